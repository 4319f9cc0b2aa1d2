// The complex-energy diagonalisation route of Sec. II.C (Eqs. 8-13) on the
// device, from eigenpairs (eps_i, U_i) of H_op = H - iW with U_i^T U_i = 1.
//
// With Gamma = 2W, Eq. 12's matrices are Gt_L = U^H Gamma_L U and
// Gt_R = U^T Gamma_R U^*.  Both K_L = U^H Gamma_L U and K_R = U^H Gamma_R U are
// Hermitian and Gt_R = conj(K_R), so Eq. 13's weight Gt_L,ij Gt_R,ji is the
// elementwise product M_ij = K_L,ij K_R,ij (Hermitian), and
//     T(E) = sum_ij M_ij a_j conj(a_i) = Re(a^H M a),   a_j = 1 / (E - eps_j).
// Both stages are dense complex contractions on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64; lane l supplies A[l % 16][l / 16], B[l / 16][l % 16]
// and holds D[4 i + l / 16][l % 16]): the Gram products over the CAP rows,
// and Y = M A over all energies with A generated on the fly, reduced to T by
// conj(A) o Y summed over rows.
#include "negf_internal.h"

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
constexpr int kT = 256;

__device__ inline d4_t mfma4(double a, double b, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// K[i][j] = sum_{r < n_rows} conj(U[i][row0 + r]) d[r] U[j][row0 + r]   (i, j < n_r)
// and, when prev != null, out = prev o K (elementwise) instead of K.
// U: [n_r][N] (eigenvector i contiguous); sel: eigenvector index per row of K.
// A work-group owns a 64 x 64 tile of K, each wave 32 x 32 as 2 x 2 blocks of
// 16 x 16; the rows are staged GRK per LDS pass, with the next pass's loads in
// flight during the MFMAs.  Each element's sum runs over r in order, four
// rows per MFMA.
constexpr int GRT = 64;  // Gram tile (rows and columns) per work-group
constexpr int GRK = 16;  // rows staged per LDS pass

__global__ __launch_bounds__(kT, 3) void k_gram(const double2* __restrict__ U, int64_t N,
                                             const int* __restrict__ sel, int n_r, int64_t row0,
                                             int n_rows, const double* __restrict__ d,
                                             const double2* __restrict__ prev,
                                             double2* __restrict__ out) {
    static_assert(GRT * GRK == 4 * kT, "four A and four B elements per thread and pass");
    __shared__ double2 sA[GRK][GRT + 1];
    __shared__ double2 sB[GRK][GRT + 1];
    const int i0 = blockIdx.y * GRT, j0 = blockIdx.x * GRT;
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    const int lr = lane % 16, lk = lane / 16;
    const d4_t z4 = {0.0, 0.0, 0.0, 0.0};
    d4_t cr[2][2] = {{z4, z4}, {z4, z4}}, ci[2][2] = {{z4, z4}, {z4, z4}};
    double2 va[4], vb[4];
    auto fetch = [&](int r0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + kT * u;
            const int m = e / GRK, r = r0 + e % GRK;
            va[u] = mk(0.0, 0.0);
            vb[u] = mk(0.0, 0.0);
            if (r < n_rows) {
                if (i0 + m < n_r) {
                    const double2 x = U[(int64_t)sel[i0 + m] * N + row0 + r];
                    va[u] = mk(x.x * d[r], -x.y * d[r]);  // conj(U) d
                }
                if (j0 + m < n_r) vb[u] = U[(int64_t)sel[j0 + m] * N + row0 + r];
            }
        }
    };
    fetch(0);
    for (int r0 = 0; r0 < n_rows; r0 += GRK) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + kT * u;
            sA[e % GRK][e / GRK] = va[u];
            sB[e % GRK][e / GRK] = vb[u];
        }
        __syncthreads();
        if (r0 + GRK < n_rows) fetch(r0 + GRK);
#pragma unroll
        for (int kk = 0; kk < GRK; kk += 4) {
            double2 a[2], b[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                a[q] = sA[kk + lk][wm + 16 * q + lr];
                b[q] = sB[kk + lk][wn + 16 * q + lr];
            }
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) {
                    cr[bi][bj] = mfma4(a[bi].x, b[bj].x, cr[bi][bj]);
                    cr[bi][bj] = mfma4(-a[bi].y, b[bj].y, cr[bi][bj]);
                    ci[bi][bj] = mfma4(a[bi].x, b[bj].y, ci[bi][bj]);
                    ci[bi][bj] = mfma4(a[bi].y, b[bj].x, ci[bi][bj]);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
        const int j = j0 + wn + 16 * bj + lr;
        if (j >= n_r) continue;
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int i = i0 + wm + 16 * bi + 4 * t + lk;
                if (i >= n_r) continue;
                double2 v = mk(cr[bi][bj][t], ci[bi][bj][t]);
                const int64_t o = (int64_t)i * n_r + j;
                if (prev) v = cmul(prev[o], v);
                out[o] = v;
            }
    }
}

// part[tile][e] = sum_{i in tile} Re( conj(a_i(E_e)) sum_j M[i][j] a_j(E_e) ),
// a_j(E) = 1 / (E - eps_j); one work-group per (64 rows i, 64 energies), each
// wave 32 x 32 as 2 x 2 blocks; the next slice of M and of a is prepared while
// the MFMAs run.  Each Y element's sum runs over j in order, four per MFMA.
__global__ __launch_bounds__(kT, 3) void k_eq13(const double2* __restrict__ M, int n_r,
                                                const double2* __restrict__ eps,
                                                const double* __restrict__ energies, int n_e,
                                                double* __restrict__ part) {
    static_assert(GRT * GRK == 4 * kT, "four M and four a elements per thread and pass");
    __shared__ double2 sM[GRK][GRT + 1];
    __shared__ double2 sA[GRK][GRT + 1];
    __shared__ double red[4][2][16];
    const int i0 = blockIdx.x * GRT, e0 = blockIdx.y * GRT;
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    const int lr = lane % 16, lk = lane / 16;
    const d4_t z4 = {0.0, 0.0, 0.0, 0.0};
    d4_t cr[2][2] = {{z4, z4}, {z4, z4}}, ci[2][2] = {{z4, z4}, {z4, z4}};
    double2 vm[4], va[4];
    auto fetch = [&](int j0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + kT * u;
            const int m = e / GRK, j = j0 + e % GRK;
            vm[u] = mk(0.0, 0.0);
            va[u] = mk(0.0, 0.0);
            if (j < n_r) {
                if (i0 + m < n_r) vm[u] = M[(int64_t)(i0 + m) * n_r + j];
                if (e0 + m < n_e)
                    va[u] = cdiv(mk(1.0, 0.0), mk(energies[e0 + m] - eps[j].x, -eps[j].y));
            }
        }
    };
    fetch(0);
    for (int j0 = 0; j0 < n_r; j0 += GRK) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + kT * u;
            sM[e % GRK][e / GRK] = vm[u];
            sA[e % GRK][e / GRK] = va[u];
        }
        __syncthreads();
        if (j0 + GRK < n_r) fetch(j0 + GRK);
#pragma unroll
        for (int kk = 0; kk < GRK; kk += 4) {
            double2 a[2], b[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                a[q] = sM[kk + lk][wm + 16 * q + lr];
                b[q] = sA[kk + lk][wn + 16 * q + lr];
            }
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) {
                    cr[bi][bj] = mfma4(a[bi].x, b[bj].x, cr[bi][bj]);
                    cr[bi][bj] = mfma4(-a[bi].y, b[bj].y, cr[bi][bj]);
                    ci[bi][bj] = mfma4(a[bi].x, b[bj].y, ci[bi][bj]);
                    ci[bi][bj] = mfma4(a[bi].y, b[bj].x, ci[bi][bj]);
                }
        }
        __syncthreads();
    }
    // this lane: Y[i][e] for i = i0 + wm + 16 bi + 4t + lk, e = e0 + wn + 16 bj + lr
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
        const int e = e0 + wn + 16 * bj + lr;
        double s = 0.0;
        if (e < n_e) {
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int i = i0 + wm + 16 * bi + 4 * t + lk;
                    if (i >= n_r) continue;
                    const double2 ai = cdiv(mk(1.0, 0.0), mk(energies[e] - eps[i].x, -eps[i].y));
                    s += ai.x * cr[bi][bj][t] + ai.y * ci[bi][bj][t];  // Re(conj(a_i) y)
                }
        }
        // the four lanes of one energy (lk = 0..3)
        s += __shfl_xor(s, 16, 64);
        s += __shfl_xor(s, 32, 64);
        if (lk == 0) red[wave][bj][lr] = s;
    }
    __syncthreads();
    if (tid < GRT) {
        // waves (0, 1) hold energies e0 .. e0 + 31, waves (2, 3) the next 32
        const int wc = tid / 32, bj = (tid / 16) % 2, l = tid % 16;
        const int ee = e0 + tid;
        if (ee < n_e) part[(int64_t)blockIdx.x * n_e + ee] = red[2 * wc][bj][l] + red[2 * wc + 1][bj][l];
    }
}

// T[e] = sum over row tiles of part[tile][e], in tile order
__global__ __launch_bounds__(kT) void k_sum_tiles(const double* __restrict__ part, int n_tiles,
                                                  int n_e, double* __restrict__ T) {
    const int e = blockIdx.x * kT + threadIdx.x;
    if (e >= n_e) return;
    double s = 0.0;
    for (int t = 0; t < n_tiles; ++t) s += part[(int64_t)t * n_e + e];
    T[e] = s;
}

}  // namespace

void launch_gram(const double2* U, int64_t N, const int* sel, int n_r, int64_t row0, int n_rows,
                 const double* d, const double2* prev, double2* out, hipStream_t s) {
    dim3 g((n_r + GRT - 1) / GRT, (n_r + GRT - 1) / GRT);
    hipLaunchKernelGGL(k_gram, g, dim3(kT), 0, s, U, N, sel, n_r, row0, n_rows, d, prev, out);
}

int eq13_tiles(int n_r) { return (n_r + GRT - 1) / GRT; }

void launch_eq13(const double2* M, int n_r, const double2* eps, const double* energies, int n_e,
                 double* part, double* T, hipStream_t s) {
    dim3 g(eq13_tiles(n_r), (n_e + GRT - 1) / GRT);
    hipLaunchKernelGGL(k_eq13, g, dim3(kT), 0, s, M, n_r, eps, energies, n_e, part);
    hipLaunchKernelGGL(k_sum_tiles, dim3((n_e + kT - 1) / kT), dim3(kT), 0, s, part, eq13_tiles(n_r),
                       n_e, T);
}
