// Per-energy solutions of the shared Krylov run and the reduction to T(E).
//
// The absorbing potential does not depend on E (the wide-band limit of
// Sec. II.B), so A(E_sigma) = A0 + delta_sigma 1 with A0 = A(E_seed): every
// energy shares the seed's Krylov space and its residuals are collinear with
// the seed's, r^sigma_k = r_k / pi^sigma_k.  The shifted COCG recurrences
//     p^s_k = r_k / pi^s_k + beta^s_{k-1} p^s_{k-1},   x^s_{k+1} = x^s_k + alpha^s_k p^s_k
// only involve the rows that are needed (the left absorbing region for T(E) of
// Eq. 7), so each energy keeps x^s and p^s on those rows only.
//
// Updating 2 x n_energies vectors every iteration would move far more bytes
// than the matvec.  Instead the seed residuals of a chunk of c iterations are
// kept in a ring buffer R (rows x c) and, per chunk, the recurrences are
// unrolled symbolically into
//     X <- X + xi o P + R CX,     P <- a o P + R CP
// with per-energy coefficients (CX, CP: c x n_energies; xi, a: n_energies)
// computed by a backward pass over the chunk's scalars.  The update is one
// batched complex GEMM per chunk (rows x c times c x 2 n_energies).
// For T(E) the epilogue-free reduction t_j(E) = 4 W_R,j sum_i W_L,i |X_i|^2
// runs once at the end.
#include "negf_internal.h"

namespace {

constexpr int kT = 256;

// One thread per (column, energy): coefficients of the column's chunk
// [kstart, kstart + cl) (kstart is a multiple of the chunk length).
__global__ __launch_bounds__(kT) void k_chunk_coef(IterState st, const int* __restrict__ kstart,
                                                   int* __restrict__ clen,
                                                   double2* __restrict__ cx,
                                                   double2* __restrict__ cp,
                                                   double2* __restrict__ xi_a,
                                                   double2* __restrict__ carry,
                                                   int* __restrict__ active) {
    const int g = blockIdx.x * kT + threadIdx.x;
    const int c = blockIdx.y;
    const int ng = st.ng, ch = st.chunk;
    if (g >= ng) return;
    const int cl = max(0, min(ch, st.k[c] - kstart[c]));
    // the chunk length for the GEMM, which may run while the next chunk
    // already advances st.k
    if (g == 0) clen[c] = cl;
    const int64_t o = (int64_t)c * ng + g;
    double2* CX = cx + (int64_t)c * ch * ng + g;
    double2* CP = cp + (int64_t)c * ch * ng + g;
    const double2* rec = st.rec + (int64_t)c * ch * 3 * ng + g;
    double2 S = mk(0.0, 0.0);   // S_j = alpha_j + beta_j S_{j+1}
    double2 B = mk(1.0, 0.0);   // B_j = prod_{i=j}^{cl-2} beta_i
    int act = 0;
    for (int j = ch - 1; j >= cl; --j) {
        CX[(int64_t)j * ng] = mk(0.0, 0.0);
        CP[(int64_t)j * ng] = mk(0.0, 0.0);
    }
    for (int j = cl - 1; j >= 0; --j) {
        const double2 rho = rec[(int64_t)(j * 3 + 0) * ng];
        const double2 al = rec[(int64_t)(j * 3 + 1) * ng];
        const double2 be = rec[(int64_t)(j * 3 + 2) * ng];
        if (j < cl - 1) B = cmul(be, B);
        S = cadd(al, cmul(be, S));
        if (al.x != 0.0 || al.y != 0.0) act = 1;
        CX[(int64_t)j * ng] = cmul(rho, S);
        CP[(int64_t)j * ng] = cmul(rho, B);
    }
    const double2 bprev = carry[o];
    if (cl > 0) {
        // S, B now hold S_0 and B_0 (B_0 = prod_{i=0}^{cl-2} beta_i)
        xi_a[2 * o] = cmul(bprev, S);
        xi_a[2 * o + 1] = cmul(bprev, B);
        carry[o] = rec[(int64_t)((cl - 1) * 3 + 2) * ng];
    } else {
        xi_a[2 * o] = mk(0.0, 0.0);
        xi_a[2 * o + 1] = mk(1.0, 0.0);
    }
    active[o] = act;
}

// The energies a column still iterates on, in order: list[c][0..n[c]) (one
// work-group per column; a wave ballot and a prefix over the waves per pass of
// 256 energies).  The GEMM tiles this list, so energies that have converged
// cost nothing once their 32-energy tile would otherwise stay live.
__global__ __launch_bounds__(kT) void k_compact_active(const int* __restrict__ active, int ng,
                                                       int all, int* __restrict__ list,
                                                       int* __restrict__ n_out) {
    __shared__ int wave_n[kT / 64];
    __shared__ int base_sh;
    const int c = blockIdx.x;
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    if (threadIdx.x == 0) base_sh = 0;
    __syncthreads();
    for (int g0 = 0; g0 < ng; g0 += kT) {
        const int g = g0 + threadIdx.x;
        const bool f = g < ng && (all || active[(int64_t)c * ng + g] != 0);
        const unsigned long long m = __ballot(f);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wave_n[wave] = __popcll(m);
        __syncthreads();
        int off = base_sh;
        for (int wv = 0; wv < wave; ++wv) off += wave_n[wv];
        if (f) list[(int64_t)c * ng + off + before] = g;
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = 0;
            for (int wv = 0; wv < kT / 64; ++wv) t += wave_n[wv];
            base_sh += t;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) n_out[c] = base_sh;
}

// X <- X + xi o P + R CX and P <- a o P + R CP for one column per grid z.
// 64 rows x 64 energies per work-group, 4 x 4 of each accumulator per thread.
constexpr int TM = 64, TN = 64, TK = 16;

__global__ __launch_bounds__(kT) void k_gemm_xp(const double2* __restrict__ ring, int ring_len,
                                                int w, int n_rows, const int* __restrict__ kstart, const int* __restrict__ clen,
                                                IterState st,
                                                const double2* __restrict__ cx,
                                                const double2* __restrict__ cp,
                                                const double2* __restrict__ xi_a,
                                                const int* __restrict__ active,
                                                double2* __restrict__ X, double2* __restrict__ P) {
    __shared__ double2 sR[TK][TM + 1];
    __shared__ double2 sX[TK][TN + 1];
    __shared__ double2 sP[TK][TN + 1];
    __shared__ int any_active;
    const int c = blockIdx.z;
    const int row0 = blockIdx.x * TM;
    const int g0 = blockIdx.y * TN;
    const int ng = st.ng, ch = st.chunk;
    const int k0 = kstart[c];
    const int cl = clen[c];
    if (cl == 0) return;
    const int tid = threadIdx.x;
    if (tid == 0) any_active = 0;
    __syncthreads();
    if (tid < TN && g0 + tid < ng && active[(int64_t)c * ng + g0 + tid]) any_active = 1;
    __syncthreads();
    if (!any_active) return;
    const int tr = tid % 16, ts = tid / 16;
    double2 ax[4][4], ap[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            ax[i][j] = mk(0.0, 0.0);
            ap[i][j] = mk(0.0, 0.0);
        }
    const double2* CX = cx + (int64_t)c * ch * ng;
    const double2* CP = cp + (int64_t)c * ch * ng;
    for (int j0 = 0; j0 < cl; j0 += TK) {
        for (int e = tid; e < TK * TM; e += kT) {
            const int jj = e / TM, rr = e % TM;
            const int j = j0 + jj, row = row0 + rr;
            double2 v = mk(0.0, 0.0);
            if (j < cl && row < n_rows) {
                const int slot = (k0 + j) % ring_len;
                v = ring[((int64_t)slot * w + c) * n_rows + row];
            }
            sR[jj][rr] = v;
        }
        for (int e = tid; e < TK * TN; e += kT) {
            const int jj = e / TN, gg = e % TN;
            const int j = j0 + jj, g = g0 + gg;
            double2 vx = mk(0.0, 0.0), vp = mk(0.0, 0.0);
            if (j < cl && g < ng) {
                vx = CX[(int64_t)j * ng + g];
                vp = CP[(int64_t)j * ng + g];
            }
            sX[jj][gg] = vx;
            sP[jj][gg] = vp;
        }
        __syncthreads();
#pragma unroll 2
        for (int jj = 0; jj < TK; ++jj) {
            double2 a[4], bx[4], bp[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = sR[jj][tr + 16 * i];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                bx[q] = sX[jj][ts + 16 * q];
                bp[q] = sP[jj][ts + 16 * q];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    ax[i][q].x = fma(a[i].x, bx[q].x, fma(-a[i].y, bx[q].y, ax[i][q].x));
                    ax[i][q].y = fma(a[i].x, bx[q].y, fma(a[i].y, bx[q].x, ax[i][q].y));
                    ap[i][q].x = fma(a[i].x, bp[q].x, fma(-a[i].y, bp[q].y, ap[i][q].x));
                    ap[i][q].y = fma(a[i].x, bp[q].y, fma(a[i].y, bp[q].x, ap[i][q].y));
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int g = g0 + ts + 16 * q;
        if (g >= ng) continue;
        const int64_t o = (int64_t)c * ng + g;
        const double2 xi = xi_a[2 * o], aa = xi_a[2 * o + 1];
        double2* Xg = X + o * n_rows;
        double2* Pg = P + o * n_rows;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = row0 + tr + 16 * i;
            if (row >= n_rows) continue;
            const double2 p0 = Pg[row];
            Xg[row] = cadd(cadd(Xg[row], cmul(xi, p0)), ax[i][q]);
            Pg[row] = cadd(cmul(aa, p0), ap[i][q]);
        }
    }
}

// The same update on the matrix cores (v_mfma_f64_16x16x4f64).  Lane layout
// of that instruction: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
// and holds D[4 i + l / 16][l % 16], i = 0..3.  A complex product takes four
// real ones: Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br.  A work-group of four
// waves owns 64 rows x 32 energies; each wave 32 rows x 16 energies as two
// 16 x 16 blocks for X and two for P (eight accumulators). The launch bound
// asks for four waves per SIMD: four work-groups per CU hid the staging loads
// better than three (10.7 ms against 12.4 ms per 128 iterations on the
// 32x32x192 wire).  Staging 8 iterations per pass leaves room in those 128
// VGPRs to keep the next pass's loads in flight during the MFMAs (+1.3 % on
// the whole bench against 16 iterations staged without prefetch); the order
// of the accumulation is the same either way.
typedef double d4_t __attribute__((ext_vector_type(4)));
constexpr int MK = 8;    // chunk iterations staged per LDS pass
constexpr int MTN = 32;  // energies per work-group

__device__ inline d4_t mfma4(double a, double b, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(kT, 4) void k_gemm_xp_mfma(const double2* __restrict__ ring, int ring_len,
                                                     int w, int n_rows,
                                                     const int* __restrict__ kstart, const int* __restrict__ clen, IterState st,
                                                     const double2* __restrict__ cx,
                                                     const double2* __restrict__ cp,
                                                     const double2* __restrict__ xi_a,
                                                     const int* __restrict__ act_list,
                                                     const int* __restrict__ act_n,
                                                     double2* __restrict__ X,
                                                     double2* __restrict__ P) {
    __shared__ double2 sR[MK][TM];
    __shared__ double2 sX[MK][MTN];
    __shared__ double2 sP[MK][MTN];
    static_assert(MK * TM == 2 * kT && MK * MTN == kT, "one pass: two ring and one coefficient element per thread");
    __shared__ int sg[MTN];  // the tile's energies (-1 past the list)
    const int c = blockIdx.z;
    const int row0 = blockIdx.x * TM;
    const int t0 = blockIdx.y * MTN;  // tile of the column's list of live energies
    const int ng = st.ng, ch = st.chunk;
    const int k0 = kstart[c];
    const int cl = clen[c];
    const int na = act_n[c];
    if (cl == 0 || t0 >= na) return;
    const int tid = threadIdx.x;
    if (tid < MTN) sg[tid] = (t0 + tid < na) ? act_list[(int64_t)c * ng + t0 + tid] : -1;
    __syncthreads();
    const int lane = tid % 64, wave = tid / 64;
    const int wr = (wave & 1) * 32, wc = (wave >> 1) * 16;  // the wave's rows / energies
    const int lr = lane % 16, lk = lane / 16;
    const d4_t zero4 = {0.0, 0.0, 0.0, 0.0};
    d4_t axr[2] = {zero4, zero4}, axi[2] = {zero4, zero4};
    d4_t apr[2] = {zero4, zero4}, api[2] = {zero4, zero4};
    const double2* CX = cx + (int64_t)c * ch * ng;
    const double2* CP = cp + (int64_t)c * ch * ng;
    // the next pass's global loads are in flight (registers) while the matrix
    // cores work on the staged one
    double2 ra[2], rx, rp;
    auto fetch = [&](int j0) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = tid + kT * u;
            const int j = j0 + e / TM, row = row0 + e % TM;
            double2 v = mk(0.0, 0.0);
            if (j < cl && row < n_rows) {
                const int slot = (k0 + j) % ring_len;
                v = ring[((int64_t)slot * w + c) * n_rows + row];
            }
            ra[u] = v;
        }
        const int j = j0 + tid / MTN, g = sg[tid % MTN];
        rx = mk(0.0, 0.0);
        rp = mk(0.0, 0.0);
        if (j < cl && g >= 0) {
            rx = CX[(int64_t)j * ng + g];
            rp = CP[(int64_t)j * ng + g];
        }
    };
    fetch(0);
    for (int j0 = 0; j0 < cl; j0 += MK) {
        sR[tid / TM][tid % TM] = ra[0];
        sR[(tid + kT) / TM][(tid + kT) % TM] = ra[1];
        sX[tid / MTN][tid % MTN] = rx;
        sP[tid / MTN][tid % MTN] = rp;
        __syncthreads();
        if (j0 + MK < cl) fetch(j0 + MK);
#pragma unroll 2
        for (int kk = 0; kk < MK; kk += 4) {
            const double2 a0 = sR[kk + lk][wr + lr];
            const double2 a1 = sR[kk + lk][wr + 16 + lr];
            const double2 bx = sX[kk + lk][wc + lr];
            const double2 bp = sP[kk + lk][wc + lr];
            axr[0] = mfma4(a0.x, bx.x, axr[0]);
            axr[0] = mfma4(-a0.y, bx.y, axr[0]);
            axi[0] = mfma4(a0.x, bx.y, axi[0]);
            axi[0] = mfma4(a0.y, bx.x, axi[0]);
            axr[1] = mfma4(a1.x, bx.x, axr[1]);
            axr[1] = mfma4(-a1.y, bx.y, axr[1]);
            axi[1] = mfma4(a1.x, bx.y, axi[1]);
            axi[1] = mfma4(a1.y, bx.x, axi[1]);
            apr[0] = mfma4(a0.x, bp.x, apr[0]);
            apr[0] = mfma4(-a0.y, bp.y, apr[0]);
            api[0] = mfma4(a0.x, bp.y, api[0]);
            api[0] = mfma4(a0.y, bp.x, api[0]);
            apr[1] = mfma4(a1.x, bp.x, apr[1]);
            apr[1] = mfma4(-a1.y, bp.y, apr[1]);
            api[1] = mfma4(a1.x, bp.y, api[1]);
            api[1] = mfma4(a1.y, bp.x, api[1]);
        }
        __syncthreads();
    }
    const int g = sg[wc + lr];
    if (g < 0) return;
    const int64_t o = (int64_t)c * ng + g;
    const double2 xi = xi_a[2 * o], aa = xi_a[2 * o + 1];
    double2* Xg = X + o * n_rows;
    double2* Pg = P + o * n_rows;
#pragma unroll
    for (int ra = 0; ra < 2; ++ra)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = row0 + wr + 16 * ra + 4 * i + lk;
            if (row >= n_rows) continue;
            const double2 p0 = Pg[row];
            Xg[row] = cadd(cadd(Xg[row], cmul(xi, p0)), mk(axr[ra][i], axi[ra][i]));
            Pg[row] = cadd(cmul(aa, p0), mk(apr[ra][i], api[ra][i]));
        }
}

// t[c][g] = col_w[c] * sum_row row_w[row] |X[c][g][row]|^2, one work-group per (g, c);
// only (nullable) selects the columns to reduce
__global__ __launch_bounds__(kT) void k_t_from_x(const double2* __restrict__ X, int n_rows, int ng,
                                                 const double* __restrict__ row_w,
                                                 const double* __restrict__ col_w,
                                                 const int* __restrict__ only,
                                                 double* __restrict__ t) {
    __shared__ double lds[kT / 64];
    const int g = blockIdx.x, c = blockIdx.y;
    if (only && !only[c]) return;
    const double2* x = X + ((int64_t)c * ng + g) * n_rows;
    double s = 0.0;
    for (int i = threadIdx.x; i < n_rows; i += kT) s += row_w[i] * cabs2(x[i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (threadIdx.x % 64 == 0) lds[threadIdx.x / 64] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int wv = 0; wv < kT / 64; ++wv) tot += lds[wv];
        t[(int64_t)c * ng + g] = col_w[c] * tot;
    }
}

// The optical theorem of one column g_j = A(E)^-1 e_j: with A = E - H + iW and
// H real symmetric, Im(g_j^H A g_j) gives sum_i W_i |g_ij|^2 = -Im g_jj, so
// |sum_i W_i |g_ij|^2 + Im g_jj| / |Im g_jj| measures how well the iterate
// solves its system.  One work-group per (energy, column).
__global__ __launch_bounds__(kT) void k_optical(const double2* __restrict__ X, int64_t stride,
                                                int n_keep, int ng,
                                                const double* __restrict__ row_w,
                                                const int* __restrict__ jloc,
                                                const int* __restrict__ only,
                                                double* __restrict__ out) {
    __shared__ double lds[kT / 64];
    const int g = blockIdx.x, c = blockIdx.y;
    if (only && !only[c]) return;
    const double2* x = X + ((int64_t)c * ng + g) * stride;
    double s = 0.0;
    for (int i = threadIdx.x; i < n_keep; i += kT) s += row_w[i] * cabs2(x[i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (threadIdx.x % 64 == 0) lds[threadIdx.x / 64] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int wv = 0; wv < kT / 64; ++wv) tot += lds[wv];
        const double im = x[jloc[c]].y;
        out[(int64_t)c * ng + g] = fabs(tot + im) / fabs(im);
    }
}

// out[g * shift_stride + c * col_stride + row] = X[c][g][row]
__global__ __launch_bounds__(kT) void k_copy_out(const double2* __restrict__ X, int n_rows, int ng,
                                                 double2* __restrict__ out, int64_t col_stride,
                                                 int64_t shift_stride) {
    const int g = blockIdx.y % ng, c = blockIdx.y / ng;
    const double2* x = X + ((int64_t)c * ng + g) * n_rows;
    double2* o = out + (int64_t)g * shift_stride + (int64_t)c * col_stride;
    for (int i = blockIdx.x * kT + threadIdx.x; i < n_rows; i += gridDim.x * kT) o[i] = x[i];
}

}  // namespace

void launch_chunk_coef(const IterState& st, const int* kstart, int* clen, double2* cx,
                       double2* cp, double2* xi_a, double2* carry, int* active, int* act_list,
                       int* act_n, hipStream_t s) {
    dim3 g((st.ng + kT - 1) / kT, st.w);
    hipLaunchKernelGGL(k_chunk_coef, g, dim3(kT), 0, s, st, kstart, clen, cx, cp, xi_a, carry,
                       active);
    // NEGF_GEMM_NO_COMPACT=1 lists every energy (a reference for tests: the
    // frozen ones then get zero coefficients, so X comes out bit for bit the same)
    const char* e = getenv("NEGF_GEMM_NO_COMPACT");
    const int all = (e && e[0] == '1') ? 1 : 0;
    hipLaunchKernelGGL(k_compact_active, dim3(st.w), dim3(kT), 0, s, active, st.ng, all, act_list,
                       act_n);
}

void launch_gemm_xp(const double2* ring, int ring_len, int w, int n_rows, const int* kstart,
                    const int* clen, const IterState& st, const double2* cx, const double2* cp,
                    const double2* xi_a, const int* active, const int* act_list,
                    const int* act_n, double2* X, double2* P, hipStream_t s) {
    dim3 g((n_rows + TM - 1) / TM, (st.ng + TN - 1) / TN, w);
    // NEGF_GEMM_VALU=1 selects the vector-ALU kernel (read per chunk)
    const char* env = getenv("NEGF_GEMM_VALU");
    const bool valu = env && env[0] == '1';
    if (valu)
        hipLaunchKernelGGL(k_gemm_xp, g, dim3(kT), 0, s, ring, ring_len, w, n_rows, kstart, clen,
                           st, cx, cp, xi_a, active, X, P);
    else
        hipLaunchKernelGGL(k_gemm_xp_mfma, dim3(g.x, (st.ng + MTN - 1) / MTN, w), dim3(kT), 0, s,
                           ring, ring_len, w, n_rows, kstart, clen, st, cx, cp, xi_a, act_list,
                           act_n, X, P);
}

void launch_t_from_x(const double2* X, int n_rows, int w, int ng, const double* row_w,
                     const double* col_w, const int* only, double* t, hipStream_t s) {
    hipLaunchKernelGGL(k_t_from_x, dim3(ng, w), dim3(kT), 0, s, X, n_rows, ng, row_w, col_w, only,
                       t);
}

void launch_optical(const double2* X, int64_t stride, int n_keep, int w, int ng,
                    const double* row_w, const int* jloc, const int* only, double* out,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_optical, dim3(ng, w), dim3(kT), 0, s, X, stride, n_keep, ng, row_w, jloc,
                       only, out);
}

void launch_copy_out(const double2* X, int n_rows, int w, int ng, double2* out, int64_t col_stride,
                     int64_t shift_stride, hipStream_t s) {
    int gx = (n_rows + kT - 1) / kT;
    if (gx > 64) gx = 64;
    hipLaunchKernelGGL(k_copy_out, dim3(gx, ng * w), dim3(kT), 0, s, X, n_rows, ng, out,
                       col_stride, shift_stride);
}
