// Per-energy coefficients of the shared Krylov basis and the reduction to T(E).
//
// The seed COCG run stores its residuals r_0 .. r_{m-1} restricted to the rows
// that are needed (the left absorbing region for T(E) of Eq. 7).  They obey
//     A0 r_k = -(beta_{k-1}/alpha_{k-1}) r_{k-1} + (1/alpha_k + beta_{k-1}/alpha_{k-1}) r_k
//              - (1/alpha_k) r_{k+1},
// i.e. A0 R_m = R_m T_m - (1/alpha_{m-1}) r_m e_m^T with a tridiagonal T_m.  For
// the shifted system (A0 + delta) x = b the Galerkin iterate is x = R_m y with
// (T_m + delta) y = e_1 ||b||-scaled, which is what shifted COCG produces; it
// is solved here per (column, energy) with partial pivoting on the
// diagonally rescaled matrix S T_m S^-1, S = diag(||r_k||), which keeps every
// entry O(1) however far the seed residual has decayed.
//
// X(rows, energies) = V (rows x m) * Gamma (m x n_energies) is then a batched
// complex GEMM; for T(E) its result is never stored: the epilogue forms
// sum_i W_L,i |X_i,e|^2 directly (the column weight 4 W_R,j is applied last).
#include "negf_internal.h"

namespace {

constexpr int kT = 256;

__device__ inline double2 diag_entry(const double2* ah, const double2* bh, int kk, double d) {
    double2 v = cdiv(mk(1.0, 0.0), ah[kk]);
    if (kk > 0) v = cadd(v, cdiv(bh[kk - 1], ah[kk - 1]));
    v.x += d;
    return v;
}

__global__ __launch_bounds__(kT) void k_tridiag(IterState st, const int* __restrict__ m_col,
                                                double2* __restrict__ gamma, int m_max,
                                                double2* __restrict__ tri,
                                                double* __restrict__ resid) {
    const int g = blockIdx.x * kT + threadIdx.x;
    const int c = blockIdx.y;
    const int ng = st.ng;
    if (g >= ng) return;
    const int m = m_col[c];
    const double2* ah = st.a_hist + (int64_t)c * st.max_iter;
    const double2* bh = st.b_hist + (int64_t)c * st.max_iter;
    const double* sh = st.s_hist + (int64_t)c * (st.max_iter + 1);
    const double d = st.deltas[(int64_t)c * ng + g];
    double2* G = gamma + (int64_t)c * m_max * ng;
    double2* Tr = tri + (int64_t)c * m_max * 4 * ng;
    if (m <= 0) {
        if (resid) resid[(int64_t)c * ng + g] = 1.0;
        return;
    }
    // forward elimination with row interchanges
    double2 cur_d = diag_entry(ah, bh, 0, d);
    double2 cur_u = (m > 1) ? cscale(-sh[0] / sh[1], cdiv(bh[0], ah[0])) : mk(0.0, 0.0);
    double2 rhs = mk(sh[0], 0.0);
    for (int kk = 0; kk + 1 < m; ++kk) {
        const double2 l = cscale(-sh[kk + 1] / sh[kk], cdiv(mk(1.0, 0.0), ah[kk]));
        const double2 nd = diag_entry(ah, bh, kk + 1, d);
        const double2 nu = (kk + 2 < m) ? cscale(-sh[kk + 1] / sh[kk + 2], cdiv(bh[kk + 1], ah[kk + 1]))
                                        : mk(0.0, 0.0);
        double2 D, DU, DU2, RH;
        if (cabs2(cur_d) >= cabs2(l)) {
            const double2 f = cdiv(l, cur_d);
            D = cur_d; DU = cur_u; DU2 = mk(0.0, 0.0); RH = rhs;
            cur_d = csub(nd, cmul(f, cur_u));
            cur_u = nu;
            rhs = csub(mk(0.0, 0.0), cmul(f, rhs));
        } else {
            const double2 f = cdiv(cur_d, l);
            D = l; DU = nd; DU2 = nu; RH = mk(0.0, 0.0);
            const double2 od = cur_d, ou = cur_u;
            (void)od;
            cur_d = csub(ou, cmul(f, nd));
            cur_u = csub(mk(0.0, 0.0), cmul(f, nu));
            rhs = rhs;  // old row kk moves down: rhs_{kk+1} = rhs_kk - f * 0
        }
        double2* row = Tr + ((int64_t)kk * 4) * ng + g;
        row[0] = D; row[ng] = DU; row[2 * ng] = DU2; row[3 * ng] = RH;
    }
    // back substitution
    double2 y1 = cdiv(rhs, cur_d);  // y_{m-1}
    const double2 ylast = y1;
    double2 y2 = mk(0.0, 0.0);
    G[(int64_t)(m - 1) * ng + g] = cscale(1.0 / sh[m - 1], y1);
    for (int kk = m - 2; kk >= 0; --kk) {
        const double2* row = Tr + ((int64_t)kk * 4) * ng + g;
        const double2 D = row[0], DU = row[ng], DU2 = row[2 * ng], RH = row[3 * ng];
        const double2 y = cdiv(csub(csub(RH, cmul(DU, y1)), cmul(DU2, y2)), D);
        G[(int64_t)kk * ng + g] = cscale(1.0 / sh[kk], y);
        y2 = y1;
        y1 = y;
    }
    if (resid) {
        // ||b - (A0 + delta) x|| / ||b|| = |T_{m,m-1}| |y_{m-1}| / s_0 (scaled basis)
        const double tsub = (sh[m] / sh[m - 1]) / sqrt(cabs2(ah[m - 1]));
        resid[(int64_t)c * ng + g] = tsub * sqrt(cabs2(ylast)) / sh[0];
    }
}

// X = V * Gamma for one column per grid z; 64 rows x 64 energies per work-group,
// 4 x 4 complex accumulators per thread.  MODE 0: weighted |X|^2 row sums;
// MODE 1: store X.
constexpr int TM = 64, TN = 64, TK = 16;

template <int MODE>
__global__ __launch_bounds__(kT) void k_gemm(double2* const* __restrict__ tab, int chunk_iters,
                                             int w, int n_rows, const int* __restrict__ m_col,
                                             const double2* __restrict__ gamma, int m_max, int ng,
                                             const double* __restrict__ row_w,
                                             double* __restrict__ tpart, double2* __restrict__ out,
                                             int64_t out_col_stride, int64_t out_shift_stride) {
    __shared__ double2 sV[TK][TM + 1];
    __shared__ double2 sG[TK][TN + 1];
    __shared__ double red[16][TN];
    const int c = blockIdx.z;
    const int row0 = blockIdx.x * TM;
    const int g0 = blockIdx.y * TN;
    const int m = m_col[c];
    const int tid = threadIdx.x;
    const int tr = tid % 16, ts = tid / 16;
    double2 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mk(0.0, 0.0);
    const double2* G = gamma + (int64_t)c * m_max * ng;
    for (int k0 = 0; k0 < m; k0 += TK) {
        // load V tile: TK slots x TM rows
        for (int e = tid; e < TK * TM; e += kT) {
            const int kk = e / TM, rr = e % TM;
            const int slot = k0 + kk, row = row0 + rr;
            double2 v = mk(0.0, 0.0);
            if (slot < m && row < n_rows)
                v = tab[slot / chunk_iters][((int64_t)(slot % chunk_iters) * w + c) * n_rows + row];
            sV[kk][rr] = v;
        }
        for (int e = tid; e < TK * TN; e += kT) {
            const int kk = e / TN, gg = e % TN;
            const int slot = k0 + kk, g = g0 + gg;
            double2 v = mk(0.0, 0.0);
            if (slot < m && g < ng) v = G[(int64_t)slot * ng + g];
            sG[kk][gg] = v;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < TK; ++kk) {
            double2 a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = sV[kk][tr + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = sG[kk][ts + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    acc[i][j].x = fma(a[i].x, b[j].x, fma(-a[i].y, b[j].y, acc[i][j].x));
                    acc[i][j].y = fma(a[i].x, b[j].y, fma(a[i].y, b[j].x, acc[i][j].y));
                }
        }
        __syncthreads();
    }
    if (MODE == 0) {
        double part[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = row0 + tr + 16 * i;
            const double wgt = (row < n_rows) ? row_w[row] : 0.0;
#pragma unroll
            for (int j = 0; j < 4; ++j) part[j] += wgt * cabs2(acc[i][j]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) red[tr][ts + 16 * j] = part[j];
        __syncthreads();
        if (tid < TN) {
            double s = 0.0;
            for (int t = 0; t < 16; ++t) s += red[t][tid];
            const int g = g0 + tid;
            const int n_tiles = gridDim.x;
            if (g < ng) tpart[((int64_t)c * n_tiles + blockIdx.x) * ng + g] = s;
        }
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = row0 + tr + 16 * i;
            if (row >= n_rows) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int g = g0 + ts + 16 * j;
                if (g < ng) out[(int64_t)g * out_shift_stride + (int64_t)c * out_col_stride + row] = acc[i][j];
            }
        }
    }
}

__global__ __launch_bounds__(kT) void k_sum_tpart(const double* __restrict__ tpart, int n_tiles,
                                                  int w, int ng, const double* __restrict__ col_w,
                                                  double* __restrict__ tcol) {
    const int g = blockIdx.x * kT + threadIdx.x;
    const int c = blockIdx.y;
    if (g >= ng) return;
    double s = 0.0;
    for (int t = 0; t < n_tiles; ++t) s += tpart[((int64_t)c * n_tiles + t) * ng + g];
    tcol[(int64_t)c * ng + g] = col_w[c] * s;
}

}  // namespace

void launch_tridiag_solve(IterState st, const int* m_col, double2* gamma, int m_max, double2* tri,
                          double* resid_out, hipStream_t s) {
    dim3 g((st.ng + kT - 1) / kT, st.w);
    hipLaunchKernelGGL(k_tridiag, g, dim3(kT), 0, s, st, m_col, gamma, m_max, tri, resid_out);
}

void launch_gemm_reduce(double2* const* chunk_tab, int chunk_iters, int w, int n_rows,
                        const int* m_col, const double2* gamma, int m_max, int ng,
                        const double* row_w, double* tpart, hipStream_t s) {
    dim3 g((n_rows + TM - 1) / TM, (ng + TN - 1) / TN, w);
    hipLaunchKernelGGL((k_gemm<0>), g, dim3(kT), 0, s, chunk_tab, chunk_iters, w, n_rows, m_col,
                       gamma, m_max, ng, row_w, tpart, (double2*)nullptr, (int64_t)0, (int64_t)0);
}

void launch_gemm_store(double2* const* chunk_tab, int chunk_iters, int w, int n_rows,
                       const int* m_col, const double2* gamma, int m_max, int ng, double2* out,
                       int64_t out_col_stride, int64_t out_shift_stride, hipStream_t s) {
    dim3 g((n_rows + TM - 1) / TM, (ng + TN - 1) / TN, w);
    hipLaunchKernelGGL((k_gemm<1>), g, dim3(kT), 0, s, chunk_tab, chunk_iters, w, n_rows, m_col,
                       gamma, m_max, ng, (const double*)nullptr, (double*)nullptr, out,
                       out_col_stride, out_shift_stride);
}

void launch_sum_tpart(const double* tpart, int n_tiles, int w, int ng, const double* col_w,
                      double* tcol, hipStream_t s) {
    dim3 g((ng + kT - 1) / kT, w);
    hipLaunchKernelGGL(k_sum_tpart, g, dim3(kT), 0, s, tpart, n_tiles, w, ng, col_w, tcol);
}
