// Row gathers and the adjoint (gradient) kernels, for gfx950.
//
// Gradient of T(E) (Eq. 7 with Gamma = 2W) with respect to the local
// potential: A = E - H + iW and dA/dV_r = -e_r e_r^T give dG_ij/dV_r = G_ir G_rj,
// hence for the columns g_j = A^-1 e_j (j on the right CAP)
//     dT/dV_r = 8 Re sum_j W_R,j g_j(r) lambda_j(r),
//     lambda_j = A^-1 (W_L o conj(g_j)),
// where the transposed solve of the adjoint uses A itself because A is complex
// symmetric (Eq. 6).
#include "negf_internal.h"

namespace {

constexpr int kT = 256;

// out[dst[c] + i] = x[c][rows[i]]   (rows == null: rows are 0..n_rows-1)
__global__ __launch_bounds__(kT) void k_gather(const double2* __restrict__ x, int64_t N,
                                               const int* __restrict__ rows, int n_rows,
                                               const int64_t* __restrict__ dst,
                                               double2* __restrict__ out) {
    const int c = blockIdx.y;
    const double2* xc = x + (int64_t)c * N;
    double2* o = out + dst[c];
    for (int i = blockIdx.x * kT + threadIdx.x; i < n_rows; i += gridDim.x * kT)
        o[i] = xc[rows ? rows[i] : i];
}

// rhs[c][i] = W_L(z(i)) * conj(g[c][i])
__global__ __launch_bounds__(kT) void k_adjoint_rhs(const double2* __restrict__ g, int64_t N,
                                                    int64_t plane, const double* __restrict__ wl,
                                                    double2* __restrict__ rhs) {
    const int c = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kT) {
        const double w = wl[i / plane];
        const double2 v = g[(int64_t)c * N + i];
        rhs[(int64_t)c * N + i] = make_double2(w * v.x, -w * v.y);
    }
}

// field[r] += scale * sum_c colw[c] Re(g[c][r] lambda[c][r])   (fixed column order)
__global__ __launch_bounds__(kT) void k_field(const double2* __restrict__ g,
                                              const double2* __restrict__ lam, int64_t N, int w,
                                              const double* __restrict__ colw, double scale,
                                              double* __restrict__ field) {
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kT) {
        double s = 0.0;
        for (int c = 0; c < w; ++c) {
            const double2 a = g[(int64_t)c * N + i], b = lam[(int64_t)c * N + i];
            s += colw[c] * (a.x * b.x - a.y * b.y);
        }
        field[i] += scale * s;
    }
}

}  // namespace

void launch_gather(const double2* x, int64_t N, int w, const int* rows, int n_rows,
                   const int64_t* dst, double2* out, hipStream_t s) {
    int gx = (n_rows + kT - 1) / kT;
    if (gx > 1024) gx = 1024;
    hipLaunchKernelGGL(k_gather, dim3(gx, w), dim3(kT), 0, s, x, N, rows, n_rows, dst, out);
}

void launch_adjoint_rhs(const double2* g, int64_t N, int64_t plane, int w, const double* wl,
                        double2* rhs, hipStream_t s) {
    hipLaunchKernelGGL(k_adjoint_rhs, dim3(part_blocks(N), w), dim3(kT), 0, s, g, N, plane, wl, rhs);
}

void launch_field(const double2* g, const double2* lam, int64_t N, int w, const double* colw,
                  double scale, double* field, hipStream_t s) {
    int gx = (int)((N + kT - 1) / kT);
    if (gx > 4096) gx = 4096;
    hipLaunchKernelGGL(k_field, dim3(gx), dim3(kT), 0, s, g, lam, N, w, colw, scale, field);
}
