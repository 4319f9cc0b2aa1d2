// Internal declarations of libnegf (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "negf.h"

// ---------------------------------------------------------------------------
// complex helpers (interleaved re/im in HIP vector types)
// ---------------------------------------------------------------------------
template <typename R> struct cplx_of;
template <> struct cplx_of<double> { using type = double2; };
template <> struct cplx_of<float> { using type = float2; };
template <typename R> using cplx_t = typename cplx_of<R>::type;

__host__ __device__ inline double2 mk(double a, double b) { return make_double2(a, b); }
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return mk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return mk(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
    return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cscale(double s, double2 a) { return mk(s * a.x, s * a.y); }
__host__ __device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline double2 cdiv(double2 a, double2 b) {
    // Smith's algorithm keeps the intermediate products in range.
    if (fabs(b.x) >= fabs(b.y)) {
        double r = b.y / b.x, den = b.x + b.y * r;
        return mk((a.x + a.y * r) / den, (a.y - a.x * r) / den);
    } else {
        double r = b.x / b.y, den = b.x * r + b.y;
        return mk((a.x * r + a.y) / den, (a.y * r - a.x) / den);
    }
}
__host__ __device__ inline bool cfinite(double2 a) { return isfinite(a.x) && isfinite(a.y); }

// ---------------------------------------------------------------------------
// operator
// ---------------------------------------------------------------------------
struct StencilCoef {
    double a[7];  // a[0]: on-site kinetic 3 c_0 / (2h^2); a[m]: c_m / (2h^2)
};

struct DeviceKB {
    int n_proj = 0;
    int64_t nnz = 0;
    int64_t* off = nullptr;   // [n_proj + 1]
    int* idx = nullptr;       // [nnz]
    double* val = nullptr;    // [nnz]
    float* valf = nullptr;    // [nnz]
    double* e = nullptr;      // [n_proj]
    // point-major transpose for the scatter: unique points and their entries
    int n_pts = 0;
    int* pts = nullptr;       // [n_pts]
    int* pt_off = nullptr;    // [n_pts + 1]
    int* pt_proj = nullptr;   // [nnz]
    double* pt_val = nullptr; // [nnz]  E_p * b_p(i)
    int max_support = 0;
};

struct Buffer {
    void* ptr = nullptr;
    size_t bytes = 0;
};

struct negf_op {
    int device = 0;
    int nx = 0, ny = 0, nz = 0, R = 0;
    double h = 0;
    int64_t N = 0;
    StencilCoef coef{};
    std::vector<double> cap_l, cap_r;   // per plane
    int zl0 = 0, zl1 = 0, zr0 = 0, zr1 = 0;  // CAP planes [z0, z1)
    double* d_v = nullptr;       // [N]
    double* d_wz = nullptr;      // [nz] W_L + W_R per plane
    double* d_wl = nullptr;      // [nz]
    double* d_wr = nullptr;      // [nz]
    DeviceKB kb;
    hipStream_t own_stream = nullptr;
    std::vector<Buffer> bufs;    // workspace, indexed by WorkSlot
    std::vector<Buffer> vchunks; // stored Krylov vectors (multi-shift)
};

// status plumbing (thread-local message)
void set_error(const char* fmt, ...);
negf_status hip_fail(hipError_t e, const char* what, int line);
#define HIPCHK(x)                                                      \
    do {                                                               \
        hipError_t _e = (x);                                           \
        if (_e != hipSuccess) return hip_fail(_e, #x, __LINE__);       \
    } while (0)

// workspace slots
enum WorkSlot {
    WS_R = 0, WS_P, WS_Q, WS_X, WS_B, WS_R64, WS_X64, WS_Q64,
    WS_PART, WS_PART2, WS_PART3, WS_KBC, WS_SHIFT, WS_COLJ,
    WS_STATE, WS_HIST, WS_PI, WS_GAMMA, WS_TRI, WS_TPART, WS_TCOL, WS_ROWS,
    WS_ROWW, WS_CHUNKTAB, WS_MISC, WS_COUNT
};
negf_status ws_get(negf_op* op, int slot, size_t bytes, void** out);

// ---------------------------------------------------------------------------
// launchers (kernels in *.hip)
// ---------------------------------------------------------------------------
// Y = A(E_c) X, column-major blocks [w][N]; skip[c] != 0 leaves column c alone.
template <typename R>
void launch_apply(const negf_op* op, const cplx_t<R>* x, cplx_t<R>* y, int w,
                  const double* d_shift, const int* d_skip, double2* d_kbc,
                  hipStream_t s);

// elementwise / reductions for the Krylov solvers
struct IterState {
    int w = 0;               // columns in the block
    int ng = 0;              // shifts per column (multi-shift)
    int max_iter = 0;
    int* k = nullptr;        // [w] completed iterations
    int* done = nullptr;     // [w] 0 running, else 1+NEGF_ITEM_*
    double2* rho = nullptr;  // [w]
    double2* alpha = nullptr;// [w]
    double2* beta = nullptr; // [w]  beta_{k-1}, used by p = r + beta p
    double* bnorm = nullptr; // [w]
    double* rnorm = nullptr; // [w]
    double2* a_hist = nullptr; // [w][max_iter]
    double2* b_hist = nullptr; // [w][max_iter]
    double* s_hist = nullptr;  // [w][max_iter + 1]
    double2* pih = nullptr;    // [w][ng] scaled pi_k
    double2* pih_prev = nullptr; // [w][ng]
    double* deltas = nullptr;  // [w][ng] real shifts E_sigma - E_seed (per column)
    int* sconv = nullptr;      // [w][ng] shift converged (sticky; its recurrence is frozen)
    int* running = nullptr;    // [1] count of running columns after a step
    double tol = 1e-10;
};

int part_blocks(int64_t n);
template <typename R>
void launch_p_update(const cplx_t<R>* r, cplx_t<R>* p, const IterState& st, int64_t N, hipStream_t s);
template <typename R>
void launch_dot_pq(const cplx_t<R>* p, const cplx_t<R>* q, double2* part, const IterState& st,
                   int64_t N, hipStream_t s);
void launch_reduce_alpha(const double2* part, int nblk, IterState st, hipStream_t s);
template <typename R>
void launch_r_update(cplx_t<R>* r, const cplx_t<R>* q, cplx_t<R>* p_or_null, cplx_t<R>* x_or_null,
                     double2* part_rr, double* part_nn, const IterState& st, int64_t N,
                     hipStream_t s);
void launch_reduce_beta_multishift(const double2* part_rr, const double* part_nn, int nblk,
                                   IterState st, hipStream_t s);
void launch_reduce_beta_single(const double2* part_rr, const double* part_nn, int nblk,
                               IterState st, double inner_tol, hipStream_t s);
template <typename R>
void launch_store_rows(const cplx_t<R>* r, int64_t N, int w, const int* rows, int64_t row0,
                       int n_rows, double2* const* chunk_tab, int chunk_iters,
                       const IterState& st, int slot_offset, hipStream_t s);
void launch_tridiag_solve(IterState st, const int* m_col, double2* gamma, int m_max,
                          double2* tri, double* resid_out, hipStream_t s);
void launch_gemm_reduce(double2* const* chunk_tab, int chunk_iters, int w, int n_rows,
                        const int* m_col, const double2* gamma, int m_max, int ng,
                        const double* row_w, double* tpart, hipStream_t s);
void launch_gemm_store(double2* const* chunk_tab, int chunk_iters, int w, int n_rows,
                       const int* m_col, const double2* gamma, int m_max, int ng,
                       double2* out, int64_t out_col_stride, int64_t out_shift_stride,
                       hipStream_t s);
void launch_sum_tpart(const double* tpart, int n_tiles, int w, int ng, const double* col_w,
                      double* tcol, hipStream_t s);
