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

// A complex element loaded with the non-temporal hint: for streams read once
// and dead afterwards, so that they do not displace data still to be reused
template <typename R>
__device__ __forceinline__ cplx_t<R> ld_once(const cplx_t<R>* p) {
    typedef R v2 __attribute__((ext_vector_type(2)));
    const v2 t = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    cplx_t<R> o;
    o.x = t.x;
    o.y = t.y;
    return o;
}

// A complex element stored with the non-temporal hint
template <typename R>
__device__ __forceinline__ void st_once(cplx_t<R>* p, const cplx_t<R>& v) {
    typedef R v2 __attribute__((ext_vector_type(2)));
    v2 t;
    t.x = v.x;
    t.y = v.y;
    __builtin_nontemporal_store(t, reinterpret_cast<v2*>(p));
}

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
    int* slot = nullptr;      // [N] index into pts, or -1
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
    void* d_sink = nullptr;      // discard target of the whole-plane stencil kernel (workspace)
    DeviceKB kb;
    hipStream_t own_stream = nullptr;
    hipStream_t side_stream = nullptr;  // the shift-accumulation GEMM, beside the iterations
    std::vector<Buffer> bufs;    // workspace, indexed by WorkSlot
    // launch shape (negf_tune); 0 / -1 = built-in choice
    int tuned_w = 0;             // source columns per multi-shift block
    int wg_target = 0;           // stencil work-groups per launch the z-chunking aims for
    int plane_kernel = -1;       // 1 whole-plane kernel, 0 row-tiled, -1 auto
};

// status plumbing (thread-local message)
void set_error(const char* fmt, ...);
negf_status hip_fail(hipError_t e, const char* what, int line);
#define HIPCHK(x)                                                      \
    do {                                                               \
        hipError_t _e = (x);                                           \
        if (_e != hipSuccess) return hip_fail(_e, #x, __LINE__);       \
    } while (0)

#define CHK(x)                                  \
    do {                                        \
        negf_status _s = (x);                   \
        if (_s != NEGF_OK) return _s;           \
    } while (0)

// workspace slots
enum WorkSlot {
    WS_R = 0, WS_P, WS_Q, WS_X, WS_B, WS_R64, WS_X64, WS_Q64,
    WS_PART, WS_PART2, WS_PART3, WS_KBC, WS_SHIFT, WS_COLJ,
    WS_STATE, WS_HIST, WS_PI, WS_GAMMA, WS_TRI, WS_TPART, WS_TCOL, WS_ROWS,
    WS_ROWW, WS_RING, WS_XS, WS_PS, WS_COEF, WS_MISC, WS_SINK, WS_SLOTS, WS_QMRD,
    WS_LANCZOS, WS_EIGTMP, WS_EIGOUT, WS_COUNT
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
    int* sconv = nullptr;      // [w][ng] 0, or the iteration at which the shift converged
                               // (sticky: its recurrence is frozen from then on)
    double* sres = nullptr;    // [w][ng] residual estimate ||r_sigma|| / ||b|| (at freeze)
    // per-iteration shifted COCG scalars for the blocked accumulation:
    // rec[((c*chunk + k%chunk)*3 + t)*ng + g], t = 0: 1/pi_k, 1: alpha^sigma_k, 2: beta^sigma_k
    double2* rec = nullptr;
    int chunk = 0;
    // simplified QMR smoothing (null for COCG): [w][8] = tau, theta^2 of the last
    // step, and the pending iterate step d = a d + b p (a, b.re, b.im)
    double* qmr = nullptr;
    int* running = nullptr;    // [1] count of running columns after a step
    double tol = 1e-10;
};

int part_blocks(int64_t n);
template <typename R>
void launch_p_update(const cplx_t<R>* r, cplx_t<R>* p, const IterState& st, int64_t N, hipStream_t s);
template <typename R>
void launch_dot_pq(const cplx_t<R>* p, const cplx_t<R>* q, double2* part, const IterState& st,
                   int64_t N, hipStream_t s);
void launch_reduce_alpha(const double2* part, int nblk, IterState st, hipStream_t s,
                         const double2* kbc = nullptr, const double* e_kb = nullptr,
                         int n_proj = 0);
// fused p-update + operator apply + p^T q partials (stencil.hip); the projector
// gather/scatter follow it.  ev0/ev1 (nullable) bracket the stencil kernel.
// live_vectors: block vectors the caller's iteration touches (r, the p pair
// and q in the multi-shift core; the iterate as well in the per-energy core),
// which decides whether the dead streams take the non-temporal hint.
template <typename R>
void launch_cocg_apply(const negf_op* op, const cplx_t<R>* r, const cplx_t<R>* pin,
                       cplx_t<R>* pout, cplx_t<R>* q, int w, const double* shift, const int* skip,
                       const int* kit, const double2* beta, double2* part, double2* d_kbc,
                       hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, bool kb_scatter = true,
                       int w_geom = 0, int live_vectors = 4);
// opts in the fused stencil kernels this op's grid can launch to more than
// 64 KB of LDS (once per kernel and device; called when the op is built)
void prepare_stencil_kernels(const negf_op* op);
// partials per column of the fused kernel when its z-chunking is chosen for w
// running columns (more chunks per column for fewer columns)
int fused_partials(const negf_op* op, int w);
// multi-shift alpha + projector term + r update + kept-row store in one launch
// (krylov.hip); ring == null skips the row store
// kept rows: n_rows in all (the ring's row stride), [row0, row0 + n_rows -
// n_rows1) followed by [row1, row1 + n_rows1)
template <typename R>
void launch_update_ms(cplx_t<R>* r, const cplx_t<R>* q, int64_t N, const IterState& st,
                      const double2* part_f, int nblk_f, const negf_op* op, const double2* kbc,
                      double2* ring, int ring_len, int64_t row0, int n_rows, double2* part_rr,
                      double* part_nn, hipStream_t s, int64_t row1 = 0, int n_rows1 = 0);
// r -= alpha q; x += alpha p (COCG), or with st.qmr the pending smoothed step
// d = a d + b p, x += d, where p is then the previous direction
template <typename R>
void launch_r_update(cplx_t<R>* r, const cplx_t<R>* q, cplx_t<R>* p_or_null, cplx_t<R>* x_or_null,
                     double2* part_rr, double* part_nn, const IterState& st, int64_t N,
                     hipStream_t s, cplx_t<R>* d_qmr = nullptr);
// the last pending QMR step of every column: d = a d + b p_K, x += d, with
// p_K in p_even (K even) or p_odd (K odd), K = k - 1
template <typename R>
void launch_qmr_flush(const cplx_t<R>* p_even, const cplx_t<R>* p_odd, cplx_t<R>* d_qmr,
                      cplx_t<R>* x, int64_t N, const IterState& st, const int* skip,
                      hipStream_t s);
void launch_reduce_beta_multishift(const double2* part_rr, const double* part_nn, int nblk,
                                   IterState st, hipStream_t s);
void launch_reduce_beta_single(const double2* part_rr, const double* part_nn, int nblk,
                               IterState st, double inner_tol, hipStream_t s);
template <typename R>
void launch_store_rows(const cplx_t<R>* r, int64_t N, int w, const int* rows, int64_t row0,
                       int n_rows, double2* ring, int ring_len, const IterState& st,
                       int slot_offset, hipStream_t s, const int* only = nullptr,
                       int64_t row1 = 0, int n_rows1 = 0);
// blocked multi-shift accumulation (shift.hip)
// kstart[c]: the column's iteration count at the start of the chunk; the
// coefficient kernel writes each column's chunk length to clen for the GEMM
// active[c][g]: energy g moved in the chunk; act_list/act_n: those energies of
// each column in order (the matrix-core GEMM tiles them)
void launch_chunk_coef(const IterState& st, const int* kstart, int* clen, double2* cx,
                       double2* cp, double2* xi_a, double2* carry, int* active, int* act_list,
                       int* act_n, hipStream_t s);
void launch_gemm_xp(const double2* ring, int ring_len, int w, int n_rows, const int* kstart,
                    const int* clen,
                    const IterState& st, const double2* cx, const double2* cp,
                    const double2* xi_a, const int* active, const int* act_list,
                    const int* act_n, double2* X, double2* P, hipStream_t s);
void launch_t_from_x(const double2* X, int n_rows, int w, int ng, const double* row_w,
                     const double* col_w, const int* only, double* t, hipStream_t s);
// optical-theorem error per (column, energy) of iterates X[c][g][stride]:
// |sum_i row_w[i] |x_i|^2 + Im x[jloc[c]]| / |Im x[jloc[c]]| over i < n_keep
void launch_optical(const double2* X, int64_t stride, int n_keep, int w, int ng,
                    const double* row_w, const int* jloc, const int* only, double* out,
                    hipStream_t s);
void launch_copy_out(const double2* X, int n_rows, int w, int ng, double2* out, int64_t col_stride,
                     int64_t shift_stride, hipStream_t s);
