// C ABI of libnegf: operator construction, the two solver cores and the
// transmission reduction.  Host orchestration only; every step of the hot
// path runs in the kernels of stencil.hip, krylov.hip and shift.hip.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <chrono>
#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <string>
#include <vector>

#include "negf_internal.h"

// launchers defined in krylov.hip (kept out of the shared header because only
// this file calls them)
// only (nullable): columns to touch; the others are left as they are
template <typename R>
void launch_init_unit(cplx_t<R>* r, double2* b64, int64_t N, int w, const int* cols, hipStream_t s,
                      const int* only = nullptr);
template <typename R>
void launch_norms(const cplx_t<R>* v, int64_t N, int w, const int* skip, double2* part_rr,
                  double* part_nn, hipStream_t s);
void launch_reduce_init(const double2* part_rr, const double* part_nn, int nblk, IterState st,
                        const int* skip, hipStream_t s, const int* only = nullptr);
void launch_residual(const double2* b, const double2* q, double2* r, int64_t N, int w,
                     const int* skip, double* part, hipStream_t s);
void launch_reduce_residual(const double* part, int nblk, int w, int* odone, const double* bnorm64,
                            double* nu, double tol, double* resid_out, hipStream_t s);
template <typename R>
void launch_scale_convert(const double2* r64, cplx_t<R>* rin, cplx_t<R>* d, int64_t N, int w,
                          const int* skip, const double* nu, hipStream_t s);
template <typename R>
void launch_accumulate(double2* x64, const cplx_t<R>* d, int64_t N, int w, const int* skip,
                       const double* nu, hipStream_t s);
void launch_weighted_norm(const double2* x64, int64_t N, int w, int64_t row0, int n_rows,
                          const double* row_w, const double* col_w, double* t, hipStream_t s);

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

negf_status hip_fail(hipError_t e, const char* what, int line) {
    set_error("HIP error %d (%s) in %s at line %d", (int)e, hipGetErrorString(e), what, line);
    return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? NEGF_E_OUT_OF_MEMORY
                                                                        : NEGF_E_DEVICE;
}


// Test hook: NEGF_TEST_FAIL_ALLOC=k makes the k-th workspace allocation of the
// process fail (exercises the out-of-memory path without exhausting HBM).
static std::atomic<long> g_alloc_count{0};

// Device allocation and release, and the capture and instantiation of the
// chunk graphs, take this lock.  Host threads of the junction batch each
// drive their own stream; hipFree synchronises the device and hipMalloc may
// too, so neither may run while another thread has a stream in capture or
// a graph half-instantiated.
static std::mutex g_device_mu;

static negf_status dev_alloc(void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    const long n_alloc = ++g_alloc_count;
    if (const char* env = getenv("NEGF_TEST_FAIL_ALLOC")) {
        if (atol(env) == n_alloc) {
            set_error("allocation of %zu bytes failed (test hook)", bytes);
            return NEGF_E_OUT_OF_MEMORY;
        }
    }
    std::lock_guard<std::mutex> lock(g_device_mu);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        set_error("device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
        return NEGF_E_OUT_OF_MEMORY;
    }
    return NEGF_OK;
}

static void dev_free(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lock(g_device_mu);
    (void)hipFree(p);
}

negf_status ws_get(negf_op* op, int slot, size_t bytes, void** out) {
    Buffer& b = op->bufs[slot];
    if (b.bytes < bytes) {
        if (b.ptr) dev_free(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
        CHK(dev_alloc(&b.ptr, bytes));
        b.bytes = bytes;
    }
    *out = b.ptr;
    return NEGF_OK;
}

template <typename T>
static negf_status ws(negf_op* op, int slot, size_t count, T** out) {
    void* p = nullptr;
    CHK(ws_get(op, slot, count * sizeof(T), &p));
    *out = static_cast<T*>(p);
    return NEGF_OK;
}

static bool is_device_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice;
}

static hipStream_t pick_stream(negf_op* op, const negf_opts* o) {
    return (o && o->stream) ? (hipStream_t)o->stream : op->own_stream;
}

// ---------------------------------------------------------------------------
// operator construction
// ---------------------------------------------------------------------------
static void fd_weights(int R, double* c) {
    // order-2R central second derivative: c_m = 2(-1)^(m+1) (R!)^2 / (m^2 (R-m)! (R+m)!),
    // c_0 = -2 sum_m c_m
    double fact[16];
    fact[0] = 1.0;
    for (int i = 1; i < 16; ++i) fact[i] = fact[i - 1] * i;
    double s = 0.0;
    for (int m = 1; m <= R; ++m) {
        c[m] = 2.0 * ((m % 2) ? 1.0 : -1.0) * fact[R] * fact[R] / ((double)m * m * fact[R - m] * fact[R + m]);
        s += c[m];
    }
    c[0] = -2.0 * s;
}

static negf_status plane_run(const double* cap, int nz, bool leading, int* z0, int* z1) {
    // supported planes must be one contiguous run touching the wall
    int first = -1, last = -1;
    for (int z = 0; z < nz; ++z) {
        if (!(cap[z] >= 0.0) || !std::isfinite(cap[z])) {
            set_error("CAP value at plane %d is negative or not finite", z);
            return NEGF_E_INVALID_ARG;
        }
        if (cap[z] > 0.0) {
            if (first < 0) first = z;
            last = z;
        }
    }
    if (first < 0) {
        set_error("a CAP profile is identically zero");
        return NEGF_E_INVALID_ARG;
    }
    for (int z = first; z <= last; ++z)
        if (!(cap[z] > 0.0)) {
            set_error("CAP support is not a contiguous run of planes");
            return NEGF_E_INVALID_ARG;
        }
    if (leading && first != 0) {
        set_error("left CAP must start at plane 0");
        return NEGF_E_INVALID_ARG;
    }
    if (!leading && last != nz - 1) {
        set_error("right CAP must end at plane nz-1");
        return NEGF_E_INVALID_ARG;
    }
    *z0 = first;
    *z1 = last + 1;
    return NEGF_OK;
}

static void free_op(negf_op* op) {
    if (!op) return;
    if (op->device < 0) {  // never reached the device
        delete op;
        return;
    }
    (void)hipSetDevice(op->device);
    if (op->own_stream) (void)hipStreamSynchronize(op->own_stream);
    if (op->side_stream) (void)hipStreamSynchronize(op->side_stream);
    void* ptrs[] = {op->d_v, op->d_wz, op->d_wl, op->d_wr, op->kb.off, op->kb.idx, op->kb.val,
                    op->kb.valf, op->kb.e, op->kb.pts, op->kb.pt_off, op->kb.pt_proj, op->kb.pt_val, op->kb.slot};
    for (void* p : ptrs) dev_free(p);
    for (auto& b : op->bufs) dev_free(b.ptr);
    if (op->own_stream) (void)hipStreamDestroy(op->own_stream);
    if (op->side_stream) (void)hipStreamDestroy(op->side_stream);
    delete op;
}

template <typename T>
static negf_status upload(T** dst, const T* src, size_t n) {
    void* p = nullptr;
    CHK(dev_alloc(&p, n * sizeof(T)));
    *dst = static_cast<T*>(p);
    if (n) HIPCHK(hipMemcpy(p, src, n * sizeof(T), hipMemcpyHostToDevice));
    return NEGF_OK;
}

static negf_status build_impl(const negf_grid* g, int32_t R, const double* v, const negf_kb* kb,
                              const double* capl, const double* capr, negf_op* op) {
    if (!g || !v || !capl || !capr) {
        set_error("null argument");
        return NEGF_E_INVALID_ARG;
    }
    if (g->nx < 1 || g->ny < 1 || g->nz < 1 || !(g->h > 0.0) || !std::isfinite(g->h)) {
        set_error("invalid grid (%d x %d x %d, h=%g)", g->nx, g->ny, g->nz, g->h);
        return NEGF_E_INVALID_ARG;
    }
    if (R < 1 || R > 6) {
        set_error("stencil radius %d outside 1..6", R);
        return NEGF_E_INVALID_ARG;
    }
    // the fused stencil step gives each point of an x-row a thread and stages
    // at least one row, with its radius-R halo, in a double-buffered FP64 LDS
    // tile of at most 160 KB
    const int max_nx = std::min(1024, 163840 / (32 * (2 * R + 1)) - 2 * R);
    if (g->nx > max_nx) {
        set_error("nx = %d exceeds %d, the widest x-row the stencil tile holds at radius %d",
                  g->nx, max_nx, R);
        return NEGF_E_INVALID_ARG;
    }
    {
        // the tile itself: a whole plane of at most 1024 points, else
        // 1024 / nx rows (256 / nx for planes of at most 256 points)
        const int64_t pts = (int64_t)g->nx * g->ny;
        const int64_t rows = pts <= 1024 ? g->ny : std::min<int64_t>(g->ny, 1024 / g->nx);
        const int64_t lds = (rows + 2 * R) * 2 * (g->nx + 2 * R) * 16;
        if (lds > 163840) {
            set_error("a %d x %d plane needs a %lld-byte stencil tile in LDS (at most 163840)",
                      g->nx, g->ny, (long long)lds);
            return NEGF_E_INVALID_ARG;
        }
    }
    const int64_t N = (int64_t)g->nx * g->ny * g->nz;
    if (N > (int64_t)1 << 31) {
        set_error("grid too large");
        return NEGF_E_INVALID_ARG;
    }
    for (int64_t i = 0; i < N; ++i)
        if (!std::isfinite(v[i])) {
            set_error("v_local[%lld] is not finite", (long long)i);
            return NEGF_E_INVALID_ARG;
        }
    op->nx = g->nx; op->ny = g->ny; op->nz = g->nz; op->h = g->h; op->R = R; op->N = N;
    CHK(plane_run(capl, g->nz, true, &op->zl0, &op->zl1));
    CHK(plane_run(capr, g->nz, false, &op->zr0, &op->zr1));
    if (op->zl1 > op->zr0) {
        set_error("left and right CAP supports overlap");
        return NEGF_E_INVALID_ARG;
    }
    if (op->zl1 - op->zl0 < R || op->zr1 - op->zr0 < R) {
        set_error("each CAP must cover at least R=%d planes", R);
        return NEGF_E_INVALID_ARG;
    }
    op->cap_l.assign(capl, capl + g->nz);
    op->cap_r.assign(capr, capr + g->nz);
    double c[7] = {0};
    fd_weights(R, c);
    const double inv2h2 = 1.0 / (2.0 * g->h * g->h);
    op->coef.a[0] = 3.0 * c[0] * inv2h2;
    for (int m = 1; m <= 6; ++m) op->coef.a[m] = (m <= R) ? c[m] * inv2h2 : 0.0;

    // projectors
    std::vector<int> pts, pt_off, pt_proj;
    std::vector<double> pt_val;
    if (kb && kb->n_proj > 0) {
        if (!kb->offsets || !kb->idx || !kb->val || !kb->e_kb || kb->offsets[0] != 0) {
            set_error("invalid projector arrays");
            return NEGF_E_INVALID_ARG;
        }
        const int P = kb->n_proj;
        for (int p = 0; p < P; ++p) {
            if (kb->offsets[p + 1] < kb->offsets[p]) {
                set_error("projector offsets decrease at %d", p);
                return NEGF_E_INVALID_ARG;
            }
            if (!std::isfinite(kb->e_kb[p])) {
                set_error("projector energy %d not finite", p);
                return NEGF_E_INVALID_ARG;
            }
        }
        const int64_t nnz = kb->offsets[P];
        const int64_t plane = (int64_t)g->nx * g->ny;
        std::map<int, std::vector<std::pair<int, double>>> by_pt;
        int max_sup = 0;
        for (int p = 0; p < P; ++p) {
            max_sup = std::max<int>(max_sup, (int)(kb->offsets[p + 1] - kb->offsets[p]));
            for (int64_t k = kb->offsets[p]; k < kb->offsets[p + 1]; ++k) {
                const int i = kb->idx[k];
                if (i < 0 || i >= N || !std::isfinite(kb->val[k])) {
                    set_error("projector entry %lld invalid", (long long)k);
                    return NEGF_E_INVALID_ARG;
                }
                const int z = (int)(i / plane);
                if (capl[z] > 0.0 || capr[z] > 0.0) {
                    set_error("projector %d reaches CAP plane %d", p, z);
                    return NEGF_E_INVALID_ARG;
                }
                by_pt[i].push_back({p, kb->e_kb[p] * kb->val[k]});
            }
        }
        pt_off.push_back(0);
        for (auto& kv : by_pt) {
            pts.push_back(kv.first);
            for (auto& e : kv.second) {
                pt_proj.push_back(e.first);
                pt_val.push_back(e.second);
            }
            pt_off.push_back((int)pt_proj.size());
        }
        op->kb.n_proj = P;
        op->kb.nnz = nnz;
        op->kb.max_support = max_sup;
        op->kb.n_pts = (int)pts.size();
    }
    // every argument is valid: device work starts here
    if (hipGetDevice(&op->device) != hipSuccess) {
        (void)hipGetLastError();
        set_error("no HIP device");
        return NEGF_E_DEVICE;
    }
    if (op->kb.n_proj > 0) {
        const int P = kb->n_proj;
        const int64_t nnz = kb->offsets[P];
        CHK(upload(&op->kb.off, kb->offsets, (size_t)P + 1));
        CHK(upload(&op->kb.idx, kb->idx, (size_t)nnz));
        CHK(upload(&op->kb.val, kb->val, (size_t)nnz));
        std::vector<float> vf(kb->val, kb->val + nnz);
        CHK(upload(&op->kb.valf, vf.data(), vf.size()));
        CHK(upload(&op->kb.e, kb->e_kb, (size_t)P));
        CHK(upload(&op->kb.pts, pts.data(), pts.size()));
        CHK(upload(&op->kb.pt_off, pt_off.data(), pt_off.size()));
        CHK(upload(&op->kb.pt_proj, pt_proj.data(), pt_proj.size()));
        CHK(upload(&op->kb.pt_val, pt_val.data(), pt_val.size()));
        std::vector<int> slot((size_t)N, -1);
        for (size_t t = 0; t < pts.size(); ++t) slot[pts[t]] = (int)t;
        CHK(upload(&op->kb.slot, slot.data(), slot.size()));
    }
    CHK(upload(&op->d_v, v, (size_t)N));
    std::vector<double> wz(g->nz);
    for (int z = 0; z < g->nz; ++z) wz[z] = capl[z] + capr[z];
    CHK(upload(&op->d_wz, wz.data(), wz.size()));
    CHK(upload(&op->d_wl, capl, (size_t)g->nz));
    CHK(upload(&op->d_wr, capr, (size_t)g->nz));
    HIPCHK(hipStreamCreateWithFlags(&op->own_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&op->side_stream, hipStreamNonBlocking));
    op->bufs.resize(WS_COUNT);
    // the large-LDS opt-in of the stencil kernels this grid can take happens
    // here, never inside a stream capture
    prepare_stencil_kernels(op);
    return NEGF_OK;
}

extern "C" negf_status negf_build_operator(const negf_grid* g, int32_t stencil_radius,
                                           const double* v_local, const negf_kb* kb,
                                           const double* cap_left_z, const double* cap_right_z,
                                           negf_op** out) {
    g_last_error.clear();
    if (!out) {
        set_error("null output pointer");
        return NEGF_E_INVALID_ARG;
    }
    *out = nullptr;
    negf_op* op = new negf_op();
    op->device = -1;
    negf_status s = build_impl(g, stencil_radius, v_local, kb, cap_left_z, cap_right_z, op);
    if (s != NEGF_OK) {
        free_op(op);
        return s;
    }
    *out = op;
    return NEGF_OK;
}

extern "C" void negf_destroy(negf_op* op) { free_op(op); }

extern "C" const char* negf_last_error(void) { return g_last_error.c_str(); }

extern "C" const char* negf_version(void) { return "libnegf 0.1 (gfx950)"; }

// ---------------------------------------------------------------------------
// operator apply (standalone entry point)
// ---------------------------------------------------------------------------
__global__ void k_d2f(const double2* a, float2* b, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = make_float2((float)a[i].x, (float)a[i].y);
}
__global__ void k_f2d(const float2* a, double2* b, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = make_double2((double)a[i].x, (double)a[i].y);
}

extern "C" negf_status negf_apply_operator(negf_op* op, int32_t precision, int32_t n_vec,
                                           const double* shifts, const negf_c64* x, negf_c64* y) {
    g_last_error.clear();
    (void)hipGetLastError();  // a stale error of an earlier call must not fail this one
    if (!op || !shifts || !x || !y || n_vec < 1 || (precision != NEGF_FP64 && precision != NEGF_MIXED)) {
        set_error("invalid argument to negf_apply_operator");
        return NEGF_E_INVALID_ARG;
    }
    HIPCHK(hipSetDevice(op->device));
    hipStream_t s = op->own_stream;
    const int64_t N = op->N, tot = N * n_vec;
    const bool dx = is_device_ptr(x), dy = is_device_ptr(y);
    double2 *bx = nullptr, *by = nullptr, *kbc = nullptr;
    double* sh = nullptr;
    CHK(ws(op, WS_X64, (size_t)tot, &bx));
    CHK(ws(op, WS_Q64, (size_t)tot, &by));
    CHK(ws(op, WS_SHIFT, (size_t)n_vec, &sh));
    CHK(ws(op, WS_KBC, (size_t)n_vec * std::max(1, op->kb.n_proj), &kbc));
    HIPCHK(hipMemcpyAsync(bx, x, tot * sizeof(double2), dx ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(sh, shifts, n_vec * sizeof(double), hipMemcpyHostToDevice, s));
    if (precision == NEGF_FP64) {
        launch_apply<double>(op, bx, by, n_vec, sh, nullptr, kbc, s);
    } else {
        float2 *fx = nullptr, *fy = nullptr;
        CHK(ws(op, WS_R, (size_t)tot, &fx));
        CHK(ws(op, WS_Q, (size_t)tot, &fy));
        const unsigned nb = (unsigned)((tot + 255) / 256);
        hipLaunchKernelGGL(k_d2f, dim3(nb), dim3(256), 0, s, bx, fx, tot);
        launch_apply<float>(op, fx, fy, n_vec, sh, nullptr, kbc, s);
        hipLaunchKernelGGL(k_f2d, dim3(nb), dim3(256), 0, s, fy, by, tot);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(y, by, tot * sizeof(double2), dy ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return NEGF_OK;
}

// ---------------------------------------------------------------------------
// shared pieces of the solver drivers
// ---------------------------------------------------------------------------
struct Defaults {
    int precision, core, solver, direction, max_iter, block_width, shift_group, max_refine;
    int col_begin, col_count, recover;
    double tol;
};

static negf_status read_opts(const negf_opts* o, Defaults* d) {
    d->precision = o ? o->precision : NEGF_FP64;
    d->core = o ? o->core : NEGF_CORE_AUTO;
    d->solver = o ? o->solver : NEGF_SOLVER_COCG;
    d->direction = o ? o->direction : NEGF_DIR_RL;
    d->tol = (o && o->tol > 0) ? o->tol : 1e-10;
    d->max_iter = (o && o->max_iter > 0) ? o->max_iter : 100000;
    d->block_width = (o && o->block_width > 0) ? o->block_width : 0;
    d->shift_group = (o && o->shift_group > 0) ? o->shift_group : 0;
    d->max_refine = (o && o->max_refine > 0) ? o->max_refine : 8;
    d->col_begin = o ? o->col_begin : 0;
    d->col_count = o ? o->col_count : 0;
    d->recover = o ? o->recover : NEGF_RECOVER_OFF;
    if (d->recover != NEGF_RECOVER_OFF && d->recover != NEGF_RECOVER_RESTART) {
        set_error("unknown recover mode %d", d->recover);
        return NEGF_E_INVALID_ARG;
    }
    if (d->col_begin < 0 || d->col_count < 0) {
        set_error("negative column range");
        return NEGF_E_INVALID_ARG;
    }
    if (d->precision != NEGF_FP64 && d->precision != NEGF_MIXED) {
        set_error("unknown precision %d", d->precision);
        return NEGF_E_INVALID_ARG;
    }
    if (d->core < NEGF_CORE_AUTO || d->core > NEGF_CORE_MULTISHIFT) {
        set_error("unknown core %d", d->core);
        return NEGF_E_INVALID_ARG;
    }
    if (d->solver != NEGF_SOLVER_COCG && d->solver != NEGF_SOLVER_QMR) {
        set_error("unknown solver %d", d->solver);
        return NEGF_E_INVALID_ARG;
    }
    if (d->solver == NEGF_SOLVER_QMR && d->core == NEGF_CORE_MULTISHIFT) {
        set_error("the QMR solver runs in the per-energy core only");
        return NEGF_E_INVALID_ARG;
    }
    if (d->direction != NEGF_DIR_RL && d->direction != NEGF_DIR_LR) {
        set_error("unknown direction %d", d->direction);
        return NEGF_E_INVALID_ARG;
    }
    if (!(d->tol < 1.0) || !std::isfinite(d->tol)) {
        set_error("tol must be in (0, 1)");
        return NEGF_E_INVALID_ARG;
    }
    return NEGF_OK;
}

static negf_status make_state(negf_op* op, int w, int ng, int max_iter, double tol, bool hist,
                              IterState* st, int chunk = 0, bool qmr = false) {
    // one allocation carved into the state arrays
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) & ~(size_t)255; return o; };
    const size_t o_k = take(w * sizeof(int)), o_done = take(w * sizeof(int));
    const size_t o_rho = take(w * sizeof(double2)), o_alpha = take(w * sizeof(double2));
    const size_t o_beta = take(w * sizeof(double2)), o_bn = take(w * sizeof(double));
    const size_t o_rn = take(w * sizeof(double));
    const size_t o_ah = hist ? take((size_t)w * max_iter * sizeof(double2)) : 0;
    const size_t o_bh = hist ? take((size_t)w * max_iter * sizeof(double2)) : 0;
    const size_t o_sh = hist ? take((size_t)w * (max_iter + 1) * sizeof(double)) : 0;
    const size_t o_pi = ng ? take((size_t)w * ng * sizeof(double2)) : 0;
    const size_t o_pp = ng ? take((size_t)w * ng * sizeof(double2)) : 0;
    const size_t o_dl = ng ? take((size_t)w * ng * sizeof(double)) : 0;
    const size_t o_sc = ng ? take((size_t)w * ng * sizeof(int)) : 0;
    const size_t o_sr = ng ? take((size_t)w * ng * sizeof(double)) : 0;
    const size_t o_rc = (ng && chunk) ? take((size_t)w * chunk * 3 * ng * sizeof(double2)) : 0;
    const size_t o_qm = qmr ? take((size_t)w * 8 * sizeof(double)) : 0;
    unsigned char* base = nullptr;
    CHK(ws(op, WS_STATE, off, &base));
    st->w = w;
    st->ng = ng;
    st->max_iter = max_iter;
    st->tol = tol;
    st->k = (int*)(base + o_k);
    st->done = (int*)(base + o_done);
    st->rho = (double2*)(base + o_rho);
    st->alpha = (double2*)(base + o_alpha);
    st->beta = (double2*)(base + o_beta);
    st->bnorm = (double*)(base + o_bn);
    st->rnorm = (double*)(base + o_rn);
    st->a_hist = hist ? (double2*)(base + o_ah) : nullptr;
    st->b_hist = hist ? (double2*)(base + o_bh) : nullptr;
    st->s_hist = hist ? (double*)(base + o_sh) : nullptr;
    st->pih = ng ? (double2*)(base + o_pi) : nullptr;
    st->pih_prev = ng ? (double2*)(base + o_pp) : nullptr;
    st->deltas = ng ? (double*)(base + o_dl) : nullptr;
    st->sconv = ng ? (int*)(base + o_sc) : nullptr;
    st->sres = ng ? (double*)(base + o_sr) : nullptr;
    st->rec = (ng && chunk) ? (double2*)(base + o_rc) : nullptr;
    st->chunk = chunk;
    st->qmr = qmr ? (double*)(base + o_qm) : nullptr;
    return NEGF_OK;
}

// HIP-event timing of the fused stencil launches (bench instrumentation):
// pairs are recorded around each launch and summed at the drivers' sync points.
struct MatvecTimer {
    bool on = false;
    bool active = true;  // whether the launches being issued are timed
    int period = 1;      // multi-shift core: time every period-th chunk
    std::vector<hipEvent_t> ev;
    int used = 0;
    double seconds = 0.0;
    int64_t launches = 0;
    double bytes = 0.0;
    static constexpr int kPool = 256;
    negf_status init(int every) {
        on = every > 0;
        period = std::max(1, every);
        if (!on) return NEGF_OK;
        ev.resize(2 * kPool);
        for (auto& e : ev) HIPCHK(hipEventCreate(&e));
        return NEGF_OK;
    }
    // events for the next launch (null when off); flushes a full pool first
    negf_status next(hipEvent_t* a, hipEvent_t* b) {
        *a = *b = nullptr;
        if (!on || !active) return NEGF_OK;
        if (used == kPool) CHK(flush());
        *a = ev[2 * used];
        *b = ev[2 * used + 1];
        ++used;
        return NEGF_OK;
    }
    negf_status flush() {
        for (int i = 0; i < used; ++i) {
            HIPCHK(hipEventSynchronize(ev[2 * i + 1]));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
            seconds += 1e-3 * ms;
            ++launches;
        }
        used = 0;
        return NEGF_OK;
    }
    ~MatvecTimer() {
        for (auto& e : ev) (void)hipEventDestroy(e);
    }
};

// A chunk of solver iterations captured once and replayed: seven small
// launches per iteration otherwise cost tens of microseconds per iteration.
// Every kernel reads its iteration state (k, done, alpha, beta, ...) from the
// device, and chunks start at even iterations, so one capture serves all
// full chunks of a block.  NEGF_NO_GRAPH=1 launches eagerly instead.
struct ChunkGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t launched_on = nullptr;  // the last replay's stream
    int timer_pairs = 0;
    bool failed = false;
    ~ChunkGraph() {
        // an error return can leave a replay in flight
        if (launched_on) (void)hipStreamSynchronize(launched_on);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

// Synchronises the given streams when it goes out of scope: declared after
// the graphs and events of a solver driver, it runs first on every return
// path, so that nothing those objects own is released while work that uses
// it may still be queued.
struct DrainGuard {
    hipStream_t a, b;
    ~DrainGuard() {
        if (a) (void)hipStreamSynchronize(a);
        if (b) (void)hipStreamSynchronize(b);
    }
};

// NEGF_NO_FUSED_UPDATE=1 runs the multi-shift iteration tail as separate kernels
static bool fused_update_disabled() {
    const char* e = std::getenv("NEGF_NO_FUSED_UPDATE");
    return e && e[0] == '1';
}

// NEGF_NO_COLUMN_STREAM=1 runs each block of source columns on its own
static bool column_stream_disabled() {
    const char* e = std::getenv("NEGF_NO_COLUMN_STREAM");
    return e && e[0] == '1';
}

static bool graphs_enabled() {
    const char* e = getenv("NEGF_NO_GRAPH");
    return !(e && atoi(e) != 0);
}

// Runs `issue` (which enqueues one full chunk on s) through the graph; falls
// back to eager launches when capture is unavailable.
template <typename F>
static negf_status run_chunk(ChunkGraph& cg, bool use_graph, hipStream_t s, MatvecTimer* tm,
                             F issue) {
    // per-kernel HIP events cannot be timed inside a graph: timed runs go eagerly
    if (tm->on && tm->active) use_graph = false;
    if (use_graph && !cg.failed && !cg.exec) {
        CHK(tm->flush());
        std::lock_guard<std::mutex> lock(g_device_mu);
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            const negf_status st = issue();
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(s, &g);
            if (st != NEGF_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (e == hipSuccess && g &&
                hipGraphInstantiate(&cg.exec, g, nullptr, nullptr, 0) == hipSuccess) {
                cg.graph = g;
                cg.timer_pairs = tm->used;
                tm->used = 0;  // recorded into the graph, not yet executed
            } else {
                if (g) (void)hipGraphDestroy(g);
                cg.exec = nullptr;
                cg.failed = true;
                tm->used = 0;
                (void)hipGetLastError();
            }
        } else {
            cg.failed = true;
            (void)hipGetLastError();
        }
    }
    if (use_graph && cg.exec) {
        cg.launched_on = s;
        HIPCHK(hipGraphLaunch(cg.exec, s));
        tm->used = cg.timer_pairs;
        return NEGF_OK;
    }
    return issue();
}

// Output of one multi-shift block.
struct MSOut {
    double* h_tcol = nullptr;   // [n_src][ng] host (transmission mode)
    double2* d_out = nullptr;   // device destination of X (column mode, n_src == w)
    int64_t out_col_stride = 0, out_shift_stride = 0;
    int* h_iters = nullptr;     // [n_src]
    int* h_status = nullptr;    // [n_src] column status
    double* h_resid = nullptr;  // [n_src][ng] residual estimate per energy
    int* h_shift_iters = nullptr; // [n_src][ng] iteration at which each energy converged (0: not)
    // optical-theorem check (transmission mode): the kept rows go on past the
    // n_rows - n_rows1 rows at row0 with the n_rows1 rows of the source side's
    // absorbing region at row1; d_row_wo [n_rows] weights W on both ranges
    int64_t row1 = 0;
    int n_rows1 = 0;
    const double* d_row_wo = nullptr;
    double* h_optical = nullptr; // [n_src][ng] |sum W |g|^2 + Im g_jj| / |Im g_jj|
};

// iterations per blocked shift update (and per ring half).  X and P move once
// per chunk, so long chunks pay on large grids (256 ran 0.9 % faster than 128
// on the 32x32x192 wire, 384 was slower); streamed slots refill only at chunk
// boundaries, so small grids, whose columns converge in ~100 iterations, keep
// 128 (the 8x8x32 wire: 113k solves/s at 256, 122k at 128).
static int shift_chunk(const negf_op* op) { return op->N >= 131072 ? 256 : 128; }

// The multi-shift core (FP64) on a block of w column slots.
//   cols (host, n_src entries) unit right-hand sides, or d_rhs (device [w][N])
//   dense ones (then n_src == w); h_col_w (host, n_src) the T weights
//   rows kept per energy: contiguous [row0, row0+n_rows) when d_rows == null
// With n_src > w (unit right-hand sides, transmission mode) the slots stream
// through the queue of source columns: at a chunk boundary every slot whose
// column has finished hands over that column's results and restarts on the
// next queued column, so the block stays full until the queue runs dry and
// only the last columns leave slots idle.  Each column's arithmetic is the
// same as in a block of its own.
//
// The run is resumable: start() queues the set-up, issue_chunk() queues one
// chunk of iterations with its shift accumulation and the read-back of the
// column flags, and after_chunk() does the host bookkeeping once that chunk
// has finished (chunk_done() polls it without blocking).  One host thread
// can so keep the streams of many runs busy (the junction batch).
template <typename R>
class MultiShiftRun {
  public:
    MultiShiftRun(negf_op* op, const Defaults& d, int w, int n_src, const int* cols,
                  const double2* d_rhs, const double* energies, int ng, const int* d_rows,
                  int64_t row0, int n_rows, const double* d_row_w, const double* h_col_w,
                  const MSOut& out, int64_t* total_iters, hipStream_t s, MatvecTimer* tm)
        : op_(op), d_(d), w_(w), n_src_(n_src), cols_(cols), d_rhs_(d_rhs), energies_(energies),
          ng_(ng), d_rows_(d_rows), row0_(row0), n_rows_(n_rows), d_row_w_(d_row_w),
          h_col_w_(h_col_w), out_(out), total_iters_(total_iters), s_(s), tm_(tm) {}
    MultiShiftRun(const MultiShiftRun&) = delete;
    MultiShiftRun& operator=(const MultiShiftRun&) = delete;
    ~MultiShiftRun() {
        // queued work may still use the events, the graph and the pinned
        // flags: drain both streams first (the graph member is released after
        // this body)
        if (s_) (void)hipStreamSynchronize(s_);
        if (side_) (void)hipStreamSynchronize(side_);
        if (ev_coef_) (void)hipEventDestroy(ev_coef_);
        if (ev_gemm_) (void)hipEventDestroy(ev_gemm_);
        if (ev_chunk_) (void)hipEventDestroy(ev_chunk_);
        if (h_flags_) {
            std::lock_guard<std::mutex> lock(g_device_mu);
            (void)hipHostFree(h_flags_);
        }
    }

    negf_status start();
    negf_status issue_chunk();
    // true once the last issued chunk has finished (or its stream failed)
    bool chunk_done() const { return hipEventQuery(ev_chunk_) != hipErrorNotReady; }
    // host bookkeeping after a chunk; *busy = false once every column is done
    negf_status after_chunk(bool* busy);
    negf_status finish();

  private:
    negf_op* op_;
    Defaults d_;
    int w_, n_src_;
    const int* cols_;
    const double2* d_rhs_;
    const double* energies_;
    int ng_;
    const int* d_rows_;
    int64_t row0_;
    int n_rows_;
    const double* d_row_w_;
    const double* h_col_w_;
    MSOut out_;
    int64_t* total_iters_;
    hipStream_t s_;
    MatvecTimer* tm_;

    int64_t N_ = 0;
    int nblk_ = 0, ch_ = 0, ring_len_ = 0;
    // the seed's Krylov vectors in R; the ring, the shifted iterates and
    // every scalar are FP64.  Only R = double is instantiated: with FP32
    // seed vectors no energy of the 32x32x192 wire converged within 100,000
    // iterations (the shifted recurrences inherit the FP32 seed's drift)
    cplx_t<R> *r_ = nullptr, *p_ = nullptr, *p2_ = nullptr, *q_ = nullptr;
    double2 *part_ = nullptr;
    double2 *kbc_ = nullptr, *ring_ = nullptr, *X_ = nullptr, *P_ = nullptr, *part_f_ = nullptr;
    double *part_nn_ = nullptr, *shift_ = nullptr;
    int* d_cols_ = nullptr;
    double2 *cx_ = nullptr, *cp_ = nullptr, *xi_a_ = nullptr, *carry_ = nullptr;
    int *active_ = nullptr, *act_list_ = nullptr, *act_n_ = nullptr;
    int* kstart_buf_[2] = {nullptr, nullptr};
    int *clen_ = nullptr, *d_mask_ = nullptr, *d_notmask_ = nullptr;
    hipStream_t side_ = nullptr;
    hipEvent_t ev_coef_ = nullptr, ev_gemm_ = nullptr, ev_chunk_ = nullptr;
    bool gemm_pending_ = false;
    IterState st_;
    bool fused_update_ = false;
    double *tcol_ = nullptr, *col_w_ = nullptr, *d_opt_ = nullptr;
    int* d_jloc_ = nullptr;
    std::vector<int> h_jloc_;
    std::vector<double> h_opt_;
    int* h_flags_ = nullptr;  // pinned: done [w], then k [w]
    std::vector<int> slot_src_, h_colsel_, h_mask_, h_notmask_, h_kprev_, h_si_;
    std::vector<double> h_t_, h_res_, h_colw_;
    int next_src_ = 0;
    int launches_ = 0;
    int steps_ = 0;
    int running_ = 0;
    ChunkGraph cg_;
    bool use_graph_ = true;
};

template <typename R>
negf_status MultiShiftRun<R>::start() {
    negf_op* op = op_;
    const int w = w_, ng = ng_, n_rows = n_rows_;
    hipStream_t s = s_;
    N_ = op->N;
    const int64_t N = N_;
    nblk_ = part_blocks(N);
    // the stencil's z-chunking follows the number of running columns (finer
    // chunks keep the CUs busy when few columns remain); partials are sized for
    // the finest
    const int nblk_f_max = fused_partials(op, 1);
    // ring of 2c + 1 slots: while the GEMM of chunk j reads its c residuals,
    // chunk j + 1 stores the next c + 1 without touching them
    ch_ = shift_chunk(op);
    ring_len_ = 2 * ch_ + 1;
    if (n_src_ < w || (n_src_ > w && (!cols_ || out_.d_out))) {
        set_error("internal: column streaming needs unit right-hand sides in transmission mode");
        return NEGF_E_INVALID_ARG;
    }
    CHK(ws(op, WS_R, (size_t)w * N, &r_));
    CHK(ws(op, WS_P, (size_t)w * N, &p_));
    CHK(ws(op, WS_Q, (size_t)w * N, &q_));
    CHK(ws(op, WS_X, (size_t)w * N, &p2_));
    CHK(ws(op, WS_PART, (size_t)w * nblk_, &part_));
    CHK(ws(op, WS_PART2, (size_t)w * nblk_, &part_nn_));
    CHK(ws(op, WS_PART3, (size_t)w * nblk_f_max, &part_f_));
    CHK(ws(op, WS_KBC, (size_t)w * std::max(1, op->kb.n_proj), &kbc_));
    CHK(ws(op, WS_SHIFT, (size_t)w, &shift_));
    CHK(ws(op, WS_COLJ, (size_t)w, &d_cols_));
    CHK(ws_get(op, WS_SINK, (size_t)w * op->nx * op->ny * sizeof(double2), &op->d_sink));
    CHK(ws(op, WS_RING, (size_t)ring_len_ * w * n_rows, &ring_));
    CHK(ws(op, WS_XS, (size_t)w * ng * n_rows, &X_));
    CHK(ws(op, WS_PS, (size_t)w * ng * n_rows, &P_));
    // coefficients: CX, CP [w][ch][ng]; xi_a [w][ng][2]; carry [w][ng];
    // ints: active [w][ng], act_list [w][ng], act_n [w]
    const size_t n_cxp = (size_t)w * ch_ * ng;
    double2* coef = nullptr;
    CHK(ws(op, WS_COEF, 2 * n_cxp + 3 * (size_t)w * ng + ((size_t)w * ng + w + 1) / 2 + 1, &coef));
    cx_ = coef;
    cp_ = coef + n_cxp;
    xi_a_ = coef + 2 * n_cxp;
    carry_ = xi_a_ + 2 * (size_t)w * ng;
    active_ = (int*)(carry_ + (size_t)w * ng);
    act_list_ = active_ + (size_t)w * ng;
    act_n_ = act_list_ + (size_t)w * ng;
    // per slot: iteration count at the chunk start (two chunks' worth: the GEMM
    // of one chunk overlaps the next), chunk length, slot masks
    int* slots = nullptr;
    CHK(ws(op, WS_SLOTS, 5 * (size_t)w, &slots));
    kstart_buf_[0] = slots;
    kstart_buf_[1] = slots + w;
    clen_ = slots + 2 * w;
    d_mask_ = slots + 3 * w;
    d_notmask_ = slots + 4 * w;
    {
        std::lock_guard<std::mutex> lock(g_device_mu);
        HIPCHK(hipHostMalloc((void**)&h_flags_, 2 * (size_t)w * sizeof(int), hipHostMallocDefault));
    }
    // the GEMM of chunk j runs on the side stream while chunk j + 1 iterates;
    // ev_coef orders it after its coefficients, ev_gemm orders later users of
    // X, P and the coefficient buffers after it; ev_chunk marks the end of the
    // chunk's read-back of the column flags
    side_ = op->side_stream;
    HIPCHK(hipEventCreateWithFlags(&ev_coef_, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ev_gemm_, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ev_chunk_, hipEventDisableTiming));
    CHK(make_state(op, w, ng, d_.max_iter, d_.tol, true, &st_, ch_));
    // fused update (alpha, projector term, r, kept rows) needs contiguous kept rows
    fused_update_ = (d_rows_ == nullptr) && !fused_update_disabled();

    // seed: the highest energy of the group (usually the slowest system)
    double e_seed = energies_[0];
    for (int g = 0; g < ng; ++g) e_seed = std::max(e_seed, energies_[g]);
    std::vector<double> h_shift(w, e_seed), h_delta((size_t)w * ng);
    for (int c = 0; c < w; ++c)
        for (int g = 0; g < ng; ++g) h_delta[(size_t)c * ng + g] = energies_[g] - e_seed;
    HIPCHK(hipMemcpyAsync(shift_, h_shift.data(), w * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(st_.deltas, h_delta.data(), h_delta.size() * sizeof(double), hipMemcpyHostToDevice, s));

    // slot -> source column (-1: idle); the first w columns start together
    slot_src_.assign(w, 0);
    h_colsel_.assign(w, 0);
    h_mask_.assign(w, 0);
    h_notmask_.assign(w, 0);
    for (int c = 0; c < w; ++c) slot_src_[c] = c;
    next_src_ = w;
    if (cols_) {
        for (int c = 0; c < w; ++c) h_colsel_[c] = cols_[c];
        HIPCHK(hipMemcpyAsync(d_cols_, h_colsel_.data(), w * sizeof(int), hipMemcpyHostToDevice, s));
        launch_init_unit<R>(r_, nullptr, N, w, d_cols_, s);
    } else {
        HIPCHK(hipMemcpyAsync(r_, d_rhs_, (size_t)w * N * sizeof(double2), hipMemcpyDeviceToDevice, s));
    }
    HIPCHK(hipMemsetAsync(X_, 0, (size_t)w * ng * n_rows * sizeof(double2), s));
    HIPCHK(hipMemsetAsync(P_, 0, (size_t)w * ng * n_rows * sizeof(double2), s));
    HIPCHK(hipMemsetAsync(carry_, 0, (size_t)w * ng * sizeof(double2), s));
    launch_norms<R>(r_, N, w, nullptr, part_, part_nn_, s);
    launch_reduce_init(part_, part_nn_, nblk_, st_, nullptr, s);
    launch_store_rows<R>(r_, N, w, d_rows_, row0_, n_rows, ring_, ring_len_, st_, 0, s,
                              nullptr, out_.row1, out_.n_rows1);
    HIPCHK(hipGetLastError());

    // per-slot readbacks and the T scratch of finishing slots
    if (out_.h_tcol || out_.h_optical) {
        // t [w][ng], column weights [w], optical errors [w][ng], source rows [w]
        CHK(ws(op, WS_TCOL, 2 * (size_t)w * ng + 2 * (size_t)w, &tcol_));
        col_w_ = tcol_ + (size_t)w * ng;
        d_opt_ = col_w_ + w;
        d_jloc_ = reinterpret_cast<int*>(d_opt_ + (size_t)w * ng);
        h_jloc_.assign(w, 0);
    }
    if (out_.h_optical && (!cols_ || out_.n_rows1 < 1 || !out_.d_row_wo)) {
        set_error("internal: the optical check needs unit sources and their own absorbing rows");
        return NEGF_E_INVALID_ARG;
    }
    h_kprev_.assign(w, 0);
    h_colw_.assign(w, 0.0);
    launches_ = 0;
    use_graph_ = graphs_enabled();
    running_ = w;  // columns still iterating at the chunk start
    return NEGF_OK;
}

template <typename R>
negf_status MultiShiftRun<R>::issue_chunk() {
    negf_op* op = op_;
    const int w = w_;
    const int64_t N = N_;
    hipStream_t s = s_;
    const int ch = ch_;
    MatvecTimer* tm = tm_;
    // a streaming block runs whole chunks (each column stops at its own
    // max_iter); a single block stops at max_iter
    steps_ = (n_src_ > w) ? ch : std::min(ch, d_.max_iter - launches_);
    const int steps = steps_;
    // the z-chunking for the running columns; the graph holds the full-width
    // shape, narrower chunks run eagerly
    const int w_geom = std::max(1, running_);
    const int nblk_f = fused_partials(op, w_geom);
    int* kstart = kstart_buf_[(launches_ / ch) & 1];
    // timing: every period-th chunk runs eagerly with its stencil launches
    // bracketed by events, the others replay as graphs; the GEMM overlaps
    // timed and untimed chunks alike, so that the timed launches share the
    // device as all the others do
    const int chunk_index = launches_ / ch;
    tm->active = tm->on && chunk_index % tm->period == 0;
    hipStream_t gemm_stream = side_;
    HIPCHK(hipMemcpyAsync(kstart, st_.k, w * sizeof(int), hipMemcpyDeviceToDevice, s));
    auto issue = [&]() -> negf_status {
        for (int it = 0; it < steps; ++it) {
            // p ping-pongs so that halo reads of the fused kernel see p_{k-1};
            // every column starts at an even k
            cplx_t<R>* pin = (it & 1) ? p2_ : p_;
            cplx_t<R>* pout = (it & 1) ? p_ : p2_;
            hipEvent_t e0, e1;
            CHK(tm->next(&e0, &e1));
            launch_cocg_apply<R>(op, r_, pin, pout, q_, w, shift_, st_.done, st_.k, st_.beta,
                                      part_f_, kbc_, s, e0, e1, !fused_update_, w_geom);
            if (fused_update_) {
                // alpha, projector term, r update and kept rows in one launch
                launch_update_ms<R>(r_, q_, N, st_, part_f_, nblk_f, op, kbc_, ring_,
                                         ring_len_, row0_, n_rows_, part_, part_nn_, s,
                                         out_.row1, out_.n_rows1);
                launch_reduce_beta_multishift(part_, part_nn_, nblk_, st_, s);
                continue;
            }
            launch_reduce_alpha(part_f_, nblk_f, st_, s, op->kb.n_proj ? kbc_ : nullptr,
                                op->kb.e, op->kb.n_proj);
            launch_r_update<R>(r_, q_, nullptr, nullptr, part_, part_nn_, st_, N, s);
            launch_store_rows<R>(r_, N, w, d_rows_, row0_, n_rows_, ring_, ring_len_, st_, 1, s,
                                      nullptr, out_.row1, out_.n_rows1);
            launch_reduce_beta_multishift(part_, part_nn_, nblk_, st_, s);
        }
        return NEGF_OK;
    };
    CHK(run_chunk(cg_, use_graph_ && steps == ch && w_geom == w, s, tm, issue));
    // fold the chunk's iterations into X and P of every energy: the
    // coefficients here (after the previous GEMM has read its own), the GEMM
    // on the side stream, overlapping the next chunk
    if (gemm_pending_) HIPCHK(hipStreamWaitEvent(s, ev_gemm_, 0));
    launch_chunk_coef(st_, kstart, clen_, cx_, cp_, xi_a_, carry_, active_, act_list_, act_n_, s);
    HIPCHK(hipEventRecord(ev_coef_, s));
    HIPCHK(hipStreamWaitEvent(gemm_stream, ev_coef_, 0));
    launch_gemm_xp(ring_, ring_len_, w, n_rows_, kstart, clen_, st_, cx_, cp_, xi_a_, active_,
                   act_list_, act_n_, X_, P_, gemm_stream);
    HIPCHK(hipEventRecord(ev_gemm_, gemm_stream));
    gemm_pending_ = true;
    HIPCHK(hipGetLastError());
    launches_ += steps;
    HIPCHK(hipMemcpyAsync(h_flags_, st_.done, w * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(h_flags_ + w, st_.k, w * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(ev_chunk_, s));
    return NEGF_OK;
}

template <typename R>
negf_status MultiShiftRun<R>::after_chunk(bool* busy) {
    negf_op* op = op_;
    const int w = w_, ng = ng_, n_rows = n_rows_;
    const int64_t N = N_;
    hipStream_t s = s_;
    MatvecTimer* tm = tm_;
    HIPCHK(hipEventSynchronize(ev_chunk_));
    const int* h_done = h_flags_;
    const int* h_k = h_flags_ + w;
    CHK(tm->flush());
    if (tm->active) {
        // algorithmic bytes of the timed launches: per column-iteration r and
        // p_{k-1} in, p_k and q out; V once per launch
        int64_t ci = 0;
        for (int c = 0; c < w; ++c) ci += h_k[c] - h_kprev_[c];
        tm->bytes += 4.0 * sizeof(cplx_t<R>) * (double)N * (double)ci + 8.0 * N * steps_;
    }
    for (int c = 0; c < w; ++c) h_kprev_[c] = h_k[c];
    const bool stop = (n_src_ == w) && launches_ >= d_.max_iter;
    // slots whose column is done hand over its results
    int n_fin = 0;
    for (int c = 0; c < w; ++c) {
        h_mask_[c] = (slot_src_[c] >= 0 && (h_done[c] != 0 || stop)) ? 1 : 0;
        n_fin += h_mask_[c];
    }
    // finished slots read X and restarted ones clear it: the GEMM first
    if (n_fin > 0) HIPCHK(hipStreamWaitEvent(s, ev_gemm_, 0));
    if (n_fin > 0 && out_.d_out) {
        // column mode: X stays in place and is copied out at the end
        for (int c = 0; c < w; ++c)
            if (h_mask_[c]) slot_src_[c] = -1;
    } else if (n_fin > 0) {
        const bool all_fin = (n_fin == w);
        HIPCHK(hipMemcpyAsync(d_mask_, h_mask_.data(), w * sizeof(int), hipMemcpyHostToDevice, s));
        if (out_.h_tcol) {
            for (int c = 0; c < w; ++c) h_colw_[c] = h_mask_[c] ? h_col_w_[slot_src_[c]] : 0.0;
            HIPCHK(hipMemcpyAsync(col_w_, h_colw_.data(), w * sizeof(double), hipMemcpyHostToDevice, s));
            launch_t_from_x(X_, n_rows, w, ng, d_row_w_, col_w_, all_fin ? nullptr : d_mask_, tcol_, s);
            h_t_.resize((size_t)w * ng);
            HIPCHK(hipMemcpyAsync(h_t_.data(), tcol_, (size_t)w * ng * sizeof(double), hipMemcpyDeviceToHost, s));
        }
        if (out_.h_optical) {
            // local kept-row index of each finishing slot's own source point
            const int n0 = n_rows - out_.n_rows1;
            for (int c = 0; c < w; ++c)
                h_jloc_[c] = h_mask_[c] ? n0 + (int)(cols_[slot_src_[c]] - out_.row1) : 0;
            HIPCHK(hipMemcpyAsync(d_jloc_, h_jloc_.data(), w * sizeof(int), hipMemcpyHostToDevice, s));
            launch_optical(X_, n_rows, n_rows, w, ng, out_.d_row_wo, d_jloc_,
                           all_fin ? nullptr : d_mask_, d_opt_, s);
            h_opt_.resize((size_t)w * ng);
            HIPCHK(hipMemcpyAsync(h_opt_.data(), d_opt_, (size_t)w * ng * sizeof(double), hipMemcpyDeviceToHost, s));
        }
        h_res_.resize((size_t)w * ng);
        h_si_.resize((size_t)w * ng);
        HIPCHK(hipMemcpyAsync(h_res_.data(), st_.sres, (size_t)w * ng * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(h_si_.data(), st_.sconv, (size_t)w * ng * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int c = 0; c < w; ++c) {
            if (!h_mask_[c]) continue;
            const int j = slot_src_[c];
            *total_iters_ += h_k[c];
            if (out_.h_iters) out_.h_iters[j] = h_k[c];
            if (out_.h_status) out_.h_status[j] = h_done[c] ? h_done[c] - 1 : NEGF_ITEM_MAX_ITER;
            for (int g = 0; g < ng; ++g) {
                const size_t so = (size_t)c * ng + g, dof = (size_t)j * ng + g;
                if (out_.h_tcol) out_.h_tcol[dof] = h_t_[so];
                if (out_.h_optical) out_.h_optical[dof] = h_opt_[so];
                if (out_.h_resid) out_.h_resid[dof] = h_res_[so];
                if (out_.h_shift_iters) out_.h_shift_iters[dof] = h_si_[so];
            }
            slot_src_[c] = -1;
        }
    }
    // restart finished slots on queued columns
    int n_new = 0;
    for (int c = 0; c < w; ++c) {
        h_mask_[c] = 0;
        if (slot_src_[c] < 0 && next_src_ < n_src_ && n_src_ > w) {
            slot_src_[c] = next_src_++;
            h_colsel_[c] = cols_[slot_src_[c]];
            h_mask_[c] = 1;
            ++n_new;
        }
        h_notmask_[c] = 1 - h_mask_[c];
    }
    if (n_new > 0) {
        HIPCHK(hipStreamWaitEvent(s, ev_gemm_, 0));  // X, P, carry are rewritten below
        HIPCHK(hipMemcpyAsync(d_mask_, h_mask_.data(), w * sizeof(int), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(d_notmask_, h_notmask_.data(), w * sizeof(int), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(d_cols_, h_colsel_.data(), w * sizeof(int), hipMemcpyHostToDevice, s));
        launch_init_unit<R>(r_, nullptr, N, w, d_cols_, s, d_mask_);
        for (int c = 0; c < w; ++c)
            if (h_mask_[c]) h_kprev_[c] = 0;
        for (int c = 0; c < w; ++c) {
            if (!h_mask_[c]) continue;
            const size_t xo = (size_t)c * ng * n_rows;
            HIPCHK(hipMemsetAsync(X_ + xo, 0, (size_t)ng * n_rows * sizeof(double2), s));
            HIPCHK(hipMemsetAsync(P_ + xo, 0, (size_t)ng * n_rows * sizeof(double2), s));
            HIPCHK(hipMemsetAsync(carry_ + (size_t)c * ng, 0, (size_t)ng * sizeof(double2), s));
        }
        launch_norms<R>(r_, N, w, d_notmask_, part_, part_nn_, s);
        launch_reduce_init(part_, part_nn_, nblk_, st_, nullptr, s, d_mask_);
        launch_store_rows<R>(r_, N, w, d_rows_, row0_, n_rows, ring_, ring_len_, st_, 0, s,
                                  d_mask_, out_.row1, out_.n_rows1);
        HIPCHK(hipGetLastError());
    }
    bool any = false;
    running_ = 0;
    for (int c = 0; c < w; ++c) {
        any = any || slot_src_[c] >= 0;
        // restarted slots run; live ones run unless their column is done
        running_ += (slot_src_[c] >= 0 && (h_mask_[c] || h_done[c] == 0)) ? 1 : 0;
    }
    (void)op;
    *busy = any;
    return NEGF_OK;
}

template <typename R>
negf_status MultiShiftRun<R>::finish() {
    const int w = w_, ng = ng_, n_rows = n_rows_;
    hipStream_t s = s_;
    if (gemm_pending_) HIPCHK(hipStreamWaitEvent(s, ev_gemm_, 0));
    if (out_.d_out) {
        // column mode: every slot is still live here (n_src == w)
        const int* h_done = h_flags_;
        const int* h_k = h_flags_ + w;
        for (int c = 0; c < w; ++c) {
            *total_iters_ += h_k[c];
            if (out_.h_iters) out_.h_iters[c] = h_k[c];
            if (out_.h_status) out_.h_status[c] = h_done[c] ? h_done[c] - 1 : NEGF_ITEM_MAX_ITER;
        }
        launch_copy_out(X_, n_rows, w, ng, out_.d_out, out_.out_col_stride, out_.out_shift_stride, s);
        if (out_.h_resid)
            HIPCHK(hipMemcpyAsync(out_.h_resid, st_.sres, (size_t)w * ng * sizeof(double), hipMemcpyDeviceToHost, s));
        if (out_.h_shift_iters)
            HIPCHK(hipMemcpyAsync(out_.h_shift_iters, st_.sconv, (size_t)w * ng * sizeof(int), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return NEGF_OK;
}

static negf_status run_multishift_block(negf_op* op, const Defaults& d, int w, int n_src,
                                        const int* cols, const double2* d_rhs,
                                        const double* energies, int ng, const int* d_rows,
                                        int64_t row0, int n_rows, const double* d_row_w,
                                        const double* h_col_w, const MSOut& out,
                                        int64_t* total_iters, hipStream_t s, MatvecTimer* tm) {
    auto go = [&](auto& run) -> negf_status {
        CHK(run.start());
        bool busy = true;
        while (busy) {
            CHK(run.issue_chunk());
            CHK(run.after_chunk(&busy));
        }
        return run.finish();
    };
    MultiShiftRun<double> run(op, d, w, n_src, cols, d_rhs, energies, ng, d_rows, row0, n_rows,
                              d_row_w, h_col_w, out, total_iters, s, tm);
    return go(run);
}

// launchers of adjoint.hip
void launch_gather(const double2* x, int64_t N, int w, const int* rows, int n_rows,
                   const int64_t* dst, double2* out, hipStream_t s);
void launch_adjoint_rhs(const double2* g, int64_t N, int64_t plane, int w, const double* wl,
                        double2* rhs, hipStream_t s);
void launch_field(const double2* g, const double2* lam, int64_t N, int w, const double* colw,
                  double scale, double* field, hipStream_t s);

// One block of w (column, energy) items through the per-energy core with
// FP64 iterative refinement.  The inner COCG runs in R (double for the FP64
// path, float for the mixed path); x, the true residual r = b - A x, its norm
// and the solution update x += ||r|| d are FP64.  On return the solutions are
// in the WS_X64 workspace ([w][N] FP64).
struct PEOut {
    int* h_iters = nullptr;    // [w] Krylov iterations summed over refinement steps
    int* h_status = nullptr;   // [w]
    double* h_resid = nullptr; // [w] final true relative residual
    int* h_refine = nullptr;   // [w] refinement steps
};

static constexpr int kInnerChunk = 16;

template <typename R>
static negf_status run_per_energy_block(negf_op* op, const Defaults& d, int w, const int* cols,
                                        const double2* d_rhs, const double* item_e,
                                        const PEOut& out, int64_t* total_iters, hipStream_t s,
                                        MatvecTimer* tm) {
    const int64_t N = op->N;
    const int nblk = part_blocks(N);
    const int nblk_f = fused_partials(op, w);
    cplx_t<R> *r, *p, *p2, *q, *dsol;
    double2 *b64, *x64, *r64, *q64, *part, *kbc, *part_f;
    double *part_nn, *shift, *misc;
    int* d_cols;
    CHK(ws(op, WS_R, (size_t)w * N, &r));
    CHK(ws(op, WS_P, (size_t)w * N, &p));
    CHK(ws(op, WS_RING, (size_t)w * N, &p2));
    CHK(ws(op, WS_Q, (size_t)w * N, &q));
    CHK(ws(op, WS_X, (size_t)w * N, &dsol));
    CHK(ws(op, WS_B, (size_t)w * N, &b64));
    CHK(ws(op, WS_PART3, (size_t)w * nblk_f, &part_f));
    CHK(ws_get(op, WS_SINK, (size_t)w * op->nx * op->ny * sizeof(double2), &op->d_sink));
    CHK(ws(op, WS_X64, (size_t)w * N, &x64));
    CHK(ws(op, WS_R64, (size_t)w * N, &r64));
    CHK(ws(op, WS_Q64, (size_t)w * N, &q64));
    CHK(ws(op, WS_PART, (size_t)w * nblk, &part));
    CHK(ws(op, WS_PART2, (size_t)w * nblk, &part_nn));
    CHK(ws(op, WS_KBC, (size_t)w * std::max(1, op->kb.n_proj), &kbc));
    CHK(ws(op, WS_SHIFT, (size_t)w, &shift));
    CHK(ws(op, WS_COLJ, (size_t)w, &d_cols));
    CHK(ws(op, WS_MISC, (size_t)w * 4, &misc));
    double* nu = misc;             // [w] current ||r64||
    double* bn64 = misc + w;       // [w] ||b||
    double* resid = misc + 2 * w;  // [w]
    int* odone = (int*)(misc + 3 * w);
    const bool qmr = d.solver == NEGF_SOLVER_QMR;
    cplx_t<R>* dq = nullptr;  // smoothed step of the simplified QMR iterate
    if (qmr) CHK(ws(op, WS_QMRD, (size_t)w * N, &dq));
    IterState st;
    CHK(make_state(op, w, 0, d.max_iter, d.tol, false, &st, 0, qmr));

    HIPCHK(hipMemcpyAsync(shift, item_e, w * sizeof(double), hipMemcpyHostToDevice, s));
    if (cols) {
        HIPCHK(hipMemcpyAsync(d_cols, cols, w * sizeof(int), hipMemcpyHostToDevice, s));
        launch_init_unit<double>(b64, nullptr, N, w, d_cols, s);
    } else {
        HIPCHK(hipMemcpyAsync(b64, d_rhs, (size_t)w * N * sizeof(double2), hipMemcpyDeviceToDevice, s));
    }
    HIPCHK(hipMemsetAsync(x64, 0, (size_t)w * N * sizeof(double2), s));
    HIPCHK(hipMemsetAsync(odone, 0, w * sizeof(int), s));
    // x = 0: r64 = b, nu = ||b||
    HIPCHK(hipMemcpyAsync(r64, b64, (size_t)w * N * sizeof(double2), hipMemcpyDeviceToDevice, s));
    launch_norms<double>(r64, N, w, nullptr, part, part_nn, s);
    launch_reduce_residual(part_nn, nblk, w, odone, nullptr, nu, d.tol, resid, s);
    HIPCHK(hipMemcpyAsync(bn64, nu, w * sizeof(double), hipMemcpyDeviceToDevice, s));

    std::vector<int> h_done(w), h_odone(w), h_k(w), iters(w, 0), refine(w, 0);
    // items whose inner COCG broke down stop refining once the outer residual
    // shows they did not converge anyway
    std::vector<int> broke(w, 0), final_break(w, 0);
    int outer = 0;
    ChunkGraph cg;
    DrainGuard drain{s, nullptr};
    const bool use_graph = graphs_enabled();
    const double inner_tol = (sizeof(R) == 8) ? 0.5 * d.tol : 2e-6;
    while (true) {
        if (outer > 0) {
            launch_apply<double>(op, x64, q64, w, shift, odone, kbc, s);
            launch_residual(b64, q64, r64, N, w, odone, part_nn, s);
            launch_reduce_residual(part_nn, nblk, w, odone, bn64, nu, d.tol, resid, s);
        }
        HIPCHK(hipMemcpyAsync(h_odone.data(), odone, w * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        bool forced = false;
        for (int c = 0; c < w; ++c)
            if (broke[c] && !h_odone[c]) {
                h_odone[c] = 1;
                final_break[c] = 1;
                forced = true;
            }
        if (forced)
            HIPCHK(hipMemcpyAsync(odone, h_odone.data(), w * sizeof(int), hipMemcpyHostToDevice, s));
        bool all = true;
        for (int c = 0; c < w; ++c) all = all && h_odone[c];
        if (all || outer >= d.max_refine) break;
        ++outer;
        for (int c = 0; c < w; ++c)
            if (!h_odone[c]) ++refine[c];
        // inner solve A d = r64 / ||r64|| in precision R
        launch_scale_convert<R>(r64, r, dsol, N, w, odone, nu, s);
        if (qmr) HIPCHK(hipMemsetAsync(dq, 0, (size_t)w * N * sizeof(cplx_t<R>), s));
        launch_norms<R>(r, N, w, odone, part, part_nn, s);
        launch_reduce_init(part, part_nn, nblk, st, odone, s);
        int k_host = 0;
        while (true) {
            const int steps = std::min(kInnerChunk, d.max_iter - k_host);
            auto issue = [&]() -> negf_status {
                for (int it = 0; it < steps; ++it) {
                    cplx_t<R>* pin = (it & 1) ? p2 : p;  // chunks start at even k
                    cplx_t<R>* pout = (it & 1) ? p : p2;
                    hipEvent_t e0, e1;
                    CHK(tm->next(&e0, &e1));
                    // r, the p pair, q and the iterate d are touched every iteration
                    launch_cocg_apply<R>(op, r, pin, pout, q, w, shift, st.done, st.k, st.beta,
                                         part_f, kbc, s, e0, e1, true, 0, 5);
                    launch_reduce_alpha(part_f, nblk_f, st, s, op->kb.n_proj ? kbc : nullptr,
                                        op->kb.e, op->kb.n_proj);
                    // COCG: x += alpha p_k; QMR: the pending smoothed step from p_{k-1}
                    launch_r_update<R>(r, q, qmr ? pin : pout, dsol, part, part_nn, st, N, s,
                                       qmr ? dq : nullptr);
                    launch_reduce_beta_single(part, part_nn, nblk, st, inner_tol, s);
                }
                return NEGF_OK;
            };
            CHK(run_chunk(cg, use_graph && steps == kInnerChunk, s, tm, issue));
            HIPCHK(hipGetLastError());
            k_host += steps;
            HIPCHK(hipMemcpyAsync(h_done.data(), st.done, w * sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            CHK(tm->flush());
            bool alld = true;
            for (int c = 0; c < w; ++c) alld = alld && h_done[c];
            if (alld || k_host >= d.max_iter) break;
        }
        HIPCHK(hipMemcpyAsync(h_k.data(), st.k, w * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(h_done.data(), st.done, w * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int c = 0; c < w; ++c)
            if (!h_odone[c] && h_done[c] == 1 + NEGF_ITEM_BREAKDOWN) broke[c] = 1;
        int64_t col_iters = 0;
        for (int c = 0; c < w; ++c)
            if (!h_odone[c]) {
                iters[c] += h_k[c];
                col_iters += h_k[c];
            }
        if (tm->on)
            tm->bytes += 4.0 * sizeof(cplx_t<R>) * (double)N * (double)col_iters + 8.0 * N * k_host;
        // QMR: the last step is still pending; p_k sits in p2 for even k, in p for odd k
        if (qmr) launch_qmr_flush<R>(p2, p, dq, dsol, N, st, odone, s);
        launch_accumulate<R>(x64, dsol, N, w, odone, nu, s);
    }
    for (int c = 0; c < w; ++c) {
        *total_iters += iters[c];
        if (out.h_iters) out.h_iters[c] = iters[c];
        if (out.h_status)
            out.h_status[c] = final_break[c] ? NEGF_ITEM_BREAKDOWN
                                             : (h_odone[c] ? NEGF_ITEM_CONVERGED : NEGF_ITEM_MAX_ITER);
        if (out.h_refine) out.h_refine[c] = refine[c];
    }
    if (out.h_resid)
        HIPCHK(hipMemcpyAsync(out.h_resid, resid, w * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return NEGF_OK;
}

static negf_status run_per_energy(negf_op* op, const Defaults& d, int w, const int* cols,
                                  const double2* d_rhs, const double* item_e, const PEOut& out,
                                  int64_t* total_iters, hipStream_t s, MatvecTimer* tm) {
    if (d.precision == NEGF_MIXED)
        return run_per_energy_block<float>(op, d, w, cols, d_rhs, item_e, out, total_iters, s, tm);
    return run_per_energy_block<double>(op, d, w, cols, d_rhs, item_e, out, total_iters, s, tm);
}

// ---------------------------------------------------------------------------
// source / row sets of the transmission (Eq. 7)
// ---------------------------------------------------------------------------
struct Sides {
    std::vector<int> cols;   // source grid indices (CAP support, ascending)
    std::vector<double> colw; // 4 W_src at the column
    int64_t row0 = 0;        // rows: contiguous CAP support of the other side
    int n_rows = 0;
    std::vector<double> roww;
};

static negf_status restrict_sides(const Defaults& d, Sides* sd) {
    const int n = (int)sd->cols.size();
    if (d.col_begin == 0 && d.col_count == 0) return NEGF_OK;
    const int cnt = d.col_count ? d.col_count : n - d.col_begin;
    if (d.col_begin >= n || cnt < 1 || d.col_begin + cnt > n) {
        set_error("column range [%d, %d) outside the %d source columns", d.col_begin,
                  d.col_begin + cnt, n);
        return NEGF_E_INVALID_ARG;
    }
    sd->cols = std::vector<int>(sd->cols.begin() + d.col_begin, sd->cols.begin() + d.col_begin + cnt);
    sd->colw = std::vector<double>(sd->colw.begin() + d.col_begin, sd->colw.begin() + d.col_begin + cnt);
    return NEGF_OK;
}

static void make_sides(const negf_op* op, int direction, Sides* sd) {
    const int64_t plane = (int64_t)op->nx * op->ny;
    const bool rl = direction == NEGF_DIR_RL;
    const int cz0 = rl ? op->zr0 : op->zl0, cz1 = rl ? op->zr1 : op->zl1;
    const int rz0 = rl ? op->zl0 : op->zr0, rz1 = rl ? op->zl1 : op->zr1;
    const std::vector<double>& wc = rl ? op->cap_r : op->cap_l;
    const std::vector<double>& wr = rl ? op->cap_l : op->cap_r;
    for (int z = cz0; z < cz1; ++z)
        for (int64_t i = 0; i < plane; ++i) {
            sd->cols.push_back((int)(z * plane + i));
            sd->colw.push_back(4.0 * wc[z]);
        }
    sd->row0 = rz0 * plane;
    sd->n_rows = (int)((rz1 - rz0) * plane);
    for (int z = rz0; z < rz1; ++z)
        for (int64_t i = 0; i < plane; ++i) sd->roww.push_back(wr[z]);
}

static negf_status check_energies(int n_e, const double* e) {
    if (n_e < 1 || !e) {
        set_error("need at least one energy");
        return NEGF_E_INVALID_ARG;
    }
    for (int i = 0; i < n_e; ++i)
        if (!std::isfinite(e[i])) {
            set_error("energy %d not finite", i);
            return NEGF_E_INVALID_ARG;
        }
    return NEGF_OK;
}

static int pick_core(const Defaults& d) {
    if (d.core != NEGF_CORE_AUTO) return d.core;
    if (d.solver == NEGF_SOLVER_QMR) return NEGF_CORE_PER_ENERGY;
    return d.precision == NEGF_FP64 ? NEGF_CORE_MULTISHIFT : NEGF_CORE_PER_ENERGY;
}

// Status of one energy of a multi-shift column: converged when its residual
// estimate met tol (energies freeze as they converge, so those that froze
// before a breakdown of the column keep their results), else the column's
// breakdown, else out of iterations
static int ms_item_status(double resid, int col_status, double tol) {
    if (resid <= tol * 1.0000001) return NEGF_ITEM_CONVERGED;
    return col_status == NEGF_ITEM_BREAKDOWN ? NEGF_ITEM_BREAKDOWN : NEGF_ITEM_MAX_ITER;
}

static negf_status final_status(int n_bad, int n_break) {
    if (n_break > 0) {
        set_error("%d items broke down", n_break);
        return NEGF_E_BREAKDOWN;
    }
    if (n_bad > 0) {
        set_error("%d items did not converge", n_bad);
        return NEGF_E_NOT_CONVERGED;
    }
    return NEGF_OK;
}

// ---------------------------------------------------------------------------
// negf_transmission
// ---------------------------------------------------------------------------
static negf_status transmission_impl(negf_op* op, const negf_opts* opts, int32_t n_e,
                                     const double* energies, double* T, negf_diag* diag) {
    Defaults d;
    CHK(read_opts(opts, &d));
    CHK(check_energies(n_e, energies));
    if (!T) {
        set_error("null T");
        return NEGF_E_INVALID_ARG;
    }
    const int core = pick_core(d);
    if (core == NEGF_CORE_MULTISHIFT && d.precision != NEGF_FP64) {
        set_error("the multi-shift core runs in FP64 only (mixed precision uses the per-energy core)");
        return NEGF_E_INVALID_ARG;
    }
    HIPCHK(hipSetDevice(op->device));
    hipStream_t s = pick_stream(op, opts);
    const auto t0 = std::chrono::steady_clock::now();
    MatvecTimer tm;
    CHK(tm.init(diag ? diag->time_matvec : 0));
    Sides sd;
    make_sides(op, d.direction, &sd);
    CHK(restrict_sides(d, &sd));
    const int n_cols = (int)sd.cols.size();
    // restarts of failed multi-shift items: the items to restart are those
    // that end in breakdown or at max_iter, or whose column fails the
    // optical-theorem check, which is then always computed
    const bool recover = d.recover == NEGF_RECOVER_RESTART && core == NEGF_CORE_MULTISHIFT;
    const bool want_opt = (diag && diag->optical_err) || recover;
    const int64_t plane = (int64_t)op->nx * op->ny;
    // the optical check keeps the source side's absorbing rows as well: T
    // weights W_dst on the destination rows and 0 on those, the check's
    // weights W on both
    const bool rl = d.direction == NEGF_DIR_RL;
    const int64_t row1 = (rl ? op->zr0 : op->zl0) * plane;
    const int n_rows1 = (want_opt && core == NEGF_CORE_MULTISHIFT)
                            ? (int)(((rl ? op->zr1 : op->zl1) - (rl ? op->zr0 : op->zl0)) * plane)
                            : 0;
    const int n_keep = sd.n_rows + n_rows1;
    std::vector<double> roww(sd.roww), row_wo;
    if (n_rows1) {
        roww.resize(n_keep, 0.0);
        row_wo = sd.roww;
        const std::vector<double>& wsrc = rl ? op->cap_r : op->cap_l;
        for (int r = 0; r < n_rows1; ++r) row_wo.push_back(wsrc[(row1 + r) / plane]);
    }
    double* d_roww = nullptr;
    CHK(ws(op, WS_ROWW, (size_t)n_keep * (n_rows1 ? 2 : 1), &d_roww));
    HIPCHK(hipMemcpyAsync(d_roww, roww.data(), n_keep * sizeof(double), hipMemcpyHostToDevice, s));
    double* d_row_wo = n_rows1 ? d_roww + n_keep : nullptr;
    if (n_rows1)
        HIPCHK(hipMemcpyAsync(d_row_wo, row_wo.data(), n_keep * sizeof(double), hipMemcpyHostToDevice, s));
    // tcol[e][c]
    std::vector<double> tcol((size_t)n_e * n_cols, 0.0);
    std::vector<int> iters((size_t)n_e * n_cols, 0), status((size_t)n_e * n_cols, 0);
    std::vector<double> resid((size_t)n_e * n_cols, 0.0);
    std::vector<double> optical(want_opt ? (size_t)n_e * n_cols : 0, 0.0);
    std::vector<int> refine((size_t)n_e * n_cols, 0);
    int64_t total_iters = 0;
    if (core == NEGF_CORE_MULTISHIFT) {
        const int ng_max = d.shift_group ? std::min(d.shift_group, n_e) : n_e;
        const int wmax = d.block_width ? d.block_width : (op->tuned_w ? op->tuned_w : 64);
        // the shard's columns stream through one block of slots; with
        // NEGF_NO_COLUMN_STREAM=1 each block of wmax columns runs on its own
        const bool stream = !column_stream_disabled();
        std::vector<double> blk_t, blk_r, blk_o;
        std::vector<int> blk_it, blk_st, blk_si;
        for (int g0 = 0; g0 < n_e; g0 += ng_max) {
            const int ng = std::min(ng_max, n_e - g0);
            const int span = stream ? n_cols : wmax;
            for (int c0 = 0; c0 < n_cols; c0 += span) {
                const int n_src = std::min(span, n_cols - c0);
                const int w = std::min(wmax, n_src);
                blk_t.assign((size_t)n_src * ng, 0.0);
                blk_r.assign((size_t)n_src * ng, 0.0);
                blk_it.assign(n_src, 0);
                blk_st.assign(n_src, 0);
                blk_si.assign((size_t)n_src * ng, 0);
                blk_o.assign(want_opt ? (size_t)n_src * ng : 0, 0.0);
                MSOut mo;
                mo.h_tcol = blk_t.data();
                mo.h_iters = blk_it.data();
                mo.h_status = blk_st.data();
                mo.h_resid = blk_r.data();
                mo.h_shift_iters = blk_si.data();
                if (want_opt) {
                    mo.row1 = row1;
                    mo.n_rows1 = n_rows1;
                    mo.d_row_wo = d_row_wo;
                    mo.h_optical = blk_o.data();
                }
                CHK(run_multishift_block(op, d, w, n_src, sd.cols.data() + c0, nullptr, energies + g0,
                                         ng, nullptr, sd.row0, n_keep, d_roww,
                                         sd.colw.data() + c0, mo, &total_iters, s, &tm));
                for (int c = 0; c < n_src; ++c)
                    for (int g = 0; g < ng; ++g) {
                        const size_t o = (size_t)(g0 + g) * n_cols + c0 + c;
                        tcol[o] = blk_t[(size_t)c * ng + g];
                        resid[o] = blk_r[(size_t)c * ng + g];
                        if (want_opt) optical[o] = blk_o[(size_t)c * ng + g];
                        // iterations this energy needed (the column's count if it never froze)
                        iters[o] = blk_si[(size_t)c * ng + g] ? blk_si[(size_t)c * ng + g] : blk_it[c];
                        // a column that hit max_iter can still have converged
                        // energies; judge each by its own residual estimate
                        status[o] = ms_item_status(resid[o], blk_st[c], d.tol);
                    }
            }
        }
    }
    // per-energy solves of the listed items (o = e * n_cols + j), in blocks
    // of up to wmax items; their diagnostics overwrite those of item o
    double* d_wfull = nullptr;  // W_L + W_R per grid point, for the optical check
    auto solve_items = [&](const Defaults& dd, const std::vector<int64_t>& items) -> negf_status {
        const int wmax = dd.block_width ? dd.block_width : 64;
        std::vector<int> icol, b_it, b_st, b_rf;
        std::vector<double> ie, colw, b_res, b_t, b_o;
        // column weights [w], t [w], optical errors [w], source points [w]
        double* d_colw = nullptr;
        CHK(ws(op, WS_TCOL, (size_t)4 * wmax, &d_colw));
        double* d_t = d_colw + wmax;
        double* d_opt = d_t + wmax;
        int* d_jg = reinterpret_cast<int*>(d_opt + wmax);
        if (want_opt && !d_wfull) {
            std::vector<double> wf((size_t)op->N);
            for (int64_t i = 0; i < op->N; ++i) {
                const int z = (int)(i / plane);
                wf[i] = op->cap_l[z] + op->cap_r[z];
            }
            CHK(ws(op, WS_GAMMA, (size_t)op->N, &d_wfull));
            HIPCHK(hipMemcpyAsync(d_wfull, wf.data(), wf.size() * sizeof(double),
                                  hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        const int64_t n_items = (int64_t)items.size();
        for (int64_t i0 = 0; i0 < n_items; i0 += wmax) {
            const int w = (int)std::min<int64_t>(wmax, n_items - i0);
            icol.resize(w); ie.resize(w); colw.resize(w);
            for (int c = 0; c < w; ++c) {
                const int64_t it = items[i0 + c];
                const int e = (int)(it / n_cols), j = (int)(it % n_cols);
                icol[c] = sd.cols[j];
                ie[c] = energies[e];
                colw[c] = sd.colw[j];
            }
            b_it.assign(w, 0); b_st.assign(w, 0); b_res.assign(w, 0.0); b_t.assign(w, 0.0);
            b_o.assign(w, 0.0); b_rf.assign(w, 0);
            PEOut po;
            po.h_iters = b_it.data();
            po.h_status = b_st.data();
            po.h_resid = b_res.data();
            po.h_refine = b_rf.data();
            CHK(run_per_energy(op, dd, w, icol.data(), nullptr, ie.data(), po, &total_iters, s, &tm));
            double2* x64 = (double2*)op->bufs[WS_X64].ptr;
            HIPCHK(hipMemcpyAsync(d_colw, colw.data(), w * sizeof(double), hipMemcpyHostToDevice, s));
            launch_weighted_norm(x64, op->N, w, sd.row0, sd.n_rows, d_roww, d_colw, d_t, s);
            HIPCHK(hipMemcpyAsync(b_t.data(), d_t, w * sizeof(double), hipMemcpyDeviceToHost, s));
            if (want_opt) {
                HIPCHK(hipMemcpyAsync(d_jg, icol.data(), w * sizeof(int), hipMemcpyHostToDevice, s));
                launch_optical(x64, op->N, (int)op->N, w, 1, d_wfull, d_jg, nullptr, d_opt, s);
                HIPCHK(hipMemcpyAsync(b_o.data(), d_opt, w * sizeof(double), hipMemcpyDeviceToHost, s));
            }
            HIPCHK(hipStreamSynchronize(s));
            for (int c = 0; c < w; ++c) {
                const size_t o = (size_t)items[i0 + c];
                tcol[o] = b_t[c];
                iters[o] = b_it[c];
                status[o] = b_st[c];
                resid[o] = b_res[c];
                refine[o] = b_rf[c];
                if (want_opt) optical[o] = b_o[c];
            }
        }
        return NEGF_OK;
    };
    if (core != NEGF_CORE_MULTISHIFT) {
        std::vector<int64_t> all((size_t)n_e * n_cols);
        for (size_t o = 0; o < all.size(); ++o) all[o] = (int64_t)o;
        CHK(solve_items(d, all));
    }
    // the optical-theorem check, when computed, must also hold
    const double opt_bar = std::max(1e4 * d.tol, 1e-8);
    auto flag_optical = [&]() {
        if (!want_opt) return;
        for (size_t o = 0; o < status.size(); ++o)
            if (status[o] == NEGF_ITEM_CONVERGED && !(optical[o] <= opt_bar))
                status[o] = NEGF_ITEM_INACCURATE;
    };
    flag_optical();
    if (recover) {
        // each failed item is restarted as its own seed system (a breakdown of
        // the shared seed ends every shift of the column at once, and the
        // shifted residuals of a restart would no longer be collinear): FP64
        // per-energy COCG with true-residual refinement, then QMR for those
        // COCG still fails
        std::vector<int> spent(iters.size(), 0);  // iterations of the earlier runs
        std::vector<int64_t> redo;
        Defaults d2 = d;
        d2.precision = NEGF_FP64;
        d2.core = NEGF_CORE_PER_ENERGY;
        for (int pass = 0; pass < 2; ++pass) {
            redo.clear();
            for (size_t o = 0; o < status.size(); ++o)
                if (status[o] != NEGF_ITEM_CONVERGED) {
                    redo.push_back((int64_t)o);
                    spent[o] += iters[o];
                }
            if (redo.empty()) break;
            d2.solver = pass == 0 ? NEGF_SOLVER_COCG : NEGF_SOLVER_QMR;
            CHK(solve_items(d2, redo));
            flag_optical();
        }
        for (size_t o = 0; o < iters.size(); ++o) iters[o] += spent[o];
    }
    int n_bad = 0, n_break = 0;
    for (int e = 0; e < n_e; ++e) {
        double acc = 0.0;
        for (int c = 0; c < n_cols; ++c) {
            const size_t o = (size_t)e * n_cols + c;
            acc += tcol[o];
            if (status[o] == NEGF_ITEM_BREAKDOWN) ++n_break;
            else if (status[o] != NEGF_ITEM_CONVERGED) ++n_bad;
        }
        T[e] = acc;
    }
    if (diag) {
        const size_t n = (size_t)n_e * n_cols;
        if (diag->iters) std::copy(iters.begin(), iters.end(), diag->iters);
        if (diag->resid) std::copy(resid.begin(), resid.end(), diag->resid);
        if (diag->t_col) std::copy(tcol.begin(), tcol.end(), diag->t_col);
        if (diag->item_status) std::copy(status.begin(), status.end(), diag->item_status);
        if (diag->optical_err) std::copy(optical.begin(), optical.end(), diag->optical_err);
        if (diag->refine_steps) std::copy(refine.begin(), refine.end(), diag->refine_steps);
        (void)n;
        diag->total_iters = total_iters;
        diag->n_not_converged = n_bad + n_break;
        diag->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        diag->matvec_seconds = tm.seconds;
        diag->matvec_launches = tm.launches;
        diag->matvec_bytes = tm.bytes;
    }
    return final_status(n_bad, n_break);
}

extern "C" negf_status negf_transmission(negf_op* op, const negf_opts* opts, int32_t n_e,
                                         const double* energies, double* T, negf_diag* diag) {
    g_last_error.clear();
    (void)hipGetLastError();  // a stale error of an earlier call must not fail this one
    if (!op) {
        set_error("null op");
        return NEGF_E_INVALID_ARG;
    }
    return transmission_impl(op, opts, n_e, energies, T, diag);
}

// ---------------------------------------------------------------------------
// negf_solve_columns
// ---------------------------------------------------------------------------
static negf_status solve_columns_impl(negf_op* op, const negf_opts* opts, int32_t n_e,
                                      const double* energies, int32_t n_rhs, const int32_t* rhs_idx,
                                      const negf_c64* rhs_dense, int32_t n_rows,
                                      const int32_t* row_idx, negf_c64* out, int32_t* item_status) {
    Defaults d;
    CHK(read_opts(opts, &d));
    CHK(check_energies(n_e, energies));
    const int64_t N = op->N;
    if (n_rhs < 1 || (!rhs_idx == !rhs_dense) || !out) {
        set_error("need n_rhs >= 1, exactly one of rhs_idx / rhs_dense, and out");
        return NEGF_E_INVALID_ARG;
    }
    if (!row_idx) n_rows = (int32_t)N;
    if (n_rows < 1) {
        set_error("n_rows must be >= 1");
        return NEGF_E_INVALID_ARG;
    }
    if (rhs_idx)
        for (int i = 0; i < n_rhs; ++i)
            if (rhs_idx[i] < 0 || rhs_idx[i] >= N) {
                set_error("rhs_idx[%d] out of range", i);
                return NEGF_E_INVALID_ARG;
            }
    if (row_idx)
        for (int i = 0; i < n_rows; ++i)
            if (row_idx[i] < 0 || row_idx[i] >= N) {
                set_error("row_idx[%d] out of range", i);
                return NEGF_E_INVALID_ARG;
            }
    const int core = pick_core(d);
    if (core == NEGF_CORE_MULTISHIFT && d.precision != NEGF_FP64) {
        set_error("the multi-shift core runs in FP64 only (mixed precision uses the per-energy core)");
        return NEGF_E_INVALID_ARG;
    }
    HIPCHK(hipSetDevice(op->device));
    hipStream_t s = pick_stream(op, opts);
    MatvecTimer tm;
    const size_t out_elems = (size_t)n_e * n_rhs * n_rows;
    const bool out_dev = is_device_ptr(out);
    double2* d_out = nullptr;
    if (out_dev) {
        d_out = (double2*)out;
    } else {
        CHK(ws(op, WS_TPART, out_elems, &d_out));
    }
    // right-hand sides on the device
    double2* d_rhs_all = nullptr;
    if (rhs_dense) {
        if (is_device_ptr(rhs_dense)) {
            d_rhs_all = (double2*)rhs_dense;
        } else {
            CHK(ws(op, WS_TCOL, (size_t)n_rhs * N, &d_rhs_all));
            HIPCHK(hipMemcpyAsync(d_rhs_all, rhs_dense, (size_t)n_rhs * N * sizeof(double2), hipMemcpyHostToDevice, s));
        }
    }
    int* d_rows = nullptr;
    if (row_idx) {
        CHK(ws(op, WS_ROWS, (size_t)n_rows, &d_rows));
        HIPCHK(hipMemcpyAsync(d_rows, row_idx, n_rows * sizeof(int), hipMemcpyHostToDevice, s));
    }
    std::vector<int> status((size_t)n_e * n_rhs, 0);
    int64_t total_iters = 0;
    if (core == NEGF_CORE_MULTISHIFT) {
        const int ng_max = d.shift_group ? std::min(d.shift_group, n_e) : n_e;
        const int wmax = d.block_width ? d.block_width : (op->tuned_w ? op->tuned_w : 64);
        std::vector<int> blk_st;
        std::vector<double> blk_r;
        for (int g0 = 0; g0 < n_e; g0 += ng_max) {
            const int ng = std::min(ng_max, n_e - g0);
            for (int c0 = 0; c0 < n_rhs; c0 += wmax) {
                const int w = std::min(wmax, n_rhs - c0);
                blk_st.assign(w, 0);
                blk_r.assign((size_t)w * ng, 0.0);
                MSOut mo;
                mo.d_out = d_out + ((size_t)g0 * n_rhs + c0) * n_rows;
                mo.out_col_stride = n_rows;
                mo.out_shift_stride = (int64_t)n_rhs * n_rows;
                mo.h_status = blk_st.data();
                mo.h_resid = blk_r.data();
                CHK(run_multishift_block(op, d, w, w, rhs_idx ? rhs_idx + c0 : nullptr,
                                         d_rhs_all ? d_rhs_all + (size_t)c0 * N : nullptr,
                                         energies + g0, ng, d_rows, 0, n_rows, nullptr, nullptr,
                                         mo, &total_iters, s, &tm));
                for (int c = 0; c < w; ++c)
                    for (int g = 0; g < ng; ++g)
                        status[(size_t)(g0 + g) * n_rhs + c0 + c] =
                            ms_item_status(blk_r[(size_t)c * ng + g], blk_st[c], d.tol);
            }
        }
    } else {
        const int wmax = d.block_width ? d.block_width : 64;
        const int64_t n_items = (int64_t)n_e * n_rhs;
        std::vector<int> icol, b_st;
        std::vector<double> ie;
        std::vector<int64_t> dst;
        int64_t* d_dst = nullptr;
        double2* d_rhs_blk = nullptr;
        CHK(ws(op, WS_ROWW, (size_t)wmax, &d_dst));
        for (int64_t i0 = 0; i0 < n_items; i0 += wmax) {
            const int w = (int)std::min<int64_t>(wmax, n_items - i0);
            icol.resize(w); ie.resize(w); dst.resize(w);
            if (d_rhs_all) CHK(ws(op, WS_GAMMA, (size_t)w * N, &d_rhs_blk));
            for (int c = 0; c < w; ++c) {
                const int64_t it = i0 + c;  // e * n_rhs + r
                const int e = (int)(it / n_rhs), rr = (int)(it % n_rhs);
                ie[c] = energies[e];
                dst[c] = it * n_rows;
                if (rhs_idx) icol[c] = rhs_idx[rr];
                else HIPCHK(hipMemcpyAsync(d_rhs_blk + (size_t)c * N, d_rhs_all + (size_t)rr * N,
                                           N * sizeof(double2), hipMemcpyDeviceToDevice, s));
            }
            std::vector<int> b_st2(w, 0);
            PEOut po;
            po.h_status = b_st2.data();
            CHK(run_per_energy(op, d, w, rhs_idx ? icol.data() : nullptr, d_rhs_blk, ie.data(), po,
                               &total_iters, s, &tm));
            HIPCHK(hipMemcpyAsync(d_dst, dst.data(), w * sizeof(int64_t), hipMemcpyHostToDevice, s));
            launch_gather((double2*)op->bufs[WS_X64].ptr, N, w, d_rows, n_rows, d_dst, d_out, s);
            HIPCHK(hipStreamSynchronize(s));
            for (int c = 0; c < w; ++c) status[(size_t)(i0 + c)] = b_st2[c];
        }
    }
    if (!out_dev)
        HIPCHK(hipMemcpyAsync(out, d_out, out_elems * sizeof(double2), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int n_bad = 0, n_break = 0;
    for (size_t i = 0; i < status.size(); ++i) {
        if (status[i] == NEGF_ITEM_BREAKDOWN) ++n_break;
        else if (status[i] != NEGF_ITEM_CONVERGED) ++n_bad;
        if (item_status) item_status[i] = status[i];
    }
    return final_status(n_bad, n_break);
}

extern "C" negf_status negf_solve_columns(negf_op* op, const negf_opts* opts, int32_t n_e,
                                          const double* energies, int32_t n_rhs,
                                          const int32_t* rhs_idx, const negf_c64* rhs_dense,
                                          int32_t n_rows, const int32_t* row_idx, negf_c64* out,
                                          int32_t* item_status) {
    g_last_error.clear();
    (void)hipGetLastError();
    if (!op) {
        set_error("null op");
        return NEGF_E_INVALID_ARG;
    }
    return solve_columns_impl(op, opts, n_e, energies, n_rhs, rhs_idx, rhs_dense, n_rows, row_idx,
                              out, item_status);
}

// ---------------------------------------------------------------------------
// negf_transmission_grad
// ---------------------------------------------------------------------------
static negf_status grad_impl(negf_op* op, const negf_opts* opts, int32_t n_e,
                             const double* energies, const double* weights, double* dL_dV,
                             double* T) {
    Defaults d;
    CHK(read_opts(opts, &d));
    CHK(check_energies(n_e, energies));
    if (!weights || !dL_dV) {
        set_error("null weights or dL_dV");
        return NEGF_E_INVALID_ARG;
    }
    HIPCHK(hipSetDevice(op->device));
    hipStream_t s = pick_stream(op, opts);
    MatvecTimer tm;
    const int64_t N = op->N;
    const int64_t plane = (int64_t)op->nx * op->ny;
    Sides sd;
    make_sides(op, NEGF_DIR_RL, &sd);
    CHK(restrict_sides(d, &sd));
    const int n_cols = (int)sd.cols.size();
    // The forward columns g_j = A(E)^-1 e_j have right-hand sides that do not
    // depend on E, so one multi-shift run per block of columns gives them at
    // every energy and every grid point (all N rows kept).  The adjoint
    // right-hand sides W_L o conj(g_j) do depend on E: those solves run in the
    // per-energy core, energy by energy.  The block width is capped so that
    // the forward columns of all energies take at most 8 GiB.
    const size_t per_col = (size_t)n_e * (size_t)N * sizeof(double2);
    const int wcap = (int)std::max<size_t>(1, ((size_t)8 << 30) / per_col);
    const int wmax = std::min(d.block_width ? d.block_width : 32, wcap);
    // adjoint solves of a block run in batches of up to kAdj (column, energy)
    // items across energies: the per-energy core gives each item its own shift
    constexpr int kAdj = 64;
    double *d_field, *d_colw, *d_roww, *d_t, *d_fw;
    double2 *d_gall, *d_rhs;
    CHK(ws(op, WS_ROWS, (size_t)N, &d_field));
    CHK(ws(op, WS_ROWW, (size_t)sd.n_rows, &d_roww));
    // per item: T weight 4 W_R,j, t_j(E), field weight 4 W_R,j w_E
    CHK(ws(op, WS_TCOL, (size_t)3 * n_e * wmax, &d_colw));
    d_t = d_colw + (size_t)n_e * wmax;
    d_fw = d_t + (size_t)n_e * wmax;
    CHK(ws(op, WS_GAMMA, (size_t)n_e * wmax * N, &d_gall));
    CHK(ws(op, WS_TRI, (size_t)kAdj * N, &d_rhs));
    HIPCHK(hipMemsetAsync(d_field, 0, N * sizeof(double), s));
    HIPCHK(hipMemcpyAsync(d_roww, sd.roww.data(), sd.n_rows * sizeof(double), hipMemcpyHostToDevice, s));
    int64_t total_iters = 0;
    int n_bad = 0, n_break = 0;
    std::vector<double> ie, colw, fw, tb, T_acc(n_e, 0.0), f_res;
    std::vector<int> f_st;
    Defaults d64 = d;
    d64.precision = NEGF_FP64;
    bool any_e = false;
    for (int e = 0; e < n_e; ++e) any_e = any_e || weights[e] != 0.0 || T;
    for (int c0 = 0; c0 < n_cols && any_e; c0 += wmax) {
        const int w = std::min(wmax, n_cols - c0);
        const int n_it = n_e * w;  // items (e, c), e-major: the layout of d_gall
        colw.resize(n_it);
        fw.resize(n_it);
        for (int e = 0; e < n_e; ++e)
            for (int c = 0; c < w; ++c) {
                colw[(size_t)e * w + c] = sd.colw[c0 + c];
                fw[(size_t)e * w + c] = sd.colw[c0 + c] * weights[e];
            }
        HIPCHK(hipMemcpyAsync(d_colw, colw.data(), n_it * sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(d_fw, fw.data(), n_it * sizeof(double), hipMemcpyHostToDevice, s));
        // forward: g[e][c][:] for every energy, one multi-shift run
        f_st.assign(w, 0);
        f_res.assign((size_t)w * n_e, 0.0);
        MSOut mo;
        mo.d_out = d_gall;
        mo.out_col_stride = N;
        mo.out_shift_stride = (int64_t)w * N;
        mo.h_status = f_st.data();
        mo.h_resid = f_res.data();
        CHK(run_multishift_block(op, d64, w, w, sd.cols.data() + c0, nullptr, energies, n_e,
                                 nullptr, 0, (int)N, nullptr, nullptr, mo, &total_iters, s, &tm));
        for (int e = 0; e < n_e; ++e) {
            if (weights[e] == 0.0 && !T) continue;
            for (int c = 0; c < w; ++c) {
                const int fs = ms_item_status(f_res[(size_t)c * n_e + e], f_st[c], d.tol);
                if (fs == NEGF_ITEM_BREAKDOWN) ++n_break;
                else if (fs != NEGF_ITEM_CONVERGED) ++n_bad;
            }
        }
        // t_j(E) of every item at once
        tb.assign(n_it, 0.0);
        launch_weighted_norm(d_gall, N, n_it, sd.row0, sd.n_rows, d_roww, d_colw, d_t, s);
        HIPCHK(hipMemcpyAsync(tb.data(), d_t, n_it * sizeof(double), hipMemcpyDeviceToHost, s));
        // adjoint right-hand sides W_L o conj(g_j), solved with the same operator,
        // over runs of items whose energy has a nonzero weight
        for (int it0 = 0; it0 < n_it;) {
            if (weights[it0 / w] == 0.0) {
                ++it0;
                continue;
            }
            int nb = 1;
            while (nb < kAdj && it0 + nb < n_it && weights[(it0 + nb) / w] != 0.0) ++nb;
            double2* d_g = d_gall + (size_t)it0 * N;
            launch_adjoint_rhs(d_g, N, plane, nb, op->d_wl, d_rhs, s);
            ie.resize(nb);
            for (int b = 0; b < nb; ++b) ie[b] = energies[(it0 + b) / w];
            std::vector<int> st2(nb, 0);
            PEOut po;
            po.h_status = st2.data();
            CHK(run_per_energy(op, d64, nb, nullptr, d_rhs, ie.data(), po, &total_iters, s, &tm));
            double2* x64 = (double2*)op->bufs[WS_X64].ptr;
            // 8 Re sum_j W_R,j w_E g_j lambda_j = 2 Re sum_j (4 W_R,j w_E) g_j lambda_j
            launch_field(d_g, x64, N, nb, d_fw + it0, 2.0, d_field, s);
            for (int b = 0; b < nb; ++b) {
                if (st2[b] == NEGF_ITEM_BREAKDOWN) ++n_break;
                else if (st2[b] != NEGF_ITEM_CONVERGED) ++n_bad;
            }
            it0 += nb;
        }
        HIPCHK(hipStreamSynchronize(s));
        for (int e = 0; e < n_e; ++e)
            for (int c = 0; c < w; ++c) T_acc[e] += tb[(size_t)e * w + c];
    }
    if (T)
        for (int e = 0; e < n_e; ++e) T[e] = T_acc[e];
    HIPCHK(hipMemcpyAsync(dL_dV, d_field, N * sizeof(double),
                          is_device_ptr(dL_dV) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return final_status(n_bad, n_break);
}

extern "C" negf_status negf_transmission_grad(negf_op* op, const negf_opts* opts, int32_t n_e,
                                              const double* energies, const double* weights,
                                              double* dL_dV, double* T) {
    g_last_error.clear();
    (void)hipGetLastError();
    if (!op) {
        set_error("null op");
        return NEGF_E_INVALID_ARG;
    }
    return grad_impl(op, opts, n_e, energies, weights, dL_dV, T);
}

// ---------------------------------------------------------------------------
// negf_transmission_batch
// ---------------------------------------------------------------------------

static void release_workspace(negf_op* op) {
    (void)hipStreamSynchronize(op->own_stream);
    (void)hipStreamSynchronize(op->side_stream);
    for (auto& b : op->bufs) {
        dev_free(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
    }
}

// ---------------------------------------------------------------------------
// negf_tune: pick the multi-shift launch shape by timing short probe runs
// ---------------------------------------------------------------------------
// device bytes of run_multishift_block's workspace for a block of w columns
static double multishift_bytes(const negf_op* op, int w, int ng, int n_rows, int max_iter) {
    const double N = (double)op->N, ch = shift_chunk(op), z = sizeof(double2);
    const double vec = 4.0 * w * N * z;                             // r, p (x2), q
    const double ring = 2.0 * ch * w * n_rows * z;
    const double xp = 2.0 * w * (double)ng * n_rows * z;
    const double coef = (2.0 * ch + 4.0) * w * ng * z;
    const double state = (double)w * max_iter * (2.0 * z + 8.0) + 3.0 * w * ch * ng * z;
    return vec + ring + xp + coef + state;
}

static negf_status tune_impl(negf_op* op, const negf_opts* opts, int32_t n_e,
                             const double* energies, int32_t probe_iters,
                             negf_tune_result* result) {
    Defaults d;
    CHK(read_opts(opts, &d));
    CHK(check_energies(n_e, energies));
    if (probe_iters < 0) {
        set_error("probe_iters must be >= 0");
        return NEGF_E_INVALID_ARG;
    }
    HIPCHK(hipSetDevice(op->device));
    hipStream_t s = pick_stream(op, opts);
    Sides sd;
    make_sides(op, d.direction, &sd);
    const int n_cols = (int)sd.cols.size();
    const int ng = d.shift_group ? std::min(d.shift_group, n_e) : n_e;
    Defaults dp = d;
    dp.max_iter = probe_iters ? probe_iters : shift_chunk(op);

    // widths whose multi-shift workspace (at the caller's max_iter) fits in
    // half of the free device memory
    size_t mem_free = 0, mem_total = 0;
    HIPCHK(hipMemGetInfo(&mem_free, &mem_total));
    auto fits = [&](int w) {
        const double b = multishift_bytes(op, w, ng, sd.n_rows, d.max_iter);
        return b <= 0.5 * (double)mem_free;
    };
    std::vector<int> widths;
    if (d.block_width) {
        widths.push_back(std::min(d.block_width, n_cols));
    } else {
        for (int w : {16, 32, 64, 128, 256})
            if (w <= n_cols && fits(w)) widths.push_back(w);
        if (widths.empty()) widths.push_back(std::min(16, n_cols));
    }
    const int pts = op->nx * op->ny;
    const bool plane_ok = pts <= 1024;
    std::vector<int> kernels = plane_ok ? std::vector<int>{1, 0} : std::vector<int>{0};
    struct Cand { int w, target, plane; double us; };
    std::vector<Cand> cands;
    for (int w : widths)
        for (int k : kernels)
            for (int t : {128, 192, 256, 512, 1024}) cands.push_back({w, t, k, 0.0});
    if ((int)cands.size() > NEGF_TUNE_MAX) cands.resize(NEGF_TUNE_MAX);

    double* d_roww = nullptr;
    CHK(ws(op, WS_ROWW, (size_t)sd.n_rows, &d_roww));
    HIPCHK(hipMemcpyAsync(d_roww, sd.roww.data(), sd.n_rows * sizeof(double), hipMemcpyHostToDevice, s));
    MatvecTimer tm;
    CHK(tm.init(false));
    const int saved_w = op->tuned_w, saved_t = op->wg_target, saved_k = op->plane_kernel;
    auto probe = [&](const Cand& c, double* us) -> negf_status {
        op->wg_target = c.target;
        op->plane_kernel = c.plane;
        MSOut mo;  // nothing copied out
        int64_t total = 0;
        HIPCHK(hipStreamSynchronize(s));
        const auto t0 = std::chrono::steady_clock::now();
        CHK(run_multishift_block(op, dp, c.w, c.w, sd.cols.data(), nullptr, energies, ng, nullptr,
                                 sd.row0, sd.n_rows, d_roww, sd.colw.data(), mo, &total, s, &tm));
        HIPCHK(hipStreamSynchronize(s));
        const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *us = 1e6 * sec / (double)std::max<int64_t>(1, total);
        return NEGF_OK;
    };
    negf_status st = NEGF_OK;
    double warm = 0.0;
    st = probe(cands[0], &warm);  // first use allocates the workspace and loads code
    for (size_t i = 0; st == NEGF_OK && i < cands.size(); ++i) st = probe(cands[i], &cands[i].us);
    if (st != NEGF_OK) {
        op->tuned_w = saved_w;
        op->wg_target = saved_t;
        op->plane_kernel = saved_k;
        return st;
    }
    size_t best = 0;
    for (size_t i = 1; i < cands.size(); ++i)
        if (cands[i].us < cands[best].us) best = i;
    op->tuned_w = cands[best].w;
    op->wg_target = cands[best].target;
    op->plane_kernel = cands[best].plane;
    release_workspace(op);  // the probes sized it for the widest candidate
    if (result) {
        result->block_width = cands[best].w;
        result->wg_target = cands[best].target;
        result->plane_kernel = cands[best].plane;
        result->n_tried = (int32_t)cands.size();
        for (size_t i = 0; i < cands.size(); ++i) {
            result->tried_block_width[i] = cands[i].w;
            result->tried_wg_target[i] = cands[i].target;
            result->tried_plane_kernel[i] = cands[i].plane;
            result->us_per_column_iteration[i] = cands[i].us;
        }
    }
    return NEGF_OK;
}

extern "C" negf_status negf_tune(negf_op* op, const negf_opts* opts, int32_t n_e,
                                 const double* energies, int32_t probe_iters,
                                 negf_tune_result* result) {
    (void)hipGetLastError();  // a stale error of an earlier call must not fail this one
    if (!op) {
        set_error("null op");
        return NEGF_E_INVALID_ARG;
    }
    return tune_impl(op, opts, n_e, energies, probe_iters, result);
}

// the cache key of a tuning request (no " => " inside: that separates the value)
static std::string tune_key(const negf_op* op, const Defaults& d, int n_e, int probe_iters) {
    Sides sd;
    make_sides(op, d.direction, &sd);
    const int ng = d.shift_group ? std::min(d.shift_group, n_e) : n_e;
    hipDeviceProp_t prop;
    std::memset(&prop, 0, sizeof prop);
    (void)hipGetDeviceProperties(&prop, op->device);
    char buf[640];
    std::snprintf(buf, sizeof buf,
                  "%s|%s|cu%d|grid%dx%dx%d|R%d|proj%d|cols%zu|rows%d|ng%d|bw%d|probe%d",
                  negf_version(), prop.gcnArchName, prop.multiProcessorCount, op->nx, op->ny,
                  op->nz, op->R, op->kb.n_proj, sd.cols.size(), sd.n_rows, ng, d.block_width,
                  probe_iters);
    return buf;
}

extern "C" negf_status negf_tune_cached(negf_op* op, const negf_opts* opts, int32_t n_e,
                                        const double* energies, int32_t probe_iters,
                                        const char* cache_path, negf_tune_result* result) {
    (void)hipGetLastError();  // a stale error of an earlier call must not fail this one
    if (!op) {
        set_error("null op");
        return NEGF_E_INVALID_ARG;
    }
    if (!cache_path || !cache_path[0]) {
        set_error("null or empty cache path");
        return NEGF_E_INVALID_ARG;
    }
    Defaults d;
    CHK(read_opts(opts, &d));
    CHK(check_energies(n_e, energies));
    if (probe_iters < 0) {
        set_error("probe_iters must be >= 0");
        return NEGF_E_INVALID_ARG;
    }
    const std::string key = tune_key(op, d, n_e, probe_iters);
    int bw = 0, tg = 0, pk = 0;
    double us = 0.0;
    bool hit = false;
    if (FILE* f = std::fopen(cache_path, "r")) {
        char line[1024];
        while (std::fgets(line, sizeof line, f)) {
            const char* sep = std::strstr(line, " => ");
            if (!sep || (size_t)(sep - line) != key.size() ||
                std::strncmp(line, key.c_str(), key.size()) != 0)
                continue;
            int a = 0, b = 0, c = 0;
            double u = 0.0;
            if (std::sscanf(sep + 4, "%d %d %d %lf", &a, &b, &c, &u) == 4 && a > 0 && b > 0 &&
                (c == 0 || c == 1)) {
                bw = a;
                tg = b;
                pk = c;
                us = u;
                hit = true;  // the last line for the key wins
            }
        }
        std::fclose(f);
    }
    if (hit) {
        CHK(negf_set_launch_shape(op, bw, tg, pk));
        if (result) {
            std::memset(result, 0, sizeof *result);
            result->block_width = bw;
            result->wg_target = tg;
            result->plane_kernel = pk;
            result->n_tried = 0;
            result->us_per_column_iteration[0] = us;
        }
        return NEGF_OK;
    }
    negf_tune_result local;
    negf_tune_result* r = result ? result : &local;
    CHK(tune_impl(op, opts, n_e, energies, probe_iters, r));
    double best = 0.0;
    for (int i = 0; i < r->n_tried; ++i)
        if (r->tried_block_width[i] == r->block_width && r->tried_wg_target[i] == r->wg_target &&
            r->tried_plane_kernel[i] == r->plane_kernel)
            best = r->us_per_column_iteration[i];
    if (FILE* f = std::fopen(cache_path, "a")) {
        std::fprintf(f, "%s => %d %d %d %.6g\n", key.c_str(), r->block_width, r->wg_target,
                     r->plane_kernel, best);
        std::fclose(f);
    }
    return NEGF_OK;
}

void launch_landauer(const double* e, const double* t, int n_e, const double* bias, int n_bias,
                     double e_fermi, double kt, double* out, hipStream_t s);

// ---------------------------------------------------------------------------
// negf_current: Landauer current (Eq. 1)
// ---------------------------------------------------------------------------
extern "C" negf_status negf_current(int32_t n_e, const double* energies, const double* T,
                                    int32_t n_bias, const double* bias, double e_fermi, double kT,
                                    double* current, void* stream) {
    (void)hipGetLastError();  // a stale error of an earlier call must not fail this one
    if (n_e < 2 || n_bias < 1 || !energies || !T || !bias || !current) {
        set_error("negf_current needs n_e >= 2, n_bias >= 1 and non-null arrays");
        return NEGF_E_INVALID_ARG;
    }
    if (!(kT >= 0.0) || !std::isfinite(kT) || !std::isfinite(e_fermi)) {
        set_error("kT must be finite and >= 0, e_fermi finite");
        return NEGF_E_INVALID_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    // host copies of the inputs (validated here), whatever side they live on
    std::vector<double> he(n_e), ht(n_e), hb(n_bias);
    auto fetch = [&](const double* src, double* dst, size_t n) -> negf_status {
        if (is_device_ptr(src)) {
            HIPCHK(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        } else {
            std::memcpy(dst, src, n * sizeof(double));
        }
        return NEGF_OK;
    };
    CHK(fetch(energies, he.data(), n_e));
    CHK(fetch(T, ht.data(), n_e));
    CHK(fetch(bias, hb.data(), n_bias));
    for (int i = 0; i < n_e; ++i) {
        if (!std::isfinite(he[i]) || !std::isfinite(ht[i]) || (i > 0 && !(he[i] > he[i - 1]))) {
            set_error("energies must be finite and strictly increasing, T finite (index %d)", i);
            return NEGF_E_INVALID_ARG;
        }
    }
    for (int b = 0; b < n_bias; ++b) {
        if (!std::isfinite(hb[b])) {
            set_error("bias %d not finite", b);
            return NEGF_E_INVALID_ARG;
        }
    }
    double* buf = nullptr;
    const size_t n_buf = 2 * (size_t)n_e + 2 * (size_t)n_bias;
    CHK(dev_alloc((void**)&buf, n_buf * sizeof(double)));
    double *de = buf, *dt = buf + n_e, *db = buf + 2 * n_e, *dout = db + n_bias;
    negf_status st = NEGF_OK;
    auto run = [&]() -> negf_status {
        HIPCHK(hipMemcpyAsync(de, he.data(), n_e * sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(dt, ht.data(), n_e * sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(db, hb.data(), n_bias * sizeof(double), hipMemcpyHostToDevice, s));
        launch_landauer(de, dt, n_e, db, n_bias, e_fermi, kT, dout, s);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(current, dout, n_bias * sizeof(double), hipMemcpyDefault, s));
        HIPCHK(hipStreamSynchronize(s));
        return NEGF_OK;
    };
    st = run();
    dev_free(buf);
    return st;
}

void launch_gram(const double2* U, int64_t N, const int* sel, int n_r, int64_t row0, int n_rows,
                 const double* d, const double2* prev, double2* out, hipStream_t s);
int eq13_tiles(int n_r);
void launch_eq13(const double2* M, int n_r, const double2* eps, const double* energies, int n_e,
                 double* part, double* T, hipStream_t s);

// ---------------------------------------------------------------------------
// negf_spectral_transmission: Eqs. 8-13 from caller-supplied eigenpairs
// ---------------------------------------------------------------------------
static negf_status spectral_impl(negf_op* op, int32_t n_r, const negf_c64* eps,
                                 const negf_c64* U, double keep, int32_t n_e,
                                 const double* energies, double* T) {
    if (n_r < 1 || !eps || !U || !T) {
        set_error("need n_r >= 1, eps, U and T");
        return NEGF_E_INVALID_ARG;
    }
    if (!(keep >= 0.0 && keep <= 1.0)) {
        set_error("keep must lie in [0, 1]");
        return NEGF_E_INVALID_ARG;
    }
    CHK(check_energies(n_e, energies));
    for (int i = 0; i < n_r; ++i) {
        if (!std::isfinite(eps[i].re) || !std::isfinite(eps[i].im)) {
            set_error("eigenvalue %d not finite", i);
            return NEGF_E_INVALID_ARG;
        }
    }
    // the kept eigenpairs: all, or those nearest the middle of the window
    double emin = energies[0], emax = energies[0];
    for (int e = 0; e < n_e; ++e) {
        emin = std::min(emin, energies[e]);
        emax = std::max(emax, energies[e]);
    }
    std::vector<int> sel(n_r);
    for (int i = 0; i < n_r; ++i) sel[i] = i;
    int n_keep = n_r;
    if (keep > 0.0 && keep < 1.0) {
        const double mid = 0.5 * (emin + emax);
        std::stable_sort(sel.begin(), sel.end(), [&](int a, int b) {
            return std::fabs(eps[a].re - mid) < std::fabs(eps[b].re - mid);
        });
        n_keep = std::max(1, (int)std::lround(keep * n_r));
        sel.resize(n_keep);
    }
    std::vector<double2> eps_k(n_keep);
    for (int i = 0; i < n_keep; ++i) {
        eps_k[i] = make_double2(eps[sel[i]].re, eps[sel[i]].im);
        for (int e = 0; e < n_e; ++e) {
            if (energies[e] == eps_k[i].x && eps_k[i].y == 0.0) {
                set_error("energy %d coincides with eigenvalue %d", e, sel[i]);
                return NEGF_E_INVALID_ARG;
            }
        }
    }
    HIPCHK(hipSetDevice(op->device));
    hipStream_t s = op->own_stream;
    const int64_t N = op->N, plane = (int64_t)op->nx * op->ny;
    const int64_t rowL = (int64_t)op->zl0 * plane, rowR = (int64_t)op->zr0 * plane;
    const int nL = (int)((op->zl1 - op->zl0) * plane), nR = (int)((op->zr1 - op->zr0) * plane);
    std::vector<double> dL(nL), dR(nR);
    for (int r = 0; r < nL; ++r) dL[r] = 2.0 * op->cap_l[op->zl0 + r / plane];
    for (int r = 0; r < nR; ++r) dR[r] = 2.0 * op->cap_r[op->zr0 + r / plane];
    // device buffers: one allocation, freed on return
    const size_t b_u = is_device_ptr(U) ? 0 : (size_t)n_r * N * sizeof(double2);
    const size_t b_m = (size_t)n_keep * n_keep * sizeof(double2);
    const size_t b_eps = (size_t)n_keep * sizeof(double2);
    const size_t b_sel = ((size_t)n_keep * sizeof(int) + 255) & ~(size_t)255;
    const size_t b_d = (size_t)(nL + nR) * sizeof(double);
    const size_t b_e = (size_t)n_e * sizeof(double) * (2 + eq13_tiles(n_keep));
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char* base = nullptr;
    CHK(dev_alloc((void**)&base, al(b_u) + al(b_m) + al(b_eps) + al(b_sel) + al(b_d) + al(b_e)));
    size_t off = 0;
    auto take = [&](size_t b) { char* p = base + off; off += al(b); return p; };
    double2* d_u = b_u ? (double2*)take(b_u) : (double2*)U;
    double2* d_m = (double2*)take(b_m);
    double2* d_eps = (double2*)take(b_eps);
    int* d_sel = (int*)take(b_sel);
    double* d_d = (double*)take(b_d);
    double* d_e = (double*)take(b_e);
    double* d_t = d_e + n_e;
    double* d_part = d_t + n_e;
    auto run = [&]() -> negf_status {
        if (b_u)
            HIPCHK(hipMemcpyAsync(d_u, U, b_u, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(d_eps, eps_k.data(), b_eps, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(d_sel, sel.data(), n_keep * sizeof(int), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(d_d, dL.data(), nL * sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(d_d + nL, dR.data(), nR * sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(d_e, energies, n_e * sizeof(double), hipMemcpyHostToDevice, s));
        // M = (U^H Gamma_L U) o (U^H Gamma_R U), then T(E) = Re(a^H M a)
        launch_gram(d_u, N, d_sel, n_keep, rowL, nL, d_d, nullptr, d_m, s);
        launch_gram(d_u, N, d_sel, n_keep, rowR, nR, d_d + nL, d_m, d_m, s);
        launch_eq13(d_m, n_keep, d_eps, d_e, n_e, d_part, d_t, s);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(T, d_t, n_e * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return NEGF_OK;
    };
    const negf_status st = run();
    (void)hipStreamSynchronize(s);
    dev_free(base);
    return st;
}

extern "C" negf_status negf_spectral_transmission(negf_op* op, int32_t n_r, const negf_c64* eps,
                                                  const negf_c64* U, double keep, int32_t n_e,
                                                  const double* energies, double* T) {
    (void)hipGetLastError();  // a stale error of an earlier call must not fail this one
    if (!op) {
        set_error("null op");
        return NEGF_E_INVALID_ARG;
    }
    return spectral_impl(op, n_r, eps, U, keep, n_e, energies, T);
}

extern "C" negf_status negf_set_launch_shape(negf_op* op, int32_t block_width, int32_t wg_target,
                                             int32_t plane_kernel) {
    if (!op) {
        set_error("null op");
        return NEGF_E_INVALID_ARG;
    }
    if (block_width < 0 || block_width > 4096 || wg_target < 0 || wg_target > 65536 ||
        plane_kernel < -1 || plane_kernel > 1) {
        set_error("launch shape out of range (block_width %d, wg_target %d, plane_kernel %d)",
                  block_width, wg_target, plane_kernel);
        return NEGF_E_INVALID_ARG;
    }
    op->tuned_w = block_width;
    op->wg_target = wg_target;
    op->plane_kernel = plane_kernel;
    return NEGF_OK;
}

// One junction of the batch in the multi-shift core: its source columns
// stream through one block of slots (a single MultiShiftRun), which the
// batch's host thread advances chunk by chunk.
struct BatchJob {
    int index = 0;
    negf_op* op = nullptr;
    Defaults d;
    Sides sd;
    int n_e = 0;
    std::vector<double> blk_t, blk_r;
    std::vector<int> blk_it, blk_st, blk_si;
    int64_t total_iters = 0;
    MatvecTimer tm;
    std::unique_ptr<MultiShiftRun<double>> run;
};

// Whether junction i of the batch runs as one resumable multi-shift run (FP64
// multi-shift core, every energy in one shift group, streamed columns, no
// restarts); the others go through negf_transmission's own driver, one at a
// time.
static bool batch_interleaves(const Defaults& d) {
    return pick_core(d) == NEGF_CORE_MULTISHIFT && d.precision == NEGF_FP64 &&
           d.shift_group == 0 && !column_stream_disabled() && d.recover == NEGF_RECOVER_OFF;
}

static negf_status batch_job_start(BatchJob* job, const negf_opts* opts, const double* energies) {
    negf_op* op = job->op;
    CHK(read_opts(opts, &job->d));
    CHK(check_energies(job->n_e, energies));
    HIPCHK(hipSetDevice(op->device));
    make_sides(op, job->d.direction, &job->sd);
    CHK(restrict_sides(job->d, &job->sd));
    const int n_cols = (int)job->sd.cols.size();
    const int ng = job->n_e;
    const int wmax = job->d.block_width ? job->d.block_width : (op->tuned_w ? op->tuned_w : 64);
    const int w = std::min(wmax, n_cols);
    hipStream_t s = op->own_stream;
    double* d_roww = nullptr;
    CHK(ws(op, WS_ROWW, (size_t)job->sd.n_rows, &d_roww));
    HIPCHK(hipMemcpyAsync(d_roww, job->sd.roww.data(), job->sd.n_rows * sizeof(double),
                          hipMemcpyHostToDevice, s));
    job->blk_t.assign((size_t)n_cols * ng, 0.0);
    job->blk_r.assign((size_t)n_cols * ng, 0.0);
    job->blk_it.assign(n_cols, 0);
    job->blk_st.assign(n_cols, 0);
    job->blk_si.assign((size_t)n_cols * ng, 0);
    MSOut mo;
    mo.h_tcol = job->blk_t.data();
    mo.h_iters = job->blk_it.data();
    mo.h_status = job->blk_st.data();
    mo.h_resid = job->blk_r.data();
    mo.h_shift_iters = job->blk_si.data();
    CHK(job->tm.init(0));
    job->run = std::make_unique<MultiShiftRun<double>>(op, job->d, w, n_cols, job->sd.cols.data(), nullptr,
                                               energies, ng, nullptr, job->sd.row0, job->sd.n_rows,
                                               d_roww, job->sd.colw.data(), mo, &job->total_iters,
                                               s, &job->tm);
    CHK(job->run->start());
    return job->run->issue_chunk();
}

// T(E) of a finished job, reduced as negf_transmission reduces it
static negf_status batch_job_result(BatchJob* job, double* T) {
    const int n_cols = (int)job->sd.cols.size();
    const int ng = job->n_e;
    int n_bad = 0, n_break = 0;
    for (int e = 0; e < ng; ++e) {
        double acc = 0.0;
        for (int c = 0; c < n_cols; ++c) {
            const size_t o = (size_t)c * ng + e;
            acc += job->blk_t[o];
            const int st = ms_item_status(job->blk_r[o], job->blk_st[c], job->d.tol);
            if (st == NEGF_ITEM_BREAKDOWN) ++n_break;
            else if (st != NEGF_ITEM_CONVERGED) ++n_bad;
        }
        T[e] = acc;
    }
    return final_status(n_bad, n_break);
}

// col_begin / col_count: per-op source-column shards (nullable: those of opts)
static negf_status batch_impl(int32_t n_ops, negf_op* const* ops, const negf_opts* opts,
                              const int32_t* n_e, const double* const* energies,
                              const int32_t* col_begin, const int32_t* col_count,
                              double* const* T, int32_t* status, int32_t max_concurrent) {
    g_last_error.clear();
    (void)hipGetLastError();
    if (n_ops < 1 || !ops || !n_e || !energies || !T) {
        set_error("invalid batch arguments");
        return NEGF_E_INVALID_ARG;
    }
    for (int i = 0; i < n_ops; ++i) {
        if (!ops[i] || !energies[i] || !T[i] || n_e[i] < 1) {
            set_error("batch entry %d is invalid", i);
            return NEGF_E_INVALID_ARG;
        }
        for (int j = 0; j < i; ++j)
            if (ops[j] == ops[i]) {
                set_error("batch entries %d and %d share an operator", j, i);
                return NEGF_E_INVALID_ARG;
            }
    }
    if (opts && opts->stream) {
        set_error("the batch runs every junction on its operator's own stream; opts->stream must be NULL");
        return NEGF_E_INVALID_ARG;
    }
    // each junction's options: the shared ones, with its own column shard
    std::vector<negf_opts> per(n_ops);
    for (int i = 0; i < n_ops; ++i) {
        if (opts) per[i] = *opts;
        else std::memset(&per[i], 0, sizeof(negf_opts));  // all defaults
        if (col_begin) per[i].col_begin = col_begin[i];
        if (col_count) per[i].col_count = col_count[i];
        if (per[i].col_begin < 0 || per[i].col_count < 0) {
            set_error("batch entry %d: negative column range", i);
            return NEGF_E_INVALID_ARG;
        }
    }
    // largest first: work ~ points x source columns x energies
    std::vector<int> order(n_ops);
    std::vector<double> cost(n_ops);
    for (int i = 0; i < n_ops; ++i) {
        order[i] = i;
        const negf_op* op = ops[i];
        const double cols = per[i].col_count > 0 ? (double)per[i].col_count
                                                 : (double)(op->zr1 - op->zr0) * op->nx * op->ny;
        cost[i] = (double)op->N * cols * n_e[i];
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    const int n_slots = std::max(1, std::min(n_ops, max_concurrent > 0 ? max_concurrent : 4));
    int device = 0;
    HIPCHK(hipGetDevice(&device));
    std::vector<negf_status> st(n_ops, NEGF_OK);
    std::vector<std::string> msg(n_ops);
    // One host thread keeps up to n_slots junctions in flight, each on its
    // operator's own stream: it queues a junction's next chunk as soon as the
    // previous one has finished (polled with event queries, no blocking wait
    // on any one stream), so the device always holds the queued chunks of
    // every slot.  Each slot hands one set of workspace buffers from junction
    // to junction (largest first, so later ones usually fit what an earlier
    // one left): no device allocation or free in between.
    std::vector<std::vector<Buffer>> pools(n_slots, std::vector<Buffer>(WS_COUNT));
    std::vector<void*> to_free;
    std::vector<std::unique_ptr<BatchJob>> slot(n_slots);
    size_t next = 0;
    auto take_buffers = [&](int k, negf_op* op) {
        for (int sl = 0; sl < WS_COUNT; ++sl)
            if (!op->bufs[sl].ptr) std::swap(op->bufs[sl], pools[k][sl]);
    };
    auto return_buffers = [&](int k, negf_op* op) {
        (void)hipStreamSynchronize(op->own_stream);
        (void)hipStreamSynchronize(op->side_stream);
        // keep the larger buffer of each kind; the other is freed after the batch
        for (int sl = 0; sl < WS_COUNT; ++sl) {
            Buffer& b = op->bufs[sl];
            if (!b.ptr) continue;
            if (pools[k][sl].ptr && pools[k][sl].bytes >= b.bytes) {
                to_free.push_back(b.ptr);
            } else {
                if (pools[k][sl].ptr) to_free.push_back(pools[k][sl].ptr);
                pools[k][sl] = b;
            }
            b = Buffer{};
        }
        op->d_sink = nullptr;
    };
    auto end_job = [&](int k, negf_status s_job) {
        BatchJob* job = slot[k].get();
        const int i = job->index;
        if (s_job == NEGF_OK && job->run) s_job = job->run->finish();
        job->run.reset();  // drains its streams
        if (s_job == NEGF_OK) {
            s_job = batch_job_result(job, T[i]);
        }
        st[i] = s_job;
        if (s_job != NEGF_OK) msg[i] = g_last_error;
        return_buffers(k, job->op);
        slot[k].reset();
    };
    // starts the next junction in slot k; junctions that do not interleave
    // run to completion here
    auto fill = [&](int k) {
        while (next < order.size()) {
            const int i = order[next++];
            negf_op* op = ops[i];
            Defaults d;
            const negf_status s_opt = read_opts(&per[i], &d);
            take_buffers(k, op);
            if (s_opt != NEGF_OK || !batch_interleaves(d)) {
                st[i] = (s_opt != NEGF_OK) ? s_opt
                                           : transmission_impl(op, &per[i], n_e[i], energies[i], T[i], nullptr);
                if (st[i] != NEGF_OK) msg[i] = g_last_error;
                return_buffers(k, op);
                continue;
            }
            slot[k] = std::make_unique<BatchJob>();
            BatchJob* job = slot[k].get();
            job->index = i;
            job->op = op;
            job->n_e = n_e[i];
            const negf_status s_start = batch_job_start(job, &per[i], energies[i]);
            if (s_start != NEGF_OK) {
                end_job(k, s_start);
                continue;
            }
            return;
        }
    };
    for (int k = 0; k < n_slots; ++k) fill(k);
    while (true) {
        bool any = false, progressed = false;
        for (int k = 0; k < n_slots; ++k) {
            BatchJob* job = slot[k].get();
            if (!job) continue;
            any = true;
            if (!job->run->chunk_done()) continue;
            progressed = true;
            (void)hipSetDevice(job->op->device);
            bool busy = false;
            negf_status s_job = job->run->after_chunk(&busy);
            if (s_job == NEGF_OK && busy) s_job = job->run->issue_chunk();
            if (s_job != NEGF_OK || !busy) {
                end_job(k, s_job);
                fill(k);
            }
        }
        if (!any) break;
        if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    (void)hipSetDevice(device);
    (void)hipDeviceSynchronize();
    for (void* ptr : to_free) dev_free(ptr);
    for (auto& pool : pools)
        for (auto& b : pool) dev_free(b.ptr);
    negf_status first = NEGF_OK;
    for (int i = 0; i < n_ops; ++i) {
        if (status) status[i] = st[i];
        if (st[i] != NEGF_OK && first == NEGF_OK) {
            first = st[i];
            set_error("junction %d: %s", i, msg[i].c_str());
        }
    }
    return first;
}

extern "C" negf_status negf_transmission_batch(int32_t n_ops, negf_op* const* ops,
                                               const negf_opts* opts, const int32_t* n_e,
                                               const double* const* energies, double* const* T,
                                               int32_t* status, int32_t max_concurrent) {
    return batch_impl(n_ops, ops, opts, n_e, energies, nullptr, nullptr, T, status,
                      max_concurrent);
}

extern "C" negf_status negf_transmission_batch_shards(int32_t n_ops, negf_op* const* ops,
                                                      const negf_opts* opts, const int32_t* n_e,
                                                      const double* const* energies,
                                                      const int32_t* col_begin,
                                                      const int32_t* col_count, double* const* T,
                                                      int32_t* status, int32_t max_concurrent) {
    if (!col_begin || !col_count) {
        g_last_error.clear();
        set_error("null col_begin or col_count");
        return NEGF_E_INVALID_ARG;
    }
    return batch_impl(n_ops, ops, opts, n_e, energies, col_begin, col_count, T, status,
                      max_concurrent);
}
