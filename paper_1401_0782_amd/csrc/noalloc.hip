// Operator apply that allocates no device memory, for callers that cannot:
// code running under HIP graph capture, tight serving loops, and harnesses
// that forbid allocation after start-up.
//
// It runs the kernels of negf_apply_operator (stencil, potential, absorbing
// potential, projector gather and scatter) directly from x to y.  Their
// scratch data, the shifts and the projector coefficients c = B^T x, live in
// `scratch`, a fixed device array of this file (each GPU that runs the
// library holds its own copy until the process ends).  Host code never uses
// the array's name as an address: the device address of each GPU's copy is
// taken once with hipGetSymbolAddress, on that GPU, and passed to the kernels.
#include <algorithm>
#include <mutex>

#include "negf_internal.h"

static __device__ __align__(256) unsigned char scratch[NEGF_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the device address of the current device's copy of scratch (set up on the
// first call on each device)
negf_status scratch_address(int dev, void** out) {
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d outside the %d devices the scratch table covers", dev, kMaxDevices);
        return NEGF_E_DEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_error("hipGetSymbolAddress of the scratch array failed on device %d: %s", dev,
                      hipGetErrorString(e));
            return NEGF_E_DEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return NEGF_OK;
}

bool device_pointer(const void* p) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

extern "C" negf_status negf_apply_operator_noalloc(negf_op* op, int32_t n_vec,
                                                   const double* shifts, const negf_c64* x,
                                                   negf_c64* y, void* stream) {
    (void)hipGetLastError();  // a stale error of an earlier call must not fail this one
    if (!op || !shifts || !x || !y || n_vec < 1) {
        set_error("invalid argument to negf_apply_operator_noalloc");
        return NEGF_E_INVALID_ARG;
    }
    const size_t shift_bytes = round256((size_t)n_vec * sizeof(double));
    const size_t kbc_bytes = (size_t)n_vec * (size_t)std::max(1, op->kb.n_proj) * sizeof(double2);
    if (shift_bytes + kbc_bytes > (size_t)NEGF_NOALLOC_SCRATCH_BYTES) {
        set_error("negf_apply_operator_noalloc: %d vectors x %d projectors need %zu bytes of "
                  "scratch, more than the %d available", n_vec, op->kb.n_proj,
                  shift_bytes + kbc_bytes, NEGF_NOALLOC_SCRATCH_BYTES);
        return NEGF_E_INVALID_ARG;
    }
    HIPCHK(hipSetDevice(op->device));
    const size_t vec_bytes = (size_t)n_vec * (size_t)op->N * sizeof(double2);
    const char* xb = reinterpret_cast<const char*>(x);
    const char* yb = reinterpret_cast<const char*>(y);
    if (xb < yb + vec_bytes && yb < xb + vec_bytes) {
        set_error("negf_apply_operator_noalloc: x and y overlap");
        return NEGF_E_INVALID_ARG;
    }
    if (!device_pointer(x) || !device_pointer(y)) {
        set_error("negf_apply_operator_noalloc: x and y must be device memory");
        return NEGF_E_INVALID_ARG;
    }
    void* base = nullptr;
    {
        const negf_status st = scratch_address(op->device, &base);
        if (st != NEGF_OK) return st;
    }
    hipStream_t s = stream ? (hipStream_t)stream : op->own_stream;
    double* d_shift = static_cast<double*>(base);
    double2* d_kbc = reinterpret_cast<double2*>(static_cast<char*>(base) + shift_bytes);
    const double* sh = shifts;
    if (!device_pointer(shifts)) {
        HIPCHK(hipMemcpyAsync(d_shift, shifts, (size_t)n_vec * sizeof(double),
                              hipMemcpyHostToDevice, s));
        sh = d_shift;
    }
    // every projector coefficient the scatter reads is written by the gather
    // of the same call, so nothing in scratch needs clearing
    launch_apply<double>(op, reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y),
                         n_vec, sh, nullptr, d_kbc, s);
    HIPCHK(hipGetLastError());
    if (!stream) HIPCHK(hipStreamSynchronize(s));
    return NEGF_OK;
}
