// Landauer current from T(E) (Eq. 1).
//
// I(V) = (2e/h) int T(E) [f(E - mu_L) - f(E - mu_R)] dE, mu_{L,R} = E_F +- V/2,
// with f the Fermi function at temperature kT (a step with f(0) = 1/2 at
// kT = 0).  Atomic units (e = hbar = 1) make 2e/h = 1/pi.  The integral is the
// trapezoid rule on the energy grid of T, which need not be uniform.
#include "negf_internal.h"

namespace {

constexpr int kT = 256;

__device__ inline double fermi(double x, double kt) {
    if (kt == 0.0) return (x < 0.0) ? 1.0 : ((x > 0.0) ? 0.0 : 0.5);
    return 0.5 * (1.0 - tanh(0.5 * x / kt));
}

// one work-group per bias point; panels reduced in a fixed order
__global__ __launch_bounds__(kT) void k_landauer(const double* __restrict__ e,
                                                 const double* __restrict__ t, int n_e,
                                                 const double* __restrict__ bias, double e_fermi,
                                                 double kt, double* __restrict__ out) {
    __shared__ double lds[kT / 64];
    const double v = bias[blockIdx.x];
    const double mu_l = e_fermi + 0.5 * v, mu_r = e_fermi - 0.5 * v;
    double s = 0.0;
    for (int i = threadIdx.x; i + 1 < n_e; i += kT) {
        const double g0 = t[i] * (fermi(e[i] - mu_l, kt) - fermi(e[i] - mu_r, kt));
        const double g1 = t[i + 1] * (fermi(e[i + 1] - mu_l, kt) - fermi(e[i + 1] - mu_r, kt));
        s += 0.5 * (e[i + 1] - e[i]) * (g0 + g1);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (threadIdx.x % 64 == 0) lds[threadIdx.x / 64] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int wv = 0; wv < kT / 64; ++wv) tot += lds[wv];
        out[blockIdx.x] = tot / M_PI;
    }
}

}  // namespace

void launch_landauer(const double* e, const double* t, int n_e, const double* bias, int n_bias,
                     double e_fermi, double kt, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_landauer, dim3(n_bias), dim3(kT), 0, s, e, t, n_e, bias, e_fermi, kt,
                       out);
}
