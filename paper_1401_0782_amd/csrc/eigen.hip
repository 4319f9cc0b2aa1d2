// Eigenpairs of the open-system operator H_op = H - i(W_L + W_R) near an
// energy window (Sec. II.C, Eq. 8), for the spectral route of Eqs. 9-13.
//
// H_op is complex symmetric (Eq. 6), so its right eigenvectors are complex
// orthogonal and can be normalised to U_i^T U_i = 1 (Eqs. 9-11).  The same
// symmetry gives a Lanczos process in the bilinear form u^T v (no
// conjugation): with v_0^T v_0 = 1,
//     beta_k v_{k+1} = H_op v_k - alpha_k v_k - beta_{k-1} v_{k-1},
//     alpha_k = v_k^T H_op v_k,  beta_k = (w^T w)^{1/2},
// and V_K^T H_op V_K = T_K, a complex symmetric tridiagonal matrix whose
// eigenpairs (theta, y) give Ritz pairs (theta, V_K y).  The paper found
// complex-symmetric Lanczos less stable than the Arnoldi process of ARPACK
// (duplicated or missed eigenpairs, from the loss of orthogonality); here
// every new vector is re-orthogonalised against all earlier ones, twice, in
// the bilinear form, which is what the Arnoldi process does.  The spectrum's
// low end, where the transport window lies, converges first.
//
// Device: the operator apply of stencil.hip, the bilinear Gram-Schmidt
// passes (dots against all kept vectors, then one multi-vector update), the
// Ritz vectors V_K Y and their true residuals.  Host: the eigenvalues of T_K
// (implicit QL with complex orthogonal rotations, O(K^2)) and the vectors y
// by inverse iteration on T_K - theta (O(K) each).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "negf_internal.h"

namespace {

constexpr int kT = 256;
using cd = std::complex<double>;

__device__ inline double2 cmul_d(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// deterministic pseudo-random start vector (splitmix64 of seed and index)
__device__ inline uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(kT) void k_rand_vec(double2* __restrict__ v, int64_t N, uint64_t seed) {
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kT) {
        const uint64_t a = mix64(seed ^ (2 * (uint64_t)i)), b = mix64(seed ^ (2 * (uint64_t)i + 1));
        v[i] = make_double2((double)(a >> 11) * 0x1.0p-52 - 1.0, (double)(b >> 11) * 0x1.0p-52 - 1.0);
    }
}

template <int NV>
__device__ inline void block_sum(double (&v)[NV], double* lds) {
#pragma unroll
    for (int j = 0; j < NV; ++j)
        for (int o = 32; o > 0; o >>= 1) v[j] += __shfl_xor(v[j], o, 64);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0)
        for (int j = 0; j < NV; ++j) lds[wave * NV + j] = v[j];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < kT / 64; ++w)
            for (int j = 0; j < NV; ++j) v[j] += lds[w * NV + j];
    __syncthreads();
}

// part[j][b] = partial of V_j^T w (bilinear) over the b-th slice; with
// w == nullptr, of V_j^T V_j together with ||V_j||^2 (third value)
__global__ __launch_bounds__(kT) void k_bidot(const double2* __restrict__ V, int64_t N,
                                              const double2* __restrict__ w,
                                              double* __restrict__ part) {
    __shared__ double lds[3 * kT / 64];
    const int j = blockIdx.y;
    const double2* vj = V + (int64_t)j * N;
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kT) {
        const double2 a = vj[i];
        const double2 b = w ? w[i] : a;
        s[0] += a.x * b.x - a.y * b.y;
        s[1] += a.x * b.y + a.y * b.x;
        s[2] += a.x * a.x + a.y * a.y;
    }
    block_sum<3>(s, lds);
    if (threadIdx.x == 0) {
        double* o = part + ((int64_t)j * gridDim.x + blockIdx.x) * 3;
        o[0] = s[0];
        o[1] = s[1];
        o[2] = s[2];
    }
}

// out[j] = (sum of the nblk partials of j), fixed order
__global__ __launch_bounds__(kT) void k_bidot_reduce(const double* __restrict__ part, int nblk,
                                                     double* __restrict__ out) {
    __shared__ double lds[3 * kT / 64];
    const int j = blockIdx.x;
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += kT)
        for (int t = 0; t < 3; ++t) s[t] += part[((int64_t)j * nblk + b) * 3 + t];
    block_sum<3>(s, lds);
    if (threadIdx.x == 0)
        for (int t = 0; t < 3; ++t) out[(int64_t)j * 3 + t] = s[t];
}

// w -= sum_{j < nv} c_j V_j   (c: [nv] complex as 3 doubles each: re, im, unused)
__global__ __launch_bounds__(kT) void k_axpy_multi(double2* __restrict__ w,
                                                   const double2* __restrict__ V, int nv,
                                                   const double* __restrict__ c, int64_t N) {
    __shared__ double2 cs[kT];
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    double ax = 0.0, ay = 0.0;
    for (int j0 = 0; j0 < nv; j0 += kT) {
        const int nj = min(kT, nv - j0);
        __syncthreads();
        if ((int)threadIdx.x < nj)
            cs[threadIdx.x] = make_double2(c[(int64_t)(j0 + threadIdx.x) * 3],
                                           c[(int64_t)(j0 + threadIdx.x) * 3 + 1]);
        __syncthreads();
        if (i < N) {
            for (int jj = 0; jj < nj; ++jj) {
                const double2 v = V[(int64_t)(j0 + jj) * N + i];
                const double2 cc = cs[jj];
                ax += v.x * cc.x - v.y * cc.y;
                ay += v.x * cc.y + v.y * cc.x;
            }
        }
    }
    if (i < N) {
        double2 o = w[i];
        o.x -= ax;
        o.y -= ay;
        w[i] = o;
    }
}

// w = -y - beta v_prev   (y = A(0) v_k = -H_op v_k)
__global__ __launch_bounds__(kT) void k_lanczos_w(double2* __restrict__ w,
                                                  const double2* __restrict__ y,
                                                  const double2* __restrict__ vprev, double2 beta,
                                                  int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kT) {
        const double2 a = y[i];
        double2 o = make_double2(-a.x, -a.y);
        if (vprev) {
            const double2 b = cmul_d(beta, vprev[i]);
            o.x -= b.x;
            o.y -= b.y;
        }
        w[i] = o;
    }
}

// dst = w * f
__global__ __launch_bounds__(kT) void k_scale_to(double2* __restrict__ dst,
                                                 const double2* __restrict__ w, double2 f,
                                                 int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kT)
        dst[i] = cmul_d(w[i], f);
}

// U[p][i] = sum_{j < K} V[j][i] Y[j][p]
__global__ __launch_bounds__(kT) void k_ritz(const double2* __restrict__ V, int K,
                                             const double2* __restrict__ Y, int P,
                                             double2* __restrict__ U, int64_t N) {
    __shared__ double2 ys[kT];
    const int p = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    double ax = 0.0, ay = 0.0;
    for (int j0 = 0; j0 < K; j0 += kT) {
        const int nj = min(kT, K - j0);
        __syncthreads();
        if ((int)threadIdx.x < nj) ys[threadIdx.x] = Y[(int64_t)(j0 + threadIdx.x) * P + p];
        __syncthreads();
        if (i < N) {
            for (int jj = 0; jj < nj; ++jj) {
                const double2 v = V[(int64_t)(j0 + jj) * N + i];
                const double2 y = ys[jj];
                ax += v.x * y.x - v.y * y.y;
                ay += v.x * y.y + v.y * y.x;
            }
        }
    }
    if (i < N) U[(int64_t)p * N + i] = make_double2(ax, ay);
}

// partials of ||-AU_p - theta_p U_p||^2 and ||U_p||^2 (AU = A(0) U = -H_op U)
__global__ __launch_bounds__(kT) void k_eig_resid(const double2* __restrict__ U,
                                                  const double2* __restrict__ AU,
                                                  const double2* __restrict__ theta, int64_t N,
                                                  double* __restrict__ part) {
    __shared__ double lds[2 * kT / 64];
    const int p = blockIdx.y;
    const double2 th = theta[p];
    double s[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kT) {
        const double2 u = U[(int64_t)p * N + i], a = AU[(int64_t)p * N + i];
        const double2 tu = cmul_d(th, u);
        const double rx = -a.x - tu.x, ry = -a.y - tu.y;
        s[0] += rx * rx + ry * ry;
        s[1] += u.x * u.x + u.y * u.y;
    }
    block_sum<2>(s, lds);
    if (threadIdx.x == 0) {
        part[((int64_t)p * gridDim.x + blockIdx.x) * 2] = s[0];
        part[((int64_t)p * gridDim.x + blockIdx.x) * 2 + 1] = s[1];
    }
}

int nblocks(int64_t N) {
    int64_t b = (N + 4 * kT - 1) / (4 * kT);
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 512));
}

// Eigenvalues of the complex symmetric tridiagonal matrix with diagonal d
// and couplings e[i] = T(i, i+1) (e[n-1] unused), by the implicit QL
// algorithm with a Wilkinson-type shift and complex orthogonal plane
// rotations (c^2 + s^2 = 1, no conjugation), which keep T complex symmetric
// and tridiagonal.  On return d holds the eigenvalues.  false if a rotation
// broke down or an eigenvalue took more than 300 sweeps.
bool tridiag_eigenvalues(std::vector<cd>& d, std::vector<cd> e) {
    const int n = (int)d.size();
    if (n == 0) return true;
    e.resize(n);
    e[n - 1] = 0.0;
    for (int l = 0; l < n; ++l) {
        int sweeps = 0;
        while (true) {
            int m = l;
            for (; m < n - 1; ++m) {
                const double dd = std::abs(d[m]) + std::abs(d[m + 1]);
                if (std::abs(e[m]) <= 1e-16 * dd) break;
            }
            if (m == l) break;
            if (++sweeps > 300) return false;
            // shift: the eigenvalue of the leading 2x2 block nearer d[l]
            cd g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            cd r = std::sqrt(g * g + 1.0);
            const cd gp = g + r, gm = g - r;
            g = d[m] - d[l] + e[l] / (std::abs(gp) >= std::abs(gm) ? gp : gm);
            cd s = 1.0, c = 1.0, p = 0.0;
            bool deflated = false;
            for (int i = m - 1; i >= l; --i) {
                const cd f = s * e[i], b = c * e[i];
                r = std::sqrt(f * f + g * g);
                e[i + 1] = r;
                if (std::abs(r) <= 1e-300 * (std::abs(f) + std::abs(g) + 1e-300)) {
                    if (std::abs(f) + std::abs(g) > 0.0) return false;  // isotropic pair
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    deflated = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
            }
            if (deflated) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    return true;
}

// Solution of (T - theta) y = b for the tridiagonal T (diagonal d, couplings
// e), by Gaussian elimination with partial pivoting (one extra
// super-diagonal); b is overwritten with y
void tridiag_solve(const std::vector<cd>& d, const std::vector<cd>& e, cd theta, std::vector<cd>& b) {
    const int n = (int)d.size();
    std::vector<cd> a(n), dg(n), u1(n), u2(n);  // sub, diag, super, super-super
    for (int i = 0; i < n; ++i) {
        dg[i] = d[i] - theta;
        a[i] = (i > 0) ? e[i - 1] : 0.0;
        u1[i] = (i < n - 1) ? e[i] : 0.0;
        u2[i] = 0.0;
    }
    const double tiny = 1e-300;
    for (int i = 0; i < n - 1; ++i) {
        // rows i and i+1: pivot on the larger of dg[i] and a[i+1]
        if (std::abs(a[i + 1]) > std::abs(dg[i])) {
            std::swap(dg[i], a[i + 1]);
            std::swap(u1[i], dg[i + 1]);
            std::swap(u2[i], u1[i + 1]);
            std::swap(b[i], b[i + 1]);
        }
        if (std::abs(dg[i]) < tiny) dg[i] = tiny;
        const cd f = a[i + 1] / dg[i];
        dg[i + 1] -= f * u1[i];
        u1[i + 1] -= f * u2[i];
        b[i + 1] -= f * b[i];
        a[i + 1] = 0.0;
    }
    if (std::abs(dg[n - 1]) < tiny) dg[n - 1] = tiny;
    for (int i = n - 1; i >= 0; --i) {
        cd v = b[i];
        if (i + 1 < n) v -= u1[i] * b[i + 1];
        if (i + 2 < n) v -= u2[i] * b[i + 2];
        b[i] = v / dg[i];
    }
}

}  // namespace

extern "C" negf_status negf_eigenpairs(negf_op* op, double e_lo, double e_hi, double margin,
                                       int32_t n_lanczos, double resid_tol, int32_t max_pairs,
                                       negf_c64* eps, negf_c64* U, double* resid,
                                       int32_t* n_found) {
    (void)hipGetLastError();  // a stale error of an earlier call must not fail this one
    if (!op || !eps || !U || !n_found || max_pairs < 1 || n_lanczos < 2 ||
        !std::isfinite(e_lo) || !std::isfinite(e_hi) || !(e_hi >= e_lo) ||
        !std::isfinite(margin) || !(margin >= 0.0) || !(resid_tol > 0.0)) {
        set_error("invalid argument to negf_eigenpairs");
        return NEGF_E_INVALID_ARG;
    }
    *n_found = 0;
    const int64_t N = op->N;
    const int K = (int)std::min<int64_t>(n_lanczos, N);
    HIPCHK(hipSetDevice(op->device));
    hipStream_t s = op->own_stream;
    const int nb = nblocks(N);
    // workspace: V [K + 1][N]; then y, w [N] each; partials; scalars; kbc
    double2* V = nullptr;
    CHK(ws_get(op, WS_LANCZOS, (size_t)(K + 1) * N * sizeof(double2), (void**)&V));
    const size_t n_tmp = 2 * (size_t)N;
    const size_t n_part = (size_t)(K + 1) * nb * 3 / 2 + 1;   // in double2 units
    const size_t n_sc = (size_t)(K + 1) * 3 / 2 + 2;
    double2* tmp = nullptr;
    CHK(ws_get(op, WS_EIGTMP,
               (n_tmp + n_part + n_sc + 2 + (size_t)std::max(1, op->kb.n_proj)) * sizeof(double2),
               (void**)&tmp));
    double2* y = tmp;
    double2* w = tmp + N;
    double* part = reinterpret_cast<double*>(tmp + n_tmp);
    double* sc = reinterpret_cast<double*>(tmp + n_tmp + n_part);
    double* zero_shift = reinterpret_cast<double*>(tmp + n_tmp + n_part + n_sc);
    double2* kbc = tmp + n_tmp + n_part + n_sc + 2;
    HIPCHK(hipMemsetAsync(zero_shift, 0, 2 * sizeof(double2), s));
    std::vector<double> h_sc(3 * (size_t)(K + 1));
    const unsigned gb = (unsigned)nb;

    // bilinear dots c_j = V_j^T x for j < nv (x == null: V_j^T V_j), into h_sc
    auto dots = [&](const double2* Vb, int nv, const double2* x) -> negf_status {
        hipLaunchKernelGGL(k_bidot, dim3(gb, nv), dim3(kT), 0, s, Vb, N, x, part);
        hipLaunchKernelGGL(k_bidot_reduce, dim3(nv), dim3(kT), 0, s, part, nb, sc);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(h_sc.data(), sc, 3 * (size_t)nv * sizeof(double),
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return NEGF_OK;
    };
    // start vector with v^T v = 1 (redrawn if its bilinear form is too small)
    uint64_t seed = 0x5eed14010782ull;
    for (int tries = 0;; ++tries) {
        hipLaunchKernelGGL(k_rand_vec, dim3(gb), dim3(kT), 0, s, V, N, seed + tries);
        CHK(dots(V, 1, nullptr));
        const cd q(h_sc[0], h_sc[1]);
        if (std::abs(q) > 1e-3 * h_sc[2]) {
            const cd f = 1.0 / std::sqrt(q);
            hipLaunchKernelGGL(k_scale_to, dim3(gb), dim3(kT), 0, s, V, V,
                               make_double2(f.real(), f.imag()), N);
            break;
        }
        if (tries > 8) {
            set_error("negf_eigenpairs: no start vector with a nonzero bilinear form");
            return NEGF_E_BREAKDOWN;
        }
    }
    std::vector<cd> alpha(K), beta(K, 0.0);
    int Kd = K;  // Lanczos steps done
    for (int k = 0; k < K; ++k) {
        double2* vk = V + (int64_t)k * N;
        launch_apply<double>(op, vk, y, 1, zero_shift, nullptr, kbc, s);
        const cd bp = k > 0 ? beta[k - 1] : 0.0;
        hipLaunchKernelGGL(k_lanczos_w, dim3(gb), dim3(kT), 0, s, w, y,
                           k > 0 ? V + (int64_t)(k - 1) * N : nullptr,
                           make_double2(bp.real(), bp.imag()), N);
        // two bilinear Gram-Schmidt passes against v_0 .. v_k
        cd a = 0.0;
        for (int pass = 0; pass < 2; ++pass) {
            CHK(dots(V, k + 1, w));
            a += cd(h_sc[3 * (size_t)k], h_sc[3 * (size_t)k + 1]);
            // the coefficients are still in sc on the device
            hipLaunchKernelGGL(k_axpy_multi, dim3((unsigned)((N + kT - 1) / kT)), dim3(kT), 0, s,
                               w, V, k + 1, sc, N);
        }
        alpha[k] = a;
        if (k == K - 1) break;
        CHK(dots(w, 1, nullptr));
        const cd q(h_sc[0], h_sc[1]);
        const double nn = h_sc[2];
        if (!(nn > 0.0) || std::abs(q) <= 1e-20 * nn) {
            // invariant subspace (w = 0) or an isotropic w (w^T w = 0):
            // the process stops here; T_k is what it has found
            Kd = k + 1;
            break;
        }
        const cd b = std::sqrt(q);
        beta[k] = b;
        const cd f = 1.0 / b;
        hipLaunchKernelGGL(k_scale_to, dim3(gb), dim3(kT), 0, s, V + (int64_t)(k + 1) * N, w,
                           make_double2(f.real(), f.imag()), N);
    }
    HIPCHK(hipGetLastError());

    // Ritz values of T_Kd in the window
    std::vector<cd> theta(alpha.begin(), alpha.begin() + Kd);
    std::vector<cd> off(beta.begin(), beta.begin() + Kd);
    if (!tridiag_eigenvalues(theta, off)) {
        set_error("negf_eigenpairs: the tridiagonal eigenvalue iteration broke down");
        return NEGF_E_BREAKDOWN;
    }
    std::vector<cd> sel;
    for (const cd& t : theta)
        if (t.real() >= e_lo - margin && t.real() <= e_hi + margin) sel.push_back(t);
    std::sort(sel.begin(), sel.end(), [](const cd& a, const cd& b) {
        return a.real() < b.real() || (a.real() == b.real() && a.imag() < b.imag());
    });
    if (sel.empty()) return NEGF_OK;
    // eigenvectors of T by inverse iteration, normalised to y^T y = 1
    const int P = (int)sel.size();
    std::vector<double2> Yh((size_t)Kd * P);
    std::vector<cd> dT(alpha.begin(), alpha.begin() + Kd), eT(beta.begin(), beta.begin() + Kd);
    std::vector<int> usable(P, 1);
    for (int p = 0; p < P; ++p) {
        std::vector<cd> v(Kd);
        for (int i = 0; i < Kd; ++i) v[i] = cd(1.0 / (1.0 + i % 7), 0.3 / (1.0 + i % 5));
        const cd th = sel[p] + cd(1e-13 * (1.0 + std::abs(sel[p])), 0.0);
        for (int it = 0; it < 3; ++it) {
            tridiag_solve(dT, eT, th, v);
            double mx = 0.0;
            for (const cd& x : v) mx = std::max(mx, std::abs(x));
            if (!(mx > 0.0) || !std::isfinite(mx)) {
                usable[p] = 0;
                break;
            }
            for (cd& x : v) x /= mx;
        }
        cd q = 0.0;
        double nn = 0.0;
        for (const cd& x : v) {
            q += x * x;
            nn += std::norm(x);
        }
        if (!usable[p] || std::abs(q) <= 1e-12 * nn) {
            usable[p] = 0;  // a (nearly) isotropic eigenvector: no U^T U = 1 normalisation
            continue;
        }
        const cd f = 1.0 / std::sqrt(q);
        for (int i = 0; i < Kd; ++i) {
            const cd x = v[i] * f;
            Yh[(size_t)i * P + p] = make_double2(x.real(), x.imag());
        }
    }
    // Ritz vectors V Y and their true residuals ||H_op u - theta u|| / ||u||
    double2 *Ud = nullptr, *AUd = nullptr, *Yd = nullptr, *thd = nullptr;
    {
        double2* buf = nullptr;
        CHK(ws_get(op, WS_EIGOUT, ((size_t)2 * P * N + (size_t)Kd * P + P) * sizeof(double2),
                   (void**)&buf));
        Ud = buf;
        AUd = buf + (size_t)P * N;
        Yd = AUd + (size_t)P * N;
        thd = Yd + (size_t)Kd * P;
    }
    double2* kbc_p = nullptr;
    CHK(ws_get(op, WS_KBC, (size_t)P * std::max(1, op->kb.n_proj) * sizeof(double2),
               (void**)&kbc_p));
    double* shifts_p = nullptr;
    CHK(ws_get(op, WS_SHIFT, (size_t)P * sizeof(double), (void**)&shifts_p));
    std::vector<double2> th_h(P);
    for (int p = 0; p < P; ++p) th_h[p] = make_double2(sel[p].real(), sel[p].imag());
    HIPCHK(hipMemcpyAsync(Yd, Yh.data(), Yh.size() * sizeof(double2), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(thd, th_h.data(), P * sizeof(double2), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(shifts_p, 0, P * sizeof(double), s));
    hipLaunchKernelGGL(k_ritz, dim3((unsigned)((N + kT - 1) / kT), P), dim3(kT), 0, s, V, Kd, Yd,
                       P, Ud, N);
    launch_apply<double>(op, Ud, AUd, P, shifts_p, nullptr, kbc_p, s);
    double* rpart = part;  // [P][nb][2] fits in the partials buffer (P <= Kd + 1)
    hipLaunchKernelGGL(k_eig_resid, dim3(gb, P), dim3(kT), 0, s, Ud, AUd, thd, N, rpart);
    HIPCHK(hipGetLastError());
    std::vector<double> rp((size_t)P * nb * 2);
    HIPCHK(hipMemcpyAsync(rp.data(), rpart, rp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const bool u_dev = [&] {
        hipPointerAttribute_t attr;
        if (hipPointerGetAttributes(&attr, U) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        return attr.type == hipMemoryTypeDevice;
    }();
    int found = 0;
    for (int p = 0; p < P && found < max_pairs; ++p) {
        if (!usable[p]) continue;
        double r2 = 0.0, u2 = 0.0;
        for (int b = 0; b < nb; ++b) {
            r2 += rp[((size_t)p * nb + b) * 2];
            u2 += rp[((size_t)p * nb + b) * 2 + 1];
        }
        const double rel = std::sqrt(r2 / u2);
        if (!(rel <= resid_tol)) continue;
        eps[found].re = sel[p].real();
        eps[found].im = sel[p].imag();
        if (resid) resid[found] = rel;
        HIPCHK(hipMemcpyAsync(U + (size_t)found * N, Ud + (size_t)p * N, N * sizeof(double2),
                              u_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
        ++found;
    }
    HIPCHK(hipStreamSynchronize(s));
    *n_found = found;
    return NEGF_OK;
}
