// Operator apply Y = A(E_c) X on a block of complex vectors, for gfx950.
//
// A(E) = E*1 - H + i(W_L + W_R) with H = -1/2 Lap_h + diag(V) + sum_p E_p b_p b_p^T
// (Sec. II.B-C).  The Laplacian is the order-2R star stencil with zero ghosts.
//
// Layout: a block holds w vectors, column-major: X[c][i], i = ix + nx*(iy + ny*iz),
// complex interleaved (double2 / float2).
//
// Kernel design (memory bound, see the roofline in the design notes): one
// work-group owns one column and a tile of TY full x-rows and marches along z.
// The 2R+1 z-values of every output point it owns sit in a register queue;
// each new plane is staged once in LDS (tile rows plus R halo rows on each
// side, x padded by R zeros) so the 4R in-plane neighbours come from LDS.
// HBM sees each input plane once per tile (halo rows are re-read through L2
// by the neighbouring tile, which runs at the same z on the same XCD because
// the tiles of one column are issued consecutively).
#include <algorithm>

#include <mutex>
#include <set>
#include <type_traits>
#include <utility>

#include "negf_internal.h"

namespace {

constexpr int kThreads = 256;

template <typename R> struct Coef { R a[7]; };

template <typename R>
__device__ inline cplx_t<R> cadd_t(cplx_t<R> a, cplx_t<R> b) {
    cplx_t<R> r; r.x = a.x + b.x; r.y = a.y + b.y; return r;
}

// ---------------------------------------------------------------------------
// reference-style kernel: one thread per (point, column), neighbours from
// global memory.  Used for planes wider than the tiled kernel supports.
// ---------------------------------------------------------------------------
template <int RAD, typename R>
__global__ __launch_bounds__(kThreads) void k_apply_direct(
    const cplx_t<R>* __restrict__ x, cplx_t<R>* __restrict__ y, int nx, int ny, int nz,
    Coef<R> cf, const double* __restrict__ v, const double* __restrict__ wz,
    const double* __restrict__ shift, const int* __restrict__ skip) {
    const int c = blockIdx.y;
    if (skip && skip[c]) return;
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= N) return;
    const int ix = (int)(i % nx);
    const int64_t t = i / nx;
    const int iy = (int)(t % ny);
    const int iz = (int)(t / ny);
    const cplx_t<R>* xc = x + (int64_t)c * N;
    const cplx_t<R> xi = xc[i];
    const R dr = (R)(shift[c] - v[i] + (double)cf.a[0]);
    const R di = (R)wz[iz];
    R accx = dr * xi.x - di * xi.y;
    R accy = dr * xi.y + di * xi.x;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
#pragma unroll
    for (int m = 1; m <= RAD; ++m) {
        R sx_ = 0, sy_ = 0;
        if (ix - m >= 0) { sx_ += xc[i - m].x; sy_ += xc[i - m].y; }
        if (ix + m < nx) { sx_ += xc[i + m].x; sy_ += xc[i + m].y; }
        if (iy - m >= 0) { sx_ += xc[i - m * sy].x; sy_ += xc[i - m * sy].y; }
        if (iy + m < ny) { sx_ += xc[i + m * sy].x; sy_ += xc[i + m * sy].y; }
        if (iz - m >= 0) { sx_ += xc[i - m * sz].x; sy_ += xc[i - m * sz].y; }
        if (iz + m < nz) { sx_ += xc[i + m * sz].x; sy_ += xc[i + m * sz].y; }
        accx += cf.a[m] * sx_;
        accy += cf.a[m] * sy_;
    }
    cplx_t<R> o; o.x = accx; o.y = accy;
    y[(int64_t)c * N + i] = o;
}

// ---------------------------------------------------------------------------
// tiled z-marching kernel
//   work-group: one column c, rows [y0, y0+TY) of every plane, z in [z0, z1)
//   thread t owns the points (x = t % nx, y = y0 + t / nx + k*(256/nx)), k < PPT
// ---------------------------------------------------------------------------
template <int RAD, typename R, int PPT>
__global__ __launch_bounds__(kThreads) void k_apply_tiled(
    const cplx_t<R>* __restrict__ x, cplx_t<R>* __restrict__ y, int nx, int ny, int nz,
    int ty, int n_ytiles, int zchunk, Coef<R> cf, const double* __restrict__ v,
    const double* __restrict__ wz, const double* __restrict__ shift,
    const int* __restrict__ skip) {
    extern __shared__ unsigned char smem_raw[];
    cplx_t<R>* tile = reinterpret_cast<cplx_t<R>*>(smem_raw);
    const int bid = blockIdx.x;
    const int c = blockIdx.y;
    if (skip && skip[c]) return;
    const int ytile = bid % n_ytiles;
    const int zc = bid / n_ytiles;
    const int z0 = zc * zchunk;
    const int z1 = min(nz, z0 + zchunk);
    const int y0 = ytile * ty;
    const int rows = min(ty, ny - y0);
    const int pitch = nx + 2 * RAD;           // LDS row pitch (x padded)
    const int lrows = rows + 2 * RAD;         // LDS rows (y halo)
    const int64_t plane = (int64_t)nx * ny;
    const int64_t N = plane * nz;
    const cplx_t<R>* xc = x + (int64_t)c * N;
    cplx_t<R>* yc = y + (int64_t)c * N;
    const int tid = threadIdx.x;
    const int rows_per_pass = kThreads / nx;  // threads beyond rows_per_pass*nx idle
    const int lx = tid % nx;
    const int ly0 = (tid < rows_per_pass * nx) ? tid / nx : (1 << 20);
    const double e_c = shift[c] + (double)cf.a[0];

    // zero the LDS tile (padding stays zero)
    for (int k = tid; k < pitch * lrows; k += kThreads) { tile[k].x = 0; tile[k].y = 0; }

    // register queue: q[k][d] = value at (point k, plane z + d - RAD)
    cplx_t<R> q[PPT][2 * RAD + 1];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int yy = ly0 + k * rows_per_pass;
#pragma unroll
        for (int d = 0; d < 2 * RAD + 1; ++d) {
            const int zz = z0 + d - RAD;
            cplx_t<R> val; val.x = 0; val.y = 0;
            if (yy < rows && zz >= 0 && zz < nz && d < 2 * RAD)
                val = xc[(int64_t)zz * plane + (int64_t)(y0 + yy) * nx + lx];
            q[k][d] = val;
        }
    }
    __syncthreads();

    for (int z = z0; z < z1; ++z) {
        // lead plane z + RAD into the queue tail
        const int zl = z + RAD;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int yy = ly0 + k * rows_per_pass;
            cplx_t<R> val; val.x = 0; val.y = 0;
            if (yy < rows && zl < nz) val = xc[(int64_t)zl * plane + (int64_t)(y0 + yy) * nx + lx];
            q[k][2 * RAD] = val;
        }
        // stage plane z: interior rows from the queue, halo rows from memory
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int yy = ly0 + k * rows_per_pass;
            if (yy < rows) tile[(yy + RAD) * pitch + RAD + lx] = q[k][RAD];
        }
        for (int k = tid; k < 2 * RAD * nx; k += kThreads) {
            const int hr = k / nx;         // 0 .. 2R-1
            const int hx = k % nx;
            const int yy = hr < RAD ? (hr - RAD) : (rows + hr - RAD);  // tile-relative row
            const int gy = y0 + yy;
            cplx_t<R> val; val.x = 0; val.y = 0;
            if (gy >= 0 && gy < ny) val = xc[(int64_t)z * plane + (int64_t)gy * nx + hx];
            tile[(yy + RAD) * pitch + RAD + hx] = val;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int yy = ly0 + k * rows_per_pass;
            if (yy < rows) {
                const int64_t gi = (int64_t)z * plane + (int64_t)(y0 + yy) * nx + lx;
                const cplx_t<R> xi = q[k][RAD];
                const R dr = (R)(e_c - v[gi]);
                const R di = (R)wz[z];
                R ax = dr * xi.x - di * xi.y;
                R ay = dr * xi.y + di * xi.x;
                const cplx_t<R>* row = tile + (yy + RAD) * pitch + RAD + lx;
#pragma unroll
                for (int m = 1; m <= RAD; ++m) {
                    const cplx_t<R> a0 = row[-m], a1 = row[m];
                    const cplx_t<R> b0 = row[-m * pitch], b1 = row[m * pitch];
                    const cplx_t<R> c0 = q[k][RAD - m], c1 = q[k][RAD + m];
                    ax += cf.a[m] * ((a0.x + a1.x) + (b0.x + b1.x) + (c0.x + c1.x));
                    ay += cf.a[m] * ((a0.y + a1.y) + (b0.y + b1.y) + (c0.y + c1.y));
                }
                cplx_t<R> o; o.x = ax; o.y = ay;
                yc[gi] = o;
            }
        }
        __syncthreads();
        // shift the queue
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
#pragma unroll
            for (int d = 0; d < 2 * RAD; ++d) q[k][d] = q[k][d + 1];
        }
    }
}

// ---------------------------------------------------------------------------
// separable projectors: gather c[col][p] = b_p^T x_col, then
// y[col][i] -= sum_{p touching i} E_p b_p(i) c[col][p]
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kThreads) void k_kb_gather(
    const cplx_t<R>* __restrict__ x, int64_t N, const int64_t* __restrict__ off,
    const int* __restrict__ idx, const double* __restrict__ val, int n_proj, int w,
    double2* __restrict__ out, const int* __restrict__ skip) {
    // one wave per (projector, column)
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int p = blockIdx.x;
    const int c = blockIdx.y * (kThreads / 64) + wave;
    if (c >= w) return;
    if (skip && skip[c]) return;
    const cplx_t<R>* xc = x + (int64_t)c * N;
    double sx = 0, sy = 0;
    int64_t k = off[p] + lane;
    const int64_t ke = off[p + 1];
    // four points per lane per step with all their loads issued together (the
    // index -> value chains are what the gather waits on); each lane still adds
    // its points in the same order
    for (; k + 192 < ke; k += 256) {
        int ii[4];
        double bb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ii[u] = idx[k + 64 * u];
            bb[u] = val[k + 64 * u];
        }
        cplx_t<R> xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u] = xc[ii[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            sx += bb[u] * (double)xv[u].x;
            sy += bb[u] * (double)xv[u].y;
        }
    }
    for (; k < ke; k += 64) {
        const cplx_t<R> xv = xc[idx[k]];
        const double b = val[k];
        sx += b * (double)xv.x;
        sy += b * (double)xv.y;
    }
    for (int o = 32; o > 0; o >>= 1) {
        sx += __shfl_xor(sx, o, 64);
        sy += __shfl_xor(sy, o, 64);
    }
    if (lane == 0) out[(int64_t)c * n_proj + p] = make_double2(sx, sy);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_kb_scatter(
    cplx_t<R>* __restrict__ y, int64_t N, const int* __restrict__ pts,
    const int* __restrict__ pt_off, const int* __restrict__ pt_proj,
    const double* __restrict__ pt_val, int n_pts, int n_proj,
    const double2* __restrict__ cproj, const int* __restrict__ skip) {
    const int c = blockIdx.y;
    if (skip && skip[c]) return;
    const int k = blockIdx.x * kThreads + threadIdx.x;
    if (k >= n_pts) return;
    double sx = 0, sy = 0;
    const double2* cc = cproj + (int64_t)c * n_proj;
    for (int e = pt_off[k]; e < pt_off[k + 1]; ++e) {
        const double2 cv = cc[pt_proj[e]];
        const double f = pt_val[e];
        sx += f * cv.x;
        sy += f * cv.y;
    }
    cplx_t<R>* yc = y + (int64_t)c * N;
    cplx_t<R> o = yc[pts[k]];
    o.x -= (R)sx;
    o.y -= (R)sy;
    yc[pts[k]] = o;
}

template <int RAD, typename R>
void apply_dispatch(const negf_op* op, const cplx_t<R>* x, cplx_t<R>* y, int w,
                    const double* d_shift, const int* d_skip, hipStream_t s) {
    Coef<R> cf;
    for (int m = 0; m < 7; ++m) cf.a[m] = (R)op->coef.a[m];
    const int nx = op->nx, ny = op->ny, nz = op->nz;
    const bool tiled = (nx >= 8) && (nx <= kThreads);
    if (tiled) {
        const int rows_per_pass = kThreads / nx;
        // points per thread: 2 passes of rows per tile when the register budget allows
        constexpr int PPT = (RAD >= 5 && sizeof(R) == 8) ? 1 : 2;
        int ty = rows_per_pass * PPT;
        if (ty > ny) ty = ny;
        const int n_ytiles = (ny + ty - 1) / ty;
        // z chunks: enough work-groups to fill the device, chunks >= 4R planes
        int zchunk = nz;
        const long target = 1024;
        long wgs = (long)n_ytiles * w;
        while (wgs * ((nz + zchunk - 1) / zchunk) < target && zchunk > 4 * RAD) zchunk = (zchunk + 1) / 2;
        const int n_z = (nz + zchunk - 1) / zchunk;
        const size_t lds = (size_t)(nx + 2 * RAD) * (ty + 2 * RAD) * sizeof(cplx_t<R>);
        dim3 grid(n_ytiles * n_z, w);
        hipLaunchKernelGGL((k_apply_tiled<RAD, R, PPT>), grid, dim3(kThreads), lds, s, x, y, nx,
                           ny, nz, ty, n_ytiles, zchunk, cf, op->d_v, op->d_wz, d_shift, d_skip);
    } else {
        const int64_t N = op->N;
        dim3 grid((unsigned)((N + kThreads - 1) / kThreads), w);
        hipLaunchKernelGGL((k_apply_direct<RAD, R>), grid, dim3(kThreads), 0, s, x, y, nx, ny,
                           nz, cf, op->d_v, op->d_wz, d_shift, d_skip);
    }
}

}  // namespace

template <typename R>
void launch_apply(const negf_op* op, const cplx_t<R>* x, cplx_t<R>* y, int w,
                  const double* d_shift, const int* d_skip, double2* d_kbc, hipStream_t s) {
    switch (op->R) {
        case 1: apply_dispatch<1, R>(op, x, y, w, d_shift, d_skip, s); break;
        case 2: apply_dispatch<2, R>(op, x, y, w, d_shift, d_skip, s); break;
        case 3: apply_dispatch<3, R>(op, x, y, w, d_shift, d_skip, s); break;
        case 4: apply_dispatch<4, R>(op, x, y, w, d_shift, d_skip, s); break;
        case 5: apply_dispatch<5, R>(op, x, y, w, d_shift, d_skip, s); break;
        default: apply_dispatch<6, R>(op, x, y, w, d_shift, d_skip, s); break;
    }
    if (op->kb.n_proj > 0) {
        const DeviceKB& kb = op->kb;
        dim3 g1(kb.n_proj, (w + 3) / 4);
        hipLaunchKernelGGL((k_kb_gather<R>), g1, dim3(kThreads), 0, s, x, op->N, kb.off, kb.idx,
                           kb.val, kb.n_proj, w, d_kbc, d_skip);
        dim3 g2((kb.n_pts + kThreads - 1) / kThreads, w);
        hipLaunchKernelGGL((k_kb_scatter<R>), g2, dim3(kThreads), 0, s, y, op->N, kb.pts,
                           kb.pt_off, kb.pt_proj, kb.pt_val, kb.n_pts, kb.n_proj, d_kbc, d_skip);
    }
}

template void launch_apply<double>(const negf_op*, const double2*, double2*, int, const double*,
                                   const int*, double2*, hipStream_t);
template void launch_apply<float>(const negf_op*, const float2*, float2*, int, const double*,
                                  const int*, double2*, hipStream_t);

// ---------------------------------------------------------------------------
// Fused COCG step on the operator (the hot loop of both solver cores):
//     p_k = r_k + beta_{k-1} p_{k-1}   (p_k = r_k at k = 0)
//     q_k = (A(E_c) - projector term) p_k,   partial sums of p_k^T q_k
// in one pass: HBM sees r and p_{k-1} once (read) and p_k, q_k once (write).
// Without FUSED the same kernel is the plain apply y = A x (x passed as pin).
//
// Work-group: NT threads own a tile of TY full x-rows (TY = NT/nx rows,
// or all ny rows when they fit; then no y-halo exists) of one column and a
// z-chunk.  Each thread owns one (x, y) column of the tile:
//   * register queue of the 2R+1 values of p along z,
//   * the next lead plane's r and p_{k-1} are prefetched one plane ahead,
//   * the centre plane (plus y-halo rows, recomputed from r and p_{k-1})
//     is staged in a double-buffered LDS tile: one barrier per plane.
// p_k is written by the owner of each plane only (no write races), and the
// p buffers ping-pong between iterations so halo reads see p_{k-1}.
// ---------------------------------------------------------------------------
// p = r + beta p_prev with the roundings fixed (explicit fused multiply-adds),
// so every thread that forms the same element (its owner, or a neighbouring
// tile's y-halo) gets the same bits
template <typename R>
__device__ __forceinline__ cplx_t<R> cocg_p(const cplx_t<R>& rv, const cplx_t<R>& pv, R bx, R by) {
    cplx_t<R> o;
    if constexpr (std::is_same<R, double>::value) {
        o.x = __builtin_fma(bx, pv.x, __builtin_fma(-by, pv.y, rv.x));
        o.y = __builtin_fma(bx, pv.y, __builtin_fma(by, pv.x, rv.y));
    } else {
        o.x = __builtin_fmaf(bx, pv.x, __builtin_fmaf(-by, pv.y, rv.x));
        o.y = __builtin_fmaf(bx, pv.y, __builtin_fmaf(by, pv.x, rv.y));
    }
    return o;
}

template <int RAD, typename R, int NT, bool FUSED>
__global__ __launch_bounds__(NT) void k_cocg_apply(
    const cplx_t<R>* __restrict__ r, const cplx_t<R>* __restrict__ pin, cplx_t<R>* __restrict__ pout,
    cplx_t<R>* __restrict__ y, int nx, int ny, int nz, int ty, int n_ytiles, int zchunk,
    Coef<R> cf, double a0, const double* __restrict__ v, const double* __restrict__ wz,
    const double* __restrict__ shift, const int* __restrict__ skip, const int* __restrict__ kit,
    const double2* __restrict__ beta, double2* __restrict__ part, int xcd_group, int nt_store) {
    extern __shared__ unsigned char smem_raw[];
    // launch index -> (tile, column).  The y-tiles of one z-chunk read each
    // other's boundary rows as halo at the same plane and time; with
    // xcd_group the G work-groups are dealt to the 8 XCDs in turn (work-group
    // i goes to XCD i mod 8) so that the i-th one an XCD receives takes
    // logical index xcd * (G / 8) + i: consecutive tiles share an XCD and the
    // halo rows come from its L2
    const int nb = gridDim.x;
    int bid = blockIdx.x, c = blockIdx.y;
    if (xcd_group) {
        const int G = nb * gridDim.y;
        const int lin = blockIdx.x + nb * blockIdx.y;
        const int G8 = G & ~7;
        const int logical = lin < G8 ? (lin & 7) * (G8 >> 3) + (lin >> 3) : lin;
        bid = logical % nb;
        c = logical / nb;
    }
    if (skip && skip[c]) return;
    const int ytile = bid % n_ytiles;
    const int z0 = (bid / n_ytiles) * zchunk;
    const int z1 = min(nz, z0 + zchunk);
    const int y0 = ytile * ty;
    const int rows = min(ty, ny - y0);
    const int pitch = nx + 2 * RAD;
    const int lrows = ty + 2 * RAD;
    cplx_t<R>* tile0 = reinterpret_cast<cplx_t<R>*>(smem_raw);
    cplx_t<R>* tile1 = tile0 + pitch * lrows;
    const int64_t plane = (int64_t)nx * ny;
    const int64_t N = plane * nz;
    const int64_t co = (int64_t)c * N;
    const int tid = threadIdx.x;
    const int lx = tid % nx;
    const int ly = tid / nx;  // < rows for the threads that own a point
    const bool own = ly < rows;
    const int col_off = (y0 + (own ? ly : 0)) * nx + lx;  // within a plane
    const double e_c = shift[c] + a0;
    const bool first = FUSED ? (kit[c] == 0) : true;
    const double2 bb = FUSED ? beta[c] : make_double2(0.0, 0.0);
    const R bx = (R)bb.x, byy = (R)bb.y;
    const bool has_halo = rows < ny;

    // p at (plane zz, tile-relative row yy, x) from r and p_{k-1} (FUSED) or x (plain)
    auto p_at = [&](int64_t gi) -> cplx_t<R> {
        if (!FUSED) return pin[co + gi];
        const cplx_t<R> rv = r[co + gi];
        if (first) return rv;
        return cocg_p<R>(rv, pin[co + gi], bx, byy);
    };

    // zero both LDS tiles (x padding and out-of-grid rows stay zero)
    for (int k = tid; k < 2 * pitch * lrows; k += NT) {
        tile0[k].x = 0;
        tile0[k].y = 0;
    }
    cplx_t<R> q[2 * RAD + 1];
#pragma unroll
    for (int d = 0; d < 2 * RAD; ++d) {
        const int zz = z0 + d - RAD;
        cplx_t<R> val;
        val.x = 0;
        val.y = 0;
        if (own && zz >= 0 && zz < nz) val = p_at((int64_t)zz * plane + col_off);
        q[d] = val;
    }
    // prefetch of the lead plane z0 + RAD and of V on the centre plane z0.
    // Vector memory counters retire in order, so every per-lane load the
    // plane step consumes is issued one step ahead: a load issued and used in
    // the same step would also wait for the prefetch behind it.
    cplx_t<R> nr, np;
    nr.x = nr.y = np.x = np.y = 0;
    double v_next = own ? v[(int64_t)z0 * plane + col_off] : 0.0;
    {
        const int zl = z0 + RAD;
        if (own && zl < nz) {
            const int64_t gi = co + (int64_t)zl * plane + col_off;
            if (FUSED) {
                nr = r[gi];
                if (!first) np = pin[gi];
            } else {
                np = pin[gi];
            }
        }
    }
    double dot_x = 0.0, dot_y = 0.0;
    __syncthreads();
    for (int z = z0; z < z1; ++z) {
        cplx_t<R>* tile = (z & 1) ? tile1 : tile0;
        const double v_cur = v_next;
        // lead plane z + RAD from the prefetched values
        {
            cplx_t<R> lead;
            if (!FUSED) {
                lead = np;
            } else if (first) {
                lead = nr;
            } else {
                lead = cocg_p<R>(nr, np, bx, byy);
            }
            q[2 * RAD] = lead;
        }
        // y-halo rows of plane z (recomputed from r and p_{k-1}), issued
        // before the next plane's prefetch: vector loads return in order, so
        // waiting for these does not wait for the prefetch behind them
        if (has_halo) {
            for (int k = tid; k < 2 * RAD * nx; k += NT) {
                const int hr = k / nx, hx = k % nx;
                const int yy = hr < RAD ? (hr - RAD) : (rows + hr - RAD);
                const int gy = y0 + yy;
                cplx_t<R> val;
                val.x = 0;
                val.y = 0;
                if (gy >= 0 && gy < ny) val = p_at((int64_t)z * plane + (int64_t)gy * nx + hx);
                tile[(yy + RAD) * pitch + RAD + hx] = val;
            }
        }
        // prefetch plane z + RAD + 1 and V of plane z + 1
        {
            const int zl = z + RAD + 1;
            nr.x = nr.y = np.x = np.y = 0;
            if (own && zl < nz && z + 1 < z1) {
                const int64_t gi = co + (int64_t)zl * plane + col_off;
                if (FUSED) {
                    nr = r[gi];
                    if (!first) np = pin[gi];
                } else {
                    np = pin[gi];
                }
            }
            if (own && z + 1 < z1) v_next = v[(int64_t)(z + 1) * plane + col_off];
        }
        // stage the centre plane
        if (own) {
            tile[(ly + RAD) * pitch + RAD + lx] = q[RAD];
            if (FUSED) {
                if (nt_store)
                    st_once<R>(pout + co + (int64_t)z * plane + col_off, q[RAD]);
                else
                    pout[co + (int64_t)z * plane + col_off] = q[RAD];
            }
        }
        __syncthreads();
        if (own) {
            const int64_t gi = (int64_t)z * plane + col_off;
            const cplx_t<R> xi = q[RAD];
            const R dr = (R)(e_c - v_cur);
            const R di = (R)wz[z];
            R ax = dr * xi.x - di * xi.y;
            R ay = dr * xi.y + di * xi.x;
            const cplx_t<R>* row = tile + (ly + RAD) * pitch + RAD + lx;
#pragma unroll
            for (int m = 1; m <= RAD; ++m) {
                const cplx_t<R> a0v = row[-m], a1v = row[m];
                const cplx_t<R> b0v = row[-m * pitch], b1v = row[m * pitch];
                const cplx_t<R> c0v = q[RAD - m], c1v = q[RAD + m];
                ax += cf.a[m] * ((a0v.x + a1v.x) + (b0v.x + b1v.x) + (c0v.x + c1v.x));
                ay += cf.a[m] * ((a0v.y + a1v.y) + (b0v.y + b1v.y) + (c0v.y + c1v.y));
            }
            cplx_t<R> o;
            o.x = ax;
            o.y = ay;
            if (nt_store)
                st_once<R>(y + co + gi, o);
            else
                y[co + gi] = o;
            if (FUSED) {
                dot_x += (double)xi.x * ax - (double)xi.y * ay;
                dot_y += (double)xi.x * ay + (double)xi.y * ax;
            }
        }
#pragma unroll
        for (int d = 0; d < 2 * RAD; ++d) q[d] = q[d + 1];
    }
    if (FUSED) {
        // block reduction of p^T q (waves, then LDS; tile0 is free to reuse)
        __syncthreads();
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            dot_x += __shfl_xor(dot_x, o, 64);
            dot_y += __shfl_xor(dot_y, o, 64);
        }
        double* red = reinterpret_cast<double*>(smem_raw);
        const int wave = tid / 64;
        if (tid % 64 == 0) {
            red[2 * wave] = dot_x;
            red[2 * wave + 1] = dot_y;
        }
        __syncthreads();
        if (tid == 0) {
            double sx = 0.0, sy = 0.0;
            for (int wv = 0; wv < NT / 64; ++wv) {
                sx += red[2 * wv];
                sy += red[2 * wv + 1];
            }
            part[(int64_t)c * nb + bid] = make_double2(sx, sy);
        }
    }
}

// Whole-plane variant of k_cocg_apply: the work-group is one z-plane of one
// column (blockDim = nx*ny <= 1024 rounded up to whole waves), so there is no
// y-halo and every thread owns a point (the padding lanes mirror the last
// one and store nothing that is kept).  Two things keep the
// in-order vector-memory queue from draining every plane:
//  * all global loads and stores are unconditional (plane indices clamped,
//    out-of-grid values discarded by selection, stores that belong to no plane
//    go to a small sink buffer), so no execution-mask branch surrounds them;
//  * the z-queue is unrolled 2R+1 ways: slot (u + d) mod (2R+1) holds plane
//    z + d - R at unrolled step u, so no register is rewritten while a store
//    that reads it may still be pending.
template <int RAD, typename R, bool FUSED, bool NTH>
__global__ __launch_bounds__(1024) void k_cocg_plane(
    const cplx_t<R>* __restrict__ r, const cplx_t<R>* __restrict__ pin, cplx_t<R>* __restrict__ pout,
    cplx_t<R>* __restrict__ y, cplx_t<R>* __restrict__ sink, int nx, int ny, int nz, int zchunk,
    Coef<R> cf, double a0, const double* __restrict__ v, const double* __restrict__ wz,
    const double* __restrict__ shift, const int* __restrict__ skip, const int* __restrict__ kit,
    const double2* __restrict__ beta, double2* __restrict__ part) {
    constexpr int Q = 2 * RAD + 1;
    extern __shared__ unsigned char smem_raw[];
    const int c = blockIdx.y;
    if (skip && skip[c]) return;
    const int z0 = blockIdx.x * zchunk;
    const int z1 = min(nz, z0 + zchunk);
    const int pitch = nx + 2 * RAD;
    const int lrows = ny + 2 * RAD;
    cplx_t<R>* tile0 = reinterpret_cast<cplx_t<R>*>(smem_raw);
    cplx_t<R>* tile1 = tile0 + pitch * lrows;
    const int64_t plane = (int64_t)nx * ny;
    const int64_t co = (int64_t)c * plane * nz;
    const int tid = threadIdx.x;
    // lanes past the plane (the block is padded to whole waves) mirror its
    // last point: same loads, same LDS value at the same place, every global
    // store sunk and no share in the dot product
    const int pts = nx * ny;
    const bool ghost = tid >= pts;
    const int pt = ghost ? pts - 1 : tid;
    const int lx = pt % nx, ly = pt / nx;
    const int64_t col_off = pt;  // = ly * nx + lx
    const int lds_at = (ly + RAD) * pitch + RAD + lx;
    cplx_t<R>* my_sink = sink + (int64_t)c * plane + col_off;
    const double e_c = shift[c] + a0;
    const bool first = FUSED ? (kit[c] == 0) : true;
    const double2 bb = FUSED ? beta[c] : make_double2(0.0, 0.0);
    const R bx = (R)bb.x, byy = (R)bb.y;
    const R zero = 0;

    auto make_p = [&](cplx_t<R> rv, cplx_t<R> pv) -> cplx_t<R> {
        if (!FUSED) return pv;
        cplx_t<R> o;
        o.x = first ? rv.x : rv.x + bx * pv.x - byy * pv.y;
        o.y = first ? rv.y : rv.y + bx * pv.y + byy * pv.x;
        return o;
    };
    auto load_plane = [&](int zz, cplx_t<R>& rv, cplx_t<R>& pv) {
        const int zc = min(max(zz, 0), nz - 1);
        const int64_t gi = co + (int64_t)zc * plane + col_off;
        if (FUSED) rv = r[gi];
        // p_{k-1} is dead after this step
        if constexpr (NTH)
            pv = ld_once<R>(pin + gi);
        else
            pv = pin[gi];
    };

    for (int k = tid; k < 2 * pitch * lrows; k += blockDim.x) {
        tile0[k].x = 0;
        tile0[k].y = 0;
    }
    cplx_t<R> q[Q];
#pragma unroll
    for (int d = 0; d < 2 * RAD; ++d) {
        const int zz = z0 + d - RAD;
        cplx_t<R> rv, pv;
        rv.x = rv.y = pv.x = pv.y = 0;
        load_plane(zz, rv, pv);
        const cplx_t<R> pp = make_p(rv, pv);
        const bool in = zz >= 0 && zz < nz;
        q[d].x = in ? pp.x : zero;
        q[d].y = in ? pp.y : zero;
    }
    cplx_t<R> nr, np;
    nr.x = nr.y = np.x = np.y = 0;
    load_plane(z0 + RAD, nr, np);
    double v_next = v[(int64_t)z0 * plane + col_off];
    double dot_x = 0.0, dot_y = 0.0;
    __syncthreads();

    // Q plane steps per trip with the queue rotated by u (a constant after
    // unrolling); the last trip runs past z1 with its loads clamped, its
    // stores sunk and its dot products dropped
    for (int zt = z0; zt < z1; zt += Q) {
#pragma unroll
        for (int u = 0; u < Q; ++u) {
            const int z = zt + u;
            cplx_t<R>* tile = (z & 1) ? tile1 : tile0;
            const double v_cur = v_next;
            {
                const cplx_t<R> pp = make_p(nr, np);
                const bool in = z + RAD < nz;
                q[(u + 2 * RAD) % Q].x = in ? pp.x : zero;
                q[(u + 2 * RAD) % Q].y = in ? pp.y : zero;
            }
            load_plane(z + RAD + 1, nr, np);
            v_next = v[(int64_t)min(z + 1, nz - 1) * plane + col_off];
            const cplx_t<R> xi = q[(u + RAD) % Q];
            tile[lds_at] = xi;
            const bool live = z < z1 && !ghost;
            const int64_t gz = co + (int64_t)min(z, nz - 1) * plane + col_off;
            if (FUSED) {
                cplx_t<R>* dst = live ? pout + gz : my_sink;
                // p_k: next read one whole step later
                if constexpr (NTH)
                    st_once<R>(dst, xi);
                else
                    *dst = xi;
            }
            __syncthreads();
            const R dr = (R)(e_c - v_cur);
            const R di = (R)wz[min(z, nz - 1)];
            R ax = dr * xi.x - di * xi.y;
            R ay = dr * xi.y + di * xi.x;
            const cplx_t<R>* row = tile + lds_at;
#pragma unroll
            for (int m = 1; m <= RAD; ++m) {
                const cplx_t<R> a0v = row[-m], a1v = row[m];
                const cplx_t<R> b0v = row[-m * pitch], b1v = row[m * pitch];
                const cplx_t<R> c0v = q[(u + RAD - m) % Q], c1v = q[(u + RAD + m) % Q];
                ax += cf.a[m] * ((a0v.x + a1v.x) + (b0v.x + b1v.x) + (c0v.x + c1v.x));
                ay += cf.a[m] * ((a0v.y + a1v.y) + (b0v.y + b1v.y) + (c0v.y + c1v.y));
            }
            cplx_t<R> o;
            o.x = ax;
            o.y = ay;
            cplx_t<R>* ydst = live ? y + gz : my_sink;
            // q: read once, by the update
            if constexpr (NTH)
                st_once<R>(ydst, o);
            else
                *ydst = o;
            if (FUSED) {
                const double dx = (double)xi.x * ax - (double)xi.y * ay;
                const double dy = (double)xi.x * ay + (double)xi.y * ax;
                dot_x += live ? dx : 0.0;
                dot_y += live ? dy : 0.0;
            }
        }
    }
    if (FUSED) {
        __syncthreads();
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            dot_x += __shfl_xor(dot_x, o, 64);
            dot_y += __shfl_xor(dot_y, o, 64);
        }
        double* red = reinterpret_cast<double*>(smem_raw);
        const int wave = tid / 64;
        if (tid % 64 == 0) {
            red[2 * wave] = dot_x;
            red[2 * wave + 1] = dot_y;
        }
        __syncthreads();
        if (tid == 0) {
            double sx = 0.0, sy = 0.0;
            for (int wv = 0; wv < (int)blockDim.x / 64; ++wv) {
                sx += red[2 * wv];
                sy += red[2 * wv + 1];
            }
            part[(int64_t)c * gridDim.x + blockIdx.x] = make_double2(sx, sy);
        }
    }
}

namespace {

struct FusedGeom {
    bool whole_plane;  // k_cocg_plane: one full plane per work-group
    int nt, ty, n_ytiles, zchunk, n_z;
    size_t lds;
};

// whole-plane kernel: one plane per work-group, z-chunks for every CU
template <int RAD, typename R>
FusedGeom plane_geom(const negf_op* op, int w) {
    FusedGeom g;
    const int nx = op->nx, ny = op->ny, nz = op->nz;
    const int pts = nx * ny;
    g.whole_plane = true;
    g.nt = (pts + 63) / 64 * 64;
    g.ty = ny;
    g.n_ytiles = 1;
    // z-chunks: enough work-groups for every CU, each a multiple of the
    // 2R+1 unrolled steps (the last trip of a chunk runs whole)
    constexpr int Q = 2 * RAD + 1;
    const int target = op->wg_target > 0 ? op->wg_target : 256;
    int nzc = std::max(1, (target + w - 1) / w);
    int zc = (nz + nzc - 1) / nzc;
    zc = std::max(Q, ((zc + Q - 1) / Q) * Q);
    g.zchunk = zc;
    g.n_z = (nz + zc - 1) / zc;
    g.lds = 2 * (size_t)(nx + 2 * RAD) * (ny + 2 * RAD) * sizeof(cplx_t<R>);
    return g;
}

// row-tiled kernel: y-tiles of whole x-rows, z-chunks for every CU
template <int RAD, typename R>
FusedGeom rowtile_geom(const negf_op* op, int w) {
    FusedGeom g;
    const int nx = op->nx, ny = op->ny, nz = op->nz;
    g.whole_plane = false;
    g.nt = (nx * ny <= 256) ? 256 : 1024;
    // as few y-tiles as the block's rows allow, with the rows spread evenly
    // over them (34 rows of 34 points: 17 + 17, not 30 + 4)
    const int rows_max = std::min(ny, g.nt / nx);
    g.n_ytiles = (ny + rows_max - 1) / rows_max;
    g.ty = (ny + g.n_ytiles - 1) / g.n_ytiles;
    // enough work-groups to give every CU work; each z-chunk re-reads 2R planes
    const long target = op->wg_target > 0 ? op->wg_target : ((g.nt == 1024) ? 256 : 1024);
    int zc = nz;
    while ((long)g.n_ytiles * w * ((nz + zc - 1) / zc) < target && zc > 8 * RAD) zc = (zc + 1) / 2;
    g.zchunk = zc;
    g.n_z = (nz + zc - 1) / zc;
    g.lds = 2 * (size_t)(nx + 2 * RAD) * (g.ty + 2 * RAD) * sizeof(cplx_t<R>);
    return g;
}

template <int RAD, typename R>
FusedGeom fused_geom(const negf_op* op, int w) {
    const bool whole_plane = op->nx * op->ny <= 1024 && op->plane_kernel != 0 &&
                             getenv("NEGF_NO_PLANE_KERNEL") == nullptr;
    return whole_plane ? plane_geom<RAD, R>(op, w) : rowtile_geom<RAD, R>(op, w);
}

// gfx950 has 160 KB of LDS per CU; dynamic allocations above 64 KB must be
// opted in, once per kernel and device (host threads of a junction batch may
// get here together)
void allow_large_lds(const void* kernel) {
    static std::mutex mu;
    static std::set<std::pair<const void*, int>> done;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lock(mu);
    if (done.insert({kernel, dev}).second)
        (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

// w columns in the grid; the z-chunking is chosen for w_geom running columns
template <int RAD, typename R, bool FUSED>
void fused_launch(const negf_op* op, const cplx_t<R>* r, const cplx_t<R>* pin, cplx_t<R>* pout,
                  cplx_t<R>* y, int w, int w_geom, const double* shift, const int* skip,
                  const int* kit, const double2* beta, double2* part, hipStream_t s,
                  int live_vectors) {
    const FusedGeom g = fused_geom<RAD, R>(op, w_geom);
    Coef<R> cf;
    for (int m = 0; m < 7; ++m) cf.a[m] = (R)op->coef.a[m];
    dim3 grid(g.n_ytiles * g.n_z, w);
    // The dead streams (p_{k-1} read; p_k and q written) take the
    // non-temporal hint only when the vectors the iteration touches outgrow
    // the last-level cache (256 MiB).  Below it q is still in the cache for
    // the kernel that reads it next: the hint cost the junction batch 6 %
    // (whole-plane) and 4 % (row-tiled), and the multi-shift core 6 % on the
    // 24x24x96 wire (4 x 57 MB), while the per-energy core there (5 x 57 MB)
    // gained 5 % from it; above it the hint gained 2 % on the 32x32x192
    // wire (4 x 201 MB) and 3 % on the 64x64x256 one (4 x 537 MB).
    const bool nth = (double)live_vectors * (double)w * (double)op->N * sizeof(cplx_t<R>) >
                     256.0 * (1 << 20);
    if (g.whole_plane) {
        auto go_plane = [&](auto kern) {
            if (g.lds > 65536) allow_large_lds((const void*)kern);
            hipLaunchKernelGGL(kern, grid, dim3(g.nt), g.lds, s, r, pin, pout, y,
                               reinterpret_cast<cplx_t<R>*>(op->d_sink), op->nx, op->ny, op->nz,
                               g.zchunk, cf, op->coef.a[0], op->d_v, op->d_wz, shift, skip, kit,
                               beta, part);
        };
        if (nth)
            go_plane(k_cocg_plane<RAD, R, FUSED, true>);
        else
            go_plane(k_cocg_plane<RAD, R, FUSED, false>);
        return;
    }
    // y-tiles of a z-chunk grouped on one XCD; NEGF_ROWTILE_XCD=0 deals them
    // out in launch order instead (A/B measurement)
    static const int xcd_group = [] {
        const char* e = getenv("NEGF_ROWTILE_XCD");
        return (e && e[0] == '0') ? 0 : 1;
    }();
    // the row-tiled loads keep no hint: a neighbouring tile re-reads r and
    // p_{k-1} rows as halo
    const int nt_store = nth ? 1 : 0;
    auto go = [&](auto kern, int nt) {
        if (g.lds > 65536) allow_large_lds((const void*)kern);
        hipLaunchKernelGGL(kern, grid, dim3(nt), g.lds, s, r, pin, pout, y, op->nx, op->ny,
                           op->nz, g.ty, g.n_ytiles, g.zchunk, cf, op->coef.a[0], op->d_v,
                           op->d_wz, shift, skip, kit, beta, part, g.n_ytiles > 1 ? xcd_group : 0,
                           nt_store);
    };
    if (g.nt == 256)
        go(k_cocg_apply<RAD, R, 256, FUSED>, 256);
    else
        go(k_cocg_apply<RAD, R, 1024, FUSED>, 1024);
}

template <int RAD, typename R>
void prepare_fused(const negf_op* op) {
    const int pts = op->nx * op->ny;
    // whole-plane kernel: the geometry does not depend on the z-chunking
    if (pts <= 1024) {
        const size_t lds = 2 * (size_t)(op->nx + 2 * RAD) * (op->ny + 2 * RAD) * sizeof(cplx_t<R>);
        if (lds > 65536) {
            allow_large_lds((const void*)k_cocg_plane<RAD, R, true, true>);
            allow_large_lds((const void*)k_cocg_plane<RAD, R, true, false>);
        }
    }
    // row-tiled kernel (also reachable for small planes through the tuner)
    for (int nt : {256, 1024}) {
        if (nt == 256 && pts > 256) continue;
        const int ty = std::min(op->ny, nt / op->nx);
        if (ty < 1) continue;
        const size_t lds = 2 * (size_t)(op->nx + 2 * RAD) * (ty + 2 * RAD) * sizeof(cplx_t<R>);
        if (lds <= 65536) continue;
        if (nt == 256) allow_large_lds((const void*)k_cocg_apply<RAD, R, 256, true>);
        else allow_large_lds((const void*)k_cocg_apply<RAD, R, 1024, true>);
    }
}

template <int RAD>
void prepare_radius(const negf_op* op) {
    prepare_fused<RAD, double>(op);
    prepare_fused<RAD, float>(op);
}

}  // namespace

void prepare_stencil_kernels(const negf_op* op) {
    switch (op->R) {
        case 1: prepare_radius<1>(op); break;
        case 2: prepare_radius<2>(op); break;
        case 3: prepare_radius<3>(op); break;
        case 4: prepare_radius<4>(op); break;
        case 5: prepare_radius<5>(op); break;
        default: prepare_radius<6>(op); break;
    }
}

int fused_partials(const negf_op* op, int w) {
    switch (op->R) {
        case 1: { auto g = fused_geom<1, double>(op, w); return g.n_ytiles * g.n_z; }
        case 2: { auto g = fused_geom<2, double>(op, w); return g.n_ytiles * g.n_z; }
        case 3: { auto g = fused_geom<3, double>(op, w); return g.n_ytiles * g.n_z; }
        case 4: { auto g = fused_geom<4, double>(op, w); return g.n_ytiles * g.n_z; }
        case 5: { auto g = fused_geom<5, double>(op, w); return g.n_ytiles * g.n_z; }
        default: { auto g = fused_geom<6, double>(op, w); return g.n_ytiles * g.n_z; }
    }
}

template <typename R>
void launch_cocg_apply(const negf_op* op, const cplx_t<R>* r, const cplx_t<R>* pin,
                       cplx_t<R>* pout, cplx_t<R>* q, int w, const double* shift, const int* skip,
                       const int* kit, const double2* beta, double2* part, double2* d_kbc,
                       hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, bool kb_scatter,
                       int w_geom, int live_vectors) {
    if (ev0) (void)hipEventRecord(ev0, s);
    const int wg = w_geom > 0 ? w_geom : w;
    const int lv = live_vectors;
    switch (op->R) {
        case 1: fused_launch<1, R, true>(op, r, pin, pout, q, w, wg, shift, skip, kit, beta, part, s, lv); break;
        case 2: fused_launch<2, R, true>(op, r, pin, pout, q, w, wg, shift, skip, kit, beta, part, s, lv); break;
        case 3: fused_launch<3, R, true>(op, r, pin, pout, q, w, wg, shift, skip, kit, beta, part, s, lv); break;
        case 4: fused_launch<4, R, true>(op, r, pin, pout, q, w, wg, shift, skip, kit, beta, part, s, lv); break;
        case 5: fused_launch<5, R, true>(op, r, pin, pout, q, w, wg, shift, skip, kit, beta, part, s, lv); break;
        default: fused_launch<6, R, true>(op, r, pin, pout, q, w, wg, shift, skip, kit, beta, part, s, lv); break;
    }
    if (ev1) (void)hipEventRecord(ev1, s);
    if (op->kb.n_proj > 0) {
        const DeviceKB& kb = op->kb;
        dim3 g1(kb.n_proj, (w + 3) / 4);
        hipLaunchKernelGGL((k_kb_gather<R>), g1, dim3(kThreads), 0, s, pout, op->N, kb.off, kb.idx,
                           kb.val, kb.n_proj, w, d_kbc, skip);
        if (kb_scatter) {
            dim3 g2((kb.n_pts + kThreads - 1) / kThreads, w);
            hipLaunchKernelGGL((k_kb_scatter<R>), g2, dim3(kThreads), 0, s, q, op->N, kb.pts,
                               kb.pt_off, kb.pt_proj, kb.pt_val, kb.n_pts, kb.n_proj, d_kbc, skip);
        }
    }
}

template void launch_cocg_apply<double>(const negf_op*, const double2*, const double2*, double2*,
                                        double2*, int, const double*, const int*, const int*,
                                        const double2*, double2*, double2*, hipStream_t,
                                        hipEvent_t, hipEvent_t, bool, int, int);
template void launch_cocg_apply<float>(const negf_op*, const float2*, const float2*, float2*,
                                       float2*, int, const double*, const int*, const int*,
                                       const double2*, double2*, double2*, hipStream_t,
                                       hipEvent_t, hipEvent_t, bool, int, int);
