/*
 * negf.h - C ABI of libnegf: real-space NEGF transmission on MI355X (gfx950).
 *
 * The library computes columns of the retarded Green's function
 *     G(E) = A(E)^-1,   A(E) = E*1 - H + i(W_L + W_R)
 * of a real-space operator H = -1/2 Lap_h + diag(V) + sum_p E_p b_p b_p^T on a
 * uniform grid (Sec. II.C: finite-difference Laplacian, local potential and a
 * non-local separable pseudopotential inside a cutoff), with z-only absorbing
 * potentials W_L, W_R (Sec. II.B, Eqs. 4-5; they play the anti-Hermitian part
 * of the lead self-energies, so the coupling matrices are Gamma = 2W).  Since
 * H is real symmetric and W diagonal, A(E) is complex symmetric (Eq. 6).  The
 * transmission is reduced from the block of G between the two absorbing
 * regions (Eq. 7, with Gamma = 2W):
 *     T(E) = 4 sum_{i in L, j in R} W_L,i W_R,j |G_ij(E)|^2 .
 *
 * Grid convention: point (ix,iy,iz) (0-based) sits at ((ix+1)h,(iy+1)h,(iz+1)h);
 * linear index i = ix + nx*(iy + ny*iz) (x fastest); Dirichlet walls one
 * spacing beyond the first and last points (ghost values are zero).  The
 * Laplacian is the order-2R central star stencil along each axis, 1 <= R <= 6.
 *
 * Ownership: every input is copied before the call returns; the caller keeps
 * ownership of all its buffers.  Outputs are caller-allocated.  Pointers are
 * host pointers unless a parameter says "host or device", in which case the
 * library asks the HIP runtime which kind it is.
 *
 * Errors: no exception crosses the ABI.  A status other than NEGF_OK leaves
 * outputs undefined, except NEGF_E_NOT_CONVERGED, which returns every result
 * together with per-item status codes.  negf_last_error() gives a message for
 * the last failing call of the calling thread.
 *
 * Concurrency: a negf_op may be used by one thread at a time; distinct ops
 * are independent.  Work is queued on opts->stream (a hipStream_t), or on a
 * stream owned by the op when that is NULL; calls return after their work on
 * that stream has finished.
 */
#ifndef NEGF_H
#define NEGF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NEGF_OK = 0,
    NEGF_E_INVALID_ARG = 1,    /* rejected before any device work */
    NEGF_E_OUT_OF_MEMORY = 2,  /* device allocation failed; nothing leaked */
    NEGF_E_DEVICE = 3,         /* a HIP call failed */
    NEGF_E_NOT_CONVERGED = 4,  /* some item missed tol within max_iter */
    NEGF_E_BREAKDOWN = 5       /* a COCG recurrence broke down (p^T A p or r^T r ~ 0) */
} negf_status;

/* per-item status codes written to item_status arrays */
enum {
    NEGF_ITEM_CONVERGED = 0,
    NEGF_ITEM_MAX_ITER = 1,
    NEGF_ITEM_BREAKDOWN = 2,
    /* the residual test passed but the optical-theorem check (negf_diag.
       optical_err, when requested) failed: error above max(1e4 tol, 1e-8).
       The multi-shift core stops on the COCG residual estimate, which on
       hard systems can drift far from the true residual */
    NEGF_ITEM_INACCURATE = 3
};

/* negf_opts.precision */
enum {
    NEGF_FP64 = 0,  /* Krylov vectors, matvec, scalars and reductions in FP64 */
    NEGF_MIXED = 1  /* FP32 matvec and Krylov vectors; FP64 scalars, dots,
                       true residual b - A x, solution accumulation and T */
};

/* negf_opts.core */
enum {
    NEGF_CORE_AUTO = 0,
    NEGF_CORE_PER_ENERGY = 1, /* one COCG run per (column, energy) item */
    NEGF_CORE_MULTISHIFT = 2  /* one COCG run per column serves every energy */
};

/* negf_opts.solver */
enum {
    NEGF_SOLVER_COCG = 0, /* conjugate orthogonal CG (bilinear form, Eq. 6 symmetry) */
    NEGF_SOLVER_QMR = 1   /* simplified (symmetric) QMR: the same Lanczos recurrences
                             with quasi-minimal-residual smoothing of the iterate;
                             per-energy core only */
};

/* negf_opts.recover for negf_transmission */
enum {
    NEGF_RECOVER_OFF = 0,     /* report what the chosen core reaches */
    NEGF_RECOVER_RESTART = 1  /* multi-shift items that end in breakdown, at
                                 max_iter or inaccurate are solved again, each
                                 as its own seed system, in the FP64
                                 per-energy core (COCG; items COCG still fails
                                 then by QMR); the optical-theorem check runs
                                 whether or not negf_diag asks for it; the
                                 re-solved items' diagnostics are those of the
                                 re-solve, iters the sum over all runs.  In a
                                 junction batch such junctions run one at a
                                 time */
};

/* negf_opts.direction for negf_transmission */
enum {
    NEGF_DIR_RL = 0, /* columns on the right CAP support, rows on the left */
    NEGF_DIR_LR = 1  /* columns on the left, rows on the right (reciprocity) */
};

typedef struct { double re, im; } negf_c64;

typedef struct {
    int32_t nx, ny, nz; /* interior grid points per axis, each >= 1 */
    double h;           /* grid spacing in bohr, > 0 */
} negf_grid;

/* Separable projectors b_p (CSR by projector): the values of b_p are
 * val[offsets[p] .. offsets[p+1]) at grid indices idx[...]; E_p = e_kb[p]. */
typedef struct {
    int32_t n_proj;
    const int64_t* offsets; /* n_proj + 1, offsets[0] = 0, non-decreasing */
    const int32_t* idx;     /* offsets[n_proj] grid indices in [0, N) */
    const double* val;      /* offsets[n_proj] real values */
    const double* e_kb;     /* n_proj energies (Ha) */
} negf_kb;

typedef struct {
    int32_t precision;   /* NEGF_FP64 or NEGF_MIXED */
    int32_t core;        /* NEGF_CORE_* */
    int32_t solver;      /* NEGF_SOLVER_*; QMR selects the per-energy core under AUTO
                            and is rejected with NEGF_CORE_MULTISHIFT */
    int32_t direction;   /* NEGF_DIR_* (negf_transmission only) */
    double tol;          /* relative residual per (column, energy); FP64 path:
                            COCG residual estimate; mixed path: true FP64
                            residual ||b - A x|| / ||b||.  0 -> 1e-10 */
    int32_t max_iter;    /* Krylov iterations per run; 0 -> 100000 */
    int32_t block_width; /* columns (or items) per block; 0 -> auto */
    int32_t shift_group; /* energies per multi-shift run; 0 -> all */
    int32_t max_refine;  /* mixed: outer refinement steps, each an FP32 solve
                            of up to max_iter iterations on the FP64 residual;
                            0 -> 8 */
    int32_t col_begin;   /* negf_transmission(_grad): first source column of the */
    int32_t col_count;   /* shard to sum over (0 -> all); T is then that shard's
                            partial sum, which shards add up to the full T(E) */
    void* stream;        /* hipStream_t or NULL */
    int32_t recover;     /* NEGF_RECOVER_* (negf_transmission, multi-shift core) */
} negf_opts;

/* Optional diagnostics of negf_transmission.  Each array is nullable and is
 * indexed [e * n_cols + c], n_cols = number of source columns
 * (nx*ny*planes of the source CAP). */
typedef struct {
    int32_t* iters;          /* Krylov iterations used for the item */
    double* resid;           /* final relative residual: per-energy core, the FP64
                                true residual ||b - A x|| / ||b||; multi-shift core,
                                the COCG residual estimate ||r_k|| / (|pi_k| ||b||)
                                at which the energy froze (that core never forms an
                                energy's full-length iterate) */
    double* t_col;           /* per-column transmission t_j(E) */
    int32_t* item_status;    /* NEGF_ITEM_* */
    int64_t total_iters;     /* out: sum of Krylov iterations over runs */
    int32_t n_not_converged; /* out */
    double seconds;          /* out: wall time of the device work */
    int32_t time_matvec;     /* in: 0 off; 1 brackets every fused stencil launch with
                                HIP events on the work stream (launched eagerly);
                                n > 1: in the multi-shift core, the launches of
                                every n-th chunk of 256 iterations are timed that
                                way and the other chunks replay as graphs (the
                                per-energy core times every launch) */
    double matvec_seconds;   /* out: summed duration of the timed launches */
    int64_t matvec_launches; /* out: number of stencil launches timed */
    double matvec_bytes;     /* out: algorithmic HBM bytes of those launches: per
                                active column r and p_{k-1} read, p_k and q written
                                (16 B per point in FP64, 8 B in FP32), plus V once */
    double* optical_err;     /* per item, the optical theorem of the column
                                g_j = A^-1 e_j (from A = E - H + iW, Eq. 4, H real):
                                |sum_i W_i |g_ij|^2 + Im g_jj| / |Im g_jj| over both
                                absorbing regions.  Requesting it makes the
                                multi-shift core also keep the source side's rows
                                (twice the kept rows), and items above
                                max(1e4 tol, 1e-8) report NEGF_ITEM_INACCURATE */
    int32_t* refine_steps;   /* per item, outer refinement steps of the per-energy
                                core (0 in the multi-shift core) */
} negf_diag;

typedef struct negf_op negf_op;

/* Builds the operator of Sec. II.B-C on the current HIP device.
 *   g           grid sizes and spacing
 *   stencil_radius  R in 1..6 (order-2R finite differences)
 *   v_local     N = nx*ny*nz local potential values (Ha), finite
 *   kb          separable projectors, or NULL for none
 *   cap_left_z  nz values W_L(z) >= 0, nonzero only on leading planes
 *   cap_right_z nz values W_R(z) >= 0, nonzero only on trailing planes
 * Requirements (else NEGF_E_INVALID_ARG): the two supports are disjoint,
 * each is a contiguous run of at least R planes touching its wall (this
 * makes A(E) nonsingular for real E without projectors), no projector
 * point lies on a CAP plane, and nx is at most the widest x-row the stencil
 * tile holds: min(1024, 163840 / (32 (2R+1)) - 2R), i.e. 1024, 1020, 725,
 * 560, 455, 381 for R = 1..6 (one thread per point of a row, and one row
 * with its radius-R halo in a double-buffered FP64 LDS tile of 160 KB);
 * the tile of t rows then needs 32 (t + 2R)(nx + 2R) <= 163840 bytes, with
 * t = ny for planes of at most 1024 points, else min(ny, 1024 / nx), which
 * excludes only narrow, tall planes (such as 2 x 512 or 3 x 400 at R = 6).
 * *out receives a new op; free with negf_destroy. */
negf_status negf_build_operator(const negf_grid* g, int32_t stencil_radius,
                                const double* v_local, const negf_kb* kb,
                                const double* cap_left_z, const double* cap_right_z,
                                negf_op** out);

/* Y = A(E_c) X for a block of n_vec complex vectors (the matvec of the hot
 * loop; Sec. II.C names it the bottleneck of iterative methods).
 *   precision   NEGF_FP64 or NEGF_MIXED (FP32 arithmetic, FP64 in and out)
 *   shifts      n_vec host energies E_c
 *   x, y        [n_vec][N] host or device (both the same kind) */
negf_status negf_apply_operator(negf_op* op, int32_t precision, int32_t n_vec,
                                const double* shifts, const negf_c64* x, negf_c64* y);

/* The FP64 operator apply of negf_apply_operator without any device
 * allocation, for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation after
 * start-up.  Its scratch data (the n_vec shifts and the n_vec x n_proj
 * projector coefficients) lives in a fixed array of
 * NEGF_NOALLOC_SCRATCH_BYTES per GPU that the library holds until the
 * process ends: 256-byte-rounded 8 n_vec plus 16 n_vec max(1, n_proj) bytes
 * must fit, else NEGF_E_INVALID_ARG (nothing is launched).  Calls that
 * overlap on one GPU share that array and race: serialise them.
 *   shifts   n_vec energies E_c, host or device (a host array is copied into
 *            the scratch array on the stream; under graph capture pass a
 *            device array)
 *   x, y     [n_vec][N] device memory, not overlapping
 *   stream   hipStream_t to queue the work on and return without waiting, or
 *            NULL: the op's own stream, waited for before returning */
#define NEGF_NOALLOC_SCRATCH_BYTES (1 << 20)
negf_status negf_apply_operator_noalloc(negf_op* op, int32_t n_vec, const double* shifts,
                                        const negf_c64* x, negf_c64* y, void* stream);

/* Columns of G(E) (Eq. 3): out[e][r][k] = (A(E_e)^-1 b_r)[row_idx[k]].
 *   n_e, energies   host energies
 *   n_rhs           number of right-hand sides
 *   rhs_idx         n_rhs grid indices (b_r = unit vector), or NULL
 *   rhs_dense       [n_rhs][N] host or device dense right-hand sides, or NULL
 *                   (exactly one of rhs_idx / rhs_dense is non-NULL)
 *   n_rows, row_idx rows to return; row_idx NULL means all N rows (n_rows = N)
 *   out             [n_e][n_rhs][n_rows] host or device
 *   item_status     [n_e][n_rhs] host, nullable */
negf_status negf_solve_columns(negf_op* op, const negf_opts* opts, int32_t n_e,
                               const double* energies, int32_t n_rhs,
                               const int32_t* rhs_idx, const negf_c64* rhs_dense,
                               int32_t n_rows, const int32_t* row_idx,
                               negf_c64* out, int32_t* item_status);

/* T(E) of Eq. 7 (factor 4 for Gamma = 2W) for n_e host energies into the
 * host array T[n_e] (FP64).  diag is nullable. */
negf_status negf_transmission(negf_op* op, const negf_opts* opts, int32_t n_e,
                              const double* energies, double* T, negf_diag* diag);

/* Batched T(E) over n_ops independent junctions (each its own operator, grid
 * and energy grid), submitted together so that the device overlaps them.
 * One host thread keeps up to max_concurrent junctions in flight, largest
 * first, each on its operator's own stream: the multi-shift core advances in
 * chunks of iterations (HIP-graph replays), and the thread queues a
 * junction's next chunk as soon as its previous one has finished (event
 * polling, no blocking wait on any one junction).  Junctions that do not run
 * in the FP64 multi-shift core with every energy in one shift group (mixed
 * precision, per-energy core, shift groups) are solved one at a time by the
 * same thread.  Each op's workspace is released when its junction finishes.
 * Equivalent to calling negf_transmission(ops[i], opts, n_e[i], energies[i],
 * T[i], NULL) for every i; the per-op results are bit-identical to that.
 *   ops         n_ops operators (distinct)
 *   n_e, energies, T   per-op energy counts, host energy arrays, host outputs
 *   status      n_ops host per-op negf_status codes (nullable); a junction
 *               whose items missed tol keeps its T and reports
 *               NEGF_E_NOT_CONVERGED, like negf_transmission
 *   max_concurrent   junctions in flight (0 -> 4)
 * Returns the first non-OK per-op status, or NEGF_OK. */
negf_status negf_transmission_batch(int32_t n_ops, negf_op* const* ops, const negf_opts* opts,
                                    const int32_t* n_e, const double* const* energies,
                                    double* const* T, int32_t* status, int32_t max_concurrent);

/* negf_transmission_batch with a source-column shard per junction: junction
 * i sums over its columns [col_begin[i], col_begin[i] + col_count[i]) (the
 * meaning of negf_opts.col_begin / col_count, which these arrays replace;
 * col_count 0 -> to the last column), e.g. to sample every junction at the
 * same relative place in its absorbing region.  Equivalent to calling
 * negf_transmission for each junction with its own shard; bit-identical.
 *   col_begin, col_count   n_ops host values each, non-null, >= 0 */
negf_status negf_transmission_batch_shards(int32_t n_ops, negf_op* const* ops,
                                           const negf_opts* opts, const int32_t* n_e,
                                           const double* const* energies, const int32_t* col_begin,
                                           const int32_t* col_count, double* const* T,
                                           int32_t* status, int32_t max_concurrent);

/* Launch-shape autotuner for the multi-shift core (the batching form's
 * tuned block width, z-chunking and stencil kernel).  It times a short run of
 * probe_iters COCG iterations (0 -> one chunk: 128 iterations, 256 on grids of
 * 131,072 points or more; so one blocked shift
 * accumulation is included) of the op's first source columns at the given
 * energies for every candidate, on the op's stream, and keeps the candidate
 * with the least device time per column-iteration in the op.  Later
 * negf_transmission / negf_solve_columns calls on this op whose
 * opts->block_width is 0 use the tuned width; the z-chunking and kernel choice
 * apply to every later stencil launch on this op.
 * Candidates: block width 16, 32, 64, 128, 256 (capped at the source column
 * count, and to widths whose workspace at opts->max_iter fits in half of the
 * free device memory; only opts->block_width when that is nonzero) x stencil
 * work-group targets
 * 128, 192, 256, 512, 1024 per launch x {whole-plane kernel, row-tiled kernel}
 * (the whole-plane kernel only where one plane fits a work-group).
 * Results are identical up to rounding for every candidate: only the launch
 * shape changes.  Probes that hit max_iter are expected and not errors.
 *   opts      direction, shift_group, block_width and stream are read
 *   result    nullable; receives the choice and the timing table */
#define NEGF_TUNE_MAX 64
typedef struct {
    int32_t block_width;  /* chosen source columns per block */
    int32_t wg_target;    /* chosen stencil work-groups per launch (z-chunking) */
    int32_t plane_kernel; /* 1 whole-plane stencil kernel, 0 row-tiled */
    int32_t n_tried;
    int32_t tried_block_width[NEGF_TUNE_MAX];
    int32_t tried_wg_target[NEGF_TUNE_MAX];
    int32_t tried_plane_kernel[NEGF_TUNE_MAX];
    double us_per_column_iteration[NEGF_TUNE_MAX];
} negf_tune_result;

negf_status negf_tune(negf_op* op, const negf_opts* opts, int32_t n_e, const double* energies,
                      int32_t probe_iters, negf_tune_result* result);

/* negf_tune with an on-disk cache of its choice.  The key is the operator's
 * shape and the tuning request: grid (nx, ny, nz), stencil radius, projector
 * count, source columns and kept rows of opts->direction, energies per shift
 * group, opts->block_width, probe_iters, and the device (architecture name
 * and compute-unit count).  A key found in cache_path sets the stored shape
 * without any probe (result->n_tried = 0, result->us_per_column_iteration[0]
 * the stored timing); otherwise negf_tune runs and one line is appended to
 * the file (created if missing).  The file is plain text, one
 * "key => block_width wg_target plane_kernel us" line per entry; the last
 * line for a key wins, and lines that do not parse are skipped.  Entries of
 * an older library version are not used (the version is part of the key).
 *   cache_path  a file path; NEGF_E_INVALID_ARG if null or empty.  File
 *               errors are not failures: a missing or unreadable cache
 *               reads as empty, and a choice that cannot be appended is
 *               still set on the operator and returned. */
negf_status negf_tune_cached(negf_op* op, const negf_opts* opts, int32_t n_e,
                             const double* energies, int32_t probe_iters,
                             const char* cache_path, negf_tune_result* result);

/* Sets the launch shape negf_tune would keep, e.g. one cached from an earlier
 * process: block_width 0 and wg_target 0 restore the built-in defaults (64
 * columns; 256 stencil work-groups per launch), plane_kernel -1 the automatic
 * kernel choice.  block_width in [0, 4096], wg_target in [0, 65536],
 * plane_kernel in {-1, 0, 1}; a whole-plane request on a grid whose plane does
 * not fit one work-group falls back to the row-tiled kernel. */
negf_status negf_set_launch_shape(negf_op* op, int32_t block_width, int32_t wg_target,
                                  int32_t plane_kernel);

/* Adjoint gradient of L = sum_e weights[e] T(E_e) with respect to the local
 * potential: dL_dV[r] = sum_e w_e 8 Re sum_{j in R} W_R,j lambda_j(r) g_j(r),
 * with g_j = A^-1 e_j and lambda_j = A^-1 (W_L o conj(g_j)) solved with the
 * same complex symmetric operator (A^T = A, Eq. 6).  The forward columns g_j
 * (right-hand sides independent of E) come from one multi-shift run per
 * block of columns at every energy, all rows kept; the adjoint solves, whose
 * right-hand sides depend on E, run in the per-energy core.  opts->tol bounds
 * both (FP64; opts->precision is not used).
 *   weights   n_e host values; dL_dV  N host or device FP64;
 *   T         optional host n_e output of T(E) (nullable). */
negf_status negf_transmission_grad(negf_op* op, const negf_opts* opts, int32_t n_e,
                                   const double* energies, const double* weights,
                                   double* dL_dV, double* T);

/* Eigenpairs (eps_i, U_i) of the open-system operator H_op = H - i(W_L + W_R)
 * (Eq. 8) whose real parts lie in [e_lo - margin, e_hi + margin], for the
 * spectral route of negf_spectral_transmission (Sec. II.C; the paper obtains
 * them with ARPACK's iterative complex diagonalisation).  Complex-symmetric
 * Lanczos in the bilinear form u^T v on the device, every new vector
 * re-orthogonalised twice against all earlier ones (this keeps the process
 * from duplicating or missing eigenpairs, the instability Sec. II.D reports
 * for plain complex-symmetric Lanczos); the eigenvalues of the tridiagonal
 * projection by implicit QL with complex orthogonal rotations, its
 * eigenvectors by inverse iteration, the Ritz vectors V y on the device.
 * The low end of the spectrum, where transport windows lie, converges first.
 *   n_lanczos   Krylov dimension K (at most N; K = N finds every eigenpair
 *               of small operators); device memory (K + 1) N complex FP64
 *   resid_tol   a Ritz pair is returned only if
 *               ||H_op U - eps U|| / ||U|| <= resid_tol (Ha)
 *   max_pairs   capacity of eps, U and resid
 *   eps         host [max_pairs] out, ascending real part
 *   U           [max_pairs][N] out (host or device), U_i^T U_i = 1 (Eqs. 9-11)
 *   resid       host [max_pairs] out (nullable): each pair's residual
 *   n_found     host out: pairs returned
 * NEGF_E_BREAKDOWN if no start vector has a nonzero bilinear form or the
 * tridiagonal eigenvalue iteration breaks down; a Krylov space that closes
 * early (an invariant subspace, or a new vector with w^T w = 0) ends the
 * process there and returns what it found. */
negf_status negf_eigenpairs(negf_op* op, double e_lo, double e_hi, double margin,
                            int32_t n_lanczos, double resid_tol, int32_t max_pairs,
                            negf_c64* eps, negf_c64* U, double* resid, int32_t* n_found);

/* Landauer current of Eq. 1 from a transmission curve, on the device:
 *   I(V_b) = (1/pi) int T(E) [f(E - mu_L) - f(E - mu_R)] dE   (atomic units,
 *   2e/h = 1/pi), mu_{L,R} = e_fermi +- V_b / 2, f the Fermi function at
 *   temperature kT (Ha; 0 gives a step with f(0) = 1/2),
 * by the trapezoid rule on the given energy grid (the bias window should lie
 * inside it; outside the grid T counts as zero).
 *   n_e >= 2 energies, strictly increasing (host or device), and T[n_e] (host
 *   or device, e.g. the output of negf_transmission);
 *   n_bias bias voltages V_b (Ha/e; host or device); current[n_bias] output
 *   (host or device).  stream: hipStream_t or NULL (the null stream).
 * Invalid arguments (non-finite or unsorted energies, kT < 0, null
 * pointers) are rejected before any device call.  Needs no operator. */
negf_status negf_current(int32_t n_e, const double* energies, const double* T, int32_t n_bias,
                         const double* bias, double e_fermi, double kT, double* current,
                         void* stream);

/* The complex-energy diagonalisation route of Sec. II.C (Eqs. 8-13) from
 * eigenpairs (eps_i, U_i) of H_op = H - i(W_L + W_R) for this op's H and CAPs,
 * supplied by the caller (the paper obtains them with ARPACK):
 *   T(E) = sum_ij Gt_L,ij Gt_R,ji / ((E - eps_j)(E - conj(eps_i)))   (Eq. 13),
 *   Gt_L = U^H Gamma_L U,  Gt_R = U^T Gamma_R conj(U),  Gamma = 2W    (Eq. 12),
 * with the eigenvectors complex-normalised, U_i^T U_i = 1 (Eqs. 9-11).  With
 * every eigenpair this equals negf_transmission's T(E); keep in (0, 1) keeps
 * the round(keep * n_r) eigenpairs whose real parts lie nearest the middle of
 * the energy window (ties by index), the truncation of Sec. II.D, whose
 * missing poles are the route's known artefact; keep 0 or 1 keeps all.
 *   eps    n_r host eigenvalues;  U  [n_r][N] eigenvectors, each contiguous
 *          (host or device);  energies  n_e host values;  T  n_e host output.
 * The Gram products over the CAP rows and the double sum over all energies
 * run on the FP64 matrix cores.  Rejects non-finite input and energies that
 * coincide with a kept eigenvalue. */
negf_status negf_spectral_transmission(negf_op* op, int32_t n_r, const negf_c64* eps,
                                       const negf_c64* U, double keep, int32_t n_e,
                                       const double* energies, double* T);

/* Frees the op and all device memory it owns.  NULL is a no-op. */
void negf_destroy(negf_op* op);

/* Message of the last failing call on this thread ("" if none). */
const char* negf_last_error(void);

/* Library version string. */
const char* negf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NEGF_H */
