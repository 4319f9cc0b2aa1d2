#!/usr/bin/env python
"""Throughput of the real-space NEGF transmission path on one MI355X.

Workload (one step): 64 source columns on the right absorbing region x 256
energies in [0.05, 0.8] Ha of the 32 x 32 x 192 wire (h = 0.4 bohr, radius-6
stencil, 20 seeded Gaussian atoms with s+p separable projectors, 16-plane
quartic absorbing regions), i.e. 16,384 G-column x energy solves reduced to
the shard's partial T(E), FP64, relative residual 1e-10 per (column, energy).
The timed steps take 64-column shards spread evenly over the 256 shards of
the right absorbing region (all 16 of its planes, innermost to outermost);
stored oracle samples that fall in a timed shard are checked.  Inputs are
synthetic (seeded) and resident on the GPU when the timed region starts.

Printed: one JSON line with the solves/s, the roofline entry of the dominant
kernel (the fused stencil step) and the CPU oracle baseline.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import pathlib
import re
import sys
import time

ROOT = pathlib.Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

METRIC = "G-column×energy solves/s at |ΔT|≤1e-6 (mixed vs FP64); matvec HBM GB/s"
HBM_PEAK_GBS = 8000.0
TOL = 1e-10
# the stencil launches of every TIME_EVERY-th chunk of 256 iterations are timed
# with HIP events (run eagerly); the other chunks replay as graphs
TIME_EVERY = 8
# the launch shape every default run uses (stencil work-groups per launch,
# whole-plane kernel); --tune asks the library's autotuner instead
LAUNCH_SHAPE = (192, 1)
COUNTERS = ROOT / "profiles" / "stencil_wire32x32x192_counters.txt"
GOLDEN = ROOT / "tests" / "golden" / "wire32x32x192_samples.json"
# --rows stream: first source column and number of 1024-column calls
STREAM_BEGIN, STREAM_CALLS = 0, 8
KERNEL_SRC = ROOT / "paper_1401_0782_amd" / "csrc" / "stencil.hip"
KERNEL_HELPERS = ROOT / "paper_1401_0782_amd" / "csrc" / "negf_internal.h"


KERNELS = {1: "k_cocg_plane<6,double,true,true>", 0: "k_cocg_apply<6,double,1024,true>"}


def _function_text(src, name):
    """The source of the function (or function template) called name: from
    its template line, or its own line, through the first closing brace at
    column 0; None if the source has no such function."""
    m = re.search(r"^(template <[^\n]*>\n)?[^\n]*\b%s\(" % re.escape(name), src, re.M)
    if not m:
        return None
    end = src.find("\n}\n", m.start())
    return src[m.start(): end + 3 if end >= 0 else len(src)]


GEOMETRY = {"k_cocg_plane": "plane_geom", "k_cocg_apply": "rowtile_geom"}


def kernel_source_hash(kernel):
    """16 hex digits of sha256 over the source the counters depend on: the
    stencil kernel's own function, the function that sets its launch geometry
    and the load / store helpers it calls.  Edits elsewhere in the stencil
    source (the other kernel, comments) leave it unchanged."""
    name = kernel.split("<", 1)[0]
    src = KERNEL_SRC.read_text()
    parts = [_function_text(src, name), _function_text(src, GEOMETRY.get(name, "fused_geom"))]
    if KERNEL_HELPERS.exists():
        helpers = KERNEL_HELPERS.read_text()
        parts += [_function_text(helpers, "ld_once"), _function_text(helpers, "st_once")]
    if parts[0] is None:  # no such kernel: the whole file stands for it
        parts = [src]
    return hashlib.sha256("".join(p or "" for p in parts).encode()).hexdigest()[:16]


def _traffic_from_profile(kernel, shape):
    """HBM bytes over algorithmic bytes of the fused stencil kernel from the
    committed rocprofv3 counter summary at this launch shape (wg_target,
    plane_kernel), or None if missing, taken on other source, on the other
    stencil kernel or at another shape."""
    if not COUNTERS.exists():
        return None, None
    fields = {}
    for line in COUNTERS.read_text().splitlines():
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel") != kernel:
        return None, f"counters were taken on {fields.get('kernel')}, this run used {kernel}"
    if fields.get("kernel_src_sha256_16") != kernel_source_hash(kernel):
        return None, "counters predate the current kernel source"
    tag = f"{shape[0]},{shape[1]}"
    key = ("traffic_over_algorithmic" if fields.get("launch_shape") == tag
           else f"traffic_over_algorithmic_at_{shape[0]}_{shape[1]}")
    if key not in fields:
        return None, f"no counters at launch shape {tag}"
    try:
        # measured with every column of the block active; per-launch traffic of
        # the timed run scales with its (smaller) average active-column count
        return float(fields[key]), None
    except ValueError:
        return None, None


# ---------------------------------------------------------------- CPU oracle leg
def _oracle_worker(args):
    """One process: the oracle's Krylov solve of one (column, energy) item,
    stopped after `seconds`; returns (iterations, seconds)."""
    j, E, seconds = args
    os.environ["OMP_NUM_THREADS"] = "1"
    import numpy as np
    import scipy.sparse.linalg as spla

    import oracle as O
    from workloads import make_wire

    w = make_wire(2)
    A = O.operator_A(w, E).tocsr()
    b = np.zeros(w.N, complex)
    b[j] = 1.0
    n = [0]
    t0 = time.perf_counter()

    class Stop(Exception):
        pass

    def cb(_x):
        n[0] += 1
        if time.perf_counter() - t0 > seconds:
            raise Stop()

    try:
        spla.bicgstab(A, b, rtol=1e-13, atol=0.0, maxiter=10 ** 7, callback=cb)
    except Stop:
        pass
    return n[0], time.perf_counter() - t0


def _oracle_to_completion(e_index):
    """One process: the oracle's BiCGSTAB on column 0 of the right absorbing
    region at energy index e_index, run to completion; returns a record."""
    os.environ["OMP_NUM_THREADS"] = "1"
    import numpy as np
    import scipy.sparse.linalg as spla

    import oracle as O
    from workloads import make_wire, rhs_columns

    w = make_wire(2)
    j = int(rhs_columns(w)[0])
    E = float(w.energies[e_index])
    A = O.operator_A(w, E).tocsr()
    b = np.zeros(w.N, complex)
    b[j] = 1.0
    n = [0]

    def cb(_x):
        n[0] += 1

    t0 = time.perf_counter()
    x, info = spla.bicgstab(A, b, rtol=1e-13, atol=0.0, maxiter=300000, callback=cb)
    res = float(np.linalg.norm(b - A @ x) / np.linalg.norm(b))
    return {"e_index": e_index, "energy": E, "iters": n[0], "info": int(info),
            "seconds": time.perf_counter() - t0, "true_res": res}


def measure_oracle_iterations(e_indices):
    """BiCGSTAB iterations per solve of the oracle at sampled energies (one
    process each; about an hour of CPU time for the slow energies)."""
    with mp.get_context("spawn").Pool(len(e_indices)) as pool:
        for rec in pool.imap(_oracle_to_completion, e_indices):
            print(json.dumps(rec), flush=True)


def _oracle_iters_per_solve():
    f = ROOT / "profiles" / "oracle_wire32x32x192_iters.txt"
    if f.exists():
        for line in f.read_text().splitlines():
            if line.startswith("iterations_per_solve"):
                return int(line.split("=")[1])
    return None


def cpu_baseline(seconds: float):
    from workloads import make_wire, rhs_columns

    w = make_wire(2)
    cols = rhs_columns(w)
    E = float(w.energies[-1])
    n_proc = max(1, min(16, os.cpu_count() or 1))
    items = [(int(cols[(k * 97) % len(cols)]), E, seconds) for k in range(n_proc)]
    with mp.get_context("spawn").Pool(n_proc) as pool:
        res = pool.map(_oracle_worker, items)
    it_rate = sum(n / t for n, t in res)  # BiCGSTAB iterations/s over all workers
    per_solve = _oracle_iters_per_solve()
    value = (it_rate / per_solve) if per_solve else None
    return {
        "value": value,
        "unit": "solves/s",
        "cores": n_proc,
        "kind": "oracle",
        "sample": (f"{n_proc} worker processes (1 BLAS thread each), each running the oracle's "
                   f"iterative route (scipy BiCGSTAB, FP64, sparse A(E)) on its own column at "
                   f"E=0.8 Ha of the same wire for {seconds:.0f} s; measured "
                   f"{it_rate:.1f} iterations/s in total, divided by the mean of "
                   f"{per_solve} iterations per solve over the energy grid (solves run to a true "
                   f"residual of 1e-12 at six sampled energies, "
                   f"profiles/oracle_wire32x32x192_iters.txt)"),
    }


# ---------------------------------------------------------- secondary rows
FP64_PEAK_TFS = 78.6
ROWS = ("small", "mixed", "batch", "full", "adjoint", "large", "large_adjoint", "spectral",
        "current", "copy", "stream")


def precision_forms(P, op, wire, n_cols=4, n_e=4):
    """The metric's comparison, after the timed region and outside it: a
    sample of the same wire (n_cols source columns spread over the right
    absorbing region x n_e energies spread over the grid) in the mixed form
    (FP32 Krylov vectors and matvec, FP64 scalars, true residual and
    refinement; per-energy core), FP64 in the same core, and FP64 in the
    multi-shift core the headline line uses, each timed whole on the host
    clock after the same call has run once.  solves/s, |dT| against the
    multi-shift core, and which form is fastest at |dT| <= 1e-6."""
    import numpy as np
    import torch

    from workloads import rhs_columns

    n_src = len(rhs_columns(wire))
    E = wire.energies[np.linspace(0, wire.energies.size - 1, n_e).astype(int)]
    cols = np.linspace(0, n_src - 1, n_cols).astype(int)
    forms = [("FP64 multi-shift (core B)", dict(core=P.NEGF_CORE_MULTISHIFT, block_width=1)),
             ("FP64 per-energy (core A)", dict(core=P.NEGF_CORE_PER_ENERGY)),
             ("mixed per-energy (core A)", dict(precision=P.NEGF_MIXED))]
    res = {}
    for name, kw in forms:
        def run(**extra):
            return sum(P.negf_transmission(op, E, tol=TOL, col_begin=int(c), col_count=1,
                                           **kw, **extra) for c in cols)
        run(max_iter=32, check=False)  # warm-up: workspace, graphs
        torch.cuda.synchronize()
        t = time.perf_counter()
        T = run()
        torch.cuda.synchronize()
        res[name] = (T, time.perf_counter() - t)
        print(f"precision form {name}: {res[name][1]:.2f} s", file=sys.stderr, flush=True)
    T0 = res[forms[0][0]][0]
    out = {"sample": f"{n_cols} source columns (spread over the right absorbing region) x "
                     f"{n_e} energies, tol {TOL:g}, one column per call"}
    for name, (T, t) in res.items():
        out[name] = {"solves_per_s": n_cols * n_e / t,
                     "max_abs_dT_vs_multishift": float(np.abs(T - T0).max())}
    ok = [n for n in res if out[n]["max_abs_dT_vs_multishift"] <= 1e-6]
    out["fastest_at_dT_1e-6"] = max(ok, key=lambda n: out[n]["solves_per_s"])
    return out


def measure_rows(names):
    """Secondary measurements (one JSON line each): the other workloads and
    forms of the path, timed whole on the host clock around synchronised
    calls, each after a warm-up call (the same call, or one on fewer columns;
    none for the 64x64x256 wire).  Not the headline line."""
    import numpy as np
    import torch

    import paper_1401_0782_amd as P
    from workloads import make_custom, make_junctions, make_wire, rhs_columns

    def emit(**kw):
        print(json.dumps(kw), flush=True)

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t

    for name in names:
        if name == "copy":
            # the practical HBM ceiling the stencil's fraction is read against:
            # torch's device copy (one read, one write) and a two-input add (two
            # reads, one write, the stencil's read/write mix), 4 GiB per operand
            n = 1 << 28
            a = torch.ones(n, dtype=torch.complex128, device="cuda")
            b = torch.ones_like(a)
            c = torch.empty_like(a)
            for form, fn, n_moved in [("copy", lambda: c.copy_(a), 2),
                                      ("add", lambda: torch.add(a, b, out=c), 3)]:
                fn()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                reps = 10
                e0.record()
                for _ in range(reps):
                    fn()
                e1.record()
                torch.cuda.synchronize()
                sec = e0.elapsed_time(e1) / 1e3 / reps
                emit(row=name, form=form, bytes_per_call=n_moved * a.numel() * 16,
                     seconds_per_call=sec, gb_per_s=n_moved * a.numel() * 16 / sec / 1e9)
            del a, b, c
            torch.cuda.empty_cache()
            continue
        if name == "small":
            w = make_wire(1)
            op = P.operator_from_wire(w)
            n, E = len(rhs_columns(w)), w.energies
            P.negf_transmission(op, E, tol=TOL)
            ref, t = timed(lambda: P.negf_transmission(op, E, tol=TOL))
            emit(row=name, workload=f"wire 8x8x32 R=2, {n} cols x {E.size} E", form="core B FP64",
                 seconds=t, solves_per_s=n * E.size / t)
            for form, kw in [("core A FP64 COCG", dict(core=P.NEGF_CORE_PER_ENERGY)),
                             ("core A FP64 QMR", dict(core=P.NEGF_CORE_PER_ENERGY,
                                                      solver=P.NEGF_SOLVER_QMR)),
                             ("core A mixed COCG", dict(precision=P.NEGF_MIXED)),
                             ("core A mixed QMR", dict(precision=P.NEGF_MIXED,
                                                       solver=P.NEGF_SOLVER_QMR))]:
                P.negf_transmission(op, E, tol=TOL, **kw)
                T, t = timed(lambda: P.negf_transmission(op, E, tol=TOL, **kw))
                emit(row=name, form=form, seconds=t, solves_per_s=n * E.size / t,
                     max_dT_vs_core_B=float(np.abs(T - ref).max()))
        elif name == "mixed":
            # the precision form: mixed (FP32 vectors, FP64 scalars, FP64 true
            # residual and refinement) against FP64 in the same per-energy
            # core and against the best FP64 form (multi-shift); each line as
            # soon as its form has run
            for wid, cols, ne in ((1, None, None), (2, 16, 4)):
                w = make_wire(wid)
                op = P.operator_from_wire(w)
                n_all = len(rhs_columns(w))
                n = cols or n_all
                E = w.energies if ne is None else w.energies[np.linspace(0, w.energies.size - 1,
                                                                         ne).astype(int)]
                kw = dict(tol=TOL, col_begin=0, col_count=n)
                ref = {}
                for form, fk in [("core B FP64", dict(core=P.NEGF_CORE_MULTISHIFT)),
                                 ("core A FP64", dict(core=P.NEGF_CORE_PER_ENERGY)),
                                 ("core A mixed", dict(precision=P.NEGF_MIXED))]:
                    (T, d), t = timed(lambda: P.negf_transmission(op, E, n_cols=n, check=False,
                                                                   **kw, **fk))
                    ref.setdefault(form, (T, t))
                    T0, tB = ref["core B FP64"]
                    tA = ref.get("core A FP64", (None, t))[1]
                    emit(row=name, workload=f"{w.name}, {n} cols x {E.size} E", form=form,
                         seconds=t, solves_per_s=n * E.size / t,
                         column_iterations=d.total_iters, status=int(d.status),
                         median_item_iterations=float(np.median(d.iters)),
                         speed_vs_core_A_fp64=tA / t, speed_vs_core_B_fp64=tB / t,
                         max_dT_vs_core_B_fp64=float(np.abs(T - T0).max()))
        elif name == "batch":
            js = make_junctions(64)
            ops = [P.operator_from_wire(j) for j in js]
            es = [j.energies for j in js]
            n_src = [len(rhs_columns(j)) for j in js]
            cols = 16
            run = lambda k: P.negf_transmission_batch(ops, es, tol=TOL, col_begin=0, col_count=k)
            run(1)
            (_, st), t = timed(lambda: run(cols))
            solves = sum(cols * e.size for e in es)
            emit(row=name, workload=f"64 junctions 16^2x64..40^2x160, first {cols} cols x all E",
                 form="batch, core B FP64", seconds=t, solves=solves, solves_per_s=solves / t,
                 statuses_ok=bool(np.all(st == 0)))
            # the same count of columns per junction at a quarter and at three
            # quarters of its absorbing region (8 + 8, one shard per call)
            t_all, ok = 0.0, True
            for f in (0.25, 0.75):
                sh = [(int(f * n) - 4, 8) for n in n_src]
                (_, st), t = timed(lambda: P.negf_transmission_batch(ops, es, tol=TOL, shards=sh))
                t_all += t
                ok = ok and bool(np.all(st == 0))
            emit(row=name, workload=f"64 junctions 16^2x64..40^2x160, 8 cols at 1/4 and 8 at 3/4 "
                 f"of each absorbing region x all E", form="batch (per-junction shards), core B FP64",
                 seconds=t_all, solves=solves, solves_per_s=solves / t_all, statuses_ok=ok)
        elif name in ("full", "adjoint"):
            w = make_wire(4)
            op = P.operator_from_wire(w)
            E, n = w.energies, len(rhs_columns(w))
            if name == "full":
                P.negf_transmission(op, E, tol=TOL, col_begin=0, col_count=64)
                _, t = timed(lambda: P.negf_transmission(op, E, tol=TOL))
                emit(row=name, workload=f"wire 24x24x96 R=4, all {n} cols x {E.size} E",
                     form="core B FP64", seconds=t, solves_per_s=n * E.size / t)
            else:
                wts = np.ones(E.size)
                run = lambda c0, k: P.negf_transmission_grad(op, E, wts, tol=TOL, col_begin=c0,
                                                             col_count=k, block_width=k)
                run(0, 2)
                # four 8-column shards spread over the 12 source planes
                shards = [int(c) for c in np.linspace(0, n - 8, 4)]
                _, t = timed(lambda: [run(c0, 8) for c0 in shards])
                cols = 8 * len(shards)
                emit(row=name, workload=f"wire 24x24x96 R=4, {cols} cols (shards at {shards}) "
                     f"x {E.size} E", form="dT/dV: forward columns from the multi-shift core, "
                     "adjoint solves in the per-energy core", seconds=t,
                     item_solves_per_s=2 * cols * E.size / t,
                     projected_full_minutes=t * n / cols / 60.0)
        elif name == "large_adjoint":
            # the 64x64x256 wire's gradient form: dT/dV summed over 16 selected
            # energies (energies[::64]), on two 2-column shards (innermost and
            # outermost absorbing plane)
            w = make_wire(5)
            op = P.operator_from_wire(w)
            E = w.energies[::64]
            n = len(rhs_columns(w))
            wts = np.ones(E.size)
            run = lambda c0, k: P.negf_transmission_grad(op, E, wts, tol=TOL, col_begin=c0,
                                                         col_count=k, block_width=k)
            run(n // 2, 1)
            shards = [0, n - 2]
            t_all = 0.0
            for c0 in shards:  # one line per shard
                _, t = timed(lambda: run(c0, 2))
                t_all += t
                emit(row=name, workload=f"wire 64x64x256 R=6 KB, cols {c0}..{c0 + 1} x {E.size} E",
                     form="dT/dV shard", seconds=t, item_solves_per_s=2 * 2 * E.size / t)
            cols = 2 * len(shards)
            emit(row=name, workload=f"wire 64x64x256 R=6 KB, {cols} cols (shards at {shards}) "
                 f"x {E.size} E", form="dT/dV: forward columns from the multi-shift core, "
                 "adjoint solves in the per-energy core", seconds=t_all,
                 item_solves_per_s=2 * cols * E.size / t_all,
                 projected_full_hours=t_all * n / cols / 3600.0)
        elif name == "stream":
            # the 32x32x192 workload the way a whole run takes it: source
            # columns streamed through 64 slots (a slot refills at a chunk
            # boundary as soon as its column has finished), by default the
            # first half of the 16,384 columns in 8 calls of 1024, one line
            # each (--stream-begin / --stream-calls pick another range)
            w = make_wire(2)
            op = P.operator_from_wire(w)
            P.negf_set_launch_shape(op, 64, 192, 1)
            E = w.energies
            golden = json.loads(GOLDEN.read_text())["samples"] if GOLDEN.exists() else []
            per, calls, t_all, worst = 1024, STREAM_CALLS, 0.0, 0.0
            first = STREAM_BEGIN
            for k in range(calls):
                c0 = first + k * per
                (T, d), t = timed(lambda: P.negf_transmission(op, E, n_cols=per, tol=TOL,
                                                               col_begin=c0, col_count=per,
                                                               block_width=64))
                t_all += t
                for smp in golden:
                    if c0 <= smp["col"] < c0 + per:
                        worst = max(worst, abs(float(d.t_col[smp["e_index"], smp["col"] - c0])
                                               - smp["t_col"]))
                emit(row=name, workload=f"wire 32x32x192 R=6 KB, columns {c0}..{c0 + per - 1} x "
                     f"{E.size} E, streamed through 64 slots", form="core B FP64", seconds=t,
                     solves_per_s=per * E.size / t, status=int(d.status),
                     column_iterations=d.total_iters)
            n_all = len(rhs_columns(w))
            emit(row=name, workload=f"wire 32x32x192 R=6 KB, columns {first}..{first + calls * per - 1}"
                 f" of {n_all} x {E.size} E", form="core B FP64, streamed", seconds=t_all,
                 solves_per_s=calls * per * E.size / t_all,
                 projected_full_minutes=t_all * n_all / (calls * per) / 60.0,
                 max_abs_dt_vs_oracle_samples=worst)
        elif name == "large":
            w = make_wire(5)
            op = P.operator_from_wire(w)
            E, cols = w.energies, 16
            run = lambda: P.negf_transmission(op, E, n_cols=cols, check=False, tol=TOL,
                                              col_begin=0, col_count=cols, block_width=cols)
            (_, d), t = timed(run)  # one 16-column block of ~50 s: not repeated
            emit(row=name, workload=f"wire 64x64x256 R=6 KB, {cols} cols x {E.size} E",
                 form="core B FP64 (cold)", seconds=t, solves_per_s=cols * E.size / t,
                 column_iterations_per_s=d.total_iters / t, status=int(d.status))
            # wider blocks: the kept-row accumulators X, P of every energy take
            # 2 w n_E n_rows 16 B (86 GB at w = 32; 128 columns would need 343
            # GB), and a whole 32-column block would run ~100 s in one call, so
            # its first 2048 iterations are timed, warm (every stencil launch
            # timed with HIP events; the shift GEMM over 1024 energies runs
            # beside them on its own stream)
            cols, iters = 32, 2048
            run = lambda k: P.negf_transmission(op, E, n_cols=cols, check=False, tol=TOL,
                                                col_begin=0, col_count=cols, block_width=cols,
                                                max_iter=k, time_matvec=1)
            run(256)  # allocates the block's workspace (~110 GB) outside the timing
            (_, d), t = timed(lambda: run(iters))
            x = d.extra
            emit(row=name, workload=f"wire 64x64x256 R=6 KB, {cols} cols x {E.size} E, "
                 f"first {iters} iterations", form=f"core B FP64, block {cols}",
                 seconds=t, column_iterations_per_s=d.total_iters / t,
                 stencil_us_per_launch=1e6 * x["matvec_seconds"] / max(1, x["matvec_launches"]),
                 stencil_gb_per_s=x["matvec_bytes"] / max(1e-30, x["matvec_seconds"]) / 1e9)
        elif name == "spectral":
            # the work depends only on the shapes: random eigenpairs of that size
            w = make_custom(16, 16, 80, 0.5, 4, 10, np.linspace(0.1, 1.0, 1024))
            op = P.operator_from_wire(w)
            n_r, n_l = 2048, 16 * 16 * 10
            rng = np.random.default_rng(5)
            eps = rng.uniform(0, 1.2, n_r) - 1j * rng.uniform(1e-3, 0.1, n_r)
            g = torch.Generator(device="cuda").manual_seed(5)
            U = torch.randn(n_r, w.N, dtype=torch.complex128, device="cuda", generator=g)
            run = lambda: P.negf_spectral_transmission(op, eps, U, w.energies)
            run()
            reps = 5
            _, t = timed(lambda: [run() for _ in range(reps)])
            # two Gram products (left, right CAP rows) and Eq. 13, complex FP64
            flops = 2 * 8.0 * n_r * n_r * n_l + 8.0 * n_r * n_r * w.energies.size
            emit(row=name, workload=f"{n_r} eigenpairs, {n_l} CAP rows per side, "
                 f"{w.energies.size} E", form="Eqs. 8-13 on FP64 MFMA",
                 ms_per_call=1e3 * t / reps, gflop_per_call=flops / 1e9,
                 tflops=flops * reps / t / 1e12,
                 frac_fp64_peak=flops * reps / t / 1e12 / FP64_PEAK_TFS)
        elif name == "current":
            n_e, n_b = 1 << 20, 64
            E = np.linspace(-1.0, 1.0, n_e)
            T = 1.0 / (1.0 + np.exp(-8 * E))
            bias = np.linspace(0.01, 0.5, n_b)
            P.negf_current(E, T, bias, 0.0, 0.01)
            _, t = timed(lambda: P.negf_current(E, T, bias, 0.0, 0.01))
            emit(row=name, workload=f"{n_e} energies x {n_b} biases",
                 form="Eq. 1, host arrays in and out", ms_per_call=1e3 * t)
        else:
            raise SystemExit(f"unknown row {name!r}: choose from {', '.join(ROWS)}")


# ---------------------------------------------------------------- GPU leg
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--block", type=int, default=64, help="source columns per step")
    ap.add_argument("--max-iter", type=int, default=60000)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stream-begin", type=int, default=0,
                    help="--rows stream: first source column (a multiple of 1024)")
    ap.add_argument("--stream-calls", type=int, default=8,
                    help="--rows stream: calls of 1024 columns each")
    ap.add_argument("--no-precision-forms", action="store_true",
                    help="skip the mixed / FP64 comparison on a sample after the timed steps")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB device copy (counter calibration under rocprofv3)")
    ap.add_argument("--launch-shape", type=str, default=None, metavar="WG_TARGET,PLANE",
                    help="stencil launch shape (default %d,%d)" % LAUNCH_SHAPE)
    ap.add_argument("--tune", action="store_true",
                    help="pick the launch shape with the library's autotuner instead")
    ap.add_argument("--oracle-iterations", type=str, default=None, metavar="E_IDX,...",
                    help="CPU only: run the oracle's BiCGSTAB to completion at these energy "
                         "indices and print the iteration counts (the CPU baseline's scale)")
    ap.add_argument("--rows", type=str, default=None, metavar="ROW,...",
                    help="instead of the headline step, time other workloads and forms: "
                         + ", ".join(ROWS))
    args = ap.parse_args()
    if args.rows:
        bad = [r for r in args.rows.split(",") if r not in ROWS]
        if bad:
            ap.error(f"unknown rows {', '.join(bad)}: choose from {', '.join(ROWS)}")
    if args.oracle_iterations:
        measure_oracle_iterations([int(v) for v in args.oracle_iterations.split(",")])
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(columns would shard across GPUs with one all-reduce of T(E)); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.rows:
        global STREAM_BEGIN, STREAM_CALLS
        STREAM_BEGIN, STREAM_CALLS = args.stream_begin, args.stream_calls
        measure_rows(args.rows.split(","))
        return
    import paper_1401_0782_amd as P
    from workloads import make_wire, rhs_columns

    wire = make_wire(2)
    op = P.operator_from_wire(wire)
    n_src = len(rhs_columns(wire))
    n_e = len(wire.energies)

    if args.calibrate_copy:
        a = torch.empty(1 << 27, dtype=torch.complex64, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    # launch shape (z-chunking, stencil kernel): fixed, so that every run, its
    # kernel statistics and its counters share one shape (the autotuner's
    # choice between close candidates varies from run to run)
    if args.tune:
        tuned = P.negf_tune(op, wire.energies, block_width=args.block)
    else:
        tgt, plane = ((int(v) for v in args.launch_shape.split(",")) if args.launch_shape
                      else LAUNCH_SHAPE)
        P.negf_set_launch_shape(op, args.block, tgt, plane)
        tuned = {"block_width": args.block, "wg_target": tgt, "plane_kernel": plane}
    plane_fits = wire.nx * wire.ny <= 1024
    kernel = KERNELS[1 if (tuned["plane_kernel"] != 0 and plane_fits) else 0]
    print(f"tuned launch shape: block {tuned['block_width']}, stencil work-groups "
          f"{tuned['wg_target']}, whole-plane kernel {tuned['plane_kernel']}",
          file=sys.stderr, flush=True)

    # timed shards spread evenly over the right absorbing region; warm-up
    # shards in between
    n_blk = n_src // args.block
    timed_blk = [int(b) for b in np.round(np.linspace(0, n_blk - 1, args.steps))]
    warm_blk = [int(b) for b in np.round(np.linspace(0, n_blk - 1, args.warmup + 2))[1:-1]]
    golden = json.loads(GOLDEN.read_text())["samples"] if GOLDEN.exists() else []
    checked = []

    def step(blk):
        c0 = blk * args.block
        T, d = P.negf_transmission(op, wire.energies, n_cols=args.block, check=False,
                                   time_matvec=TIME_EVERY, col_begin=c0, col_count=args.block,
                                   block_width=args.block, tol=TOL, max_iter=args.max_iter)
        if d.status not in (0, 4):  # anything but OK / NOT_CONVERGED is a failure
            raise RuntimeError(f"negf_transmission failed: status {d.status}: "
                               f"{P.api._lib().negf_last_error().decode()}")
        return T, d

    for i in range(args.warmup):
        step(warm_blk[i])
        print(f"warmup step {i} done (shard {warm_blk[i]})", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mv_s = mv_b = 0.0
    mv_n = 0
    not_conv = 0
    iters = 0
    for i in range(args.steps):
        T, d = step(timed_blk[i])
        for smp in golden:
            if smp["col"] // args.block == timed_blk[i]:
                t = float(d.t_col[smp["e_index"], smp["col"] - timed_blk[i] * args.block])
                checked.append((smp["col"], smp["e_index"], abs(t - smp["t_col"]), smp["t_col"]))
        mv_s += d.extra["matvec_seconds"]
        mv_b += d.extra["matvec_bytes"]
        mv_n += d.extra["matvec_launches"]
        not_conv += d.n_not_converged
        iters += d.total_iters
        print(f"step {i} done (shard {timed_blk[i]}, {d.seconds:.2f} s, "
              f"{d.total_iters} column-iterations)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    solves = args.steps * args.block * n_e
    value = solves / elapsed
    achieved = mv_b / mv_s / 1e9 if mv_s > 0 else None
    ratio, why = _traffic_from_profile(kernel, (tuned["wg_target"], tuned["plane_kernel"]))
    traffic = ratio * mv_b / max(1, mv_n) if ratio else None
    roofline = {
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
        "traffic": traffic,  # HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)
        "kernel": kernel + " (fused p = r + beta p, stencil + potential + CAP apply, p^T q partials)",
        "launches": mv_n,
        "timed_sample": f"stencil launches of every {TIME_EVERY}th chunk of 256 iterations "
                        f"(launched eagerly, the shift GEMM overlapping as in the other chunks), "
                        f"{mv_n} launches over the timed steps",
        "avg_launch_us": 1e6 * mv_s / max(1, mv_n),
        "bytes_per_launch": mv_b / max(1, mv_n),
    }
    if why:
        roofline["traffic_note"] = why
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": ("wire 32x32x192 h=0.4 R=6, 20 atoms + s,p KB projectors, CAP 16 planes; "
                         f"{args.block} source columns x {n_e} energies per step, FP64 multi-shift "
                         f"COCG, tol {TOL:g}"),
            "solves_per_step": args.block * n_e,
            "launch_shape": {k: tuned[k] for k in ("block_width", "wg_target", "plane_kernel")},
            "column_iterations": iters,
            "not_converged": not_conv,
            "timed_shards": timed_blk,
            "oracle_samples_checked": [
                {"col": c, "e_index": e, "abs_dt": dt, "t_oracle": t} for c, e, dt, t in checked],
            "max_abs_dt_vs_oracle": max((c[2] for c in checked), default=None),
        },
        "roofline": roofline,
    }
    if not args.no_precision_forms:
        out["precision_forms"] = precision_forms(P, op, wire)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
