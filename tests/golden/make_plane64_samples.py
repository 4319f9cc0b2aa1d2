"""Write oracle samples of a short wire with 64 x 64 planes at radius 6.

Planes of 4,096 points (the cross-section of the 64x64x256 workload) take the
row-tiled stencil kernel, split into y-tiles whose radius-6 halo crosses the
tile boundaries.  The oracle's iterative route (scipy Krylov on the oracle's
sparse A(E), true relative residual <= 1e-12) solves each requested source
column at each energy; the file keeps G at chosen rows and
t_j(E) = 4 W_R,j sum_{i in L} W_L,i |G_ij|^2 (Eq. 7 with Gamma = 2W).
Only oracle/ and the input generator are used.

usage: python tests/golden/make_plane64_samples.py
writes tests/golden/plane64x64x25_samples.json (one process per solve)
"""

import json
import multiprocessing as mp
import os
import pathlib
import sys
import time

ROOT = pathlib.Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))
OUT = pathlib.Path(__file__).resolve().parent / "plane64x64x25_samples.json"

# make_custom arguments: 64 x 64 x 25 grid, h = 0.35, R = 6, 6-plane CAPs,
# one atom with s+p projectors on the axis (its 2-bohr sphere spans planes
# 7..17, one plane clear of both CAPs) and one off-axis well
WIRE = {
    "nx": 64, "ny": 64, "nz": 25, "h": 0.35, "R": 6, "n_cap": 6,
    "energies": [0.45, 0.9],
    "wells": [[11.375, 11.375, 4.55, 0.5], [6.0, 17.0, 4.2, 0.35]],
    "atoms_kb": [[0.8, 0.3, 0.12], [0.7, 0.25, 0.1]],
}
# source columns (x, y) on the innermost right-CAP plane: both sides of the
# y-tile boundaries at y = 16 and y = 48 (16 rows per tile), and the corners
SOURCES = [(10, 15), (40, 16), (63, 47), (0, 48)]


def make():
    from workloads import make_custom

    p = WIRE
    return make_custom(p["nx"], p["ny"], p["nz"], p["h"], p["R"], p["n_cap"], p["energies"],
                       wells=[tuple(w) for w in p["wells"]],
                       atoms_kb=[tuple(a) for a in p["atoms_kb"]], name="plane64")


def rows_of(w):
    """Kept rows: every 37th point of the left CAP, the innermost left plane
    around the tile boundary (y = 12..20 at x = 5 and x = 60), and the source
    plane around the same boundary."""
    import numpy as np

    from workloads import left_support

    per = w.nx * w.ny
    zl = w.n_cap - 1
    zs = w.nz - w.n_cap
    near = [zl * per + y * w.nx + x for y in range(12, 21) for x in (5, 60)]
    src = [zs * per + y * w.nx + x for y in range(12, 21) for x in (10, 40)]
    rows = np.unique(np.concatenate([left_support(w)[::37], near, src]))
    return rows.astype(np.int64)


def one(spec):
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import numpy as np

    import oracle as O
    from workloads import left_support

    k, e = spec
    w = make()
    per = w.nx * w.ny
    x, y = SOURCES[k]
    j = (w.nz - w.n_cap) * per + y * w.nx + x
    E = float(w.energies[e])
    t0 = time.time()
    A = O.operator_A(w, E).tocsr()
    b = np.zeros(w.N, complex)
    b[j] = 1.0
    g, res = O.solve_iterative(A, b, tol=1e-12)
    wl, wr = O.cap_diagonals(w)
    L = left_support(w)
    t = 4.0 * wr[j] * float(np.sum(wl[L] * np.abs(g[L]) ** 2))
    rows = rows_of(w)
    return {"source": k, "grid_index": int(j), "e_index": e, "energy": E, "t_col": t,
            "g_rows": [[float(v.real), float(v.imag)] for v in g[rows]],
            "g_scale": float(np.abs(g).max()), "true_residual": float(res),
            "seconds": time.time() - t0}


if __name__ == "__main__":
    specs = [(k, e) for k in range(len(SOURCES)) for e in range(len(WIRE["energies"]))]
    with mp.get_context("spawn").Pool(int(os.environ.get("WORKERS", "4"))) as pool:
        results = pool.map(one, specs)
    w = make()
    data = {"workload": "wire 64x64x25 h=0.35 R=6, CAP 6, one atom with s,p KB + one well",
            "generator": "tests/golden/make_plane64_samples.py (oracle iterative route)",
            "wire": WIRE, "sources": SOURCES, "rows": [int(r) for r in rows_of(w)],
            "samples": results}
    OUT.write_text(json.dumps(data) + "\n")
    print(json.dumps([{k: v for k, v in r.items() if k != "g_rows"} for r in results], indent=1))
