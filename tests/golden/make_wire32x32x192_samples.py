"""Write oracle samples of the 32x32x192 R=6 wire with projectors.

For each requested (source column index, energy index) this runs the oracle's
iterative route (scipy Krylov on the oracle's sparse A(E), true relative
residual <= 1e-12) and stores t_j(E) = 4 W_R,j sum_{i in L} W_L,i |G_ij|^2
(Eq. 7 with Gamma = 2W) plus G_jj, in tests/golden/wire32x32x192_samples.json.
Only oracle/ and the input generator are used.

usage: python tests/golden/make_wire32x32x192_samples.py [--drop COL:E ...] COL:E [COL:E ...]
(samples are merged into the existing file; each sample is one process;
--drop removes a stored sample, e.g. one whose t_j is too small to inform)
"""

import json
import multiprocessing as mp
import os
import pathlib
import sys
import time

ROOT = pathlib.Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))
OUT = pathlib.Path(__file__).resolve().parent / "wire32x32x192_samples.json"


def one(spec):
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import numpy as np

    import oracle as O
    from workloads import left_support, make_wire, rhs_columns

    ci, ei = spec
    w = make_wire(2)
    j = int(rhs_columns(w)[ci])
    E = float(w.energies[ei])
    wl, wr = O.cap_diagonals(w)
    t0 = time.time()
    A = O.operator_A(w, E).tocsr()
    b = np.zeros(w.N, complex)
    b[j] = 1.0
    x, res = O.solve_iterative(A, b, tol=1e-12)
    L = left_support(w)
    t = 4.0 * wr[j] * float(np.sum(wl[L] * np.abs(x[L]) ** 2))
    return {"col": ci, "grid_index": j, "e_index": ei, "energy": E, "t_col": t,
            "g_jj": [float(x[j].real), float(x[j].imag)], "true_residual": float(res),
            "seconds": time.time() - t0}


if __name__ == "__main__":
    args = sys.argv[1:]
    drop = {tuple(int(v) for v in args[i + 1].split(":")) for i, a in enumerate(args) if a == "--drop"}
    specs = [tuple(int(v) for v in a.split(":")) for i, a in enumerate(args)
             if a != "--drop" and (i == 0 or args[i - 1] != "--drop")]
    results = []
    if specs:
        with mp.get_context("spawn").Pool(len(specs)) as pool:
            results = pool.map(one, specs)
    data = json.loads(OUT.read_text()) if OUT.exists() else {
        "workload": "wire 32x32x192 h=0.4 R=6, 20 atoms + s,p KB, CAP 16 (make_wire(2))",
        "generator": "tests/golden/make_wire32x32x192_samples.py (oracle iterative route)",
        "samples": []}
    keep = {(s["col"], s["e_index"]) for s in results} | drop
    data["samples"] = [s for s in data["samples"] if (s["col"], s["e_index"]) not in keep] + results
    OUT.write_text(json.dumps(data, indent=1) + "\n")
    print(json.dumps(results, indent=1))
