"""Write oracle samples for the full-size parity tests (calls only oracle/).

For each workload the FP64 oracle runs the whole method; the file keeps, per
component grid, the values at a few seeded nodes and the grid sum, plus the
combined solution at seeded finest-grid nodes and the error norms.  The GPU
tests compare the library's FP64 run with these samples.

    python tests/golden/make_golden.py c3 c4      # minutes on 8 cores
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import sgw_inputs as W  # noqa: E402

WORKLOADS = {
    "c3": lambda: W.c3_advection_3d(precision=W.PREC_FP64),
    "c4": lambda: W.c4_vlasov_4d(precision=W.PREC_FP64),
}


def make(name: str, nodes_per_grid: int = 12, fine_points: int = 256) -> dict:
    pb = WORKLOADS[name]()
    t0 = time.time()
    st = O.restrict(pb)
    stats = O.evolve(pb, st)
    t_evolve = time.time() - t0
    rng = np.random.default_rng(2007_10196)
    grids = []
    for lev, coef, shp, off in O.grid_layout(pb):
        n = int(np.prod(shp))
        idx = np.sort(rng.choice(n, size=min(nodes_per_grid, n), replace=False))
        grids.append(dict(level=list(lev), coef=coef, shape=list(shp), offset=int(off),
                          idx=[int(i) for i in idx], val=[float(st[off + i]) for i in idx],
                          sum=float(st[off:off + n].sum())))
    J = rng.integers(0, pb.n_fine, size=(fine_points, pb.d)).astype(np.int32)
    fine = O.prolong_combine_points(pb, st, J)
    exact = np.array([O.exact(pb, [pb.lo[k] + J[i, k] * (pb.hi[k] - pb.lo[k]) / pb.n_fine for k in range(pb.d)],
                              stats["t"]) for i in range(J.shape[0])])
    return dict(workload=name, problem=pb.name, nr=pb.nr, nl=pb.nl, T=pb.T, eps_flux=pb.eps_flux,
                eps_interp=pb.eps_interp, steps=int(stats["steps"]), t=stats["t"], grids=grids,
                fine_J=J.tolist(), fine_val=[float(v) for v in fine], fine_exact=[float(v) for v in exact],
                oracle_evolve_s=t_evolve, oracle_threads=O.max_threads())


if __name__ == "__main__":
    for name in sys.argv[1:] or list(WORKLOADS):
        out = make(name)
        path = os.path.join(HERE, f"oracle_{name}_full.json")
        with open(path, "w") as f:
            json.dump(out, f)
        print(path, out["steps"], f"{out['oracle_evolve_s']:.1f}s", flush=True)
