"""Writes tests/golden/fullsize_oracle.json: the oracle's FGMRES solve of the
3D 32^3 sinker workload (881,213 unknowns; minutes of CPU time and tens of
GB of memory, so it is recorded once): iteration count, residual history,
solution norms, and the solution at 2,000 seeded unknowns. Calls only the
oracle.

    python tests/golden/make_fullsize_golden.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.krylov import StokesSolver  # noqa: E402
from workloads import CONFIGS  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_oracle.json")
SAMPLE_SEED = 11
N_SAMPLE = 2000


def main():
    out = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in sys.argv[1:] or ["sinker_3d_32cu_L3"]:
        wl = CONFIGS[name]
        t0 = time.perf_counter()
        S = StokesSolver(wl)
        t1 = time.perf_counter()
        x, info = S.solve()
        t2 = time.perf_counter()
        nu = S.ops.level.n_u
        rng = np.random.default_rng(SAMPLE_SEED)
        idx = np.sort(rng.choice(x.size, N_SAMPLE, replace=False))
        out[name] = {"iters": info["iters"], "converged": bool(info["converged"]), "rel_res": info["rel_res"],
                     "hist": [float(h) for h in info["hist"]], "n_u": int(nu), "n_p": int(x.size - nu),
                     "norm_u": float(np.linalg.norm(x[:nu])), "norm_p": float(np.linalg.norm(x[nu:])),
                     "sample_seed": SAMPLE_SEED, "sample_index": idx.tolist(), "sample_value": x[idx].tolist(),
                     "setup_s": t1 - t0, "solve_s": t2 - t1}
        json.dump(out, open(OUT, "w"), indent=1, sort_keys=True)
        print(f"{name}: {info['iters']} iterations, converged {info['converged']}, setup {t1 - t0:.0f} s, "
              f"solve {t2 - t1:.0f} s", flush=True)


if __name__ == "__main__":
    main()
