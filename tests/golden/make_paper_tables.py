"""Writes tests/golden/paper_tables_oracle.json: the oracle's FGMRES
iteration counts at the settings of the paper's iteration tables
(workloads.PAPER_VANKA_AL: table "vanka", AL column; workloads.PAPER_K2_SMALL:
table "k", k = 2, on a 12^3 mesh; workloads.PAPER_LINEAR_Q3: table "linear",
2D, [Q3]^2 x P2disc, robust rows; workloads.PAPER_LINEAR_Q3_3D: its 3D
settings on 8^3 cells). Calls only the oracle.

    python tests/golden/make_paper_tables.py [--only vanka|k2|linear_q3|linear_q3_3d]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.krylov import StokesSolver  # noqa: E402
from workloads import PAPER_VANKA_AL, PAPER_K2_SMALL, PAPER_LINEAR_Q3, PAPER_LINEAR_Q3_3D  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_tables_oracle.json")


def run(wl):
    t0 = time.perf_counter()
    x, info = StokesSolver(wl).solve()
    print(f"{wl.name}: {info['iters']} iterations, converged {info['converged']}, "
          f"{time.perf_counter() - t0:.0f} s", flush=True)
    return {"iters": info["iters"], "converged": bool(info["converged"]), "rel_res": info["rel_res"]}


def main():
    only = sys.argv[sys.argv.index("--only") + 1] if "--only" in sys.argv else None
    out = json.load(open(OUT)) if os.path.exists(OUT) else {}
    if only in (None, "vanka"):
        for wl in PAPER_VANKA_AL.values():
            out[wl.name] = run(wl)
            json.dump(out, open(OUT, "w"), indent=1, sort_keys=True)
    if only in (None, "k2"):
        for wl in PAPER_K2_SMALL.values():
            out[wl.name] = run(wl)
            json.dump(out, open(OUT, "w"), indent=1, sort_keys=True)
    if only in (None, "linear_q3"):
        for wl in PAPER_LINEAR_Q3.values():
            out[wl.name] = run(wl)
            json.dump(out, open(OUT, "w"), indent=1, sort_keys=True)
    if only in (None, "linear_q3_3d"):
        for wl in PAPER_LINEAR_Q3_3D.values():
            out[wl.name] = run(wl)
            json.dump(out, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
