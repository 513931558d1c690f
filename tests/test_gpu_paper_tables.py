"""The paper's iteration tables, run on the GPU with the paper's solver
options (5 + 5 relaxation steps, F-cycles, FGMRES(30) to a 1e6 residual
reduction; preconditioner P2 unless stated):

* table "vanka", AL column (2D 128^2, 4 levels, gamma 100, 1/6/24 sinkers,
  contrast 1e4..1e10): the GPU count must equal the oracle's
  (tests/golden/paper_tables_oracle.json, written by make_paper_tables.py
  from the oracle alone); the paper's printed count is logged beside them
  (the sinker positions differ, so that comparison is qualitative);
* table "k", k = 2 (3D, 2 levels, contrast 1e6, gamma 0/10/1000): GPU =
  oracle on a 12^3 mesh, and the GPU count on the paper's 30^3 mesh logged
  beside the printed one; the augmentation must pay at gamma 1000 (count
  well below the one at gamma 0). With these seeded sinkers gamma 10 needs
  far more iterations than the paper prints (the Schur approximation's
  quality depends on the viscosity field), so it is reported, not bounded;
* table "linear", 2D ([Q3]^2 x P2disc on 128^2, 4 levels, 24 sinkers, P1 and
  P2, gamma 10 / 1000, contrast 1e6 / 1e10, robust smoother and transfer):
  GPU = oracle, the printed count logged beside them, and every count within
  the paper's observation of convergence in at most 30 iterations for gamma
  from 10 to 1000; its 3D settings ([Q3]^3 x P2disc, contrast 1e8, P1 and P2,
  gamma 10 / 1000) on 8^3 cells with 2 levels (the paper's 80^3 is beyond the
  explicit patch inverses): GPU = oracle, printed counts logged. On this
  mesh a cell is wider than a sinker, and P2 at gamma 10 stalls above the
  1e6 reduction within 300 iterations in the oracle too: there the GPU must
  stop at the same count with a true residual within 10% of the oracle's.
  At gamma 1000 both preconditioners converge.
"""
import json
import os

import pytest

from gpu_common import log

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_tables_oracle.json")


def gpu_count(wl):
    from paper_2107_00820_amd import Hierarchy
    h = Hierarchy.from_workload(wl)
    bu, bp = h.stk_rhs()
    _, _, info = h.stk_solve(bu, bp, rtol=wl.rtol, restart=wl.restart, maxit=wl.maxit, cycle=wl.cycle,
                             allow_notconv=True)
    h.close()
    return info


def test_table_vanka_al_column():
    from workloads import PAPER_VANKA_AL, PAPER_VANKA_AL_PRINTED
    orc = json.load(open(GOLDEN))
    for key, wl in PAPER_VANKA_AL.items():
        info = gpu_count(wl)
        o = orc[wl.name]
        log(f"[vanka] {key[0]:2d} sinkers, DR {key[1]:.0e}: GPU {info['iters']}, oracle {o['iters']}, "
            f"paper {PAPER_VANKA_AL_PRINTED[key]}")
        assert info["converged"] and o["converged"]
        assert info["iters"] == o["iters"]


def test_table_k_quadratic_column():
    from workloads import PAPER_K2, PAPER_K2_SMALL, PAPER_K2_PRINTED
    orc = json.load(open(GOLDEN))
    for g, wl in PAPER_K2_SMALL.items():
        info = gpu_count(wl)
        o = orc[wl.name]
        log(f"[k=2, 12^3] gamma {g:g}: GPU {info['iters']}, oracle {o['iters']}")
        assert info["converged"] == o["converged"]
        assert info["iters"] == o["iters"]
    its = {}
    for g, wl in PAPER_K2.items():
        info = gpu_count(wl)
        its[g] = info["iters"]
        log(f"[k=2, 30^3] gamma {g:g}: GPU {info['iters']} (converged {info['converged']}), "
            f"paper {PAPER_K2_PRINTED[g]}")
        # without augmentation (gamma = 0) the count may reach maxit, as it
        # does on the 12^3 mesh; with it the solver must converge
        if g > 0:
            assert info["converged"]
    assert its[1000.0] < its[0.0] / 2


def test_table_linear_q3_2d():
    from workloads import PAPER_LINEAR_Q3, PAPER_LINEAR_Q3_PRINTED
    orc = json.load(open(GOLDEN))
    for key, wl in PAPER_LINEAR_Q3.items():
        info = gpu_count(wl)
        o = orc[wl.name]
        log(f"[linear Q3 2D] P{key[0]} gamma {key[1]:g} DR {key[2]:.0e}: GPU {info['iters']}, oracle {o['iters']}, "
            f"paper {PAPER_LINEAR_Q3_PRINTED[key]}")
        assert info["converged"] and o["converged"]
        assert info["iters"] == o["iters"]
        assert info["iters"] <= 30


def test_table_linear_q3_3d():
    from workloads import PAPER_LINEAR_Q3_3D, PAPER_LINEAR_Q3_3D_PRINTED
    orc = json.load(open(GOLDEN))
    for key, wl in PAPER_LINEAR_Q3_3D.items():
        info = gpu_count(wl)
        o = orc[wl.name]
        log(f"[linear Q3 3D, 8^3] P{key[0]} gamma {key[1]:g}: GPU {info['iters']} (residual "
            f"{info['rel_res']:.3e}), oracle {o['iters']} ({o['rel_res']:.3e}), "
            f"paper (80^3) {PAPER_LINEAR_Q3_3D_PRINTED[key]}")
        assert info["converged"] == o["converged"]
        assert info["iters"] == o["iters"]
        if not o["converged"]:
            assert abs(info["rel_res"] - o["rel_res"]) <= 0.1 * o["rel_res"]
        if key[1] >= 1000.0:
            assert info["converged"]
