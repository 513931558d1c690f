"""GPU parity at the benchmark's full size (2D 128x128, 4 levels, 16 sinkers,
contrast 1e6, gamma 1e3), in the launch configuration bench.py times (HIP
graph replays of the Arnoldi steps): identical FGMRES iteration count to the
oracle, solution within 1e-8 relative, true residual checked with the
oracle's assembled operator, and element-wise checks of the fine-level
operator and smoother applications."""
import numpy as np
import pytest

from workloads import CONFIGS
from gpu_common import to_dev, to_host, rel, rand_u, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pair():
    from oracle.krylov import StokesSolver
    from paper_2107_00820_amd import Hierarchy
    wl = CONFIGS["sinker_2d_128sq_L4"]
    log("[fullsize] oracle setup c2")
    orc = StokesSolver(wl)
    log("[fullsize] gpu setup c2")
    gpu = Hierarchy.from_workload(wl)
    return wl, orc, gpu


def test_c2_operators(pair):
    wl, orc, gpu = pair
    lf = wl.levels - 1
    lv = orc.mg.hier[lf]
    u, us = rand_u(lv, 1)
    y = lv.from_stored(to_host(gpu.stk_apply_Agamma(lf, to_dev(us))))
    ref = orc.mg.ops[lf].Agamma @ u
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))
    r, rs = rand_u(lv, 2)
    z = lv.from_stored(to_host(gpu.stk_asm(lf, to_dev(rs))))
    zr = orc.mg.smoothers[lf].apply(r)
    log(f"[fullsize] asm rel err {rel(z, zr):.2e}")
    assert rel(z, zr) <= 1e-9


def test_c2_solve(pair):
    wl, orc, gpu = pair
    lv = orc.mg.hier[-1]
    log("[fullsize] oracle solve c2")
    x_o, info_o = orc.solve()
    bu, bp = gpu.stk_rhs()
    xu, xp, info = gpu.stk_solve(bu, bp, rtol=wl.rtol, restart=wl.restart, maxit=wl.maxit)
    log(f"[fullsize] iterations gpu {info['iters']} oracle {info_o['iters']}")
    assert info["converged"] and info["iters"] == info_o["iters"]
    x = np.concatenate([lv.from_stored(to_host(xu)), to_host(xp)])
    assert rel(x, x_o) <= 1e-8
    b = orc.rhs()
    assert np.linalg.norm(b - orc.K @ x) <= wl.rtol * np.linalg.norm(b)
