"""Degenerate and extreme inputs of the method through the C ABI, against the
oracle where there is something to compare:
- a zero right-hand side (no sinkers, so no forcing): x = 0 exactly, no
  iteration, converged;
- gamma = 0 (A_gamma = A; P1 reduces to the inverse viscosity-weighted mass)
  and a constant viscosity (contrast 1): operator, smoother and solve parity;
- the smallest hierarchies (one coarse cell, 2 x 2 / 2 x 2 x 2 fine cells;
  Q2 and Q3, in 2D and 3D): every patch class a boundary class but one,
  coarse problems of 2, 3, 8 and 24 unknowns in one padded tile; operator,
  smoother, transfer and solve parity.
Tolerances as in test_gpu_parity (these meshes have small condition
numbers, so the applies and solves use the strict 1e-12 / 1e-8 bars)."""
import numpy as np
import pytest

from workloads import small
from gpu_common import to_dev, to_host, rel, rand_u, log

pytestmark = pytest.mark.gpu

EDGE = {
    "gamma0": small(2, 16, 2, gamma=0.0, dr=1e2, n_sinkers=4, seed=901),
    "const_mu": small(3, 8, 2, gamma=1e2, dr=1.0, n_sinkers=4, seed=902),
    "min_2d": small(2, 2, 2, gamma=1e2, dr=1e2, n_sinkers=2, seed=903),
    "min_3d": small(3, 2, 2, gamma=1e2, dr=1e2, n_sinkers=2, seed=904),
    "min_q3": small(2, 2, 2, gamma=1e2, dr=1e2, n_sinkers=2, seed=905, degree=3),
    "min_q3_3d": small(3, 2, 2, gamma=1e2, dr=1e2, n_sinkers=2, seed=907, degree=3),
}


def pair(name):
    from oracle.krylov import StokesSolver
    from paper_2107_00820_amd import Hierarchy
    wl = EDGE[name]
    return wl, StokesSolver(wl), Hierarchy.from_workload(wl)


@pytest.mark.parametrize("degree", [2, 3])
def test_zero_rhs_gives_zero_solution(degree):
    from paper_2107_00820_amd import Hierarchy
    wl = small(2, 8, 2, gamma=1e2, dr=1e2, n_sinkers=0, seed=906, degree=degree)
    h = Hierarchy.from_workload(wl)
    bu, bp = h.stk_rhs()
    assert np.all(to_host(bu) == 0.0) and np.all(to_host(bp) == 0.0)
    xu, xp = h.zeros_u() + 1.0, h.zeros_p() + 1.0     # overwritten
    xu, xp, info = h.stk_solve(bu, bp, xu=xu, xp=xp)
    log(f"[edge] zero rhs, degree {degree}: {info['iters']} iterations")
    assert info["converged"] and info["iters"] == 0
    assert np.all(to_host(xu) == 0.0) and np.all(to_host(xp) == 0.0)
    h.close()


@pytest.mark.parametrize("name", list(EDGE))
def test_edge_operators_smoother_transfers(name):
    wl, orc, gpu = pair(name)
    log(f"[edge] {name}")
    for l in range(wl.levels):
        lv = orc.mg.hier[l]
        u, us = rand_u(lv, 10 + l)
        y = lv.from_stored(to_host(gpu.stk_apply_Agamma(l, to_dev(us))))
        assert rel(y, orc.mg.ops[l].Agamma @ u) <= 1e-12, l
    for l in range(1, wl.levels):
        lv = orc.mg.hier[l]
        r, rs = rand_u(lv, 20 + l)
        y = lv.from_stored(to_host(gpu.stk_asm(l, to_dev(rs))))
        assert rel(y, orc.mg.smoothers[l].apply(r)) <= 1e-10, l
        coarse = orc.mg.hier[l - 1]
        xc, xcs = rand_u(coarse, 30 + l)
        xf = lv.from_stored(to_host(gpu.stk_prolong(l - 1, to_dev(xcs))))
        assert rel(xf, orc.mg.transfers[l].prolong(xc)) <= 1e-10, l
        rc = coarse.from_stored(to_host(gpu.stk_restrict(l, to_dev(rs))))
        assert rel(rc, orc.mg.transfers[l].restrict(r)) <= 1e-10, l
    lv0 = orc.mg.hier[0]
    b, bs = rand_u(lv0, 50)
    x = lv0.from_stored(to_host(gpu.stk_coarse_solve(to_dev(bs))))
    assert rel(x, orc.mg.coarse_lu.solve(b)) <= 1e-10
    gpu.close()


@pytest.mark.parametrize("name", list(EDGE))
def test_edge_solves(name):
    wl, orc, gpu = pair(name)
    lv = orc.mg.hier[-1]
    x_o, info_o = orc.solve()
    bu, bp = gpu.stk_rhs()
    xu, xp, info = gpu.stk_solve(bu, bp, rtol=wl.rtol, restart=wl.restart, maxit=wl.maxit)
    log(f"[edge solve] {name}: GPU {info['iters']}, oracle {info_o['iters']}")
    assert info["converged"] and info["iters"] == info_o["iters"]
    x = np.concatenate([lv.from_stored(to_host(xu)), to_host(xp)])
    assert rel(x, x_o) <= 1e-8
    gpu.close()
