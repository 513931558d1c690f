"""GPU parity: every operation of the hot path through the C ABI against the
CPU FP64 oracle on the same seeded inputs.

Tolerances: operator applications (A_gamma, K) 1e-12 relative; patch solves
(star smoother, local transfer solves, coarse solve) 50 kappa eps64 with
kappa the largest condition number of the patch (or coarse) matrices, at
least 1e-12; compositions (relaxation, V-cycle, preconditioner), which chain
several such solves and small least-squares problems, 50 kappa eps64, at
least 1e-10; solves: identical iteration count and solutions within 1e-8
relative.
"""
import numpy as np
import pytest

from gpu_common import CASES, oracle_for, gpu_for, to_dev, to_host, rel, rand_u, log

pytestmark = pytest.mark.gpu

NAMES = list(CASES)


def cond_bound(orc, l):
    """Largest condition number of the star patch matrices of level l (oracle)."""
    import scipy.linalg as sla
    from oracle.multigrid import extract_dense
    A = orc.mg.ops[l].Agamma
    worst = 1.0
    for idx in orc.mg.smoothers[l].patches[::7]:
        worst = max(worst, np.linalg.cond(extract_dense(A, idx)))
    return worst


@pytest.mark.parametrize("name", NAMES)
def test_apply_agamma_all_levels(name):
    log(f"[apply] {name}")
    orc, gpu = oracle_for(name), gpu_for(name)
    for l in range(CASES[name].levels):
        lv = orc.mg.hier[l]
        u, us = rand_u(lv, 10 + l)
        y = to_host(gpu.stk_apply_Agamma(l, to_dev(us)))
        ref = orc.mg.ops[l].Agamma @ u
        assert rel(lv.from_stored(y), ref) <= 1e-12
        # Dirichlet entries written as zero
        mask = np.ones(lv.n_stored, dtype=bool)
        mask[lv.stored_index()] = False
        assert np.all(y[mask] == 0.0)


@pytest.mark.parametrize("name", NAMES)
def test_apply_stokes_and_rhs(name):
    log(f"[stokes] {name}")
    orc, gpu = oracle_for(name), gpu_for(name)
    lv = orc.mg.hier[-1]
    u, us = rand_u(lv, 3)
    p = np.random.default_rng(4).standard_normal(lv.n_p)
    yu, yp = gpu.stk_apply_stokes(to_dev(us), to_dev(p))
    ref = orc.K @ np.concatenate([u, p])
    assert rel(lv.from_stored(to_host(yu)), ref[:lv.n_u]) <= 1e-12
    assert rel(to_host(yp), ref[lv.n_u:]) <= 1e-12
    bu, bp = gpu.stk_rhs()
    assert rel(lv.from_stored(to_host(bu)), orc.ops.rhs()) <= 1e-12
    assert np.all(to_host(bp) == 0.0)


@pytest.mark.parametrize("name", NAMES)
def test_star_asm_all_levels(name):
    log(f"[asm] {name}")
    orc, gpu = oracle_for(name), gpu_for(name)
    for l in range(1, CASES[name].levels):
        lv = orc.mg.hier[l]
        r, rs = rand_u(lv, 20 + l)
        y = lv.from_stored(to_host(gpu.stk_asm(l, to_dev(rs))))
        ref = orc.mg.smoothers[l].apply(r)
        tol = max(1e-12, 50 * cond_bound(orc, l) * np.finfo(float).eps)
        err = rel(y, ref)
        log(f"  level {l}: rel err {err:.2e} (tol {tol:.1e})")
        assert err <= tol


@pytest.mark.parametrize("name", NAMES)
def test_robust_transfers(name):
    log(f"[transfer] {name}")
    orc, gpu = oracle_for(name), gpu_for(name)
    for l in range(1, CASES[name].levels):
        fine, coarse = orc.mg.hier[l], orc.mg.hier[l - 1]
        T = orc.mg.transfers[l]
        tol = max(1e-12, 50 * cond_bound(orc, l) * np.finfo(float).eps)
        xc, xcs = rand_u(coarse, 30 + l)
        xf = fine.from_stored(to_host(gpu.stk_prolong(l - 1, to_dev(xcs))))
        e1 = rel(xf, T.prolong(xc))
        rf, rfs = rand_u(fine, 40 + l)
        rc = coarse.from_stored(to_host(gpu.stk_restrict(l, to_dev(rfs))))
        e2 = rel(rc, T.restrict(rf))
        log(f"  level {l}: prolong {e1:.2e} restrict {e2:.2e} (tol {tol:.1e})")
        assert e1 <= tol and e2 <= tol


@pytest.mark.parametrize("name", NAMES)
def test_coarse_solve(name):
    log(f"[coarse] {name}")
    orc, gpu = oracle_for(name), gpu_for(name)
    lv = orc.mg.hier[0]
    b, bs = rand_u(lv, 50)
    x = lv.from_stored(to_host(gpu.stk_coarse_solve(to_dev(bs))))
    A = orc.mg.ops[0].Agamma.toarray()
    ref = orc.mg.coarse_lu.solve(b)
    err = rel(x, ref)
    # the inverse is formed through Cholesky factors (square-root sweep), whose
    # forward error is a small fraction of kappa eps (at most 0.07 kappa eps
    # over these cases; the explicit-pivot-inverse sweep reached 87)
    tol = max(1e-12, 2 * np.linalg.cond(A) * np.finfo(float).eps)
    log(f"  rel err {err:.2e} (tol {tol:.1e})")
    assert err <= tol


@pytest.mark.parametrize("name", NAMES)
def test_relaxation_vcycle_precond(name):
    log(f"[compose] {name}")
    from oracle.multigrid import gmres_relax
    orc, gpu = oracle_for(name), gpu_for(name)
    wl = CASES[name]
    lf = wl.levels - 1
    lv = orc.mg.hier[lf]
    b, bs = rand_u(lv, 60)
    x0, x0s = rand_u(lv, 61)
    tol = max(1e-10, 50 * cond_bound(orc, lf) * np.finfo(float).eps)
    log(f"  composition tolerance {tol:.1e}")
    x = to_dev(x0s)
    gpu.stk_smooth(lf, to_dev(bs), x, 3)
    ref = gmres_relax(orc.mg.ops[lf].Agamma, orc.mg.smoothers[lf].apply, b, x0, 3)
    e = rel(lv.from_stored(to_host(x)), ref)
    log(f"  relax {e:.2e}")
    assert e <= tol
    v = lv.from_stored(to_host(gpu.stk_vcycle(to_dev(bs))))
    e = rel(v, orc.mg.vcycle(b))
    log(f"  vcycle {e:.2e}")
    assert e <= tol
    p = np.random.default_rng(62).standard_normal(lv.n_p)
    zu, zp = gpu.stk_precond(to_dev(bs), to_dev(p))
    ref = orc.pc.apply(np.concatenate([b, p]))
    e1 = rel(lv.from_stored(to_host(zu)), ref[:lv.n_u])
    e2 = rel(to_host(zp), ref[lv.n_u:])
    log(f"  precond u {e1:.2e} p {e2:.2e}")
    assert e1 <= tol and e2 <= tol
    # block upper-triangular variant
    from oracle.krylov import BlockPreconditioner
    zu, zp = gpu.stk_precond(to_dev(bs), to_dev(p), pc="upper")
    ref = BlockPreconditioner(orc.mg, "upper").apply(np.concatenate([b, p]))
    e1 = rel(lv.from_stored(to_host(zu)), ref[:lv.n_u])
    e2 = rel(to_host(zp), ref[lv.n_u:])
    log(f"  upper precond u {e1:.2e} p {e2:.2e}")
    assert e1 <= tol and e2 <= tol


@pytest.mark.parametrize("name", NAMES)
def test_solve_matches_oracle(name):
    log(f"[solve] {name}")
    orc, gpu = oracle_for(name), gpu_for(name)
    wl = CASES[name]
    lv = orc.mg.hier[-1]
    x_o, info_o = orc.solve()
    bu, bp = gpu.stk_rhs()
    xu, xp, info = gpu.stk_solve(bu, bp, rtol=wl.rtol, restart=wl.restart, maxit=wl.maxit)
    log(f"  iterations gpu {info['iters']} oracle {info_o['iters']}; rel res {info['rel_res']:.2e}")
    assert info["converged"] and info["rel_res"] <= wl.rtol
    assert info["iters"] == info_o["iters"]
    x = np.concatenate([lv.from_stored(to_host(xu)), to_host(xp)])
    assert rel(x, x_o) <= 1e-8
    # true residual checked with the oracle's assembled operator
    b = orc.rhs()
    assert np.linalg.norm(b - orc.K @ x) <= wl.rtol * np.linalg.norm(b)
    # residual histories agree. Within the first cycle both are Arnoldi
    # estimates; each restart recomputes b - K x, whose rounding error is up
    # to eps || |b| + |K| |x| || (componentwise bound of a computed residual),
    # so the entries after a restart are compared to that bound
    h_o = np.array(info_o["hist"])
    h_g = np.array(info["hist"])
    assert h_g.shape == h_o.shape
    m = min(len(h_o), wl.restart + 1)
    assert np.allclose(h_g[:m], h_o[:m], rtol=1e-6, atol=1e-14)
    if len(h_o) > m:
        eps = np.finfo(float).eps
        atol = eps * np.linalg.norm(np.abs(b) + abs(orc.K) @ np.abs(x)) / np.linalg.norm(b)
        log(f"  history after restart: max diff {np.max(np.abs(h_g[m:] - h_o[m:])):.1e} (bound {atol:.1e})")
        assert np.allclose(h_g[m:], h_o[m:], rtol=1e-6, atol=atol)
    # determinism: a second solve is bit-identical
    xu2, xp2, info2 = gpu.stk_solve(bu, bp, rtol=wl.rtol, restart=wl.restart, maxit=wl.maxit)
    assert info2["iters"] == info["iters"]
    assert np.array_equal(to_host(xu2), to_host(xu)) and np.array_equal(to_host(xp2), to_host(xp))


@pytest.mark.parametrize("name", ["sinker_2d_16sq_L2", "2d_32_L3", "3d_8_L2", "3d_8_L2_tensor"])
def test_solve_upper_matches_oracle(name):
    """FGMRES with the block upper-triangular preconditioner: same iteration
    count as the oracle's, solution within 1e-8, true residual checked with
    the oracle's operator."""
    log(f"[solve upper] {name}")
    orc, gpu = oracle_for(name), gpu_for(name)
    wl = CASES[name]
    lv = orc.mg.hier[-1]
    x_o, info_o = orc.solve(pc="upper")
    bu, bp = gpu.stk_rhs()
    xu, xp, info = gpu.stk_solve(bu, bp, rtol=wl.rtol, restart=wl.restart, maxit=wl.maxit, pc="upper")
    log(f"  iterations gpu {info['iters']} oracle {info_o['iters']}")
    assert info["converged"] and info["iters"] == info_o["iters"]
    x = np.concatenate([lv.from_stored(to_host(xu)), to_host(xp)])
    assert rel(x, x_o) <= 1e-8
    b = orc.rhs()
    assert np.linalg.norm(b - orc.K @ x) <= wl.rtol * np.linalg.norm(b)


@pytest.mark.parametrize("name", ["sinker_2d_16sq_L2", "3d_8_L2"])
def test_graph_replay_matches_eager(name):
    """Each Arnoldi step is captured once as a HIP graph and replayed; every
    replay must reproduce the plain-launch solve bit for bit, also with
    eager work and synchronisations between replays."""
    log(f"[graph] {name}")
    import torch
    gpu = gpu_for(name)
    wl = CASES[name]
    bu, bp = gpu.stk_rhs()
    xe_u, xe_p, ie = gpu.stk_solve(bu, bp, rtol=wl.rtol, restart=wl.restart, maxit=wl.maxit, eager=True)
    ref_u, ref_p = to_host(xe_u), to_host(xe_p)
    for rep in range(3):
        xg_u, xg_p, ig = gpu.stk_solve(bu, bp, rtol=wl.rtol, restart=wl.restart, maxit=wl.maxit)
        assert ig["iters"] == ie["iters"]
        assert np.array_equal(to_host(xg_u), ref_u) and np.array_equal(to_host(xg_p), ref_p), rep
        # unrelated eager work in between replays
        y = gpu.stk_vcycle(bu)
        torch.cuda.synchronize()
        assert np.isfinite(to_host(y)).all()
