"""GPU parity: every operation of the hot path through the C ABI against the
CPU FP64 oracle on the same seeded inputs.

Tolerances: operator applications (A_gamma, K) 1e-12 relative. Patch
solves are only defined to kappa eps: the star smoother is checked entry by
entry against the sum, over the patches containing the entry, of the
per-patch forward-error bound 50 kappa_i eps64 ||A_i^{-1}||_2 ||r_i||_2 (kappa_i
and ||A_i^{-1}|| from the SVD of every patch matrix), and the transfers
likewise per coarse cell (their local solves), plus 32 eps64 times the
absolute values of the other terms; on the 2D 16^2 workload, whose patches
have kappa <= 1.4e3, both must also hold to 1e-12 relative. Coarse solve:
2 kappa eps64. Compositions (relaxation, V- and F-cycle, preconditioner),
which chain several such solves and small least-squares problems:
100 kappa eps64 with kappa the largest patch condition number, at least
1e-10 (the preconditioner's velocity block on F-cycles 2000 kappa eps64; a
plain FP64 CPU run of the same algorithm with Cholesky-based explicit
inverses differs from the oracle's LU solves by up to 33 and 457 kappa eps64
on the 3D 16^3 cases, so these bars are the rounding of the method). Solves: identical iteration count and solutions within 1e-8 relative.
"""
import functools

import numpy as np
import pytest

from gpu_common import CASES, oracle_for, gpu_for, to_dev, to_host, rel, rand_u, log

pytestmark = pytest.mark.gpu

NAMES = list(CASES)
EPS = np.finfo(float).eps
STRICT = "sinker_2d_16sq_L2"


@functools.lru_cache(maxsize=None)
def patch_svd(name, l, which):
    """(index arrays, kappa_i, ||A_i^{-1}||_2) of the star patches (which =
    "star") or the coarse-cell blocks of the transfer into level l ("cell")."""
    from oracle.multigrid import extract_dense
    orc = oracle_for(name)
    A = orc.mg.ops[l].Agamma
    blocks = orc.mg.smoothers[l].patches if which == "star" else orc.mg.transfers[l].blocks
    kap, ninv = [], []
    for idx in blocks:
        sv = np.linalg.svd(extract_dense(A, idx), compute_uv=False)
        kap.append(sv[0] / sv[-1])
        ninv.append(1.0 / sv[-1])
    return blocks, np.array(kap), np.array(ninv)


def local_bound(name, l, which, r, kappa=True):
    """Entrywise sum over the blocks containing each unknown of 50 kappa_i
    eps ||A_i^{-1}|| ||r_i|| (the forward error of a solve with A_i), or
    without kappa_i (the effect of an error r in the right-hand side)."""
    blocks, kap, ninv = patch_svd(name, l, which)
    out = np.zeros_like(r)
    for idx, k, ni in zip(blocks, kap, ninv):
        out[idx] += 50.0 * (k if kappa else 1.0) * EPS * ni * np.linalg.norm(r[idx])
    return out


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
        bnd = local_bound(name, l, "star", r)
        worst = np.max(np.abs(y - ref) / bnd)
        log(f"  level {l}: rel err {rel(y, ref):.2e}, largest error / per-patch bound {worst:.2e}")
        assert np.all(np.abs(y - ref) <= bnd)
        if name == STRICT:
            assert rel(y, ref) <= 1e-12


@pytest.mark.parametrize("name", NAMES)
def test_robust_transfers(name):
    log(f"[transfer] {name}")
    orc, gpu = oracle_for(name), gpu_for(name)
    for l in range(1, CASES[name].levels):
        fine, coarse = orc.mg.hier[l], orc.mg.hier[l - 1]
        T = orc.mg.transfers[l]
        absP, absG = abs(T.P), abs(T.G)
        xc, xcs = rand_u(coarse, 30 + l)
        xf = fine.from_stored(to_host(gpu.stk_prolong(l - 1, to_dev(xcs))))
        t = T.P @ xc
        g = T.G @ t
        corr = T.local_correction(g)
        ref = t - corr
        # local solves of each coarse cell, the rounding of G P xc seen
        # through them, and the rounding of P xc and of the difference
        bnd = (local_bound(name, l, "cell", g) + local_bound(name, l, "cell", absG @ (absP @ np.abs(xc)), False)
               + 32 * EPS * (absP @ np.abs(xc) + np.abs(corr)))
        e1 = np.max(np.abs(xf - ref) / bnd)
        assert np.all(np.abs(xf - ref) <= bnd), e1
        rf, rfs = rand_u(fine, 40 + l)
        rc = coarse.from_stored(to_host(gpu.stk_restrict(l, to_dev(rfs))))
        s_loc = T.local_correction(rf, trans=1)
        ref_c = T.P.T @ (rf - T.GT @ s_loc)
        ds = local_bound(name, l, "cell", rf)
        bnd_c = abs(T.P.T) @ (absG.T @ ds) + 32 * EPS * (abs(T.P.T) @ (np.abs(rf) + absG.T @ np.abs(s_loc)))
        e2 = np.max(np.abs(rc - ref_c) / bnd_c)
        log(f"  level {l}: prolong rel {rel(xf, ref):.2e} ({e1:.2e} of bound), "
            f"restrict rel {rel(rc, ref_c):.2e} ({e2:.2e} of bound)")
        assert np.all(np.abs(rc - ref_c) <= bnd_c), e2
        if name == STRICT:
            assert rel(xf, ref) <= 1e-12 and rel(rc, ref_c) <= 1e-12


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
    tol = max(1e-10, 100 * patch_svd(name, lf, "star")[1].max() * EPS)
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
    v = lv.from_stored(to_host(gpu.stk_fcycle(to_dev(bs))))
    e = rel(v, orc.mg.fcycle(b))
    log(f"  fcycle {e:.2e}")
    assert e <= tol
    p = np.random.default_rng(62).standard_normal(lv.n_p)
    ops = orc.ops
    for pc, cycle in (("full", "V"), ("upper", "V"), ("full", "F")):
        zu, zp = gpu.stk_precond(to_dev(bs), to_dev(p), pc=pc, cycle=cycle)
        # the oracle's eq. (precond) step by step; z_u = y - w (full) ends in
        # a difference of two cycles, so its error is measured against the
        # size of the two terms
        ahat = orc.mg.vcycle if cycle == "V" else orc.mg.fcycle
        if pc == "full":
            y = ahat(b)
            zp_ref = ops.project_mean(-(ops.Shat_inv @ (p - ops.B @ y)))
            w = ahat(ops.B.T @ zp_ref)
            zu_ref, scale = y - w, np.linalg.norm(y) + np.linalg.norm(w)
        else:
            zp_ref = ops.project_mean(-(ops.Shat_inv @ p))
            zu_ref = ahat(b - ops.B.T @ zp_ref)
            scale = np.linalg.norm(zu_ref)
        e1 = np.linalg.norm(lv.from_stored(to_host(zu)) - zu_ref) / scale
        e2 = rel(to_host(zp), zp_ref)
        # with F-cycles the second cycle runs on B^T z_p, which lies in the
        # stiff range of A_gamma, through more chained patch solves: a plain
        # FP64 CPU run of the same algorithm (explicit Cholesky-based
        # inverses) differs from the oracle's LU solves by 87 kappa eps on the
        # 3D 16^3 case and 457 kappa eps on its tensor variant (33 kappa eps
        # with V-cycles), so this block gets 2000 kappa eps
        tol_u = tol if cycle == "V" else 20 * tol
        log(f"  precond {pc} {cycle}: u {e1:.2e} (of |y| + |w|; tol {tol_u:.1e}) p {e2:.2e}")
        assert e1 <= tol_u and e2 <= tol


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


@pytest.mark.parametrize("name", ["sinker_2d_16sq_L2", "2d_32_L3", "3d_8_L2", "3d_8_L2_tensor", "q3_2d_16_L3"])
@pytest.mark.parametrize("cycle", ["V", "F"])
def test_solve_variants_match_oracle(name, cycle):
    """FGMRES with the block upper-triangular preconditioner (V-cycle) or
    with the full preconditioner on F-cycles: same iteration count as the
    oracle's, solution within 1e-8, true residual checked with the oracle's
    operator."""
    pc = "upper" if cycle == "V" else "full"
    log(f"[solve {pc} {cycle}] {name}")
    orc, gpu = oracle_for(name), gpu_for(name)
    wl = CASES[name]
    lv = orc.mg.hier[-1]
    x_o, info_o = orc.solve(pc=pc, cycle=cycle)
    bu, bp = gpu.stk_rhs()
    xu, xp, info = gpu.stk_solve(bu, bp, rtol=wl.rtol, restart=wl.restart, maxit=wl.maxit, pc=pc, cycle=cycle)
    log(f"  iterations gpu {info['iters']} oracle {info_o['iters']}")
    assert info["converged"] and info["iters"] == info_o["iters"]
    x = np.concatenate([lv.from_stored(to_host(xu)), to_host(xp)])
    assert rel(x, x_o) <= 1e-8
    b = orc.rhs()
    assert np.linalg.norm(b - orc.K @ x) <= wl.rtol * np.linalg.norm(b)


@pytest.mark.parametrize("name", ["sinker_2d_16sq_L2", "3d_8_L2", "q3_2d_8_L2"])
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
