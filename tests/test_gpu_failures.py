"""Failure paths of the C ABI on the GPU, each forced from the host so that
every kernel still exits normally: FGMRES reaching maxit (STK_ENOTCONV with
the last iterate written and the info filled), a non-finite right-hand side
(STK_ENAN, found by the norm of b before any solve kernel runs), a second
solve or a level operation on a hierarchy with a resumable solve in progress
(STK_EBUSY, the running solve unaffected), and a patch factorisation that
breaks down (STK_ENOTSPD: at gamma = 1e300 the augmented term swamps the
viscous one, so the patch matrices are numerically singular and Cholesky
meets non-positive pivots)."""
import numpy as np
import pytest

from gpu_common import CASES, oracle_for, gpu_for, to_dev, to_host, rel, log

pytestmark = pytest.mark.gpu

NAME = "sinker_2d_16sq_L2"


def test_maxit_returns_notconv_with_last_iterate():
    from paper_2107_00820_amd.stk import STK_ENOTCONV
    log("[fail] maxit = 1")
    orc, gpu = oracle_for(NAME), gpu_for(NAME)
    lv = orc.mg.hier[-1]
    bu, bp = gpu.stk_rhs()
    xu, xp, info = gpu.stk_solve(bu, bp, rtol=1e-8, restart=30, maxit=1, allow_notconv=True)
    assert info["status"] == STK_ENOTCONV and not info["converged"] and info["iters"] == 1
    x_o, info_o = orc.solve(maxit=1)
    x = np.concatenate([lv.from_stored(to_host(xu)), to_host(xp)])
    assert not info_o["converged"] and info_o["iters"] == 1
    assert rel(x, x_o) <= 1e-10
    # rel_res is the true residual of the returned iterate
    b = orc.rhs()
    rr = np.linalg.norm(b - orc.K @ x) / np.linalg.norm(b)
    assert abs(info["rel_res"] - rr) <= 1e-8 * rr and 0.0 < rr < 1.0
    assert len(info["hist"]) == 2


def test_nonfinite_rhs_returns_enan():
    from paper_2107_00820_amd.stk import STK_ENAN, StkError
    log("[fail] NaN in b_u")
    gpu = gpu_for(NAME)
    bu, bp = gpu.stk_rhs()
    bad = bu.clone()
    bad[bad.numel() // 2] = float("nan")
    xu, xp, info = gpu.stk_solve(bad, bp, allow=(STK_ENAN,))
    assert info["status"] == STK_ENAN and not info["converged"] and info["iters"] == 0
    with pytest.raises(StkError) as e:
        gpu.stk_solve_begin(bad, bp, eager=True)
    assert e.value.status == STK_ENAN
    # the hierarchy is usable afterwards
    xu, xp, info = gpu.stk_solve(bu, bp)
    assert info["converged"]


def test_busy_hierarchy_rejects_other_work():
    import torch
    from paper_2107_00820_amd import stk_step_batch
    from paper_2107_00820_amd.stk import STK_EBUSY, StkError
    log("[fail] calls during a resumable solve")
    gpu = gpu_for(NAME)
    bu, bp = gpu.stk_rhs()
    ref_u, ref_p, ref = gpu.stk_solve(bu, bp, eager=True)
    ref_u, ref_p = to_host(ref_u), to_host(ref_p)
    xu, xp = gpu.stk_solve_begin(bu, bp, eager=True)
    y = gpu.zeros_u()
    calls = [lambda: gpu.stk_solve_begin(bu, bp, eager=True),
             lambda: gpu.stk_solve(bu, bp),
             lambda: gpu.stk_vcycle(bu, y),
             lambda: gpu.stk_fcycle(bu, y),
             lambda: gpu.stk_apply_Agamma(1, bu, y),
             lambda: gpu.stk_asm(1, bu, y),
             lambda: gpu.stk_smooth(1, bu, y, 2),
             lambda: gpu.stk_precond(bu, bp),
             lambda: gpu.stk_apply_stokes(bu, bp),
             lambda: gpu.stk_rhs(),
             lambda: gpu.stk_autotune(reps=1),
             lambda: gpu.stk_set_asm_variant(1, 0)]
    info = None
    for k in range(100000):
        if k < len(calls):
            with pytest.raises(StkError) as e:
                calls[k]()
            assert e.value.status == STK_EBUSY, k
        info = gpu.stk_poll()
        if info is not None:
            break
        stk_step_batch([gpu])
    assert info is not None and info["converged"] and info["iters"] == ref["iters"]
    torch.cuda.synchronize()
    assert np.array_equal(to_host(xu), ref_u) and np.array_equal(to_host(xp), ref_p)
    # idle again: the level operations work
    gpu.stk_vcycle(bu, y)


def test_breakdown_of_patch_factorisation_returns_enotspd():
    from paper_2107_00820_amd import Hierarchy, desc_from_workload
    from paper_2107_00820_amd.stk import STK_ENOTSPD, StkError
    from workloads import small
    log("[fail] gamma = 1e300")
    wl = small(2, 8, 2, gamma=1e300, dr=1e2, n_sinkers=4, seed=3)
    with pytest.raises(StkError) as e:
        Hierarchy(desc_from_workload(wl))
    assert e.value.status == STK_ENOTSPD
