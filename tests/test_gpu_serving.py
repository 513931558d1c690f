"""Serving loop on the GPU: requests that arrive while others run are
admitted as memory and slots free up, their solves overlap on the device, and
every result is bit-identical to the same request solved alone (the
resumable solve runs the same kernels in the same order on each hierarchy;
no state is shared between requests)."""
import numpy as np
import pytest

from workloads import small
from gpu_common import log

pytestmark = pytest.mark.gpu


def _requests():
    # mixed 2D/3D sizes and contrasts, arriving 5 ms apart (so that they overlap)
    specs = [
        (2, 32, 2, 1e3, 1e6, 1),
        (3, 8, 2, 1e4, 1e8, 2),
        (2, 64, 3, 1e3, 1e4, 3),
        (2, 16, 2, 1e3, 1e6, 4),
        (3, 16, 2, 1e4, 1e5, 5),
        (2, 32, 2, 1e3, 1e8, 6),
    ]
    return [(0.005 * k, small(d, n, L, gamma=g, dr=dr, n_sinkers=24, seed=10 ** 6 + s))
            for k, (d, n, L, g, dr, s) in enumerate(specs)]


@pytest.mark.parametrize("cross", ["0", "1"])
def test_mix_equals_alone_and_overlaps(cross, monkeypatch):
    import torch
    from paper_2107_00820_amd import Hierarchy
    from paper_2107_00820_amd.serve import Server
    monkeypatch.setenv("STK_CROSS_BATCH", cross)
    reqs = _requests()
    log(f"[serving] mix of 6 requests, STK_CROSS_BATCH={cross}")
    out = Server(hbm_budget=8 << 30, max_active=4, keep_solutions=True).run(reqs)
    assert out["completed"] == len(reqs), [r.error for r in out["results"]]
    assert out["peak_active"] >= 2            # solves were in flight together
    for r in out["results"]:
        wl = reqs[r.index][1]
        h = Hierarchy.from_workload(wl)
        bu, bp = h.stk_rhs()
        xu, xp, info = h.stk_solve(bu, bp)
        torch.cuda.synchronize()
        log(f"  {wl.name}: mix {r.iters} it, alone {info['iters']} it")
        assert info["iters"] == r.iters
        assert np.array_equal(xu.cpu().numpy(), r.solution[0])
        assert np.array_equal(xp.cpu().numpy(), r.solution[1])
        h.close()


def test_admission_respects_budget():
    """With a budget that holds one request at a time, requests are served
    one after another and the peak footprint never exceeds the budget; a
    request larger than the budget is rejected without touching the device."""
    from paper_2107_00820_amd import desc_from_workload, stk_footprint
    from paper_2107_00820_amd.serve import Server
    reqs = _requests()[:3]
    fps = [stk_footprint(desc_from_workload(w)) for _, w in reqs]
    budget = max(fps) + 1
    out = Server(hbm_budget=budget, max_active=4).run(reqs)
    assert out["completed"] == 3
    assert out["peak_footprint_bytes"] <= budget
    big = [(0.0, small(3, 32, 3, gamma=1e4, dr=1e4, n_sinkers=24, seed=9))]
    out = Server(hbm_budget=budget, max_active=4).run(big)
    assert out["completed"] == 0 and out["results"][0].error


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("cross", ["1", "0"])
def test_same_shape_requests_step_together_and_equal_alone(dim, cross, monkeypatch):
    """Same-shape requests started together step in lockstep with batched
    star-patch solve launches (STK_CROSS_BATCH=1) or each on its own (0,
    the default); either way every solution and iteration count is
    bit-identical to the request solved alone."""
    import torch
    from paper_2107_00820_amd import Hierarchy, stk_step_batch
    monkeypatch.setenv("STK_CROSS_BATCH", cross)
    n, L, g = (32, 2, 1e3) if dim == 2 else (8, 2, 1e4)
    wls = [small(dim, n, L, gamma=g, dr=dr, n_sinkers=24, seed=2 * 10 ** 6 + k)
           for k, dr in enumerate((1e4, 1e6, 1e8, 1e5, 1e7))]
    log(f"[cohort] {len(wls)} x {dim}D {n} L{L}, STK_CROSS_BATCH={cross}")
    hs = [Hierarchy.from_workload(w) for w in wls]
    outs = []
    for h in hs:
        bu, bp = h.stk_rhs()
        outs.append(h.stk_solve_begin(bu, bp, eager=True))
    infos = [None] * len(hs)
    for _ in range(100000):
        if all(i is not None for i in infos):
            break
        stk_step_batch([h for h, i in zip(hs, infos) if i is None])
        for k, h in enumerate(hs):
            if infos[k] is None:
                infos[k] = h.stk_poll()
    assert all(i is not None and i["converged"] for i in infos)
    for k, (h, w) in enumerate(zip(hs, wls)):
        bu, bp = h.stk_rhs()
        xu, xp, info = h.stk_solve(bu, bp, eager=True)
        torch.cuda.synchronize()
        assert info["iters"] == infos[k]["iters"]
        assert np.array_equal(xu.cpu().numpy(), outs[k][0].cpu().numpy())
        assert np.array_equal(xp.cpu().numpy(), outs[k][1].cpu().numpy())
        h.close()


def test_degree_three_requests_in_the_mix():
    """[Q3]^2 x P2disc requests served beside Q2 ones (same-size meshes, so
    the cross-request cohorts must keep the degrees apart): results
    bit-identical to each request solved alone."""
    import os
    import torch
    from paper_2107_00820_amd import Hierarchy
    from paper_2107_00820_amd.serve import Server
    reqs = [(0.002 * k, small(2, 32, 2, gamma=1e3, dr=1e4, n_sinkers=24, seed=3 * 10 ** 6 + k, degree=d))
            for k, d in enumerate((3, 2, 3, 2, 3))]
    for cross in ("0", "1"):
        os.environ["STK_CROSS_BATCH"] = cross
        try:
            out = Server(hbm_budget=8 << 30, max_active=5, keep_solutions=True).run(reqs)
        finally:
            del os.environ["STK_CROSS_BATCH"]
        assert out["completed"] == len(reqs), [r.error for r in out["results"]]
        for r in out["results"]:
            wl = reqs[r.index][1]
            h = Hierarchy.from_workload(wl)
            bu, bp = h.stk_rhs()
            xu, xp, info = h.stk_solve(bu, bp, eager=True)
            torch.cuda.synchronize()
            log(f"  [q3 mix, cross {cross}] {wl.name} (degree {wl.degree}): {r.iters} it, alone {info['iters']}")
            assert info["iters"] == r.iters
            assert np.array_equal(xu.cpu().numpy(), r.solution[0])
            assert np.array_equal(xp.cpu().numpy(), r.solution[1])
            h.close()
