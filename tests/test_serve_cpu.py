"""The request loop's bookkeeping on the CPU, with stand-in hierarchies: a
request whose setup, start or solve fails is recorded with its error, its
memory is released (so requests waiting behind it are admitted) and the
loop goes on; the others complete."""
import pytest

from workloads import small
from paper_2107_00820_amd.stk import StkError, STK_ENAN, STK_EDEVICE, STK_ENOTSPD
from paper_2107_00820_amd.serve import Server


class StubHierarchy:
    """Fails at start ("start"), at the n-th poll ("poll"), or finishes after n polls."""
    closed = []

    def __init__(self, wl, mode, n=2):
        self.wl, self.mode, self.n, self.polls = wl, mode, n, 0

    def stk_rhs(self):
        return None, None

    def stk_solve_begin(self, bu, bp, **kw):
        if self.mode == "start":
            raise StkError(STK_ENAN, "right-hand side is not finite")
        return "xu", "xp"

    def stk_poll(self):
        self.polls += 1
        if self.polls < self.n:
            return None
        if self.mode == "poll":
            raise StkError(STK_EDEVICE, "phase enqueue failed")
        return dict(iters=7, converged=True, rel_res=1e-9, t_solve=0.0, hist=[], status=0)

    def close(self):
        StubHierarchy.closed.append(self.wl.name)


@pytest.mark.timeout(60)
def test_failed_requests_are_recorded_and_release_memory():
    modes = {0: "ok", 1: "start", 2: "poll", 3: "setup", 4: "ok", 5: "ok"}
    reqs = [(0.001 * i, small(2, 8, 2, seed=100 + i)) for i in range(6)]
    by_name = {wl.name: modes[i] for i, (_, wl) in enumerate(reqs)}

    def build(wl, mixed):
        if by_name[wl.name] == "setup":
            raise StkError(STK_ENOTSPD, "non-positive pivot")
        return StubHierarchy(wl, by_name[wl.name], n=3)

    steps = []
    StubHierarchy.closed = []
    # the budget admits one request at a time: a leaked footprint would stall the loop
    srv = Server(hbm_budget=100, max_active=4, setup_workers=1, build=build,
                 step=lambda hs: steps.append(len(hs)), footprint=lambda wl, mixed: 60)
    out = srv.run(reqs)
    res = out["results"]
    assert out["completed"] == 3 and out["failed"] == 3
    assert [r.converged for r in res] == [True, False, False, False, True, True]
    assert res[1].status == STK_ENAN and "not finite" in res[1].error
    assert res[2].status == STK_EDEVICE and res[2].error
    assert res[3].status == STK_ENOTSPD and res[3].error
    # every hierarchy that was built got closed exactly once
    built = [wl.name for i, (_, wl) in enumerate(reqs) if modes[i] != "setup"]
    assert sorted(StubHierarchy.closed) == sorted(built)
    assert max(steps) == 1 and out["peak_footprint_bytes"] == 60


def test_oversized_request_is_rejected_without_setup():
    calls = []
    srv = Server(hbm_budget=10, build=lambda wl, m: calls.append(wl) or StubHierarchy(wl, "ok"),
                 step=lambda hs: None, footprint=lambda wl, mixed: 11)
    out = srv.run([(0.0, small(2, 8, 2, seed=1))])
    assert out["failed"] == 1 and not calls
    assert "budget" in out["results"][0].error
