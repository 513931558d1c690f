"""Autotuning of the batched star-patch solve: every variant of the kernel
performs the same multiply-adds in the same order, so the patch-solve output
must be bit-identical across variants (FP64 and FP32), the tuner must return
a valid choice per smoothed level and precision, and a solve after tuning
must reproduce the solve before it bit for bit."""
import numpy as np
import pytest

from gpu_common import CASES, log
from paper_2107_00820_amd.stk import STK_ASM_VARIANTS

pytestmark = pytest.mark.gpu

NAMES = ["2d_32_L3", "3d_8_L2"]
NVAR = STK_ASM_VARIANTS


@pytest.mark.parametrize("name", NAMES)
def test_variants_bit_identical_and_tuning(name):
    import torch
    from paper_2107_00820_amd import Hierarchy
    wl = CASES[name]
    h = Hierarchy.from_workload(wl, mixed=1)
    try:
        gen = torch.Generator(device="cuda").manual_seed(7)
        for l in range(1, h.L):
            nv, _ = h.sizes(l)
            r64 = torch.randn(nv, dtype=torch.float64, device="cuda", generator=gen)
            for dt, r in ((torch.float64, r64), (torch.float32, r64.float())):
                outs = []
                for v in range(NVAR):
                    h.stk_set_asm_variant(l, v, dt)
                    outs.append(h.stk_asm(l, r).cpu().numpy())
                log(f"  {name} level {l} {dt}: variants {NVAR}, max |y| {np.abs(outs[0]).max():.3e}")
                for v in range(1, NVAR):
                    assert np.array_equal(outs[0], outs[v]), (l, dt, v)
                h.stk_set_asm_variant(l, 0, dt)
        bu, bp = h.stk_rhs()
        xu0, xp0, i0 = h.stk_solve(bu, bp, rtol=wl.rtol, restart=wl.restart, maxit=wl.maxit)
        xu0, xp0 = xu0.cpu().numpy(), xp0.cpu().numpy()
        choice = h.stk_autotune(reps=3)
        log(f"  {name} autotune: {choice}")
        assert set(choice) == {(l, p) for l in range(1, h.L) for p in ("f64", "f32")}
        assert all(0 <= v < NVAR for v in choice.values())
        xu1, xp1, i1 = h.stk_solve(bu, bp, rtol=wl.rtol, restart=wl.restart, maxit=wl.maxit)
        assert i1["iters"] == i0["iters"]
        assert np.array_equal(xu1.cpu().numpy(), xu0) and np.array_equal(xp1.cpu().numpy(), xp0)
    finally:
        h.close()
