"""stk_asm_noalloc (the star-patch solve with its patch-output buffer in the
library's fixed device array) against stk_asm on the same hierarchy: two
calls in a row, the second on a smaller level, each bit-identical to stk_asm
(the same kernels run on the same data), in FP64 and FP32; a level whose
patch outputs exceed the fixed array is rejected before any launch."""
import ctypes as C

import numpy as np
import pytest

from gpu_common import CASES, oracle_for, gpu_for, gpu_mixed_for, to_dev, to_dev32, to_host, rand_u, log

pytestmark = pytest.mark.gpu


def noalloc(h, level, r, y):
    """The C entry point through ctypes; returns its status."""
    from paper_2107_00820_amd import stk
    code, pr, py = stk._dptr(r, y)
    return stk.load().stk_asm_noalloc(h._h, level, code, pr, py, stk._stream())


@pytest.mark.parametrize("name", ["2d_32_L3", "3d_16_L3", "q3_2d_16_L3"])
def test_noalloc_asm_equals_asm_twice(name):
    log(f"[noalloc] {name}")
    orc, gpu = oracle_for(name), gpu_for(name)
    L = CASES[name].levels
    for l in (L - 1, L - 2):             # the second call on a smaller level
        lv = orc.mg.hier[l]
        _, rs = rand_u(lv, 70 + l)
        r = to_dev(rs)
        y_ref = to_host(gpu.stk_asm(l, r))
        y = gpu.zeros_u(l)
        assert noalloc(gpu, l, r, y) == 0
        assert np.array_equal(to_host(y), y_ref), l


def test_noalloc_asm_equals_asm_twice_q3_3d():
    """[Q3]^3: 375 patch outputs per vertex; the fine level of 4^3 cells, then
    the 2^3 level of the same hierarchy."""
    from paper_2107_00820_amd import Hierarchy
    from workloads import small
    log("[noalloc] q3 3d 4^3 L3")
    h = Hierarchy.from_workload(small(3, 4, 3, gamma=1e3, dr=1e4, n_sinkers=4, seed=523, degree=3))
    rng = np.random.default_rng(90)
    for l in (2, 1):
        r = to_dev(rng.standard_normal(h.zeros_u(l).numel()))
        y_ref = to_host(h.stk_asm(l, r))
        y = h.zeros_u(l)
        assert noalloc(h, l, r, y) == 0
        assert np.array_equal(to_host(y), y_ref), l
    h.close()


def test_noalloc_asm_fp32():
    name = "2d_32_L3"
    log(f"[noalloc f32] {name}")
    import torch
    orc, gpu = oracle_for(name), gpu_mixed_for(name)
    for l in (2, 1):
        lv = orc.mg.hier[l]
        _, rs = rand_u(lv, 80 + l)
        r = to_dev32(rs)
        y_ref = to_host(gpu.stk_asm(l, r))
        y = gpu.zeros_u(l, torch.float32)
        assert noalloc(gpu, l, r, y) == 0
        assert np.array_equal(to_host(y), y_ref), l


def test_noalloc_rejects_oversized_level():
    from paper_2107_00820_amd import Hierarchy, stk
    from workloads import small
    log("[noalloc] oversized level")
    h = Hierarchy.from_workload(small(2, 1024, 5, gamma=1e2, dr=1e2, n_sinkers=4, seed=5))
    r, y = h.zeros_u(4), h.zeros_u(4)
    st = noalloc(h, 4, r, y)
    assert st == stk.STK_EINVAL and b"static buffer" in stk.load().stk_last_error()
    # a smaller level of the same hierarchy fits
    assert noalloc(h, 3, h.zeros_u(3), h.zeros_u(3)) == 0
    h.close()
    # degree 3: 50 patch outputs per vertex, so 2D 512^2 (263,169 vertices,
    # 105 MB) is over the limit where Q2 (38 MB) is not
    h = Hierarchy.from_workload(small(2, 512, 5, gamma=1e2, dr=1e2, n_sinkers=4, seed=5, degree=3))
    st = noalloc(h, 4, h.zeros_u(4), h.zeros_u(4))
    assert st == stk.STK_EINVAL and b"static buffer" in stk.load().stk_last_error()
    assert noalloc(h, 3, h.zeros_u(3), h.zeros_u(3)) == 0
    h.close()
