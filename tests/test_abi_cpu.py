"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/stk.h declares, validates descriptors and computes the
HBM footprint without touching a device."""
import os
import re

import pytest

from workloads import CONFIGS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    hdr = open(os.path.join(ROOT, "include", "stk.h")).read()
    return re.findall(r"^\s*(?:stk_status|const char\*)\s+(stk_\w+)\s*\(", hdr, re.M)


def test_library_exports_every_declared_symbol():
    from paper_2107_00820_amd import stk
    lib = stk.load()
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_footprint_and_validation():
    from paper_2107_00820_amd import stk
    d = stk.desc_from_workload(CONFIGS["sinker_2d_128sq_L4"])
    fp = stk.stk_footprint(d)
    # packed interior inverses alone: 16129 patches of 18x18
    assert fp > 16129 * 171 * 8
    assert fp < 2 ** 30
    d3 = stk.desc_from_workload(CONFIGS["sinker_3d_32cu_L3"])
    assert stk.stk_footprint(d3) > 29791 * (81 * 82 // 2) * 8
    bad = stk.desc_from_workload(CONFIGS["sinker_2d_128sq_L4"])
    bad.n_fine = 100          # not a multiple of 2^(levels-1)
    with pytest.raises(stk.StkError) as e:
        stk.stk_footprint(bad)
    assert e.value.status == stk.STK_EINVAL
    bad = stk.desc_from_workload(CONFIGS["sinker_2d_128sq_L4"])
    bad.sinker.mu_min = -1.0
    with pytest.raises(stk.StkError):
        stk.stk_footprint(bad)
    bad = stk.desc_from_workload(CONFIGS["sinker_2d_128sq_L4"])
    bad.nu_pre = 9
    with pytest.raises(stk.StkError):
        stk.stk_footprint(bad)


def test_setup_rejects_budget_before_touching_the_device():
    from paper_2107_00820_amd import stk
    import ctypes
    d = stk.desc_from_workload(CONFIGS["sinker_2d_16sq_L2"], hbm_budget=1024)
    h = ctypes.c_void_p()
    st = stk.load().stk_setup_hierarchy(ctypes.byref(d), None, ctypes.byref(h))
    assert st == stk.STK_ENOMEM and not h.value
    assert b"exceeds budget" in stk.load().stk_last_error()


def test_tensor_and_mixed_descriptors():
    """The viscoplastic tensor adds mu_eff and w (d(d+1)/2 values) per Gauss
    point on every level; the mixed form adds FP32 copies. Bad tensor
    parameters are rejected on the host."""
    from paper_2107_00820_amd import stk
    wl = CONFIGS["viscoplastic_3d_48cu_L3"]
    d_t = stk.desc_from_workload(wl)
    assert d_t.coef_kind == 1 and d_t.vp.modes == wl.fourier_modes
    d_s = stk.desc_from_workload(wl)
    d_s.coef_kind = 0
    gauss_pts = sum(27 * (wl.n_level(l) ** 3) for l in range(wl.levels))
    assert stk.stk_footprint(d_t) - stk.stk_footprint(d_s) >= 6 * 8 * gauss_pts
    d_m = stk.desc_from_workload(wl, mixed=1)
    assert stk.stk_footprint(d_m) > stk.stk_footprint(d_t)
    bad = stk.desc_from_workload(wl)
    bad.vp.modes = 9
    with pytest.raises(stk.StkError):
        stk.stk_footprint(bad)
    bad = stk.desc_from_workload(wl)
    bad.vp.tau_y = 0.0
    with pytest.raises(stk.StkError):
        stk.stk_footprint(bad)
    bad = stk.desc_from_workload(CONFIGS["sinker_2d_128sq_L4"])
    bad.mixed = 2
    with pytest.raises(stk.StkError):
        stk.stk_footprint(bad)


def test_descriptor_fields_of_the_boundary():
    """qpts_1d accepts the default (0) and the 3-point rule only; the
    viscoplastic floor and strain-rate scale must be finite."""
    from paper_2107_00820_amd import stk
    for q, ok in ((0, True), (3, True), (2, False), (4, False)):
        d = stk.desc_from_workload(CONFIGS["sinker_2d_16sq_L2"])
        d.qpts_1d = q
        if ok:
            assert stk.stk_footprint(d) > 0
        else:
            with pytest.raises(stk.StkError) as e:
                stk.stk_footprint(d)
            assert e.value.status == stk.STK_EINVAL and b"qpts_1d" in stk.load().stk_last_error()
    d = stk.desc_from_workload(CONFIGS["viscoplastic_3d_48cu_L3"])
    assert stk.stk_footprint(d) > 0
    d.vp.mu_floor = float("nan")
    with pytest.raises(stk.StkError):
        stk.stk_footprint(d)
    d = stk.desc_from_workload(CONFIGS["viscoplastic_3d_48cu_L3"])
    d.vp.eps_scale = float("inf")
    with pytest.raises(stk.StkError):
        stk.stk_footprint(d)


def test_degree_three_descriptor():
    """degree 3 ([Q3]^d x P2disc) is accepted with the scalar law and the
    FP64 form (3D up to 32^3 cells); its footprint holds 16 Gauss points per
    cell, 6 pressure unknowns per cell and 50-unknown patch inverses in 2D,
    and the stored 375-unknown inverses in 3D; other combinations (a 3D mesh
    over 32^3 cells, the mixed form, the tensor law, degree 4) are rejected
    on the host."""
    from paper_2107_00820_amd import stk
    from workloads import small
    wl3 = small(2, 64, 3, gamma=1e3, dr=1e4, degree=3)
    wl2 = small(2, 64, 3, gamma=1e3, dr=1e4)
    f3, f2 = stk.stk_footprint(stk.desc_from_workload(wl3)), stk.stk_footprint(stk.desc_from_workload(wl2))
    # packed 50-unknown inverses on the finest level alone: 65^2 patches x 1275 doubles
    assert f3 - f2 >= 8 * 65 * 65 * (1275 - 171)
    for q, ok in ((0, True), (4, True), (3, False)):
        d = stk.desc_from_workload(wl3)
        d.qpts_1d = q
        if ok:
            assert stk.stk_footprint(d) > 0
        else:
            with pytest.raises(stk.StkError):
                stk.stk_footprint(d)
    # 3D degree 3 up to 32^3 (explicit 375-unknown patch inverses): the finest
    # level of 16^3 alone holds 17^3 inverses of 74,496 doubles (15 full 64 x 64
    # tiles and 6 diagonal tiles of 2,176); 32^3 is accepted, 36^3 is not
    f16 = stk.stk_footprint(stk.desc_from_workload(small(3, 16, 2, gamma=1e3, dr=1e4, degree=3)))
    assert f16 >= 8 * 17 ** 3 * (15 * 4096 + 6 * 2176)
    assert stk.stk_footprint(stk.desc_from_workload(small(3, 32, 4, gamma=1e3, dr=1e4, degree=3))) > f16
    with pytest.raises(stk.StkError) as e:
        stk.stk_footprint(stk.desc_from_workload(small(3, 36, 3, gamma=1e3, dr=1e4, degree=3)))
    assert e.value.status == stk.STK_EINVAL
    for field, value in (("mixed", 1), ("dim", 3), ("coef_kind", 1), ("degree", 4)):
        d = stk.desc_from_workload(wl3)
        setattr(d, field, value)
        with pytest.raises(stk.StkError) as e:
            stk.stk_footprint(d)
        assert e.value.status == stk.STK_EINVAL
