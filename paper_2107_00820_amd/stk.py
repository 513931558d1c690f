"""ctypes binding of libstk.so (argument marshalling only).

Names follow the C ABI in include/stk.h. Buffers are torch tensors on the
current HIP device (contiguous float64; the level operations also take
float32 tensors on a hierarchy built with mixed=1, and the dtype passed to
the library follows the tensors); every device step runs in the HIP kernels
of libstk.so. There is no fallback path: if the library is missing
or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstk.so")

STK_OK, STK_EINVAL, STK_ENOMEM, STK_EDEVICE, STK_ENOTCONV, STK_ENOTSPD, STK_ENAN, STK_EBUSY = 0, -1, -2, -3, -4, -5, -6, -7
STK_F64, STK_F32 = 0, 1
STK_ASM_VARIANTS = 4
STK_PC_MIXED, STK_PC_UPPER, STK_PC_FCYCLE = 1, 2, 4
STK_BATCH_MAX = 8
_PC = {"full": 0, "upper": 1}
_CYCLE = {"V": 0, "F": 1}
_NAMES = {0: "STK_OK", -1: "STK_EINVAL", -2: "STK_ENOMEM", -3: "STK_EDEVICE", -4: "STK_ENOTCONV",
          -5: "STK_ENOTSPD", -6: "STK_ENAN", -7: "STK_EBUSY"}


class StkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class Sinker(C.Structure):
    _fields_ = [("n", C.c_int), ("centers", C.POINTER(C.c_double)), ("omega", C.c_double),
                ("delta", C.c_double), ("mu_min", C.c_double), ("mu_max", C.c_double), ("beta", C.c_double)]


class Viscoplastic(C.Structure):
    _fields_ = [("modes", C.c_int), ("amp", C.POINTER(C.c_double)), ("tau_y", C.c_double),
                ("mu_floor", C.c_double), ("eps_scale", C.c_double)]


class Desc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_fine", C.c_int), ("n_levels", C.c_int), ("qpts_1d", C.c_int),
                ("gamma", C.c_double),
                ("schur", C.c_int), ("coef_kind", C.c_int), ("sinker", Sinker), ("vp", Viscoplastic),
                ("nu_pre", C.c_int), ("nu_post", C.c_int), ("mixed", C.c_int), ("hbm_budget", C.c_size_t),
                ("degree", C.c_int)]


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("restart", C.c_int), ("maxit", C.c_int), ("eager", C.c_int),
                ("mixed", C.c_int), ("pc", C.c_int), ("cycle", C.c_int)]


class NewtonOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int), ("lin_rtol", C.c_double), ("lin_maxit", C.c_int),
                ("restart", C.c_int), ("max_halvings", C.c_int), ("pc", C.c_int), ("cycle", C.c_int),
                ("eager", C.c_int)]


STK_NEWTON_MAXIT = 64


class NewtonInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("rel_res", C.c_double), ("res0", C.c_double),
                ("t_s", C.c_double), ("hist", C.c_double * (STK_NEWTON_MAXIT + 1)),
                ("alpha", C.c_double * STK_NEWTON_MAXIT), ("lin_iters", C.c_int * STK_NEWTON_MAXIT)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("rel_res", C.c_double),
                ("t_solve_s", C.c_double), ("hist", C.c_double * 1001)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libstk.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2107_00820_amd.build` "
                           "(or __graft_entry__.build())")
    # torch first: its HIP runtime must be the one the library binds to, so
    # that device memory and streams are shared
    import torch  # noqa: F401
    lib = C.CDLL(path)
    vp, i32, i64p, dp = C.c_void_p, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double)
    sig = {
        "stk_footprint": [C.POINTER(Desc), C.POINTER(C.c_size_t)],
        "stk_setup_hierarchy": [C.POINTER(Desc), vp, C.POINTER(vp)],
        "stk_destroy": [vp],
        "stk_sizes": [vp, i32, i64p, i64p],
        "stk_rhs": [vp, vp, vp, vp],
        "stk_apply_Agamma": [vp, i32, i32, vp, vp, vp],
        "stk_apply_stokes": [vp, vp, vp, vp, vp, vp],
        "stk_asm": [vp, i32, i32, vp, vp, vp],
        "stk_asm_noalloc": [vp, i32, i32, vp, vp, vp],
        "stk_smooth": [vp, i32, i32, vp, vp, i32, vp],
        "stk_prolong": [vp, i32, i32, vp, vp, vp],
        "stk_restrict": [vp, i32, i32, vp, vp, vp],
        "stk_coarse_solve": [vp, vp, vp, vp],
        "stk_vcycle": [vp, i32, vp, vp, vp],
        "stk_fcycle": [vp, i32, vp, vp, vp],
        "stk_precond": [vp, i32, vp, vp, vp, vp, vp],
        "stk_solve": [vp, vp, vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp],
        "stk_solve_begin": [vp, vp, vp, vp, vp, C.POINTER(SolveOpts), vp],
        "stk_step_batch": [C.POINTER(vp), i32, vp],
        "stk_poll": [vp, C.POINTER(SolveInfo)],
        "stk_profile": [vp, i32],
        "stk_profile_read": [vp, i32, i64p, dp, dp],
        "stk_autotune": [vp, i32, C.POINTER(C.c_int), C.POINTER(C.c_float), vp],
        "stk_set_asm_variant": [vp, i32, i32, i32],
        "stk_relinearize": [vp, vp, vp],
        "stk_nl_residual": [vp, vp, vp, vp, vp, vp],
        "stk_newton": [vp, vp, vp, C.POINTER(NewtonOpts), C.POINTER(NewtonInfo), vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.stk_last_error.argtypes = []
    lib.stk_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _check(st: int, allow=()):
    if st != STK_OK and st not in allow:
        raise StkError(st, load().stk_last_error().decode())
    return st


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> C.c_void_p:
    import torch
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), "expected a contiguous float64 GPU tensor"
    return C.c_void_p(t.data_ptr())


def _dptr(*ts):
    """dtype code and pointers for tensors that must share one float dtype."""
    import torch
    dt = ts[0].dtype
    code = {torch.float64: STK_F64, torch.float32: STK_F32}.get(dt)
    assert code is not None, "expected float64 or float32 tensors"
    for t in ts:
        assert t.is_cuda and t.dtype == dt and t.is_contiguous(), "expected contiguous GPU tensors of one dtype"
    return (code,) + tuple(C.c_void_p(t.data_ptr()) for t in ts)


def make_desc(dim, n_fine, n_levels, gamma, centers, mu_min, mu_max, omega=0.1, delta=200.0, beta=10.0,
              nu_pre=2, nu_post=2, hbm_budget=0, mixed=0, vp_amp=None, vp_tau_y=0.0, vp_eps_scale=0.0, schur=1,
              vp_mu_floor=0.0, qpts_1d=0, newton=False, degree=2):
    """Descriptor; vp_amp (array [d][M]^d) selects the viscoplastic Newton
    tensor over the sinker base field (coef_kind 1); newton=True the
    viscoplastic state for the Newton loop (coef_kind 2, with vp_tau_y);
    degree=3 the [Q3]^2 x P2disc discretisation."""
    centers = np.ascontiguousarray(np.asarray(centers, dtype=np.float64).reshape(-1, dim))
    d = Desc()
    d.dim, d.n_fine, d.n_levels, d.gamma = dim, n_fine, n_levels, float(gamma)
    d.qpts_1d = int(qpts_1d)
    d.schur, d.coef_kind, d.mixed = int(schur), 0, int(mixed)
    if vp_amp is not None:
        amp = np.ascontiguousarray(np.asarray(vp_amp, dtype=np.float64))
        assert amp.ndim == dim + 1 and amp.shape[0] == dim and all(s == amp.shape[1] for s in amp.shape[1:])
        d.coef_kind = 1
        d.vp.modes = amp.shape[1]
        d.vp.amp = amp.ctypes.data_as(C.POINTER(C.c_double))
        d.vp.tau_y, d.vp.eps_scale, d.vp.mu_floor = float(vp_tau_y), float(vp_eps_scale), float(vp_mu_floor)
        d._keep_amp = amp
    if newton:
        d.coef_kind = 2
        d.vp.tau_y, d.vp.mu_floor = float(vp_tau_y), float(vp_mu_floor)
    d.sinker.n = centers.shape[0]
    d.sinker.centers = centers.ctypes.data_as(C.POINTER(C.c_double))
    d.sinker.omega, d.sinker.delta, d.sinker.beta = omega, delta, beta
    d.sinker.mu_min, d.sinker.mu_max = mu_min, mu_max
    d.nu_pre, d.nu_post = nu_pre, nu_post
    d.hbm_budget = int(hbm_budget)
    d.degree = int(degree)
    d._keep = centers          # keep the host array alive while the desc is used
    return d


def desc_from_workload(wl, hbm_budget=0, mixed=0):
    """Descriptor of a workload. For the viscoplastic workloads the yield
    stress is 2 mu_max and the velocity scale is left to the library (root
    mean square of eps_II over the finest Gauss points equal to 1)."""
    from workloads import OMEGA, DELTA, BETA
    vp = {}
    if wl.coef_kind == 1:
        vp = dict(vp_amp=wl.fourier_amplitudes(), vp_tau_y=wl.tau_y if wl.tau_y > 0 else 2.0 * wl.mu_max,
                  vp_mu_floor=wl.mu_floor)
    elif wl.coef_kind == 2:
        vp = dict(newton=True, vp_tau_y=wl.tau_y, vp_mu_floor=wl.mu_floor)
    return make_desc(wl.dim, wl.n_fine, wl.levels, wl.gamma, wl.centers(), wl.mu_min, wl.mu_max,
                     OMEGA, DELTA, BETA, wl.nu_pre, wl.nu_post, hbm_budget, mixed, schur=getattr(wl, "schur", 1),
                     degree=getattr(wl, "degree", 2), **vp)


def stk_step_batch(hierarchies) -> int:
    """One phase of every listed hierarchy's solve (their device work overlaps)."""
    arr = (C.c_void_p * len(hierarchies))(*[h._h.value for h in hierarchies])
    return _check(load().stk_step_batch(arr, len(hierarchies), None), allow=(STK_ENOTCONV, STK_ENAN))


def stk_footprint(desc: Desc) -> int:
    out = C.c_size_t(0)
    _check(load().stk_footprint(C.byref(desc), C.byref(out)))
    return out.value


class Hierarchy:
    """A device hierarchy (stk_setup_hierarchy ... stk_destroy)."""

    def __init__(self, desc: Desc):
        import torch
        lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("libstk needs a HIP GPU; none is visible")
        self.desc = desc
        self.dim, self.L = desc.dim, desc.n_levels
        h = C.c_void_p()
        _check(lib.stk_setup_hierarchy(C.byref(desc), _stream(), C.byref(h)))
        self._h = h

    @classmethod
    def from_workload(cls, wl, hbm_budget=0, mixed=0):
        return cls(desc_from_workload(wl, hbm_budget, mixed))

    def close(self):
        if getattr(self, "_h", None):
            load().stk_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- sizes and buffers
    def sizes(self, level: int):
        nv, npr = C.c_int64(), C.c_int64()
        _check(load().stk_sizes(self._h, level, C.byref(nv), C.byref(npr)))
        return nv.value, npr.value

    def zeros_u(self, level: Optional[int] = None, dtype=None):
        import torch
        nv, _ = self.sizes(self.L - 1 if level is None else level)
        return torch.zeros(nv, dtype=torch.float64 if dtype is None else dtype, device="cuda")

    def zeros_p(self):
        import torch
        _, npr = self.sizes(self.L - 1)
        return torch.zeros(npr, dtype=torch.float64, device="cuda")

    # ---- operations (same names as the C ABI)
    def stk_rhs(self):
        bu, bp = self.zeros_u(), self.zeros_p()
        _check(load().stk_rhs(self._h, _ptr(bu), _ptr(bp), _stream()))
        return bu, bp

    def stk_apply_Agamma(self, level, x, y=None):
        y = self.zeros_u(level, x.dtype) if y is None else y
        _check(load().stk_apply_Agamma(self._h, level, *_dptr(x, y), _stream()))
        return y

    def stk_apply_stokes(self, xu, xp, yu=None, yp=None):
        yu = self.zeros_u() if yu is None else yu
        yp = self.zeros_p() if yp is None else yp
        _check(load().stk_apply_stokes(self._h, _ptr(xu), _ptr(xp), _ptr(yu), _ptr(yp), _stream()))
        return yu, yp

    def stk_asm(self, level, r, y=None):
        y = self.zeros_u(level, r.dtype) if y is None else y
        _check(load().stk_asm(self._h, level, *_dptr(r, y), _stream()))
        return y

    def stk_asm_noalloc(self, level, r, y=None):
        """stk_asm with the patch outputs in the library's fixed device array
        (the call allocates nothing; y must be preallocated for that)."""
        y = self.zeros_u(level, r.dtype) if y is None else y
        _check(load().stk_asm_noalloc(self._h, level, *_dptr(r, y), _stream()))
        return y

    def stk_smooth(self, level, b, x, nsteps):
        code, pb, px = _dptr(b, x)
        _check(load().stk_smooth(self._h, level, code, pb, px, nsteps, _stream()))
        return x

    def stk_prolong(self, coarse_level, xc, xf=None):
        xf = self.zeros_u(coarse_level + 1, xc.dtype) if xf is None else xf
        _check(load().stk_prolong(self._h, coarse_level, *_dptr(xc, xf), _stream()))
        return xf

    def stk_restrict(self, fine_level, rf, rc=None):
        rc = self.zeros_u(fine_level - 1, rf.dtype) if rc is None else rc
        _check(load().stk_restrict(self._h, fine_level, *_dptr(rf, rc), _stream()))
        return rc

    def stk_coarse_solve(self, b, x=None):
        x = self.zeros_u(0) if x is None else x
        _check(load().stk_coarse_solve(self._h, _ptr(b), _ptr(x), _stream()))
        return x

    def stk_vcycle(self, b, x=None):
        x = self.zeros_u(None, b.dtype) if x is None else x
        _check(load().stk_vcycle(self._h, *_dptr(b, x), _stream()))
        return x

    def stk_fcycle(self, b, x=None):
        x = self.zeros_u(None, b.dtype) if x is None else x
        _check(load().stk_fcycle(self._h, *_dptr(b, x), _stream()))
        return x

    def stk_precond(self, vu, vp, zu=None, zp=None, mixed=False, pc="full", cycle="V"):
        zu = self.zeros_u() if zu is None else zu
        zp = self.zeros_p() if zp is None else zp
        flags = ((STK_PC_MIXED if mixed else 0) | (STK_PC_UPPER if pc == "upper" else 0) |
                 (STK_PC_FCYCLE if cycle == "F" else 0))
        _check(load().stk_precond(self._h, flags, _ptr(vu), _ptr(vp), _ptr(zu), _ptr(zp), _stream()))
        return zu, zp

    # ---- serving (resumable solves)
    def stk_solve_begin(self, bu, bp=None, rtol=1e-8, restart=30, maxit=300, xu=None, xp=None, eager=False,
                        mixed=False, pc="full", cycle="V"):
        """Starts a solve; the returned output tensors are filled once
        stk_poll reports completion."""
        xu = self.zeros_u() if xu is None else xu
        xp = self.zeros_p() if xp is None else xp
        opts = SolveOpts(rtol, restart, maxit, 1 if eager else 0, 1 if mixed else 0, _PC[pc], _CYCLE[cycle])
        self._solve_refs = (bu, bp, xu, xp)        # keep the buffers alive while the solve runs
        _check(load().stk_solve_begin(self._h, _ptr(bu), _ptr(bp) if bp is not None else None, _ptr(xu),
                                      _ptr(xp), C.byref(opts), _stream()))
        return xu, xp

    def stk_poll(self):
        """None while running, else the info dict (status included)."""
        info = SolveInfo()
        st = load().stk_poll(self._h, C.byref(info))
        if st == STK_EBUSY:
            return None
        _check(st, allow=(STK_ENOTCONV, STK_ENAN))
        return dict(iters=info.iters, converged=bool(info.converged), rel_res=info.rel_res,
                    t_solve=info.t_solve_s, hist=list(info.hist[:info.iters + 1]), status=st)

    # ---- viscoplastic Newton (hierarchies set up with coef_kind 2)
    def stk_relinearize(self, xu):
        _check(load().stk_relinearize(self._h, _ptr(xu), _stream()))

    def stk_nl_residual(self, xu, xp, ru=None, rp=None):
        ru = self.zeros_u() if ru is None else ru
        rp = self.zeros_p() if rp is None else rp
        _check(load().stk_nl_residual(self._h, _ptr(xu), _ptr(xp), _ptr(ru), _ptr(rp), _stream()))
        return ru, rp

    def stk_newton(self, rtol=1e-8, maxit=30, lin_rtol=1e-6, lin_maxit=300, restart=30, max_halvings=10,
                   pc="full", cycle="V", eager=False, xu=None, xp=None, allow_notconv=False):
        xu = self.zeros_u() if xu is None else xu
        xp = self.zeros_p() if xp is None else xp
        o = NewtonOpts(rtol, maxit, lin_rtol, lin_maxit, restart, max_halvings, _PC[pc], _CYCLE[cycle],
                       1 if eager else 0)
        info = NewtonInfo()
        st = load().stk_newton(self._h, _ptr(xu), _ptr(xp), C.byref(o), C.byref(info), _stream())
        _check(st, allow=(STK_ENOTCONV,) if allow_notconv else ())
        k = info.iters
        return xu, xp, dict(iters=k, converged=bool(info.converged), rel_res=info.rel_res, res0=info.res0,
                            t_s=info.t_s, hist=list(info.hist[:k + 1]), alpha=list(info.alpha[:k]),
                            lin_iters=list(info.lin_iters[:k]), status=st)

    def stk_autotune(self, reps: int = 5, with_times: bool = False):
        """Time the bit-identical patch-solve variants on every smoothed level
        and keep the fastest; returns {(level, "f64"|"f32"): variant} (and the
        per-variant average launch times in ms if with_times)."""
        nl = max(self.L - 1, 1)
        out = (C.c_int * (2 * nl))()
        tm = (C.c_float * (2 * nl * STK_ASM_VARIANTS))()
        _check(load().stk_autotune(self._h, int(reps), out, tm, _stream()))
        res, times = {}, {}
        for l in range(1, self.L):
            for dt, name in ((0, "f64"), (1, "f32")):
                v = out[(l - 1) * 2 + dt]
                if v >= 0:
                    res[(l, name)] = v
                    k = ((l - 1) * 2 + dt) * STK_ASM_VARIANTS
                    times[(l, name)] = [tm[k + i] for i in range(STK_ASM_VARIANTS)]
        return (res, times) if with_times else res

    def level_cells(self, level: int) -> int:
        """Cells per axis of a level (level L-1 is the finest)."""
        return int(self.desc.n_fine) >> (self.L - 1 - int(level))

    def apply_asm_tuning(self, table) -> dict:
        """Apply a recorded choice {(dim, cells per axis, "f64"|"f32"): variant}
        to every level it covers; returns {(level, dtype): variant} applied."""
        applied = {}
        for l in range(1, self.L):
            for name in ("f64", "f32"):
                if name == "f32" and not self.desc.mixed:
                    continue
                v = table.get((int(self.dim), self.level_cells(l), name))
                if v is not None:
                    self.stk_set_asm_variant(l, v, name)
                    applied[(l, name)] = v
        return applied

    def stk_set_asm_variant(self, level: int, variant: int, dtype=None):
        import torch
        dt = STK_F32 if dtype in (torch.float32, "f32") else STK_F64
        _check(load().stk_set_asm_variant(self._h, int(level), dt, int(variant)))

    def stk_profile(self, enable, reps: int = 1):
        """Start (enable) or stop kernel timing; each instrumented launch is
        repeated `reps` times inside its event bracket."""
        _check(load().stk_profile(self._h, int(reps) if enable else 0))

    def stk_profile_read(self, kernel: int):
        n, ms, by = C.c_int64(), C.c_double(), C.c_double()
        _check(load().stk_profile_read(self._h, kernel, C.byref(n), C.byref(ms), C.byref(by)))
        return n.value, ms.value, by.value

    def stk_solve(self, bu, bp=None, rtol=1e-8, restart=30, maxit=300, xu=None, xp=None, allow_notconv=False,
                  eager=False, mixed=False, pc="full", cycle="V", allow=()):
        xu = self.zeros_u() if xu is None else xu
        xp = self.zeros_p() if xp is None else xp
        opts = SolveOpts(rtol, restart, maxit, 1 if eager else 0, 1 if mixed else 0, _PC[pc], _CYCLE[cycle])
        info = SolveInfo()
        st = load().stk_solve(self._h, _ptr(bu), _ptr(bp) if bp is not None else None, _ptr(xu), _ptr(xp),
                              C.byref(opts), C.byref(info), _stream())
        _check(st, allow=((STK_ENOTCONV,) if allow_notconv else ()) + tuple(allow))
        out = dict(iters=info.iters, converged=bool(info.converged), rel_res=info.rel_res,
                   t_solve=info.t_solve_s, hist=list(info.hist[:info.iters + 1]), status=st)
        return xu, xp, out
