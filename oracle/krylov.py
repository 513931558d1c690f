"""Outer FGMRES with the augmented-Lagrangian block preconditioner (oracle).

Test infrastructure: see package docstring.

Block preconditioner (Section 2, eq. (precond)), applied to the augmented
system of eq. (augstokessys):
    P = [I, -Ahat^{-1} B^T; 0, I] diag(Ahat^{-1}, -Shat^{-1}) [I, 0; -B Ahat^{-1}, I]
with Ahat^{-1} one multigrid V-cycle on A_gamma and, for preconditioner P1 of
eq. (P1P2), Shat_gamma^{-1} = M_p(1/mu)^{-1} + gamma M_p^{-1} (P2:
(1 + gamma) M_p(1/mu)^{-1}), both assembled and inverted cell by cell
(Section 5.1). Applied to (v_u, v_p) the three factors give
    y   = Ahat^{-1} v_u
    z_p = -Shat^{-1} (v_p - B y),   then the constant mode of z_p removed
    z_u = y - Ahat^{-1} B^T z_p.
Reading taken: the full factorisation as printed (two V-cycles per
application); the zero-mean projection after each Schur application keeps the
pressure in L^2_0 (the constant pressure is the kernel of B^T).

FGMRES (Section 5.1: "flexible Krylov solver FGMRES"): right preconditioned,
x0 = 0, restart m, Arnoldi by classical Gram-Schmidt applied twice, Givens
rotations; stop when the Arnoldi residual estimate |g_{j+1}| <= rtol ||b||_2,
then confirm with the true residual ||b - K x||_2 and restart if it is not
below the threshold. The paper stops at a 1e6 reduction; the workloads here
use rtol = 1e-8.
"""
from __future__ import annotations

import time

import numpy as np

from .multigrid import Multigrid


class BlockPreconditioner:
    """Eq. (precond): P = [I, -Ahat^{-1}B^T; 0, I] diag(Ahat^{-1}, -Shat^{-1})
    [I, 0; -B Ahat^{-1}, I] (kind "full", two V-cycles per application), or
    its block upper-triangular part P = [Ahat, B^T; 0, -Shat]^{-1} (kind
    "upper", one V-cycle; the block-triangular family the paper's
    introduction cites), with Ahat^{-1} = one V-cycle."""

    def __init__(self, mg: Multigrid, kind: str = "full", cycle: str = "V"):
        assert kind in ("full", "upper") and cycle in ("V", "F")
        self.mg = mg
        self.kind = kind
        self.ops = mg.ops[-1]
        self.nu = self.ops.level.n_u
        # Ahat^{-1}: one V-cycle, or one F-cycle (the paper's cycle)
        self.ahat_inv = mg.vcycle if cycle == "V" else mg.fcycle

    def apply(self, v: np.ndarray) -> np.ndarray:
        ops = self.ops
        vu, vp = v[:self.nu], v[self.nu:]
        if self.kind == "upper":
            zp = ops.project_mean(-(ops.Shat_inv @ vp))
            zu = self.ahat_inv(vu - ops.B.T @ zp)
            return np.concatenate([zu, zp])
        y = self.ahat_inv(vu)
        zp = -(ops.Shat_inv @ (vp - ops.B @ y))
        zp = ops.project_mean(zp)
        zu = y - self.ahat_inv(ops.B.T @ zp)
        return np.concatenate([zu, zp])


def _givens(a: float, b: float):
    """Rotation (c, s) with [c s; -s c] [a; b] = [r; 0]."""
    if b == 0.0:
        return 1.0, 0.0
    r = np.hypot(a, b)
    return a / r, b / r


def fgmres(K, M, b: np.ndarray, rtol: float = 1e-8, restart: int = 30, maxit: int = 300):
    """Right-preconditioned flexible GMRES for K x = b.

    K, M are callables (matrix apply, preconditioner apply). Returns (x, info)
    with info = dict(iters, converged, rel_res, hist) where hist[i] is the
    Arnoldi residual estimate after i iterations relative to ||b||."""
    n = b.size
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    hist = [1.0]
    if bnorm == 0.0:
        return x, dict(iters=0, converged=True, rel_res=0.0, hist=hist)
    r = b.copy()
    beta = bnorm
    it = 0
    converged = False
    while True:
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs, sn = [], []
        g = np.zeros(restart + 1)
        g[0] = beta
        j_used = 0
        for j in range(restart):
            z = M(V[j])
            Z.append(z)
            w = K(z)
            for _ in range(2):
                h = np.array([v @ w for v in V])
                w = w - sum(hi * v for hi, v in zip(h, V))
                H[:j + 1, j] += h
            H[j + 1, j] = np.linalg.norm(w)
            V.append(w / H[j + 1, j] if H[j + 1, j] != 0.0 else np.zeros(n))
            for i in range(j):
                a, c = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * c
                H[i + 1, j] = -sn[i] * a + cs[i] * c
            c, s = _givens(H[j, j], H[j + 1, j])
            cs.append(c); sn.append(s)
            H[j, j] = c * H[j, j] + s * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -s * g[j]
            g[j] = c * g[j]
            it += 1
            j_used = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= rtol * bnorm or it >= maxit:
                break
        k = j_used
        y = np.zeros(k)
        for i in reversed(range(k)):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + sum(yi * zi for yi, zi in zip(y, Z))
        r = b - K(x)
        beta = np.linalg.norm(r)
        if beta <= rtol * bnorm:
            converged = True
            break
        if it >= maxit:
            break
    return x, dict(iters=it, converged=converged, rel_res=beta / bnorm, hist=hist)


class StokesSolver:
    """Everything for one workload: hierarchy, operators, preconditioner, FGMRES."""

    def __init__(self, wl, schur: int = None, robust: bool = True, coef=None):
        if schur is None:
            schur = getattr(wl, "schur", 1)
        from .coefficients import SinkerField, ViscoplasticNewton
        from .fem import Level
        self.wl = wl
        if coef is None:
            if wl.coef_kind == 0:
                coef = SinkerField.from_workload(wl)
            else:
                coef = ViscoplasticNewton.from_workload(
                    wl, Level(wl.dim, wl.n_fine, getattr(wl, "degree", 2)).quad_points())
        self.coef = coef
        t0 = time.perf_counter()
        self.mg = Multigrid(wl.dim, wl.n_fine, wl.levels, coef, wl.gamma, wl.nu_pre, wl.nu_post,
                            schur=schur, robust=robust, k=getattr(wl, "degree", 2))
        self.ops = self.mg.ops[-1]
        self.K = self.ops.stokes(augmented=True)
        self.pc = BlockPreconditioner(self.mg)
        self.t_setup = time.perf_counter() - t0

    def rhs(self) -> np.ndarray:
        return np.concatenate([self.ops.rhs(), np.zeros(self.ops.level.n_p)])

    def solve(self, b=None, rtol=None, maxit=None, pc: str = "full", cycle: str = None):
        wl = self.wl
        if b is None:
            b = self.rhs()
        if cycle is None:
            cycle = getattr(wl, "cycle", "V")
        t0 = time.perf_counter()
        apply = self.pc.apply if (pc == "full" and cycle == "V") else BlockPreconditioner(self.mg, pc, cycle).apply
        x, info = fgmres(lambda v: self.K @ v, apply, b,
                         rtol=wl.rtol if rtol is None else rtol, restart=wl.restart,
                         maxit=wl.maxit if maxit is None else maxit)
        nu = self.ops.level.n_u
        x[nu:] = self.ops.project_mean(x[nu:])
        info["t_solve"] = time.perf_counter() - t0
        return x, info
