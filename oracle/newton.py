"""Newton's method for viscoplastic Stokes flow (oracle). Test infrastructure:
see the package docstring.

Nonlinear problem (Section 5.3.1, with the reading of coefficients.py: the
capped law over the multi-sinker base field mu0, floor mu_f, yield stress
tau_y; homogeneous Dirichlet walls, the multi-sinker forcing): find (u, p) with
    F_u(u, p) = a(u; u) + gamma B^T W^{-1} B u + B^T p - b = 0,
    F_p(u)    = B u = 0,
    a(w; v)   = (2 mu_eff(eps_II(w)) eps(w), eps(v)),
    mu_eff    = mu_f + min(mu0 - mu_f, tau_y / (2 eps_II)).
The augmented term vanishes wherever B u = 0, so the solutions are those of
the unaugmented problem (Section 3). Its Jacobian at (u_k, p_k) is the
augmented Stokes operator of eq. (augstokessys) with the fourth-order
viscosity C = d tau / d eps at eps(u_k) (coefficients.capped_law), so each
Newton step is one solve of the linear system the paper's solver targets:
FGMRES with the augmented-Lagrangian block preconditioner, its multigrid
rediscretised on every level.

Readings taken (the paper gives the structure, not these details):
  * standard Newton: the paper uses a stress-velocity variant whose update
    formula is in another reference, and notes that the standard
    linearisation differs only in using eps(u_{k-1}) where the stress
    variable appears;
  * the coarse-level linearisations use the velocity injected to the coarse
    nodes (nested Q2 spaces: coarse node i is fine node 2i);
  * line search: backtracking alpha = 1, 1/2, ... until the residual norm
    decreases sufficiently, ||F(x + alpha d)|| <= (1 - 1e-4 alpha) ||F(x)||,
    at most `max_halvings` halvings (the last step is taken regardless);
  * stop when ||F|| <= rtol ||F(x_0)|| (the paper: a 1e8 reduction), start
    from x_0 = 0 (whose linearisation is the Newtonian problem with mu0);
  * linear solves to a relative residual lin_rtol (the paper: 1e6 reduction).
"""
from __future__ import annotations

import numpy as np

from .assembly import basis_strain, Operators
from .coefficients import SinkerField, capped_law
from .fem import Level, Hierarchy, reference_tables


def fe_strain(level: Level, u: np.ndarray) -> np.ndarray:
    """Strain rate eps(u)[cell, q, a, b] of the FE velocity u (interior
    unknowns) at the level's Gauss points."""
    eps_b, _ = basis_strain(level)                                 # [q, i, a, b]
    ed = level.element_dofs()
    ue = np.where(ed >= 0, u[np.maximum(ed, 0)], 0.0)              # (nc, nl)
    return np.einsum("qiab,ki->kqab", eps_b, ue)


def inject(fine: Level, coarse: Level, u: np.ndarray) -> np.ndarray:
    """Coarse interior unknowns taken from the fine unknowns at the same
    nodes (coarse node i is fine node 2i)."""
    d = coarse.dim
    from .fem import unlex
    cn = unlex(np.arange(coarse.n_int_nodes), coarse.ni, d) + 1
    out = np.zeros(coarse.n_u)
    for c in range(d):
        out[c * coarse.n_int_nodes + np.arange(coarse.n_int_nodes)] = u[fine.u_dof(c, 2 * cn)]
    return out


class ViscoplasticFE:
    """The capped law's coefficients at an FE velocity, per level: the
    viscosity and tensor at the Gauss points of a level (identified by its
    cell count) come from the strain rate of the velocity injected there."""

    kind = "tensor"

    def __init__(self, base: SinkerField, tau_y: float, mu_floor: float, hier: Hierarchy, u_fine: np.ndarray):
        self.base, self.tau_y = base, float(tau_y)
        self.dim = base.dim
        self.mu_min = float(mu_floor) if mu_floor > 0.0 else base.mu_min
        self.eps = {}
        u = u_fine
        for l in range(len(hier) - 1, -1, -1):
            lv = hier[l]
            self.eps[lv.n_cells] = fe_strain(lv, u)
            if l > 0:
                u = inject(lv, hier[l - 1], u)

    def _state(self, x):
        eps = self.eps[x.shape[0]]
        assert eps.shape[:2] == x.shape[:2], "coefficients are defined at a level's Gauss points only"
        return capped_law(eps, self.base.mu(x), self.tau_y, self.mu_min)

    def mu_eff(self, x):
        return self._state(x)[0]

    def scalar_viscosity(self, x):
        return self.mu_eff(x)

    def stress_tensor(self, x):
        return self._state(x)[1]


def stress_form(level: Level, base: SinkerField, tau_y: float, mu_f: float, u: np.ndarray) -> np.ndarray:
    """a(u; v) for every velocity basis function v: the vector of
    (2 mu_eff(eps_II(u)) eps(u), eps(phi_i)) over the interior unknowns."""
    d = level.dim
    xi, w, phi, dphi = reference_tables(d)
    eps_b, _ = basis_strain(level)                                 # [q, i, a, b]
    eps = fe_strain(level, u)                                      # [k, q, a, b]
    mu_eff, _ = capped_law(eps, base.mu(level.quad_points()), tau_y, mu_f)
    tau = 2.0 * mu_eff[..., None, None] * eps
    be = np.einsum("q,kqab,qiab->ki", w * level.h ** d, tau, eps_b)
    ed = level.element_dofs()
    out = np.zeros(level.n_u)
    keep = ed >= 0
    np.add.at(out, ed[keep], be[keep])
    return out


class NewtonSolver:
    """Newton with backtracking line search; each step is solved by the
    oracle's FGMRES with the block preconditioner and robust multigrid."""

    def __init__(self, wl, tau_y: float, mu_floor: float = 0.0):
        from .krylov import StokesSolver
        assert getattr(wl, "degree", 2) == 2, "the Newton loop is built for [Q2]^d x P1disc"
        self.wl = wl
        self.base = SinkerField.from_workload(wl)
        self.tau_y = float(tau_y)
        self.mu_f = float(mu_floor) if mu_floor > 0.0 else self.base.mu_min
        self.hier = Hierarchy(wl.dim, wl.n_fine, wl.levels)
        self.fine = self.hier[-1]
        # W, B, the right-hand side and the mean projection do not depend on the state
        self.ops0 = Operators(self.fine, self.base, wl.gamma, getattr(wl, "schur", 1))
        self.b = self.ops0.rhs()
        self._solver_cls = StokesSolver

    def residual(self, u: np.ndarray, p: np.ndarray):
        """(F_u, F_p)."""
        ops = self.ops0
        Fu = stress_form(self.fine, self.base, self.tau_y, self.mu_f, u) + ops.G @ u + ops.B.T @ p - self.b
        return Fu, ops.B @ u

    def linearisation(self, u: np.ndarray):
        coef = ViscoplasticFE(self.base, self.tau_y, self.mu_f, self.hier, u)
        return self._solver_cls(self.wl, coef=coef)

    def solve(self, rtol=1e-8, maxit=30, lin_rtol=1e-6, max_halvings=10, cycle=None, pc="full"):
        nu, npr = self.fine.n_u, self.fine.n_p
        u, p = np.zeros(nu), np.zeros(npr)
        Fu, Fp = self.residual(u, p)
        fn = np.sqrt(Fu @ Fu + Fp @ Fp)
        f0 = fn
        hist, lin, alphas = [1.0], [], []
        converged = False
        for k in range(maxit):
            if fn <= rtol * f0:
                converged = True
                break
            S = self.linearisation(u)
            d, info = S.solve(b=-np.concatenate([Fu, Fp]), rtol=lin_rtol, pc=pc, cycle=cycle)
            lin.append(info["iters"])
            du, dp = d[:nu], d[nu:]
            alpha = 1.0
            for h in range(max_halvings + 1):
                ut, pt = u + alpha * du, p + alpha * dp
                Fut, Fpt = self.residual(ut, pt)
                ft = np.sqrt(Fut @ Fut + Fpt @ Fpt)
                if ft <= (1.0 - 1e-4 * alpha) * fn or h == max_halvings:
                    break
                alpha *= 0.5
            u, p, Fu, Fp, fn = ut, pt, Fut, Fpt, ft
            alphas.append(alpha)
            hist.append(fn / f0)
        else:
            converged = fn <= rtol * f0
        return u, p, dict(iters=len(lin), converged=converged, rel_res=fn / f0, hist=hist, lin_iters=lin,
                          alpha=alphas, res0=f0)
