"""Assembled sparse operators of the (augmented) Stokes system (oracle).

Test infrastructure: see package docstring.

Entries (Section 2, eq. (stokessys) and the definitions following it):
    [A]_ij   = (2 mu eps(phi_j), eps(phi_i))       (tensor case: (C:eps(phi_j), eps(phi_i)))
    [B]_mj   = -(psi_m, div phi_j)
    [M_p(w)]_mn = (w psi_m, psi_n)                   (eq. (inv-visc-mass) with w = 1/mu)
Augmented block (Section 3, eq. (augstokessys)):
    A_gamma = A + gamma B^T W^{-1} B,   W = M_p (preconditioner P1) or M_p(1/mu) (P2).
Right-hand side: (f, phi_i) for the velocity and 0 for the pressure (r_2 = 0,
so the augmented right-hand side equals the original one).

All integrals use the tensor (k+1)-point Gauss rule on every cell (the paper
does not state its rule; this rule is exact for the constant-coefficient Q_k
stiffness on affine cells and it defines the discrete problem otherwise).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import Level, reference_tables, pressure_basis


def basis_strain(level: Level):
    """Strain eps(phi_i) of every local vector basis function at every
    reference quadrature point: array [q, i, a, b], i = comp * (k+1)^d + node,
    physical units (reference gradient / h)."""
    d = level.dim
    xi, w, phi, dphi = reference_tables(d, level.k)
    nq, nn = phi.shape
    grad = np.zeros((nq, d * nn, d, d))
    for c in range(d):
        grad[:, c * nn:(c + 1) * nn, c, :] = dphi / level.h     # d(phi)_c / dx_b
    return 0.5 * (grad + np.swapaxes(grad, -1, -2)), grad


def element_viscous(level: Level, coef, cells=None) -> np.ndarray:
    """Element matrices (n_cells, nl, nl) of a(u, v) = (sigma(u), eps(v));
    only those of `cells` (an index array) if given."""
    d = level.dim
    xi, w, phi, dphi = reference_tables(d, level.k)
    eps, _ = basis_strain(level)
    nq, nl = eps.shape[0], eps.shape[1]
    vol = level.h ** d
    x = level.quad_points()
    if cells is not None:
        x = x[cells]
    E = eps.reshape(nq, nl, d * d)
    if coef.kind == "scalar":
        mu = coef.mu(x)                                            # (nc, nq)
        # per quadrature point the matrix eps_i : eps_j, weighted by 2 mu w |K|
        P = np.einsum("qix,qjx->qij", E, E).reshape(nq, nl * nl)
        Ae = (2.0 * mu * (w * vol)[None, :]) @ P
        return Ae.reshape(-1, nl, nl)
    C = coef.stress_tensor(x).reshape(x.shape[0], nq, d * d, d * d)
    Ae = np.zeros((x.shape[0], nl, nl))
    for q in range(nq):
        CE = np.einsum("kxy,jy->kxj", C[:, q], E[q])              # C : eps_j
        Ae += (w[q] * vol) * np.einsum("ix,kxj->kij", E[q], CE)
    return Ae


def element_divergence(level: Level) -> np.ndarray:
    """Be[m, j] = -(psi_m, div phi_j) on one cell (identical on all cells)."""
    d = level.dim
    xi, w, phi, dphi = reference_tables(d, level.k)
    _, grad = basis_strain(level)
    div = np.trace(grad, axis1=-2, axis2=-1)                      # (nq, nl)
    psi = pressure_basis(xi, level.k)                             # (nq, n_pb)
    return -np.einsum("q,qm,qj->mj", w * level.h ** d, psi, div)


def element_pressure_mass(level: Level, weight=None) -> np.ndarray:
    """(w psi_m, psi_n) on every cell: (n_cells, n_pb, n_pb); weight(x) optional."""
    d = level.dim
    xi, w, phi, dphi = reference_tables(d, level.k)
    psi = pressure_basis(xi, level.k)
    vol = level.h ** d
    if weight is None:
        wq = np.ones((level.n_cells, len(w)))
    else:
        wq = weight(level.quad_points())
    return np.einsum("kq,q,qm,qn->kmn", wq, w * vol, psi, psi)


def _assemble(rows_e, cols_e, vals_e, shape):
    r = np.broadcast_to(rows_e, vals_e.shape).ravel()
    c = np.broadcast_to(cols_e, vals_e.shape).ravel()
    v = vals_e.ravel()
    keep = (r >= 0) & (c >= 0)
    return sp.coo_matrix((v[keep], (r[keep], c[keep])), shape=shape).tocsr()


def pressure_dofs(level: Level) -> np.ndarray:
    return np.arange(level.n_p).reshape(level.n_cells, level.n_pb)


class Operators:
    """All assembled matrices of one level."""

    def __init__(self, level: Level, coef, gamma: float, schur: int = 1):
        self.level, self.coef, self.gamma, self.schur = level, coef, float(gamma), schur
        d = level.dim
        ed = level.element_dofs()                                   # (nc, nl)
        pd = pressure_dofs(level)                                   # (nc, n_pb)
        Ae = element_viscous(level, coef)
        self.A = _assemble(ed[:, :, None], ed[:, None, :], Ae, (level.n_u, level.n_u))
        Be = np.broadcast_to(element_divergence(level), (level.n_cells,) + (level.n_pb, ed.shape[1]))
        self.B = _assemble(pd[:, :, None], ed[:, None, :], Be, (level.n_p, level.n_u))
        Me = element_pressure_mass(level)
        Mmu = element_pressure_mass(level, lambda x: 1.0 / coef.scalar_viscosity(x))
        self.Mp = _assemble(pd[:, :, None], pd[:, None, :], Me, (level.n_p, level.n_p))
        self.Mp_invmu = _assemble(pd[:, :, None], pd[:, None, :], Mmu, (level.n_p, level.n_p))
        We = Me if schur == 1 else Mmu                              # W in A_gamma
        self.Winv = _assemble(pd[:, :, None], pd[:, None, :], np.linalg.inv(We),
                              (level.n_p, level.n_p))
        self.G = (self.gamma * (self.B.T @ self.Winv @ self.B)).tocsr()
        self.Agamma = (self.A + self.G).tocsr()
        # Schur approximation of eq. (P1P2), assembled and inverted cellwise
        if schur == 1:
            Sinv = np.linalg.inv(Mmu) + self.gamma * np.linalg.inv(Me)
        else:
            Sinv = (1.0 + self.gamma) * np.linalg.inv(Mmu)
        self.Shat_inv = _assemble(pd[:, :, None], pd[:, None, :], Sinv, (level.n_p, level.n_p))
        # one-vector of the pressure constants: m = M_p 1 (used for int p = 0)
        ones = np.zeros(level.n_p)
        ones[pd[:, 0]] = 1.0
        self.p_const = ones
        self.p_mass_const = self.Mp @ ones

    def stokes(self, augmented: bool = True):
        """K = [[A_gamma, B^T], [B, 0]] (or the unaugmented A)."""
        Auu = self.Agamma if augmented else self.A
        return sp.bmat([[Auu, self.B.T], [self.B, None]], format="csr")

    def rhs(self) -> np.ndarray:
        """Velocity right-hand side (f, phi_i)."""
        level = self.level
        d = level.dim
        xi, w, phi, dphi = reference_tables(d, level.k)
        x = level.quad_points()
        f = self.coef_force(x)                                      # (nc, nq, d)
        vol = level.h ** d
        # element vector: local i = c * nn + n
        be = np.einsum("q,kqc,qn->kcn", w * vol, f, phi).reshape(level.n_cells, -1)
        ed = level.element_dofs()
        b = np.zeros(level.n_u)
        keep = ed >= 0
        np.add.at(b, ed[keep], be[keep])
        return b

    def coef_force(self, x):
        base = self.coef if self.coef.kind == "scalar" else self.coef.base
        return base.force(x)

    def project_mean(self, p: np.ndarray) -> np.ndarray:
        """Remove the constant-pressure component so that int p = 0 (Q_h in L^2_0)."""
        m = self.p_mass_const
        return p - (m @ p) / (m @ self.p_const) * self.p_const


def stokes_rows(level: Level, coef, gamma: float, u: np.ndarray, p: np.ndarray, vel_rows, pres_cells):
    """Selected entries of K [u; p], K = [[A_gamma, B^T], [B, 0]] (W = M_p),
    summed from the element matrices of only the cells those entries touch:
    the same entries as the assembled operators of `Operators`, for spot
    checks on meshes too large to assemble. Returns (velocity entries at
    `vel_rows`, pressure entries of the cells `pres_cells` as (len, n_pb))."""
    vel_rows = np.asarray(vel_rows)
    pres_cells = np.asarray(pres_cells)
    ed = level.element_dofs()
    pd = pressure_dofs(level)
    cells = np.unique(np.concatenate([np.nonzero(np.isin(ed, vel_rows).any(axis=1))[0], pres_cells]))
    Ae = element_viscous(level, coef, cells)
    Be = element_divergence(level)
    Winv = np.linalg.inv(element_pressure_mass(level)[0])
    Ke = Ae + gamma * (Be.T @ Winv @ Be)[None]
    ue = np.where(ed[cells] >= 0, u[np.maximum(ed[cells], 0)], 0.0)
    pe = p[pd[cells]]
    ye = np.einsum("kij,kj->ki", Ke, ue) + pe @ Be
    yv = np.zeros(len(vel_rows))
    pos = {int(r): i for i, r in enumerate(vel_rows)}
    for k in range(len(cells)):
        for loc, dof in enumerate(ed[cells[k]]):
            i = pos.get(int(dof))
            if i is not None:
                yv[i] += ye[k, loc]
    where = {int(c): k for k, c in enumerate(cells)}
    yp = np.array([Be @ ue[where[int(c)]] for c in pres_cells]).reshape(len(pres_cells), -1)
    return yv, yp


def rhs_rows(level: Level, coef, vel_rows) -> np.ndarray:
    """Selected entries of the velocity right-hand side (f, phi_i), from the
    cells that touch them (same element loads as `Operators.rhs`)."""
    vel_rows = np.asarray(vel_rows)
    d = level.dim
    xi, w, phi, dphi = reference_tables(d, level.k)
    ed = level.element_dofs()
    cells = np.nonzero(np.isin(ed, vel_rows).any(axis=1))[0]
    base = coef if coef.kind == "scalar" else coef.base
    f = base.force(level.quad_points()[cells])
    be = np.einsum("q,kqc,qn->kcn", w * level.h ** d, f, phi).reshape(len(cells), -1)
    out = np.zeros(len(vel_rows))
    pos = {int(r): i for i, r in enumerate(vel_rows)}
    for k in range(len(cells)):
        for loc, dof in enumerate(ed[cells[k]]):
            i = pos.get(int(dof))
            if i is not None:
                out[i] += be[k, loc]
    return out
