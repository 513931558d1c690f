"""Robust geometric multigrid for A_gamma (oracle). Test infrastructure: see package docstring.

* Smoother (Section 4.1): parallel subspace correction
      D^{-1} r = sum_i I_i A_i^{-1} I_i^* r
  over the vertex-star decomposition of eq. (viim): V_i holds the velocity
  fields supported in star(v_i), i.e. the unknowns at nodes strictly inside
  the union of the cells around vertex v_i, for every vertex of the level
  (boundary vertices included). As in Section 5.1, each A_i is extracted from
  the globally assembled A_gamma and factored by dense LU.
  Relaxation (Section 5.1 and the algorithm outline): a fixed number nu of
  GMRES steps preconditioned by D^{-1}. Reading taken (the paper gives neither
  the side of preconditioning nor a damping): right preconditioning, exactly
  nu Arnoldi steps with classical Gram-Schmidt applied twice, no damping, the
  small least-squares problem solved exactly.
* Prolongation (Section 4.2, eq. (Ptilde)): P~ u_H = P_H u_H - u~_h, where u~_h
  solves a_{h,gamma}(u~_h, v) = gamma (Pi div P_H u_H, Pi div v) for all v
  supported inside one coarse cell. Reading taken for the garbled right-hand
  side: the divergence is applied to P_H u_H, so that the right-hand side is
  (G_h P_H u_H) restricted to those unknowns with G_h = gamma B^T W^{-1} B.
  Each coarse cell gives an independent local problem on the fine unknowns
  strictly inside it, extracted from the assembled fine A_gamma and solved
  exactly (Section 5.1).
* Restriction: the transpose of P~ (the paper does not state it; the
  transpose keeps the V-cycle symmetric in structure).
* Coarse level: sparse direct LU of A_gamma (the paper uses MUMPS).
* Cycles. V-cycle: pre-smooth (from zero, or from a given iterate),
  residual, restrict, recurse from zero, prolongate and add, post-smooth.
  F-cycle, the paper's "full" multigrid cycle (Section 5.1 and the algorithm
  outline); reading taken: the full multigrid cycle of PETSc, which the
  paper's Firedrake solver uses: the right-hand side is restricted to every
  coarser level, the coarsest level is solved directly, and going up, each
  level's start is the prolongated coarser result, improved by one V-cycle.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import Level, Hierarchy, lagrange_1d, unlex, lex
from .assembly import Operators


# --------------------------------------------------------------------------- patches
def star_patch_dofs(level: Level, vertex) -> np.ndarray:
    """Unknowns strictly inside star(vertex): per axis the nodes kv-(k-1) ..
    kv+(k-1) that are interior to the domain, all components; sorted
    ascending ((2k-1)^d nodes at an interior vertex)."""
    d, k = level.dim, level.k
    ranges = []
    for a in range(d):
        v = int(vertex[a])
        ranges.append([i for i in range(k * v - (k - 1), k * v + k) if 1 <= i <= k * level.n - 1])
    nodes = np.array(list(itertools.product(*ranges)), dtype=np.int64)
    if nodes.size == 0:
        return np.zeros(0, dtype=np.int64)
    dofs = np.concatenate([level.u_dof(c, nodes) for c in range(d)])
    return np.sort(dofs)


def all_vertices(level: Level) -> np.ndarray:
    return unlex(np.arange((level.n + 1) ** level.dim), level.n + 1, level.dim)


def coarse_cell_dofs(fine: Level, coarse_cell) -> np.ndarray:
    """Fine unknowns strictly inside a coarse cell (fine nodes 2kc+1 .. 2kc+2k-1
    per axis)."""
    d, k = fine.dim, fine.k
    ranges = [range(2 * k * int(c) + 1, 2 * k * int(c) + 2 * k) for c in coarse_cell]
    nodes = np.array(list(itertools.product(*ranges)), dtype=np.int64)
    dofs = np.concatenate([fine.u_dof(c, nodes) for c in range(d)])
    return np.sort(dofs)


def extract_dense(M: sp.csr_matrix, idx: np.ndarray) -> np.ndarray:
    return M[idx][:, idx].toarray()


class StarASM:
    """D^{-1} = sum_i I_i A_i^{-1} I_i^*, A_i extracted from the assembled matrix, dense LU."""

    def __init__(self, level: Level, Agamma: sp.csr_matrix):
        self.level = level
        self.patches = []
        self.lus = []
        for v in all_vertices(level):
            idx = star_patch_dofs(level, v)
            if idx.size == 0:
                continue
            self.patches.append(idx)
            self.lus.append(sla.lu_factor(extract_dense(Agamma, idx), check_finite=False))

    def apply(self, r: np.ndarray) -> np.ndarray:
        y = np.zeros_like(r)
        for idx, lu in zip(self.patches, self.lus):
            y[idx] += sla.lu_solve(lu, r[idx], check_finite=False)
        return y


# --------------------------------------------------------------------------- transfers
def standard_prolongation(coarse: Level, fine: Level) -> sp.csr_matrix:
    """P_H: coarse Q_k field evaluated at the fine nodes (nested spaces)."""
    d, kk = coarse.dim, coarse.k
    assert fine.n == 2 * coarse.n and fine.k == kk
    fnodes = unlex(np.arange(fine.n_int_nodes), fine.ni, d) + 1      # fine node indices
    # position in coarse-cell units: fine node i sits at i/(2k) coarse cells,
    # in cell floor(i/(2k)) at the local coordinate (i - 2k cell)/(2k), formed
    # from the integer offset so that it is correctly rounded
    cell = np.minimum(fnodes // (2 * kk), coarse.n - 1)
    xi = (fnodes - 2 * kk * cell) / (2.0 * kk)
    val, _ = lagrange_1d(xi, kk)                                      # (nf, d, k+1)
    rows, cols, vals = [], [], []
    for loc in itertools.product(range(kk + 1), repeat=d):
        w = np.ones(len(fnodes))
        for k in range(d):
            w = w * val[:, k, loc[k]]
        cnode = kk * cell + np.array(loc)[None, :]
        for c in range(d):
            cd = coarse.u_dof(c, cnode)
            fd = c * fine.n_int_nodes + np.arange(fine.n_int_nodes)
            keep = (cd >= 0) & (w != 0.0)
            rows.append(fd[keep]); cols.append(cd[keep]); vals.append(w[keep])
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(fine.n_u, coarse.n_u)).tocsr()


class RobustTransfer:
    """P~ = P_H - sum_K E_K^T A_K^{-1} E_K G_h P_H and R = P~^T."""

    def __init__(self, coarse: Level, fine: Level, fine_ops: Operators):
        self.P = standard_prolongation(coarse, fine)
        self.G = fine_ops.G
        self.GT = fine_ops.G.T.tocsr()
        self.blocks, self.lus = [], []
        for cc in unlex(np.arange(coarse.n_cells), coarse.n, coarse.dim):
            idx = coarse_cell_dofs(fine, cc)
            self.blocks.append(idx)
            self.lus.append(sla.lu_factor(extract_dense(fine_ops.Agamma, idx), check_finite=False))

    def local_correction(self, g: np.ndarray, trans: int = 0) -> np.ndarray:
        s = np.zeros_like(g)
        for idx, lu in zip(self.blocks, self.lus):
            s[idx] = sla.lu_solve(lu, g[idx], trans=trans, check_finite=False)
        return s

    def prolong(self, xc: np.ndarray) -> np.ndarray:
        t = self.P @ xc
        return t - self.local_correction(self.G @ t)

    def restrict(self, r: np.ndarray) -> np.ndarray:
        s = self.local_correction(r, trans=1)
        return self.P.T @ (r - self.GT @ s)

    def standard_restrict(self, r):
        return self.P.T @ r


# --------------------------------------------------------------------------- relaxation
def gmres_relax(A, Dinv, b: np.ndarray, x0, nu: int) -> np.ndarray:
    """nu steps of GMRES on A x = b, right-preconditioned by Dinv, from x0.

    Minimises the true residual ||b - A x||_2 over x0 + Dinv K_nu(A Dinv, r0),
    r0 = b - A x0; Arnoldi with classical Gram-Schmidt applied twice; stops
    early only on an exact breakdown (zero new Arnoldi vector).

    Reading taken: right preconditioning. Left preconditioning (minimising
    ||Dinv r||) loses the gamma-robustness the paper reports: at gamma = 1e4
    the V-cycle preconditioned solve stagnates, while right preconditioning
    keeps the iteration count flat in gamma (measured on 2D 8x8 to 16x16
    sinker problems)."""
    if x0 is None:
        x0 = np.zeros_like(b)
        r = b.copy()
    else:
        r = b - A @ x0
    beta = np.linalg.norm(r)
    if beta == 0.0:
        return x0.copy()
    V = [r / beta]
    Z = []
    H = np.zeros((nu + 1, nu))
    k = nu
    for j in range(nu):
        Z.append(Dinv(V[j]))
        w = A @ Z[j]
        for _ in range(2):
            h = np.array([v @ w for v in V])
            w = w - sum(hi * v for hi, v in zip(h, V))
            H[:j + 1, j] += h
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] == 0.0:
            k = j + 1
            break
        V.append(w / H[j + 1, j])
    e1 = np.zeros(k + 1)
    e1[0] = beta
    y, *_ = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)
    return x0 + sum(yi * z for yi, z in zip(y, Z[:k]))


# --------------------------------------------------------------------------- hierarchy
class Multigrid:
    """Rediscretised hierarchy with star-ASM relaxation and robust transfers."""

    def __init__(self, dim: int, n_fine: int, n_levels: int, coef, gamma: float,
                 nu_pre: int = 2, nu_post: int = 2, schur: int = 1, robust: bool = True, k: int = 2):
        self.hier = Hierarchy(dim, n_fine, n_levels, k)
        self.nu_pre, self.nu_post = nu_pre, nu_post
        self.ops = [Operators(lv, coef, gamma, schur) for lv in self.hier.levels]
        self.robust = robust
        self.smoothers = [None] + [StarASM(self.hier[l], self.ops[l].Agamma)
                                   for l in range(1, n_levels)]
        self.transfers = [None] + [RobustTransfer(self.hier[l - 1], self.hier[l], self.ops[l])
                                   for l in range(1, n_levels)]
        self.coarse_lu = spla.splu(self.ops[0].Agamma.tocsc())

    @property
    def L(self):
        return len(self.hier)

    def smooth(self, l: int, b: np.ndarray, x0, nu: int) -> np.ndarray:
        return gmres_relax(self.ops[l].Agamma, self.smoothers[l].apply, b, x0, nu)

    def prolong(self, l: int, xc):
        """Coarse level l-1 -> fine level l."""
        T = self.transfers[l]
        return T.prolong(xc) if self.robust else T.P @ xc

    def restrict(self, l: int, r):
        """Fine level l -> coarse level l-1."""
        T = self.transfers[l]
        return T.restrict(r) if self.robust else T.P.T @ r

    def vcycle(self, b: np.ndarray, l: int | None = None, x0=None) -> np.ndarray:
        """One V-cycle on level l (default: finest) from x0 (default: zero)."""
        if l is None:
            l = self.L - 1
        if l == 0:
            return self.coarse_lu.solve(b)
        x = self.smooth(l, b, x0, self.nu_pre)
        r = b - self.ops[l].Agamma @ x
        xc = self.vcycle(self.restrict(l, r), l - 1)
        x = x + self.prolong(l, xc)
        return self.smooth(l, b, x, self.nu_post)

    def fcycle(self, b: np.ndarray) -> np.ndarray:
        """One F-cycle (full multigrid cycle) on the finest level."""
        L = self.L
        rhs = [None] * L
        rhs[L - 1] = b
        for l in range(L - 1, 0, -1):
            rhs[l - 1] = self.restrict(l, rhs[l])
        x = self.coarse_lu.solve(rhs[0])
        for l in range(1, L):
            x = self.vcycle(rhs[l], l, x0=self.prolong(l, x))
        return x

    def cycle(self, b: np.ndarray, kind: str = "V") -> np.ndarray:
        return self.fcycle(b) if kind == "F" else self.vcycle(b)
