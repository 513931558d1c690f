"""Structured [Q2]^d x P1disc discretisation on the unit square/cube (oracle).

Test infrastructure: see the package docstring.

Spaces (Section 4, definition of V_h^k and Q_h^{k-1}, k = 2):
  * velocity: continuous, piecewise tensor-product quadratic (Q2) in each of
    the d components, zero on the whole boundary (homogeneous Dirichlet,
    Section 2, eq. (stokes-linear));
  * pressure: discontinuous, total degree <= 1 on every cell (P1disc), with
    zero mean (Q_h subset of L^2_0).

Mesh: [0,1]^d split into N^d axis-aligned cells of width h = 1/N; uniform
refinement gives the multigrid levels (Section 5.1). On axis-aligned cells the
"mapped" and the physical P1 spaces coincide, so the pressure basis on cell K
with centre c_K is psi_0 = 1, psi_j = (x_j - c_{K,j}) / h (j = 1..d).

Index conventions (shared with nothing; the GPU library defines its own):
  * multi-indices are ordered (x, y[, z]) and flattened lexicographically with
    x fastest;
  * a Q2 cell with lower corner index (i, j[, k]) owns the full-grid nodes
    (2i + a, 2j + b[, 2k + c]), a, b, c in {0, 1, 2}; local node = a + 3b + 9c;
  * velocity unknowns are the interior nodes (all indices in 1..2N-1),
    numbered component-major: dof = comp * (2N-1)^d + lex(node - 1);
  * the "stored" layout is the full node grid, comp-major, x fastest, with
    zeros on Dirichlet nodes: index = comp * (2N+1)^d + lex(node).
  * pressure unknowns: dof = cell * (d + 1) + m, m = 0..d.
"""
from __future__ import annotations

import itertools
from functools import lru_cache

import numpy as np

Q1D = 3          # Gauss points per axis (exact for degree <= 5)
NODES_1D = np.array([0.0, 0.5, 1.0])


@lru_cache(maxsize=None)
def gauss_legendre_01(n: int = Q1D):
    """Gauss-Legendre points and weights mapped from [-1, 1] to [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_1d(xi: np.ndarray):
    """Values and derivatives of the three quadratic Lagrange polynomials on
    nodes {0, 1/2, 1} at points xi; returns (val[..., 3], der[..., 3]).

    Written from the Lagrange product formula l_a(x) = prod_{b != a}
    (x - x_b) / (x_a - x_b) and its product-rule derivative.
    """
    xi = np.asarray(xi, dtype=np.float64)
    val = np.ones(xi.shape + (3,))
    der = np.zeros(xi.shape + (3,))
    for a in range(3):
        others = [b for b in range(3) if b != a]
        den = np.prod([NODES_1D[a] - NODES_1D[b] for b in others])
        val[..., a] = np.prod([xi - NODES_1D[b] for b in others], axis=0) / den
        d = np.zeros(xi.shape)
        for skip in others:
            d = d + np.prod([xi - NODES_1D[b] for b in others if b != skip], axis=0)
        der[..., a] = d / den
    return val, der


@lru_cache(maxsize=None)
def reference_tables(dim: int):
    """Reference-cell tables at the tensor Gauss points.

    Returns (xi[q, dim], w[q], phi[q, n], dphi[q, n, dim]) with q and n
    flattened x-fastest; dphi is the gradient in reference coordinates
    (divide by h for the physical gradient).
    """
    g, gw = gauss_legendre_01(Q1D)
    val, der = lagrange_1d(g)          # [qpt, node]
    qs = list(itertools.product(range(Q1D), repeat=dim))
    ns = list(itertools.product(range(3), repeat=dim))
    # itertools.product varies the LAST index fastest; we want x (index 0) fastest
    qs = [tuple(reversed(t)) for t in qs]
    ns = [tuple(reversed(t)) for t in ns]
    nq, nn = len(qs), len(ns)
    xi = np.array([[g[t[k]] for k in range(dim)] for t in qs])
    w = np.array([np.prod([gw[t[k]] for k in range(dim)]) for t in qs])
    phi = np.zeros((nq, nn))
    dphi = np.zeros((nq, nn, dim))
    for iq, tq in enumerate(qs):
        for inn, tn in enumerate(ns):
            phi[iq, inn] = np.prod([val[tq[k], tn[k]] for k in range(dim)])
            for j in range(dim):
                dphi[iq, inn, j] = np.prod([der[tq[k], tn[k]] if k == j else val[tq[k], tn[k]]
                                            for k in range(dim)])
    return xi, w, phi, dphi


def pressure_basis(xi: np.ndarray) -> np.ndarray:
    """P1disc basis at reference points xi[..., dim]: [1, xi_1 - 1/2, ...]."""
    xi = np.asarray(xi)
    return np.concatenate([np.ones(xi.shape[:-1] + (1,)), xi - 0.5], axis=-1)


def lex(idx: np.ndarray, n: int) -> np.ndarray:
    """Lexicographic index (x fastest) of multi-indices idx[..., dim] in an n^dim box."""
    idx = np.asarray(idx)
    out = np.zeros(idx.shape[:-1], dtype=np.int64)
    for k in reversed(range(idx.shape[-1])):
        out = out * n + idx[..., k]
    return out


def unlex(i: np.ndarray, n: int, dim: int) -> np.ndarray:
    i = np.asarray(i, dtype=np.int64)
    out = np.zeros(i.shape + (dim,), dtype=np.int64)
    for k in range(dim):
        out[..., k] = i % n
        i = i // n
    return out


class Level:
    """One level of the uniformly refined hierarchy: N cells per axis."""

    def __init__(self, dim: int, n: int):
        assert dim in (2, 3) and n >= 1
        self.dim, self.n = dim, n
        self.h = 1.0 / n
        self.n1 = 2 * n + 1                    # nodes per axis
        self.ni = 2 * n - 1                    # interior nodes per axis
        self.n_nodes = self.n1 ** dim
        self.n_int_nodes = self.ni ** dim
        self.n_u = dim * self.n_int_nodes      # velocity unknowns
        self.n_cells = n ** dim
        self.n_p = (dim + 1) * self.n_cells    # pressure unknowns
        self.n_stored = dim * self.n_nodes

    # ---- node / dof numbering -------------------------------------------------
    def interior_node(self, node: np.ndarray) -> np.ndarray:
        """Interior lex index of full-grid nodes node[..., dim], or -1 on the boundary."""
        node = np.asarray(node)
        inside = np.all((node >= 1) & (node <= 2 * self.n - 1), axis=-1)
        out = lex(np.clip(node - 1, 0, self.ni - 1), self.ni)
        return np.where(inside, out, -1)

    def u_dof(self, comp, node) -> np.ndarray:
        """Velocity unknown of component comp at full-grid node, or -1 (Dirichlet)."""
        inn = self.interior_node(node)
        return np.where(inn >= 0, np.asarray(comp) * self.n_int_nodes + inn, -1)

    def cells(self) -> np.ndarray:
        """Cell multi-indices (n_cells, dim) in lex order."""
        return unlex(np.arange(self.n_cells), self.n, self.dim)

    def element_dofs(self) -> np.ndarray:
        """(n_cells, dim * 3^dim) velocity unknowns of every cell (local index
        comp * 3^dim + a + 3b + 9c), -1 for Dirichlet nodes."""
        cells = self.cells()
        loc = unlex(np.arange(3 ** self.dim), 3, self.dim)          # (nn, dim)
        nodes = 2 * cells[:, None, :] + loc[None, :, :]             # (nc, nn, dim)
        out = [self.u_dof(c, nodes) for c in range(self.dim)]
        return np.concatenate(out, axis=1)

    def quad_points(self) -> np.ndarray:
        """Physical quadrature points (n_cells, nq, dim)."""
        xi, _, _, _ = reference_tables(self.dim)
        return self.h * (self.cells()[:, None, :] + xi[None, :, :])

    # ---- stored (full grid) <-> unknowns --------------------------------------
    def stored_index(self) -> np.ndarray:
        """For every velocity unknown, its index in the stored full-grid layout."""
        inn = unlex(np.arange(self.n_int_nodes), self.ni, self.dim) + 1
        base = lex(inn, self.n1)
        return np.concatenate([c * self.n_nodes + base for c in range(self.dim)])

    def to_stored(self, u: np.ndarray) -> np.ndarray:
        out = np.zeros(self.n_stored)
        out[self.stored_index()] = u
        return out

    def from_stored(self, us: np.ndarray) -> np.ndarray:
        return np.asarray(us)[self.stored_index()]


class Hierarchy:
    """Levels 0 (coarsest) .. L-1 (finest), N_l = N_fine / 2^(L-1-l)."""

    def __init__(self, dim: int, n_fine: int, n_levels: int):
        assert n_fine % (1 << (n_levels - 1)) == 0
        self.dim = dim
        self.levels = [Level(dim, n_fine >> (n_levels - 1 - l)) for l in range(n_levels)]

    def __len__(self):
        return len(self.levels)

    def __getitem__(self, l):
        return self.levels[l]
