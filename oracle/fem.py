"""Structured [Q_k]^d x P_{k-1}^disc discretisation on the unit square/cube,
k = 2 (the path's discretisation) or k = 3 (oracle).

Test infrastructure: see the package docstring.

Spaces (Section 4, definition of V_h^k and Q_h^{k-1}):
  * velocity: continuous, piecewise tensor-product polynomials of degree k
    (Q_k) in each of the d components, zero on the whole boundary
    (homogeneous Dirichlet, Section 2, eq. (stokes-linear));
  * pressure: discontinuous, total degree <= k-1 on every cell (P_{k-1}^disc),
    with zero mean (Q_h subset of L^2_0).

Mesh: [0,1]^d split into N^d axis-aligned cells of width h = 1/N; uniform
refinement gives the multigrid levels (Section 5.1). On axis-aligned cells the
"mapped" and the physical P_{k-1} spaces coincide, so the pressure basis on
cell K with centre c_K is the monomials of total degree <= k-1 in
(x - c_K) / h: psi_0 = 1, psi_j = (x_j - c_{K,j}) / h (j = 1..d), then for
k = 3 the quadratic ones (pressure_exponents gives the order).

Readings (the paper names the spaces, not these details): the velocity
Lagrange nodes are equispaced, {0, 1/k, .., 1} on the reference interval;
quadrature is tensor Gauss-Legendre with k+1 points per axis (exact through
degree 2k+1 per axis: the constant-coefficient stiffness is integrated
exactly on affine cells).

Index conventions (shared with nothing; the GPU library defines its own):
  * multi-indices are ordered (x, y[, z]) and flattened lexicographically with
    x fastest;
  * a cell with lower corner index (i, j[, k']) owns the full-grid nodes
    (k i + a, k j + b[, k k' + c]), a, b, c in {0..k}; local node =
    a + (k+1) b + (k+1)^2 c;
  * velocity unknowns are the interior nodes (all indices in 1..kN-1),
    numbered component-major: dof = comp * (kN-1)^d + lex(node - 1);
  * the "stored" layout is the full node grid, comp-major, x fastest, with
    zeros on Dirichlet nodes: index = comp * (kN+1)^d + lex(node).
  * pressure unknowns: dof = cell * n_pb + m, m = 0..n_pb-1 (n_pb = d+1
    for k = 2; 6 (2D) or 10 (3D) for k = 3).
"""
from __future__ import annotations

import itertools
from functools import lru_cache

import numpy as np

Q1D = 3          # Gauss points per axis for k = 2 (exact for degree <= 5)
NODES_1D = np.array([0.0, 0.5, 1.0])


def nodes_1d(k: int = 2) -> np.ndarray:
    """Equispaced Lagrange nodes {0, 1/k, .., 1} of the degree-k basis."""
    return np.arange(k + 1) / float(k)


@lru_cache(maxsize=None)
def gauss_legendre_01(n: int = Q1D):
    """Gauss-Legendre points and weights mapped from [-1, 1] to [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_1d(xi: np.ndarray, k: int = 2):
    """Values and derivatives of the k+1 Lagrange polynomials of degree k on
    the nodes {0, 1/k, .., 1} at points xi; returns (val[..., k+1],
    der[..., k+1]) (k = 2: nodes {0, 1/2, 1}).

    Written from the Lagrange product formula l_a(x) = prod_{b != a}
    (x - x_b) / (x_a - x_b) and its product-rule derivative.
    """
    xi = np.asarray(xi, dtype=np.float64)
    nd = nodes_1d(k)
    val = np.ones(xi.shape + (k + 1,))
    der = np.zeros(xi.shape + (k + 1,))
    for a in range(k + 1):
        others = [b for b in range(k + 1) if b != a]
        den = np.prod([nd[a] - nd[b] for b in others])
        val[..., a] = np.prod([xi - nd[b] for b in others], axis=0) / den
        d = np.zeros(xi.shape)
        for skip in others:
            d = d + np.prod([xi - nd[b] for b in others if b != skip], axis=0)
        der[..., a] = d / den
    return val, der


@lru_cache(maxsize=None)
def reference_tables(dim: int, k: int = 2):
    """Reference-cell tables of Q_k at the tensor Gauss points (k+1 per axis).

    Returns (xi[q, dim], w[q], phi[q, n], dphi[q, n, dim]) with q and n
    flattened x-fastest; dphi is the gradient in reference coordinates
    (divide by h for the physical gradient).
    """
    nq1 = k + 1
    g, gw = gauss_legendre_01(nq1)
    val, der = lagrange_1d(g, k)       # [qpt, node]
    qs = list(itertools.product(range(nq1), repeat=dim))
    ns = list(itertools.product(range(k + 1), repeat=dim))
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


def pressure_exponents(dim: int, k: int = 2):
    """Exponent tuples of the P_{k-1} monomials: by total degree, and within
    a degree by decreasing power of x, then of y (k = 2: 1, x, y[, z];
    k = 3 in 2D: 1, x, y, x^2, xy, y^2)."""
    out = []
    for deg in range(k):
        tup = [t for t in itertools.product(range(deg + 1), repeat=dim) if sum(t) == deg]
        tup.sort(reverse=True)
        out += tup
    return out


def pressure_basis(xi: np.ndarray, k: int = 2) -> np.ndarray:
    """P_{k-1}^disc basis at reference points xi[..., dim]: the monomials of
    pressure_exponents in (xi - 1/2); k = 2: [1, xi_1 - 1/2, ...]."""
    xi = np.asarray(xi) - 0.5
    dim = xi.shape[-1]
    cols = [np.prod([xi[..., j] ** e[j] for j in range(dim)], axis=0) for e in pressure_exponents(dim, k)]
    return np.stack(cols, axis=-1)


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
    """One level of the uniformly refined hierarchy: N cells per axis, velocity
    degree k (2 or 3)."""

    def __init__(self, dim: int, n: int, k: int = 2):
        assert dim in (2, 3) and n >= 1 and k in (2, 3)
        self.dim, self.n, self.k = dim, n, k
        self.h = 1.0 / n
        self.n1 = k * n + 1                    # nodes per axis
        self.ni = k * n - 1                    # interior nodes per axis
        self.nn = (k + 1) ** dim               # nodes per cell
        self.n_nodes = self.n1 ** dim
        self.n_int_nodes = self.ni ** dim
        self.n_u = dim * self.n_int_nodes      # velocity unknowns
        self.n_cells = n ** dim
        self.n_pb = len(pressure_exponents(dim, k))   # pressure unknowns per cell
        self.n_p = self.n_pb * self.n_cells    # pressure unknowns
        self.n_stored = dim * self.n_nodes

    # ---- node / dof numbering -------------------------------------------------
    def interior_node(self, node: np.ndarray) -> np.ndarray:
        """Interior lex index of full-grid nodes node[..., dim], or -1 on the boundary."""
        node = np.asarray(node)
        inside = np.all((node >= 1) & (node <= self.k * self.n - 1), axis=-1)
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
        """(n_cells, dim * (k+1)^dim) velocity unknowns of every cell (local
        index comp * (k+1)^dim + local node), -1 for Dirichlet nodes."""
        cells = self.cells()
        loc = unlex(np.arange(self.nn), self.k + 1, self.dim)       # (nn, dim)
        nodes = self.k * cells[:, None, :] + loc[None, :, :]        # (nc, nn, dim)
        out = [self.u_dof(c, nodes) for c in range(self.dim)]
        return np.concatenate(out, axis=1)

    def quad_points(self) -> np.ndarray:
        """Physical quadrature points (n_cells, nq, dim)."""
        xi, _, _, _ = reference_tables(self.dim, self.k)
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

    def __init__(self, dim: int, n_fine: int, n_levels: int, k: int = 2):
        assert n_fine % (1 << (n_levels - 1)) == 0
        self.dim, self.k = dim, k
        self.levels = [Level(dim, n_fine >> (n_levels - 1 - l), k) for l in range(n_levels)]

    def __len__(self):
        return len(self.levels)

    def __getitem__(self, l):
        return self.levels[l]
