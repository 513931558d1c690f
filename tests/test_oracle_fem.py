"""Pins of the oracle's discretisation against facts fixed outside the oracle:
counts printed in the paper, exact polynomial integrals, closed forms."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle.fem import Level, lagrange_1d, gauss_legendre_01, reference_tables, lex
from oracle.assembly import Operators, element_pressure_mass
from oracle.multigrid import standard_prolongation

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------- tiny exact polynomial algebra
class Poly:
    """Multivariate polynomial {exponent tuple: coefficient}, exact integration."""

    def __init__(self, terms, dim):
        self.t = {k: v for k, v in terms.items() if v != 0.0}
        self.dim = dim

    @staticmethod
    def var(k, dim, shift=0.0, scale=1.0):
        e = [0] * dim
        e[k] = 1
        terms = {tuple(e): scale}
        if shift:
            terms[(0,) * dim] = -shift * scale
        return Poly(terms, dim)

    @staticmethod
    def const(c, dim):
        return Poly({(0,) * dim: c}, dim)

    def __add__(self, o):
        t = dict(self.t)
        for k, v in o.t.items():
            t[k] = t.get(k, 0.0) + v
        return Poly(t, self.dim)

    def __sub__(self, o):
        return self + o * (-1.0)

    def __mul__(self, o):
        if not isinstance(o, Poly):
            return Poly({k: v * o for k, v in self.t.items()}, self.dim)
        t = {}
        for (k1, v1), (k2, v2) in itertools.product(self.t.items(), o.t.items()):
            k = tuple(a + b for a, b in zip(k1, k2))
            t[k] = t.get(k, 0.0) + v1 * v2
        return Poly(t, self.dim)

    def d(self, k):
        t = {}
        for e, v in self.t.items():
            if e[k] > 0:
                e2 = list(e)
                e2[k] -= 1
                t[tuple(e2)] = t.get(tuple(e2), 0.0) + v * e[k]
        return Poly(t, self.dim)

    def integrate(self, lo, hi):
        s = 0.0
        for e, v in self.t.items():
            s += v * np.prod([(hi[k] ** (e[k] + 1) - lo[k] ** (e[k] + 1)) / (e[k] + 1)
                              for k in range(self.dim)])
        return s

    def __call__(self, x):
        x = np.asarray(x, dtype=np.float64)
        out = np.zeros(x.shape[:-1])
        for e, v in self.t.items():
            out = out + v * np.prod([x[..., k] ** e[k] for k in range(self.dim)], axis=0)
        return out


def bubble(dim):
    b = Poly.const(1.0, dim)
    for k in range(dim):
        xk = Poly.var(k, dim)
        b = b * xk * (Poly.const(1.0, dim) - xk)
    return b


class PolyCoef:
    """Coefficient object with a polynomial viscosity and force (test only)."""
    kind = "scalar"

    def __init__(self, mu, force):
        self._mu, self._f = mu, force

    def mu(self, x):
        return self._mu(x)

    def scalar_viscosity(self, x):
        return self._mu(x)

    def force(self, x):
        return np.stack([f(x) for f in self._f], axis=-1)


def nodal(level, fields):
    """Interpolate a vector field (list of callables) at the velocity unknowns."""
    nodes = np.stack(np.meshgrid(*[np.arange(1, 2 * level.n)] * level.dim, indexing="ij"), -1)
    nodes = nodes.reshape(-1, level.dim)
    out = np.zeros(level.n_u)
    for c, f in enumerate(fields):
        dofs = level.u_dof(c, nodes)
        out[dofs] = f(nodes * level.h / 2.0)
    return out


# --------------------------------------------------------------------------- tests
def test_dof_counts_match_paper():
    g = json.load(open(os.path.join(GOLDEN, "paper_counts.json")))
    lv = Level(g["dim"], g["n_fine"])
    assert lv.n_stored == g["velocity_unknowns_including_boundary_nodes"]
    assert lv.n_p == g["pressure_unknowns_p1disc"]


def test_lagrange_basis_closed_form():
    val, der = lagrange_1d(np.array([0.0, 0.5, 1.0]))
    assert np.allclose(val, np.eye(3), atol=0, rtol=0)
    xs = np.linspace(0, 1, 7)
    v, d = lagrange_1d(xs)
    assert np.allclose(v.sum(-1), 1.0, atol=1e-15)
    assert np.allclose(d.sum(-1), 0.0, atol=1e-14)
    # l0 = 2(x-1/2)(x-1), l1 = 4x(1-x), l2 = 2x(x-1/2)
    assert np.allclose(v[:, 0], 2 * (xs - 0.5) * (xs - 1), atol=1e-15)
    assert np.allclose(v[:, 1], 4 * xs * (1 - xs), atol=1e-15)
    assert np.allclose(d[:, 2], 4 * xs - 1, atol=1e-14)
    q, _ = lagrange_1d(np.array([0.25, 0.75]))
    assert np.allclose(q[0], [3 / 8, 3 / 4, -1 / 8], atol=0)
    assert np.allclose(q[1], [-1 / 8, 3 / 4, 3 / 8], atol=0)


def test_gauss_rule_exactness():
    x, w = gauss_legendre_01(3)
    for k in range(6):
        assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-15
    assert abs(np.sum(w * x ** 6) - 1.0 / 7) > 1e-6


@pytest.mark.parametrize("dim,n", [(2, 4), (3, 2)])
def test_prolongation_reproduces_coarse_q2(dim, n):
    """Nested spaces: P_H is the identity on V_H (Lemma P(d) proof, Section 4.2)."""
    coarse, fine = Level(dim, n), Level(dim, 2 * n)
    b = bubble(dim)
    xk = [Poly.var(k, dim) for k in range(dim)]
    # per-cell Q2 field that is not a global polynomial: bubble plus a kink-free
    # random coarse vector
    rng = np.random.default_rng(3)
    uc = rng.standard_normal(coarse.n_u)
    P = standard_prolongation(coarse, fine)
    uf = P @ uc
    # evaluate the coarse FE function at fine nodes by direct summation over cells
    for c in range(dim):
        fnodes = np.stack(np.meshgrid(*[np.arange(1, 2 * fine.n)] * dim, indexing="ij"), -1).reshape(-1, dim)
        sample = fnodes[rng.choice(len(fnodes), 25, replace=False)]
        for node in sample:
            xq = node / (2.0 * fine.n)
            cell = np.minimum((xq * coarse.n).astype(int), coarse.n - 1)
            xi = xq * coarse.n - cell
            val, _ = lagrange_1d(xi)
            s = 0.0
            for loc in itertools.product(range(3), repeat=dim):
                cn = 2 * cell + np.array(loc)
                dof = coarse.u_dof(c, cn[None, :])[0]
                if dof >= 0:
                    s += uc[dof] * np.prod([val[k, loc[k]] for k in range(dim)])
            assert abs(uf[fine.u_dof(c, node[None, :])[0]] - s) < 1e-13
    # a global Q2 polynomial interpolates identically on both levels
    fields = [b * (c + 1.0) for c in range(dim)]
    assert np.allclose(P @ nodal(coarse, fields), nodal(fine, fields), atol=1e-15)


@pytest.mark.parametrize("dim,n", [(2, 3), (3, 2)])
def test_viscous_form_exact_polynomials(dim, n):
    """u^T A v equals the exact integral of 2 mu eps(u):eps(v) for Q2
    polynomials vanishing on the boundary and a linear viscosity (the
    integrand is within the exactness of the 3-point rule)."""
    b = bubble(dim)
    mu = Poly.const(1.0, dim) + Poly.var(0, dim) * 0.7 + Poly.var(dim - 1, dim) * 1.3
    coef = PolyCoef(mu, [Poly.const(0.0, dim)] * dim)
    lv = Level(dim, n)
    ops = Operators(lv, coef, gamma=0.0)
    rng = np.random.default_rng(5)
    au = rng.standard_normal(dim)
    av = rng.standard_normal(dim)
    u = [b * a for a in au]
    v = [b * a for a in av]
    # exact: int 2 mu eps(u) : eps(v)
    total = Poly.const(0.0, dim)
    for i in range(dim):
        for j in range(dim):
            eu = (u[i].d(j) + u[j].d(i)) * 0.5
            ev = (v[i].d(j) + v[j].d(i)) * 0.5
            total = total + mu * eu * ev * 2.0
    exact = total.integrate([0.0] * dim, [1.0] * dim)
    got = nodal(lv, v) @ (ops.A @ nodal(lv, u))
    assert abs(got - exact) <= 1e-13 * abs(exact)


@pytest.mark.parametrize("dim,n", [(2, 3), (3, 2)])
def test_divergence_form_exact_polynomials(dim, n):
    """(B u)_{K,m} = -int_K psi_m div u, psi_0 = 1, psi_j = (x_j - c_j)/h."""
    b = bubble(dim)
    lv = Level(dim, n)
    coef = PolyCoef(Poly.const(1.0, dim), [Poly.const(0.0, dim)] * dim)
    ops = Operators(lv, coef, gamma=0.0)
    u = [b * (1.0 + 2.0 * c) for c in range(dim)]
    div = Poly.const(0.0, dim)
    for c in range(dim):
        div = div + u[c].d(c)
    Bu = ops.B @ nodal(lv, u)
    for cell in itertools.product(range(n), repeat=dim):
        cell = np.array(cell)
        k = lex(cell, n)
        lo, hi = cell * lv.h, (cell + 1) * lv.h
        for m in range(dim + 1):
            psi = Poly.const(1.0, dim) if m == 0 else \
                Poly.var(m - 1, dim, shift=(cell[m - 1] + 0.5) * lv.h, scale=1.0 / lv.h)
            exact = -(psi * div).integrate(lo, hi)
            assert abs(Bu[k * (dim + 1) + m] - exact) < 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_pressure_mass_closed_form(dim):
    lv = Level(dim, 3)
    M = element_pressure_mass(lv)
    expect = lv.h ** dim * np.diag([1.0] + [1.0 / 12] * dim)
    assert np.allclose(M, expect[None], atol=1e-17, rtol=1e-14)


@pytest.mark.parametrize("dim,n", [(2, 3), (3, 2)])
def test_rhs_exact_polynomial_force(dim, n):
    """(f, v) for a polynomial force and v in V_h (integrand degree <= 5 per axis)."""
    b = bubble(dim)
    f = [Poly.var(0, dim) * (c + 1.0) + Poly.const(0.5, dim) for c in range(dim)]
    coef = PolyCoef(Poly.const(1.0, dim), f)
    lv = Level(dim, n)
    ops = Operators(lv, coef, gamma=0.0)
    v = [b * (2.0 - c) for c in range(dim)]
    exact = sum((f[c] * v[c]).integrate([0.0] * dim, [1.0] * dim) for c in range(dim))
    assert abs(ops.rhs() @ nodal(lv, v) - exact) < 1e-14


@pytest.mark.parametrize("dim,n", [(2, 4), (3, 2)])
def test_augmented_block_symmetric_positive_definite(dim, n):
    from oracle.coefficients import SinkerField
    rng = np.random.default_rng(1)
    coef = SinkerField(rng.random((3, dim)), 0.01, 100.0)
    ops = Operators(Level(dim, n), coef, gamma=1e3)
    A = ops.Agamma.toarray()
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    np.linalg.cholesky(A)
    # constants are the kernel of B^T (velocity vanishes on the boundary)
    assert np.abs(ops.B.T @ ops.p_const).max() < 1e-14


@pytest.mark.parametrize("tensor", [False, True])
def test_local_rows_equal_assembled_operator(tensor):
    """stokes_rows / rhs_rows (used for spot checks at sizes too large to
    assemble) give the same entries as the assembled K and right-hand side."""
    from workloads import small
    from oracle.krylov import StokesSolver
    from oracle.assembly import stokes_rows, rhs_rows
    if tensor:
        wl = small(3, 4, 2, gamma=1e2, dr=1e6, n_sinkers=4, seed=4, coef_kind=1, fourier_seed=5)
    else:
        wl = small(2, 8, 2, gamma=1e3, dr=1e4, n_sinkers=4, seed=3)
    S = StokesSolver(wl)
    lv = S.ops.level
    rng = np.random.default_rng(0)
    u, p = rng.standard_normal(lv.n_u), rng.standard_normal(lv.n_p)
    rows = rng.choice(lv.n_u, 30, replace=False)
    pc = rng.choice(lv.n_cells, 5, replace=False)
    yv, yp = stokes_rows(lv, S.coef, wl.gamma, u, p, rows, pc)
    full = S.K @ np.concatenate([u, p])
    scale = np.max(np.abs(full))
    assert np.max(np.abs(yv - full[rows])) <= 1e-14 * scale
    pidx = (pc[:, None] * (lv.dim + 1) + np.arange(lv.dim + 1)).ravel()
    assert np.max(np.abs(yp.ravel() - full[lv.n_u:][pidx])) <= 1e-14 * scale
    assert np.allclose(rhs_rows(lv, S.coef, rows), S.ops.rhs()[rows], rtol=1e-14, atol=1e-16)
