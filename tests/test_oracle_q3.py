"""Pins of the oracle's [Q3]^d x P2disc discretisation and multigrid (k = 3)
against facts fixed outside the oracle: unknown counts printed in the paper,
exact polynomial integrals, closed forms of the basis and the pressure mass,
the vertex-star kernel decomposition, and the direct solution."""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle.fem import Level, lagrange_1d, gauss_legendre_01, lex, pressure_exponents
from oracle.assembly import Operators, element_pressure_mass
from oracle.multigrid import (standard_prolongation, star_patch_dofs, all_vertices, coarse_cell_dofs,
                              StarASM, RobustTransfer)
from test_oracle_fem import Poly, PolyCoef, bubble

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
K = 3


def nodal(level, fields):
    """Interpolate a vector field (list of callables) at the velocity unknowns
    (node i sits at x = i h / k)."""
    k = level.k
    nodes = np.stack(np.meshgrid(*[np.arange(1, k * level.n)] * level.dim, indexing="ij"), -1)
    nodes = nodes.reshape(-1, level.dim)
    out = np.zeros(level.n_u)
    for c, f in enumerate(fields):
        out[level.u_dof(c, nodes)] = f(nodes * level.h / k)
    return out


def cubic_field(dim, scale):
    """A global field in [Q3]^d vanishing on the boundary: bubble times an
    affine factor (degree 3 per axis)."""
    aff = Poly.const(1.0, dim)
    for a in range(dim):
        aff = aff + Poly.var(a, dim) * (0.3 + 0.4 * a)
    return bubble(dim) * aff * scale


def test_q3_unknown_counts_match_paper():
    g = json.load(open(os.path.join(GOLDEN, "paper_counts_q3.json")))
    for c in g["cases"]:
        lv = Level(c["dim"], c["n_fine"], K)
        if "velocity_plus_pressure_unknowns" in c:
            assert lv.n_stored + lv.n_p == c["velocity_plus_pressure_unknowns"], c["_cite"]
        else:
            assert lv.n_stored == c["velocity_unknowns_including_boundary_nodes"], c["_cite"]


def test_cubic_lagrange_basis_closed_form():
    nodes = np.array([0.0, 1 / 3, 2 / 3, 1.0])
    val, der = lagrange_1d(nodes, K)
    assert np.allclose(val, np.eye(4), atol=1e-15)
    xs = np.linspace(0, 1, 11)
    v, d = lagrange_1d(xs, K)
    assert np.allclose(v.sum(-1), 1.0, atol=1e-14)
    assert np.allclose(d.sum(-1), 0.0, atol=1e-12)
    # l_1(x) = 27/2 x (x - 2/3)(x - 1), l_3(x) = 9/2 x (x - 1/3)(x - 2/3)
    assert np.allclose(v[:, 1], 13.5 * xs * (xs - 2 / 3) * (xs - 1), atol=1e-14)
    assert np.allclose(v[:, 3], 4.5 * xs * (xs - 1 / 3) * (xs - 2 / 3), atol=1e-14)
    # l_0'(x) = -9/2 [(x-2/3)(x-1) + (x-1/3)(x-1) + (x-1/3)(x-2/3)]
    d0 = -4.5 * ((xs - 2 / 3) * (xs - 1) + (xs - 1 / 3) * (xs - 1) + (xs - 1 / 3) * (xs - 2 / 3))
    assert np.allclose(d[:, 0], d0, atol=1e-13)


def test_four_point_gauss_rule_exactness():
    x, w = gauss_legendre_01(4)
    for e in range(8):
        assert abs(np.sum(w * x ** e) - 1.0 / (e + 1)) < 1e-15
    assert abs(np.sum(w * x ** 8) - 1.0 / 9) > 1e-7


def test_pressure_monomials():
    assert pressure_exponents(2, K) == [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]
    for dim in (2, 3):
        assert len(pressure_exponents(dim, K)) == math.comb(K - 1 + dim, dim)
        assert Level(dim, 2, K).n_pb == math.comb(K - 1 + dim, dim)


@pytest.mark.parametrize("dim", [2, 3])
def test_pressure_mass_closed_form(dim):
    """(psi_a, psi_b)_K = h^d prod_j int_{-1/2}^{1/2} s^(a_j + b_j) ds, which is
    0 for an odd power and 1 / (2^e (e + 1)) for an even power e."""
    lv = Level(dim, 2, K)
    M = element_pressure_mass(lv)
    ex = pressure_exponents(dim, K)

    def m1(e):
        return 0.0 if e % 2 else 1.0 / (2 ** e * (e + 1))
    expect = np.array([[lv.h ** dim * np.prod([m1(a[j] + b[j]) for j in range(dim)]) for b in ex] for a in ex])
    assert np.allclose(M, expect[None], atol=1e-17, rtol=1e-13)


@pytest.mark.parametrize("dim,n", [(2, 2), (3, 1)])
def test_prolongation_reproduces_coarse_q3(dim, n):
    """Nested spaces: P_H evaluates the coarse Q3 function at the fine nodes."""
    coarse, fine = Level(dim, n, K), Level(dim, 2 * n, K)
    P = standard_prolongation(coarse, fine)
    fields = [cubic_field(dim, c + 1.0) for c in range(dim)]
    assert np.allclose(P @ nodal(coarse, fields), nodal(fine, fields), atol=1e-14)
    if dim == 2:
        # a random coarse vector (not a global polynomial), summed over cells by hand
        rng = np.random.default_rng(3)
        uc = rng.standard_normal(coarse.n_u)
        uf = P @ uc
        fnodes = np.stack(np.meshgrid(*[np.arange(1, K * fine.n)] * dim, indexing="ij"), -1).reshape(-1, dim)
        for node in fnodes[rng.choice(len(fnodes), 30, replace=False)]:
            xq = node / (K * fine.n)
            cell = np.minimum((xq * coarse.n).astype(int), coarse.n - 1)
            val, _ = lagrange_1d(xq * coarse.n - cell, K)
            for c in range(dim):
                s = 0.0
                for loc in itertools.product(range(K + 1), repeat=dim):
                    dof = coarse.u_dof(c, (K * cell + np.array(loc))[None, :])[0]
                    if dof >= 0:
                        s += uc[dof] * np.prod([val[a, loc[a]] for a in range(dim)])
                assert abs(uf[fine.u_dof(c, node[None, :])[0]] - s) < 1e-13


@pytest.mark.parametrize("dim,n", [(2, 3), (3, 1)])
def test_viscous_form_exact_polynomials(dim, n):
    """u^T A v = int 2 mu eps(u):eps(v) for [Q3]^d fields vanishing on the
    boundary and a linear viscosity (degree <= 7 per axis: exact for the
    4-point rule)."""
    mu = Poly.const(1.0, dim) + Poly.var(0, dim) * 0.7 + Poly.var(dim - 1, dim) * 1.3
    lv = Level(dim, n, K)
    ops = Operators(lv, PolyCoef(mu, [Poly.const(0.0, dim)] * dim), gamma=0.0)
    u = [cubic_field(dim, a) for a in (1.0, -0.6, 0.8)[:dim]]
    v = [cubic_field(dim, a) * Poly.const(1.0, dim) for a in (0.5, 1.1, -0.9)[:dim]]
    total = Poly.const(0.0, dim)
    for i in range(dim):
        for j in range(dim):
            eu = (u[i].d(j) + u[j].d(i)) * 0.5
            ev = (v[i].d(j) + v[j].d(i)) * 0.5
            total = total + mu * eu * ev * 2.0
    exact = total.integrate([0.0] * dim, [1.0] * dim)
    got = nodal(lv, v) @ (ops.A @ nodal(lv, u))
    assert abs(got - exact) <= 1e-12 * abs(exact)


@pytest.mark.parametrize("dim,n", [(2, 2), (3, 1)])
def test_divergence_form_exact_polynomials(dim, n):
    """(B u)_{K,m} = -int_K psi_m div u with the P2 monomials in (x - c_K)/h."""
    lv = Level(dim, n, K)
    ops = Operators(lv, PolyCoef(Poly.const(1.0, dim), [Poly.const(0.0, dim)] * dim), gamma=0.0)
    u = [cubic_field(dim, 1.0 + 2.0 * c) for c in range(dim)]
    div = Poly.const(0.0, dim)
    for c in range(dim):
        div = div + u[c].d(c)
    Bu = ops.B @ nodal(lv, u)
    ex = pressure_exponents(dim, K)
    for cell in itertools.product(range(n), repeat=dim):
        cell = np.array(cell)
        kc = lex(cell, n)
        lo, hi = cell * lv.h, (cell + 1) * lv.h
        for m, e in enumerate(ex):
            psi = Poly.const(1.0, dim)
            for j in range(dim):
                for _ in range(e[j]):
                    psi = psi * Poly.var(j, dim, shift=(cell[j] + 0.5) * lv.h, scale=1.0 / lv.h)
            exact = -(psi * div).integrate(lo, hi)
            assert abs(Bu[kc * len(ex) + m] - exact) < 1e-13


@pytest.mark.parametrize("dim,n", [(2, 2), (3, 1)])
def test_rhs_exact_polynomial_force(dim, n):
    f = [Poly.var(0, dim) * (c + 1.0) + Poly.const(0.5, dim) for c in range(dim)]
    lv = Level(dim, n, K)
    ops = Operators(lv, PolyCoef(Poly.const(1.0, dim), f), gamma=0.0)
    v = [cubic_field(dim, 2.0 - c) for c in range(dim)]
    exact = sum((f[c] * v[c]).integrate([0.0] * dim, [1.0] * dim) for c in range(dim))
    assert abs(ops.rhs() @ nodal(lv, v) - exact) < 1e-13


def sinker(dim, dr=1.0, seed=0):
    from oracle.coefficients import SinkerField
    rng = np.random.default_rng(seed)
    return SinkerField(rng.random((2, dim)), dr ** -0.5, dr ** 0.5, omega=0.3)


@pytest.mark.parametrize("dim,n", [(2, 3), (3, 2)])
def test_augmented_block_spd_and_constants_in_kernel_of_bt(dim, n):
    ops = Operators(Level(dim, n, K), sinker(dim, 1e2), gamma=1e3)
    A = ops.Agamma.toarray()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    np.linalg.cholesky(A)
    assert np.abs(ops.B.T @ ops.p_const).max() < 1e-13


def test_q3_patch_sizes():
    """Star interiors hold d (2k-1)^d unknowns, 50 in 2D and 375 in 3D, at
    interior vertices; boundary stars lose the nodes on the boundary."""
    for dim, n, sizes in [(2, 3, {50, 20, 8}), (3, 3, {375, 150, 60, 24})]:
        lv = Level(dim, n, K)
        assert {star_patch_dofs(lv, v).size for v in all_vertices(lv)} == sizes


def test_q3_center_patch_is_coarse_cell_interior():
    for dim in (2, 3):
        fine = Level(dim, 2 if dim == 3 else 4, K)
        for cc in itertools.product(range(fine.n // 2), repeat=dim):
            centre = np.array([2 * c + 1 for c in cc])
            assert np.array_equal(coarse_cell_dofs(fine, cc), star_patch_dofs(fine, centre))
            assert coarse_cell_dofs(fine, cc).size == dim * (2 * K - 1) ** dim


@pytest.mark.parametrize("dim,n", [(2, 3), (3, 2)])
def test_q3_kernel_decomposition_vertex_stars(dim, n):
    """eq. (kdp) for k = 3: the vertex stars span the discrete kernel of B."""
    lv = Level(dim, n, K)
    B = Operators(lv, sinker(dim), gamma=1.0).B.toarray()
    dim_kernel = lv.n_u - np.linalg.matrix_rank(B)
    cols = []
    for v in all_vertices(lv):
        idx = star_patch_dofs(lv, v)
        if idx.size == 0:
            continue
        for z in sla.null_space(B[:, idx]).T:
            full = np.zeros(lv.n_u)
            full[idx] = z
            cols.append(full)
    assert np.linalg.matrix_rank(np.array(cols).T) == dim_kernel


def test_q3_star_smoother_gamma_robust():
    """Section 4.1 for k = 3: the smallest eigenvalue of D A stays put as
    gamma grows, point Jacobi's falls like 1/gamma."""
    lv = Level(2, 3, K)
    lam_star, lam_jac = [], []
    for gamma in (1e2, 1e4, 1e6):
        A = Operators(lv, sinker(2, 1e2), gamma=gamma).Agamma
        Ad = A.toarray()
        asm = StarASM(lv, A)
        D = np.column_stack([asm.apply(e) for e in np.eye(lv.n_u)])
        ev = np.sort(np.real(np.linalg.eigvals(D @ Ad)))
        lam_star.append(ev[0])
        lam_jac.append(np.sort(np.real(np.linalg.eigvals(Ad / np.diag(Ad)[:, None])))[0])
    assert lam_star[2] > 0.5 * lam_star[1] > 0.0
    assert lam_jac[2] < 0.05 * lam_jac[1]
    # at most 2^d stars overlap; the eigenvalues of the product D A carry a
    # rounding error of order kappa(A) eps ~ 1e-7 at gamma = 1e6
    assert ev[-1] <= 4 * (1 + 1e-6)


def test_q3_robust_prolongation_properties():
    """Section 4.2 for k = 3 (2D): divergence of prolongated coarse
    divergence-free fields decays like 1/gamma, bounded energy, the
    restriction is the transpose."""
    coarse, fine = Level(2, 2, K), Level(2, 4, K)
    coef = sinker(2, 1.0)
    divs, ratios = [], []
    for gamma in (1e2, 1e4, 1e6):
        oc, of = Operators(coarse, coef, gamma), Operators(fine, coef, gamma)
        T = RobustTransfer(coarse, fine, of)
        kerH = sla.null_space(oc.B.toarray())
        uH = kerH @ np.random.default_rng(4).standard_normal(kerH.shape[1])
        Mp = of.Mp.toarray()
        Winv = of.Winv.toarray()
        bt = of.B @ T.prolong(uH)
        bs = of.B @ (T.P @ uH)
        divs.append((np.sqrt(bt @ Winv @ bt), np.sqrt(bs @ Winv @ bs)))
        Pt = np.column_stack([T.prolong(e) for e in np.eye(coarse.n_u)])
        ratios.append(sla.eigh(Pt.T @ of.Agamma.toarray() @ Pt, oc.Agamma.toarray(), eigvals_only=True)[-1])
        R = np.column_stack([T.restrict(e) for e in np.eye(fine.n_u)])
        assert np.abs(R - Pt.T).max() <= 1e-9 * np.abs(Pt).max()
        assert Mp.shape[0] == fine.n_p
    assert divs[1][0] < 0.02 * divs[0][0] and divs[2][0] < 0.02 * divs[1][0]
    assert divs[2][1] > 0.5 * divs[0][1]
    assert max(ratios) < 4.0


@pytest.mark.parametrize("cycle", ["V", "F"])
def test_q3_fgmres_matches_direct_solution(cycle):
    """The whole k = 3 solver (FGMRES, block preconditioner, star-ASM
    multigrid with robust transfers) reaches the direct solution of the
    bordered system (the plain definition of the discrete solution)."""
    from workloads import small
    from oracle.krylov import StokesSolver
    from oracle.direct import solve_direct
    wl = small(2, 8, 2, gamma=1e3, dr=1e4, n_sinkers=3, seed=11, degree=K, cycle=cycle)
    S = StokesSolver(wl)
    x, info = S.solve()
    assert info["converged"] and info["iters"] <= 30
    xd = solve_direct(S.ops, S.ops.rhs())
    nu = S.ops.level.n_u
    assert np.linalg.norm(x[:nu] - xd[:nu]) <= 1e-6 * np.linalg.norm(xd[:nu])
    assert np.linalg.norm(x[nu:] - xd[nu:]) <= 1e-6 * np.linalg.norm(xd[nu:])
