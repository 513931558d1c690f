"""Pins of three oracle functions against values fixed outside the oracle:

* the multi-sinker viscosity and forcing of Section 5.2 (reading: floor
  mu_min and squared Gaussian) at points where the closed form reduces to a
  number by hand: a sinker centre, a point at distance omega/2 + s from a lone
  sinker, points far from every sinker, and a point between two sinkers
  (product over sinkers);
* the block preconditioner of eq. (precond) (kind "full") with exact inner
  solves against the dense product of its three block factors;
* the tensor branch of the element viscous matrix: equal to the scalar branch
  for C = 2 mu I_sym, and equal to the exact polynomial integral of
  (C : eps(u)) : eps(v) for a constant anisotropic C without major symmetry
  (so a transposed contraction would be caught).
"""
import itertools
from types import SimpleNamespace

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.assembly import Operators, element_viscous
from oracle.coefficients import SinkerField
from oracle.fem import Level
from test_oracle_fem import Poly, bubble, nodal

MU_MIN, MU_MAX, OMEGA, DELTA, BETA = 1e-3, 1e3, 0.1, 200.0, 10.0


def lone(center):
    return SinkerField(np.array([center], dtype=float), MU_MIN, MU_MAX, OMEGA, DELTA, BETA)


# --------------------------------------------------------------------------- sinker field
@pytest.mark.parametrize("dim", [2, 3])
def test_sinker_value_at_centre_and_inside(dim):
    """Inside a sinker (|x - c| <= omega/2) the Gaussian factor is 1, so
    chi = 0, mu = mu_max and f = (0, .., -beta)."""
    c = np.full(dim, 0.4)
    f = lone(c)
    for x in (c, c + np.eye(dim)[0] * 0.5 * OMEGA * 0.999):
        assert f.chi(x[None])[0] == 0.0
        assert f.mu(x[None])[0] == MU_MAX
        force = f.force(x[None])[0]
        assert np.all(force[:-1] == 0.0) and force[-1] == -BETA


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("s", [0.02, 0.05, 0.1])
def test_sinker_value_at_distance(dim, s):
    """At distance omega/2 + s from a lone sinker, chi = 1 - exp(-delta s^2)
    and mu = (mu_max - mu_min) exp(-delta s^2) + mu_min (hand values: delta s^2
    = 0.08, 0.5, 2). An unsquared exponent gives exp(-delta s) instead, and a
    missing floor drops the mu_min term."""
    c = np.full(dim, 0.3)
    direction = np.arange(1.0, dim + 1.0)
    direction /= np.linalg.norm(direction)
    x = c + (0.5 * OMEGA + s) * direction
    g = {0.02: np.exp(-0.08), 0.05: np.exp(-0.5), 0.1: np.exp(-2.0)}[s]
    f = lone(c)
    assert abs(f.chi(x[None])[0] - (1.0 - g)) <= 1e-14
    mu = f.mu(x[None])[0]
    assert abs(mu - ((MU_MAX - MU_MIN) * g + MU_MIN)) <= 1e-13 * MU_MAX
    assert abs(f.force(x[None])[0][-1] - (-BETA * g)) <= 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_sinker_far_field_is_the_floor(dim):
    """Far from every sinker chi = 1 to rounding, so mu = mu_min (not 0) and
    the forcing vanishes."""
    rng = np.random.default_rng(0)
    f = SinkerField(rng.random((5, dim)) * 0.2, MU_MIN, MU_MAX, OMEGA, DELTA, BETA)
    x = np.full((3, dim), 0.9) + rng.random((3, dim)) * 0.1   # >= 0.6 from every centre
    assert np.all(np.abs(f.chi(x) - 1.0) <= 1e-15)
    assert np.allclose(f.mu(x), MU_MIN, rtol=1e-9, atol=0.0)
    assert np.all(np.abs(f.force(x)[..., -1]) <= 1e-14)


def test_sinker_product_over_two_sinkers():
    """chi multiplies the factors of the sinkers: at distances omega/2 + s1
    and omega/2 + s2 from two sinkers, chi = (1 - e^{-delta s1^2})(1 - e^{-delta s2^2})."""
    c1, c2 = np.array([0.3, 0.5]), np.array([0.6, 0.5])
    x = np.array([[0.45, 0.5]])             # 0.15 from both: s = 0.1, delta s^2 = 2
    f = SinkerField(np.stack([c1, c2]), MU_MIN, MU_MAX, OMEGA, DELTA, BETA)
    chi = (1.0 - np.exp(-2.0)) ** 2
    assert abs(f.chi(x)[0] - chi) <= 1e-14
    assert abs(f.mu(x)[0] - ((MU_MAX - MU_MIN) * (1.0 - chi) + MU_MIN)) <= 1e-13 * MU_MAX


# --------------------------------------------------------------------------- block preconditioner
def exact_pc(ops, kind):
    from oracle.krylov import BlockPreconditioner
    lu = spla.splu(ops.Agamma.tocsc())
    return BlockPreconditioner(SimpleNamespace(ops=[ops], vcycle=lu.solve), kind)


def dense_factors(ops):
    """The three block factors of eq. (precond) with Ahat = A_gamma exactly:
    [I, -A^{-1}B^T; 0, I] diag(A^{-1}, -Shat^{-1}) [I, 0; -B A^{-1}, I]."""
    nu, npres = ops.level.n_u, ops.level.n_p
    Ainv = np.linalg.inv(ops.Agamma.toarray())
    Sinv = ops.Shat_inv.toarray()
    B = ops.B.toarray()
    I_u, I_p, Z_up = np.eye(nu), np.eye(npres), np.zeros((nu, npres))
    left = np.block([[I_u, -Ainv @ B.T], [Z_up.T, I_p]])
    mid = np.block([[Ainv, Z_up], [Z_up.T, -Sinv]])
    right = np.block([[I_u, Z_up], [-B @ Ainv, I_p]])
    return left, mid, right, Ainv, Sinv, B


@pytest.mark.parametrize("dim,n,schur", [(2, 3, 1), (2, 3, 2), (3, 2, 1)])
def test_full_block_preconditioner_equals_dense_factors(dim, n, schur):
    """With exact inner solves, BlockPreconditioner("full").apply equals the
    dense product of the three factors applied to v: exactly when the
    Schur output has zero mean (the projection is then inactive), and with
    the mean projection of the pressure block inserted after the middle
    factor for a general v. A sign error in z_p or in either off-diagonal
    factor changes the result."""
    rng = np.random.default_rng(7)
    coef = SinkerField(rng.random((3, dim)), 1e-2, 1e2, omega=0.3)
    ops = Operators(Level(dim, n), coef, gamma=30.0, schur=schur)
    nu, npres = ops.level.n_u, ops.level.n_p
    left, mid, right, Ainv, Sinv, B = dense_factors(ops)
    P = left @ mid @ right
    pc = exact_pc(ops, "full")
    # (1) data for which -Shat^{-1}(v_p - B A^{-1} v_u) is mean-free
    vu = rng.standard_normal(nu)
    p0 = ops.project_mean(rng.standard_normal(npres))
    vp = B @ (Ainv @ vu) - np.linalg.solve(Sinv, p0)
    v = np.concatenate([vu, vp])
    ref = P @ v
    got = pc.apply(v)
    assert np.allclose(got[nu:], p0, rtol=1e-9, atol=1e-9 * np.abs(p0).max())
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()
    # (2) general v: the projection Q = I - 1 m^T / (m^T 1) acts on the pressure
    m, one = ops.p_mass_const, ops.p_const
    Q = np.eye(npres) - np.outer(one, m) / (m @ one)
    Qb = np.block([[np.eye(nu), np.zeros((nu, npres))], [np.zeros((npres, nu)), Q]])
    Pq = left @ Qb @ mid @ right
    v = rng.standard_normal(nu + npres)
    ref = Pq @ v
    assert np.abs(pc.apply(v) - ref).max() <= 1e-9 * np.abs(ref).max()


# --------------------------------------------------------------------------- tensor element matrices
class TensorCoef:
    """Test coefficient: kind "tensor" with a given C(x) of shape [.., d, d, d, d]."""
    kind = "tensor"

    def __init__(self, fn):
        self.fn = fn

    def stress_tensor(self, x):
        return self.fn(x)


@pytest.mark.parametrize("dim,n", [(2, 3), (3, 2)])
def test_tensor_branch_equals_scalar_branch_for_isotropic_c(dim, n):
    """C = 2 mu I_sym (I_sym the identity on symmetric tensors) gives the
    scalar-branch element matrices of the same mu."""
    rng = np.random.default_rng(2)
    base = SinkerField(rng.random((3, dim)), 1e-2, 1e2, omega=0.3)
    lv = Level(dim, n)
    As = element_viscous(lv, base)
    At = element_viscous(lv, TensorCoef(base.stress_tensor))
    assert np.abs(At - As).max() <= 1e-13 * np.abs(As).max()


def anisotropic_constant_tensor(dim, seed):
    """A constant fourth-order tensor with both minor symmetries but no major
    symmetry: C_abcd = C_bacd = C_abdc, C_abcd != C_cdab in general."""
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((dim, dim, dim, dim))
    C = 0.5 * (C + C.transpose(1, 0, 2, 3))
    C = 0.5 * (C + C.transpose(0, 1, 3, 2))
    assert np.abs(C - C.transpose(2, 3, 0, 1)).max() > 0.1
    return C


@pytest.mark.parametrize("dim,n", [(2, 3), (3, 2)])
def test_tensor_branch_exact_polynomial_integral(dim, n):
    """v^T A u equals int (C : eps(u)) : eps(v) computed exactly for Q2
    polynomial fields vanishing on the boundary and a constant C (the
    integrand has degree <= 4 per axis, within the 3-point rule)."""
    C = anisotropic_constant_tensor(dim, 11)
    coef = TensorCoef(lambda x: np.broadcast_to(C, x.shape[:-1] + C.shape))
    lv = Level(dim, n)
    Ae = element_viscous(lv, coef)
    ed = lv.element_dofs()
    A = np.zeros((lv.n_u, lv.n_u))
    for k in range(lv.n_cells):
        keep = ed[k] >= 0
        A[np.ix_(ed[k][keep], ed[k][keep])] += Ae[k][np.ix_(keep, keep)]
    b = bubble(dim)
    rng = np.random.default_rng(5)
    # two different vector fields in V_h (the bubble, of degree 2 per axis,
    # times random constants per component)
    u = [b * rng.standard_normal() for _ in range(dim)]
    v = [b * rng.standard_normal() for _ in range(dim)]

    def eps(w):
        return [[(w[i].d(j) + w[j].d(i)) * 0.5 for j in range(dim)] for i in range(dim)]

    eu, ev = eps(u), eps(v)
    total = Poly.const(0.0, dim)
    for a, bb, c, d in itertools.product(range(dim), repeat=4):
        if C[a, bb, c, d] != 0.0:
            total = total + ev[a][bb] * eu[c][d] * C[a, bb, c, d]
    exact = total.integrate([0.0] * dim, [1.0] * dim)
    got = nodal(lv, v) @ (A @ nodal(lv, u))
    assert abs(got - exact) <= 1e-12 * max(abs(exact), 1e-300)
    # the transposed contraction gives a different number for this C
    totalT = Poly.const(0.0, dim)
    for a, bb, c, d in itertools.product(range(dim), repeat=4):
        totalT = totalT + eu[a][bb] * ev[c][d] * C[a, bb, c, d]
    assert abs(totalT.integrate([0.0] * dim, [1.0] * dim) - exact) > 1e-6 * abs(exact)
