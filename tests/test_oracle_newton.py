"""Pins of the oracle's Newton loop for the viscoplastic problem
(Section 5.3): without yielding the residual is the linear operator and one
Newton step solves the problem; the Jacobian the step uses is the derivative
of the residual (central differences); injection reproduces coarse fields;
near the solution the residual falls quadratically."""
import numpy as np
import pytest

from oracle.fem import Level, Hierarchy
from oracle.newton import NewtonSolver, inject, stress_form, ViscoplasticFE
from oracle.multigrid import standard_prolongation
from workloads import small


def wl2(tau_y):
    return small(2, 8, 2, gamma=1e3, dr=1e4, n_sinkers=4, seed=11, coef_kind=2, tau_y=tau_y)


@pytest.mark.parametrize("dim,n", [(2, 4), (3, 2)])
def test_injection_reproduces_coarse_fields(dim, n):
    """Nested Q2 spaces: the prolongation of a coarse field, injected back to
    the coarse nodes, is the field itself."""
    coarse, fine = Level(dim, n), Level(dim, 2 * n)
    xc = np.random.default_rng(1).standard_normal(coarse.n_u)
    assert np.array_equal(inject(fine, coarse, standard_prolongation(coarse, fine) @ xc), xc)


def test_residual_without_yield_is_the_linear_operator():
    """With an unreachable yield stress mu_eff = mu0, so a(u; .) = A u with
    the assembled viscous matrix of the sinker field."""
    ns = NewtonSolver(wl2(1e300), tau_y=1e300)
    u = np.random.default_rng(2).standard_normal(ns.fine.n_u)
    ref = ns.ops0.A @ u
    assert np.abs(stress_form(ns.fine, ns.base, ns.tau_y, ns.mu_f, u) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_jacobian_is_the_derivative_of_the_residual():
    """K(u) d = (F(u + h d) - F(u - h d)) / 2h for the linearisation at a
    state u where part of the domain yields."""
    ns = NewtonSolver(wl2(0.5), tau_y=0.5)
    rng = np.random.default_rng(3)
    u = rng.standard_normal(ns.fine.n_u)
    coef = ViscoplasticFE(ns.base, ns.tau_y, ns.mu_f, ns.hier, u)
    x = ns.fine.quad_points()
    yielded = coef.mu_eff(x) < ns.base.mu(x) - 1e-9
    assert yielded.any() and (~yielded).any()
    K = ns.linearisation(u).K
    p = rng.standard_normal(ns.fine.n_p)
    du, dp = rng.standard_normal(ns.fine.n_u), rng.standard_normal(ns.fine.n_p)
    h = 1e-6
    Fp1 = np.concatenate(ns.residual(u + h * du, p + h * dp))
    Fm1 = np.concatenate(ns.residual(u - h * du, p - h * dp))
    fd = (Fp1 - Fm1) / (2 * h)
    an = K @ np.concatenate([du, dp])
    assert np.linalg.norm(fd - an) <= 1e-6 * np.linalg.norm(an)


def test_newtonian_limit_takes_one_step():
    """Without yielding the problem is linear: one Newton step (solved to
    1e-11) meets a 1e-8 reduction, and the result is the linear Stokes
    solution of the sinker field."""
    from oracle.krylov import StokesSolver
    from oracle.direct import solve_direct
    wl = wl2(1e300)
    ns = NewtonSolver(wl, tau_y=1e300)
    u, p, info = ns.solve(rtol=1e-8, lin_rtol=1e-11)
    assert info["converged"] and info["iters"] == 1 and info["alpha"] == [1.0]
    st = StokesSolver(small(2, 8, 2, gamma=1e3, dr=1e4, n_sinkers=4, seed=11))
    x_d = solve_direct(st.ops, st.ops.rhs())
    assert np.linalg.norm(np.concatenate([u, p]) - x_d) <= 1e-9 * np.linalg.norm(x_d)


def test_newton_converges_quadratically_near_the_solution():
    """With accurate linear solves the last reductions are quadratic:
    r_{k+1} <= C r_k^2 with C from the step before."""
    ns = NewtonSolver(wl2(0.5), tau_y=0.5)
    u, p, info = ns.solve(rtol=1e-10, maxit=30, lin_rtol=1e-12)
    r = info["hist"]
    assert info["converged"] and len(r) >= 4, r
    # the final steps: at least super-linear with order close to 2
    k = len(r) - 1
    assert np.log(r[k]) <= 1.7 * np.log(r[k - 1]) - 0.0 or r[k] <= 1e-13, r
    Fu, Fp = ns.residual(u, p)
    assert np.linalg.norm(np.concatenate([Fu, Fp])) <= 1e-10 * info["res0"]
