"""Pins of the augmented system and the Schur approximations (Section 3):
the Woodbury identity, the closed-form spectrum of the remark for Shat = W,
and the eigenvalue bounds of the lemma on the spectrum of Shat_gamma^{-1} S_gamma."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.fem import Level
from oracle.assembly import Operators
from oracle.coefficients import SinkerField


def setup(dim, n, gamma, schur, seed=2, dr=1e4):
    rng = np.random.default_rng(seed)
    coef = SinkerField(rng.random((3, dim)), dr ** -0.5, dr ** 0.5, omega=0.3)
    ops = Operators(Level(dim, n), coef, gamma=gamma, schur=schur)
    # orthonormal basis of the complement of the constant pressure (kernel of B^T)
    c = ops.p_const / np.linalg.norm(ops.p_const)
    Z = sla.null_space(c[None, :])
    return ops, Z


def dense(M):
    return M.toarray()


def compress(M, Z):
    """Operator on the mean-free quotient whose inverse is the compression of
    M^{-1}: the form in which M^{-1} acts when followed by the mean projection
    (and the form in which W^{-1} enters S_gamma^{-1} = S^{-1} + gamma W^{-1})."""
    return np.linalg.inv(Z.T @ np.linalg.inv(dense(M)) @ Z)


@pytest.mark.parametrize("dim,n", [(2, 4), (3, 2)])
@pytest.mark.parametrize("schur", [1, 2])
def test_woodbury_identity(dim, n, schur):
    """S_gamma^{-1} = S^{-1} + gamma W^{-1} (eq. (AL-Schur)) on the mean-free subspace."""
    gamma = 37.0
    ops, Z = setup(dim, n, gamma, schur)
    Bt = Z.T @ dense(ops.B)
    S = Bt @ np.linalg.solve(dense(ops.A), Bt.T)
    Sg = Bt @ np.linalg.solve(dense(ops.Agamma), Bt.T)
    Winv = Z.T @ dense(ops.Winv) @ Z
    lhs = np.linalg.inv(Sg)
    rhs = np.linalg.inv(S) + gamma * Winv
    assert np.abs(lhs - rhs).max() <= 1e-9 * np.abs(rhs).max()


@pytest.mark.parametrize("gamma", [0.0, 1.0, 1e2, 1e4])
def test_p2_closed_form_spectrum(gamma):
    """Remark after the eigenvalue lemma: with Shat = W the eigenvalues of
    S_gamma x = lambda Shat_gamma x are (1 + gamma) / (nu^{-1} + gamma), nu the
    eigenvalues of S y = nu Shat y. P2 is this case (W = Shat = M_p(1/mu))."""
    ops, Z = setup(2, 4, gamma, schur=2)
    Bt = Z.T @ dense(ops.B)
    S = Bt @ np.linalg.solve(dense(ops.A), Bt.T)
    Sg = Bt @ np.linalg.solve(dense(ops.Agamma), Bt.T)
    Shat = compress(ops.Mp_invmu, Z)
    nu = sla.eigh(S, Shat, eigvals_only=True)
    # Shat_gamma^{-1} = (1+gamma) M_p(1/mu)^{-1}: the operator P2 applies
    Shat_g = np.linalg.inv(Z.T @ dense(ops.Shat_inv) @ Z)
    lam = sla.eigh(Sg, Shat_g, eigvals_only=True)
    expect = np.sort((1.0 + gamma) / (1.0 / nu + gamma))
    assert np.allclose(np.sort(lam), expect, rtol=1e-9, atol=0)


def gen_eig_range(A, B):
    ev = sla.eigh(A, B, eigvals_only=True)
    return ev[0], ev[-1]


@pytest.mark.parametrize("gamma", [0.0, 10.0, 1e3, 1e5])
def test_lemma_eigenvalue_bounds_p1(gamma):
    """Lemma (eigenvalue bounds): sigma(Shat_gamma^{-1} S_gamma) in [f_mu, F_mu]
    with the constants of the three spectral equivalences, for P1
    (Shat = M_p(1/mu), W = M_p); f_mu, F_mu -> 1 as gamma grows."""
    ops, Z = setup(2, 4, gamma, schur=1, dr=1e6)
    Bt = Z.T @ dense(ops.B)
    S = Bt @ np.linalg.solve(dense(ops.A), Bt.T)
    Sg = Bt @ np.linalg.solve(dense(ops.Agamma), Bt.T)
    Shat = compress(ops.Mp_invmu, Z)
    W = compress(ops.Mp, Z)
    c, C = gen_eig_range(S, Shat)       # c Shat <= S <= C Shat
    d, D = gen_eig_range(S, W)          # d W <= S <= D W
    e, E = gen_eig_range(Shat, W)       # e W <= Shat <= E W
    g = gamma
    f = max(c / (1 + g * c * E) + g * d / (1 + g * d), (1 + g * e) / (max(1, 1 / c) + g * e))
    F = min(C / (1 + g * C * e) + g * D / (1 + g * D), (1 + g * e) / (min(1, 1 / C) + g * e))
    Shat_g = np.linalg.inv(Z.T @ dense(ops.Shat_inv) @ Z)
    lo, hi = gen_eig_range(Sg, Shat_g)
    assert lo >= f * (1 - 1e-9) and hi <= F * (1 + 1e-9)
    if gamma >= 1e5:
        assert 0.9 < lo and hi < 1.1


def test_exact_block_gives_triangular_spectrum():
    """Remark: with A_gamma inverted exactly, P K is block upper triangular with
    the identity and Shat_gamma^{-1} S_gamma on the diagonal (the oracle's
    BlockPreconditioner is pinned to the same dense factors in
    test_oracle_pins.py)."""
    gamma = 50.0
    ops, Z = setup(2, 3, gamma, schur=1)
    K = dense(ops.stokes())
    nu, npres = ops.level.n_u, ops.level.n_p
    Ainv = np.linalg.inv(dense(ops.Agamma))
    Sinv = dense(ops.Shat_inv)
    B = dense(ops.B)
    P = np.block([[np.eye(nu), -Ainv @ B.T], [np.zeros((npres, nu)), np.eye(npres)]]) @ \
        np.block([[Ainv, np.zeros((nu, npres))], [np.zeros((npres, nu)), -Sinv]]) @ \
        np.block([[np.eye(nu), np.zeros((nu, npres))], [-B @ Ainv, np.eye(npres)]])
    PK = P @ K
    assert np.abs(PK[:nu, :nu] - np.eye(nu)).max() < 1e-9
    assert np.abs(PK[nu:, :nu]).max() < 1e-9
    Sg = B @ Ainv @ B.T
    assert np.allclose(PK[nu:, nu:], Sinv @ Sg, atol=1e-9)


def test_upper_triangular_block_preconditioner():
    """The upper block-triangular variant with an exact inner solve equals the
    dense solve of [[A_gamma, B^T], [0, -Shat]] (pressure data chosen so that
    the mean projection is inactive), and as an FGMRES preconditioner it
    reaches the direct solution."""
    from types import SimpleNamespace
    import scipy.sparse.linalg as spla
    from oracle.krylov import BlockPreconditioner, StokesSolver
    from workloads import small
    gamma = 50.0
    ops, Z = setup(2, 3, gamma, schur=1)
    nu, npres = ops.level.n_u, ops.level.n_p
    A = dense(ops.Agamma)
    B = dense(ops.B)
    S = np.linalg.inv(dense(ops.Shat_inv))
    lu = spla.splu(ops.Agamma.tocsc())
    fake_mg = SimpleNamespace(ops=[ops], vcycle=lambda r: lu.solve(r))
    pc = BlockPreconditioner(fake_mg, "upper")
    rng = np.random.default_rng(3)
    p0 = ops.project_mean(rng.standard_normal(npres))
    v = np.concatenate([rng.standard_normal(nu), S @ p0])
    U = np.block([[A, B.T], [np.zeros((npres, nu)), -S]])
    assert np.allclose(pc.apply(v), np.linalg.solve(U, v), rtol=1e-9, atol=1e-11)
    wl = small(2, 8, 2, gamma=1e3, dr=1e4, n_sinkers=4, seed=3)
    st = StokesSolver(wl)
    from oracle.direct import solve_direct
    x_d = solve_direct(st.ops, st.ops.rhs())
    x, info = st.solve(rtol=1e-11, pc="upper")
    assert info["converged"]
    assert np.linalg.norm(x - x_d) <= 1e-8 * np.linalg.norm(x_d)
