"""Pins of the oracle's robust multigrid pieces (Section 4): kernel
decomposition of the vertex stars, gamma-robust spectral equivalence of the
star smoother, the robust prolongation's divergence and energy properties,
and the GMRES relaxation against a brute-force Krylov minimisation."""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla

from oracle.fem import Level
from oracle.assembly import Operators
from oracle.coefficients import SinkerField
from oracle.multigrid import (StarASM, RobustTransfer, star_patch_dofs, all_vertices,
                              coarse_cell_dofs, gmres_relax, Multigrid)


def sinker(dim, dr=1.0, seed=0):
    rng = np.random.default_rng(seed)
    return SinkerField(rng.random((2, dim)), dr ** -0.5, dr ** 0.5, omega=0.3)


@pytest.mark.parametrize("dim,n", [(2, 4), (3, 2)])
def test_kernel_decomposition_vertex_stars(dim, n):
    """eq. (kdp): N_h = sum_i (V_i cap N_h) for the vertex stars of eq. (viim);
    a decomposition into cell interiors (which misses the vertex-centred
    unknowns) does not have it."""
    lv = Level(dim, n)
    ops = Operators(lv, sinker(dim), gamma=1.0)
    B = ops.B.toarray()
    dim_kernel = lv.n_u - np.linalg.matrix_rank(B)

    def span_rank(patches):
        cols = []
        for idx in patches:
            ns = sla.null_space(B[:, idx])
            for v in ns.T:
                full = np.zeros(lv.n_u)
                full[idx] = v
                cols.append(full)
        return np.linalg.matrix_rank(np.array(cols).T) if cols else 0

    stars = [star_patch_dofs(lv, v) for v in all_vertices(lv)]
    assert span_rank([s for s in stars if s.size]) == dim_kernel
    # negative control: patches = interior nodes of single cells (2i+1)
    cells = []
    for c in itertools.product(range(n), repeat=dim):
        node = np.array([[2 * ci + 1 for ci in c]])
        cells.append(np.array([lv.u_dof(k, node)[0] for k in range(dim)]))
    assert span_rank(cells) < dim_kernel


def test_patch_sizes():
    """Star interiors hold d*3^d unknowns (18 in 2D, 81 in 3D) at interior
    vertices and fewer at boundary vertices."""
    for dim, n, sizes in [(2, 4, {18, 6, 2}), (3, 4, {81, 27, 9, 3})]:
        lv = Level(dim, n)
        got = {star_patch_dofs(lv, v).size for v in all_vertices(lv)}
        assert got == sizes


def test_center_patch_is_coarse_cell_interior():
    """The local problem of a coarse cell (fine unknowns strictly inside it)
    is the star patch of the fine vertex at the cell centre."""
    for dim in (2, 3):
        fine = Level(dim, 4)
        for cc in itertools.product(range(2), repeat=dim):
            centre = np.array([2 * c + 1 for c in cc])
            assert np.array_equal(coarse_cell_dofs(fine, cc), star_patch_dofs(fine, centre))


@pytest.mark.parametrize("dim,n", [(2, 4), (3, 2)])
def test_star_smoother_gamma_robust(dim, n):
    """Section 4.1: D_{h,gamma} is spectrally equivalent to A_{h,gamma} with
    gamma-independent constants; point Jacobi loses a factor ~gamma."""
    lv = Level(dim, n)
    lam_star, lam_jac = [], []
    for gamma in (1e2, 1e4, 1e6):
        A = Operators(lv, sinker(dim, 1e2), gamma=gamma).Agamma
        Ad = A.toarray()
        asm = StarASM(lv, A)
        D = np.column_stack([asm.apply(e) for e in np.eye(lv.n_u)])
        # D^{-1} is SPD; generalized eigenvalues of A x = lam D^{-1}... via D A
        ev = np.sort(np.real(np.linalg.eigvals(D @ Ad)))
        lam_star.append(ev[0])
        evj = np.sort(np.real(np.linalg.eigvals(Ad / np.diag(Ad)[:, None])))
        lam_jac.append(evj[0])
    assert lam_star[2] > 0.5 * lam_star[1] > 0.0
    assert lam_jac[2] < 0.05 * lam_jac[1]
    # largest eigenvalue is bounded by the number of overlapping stars (2^d)
    assert ev[-1] <= 2 ** dim * (1 + 1e-9)


@pytest.mark.parametrize("dim,nc", [(2, 2), (3, 2)])
def test_robust_prolongation_properties(dim, nc):
    """Section 4.2: (1) P~ maps coarse discretely divergence-free fields to
    fine fields whose divergence decays like 1/gamma, while P_H does not;
    (2) energy continuity eq. (conP) with a gamma-independent constant;
    (3) Lemma P(b)/(d): coarse-cell means of the divergence are preserved;
    (4) the restriction is the transpose."""
    coarse, fine = Level(dim, nc), Level(dim, 2 * nc)
    coef = sinker(dim, 1.0)
    divs, ratios = [], []
    for gamma in (1e2, 1e4, 1e6):
        oc, of = Operators(coarse, coef, gamma), Operators(fine, coef, gamma)
        T = RobustTransfer(coarse, fine, of)
        kerH = sla.null_space(oc.B.toarray())
        uH = kerH @ np.random.default_rng(4).standard_normal(kerH.shape[1])
        Wih = np.sqrt(of.Winv.diagonal())
        div_t = np.linalg.norm(Wih * (of.B @ T.prolong(uH)))
        div_s = np.linalg.norm(Wih * (of.B @ (T.P @ uH)))
        divs.append((div_t, div_s))
        Pt = np.column_stack([T.prolong(e) for e in np.eye(coarse.n_u)])
        ratios.append(sla.eigh(Pt.T @ of.Agamma.toarray() @ Pt, oc.Agamma.toarray(),
                               eigvals_only=True)[-1])
        # cell means of the divergence: sum of fine psi_0 rows inside each coarse cell
        x = np.random.default_rng(5).standard_normal(coarse.n_u)
        Bf0 = (of.B @ T.prolong(x))[0::dim + 1].reshape((fine.n,) * dim)
        Bc0 = (oc.B @ x)[0::dim + 1].reshape((coarse.n,) * dim)
        agg = Bf0
        for ax in range(dim):
            agg = agg.reshape(agg.shape[:ax] + (coarse.n, 2) + agg.shape[ax + 1:]).sum(axis=ax + 1)
        assert np.allclose(agg, Bc0, atol=1e-12 * np.abs(Bf0).max())
        R = np.column_stack([T.restrict(e) for e in np.eye(fine.n_u)])
        assert np.abs(R - Pt.T).max() <= 1e-9 * np.abs(Pt).max()
    assert divs[1][0] < 0.02 * divs[0][0] and divs[2][0] < 0.02 * divs[1][0]
    assert divs[2][1] > 0.5 * divs[0][1]
    assert max(ratios) < 4.0


def test_gmres_relax_minimises_true_residual():
    """Brute force: the relaxation result minimises ||b - A x|| over
    x0 + Dinv span{r0, A Dinv r0, ..., (A Dinv)^{nu-1} r0}."""
    rng = np.random.default_rng(0)
    n = 30
    M = rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)
    Dm = np.diag(1 / np.diag(A)) + 0.01 * np.eye(n)
    b, x0 = rng.standard_normal(n), rng.standard_normal(n)
    for nu in (1, 2, 3):
        x = gmres_relax(A, lambda r: Dm @ r, b, x0, nu)
        r0 = b - A @ x0
        K = [r0]
        for _ in range(nu - 1):
            K.append(A @ (Dm @ K[-1]))
        DK = Dm @ np.column_stack(K)
        c, *_ = np.linalg.lstsq(A @ DK, r0, rcond=None)
        assert np.linalg.norm(x - (x0 + DK @ c)) <= 1e-12 * np.linalg.norm(x)
    assert np.array_equal(gmres_relax(A, lambda r: Dm @ r, np.zeros(n), None, 2), np.zeros(n))


def test_vcycle_gamma_robust_iterations():
    """Section 4 / table fig:topleftsolve: with the robust smoother and
    transfer, V-cycle-preconditioned FGMRES on A_gamma needs about the same
    iterations for gamma from 1 to 1e4; the standard transfer degrades."""
    from oracle.krylov import fgmres
    its = {}
    for robust in (True, False):
        for gamma in (1.0, 1e2, 1e4):
            mg = Multigrid(2, 8, 2, sinker(2, 1e2), gamma, nu_pre=2, nu_post=2, robust=robust)
            A = mg.ops[-1].Agamma
            b = mg.ops[-1].rhs()
            _, info = fgmres(lambda v: A @ v, mg.vcycle, b, rtol=1e-8, restart=30, maxit=60)
            its[(robust, gamma)] = info["iters"]
    assert max(its[(True, g)] for g in (1.0, 1e2, 1e4)) <= its[(True, 1.0)] + 6
    assert its[(False, 1e4)] >= 2 * its[(True, 1e4)]


@pytest.mark.parametrize("dim,n", [(2, 4), (3, 2)])
def test_fcycle_two_level_without_relaxation(dim, n):
    """With no relaxation (nu = 0) the two-level F-cycle is two steps of the
    coarse-grid-correction iteration x <- x + M (b - A x) from x = 0, with
    M = P~ A_0^{-1} P~^T: the coarse solve of the restricted b, prolongated,
    then one V-cycle from that start. Ignoring the start (a V-cycle from
    zero) would give one step, M b."""
    mg = Multigrid(dim, n, 2, sinker(dim, 1e2, seed=3), 50.0, nu_pre=0, nu_post=0)
    A = mg.ops[1].Agamma
    b = np.random.default_rng(1).standard_normal(A.shape[0])

    def M(r):
        return mg.prolong(1, mg.coarse_lu.solve(mg.restrict(1, r)))

    x1 = M(b)
    x2 = x1 + M(b - A @ x1)
    f = mg.fcycle(b)
    assert np.linalg.norm(f - x2) <= 1e-10 * np.linalg.norm(x2)
    assert np.linalg.norm(f - x1) > 1e-3 * np.linalg.norm(x2)


def test_fcycle_with_exact_relaxation_is_exact():
    """GMRES relaxation with as many steps as unknowns solves the level
    exactly, so the F-cycle (like the V-cycle) returns A_gamma^{-1} b."""
    mg = Multigrid(2, 2, 2, sinker(2, 1e2, seed=4), 10.0, nu_pre=18, nu_post=18)
    A = mg.ops[1].Agamma
    b = np.random.default_rng(2).standard_normal(A.shape[0])
    x = np.linalg.solve(A.toarray(), b)
    assert np.linalg.norm(mg.fcycle(b) - x) <= 1e-9 * np.linalg.norm(x)


def test_fcycle_three_levels_preconditions_like_the_v_cycle():
    """On three levels the F-cycle is a better approximate inverse than the
    V-cycle it ends with: FGMRES on A_gamma needs at most as many iterations
    (the coarse levels see a V-cycle of their own before the finest one)."""
    from oracle.krylov import fgmres
    mg = Multigrid(2, 16, 3, sinker(2, 1e4, seed=5), 1e3, nu_pre=2, nu_post=2)
    A = mg.ops[-1].Agamma
    b = mg.ops[-1].rhs()
    _, iv = fgmres(lambda v: A @ v, mg.vcycle, b, rtol=1e-8, restart=30, maxit=60)
    _, jf = fgmres(lambda v: A @ v, mg.fcycle, b, rtol=1e-8, restart=30, maxit=60)
    assert iv["converged"] and jf["converged"]
    assert jf["iters"] <= iv["iters"]
