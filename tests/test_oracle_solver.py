"""Pins of the oracle's full solver: convergence to the direct solution of the
bordered saddle-point system, manufactured-solution convergence rates of the
discretisation (forcing computed by automatic differentiation, independent of
the finite element code), the FGMRES routine, and the viscoplastic Newton tensor."""
import numpy as np
import pytest
import torch

from workloads import CONFIGS, small
from oracle.fem import Level, lagrange_1d, gauss_legendre_01, unlex
from oracle.assembly import Operators
from oracle.coefficients import SinkerField, ViscoplasticNewton, FourierVelocity, second_invariant
from oracle.direct import solve_direct
from oracle.krylov import StokesSolver, fgmres


def test_fgmres_routine_on_small_system():
    rng = np.random.default_rng(1)
    n = 40
    K = rng.standard_normal((n, n)) + 8 * np.eye(n)
    b = rng.standard_normal(n)
    Minv = np.linalg.inv(np.diag(np.diag(K)))
    x, info = fgmres(lambda v: K @ v, lambda v: Minv @ v, b, rtol=1e-12, restart=7, maxit=200)
    assert info["converged"]
    assert np.linalg.norm(x - np.linalg.solve(K, b)) <= 1e-10 * np.linalg.norm(x)
    # the recorded estimate after the last iteration is the true residual
    assert info["rel_res"] <= 1e-12


@pytest.mark.parametrize("wl", [CONFIGS["sinker_2d_16sq_L2"], small(3, 4, 2, gamma=1e3, dr=1e4, n_sinkers=3)],
                         ids=["sinker_2d_16sq_L2", "3d_4cu"])
def test_fgmres_solution_matches_direct(wl):
    s = StokesSolver(wl)
    x, info = s.solve()
    assert info["converged"] and info["rel_res"] <= wl.rtol
    # iterate further: the limit is the direct solution of the bordered system
    x, info = s.solve(rtol=1e-11)
    assert info["converged"]
    xd = solve_direct(s.ops, s.ops.rhs())
    nu = s.ops.level.n_u
    err_u = np.linalg.norm(x[:nu] - xd[:nu]) / np.linalg.norm(xd[:nu])
    err = np.linalg.norm(x - xd) / np.linalg.norm(xd)
    assert err_u < 1e-9 and err < 1e-8, (err_u, err)
    # the discrete solution is (weakly) divergence free
    assert np.linalg.norm(s.ops.B @ xd[:nu]) < 1e-9 * np.linalg.norm(s.ops.rhs())


def test_iterations_fall_with_gamma_exact_block():
    """table:exacttopleft trend: with the (1,1) block solved exactly the
    iteration count decreases as gamma grows (Section 3)."""
    import scipy.sparse.linalg as spla
    its = []
    for gamma in (0.0, 10.0, 1e3):
        wl = small(2, 16, 2, gamma=gamma, dr=1e4, n_sinkers=6)
        ops = Operators(Level(2, 16), SinkerField.from_workload(wl), gamma)
        lu = spla.splu(ops.Agamma.tocsc())
        K = ops.stokes()
        nu = ops.level.n_u

        def pc(v):
            y = lu.solve(v[:nu])
            zp = ops.project_mean(-(ops.Shat_inv @ (v[nu:] - ops.B @ y)))
            return np.concatenate([y - lu.solve(ops.B.T @ zp), zp])
        b = np.concatenate([ops.rhs(), np.zeros(ops.level.n_p)])
        _, info = fgmres(lambda v: K @ v, pc, b, rtol=1e-6, maxit=200)
        its.append(info["iters"])
    assert its[0] > its[1] > its[2]
    assert its[2] <= 5


# --------------------------------------------------------------------------- manufactured solution
def _mms_fields():
    def psi(x, y):
        return (x * (1 - x) * y * (1 - y)) ** 2

    def mu(x, y):
        return 1.0 + 0.5 * torch.sin(2 * np.pi * x) * torch.cos(np.pi * y)

    def p(x, y):
        return torch.cos(np.pi * x) * torch.cos(np.pi * y)

    def vel(x, y):
        s = psi(x, y).sum()
        gx, gy = torch.autograd.grad(s, (x, y), create_graph=True)
        return gy, -gx

    def force(pts):
        x = torch.tensor(pts[:, 0], requires_grad=True)
        y = torch.tensor(pts[:, 1], requires_grad=True)
        u = vel(x, y)
        G = [[None, None], [None, None]]
        for a in range(2):
            ga = torch.autograd.grad(u[a].sum(), (x, y), create_graph=True)
            G[a] = list(ga)
        m = mu(x, y)
        pp = p(x, y)
        dp = torch.autograd.grad(pp.sum(), (x, y), create_graph=True)
        f = []
        for a in range(2):
            div_sig = 0
            for b, var in enumerate((x, y)):
                sig_ab = m * (G[a][b] + G[b][a])
                div_sig = div_sig + torch.autograd.grad(sig_ab.sum(), var, create_graph=True)[0]
            f.append((-div_sig + dp[a]).detach().numpy())
        return np.stack(f, -1)

    def exact(pts):
        x = torch.tensor(pts[:, 0], requires_grad=True)
        y = torch.tensor(pts[:, 1], requires_grad=True)
        u = vel(x, y)
        return np.stack([u[0].detach().numpy(), u[1].detach().numpy()], -1), \
            p(x, y).detach().numpy()

    return mu, force, exact


class _MMSCoef:
    kind = "scalar"

    def __init__(self):
        self._mu, self._force, _ = _mms_fields()

    def mu(self, x):
        sh = x.shape[:-1]
        pts = torch.tensor(x.reshape(-1, 2))
        return self._mu(pts[:, 0], pts[:, 1]).numpy().reshape(sh)

    scalar_viscosity = mu

    def force(self, x):
        return self._force(x.reshape(-1, 2)).reshape(x.shape)


@pytest.mark.slow
def test_manufactured_solution_rates():
    """Inf-sup stable [Q2]^2 x P1disc: ||u - u_h||_0 = O(h^3), ||p - p_h||_0 = O(h^2)."""
    _, _, exact = _mms_fields()
    g5, w5 = gauss_legendre_01(5)
    val, _ = lagrange_1d(g5)
    eu, ep = [], []
    for n in (4, 8, 16):
        lv = Level(2, n)
        ops = Operators(lv, _MMSCoef(), gamma=1.0)
        sol = solve_direct(ops, ops.rhs())
        u, p = sol[:lv.n_u], sol[lv.n_u:]
        ed = lv.element_dofs()
        cells = lv.cells()
        err_u = err_p = 0.0
        for qy in range(5):
            for qx in range(5):
                xi = np.array([g5[qx], g5[qy]])
                pts = lv.h * (cells + xi)
                ue, pe = exact(pts)
                phi = np.array([val[qx, a] * val[qy, b] for b in range(3) for a in range(3)])
                uh = np.zeros((lv.n_cells, 2))
                for c in range(2):
                    dofs = ed[:, c * 9:(c + 1) * 9]
                    vals = np.where(dofs >= 0, u[np.maximum(dofs, 0)], 0.0)
                    uh[:, c] = vals @ phi
                pk = p.reshape(-1, 3)
                ph = pk[:, 0] + pk[:, 1] * (xi[0] - 0.5) + pk[:, 2] * (xi[1] - 0.5)
                wq = w5[qx] * w5[qy] * lv.h ** 2
                err_u += wq * np.sum((uh - ue) ** 2)
                err_p += wq * np.sum((ph - pe) ** 2)
        eu.append(np.sqrt(err_u))
        ep.append(np.sqrt(err_p))
    ru = np.log2(np.array(eu[:-1]) / np.array(eu[1:]))
    rp = np.log2(np.array(ep[:-1]) / np.array(ep[1:]))
    assert ru[-1] > 2.7, (eu, ru)
    assert rp[-1] > 1.8, (ep, rp)


# --------------------------------------------------------------------------- viscoplastic tensor
def _vp(dim=3):
    wl = CONFIGS["viscoplastic_3d_48cu_L3"]
    lv = Level(dim, 4)
    base = SinkerField(np.random.default_rng(0).random((4, dim)), 1e-5, 1e5, omega=0.3)
    vel = FourierVelocity(np.random.default_rng(1).standard_normal((dim,) + (3,) * dim), 1.0)
    eii = second_invariant(vel.strain_rate(lv.quad_points()))
    vel.scale = 1.0 / np.sqrt(np.mean(eii ** 2))
    return ViscoplasticNewton(base, vel, 2.0 * base.mu_max), lv


def test_newton_tensor_is_derivative_of_stress():
    """C = d tau / d eps for tau = 2 mu_eff(eps_II) eps (central differences)."""
    law, lv = _vp()
    x = lv.quad_points().reshape(-1, 3)[::7]
    eps0 = law.vel.strain_rate(x)
    C = law.stress_tensor(x)
    h = 1e-6
    for a in range(3):
        for b in range(a, 3):
            dE = np.zeros((3, 3))
            dE[a, b] += 0.5
            dE[b, a] += 0.5
            fd = (law.stress(eps0 + h * dE, x) - law.stress(eps0 - h * dE, x)) / (2 * h)
            an = np.einsum("pijkl,kl->pij", C, dE)
            scale = np.abs(C).reshape(len(x), -1).max(axis=1)[:, None, None]
            assert np.all(np.abs(fd - an) <= 1e-5 * scale)


def test_newton_tensor_spd_and_scalar_limit():
    law, lv = _vp()
    x = lv.quad_points().reshape(-1, 3)
    C = law.stress_tensor(x)
    # as an operator on symmetric tensors (Mandel basis) it is SPD with eigenvalues >= 2 mu_min
    idx = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    wts = [1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)]
    Mm = np.zeros((len(x), 6, 6))
    for i, (a, b) in enumerate(idx):
        for j, (c, d) in enumerate(idx):
            Mm[:, i, j] = wts[i] * wts[j] * C[:, a, b, c, d]
    assert np.abs(Mm - np.swapaxes(Mm, 1, 2)).max() <= 1e-12 * np.abs(Mm).max()
    ev = np.linalg.eigvalsh(Mm)
    assert ev.min() >= 2 * law.mu_min - 1e-14 * ev.max()
    mu_eff, yielded = law.mu_eff(x), law.yielded(x)
    assert yielded.any() and (~yielded).any()
    # where nothing yields the tensor is 2 mu I
    iso = Mm[~yielded]
    assert np.allclose(iso, 2 * mu_eff[~yielded][:, None, None] * np.eye(6), rtol=1e-12, atol=0)


@pytest.mark.parametrize("dim", [2, 3])
def test_fourier_gradient_against_brute_force(dim):
    """The mode-by-mode contraction of the Fourier velocity gradient equals
    the plain sum over all modes (written out here term by term) and the
    central difference of the velocity itself."""
    M = 3
    a = np.random.default_rng(5).standard_normal((dim,) + (M,) * dim)
    vel = FourierVelocity(a, 0.7)
    x = np.random.default_rng(6).random((5, dim))

    def u(p):
        out = np.zeros(dim)
        for m in np.ndindex(*(M,) * dim):
            mm = np.array(m) + 1
            prod = np.prod(np.sin(np.pi * mm * p))
            out += a[(slice(None),) + m] / (1.0 + np.sum(mm ** 2)) * prod
        return 0.7 * out

    G = vel.grad(x)
    for i, p in enumerate(x):
        ref = np.zeros((dim, dim))
        for m in np.ndindex(*(M,) * dim):
            mm = np.array(m) + 1
            for k in range(dim):
                f = np.prod([np.pi * mm[j] * np.cos(np.pi * mm[j] * p[j]) if j == k else np.sin(np.pi * mm[j] * p[j])
                             for j in range(dim)])
                ref[:, k] += 0.7 * a[(slice(None),) + m] / (1.0 + np.sum(mm ** 2)) * f
        assert np.allclose(G[i], ref, rtol=1e-13, atol=1e-13)
        h = 1e-6
        for k in range(dim):
            e = np.zeros(dim)
            e[k] = h
            fd = (u(p + e) - u(p - e)) / (2 * h)
            assert np.allclose(G[i][:, k], fd, rtol=1e-7, atol=1e-7)
