"""Viscosity fields and forcing (oracle). Test infrastructure: see package docstring.

Multi-sinker benchmark (Section 5.2). The paper prints
    mu(x) = (mu_max - mu_min)(1 - chi(x)),
    chi(x) = prod_i [1 - exp(-delta max(0, |c_i - x| - omega/2))],
    f(x)   = (0, ..., beta (chi(x) - 1)).
Reading taken (the printed formula loses the floor mu_min and the square of
the Gaussian, so that mu would vanish far from all sinkers):
    mu(x)  = (mu_max - mu_min)(1 - chi(x)) + mu_min,
    chi(x) = prod_i [1 - exp(-delta max(0, |c_i - x| - omega/2)^2)].
Inside a sinker chi = 0 and mu = mu_max; far away chi -> 1 and mu -> mu_min.
In 2D the forcing is f = (0, beta (chi - 1)).

Viscoplastic Newton tensor (Section 5.3.1). The paper linearises
tau(eps) = 2 mu_eff(eps_II) eps with eps_II = (eps:eps / 2)^(1/2) and obtains a
fourth-order tensor viscosity. Reading taken for the synthetic workload: a
base field mu0(x) (the multi-sinker field) capped by a yield stress tau_y
above a floor mu_f (mu_min of the sinker field unless given),
    mu_eff = mu_f + min(mu0 - mu_f, tau_y / (2 eps_II)),
whose exact derivative is
    C = 2 mu_eff I - 2 (mu_eff - mu_f) [yielded] n (x) n,  n = eps / |eps|_F,
symmetric positive definite with smallest eigenvalue >= 2 mu_f. The strain
rate is that of a smooth Fourier velocity
    u_c(x) = s sum_{m in {1..M}^d} a_{c,m} / (1 + |m|^2) prod_j sin(pi m_j x_j),
with standard-normal amplitudes a (seeded) and s set so that the RMS of
eps_II over the finest level's quadrature points is 1; tau_y = 2 mu_max.
"""
from __future__ import annotations

import numpy as np


class SinkerField:
    """Scalar multi-sinker viscosity with the forcing that drives it."""

    kind = "scalar"

    def __init__(self, centers, mu_min: float, mu_max: float, omega: float = 0.1,
                 delta: float = 200.0, beta: float = 10.0):
        self.centers = np.asarray(centers, dtype=np.float64)
        self.dim = self.centers.shape[1]
        self.mu_min, self.mu_max = float(mu_min), float(mu_max)
        self.omega, self.delta, self.beta = float(omega), float(delta), float(beta)

    @classmethod
    def from_workload(cls, wl):
        from workloads import OMEGA, DELTA, BETA
        return cls(wl.centers(), wl.mu_min, wl.mu_max, OMEGA, DELTA, BETA)

    def chi(self, x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        out = np.ones(x.shape[:-1])
        for c in self.centers:
            dist = np.sqrt(np.sum((x - c) ** 2, axis=-1))
            s = np.maximum(0.0, dist - 0.5 * self.omega)
            out = out * (1.0 - np.exp(-self.delta * s * s))
        return out

    def mu(self, x: np.ndarray) -> np.ndarray:
        return (self.mu_max - self.mu_min) * (1.0 - self.chi(x)) + self.mu_min

    def force(self, x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        f = np.zeros(x.shape)
        f[..., -1] = self.beta * (self.chi(x) - 1.0)
        return f

    # Uniform interface used by the assembly
    def scalar_viscosity(self, x):
        """Scalar viscosity used in the Schur approximation M_p(1/mu)."""
        return self.mu(x)

    def stress_tensor(self, x):
        """Fourth-order C with sigma = C : eps; here C = 2 mu I (on symmetric eps)."""
        mu = self.mu(x)
        d = self.dim
        eye = np.eye(d)
        ident = 0.5 * (np.einsum("ac,bd->abcd", eye, eye) + np.einsum("ad,bc->abcd", eye, eye))
        return 2.0 * mu[..., None, None, None, None] * ident


class FourierVelocity:
    """Smooth random velocity u = s sum_m a_m/(1+|m|^2) prod_j sin(pi m_j x_j)."""

    def __init__(self, amplitudes: np.ndarray, scale: float = 1.0):
        self.a = np.asarray(amplitudes, dtype=np.float64)    # (d, M, ..., M)
        self.dim = self.a.shape[0]
        self.modes = self.a.shape[1]
        self.scale = float(scale)

    def grad(self, x: np.ndarray) -> np.ndarray:
        """Velocity gradient G[..., c, k] = d u_c / d x_k (analytic)."""
        x = np.asarray(x, dtype=np.float64)
        d, M = self.dim, self.modes
        ms = np.arange(1, M + 1)
        msq = np.zeros((M,) * d)
        for j in range(d):
            shape = [1] * d
            shape[j] = M
            msq = msq + (ms ** 2).reshape(shape)
        A = self.a / (1.0 + msq)[None]                               # (d, M, .., M)
        pts = x.reshape(-1, d)
        out = np.zeros((pts.shape[0], d, d))
        for p0 in range(0, pts.shape[0], 16384):
            P = pts[p0:p0 + 16384]
            S = np.sin(np.pi * ms[None, None, :] * P[:, :, None])    # (P, d, M)
            C = np.cos(np.pi * ms[None, None, :] * P[:, :, None]) * (np.pi * ms)
            for k in range(d):
                # factor of axis j: derivative (C) for j == k, value (S) otherwise;
                # sum over the modes one axis at a time, last axis first
                facs = [C[:, j, :] if j == k else S[:, j, :] for j in range(d)]
                Z = np.tensordot(facs[d - 1], A, axes=([1], [d]))     # (P, c, m_0 .. m_{d-2})
                for j in range(d - 2, -1, -1):
                    Z = np.einsum("pc...m,pm->pc...", Z, facs[j])
                out[p0:p0 + 16384, :, k] = Z
        return self.scale * out.reshape(x.shape[:-1] + (d, d))

    def strain_rate(self, x):
        g = self.grad(x)
        return 0.5 * (g + np.swapaxes(g, -1, -2))


def second_invariant(eps: np.ndarray) -> np.ndarray:
    """eps_II = (eps:eps / 2)^(1/2)."""
    return np.sqrt(0.5 * np.sum(eps * eps, axis=(-1, -2)))


def capped_law(eps: np.ndarray, mu0: np.ndarray, tau_y: float, mu_f: float):
    """The capped viscoplastic law at strain rates eps[..., d, d] over base
    viscosities mu0[...]: (mu_eff, C) with
        mu_eff = mu_f + min(mu0 - mu_f, tau_y / (2 eps_II)),
        C = 2 mu_eff I_sym - 2 (mu_eff - mu_f) [yielded] n (x) n,  n = eps/|eps|_F,
    the derivative of tau(eps) = 2 mu_eff(eps_II) eps (yielded: the cap is
    below mu0 - mu_f; eps = 0 never yields)."""
    eii = second_invariant(eps)
    with np.errstate(divide="ignore"):
        cap = np.where(eii > 0, tau_y / (2.0 * np.where(eii > 0, eii, 1.0)), np.inf)
    yielded = cap < (mu0 - mu_f)
    mu_eff = mu_f + np.minimum(mu0 - mu_f, cap)
    d = eps.shape[-1]
    eye = np.eye(d)
    ident = 0.5 * (np.einsum("ac,bd->abcd", eye, eye) + np.einsum("ad,bc->abcd", eye, eye))
    nrm = np.sqrt(np.sum(eps * eps, axis=(-1, -2)))
    n = eps / np.where(nrm > 0, nrm, 1.0)[..., None, None]
    C = 2.0 * mu_eff[..., None, None, None, None] * ident
    coef = 2.0 * (mu_eff - mu_f) * yielded
    C = C - coef[..., None, None, None, None] * np.einsum("...ab,...cd->...abcd", n, n)
    return mu_eff, C


class ViscoplasticNewton:
    """Newton tensor of tau(eps) = 2 mu_eff(eps_II) eps for the capped law."""

    kind = "tensor"

    def __init__(self, base: SinkerField, velocity: FourierVelocity, tau_y: float, mu_floor: float = 0.0):
        self.base, self.vel, self.tau_y = base, velocity, float(tau_y)
        self.dim = base.dim
        # the floor of the capped law (mu_f); mu_min of the base field unless given
        self.mu_min = float(mu_floor) if mu_floor > 0.0 else base.mu_min

    @classmethod
    def from_workload(cls, wl, fine_quad_points: np.ndarray):
        base = SinkerField.from_workload(wl)
        vel = FourierVelocity(wl.fourier_amplitudes(), 1.0)
        eii = second_invariant(vel.strain_rate(fine_quad_points))
        vel.scale = 1.0 / np.sqrt(np.mean(eii ** 2))
        tau_y = getattr(wl, "tau_y", 0.0)
        return cls(base, vel, tau_y if tau_y > 0 else 2.0 * wl.mu_max, getattr(wl, "mu_floor", 0.0))

    def yielded(self, x):
        """Where the cap is active (tau_y / (2 eps_II) < mu0 - mu_f)."""
        eii = second_invariant(self.vel.strain_rate(x))
        with np.errstate(divide="ignore"):
            cap = np.where(eii > 0, self.tau_y / (2.0 * np.where(eii > 0, eii, 1.0)), np.inf)
        return cap < self.base.mu(x) - self.mu_min

    def mu_eff(self, x):
        return capped_law(self.vel.strain_rate(x), self.base.mu(x), self.tau_y, self.mu_min)[0]

    def scalar_viscosity(self, x):
        """The scalar in front of the tensor, used for M_p(1/mu) (Section 5.3.2)."""
        return self.mu_eff(x)

    def stress_tensor(self, x):
        return capped_law(self.vel.strain_rate(x), self.base.mu(x), self.tau_y, self.mu_min)[1]

    def stress(self, eps: np.ndarray, x: np.ndarray) -> np.ndarray:
        """tau(eps) = 2 mu_eff(eps_II) eps at positions x (for derivative checks)."""
        mu_eff = capped_law(eps, self.base.mu(x), self.tau_y, self.mu_min)[0]
        return 2.0 * mu_eff[..., None, None] * eps
