"""Seeded synthetic workloads for the augmented-Lagrangian Stokes multigrid.

This module is the only code shared by the CPU oracle and the GPU path. It
holds workload *descriptions* and the random numbers they draw (sinker
centres, Fourier amplitudes, request arrival times); it holds none of the
method's arithmetic (no basis functions, no viscosity law, no operators).

Workloads follow the multi-sinker benchmark of Section 5.2 (Rudi-Stadler-
Ghattas setup): unit square/cube, homogeneous Dirichlet walls, n sinkers of
diameter omega with Gaussian-smoothed edges (parameter delta), contrast
DR = mu_max/mu_min with mu_max = DR^(1/2), mu_min = DR^(-1/2), forcing
strength beta. The paper draws the sinker centres "randomly" without a
distribution or seed; here they are uniform on [0,1)^d from numpy's PCG64
generator with the seed stored in the workload.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

OMEGA = 0.1     # sinker diameter (Section 5.2)
DELTA = 200.0   # edge smoothing parameter (Section 5.2)
BETA = 10.0     # forcing strength (Section 5.2)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One Stokes solve: mesh hierarchy, coefficient field and solver knobs."""
    name: str
    dim: int              # 2 or 3
    n_fine: int           # cells per axis on the finest level
    levels: int           # number of multigrid levels (level 0 = coarsest)
    n_sinkers: int
    dr: float             # dynamic ratio mu_max / mu_min
    gamma: float          # augmented-Lagrangian parameter
    seed: int             # seed for the sinker centres
    nu_pre: int = 2       # GMRES-accelerated ASM steps before coarse correction
    nu_post: int = 2      # ... and after
    restart: int = 30     # FGMRES restart length
    rtol: float = 1e-8    # relative residual target ||b - Kx|| <= rtol ||b||
    maxit: int = 300
    coef_kind: int = 0    # 0 = scalar sinker viscosity, 1 = viscoplastic Newton tensor at the
                          # Fourier velocity, 2 = viscoplastic problem solved by Newton's method
    fourier_seed: Optional[int] = None   # seed of the Fourier velocity (coef_kind 1)
    fourier_modes: int = 8               # modes per axis (coef_kind 1)
    schur: int = 1        # W in A_gamma: 1 = M_p (preconditioner P1), 2 = M_p(1/mu) (P2)
    mu_floor: float = 0.0  # floor of the capped viscoplastic law (coef_kind 1, 2); 0 selects mu_min
    tau_y: float = 0.0     # yield stress of the capped law; 0 selects 2 mu_max (coef_kind 1)
    cycle: str = "V"       # multigrid cycle of the block preconditioner: "V" or "F"
    degree: int = 2        # velocity degree k of [Q_k]^d x P_{k-1}^disc (2 or 3)

    @property
    def mu_max(self) -> float:
        return math.sqrt(self.dr)

    @property
    def mu_min(self) -> float:
        return 1.0 / math.sqrt(self.dr)

    def n_level(self, level: int) -> int:
        """Cells per axis on `level` (0 = coarsest)."""
        return self.n_fine >> (self.levels - 1 - level)

    def centers(self) -> np.ndarray:
        """Sinker centres, shape (n_sinkers, dim), uniform on [0,1)^dim."""
        return sinker_centers(self.n_sinkers, self.dim, self.seed)

    def fourier_amplitudes(self) -> np.ndarray:
        """Standard-normal amplitudes a[c, m_1..m_d] for the Fourier velocity."""
        assert self.fourier_seed is not None
        return fourier_amplitudes(self.dim, self.fourier_modes, self.fourier_seed)

    def unknowns(self) -> Tuple[int, int]:
        """(interior velocity unknowns, pressure unknowns) on the finest level."""
        d, n, k = self.dim, self.n_fine, self.degree
        n_pb = math.comb(k - 1 + d, d)       # monomials of total degree <= k-1
        return d * (k * n - 1) ** d, n_pb * n ** d


def sinker_centers(n: int, dim: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).random((n, dim))


def fourier_amplitudes(dim: int, modes: int, seed: int) -> np.ndarray:
    shape = (dim,) + (modes,) * dim
    return np.random.default_rng(seed).standard_normal(shape)


CONFIGS = {
    # 2D 16x16, 2 levels, V(2,2), gamma 1e2, 4 sinkers, DR 1e2
    "sinker_2d_16sq_L2": Workload("sinker_2d_16sq_L2", 2, 16, 2, 4, 1e2, 1e2, 101),
    # 2D 128x128, 4 levels, 16 sinkers, DR 1e6, gamma 1e3, FGMRES(30) to 1e-8
    "sinker_2d_128sq_L4": Workload("sinker_2d_128sq_L4", 2, 128, 4, 16, 1e6, 1e3, 201),
    # 3D 32^3, 3 levels, 24 sinkers, DR 1e8, gamma 1e4
    "sinker_3d_32cu_L3": Workload("sinker_3d_32cu_L3", 3, 32, 3, 24, 1e8, 1e4, 301),
    # 3D 48^3, 3 levels, viscoplastic Newton tensor over a 24-sinker base field, DR 1e10
    "viscoplastic_3d_48cu_L3": Workload("viscoplastic_3d_48cu_L3", 3, 48, 3, 24, 1e10, 1e4, 401,
                   coef_kind=1, fourier_seed=402),
}


# Settings of the paper's two tables of Q2 iteration counts, run with its
# solver options: preconditioner P2 (W = M_p(1/mu)), 5 pre- and 5
# post-relaxation steps, F-cycles, FGMRES(30) to a 1e6 residual reduction.
# Sinker centres are seeded here (the paper's are not published), so the
# comparison with the printed counts is qualitative.
PAPER_VANKA_AL = {   # table "vanka", AL column: 2D 128^2, 4 levels, gamma 100
    (ns, dr): Workload(f"vanka_al_{ns}s_dr{dr:g}", 2, 128, 4, ns, dr, 100.0, 600 + ns, nu_pre=5, nu_post=5,
                       rtol=1e-6, schur=2, cycle="F")
    for ns in (1, 6, 24) for dr in (1e4, 1e6, 1e8, 1e10)}
PAPER_VANKA_AL_PRINTED = {(1, 1e4): 4, (1, 1e6): 6, (1, 1e8): 8, (1, 1e10): 9,
                          (6, 1e4): 10, (6, 1e6): 14, (6, 1e8): 16, (6, 1e10): 16,
                          (24, 1e4): 9, (24, 1e6): 15, (24, 1e8): 20, (24, 1e10): 25}
# table "k", k = 2 column (robust smoother and transfer): 3D 30^3, 2 levels,
# contrast 1e6; the paper's sinker count for this table is not stated: 24
PAPER_K2 = {g: Workload(f"k2_30cu_g{g:g}", 3, 30, 2, 24, 1e6, g, 700, nu_pre=5, nu_post=5, rtol=1e-6,
                        schur=2, cycle="F") for g in (0.0, 10.0, 1000.0)}
PAPER_K2_PRINTED = {0.0: 95, 10.0: 28, 1000.0: 27}
# the same settings on a 12^3 mesh (2 levels), where the oracle solves in minutes
PAPER_K2_SMALL = {g: Workload(f"k2_12cu_g{g:g}", 3, 12, 2, 24, 1e6, g, 700, nu_pre=5, nu_post=5, rtol=1e-6,
                              schur=2, cycle="F") for g in (0.0, 10.0, 1000.0)}


# table "linear", 2D (robust smoother and transfer): [Q3]^2 x P2disc on the
# 2D 128^2 mesh with 4 levels, 24 sinkers, F-cycles with 5 pre- and 5
# post-relaxation steps, FGMRES(30) to a 1e6 residual reduction, P1 and P2
PAPER_LINEAR_Q3 = {(schur, g, dr): Workload(f"linear_q3_p{schur}_g{g:g}_dr{dr:g}", 2, 128, 4, 24, dr, g, 800,
                                            nu_pre=5, nu_post=5, rtol=1e-6, schur=schur, cycle="F", degree=3)
                   for schur in (1, 2) for g in (10.0, 1000.0) for dr in (1e6, 1e10)}
PAPER_LINEAR_Q3_PRINTED = {(1, 10.0, 1e6): 11, (1, 10.0, 1e10): 22, (1, 1000.0, 1e6): 13, (1, 1000.0, 1e10): 15,
                           (2, 10.0, 1e6): 19, (2, 10.0, 1e10): 27, (2, 1000.0, 1e6): 12, (2, 1000.0, 1e10): 16}
# the same table's 3D settings (contrast 1e8, P1 and P2, gamma 10 / 1000) on
# 8^3 cells with 2 levels: the paper's 80^3 with 3 levels is beyond the
# explicit 375-unknown patch inverses (its finest level alone would take
# about 320 GB)
PAPER_LINEAR_Q3_3D = {(schur, g): Workload(f"linear_q3_3d_p{schur}_g{g:g}", 3, 8, 2, 24, 1e8, g, 810, nu_pre=5,
                                           nu_post=5, rtol=1e-6, schur=schur, cycle="F", degree=3)
                      for schur in (1, 2) for g in (10.0, 1000.0)}
PAPER_LINEAR_Q3_3D_PRINTED = {(1, 10.0): 15, (1, 1000.0): 14, (2, 10.0): 15, (2, 1000.0): 14}
# the 3D degree-3 benchmark setting: the same solver options on 16^3 cells
# with 3 levels (P1, gamma 1000), the largest mesh whose setup stays well
# under a second
Q3_3D_BENCH = Workload("q3_3d_16cu_L3", 3, 16, 3, 24, 1e8, 1000.0, 810, nu_pre=5, nu_post=5, rtol=1e-6, schur=1,
                       cycle="F", degree=3)


# Viscoplastic Newton problems (capped law over a multi-sinker base field,
# solved from rest): 8 sinkers, contrast 1e4; tau_y is about the 90th
# percentile of 2 mu0 eps_II of the first (Newtonian) iterate, so roughly a
# tenth of the domain yields at the start.
NEWTON = {
    "newton_2d_32sq_L3": Workload("newton_2d_32sq_L3", 2, 32, 3, 8, 1e4, 1e3, 503, coef_kind=2, tau_y=1.0),
    "newton_3d_8cu_L2": Workload("newton_3d_8cu_L2", 3, 8, 2, 8, 1e4, 1e4, 504, coef_kind=2, tau_y=0.12),
    "newton_3d_32cu_L3": Workload("newton_3d_32cu_L3", 3, 32, 3, 8, 1e4, 1e4, 504, coef_kind=2, tau_y=0.12),
}


def small(dim: int, n_fine: int, levels: int, *, n_sinkers: int = 4, dr: float = 1e2,
          gamma: float = 1e2, seed: int = 7, **kw) -> Workload:
    """A small workload for tests, same recipe as the named configurations."""
    name = f"t{dim}d_{n_fine}_L{levels}_g{gamma:g}_dr{dr:g}_s{seed}"
    return Workload(name, dim, n_fine, levels, n_sinkers, dr, gamma, seed, **kw)


def serving_stream(n_requests: int = 200, rate_hz: float = 20.0, seed: int = 501):
    """Poisson stream of mixed 2D/3D requests: list of (arrival_s, Workload).

    Each request is 2D or 3D with probability 1/2; N is uniform over
    {32,64,128,256} (2D) or {8,16,32} (3D); the contrast is log-uniform in
    [1e4, 1e8]; 24 sinkers seeded by 10^6 + i. Coarsest mesh 16^2 in 2D,
    8^3 in 3D (4^3 for an 8^3 request); gamma 1e3 (2D) / 1e4 (3D).
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        dim = 2 if rng.random() < 0.5 else 3
        if dim == 2:
            n = int(rng.choice([32, 64, 128, 256]))
            coarse = 16
            gamma = 1e3
        else:
            n = int(rng.choice([8, 16, 32]))
            coarse = 8 if n > 8 else 4
            gamma = 1e4
        levels = int(round(math.log2(n // coarse))) + 1
        dr = float(10.0 ** rng.uniform(4.0, 8.0))
        w = Workload(f"req{i}_{dim}d_{n}", dim, n, levels, 24, dr, gamma, 10 ** 6 + i)
        out.append((t, w))
    return out
