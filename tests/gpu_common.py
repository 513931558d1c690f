"""Shared helpers of the GPU parity tests: build the oracle and the GPU
hierarchy for one workload, convert between the oracle's unknown vectors and
the stored full-grid layout."""
from __future__ import annotations

import functools
import sys

import numpy as np

from workloads import CONFIGS, small


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


CASES = {
    "sinker_2d_16sq_L2": CONFIGS["sinker_2d_16sq_L2"],
    "2d_32_L3": small(2, 32, 3, gamma=1e3, dr=1e6, n_sinkers=16, seed=201),
    "3d_8_L2": small(3, 8, 2, gamma=1e4, dr=1e8, n_sinkers=24, seed=301),
    # viscoplastic Newton tensor over a sinker base field (the recipe of the 3D 48^3 workload)
    "2d_16_L2_tensor": small(2, 16, 2, gamma=1e3, dr=1e6, n_sinkers=16, seed=411, coef_kind=1, fourier_seed=412),
    "3d_8_L2_tensor": small(3, 8, 2, gamma=1e4, dr=1e10, n_sinkers=24, seed=401, coef_kind=1, fourier_seed=402),
    # W = M_p(1/mu) (preconditioner P2)
    "2d_16_L3_p2": small(2, 16, 3, gamma=1e3, dr=1e6, n_sinkers=16, seed=421, schur=2),
    "3d_8_L2_p2": small(3, 8, 2, gamma=1e4, dr=1e4, n_sinkers=24, seed=431, schur=2),
    # odd cell counts per axis (coarse 3, fine 6): no level is a power of two.
    # The 3D contrast is moderate: at 1e8 this mesh cannot resolve the
    # sinkers, FGMRES stagnates over three restart cycles (90 iterations, equal
    # on both sides) and the residual histories drift apart by 1e-4, beyond
    # the history tolerance, though the solutions still agree to 1e-8.
    "2d_6_L2": small(2, 6, 2, gamma=1e3, dr=1e6, n_sinkers=4, seed=441),
    "3d_6_L2": small(3, 6, 2, gamma=1e4, dr=1e4, n_sinkers=6, seed=451),
    # three 3D levels with a middle level (a prolongation in and a restriction
    # out, split centre solves): the 32^3 workload's parameters (24 sinkers,
    # contrast 1e8, gamma 1e4) and the 48^3 workload's tensor law (contrast
    # 1e10) on 16^3 / 8^3 / 4^3
    "3d_16_L3": small(3, 16, 3, gamma=1e4, dr=1e8, n_sinkers=24, seed=301),
    "3d_16_L3_tensor": small(3, 16, 3, gamma=1e4, dr=1e10, n_sinkers=24, seed=401, coef_kind=1, fourier_seed=402),
    # 3D 4^3 fine level: one tile of coarse cells, too few fine cells for the
    # split centre solves, so the transfers take the in-workgroup path
    "3d_4_L2": small(3, 4, 2, gamma=1e3, dr=1e4, n_sinkers=4, seed=461),
    # [Q3]^2 x P2disc (velocity degree 3): two levels, three levels (a middle
    # level), and W = M_p(1/mu)
    "q3_2d_8_L2": small(2, 8, 2, gamma=1e3, dr=1e4, n_sinkers=4, seed=471, degree=3),
    "q3_2d_16_L3": small(2, 16, 3, gamma=1e3, dr=1e6, n_sinkers=8, seed=481, degree=3),
    "q3_2d_16_L2_p2": small(2, 16, 2, gamma=1e2, dr=1e4, n_sinkers=6, seed=491, schur=2, degree=3),
    # [Q3]^3 x P2disc: 4^3 fine cells over 2^3 (27 interior 375-unknown stars)
    "q3_3d_4_L2": small(3, 4, 2, gamma=1e3, dr=1e4, n_sinkers=4, seed=521, degree=3),
}
Q3_CASES = ["q3_2d_8_L2", "q3_2d_16_L3", "q3_2d_16_L2_p2", "q3_3d_4_L2"]
SCALAR_CASES = ["sinker_2d_16sq_L2", "2d_32_L3", "3d_8_L2"]
# the slow oracle cases (about a minute of oracle setup and solve each)
BIG_CASES = ["3d_16_L3", "3d_16_L3_tensor"]
P2_CASES = ["2d_16_L3_p2", "3d_8_L2_p2"]


@functools.lru_cache(maxsize=None)
def oracle_for(name: str):
    from oracle.krylov import StokesSolver
    return StokesSolver(CASES[name])


@functools.lru_cache(maxsize=None)
def gpu_for(name: str):
    from paper_2107_00820_amd import Hierarchy
    return Hierarchy.from_workload(CASES[name])


def to_dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def rand_u(level, seed):
    """Random unknown vector of a level and its stored layout (with garbage on
    Dirichlet nodes, which the library must ignore)."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(level.n_u)
    s = level.to_stored(u)
    mask = np.ones(level.n_stored, dtype=bool)
    mask[level.stored_index()] = False
    s[mask] = rng.standard_normal(mask.sum()) * 1e3
    return u, s


@functools.lru_cache(maxsize=None)
def gpu_mixed_for(name: str):
    """Hierarchy with the FP32 tables of the mixed form."""
    from paper_2107_00820_amd import Hierarchy
    return Hierarchy.from_workload(CASES[name], mixed=1)


def to_dev32(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


def f32(x):
    """Round an FP64 array to FP32 and back (the values an FP32 input holds)."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)
