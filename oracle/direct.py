"""Direct solve of the discrete Stokes system: the plain definition (oracle).

Test infrastructure: see package docstring.

The discrete solution is the (u, p) with p in L^2_0 solving eq. (stokessys)
(Section 2); with r_2 = 0 it also solves the augmented system of eq.
(augstokessys) (Section 3). The constant pressure is the kernel of B^T, so the
zero-mean condition int p = m^T p = 0 (m = M_p 1) is imposed by a Lagrange
multiplier, giving the bordered system
    [A_gamma  B^T  0] [u]   [r_1]
    [B        0    m] [p] = [0  ]
    [0        m^T  0] [l]   [0  ]
which is nonsingular and is factored by sparse LU.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assembly import Operators


def solve_direct(ops: Operators, b_u: np.ndarray, augmented: bool = True) -> np.ndarray:
    m = sp.csr_matrix(ops.p_mass_const.reshape(-1, 1))
    Auu = ops.Agamma if augmented else ops.A
    K = sp.bmat([[Auu, ops.B.T, None],
                 [ops.B, None, m],
                 [None, m.T, None]], format="csc")
    rhs = np.concatenate([b_u, np.zeros(ops.level.n_p + 1)])
    sol = spla.splu(K).solve(rhs)
    return sol[:ops.level.n_u + ops.level.n_p]
