"""Preconditioners applied to a residual, by their definitions.

ORACLE / TEST INFRASTRUCTURE ONLY: see oracle/__init__.py.

  * Eq. (17) (truncated Laplacian Green's function): P g(r) = C0 g(r) + C1 sum
    of g at the neighbouring grid points; C0 = 1, C1 = exp(-alpha) (Sec. III).
    The neighbour set is read as the six face neighbours (+-h_x, +-h_y, +-h_z),
    laterally periodic, zero outside the transition region along z.
  * the lateral-Fourier preconditioner: the exact inverse of the IOBM matrix
    of the flat wire (V = 0, no nonlocal term), computed here by a sparse
    direct solve with that matrix; no Fourier transform is used.
These change iteration counts only, never the converged psi.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .system import Problem


def truncated_laplacian(g, r, alpha):
    r = np.asarray(r).reshape((-1,) + g.shape)
    c1 = np.exp(-alpha)
    z = r.copy()
    for ax in (2, 3):
        z += c1 * (np.roll(r, 1, axis=ax) + np.roll(r, -1, axis=ax))
    z[:, 1:] += c1 * r[:, :-1]
    z[:, :-1] += c1 * r[:, 1:]
    return z


def flat_wire_inverse(g, E, r):
    r = np.asarray(r).reshape(-1, g.npts)
    P0 = Problem(g, np.zeros(g.shape))
    lu = spla.splu(P0.matrix(E), permc_spec="COLAMD")
    return np.stack([lu.solve(v) for v in r]).reshape((-1,) + g.shape)
