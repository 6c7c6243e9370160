"""Preconditioners applied to a residual, by their definitions.

ORACLE / TEST INFRASTRUCTURE ONLY: see oracle/__init__.py.

  * Eq. (17) (truncated Laplacian Green's function): P g(r) = C0 g(r) + C1 sum
    of g at the neighbouring grid points; C0 = 1, C1 = exp(-alpha) (Sec. III).
    The neighbour set is read as the six face neighbours (+-h_x, +-h_y, +-h_z),
    laterally periodic, zero outside the transition region along z.
  * the lateral-Fourier preconditioner: the exact inverse of the IOBM matrix
    of the flat wire (V = 0, no nonlocal term), computed here by a sparse
    direct solve with that matrix; no Fourier transform is used.
  * Jacobi (diagonal scaling, named alongside Eq. (17) in Sec. II): z = r / a
    with a the diagonal of A(E), i.e. E - V - the kinetic diagonal, minus the
    diagonal of the self-energies on the boundary planes and of the nonlocal
    term.
These change iteration counts only, never the converged psi.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .system import Problem


def truncated_laplacian(g, r, alpha, kappa=(0.0, 0.0)):
    """Lateral neighbours of a Bloch-periodic r across the cell carry the
    phase exp(+-i kappa_mu L_mu)."""
    r = np.asarray(r).reshape((-1,) + g.shape).astype(complex)
    c1 = np.exp(-alpha)
    z = r.copy()
    for ax, n, ph in ((3, g.nx, np.exp(1j * kappa[0] * g.nx * g.hx)), (2, g.ny, np.exp(1j * kappa[1] * g.ny * g.hy))):
        up = np.roll(r, -1, axis=ax)   # r(i + 1): the last index wraps to 0 of the next cell
        dn = np.roll(r, 1, axis=ax)    # r(i - 1): the first index wraps to n - 1 of the previous cell
        sl_last = [slice(None)] * 4
        sl_last[ax] = n - 1
        sl_first = [slice(None)] * 4
        sl_first[ax] = 0
        up[tuple(sl_last)] *= ph
        dn[tuple(sl_first)] /= ph
        z += c1 * (up + dn)
    z[:, 1:] += c1 * r[:, :-1]
    z[:, :-1] += c1 * r[:, 1:]
    return z


def flat_wire_inverse(g, E, r, kappa=(0.0, 0.0)):
    r = np.asarray(r).reshape(-1, g.npts)
    P0 = Problem(g, np.zeros(g.shape), kappa=kappa)
    lu = spla.splu(P0.matrix(E), permc_spec="COLAMD")
    return np.stack([lu.solve(v) for v in r]).reshape((-1,) + g.shape)


def jacobi_diagonal(prob, E):
    """Diagonal of A(E) = E - H_T - V_NL - Sigma_L - Sigma_R, entry by entry
    from its parts."""
    g = prob.g
    a = (E - prob.H_loc.diagonal()).astype(complex)
    if prob.B is not None:
        B = prob.B.tocsr()
        a -= np.einsum("ip,pq,iq->i", B.toarray(), prob.hD, B.toarray())
    for side in ("L", "R"):
        s = prob.boundary_slice(side)
        a[s] -= np.diag(prob.sigma(E, side))
    return a.reshape(g.shape)


def jacobi(prob, E, r):
    r = np.asarray(r).reshape((-1,) + prob.g.shape)
    return r / jacobi_diagonal(prob, E)[None]
