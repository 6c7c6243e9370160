"""Gradient of the total transmission with respect to the local potential.

ORACLE / TEST INFRASTRUCTURE ONLY: see oracle/__init__.py.

The paper computes transmissions only; the derivative is the plain
consequence of its linear system (Eq. (6)):
  * A depends on V only through -diag(V), b does not depend on V, so
    d psi / d V_i = A^-1 (e_i psi_i);
  * T_mu = psi_B^H Gamma psi_B / J_mu, hence
    d T_mu / d V_i = 2 Re(lambda_i psi_i) with A^T lambda = conj(Gamma psi_B) / J_mu
    (adjoint vector placed on the far boundary planes);
  * the transposed solve reuses the LU factors (trans='T'): SuperLU's, or
    for wide cross-sections (dense self-energy blocks) a dense LAPACK LU of
    the same matrix.
With a nonlocal term the same holds for the bordered matrix; lambda is its
first N_pts entries.
"""
from __future__ import annotations

import numpy as np

from .lead import open_channels


class _DenseLU:
    """LAPACK LU of the dense matrix with SuperLU's solve(rhs, trans) call."""

    def __init__(self, A):
        import scipy.linalg as sla
        self._sla = sla
        self._f = sla.lu_factor(A.toarray(), check_finite=False)

    def solve(self, rhs, trans="N"):
        return self._sla.lu_solve(self._f, rhs, trans={"N": 0, "T": 1}[trans], check_finite=False)


def total_transmission_and_gradient(prob, energies, side="L", dense=False):
    """(T_total, dT_total/dV as (nz, ny, nx)) summed over every open channel
    at every energy in `energies`."""
    g = prob.g
    far = "R" if side == "L" else "L"
    sf = prob.boundary_slice(far)
    nb = 0 if prob.B is None else prob.B.shape[1]
    T_total = 0.0
    grad = np.zeros(g.npts)
    for E in energies:
        modes = open_channels(g, E, prob.kappa)
        lu = _DenseLU(prob.matrix(E)) if dense else prob.factor(E)
        psi = prob.solve(E, modes, side, lu=lu)
        G = prob.gamma(E, far)
        for m, p in zip(modes, psi):
            p = p.ravel()
            J = prob.incident_current(E, m, side)
            T_total += np.real(np.vdot(p[sf], G @ p[sf])) / J
            rhs = np.zeros(g.npts + nb, dtype=complex)
            rhs[sf] = np.conj(G @ p[sf]) / J
            lam = lu.solve(rhs, trans="T")[:g.npts]
            grad += 2.0 * np.real(lam * p)
    return T_total, grad.reshape(g.shape)


def total_transmission(prob, energies, side="L"):
    g = prob.g
    T = 0.0
    for E in energies:
        modes = open_channels(g, E, prob.kappa)
        psi = prob.solve(E, modes, side)
        for m, p in zip(modes, psi):
            T += prob.currents(E, m, p, side)[0]
    return T
