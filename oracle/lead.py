"""Semi-infinite jellium leads: lateral modes, generalized Bloch states and
retarded self-energies.

ORACLE / TEST INFRASTRUCTURE ONLY: see oracle/__init__.py.

Follows Sec. II of the paper:
  * the lead is the discretised free-electron problem (V = 0), laterally
    periodic, so it is diagonal in the lateral plane waves
    exp(i G_nu . r) with G_nu = (2 pi nu_x / L_x, 2 pi nu_y / L_y)
    (Eqs. (11)-(13), (14)-(16));
  * along z, in each lateral mode, the discretised Kohn-Sham equation
    (Eq. (2), generalised to N_f neighbour planes) is a linear recurrence
    whose solutions are the generalized Bloch states x^k (propagating for
    |x| = 1, evanescent otherwise);
  * the self-energies follow Eqs. (9)-(10): Sigma = (coupling to the lead)
    x Q(lead planes) x Q(boundary planes)^-1, where the columns of Q are the
    generalized Bloch states that leave the transition region
    ("tra" states for the right lead, "ref" states for the left one).
    For N_f > 1 the coupling and the Q matrices span N_f planes (the
    extension the paper calls straightforward).
  * a propagating state leaves through the right lead if it carries current
    to the right.  The current is computed from its definition (bond current
    across a plane cut), not from a dispersion derivative.

Lateral mode numbering (interface convention shared with the library as
data): mode id m = iy * nx + ix with ix, iy in FFT order, i.e.
nu_x = ix for ix < nx/2 and ix - nx otherwise (same for y).

Lateral Bloch vector kappa = (kappa_x, kappa_y) (Eqs. (2), (12)-(13) and
(16) carry it; the workloads use kappa = 0): the wave functions obey
psi(r + L_x e_x) = exp(i kappa_x L_x) psi(r), so the lateral plane waves
are exp(i (G_nu + kappa) . r) and every lateral energy is taken at
G_nu + kappa.

Quantities are per unit lateral plane wave; the real-space matrices
(Eq. (11) generalised) are built by explicit DFT sums, without an FFT.
"""
from __future__ import annotations

import numpy as np

from .fd import fd_coefficients


class AtThreshold(ValueError):
    """Energy (numerically) at a channel threshold: a propagating pair of
    Bloch states merges, the velocity vanishes and Sigma is singular."""


def mode_numbers(n: int):
    """nu for index 0..n-1 in FFT order."""
    return np.array([i if i < n // 2 else i - n for i in range(n)])


def lateral_energy(g, mode, kappa=(0.0, 0.0)):
    """eps_nu: lateral kinetic energy of the plane wave exp(i (G_nu + kappa).r)
    of mode id `mode` under the lateral part of the FD Laplacian (Eq. (1),
    spacing h_x along x and h_y along y)."""
    c = fd_coefficients(g.nf)
    ix, iy = mode % g.nx, mode // g.nx
    e = 0.0
    for nu, n_, h, k in ((mode_numbers(g.nx)[ix], g.nx, g.hx, kappa[0]),
                         (mode_numbers(g.ny)[iy], g.ny, g.hy, kappa[1])):
        th = 2.0 * np.pi * nu / n_ + k * h  # (G_nu + kappa) * h_mu
        e += -(c[0] + 2.0 * sum(c[n] * np.cos(n * th) for n in range(1, g.nf + 1))) / (2.0 * h ** 2)
    return e


def z_hopping(g):
    """a_n, n = 0..nf: the z part of H couples planes k and k+-n by
    a_n = -chat_n / (2 h_z^2)."""
    c = fd_coefficients(g.nf)
    return np.array([-c[n] / (2.0 * g.hz ** 2) for n in range(g.nf + 1)])


def transfer_matrix(g, E, eps):
    """One-plane transfer matrix of the lead recurrence in one lateral mode.

    sum_{n=-nf}^{nf} a_|n| psi(k+n) = (E - eps) psi(k); the state vector is
    u(k) = (psi(k-nf+1), ..., psi(k+nf)) and u(k+1) = M u(k)."""
    a = z_hopping(g)
    nf = g.nf
    M = np.zeros((2 * nf, 2 * nf), dtype=complex)
    for r in range(2 * nf - 1):
        M[r, r + 1] = 1.0
    # psi(k+nf+1) = [(E - eps) psi(k+1) - sum_{n=-nf}^{nf-1} a_|n| psi(k+1+n)] / a_nf
    # entries of u(k) are psi(k-nf+1+s), s = 0..2nf-1, i.e. offset n = s - nf from k+1
    for s in range(2 * nf):
        n = s - nf
        coef = -a[abs(n)]
        if n == 0:
            coef += E - eps
        M[-1, s] = coef / a[nf]
    return M


def bloch_current(g, x):
    """Bond current carried by the Bloch state psi(k) = x^k (|x| = 1) across a
    cut between two planes, per lateral point:
    J = -2 sum_{p <= 0 < q} a_{q-p} Im(conj(psi_p) psi_q)."""
    a = z_hopping(g)
    J = 0.0
    for n in range(1, g.nf + 1):
        for p in range(1 - n, 1):  # n bonds of length n straddle the cut
            q = p + n
            J += -2.0 * a[n] * np.imag(np.conj(x ** p) * x ** q)
    return J


def _polish(g, dE, x, steps=3):
    """Newton refinement of an eigenvalue x of the transfer matrix on its
    characteristic equation sum_n a_|n| x^(n+nf) - dE x^nf = 0."""
    a = z_hopping(g)
    nf = g.nf
    for _ in range(steps):
        f = -dE * x ** nf
        df = -dE * nf * x ** (nf - 1)
        for n in range(-nf, nf + 1):
            e = n + nf
            f += a[abs(n)] * x ** e
            if e:
                df += a[abs(n)] * e * x ** (e - 1)
        if df == 0:
            break
        step = f / df
        x = x - step
        if abs(step) < 1e-17 * max(1.0, abs(x)):
            break
    return x


class LeadMode:
    """Generalized Bloch states and self-energies of one lateral mode."""

    def __init__(self, g, E, mode, tol=1e-9, kappa=(0.0, 0.0)):
        self.g, self.E, self.mode = g, E, mode
        self.eps = lateral_energy(g, mode, kappa)
        roots = np.linalg.eigvals(transfer_matrix(g, E, self.eps))
        roots = np.array([_polish(g, E - self.eps, x) for x in roots])
        self.roots = roots
        right, left = [], []
        self.x_in = None   # right-moving propagating state (incident from the left)
        self.x_back = None  # left-moving propagating state
        for x in roots:
            if abs(abs(x) - 1.0) < tol:
                J = bloch_current(g, x / abs(x))
                if abs(J) < tol:
                    raise AtThreshold(f"mode {mode}: zero-velocity state at E={E}")
                if J > 0:
                    right.append(x)
                    self.x_in = x / abs(x)
                    self.J = J
                else:
                    left.append(x)
                    self.x_back = x / abs(x)
            elif abs(x) < 1.0:
                right.append(x)
            else:
                left.append(x)
        if len(right) != g.nf or len(left) != g.nf:
            raise AtThreshold(f"mode {mode}: cannot split roots at E={E}: {roots}")
        dmin = min(abs(r1 - r2) for i, r1 in enumerate(roots) for r2 in roots[i + 1:])
        if dmin < 1e-7:
            raise AtThreshold(f"mode {mode}: degenerate Bloch states at E={E}")
        self.right = np.array(right)  # states leaving through the right lead
        self.left = np.array(left)    # states leaving through the left lead
        self.open = self.x_in is not None

    def sigma_right(self):
        """N_f x N_f retarded self-energy of the right lead on the last N_f
        planes (index i <-> plane nz-nf+i), Eq. (10) generalised:
        Sigma_R = C_R Q_tra(lead) Q_tra(boundary)^-1."""
        nf, a = self.g.nf, z_hopping(self.g)
        Qb = np.array([[x ** m for x in self.right] for m in range(nf)])
        Ql = np.array([[x ** (nf + m) for x in self.right] for m in range(nf)])
        C = np.zeros((nf, nf))
        for i in range(nf):
            for m in range(nf):
                n = nf + m - i  # plane distance from boundary plane i to lead plane m
                if n <= nf:
                    C[i, m] = a[n]
        return C @ Ql @ np.linalg.inv(Qb)

    def sigma_left(self):
        """Left-lead self-energy on planes 0..nf-1, Eq. (9) generalised:
        Sigma_L = C_L Q_ref(lead) Q_ref(boundary)^-1 (lead planes -1..-nf)."""
        nf, a = self.g.nf, z_hopping(self.g)
        Qb = np.array([[y ** m for y in self.left] for m in range(nf)])
        Ql = np.array([[y ** (-(m + 1)) for y in self.left] for m in range(nf)])
        C = np.zeros((nf, nf))
        for i in range(nf):
            for m in range(nf):
                n = i + m + 1
                if n <= nf:
                    C[i, m] = a[n]
        return C @ Ql @ np.linalg.inv(Qb)


def lead_modes(g, E, kappa=(0.0, 0.0)):
    return [LeadMode(g, E, m, kappa=kappa) for m in range(g.nx * g.ny)]


def open_channels(g, E, kappa=(0.0, 0.0)):
    """Mode ids of the propagating lateral modes at E (ascending)."""
    return [m for m in range(g.nx * g.ny) if LeadMode(g, E, m, kappa=kappa).open]


def plane_wave_matrix(g, kappa=(0.0, 0.0)):
    """F[l, m] = exp(i (G_m + kappa) . r_l) for lateral points l = j*nx + i."""
    jj, ii = np.meshgrid(np.arange(g.ny), np.arange(g.nx), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    mx = mode_numbers(g.nx)
    my = mode_numbers(g.ny)
    modes = np.arange(g.nx * g.ny)
    nux, nuy = mx[modes % g.nx], my[modes // g.nx]
    ph = 2.0 * np.pi * (np.outer(ii, nux) / g.nx + np.outer(jj, nuy) / g.ny)
    ph = ph + (kappa[0] * g.hx * ii + kappa[1] * g.hy * jj)[:, None]
    return np.exp(1j * ph)


def sigma_realspace(g, E, side, kappa=(0.0, 0.0)):
    """Dense real-space self-energy on the N_f boundary planes (Eq. (11),
    generalised): Sigma[(i,l),(j,l')] = 1/N_xy sum_nu e^{i(G+kappa).(r_l - r_l')}
    Sigma_nu[i, j], as explicit sums.  Shape (nf*Nxy, nf*Nxy); plane index i
    is the slow one.  side = 'L' (planes 0..nf-1) or 'R' (nz-nf..nz-1)."""
    nf, nxy = g.nf, g.nx * g.ny
    F = plane_wave_matrix(g, kappa)
    sig = np.zeros((nxy, nf, nf), dtype=complex)
    for m in range(nxy):
        lm = LeadMode(g, E, m, kappa=kappa)
        sig[m] = lm.sigma_left() if side == "L" else lm.sigma_right()
    S = np.zeros((nf * nxy, nf * nxy), dtype=complex)
    for i in range(nf):
        for j in range(nf):
            S[i * nxy:(i + 1) * nxy, j * nxy:(j + 1) * nxy] = (F * sig[:, i, j][None, :]) @ F.conj().T / nxy
    return S
