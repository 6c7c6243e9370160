"""The IOBM scattering system and its direct solution.

ORACLE / TEST INFRASTRUCTURE ONLY: see oracle/__init__.py.

What is computed (Sec. II of the paper):
  * H_T, the truncated real-space FD Kohn-Sham Hamiltonian on planes
    0 .. nz-1 (Eqs. (1)-(4); laterally periodic with kappa = 0, couplings
    beyond the first and last plane dropped), plus the local potential V(r)
    and, optionally, a separable nonlocal term sum_a B_a D_a h^3 B_a^T;
  * the IOBM matrix A(E) = E - H_T - Htilde (Eq. (6), Eq. (8)) with
    Htilde = diag(Sigma_L, 0, ..., 0, Sigma_R) acting on the first and last
    N_f planes (self-energies of lead.py, in real space);
  * the right-hand side of Eq. (6): b = C_L Phi_in(lead planes)
    - Sigma_L Phi_in(boundary planes), C_L being the couplings of H_T to the
    left-lead planes that truncation dropped (B_z^dagger for N_f = 1), with
    the incident wave Phi_in a right-moving lateral plane wave x^k;
  * psi = A^-1 b by sparse direct LU (scipy SuperLU), one factorisation per
    energy shared by every incident channel (or, for wide cross-sections
    whose dense self-energy blocks defeat the sparse ordering, by a dense
    LAPACK solve of the same matrix);
  * transmission and reflection from the probability current, as ratios of
    the current leaving through each lead to the incident current (the
    Landauer-Buttiker transmission quoted in Sec. III): the current into a
    lead is psi_B^H Gamma psi_B with Gamma = i (Sigma - Sigma^H), and the
    incident current is the bond current of Phi_in across a plane cut.

The nonlocal term is carried by the bordered (augmented) matrix
[[A_loc, B], [B^T, (h^3 D)^-1]] whose Schur complement is A_loc - B h^3 D B^T,
so the sparse LU keeps its sparsity.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fd import fd_coefficients
from .lead import LeadMode, mode_numbers, sigma_realspace, z_hopping


def _second_difference_1d(n, nf, periodic, phase=1.0):
    """Matrix of sum_{m=-nf}^{nf} chat_|m| f(k+m) on n points (h = 1).
    periodic: f(k + n) = phase f(k) (a Bloch phase exp(i kappa L))."""
    c = fd_coefficients(nf)
    D = sp.lil_matrix((n, n), dtype=complex)
    for k in range(n):
        for m in range(-nf, nf + 1):
            q = k + m
            if periodic:
                D[k, q % n] += c[abs(m)] * phase ** (q // n)
            elif 0 <= q < n:
                D[k, q] += c[abs(m)]
    return D.tocsr()


def kinetic(g, kappa=(0.0, 0.0)):
    """-1/2 Laplacian (Eq. (1), c_{mu,n} = chat_n / h_mu^2 per direction) on
    the truncated grid, flat index (k*ny + j)*nx + i: Bloch periodic in x and
    y (phase exp(i kappa_mu L_mu) across the cell), z couplings outside
    0..nz-1 dropped (Eq. (4))."""
    px = np.exp(1j * kappa[0] * g.nx * g.hx)
    py = np.exp(1j * kappa[1] * g.ny * g.hy)
    Dx = _second_difference_1d(g.nx, g.nf, True, px) / g.hx ** 2
    Dy = _second_difference_1d(g.ny, g.nf, True, py) / g.hy ** 2
    Dz = _second_difference_1d(g.nz, g.nf, False) / g.hz ** 2
    Ix, Iy, Iz = (sp.identity(n, format="csr") for n in (g.nx, g.ny, g.nz))
    lap = sp.kron(Iz, sp.kron(Iy, Dx)) + sp.kron(Iz, sp.kron(Dy, Ix)) + sp.kron(Dz, sp.kron(Iy, Ix))
    return (-0.5 * lap).tocsr()


def lead_coupling(g, side):
    """Couplings of H between the N_f boundary planes and the N_f adjacent
    lead planes, dropped by truncation: dense (nf*Nxy, nf*Nxy), rows =
    boundary planes (0..nf-1 or nz-nf..nz-1), columns = lead planes
    (-nf..-1 or nz..nz+nf-1), plane index slow."""
    nf, nxy = g.nf, g.nx * g.ny
    a = z_hopping(g)
    Cz = np.zeros((nf, nf))
    for i in range(nf):
        for m in range(nf):
            if side == "L":
                dist = i - (m - nf)       # boundary plane i, lead plane m - nf
            else:
                dist = (g.nz + m) - (g.nz - nf + i)
            if 1 <= dist <= nf:
                Cz[i, m] = a[dist]
    return np.kron(Cz, np.eye(nxy))


def kb_matrix(g, nl):
    """Sparse B (N_pts x nproj) and the per-projector coupling block
    diag_a(h^3 D_a) (nproj x nproj), h^3 = hx hy hz the volume element."""
    if nl is None:
        return None, None
    rows, cols, vals = [], [], []
    col = 0
    blocks = []
    for idx, beta, D in zip(nl.support, nl.beta, nl.D):
        r = beta.shape[0]
        for p in range(r):
            rows.append(idx)
            cols.append(np.full(idx.size, col + p))
            vals.append(beta[p])
        blocks.append(g.hx * g.hy * g.hz * np.asarray(D, dtype=float))
        col += r
    B = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(g.npts, col))
    from scipy.linalg import block_diag
    return B, block_diag(*blocks)


class Problem:
    """One transition region: grid, local potential, optional nonlocal term,
    lateral Bloch vector kappa (A(kappa)^T = A(-kappa); symmetric at 0)."""

    def __init__(self, g, V, nl=None, kappa=(0.0, 0.0)):
        self.g = g
        self.V = np.asarray(V, dtype=float).reshape(g.shape)
        self.nl = nl
        self.kappa = (float(kappa[0]), float(kappa[1]))
        H = kinetic(g, self.kappa)
        if self.kappa == (0.0, 0.0):
            H = H.real
        self.H_loc = (H + sp.diags(self.V.ravel())).tocsr()
        self.B, self.hD = kb_matrix(g, nl)
        self._sig = {}

    # --- boundary blocks -------------------------------------------------
    def sigma(self, E, side):
        key = (float(E), side)
        if key not in self._sig:
            self._sig[key] = sigma_realspace(self.g, E, side, self.kappa)
        return self._sig[key]

    def boundary_slice(self, side):
        nf, nxy = self.g.nf, self.g.nx * self.g.ny
        if side == "L":
            return slice(0, nf * nxy)
        return slice(self.g.npts - nf * nxy, self.g.npts)

    # --- operator ----------------------------------------------------------
    def apply(self, E, x):
        """y = A(E) x for x of shape (..., N_pts) or (N_pts,), by the plain
        definition: E x - H_T x - V_NL x - Sigma_L x_B - Sigma_R x_B."""
        x = np.asarray(x)
        X = x.reshape(-1, self.g.npts).T  # (N_pts, nrhs)
        Y = E * X - self.H_loc @ X
        if self.B is not None:
            Y = Y - self.B @ (self.hD @ (self.B.T @ X))
        for side in ("L", "R"):
            s = self.boundary_slice(side)
            Y[s] -= self.sigma(E, side) @ X[s]
        return Y.T.reshape(x.shape)

    def matrix(self, E):
        """Sparse A(E) (bordered by the nonlocal projectors when present)."""
        g = self.g
        A = (E * sp.identity(g.npts, format="csr") - self.H_loc).astype(complex)
        for side in ("L", "R"):
            s = self.boundary_slice(side)
            S = sp.coo_matrix(self.sigma(E, side))
            A = A - sp.csr_matrix((S.data, (S.row + s.start, S.col + s.start)), shape=A.shape)
        A = A.tocsc()
        if self.B is not None:
            C = sp.csc_matrix(np.linalg.inv(self.hD))
            A = sp.bmat([[A, self.B], [self.B.T, C]], format="csc")
        return A

    # --- incident wave and right-hand side (Eq. (6)) ------------------------
    def incident(self, E, mode, side="L"):
        """Phi_in on planes -nf .. nz-1+nf, shape (nz + 2nf, ny, nx): lateral
        plane wave exp(i G.r) times the propagating Bloch state moving away
        from the source lead, unit amplitude on the first transition plane
        it enters (plane 0 from the left, plane nz-1 from the right)."""
        g = self.g
        lm = LeadMode(g, E, mode, kappa=self.kappa)
        if not lm.open:
            raise ValueError(f"mode {mode} is closed at E={E}")
        x = lm.x_in if side == "L" else lm.x_back
        k = np.arange(-g.nf, g.nz + g.nf)
        kref = 0 if side == "L" else g.nz - 1
        zpart = x ** (k - kref)
        nux = mode_numbers(g.nx)[mode % g.nx]
        nuy = mode_numbers(g.ny)[mode // g.nx]
        jj, ii = np.meshgrid(np.arange(g.ny), np.arange(g.nx), indexing="ij")
        lat = np.exp(2j * np.pi * (nux * ii / g.nx + nuy * jj / g.ny)
                     + 1j * (self.kappa[0] * g.hx * ii + self.kappa[1] * g.hy * jj))
        return zpart[:, None, None] * lat[None, :, :]

    def rhs(self, E, mode, side="L"):
        g = self.g
        nf, nxy = g.nf, g.nx * g.ny
        Phi = self.incident(E, mode, side)
        b = np.zeros(g.npts, dtype=complex)
        if side == "L":
            lead = Phi[:nf].ravel()                  # planes -nf..-1
            bnd = Phi[nf:2 * nf].ravel()             # planes 0..nf-1
        else:
            lead = Phi[nf + g.nz: 2 * nf + g.nz].ravel()  # planes nz..nz+nf-1
            bnd = Phi[g.nz: g.nz + nf].ravel()            # planes nz-nf..nz-1
        s = self.boundary_slice(side)
        b[s] = lead_coupling(g, side) @ lead - self.sigma(E, side) @ bnd
        return b

    def incident_current(self, E, mode, side="L"):
        """Bond current of Phi_in across the cut between lead planes -1 and 0
        (left) or nz-1 and nz (right), summed over the lateral points:
        J = -2 sum a_{q-p} Im(conj(Phi_p) Phi_q) over bonds p < cut <= q.
        Positive in the direction of incidence."""
        g = self.g
        a = z_hopping(g)
        Phi = self.incident(E, mode, side)
        off = g.nf  # array plane index of transition plane 0
        cut = 0 if side == "L" else g.nz  # first plane to the right of the cut
        J = 0.0
        for n in range(1, g.nf + 1):
            for p in range(cut - n, cut):
                q = p + n
                J += -2.0 * a[n] * np.sum(np.imag(np.conj(Phi[p + off]) * Phi[q + off]))
        return J if side == "L" else -J

    # --- solve and read out -------------------------------------------------
    def factor(self, E):
        return spla.splu(self.matrix(E), permc_spec="COLAMD")

    def solve(self, E, modes, side="L", lu=None, check=True, dense=False):
        """psi for every incident mode in `modes`: array (len(modes), nz, ny, nx).
        dense=True solves with the dense matrix (numpy.linalg.solve)."""
        g = self.g
        nb = 0 if self.B is None else self.B.shape[1]
        Bm = np.zeros((g.npts + nb, len(modes)), dtype=complex)
        for c, m in enumerate(modes):
            Bm[:g.npts, c] = self.rhs(E, m, side)
        if dense:
            X = np.linalg.solve(self.matrix(E).toarray(), Bm)
        else:
            lu = lu or self.factor(E)
            X = lu.solve(Bm)
        psi = X[:g.npts].T.reshape((len(modes),) + g.shape)
        if check:
            res = self.apply(E, psi.reshape(len(modes), -1)) - Bm[:g.npts].T
            rel = np.linalg.norm(res, axis=1) / np.linalg.norm(Bm[:g.npts], axis=0)
            if rel.max() > 1e-10:
                raise RuntimeError(f"direct solve residual {rel.max():.3e}")
        return psi

    def gamma(self, E, side):
        key = (float(E), side, "gamma")
        if key not in self._sig:
            S = self.sigma(E, side)
            self._sig[key] = 1j * (S - S.conj().T)
        return self._sig[key]

    def currents(self, E, mode, psi, side="L"):
        """(T, R): current leaving through the far / near lead divided by the
        incident current."""
        far, near = ("R", "L") if side == "L" else ("L", "R")
        psi = psi.ravel()
        Phi = self.incident(E, mode, side)[self.g.nf:self.g.nf + self.g.nz].ravel()
        J = self.incident_current(E, mode, side)
        sf, sn = self.boundary_slice(far), self.boundary_slice(near)
        Jt = np.real(np.vdot(psi[sf], self.gamma(E, far) @ psi[sf]))
        d = psi[sn] - Phi[sn]
        Jr = np.real(np.vdot(d, self.gamma(E, near) @ d))
        return Jt / J, Jr / J

    def lateral_components(self, psi, planes):
        """psi~_nu(plane) = (1/Nxy) sum_l exp(-i G_nu . r_l) psi(plane, l) for
        every lateral mode nu (Eq. (16)), by explicit sums: (len(planes), Nxy)."""
        from .lead import plane_wave_matrix
        F = plane_wave_matrix(self.g, self.kappa)
        P = np.stack([np.asarray(psi)[k].ravel() for k in planes])
        return P @ F.conj() / (self.g.nx * self.g.ny)

    def amplitudes(self, E, mode, psi, side="L"):
        """Outgoing amplitudes of psi in every open channel (the scattering
        condition, Eq. (7)): on the nf planes next to each lead, the lateral
        component of every open channel nu is expanded in the nf Bloch states
        that leave through that lead; the coefficient of the propagating one,
        referred to the plane next to the lead (plane 0 or nz-1), is the
        amplitude.  On the side of incidence the incident wave (unit amplitude
        at that plane) is subtracted first.  Returns dicts {nu: amplitude} for
        the left and right leads."""
        from .lead import LeadMode, open_channels
        g = self.g
        nf, nz = g.nf, g.nz
        lo, hi = list(range(nf)), list(range(nz - nf, nz))
        cl, cr = self.lateral_components(psi, lo), self.lateral_components(psi, hi)
        out = {"L": {}, "R": {}}
        for nu in open_channels(g, E, self.kappa):
            lm = LeadMode(g, E, nu, kappa=self.kappa)
            # right lead: states leaving to the right, x^(k - (nz-1)) on planes nz-nf..nz-1
            vals = cr[:, nu].copy()
            if side == "R" and nu == mode:
                vals -= lm.x_back ** (np.array(hi) - (nz - 1))
            X = np.array([[x ** (k - (nz - 1)) for x in lm.right] for k in hi])
            c = np.linalg.solve(X, vals)
            out["R"][nu] = c[np.argmin(np.abs(np.abs(lm.right) - 1))]
            # left lead: states leaving to the left, y^k on planes 0..nf-1
            vals = cl[:, nu].copy()
            if side == "L" and nu == mode:
                vals -= lm.x_in ** np.array(lo)
            Y = np.array([[y ** k for y in lm.left] for k in lo])
            c = np.linalg.solve(Y, vals)
            out["L"][nu] = c[np.argmin(np.abs(np.abs(lm.left) - 1))]
        return out

    def smatrix(self, E):
        """Flux-normalised scattering matrix at E: rows and columns ordered
        [left channels | right channels] (ascending ids), S[b nu, a mu] =
        sqrt(J_nu / J_mu) x (amplitude of channel nu in lead b for unit
        incidence in channel mu from lead a), every amplitude referred to the
        plane next to its lead; J is the current of the unit Bloch wave."""
        from .lead import LeadMode, open_channels
        modes = open_channels(self.g, E, self.kappa)
        n = len(modes)
        J = np.array([LeadMode(self.g, E, m, kappa=self.kappa).J for m in modes])
        S = np.zeros((2 * n, 2 * n), dtype=complex)
        lu = self.factor(E)
        for a, side in enumerate(("L", "R")):
            psis = self.solve(E, modes, side, lu=lu)
            for j, (mu, p) in enumerate(zip(modes, psis)):
                amp = self.amplitudes(E, mu, p, side)
                for b, lead in enumerate(("L", "R")):
                    for i, nu in enumerate(modes):
                        S[b * n + i, a * n + j] = np.sqrt(J[i] / J[j]) * amp[lead][nu]
        return modes, S

    def transmission_matrix_eigs(self, E, modes, psis, side="L"):
        """Eigenvalues of t^dagger t for the incident channels `modes` at E:
        the flux-normalised matrix M[m, m'] = psi_m^H Gamma_far psi_m' /
        sqrt(J_m J_m') (eigenchannel transmissions, Sec. IV)."""
        far = "R" if side == "L" else "L"
        sf = self.boundary_slice(far)
        G = self.gamma(E, far)
        P = np.stack([p.ravel()[sf] for p in psis], axis=1)
        J = np.array([self.incident_current(E, m, side) for m in modes])
        M = (P.conj().T @ G @ P) / np.sqrt(np.outer(J, J))
        return np.linalg.eigvalsh(0.5 * (M + M.conj().T))


def solve_workload(prob, energies, side="L", channels=None):
    """Solve every (energy, open channel) pair; returns a list of dicts per
    energy with keys E, modes, psi, T, R."""
    from .lead import open_channels
    out = []
    for E in energies:
        modes = open_channels(prob.g, E, prob.kappa)
        if channels == "lowest":
            modes = modes[:1]
        lu = prob.factor(E)
        psi = prob.solve(E, modes, side, lu=lu)
        TR = [prob.currents(E, m, p, side) for m, p in zip(modes, psi)]
        out.append({"E": E, "modes": modes, "psi": psi, "lu": lu,
                    "T": np.array([t for t, _ in TR]), "R": np.array([r for _, r in TR])})
    return out
