"""Pins of the CPU oracle against facts that do not come from the oracle:
values printed in the paper, closed forms, an independent published
algorithm (Lopez Sancho-Rubio decimation), the Caroli/Fisher-Lee trace
formula, exact invariants of the discrete system, and finite differences.

Each test names what a plausible mistake would break.
"""
from fractions import Fraction
import math
import os

import numpy as np
import pytest

import oracle as O
from workloads import Grid, make, random_field

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- Eq. (1)
def _golden_fd():
    out = {}
    for line in open(os.path.join(GOLDEN, "fd_coefficients.txt")):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        out[int(f[0])] = [Fraction(v) for v in f[1:]]
    return out


@pytest.mark.parametrize("nf", [1, 2, 3])
def test_fd_coefficients_match_printed_and_textbook_values(nf):
    assert list(O.fd_coefficients_exact(nf)) == _golden_fd()[nf]


@pytest.mark.parametrize("nf", [1, 2, 3])
def test_fd_order_of_accuracy(nf):
    # the 2nf-order stencil on sin(x): error ~ h^(2 nf)
    c = O.fd_coefficients(nf)
    errs = []
    for h in (0.2, 0.1):
        x0 = 0.3
        d2 = sum(c[abs(n)] * math.sin(x0 + n * h) for n in range(-nf, nf + 1)) / h ** 2
        errs.append(abs(d2 + math.sin(x0)))
    order = math.log(errs[0] / errs[1], 2)
    assert abs(order - 2 * nf) < 0.3


# ------------------------------------- Eqs. (11)-(15) and the appendix
def _chi(g, E, mode):
    """Eq. (13) with kappa = 0 (N_f = 1), spacings h_x, h_y, h_z."""
    nux = O.mode_numbers(g.nx)[mode % g.nx]
    nuy = O.mode_numbers(g.ny)[mode // g.nx]
    hz2 = g.hz * g.hz
    return (hz2 * E - hz2 / g.hx ** 2 * (1 - math.cos(2 * math.pi * nux / g.nx))
            - hz2 / g.hy ** 2 * (1 - math.cos(2 * math.pi * nuy / g.ny)) - 1.0)


def _sigma_closed_form(g, E, mode):
    """Eq. (15): Sigma_nu = -exp(i k_z h) / (2 h^2), with k_z from Eq. (12)
    and the branch rule stated after Eq. (13); for chi > 1 (above the
    discrete band top) the decaying root of x^2 + 2 chi x + 1 = 0 (the
    appendix's pole pair omega_1, omega_2 with omega_1 omega_2 = 1) is taken."""
    chi = _chi(g, E, mode)
    h = g.hz
    if abs(chi) < 1:
        x = complex(math.cos(math.acos(-chi)), math.sin(math.acos(-chi)))
    elif chi < -1:
        x = math.exp(-math.acosh(-chi))
    else:
        x = -chi + math.sqrt(chi * chi - 1)
    return -x / (2 * h * h)


ANISO = Grid(8, 6, 10, 0.4, 1, hy_=0.55, hz_=0.3)


@pytest.mark.parametrize("g", [Grid(8, 6, 10, 0.4, 1), ANISO], ids=["iso", "aniso"])
@pytest.mark.parametrize("E", [0.05, 0.4, 2.0, 30.0])
def test_sigma_nf1_equals_closed_form(g, E):
    for m in range(g.nx * g.ny):
        lm = O.LeadMode(g, E, m)
        s = lm.sigma_right()
        assert s.shape == (1, 1)
        assert abs(s[0, 0] - _sigma_closed_form(g, E, m)) < 1e-12 * 2 / g.hz ** 2
        assert lm.open == (abs(_chi(g, E, m)) < 1)


def _sancho_rubio(g, E, mode, eta=1e-9, itmax=200):
    """Lopez Sancho, Lopez Sancho & Rubio, J. Phys. F 15, 851 (1985):
    decimation for the surface Green function of a semi-infinite chain of
    principal layers (here N_f planes of one lateral mode); returns the
    right-lead self-energy H01 g_s H10."""
    nf = g.nf
    c = O.fd_coefficients(nf)
    a = [-c[n] / (2 * g.hz ** 2) for n in range(nf + 1)]
    eps = O.lateral_energy(g, mode)
    H00 = np.zeros((nf, nf))
    H01 = np.zeros((nf, nf))
    for i in range(nf):
        for j in range(nf):
            d = abs(i - j)
            H00[i, j] = a[d] + (eps if d == 0 else 0.0)
            dd = nf + j - i
            if dd <= nf:
                H01[i, j] = a[dd]
    w = (E + 1j * eta) * np.eye(nf)
    es, e, al, be = H00.astype(complex), H00.astype(complex), H01.astype(complex), H01.T.astype(complex)
    for _ in range(itmax):
        gg = np.linalg.inv(w - e)
        agb, bga = al @ gg @ be, be @ gg @ al
        es = es + agb
        e = e + agb + bga
        al, be = al @ gg @ al, be @ gg @ be
        if np.abs(al).max() + np.abs(be).max() < 1e-15:
            break
    gs = np.linalg.inv(w - es)
    return H01 @ gs @ H01.T


@pytest.mark.parametrize("aniso", [False, True])
@pytest.mark.parametrize("nf", [2, 3])
@pytest.mark.parametrize("E", [0.1, 0.9, 3.0])
def test_sigma_matches_sancho_rubio(nf, E, aniso):
    g = Grid(6, 4, 10, 0.4, nf, hy_=0.5, hz_=0.33) if aniso else Grid(6, 4, 10, 0.4, nf)
    for m in range(g.nx * g.ny):
        s = O.LeadMode(g, E, m).sigma_right()
        ref = _sancho_rubio(g, E, m)
        assert np.abs(s - ref).max() < 1e-6 * np.abs(ref).max()


@pytest.mark.parametrize("nf", [1, 2, 3])
def test_sigma_symmetric_and_mirror_and_root_pairing(nf):
    g = Grid(6, 6, 10, 0.35, nf)
    for E in (0.2, 1.1):
        for m in range(g.nx * g.ny):
            lm = O.LeadMode(g, E, m)
            S, SL = lm.sigma_right(), lm.sigma_left()
            assert np.abs(S - S.T).max() < 1e-12 * np.abs(S).max()
            # jellium leads: left = right with the plane order reversed
            assert np.abs(SL - S[::-1, ::-1]).max() < 1e-12 * np.abs(S).max()
            # palindromic recurrence: roots pair as x <-> 1/x (omega_1 omega_2 = 1)
            for x in lm.right:
                assert np.min(np.abs(lm.left - 1 / x)) < 1e-9 * max(1, abs(1 / x))
            # retarded: Im Sigma <= 0 (negative semidefinite broadening)
            G = 1j * (S - S.conj().T)
            assert np.linalg.eigvalsh(G).min() > -1e-12 * np.abs(S).max()


def _golden_counts():
    rows = []
    for line in open(os.path.join(GOLDEN, "paper_channel_counts.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, L, N, rs, nin = line.split()
        rows.append((name, float(L), int(N), float(rs), int(nin)))
    return rows


@pytest.mark.parametrize("row", _golden_counts(), ids=lambda r: r[0])
def test_channel_count_of_ir_and_au_wires(row):
    name, L, N, rs, nin = row
    EF = (9 * math.pi / 4) ** (2 / 3) / (2 * rs * rs)
    g = Grid(N, N, 4, L / N, 1)
    assert len(O.open_channels(g, EF)) == nin


# ------------------------------------------------------------ whole solve
@pytest.mark.parametrize("aniso", [False, True])
@pytest.mark.parametrize("nf", [1, 2, 3])
def test_flat_wire_transmits_every_open_channel(nf, aniso):
    # h = 0.9 on a 6x6 cell: several lateral channels open at E = 1.0
    g = Grid(6, 6, 12, 0.9, nf, hy_=0.8, hz_=0.6) if aniso else Grid(6, 6, 12, 0.9, nf)
    P = O.Problem(g, np.zeros(g.shape))
    E = 1.0
    modes = O.open_channels(g, E)
    assert len(modes) >= 5
    psi = P.solve(E, modes)
    Ts = []
    for m, p in zip(modes, psi):
        Phi = P.incident(E, m)[nf:nf + g.nz]
        assert np.abs(p - Phi).max() < 1e-11
        T, R = P.currents(E, m, p)
        Ts.append(T)
        assert abs(T - 1) < 1e-11 and abs(R) < 1e-11
    assert abs(sum(Ts) - len(modes)) < 1e-10


def _barrier_closed_form(E, V0, n, h):
    """Transmission of a tight-binding chain (N_f = 1, t = 1/(2h^2)) through n
    consecutive sites raised by V0: T = [1 + (V0 h^2)^2 |sin(n phi)/sin(phi)|^2
    / sin^2(theta)]^-1 with cos(theta) = 1 - E h^2, cos(phi) = 1 - (E - V0) h^2."""
    th = np.arccos(1 - E * h * h)
    cphi = 1 - (E - V0) * h * h
    phi = np.arccos(complex(cphi))
    ratio = n if abs(np.sin(phi)) < 1e-14 else np.sin(n * phi) / np.sin(phi)
    return 1.0 / (1.0 + (V0 * h * h) ** 2 * abs(ratio) ** 2 / np.sin(th) ** 2)


@pytest.mark.parametrize("E,V0,n", [(0.3, 0.5, 7), (0.6, 0.2, 11), (0.25, -0.3, 5)])
def test_lattice_square_barrier_closed_form(E, V0, n):
    g = Grid(4, 4, 24, 0.5, 1)
    V = np.zeros(g.shape)
    V[8:8 + n] = V0
    P = O.Problem(g, V)
    psi = P.solve(E, [0])
    T, R = P.currents(E, 0, psi[0])
    assert abs(T - _barrier_closed_form(E, V0, n, g.hz)) < 1e-12
    assert abs(T + R - 1) < 1e-12


def _eps_nf1(g, mode):
    """Lateral energy of a plane wave on the 3-point stencil (the textbook
    tight-binding band of each lateral direction, spacing h_x or h_y)."""
    nux = O.mode_numbers(g.nx)[mode % g.nx]
    nuy = O.mode_numbers(g.ny)[mode // g.nx]
    return ((1 - math.cos(2 * math.pi * nux / g.nx)) / g.hx ** 2
            + (1 - math.cos(2 * math.pi * nuy / g.ny)) / g.hy ** 2)


# h_x, h_y, h_z all different: a swapped spacing anywhere (kinetic operator,
# lateral energy, lead hopping, incident current) changes every E_nu below
UNIFORM = Grid(6, 4, 24, 0.9, 1, hy_=0.8, hz_=0.5)


@pytest.mark.parametrize("E,V0,n", [(1.8, 0.5, 7), (2.4, -0.3, 5)])
def test_uniform_barrier_eigenchannels_closed_form(E, V0, n):
    """A laterally uniform barrier does not mix lateral modes, so t is
    diagonal and the eigenvalues of t^dagger t (Sec. IV's eigenchannel
    transmissions) are the lattice square-barrier transmissions of each open
    mode at its longitudinal energy E - eps_nu (spacing h_z along z).  Pins
    the per-channel flux normalisation of the eigenchannel matrix, and the
    anisotropic grid."""
    g = UNIFORM
    V = np.zeros(g.shape)
    V[8:8 + n] = V0
    P = O.Problem(g, V)
    modes = O.open_channels(g, E)
    assert len(modes) >= 5
    ref = sorted(_barrier_closed_form(E - _eps_nf1(g, m), V0, n, g.hz) for m in modes)
    for side in ("L", "R"):
        psi = P.solve(E, modes, side)
        eig = np.sort(P.transmission_matrix_eigs(E, modes, psi, side))
        assert np.abs(eig - ref).max() < 1e-11
        for m, p in zip(modes, psi):
            T, R = P.currents(E, m, p, side)
            assert abs(T - _barrier_closed_form(E - _eps_nf1(g, m), V0, n, g.hz)) < 1e-11


def test_eigenchannels_match_caroli_matrix():
    """The nonzero eigenvalues of the Caroli matrix Gamma_L G_LR Gamma_R
    G_LR^H (Green's function of the dense matrix, no wave functions) are the
    eigenchannel transmissions: pins the off-diagonal (channel-mixing)
    normalisation of the oracle's eigenchannel matrix on a random potential
    with an anisotropic grid."""
    g = Grid(4, 4, 10, 0.9, 2, hy_=0.85, hz_=0.7)
    rng = np.random.default_rng(17)
    V = 0.4 * rng.standard_normal(g.shape)
    P = O.Problem(g, V)
    E = 2.2
    modes = O.open_channels(g, E)
    assert len(modes) >= 5
    G = np.linalg.inv(P.matrix(E).toarray())
    sL, sR = P.boundary_slice("L"), P.boundary_slice("R")
    M = P.gamma(E, "L") @ G[sL, sR] @ P.gamma(E, "R") @ G[sL, sR].conj().T
    lam = np.sort(np.real(np.linalg.eigvals(M)))[::-1][:len(modes)]
    psi = P.solve(E, modes)
    eig = np.sort(P.transmission_matrix_eigs(E, modes, psi))[::-1]
    assert np.abs(eig - lam).max() < 1e-10
    assert eig.max() - eig.min() > 1e-3  # the eigenvalues are distinct: mixing is tested


def test_truncated_laplacian_on_plane_waves():
    """Eq. (17) on r(i, j, k) = exp(i(tx i + ty j)) f(k): the lateral
    neighbours multiply the plane wave by 2 cos t, so interior planes give
    [1 + 2 e^-alpha (cos tx + cos ty)] f(k) + e^-alpha (f(k-1) + f(k+1)) and
    the first and last planes lose their missing z neighbour."""
    g = Grid(6, 4, 9, 0.5, 2)
    alpha = 1.8
    c1 = math.exp(-alpha)
    f = random_field(g.nz, 3)
    for mx, my in ((0, 0), (1, 0), (2, 3), (5, 1)):
        tx, ty = 2 * math.pi * mx / g.nx, 2 * math.pi * my / g.ny
        jj, ii = np.meshgrid(np.arange(g.ny), np.arange(g.nx), indexing="ij")
        lat = np.exp(1j * (tx * ii + ty * jj))
        r = f[:, None, None] * lat[None]
        z = O.precond.truncated_laplacian(g, r[None], alpha)[0]
        fm = np.concatenate([[0], f[:-1]])  # f(k-1), zero below plane 0
        fp = np.concatenate([f[1:], [0]])   # f(k+1), zero above plane nz-1
        ref = ((1 + 2 * c1 * (math.cos(tx) + math.cos(ty))) * f + c1 * (fm + fp))[:, None, None] * lat[None]
        assert np.abs(z - ref).max() < 1e-14 * np.abs(ref).max()


def test_continuum_barrier_limit_is_second_order():
    # the continuum formula is approached as O(h^2) (the sharp step limits
    # the order for every N_f); checks that the discretisation is the
    # Schrodinger operator with the right units (hbar = m = 1)
    V0, a, E = 0.5, 2.0, 0.3
    kap = math.sqrt(2 * (V0 - E))
    Tc = 1 / (1 + V0 ** 2 * math.sinh(kap * a) ** 2 / (4 * E * (V0 - E)))
    errs = []
    for h in (0.2, 0.1):
        n = int(round(a / h))
        nz = n + 16
        g = Grid(2, 2, nz, h, 2)
        V = np.zeros(g.shape)
        V[8:8 + n] = V0
        P = O.Problem(g, V)
        psi = P.solve(E, [0])
        errs.append(abs(P.currents(E, 0, psi[0])[0] - Tc))
    assert errs[1] < errs[0] / 2.5


def _random_problem(nf, seed, kb=False, shape=(6, 6, 14), h=0.9, hz=None):
    g = Grid(shape[0], shape[1], shape[2], h, nf, hz_=hz)
    rng = np.random.default_rng(seed)
    V = 0.3 * rng.standard_normal(g.shape)
    nl = None
    if kb:
        from workloads.synth import _kb_projectors
        centres = [np.array([1.5, 1.8, 4.0]), np.array([2.0, 1.0, 5.5])]
        nl = _kb_projectors(g, centres, 0.8, 3, rng)
    return O.Problem(g, V, nl)


@pytest.mark.parametrize("nf,kb,hz", [(1, False, None), (2, False, None), (3, False, None), (2, True, None),
                                       (1, False, 0.7), (2, True, 0.75)])
def test_flux_conservation_and_reciprocity(nf, kb, hz):
    P = _random_problem(nf, 7 + nf, kb, hz=hz)
    E = 1.6
    modes = O.open_channels(P.g, E)
    assert len(modes) >= 5
    psiL = P.solve(E, modes, "L")
    TL = 0.0
    for m, p in zip(modes, psiL):
        T, R = P.currents(E, m, p, "L")
        assert abs(T + R - 1) < 1e-10
        assert -1e-12 < T < 1 + 1e-12
        TL += T
    psiR = P.solve(E, modes, "R")
    TR = sum(P.currents(E, m, p, "R")[0] for m, p in zip(modes, psiR))
    assert abs(TL - TR) < 1e-10
    eig = P.transmission_matrix_eigs(E, modes, psiL)
    assert abs(eig.sum() - TL) < 1e-10
    assert eig.min() > -1e-10 and eig.max() < 1 + 1e-10


@pytest.mark.parametrize("nf", [1, 2, 3])
def test_matrix_is_complex_symmetric(nf):
    P = _random_problem(nf, 3, kb=(nf == 2))
    A = P.matrix(0.9)
    assert abs(A - A.T).max() < 1e-12


def test_dense_solve_and_caroli_trace():
    """Total transmission equals the Caroli / Fisher-Lee trace
    Tr[Gamma_L G Gamma_R G^H] with G = A^-1 (dense): pins b, the incident
    current normalisation and the readout together."""
    P = _random_problem(2, 11)
    g = P.g
    E = 1.3
    A = P.matrix(E).toarray()
    G = np.linalg.inv(A)
    sL, sR = P.boundary_slice("L"), P.boundary_slice("R")
    caroli = np.real(np.trace(P.gamma(E, "L") @ G[sL, sR] @ P.gamma(E, "R") @ G[sL, sR].conj().T))
    modes = O.open_channels(g, E)
    psi = P.solve(E, modes)
    T = sum(P.currents(E, m, p)[0] for m, p in zip(modes, psi))
    assert abs(T - caroli) < 1e-10 * max(1, caroli)
    b = P.rhs(E, modes[0])
    assert np.abs(np.linalg.solve(A, b) - psi[0].ravel()).max() < 1e-10
    # the dense path of the oracle's solve equals the sparse LU
    psid = P.solve(E, modes, dense=True)
    assert np.abs(psid - psi).max() < 1e-10 * np.abs(psi).max()


def test_bordered_nonlocal_equals_dense_schur_complement():
    P = _random_problem(2, 5, kb=True)
    E = 0.8
    x = random_field(P.g.npts, 4)
    y = P.apply(E, x)
    A_loc = (E * np.eye(P.g.npts) - P.H_loc.toarray()).astype(complex)
    for side in ("L", "R"):
        s = P.boundary_slice(side)
        A_loc[s, s] -= P.sigma(E, side)
    Bd = P.B.toarray()
    A_dense = A_loc - Bd @ P.hD @ Bd.T
    assert np.abs(y - A_dense @ x).max() < 1e-11 * np.abs(y).max()
    modes = O.open_channels(P.g, E)
    psi = P.solve(E, modes[:2])
    for m, p in zip(modes[:2], psi):
        assert np.abs(A_dense @ p.ravel() - P.rhs(E, m)).max() < 1e-10


def test_interior_bond_current_equals_transmitted_current():
    """Current conservation across every plane cut inside the transition
    region (real V): the Gamma-based transmitted current must equal the bond
    current through each interior cut."""
    P = _random_problem(3, 21)
    g = P.g
    E = 1.1
    modes = O.open_channels(g, E)
    psi = P.solve(E, modes[:3])
    a = O.lead.z_hopping(g)
    for m, p in zip(modes[:3], psi):
        T, _ = P.currents(E, m, p)
        J = P.incident_current(E, m)
        for cut in range(g.nf, g.nz - g.nf + 1):
            Jc = 0.0
            for n in range(1, g.nf + 1):
                for q0 in range(cut - n, cut):
                    Jc += -2 * a[n] * np.sum(np.imag(np.conj(p[q0]) * p[q0 + n]))
            assert abs(Jc / J - T) < 1e-10


def test_gradient_matches_central_differences():
    P = _random_problem(2, 31, shape=(4, 4, 10), h=0.7)
    g = P.g
    Es = [0.9, 1.4]
    T0, grad = O.total_transmission_and_gradient(P, Es)
    assert abs(T0 - O.total_transmission(P, Es)) < 1e-11
    # the dense-LU path equals the sparse one
    T1, grad1 = O.total_transmission_and_gradient(P, Es, dense=True)
    assert abs(T1 - T0) < 1e-11 and np.abs(grad1 - grad).max() < 1e-10 * np.abs(grad).max()
    rng = np.random.default_rng(0)
    vox = rng.choice(g.npts, 12, replace=False)
    d = 1e-5
    for v in vox:
        Vp, Vm = P.V.copy(), P.V.copy()
        Vp.flat[v] += d
        Vm.flat[v] -= d
        fd = (O.total_transmission(O.Problem(g, Vp), Es) - O.total_transmission(O.Problem(g, Vm), Es)) / (2 * d)
        assert abs(fd - grad.flat[v]) < 1e-6 * max(1e-3, np.abs(grad).max())


def test_threshold_is_rejected():
    g = Grid(4, 4, 8, 0.5, 2)
    # the (1,0) lateral threshold is exactly eps of that mode
    eps = O.lateral_energy(g, 1)
    with pytest.raises(O.AtThreshold):
        O.LeadMode(g, eps, 1)


def test_workload_channel_counts():
    """Open-channel counts of the five workloads (Eq. (13) generalised to the
    workloads' FD orders): flat 1 at E=0.1; barrier 1 per energy; adjoint
    1/5/9/13; wide 45..57 per energy."""
    w1 = make(1)
    assert len(O.open_channels(w1.grid, 0.1)) >= 1
    w2 = make(2)
    assert [len(O.open_channels(w2.grid, E)) for E in w2.energies] == [1] * 8
    w5 = make(5)
    assert [len(O.open_channels(w5.grid, E)) for E in w5.energies] == [1, 5, 9, 13]
    from workloads import Grid as G_
    g4 = G_(48, 48, 4, 0.4, 2)
    n4 = [len(O.open_channels(g4, E)) for E in make(4, G_(48, 48, 4, 0.4, 2)).energies]
    assert min(n4) >= 40 and max(n4) <= 60 and sum(n4) == 768


def test_na_wire_stand_in():
    """The synthetic Na-like wires: the paper's cell (36 x 36 lateral points
    over 25.66 bohr, nz = 60 + 10 (n_atom - 1), length (n_atom - 1) d + 42.12
    with d = sqrt(3) a0 / 2), V = 0 in the electrodes, and the jellium Fermi
    energy of r_s = 3.99 (3.15 eV)."""
    from workloads import na_wire, jellium_fermi_energy
    assert abs(jellium_fermi_energy() * 27.211386 - 3.148) < 2e-3
    for n in (3, 8):
        w = na_wire(n)
        g = w.grid
        assert (g.nx, g.ny, g.nz, g.nf) == (36, 36, 60 + 10 * (n - 1), 1)
        assert abs(g.hx * 36 - 25.66) < 1e-12 and g.hy == g.hx
        assert abs(g.hz * g.nz - ((n - 1) * 8.11 * 3 ** 0.5 / 2 + 42.12)) < 1e-9
        assert g.hz == w.extra["hz"]
        assert np.abs(w.V[:3]).max() < 1e-6 and np.abs(w.V[-3:]).max() < 1e-6
        assert 0.19 < w.V.max() <= 0.2 and w.V.min() < -0.3
        # the lateral dispersion gives 9 open channels at E_F (the paper quotes 13
        # for its SCF wire; see the design notes)
        assert len(O.open_channels(g, float(w.energies[0]))) == 9


@pytest.mark.parametrize("nf,kb,hz", [(1, False, None), (2, True, 0.75), (3, False, None)])
def test_mode_amplitudes_and_scattering_matrix(nf, kb, hz):
    """The amplitude readout (the nf boundary values of each open channel
    expanded in the Bloch states leaving through that lead, Eq. (7)) against
    the current-based readout: T_mu = sum_nu (J_nu / J_mu) |t_nu mu|^2 and
    R_mu likewise, for incidence from both leads.  The assembled flux-
    normalised S-matrix is unitary (current conservation) and obeys the
    time-reversal relation S[b nu, a mu] = S[a -mu, b -nu] (real V,
    kappa = 0: time reversal maps the lateral wave G to -G)."""
    P = _random_problem(nf, 40 + nf, kb, hz=hz)
    g = P.g
    E = 1.6
    modes, S = P.smatrix(E)
    n = len(modes)
    assert n >= 5
    J = {m: O.LeadMode(g, E, m).J for m in modes}
    for side in ("L", "R"):
        psis = P.solve(E, modes, side)
        far, near = ("R", "L") if side == "L" else ("L", "R")
        for mu, p in zip(modes, psis):
            amp = P.amplitudes(E, mu, p, side)
            T = sum(J[nu] / J[mu] * abs(amp[far][nu]) ** 2 for nu in modes)
            R = sum(J[nu] / J[mu] * abs(amp[near][nu]) ** 2 for nu in modes)
            Tc, Rc = P.currents(E, mu, p, side)
            assert abs(T - Tc) < 1e-10 and abs(R - Rc) < 1e-10
    assert np.abs(S.conj().T @ S - np.eye(2 * n)).max() < 1e-10
    neg = [modes.index(((g.ny - m // g.nx) % g.ny) * g.nx + (g.nx - m % g.nx) % g.nx) for m in modes]
    perm = neg + [n + i for i in neg]
    assert np.abs(S - S[np.ix_(perm, perm)].T).max() < 1e-10


def test_scattering_matrix_of_the_flat_wire_is_pure_transmission():
    """V = 0: every channel passes with amplitude 1 referred to the plane
    next to each lead, i.e. S = [[0, D], [D, 0]] with D the phase of the free
    propagation from plane 0 to plane nz-1, x_mu^(nz-1)."""
    g = Grid(6, 6, 12, 0.9, 2, hy_=0.8, hz_=0.6)
    P = O.Problem(g, np.zeros(g.shape))
    E = 1.0
    modes, S = P.smatrix(E)
    n = len(modes)
    D = np.diag([O.LeadMode(g, E, m).x_in ** (g.nz - 1) for m in modes])
    assert np.abs(S[:n, :n]).max() < 1e-10 and np.abs(S[n:, n:]).max() < 1e-10
    assert np.abs(S[n:, :n] - D).max() < 1e-10 and np.abs(S[:n, n:] - D).max() < 1e-10


@pytest.mark.parametrize("nf,kb", [(1, False), (2, True), (3, False)])
def test_jacobi_diagonal_is_the_operator_diagonal(nf, kb):
    """Brute force on a small grid: the Jacobi diagonal equals e_i^T A e_i
    for every voxel i, with A applied to unit vectors by the operator's
    plain definition (Problem.apply)."""
    P = _random_problem(nf, 60 + nf, kb, shape=(4, 3, 2 * nf + 3), hz=0.7)
    g = P.g
    E = 0.9
    a = O.precond.jacobi_diagonal(P, E).ravel()
    I = np.eye(g.npts, dtype=complex)
    diag = np.array([P.apply(E, I[i])[i] for i in range(g.npts)])
    assert np.abs(a - diag).max() < 1e-12 * np.abs(diag).max()
    r = random_field((2,) + g.shape, 5)
    z = O.precond.jacobi(P, E, r)
    assert np.abs(z.reshape(2, -1) * diag[None] - r.reshape(2, -1)).max() < 1e-12 * np.abs(r).max()


# ------------------------------------------------ lateral Bloch vector kappa
KAPPAS = [(0.31, 0.0), (0.17, -0.42)]


@pytest.mark.parametrize("kappa", KAPPAS)
@pytest.mark.parametrize("nf", [1, 2, 3])
def test_flat_wire_at_nonzero_kappa(nf, kappa):
    """V = 0 at a lateral Bloch vector kappa: every open channel (counted at
    G + kappa) passes with T = 1, R = 0 and psi = Phi_in."""
    g = Grid(6, 5, 12, 0.9, nf, hz_=0.7)
    P = O.Problem(g, np.zeros(g.shape), kappa=kappa)
    E = 1.2
    modes = O.open_channels(g, E, kappa)
    assert len(modes) >= 3
    psi = P.solve(E, modes)
    for m, p in zip(modes, psi):
        Phi = P.incident(E, m)[nf:nf + g.nz]
        assert np.abs(p - Phi).max() < 1e-11
        T, R = P.currents(E, m, p)
        assert abs(T - 1) < 1e-11 and abs(R) < 1e-11


@pytest.mark.parametrize("nf", [1, 2])
def test_kappa_transpose_identity(nf):
    """A(kappa)^T = A(-kappa) (the Bloch phases of the lateral wrap and of the
    self-energies conjugate under transposition), and A(kappa) is not
    complex symmetric for kappa != 0."""
    P = _random_problem(nf, 70 + nf, kb=(nf == 2))
    Pp = O.Problem(P.g, P.V, P.nl, kappa=(0.23, -0.11))
    Pm = O.Problem(P.g, P.V, P.nl, kappa=(-0.23, 0.11))
    A, Am = Pp.matrix(0.9), Pm.matrix(0.9)
    assert abs(A - Am.T).max() < 1e-12
    assert abs(A - A.T).max() > 1e-3


def _eps_nf1_kappa(g, mode, kappa):
    nux = O.mode_numbers(g.nx)[mode % g.nx]
    nuy = O.mode_numbers(g.ny)[mode // g.nx]
    return ((1 - math.cos(2 * math.pi * nux / g.nx + kappa[0] * g.hx)) / g.hx ** 2
            + (1 - math.cos(2 * math.pi * nuy / g.ny + kappa[1] * g.hy)) / g.hy ** 2)


@pytest.mark.parametrize("kappa", KAPPAS)
def test_uniform_barrier_closed_form_at_nonzero_kappa(kappa):
    """Laterally uniform barrier: the channels decouple, and each one follows
    the lattice square-barrier closed form at E - eps(G + kappa)."""
    g = UNIFORM
    V = np.zeros(g.shape)
    V[8:15] = 0.5
    P = O.Problem(g, V, kappa=kappa)
    E = 1.8
    modes = O.open_channels(g, E, kappa)
    assert len(modes) >= 4
    psi = P.solve(E, modes)
    for m, p in zip(modes, psi):
        T, R = P.currents(E, m, p)
        assert abs(T - _barrier_closed_form(E - _eps_nf1_kappa(g, m, kappa), 0.5, 7, g.hz)) < 1e-11
        assert abs(T + R - 1) < 1e-11


@pytest.mark.parametrize("nf", [1, 2])
def test_flux_caroli_and_reciprocity_at_nonzero_kappa(nf):
    """Random V at kappa != 0: T + R = 1 per channel, the total transmission
    equals the Caroli trace and is the same from both leads, the S-matrix is
    unitary, and time reversal maps (kappa, G) to (-kappa, -G):
    S(kappa)[b nu, a mu] = S(-kappa)[a -mu, b -nu]."""
    P0 = _random_problem(nf, 80 + nf, kb=(nf == 2))
    kappa = (0.29, -0.13)
    P = O.Problem(P0.g, P0.V, P0.nl, kappa=kappa)
    Pm = O.Problem(P0.g, P0.V, P0.nl, kappa=(-kappa[0], -kappa[1]))
    g = P.g
    E = 1.6
    modes = O.open_channels(g, E, kappa)
    assert len(modes) >= 4
    TL = 0.0
    for m, p in zip(modes, P.solve(E, modes, "L")):
        T, R = P.currents(E, m, p, "L")
        assert abs(T + R - 1) < 1e-10
        TL += T
    TR = sum(P.currents(E, m, p, "R")[0] for m, p in zip(modes, P.solve(E, modes, "R")))
    assert abs(TL - TR) < 1e-10
    A = P.matrix(E).toarray()
    G = np.linalg.inv(A)
    sL, sR = P.boundary_slice("L"), P.boundary_slice("R")
    n = g.npts
    caroli = np.real(np.trace(P.gamma(E, "R") @ G[:n, :n][sR, sL] @ P.gamma(E, "L") @ G[:n, :n][sR, sL].conj().T))
    assert abs(TL - caroli) < 1e-10 * max(1, caroli)
    modes_p, S = P.smatrix(E)
    modes_m, Sm = Pm.smatrix(E)
    k = len(modes_p)
    assert np.abs(S.conj().T @ S - np.eye(2 * k)).max() < 1e-10
    neg = [modes_m.index(((g.ny - m // g.nx) % g.ny) * g.nx + (g.nx - m % g.nx) % g.nx) for m in modes_p]
    perm = neg + [k + i for i in neg]
    assert np.abs(S - Sm[np.ix_(perm, perm)].T).max() < 1e-10


def test_truncated_laplacian_bloch_phases():
    """Eq. (17) on a Bloch wave exp(i (G + kappa) . r) f(k): the lateral
    neighbours multiply it by 2 cos((G_mu + kappa_mu) h_mu) across the cell."""
    g = Grid(6, 4, 7, 0.5, 2, hy_=0.6)
    kappa = (0.4, -0.7)
    alpha = 2.4
    c1 = math.exp(-alpha)
    f = random_field(g.nz, 9)
    jj, ii = np.meshgrid(np.arange(g.ny), np.arange(g.nx), indexing="ij")
    for mx, my in ((0, 0), (2, 1), (5, 3)):
        tx = 2 * math.pi * mx / g.nx + kappa[0] * g.hx
        ty = 2 * math.pi * my / g.ny + kappa[1] * g.hy
        lat = np.exp(1j * (tx * ii + ty * jj))
        r = f[:, None, None] * lat[None]
        z = O.precond.truncated_laplacian(g, r[None], alpha, kappa)[0]
        fm = np.concatenate([[0], f[:-1]])
        fp = np.concatenate([f[1:], [0]])
        ref = ((1 + 2 * c1 * (math.cos(tx) + math.cos(ty))) * f + c1 * (fm + fp))[:, None, None] * lat[None]
        assert np.abs(z - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("nf", [2, 3])
def test_kinetic_on_the_shortest_lateral_period(nf):
    """nx = ny = nf: lateral neighbours at distance n <= nf wrap across the
    cell (onto the point itself at n = nx).  Lateral plane waves stay
    eigenvectors of the lateral couplings, with the lateral energy of Eq. (13)
    generalised to order 2 nf."""
    from oracle.fd import fd_coefficients
    from oracle.system import kinetic
    g = Grid(nf, nf, 4 * nf, 0.5, nf)
    H = kinetic(g).toarray()
    N = g.nx * g.ny
    c = fd_coefficients(nf)
    B = H[N:2 * N, N:2 * N] - np.eye(N) * (-0.5 * c[0] / g.hz ** 2)  # one plane, z diagonal removed
    jj, ii = np.meshgrid(np.arange(g.ny), np.arange(g.nx), indexing="ij")
    for m in range(N):
        lat = np.exp(2j * np.pi * ((m % g.nx) * ii / g.nx + (m // g.nx) * jj / g.ny)).ravel()
        assert np.allclose(B @ lat, O.lateral_energy(g, m) * lat, atol=1e-12)
