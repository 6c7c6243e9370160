"""Seeded synthetic inputs for the IOBM scattering solve.

This module only *generates inputs*: grids, local potentials V(r), energies,
and the real Kleinman-Bylander projector data of the nonlocal term.  It holds
none of the method's arithmetic (no stencil, no self-energy, no solve), so the
CPU oracle and the GPU library can both be fed from it without sharing code.

The paper's own potentials (self-consistent LDA potentials of Na, Ir and Au
wires, Sec. III and IV) are not available; every workload below is a
synthetic stand-in with the geometry class of the paper's wires: a periodic
lateral cell, a transition region along z, jellium leads at V = 0.

Conventions (Hartree atomic units):
  * grid point (i, j, k) sits at r = (i*hx, j*hy, k*hz), i < nx, j < ny,
    k < nz (the spacings may differ per direction, as in Eq. (1));
  * arrays are indexed [k][j][i] (x fastest), float64;
  * the lateral cell is periodic with L = n*h; distances to atoms use the
    minimum image laterally and the plain difference along z.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Grid:
    """Grid of the transition region.  `h` is the spacing along x; y and z
    use it too unless `hy_` / `hz_` give their own."""
    nx: int
    ny: int
    nz: int
    h: float
    nf: int  # finite-difference half width: 1, 2 or 3 (2nd/4th/6th order)
    hy_: float | None = None
    hz_: float | None = None

    @property
    def hx(self):
        return self.h

    @property
    def hy(self):
        return self.h if self.hy_ is None else self.hy_

    @property
    def hz(self):
        return self.h if self.hz_ is None else self.hz_

    @property
    def spacings(self):
        return (self.hx, self.hy, self.hz)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def npts(self):
        return self.nx * self.ny * self.nz


@dataclass
class Nonlocal:
    """Separable nonlocal term V_NL = sum_a B_a D_a h^3 B_a^T.

    support[a]: int64 flat voxel indices (k*ny + j)*nx + i of centre a,
    beta[a]:    float64 [rank][len(support[a])] projector values there,
    D[a]:       float64 [rank][rank] symmetric coupling matrix (Ha).
    """
    support: list
    beta: list
    D: list

    @property
    def rank(self):
        return self.D[0].shape[0]


@dataclass
class Workload:
    name: str
    grid: Grid
    V: np.ndarray
    energies: np.ndarray
    nonlocal_: Nonlocal | None = None
    # incident channels: None = every open channel at each energy,
    # "lowest" = only the (0, 0) lateral mode
    channels: str | None = None
    extra: dict = field(default_factory=dict)


def _coords(g: Grid):
    k, j, i = np.meshgrid(np.arange(g.nz), np.arange(g.ny), np.arange(g.nx),
                          indexing="ij")
    return i * g.hx, j * g.hy, k * g.hz


def _min_image(d, L):
    return d - L * np.round(d / L)


def _wells(g: Grid, centres, depth, sigma):
    X, Y, Z = _coords(g)
    Lx, Ly = g.nx * g.hx, g.ny * g.hy
    V = np.zeros(g.shape)
    for R in centres:
        dx = _min_image(X - R[0], Lx)
        dy = _min_image(Y - R[1], Ly)
        dz = Z - R[2]
        V -= depth * np.exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * sigma * sigma))
    return V


def _well_centres(g: Grid, n, spacing, jitter, rng):
    zc = (g.nz - 1) * g.hz / 2.0
    base = [(g.nx * g.hx / 2.0, g.ny * g.hy / 2.0, zc + spacing * (a - (n - 1) / 2.0))
            for a in range(n)]
    return [np.array(b) + rng.uniform(-jitter, jitter, 3) for b in base]


def flat(grid: Grid | None = None) -> Workload:
    """Flat jellium wire: V = 0, E = 0.1 Ha, lowest lateral channel only."""
    g = grid or Grid(8, 8, 24, 0.4, 2)
    return Workload("flat", g, np.zeros(g.shape), np.array([0.1]), channels="lowest")


def barrier(grid: Grid | None = None, seed: int = 1002) -> Workload:
    """Laterally uniform Gaussian barrier (0.05 Ha, width 3 bohr, centred in z)
    plus a smooth random perturbation built from the four lowest Fourier
    modes, rescaled to max |dV| = 0.005 Ha.  8 energies in [0.02, 0.30] Ha."""
    g = grid or Grid(16, 16, 48, 0.4, 2)
    rng = np.random.default_rng(seed)
    X, Y, Z = _coords(g)
    zc = (g.nz - 1) * g.hz / 2.0
    V = 0.05 * np.exp(-(Z - zc) ** 2 / (2.0 * 3.0 ** 2))
    L = (g.nx * g.hx, g.ny * g.hy, g.nz * g.hz)
    dV = np.zeros(g.shape)
    for n in ((1, 0, 0), (0, 1, 0), (1, 1, 0), (0, 0, 1)):
        a = rng.uniform(-1.0, 1.0)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        arg = 2 * np.pi * (n[0] * X / L[0] + n[1] * Y / L[1] + n[2] * Z / L[2])
        dV += a * np.cos(arg + ph)
    V = V + 0.005 * dV / np.abs(dV).max()
    return Workload("barrier", g, V, np.linspace(0.02, 0.30, 8))


def _kb_projectors(g: Grid, centres, sigma, rank, rng):
    """Rank-`rank` real projectors per centre: beta_p = sum_q M_pq phi_q with
    phi_q in {1, x/s, y/s, z/s} * exp(-r^2/(2 s^2)), cut at r = 3 s, each
    normalised to h^3 sum beta^2 = 1; D = diag(U(0.05, 0.5)) Ha."""
    X, Y, Z = _coords(g)
    Lx, Ly = g.nx * g.hx, g.ny * g.hy
    support, beta, D = [], [], []
    for R in centres:
        dx = _min_image(X - R[0], Lx)
        dy = _min_image(Y - R[1], Ly)
        dz = Z - R[2]
        r2 = dx * dx + dy * dy + dz * dz
        mask = r2 <= (3.0 * sigma) ** 2
        idx = np.flatnonzero(mask.ravel()).astype(np.int64)
        env = np.exp(-r2.ravel()[idx] / (2.0 * sigma * sigma))
        phi = np.stack([env,
                        dx.ravel()[idx] / sigma * env,
                        dy.ravel()[idx] / sigma * env,
                        dz.ravel()[idx] / sigma * env])[:rank]
        M = rng.standard_normal((rank, phi.shape[0]))
        b = M @ phi
        b /= np.sqrt(g.hx * g.hy * g.hz * np.sum(b * b, axis=1))[:, None]
        support.append(idx)
        beta.append(np.ascontiguousarray(b))
        D.append(np.diag(rng.uniform(0.05, 0.5, rank)))
    return Nonlocal(support, beta, D)


def chain(grid: Grid | None = None, seed: int = 1003, kb: bool = True) -> Workload:
    """Atomic-chain-like wire: 6 Gaussian wells (depth 0.4 Ha, sigma 1.2 bohr,
    6 bohr apart along the axis, jitter +-0.2 bohr) and a rank-4 KB term per
    well.  32 energies in [0.05, 1.35] Ha, every open channel."""
    g = grid or Grid(24, 24, 96, 0.35, 3)
    rng = np.random.default_rng(seed)
    centres = _well_centres(g, 6, 6.0, 0.2, rng)
    V = _wells(g, centres, 0.4, 1.2)
    nl = _kb_projectors(g, centres, 1.2, 4, rng) if kb else None
    return Workload("chain", g, V, np.linspace(0.05, 1.35, 32), nonlocal_=nl,
                    extra={"centres": centres})


CONFIG4_ENERGIES = np.array([0.71, 0.725, 0.74, 0.755, 0.77, 0.785, 0.80, 0.815,
                             0.83, 0.845, 0.87, 0.885, 0.90, 0.92, 0.935, 0.95])


def wide(grid: Grid | None = None, seed: int = 1004) -> Workload:
    """Large cross-section: smooth random V of amplitude 0.02 Ha, built from
    white noise convolved (periodically, via FFT) with a Gaussian of
    correlation length 2 bohr.  16 energies with 45-57 open channels each."""
    g = grid or Grid(48, 48, 128, 0.4, 2)
    rng = np.random.default_rng(seed)
    F = rng.standard_normal(g.shape)
    d2 = 0.0
    for ax, (n, h) in enumerate(zip(g.shape, (g.hz, g.hy, g.hx))):
        m = np.arange(n)
        m = np.minimum(m, n - m).astype(float) * h
        sh = [1, 1, 1]
        sh[ax] = n
        d2 = d2 + (m ** 2).reshape(sh)
    kern = np.exp(-d2 / (2.0 * 2.0 ** 2))
    F = np.real(np.fft.ifftn(np.fft.fftn(F) * np.fft.fftn(kern)))
    V = 0.02 * F / np.abs(F).max()
    return Workload("wide", g, V, CONFIG4_ENERGIES.copy())


def adjoint(grid: Grid | None = None, seed: int = 1005) -> Workload:
    """Adjoint workload: 4 Gaussian wells (well parameters of the chain
    workload), no KB term; total transmission over every open channel at
    4 energies.  64 finite-difference voxels are drawn with the same seed."""
    g = grid or Grid(32, 32, 96, 0.4, 2)
    rng = np.random.default_rng(seed)
    centres = _well_centres(g, 4, 6.0, 0.2, rng)
    V = _wells(g, centres, 0.4, 1.2)
    return Workload("adjoint", g, V, np.array([0.08, 0.20, 0.35, 0.55]),
                    extra={"centres": centres, "fd_rng_seed": seed})


NA_RS = 3.99              # Wigner-Seitz radius of the jellium electrodes (bohr)
NA_A0 = 8.11              # Na bulk lattice constant (bohr)
NA_D = 3.0 ** 0.5 * NA_A0 / 2.0   # interatomic distance of the [110] strand


def jellium_fermi_energy(rs: float = NA_RS) -> float:
    """Free-electron Fermi energy (Ha) of jellium of Wigner-Seitz radius rs,
    measured from the band bottom: k_F = (9 pi / 4)^(1/3) / rs."""
    kf = (9.0 * np.pi / 4.0) ** (1.0 / 3.0) / rs
    return 0.5 * kf * kf


def na_wire(n_atom: int, seed: int = 1006, nx: int = 36, nz: int | None = None) -> Workload:
    """Synthetic stand-in for the paper's single-row Na wires between jellium
    electrodes (Sec. III): n_atom = 3..8 atoms NA_D apart on the axis of a
    36 x 36 lateral cell of 25.66 bohr, nz = 60 + 10 (n_atom - 1) planes over
    (n_atom - 1) NA_D + 42.12 bohr, 2nd-order FD, one energy at the jellium
    Fermi level.  V is 0 inside the electrodes, which end 2.867 bohr
    (sqrt(2) a0 / 4) beyond the edge atoms; between them V rises to 0.2 Ha
    (logistic steps 0.5 bohr wide) and each atom is a Gaussian well of depth
    0.6 Ha and width 3 bohr (positions jittered by U(+-0.1) bohr), which
    overlap into one conducting channel along the axis.  The grid spacing
    differs along z (grid.hz; also extra["hz"]).

    nx < 36 keeps the lateral spacing and narrows the cell; nz sets another
    plane count over the same length (both for oracle-sized parity cases)."""
    if not 1 <= n_atom <= 20:
        raise ValueError("n_atom out of range")
    hx = 25.66 / 36
    if nz is None:
        nz = 60 + 10 * (n_atom - 1)
    hz = ((n_atom - 1) * NA_D + 42.12) / nz
    g = Grid(nx, nx, nz, hx, 1, hz_=hz)
    rng = np.random.default_rng(seed + n_atom)
    X, Y, Z = _coords(g)
    L = nx * hx
    zc = (nz - 1) * hz / 2.0
    za = [zc + NA_D * (a - (n_atom - 1) / 2.0) for a in range(n_atom)]
    zl, zr = za[0] - 2.0 ** 0.5 * NA_A0 / 4.0, za[-1] + 2.0 ** 0.5 * NA_A0 / 4.0
    w = 0.5
    V = 0.2 / (1.0 + np.exp(-(Z - zl) / w)) / (1.0 + np.exp(-(zr - Z) / w))
    centres = []
    for z0 in za:
        R = np.array([L / 2.0, L / 2.0, z0]) + rng.uniform(-0.1, 0.1, 3)
        centres.append(R)
        dx = _min_image(X - R[0], L)
        dy = _min_image(Y - R[1], L)
        V = V - 0.6 * np.exp(-(dx * dx + dy * dy + (Z - R[2]) ** 2) / (2.0 * 3.0 ** 2))
    return Workload(f"na{n_atom}", g, V, np.array([jellium_fermi_energy()]),
                    extra={"hz": hz, "centres": centres})


CONFIGS = {1: flat, 2: barrier, 3: chain, 4: wide, 5: adjoint}


def make(cfg: int, grid: Grid | None = None) -> Workload:
    """Workload of configuration `cfg` (1..5), optionally on another grid
    with the same recipe (used for oracle-sized parity cases)."""
    return CONFIGS[cfg](grid)


def random_field(shape, seed, complex_=True):
    """Seeded complex (or real) Gaussian test vector, e.g. for matvec parity."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(shape)
    if complex_:
        x = x + 1j * rng.standard_normal(shape)
    return x
