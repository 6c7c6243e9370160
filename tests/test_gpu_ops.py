"""Parity of the individual HIP kernels (through the C ABI) with the CPU
oracle, on seeded inputs: electrode mode setup, right-hand side, operator,
both preconditioners.  Sizes span several blocks and ragged tails (lateral
planes of 120 and 480 points, z chunks of 16 planes over 40), the 32 x 32
and 48 x 48 cross-sections of the adjoint and wide-wire workloads, grids
with a different spacing per direction, and every launch shape."""
import numpy as np
import pytest

import oracle as O
from workloads import Grid, random_field, make

pytestmark = pytest.mark.gpu

GRIDS = [Grid(12, 10, 40, 0.4, 2), Grid(24, 20, 40, 0.45, 3), Grid(10, 12, 18, 0.6, 1),
         Grid(12, 10, 40, 0.4, 2, hy_=0.45, hz_=0.35)]


def gid(g):
    s = f"{g.nx}x{g.ny}x{g.nz}nf{g.nf}"
    return s if g.spacings == (g.h,) * 3 else s + "h" + "-".join(f"{h:g}" for h in g.spacings)


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _solver(g, V, nl=None):
    from paper_1009_5300_amd import iobm
    s = iobm.Solver(g.nx, g.ny, g.nz, g.spacings, g.nf)
    s.set_potential(V)
    if nl is not None:
        s.set_nonlocal(nl)
    return s


def _V(g, seed):
    return 0.2 * random_field(g.shape, seed, complex_=False)


@pytest.mark.parametrize("g", GRIDS, ids=gid)
@pytest.mark.parametrize("E", [0.3, 1.7])
def test_channels_and_self_energy(torch, g, E):
    s = _solver(g, np.zeros(g.shape))
    ids, kz, v = s.channels(E)
    ref = O.open_channels(g, E)
    assert list(ids) == list(ref)
    for m, k in zip(ids, kz):
        x = O.LeadMode(g, E, m).x_in
        assert abs(k - np.angle(x) / g.hz) < 1e-12
    sig = s.self_energy(E)
    for m in range(g.nx * g.ny):
        S = O.LeadMode(g, E, m).sigma_right()
        assert np.abs(sig[m] - S).max() <= 1e-12 * np.abs(S).max()


def test_threshold_energy_is_rejected(torch):
    from paper_1009_5300_amd import iobm
    g = Grid(8, 8, 16, 0.5, 2)
    s = _solver(g, np.zeros(g.shape))
    with pytest.raises(iobm.IobmError) as e:
        s.channels(O.lateral_energy(g, 1))
    assert e.value.status == 7


@pytest.mark.parametrize("g", GRIDS, ids=gid)
def test_rhs(torch, g):
    E = 1.7
    s = _solver(g, np.zeros(g.shape))
    P = O.Problem(g, np.zeros(g.shape))
    modes = O.open_channels(g, E)
    for side, sname in ((0, "L"), (1, "R")):
        b = s.rhs(E, modes, side).cpu().numpy()
        for k, m in enumerate(modes):
            ref = P.rhs(E, m, sname).reshape(g.shape)
            assert np.abs(b[k] - ref).max() <= 1e-12 * np.abs(ref).max()


# square lateral planes take the in-register FFT path of the electrode term;
# 32 x 32 and 48 x 48 are the cross-sections of the adjoint and wide-wire
# workloads (the latter runs the 768-thread stencil and the 48-point
# electrode kernel), the last grid the Na-like cell with h_z != h_x
APPLY_GRIDS = GRIDS + [Grid(8, 8, 24, 0.4, 1), Grid(16, 16, 20, 0.4, 2), Grid(24, 24, 16, 0.35, 3),
                       Grid(32, 32, 40, 0.4, 2), Grid(48, 48, 40, 0.4, 2),
                       Grid(12, 12, 40, 25.66 / 36, 1, hz_=1.4052)]


@pytest.mark.parametrize("g", APPLY_GRIDS, ids=gid)
@pytest.mark.parametrize("kb", [False, True])
def test_apply_matches_oracle(torch, g, kb):
    from paper_1009_5300_amd import iobm
    from workloads.synth import _kb_projectors
    V = _V(g, 11)
    nl = None
    if kb:
        rng = np.random.default_rng(5)
        Lx, Ly, Lz = g.nx * g.hx, g.ny * g.hy, g.nz * g.hz
        centres = [np.array([Lx / 2, Ly / 3, 0.3 * Lz]), np.array([Lx / 3, Ly / 2, 0.6 * Lz]),
                   np.array([0.1, 0.2, 0.2])]  # last one straddles the periodic edge and plane 0
        nl = _kb_projectors(g, centres, 1.0, 4, rng)
    s = _solver(g, V, nl)
    P = O.Problem(g, V, nl)
    E = 0.9  # 44 mHa and 10 mHa from the nearest channel thresholds of the 32 and 48 point planes
    x = random_field((3,) + g.shape, 21)
    ref = P.apply(E, x.reshape(3, -1)).reshape(x.shape)
    xt = torch.as_tensor(x, device="cuda")
    y = s.apply(E, xt, iobm.C128).cpu().numpy()
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    y32 = s.apply(E, xt.to(torch.complex64), iobm.C64_REFINED).cpu().numpy()
    assert np.abs(y32 - ref).max() <= 2e-5 * np.abs(ref).max()


def _random_projectors(g, ncen, rank, seed):
    """ncen centres of rank-`rank` projectors with random values on the
    sphere supports of the synthetic generator (overlapping, some wrapping
    the periodic edge) and random symmetric D."""
    from workloads.synth import Nonlocal, _kb_projectors
    rng = np.random.default_rng(seed)
    L = np.array([g.nx * g.hx, g.ny * g.hy, g.nz * g.hz])
    centres = [rng.uniform(0, 1, 3) * L for _ in range(ncen)]
    base = _kb_projectors(g, centres, 1.0, 1, rng)
    beta, D = [], []
    for idx in base.support:
        b = rng.standard_normal((rank, len(idx)))
        beta.append(b / np.sqrt(g.hx * g.hy * g.hz * np.sum(b * b, axis=1))[:, None])
        M = rng.uniform(-1.0, 1.0, (rank, rank))
        D.append(M + M.T)
    return Nonlocal(base.support, beta, D)


@pytest.mark.parametrize("ncen,rank,nrhs", [(1, 1, 5), (10, 4, 37), (16, 8, 70)],
                         ids=["1proj_5rhs", "40proj_37rhs", "128proj_70rhs"])
def test_nonlocal_apply_projector_tiles_and_rhs_groups(torch, ncen, rank, nrhs):
    """The nonlocal term with 1 to 128 projectors (one to eight 16-wide MFMA
    projector tiles) and right-hand-side counts that leave the last 32-wide
    projection group and the last 16-wide back-projection group partly
    filled, on a grid whose support union spans many 64-voxel chunks and
    voxel splits: complex128 to 1e-12 and complex64 to 2e-5 of the oracle's
    operator, and the nonlocal contribution alone (with the term minus
    without it, 0.3 to 1.5 percent of the operator here) to 1e-10 of its size."""
    from paper_1009_5300_amd import iobm
    g = Grid(24, 24, 32, 0.4, 2)
    nl = _random_projectors(g, ncen, rank, 60 + ncen)
    V = _V(g, 12)
    s = _solver(g, V, nl)
    P = O.Problem(g, V, nl)
    E = 0.9
    x = random_field((nrhs,) + g.shape, 22)
    ref = P.apply(E, x.reshape(nrhs, -1)).reshape(x.shape)
    xt = torch.as_tensor(x, device="cuda")
    y = s.apply(E, xt, iobm.C128).cpu().numpy()
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    y32 = s.apply(E, xt.to(torch.complex64), iobm.C64_REFINED).cpu().numpy()
    assert np.abs(y32 - ref).max() <= 2e-5 * np.abs(ref).max()
    # the nonlocal contribution alone: with the term minus without it
    ref_nl = ref - O.Problem(g, V).apply(E, x.reshape(nrhs, -1)).reshape(x.shape)
    y_nl = y - _solver(g, V).apply(E, xt, iobm.C128).cpu().numpy()
    assert np.abs(y_nl - ref_nl).max() <= 1e-10 * np.abs(ref_nl).max()


@pytest.mark.parametrize("g", GRIDS, ids=gid)
def test_truncated_laplacian_preconditioner(torch, g):
    from paper_1009_5300_amd import iobm
    s = _solver(g, np.zeros(g.shape))
    r = random_field((2,) + g.shape, 3)
    for alpha in (1.8, 3.0):
        ref = O.precond.truncated_laplacian(g, r, alpha)
        z = s.precondition(iobm.PC_TRUNCATED_LAPLACIAN, torch.as_tensor(r, device="cuda"), alpha=alpha).cpu().numpy()
        assert np.abs(z - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("g", GRIDS, ids=gid)
def test_lateral_fft_preconditioner_is_flat_wire_inverse(torch, g):
    from paper_1009_5300_amd import iobm
    s = _solver(g, np.zeros(g.shape))
    E = 1.7
    r = random_field((2,) + g.shape, 4)
    ref = O.precond.flat_wire_inverse(g, E, r)
    rt = torch.as_tensor(r, device="cuda")
    z = s.precondition(iobm.PC_LATERAL_FFT, rt, E=E).cpu().numpy()
    assert np.abs(z - ref).max() <= 1e-10 * np.abs(ref).max()
    z32 = s.precondition(iobm.PC_LATERAL_FFT, rt.to(torch.complex64), E=E, precision=iobm.C64_REFINED).cpu().numpy()
    assert np.abs(z32 - ref).max() <= 1e-4 * np.abs(ref).max()


def test_bad_arguments_return_status(torch):
    from paper_1009_5300_amd import iobm
    g = Grid(8, 8, 16, 0.5, 2)
    s = iobm.Solver(g.nx, g.ny, g.nz, g.spacings, g.nf)
    with pytest.raises(iobm.IobmError) as e:  # solve before the potential is set
        s.solve([0.3])
    assert e.value.status == 2
    V = np.zeros(g.shape)
    V[3, 2, 1] = np.nan
    with pytest.raises(iobm.IobmError) as e:
        s.set_potential(V)
    assert e.value.status == 1
    s.set_potential(np.zeros(g.shape))
    with pytest.raises(iobm.IobmError) as e:  # closed channel requested
        s.solve([0.3], channels=[[5]])
    assert e.value.status == 1
    with pytest.raises(iobm.IobmError) as e:
        s.solve([0.3], opts=iobm.default_opts(tol=0.0))
    assert e.value.status == 1


SQUARE = [Grid(8, 8, 24, 0.4, 1), Grid(16, 16, 20, 0.4, 2), Grid(24, 24, 16, 0.35, 3), Grid(12, 12, 40, 0.4, 2)]


@pytest.mark.parametrize("g", SQUARE, ids=gid)
def test_lateral_fft_preconditioner_square_planes(torch, g):
    """Square lateral planes take the in-register FFT path."""
    from paper_1009_5300_amd import iobm
    s = _solver(g, np.zeros(g.shape))
    E = 1.1
    r = random_field((2,) + g.shape, 8)
    ref = O.precond.flat_wire_inverse(g, E, r)
    rt = torch.as_tensor(r, device="cuda")
    z = s.precondition(iobm.PC_LATERAL_FFT, rt, E=E).cpu().numpy()
    assert np.abs(z - ref).max() <= 1e-10 * np.abs(ref).max()
    z32 = s.precondition(iobm.PC_LATERAL_FFT, rt.to(torch.complex64), E=E, precision=iobm.C64_REFINED).cpu().numpy()
    assert np.abs(z32 - ref).max() <= 1e-4 * np.abs(ref).max()


@pytest.mark.parametrize("n,nz", [(32, 96), (48, 128)])
def test_lateral_fft_preconditioner_inverts_flat_operator(torch, n, nz):
    """At the workloads' cross-sections (any size): P (A_0 x) = x, with A_0 x
    the oracle's flat-wire operator applied to a seeded x."""
    from paper_1009_5300_amd import iobm
    g = Grid(n, n, nz, 0.4, 2)
    s = _solver(g, np.zeros(g.shape))
    E = 0.8
    x = random_field((1,) + g.shape, 9)
    y = O.Problem(g, np.zeros(g.shape)).apply(E, x.reshape(1, -1)).reshape(x.shape)
    z = s.precondition(iobm.PC_LATERAL_FFT, torch.as_tensor(y, device="cuda"), E=E).cpu().numpy()
    assert np.abs(z - x).max() <= 1e-9 * np.abs(x).max()
    z32 = s.precondition(iobm.PC_LATERAL_FFT, torch.as_tensor(y, device="cuda").to(torch.complex64), E=E,
                         precision=iobm.C64_REFINED).cpu().numpy()
    assert np.abs(z32 - x).max() <= 1e-3 * np.abs(x).max()


# square planes of the register transforms take the partials in the z filter
# (16x16: 4 full pair blocks, nf 2 and 3; 12x12: a ragged third block),
# unless the pair blocks outnumber the planes (24x24x8: 9 blocks, 8 planes),
# which keeps them in the inverse transform (sizes kept to what the oracle's
# dense per-mode inverse finishes in seconds)
RZ_GRIDS = [GRIDS[0], GRIDS[2], Grid(16, 16, 20, 0.4, 2), Grid(12, 12, 40, 0.4, 2), Grid(9, 7, 20, 0.5, 2),
            Grid(7, 10, 33, 0.5, 3), Grid(16, 16, 20, 0.4, 3), Grid(24, 24, 8, 0.4, 2)]


@pytest.mark.parametrize("g", RZ_GRIDS, ids=gid)
def test_preconditioner_rz_partials(torch, g):
    """r^T z from the solver's own reductions (for the lateral-Fourier
    preconditioner taken in mode space, sum_k R(-k) Z(k) / Nxy, which pairs
    every lateral mode with its negative: odd plane sizes have one
    self-paired mode, even ones four) against the bilinear form of the
    oracle's z = P r."""
    from paper_1009_5300_amd import iobm
    s = _solver(g, np.zeros(g.shape))
    E = 1.3
    r = random_field((3,) + g.shape, 11)
    rt = torch.as_tensor(r, device="cuda")
    refs = {iobm.PC_LATERAL_FFT: O.precond.flat_wire_inverse(g, E, r),
            iobm.PC_TRUNCATED_LAPLACIAN: O.precond.truncated_laplacian(g, r, 1.8),
            iobm.PC_NONE: r}
    for kind, ref in refs.items():
        a, b = r.reshape(len(r), -1), ref.reshape(len(r), -1)
        rz_ref = (a * b).sum(axis=1)  # no conjugation
        scale = (np.abs(a) * np.abs(b)).sum(axis=1)
        for prec, rr, tol in ((iobm.C128, rt, 1e-11), (iobm.C64_REFINED, rt.to(torch.complex64), 2e-5)):
            _, rz = s.precondition(kind, rr, alpha=1.8, E=E, precision=prec, want_rz=True)
            assert np.all(np.abs(rz - rz_ref) <= tol * scale), (kind, prec, rz, rz_ref)


def _shapes(s, g):
    """Every launch shape the library accepts for this grid: the cache-based
    stencil, and the 2.5D stencil at each points-per-thread and chunk length,
    with the register and the LDS plane FFT."""
    from paper_1009_5300_amd import iobm
    out = []
    cands = [dict(stencil=2, plane_fft=2)]
    for ppt in (1, 2, 3, 4):
        for zc in (8, 16, 32, 64):
            cands.append(dict(stencil=1, points_per_thread=ppt, planes_per_block=zc, plane_fft=1))
    cands.append(dict(stencil=1, plane_fft=2))
    for c in cands:
        try:
            s.set_launch_shape(iobm.C128, c)
        except iobm.IobmError as e:
            assert e.status == 8, e  # UNSUPPORTED for this grid, never another error
            continue
        out.append(c)
    return out


SHAPE_GRIDS = [Grid(48, 48, 40, 0.4, 2), Grid(32, 32, 24, 0.4, 2), Grid(16, 16, 20, 0.4, 3), Grid(8, 8, 24, 0.4, 1),
               Grid(12, 10, 40, 0.4, 2)]


@pytest.mark.parametrize("g", SHAPE_GRIDS, ids=gid)
def test_apply_every_launch_shape(torch, g):
    """y = A x at every admissible launch shape: each against the oracle
    (complex128 to 1e-12, complex64 to 2e-5), and the 2.5D stencil shapes
    bit-identical to each other (every point sums its terms in the same
    order whatever the block shape)."""
    from paper_1009_5300_amd import iobm
    V = _V(g, 12)
    s = _solver(g, V)
    P = O.Problem(g, V)
    E = 0.9
    x = random_field((2,) + g.shape, 22)
    ref = P.apply(E, x.reshape(2, -1)).reshape(x.shape)
    xt = torch.as_tensor(x, device="cuda")
    xf = xt.to(torch.complex64)
    shapes = _shapes(s, g)
    assert any(c["stencil"] == 1 for c in shapes) and any(c["stencil"] == 2 for c in shapes)
    first = {}
    for c in shapes:
        for prec in (iobm.C128, iobm.C64_REFINED):
            s.set_launch_shape(prec, c)
            got = s.get_launch_shape(prec)
            assert got["stencil"] == c["stencil"] and got["plane_fft"] == c["plane_fft"]
            y = s.apply(E, xt if prec == iobm.C128 else xf, prec).cpu().numpy()
            tol = 1e-12 if prec == iobm.C128 else 2e-5
            assert np.abs(y - ref).max() <= tol * np.abs(ref).max(), (c, prec)
            key = (prec, c["plane_fft"])
            if c["stencil"] == 1:
                if key in first:
                    assert np.array_equal(y, first[key]), (c, prec)
                else:
                    first[key] = y
    s.set_launch_shape(iobm.C128, None)
    s.set_launch_shape(iobm.C64_REFINED, None)


def test_launch_shape_rejections(torch):
    from paper_1009_5300_amd import iobm
    g = Grid(48, 48, 40, 0.4, 2)
    s = _solver(g, np.zeros(g.shape))
    for bad, status in ((dict(stencil=1, points_per_thread=1), 8),   # 2304 threads per block
                        (dict(stencil=1, points_per_thread=4), 8),   # 4 points per thread only for nf = 1
                        (dict(planes_per_block=12), 8), (dict(zfilter_chunk=4), 8),
                        (dict(stencil=3), 1), (dict(planes_per_block=-1), 1), (dict(rz_pass=3), 1)):
        with pytest.raises(iobm.IobmError) as e:
            s.set_launch_shape(iobm.C64_REFINED, bad)
        assert e.value.status == status, bad
    g2 = Grid(12, 10, 40, 0.4, 2)
    s2 = _solver(g2, np.zeros(g2.shape))
    with pytest.raises(iobm.IobmError) as e:  # register FFT needs square planes
        s2.set_launch_shape(iobm.C128, dict(plane_fft=1))
    assert e.value.status == 8
    assert s2.get_launch_shape(iobm.C128)["plane_fft"] == 2


@pytest.mark.parametrize("plane_fft", [1, 2])
def test_lateral_fft_preconditioner_48x48_both_plane_ffts(torch, plane_fft):
    """The wide-wire cross-section with the register and the LDS plane FFT:
    P is the exact inverse of the flat-wire operator, so P (A_0 x) = x with
    A_0 x from the oracle (its direct solve is out of reach at 48 x 48)."""
    from paper_1009_5300_amd import iobm
    g = Grid(48, 48, 24, 0.4, 2)
    s = _solver(g, np.zeros(g.shape))
    for prec in (iobm.C128, iobm.C64_REFINED):
        s.set_launch_shape(prec, dict(plane_fft=plane_fft))
        assert s.get_launch_shape(prec)["plane_fft"] == plane_fft
    E = 0.74
    x = random_field((2,) + g.shape, 31)
    y = O.Problem(g, np.zeros(g.shape)).apply(E, x.reshape(2, -1)).reshape(x.shape)
    yt = torch.as_tensor(y, device="cuda")
    z = s.precondition(iobm.PC_LATERAL_FFT, yt, E=E).cpu().numpy()
    assert np.abs(z - x).max() <= 1e-9 * np.abs(x).max()
    z32 = s.precondition(iobm.PC_LATERAL_FFT, yt.to(torch.complex64), E=E, precision=iobm.C64_REFINED).cpu().numpy()
    assert np.abs(z32 - x).max() <= 1e-3 * np.abs(x).max()



@pytest.mark.parametrize("g", GRIDS, ids=gid)
@pytest.mark.parametrize("kb", [False, True])
def test_jacobi_preconditioner(torch, g, kb):
    """z = r / diag A(E) against the oracle's diagonal (potential, kinetic,
    nonlocal and face-plane self-energy parts), with the r^T z partials."""
    from paper_1009_5300_amd import iobm
    from workloads.synth import _kb_projectors
    V = _V(g, 13)
    nl = None
    if kb:
        Lx, Ly, Lz = g.nx * g.hx, g.ny * g.hy, g.nz * g.hz
        nl = _kb_projectors(g, [np.array([Lx / 2, Ly / 2, 0.5 * Lz]), np.array([0.1, 0.2, 0.1])], 1.0, 3,
                            np.random.default_rng(8))
    s = _solver(g, V, nl)
    P = O.Problem(g, V, nl)
    E = 1.3
    r = random_field((3,) + g.shape, 14)
    ref = O.precond.jacobi(P, E, r)
    rt = torch.as_tensor(r, device="cuda")
    for prec, rr, tol in ((iobm.C128, rt, 1e-13), (iobm.C64_REFINED, rt.to(torch.complex64), 2e-6)):
        z, rz = s.precondition(iobm.PC_JACOBI, rr, E=E, precision=prec, want_rz=True)
        z = z.cpu().numpy()
        assert np.abs(z - ref).max() <= tol * np.abs(ref).max()
        a, b = r.reshape(3, -1), ref.reshape(3, -1)
        assert np.all(np.abs(rz - (a * b).sum(axis=1)) <= 10 * tol * (np.abs(a) * np.abs(b)).sum(axis=1))
