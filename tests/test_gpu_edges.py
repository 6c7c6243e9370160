"""Edge cases through the C ABI on the GPU: an empty energy list, energies
without an open channel inside a ragged batch (per-energy channel lists of
different lengths, some empty), the thinnest transition region (nz = 2 nf:
the planes next to the two electrodes fill it), the shortest lateral period
(nx = ny = nf), the largest admitted grids, and the size limits."""
import numpy as np
import pytest

import oracle as O
from workloads import Grid, make

pytestmark = pytest.mark.gpu

DT = 1e-6


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _solver(g, V):
    from paper_1009_5300_amd import iobm
    s = iobm.Solver(g.nx, g.ny, g.nz, g.spacings, g.nf)
    s.set_potential(V)
    return s


def test_empty_energy_list(torch):
    from paper_1009_5300_amd import iobm
    w = make(2)
    s = _solver(w.grid, w.V)
    out = s.solve([])
    assert out["status"] == 0 and len(out["T"]) == 0 and out["stats"] == []
    S, st, status = s.smatrix([])
    assert status == 0 and S == [] and st == []
    Sp, Sm, st, status = s.smatrix_bloch([], (0.1, 0.0), opts=iobm.default_opts(precision=iobm.C128))
    assert status == 0 and Sp == [] and Sm == []


def test_energies_without_open_channels_in_a_ragged_batch(torch):
    """Energies below the lead band bottom (no open channel) mixed with
    energies of 1 and 9 channels, in one batch; explicit channel lists of
    different lengths, one of them empty.  The open ones match the oracle;
    the empty ones produce no state and an empty scattering matrix."""
    from paper_1009_5300_amd import iobm
    w = make(5, Grid(16, 16, 24, 0.4, 2))
    g = w.grid
    s = _solver(g, w.V)
    Es = [-0.05, 0.3, -0.2, 1.2]
    counts = [len(O.open_channels(g, E)) for E in Es]
    assert counts == [0, 1, 0, 9]
    P = O.Problem(g, w.V)
    ref = {}
    for E in (0.3, 1.2):
        modes = O.open_channels(g, E)
        psi = P.solve(E, modes)
        ref[E] = (modes, np.array([P.currents(E, m, p)[0] for m, p in zip(modes, psi)]))
    for prec in (iobm.C128, iobm.C64_REFINED):
        out = s.solve(Es, opts=iobm.default_opts(precision=prec))
        assert out["status"] == 0 and len(out["T"]) == 10
        assert [len(m) for m in out["modes"]] == counts
        assert np.abs(out["T"][0] - ref[0.3][1][0]) <= DT
        assert np.abs(out["T"][1:] - ref[1.2][1]).max() <= DT
        ids = list(ref[1.2][0])
        pick = ids[::3]
        part = s.solve(Es, channels=[[], [int(ref[0.3][0][0])], [], pick], opts=iobm.default_opts(precision=prec))
        assert part["status"] == 0 and len(part["T"]) == 1 + len(pick)
        assert abs(part["T"][0] - out["T"][0]) <= 1e-8
        for k, m in enumerate(pick):
            assert abs(part["T"][1 + k] - out["T"][1 + ids.index(m)]) <= 1e-8
    S, st, status = s.smatrix(Es, opts=iobm.default_opts(precision=iobm.C128))
    assert status == 0 and [x.shape for x in S] == [(0, 0), (2, 2), (0, 0), (18, 18)]
    for E, Sx in ((0.3, S[1]), (1.2, S[3])):
        assert np.abs(Sx - P.smatrix(E)[1]).max() <= 1e-7
    Sp, Sm, st, status = s.smatrix_bloch(Es, (0.2, -0.1), opts=iobm.default_opts(precision=iobm.C128))
    assert status == 0 and Sp[0].shape == (0, 0) and Sp[2].shape == (0, 0)
    for Sx in Sp[1:2] + Sp[3:]:
        n = Sx.shape[0]
        assert n > 0 and np.abs(Sx.conj().T @ Sx - np.eye(n)).max() <= 1e-8


@pytest.mark.parametrize("nf", [1, 2, 3])
def test_thinnest_transition_region(torch, nf):
    """nz = 2 nf: every plane is next to an electrode (the left face planes
    0..nf-1 and the right face planes nf..2nf-1 fill the region), both
    precisions and incidence from both sides, against the oracle."""
    from paper_1009_5300_amd import iobm
    g = Grid(8, 8, 2 * nf, 0.5, nf)
    rng = np.random.default_rng(40 + nf)
    V = 0.3 * rng.random(g.shape)
    s = _solver(g, V)
    P = O.Problem(g, V)
    E = 2.2
    modes = O.open_channels(g, E)
    assert len(modes) >= 3
    for side in ("L", "R"):
        psi = P.solve(E, modes, side)
        TR = np.array([P.currents(E, m, p, side) for m, p in zip(modes, psi)])
        for prec in (iobm.C128, iobm.C64_REFINED):
            out = s.solve([E], opts=iobm.default_opts(precision=prec, side=0 if side == "L" else 1), want_psi=True)
            assert out["status"] == 0, out.get("error")
            assert np.abs(out["T"] - TR[:, 0]).max() <= DT and np.abs(out["R"] - TR[:, 1]).max() <= DT
            got = out["psi"].cpu().numpy()
            assert np.abs(got - psi).max() <= 1e-6 * np.abs(psi).max()


@pytest.mark.parametrize("nf", [2, 3])
def test_shortest_lateral_period(torch, nf):
    """nx = ny = nf: the lateral neighbours at distance nf wrap onto the point
    itself.  The operator against the oracle's (complex128 to 1e-12), and a
    solve."""
    from paper_1009_5300_amd import iobm
    g = Grid(nf, nf, 16, 0.5, nf)
    rng = np.random.default_rng(50 + nf)
    V = 0.2 * rng.random(g.shape)
    s = _solver(g, V)
    P = O.Problem(g, V)
    E = 0.6
    x = rng.standard_normal((2,) + g.shape) + 1j * rng.standard_normal((2,) + g.shape)
    ref = P.apply(E, x.reshape(2, -1)).reshape(x.shape)
    y = s.apply(E, torch.as_tensor(x, device="cuda")).cpu().numpy()
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    modes = O.open_channels(g, E)
    assert len(modes) >= 1
    psi = P.solve(E, modes)
    TR = np.array([P.currents(E, m, p) for m, p in zip(modes, psi)])
    out = s.solve([E], opts=iobm.default_opts(precision=iobm.C128))
    assert out["status"] == 0
    assert np.abs(out["T"] - TR[:, 0]).max() <= DT and np.abs(out["R"] - TR[:, 1]).max() <= DT


@pytest.mark.parametrize("nx,ny,nz,nf", [(64, 64, 256, 1), (48, 64, 128, 2)])
def test_largest_admitted_grids(torch, nx, ny, nz, nf):
    """The largest cross-sections the LDS kernels admit at their FD order
    (64 x 64 at nf = 1, 48 x 64 = 3072 <= 3413 at nf = 2) and the longest
    region (256 planes): a flat wire, where every open channel transmits
    fully and psi is the incident wave."""
    from paper_1009_5300_amd import iobm
    g = Grid(nx, ny, nz, 0.4, nf)
    s = _solver(g, np.zeros(g.shape))
    P = O.Problem(g, np.zeros(g.shape))
    E = 0.1
    ids, _, _ = s.channels(E)
    assert len(ids) >= 3
    pick = [int(m) for m in ids[:3]]
    for prec in (iobm.C128, iobm.C64_REFINED):
        out = s.solve([E], channels=[pick], opts=iobm.default_opts(precision=prec), want_psi=True)
        assert out["status"] == 0, out.get("error")
        assert np.abs(out["T"] - 1.0).max() <= 1e-9 and np.abs(out["R"]).max() <= 1e-9
        got = out["psi"].cpu().numpy()
        for k, m in enumerate(pick):
            Phi = P.incident(E, m)[nf:nf + nz]
            assert np.abs(got[k] - Phi).max() <= 1e-8


def test_size_limits(torch):
    """Grids beyond the limits are refused at creation: more than 4096
    lateral points, more than 256 planes, and a cross-section whose nf + 1
    complex128 planes exceed a workgroup's LDS."""
    import ctypes as C
    from paper_1009_5300_amd import iobm
    lib = iobm.lib()
    for nx, ny, nz, nf in ((65, 64, 16, 1), (8, 8, 257, 2), (64, 64, 16, 2), (52, 52, 16, 3)):
        g = iobm.Grid(nx, ny, nz, 0.4, 0.4, 0.4, nf)
        ctx = C.c_void_p()
        assert lib.iobm_create(C.byref(g), None, C.byref(ctx)) == 8, (nx, ny, nz, nf)
        assert not ctx.value
    for nx, ny, nz, nf in ((64, 64, 16, 1), (56, 56, 16, 2), (50, 50, 16, 3)):
        g = iobm.Grid(nx, ny, nz, 0.4, 0.4, 0.4, nf)
        ctx = C.c_void_p()
        assert lib.iobm_create(C.byref(g), None, C.byref(ctx)) == 0, (nx, ny, nz, nf)
        assert lib.iobm_destroy(ctx) == 0
