"""Python binding of libiobm (ctypes).  Argument marshalling only: every step
of the scattering solve runs in the library's HIP kernels; PyTorch supplies
device memory and the current HIP stream.  There is no CPU fallback: if the
library is missing the import of this module fails.

The functions mirror the C ABI in include/iobm.h (same names without the
`iobm_` prefix on the Solver methods); see that header for units, layouts
and error behaviour.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libiobm.so")

C128, C64_REFINED = 0, 1
PC_NONE, PC_TRUNCATED_LAPLACIAN, PC_LATERAL_FFT, PC_JACOBI = 0, 1, 2, 3
(K_STENCIL, K_BOUNDARY, K_PRECOND_FFT, K_PRECOND_LAP, K_NONLOCAL, K_DOT, K_UPDATE, K_STENCIL_C128,
 K_FFT_PLANES, K_ZFILTER, K_ACCUMULATE, K_NONLOCAL_C128, K_FFT_PLANES_DOT, K_FFT_PLANES_UPD,
 K_PRECOND_JACOBI, K_BLOCK_GRAM, K_BLOCK_UPDATE, K_BLOCH_STENCIL, K_BLOCH_VECTOR) = range(1, 20)
STATUS = ["ok", "invalid argument", "bad state", "out of device memory", "device error",
          "not converged", "Krylov breakdown", "energy at a channel threshold", "unsupported"]


class IobmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS[status] if 0 <= status < len(STATUS) else status}: {msg}")
        self.status = status


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("hx", C.c_double), ("hy", C.c_double), ("hz", C.c_double), ("nf", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("precond", C.c_int32), ("alpha", C.c_double),
                ("tol", C.c_double), ("inner_tol", C.c_double), ("max_iter", C.c_int32),
                ("side", C.c_int32), ("check_every", C.c_int32), ("keep_direction", C.c_int32), ("graph", C.c_int32),
                ("block", C.c_int32), ("pad_", C.c_int32)]


class SolveStat(C.Structure):
    _fields_ = [("iters", C.c_int32), ("refinements", C.c_int32), ("status", C.c_int32),
                ("pad_", C.c_int32), ("rel_residual", C.c_double), ("flux_error", C.c_double)]


class LaunchShape(C.Structure):
    _fields_ = [("stencil", C.c_int32), ("points_per_thread", C.c_int32), ("planes_per_block", C.c_int32),
                ("zfilter_chunk", C.c_int32), ("plane_fft", C.c_int32), ("rz_pass", C.c_int32)]


SHAPE_FIELDS = [f for f, _ in LaunchShape._fields_]

EXPORTS = {
    "iobm_default_opts": (None, [C.POINTER(SolveOpts)]),
    "iobm_create": (C.c_int, [C.POINTER(Grid), C.c_void_p, C.POINTER(C.c_void_p)]),
    "iobm_set_potential": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32]),
    "iobm_set_nonlocal": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p]),
    "iobm_channels": (C.c_int, [C.c_void_p, C.c_double, C.POINTER(C.c_int32), C.c_void_p,
                                C.c_void_p, C.c_void_p]),
    "iobm_self_energy": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p]),
    "iobm_apply": (C.c_int, [C.c_void_p, C.c_double, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32]),
    "iobm_precondition": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                    C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "iobm_precondition_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                            C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "iobm_rhs": (C.c_int, [C.c_void_p, C.c_double, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p]),
    "iobm_solve": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_int32, C.c_void_p, C.c_void_p,
                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_void_p]),
    "iobm_smatrix": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "iobm_channels_bloch": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double, C.POINTER(C.c_int32),
                                      C.c_void_p, C.c_void_p, C.c_void_p]),
    "iobm_smatrix_bloch": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_double, C.c_double, C.c_int32,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "iobm_grad_transmission": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_int32, C.c_void_p,
                                         C.POINTER(C.c_double), C.c_void_p]),
    "iobm_get_launch_shape": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(LaunchShape)]),
    "iobm_set_launch_shape": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(LaunchShape)]),
    "iobm_profile_begin": (C.c_int, [C.c_void_p, C.c_int32]),
    "iobm_profile_end": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "iobm_destroy": (C.c_int, [C.c_void_p]),
    "iobm_status_str": (C.c_char_p, [C.c_int]),
    "iobm_last_error": (C.c_char_p, [C.c_void_p]),
}


def load(path: str = LIBPATH):
    if not os.path.exists(path):
        raise ImportError(f"libiobm is not built ({path} missing); run __graft_entry__.build()")
    lib = C.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    lib().iobm_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ptr(a):
    """Raw pointer of a torch tensor or numpy array (no copy)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


class Solver:
    """One transition region (grid) on the current HIP device."""

    def __init__(self, nx, ny, nz, h, nf, stream=None):
        import torch
        self.torch = torch
        self.shape = (nz, ny, nx)
        hx, hy, hz = (h, h, h) if np.isscalar(h) else h
        self.grid = Grid(nx, ny, nz, hx, hy, hz, nf)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self._ctx = C.c_void_p()
        self._check(lib().iobm_create(C.byref(self.grid), C.c_void_p(stream), C.byref(self._ctx)), None)

    # -- helpers
    def _check(self, st, ctx="self"):
        if st != 0:
            msg = lib().iobm_last_error(self._ctx if ctx else None)
            raise IobmError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_ctx", None):
            lib().iobm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def npts(self):
        return int(np.prod(self.shape))

    def _dev(self, a, dtype):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device="cuda", dtype=dtype).contiguous()
        return t.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")

    # -- ABI calls
    def set_potential(self, V):
        V = self._dev(V, self.torch.float64).reshape(-1)
        assert V.numel() == self.npts
        self._check(lib().iobm_set_potential(self._ctx, _ptr(V), 1))
        self.torch.cuda.current_stream().synchronize()

    def set_nonlocal(self, nl):
        if nl is None:
            self._check(lib().iobm_set_nonlocal(self._ctx, 0, 0, None, None, None, None))
            return
        rank = nl.beta[0].shape[0]
        nsup = np.array([len(s) for s in nl.support], dtype=np.int32)
        idx = np.ascontiguousarray(np.concatenate(nl.support).astype(np.int64))
        # per-centre [rank][nsupport] blocks, concatenated
        beta = np.ascontiguousarray(np.concatenate([np.asarray(b, float).ravel() for b in nl.beta]))
        D = np.ascontiguousarray(np.stack([np.asarray(d, float) for d in nl.D]))
        self._check(lib().iobm_set_nonlocal(self._ctx, len(nl.support), rank, _ptr(nsup), _ptr(idx),
                                            _ptr(beta), _ptr(D)))

    def get_launch_shape(self, precision):
        """The launch shape in effect for `precision` (dict of iobm_launch_shape)."""
        sh = LaunchShape()
        self._check(lib().iobm_get_launch_shape(self._ctx, precision, C.byref(sh)))
        return {f: getattr(sh, f) for f in SHAPE_FIELDS}

    def set_launch_shape(self, precision, shape):
        """Pin a launch shape (dict; missing fields 0 = default rule), or
        unpin with None."""
        if shape is None:
            self._check(lib().iobm_set_launch_shape(self._ctx, precision, None))
            return
        sh = LaunchShape(*[int(shape.get(f, 0)) for f in SHAPE_FIELDS])
        self._check(lib().iobm_set_launch_shape(self._ctx, precision, C.byref(sh)))

    def profile_begin(self, classes):
        mask = 0
        for k in classes:
            mask |= 1 << k
        self._check(lib().iobm_profile_begin(self._ctx, mask))

    def profile_end(self, kernel_class):
        """(launches, total ms, algorithmic bytes) of one timed kernel class."""
        n = C.c_int32()
        ms = C.c_double()
        b = C.c_double()
        self._check(lib().iobm_profile_end(self._ctx, kernel_class, C.byref(n), C.byref(ms), C.byref(b)))
        return n.value, ms.value, b.value

    def channels(self, E):
        key = float(E)
        cache = self.__dict__.setdefault("_chan_cache", {})
        if key not in cache:
            cache[key] = self._channels(key)
        return tuple(a.copy() for a in cache[key])

    def _channels(self, E):
        n = C.c_int32()
        cap = self.shape[1] * self.shape[2]
        ids = np.zeros(cap, np.int32)
        kz = np.zeros(cap)
        v = np.zeros(cap)
        self._check(lib().iobm_channels(self._ctx, float(E), C.byref(n), _ptr(ids), _ptr(kz), _ptr(v)))
        k = n.value
        return ids[:k].copy(), kz[:k].copy(), v[:k].copy()

    def self_energy(self, E):
        nf = self.grid.nf
        s = np.zeros((self.shape[1] * self.shape[2], nf, nf, 2))
        self._check(lib().iobm_self_energy(self._ctx, float(E), _ptr(s)))
        return s[..., 0] + 1j * s[..., 1]

    def apply(self, E, x, precision=C128):
        t = self.torch
        x = x.contiguous()
        y = t.empty_like(x)
        nrhs = x.numel() // self.npts
        self._check(lib().iobm_apply(self._ctx, float(E), nrhs, _ptr(x), _ptr(y), precision))
        return y

    def precondition(self, kind, r, alpha=1.8, E=0.0, precision=C128, want_rz=False):
        """z = P r; with want_rz, also (z, rz) with rz[i] = r_i^T z_i (complex128,
        numpy) from the solver's own reduction."""
        r = r.contiguous()
        z = self.torch.empty_like(r)
        nrhs = r.numel() // self.npts
        rz = np.zeros(nrhs, dtype=np.complex128) if want_rz else None
        self._check(lib().iobm_precondition(self._ctx, kind, float(alpha), float(E), nrhs, _ptr(r),
                                            _ptr(z), precision, _ptr(rz)))
        return (z, rz) if want_rz else z

    def precondition_noalloc(self, kind, r, z, alpha=1.8, E=0.0, precision=C128, want_rz=False):
        """z = P r into the caller's z through the allocation-free entry
        point (the library's static workspace); returns rz as precondition."""
        nrhs = r.numel() // self.npts
        assert r.is_contiguous() and z.is_contiguous() and z.numel() == r.numel()
        rz = np.zeros(nrhs, dtype=np.complex128) if want_rz else None
        self._check(lib().iobm_precondition_noalloc(self._ctx, kind, float(alpha), float(E), nrhs, _ptr(r),
                                                    _ptr(z), precision, _ptr(rz)))
        return rz

    def rhs(self, E, ids, side=0):
        ids = np.ascontiguousarray(np.asarray(ids, dtype=np.int32))
        b = self.torch.empty((len(ids),) + self.shape, dtype=self.torch.complex128, device="cuda")
        self._check(lib().iobm_rhs(self._ctx, float(E), len(ids), _ptr(ids), side, _ptr(b)))
        return b

    def solve(self, energies, channels=None, opts=None, want_psi=False, want_t=False):
        """channels: None (every open channel at each energy) or a list with one
        entry per energy (None = all open, else a list of channel ids)."""
        energies = np.ascontiguousarray(np.asarray(energies, dtype=np.float64))
        nE = len(energies)
        if channels is None:
            channels = [None] * nE
        ninc = np.array([-1 if c is None else len(c) for c in channels], dtype=np.int32)
        inc = np.ascontiguousarray(np.concatenate(
            [np.asarray(c, np.int32) for c in channels if c is not None] or [np.zeros(0, np.int32)]
        ).astype(np.int32))
        opened = [self.channels(E)[0] for E in energies]
        counts = [len(opened[e]) if ninc[e] < 0 else ninc[e] for e in range(nE)]
        nrhs = int(sum(counts))
        T = np.zeros(nrhs)
        R = np.zeros(nrhs)
        st = (SolveStat * max(1, nrhs))()
        psi = None
        if want_psi:
            psi = self.torch.empty((nrhs,) + self.shape, dtype=self.torch.complex128, device="cuda")
        tlen = sum(len(opened[e]) * counts[e] for e in range(nE))
        t = np.zeros((max(1, tlen), 2)) if want_t else None
        o = opts or default_opts()
        status = lib().iobm_solve(self._ctx, C.byref(o), nE, _ptr(energies), _ptr(ninc), _ptr(inc),
                                  _ptr(psi), _ptr(t), _ptr(T), _ptr(R), st)
        stats = [(s.iters, s.refinements, s.status, s.rel_residual, s.flux_error) for s in st[:nrhs]]
        out = {"T": T, "R": R, "stats": stats, "psi": psi, "status": status,
               "modes": [opened[e] if ninc[e] < 0 else np.asarray(channels[e]) for e in range(nE)],
               "open": opened}
        if want_t:
            tm, off = [], 0
            tc = t[:, 0] + 1j * t[:, 1]
            for e in range(nE):
                n = len(opened[e]) * counts[e]
                tm.append(tc[off:off + n].reshape(len(opened[e]), counts[e]))
                off += n
            out["t"] = tm
        if status not in (0,):
            msg = lib().iobm_last_error(self._ctx)
            out["error"] = msg.decode() if msg else ""
            if status not in (5, 6):
                raise IobmError(status, out["error"])
        return out

    def smatrix(self, energies, opts=None):
        """Per energy the flux-normalised scattering matrix (2n x 2n complex
        numpy array, [left | right] channels); returns (list of S, stats)."""
        energies = np.ascontiguousarray(np.asarray(energies, dtype=np.float64))
        n = [len(self.channels(E)[0]) for E in energies]
        tot = sum(4 * k * k for k in n)
        S = np.zeros((max(1, tot), 2))
        st = (SolveStat * max(1, 2 * sum(n)))()
        o = opts or default_opts()
        status = lib().iobm_smatrix(self._ctx, C.byref(o), len(energies), _ptr(energies), _ptr(S), st)
        if status not in (0, 5, 6):
            self._check(status)
        Sc = S[:, 0] + 1j * S[:, 1]
        out, off = [], 0
        for k in n:
            out.append(Sc[off:off + 4 * k * k].reshape(2 * k, 2 * k))
            off += 4 * k * k
        stats = [(x.iters, x.refinements, x.status, x.rel_residual, x.flux_error) for x in st[:2 * sum(n)]]
        return out, stats, status

    def channels_bloch(self, E, kappa):
        """(ids, kz, v) of the open channels at E and lateral Bloch vector kappa."""
        n = C.c_int32()
        cap = self.shape[1] * self.shape[2]
        ids = np.zeros(cap, np.int32)
        kz = np.zeros(cap)
        v = np.zeros(cap)
        self._check(lib().iobm_channels_bloch(self._ctx, float(E), float(kappa[0]), float(kappa[1]), C.byref(n),
                                              _ptr(ids), _ptr(kz), _ptr(v)))
        k = n.value
        return ids[:k].copy(), kz[:k].copy(), v[:k].copy()

    def smatrix_bloch(self, energies, kappa, opts=None):
        """Scattering matrices at kappa and -kappa per energy: returns
        (list of S(kappa), list of S(-kappa), stats, status)."""
        energies = np.ascontiguousarray(np.asarray(energies, dtype=np.float64))
        n = [len(self.channels_bloch(E, kappa)[0]) for E in energies]
        tot = sum(4 * k * k for k in n)
        Sp = np.zeros((max(1, tot), 2))
        Sm = np.zeros((max(1, tot), 2))
        st = (SolveStat * max(1, 2 * sum(n)))()
        o = opts or default_opts()
        status = lib().iobm_smatrix_bloch(self._ctx, C.byref(o), float(kappa[0]), float(kappa[1]), len(energies),
                                          _ptr(energies), _ptr(Sp), _ptr(Sm), st)
        if status not in (0, 5, 6):
            self._check(status)
        outs = []
        for S in (Sp, Sm):
            Sc = S[:, 0] + 1j * S[:, 1]
            out, off = [], 0
            for k in n:
                out.append(Sc[off:off + 4 * k * k].reshape(2 * k, 2 * k))
                off += 4 * k * k
            outs.append(out)
        stats = [(x.iters, x.refinements, x.status, x.rel_residual, x.flux_error) for x in st[:2 * sum(n)]]
        return outs[0], outs[1], stats, status

    def grad_transmission(self, energies, opts=None):
        energies = np.ascontiguousarray(np.asarray(energies, dtype=np.float64))
        g = self.torch.empty(self.shape, dtype=self.torch.float64, device="cuda")
        T = C.c_double()
        o = opts or default_opts()
        self._check(lib().iobm_grad_transmission(self._ctx, C.byref(o), len(energies), _ptr(energies),
                                                 C.byref(T), _ptr(g)))
        return T.value, g
