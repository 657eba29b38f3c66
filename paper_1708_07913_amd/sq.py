"""Thin Python binding of libsq (include/sq.h): argument marshalling only.

PyTorch provides the device memory (workspace, V_eff, bounds, moments,
density) and the stream; every step of the SQ density/energy path runs in the
HIP kernels of libsq.so.  Loading fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsq.so")

FP64 = 0
FP32_MIXED = 1

SQ_OK = 0
_STATUS = {-1: "SQ_EINVAL", -2: "SQ_ENOMEM", -3: "SQ_EDEVICE", -4: "SQ_ESTATE", -5: "SQ_ENOCONV",
           -6: "SQ_EBOUNDS", -7: "SQ_ECAPACITY"}


class SQError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{_STATUS.get(code, code)}: {message}")
        self.code = code


class Options(ct.Structure):
    _fields_ = [("precision", ct.c_int), ("n_lanczos", ct.c_int), ("margin", ct.c_double),
                ("mu_xtol", ct.c_double), ("ne_rtol", ct.c_double), ("max_brent", ct.c_int),
                ("workgroups", ct.c_int)]


class BatchOptions(ct.Structure):
    _fields_ = [("block_nodes", ct.c_int), ("wg_per_cu", ct.c_int), ("use_graph", ct.c_int),
                ("bounds_every", ct.c_int), ("reuse_check", ct.c_int), ("shape", ct.c_int)]


# kernel shapes of the batched recurrence launches (bits of BatchOptions.shape)
SHAPE_TWO_ROWS = 1    # two cube columns per thread (21-27-point cubes)
SHAPE_TWO_PLANES = 2  # two planes per barrier in the FP64 sweeps (21-31-point cubes)


_lib = None


def load_library():
    """Load libsq.so from the package directory (never a CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ct.CDLL(LIB_PATH)
    P, D, I, S = ct.c_void_p, ct.c_double, ct.c_int, ct.c_size_t
    dp = ct.POINTER(ct.c_double)
    lib.sq_default_options.argtypes = [ct.POINTER(Options)]
    lib.sq_default_options.restype = None
    lib.sq_last_error.restype = ct.c_char_p
    lib.sq_setup.argtypes = [ct.POINTER(P), D, D, I, D, I, D, I, dp, dp, ct.POINTER(Options)]
    lib.sq_query.argtypes = [P, ct.POINTER(I), ct.POINTER(I), ct.POINTER(ct.c_longlong), ct.POINTER(S)]
    lib.sq_bind.argtypes = [P, P, S, P, P]
    lib.sq_update_veff.argtypes = [P, P, P]
    lib.sq_spectral_bounds.argtypes = [P, P, P, P]
    lib.sq_set_bounds.argtypes = [P, P, P, P]
    lib.sq_moments.argtypes = [P, P, P]
    lib.sq_fermi_level.argtypes = [P, P, D, dp, P]
    lib.sq_density_energy.argtypes = [P, P, D, P, dp, P]
    lib.sq_density_energy_static.argtypes = [P, P, D, P, dp, P]
    lib.sq_nl_forces.argtypes = [P, D, dp, P]
    lib.sq_destroy.argtypes = [P]
    lib.sq_destroy.restype = None
    lib.sq_batch_default_options.argtypes = [ct.POINTER(BatchOptions)]
    lib.sq_batch_default_options.restype = None
    lib.sq_batch_create.argtypes = [ct.POINTER(P), ct.POINTER(P), I, ct.POINTER(P), ct.POINTER(P), dp,
                                    ct.POINTER(BatchOptions)]
    lib.sq_batch_query.argtypes = [P, ct.POINTER(S)]
    lib.sq_batch_bind.argtypes = [P, P, S, P]
    lib.sq_batch_step.argtypes = [P, dp, dp, P]
    lib.sq_batch_autotune.argtypes = [P, ct.c_char_p, P]
    lib.sq_batch_tiles.argtypes = [P, ct.POINTER(I), ct.POINTER(I), ct.POINTER(I)]
    lib.sq_batch_group.argtypes = [P, I, ct.POINTER(I), ct.POINTER(I), ct.POINTER(I), ct.POINTER(I)]
    lib.sq_batch_destroy.argtypes = [P]
    lib.sq_batch_destroy.restype = None
    for name in ("sq_setup", "sq_query", "sq_bind", "sq_update_veff", "sq_spectral_bounds",
                 "sq_set_bounds", "sq_moments", "sq_fermi_level", "sq_density_energy",
                 "sq_density_energy_static", "sq_nl_forces",
                 "sq_batch_create", "sq_batch_query", "sq_batch_bind", "sq_batch_step",
                 "sq_batch_autotune", "sq_batch_tiles", "sq_batch_group"):
        getattr(lib, name).restype = ct.c_int
    _lib = lib
    return lib


def _check(code: int):
    if code != SQ_OK:
        raise SQError(code, _lib.sq_last_error().decode())


def default_options() -> Options:
    o = Options()
    load_library().sq_default_options(ct.byref(o))
    return o


def _dptr(t) -> int:
    return t.data_ptr()


class SQ:
    """One snapshot on the current CUDA (HIP) device.

    veff: torch float64 tensor of n^3 values on the device (kept alive here).
    """

    def __init__(self, cell, h, fd_order, rcut, npl, kT, atoms, kb, veff, precision=FP64,
                 n_lanczos=50, margin=0.05, workgroups=0, stream=None):
        import torch
        lib = load_library()
        self.torch = torch
        opt = default_options()
        opt.precision = int(precision)
        opt.n_lanczos = int(n_lanczos)
        opt.margin = float(margin)
        opt.workgroups = int(workgroups)
        atoms = np.ascontiguousarray(np.asarray(atoms, dtype=np.float64).reshape(-1, 3))
        kb = np.ascontiguousarray(np.asarray(kb, dtype=np.float64).reshape(-1, 3))
        natom = atoms.shape[0]
        self.natom = natom
        ctx = ct.c_void_p()
        dp = ct.POINTER(ct.c_double)
        _check(lib.sq_setup(ct.byref(ctx), float(cell), float(h), int(fd_order), float(rcut), int(npl),
                            float(kT), natom, atoms.ctypes.data_as(dp) if natom else None,
                            kb.ctypes.data_as(dp) if natom else None, ct.byref(opt)))
        self._ctx = ctx
        n, m, nd, ws = ct.c_int(), ct.c_int(), ct.c_longlong(), ct.c_size_t()
        _check(lib.sq_query(ctx, ct.byref(n), ct.byref(m), ct.byref(nd), ct.byref(ws)))
        self.n, self.m, self.nd, self.workspace_bytes = n.value, m.value, nd.value, ws.value
        self.npl = int(npl)
        self.kT = float(kT)
        self.precision = int(precision)
        self.h = float(cell) / self.n
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._stream = stream
        self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.veff = self._as_veff(veff)
        _check(lib.sq_bind(ctx, self._ws_ptr, self.workspace_bytes, _dptr(self.veff), self._stream_ptr()))

    @classmethod
    def from_workload(cls, wl, veff=None, precision=None, **kw):
        import torch
        if veff is None:
            veff = torch.from_numpy(wl.veff()).to("cuda")
        if precision is None:
            precision = FP32_MIXED if wl.precision == "mixed" else FP64
        return cls(wl.cell, wl.h, wl.fd_order, wl.rcut, wl.npl, wl.kT, wl.atoms, wl.kb, veff,
                   precision=precision, **kw)

    def _as_veff(self, veff):
        torch = self.torch
        if not isinstance(veff, torch.Tensor):
            veff = torch.from_numpy(np.ascontiguousarray(veff, dtype=np.float64))
        veff = veff.to(device=self.device, dtype=torch.float64).contiguous()
        if veff.numel() != self.nd:
            raise ValueError(f"veff must have {self.nd} entries")
        return veff

    def _stream_ptr(self):
        s = self._stream if self._stream is not None else self.torch.cuda.current_stream(self.device)
        return s.cuda_stream

    def __del__(self):
        if getattr(self, "_ctx", None) and _lib is not None:
            _lib.sq_destroy(self._ctx)
            self._ctx = None

    # -- the five steps -------------------------------------------------------------
    def update_veff(self, veff):
        self.veff = self._as_veff(veff)
        _check(_lib.sq_update_veff(self._ctx, _dptr(self.veff), self._stream_ptr()))

    def spectral_bounds(self):
        torch = self.torch
        lmin = torch.empty(self.nd, dtype=torch.float64, device=self.device)
        lmax = torch.empty(self.nd, dtype=torch.float64, device=self.device)
        _check(_lib.sq_spectral_bounds(self._ctx, _dptr(lmin), _dptr(lmax), self._stream_ptr()))
        return lmin, lmax

    def set_bounds(self, lmin, lmax):
        torch = self.torch
        self._lmin = torch.as_tensor(lmin, dtype=torch.float64).to(self.device).contiguous()
        self._lmax = torch.as_tensor(lmax, dtype=torch.float64).to(self.device).contiguous()
        if self._lmin.numel() != self.nd or self._lmax.numel() != self.nd:
            raise ValueError("bounds must have N_d entries")
        _check(_lib.sq_set_bounds(self._ctx, _dptr(self._lmin), _dptr(self._lmax), self._stream_ptr()))

    def moments(self, out=None):
        torch = self.torch
        if out is None:
            out = torch.empty((self.nd, self.npl + 1), dtype=torch.float64, device=self.device)
        _check(_lib.sq_moments(self._ctx, _dptr(out), self._stream_ptr()))
        return out

    def fermi_level(self, moments, n_electrons) -> float:
        mu = ct.c_double()
        _check(_lib.sq_fermi_level(self._ctx, _dptr(moments), float(n_electrons), ct.byref(mu),
                                   self._stream_ptr()))
        return mu.value

    def density_energy(self, moments, mu, rho=None):
        torch = self.torch
        if rho is None:
            rho = torch.empty(self.nd, dtype=torch.float64, device=self.device)
        e = (ct.c_double * 4)()
        _check(_lib.sq_density_energy(self._ctx, _dptr(moments), float(mu), _dptr(rho), e,
                                      self._stream_ptr()))
        return rho, np.array(list(e))

    def density_energy_static(self, moments, mu, rho):
        """sq_density_energy_static: the allocation-free variant; rho must be
        a caller-allocated device tensor of N_d FP64."""
        e = (ct.c_double * 4)()
        _check(_lib.sq_density_energy_static(self._ctx, _dptr(moments), float(mu), _dptr(rho), e,
                                             self._stream_ptr()))
        return rho, np.array(list(e))

    def nl_forces(self, mu):
        """sq_nl_forces: nonlocal atomic forces (natom x 3, Ha/Bohr) at Fermi
        level mu and the current bounds."""
        f = np.zeros((self.natom, 3))
        _check(_lib.sq_nl_forces(self._ctx, float(mu), f.ctypes.data_as(ct.POINTER(ct.c_double)),
                                 self._stream_ptr()))
        return f

    def scf_pass(self, n_electrons):
        """bounds -> moments -> Fermi level -> density and energies (fixed V_eff)."""
        self.spectral_bounds()
        mom = self.moments()
        mu = self.fermi_level(mom, n_electrons)
        rho, e = self.density_energy(mom, mu)
        return mom, mu, rho, e


class Batch:
    """Many snapshots (bound SQ objects of one precision) advanced together:
    one call runs bounds, moments, Fermi level, density and energies of all
    of them (persistent work-queue launches; optionally one hipGraph)."""

    def __init__(self, snaps, n_electrons, block_nodes=0, wg_per_cu=0, use_graph=True, bounds_every=1,
                 stream=None, reuse_check=True, shape=0):
        import torch
        lib = load_library()
        self.torch = torch
        self.snaps = list(snaps)
        n = len(self.snaps)
        self.n_electrons = np.ascontiguousarray(np.asarray(n_electrons, dtype=np.float64).reshape(n))
        dev = self.snaps[0].device
        self.moments = [torch.empty((s.nd, s.npl + 1), dtype=torch.float64, device=dev) for s in self.snaps]
        self.rho = [torch.empty(s.nd, dtype=torch.float64, device=dev) for s in self.snaps]
        opt = BatchOptions()
        lib.sq_batch_default_options(ct.byref(opt))
        opt.block_nodes, opt.wg_per_cu, opt.use_graph = int(block_nodes), int(wg_per_cu), int(bool(use_graph))
        opt.bounds_every = int(bounds_every)
        opt.reuse_check = int(bool(reuse_check))
        opt.shape = int(shape)
        ctxs = (ct.c_void_p * n)(*[s._ctx for s in self.snaps])
        mom = (ct.c_void_p * n)(*[t.data_ptr() for t in self.moments])
        rho = (ct.c_void_p * n)(*[t.data_ptr() for t in self.rho])
        b = ct.c_void_p()
        dp = ct.POINTER(ct.c_double)
        _check(lib.sq_batch_create(ct.byref(b), ctxs, n, mom, rho, self.n_electrons.ctypes.data_as(dp),
                                   ct.byref(opt)))
        self._b = b
        self._stream = stream
        ws = ct.c_size_t()
        _check(lib.sq_batch_query(b, ct.byref(ws)))
        self.workspace_bytes = ws.value
        self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=dev)
        self._ws_ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        _check(lib.sq_batch_bind(b, self._ws_ptr, self.workspace_bytes, self._stream_ptr()))

    def _stream_ptr(self):
        s = self._stream if self._stream is not None else self.torch.cuda.current_stream()
        return s.cuda_stream

    def step(self):
        """One pass of every snapshot; returns (mu[n], energies[n, 4])."""
        n = len(self.snaps)
        mu = np.zeros(n)
        e = np.zeros((n, 4))
        dp = ct.POINTER(ct.c_double)
        _check(_lib.sq_batch_step(self._b, mu.ctypes.data_as(dp), e.ctypes.data_as(dp), self._stream_ptr()))
        return mu, e

    def autotune(self, cache_path=None):
        _check(_lib.sq_batch_autotune(self._b, cache_path.encode() if cache_path else None, self._stream_ptr()))
        return self.tiles()

    def tiles(self):
        b, w, k = ct.c_int(), ct.c_int(), ct.c_int()
        _check(_lib.sq_batch_tiles(self._b, ct.byref(b), ct.byref(w), ct.byref(k)))
        return {"block_nodes": b.value, "wg_per_cu": w.value, "n_items": k.value}

    def groups(self):
        """Launch groups: [(cube side, projector chains, shape bits), ...]."""
        n = ct.c_int()
        _check(_lib.sq_batch_group(self._b, -1, None, None, None, ct.byref(n)))
        out = []
        for i in range(n.value):
            c, k, s = ct.c_int(), ct.c_int(), ct.c_int()
            _check(_lib.sq_batch_group(self._b, i, ct.byref(c), ct.byref(k), ct.byref(s), None))
            out.append((c.value, k.value, s.value))
        return out

    def __del__(self):
        if getattr(self, "_b", None) and _lib is not None:
            _lib.sq_batch_destroy(self._b)
            self._b = None
