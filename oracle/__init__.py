"""FP64 CPU oracle for the spectral-quadrature density/energy step.

TEST INFRASTRUCTURE ONLY: the slow, obviously-correct reference that the GPU
library is checked against.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.
It shares no code with the GPU library (its C source is ``sq_oracle.c``).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sq_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_sq.so")

INFINITE_CELL = 0
GAMMA = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fPIC",
               "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ct.CDLL(_LIB)
    P = ct.c_void_p
    dp = ct.POINTER(ct.c_double)
    lp = ct.POINTER(ct.c_long)
    ip = ct.POINTER(ct.c_int)
    lib.sqo_create.restype = P
    lib.sqo_create.argtypes = [ct.c_double, ct.c_double, ct.c_int, ct.c_double, ct.c_int,
                               ct.c_double, ct.c_int, dp, dp, dp, ct.c_int, ct.c_int, ct.c_double]
    lib.sqo_destroy.argtypes = [P]
    lib.sqo_info.argtypes = [P, ip, ip, lp, lp, dp]
    lib.sqo_fd_weights.argtypes = [ct.c_int, ct.c_double, dp]
    lib.sqo_splitmix64.restype = ct.c_uint64
    lib.sqo_splitmix64.argtypes = [ct.c_uint64]
    lib.sqo_unit.restype = ct.c_double
    lib.sqo_unit.argtypes = [ct.c_uint64]
    lib.sqo_matvec.argtypes = [P, ct.c_long, dp, dp]
    lib.sqo_region_images.argtypes = [P, ct.c_long]
    lib.sqo_atom_table.argtypes = [P, ct.c_int, ip, ct.POINTER(ip), ct.POINTER(dp)]
    lib.sqo_tridiag_extremes.argtypes = [ct.c_int, dp, dp, dp, dp]
    lib.sqo_lanczos.argtypes = [P, ct.c_long, dp, dp, ip]
    lib.sqo_bounds.argtypes = [P, lp, ct.c_long, dp, dp, ip]
    lib.sqo_moments.argtypes = [P, lp, ct.c_long, dp, dp, dp]
    lib.sqo_coefficients.argtypes = [P, ct.c_double, ct.c_double, ct.c_double, dp, dp, dp]
    lib.sqo_electron_count.restype = ct.c_double
    lib.sqo_electron_count.argtypes = [P, ct.c_long, dp, dp, dp, ct.c_double]
    lib.sqo_fermi_level.argtypes = [P, ct.c_long, dp, dp, dp, ct.c_double, ct.c_double,
                                    ct.c_double, ct.c_int, dp, ip]
    lib.sqo_density_energy.argtypes = [P, ct.c_long, dp, dp, dp, ct.c_double, dp, dp]
    lib.sqo_nl_forces.argtypes = [P, lp, ct.c_long, dp, dp, ct.c_double, dp]
    lib.sqo_num_threads.restype = ct.c_int
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def fd_weights(fd_order: int, h: float) -> np.ndarray:
    lib = _load()
    w = np.zeros(7)
    if lib.sqo_fd_weights(int(fd_order), float(h), _dp(w)) != 0:
        raise ValueError("fd_order must be even in [2, 12]")
    return w[: fd_order // 2 + 1].copy()


def splitmix64(seed: int) -> int:
    return int(_load().sqo_splitmix64(ct.c_uint64(seed)))


def unit(a: int) -> float:
    return float(_load().sqo_unit(ct.c_uint64(a)))


def tridiag_extremes(alpha, beta):
    lib = _load()
    a = _f64(alpha)
    b = _f64(beta) if len(beta) else np.zeros(1)
    lo, hi = ct.c_double(), ct.c_double()
    if lib.sqo_tridiag_extremes(len(a), _dp(a), _dp(b), ct.byref(lo), ct.byref(hi)) != 0:
        raise ValueError("empty tridiagonal")
    return lo.value, hi.value


def num_threads() -> int:
    return int(_load().sqo_num_threads())


class Oracle:
    """One snapshot: grid, FD weights, projector tables and V_eff (borrowed)."""

    def __init__(self, cell, h, fd_order, rcut, npl, kT, atoms, kb, veff,
                 region=INFINITE_CELL, n_lanczos=50, margin=0.05):
        lib = _load()
        self._atoms = _f64(atoms).reshape(-1, 3)
        self._kb = _f64(kb).reshape(-1, 3)
        self._veff = _f64(veff)
        natom = self._atoms.shape[0]
        self.kT = float(kT)
        self.npl = int(npl)
        self.margin = float(margin)
        self._p = lib.sqo_create(float(cell), float(h), int(fd_order), float(rcut), int(npl),
                                 float(kT), natom, _dp(self._atoms) if natom else None,
                                 _dp(self._kb) if natom else None, _dp(self._veff),
                                 int(region), int(n_lanczos), float(margin))
        if not self._p:
            raise ValueError("invalid SQ parameters")
        n, m, nd, ns, hh = ct.c_int(), ct.c_int(), ct.c_long(), ct.c_long(), ct.c_double()
        lib.sqo_info(self._p, ct.byref(n), ct.byref(m), ct.byref(nd), ct.byref(ns), ct.byref(hh))
        self.n, self.m, self.nd, self.ns, self.h = n.value, m.value, nd.value, ns.value, hh.value
        if self._veff.size != self.nd:
            lib.sqo_destroy(self._p)
            self._p = None
            raise ValueError("veff must have n^3 entries")
        self.region = region

    @classmethod
    def from_workload(cls, wl, region=INFINITE_CELL, **kw):
        veff = kw.pop("veff", None)
        if veff is None:
            veff = wl.veff()
        return cls(wl.cell, wl.h, wl.fd_order, wl.rcut, wl.npl, wl.kT, wl.atoms, wl.kb,
                   veff, region=region, **kw)

    def __del__(self):
        if getattr(self, "_p", None):
            _load().sqo_destroy(self._p)
            self._p = None

    def _nodes(self, nodes):
        if nodes is None:
            return None, self.nd
        arr = np.ascontiguousarray(np.asarray(nodes, dtype=np.int64))
        return arr, arr.size

    def matvec(self, q: int, x) -> np.ndarray:
        x = _f64(x)
        y = np.zeros(self.ns)
        if _load().sqo_matvec(self._p, int(q), _dp(x), _dp(y)) != 0:
            raise ValueError("bad node")
        return y

    def region_images(self, q: int) -> int:
        return int(_load().sqo_region_images(self._p, int(q)))

    def atom_table(self, a: int):
        cnt = ct.c_int()
        ijk = ct.POINTER(ct.c_int)()
        p = ct.POINTER(ct.c_double)()
        if _load().sqo_atom_table(self._p, int(a), ct.byref(cnt), ct.byref(ijk), ct.byref(p)) != 0:
            raise IndexError(a)
        k = cnt.value
        return (np.ctypeslib.as_array(ijk, shape=(k * 3,)).reshape(k, 3).copy(),
                np.ctypeslib.as_array(p, shape=(k,)).copy())

    def lanczos(self, q: int):
        al = np.zeros(256)
        be = np.zeros(256)
        k = ct.c_int()
        _load().sqo_lanczos(self._p, int(q), _dp(al), _dp(be), ct.byref(k))
        return al[: k.value].copy(), be[: k.value].copy()

    def bounds(self, nodes=None):
        arr, cnt = self._nodes(nodes)
        lmin = np.zeros(cnt)
        lmax = np.zeros(cnt)
        steps = np.zeros(cnt, dtype=np.int32)
        lp = arr.ctypes.data_as(ct.POINTER(ct.c_long)) if arr is not None else None
        rc = _load().sqo_bounds(self._p, lp, cnt, _dp(lmin), _dp(lmax),
                                steps.ctypes.data_as(ct.POINTER(ct.c_int)))
        if rc != 0:
            raise RuntimeError(f"sqo_bounds failed ({rc})")
        return lmin, lmax

    def moments(self, lmin, lmax, nodes=None) -> np.ndarray:
        arr, cnt = self._nodes(nodes)
        lmin = _f64(lmin)
        lmax = _f64(lmax)
        assert lmin.size == cnt and lmax.size == cnt
        mom = np.zeros((cnt, self.npl + 1))
        lp = arr.ctypes.data_as(ct.POINTER(ct.c_long)) if arr is not None else None
        rc = _load().sqo_moments(self._p, lp, cnt, _dp(lmin), _dp(lmax), _dp(mom))
        if rc != 0:
            raise RuntimeError(f"sqo_moments failed ({rc})")
        return mom

    def coefficients(self, mu, lmin, lmax):
        c = np.zeros(self.npl + 1)
        d = np.zeros(self.npl + 1)
        e = np.zeros(self.npl + 1)
        _load().sqo_coefficients(self._p, float(mu), float(lmin), float(lmax), _dp(c), _dp(d), _dp(e))
        return c, d, e

    def electron_count(self, lmin, lmax, mom, mu) -> float:
        lmin, lmax, mom = _f64(lmin), _f64(lmax), _f64(mom)
        return float(_load().sqo_electron_count(self._p, lmin.size, _dp(lmin), _dp(lmax), _dp(mom),
                                                float(mu)))

    def fermi_level(self, lmin, lmax, mom, n_electrons, xtol=1e-14, frtol=1e-13, maxit=200):
        lmin, lmax, mom = _f64(lmin), _f64(lmax), _f64(mom)
        mu = ct.c_double()
        it = ct.c_int()
        rc = _load().sqo_fermi_level(self._p, lmin.size, _dp(lmin), _dp(lmax), _dp(mom),
                                     float(n_electrons), float(xtol), float(frtol), int(maxit),
                                     ct.byref(mu), ct.byref(it))
        if rc != 0:
            raise RuntimeError(f"sqo_fermi_level failed ({rc})")
        return mu.value, it.value

    def density_energy(self, lmin, lmax, mom, mu):
        lmin, lmax, mom = _f64(lmin), _f64(lmax), _f64(mom)
        rho = np.zeros(lmin.size)
        out = np.zeros(4)
        _load().sqo_density_energy(self._p, lmin.size, _dp(lmin), _dp(lmax), _dp(mom), float(mu),
                                   _dp(rho), _dp(out))
        return rho, out

    def nl_forces(self, lmin, lmax, mu, nodes=None) -> np.ndarray:
        """Nonlocal atomic forces (natom x 3, Ha/Bohr) from the given nodes
        (all by default; lmin/lmax per listed node), Sec. 3.4."""
        arr, cnt = self._nodes(nodes)
        lmin = _f64(lmin)
        lmax = _f64(lmax)
        assert lmin.size == cnt and lmax.size == cnt
        f = np.zeros((self._atoms.shape[0], 3))
        lp = arr.ctypes.data_as(ct.POINTER(ct.c_long)) if arr is not None else None
        rc = _load().sqo_nl_forces(self._p, lp, cnt, _dp(lmin), _dp(lmax), float(mu), _dp(f))
        if rc != 0:
            raise RuntimeError(f"sqo_nl_forces failed ({rc})")
        return f
