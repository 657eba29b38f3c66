"""CPU-side checks of the C ABI: the library loads, exports every function
that include/sq.h declares, and rejects invalid arguments before it touches a
device (no compute call is made here)."""
from __future__ import annotations

import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_1708_07913_amd import sq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "sq.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sq_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = sq.load_library()
    names = _declared()
    assert {"sq_setup", "sq_spectral_bounds", "sq_moments", "sq_fermi_level",
            "sq_density_energy"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def test_default_options():
    o = sq.default_options()
    assert (o.precision, o.n_lanczos, o.margin, o.max_brent) == (0, 50, 0.05, 200)
    assert o.mu_xtol == 1e-14 and o.ne_rtol == 1e-13


def _setup(**over):
    lib = sq.load_library()
    args = dict(cell=8.0, h=0.5, fd_order=12, rcut=2.5, npl=24, kT=0.0367, natom=1,
                xyz=np.array([[1.0, 2.0, 3.0]]), kb=np.array([[0.7, 2.5, 0.5]]), opt=None)
    args.update(over)
    dp = ct.POINTER(ct.c_double)
    ctx = ct.c_void_p()
    xyz = None if args["xyz"] is None else np.ascontiguousarray(args["xyz"], dtype=np.float64)
    kb = None if args["kb"] is None else np.ascontiguousarray(args["kb"], dtype=np.float64)
    rc = lib.sq_setup(ct.byref(ctx), args["cell"], args["h"], args["fd_order"], args["rcut"],
                      args["npl"], args["kT"], args["natom"],
                      xyz.ctypes.data_as(dp) if xyz is not None else None,
                      kb.ctypes.data_as(dp) if kb is not None else None,
                      ct.byref(args["opt"]) if args["opt"] is not None else None)
    return rc, lib.sq_last_error().decode()


@pytest.mark.parametrize("over,fragment", [
    (dict(cell=-1.0), "cell"),
    (dict(cell=float("nan")), "cell"),
    (dict(h=0.0), "h must"),
    (dict(fd_order=7), "fd_order"),
    (dict(fd_order=14), "fd_order"),
    (dict(npl=22), "npl"),
    (dict(npl=0), "npl"),
    (dict(kT=0.0), "kT"),
    (dict(rcut=0.2), "m >= 1"),
    (dict(rcut=9.5), "wider than 37"),
    (dict(natom=-1), "natom"),
    (dict(xyz=None), "atom_xyz"),
    (dict(kb=np.array([[0.0, 2.5, 0.5]])), "projector"),
    (dict(kb=np.array([[0.7, 60.0, 0.5]])), "100 mesh"),
    (dict(xyz=np.array([[np.inf, 0.0, 0.0]])), "non-finite"),
])
def test_setup_rejects_invalid_arguments(over, fragment):
    rc, msg = _setup(**over)
    assert rc == -1, (rc, msg)
    assert fragment in msg


def test_streamed_regions_reject_deep_projector_overlap():
    # three coincident spheres: depth 3 is served by four chains on resident
    # cubes, but streamed cubes (wider than 31 points) carry two
    xyz = np.array([[1.0, 2.0, 3.0]] * 3)
    kb = np.array([[0.7, 2.5, 0.5]] * 3)
    rc, msg = _setup(natom=3, xyz=xyz, kb=kb, rcut=8.0)
    assert rc == -7, (rc, msg)
    assert "two overlapping" in msg
    rc, msg = _setup(natom=3, xyz=xyz, kb=kb, rcut=7.5)
    assert rc != -7, (rc, msg)  # without a GPU, set-up stops later (SQ_EDEVICE)


def test_setup_rejects_bad_options():
    o = sq.default_options()
    o.n_lanczos = 0
    rc, msg = _setup(opt=o)
    assert rc == -1 and "n_lanczos" in msg
    o = sq.default_options()
    o.precision = 7
    rc, msg = _setup(opt=o)
    assert rc == -1 and "precision" in msg


def test_null_context_calls():
    lib = sq.load_library()
    assert lib.sq_moments(None, None, None) == -1
    assert lib.sq_spectral_bounds(None, None, None, None) == -1
    assert lib.sq_query(None, None, None, None, None) == -1
    lib.sq_destroy(None)


def test_batch_options_and_null_batch_calls():
    lib = sq.load_library()
    o = sq.BatchOptions()
    lib.sq_batch_default_options(ct.byref(o))
    assert (o.block_nodes, o.wg_per_cu, o.use_graph, o.bounds_every, o.reuse_check, o.shape) == (0, 0, 1, 1, 1, 0)
    n = ct.c_int(-1)
    assert lib.sq_batch_group(None, 0, None, None, None, ct.byref(n)) == -1
    assert lib.sq_batch_tiles(None, None, None, None) == -1
    assert lib.sq_batch_query(None, None) == -1
    # options are validated before any context is looked at (no device call)
    ctxs = (ct.c_void_p * 1)(None)
    ptrs = (ct.c_void_p * 1)(1)
    ne = (ct.c_double * 1)(4.0)
    b = ct.c_void_p()
    for field, value, fragment in (("shape", 4, "shape"), ("block_nodes", 4, "block_nodes"),
                                   ("bounds_every", -1, "invalid batch options")):
        lib.sq_batch_default_options(ct.byref(o))
        setattr(o, field, value)
        rc = lib.sq_batch_create(ct.byref(b), ctxs, 1, ptrs, ptrs, ne, ct.byref(o))
        assert rc == -1 and fragment in lib.sq_last_error().decode(), (field, lib.sq_last_error())
        assert not b.value


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU: --gpus above 1 exits with a message."""
    import json
    import subprocess
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]
