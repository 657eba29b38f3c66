"""Full-cell oracle results for the two large workloads, written once and read by
the GPU parity tests (``tests/test_gpu_fullcell.py``).

    python tests/golden/make_goldens.py paper [--scratch DIR]
    python tests/golden/make_goldens.py large [--scratch DIR]

Only the FP64 CPU oracle (``oracle/``) and the seeded input generator
(``paper_1708_07913_amd.workloads``, inputs only) are called; nothing here
touches the GPU library.  For every node of the cell:

1. spectral bounds by the oracle's Lanczos (Sec. 3.2).  They are stored
   rounded OUTWARD to multiples of 1/256 Ha (lmin down, lmax up; int16), so
   that the injected bounds still enclose each nodal spectrum and the file
   stays small.  Every later step uses these stored bounds, on both sides.
   The unrounded Lanczos bounds of every BOUNDS_STRIDE-th node are stored too
   (FP64), for bounds parity;
2. Chebyshev moments at the stored bounds (Sec. 3.2), for every node;
3. the Fermi level by Brent's method on the electron-count constraint
   (Sec. 3.2) over all nodes;
4. the density and the band / entropy energies at that Fermi level
   (Sec. 3.2-3.3).

Stored: the quantised bounds of every node, mu, {E_band, E_ent, F_el,
h^3 sum rho}, rho of every RHO_STRIDE-th node, the moment rows of every
MOM_STRIDE-th node, and the run's parameters.  Partial results are kept in
the scratch directory, so an interrupted run resumes where it stopped.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1708_07913_amd import workloads as W  # noqa: E402

QSCALE = 256.0        # bounds are integer multiples of 1/QSCALE Ha
RHO_STRIDE = 13       # rho kept at nodes q = 0, 13, 26, ...
MOM_STRIDE = 2999     # moment rows kept at nodes q = 0, 2999, ...
BOUNDS_STRIDE = 61    # exact (unrounded) Lanczos bounds kept at q = 0, 61, ...
CHUNK = 2048          # nodes per oracle call (one checkpoint file each)

WORKLOADS = {"paper": W.paper_size_cell, "large": W.large_cell, "tiny": W.tiny_cell}
HERE = os.path.dirname(os.path.abspath(__file__))


def golden_path(name: str) -> str:
    return os.path.join(HERE, f"full_{name}.npz")


def quantise_outward(lmin: np.ndarray, lmax: np.ndarray):
    qlo = np.floor(lmin * QSCALE)
    qhi = np.ceil(lmax * QSCALE)
    if qlo.min() < -32768 or qhi.max() > 32767:
        raise ValueError("bounds outside the int16 range of the stored grid")
    return qlo.astype(np.int16), qhi.astype(np.int16)


def dequantise(q: np.ndarray) -> np.ndarray:
    return q.astype(np.float64) / QSCALE


def _chunked(o, nd, scratch, tag, fn, width):
    """Run fn(nodes) -> array (len(nodes), width) over all nodes in CHUNK pieces,
    each saved to scratch/tag_<i>.npy (skipped if present)."""
    out = np.empty((nd, width))
    nchunks = (nd + CHUNK - 1) // CHUNK
    t0 = time.perf_counter()
    done = 0
    for i in range(nchunks):
        f = os.path.join(scratch, f"{tag}_{i:05d}.npy")
        q0, q1 = i * CHUNK, min(nd, (i + 1) * CHUNK)
        if os.path.exists(f):
            out[q0:q1] = np.load(f)
            continue
        res = fn(np.arange(q0, q1, dtype=np.int64))
        np.save(f + ".tmp.npy", res)
        os.replace(f + ".tmp.npy", f)
        out[q0:q1] = res
        done += 1
        if done % 10 == 0 or i == nchunks - 1:
            el = time.perf_counter() - t0
            print(f"[golden] {tag}: chunk {i + 1}/{nchunks} ({el:.0f} s this run)", flush=True)
    return out


def make(name: str, scratch: str) -> str:
    wl = WORKLOADS[name]()
    os.makedirs(scratch, exist_ok=True)
    V = wl.veff()
    o = oracle.Oracle.from_workload(wl, veff=V)
    nd = o.nd
    print(f"[golden] {wl.name}: n={o.n} nodes={nd} cube={2 * o.m + 1} npl={wl.npl} "
          f"threads={oracle.num_threads()}", flush=True)
    t_start = time.perf_counter()

    def bounds_fn(nodes):
        lo, hi = o.bounds(nodes)
        return np.stack([lo, hi], axis=1)

    b = _chunked(o, nd, scratch, f"{wl.name}_bounds", bounds_fn, 2)
    lmin_exact, lmax_exact = b[:, 0].copy(), b[:, 1].copy()
    qlo, qhi = quantise_outward(lmin_exact, lmax_exact)
    lmin, lmax = dequantise(qlo), dequantise(qhi)

    def moments_fn(nodes):
        return o.moments(lmin[nodes], lmax[nodes], nodes=nodes)

    mom = _chunked(o, nd, scratch, f"{wl.name}_moments", moments_fn, wl.npl + 1)
    t_rec = time.perf_counter() - t_start
    mu, iters = o.fermi_level(lmin, lmax, mom, wl.n_electrons)
    rho, energies = o.density_energy(lmin, lmax, mom, mu)
    elapsed = time.perf_counter() - t_start
    print(f"[golden] mu={mu:.15f} ({iters} Brent iterations) E={energies.tolist()} "
          f"({elapsed:.0f} s)", flush=True)

    rho_nodes = np.arange(0, nd, RHO_STRIDE, dtype=np.int64)
    mom_nodes = np.arange(0, nd, MOM_STRIDE, dtype=np.int64)
    b_nodes = np.arange(0, nd, BOUNDS_STRIDE, dtype=np.int64)
    meta = {"workload": wl.name, "n": o.n, "nodes": nd, "cube": 2 * o.m + 1, "npl": wl.npl,
            "kT_eV": wl.kT_eV, "natom": wl.natom, "n_electrons": wl.n_electrons,
            "qscale": QSCALE, "rho_stride": RHO_STRIDE, "mom_stride": MOM_STRIDE,
            "bounds_stride": BOUNDS_STRIDE, "brent_iterations": iters,
            "oracle_threads": oracle.num_threads(), "oracle_seconds": elapsed,
            "oracle_recurrence_seconds": t_rec,
            "bounds_rule": "oracle Lanczos extremes rounded outward to multiples of 1/qscale Ha",
            "max_rho": float(rho.max())}
    path = golden_path(name)
    tmp = path + ".tmp.npz"
    np.savez_compressed(tmp, qlo=qlo, qhi=qhi, mu=np.float64(mu), energies=energies,
                        rho_nodes=rho_nodes, rho=rho[rho_nodes], rho_max=np.float64(rho.max()),
                        mom_nodes=mom_nodes, moments=mom[mom_nodes],
                        bounds_nodes=b_nodes, lmin_exact=lmin_exact[b_nodes],
                        lmax_exact=lmax_exact[b_nodes], meta=np.array(json.dumps(meta)))
    os.replace(tmp, path)
    print(f"[golden] wrote {path} ({os.path.getsize(path) / 1e6:.2f} MB)", flush=True)
    return path


def load(name: str):
    """The stored results as a dict (bounds dequantised to FP64)."""
    with np.load(golden_path(name), allow_pickle=False) as z:
        d = {k: z[k] for k in z.files}
    d["meta"] = json.loads(str(d["meta"]))
    d["lmin"] = dequantise(d["qlo"])
    d["lmax"] = dequantise(d["qhi"])
    d["mu"] = float(d["mu"])
    d["rho_max"] = float(d["rho_max"])
    return d


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(WORKLOADS))
    ap.add_argument("--scratch", default=os.path.join(tempfile.gettempdir(), "sq_golden_scratch"))
    args = ap.parse_args()
    make(args.workload, args.scratch)


if __name__ == "__main__":
    main()
