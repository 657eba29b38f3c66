"""The stored full-cell oracle results (tests/golden/full_*.npz) against the
oracle itself and the invariants the method fixes (CPU only).

Each file must be what the oracle computes: a few stored nodes are recomputed
(Lanczos bounds, moment rows at the stored bounds, density at the stored
Fermi level), and the stored whole-cell numbers must satisfy the electron-count
constraint h^3 sum rho = N_e at mu (Sec. 3.2), F_el = E_band + E_ent
(Sec. 3.3), rho^0 = 1 and |rho^j| <= 1 (spectrum scaled into [-1, 1]), and
bounds that enclose the unrounded Lanczos bounds by at most one grid step.
"""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

import oracle
from paper_1708_07913_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_goldens  # noqa: E402

CELLS = {"paper": W.paper_size_cell, "large": W.large_cell}


def _golden(name):
    if not os.path.exists(make_goldens.golden_path(name)):
        pytest.skip(f"stored oracle results for '{name}' not generated")
    return make_goldens.load(name)


@pytest.mark.parametrize("name", sorted(CELLS))
def test_golden_invariants(name):
    g = _golden(name)
    wl = CELLS[name]()
    meta = g["meta"]
    assert meta["nodes"] == wl.n ** 3 and meta["npl"] == wl.npl
    e = g["energies"]
    assert abs(e[3] - wl.n_electrons) < 1e-10 * wl.n_electrons
    assert abs(e[2] - (e[0] + e[1])) < 1e-12 * abs(e[2])
    assert e[1] < 0.0  # entropy term -sigma S <= 0
    m = g["moments"]
    assert np.all(m[:, 0] == 1.0) and np.abs(m).max() <= 1.0 + 1e-10
    # stored bounds enclose the unrounded Lanczos bounds, by at most one step
    q = 1.0 / meta["qscale"]
    lo, hi = g["lmin"][g["bounds_nodes"]], g["lmax"][g["bounds_nodes"]]
    assert np.all(lo <= g["lmin_exact"]) and np.all(g["lmin_exact"] - lo < q)
    assert np.all(hi >= g["lmax_exact"]) and np.all(hi - g["lmax_exact"] < q)
    assert np.all(g["rho"] >= 0.0) and g["rho"].max() <= g["rho_max"]


@pytest.mark.parametrize("name", sorted(CELLS))
def test_golden_matches_oracle(name):
    g = _golden(name)
    wl = CELLS[name]()
    o = oracle.Oracle.from_workload(wl)
    # bounds of two stored nodes
    bn = g["bounds_nodes"][[0, len(g["bounds_nodes"]) // 2]]
    lo, hi = o.bounds(bn)
    idx = np.searchsorted(g["bounds_nodes"], bn)
    assert np.array_equal(lo, g["lmin_exact"][idx]) and np.array_equal(hi, g["lmax_exact"][idx])
    # moment rows of two stored nodes at the stored bounds (nodes 13 * 2999 k
    # are also rho nodes)
    mn = g["mom_nodes"][[13, 26]]
    mom = o.moments(g["lmin"][mn], g["lmax"][mn], nodes=mn)
    idx = np.searchsorted(g["mom_nodes"], mn)
    assert np.array_equal(mom, g["moments"][idx])
    # density of those nodes at the stored Fermi level, where they are stored
    rho, _ = o.density_energy(g["lmin"][mn], g["lmax"][mn], mom, g["mu"])
    k = np.searchsorted(g["rho_nodes"], mn)
    assert np.array_equal(g["rho_nodes"][k], mn)
    assert np.array_equal(rho, g["rho"][k])
