"""Pins of the oracle's nonlocal atomic forces (Sec. 3.4) against facts that
do not come from the oracle (CPU only):

* an undisplaced FCC crystal on grid nodes has every atom at an inversion
  centre, so each force vanishes;
* in the whole-cell (Gamma) mode the SQ force converges, as n_pl grows, to
  -4 gamma h^3 p^T grad_h f((H - mu)/sigma) p with H the periodic FD
  Hamiltonian diagonalised by LAPACK and grad_h built from exact Taylor
  weights;
* that force is minus the derivative of the grand potential
  Omega = -2 sigma sum_i log(1 + exp(-(lambda_i - mu)/sigma)) with respect to
  the atom position, up to the FD representation of the projector's
  derivative (central differences of the exact Omega).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import ref
from paper_1708_07913_amd import workloads as W


def _exact_setup(wl, atoms=None):
    V = wl.veff()
    n = W.grid_points_per_axis(wl.cell, wl.h)
    h = wl.cell / n
    w = [float(x) / h ** 2 for x in ref.fd_weights_taylor(6)]
    tabs = ref.projector_tables(wl.atoms if atoms is None else atoms, wl.kb, h)
    H = ref.bloch_hamiltonian(n, h, w, V, tabs, np.zeros(3)).real
    return V, n, h, tabs, H


def _exact_forces(n, h, tabs, lam, U, mu, kT):
    D = (U * ref.fermi((lam - mu) / kT)[None, :]) @ U.T
    g = ref.fd_gradient_weights_taylor(6)
    G = [ref.periodic_gradient(n, h, g, ax) for ax in range(3)]
    F = np.zeros((len(tabs), 3))
    for I, (p, gam) in enumerate(ref.projector_vectors(n, tabs)):
        Dp = D @ p
        for ax in range(3):
            F[I, ax] = -4.0 * gam * h ** 3 * p @ (G[ax] @ Dp)
    return F


def test_forces_vanish_on_undisplaced_fcc():
    wl = W.fcc_workload("sym", 1, 8.0, 0.0, 0, 0.5, 2.5, 24, 1.0)
    o = oracle.Oracle.from_workload(wl)
    lmin, lmax = o.bounds()
    # mirror nodes get slightly different Ritz values from the fixed start
    # vector; common bounds keep the quadrature symmetric
    lmin = np.full(o.nd, lmin.min())
    lmax = np.full(o.nd, lmax.max())
    mom = o.moments(lmin, lmax)
    mu, _ = o.fermi_level(lmin, lmax, mom, wl.n_electrons)
    F = o.nl_forces(lmin, lmax, mu)
    # the displaced tiny cell's forces are ~1e-4 Ha/Bohr
    assert np.abs(F).max() < 1e-14


def test_forces_antisymmetric_under_inversion():
    """Inverting the displaced cell about the origin (grid node) maps every
    atom's force f to -f of its image atom."""
    wl = W.tiny_cell()
    inv = W.Workload(**{**wl.__dict__, "atoms": np.mod(-wl.atoms, wl.cell)})
    out = []
    for w_ in (wl, inv):
        o = oracle.Oracle.from_workload(w_)
        lmin, lmax = np.full(o.nd, -1.0), np.full(o.nd, 60.0)
        mom = o.moments(lmin, lmax)
        mu, _ = o.fermi_level(lmin, lmax, mom, w_.n_electrons)
        out.append((mu, o.nl_forces(lmin, lmax, mu)))
    (mu0, F0), (mu1, F1) = out
    assert abs(mu0 - mu1) < 1e-12
    assert np.abs(F0).max() > 1e-6
    assert np.abs(F0 + F1).max() < 1e-9 * np.abs(F0).max()


@pytest.mark.slow
def test_gamma_forces_match_diagonalisation():
    wl = W.fcc_workload("g", 1, 8.0, 0.1, 3, 0.8, 2.5, 24, 5.0)
    V, n, h, tabs, H = _exact_setup(wl)
    lam, U = np.linalg.eigh(H)
    from scipy.optimize import brentq
    mu = brentq(lambda m: 2 * ref.fermi((lam - m) / wl.kT).sum() - wl.n_electrons,
                lam[0] - 5, lam[-1] + 5, xtol=1e-14)
    exact = _exact_forces(n, h, tabs, lam, U, mu, wl.kT)
    errs = []
    for npl in (64, 160, 320):
        o = oracle.Oracle(wl.cell, wl.h, 12, wl.rcut, npl, wl.kT, wl.atoms, wl.kb, V,
                          region=oracle.GAMMA)
        lo, hi = o.bounds([0])
        F = o.nl_forces(np.full(o.nd, lo[0]), np.full(o.nd, hi[0]), mu)
        errs.append(np.abs(F - exact).max() / np.abs(exact).max())
    assert np.abs(exact).max() > 1e-5
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-9


@pytest.mark.slow
def test_forces_are_minus_grand_potential_gradient():
    """-dOmega/dR_I by central differences of the exact grand potential at fixed
    V_eff and mu, for projectors smooth enough that Omega is smooth in R: a
    4.8 Bohr cell at h = 0.4 with two atoms, Gaussian width 0.6 and cut radius
    4.1 (chi(r_c) ~ 1e-10, so no grid point entering the sphere moves Omega).
    The force formula replaces dp/dR by -grad_h p (12th-order FD); the two
    agree to about 1e-5 of the largest force here."""
    atoms = np.array([[0.9, 1.3, 2.2], [3.1, 3.4, 0.7]])
    kb = np.array([[0.6, 4.1, 0.5], [0.6, 4.1, 0.5]])
    wl = W.Workload(name="smooth", cell=4.8, h=0.4, fd_order=12, rcut=2.4, npl=24, kT_eV=5.0,
                    atoms=atoms, kb=kb, n_electrons=6.0, seed=0, amplitude=0.0)
    V, n, h, tabs, H = _exact_setup(wl)
    lam, U = np.linalg.eigh(H)
    mu = 0.3
    F = _exact_forces(n, h, tabs, lam, U, mu, wl.kT)

    def omega(at):
        _, _, _, _, Hd = _exact_setup(wl, at)
        x = (np.linalg.eigvalsh(Hd) - mu) / wl.kT
        return -2.0 * wl.kT * np.sum(np.logaddexp(0.0, -x))

    delta = 0.005  # central-difference error ~delta^2: 1.2e-5 of max |F| here
    assert np.abs(F).max() > 1e-4
    for I in range(2):
        for ax in range(3):
            ap, am = atoms.copy(), atoms.copy()
            ap[I, ax] += delta
            am[I, ax] -= delta
            fd = -(omega(ap) - omega(am)) / (2 * delta)
            assert abs(fd - F[I, ax]) < 1e-4 * np.abs(F).max(), (I, ax, fd, F[I, ax])
