"""Batched snapshots on the GPU: one pass of many snapshots (persistent
work-queue launches per cube size, device-side Brent, hipGraph replay)
against the single-snapshot path and the FP64 oracle, through the C ABI."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import oracle
from paper_1708_07913_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_07913_amd import sq
    sq.load_library()
    torch.cuda.set_device(0)


def _sq():
    from paper_1708_07913_amd import sq
    return sq


def _small_ensemble(precision="fp64"):
    """Four uneven snapshots: three cube sizes (one streamed), three n_pl."""
    return [
        W.fcc_workload("b0_al4_c11", 1, 8.0, 0.1, 21, 0.5, 2.5, 24, 1.0, precision=precision),
        W.fcc_workload("b1_al4_c15", 1, 8.0, 0.15, 22, 0.5, 3.5, 16, 3.0, precision=precision),
        W.fcc_workload("b2_al32_c11", 2, 7.78, 0.2, 23, 0.5, 2.5, 32, 1.0, precision=precision),
        W.fcc_workload("b3_al4_c33", 1, 8.0, 0.1, 24, 0.5, 8.0, 16, 1.0, precision=precision),
    ]


def _snaps(wls):
    sq = _sq()
    return [sq.SQ.from_workload(wl, veff=torch.from_numpy(wl.veff()).cuda()) for wl in wls]


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _single(snaps, wls):
    out = []
    for g, wl in zip(snaps, wls):
        mom, mu, rho, e = g.scf_pass(wl.n_electrons)
        out.append((_np(mom), mu, _np(rho), e))
    return out


def _compare(batch, mu, e, ref, wls, tol_rho=1e-12):
    for i, (wl, (mom1, mu1, rho1, e1)) in enumerate(zip(wls, ref)):
        m = _np(batch.moments[i])
        r = _np(batch.rho[i])
        assert np.abs(m - mom1).max() < 1e-12, (wl.name, np.abs(m - mom1).max())
        assert abs(mu[i] - mu1) < 1e-11, (wl.name, mu[i], mu1)
        assert np.abs(r - rho1).max() < tol_rho * rho1.max(), wl.name
        assert np.abs(e[i] - e1).max() < 1e-10 * np.abs(e1).max(), wl.name
        assert abs(e[i][3] - wl.n_electrons) < 1e-10 * wl.n_electrons


def test_batch_matches_single_snapshots_and_oracle():
    sq = _sq()
    wls = _small_ensemble()
    print("case small ensemble fp64 eager", flush=True)
    snaps = _snaps(wls)
    ref = _single(snaps, wls)
    b = sq.Batch(snaps, [wl.n_electrons for wl in wls], use_graph=False)
    mu, e = b.step()
    _compare(b, mu, e, ref, wls)
    # the tiny snapshot against the oracle (bounds of the GPU, density at the GPU's mu)
    wl = wls[0]
    o = oracle.Oracle.from_workload(wl, veff=wl.veff())
    lmin, lmax = o.bounds()
    mom_ref = o.moments(lmin, lmax)
    assert np.abs(_np(b.moments[0]) - mom_ref).max() < 1e-8  # bounds differ at rounding level
    mu_ref, _ = o.fermi_level(lmin, lmax, mom_ref, wl.n_electrons)
    assert abs(mu[0] - mu_ref) < 1e-8
    rho_ref, e_ref = o.density_energy(lmin, lmax, mom_ref, mu[0])
    r = _np(b.rho[0])
    assert np.abs(r - rho_ref).max() < 1e-8 * rho_ref.max()


def test_batch_graph_replays_match_eager():
    sq = _sq()
    wls = _small_ensemble()
    print("case small ensemble fp64 graph", flush=True)
    snaps = _snaps(wls)
    ref = _single(snaps, wls)
    b = sq.Batch(snaps, [wl.n_electrons for wl in wls], use_graph=True)
    for rep in range(3):
        mu, e = b.step()
        _compare(b, mu, e, ref, wls)
        # eager work of the program between replays
        snaps[0].spectral_bounds()
        snaps[0].moments()
        torch.cuda.synchronize()


def test_batch_mixed_precision():
    sq = _sq()
    wls = _small_ensemble("mixed")[:3]
    print("case small ensemble mixed", flush=True)
    snaps = _snaps(wls)
    ref = _single(snaps, wls)
    b = sq.Batch(snaps, [wl.n_electrons for wl in wls], use_graph=True)
    mu, e = b.step()
    for i, wl in enumerate(wls):
        rho1 = ref[i][2]
        r = _np(b.rho[i])
        # same kernels; FP32 rounding can flip where projector-dot atomics
        # change the FP64 summation order
        assert np.abs(r - rho1).max() < 1e-7 * rho1.max(), wl.name
        assert abs(e[i][3] - wl.n_electrons) < 1e-9 * wl.n_electrons


def _shape_cells(precision="fp64"):
    """Cells whose regions have the alternative kernel shapes: 21- and
    27-point cubes (two rows, two planes) and a 29-point cube (two planes)."""
    return [
        W.fcc_workload("s0_al4_c21", 1, 8.0, 0.1, 31, 0.5, 5.0, 24, 1.0, precision=precision),
        W.fcc_workload("s1_al4_c27", 1, 8.0, 0.1, 32, 0.5, 6.5, 16, 1.0, precision=precision),
        W.fcc_workload("s2_al4_c29", 1, 8.0, 0.15, 33, 0.5, 7.0, 16, 1.0, precision=precision),
    ]


def _shape_bits(cube):
    """Kernel shapes a cube side has (SHAPE_TWO_ROWS: 21-27, SHAPE_TWO_PLANES: 21-31)."""
    sq = _sq()
    return (sq.SHAPE_TWO_ROWS if 21 <= cube <= 27 else 0) | (sq.SHAPE_TWO_PLANES if 21 <= cube <= 31 else 0)


@pytest.mark.parametrize("precision,shape", [("fp64", 1), ("fp64", 2), ("fp64", 3), ("mixed", 3)])
def test_batch_kernel_shapes(precision, shape):
    """Every kernel shape against the single-snapshot path (default shape) and,
    on two sampled nodes per cell, against the FP64 oracle."""
    sq = _sq()
    wls = _shape_cells(precision)
    print(f"case kernel shape {shape} {precision}", flush=True)
    snaps = _snaps(wls)
    ref = _single(snaps, wls)
    b = sq.Batch(snaps, [wl.n_electrons for wl in wls], use_graph=False, shape=shape)
    groups = b.groups()
    assert sorted(c for c, _, _ in groups) == [21, 27, 29]
    for c, _, s in groups:
        assert s == shape & _shape_bits(c), (c, s)
    mu, e = b.step()
    if precision == "fp64":
        _compare(b, mu, e, ref, wls)
    else:
        for i, wl in enumerate(wls):
            rho1 = ref[i][2]
            assert np.abs(_np(b.rho[i]) - rho1).max() < 1e-7 * rho1.max(), wl.name
            assert abs(e[i][3] - wl.n_electrons) < 1e-9 * wl.n_electrons
    rng = np.random.default_rng(11)
    for i, (wl, g) in enumerate(zip(wls, snaps)):
        nodes = rng.choice(g.nd, 2, replace=False)
        o = oracle.Oracle.from_workload(wl, veff=wl.veff())
        lo, hi = o.bounds(nodes)
        mom_ref = o.moments(lo, hi, nodes=nodes)
        rho_ref, _ = o.density_energy(lo, hi, mom_ref, mu[i])
        r = _np(b.rho[i])
        err = np.abs(r[nodes] - rho_ref).max() / r.max()
        print(f"  {wl.name}: sampled rho rel err {err:.2e}", flush=True)
        assert err < (1e-10 if precision == "fp64" else 1e-5)


def test_batch_shape_bits_ignored_where_absent():
    """Shape bits a cube side does not have (11-, 15- and streamed 33-point
    cubes) leave its launches at the default shape."""
    sq = _sq()
    wls = _small_ensemble()
    print("case shape bits on cubes without shapes", flush=True)
    snaps = _snaps(wls)
    ref = _single(snaps, wls)
    b = sq.Batch(snaps, [wl.n_electrons for wl in wls], use_graph=False,
                 shape=sq.SHAPE_TWO_ROWS | sq.SHAPE_TWO_PLANES)
    assert all(s == 0 for _, _, s in b.groups()), b.groups()
    mu, e = b.step()
    _compare(b, mu, e, ref, wls)


def test_batch_autotune_and_cache(tmp_path):
    """The tuner picks a tile (block_nodes x wg_per_cu) and, per launch group,
    a kernel shape among those its cube side has; the choice is cached and a
    second batch of the same signature reads it back."""
    sq = _sq()
    wls = _small_ensemble()[:3] + _shape_cells()[:2]
    print("case autotune", flush=True)
    snaps = _snaps(wls)
    ref = _single(snaps, wls)
    cache = str(tmp_path / "tiles.json")
    b = sq.Batch(snaps, [wl.n_electrons for wl in wls])
    t = b.autotune(cache)
    assert t["block_nodes"] in (8, 32, 128) and t["n_items"] > 0
    groups = b.groups()
    for c, _, s in groups:
        assert s & ~_shape_bits(c) == 0, (c, s)
    data = json.load(open(cache))
    assert len(data) == 1
    entry = next(iter(data.values()))
    assert entry["block_nodes"] == t["block_nodes"] and entry["wg_per_cu"] == t["wg_per_cu"]
    # one shape entry per group that has alternatives: cubes 21 and 27
    assert sorted((c, k, s) for c, k, s in entry["shapes"]) == sorted(
        (c, k, s) for c, k, s in groups if _shape_bits(c))
    assert sorted(c for c, _, _ in entry["shapes"]) == [21, 27]
    # the sample time of every shape the group's cube side has; the chosen one is the fastest
    chosen = {(c, k): s for c, k, s in entry["shapes"]}
    for c, k, *ms in entry["shape_ms"]:
        have = [s for s in range(4) if s & ~_shape_bits(c) == 0]
        assert all((ms[s] >= 0) == (s in have) for s in range(4)), (c, ms)
        assert ms[chosen[(c, k)]] == min(ms[s] for s in have), (c, ms)
    print(f"  tiles {t}, groups {groups}", flush=True)
    mu, e = b.step()
    _compare(b, mu, e, ref, wls)
    # a second batch of the same shapes reads the cache
    b2 = sq.Batch(snaps, [wl.n_electrons for wl in wls])
    t2 = b2.autotune(cache)
    assert t2["block_nodes"] == t["block_nodes"] and t2["wg_per_cu"] == t["wg_per_cu"]
    assert b2.groups() == groups
    assert len(json.load(open(cache))) == 1
    # an entry edited by hand (every shape bit the cubes have, 32 nodes per
    # item) is applied as read, and the pass keeps its parity
    data = json.load(open(cache))
    key = next(iter(data))
    data[key]["block_nodes"] = 32
    data[key]["shapes"] = [[c, k, _shape_bits(c)] for c, k, _ in data[key]["shapes"]]
    json.dump(data, open(cache, "w"))
    b3 = sq.Batch(snaps, [wl.n_electrons for wl in wls])
    t3 = b3.autotune(cache)
    assert t3["block_nodes"] == 32
    assert all(s == _shape_bits(c) for c, _, s in b3.groups())
    mu, e = b3.step()
    _compare(b3, mu, e, ref, wls)


def test_batch_ensemble_sampled():
    """The 12-snapshot ensemble (32-500 atoms, cubes 21-37, n_pl 32-64, FP32-mixed)
    in one batched pass; sampled nodes of every snapshot against the oracle."""
    sq = _sq()
    wls = W.qmd_ensemble()
    print(f"case qmd ensemble: {len(wls)} snapshots", flush=True)
    snaps = _snaps(wls)
    b = sq.Batch(snaps, [wl.n_electrons for wl in wls], use_graph=True)
    mu, e = b.step()
    rng = np.random.default_rng(7)
    for i, (wl, g) in enumerate(zip(wls, snaps)):
        print(f"  {wl.name}: n={wl.n} mu={mu[i]:.10f} N={e[i][3]:.10f}", flush=True)
        assert abs(e[i][3] - wl.n_electrons) < 1e-9 * wl.n_electrons
        # FP64 reference on two sampled nodes, on FP64 bounds from the oracle
        nodes = rng.choice(g.nd, 2, replace=False)
        o = oracle.Oracle.from_workload(wl, veff=wl.veff())
        lo, hi = o.bounds(nodes)
        mom_ref = o.moments(lo, hi, nodes=nodes)
        rho_ref, _ = o.density_energy(lo, hi, mom_ref, mu[i])
        r = _np(b.rho[i])
        err = np.abs(r[nodes] - rho_ref).max() / r.max()
        print(f"    sampled rho rel err {err:.2e}", flush=True)
        assert err < 1e-5


def test_batch_bounds_reuse_across_veff_update():
    """bounds_every = 1000: pass 2 reuses the first pass's bounds after a small
    V_eff change and matches a fresh single-snapshot pass on those same bounds.
    Bounds rewritten outside the batch (sq_set_bounds) are not reused: the next
    pass computes fresh ones.  After a large V_eff change (beyond the margin
    slack) the pass also computes fresh bounds."""
    sq = _sq()
    wls = _small_ensemble()[:2]
    print("case bounds reuse", flush=True)
    snaps = _snaps(wls)
    refs = _snaps(wls)  # separate contexts for the reference passes
    b = sq.Batch(snaps, [wl.n_electrons for wl in wls], use_graph=True, bounds_every=1000)
    b.step()
    lo_hi = [g.spectral_bounds() for g in refs]  # the bounds the batch just computed

    def set_veff(scale):
        for g, r, wl in zip(snaps, refs, wls):
            v = torch.from_numpy(scale * wl.veff()).cuda()
            g.update_veff(v)
            r.update_veff(v)

    def check_fresh(mu, e):
        for i, (r, wl) in enumerate(zip(refs, wls)):
            mom1, mu1, rho1, e1 = r.scf_pass(wl.n_electrons)
            assert abs(mu[i] - mu1) < 1e-11, (mu[i], mu1)
            assert np.abs(_np(b.rho[i]) - _np(rho1)).max() < 1e-12 * _np(rho1).max()

    set_veff(0.98)
    mu, e = b.step()  # reuses the first pass's bounds
    for i, (r, wl) in enumerate(zip(refs, wls)):
        r.set_bounds(*lo_hi[i])
        mom = r.moments()
        mu1 = r.fermi_level(mom, wl.n_electrons)
        rho1, e1 = r.density_energy(mom, mu1)
        assert abs(mu[i] - mu1) < 1e-11
        assert np.abs(_np(b.rho[i]) - _np(rho1)).max() < 1e-12 * _np(rho1).max()
        assert abs(e[i][3] - wl.n_electrons) < 1e-10 * wl.n_electrons
    # the reusing pass of the 16^3 snapshot against the oracle at the new
    # V_eff on the same (reused) bounds
    wl = wls[0]
    o = oracle.Oracle.from_workload(wl, veff=0.98 * wl.veff())
    lmin, lmax = (_np(t) for t in lo_hi[0])
    mom_ref = o.moments(lmin, lmax)
    assert np.abs(_np(b.moments[0]) - mom_ref).max() < 1e-12
    mu_ref, _ = o.fermi_level(lmin, lmax, mom_ref, wl.n_electrons)
    assert abs(mu[0] - mu_ref) < 1e-10, (mu[0], mu_ref)
    rho_ref, e_ref = o.density_energy(lmin, lmax, mom_ref, mu[0])
    assert np.abs(_np(b.rho[0]) - rho_ref).max() < 1e-10 * rho_ref.max()
    assert np.abs(e[0] - e_ref).max() < 1e-10 * np.abs(e_ref).max(), (e[0], e_ref)
    # bounds injected from outside (here far too tight): not reused
    lo, hi = lo_hi[0]
    mid = 0.5 * (lo + hi)
    snaps[0].set_bounds(mid - 0.1, mid + 0.1)
    mu, e = b.step()
    check_fresh(mu, e)
    # a large change: beyond the margin slack, the previous bounds no longer hold
    set_veff(3.0)
    mu, e = b.step()
    check_fresh(mu, e)


def test_batch_redo_when_reused_bounds_fail():
    """reuse_check = 0: the batch trusts its previous bounds after V_eff is
    shifted down by 30 Ha, so every eigenvalue leaves the old interval and the
    moments leave [-1, 1] (SQ_EBOUNDS inside the pass); the pass is redone
    with fresh bounds and matches a fresh single-snapshot pass.  (A moderate
    escape can keep every moment within [-1, 1] at low n_pl, which is why the
    V_eff change test is on by default.)"""
    sq = _sq()
    wls = _small_ensemble()[:2]
    print("case bounds redo", flush=True)
    snaps = _snaps(wls)
    refs = _snaps(wls)
    b = sq.Batch(snaps, [wl.n_electrons for wl in wls], use_graph=True, bounds_every=1000, reuse_check=False)
    b.step()
    for g, r, wl in zip(snaps, refs, wls):
        v = torch.from_numpy(wl.veff() - 30.0).cuda()
        g.update_veff(v)
        r.update_veff(v)
    mu, e = b.step()
    for i, (r, wl) in enumerate(zip(refs, wls)):
        mom1, mu1, rho1, e1 = r.scf_pass(wl.n_electrons)
        assert abs(mu[i] - mu1) < 1e-11, (mu[i], mu1)
        assert np.abs(_np(b.rho[i]) - _np(rho1)).max() < 1e-12 * _np(rho1).max()
        assert abs(e[i][3] - wl.n_electrons) < 1e-10 * wl.n_electrons
