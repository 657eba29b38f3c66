"""The allocation-free entry point sq_density_energy_static against
sq_density_energy on the GPU, through the C ABI: two calls in a row on one
GPU (the second on a smaller cell), each compared with the workspace-based
entry point on the same moments and Fermi level."""
from __future__ import annotations

import numpy as np
import pytest

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


def _case(wl):
    from paper_1708_07913_amd import sq
    g = sq.SQ.from_workload(wl, veff=torch.from_numpy(wl.veff()).cuda(), precision=sq.FP64)
    g.spectral_bounds()
    mom = g.moments()
    mu = g.fermi_level(mom, wl.n_electrons)
    rho_ref, e_ref = g.density_energy(mom, mu)
    rho = torch.full((g.nd,), float("nan"), dtype=torch.float64, device="cuda")
    rho, e = g.density_energy_static(mom, mu, rho)
    torch.cuda.synchronize()
    r, r0 = rho.cpu().numpy(), rho_ref.cpu().numpy()
    print(f"case {wl.name}: nodes {g.nd}  rho {np.abs(r - r0).max() / r0.max():.2e}  "
          f"E {np.abs(e - e_ref).max() / np.abs(e_ref).max():.2e}", flush=True)
    assert np.all(np.isfinite(r))
    assert np.abs(r - r0).max() <= 1e-12 * r0.max()
    assert np.abs(e - e_ref).max() <= 1e-12 * np.abs(e_ref).max()
    assert abs(e[3] - wl.n_electrons) < 1e-10 * wl.n_electrons


def test_static_density_matches_workspace_entry_twice():
    # a larger cell first, then a smaller one: the second call reuses the
    # scratch the first one left behind
    _case(W.fcc_workload("static_al32_c11", 2, 7.78, 0.15, 31, 0.5, 2.5, 32, 1.0))
    _case(W.tiny_cell())
