import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
for p in (ROOT, os.path.join(ROOT, "tests")):
    if p not in sys.path:
        sys.path.insert(0, p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes tens of seconds")


@pytest.fixture(scope="session")
def tiny():
    """Tiny-cell oracle run shared by several pins: (workload, V, oracle, bounds, moments, mu)."""
    import oracle
    from paper_1708_07913_amd import workloads as W
    wl = W.tiny_cell()
    V = wl.veff()
    o = oracle.Oracle.from_workload(wl, veff=V)
    lmin, lmax = o.bounds()
    mom = o.moments(lmin, lmax)
    mu, _ = o.fermi_level(lmin, lmax, mom, wl.n_electrons)
    return dict(wl=wl, V=V, o=o, lmin=lmin, lmax=lmax, mom=mom, mu=mu)
