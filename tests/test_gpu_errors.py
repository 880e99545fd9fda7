"""Error returns of the C ABI that need a device: the stability check of
lsb_step (LSB_EUNSTABLE on a non-finite or non-positive density).

The unstable states are ordinary inputs: a non-finite or strongly negative
LB density in one bulk cell, far from the level-set band, so that only the
collide-stream arithmetic sees it (no index is ever computed from it).  A
mildly negative one (-0.5) is no test: pull streaming replaces the cell's
populations by its neighbours' in one step and no density stays below zero.
"""
import numpy as np
import pytest

from paper_2601_05936_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("bad", [np.nan, np.inf, -20.0])
def test_step_reports_unstable_state(require_gpu, bad):
    from paper_2601_05936_amd.lsb import Sim, LsbError, LSB_EUNSTABLE
    w = W.seeded_bubble(0, lattice=W.D2Q9, shape=(48, 40, 1), walls="periodic")
    phi0 = w["phi0"]
    rho0 = np.ones_like(phi0) if w["rho0"] is None else np.array(w["rho0"], dtype=np.float64)
    far = np.unravel_index(np.argmax(np.abs(phi0)), phi0.shape)
    assert abs(phi0[far]) > w["params"]["band"] + 3  # outside the band and its neighbourhood
    rho0 = rho0.copy()
    rho0[far] = bad
    Sim(w["params"]).init(phi0, rho0, w["u0"]).step(3)  # without the check the steps run through
    s = Sim(w["params"]).init(phi0, rho0, w["u0"])
    with pytest.raises(LsbError) as e:
        s.step(5, check_every=1)  # checked after the first step
    assert e.value.code == LSB_EUNSTABLE
    assert "unstable" in str(e.value)


def test_step_check_passes_on_a_stable_state(require_gpu):
    from paper_2601_05936_amd.lsb import Sim
    w = W.seeded_bubble(0, lattice=W.D2Q9, shape=(48, 40, 1), walls="periodic")
    s = Sim(w["params"]).init(w["phi0"], w["rho0"], w["u0"])
    s.step(6, check_every=2)
    assert s.integrals()["step"] == 6
