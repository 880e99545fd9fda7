"""lsb_get_integrals_static (no allocation: partial sums in the library's
static device array) against lsb_get_integrals, through the C ABI: two
calls in a row on one GPU, the second on a smaller grid, each equal to the
allocating entry point bit for bit."""
import numpy as np
import pytest

from paper_2601_05936_amd import workloads as W

pytestmark = pytest.mark.gpu


def _pair(s, torch):
    I = s.integrals()
    out = torch.full((16,), float("nan"), dtype=torch.float64, device="cuda:0")
    s.integrals_static(out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want = np.array(list(I["mass"]) + [I["volume_gas"]] + list(I["centroid"]) + list(I["vel_b"]) + [I["pb"], I["umax"]])
    return got, want


def test_static_integrals_match_allocating_entry_point(require_gpu):
    import torch
    from paper_2601_05936_amd.lsb import Sim
    cases = [W.seeded_bubble(3, lattice=W.D3Q19, shape=(41, 38, 36), g=2e-4, u_amp=0.02),
             W.seeded_bubble(4, lattice=W.D2Q9, shape=(37, 29, 1))]
    for w in cases:
        s = Sim(w["params"]).init(w["phi0"], w["rho0"], w["u0"])
        s.step(7)
        got, want = _pair(s, torch)
        print(w["params"]["lattice"], got[:12], flush=True)
        np.testing.assert_array_equal(got[:11], want)
        assert got[11] == 0.0 and np.all(got[12:] == 0.0)  # no unstable cell; pads
        assert want[2] > 0  # the gas volume is not trivial
