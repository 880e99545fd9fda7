"""The reduced-precision population codec through the C ABI.

FP16 deviation storage keeps s (f - w_i rho_ref) / w_i (s = 2^12) rounded to
nearest even with 11 significant bits, BF16 keeps (f - w_i rho_ref) / w_i
with 8: after a round trip a population is off by at most 2^-11 (FP16) or
2^-8 (BF16) of its deviation, plus the FP32 arithmetic around the codec
(a few 2^-24 of the deviation) and, below FP16's normal range, half its
subnormal spacing (w_i 2^-25 / s).  The rest state is all zero deviations
and is kept bit for bit, with a flat interface at any offset as well.
"""
import numpy as np
import pytest

from paper_2601_05936_amd import workloads as W

pytestmark = pytest.mark.gpu

BITS = {W.F16DEV: 11, W.BF16DEV: 8}


@pytest.mark.parametrize("storage", [W.F16DEV, W.BF16DEV])
@pytest.mark.parametrize("lat", [W.D2Q9, W.D3Q27])
@pytest.mark.parametrize("case", ["large", "tiny"])
def test_codec_round_trip_bound(require_gpu, storage, lat, case):
    """Equilibria of random density and velocity ('large': |u| ~ 0.05,
    |rho - 1| ~ 0.02) or of density 1 and velocities down to 1e-9 ('tiny':
    deviations deep into FP16's subnormal range; the phase's reference
    density is then exactly 1) are stored at initialisation and read back:
    every population within the codec's bound of its FP64 value."""
    import oracle as O
    from paper_2601_05936_amd.lsb import Sim
    shape = (12, 10, 1) if lat == W.D2Q9 else (10, 9, 8)
    p = W.default_params(lattice=lat, storage=storage, nx=shape[0], ny=shape[1], nz=shape[2])
    rng = np.random.default_rng(21)
    N = shape[0] * shape[1] * shape[2]
    if case == "large":
        rho = 1.0 + 0.02 * rng.standard_normal(N)
        u = 0.05 * rng.standard_normal((N, 3))
    else:
        rho = np.ones(N)
        u = 10.0 ** rng.uniform(-9, -5, (N, 1)) * rng.standard_normal((N, 3))
    if lat == W.D2Q9:
        u[:, 2] = 0.0
    s = Sim(p).init(-6.0 * np.ones(N), rho, u)  # one phase everywhere
    got = s.populations().reshape(-1, N)
    D, Q, c, w, _ = O.lattice(lat)
    exact = np.stack([O.feq(lat, rho[k], u[k]) for k in range(N)], axis=1)
    # the reference density is the mean initial density as stored, rounded
    # to FP32: 1 exactly in the tiny case; in the large case it may differ
    # from the exact mean by dr
    rho_ref = 1.0 if case == "tiny" else float(np.float32(np.mean(rho)))
    dr = 0.0 if case == "tiny" else 2.0 ** -BITS[storage] * float(np.max(np.abs(rho - 1.0))) + 2.0 ** -23
    dev = np.abs(exact - w[:, None] * rho_ref) + w[:, None] * dr
    scale = 4096.0 if storage == W.F16DEV else 1.0
    bound = dev * (2.0 ** -BITS[storage] + 8 * 2.0 ** -24) + w[:, None] * 2.0 ** -25 / scale + 1e-17
    err = np.abs(got - exact)
    print(storage, lat, case, "max err / bound", float(np.max(err / bound)), flush=True)
    assert np.all(err <= bound)


@pytest.mark.parametrize("storage", [W.F16DEV, W.BF16DEV])
@pytest.mark.parametrize("lat", [W.D2Q9, W.D3Q19, W.D3Q27])
def test_rest_state_with_flat_interface_bit_exact(require_gpu, storage, lat):
    """Uniform density 1 at rest on both sides of a flat interface off the
    lattice (sigma and the density ratio arbitrary, no gravity): every
    population stays exactly w_i through 20 steps with reinitialisation."""
    import oracle as O
    from paper_2601_05936_amd.lsb import Sim
    shape = (16, 20, 1) if lat == W.D2Q9 else (12, 16, 10)
    p = W.default_params(lattice=lat, storage=storage, nx=shape[0], ny=shape[1], nz=shape[2],
                         rho_phys=[1.0, 0.01], tau=[0.7, 1.1], sigma=3e-3, reinit_every=5, n_reinit=2,
                         bc=[W.PERIODIC, W.PERIODIC, W.NOSLIP, W.NOSLIP, W.PERIODIC, W.PERIODIC])
    x, y, z = W.grid(p)
    s = Sim(p).init(y - 10.3)
    s.step(20)
    D, Q, c, w, _ = O.lattice(lat)
    pop = s.populations()
    np.testing.assert_array_equal(pop, np.broadcast_to(w.reshape((Q, 1, 1, 1)), pop.shape))
