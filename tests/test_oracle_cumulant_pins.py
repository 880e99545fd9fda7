"""Pins of the oracle's cumulant collision (Sec. 2.1, D3Q27).

The oracle computes joint cumulants from the moment-cumulant formula over set
partitions and inverts them the same way.  These tests fix that machinery and
the collision built on it against facts that do not come from the oracle:
the cumulants of a Gaussian (exact Gauss-Hermite quadrature), additivity of
cumulants over independent sums, shift and scale behaviour, vanishing mixed
cumulants of independent axes, raw moments summed directly, conservation,
the product equilibrium as the fixed point (its cumulants are those of the
Maxwell distribution), the BGK operator's shear moments, axis-permutation
covariance, and the viscosity of a decaying shear wave.
"""
import math
from itertools import product

import numpy as np
import pytest

import oracle as O
from paper_2601_05936_amd import workloads as W

ORDER = np.array([[[a + b + c for c in range(3)] for b in range(3)] for a in range(3)])
_, _, C27, W27, _ = O.lattice(W.D3Q27)
C27F = C27.astype(float)


def direct_moments(pts, w):
    """Normalised raw moments m[a, b, c] = E[x^a y^b z^c], summed directly."""
    m = np.zeros((3, 3, 3))
    for a, b, c in product(range(3), repeat=3):
        m[a, b, c] = np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c) / w.sum()
    return m


def random_points(rng, n):
    return rng.normal(size=(n, 3)), rng.uniform(0.2, 1.0, n)


def product_equilibrium(rho, u):
    """D3Q27 distribution rho prod_a phi(c_a, u_a) with the three-point
    marginal of mean u_a and variance cs^2 = 1/3: phi(0) = 2/3 - u^2,
    phi(+-1) = (1/3 + u^2 +- u) / 2."""
    def phi(c, v):
        return 2.0 / 3.0 - v * v if c == 0 else (1.0 / 3.0 + v * v + c * v) / 2.0
    return np.array([rho * phi(c[0], u[0]) * phi(c[1], u[1]) * phi(c[2], u[2]) for c in C27])


def random_state(rng, amp):
    """Populations near a random equilibrium with a random non-equilibrium part."""
    rho = 1.0 + rng.uniform(-0.05, 0.05)
    u = rng.uniform(-0.08, 0.08, 3)
    return product_equilibrium(rho, u) * (1.0 + amp * rng.uniform(-1, 1, 27))


def bgk(f, omega):
    rho = f.sum()
    u = C27F.T @ f / rho
    cu = C27F @ u
    feq = W27 * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * u @ u)
    return f - omega * (f - feq)


def second_moment(f):
    return np.einsum("i,ia,ib->ab", f, C27F, C27F)


def dev(t):
    return t - np.trace(t) / 3.0 * np.eye(3)


# ---------------------------------------------------------------------------
# the cumulant transform
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cumulants_of_a_gaussian_by_exact_quadrature(seed):
    """A Gauss-Hermite tensor rule with 8 nodes integrates polynomials of
    degree <= 15 per axis exactly, so the point set has the moments of the
    normal distribution N(mu, L L^T) up to order 6: first cumulants mu,
    second L L^T, all others zero (textbook property of the Gaussian)."""
    rng = np.random.default_rng(seed)
    x, w = np.polynomial.hermite_e.hermegauss(8)
    w = w / math.sqrt(2 * math.pi)
    Z = np.array(list(product(x, x, x)))
    Wt = np.array([a * b * c for a, b, c in product(w, w, w)])
    L = np.tril(rng.uniform(-0.7, 0.7, (3, 3))) + np.eye(3)
    mu = rng.uniform(-0.3, 0.3, 3)
    k = O.cumulants_points(Z @ L.T + mu, Wt)
    S = L @ L.T
    np.testing.assert_allclose([k[1, 0, 0], k[0, 1, 0], k[0, 0, 1]], mu, atol=1e-13)
    for (a, b), idx in {(0, 0): (2, 0, 0), (1, 1): (0, 2, 0), (2, 2): (0, 0, 2),
                        (0, 1): (1, 1, 0), (0, 2): (1, 0, 1), (1, 2): (0, 1, 1)}.items():
        assert abs(k[idx] - S[a, b]) < 1e-12
    assert np.abs(k[ORDER >= 3]).max() < 1e-11


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_cumulants_add_over_independent_sums(seed):
    """Cumulants of X + Y with X, Y independent are the sums of theirs (the
    cumulant generating function of a convolution is the sum)."""
    rng = np.random.default_rng(seed)
    X, wx = random_points(rng, 5)
    Y, wy = random_points(rng, 4)
    Zp = (X[:, None, :] + Y[None, :, :]).reshape(-1, 3)
    Zw = (wx[:, None] * wy[None, :]).reshape(-1)
    kx, ky, kz = O.cumulants_points(X, wx), O.cumulants_points(Y, wy), O.cumulants_points(Zp, Zw)
    np.testing.assert_allclose(kz[ORDER >= 1], (kx + ky)[ORDER >= 1], atol=1e-12)


def test_cumulants_shift_and_scale():
    """Translation moves only the first cumulants; scaling axis a by s_a
    multiplies kappa_abc by sx^a sy^b sz^c."""
    rng = np.random.default_rng(6)
    X, w = random_points(rng, 7)
    k0 = O.cumulants_points(X, w)
    v = np.array([0.4, -1.3, 2.2])
    k1 = O.cumulants_points(X + v, w)
    np.testing.assert_allclose(k1[ORDER >= 2], k0[ORDER >= 2], atol=1e-12)
    np.testing.assert_allclose([k1[1, 0, 0] - k0[1, 0, 0], k1[0, 1, 0] - k0[0, 1, 0], k1[0, 0, 1] - k0[0, 0, 1]], v,
                               atol=1e-13)
    s = np.array([0.5, 2.0, -1.5])
    k2 = O.cumulants_points(X * s, w)
    scale = np.array([[[s[0] ** a * s[1] ** b * s[2] ** c for c in range(3)] for b in range(3)] for a in range(3)])
    np.testing.assert_allclose(k2[ORDER >= 1], (k0 * scale)[ORDER >= 1], rtol=1e-12, atol=1e-12)


def test_mixed_cumulants_of_independent_axes_vanish():
    """A product of three one-dimensional distributions has independent
    coordinates: every cumulant that involves two or more axes is zero, and
    kappa_200 is the variance of the x marginal."""
    rng = np.random.default_rng(8)
    xs = [rng.normal(size=4) for _ in range(3)]
    ws = [rng.uniform(0.1, 1.0, 4) for _ in range(3)]
    pts = np.array([[a, b, c] for a in xs[0] for b in xs[1] for c in xs[2]])
    wt = np.array([a * b * c for a in ws[0] for b in ws[1] for c in ws[2]])
    k = O.cumulants_points(pts, wt)
    mixed = np.array([[[(a > 0) + (b > 0) + (c > 0) >= 2 for c in range(3)] for b in range(3)] for a in range(3)])
    assert np.abs(k[mixed]).max() < 1e-12
    mx = np.sum(ws[0] * xs[0]) / ws[0].sum()
    var = np.sum(ws[0] * (xs[0] - mx) ** 2) / ws[0].sum()
    assert abs(k[2, 0, 0] - var) < 1e-13


def test_moments_from_cumulants_returns_the_raw_moments():
    rng = np.random.default_rng(9)
    X, w = random_points(rng, 6)
    m = O.moments_from_cumulants(O.cumulants_points(X, w))
    np.testing.assert_allclose(m, direct_moments(X, w), rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------
# the collision
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_cumulant_collision_conserves_mass_and_momentum(seed):
    rng = np.random.default_rng(10 + seed)
    f = random_state(rng, 0.2)
    acc = rng.uniform(-1e-3, 1e-3, 3)
    out = O.cumulant_collide(f, rng.uniform(0.3, 1.9), acc=acc)
    rho = f.sum()
    assert abs(out.sum() - rho) < 1e-14
    np.testing.assert_allclose(C27F.T @ out, C27F.T @ f + rho * acc, atol=1e-15)


@pytest.mark.parametrize("omega1", [0.4, 1.0, 1.7])
def test_product_equilibrium_is_the_fixed_point(omega1):
    """The product equilibrium has the Maxwell cumulants (variance cs^2 per
    axis, independent axes): the collision leaves it unchanged."""
    rng = np.random.default_rng(20)
    for _ in range(4):
        f = product_equilibrium(1.0 + rng.uniform(-0.1, 0.1), rng.uniform(-0.1, 0.1, 3))
        np.testing.assert_allclose(O.cumulant_collide(f, omega1), f, rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", range(4))
def test_unit_rates_give_the_product_equilibrium(seed):
    """With every rate one all cumulants take their Maxwell values, and the
    only D3Q27 distribution with those (given rho and u) is the product
    equilibrium."""
    rng = np.random.default_rng(30 + seed)
    f = random_state(rng, 0.3)
    rho = f.sum()
    u = C27F.T @ f / rho
    np.testing.assert_allclose(O.cumulant_collide(f, 1.0), product_equilibrium(rho, u), atol=1e-15)


@pytest.mark.parametrize("seed", range(4))
def test_shear_moments_equal_bgk_and_trace_is_relaxed(seed):
    """The deviatoric second moment after the collision is that of BGK with
    the same omega (both relax the deviatoric central second moment by
    1 - omega and keep rho u u); with omega_2 = 1 the trace of the central
    second moment becomes 3 cs^2 = 1 per unit density."""
    rng = np.random.default_rng(40 + seed)
    f = random_state(rng, 0.3)
    om = rng.uniform(0.3, 1.9)
    out = O.cumulant_collide(f, om)
    np.testing.assert_allclose(dev(second_moment(out)), dev(second_moment(bgk(f, om))), atol=1e-15)
    rho = f.sum()
    u = C27F.T @ f / rho
    assert abs(np.trace(second_moment(out)) / rho - u @ u - 1.0) < 1e-14


def test_rates_zero_is_the_identity_and_bulk_rate_acts_on_the_trace():
    """All rates zero: nothing relaxes, the transform and its inverse return
    the populations.  Bulk rate omega_2 alone: the trace of the central second
    moment relaxes by 1 - omega_2 towards 1, the deviatoric part is kept."""
    rng = np.random.default_rng(50)
    f = random_state(rng, 0.3)
    np.testing.assert_allclose(O.cumulant_collide(f, 0.0, 0.0, 0.0), f, atol=1e-15)
    rho = f.sum()
    u = C27F.T @ f / rho
    om2 = 0.6
    out = O.cumulant_collide(f, 0.0, om2, 0.0)
    tr_in = np.trace(second_moment(f)) / rho - u @ u
    tr_out = np.trace(second_moment(out)) / rho - u @ u
    assert abs((tr_out - 1.0) - (1 - om2) * (tr_in - 1.0)) < 1e-14
    np.testing.assert_allclose(dev(second_moment(out)), dev(second_moment(f)), atol=1e-15)


def test_axis_permutation_covariance():
    """Renaming the axes (x, y, z) -> (y, z, x) commutes with the collision."""
    rng = np.random.default_rng(60)
    f = random_state(rng, 0.3)
    perm = [1, 2, 0]
    # direction j of the renamed lattice is the image of direction i
    img = [int(np.flatnonzero((C27 == C27[i][perm]).all(1))[0]) for i in range(27)]
    g = np.zeros(27)
    g[img] = f
    out_f = O.cumulant_collide(f, 1.3, acc=(1e-4, -2e-4, 3e-4))
    out_g = O.cumulant_collide(g, 1.3, acc=(-2e-4, 3e-4, 1e-4))
    np.testing.assert_allclose(out_g[img], out_f, atol=1e-15)


def test_cumulant_shear_wave_decays_with_the_bgk_viscosity():
    """Whole-step check of the cumulant gas phase: a periodic shear wave in a
    gas-filled D3Q27 box decays as exp(-nu k^2 t), nu = cs^2 (tau - 1/2), to
    second order in the resolution (the same decay time in lattice units of
    the wavelength at 32 and 64 cells)."""
    tau, U = 0.7, 1e-4
    nu = (tau - 0.5) / 3.0
    errs = []
    for ny in (32, 64):
        t = 200 * (ny // 32) ** 2
        p = W.default_params(lattice=W.D3Q27, nx=1, ny=ny, nz=1, tau=[tau, tau], collision=[W.BGK, W.CUMULANT])
        x, y, z = W.grid(p)
        k = 2 * np.pi / ny
        u0 = np.zeros((1, ny, 1, 3))
        u0[..., 0] = U * np.sin(k * y)
        o = O.Oracle(p, 6.0 * np.ones((1, ny, 1)), u0=u0)
        o.step(t)
        u = o.fields()["u"][0, :, 0, 0]
        amp = 2 * np.mean(u * np.sin(k * y[0, :, 0]))
        errs.append(abs(amp / (U * math.exp(-nu * k * k * t)) - 1))
    assert errs[1] < 2e-3
    assert errs[0] / errs[1] > 3.0


def test_cumulant_needs_d3q27():
    p = W.default_params(lattice=W.D3Q19, nx=4, ny=4, nz=4, collision=[W.BGK, W.CUMULANT])
    with pytest.raises(Exception):
        O.Oracle(p, np.ones((4, 4, 4)))
