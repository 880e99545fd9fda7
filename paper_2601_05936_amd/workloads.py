"""Synthetic workloads: parameter sets and seeded initial fields.

This module only describes *problems* (box, boundary faces, fluid properties,
initial signed-distance level set, optional initial density/velocity).  It
holds none of the method's arithmetic, so both the GPU path and the CPU
oracle may use it.  Coordinates are cell centred, x = i + 1/2, and arrays are
row-major [nz][ny][nx].

The paper's experiments (Sec. 3) measure against third-party rising-bubble
benchmark data that is not available here; the workloads below are synthetic
stand-ins with the benchmark's dimensionless groups (Re, Eo, density and
viscosity ratios, Sec. 3.2 table of parameters) and the stratified-flow setup
of Sec. 3.1.
"""
from __future__ import annotations

import math

import numpy as np

D2Q9, D3Q19, D3Q27 = 0, 1, 2
F64, F32, F16DEV, BF16DEV = 0, 1, 2, 3
PERIODIC, NOSLIP, FREESLIP = 0, 1, 2
LIQUID, GAS = 0, 1
BGK, CUMULANT = 0, 1


def default_params(**kw) -> dict:
    """Every field of the parameter block with its default value."""
    p = dict(
        lattice=D3Q27, storage=F64, nx=8, ny=8, nz=8,
        bc=[PERIODIC] * 6, wall_u=[[0.0, 0.0, 0.0] for _ in range(6)],
        rho_phys=[1.0, 1.0], tau=[0.8, 0.8], accel=[[0.0] * 3, [0.0] * 3],
        sigma=0.0, band=6.0, n_ext=8, ext_dtau=0.5,
        reinit_every=10, n_reinit=5, reinit_dtau=0.3, heaviside_eps=1.5,
        use_pb=0, pb0=0.0, init_hydrostatic=0, fp16_scale_log2=12, collision=[BGK, BGK],
    )
    p.update(kw)
    return p


def tau_from_eta(eta: float, rho: float) -> float:
    """BGK relaxation time for dynamic viscosity eta at physical density rho
    (lattice units, cs^2 = 1/3): nu = eta/rho, tau = 1/2 + 3 nu."""
    return 0.5 + 3.0 * eta / rho


def grid(p: dict):
    """Cell-centre coordinate arrays X, Y, Z of shape [nz][ny][nx]."""
    z, y, x = np.meshgrid(np.arange(p["nz"]) + 0.5, np.arange(p["ny"]) + 0.5,
                          np.arange(p["nx"]) + 0.5, indexing="ij")
    return x, y, z


# ---------------------------------------------------------------------------
# The five named workloads.
# ---------------------------------------------------------------------------

def stratified_channel_2d(nx=64, ny=32, h_liquid=16.0, force=1e-6, steps=2000, storage=F64):
    """Two-layer channel: D2Q9, liquid y < h, gas above, density ratio 10,
    kinematic viscosity ratio 1 (tau 0.8 both), body-force density along x,
    periodic x, no-slip walls at y = 0 and y = ny (two-layer Poiseuille of
    Sec. 3.1)."""
    rho = [1.0, 0.1]
    p = default_params(
        lattice=D2Q9, storage=storage, nx=nx, ny=ny, nz=1,
        bc=[PERIODIC, PERIODIC, NOSLIP, NOSLIP, PERIODIC, PERIODIC],
        rho_phys=rho, tau=[0.8, 0.8],
        # a force density G acts on each phase as the acceleration G / rho_k
        accel=[[force / rho[0], 0.0, 0.0], [force / rho[1], 0.0, 0.0]],
    )
    x, y, z = grid(p)
    phi = y - h_liquid
    return dict(params=p, phi0=phi, rho0=None, u0=None, steps=steps,
                name=f"D2Q9 stratified channel {nx}x{ny}")


def static_droplet_3d(n=128, radius=20.0, sigma=1e-3, lattice=D3Q19, storage=F32, steps=5000):
    """Static droplet: periodic box, density ratio 1000, dynamic viscosity
    ratio 100, liquid inside a sphere.  The liquid starts at the Laplace
    pressure 2 sigma / R above the gas."""
    rho = [1.0, 1e-3]
    tau_l = 0.6
    eta_l = rho[0] * (tau_l - 0.5) / 3.0
    tau_g = tau_from_eta(eta_l / 100.0, rho[1])
    p = default_params(lattice=lattice, storage=storage, nx=n, ny=n, nz=n,
                       rho_phys=rho, tau=[tau_l, tau_g], sigma=sigma)
    x, y, z = grid(p)
    c = n / 2.0
    phi = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2) - radius
    dp = 2.0 * sigma / radius
    rho0 = np.where(phi < 0, 1.0 + dp / (rho[0] / 3.0), 1.0)
    return dict(params=p, phi0=phi, rho0=rho0, u0=None, steps=steps,
                name=f"static droplet {n}^3 R={radius}")


def rising_bubble_3d(nx=128, ny=128, nz=256, radius=16.0, zc=48.0, g=1e-5, eotvos=10.0,
                     morton=1e-3, rho_ratio=1000.0, eta_ratio=100.0, storage=F16DEV, steps=10000):
    """Rising bubble: D3Q27, gas sphere in liquid, gravity -z; sigma from the
    Eotvos number, liquid viscosity from the Morton number
    Mo = g eta_l^4 (rho_l - rho_g) / (rho_l^2 sigma^3); no-slip z, free-slip
    x and y (container walls of Sec. 3.2)."""
    rho = [1.0, 1.0 / rho_ratio]
    d = 2.0 * radius
    sigma = rho[0] * g * d * d / eotvos
    eta_l = (morton * rho[0] ** 2 * sigma ** 3 / (g * (rho[0] - rho[1]))) ** 0.25
    p = default_params(
        lattice=D3Q27, storage=storage, nx=nx, ny=ny, nz=nz,
        bc=[FREESLIP, FREESLIP, FREESLIP, FREESLIP, NOSLIP, NOSLIP],
        rho_phys=rho, tau=[tau_from_eta(eta_l, rho[0]), tau_from_eta(eta_l / eta_ratio, rho[1])],
        accel=[[0.0, 0.0, -g], [0.0, 0.0, -g]], sigma=sigma,
        use_pb=1, pb0=2.0 * sigma / radius, init_hydrostatic=1,
    )
    x, y, z = grid(p)
    phi = radius - np.sqrt((x - nx / 2.0) ** 2 + (y - ny / 2.0) ** 2 + (z - zc) ** 2)
    return dict(params=p, phi0=phi, rho0=None, u0=None, steps=steps,
                name=f"D3Q27 rising bubble {nx}x{ny}x{nz}")


def rising_bubble_2d(nx=256, ny=512, radius=24.0, yc=64.0, g=1e-5, sigma=5e-3, reynolds=35.0,
                     rho_ratio=100.0, eta_ratio=10.0, storage=F32, steps=2000):
    """2D rising bubble (the differentiation workload): D2Q9, gravity -y,
    liquid viscosity from Re = rho_l sqrt(g d^3) / eta_l (Sec. 3.2), no-slip
    y, free-slip x, reinitialisation off."""
    rho = [1.0, 1.0 / rho_ratio]
    d = 2.0 * radius
    eta_l = rho[0] * math.sqrt(g * d ** 3) / reynolds
    p = default_params(
        lattice=D2Q9, storage=storage, nx=nx, ny=ny, nz=1,
        bc=[FREESLIP, FREESLIP, NOSLIP, NOSLIP, PERIODIC, PERIODIC],
        rho_phys=rho, tau=[tau_from_eta(eta_l, rho[0]), tau_from_eta(eta_l / eta_ratio, rho[1])],
        accel=[[0.0, -g, 0.0], [0.0, -g, 0.0]], sigma=sigma,
        use_pb=1, pb0=sigma / radius, init_hydrostatic=1, reinit_every=0,
    )
    x, y, z = grid(p)
    phi = radius - np.sqrt((x - nx / 2.0) ** 2 + (y - yc) ** 2)
    return dict(params=p, phi0=phi, rho0=None, u0=None, steps=steps,
                name=f"D2Q9 rising bubble {nx}x{ny}")


def wavy_stratified_3d(n=512, amplitude=8.0, storage=F16DEV, steps=1000):
    """Throughput workload: D3Q27 n^3, periodic x and y, no-slip z, liquid
    below the wavy surface z = n/2 + a sin(2 pi x/n) cos(2 pi y/n), density
    ratio 1000, dynamic viscosity ratio 50, sigma 1e-3, no gravity."""
    rho = [1.0, 1e-3]
    tau_l = 0.55
    eta_l = rho[0] * (tau_l - 0.5) / 3.0
    p = default_params(
        lattice=D3Q27, storage=storage, nx=n, ny=n, nz=n,
        bc=[PERIODIC, PERIODIC, PERIODIC, PERIODIC, NOSLIP, NOSLIP],
        rho_phys=rho, tau=[tau_l, tau_from_eta(eta_l / 50.0, rho[1])], sigma=1e-3,
    )
    return dict(params=p, phi0=None, phi0_fn=lambda: wavy_phi(p, amplitude), rho0=None, u0=None,
                steps=steps, name=f"D3Q27 wavy stratified {n}^3")


def wavy_phi(p: dict, amplitude: float, dtype=np.float64) -> np.ndarray:
    """phi = z - nz/2 - a sin(2 pi x / nx) cos(2 pi y / ny), built plane by
    plane to bound host memory."""
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    xs = np.arange(nx) + 0.5
    ys = np.arange(ny) + 0.5
    surf = nz / 2.0 + amplitude * np.sin(2 * np.pi * xs / nx)[None, :] * np.cos(2 * np.pi * ys / ny)[:, None]
    out = np.empty((nz, ny, nx), dtype=dtype)
    for k in range(nz):
        out[k] = (k + 0.5) - surf
    return out


# ---------------------------------------------------------------------------
# Small seeded cases for parity tests.
# ---------------------------------------------------------------------------

def bubble_cluster(centers, radius, shape, lattice=D2Q9, g=1e-5, sigma=5e-3, rho_ratio=100.0, eta_ratio=10.0,
                   tau_l=0.6, storage=F64, reinit_every=10, n_reinit=3, collision=None):
    """Several gas bubbles of one radius in liquid, gravity along -y, one
    gas-pressure baseline per bubble (use_pb = 2), hydrostatic start; no-slip
    on the y faces, free slip on the others.  The level set is the union of
    the bubbles' signed distances, max_k (R - |x - c_k|)."""
    nx, ny, nz = shape
    dim = 2 if lattice == D2Q9 else 3
    rho = [1.0, 1.0 / rho_ratio]
    eta_l = rho[0] * (tau_l - 0.5) / 3.0
    bc = [FREESLIP, FREESLIP, NOSLIP, NOSLIP, PERIODIC, PERIODIC] if dim == 2 else \
         [FREESLIP, FREESLIP, NOSLIP, NOSLIP, FREESLIP, FREESLIP]
    p = default_params(lattice=lattice, storage=storage, nx=nx, ny=ny, nz=nz, bc=bc, rho_phys=rho,
                       tau=[tau_l, tau_from_eta(eta_l / eta_ratio, rho[1])],
                       accel=[[0.0, -g, 0.0], [0.0, -g, 0.0]], sigma=sigma, use_pb=2,
                       pb0=sigma * (1.0 if dim == 2 else 2.0) / radius, init_hydrostatic=1,
                       reinit_every=reinit_every, n_reinit=n_reinit,
                       collision=list(collision) if collision else [BGK, BGK])
    x, y, z = grid(p)
    phi = np.full(x.shape, -1e30)
    for c in centers:
        d2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + ((z - c[2]) ** 2 if dim == 3 else 0.0)
        phi = np.maximum(phi, radius - np.sqrt(d2))
    return dict(params=p, phi0=phi, rho0=None, u0=None, steps=200,
                name=f"{len(centers)} bubbles lattice={lattice} {nx}x{ny}x{nz}")


def nine_bubble_cluster_3d(d=32, storage=F16DEV, steps=1000):
    """The paper's cluster of nine rising bubbles (Sec. 3, last case) as a
    synthetic layout: domain 10 x 20 x 10 bubble diameters, gravity along
    -y, a lower layer of five bubbles (one at the axis, four on the
    diagonals 1.5 d off it) two diameters above the floor and an upper layer
    of four (0.75 d off the axis on the diagonals) two diameters higher;
    the physical parameters of the single 3D rising bubble (Eo 10,
    Mo 1e-3, density ratio 1000, viscosity ratio 100) with the paper's 3D
    pairing of collision operators (BGK liquid, cumulant gas)."""
    nx, ny, nz = 10 * d, 20 * d, 10 * d
    R = d / 2.0
    g = 1e-5
    ref = rising_bubble_3d(nx=8, ny=8, nz=8, radius=R, zc=4.0, g=g)["params"]
    cx, cz = nx / 2.0, nz / 2.0
    y0, y1 = 2.0 * d, 4.0 * d
    centers = [(cx, y0, cz)] + [(cx + sx * 1.5 * d, y0, cz + sz * 1.5 * d) for sx in (-1, 1) for sz in (-1, 1)]
    centers += [(cx + sx * 0.75 * d, y1, cz + sz * 0.75 * d) for sx in (-1, 1) for sz in (-1, 1)]
    w = bubble_cluster(centers, R, (nx, ny, nz), lattice=D3Q27, g=g, sigma=ref["sigma"], rho_ratio=1000.0,
                       eta_ratio=100.0, tau_l=ref["tau"][0], storage=storage, collision=[BGK, CUMULANT])
    w["steps"] = steps
    w["name"] = f"nine-bubble cluster D3Q27 {nx}x{ny}x{nz}"
    return w


def seeded_bubble(seed: int, lattice=D2Q9, shape=(37, 29, 1), storage=F64, gas_inside=True,
                  u_amp=0.02, sigma=2e-3, rho_ratio=10.0, eta_ratio=5.0, g=0.0, walls="mixed"):
    """A randomly placed circle/sphere with a seeded random initial velocity
    field, so that the interface moves and cells change phase within a few
    tens of steps.  Ragged sizes exercise partial tiles."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    rho = [1.0, 1.0 / rho_ratio]
    tau_l = 0.5 + rng.uniform(0.2, 0.5)
    eta_l = rho[0] * (tau_l - 0.5) / 3.0
    tau_g = tau_from_eta(eta_l / eta_ratio, rho[1])
    dim = 2 if lattice == D2Q9 else 3
    if walls == "periodic":
        bc = [PERIODIC] * 6
    elif walls == "mixed":
        bc = [PERIODIC, PERIODIC, NOSLIP, NOSLIP, FREESLIP, FREESLIP] if dim == 3 else \
             [FREESLIP, FREESLIP, NOSLIP, NOSLIP, PERIODIC, PERIODIC]
    else:
        raise ValueError(walls)
    wall_u = [[0.0] * 3 for _ in range(6)]
    wall_u[3] = [float(rng.uniform(-0.02, 0.02)), 0.0, 0.0]  # moving +y wall
    p = default_params(lattice=lattice, storage=storage, nx=nx, ny=ny, nz=nz, bc=bc, wall_u=wall_u,
                       rho_phys=rho, tau=[tau_l, tau_g], sigma=sigma,
                       accel=[[0.0, -g, 0.0], [0.0, -g, 0.0]] if dim == 2 else
                       [[0.0, 0.0, -g], [0.0, 0.0, -g]],
                       reinit_every=5, n_reinit=2)
    if g != 0.0:
        p.update(use_pb=1, init_hydrostatic=1)
    x, y, z = grid(p)
    r = rng.uniform(0.22, 0.3) * min(nx, ny)
    cx = nx / 2 + rng.uniform(-2, 2)
    cy = ny / 2 + rng.uniform(-2, 2)
    if dim == 3:
        cz = nz / 2 + rng.uniform(-2, 2)
        dist = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2)
    else:
        dist = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    phi = (r - dist) if gas_inside else (dist - r)
    if g != 0.0:
        p["pb0"] = sigma * (1.0 if dim == 2 else 2.0) / r
    # smooth random velocity: a few random Fourier modes
    u0 = np.zeros((nz, ny, nx, 3))
    for a in range(dim):
        for _ in range(3):
            kx, ky = rng.integers(1, 3, size=2)
            kz = rng.integers(0, 2)
            ph = rng.uniform(0, 2 * np.pi)
            u0[..., a] += u_amp / 3 * np.sin(2 * np.pi * (kx * x / nx + ky * y / ny + kz * z / max(nz, 1)) + ph)
    if walls == "mixed":  # keep the no-slip walls quiet at start
        u0 *= np.sin(np.pi * y / ny)[..., None]
    rho0 = 1.0 + 0.01 * rng.standard_normal((nz, ny, nx)) * 0.1
    return dict(params=p, phi0=phi, rho0=rho0, u0=u0, steps=30,
                name=f"seeded bubble seed={seed} lattice={lattice} {nx}x{ny}x{nz}")


# ---------------------------------------------------------------------------
# Two-level grids (the interface on the finest level).
# ---------------------------------------------------------------------------

def two_level_bubble(lattice=D2Q9, n=(48, 48, 1), box=(10, 38, 10, 38), centre=None, radius=7.0, gas_inside=True,
                     rho_ratio=10.0, tau=(0.8, 0.8), sigma=1e-2, g=0.0, u_amp=0.0, seed=0, storage=F64,
                     reinit_every=10, n_reinit=3, bc=None, wall_u=None):
    """A circle or sphere of radius R (coarse cells) in a periodic coarse
    grid of n nodes, held on the fine level of the box (ia, ib, ja, jb[, ka,
    kb]) of coarse nodes.  Coarse node (I, J, K) sits at (I, J, K), fine node
    (i, j, k) at (ia + i/2, ja + j/2, ka + k/2); phi is the signed distance
    (gas >= 0) in each level's cells.  Density 1 everywhere; the velocity is
    zero or a seeded sum of smooth periodic modes of amplitude u_amp, the
    same function on both levels; gravity g along -y (2D) or -z (3D) with
    the gas pressure baseline of the bubble; coarse faces bc (periodic by
    default) with wall velocities wall_u."""
    nx, ny, nz = n
    dim = 2 if lattice == D2Q9 else 3
    b = (tuple(int(v) for v in box) + (0, 0))[:6]
    if centre is None:
        centre = (0.5 * (b[0] + b[1]), 0.5 * (b[2] + b[3]), 0.5 * (b[4] + b[5]) if dim == 3 else 0.0)
    rho = [1.0, 1.0 / rho_ratio]
    acc = [0.0, -g, 0.0] if dim == 2 else [0.0, 0.0, -g]
    p = default_params(lattice=lattice, storage=storage, nx=nx, ny=ny, nz=nz,
                       bc=list(bc) if bc is not None else [PERIODIC] * 6, rho_phys=rho,
                       tau=list(tau), sigma=sigma, accel=[list(acc), list(acc)],
                       reinit_every=reinit_every, n_reinit=n_reinit)
    if wall_u is not None:
        p["wall_u"] = [list(map(float, v)) for v in wall_u]
    if g != 0.0:
        p.update(use_pb=1, pb0=sigma * (1.0 if dim == 2 else 2.0) / radius)
    rng = np.random.default_rng(seed)
    modes = []
    if u_amp:
        for a in range(dim):
            for _ in range(3):
                kx, ky = rng.integers(1, 3, size=2)
                kz = int(rng.integers(0, 2)) if dim == 3 else 0
                modes.append((a, kx, ky, kz, rng.uniform(0, 2 * np.pi)))

    def fields(x, y, z, scale):
        d2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + ((z - centre[2]) ** 2 if dim == 3 else 0.0)
        dist = np.sqrt(d2)
        phi = scale * ((radius - dist) if gas_inside else (dist - radius))
        u = np.zeros(x.shape + (3,))
        for a, kx, ky, kz, ph in modes:
            u[..., a] += u_amp / 3 * np.sin(2 * np.pi * (kx * x / nx + ky * y / ny + kz * z / nz) + ph)
        return phi.reshape(-1), np.ones(x.size), u.reshape(-1, 3)

    K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phi_c, rho_c, u_c = fields(1.0 * I, 1.0 * J, 1.0 * K, 1.0)
    fx, fy = 2 * (b[1] - b[0]) + 1, 2 * (b[3] - b[2]) + 1
    fz = 2 * (b[5] - b[4]) + 1 if dim == 3 else 1
    k, j, i = np.meshgrid(np.arange(fz), np.arange(fy), np.arange(fx), indexing="ij")
    zf = b[4] + 0.5 * k if dim == 3 else 0.0 * k
    phi_f, rho_f, u_f = fields(b[0] + 0.5 * i, b[2] + 0.5 * j, zf, 2.0)
    return dict(params=p, box=b, phi_c=phi_c, rho_c=rho_c, u_c=u_c, phi_f=phi_f, rho_f=rho_f, u_f=u_f,
                fine_shape=(fz, fy, fx),
                name=f"two-level {'bubble' if gas_inside else 'droplet'} lattice={lattice} {nx}x{ny}x{nz} box={b}")
