"""Pins of the oracle's several-bubble gas baseline.

Bubbles are the connected components of the smoothed Heaviside's support
(phi > -eps) over the lattice links; each has the single-bubble baseline at
its own centroid.  Fixed here against: connected-component labelling by
scipy.ndimage with the lattice's neighbourhood, numbering by smallest cell,
wrap across periodic faces, identity with the single-bubble baseline when
there is one bubble, and the physics the per-bubble baseline exists for
(bubbles at different heights keep their volume).
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle as O
from paper_2601_05936_amd import workloads as W


def _blobs(seed, shape, dim, n=7):
    rng = np.random.default_rng(seed)
    p = W.default_params(lattice={2: W.D2Q9, 3: W.D3Q27}[dim], nx=shape[0], ny=shape[1], nz=shape[2])
    x, y, z = W.grid(p)
    phi = np.full(x.shape, -1e30)
    for _ in range(n):
        c = rng.uniform(3, np.array(shape[:dim]) - 3)
        r = rng.uniform(1.0, 3.0) if dim == 2 else rng.uniform(0.8, 2.2)
        d2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + ((z - c[2]) ** 2 if dim == 3 else 0.0)
        phi = np.maximum(phi, r - np.sqrt(d2))
    return phi


@pytest.mark.parametrize("lat,shape,conn", [(W.D2Q9, (40, 36, 1), 2), (W.D3Q27, (28, 26, 24), 3),
                                            (W.D3Q19, (28, 26, 24), 2)])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bubble_labels_match_scipy(lat, shape, conn, seed):
    """The same partition as scipy.ndimage.label of {phi > -eps} with the
    velocity set's neighbourhood (D2Q9: 8, D3Q27: 26, D3Q19: 18 neighbours),
    walls on every face, and bubbles numbered by their smallest cell."""
    dim = 2 if lat == W.D2Q9 else 3
    phi = _blobs(seed, shape, dim)
    bc = [W.NOSLIP] * 4 + ([W.PERIODIC] * 2 if dim == 2 else [W.NOSLIP] * 2)
    p = W.default_params(lattice=lat, nx=shape[0], ny=shape[1], nz=shape[2], bc=bc, use_pb=2)
    lab = O.Oracle(p, phi).bubbles()["labels"]
    supp = np.clip(phi, -p["band"], p["band"]) > -p["heaviside_eps"]
    if dim == 2:
        ref, n = ndimage.label(supp[0], structure=ndimage.generate_binary_structure(2, 2))
        ref = ref[None]
    else:
        ref, n = ndimage.label(supp, structure=ndimage.generate_binary_structure(3, conn))
    assert n > 1
    assert ((lab >= 0) == supp).all()
    # same partition: one-to-one correspondence of the labels
    pairs = set(zip(lab[supp].tolist(), ref[supp].tolist()))
    assert len(pairs) == n == len(set(lab[supp].tolist()))
    # numbered by smallest cell index
    flat = lab.reshape(-1)
    first = [int(np.flatnonzero(flat == k)[0]) for k in range(n)]
    assert first == sorted(first)


def test_bubble_across_periodic_face_is_one():
    p = W.default_params(lattice=W.D2Q9, nx=32, ny=24, nz=1, bc=[W.PERIODIC, W.PERIODIC, W.NOSLIP, W.NOSLIP,
                                                               W.PERIODIC, W.PERIODIC], use_pb=2)
    x, y, z = W.grid(p)
    dx = np.minimum(np.abs(x - 1.0), 32 - np.abs(x - 1.0))  # circle centred on the x = 0 face
    phi = 5.0 - np.sqrt(dx ** 2 + (y - 12.0) ** 2)
    b = O.Oracle(p, phi).bubbles()
    assert b["count"] == 1


def test_single_bubble_reduces_to_the_single_baseline():
    """With one bubble the per-bubble baseline is the single-bubble one: the
    two modes give identical states, step for step."""
    w = W.rising_bubble_2d(nx=48, ny=64, radius=8.0, yc=22.0, g=4e-5, sigma=5e-3, storage=W.F64)
    p1 = dict(w["params"])
    p2 = dict(w["params"], use_pb=2)
    o1, o2 = O.Oracle(p1, w["phi0"]), O.Oracle(p2, w["phi0"])
    o1.step(40)
    o2.step(40)
    assert np.array_equal(o1.populations(), o2.populations())
    b = o2.bubbles()
    assert b["count"] == 1
    assert b["pb"][0] == o1.integrals()["pb"]


def test_bubbles_at_different_heights_keep_their_volume():
    """Two equal bubbles two diameters apart in height under gravity.  One
    baseline from the joint centroid puts the lower bubble's gas below and
    the upper one's above the surrounding liquid pressure by rho_l g dh / 2,
    which compresses / expands them; a baseline per bubble does not."""
    drift = {}
    for mode in (1, 2):
        w = W.bubble_cluster([(24.0, 24.0, 0.0), (24.0, 56.0, 0.0)], 6.0, (48, 96, 1), g=2e-5, sigma=5e-3,
                             rho_ratio=100.0, reinit_every=10, n_reinit=3)
        p = dict(w["params"], use_pb=mode)
        o = O.Oracle(p, w["phi0"])
        v0 = _volumes(o)
        o.step(300)
        v1 = _volumes(o)
        drift[mode] = np.abs(v1 / v0 - 1.0)
    print(drift)
    assert drift[2].max() < 0.25 * drift[1].max()


def _volumes(o):
    """Gas volume of the lower and upper half of the domain (one bubble each)."""
    phi = o.interface()["phi"][0]
    h = np.vectorize(lambda v: O.heaviside(v, 1.5))(phi)
    ny = phi.shape[0]
    return np.array([h[: ny // 2].sum(), h[ny // 2:].sum()])
