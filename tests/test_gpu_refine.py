"""Static refinement (D2Q9, D3Q19, D3Q27; BGK, FP64, ratio 2; two to four
nested levels) on the GPU against the CPU oracle, element by element on
every level.

The coupling follows the Dupuis-Chopard approach the paper adopts for its
refinement jumps (Sec. 2, lattice Boltzmann method); lsb_refine.h states
the steps.  Cases: a small grid, a grid wider than one 256-lane block (the
fine rows span two blocks with a ragged tail), the minimal 2 x 2-cell patch,
and the benchmark's configurations (2D: 2048^2 coarse nodes with a
1024^2-cell patch; 3D: D3Q27 192^3 with a 96^3-cell patch), which the oracle
still finishes in seconds; in 3D also D3Q19 and a minimal patch.  Nested
levels: three and four levels in 2D and 3D, rows of the innermost level
spanning three blocks with a ragged tail, minimal inner patches, and the
benchmark's three-level configuration (2048^2 coarse, a 1024^2-cell level
1, a 512^2-coarse-cell level 2 with 2049^2 nodes).  Trees of boxes (several
boxes per grid, nested boxes under some), including the benchmark's
nine-box tree; the level-set sensors (one box, one per level, one per
seed) and re-meshing of chains and trees; graph-launched steps against
plain launches, bit for bit.  Bar:
max |f_gpu - f_oracle| <= 1e-13 (populations are O(0.1); the two sides
differ only in the rounding of fused multiply-adds, measured at a few 1e-16
per step).
"""
import numpy as np
import pytest

from oracle import RefineOracle

pytestmark = pytest.mark.gpu

TOL = 1e-13


def _fields(nx, ny, patch, seed, amp=0.02):
    """Smooth random velocity and density fields sampled on both levels."""
    rng = np.random.default_rng(seed)
    kx, ky = rng.integers(1, 4, 4), rng.integers(1, 4, 4)
    ph = rng.uniform(0, 2 * np.pi, 4)

    def sample(x, y):
        s = [np.sin(2 * np.pi * (kx[m] * x / nx + ky[m] * y / ny) + ph[m]) for m in range(4)]
        return 1.0 + 0.5 * amp * s[0], np.stack([amp * s[1] + 0.3 * amp * s[3], amp * s[2]], 1)

    J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    rc, uc = sample(I.reshape(-1).astype(float), J.reshape(-1).astype(float))
    o = RefineOracle(nx, ny, patch, 0.7)
    xf, yf = o.fine_coords()
    rf, uf = sample(xf, yf)
    return rc, uc, rf, uf


def _run_both(nx, ny, patch, tau_c, steps, seed):
    from paper_2601_05936_amd.lsb import Refine
    rc, uc, rf, uf = _fields(nx, ny, patch, seed)
    o = RefineOracle(nx, ny, patch, tau_c).init(rc, uc, rf, uf)
    g = Refine(nx, ny, patch, tau_c).init(rc, uc, rf, uf)
    o.step(steps)
    g.step(steps)
    return o.populations(), g.populations()


@pytest.mark.parametrize("nx,ny,patch,tau_c,steps", [
    (37, 29, (5, 20, 3, 17), 0.7, 40),
    (300, 40, (100, 290, 5, 30), 0.62, 20),   # fine rows of 381 nodes: two blocks, ragged tail
    (8, 8, (1, 3, 1, 3), 0.9, 30),            # the minimal patch
])
def test_refine_matches_oracle(require_gpu, nx, ny, patch, tau_c, steps):
    (oc, of), (gc, gf) = _run_both(nx, ny, patch, tau_c, steps, seed=nx)
    ec, ef = np.max(np.abs(gc - oc)), np.max(np.abs(gf - of))
    print(f"refine {nx}x{ny} patch {patch}: coarse {ec:.2e} fine {ef:.2e}", flush=True)
    assert ec <= TOL and ef <= TOL


def test_refine_benchmark_configuration(require_gpu):
    """2048^2 coarse nodes, patch over [512, 1536]^2 (2049^2 fine nodes), the
    launch configuration of the benchmark, 2 coarse steps."""
    nx = ny = 2048
    patch = (512, 1536, 512, 1536)
    (oc, of), (gc, gf) = _run_both(nx, ny, patch, 0.6, 2, seed=7)
    ec, ef = np.max(np.abs(gc - oc)), np.max(np.abs(gf - of))
    print(f"refine 2048^2: coarse {ec:.2e} fine {ef:.2e}", flush=True)
    assert ec <= TOL and ef <= TOL


def test_refine_uniform_state_is_fixed(require_gpu):
    """Any uniform state is a fixed point of the coupled step (exact up to
    rounding), on the benchmark's grid."""
    from paper_2601_05936_amd.lsb import Refine
    nx = ny = 2048
    patch = (512, 1536, 512, 1536)
    g = Refine(nx, ny, patch, 0.6)
    u = np.array([0.04, -0.03])
    g.init(np.full(g.n_coarse, 1.02), np.tile(u, g.n_coarse), np.full(g.n_fine, 1.02), np.tile(u, g.n_fine))
    c0, f0 = g.populations()
    g.step(3)
    c1, f1 = g.populations()
    assert np.max(np.abs(c1 - c0)) < 1e-15 and np.max(np.abs(f1 - f0)) < 1e-15


# --- 3D: D3Q19 and D3Q27, face interpolation ---

def _fields3(n3, lattice, patch, seed, amp=0.02):
    nx, ny, nz = n3
    rng = np.random.default_rng(seed)
    kk = rng.integers(1, 3, (4, 3))
    ph = rng.uniform(0, 2 * np.pi, 4)

    def sample(x, y, z):
        s = [np.sin(2 * np.pi * (kk[m, 0] * x / nx + kk[m, 1] * y / ny + kk[m, 2] * z / nz) + ph[m]) for m in range(4)]
        return 1.0 + 0.5 * amp * s[0], np.stack([amp * s[1], amp * s[2], amp * s[3]], 1)

    K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    rc, uc = sample(I.reshape(-1).astype(float), J.reshape(-1).astype(float), K.reshape(-1).astype(float))
    o = RefineOracle(nx, ny, patch, 0.7, lattice=lattice, nz=nz)
    rf, uf = sample(*o.fine_coords())
    return rc, uc, rf, uf


def _run_both3(n3, lattice, patch, tau_c, steps, seed):
    from paper_2601_05936_amd.lsb import Refine
    nx, ny, nz = n3
    rc, uc, rf, uf = _fields3(n3, lattice, patch, seed)
    o = RefineOracle(nx, ny, patch, tau_c, lattice=lattice, nz=nz).init(rc, uc, rf, uf)
    g = Refine(nx, ny, patch, tau_c, lattice=lattice, nz=nz).init(rc, uc, rf, uf)
    o.step(steps)
    g.step(steps)
    return o.populations(), g.populations()


@pytest.mark.parametrize("lattice,n3,patch,tau_c,steps", [
    (1, (20, 18, 16), (5, 12, 4, 13, 6, 11), 0.7, 12),
    (2, (20, 18, 16), (5, 12, 4, 13, 6, 11), 0.62, 12),
    (2, (300, 12, 10), (100, 290, 3, 8, 3, 6), 0.9, 6),  # fine rows of 381 nodes: two blocks, ragged tail
    (2, (9, 8, 8), (2, 4, 2, 4, 3, 5), 0.8, 10),          # the minimal patch
])
def test_refine_3d_matches_oracle(require_gpu, lattice, n3, patch, tau_c, steps):
    (oc, of), (gc, gf) = _run_both3(n3, lattice, patch, tau_c, steps, seed=sum(n3))
    ec, ef = np.max(np.abs(gc - oc)), np.max(np.abs(gf - of))
    print(f"refine D3Q{19 if lattice == 1 else 27} {n3} patch {patch}: coarse {ec:.2e} fine {ef:.2e}", flush=True)
    assert ec <= TOL and ef <= TOL


def test_refine_3d_benchmark_configuration(require_gpu):
    """D3Q27, 192^3 coarse nodes, patch over [48, 144]^3 (193^3 fine nodes),
    the launch configuration of the benchmark's 3D leg, 2 coarse steps."""
    n3, patch = (192, 192, 192), (48, 144, 48, 144, 48, 144)
    (oc, of), (gc, gf) = _run_both3(n3, 2, patch, 0.6, 2, seed=11)
    ec, ef = np.max(np.abs(gc - oc)), np.max(np.abs(gf - of))
    print(f"refine D3Q27 192^3: coarse {ec:.2e} fine {ef:.2e}", flush=True)
    assert ec <= TOL and ef <= TOL


# --- level-set sensor and re-meshing ---

@pytest.mark.parametrize("lattice,n3,patch,max_ext,steps", [
    (0, (64, 56, 1), (20, 30, 18, 28), (50, 50, 0), 6),
    (2, (30, 28, 26), (10, 16, 9, 15, 8, 14), (24, 24, 22), 4),
])
def test_refine_sensor_and_remesh_match_oracle(require_gpu, lattice, n3, patch, max_ext, steps):
    """Steps, the level-set sensor on a gas sphere (box compared with the
    oracle's), re-meshing onto it, more steps, then a shrunk and shifted
    patch; both levels against the oracle after each phase."""
    from paper_2601_05936_amd.lsb import Refine
    nx, ny, nz = n3
    if lattice == 0:
        rc, uc, rf, uf = _fields(nx, ny, patch, seed=5)
        o = RefineOracle(nx, ny, patch, 0.7)
        g = Refine(nx, ny, patch, 0.7, max_extent=max_ext)
        J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        phi = 9.5 - np.hypot(I - 33.2, J - 24.7)
    else:
        rc, uc, rf, uf = _fields3(n3, lattice, patch, seed=6)
        o = RefineOracle(nx, ny, patch, 0.7, lattice=lattice, nz=nz)
        g = Refine(nx, ny, patch, 0.7, lattice=lattice, nz=nz, max_extent=max_ext)
        K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        phi = 5.5 - np.sqrt((I - 14.6) ** 2 + (J - 13.2) ** 2 + (K - 12.9) ** 2)
    o.init(rc, uc, rf, uf)
    g.init(rc, uc, rf, uf)

    def check(label):
        (oc, of), (gc, gf) = o.populations(), g.populations()
        ec, ef = np.max(np.abs(gc - oc)), np.max(np.abs(gf - of))
        print(f"remesh D={g.D} {label}: coarse {ec:.2e} fine {ef:.2e}", flush=True)
        assert gf.shape == of.shape and ec <= TOL and ef <= TOL

    o.step(steps)
    g.step(steps)
    check("before")
    box = g.sensor(phi.reshape(-1), 2.0, 1)
    assert box == o.sensor(phi.reshape(-1), 2.0, 1)
    assert box[:4] != tuple(patch[:4])
    o.remesh(box)
    g.remesh(box)
    check("re-meshed")
    o.step(steps)
    g.step(steps)
    check("after")
    small = tuple(v + (1 if d % 2 == 0 else -2) for d, v in enumerate(box[:2 * g.D]))
    o.remesh(small)
    g.remesh(small)
    o.step(steps)
    g.step(steps)
    check("shrunk")


def test_refine_remesh_rejects_patches_beyond_the_workspace(require_gpu):
    from paper_2601_05936_amd.lsb import LsbError, Refine
    g = Refine(40, 40, (10, 20, 10, 20), 0.7, max_extent=(14, 14, 0))
    g.init(np.ones(g.n_coarse), np.zeros(2 * g.n_coarse), np.ones(g.n_fine), np.zeros(2 * g.n_fine))
    with pytest.raises(LsbError):
        g.remesh((5, 20, 10, 20))      # 15 cells in x > 14
    g.remesh((6, 20, 10, 24))          # 14 x 14 fits


# --- nested levels ---

def _fields_nested(o, seed, amp=0.02):
    """Smooth random density and velocity sampled on every level of oracle o."""
    rng = np.random.default_rng(seed)
    n = np.array([o.nx, o.ny, o.nz], dtype=float)
    kk = rng.integers(1, 3, (4, 3))
    ph = rng.uniform(0, 2 * np.pi, 4)
    args = []
    for lv in range(o.levels):
        xyz = list(o.coords(lv)) + [0.0] * (3 - o.D)
        s = [np.sin(2 * np.pi * sum(kk[m, d] * xyz[d] / n[d] for d in range(3)) + ph[m]) for m in range(4)]
        u = np.stack([amp * s[1], amp * s[2], amp * s[3]][:o.D], 1)
        args += [1.0 + 0.5 * amp * s[0], u]
    return args


def _run_nested(lattice, n3, boxes, tau_c, steps, seed):
    from paper_2601_05936_amd.lsb import Refine
    nx, ny, nz = n3
    o = RefineOracle(nx, ny, boxes, tau_c, lattice=lattice, nz=nz)
    args = _fields_nested(o, seed)
    g = Refine(nx, ny, boxes, tau_c, lattice=lattice, nz=nz)
    o.init(*args)
    g.init(*args)
    o.step(steps)
    g.step(steps)
    return o.populations(), g.populations()


@pytest.mark.parametrize("lattice,n3,boxes,tau_c,steps", [
    (0, (40, 36, 1), [(8, 30, 7, 28), (3, 40, 4, 38)], 0.7, 10),
    (0, (300, 30, 1), [(50, 250, 4, 25), (10, 390, 3, 40)], 0.62, 4),   # level-2 rows of 761 nodes
    (0, (30, 30, 1), [(6, 22, 5, 21), (3, 27, 4, 30), (2, 44, 3, 50)], 0.8, 6),   # four levels
    (0, (12, 12, 1), [(3, 6, 2, 5), (1, 3, 1, 3)], 0.9, 8),             # minimal inner patch
    (1, (14, 14, 14), [(3, 10, 4, 11, 2, 9), (2, 12, 1, 12, 3, 11)], 0.7, 6),
    (2, (20, 18, 16), [(5, 12, 4, 13, 6, 11), (2, 12, 3, 15, 1, 9)], 0.62, 4),
    (2, (10, 10, 10), [(2, 6, 2, 6, 2, 6), (2, 5, 2, 6, 1, 4), (1, 4, 2, 5, 1, 4)], 0.75, 3),  # four levels
])
def test_nested_matches_oracle(require_gpu, lattice, n3, boxes, tau_c, steps):
    ref, got = _run_nested(lattice, n3, boxes, tau_c, steps, seed=sum(n3) + len(boxes))
    errs = [float(np.max(np.abs(g - o))) for o, g in zip(ref, got)]
    print(f"nested D={2 if lattice == 0 else 3} Q{ref[0].shape[0]} {n3} {len(boxes) + 1} levels: "
          + " ".join(f"{e:.2e}" for e in errs), flush=True)
    assert all(g.shape == o.shape for o, g in zip(ref, got))
    assert max(errs) <= TOL


def test_nested_benchmark_configuration(require_gpu):
    """2048^2 coarse nodes, level 1 over [512, 1536]^2, level 2 over level-1
    nodes [512, 1536]^2 (2049^2 nodes each), the launch configuration of the
    benchmark's three-level leg, 2 coarse steps."""
    ref, got = _run_nested(0, (2048, 2048, 1), [(512, 1536, 512, 1536)] * 2, 0.6, 2, seed=3)
    errs = [float(np.max(np.abs(g - o))) for o, g in zip(ref, got)]
    print("nested 2048^2 three levels: " + " ".join(f"{e:.2e}" for e in errs), flush=True)
    assert max(errs) <= TOL


def test_nested_uniform_state_is_fixed(require_gpu):
    from paper_2601_05936_amd.lsb import Refine
    boxes = [(5, 12, 4, 13, 6, 11), (2, 12, 3, 15, 1, 9)]
    g = Refine(20, 18, boxes, 0.7, lattice=2, nz=16)
    u = np.array([0.04, -0.03, 0.02])
    args = []
    for lv in range(3):
        args += [np.full(g.n_level(lv), 1.02), np.tile(u, g.n_level(lv))]
    g.init(*args)
    f0 = g.populations()
    g.step(3)
    for a, b in zip(g.populations(), f0):
        assert np.max(np.abs(a - b)) < 1e-15


def test_nested_rejects_two_level_calls(require_gpu):
    from paper_2601_05936_amd.lsb import LsbError, Refine
    g = Refine(30, 30, [(6, 22, 5, 21), (3, 27, 4, 30)], 0.7)
    with pytest.raises(LsbError):
        g.remesh((5, 20, 5, 20))   # before init: state error
    args = []
    for lv in range(3):
        args += [np.ones(g.n_level(lv)), np.zeros(2 * g.n_level(lv))]
    g.init(*args)
    with pytest.raises(LsbError):
        g.remesh((5, 20, 5, 20))   # re-meshing takes two levels


@pytest.mark.parametrize("lattice,n3,boxes,max_ext,max_inner,margins", [
    (0, (64, 56, 1), [(20, 30, 18, 28), (4, 16, 5, 15)], (40, 40, 0), [(60, 60, 0)], (3, 1)),
    (2, (30, 28, 26), [(10, 16, 9, 15, 8, 14), (2, 10, 3, 9, 2, 10)], (24, 24, 22), [(40, 40, 40)], (2, 1)),
])
def test_nested_sensor_and_remesh_match_oracle(require_gpu, lattice, n3, boxes, max_ext, max_inner, margins):
    """Three levels: steps, the sensor's boxes on a gas disk/sphere against
    the oracle's, re-meshing every level onto them, steps, then onto the
    boxes of a narrower band (smaller d_ref), steps; every level against the
    oracle after each phase."""
    from paper_2601_05936_amd.lsb import Refine
    nx, ny, nz = n3
    o = RefineOracle(nx, ny, boxes, 0.7, lattice=lattice, nz=nz)
    args = _fields_nested(o, seed=9)
    g = Refine(nx, ny, boxes, 0.7, lattice=lattice, nz=nz, max_extent=max_ext, max_inner_extent=max_inner)
    o.init(*args)
    g.init(*args)
    if lattice == 0:
        J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        phi = 9.5 - np.hypot(I - 33.2, J - 24.7)
    else:
        K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        phi = 5.5 - np.sqrt((I - 14.6) ** 2 + (J - 13.2) ** 2 + (K - 12.9) ** 2)

    def check(label):
        errs = [float(np.max(np.abs(b - a))) for a, b in zip(o.populations(), g.populations())]
        print(f"nested remesh D={g.D} {label}: " + " ".join(f"{e:.2e}" for e in errs), flush=True)
        assert max(errs) <= TOL

    o.step(4)
    g.step(4)
    check("before")
    for d_ref in (2.0, 0.5):
        got = g.sensor_levels(phi.reshape(-1), d_ref, margins)
        want = o.sensor_levels(phi.reshape(-1), d_ref, margins)
        assert got == want, (got, want)
        o.remesh_levels(want)
        g.remesh_levels(got)
        check(f"re-meshed (d_ref {d_ref})")
        o.step(3)
        g.step(3)
        check(f"after (d_ref {d_ref})")


def test_nested_remesh_rejects_boxes_beyond_the_workspace(require_gpu):
    from paper_2601_05936_amd.lsb import LsbError, Refine
    boxes = [(10, 20, 10, 20), (4, 12, 4, 12)]
    g = Refine(40, 40, boxes, 0.7, max_extent=(14, 14, 0), max_inner_extent=[(10, 10, 0)])
    args = []
    for lv in range(3):
        args += [np.ones(g.n_level(lv)), np.zeros(2 * g.n_level(lv))]
    g.init(*args)
    with pytest.raises(LsbError):
        g.remesh_levels([(10, 20, 10, 20), (4, 15, 4, 12)])   # 11 cells > 10
    with pytest.raises(LsbError):
        g.remesh_levels([(10, 20, 10, 20), (4, 20, 4, 12)])   # beyond level 1's last node - 1
    g.remesh_levels([(6, 20, 10, 24), (2, 12, 16, 26)])      # fits
    assert g.boxes[1][:4] == (2, 12, 16, 26)


# --- trees: several boxes refining one grid ---

@pytest.mark.parametrize("lattice,n3,boxes,parents,tau_c,steps", [
    (0, (48, 40, 1), [(4, 16, 6, 30), (18, 40, 4, 20), (3, 20, 5, 40)], [0, 0, 1], 0.7, 8),
    (0, (48, 48, 1), [(5, 19, 8, 40), (28, 42, 8, 40), (4, 20, 6, 50), (8, 24, 6, 50)], [0, 0, 1, 2], 0.7, 6),
    (0, (400, 30, 1), [(10, 150, 4, 25), (160, 390, 3, 20), (20, 270, 3, 30), (30, 440, 4, 28)], [0, 0, 1, 2], 0.62, 3),
    (2, (24, 20, 18), [(3, 9, 4, 14, 3, 12), (11, 20, 3, 10, 4, 13), (2, 10, 3, 12, 2, 14)], [0, 0, 2], 0.7, 3),
    (1, (16, 16, 16), [(2, 6, 3, 12, 2, 13), (8, 13, 2, 9, 4, 10)], [0, 0], 0.8, 4),
])
def test_tree_matches_oracle(require_gpu, lattice, n3, boxes, parents, tau_c, steps):
    from paper_2601_05936_amd.lsb import Refine
    nx, ny, nz = n3
    o = RefineOracle(nx, ny, boxes, tau_c, lattice=lattice, nz=nz, parents=parents)
    args = _fields_nested(o, seed=sum(n3) + 3 * len(boxes))
    g = Refine(nx, ny, boxes, tau_c, lattice=lattice, nz=nz, parents=parents)
    o.init(*args)
    g.init(*args)
    o.step(steps)
    g.step(steps)
    errs = [float(np.max(np.abs(b - a))) for a, b in zip(o.populations(), g.populations())]
    print(f"tree D={2 if lattice == 0 else 3} {n3} parents {parents}: " + " ".join(f"{e:.2e}" for e in errs), flush=True)
    assert max(errs) <= TOL


def test_tree_benchmark_configuration(require_gpu):
    """The benchmark's tree leg: 2048^2 coarse nodes, nine 200^2-cell boxes
    on a 3 x 3 lattice (401^2 nodes each), stepped from the captured graphs
    with the boxes on parallel branches; 2 coarse steps against the oracle."""
    from paper_2601_05936_amd.lsb import Refine
    n = 2048
    boxes = [(224 + 600 * a, 424 + 600 * a, 224 + 600 * b, 424 + 600 * b) for b in range(3) for a in range(3)]
    o = RefineOracle(n, n, boxes, 0.6, parents=[0] * 9)
    args = _fields_nested(o, seed=41)
    g = Refine(n, n, boxes, 0.6, parents=[0] * 9)
    o.init(*args)
    g.init(*args)
    o.step(2)
    g.step(2)
    errs = [float(np.max(np.abs(b - a))) for a, b in zip(o.populations(), g.populations())]
    print("tree 2048^2 nine boxes: " + " ".join(f"{e:.2e}" for e in errs), flush=True)
    assert max(errs) <= TOL


def test_tree_refuses_the_sensor(require_gpu):
    from paper_2601_05936_amd.lsb import LsbError, Refine
    g = Refine(48, 40, [(4, 16, 6, 30), (18, 40, 4, 20)], 0.7, parents=[0, 0])
    args = []
    for lv in range(3):
        args += [np.ones(g.n_level(lv)), np.zeros(2 * g.n_level(lv))]
    g.init(*args)
    with pytest.raises(LsbError):
        g.sensor_levels(np.zeros(48 * 40), 1.0, (1, 1))
    with pytest.raises(LsbError):   # siblings one node too close
        g.remesh_levels([(4, 17, 6, 30), (18, 40, 4, 20)])


@pytest.mark.parametrize("lattice,n3,boxes,parents,new", [
    (0, (40, 40, 1), [(4, 16, 6, 30), (20, 34, 4, 20), (3, 20, 5, 40)], [0, 0, 1],
     [(5, 16, 4, 28), (20, 34, 6, 22), (2, 19, 8, 42)]),
    (2, (24, 20, 18), [(3, 9, 4, 14, 3, 12), (11, 20, 3, 10, 4, 13), (2, 10, 3, 12, 2, 14)], [0, 0, 2],
     [(2, 9, 5, 14, 3, 11), (11, 19, 4, 11, 4, 12), (3, 11, 3, 11, 2, 14)]),
])
def test_tree_remesh_matches_oracle(require_gpu, lattice, n3, boxes, parents, new):
    """Steps, a re-mesh of every box of a tree (boxes no larger than before:
    a tree's workspace holds its initial boxes), steps; every grid against
    the oracle after each phase."""
    from paper_2601_05936_amd.lsb import Refine
    nx, ny, nz = n3
    o = RefineOracle(nx, ny, boxes, 0.7, lattice=lattice, nz=nz, parents=parents)
    args = _fields_nested(o, seed=33)
    g = Refine(nx, ny, boxes, 0.7, lattice=lattice, nz=nz, parents=parents,
               max_extent=(14, 14, 10) if lattice else (14, 26, 0))
    o.init(*args)
    g.init(*args)
    for phase in ("before", "re-meshed", "after"):
        if phase == "re-meshed":
            o.remesh_levels(new)
            g.remesh_levels(new)
        else:
            o.step(3)
            g.step(3)
        errs = [float(np.max(np.abs(b - a))) for a, b in zip(o.populations(), g.populations())]
        print(f"tree remesh D={g.D} {phase}: " + " ".join(f"{e:.2e}" for e in errs), flush=True)
        assert max(errs) <= TOL


@pytest.mark.parametrize("kind", ["tree", "chain"])
def test_graph_steps_match_plain_launches(require_gpu, kind):
    """Coarse steps replayed from the two captured graphs against plain
    launches, bit for bit, one step per call with a read-back (and so a
    synchronisation) between replays, across a re-mesh that rebuilds the
    graphs (chain) and against the oracle at the end."""
    from paper_2601_05936_amd.lsb import Refine
    if kind == "tree":
        n3, boxes, parents, kw = (48, 40, 1), [(4, 16, 6, 30), (18, 40, 4, 20), (3, 20, 5, 40)], [0, 0, 1], {}
    else:
        n3, boxes, parents = (40, 36, 1), [(8, 30, 7, 28), (3, 40, 4, 38)], None
        kw = dict(max_extent=(30, 30, 0), max_inner_extent=[(50, 50, 0)])
    nx, ny, nz = n3
    o = RefineOracle(nx, ny, boxes, 0.7, parents=parents)
    args = _fields_nested(o, seed=21)
    o.init(*args)
    gr = Refine(nx, ny, boxes, 0.7, parents=parents, **kw).init(*args)
    pl = Refine(nx, ny, boxes, 0.7, parents=parents, **kw).set_graphs(False).init(*args)
    for s in range(5):
        o.step(1)
        gr.step(1)
        pl.step(1)
        for a, b in zip(gr.populations(), pl.populations()):
            assert np.array_equal(a, b), s
        if kind == "chain" and s == 2:
            new = [(6, 31, 5, 29), (4, 44, 6, 40)]
            o.remesh_levels(new)
            gr.remesh_levels(new)
            pl.remesh_levels(new)
    errs = [float(np.max(np.abs(b - a))) for a, b in zip(o.populations(), gr.populations())]
    print(f"graph steps {kind}: " + " ".join(f"{e:.2e}" for e in errs), flush=True)
    assert max(errs) <= TOL


@pytest.mark.parametrize("lattice", [0, 2])
def test_seeded_sensor_matches_oracle_and_drives_a_tree(require_gpu, lattice):
    """The seeded sensor's boxes against the oracle's (gas disks/spheres,
    one seed each, plus a seed with no tagged node), a tree built on them,
    steps, a second sensor call with the gas moved and a re-mesh of the tree
    onto its boxes, steps; every grid against the oracle."""
    from paper_2601_05936_amd.lsb import Refine
    if lattice == 0:
        n3 = (96, 96, 1)
        J, I = np.meshgrid(np.arange(96), np.arange(96), indexing="ij")
        K = 0 * I
        blobs = [(20.3, 24.6, 0, 6.5), (70.2, 30.1, 0, 8.2), (45.5, 75.4, 0, 5.1)]
        seeds = [(20, 25, 0), (70, 30, 0), (45, 75, 0), (90, 5, 0)]
    else:
        n3 = (40, 36, 32)
        K, J, I = np.meshgrid(np.arange(32), np.arange(36), np.arange(40), indexing="ij")
        blobs = [(11.2, 12.7, 15.1, 4.2), (27.6, 22.3, 14.4, 4.8)]
        seeds = [(11, 13, 15), (28, 22, 14)]
    nx, ny, nz = n3

    def gas(shift):
        return np.max([r - np.sqrt((I - x - shift) ** 2 + (J - y) ** 2 + (K - z) ** 2) for x, y, z, r in blobs],
                      axis=0).reshape(-1)
    # a one-box tree holds the coarse grid for the sensor calls
    probe_o = RefineOracle(nx, ny, [(2, 6, 2, 6, 2, 6)], 0.7, lattice=lattice, nz=nz)
    probe_g = Refine(nx, ny, [(2, 6, 2, 6, 2, 6)], 0.7, lattice=lattice, nz=nz)
    want = probe_o.sensor_seeded(gas(0.0), 1.5, 2, seeds)
    got = probe_g.sensor_seeded(gas(0.0), 1.5, 2, seeds)
    assert got == want and len(got) == len(blobs), (got, want)
    parents = [0] * len(got)
    o = RefineOracle(nx, ny, got, 0.7, lattice=lattice, nz=nz, parents=parents)
    args = _fields_nested(o, seed=51)
    g = Refine(nx, ny, got, 0.7, lattice=lattice, nz=nz, parents=parents)
    o.init(*args)
    g.init(*args)
    o.step(3)
    g.step(3)
    moved_o = o.sensor_seeded(gas(-1.0), 1.0, 1, seeds)       # smaller boxes: within the tree's workspace
    moved_g = g.sensor_seeded(gas(-1.0), 1.0, 1, seeds)
    assert moved_g == moved_o and len(moved_g) == len(got)
    o.remesh_levels(moved_o)
    g.remesh_levels(moved_g)
    o.step(3)
    g.step(3)
    errs = [float(np.max(np.abs(b - a))) for a, b in zip(o.populations(), g.populations())]
    print(f"seeded sensor D={g.D}: boxes {got} -> {moved_g}; " + " ".join(f"{e:.2e}" for e in errs), flush=True)
    assert max(errs) <= TOL
