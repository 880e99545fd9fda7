"""The C-ABI library loads and exports every entry point include/*.h
declares; parameter validation and the workspace layout need no GPU."""
import ctypes as C
import os
import re

import pytest

from paper_2601_05936_amd import lsb, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsb.h")


def declared_symbols():
    inc = os.path.join(ROOT, "include")
    text = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    return sorted(set(re.findall(r"\b(lsb_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = lsb.load()
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(lsb.EXPORTS)


def test_params_struct_matches_header_field_order():
    text = open(HEADER).read()
    body = text[text.index("typedef struct lsb_params"):text.index("} lsb_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"\b([a-z_0-9]+)(?:\[[0-9]+\])*\s*[;,]", body)
    assert [n for n in names if n != "int"] == [f for f, _ in lsb.Params._fields_]


def _create(p):
    lib = lsb.load()
    h = C.c_void_p()
    rc = lib.lsb_create(C.byref(lsb.to_params(p)), C.byref(h))
    return rc, h


@pytest.mark.parametrize("bad", [
    dict(lattice=7), dict(storage=9), dict(nz=3),  # D2Q9 with nz != 1
    dict(tau=[0.5, 0.8]), dict(band=1.0), dict(bc=[0, 1, 0, 0, 0, 0]), dict(nx=2),
    dict(collision=[W.BGK, W.CUMULANT]),  # cumulant needs D3Q27
    dict(collision=[2, W.BGK]),  # unknown operator
    dict(use_pb=3),  # unknown baseline mode
])
def test_create_rejects_invalid_parameters(bad):
    p = W.default_params(lattice=W.D2Q9, nx=16, ny=16, nz=1,
                         bc=[W.PERIODIC] * 6)
    p.update(bad)
    rc, h = _create(p)
    assert rc == lsb.LSB_EINVAL
    assert lsb.load().lsb_last_error().decode()


@pytest.mark.parametrize("lat,storage,shape,pop_bytes", [
    (W.D2Q9, W.F64, (64, 32, 1), 8), (W.D3Q19, W.F32, (20, 18, 22), 4), (W.D3Q27, W.F16DEV, (16, 16, 16), 2),
])
def test_workspace_layout_and_state_image(lat, storage, shape, pop_bytes):
    nx, ny, nz = shape
    p = W.default_params(lattice=lat, storage=storage, nx=nx, ny=ny, nz=nz)
    rc, h = _create(p)
    assert rc == 0
    lib = lsb.load()
    nb = C.c_size_t()
    assert lib.lsb_workspace_bytes(h, C.byref(nb)) == 0
    N = nx * ny * nz
    Q = {W.D2Q9: 9, W.D3Q19: 19, W.D3Q27: 27}[lat]
    assert nb.value >= 2 * Q * N * pop_bytes
    sb = C.c_size_t()
    assert lib.lsb_state_bytes(h, C.byref(sb)) == 0
    assert sb.value >= Q * N * pop_bytes
    # binding a too small buffer is refused before any device access
    assert lib.lsb_bind(h, C.c_void_p(256), 16) == lsb.LSB_ENOMEM
    # stepping before init is a state error
    assert lib.lsb_step(h, 1, 0, None) == lsb.LSB_ESTATE
    lib.lsb_destroy(h)


def test_schedule_selection_is_validated():
    p = W.default_params(lattice=W.D3Q19, nx=16, ny=16, nz=16)
    rc, h = _create(p)
    assert rc == 0
    lib = lsb.load()
    assert lib.lsb_set_schedule(h, lsb.SCHED_OVERLAP) == lsb.LSB_OK
    assert lib.lsb_set_schedule(h, lsb.SCHED_SERIAL) == lsb.LSB_OK
    assert lib.lsb_set_schedule(h, 7) == lsb.LSB_EINVAL
    assert lib.lsb_set_schedule(None, 0) == lsb.LSB_EINVAL
    lib.lsb_destroy(h)


def test_static_integrals_validate_before_device_access():
    """The no-allocation integrals entry point refuses NULL arguments and a
    plan without state before touching the device."""
    p = W.default_params(lattice=W.D2Q9, nx=16, ny=16, nz=1)
    rc, h = _create(p)
    assert rc == 0
    lib = lsb.load()
    assert lib.lsb_get_integrals_static(None, C.c_void_p(1 << 20), None) == lsb.LSB_EINVAL
    assert lib.lsb_get_integrals_static(h, None, None) == lsb.LSB_EINVAL
    assert lib.lsb_get_integrals_static(h, C.c_void_p(1 << 20), None) == lsb.LSB_ESTATE
    lib.lsb_destroy(h)


def test_reverse_mode_rejects_per_bubble_baselines():
    """The reverse mode differentiates one gas baseline (use_pb 0 or 1)."""
    lib = lsb.load()
    for mode, want in ((1, lsb.LSB_OK), (2, lsb.LSB_EINVAL)):
        p = W.default_params(lattice=W.D2Q9, nx=16, ny=16, nz=1, bc=[W.PERIODIC] * 6, use_pb=mode)
        rc, h = _create(p)
        assert rc == 0
        nb = C.c_size_t()
        assert lib.lsb_adjoint_workspace_bytes(h, 10, C.byref(nb)) == want
        lib.lsb_destroy(h)


def _pitch(mx):
    """Row pitch of a refined level: node 0 at column 16, rounded up to 16."""
    return (mx + 18 + 15) // 16 * 16


def _ref_create(**kw):
    p = dict(lattice=lsb.D2Q9, nx=32, ny=24, nz=1, patch=(8, 20, 6, 16, 0, 0), tau_c=0.7)
    p.update(kw)
    inner = ((C.c_int * 6) * (lsb.REF_MAX_LEVELS - 2))()
    for l, bx in enumerate(p.get("inner", ())):
        inner[l] = (C.c_int * 6)(*bx)
    mie = ((C.c_int * 3) * (lsb.REF_MAX_LEVELS - 2))()
    for l, e in enumerate(p.get("max_inner_extent", ())):
        mie[l] = (C.c_int * 3)(*e)
    cp = lsb.RefParams(p["lattice"], p["nx"], p["ny"], p["nz"], (C.c_int * 6)(*p["patch"]), p["tau_c"],
                       (C.c_int * 3)(*p.get("max_extent", (0, 0, 0))), p.get("levels", 0), inner, mie)
    h = C.c_void_p()
    rc = lsb.load().lsb_ref_create(C.byref(cp), C.byref(h))
    return rc, h


@pytest.mark.parametrize("bad", [
    dict(lattice=5), dict(nx=3), dict(nz=2),                                   # 2D needs nz = 1
    dict(patch=(0, 20, 6, 16, 0, 0)), dict(patch=(8, 31, 6, 16, 0, 0)),        # no spare node at the edge
    dict(patch=(8, 9, 6, 16, 0, 0)),                                            # fewer than 2 cells
    dict(tau_c=0.5),
    dict(lattice=lsb.D3Q27, nz=16, patch=(8, 20, 6, 16, 0, 9)),                 # 3D: ka < 1
    dict(lattice=lsb.D3Q19, nz=3, patch=(8, 20, 6, 16, 1, 2)),                  # 3D: nz < 4
    dict(max_extent=(30, 0, 0)),                                                # beyond n - 3
    dict(levels=1), dict(levels=5),
    dict(levels=3, inner=[(0, 10, 2, 12, 0, 0)]),                               # level 2 touches level 1's edge
    dict(levels=3, inner=[(2, 24, 2, 12, 0, 0)]),                               # level 1 has nodes 0 .. 24
    dict(levels=3, inner=[(2, 3, 2, 12, 0, 0)]),                                # fewer than 2 cells
    dict(levels=4, inner=[(2, 20, 2, 12, 0, 0), (1, 36, 3, 9, 0, 0)]),         # level 2 has nodes 0 .. 36
    dict(lattice=lsb.D3Q19, nz=16, patch=(8, 20, 6, 16, 4, 12), levels=3,
         inner=[(2, 20, 2, 12, 3, 16)]),                                        # 3D: kb > m - 1
    dict(levels=3, inner=[(2, 20, 2, 12, 0, 0)], max_inner_extent=[(23, 0, 0)]),  # > 2 x 12 - 2
    dict(levels=3, inner=[(2, 20, 2, 12, 0, 0)], max_inner_extent=[(0, -1, 0)]),
])
def test_refine_create_rejects_invalid_parameters(bad):
    rc, h = _ref_create(**bad)
    assert rc == lsb.LSB_EINVAL
    assert lsb.load().lsb_last_error().decode()


def test_refine_workspace_layout():
    """Workspace = 2 x (coarse + fine with a one-node ghost shell + the box
    surface), Q doubles per node, each part aligned to 256 bytes, sized for
    the largest patch, plus the sensor's partial boxes.  Fine rows start
    node 0 at column 16 of a pitch rounded up to 16 doubles."""
    def up(v):
        return (v + 255) // 256 * 256
    lib = lsb.load()
    for lat, Q, n3, patch in [(lsb.D2Q9, 9, (32, 24, 1), (8, 20, 6, 16, 0, 0)),
                              (lsb.D3Q27, 27, (20, 18, 16), (5, 12, 4, 13, 6, 11))]:
        rc, h = _ref_create(lattice=lat, nx=n3[0], ny=n3[1], nz=n3[2], patch=patch)
        assert rc == lsb.LSB_OK
        nb = C.c_size_t()
        assert lib.lsb_ref_workspace_bytes(h, C.byref(nb)) == lsb.LSB_OK
        ia, ib, ja, jb, ka, kb = patch
        mx, my, mz = 2 * (ib - ia), 2 * (jb - ja), 2 * (kb - ka)
        nc = n3[0] * n3[1] * n3[2]
        if lat == lsb.D2Q9:
            nf = _pitch(mx) * (my + 3)
            ns = 2 * (jb - ja + 1) + 2 * (ib - ia + 1)
        else:
            bw, bh, bd = ib - ia + 1, jb - ja + 1, kb - ka + 1
            nf = _pitch(mx) * (my + 3) * (mz + 3)
            ns = 2 * bh * bd + 2 * bw * bd + 2 * bw * bh
        assert nb.value == 2 * (up(8 * Q * nc) + up(8 * Q * nf) + up(8 * Q * ns)) + up(4 * 6 * 15 * 1025)
        assert lib.lsb_ref_bind(h, C.c_void_p(1 << 20), nb.value - 1) == lsb.LSB_ENOMEM
        lib.lsb_ref_destroy(h)


def test_refine_nested_workspace_layout():
    """Nested levels append, per deeper level, 2 x (its nodes with the ghost
    shell + its box surface) to the two-level layout."""
    def up(v):
        return (v + 255) // 256 * 256
    lib = lsb.load()
    base = dict(lattice=lsb.D3Q27, nx=20, ny=18, nz=16, patch=(5, 12, 4, 13, 6, 11))
    rc, h2 = _ref_create(**base)
    assert rc == lsb.LSB_OK
    n2 = C.c_size_t()
    assert lib.lsb_ref_workspace_bytes(h2, C.byref(n2)) == lsb.LSB_OK
    boxes = [(2, 12, 3, 15, 1, 9), (4, 18, 2, 20, 3, 14)]
    rc, h = _ref_create(levels=4, inner=boxes, **base)
    assert rc == lsb.LSB_OK, lib.lsb_last_error()
    nb = C.c_size_t()
    assert lib.lsb_ref_workspace_bytes(h, C.byref(nb)) == lsb.LSB_OK
    extra = 0
    for ia, ib, ja, jb, ka, kb in boxes:
        mx, my, mz = 2 * (ib - ia), 2 * (jb - ja), 2 * (kb - ka)
        bw, bh, bd = ib - ia + 1, jb - ja + 1, kb - ka + 1
        nf = _pitch(mx) * (my + 3) * (mz + 3)
        ns = 2 * bh * bd + 2 * bw * bd + 2 * bw * bh
        extra += 2 * (up(8 * 27 * nf) + up(8 * 27 * ns))
    assert nb.value == n2.value + extra
    # max_inner_extent sizes a deeper level for its largest box
    rc, h3 = _ref_create(levels=3, inner=boxes[:1], max_inner_extent=[(12, 14, 8)], **base)
    assert rc == lsb.LSB_OK
    n3 = C.c_size_t()
    assert lib.lsb_ref_workspace_bytes(h3, C.byref(n3)) == lsb.LSB_OK
    e = (12, 14, 8)
    nf = _pitch(2 * e[0]) * (2 * e[1] + 3) * (2 * e[2] + 3)
    ns = 2 * (e[1] + 1) * (e[2] + 1) + 2 * (e[0] + 1) * (e[2] + 1) + 2 * (e[0] + 1) * (e[1] + 1)
    assert n3.value == n2.value + 2 * (up(8 * 27 * nf) + up(8 * 27 * ns))
    lib.lsb_ref_destroy(h3)
    # two-level entry points refuse the deeper hierarchy before any device access
    dummy = C.c_void_p(1)
    assert lib.lsb_ref_init(h, dummy, dummy, dummy, dummy, None) == lsb.LSB_EINVAL
    assert "lsb_ref_init_levels" in lib.lsb_last_error().decode()
    assert lib.lsb_ref_get_level(h, 4, C.c_void_p(1), None) == lsb.LSB_EINVAL
    assert lib.lsb_ref_get_level(h, 3, C.c_void_p(1), None) == lsb.LSB_ESTATE
    lib.lsb_ref_destroy(h)
    lib.lsb_ref_destroy(h2)


def _tree_create(parents, boxes, **kw):
    p = dict(lattice=lsb.D2Q9, nx=48, ny=40, nz=1, tau_c=0.7)
    p.update(kw)
    cp = lsb.RefParams(p["lattice"], p["nx"], p["ny"], p["nz"], (C.c_int * 6)(), p["tau_c"], (C.c_int * 3)(), 0,
                       ((C.c_int * 6) * (lsb.REF_MAX_LEVELS - 2))(), ((C.c_int * 3) * (lsb.REF_MAX_LEVELS - 2))())
    flat = [v for bx in boxes for v in bx]
    h = C.c_void_p()
    rc = lsb.load().lsb_ref_create_tree(C.byref(cp), len(boxes), (C.c_int * len(parents))(*parents),
                                        (C.c_int * len(flat))(*flat), C.byref(h))
    return rc, h


_SIB = [(4, 16, 6, 30, 0, 0), (18, 40, 4, 20, 0, 0), (3, 20, 5, 40, 0, 0)]


@pytest.mark.parametrize("parents,boxes", [
    ([1, 0, 1], _SIB),                                              # box 1 must refine the coarse grid
    ([0, 2, 1], _SIB),                                              # a parent must come first
    ([0, 0, 1], [_SIB[0], (17, 40, 4, 20, 0, 0), _SIB[2]]),         # siblings without a node between
    ([0, 0, 1], [_SIB[0], _SIB[1], (3, 24, 5, 40, 0, 0)]),          # box 3 beyond box 1's last node - 1
    ([0] * 16, [(1, 3, 2, 8, 0, 0)] * 16),                          # more than 15 boxes
])
def test_refine_tree_rejects_invalid_trees(parents, boxes):
    rc, h = _tree_create(parents, boxes)
    assert rc == lsb.LSB_EINVAL
    assert lsb.load().lsb_last_error().decode()


def test_refine_tree_layout_and_chain_only_calls():
    """A tree's workspace is the two-level layout of box 1 plus, per further
    box, 2 x (its nodes with the ghost shell + its box surface); the sensor
    and re-meshing refuse trees before any device access."""
    def up(v):
        return (v + 255) // 256 * 256
    lib = lsb.load()
    rc, h = _tree_create([0, 0, 1], _SIB)
    assert rc == lsb.LSB_OK, lib.lsb_last_error()
    rc2, h2 = _ref_create(nx=48, ny=40, patch=_SIB[0])
    assert rc2 == lsb.LSB_OK
    nb, nb2 = C.c_size_t(), C.c_size_t()
    assert lib.lsb_ref_workspace_bytes(h, C.byref(nb)) == lsb.LSB_OK
    assert lib.lsb_ref_workspace_bytes(h2, C.byref(nb2)) == lsb.LSB_OK
    extra = 0
    for ia, ib, ja, jb, _, _ in _SIB[1:]:
        mx, my = 2 * (ib - ia), 2 * (jb - ja)
        extra += 2 * (up(8 * 9 * _pitch(mx) * (my + 3)) + up(8 * 9 * (2 * (jb - ja + 1) + 2 * (ib - ia + 1))))
    assert nb.value == nb2.value + extra
    assert lib.lsb_ref_bind(h, C.c_void_p(1 << 20), nb.value) == lsb.LSB_OK   # stores the pointer only
    out = (C.c_int * 18)()
    assert lib.lsb_ref_sensor_levels(h, C.c_void_p(1), 0.5, (C.c_int * 3)(1, 1, 1), out, None) == lsb.LSB_EINVAL
    assert "tree" in lib.lsb_last_error().decode()
    lib.lsb_ref_destroy(h)
    lib.lsb_ref_destroy(h2)


def test_refine_seeded_sensor_validates_before_device_access():
    lib = lsb.load()
    rc, h = _tree_create([0, 0, 1], _SIB)
    assert rc == lsb.LSB_OK
    out, nb = (C.c_int * 96)(), C.c_int()
    seeds = (C.c_int * 48)()
    assert lib.lsb_ref_sensor_seeded(h, C.c_void_p(1), 0.5, 1, 2, seeds, out, C.byref(nb), None) == lsb.LSB_ESTATE
    nbytes = C.c_size_t()
    assert lib.lsb_ref_workspace_bytes(h, C.byref(nbytes)) == lsb.LSB_OK
    assert lib.lsb_ref_bind(h, C.c_void_p(1 << 20), nbytes.value) == lsb.LSB_OK
    for ns, margin in [(0, 1), (16, 1), (2, -1)]:
        assert lib.lsb_ref_sensor_seeded(h, C.c_void_p(1), 0.5, margin, ns, seeds, out, C.byref(nb), None) == lsb.LSB_EINVAL
    assert lib.lsb_ref_sensor_seeded(h, None, 0.5, 1, 2, seeds, out, C.byref(nb), None) == lsb.LSB_EINVAL
    lib.lsb_ref_destroy(h)


def test_refine_remesh_levels_checks_the_box_count_first():
    """Re-meshing takes exactly one box per refined grid: a seeded sensor
    result with merged boxes (fewer than the tree has) is refused before any
    device access, and so is a longer list."""
    lib = lsb.load()
    rc, h = _tree_create([0, 0, 1], _SIB)
    assert rc == lsb.LSB_OK
    flat = [v for bx in _SIB for v in bx]
    arr = (C.c_int * len(flat))(*flat)
    for n in (0, 1, 2, 4):
        assert lib.lsb_ref_remesh_levels(h, arr, n, None) == lsb.LSB_EINVAL
        assert "number of boxes" in lib.lsb_last_error().decode()
    assert lib.lsb_ref_remesh_levels(h, arr, 3, None) == lsb.LSB_ESTATE   # right count, not initialised
    g = lsb.Refine.__new__(lsb.Refine)
    g.levels = 4
    with pytest.raises(ValueError, match="rebuilding"):
        lsb.Refine.remesh_levels(g, _SIB[:2])
    lib.lsb_ref_destroy(h)


def test_two_level_create_validates_without_a_device():
    """lsb_ref2_create: a periodic coarse grid, BGK phases, a box keeping a
    node to every face and spanning 4 cells per axis; host memory only."""
    lib = lsb.load()
    w = W.two_level_bubble(W.D2Q9)

    def create(p, box):
        h = C.c_void_p()
        rc = lib.lsb_ref2_create(C.byref(lsb.to_params(p)), (C.c_int * 6)(*(tuple(box) + (0, 0))[:6]), C.byref(h))
        return rc, h

    for p, box in [(dict(w["params"], bc=[W.NOSLIP] * 4 + [W.PERIODIC] * 2), w["box"]),
                   (dict(w["params"], collision=[W.BGK, W.CUMULANT], lattice=W.D3Q27, nz=48), (10, 38, 10, 38, 10, 38)),
                   (w["params"], (10, 13, 10, 38)), (w["params"], (0, 38, 10, 38)), (w["params"], (10, 47, 10, 38)),
                   (dict(w["params"], tau=[0.5, 0.8]), w["box"])]:
        rc, h = create(p, box)
        assert rc == lsb.LSB_EINVAL and not h.value, (p["bc"], box)
    rc, h = create(w["params"], w["box"])
    assert rc == lsb.LSB_OK and h.value
    nb = C.c_size_t()
    assert lib.lsb_ref2_workspace_bytes(h, C.byref(nb)) == 0
    sh = (C.c_int * 3)()
    assert lib.lsb_ref2_fine_shape(h, sh) == 0 and tuple(sh) == (57, 57, 1)
    # coarse populations twice (FP64) at least, plus the fine level's workspace
    assert nb.value > 2 * 9 * 48 * 48 * 8 + 2 * 9 * 57 * 57 * 8
    lib.lsb_ref2_destroy(h)


def test_traffic_record_is_tied_to_the_bulk_kernel_sources():
    """The benchmark reports counter traffic only for the sources it was
    measured on: the hash covers the D3Q27 unit, every header it includes,
    the plan set-up and the build flags, and nothing the kernel is not built
    from."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    files = bench.kernel_sources()
    for f in ("paper_2601_05936_amd/csrc/kernels.h", "paper_2601_05936_amd/csrc/common.h",
              "paper_2601_05936_amd/csrc/driver.h", "paper_2601_05936_amd/csrc/plan.h",
              "paper_2601_05936_amd/csrc/api.hip", "paper_2601_05936_amd/csrc/lsb_d3q27.hip",
              "include/lsb.h", "paper_2601_05936_amd/build.py"):
        assert f in files, f
    assert not any(f.endswith(("refine.hip", "refine2.hip", "adjoint.h")) for f in files)
    h = bench.kernel_sources_hash()
    assert len(h) == 16 and h == bench.kernel_sources_hash()
    if bench.MEASURED_TRAFFIC["sources"] != h:
        assert bench.measured_traffic(("f16dev", "serial", 512)) is None
