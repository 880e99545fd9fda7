"""ctypes binding of the CPU oracle (lsb_oracle.cpp, refine_oracle.cpp).

TEST INFRASTRUCTURE ONLY.  The parameter block below mirrors orc::Params of
the oracle's own source; it is not shared with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lsb_oracle.cpp")
SRCS = [SRC, os.path.join(HERE, "refine_oracle.cpp")]
LIB_PATH = os.path.join(HERE, "liblsb_oracle.so")


def build(verbose: bool = False) -> str:
    """Compile the oracle with the host compiler (plain C++17, OpenMP)."""
    cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", LIB_PATH] + SRCS
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB_PATH


class _Params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int), ("storage", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("bc", C.c_int * 6), ("wall_u", (C.c_double * 3) * 6),
        ("rho_phys", C.c_double * 2), ("tau", C.c_double * 2), ("accel", (C.c_double * 3) * 2),
        ("sigma", C.c_double), ("band", C.c_double), ("n_ext", C.c_int), ("ext_dtau", C.c_double),
        ("reinit_every", C.c_int), ("n_reinit", C.c_int), ("reinit_dtau", C.c_double),
        ("heaviside_eps", C.c_double), ("use_pb", C.c_int), ("pb0", C.c_double),
        ("init_hydrostatic", C.c_int), ("fp16_scale_log2", C.c_int), ("collision", C.c_int * 2),
    ]


def _params(p: dict) -> _Params:
    s = _Params()
    for k, _ in _Params._fields_:
        v = p[k]
        if k == "bc":
            for i in range(6):
                s.bc[i] = int(v[i])
        elif k == "wall_u":
            for i in range(6):
                for a in range(3):
                    s.wall_u[i][a] = float(v[i][a])
        elif k in ("rho_phys", "tau"):
            for i in range(2):
                getattr(s, k)[i] = float(v[i])
        elif k == "accel":
            for i in range(2):
                for a in range(3):
                    s.accel[i][a] = float(v[i][a])
        elif k == "collision":
            for i in range(2):
                s.collision[i] = int(v[i])
        else:
            setattr(s, k, v)
    return s


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(os.path.getmtime(f) for f in SRCS):
        build()
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER(_Params)
    dp = C.POINTER(C.c_double)
    ub = C.POINTER(C.c_ubyte)
    lib.orc_create.restype = C.c_void_p
    lib.orc_create.argtypes = [P]
    lib.orc_destroy.argtypes = [C.c_void_p]
    lib.orc_init.argtypes = [C.c_void_p, dp, dp, dp]
    lib.orc_step.argtypes = [C.c_void_p, C.c_int]
    lib.orc_nstep.restype = C.c_long
    lib.orc_nstep.argtypes = [C.c_void_p]
    lib.orc_get_pop.argtypes = [C.c_void_p, dp]
    lib.orc_set_decisions.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
    lib.orc_replay_failed.argtypes = [C.c_void_p]
    lib.orc_r2_create.restype = C.c_void_p
    lib.orc_r2_create.argtypes = [P, C.POINTER(C.c_int)]
    lib.orc_r2_destroy.argtypes = [C.c_void_p]
    lib.orc_r2_fine_shape.argtypes = [C.c_void_p, C.POINTER(C.c_int)]
    lib.orc_r2_init.argtypes = [C.c_void_p, dp, dp, dp, dp, dp, dp]
    lib.orc_r2_step.argtypes = [C.c_void_p, C.c_int]
    lib.orc_r2_get_coarse.argtypes = [C.c_void_p, dp, C.POINTER(C.c_ubyte)]
    lib.orc_r2_fine.restype = C.c_void_p
    lib.orc_r2_fine.argtypes = [C.c_void_p]
    lib.orc_r2_sensor.argtypes = [C.c_void_p, C.c_double, C.POINTER(C.c_int)]
    lib.orc_r2_remesh.argtypes = [C.c_void_p, C.POINTER(C.c_int)]
    lib.orc_r2_box.argtypes = [C.c_void_p, C.POINTER(C.c_int)]
    lib.orc_decisions.restype = C.c_long
    lib.orc_decisions.argtypes = [C.c_void_p, C.POINTER(C.c_uint64), C.c_long]
    lib.orc_get_sample.argtypes = [C.c_void_p, C.POINTER(C.c_long), C.c_int, dp, dp, C.POINTER(C.c_ubyte)]
    lib.orc_get_sample.restype = C.c_int
    lib.orc_get_fields.argtypes = [C.c_void_p, dp, dp, dp, ub]
    lib.orc_get_interface.argtypes = [C.c_void_p, dp, dp, dp, ub]
    lib.orc_get_moments.argtypes = [C.c_void_p, dp]
    lib.orc_get_integrals.argtypes = [C.c_void_p, dp]
    lib.orc_lattice.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int), dp,
                                C.POINTER(C.c_int)]
    lib.orc_feq.argtypes = [C.c_int, C.c_double, dp, dp]
    lib.orc_refill_weights.argtypes = [C.c_double, dp]
    lib.orc_get_bubbles.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int), dp, C.POINTER(C.c_int)]
    lib.orc_cumulants_points.argtypes = [C.c_int, dp, dp, dp]
    lib.orc_moments_from_cumulants.argtypes = [dp, dp]
    lib.orc_cumulant_collide.argtypes = [dp, C.c_double, C.c_double, C.c_double, dp, dp]
    lib.orc_heaviside.restype = C.c_double
    lib.orc_heaviside.argtypes = [C.c_double, C.c_double]
    lib.orc_geometry.argtypes = [P, dp, dp, dp]
    lib.orc_advect_rate.argtypes = [P, dp, dp, dp]
    lib.orc_advect.argtypes = [P, dp, dp, C.c_int]
    lib.orc_reinit.argtypes = [P, dp, C.c_int]
    lib.orc_extend.argtypes = [P, dp, ub, dp]
    lib.orc_refill.argtypes = [P, dp, ub, dp, dp, dp, dp, C.c_double]
    lib.orc_tan_create.restype = C.c_void_p
    lib.orc_tan_create.argtypes = [P]
    lib.orc_tan_destroy.argtypes = [C.c_void_p]
    lib.orc_tan_init.argtypes = [C.c_void_p, dp, dp, C.c_double, dp, dp]
    lib.orc_tan_step.argtypes = [C.c_void_p, C.c_int]
    lib.orc_tan_centroid.argtypes = [C.c_void_p, C.c_int, dp, dp]
    lib.orc_tan_get_pop.argtypes = [C.c_void_p, dp, dp]
    lib.orc_ref_create.restype = C.c_void_p
    lib.orc_ref_create.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_double, C.c_double]
    lib.orc_ref_destroy.argtypes = [C.c_void_p]
    lib.orc_ref_init.argtypes = [C.c_void_p, dp, dp, dp, dp]
    lib.orc_ref_step.argtypes = [C.c_void_p, C.c_int]
    lib.orc_ref_get.argtypes = [C.c_void_p, dp, dp]
    lib.orc_ref_sensor.argtypes = [C.c_void_p, dp, C.c_double, C.c_int, C.POINTER(C.c_int)]
    lib.orc_ref_remesh.argtypes = [C.c_void_p, C.POINTER(C.c_int)]
    lib.orc_mref_create.restype = C.c_void_p
    lib.orc_mref_create.argtypes = [C.c_int, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_int), C.c_double,
                                    C.POINTER(C.c_double)]
    lib.orc_tree_create.restype = C.c_void_p
    lib.orc_tree_create.argtypes = [C.c_int, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                    C.c_double, C.POINTER(C.c_double)]
    lib.orc_mref_init.argtypes = [C.c_void_p, C.POINTER(dp), C.POINTER(dp)]
    lib.orc_mref_get.argtypes = [C.c_void_p, C.c_int, dp]
    lib.orc_ref_sensor_levels.argtypes = [C.c_void_p, dp, C.c_double, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.orc_ref_remesh_levels.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.c_int]
    lib.orc_ref_sensor_seeded.restype = C.c_int
    lib.orc_ref_sensor_seeded.argtypes = [C.c_void_p, dp, C.c_double, C.c_int, C.c_int, C.POINTER(C.c_int),
                                          C.POINTER(C.c_int)]
    _lib = lib
    return lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, n=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


def lattice(lat: int):
    lib = _load()
    D, Q = C.c_int(), C.c_int()
    c = (C.c_int * 81)()
    w = np.zeros(27)
    opp = (C.c_int * 27)()
    assert lib.orc_lattice(lat, C.byref(D), C.byref(Q), c, _dp(w), opp) == 0
    q = Q.value
    cc = np.array(c[:3 * q], dtype=np.int64).reshape(q, 3)
    return D.value, q, cc, w[:q].copy(), np.array(opp[:q])


def feq(lat: int, rho: float, u) -> np.ndarray:
    lib = _load()
    u = _f64(np.asarray(u, dtype=np.float64).reshape(3))
    out = np.zeros(27)
    assert lib.orc_feq(lat, float(rho), _dp(u), _dp(out)) == 0
    return out[: lattice(lat)[1]]


def cumulants_points(pts, w) -> np.ndarray:
    """Joint cumulants kappa[a, b, c] (a, b, c in 0..2) of a weighted point set
    in R^3 (normalised by the total weight; kappa[0, 0, 0] = total weight)."""
    pts = _f64(np.asarray(pts, dtype=np.float64).reshape(-1, 3))
    w = _f64(w, pts.shape[0])
    out = np.zeros(27)
    assert _load().orc_cumulants_points(pts.shape[0], _dp(pts), _dp(w), _dp(out)) == 0
    return out.reshape(3, 3, 3)


def moments_from_cumulants(kappa) -> np.ndarray:
    """Normalised moments m[a, b, c] from joint cumulants (kappa[0, 0, 0] ignored)."""
    k = _f64(np.asarray(kappa, dtype=np.float64).reshape(27))
    out = np.zeros(27)
    _load().orc_moments_from_cumulants(_dp(k), _dp(out))
    return out.reshape(3, 3, 3)


def cumulant_collide(f, omega1: float, omega2: float = 1.0, omega3: float = 1.0, acc=(0.0, 0.0, 0.0)):
    """One D3Q27 cell (oracle direction order) through the cumulant collision."""
    f = _f64(f, 27)
    a = _f64(np.asarray(acc, dtype=np.float64), 3)
    out = np.zeros(27)
    assert _load().orc_cumulant_collide(_dp(f), float(omega1), float(omega2), float(omega3), _dp(a), _dp(out)) == 0
    return out


def refill_weights(q: float) -> np.ndarray:
    out = np.zeros(3)
    _load().orc_refill_weights(float(q), _dp(out))
    return out


def heaviside(phi: float, eps: float) -> float:
    return _load().orc_heaviside(float(phi), float(eps))


def _ncell(p):
    return p["nx"] * p["ny"] * p["nz"]


def _dim(p):
    return 2 if p["lattice"] == 0 else 3


def geometry(p: dict, phi):
    lib = _load()
    N = _ncell(p)
    phi = _f64(phi, N)
    n = np.zeros(N * _dim(p))
    k = np.zeros(N)
    assert lib.orc_geometry(C.byref(_params(p)), _dp(phi), _dp(n), _dp(k)) == 0
    shp = (p["nz"], p["ny"], p["nx"])
    return n.reshape(shp + (_dim(p),)), k.reshape(shp)


def advect_rate(p: dict, phi, u):
    lib = _load()
    N = _ncell(p)
    phi = _f64(phi, N)
    u = _f64(u, 3 * N)
    out = np.zeros(N)
    assert lib.orc_advect_rate(C.byref(_params(p)), _dp(phi), _dp(u), _dp(out)) == 0
    return out.reshape(p["nz"], p["ny"], p["nx"])


def advect(p: dict, phi, u, nsteps: int):
    lib = _load()
    N = _ncell(p)
    phi = _f64(phi, N).copy()
    u = _f64(u, 3 * N)
    assert lib.orc_advect(C.byref(_params(p)), _dp(phi), _dp(u), int(nsteps)) == 0
    return phi.reshape(p["nz"], p["ny"], p["nx"])


def reinit(p: dict, phi, calls: int = 1):
    lib = _load()
    N = _ncell(p)
    phi = _f64(phi, N).copy()
    assert lib.orc_reinit(C.byref(_params(p)), _dp(phi), int(calls)) == 0
    return phi.reshape(p["nz"], p["ny"], p["nx"])


def extend(p: dict, phi, fixed, u):
    lib = _load()
    N = _ncell(p)
    phi = _f64(phi, N)
    fx = np.ascontiguousarray(fixed, dtype=np.uint8).reshape(N)
    u = _f64(u, 3 * N).copy()
    assert lib.orc_extend(C.byref(_params(p)), _dp(phi), fx.ctypes.data_as(C.POINTER(C.c_ubyte)), _dp(u)) == 0
    return u.reshape(p["nz"], p["ny"], p["nx"], 3)


def refill(p: dict, phi_new, old_gas, pop, rho, u, S=None, pb: float = 0.0):
    """Refill (Sec. 2.4) on a crafted state through the oracle step's own
    refill: phi_new (N) gives the new phase and the geometry, old_gas (N)
    the tags before the step, pop (Q, N) the post-collision populations,
    rho (N), u (N, 3) and S (N, 6) the collision's moments.  Returns the
    refilled (pop, rho, u, S)."""
    lib = _load()
    N = _ncell(p)
    phi = _f64(phi_new, N)
    g = np.ascontiguousarray(old_gas, dtype=np.uint8).reshape(N)
    pop = _f64(pop).reshape(-1).copy()
    rho = _f64(rho, N).copy()
    u = _f64(u, 3 * N).copy()
    S = np.zeros(6 * N) if S is None else _f64(S, 6 * N).copy()
    assert lib.orc_refill(C.byref(_params(p)), _dp(phi), g.ctypes.data_as(C.POINTER(C.c_ubyte)), _dp(pop),
                          _dp(rho), _dp(u), _dp(S), float(pb)) == 0
    return pop.reshape(-1, N), rho, u.reshape(N, 3), S.reshape(N, 6)


class TwoPhaseRefineOracle:
    """Two-level refinement of the two-phase step (oracle): a coarse grid
    (params in coarse lattice units; periodic, no-slip or free-slip faces)
    with one box (6 ints, coarse
    nodes) refined at ratio 2 that holds the interface and its band.  The
    fine level is an Oracle view in fine lattice units (self.fine)."""

    def __init__(self, params: dict, box):
        self.lib = _load()
        self.p = dict(params)
        self._cp = _params(self.p)
        b = (tuple(int(v) for v in box) + (0, 0))[:6]
        self.box = b
        self.h = self.lib.orc_r2_create(C.byref(self._cp), (C.c_int * 6)(*b))
        if not self.h:
            raise ValueError("refinement oracle rejected the parameters or the box")
        nf = (C.c_int * 3)()
        self.lib.orc_r2_fine_shape(self.h, nf)
        self.fine_shape = (nf[2], nf[1], nf[0])
        pf = dict(self.p, nx=nf[0], ny=nf[1], nz=nf[2], tau=[2 * t - 0.5 for t in self.p["tau"]],
                  sigma=2 * self.p["sigma"], accel=[[0.5 * a for a in ac] for ac in self.p["accel"]])
        self.fine = Oracle._view(self.lib, self.lib.orc_r2_fine(self.h), pf, self)
        self.Q = self.fine.Q
        self.coarse_shape = (self.p["nz"], self.p["ny"], self.p["nx"])

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.orc_r2_destroy(self.h)
            self.h = None

    def init(self, phi_c, rho_c, u_c, phi_f, rho_f, u_f):
        nc = int(np.prod(self.coarse_shape))
        nf = int(np.prod(self.fine_shape))
        self._keep = [_f64(phi_c, nc), _f64(rho_c, nc), _f64(u_c, 3 * nc), _f64(phi_f, nf), _f64(rho_f, nf),
                      _f64(u_f, 3 * nf)]
        assert self.lib.orc_r2_init(self.h, *[_dp(a) for a in self._keep]) == 0
        return self

    def step(self, n: int = 1):
        rc = self.lib.orc_r2_step(self.h, int(n))
        if rc == -2:
            raise RuntimeError("the level-set band reached the refined box's faces")
        assert rc == 0
        return self

    def sensor(self, d_ref: float):
        """Box (6 ints) that the level-set sensor moves the refined box to."""
        out = (C.c_int * 6)()
        self.lib.orc_r2_sensor(self.h, float(d_ref), out)
        return tuple(out)

    def remesh(self, box):
        """Re-mesh onto a box of the same extents (6 ints)."""
        b = (tuple(int(v) for v in box) + (0, 0))[:6]
        rc = self.lib.orc_r2_remesh(self.h, (C.c_int * 6)(*b))
        if rc == -1:
            raise ValueError("re-meshing needs a box of the same extents inside the grid")
        if rc == -2:
            raise RuntimeError("the level-set band is not inside the new box")
        self.box = b
        return self

    @property
    def current_box(self):
        out = (C.c_int * 6)()
        self.lib.orc_r2_box(self.h, out)
        return tuple(out)

    def coarse(self):
        """(populations [Q][nz][ny][nx], phase [nz][ny][nx]) of the coarse grid
        (covered nodes hold the fine state restricted to the coarse level)."""
        nc = int(np.prod(self.coarse_shape))
        pop = np.zeros(self.Q * nc)
        ph = np.zeros(nc, dtype=np.uint8)
        self.lib.orc_r2_get_coarse(self.h, _dp(pop), ph.ctypes.data_as(C.POINTER(C.c_ubyte)))
        return pop.reshape((self.Q,) + self.coarse_shape), ph.reshape(self.coarse_shape)


class Oracle:
    """One oracle simulation (FP64)."""

    def __init__(self, params: dict, phi0, rho0=None, u0=None, record=False, replay=None):
        """record: keep every decision of this run (tags, branches); replay:
        an Oracle created with record=True whose decisions this run takes
        (the frozen-decision program, for finite differences)."""
        self.lib = _load()
        self.p = dict(params)
        self._cp = _params(self.p)
        self.h = self.lib.orc_create(C.byref(self._cp))
        if not self.h:
            raise ValueError("oracle rejected the parameters")
        self.N = _ncell(self.p)
        self.shape = (self.p["nz"], self.p["ny"], self.p["nx"])
        self.D, self.Q = lattice(self.p["lattice"])[:2]
        if record:
            self.lib.orc_set_decisions(self.h, 1, None)
        if replay is not None:
            self._replay_src = replay  # the record lives as long as the replaying run
            if self.lib.orc_set_decisions(self.h, 2, replay.h) != 0:
                raise ValueError("replay needs an Oracle created with record=True")
        phi0 = _f64(phi0, self.N)
        rho0 = _f64(rho0, self.N)
        u0 = _f64(u0, 3 * self.N)
        assert self.lib.orc_init(self.h, _dp(phi0), _dp(rho0), _dp(u0)) == 0

    def replay_failed(self) -> bool:
        """True if a replayed run met a decision the record does not hold."""
        return bool(self.lib.orc_replay_failed(self.h))

    def __del__(self):
        if getattr(self, "h", None) and not getattr(self, "_borrowed", False):
            self.lib.orc_destroy(self.h)
        self.h = None

    @classmethod
    def _view(cls, lib, handle, params, owner):
        """An Oracle over a simulation owned by another object (no init)."""
        o = cls.__new__(cls)
        o.lib, o.h, o.p, o._borrowed, o._owner = lib, handle, dict(params), True, owner
        o._cp = _params(o.p)
        o.N = _ncell(o.p)
        o.shape = (o.p["nz"], o.p["ny"], o.p["nx"])
        o.D, o.Q = lattice(o.p["lattice"])[:2]
        return o

    def step(self, n: int = 1):
        assert self.lib.orc_step(self.h, int(n)) == 0

    @property
    def nstep(self):
        return self.lib.orc_nstep(self.h)

    def decisions(self) -> np.ndarray:
        """One 64-bit hash per step taken of every decision the step's values
        made (tags, bounce-back branches, upwind directions, clamps, refill
        directions and fallbacks, Heaviside regions, bubble labels)."""
        n = self.lib.orc_decisions(self.h, None, 0)
        out = np.zeros(max(n, 1), dtype=np.uint64)
        self.lib.orc_decisions(self.h, out.ctypes.data_as(C.POINTER(C.c_uint64)), n)
        return out[:n]

    def populations(self):
        out = np.zeros(self.Q * self.N)
        self.lib.orc_get_pop(self.h, _dp(out))
        return out.reshape((self.Q,) + self.shape)

    def sample(self, cells):
        """Populations [Q, n], phi [n] and tags [n] at flat cell indices."""
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        n = len(cells)
        pop = np.zeros(self.Q * n)
        phi = np.zeros(n)
        t = np.zeros(n, dtype=np.uint8)
        assert self.lib.orc_get_sample(self.h, cells.ctypes.data_as(C.POINTER(C.c_long)), n, _dp(pop), _dp(phi),
                                       t.ctypes.data_as(C.POINTER(C.c_ubyte))) == 0
        return pop.reshape(self.Q, n), phi, t

    def fields(self):
        rho = np.zeros(self.N)
        u = np.zeros(self.N * self.D)
        p = np.zeros(self.N)
        ph = np.zeros(self.N, dtype=np.uint8)
        self.lib.orc_get_fields(self.h, _dp(rho), _dp(u), _dp(p), ph.ctypes.data_as(C.POINTER(C.c_ubyte)))
        return dict(rho=rho.reshape(self.shape), u=u.reshape(self.shape + (self.D,)), p=p.reshape(self.shape),
                    phase=ph.reshape(self.shape))

    def interface(self):
        phi = np.zeros(self.N)
        n = np.zeros(self.N * self.D)
        k = np.zeros(self.N)
        t = np.zeros(self.N, dtype=np.uint8)
        self.lib.orc_get_interface(self.h, _dp(phi), _dp(n), _dp(k), t.ctypes.data_as(C.POINTER(C.c_ubyte)))
        return dict(phi=phi.reshape(self.shape), normal=n.reshape(self.shape + (self.D,)),
                    kappa=k.reshape(self.shape), tags=t.reshape(self.shape))

    def moments(self):
        out = np.zeros(10 * self.N)
        self.lib.orc_get_moments(self.h, _dp(out))
        return out.reshape(self.shape + (10,))

    def bubbles(self):
        """Several-bubble mode: per bubble (numbered by smallest cell) volume,
        centroid and baseline, and the bubble of every cell (-1 outside the
        Heaviside support)."""
        n = C.c_int()
        assert self.lib.orc_get_bubbles(self.h, 0, C.byref(n), None, None) == 0
        out = np.zeros(5 * max(n.value, 1))
        lab = np.zeros(self.N, dtype=np.int32)
        assert self.lib.orc_get_bubbles(self.h, n.value, C.byref(n), _dp(out),
                                        lab.ctypes.data_as(C.POINTER(C.c_int))) == 0
        b = out[:5 * n.value].reshape(-1, 5)
        return dict(count=n.value, volume=b[:, 0].copy(), centroid=b[:, 1:4].copy(), pb=b[:, 4].copy(),
                    labels=lab.reshape(self.shape))

    def integrals(self):
        out = np.zeros(16)
        self.lib.orc_get_integrals(self.h, _dp(out))
        return dict(mass=out[0:2].copy(), volume_gas=out[2], centroid=out[3:6].copy(), vel_b=out[6:9].copy(),
                    pb=out[9], umax=out[10], step=int(out[11]))


class TangentOracle:
    """Forward-mode tangent of the oracle (dual numbers, frozen decisions)."""

    def __init__(self, params: dict, phi0, dphi0=None, dsigma=0.0, rho0=None, u0=None):
        self.lib = _load()
        self.p = dict(params)
        self._cp = _params(self.p)
        self.h = self.lib.orc_tan_create(C.byref(self._cp))
        if not self.h:
            raise ValueError("oracle rejected the parameters")
        N = _ncell(self.p)
        self.N = N
        assert self.lib.orc_tan_init(self.h, _dp(_f64(phi0, N)), _dp(_f64(dphi0, N)), float(dsigma),
                                     _dp(_f64(rho0, N)), _dp(_f64(u0, 3 * N))) == 0

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.orc_tan_destroy(self.h)
            self.h = None

    def step(self, n: int = 1):
        assert self.lib.orc_tan_step(self.h, int(n)) == 0

    def centroid(self, axis: int):
        v, t = C.c_double(), C.c_double()
        self.lib.orc_tan_centroid(self.h, int(axis), C.byref(v), C.byref(t))
        return v.value, t.value


class RefineOracle:
    """Static refinement of the BGK solver (ratio 2), FP64, two to four
    nested levels.

    lattice 0 (D2Q9), 1 (D3Q19) or 2 (D3Q27).  Coarse nodes nx x ny (x nz),
    periodic.  patch is one box (ia, ib, ja, jb) (+ (ka, kb) in 3D), the
    coarse nodes the fine level covers, inclusive, at half spacing (fine node
    (i, j, k) at (ia + i/2, ja + j/2, ka + k/2)); or a list of such boxes,
    level 1 first, each in its parent level's node coordinates.  With
    parents (one index per box: 0 for the coarse grid, else an earlier box,
    counted from 1) the boxes form a tree: several disjoint boxes may refine
    one grid.  Populations are [Q][nodes] (x fastest), the paper's ordering;
    velocities [nodes][D].
    tau_f = None takes 2 tau - 1/2 from level to level (constant viscosity);
    a number overrides level 1's, a list (one entry per refined level, None
    for the derived value) any level's: the tests pass other values only to
    plant a mistake.
    """

    def __init__(self, nx: int, ny: int, patch, tau_c: float, tau_f=None, lattice: int = 0, nz: int = 1,
                 parents=None):
        lib = _load()
        self.lattice = int(lattice)
        self.D, self.Q = (2, 9) if self.lattice == 0 else (3, 19 if self.lattice == 1 else 27)
        self.nx, self.ny, self.nz = int(nx), int(ny), (int(nz) if self.D == 3 else 1)
        boxes = [patch] if np.isscalar(patch[0]) else list(patch)
        self.boxes = []
        for bx in boxes:
            p = tuple(int(v) for v in bx)
            self.boxes.append(p[:6] if self.D == 3 else p[:4] + (0, 0))
        self.levels = len(self.boxes) + 1
        self.parents = list(range(len(self.boxes))) if parents is None else [int(v) for v in parents]
        over = [None] * (self.levels - 1)
        if tau_f is not None:
            if np.isscalar(tau_f):
                over[0] = float(tau_f)
            else:
                over = [None if t is None else float(t) for t in tau_f]
        self.taus = [float(tau_c)]
        for l in range(1, self.levels):
            par = self.parents[l - 1] if 0 <= self.parents[l - 1] < l else 0
            self.taus.append(2.0 * self.taus[par] - 0.5 if over[l - 1] is None else over[l - 1])
        n3 = (C.c_int * 3)(self.nx, self.ny, self.nz)
        flat = [v for bx in self.boxes for v in bx]
        pp = (C.c_int * len(flat))(*flat)
        tt = (C.c_double * self.levels)(*self.taus)
        par = (C.c_int * len(self.parents))(*self.parents)
        self._h = lib.orc_tree_create(self.lattice, n3, len(self.boxes), par, pp, float(tau_c), tt)
        if not self._h:
            raise ValueError("invalid refinement configuration")
        self._lib = lib
        self._sync_level1()

    def _sync_level1(self):
        ia, ib, ja, jb, ka, kb = self.boxes[0]
        self.patch = self.boxes[0] if self.D == 3 else self.boxes[0][:4]
        self.mx, self.my, self.mz = 2 * (ib - ia), 2 * (jb - ja), 2 * (kb - ka)

    @property
    def tau_c(self) -> float:
        return self.taus[0]

    @property
    def tau_f(self) -> float:
        return self.taus[1]

    def shape(self, level: int):
        """Nodes per axis (x, y, z) of a level."""
        if level == 0:
            return self.nx, self.ny, self.nz
        ia, ib, ja, jb, ka, kb = self.boxes[level - 1]
        return 2 * (ib - ia) + 1, 2 * (jb - ja) + 1, 2 * (kb - ka) + 1

    def n_level(self, level: int) -> int:
        return int(np.prod(self.shape(level)))

    @property
    def n_coarse(self) -> int:
        return self.n_level(0)

    @property
    def n_fine(self) -> int:
        return self.n_level(1)

    def coords(self, level: int):
        """Coarse-unit coordinates of a level's nodes, [nodes] each: (x, y)
        in 2D, (x, y, z) in 3D."""
        path = []
        l = level
        while l > 0:
            path.append(l)
            l = self.parents[l - 1]
        o, h = np.zeros(3), 1.0
        for l in reversed(path):
            bx = self.boxes[l - 1]
            o = o + h * np.array([bx[0], bx[2], bx[4]], dtype=float)
            h *= 0.5
        sx, sy, sz = self.shape(level)
        k, j, i = np.meshgrid(np.arange(sz), np.arange(sy), np.arange(sx), indexing="ij")
        xyz = (o[0] + h * i.reshape(-1), o[1] + h * j.reshape(-1), o[2] + h * k.reshape(-1))
        return xyz[:self.D]

    def fine_coords(self):
        """Coarse-unit coordinates of level 1's nodes."""
        return self.coords(1)

    def init(self, rho_c, u_c, rho_f, u_f, *deeper):
        """Equilibrium state from rho and u on every level: the coarse and
        level-1 arrays, then (rho, u) of each deeper level."""
        arrs = [rho_c, u_c, rho_f, u_f] + list(deeper)
        if len(arrs) != 2 * self.levels:
            raise ValueError("one (rho, u) pair per level expected")
        self._keep = []
        for l in range(self.levels):
            n = self.n_level(l)
            self._keep += [_f64(arrs[2 * l], n), _f64(arrs[2 * l + 1], self.D * n)]
        dpt = C.POINTER(C.c_double)
        rho = (dpt * self.levels)(*[_dp(self._keep[2 * l]) for l in range(self.levels)])
        u = (dpt * self.levels)(*[_dp(self._keep[2 * l + 1]) for l in range(self.levels)])
        self._lib.orc_mref_init(self._h, rho, u)
        return self

    def step(self, n: int = 1):
        self._lib.orc_ref_step(self._h, int(n))
        return self

    def sensor(self, phi, d_ref: float, margin: int):
        """Patch box (6 ints) of the level-set sensor on the coarse level set
        phi [n_coarse], or None when no node is tagged."""
        out = (C.c_int * 6)()
        keep = _f64(phi, self.n_coarse)
        if not self._lib.orc_ref_sensor(self._h, _dp(keep), float(d_ref), int(margin), out):
            return None
        return tuple(out)

    def remesh(self, patch):
        """Re-mesh a two-level hierarchy onto patch (6 ints; ka, kb ignored in
        2D)."""
        p = tuple(int(v) for v in patch) + (0, 0)
        p6 = (C.c_int * 6)(*p[:6])
        if self._lib.orc_ref_remesh(self._h, p6) != 0:
            raise ValueError("patch does not fit the grid")
        ia, ib, ja, jb, ka, kb = p[:6]
        if self.D == 2:
            ka = kb = 0
        self.boxes[0] = (ia, ib, ja, jb, ka, kb)
        self._sync_level1()
        return self

    def sensor_levels(self, phi, d_ref: float, margins):
        """Boxes of every refined level (6 ints each, each in its parent's
        node coordinates) from the level-set sensor on the coarse level set,
        with margins[l - 1] coarse nodes for level l; None when no node is
        tagged."""
        nl = self.levels - 1
        out = (C.c_int * (6 * nl))()
        mg = (C.c_int * nl)(*[int(m) for m in margins])
        keep = _f64(phi, self.n_coarse)
        rc = self._lib.orc_ref_sensor_levels(self._h, _dp(keep), float(d_ref), mg, out)
        if rc < 0:
            raise ValueError("the sensor's boxes need a chain of nested levels")
        if not rc:
            return None
        return [tuple(out[6 * l:6 * l + 6]) for l in range(nl)]

    def sensor_seeded(self, phi, d_ref: float, margin: int, seeds):
        """Boxes for a tree of root boxes (6 ints each): tagged coarse nodes
        go to their nearest seed (seeds: coarse nodes, (x, y[, z]) each),
        each seed's bounding box grown by margin and clamped, boxes closer
        than one node merged."""
        sd = [tuple(int(v) for v in p) + (0,) * (3 - len(p)) for p in seeds]
        flat = [v for p in sd for v in p]
        out = (C.c_int * (6 * len(sd)))()
        keep = _f64(phi, self.n_coarse)
        nb = self._lib.orc_ref_sensor_seeded(self._h, _dp(keep), float(d_ref), int(margin), len(sd),
                                             (C.c_int * len(flat))(*flat), out)
        return [tuple(out[6 * k:6 * k + 6]) for k in range(nb)]

    def remesh_levels(self, boxes):
        """Re-mesh every refined level onto boxes (6 ints each, level 1
        first, each in its new parent's node coordinates), one box per
        refined grid."""
        if len(boxes) != self.levels - 1:
            raise ValueError(f"{len(boxes)} boxes for {self.levels - 1} refined grids: the tree needs rebuilding")
        flat = []
        for bx in boxes:
            p = (tuple(int(v) for v in bx) + (0, 0))[:6]
            flat += list(p if self.D == 3 else p[:4] + (0, 0))
        if self._lib.orc_ref_remesh_levels(self._h, (C.c_int * max(1, len(flat)))(*flat), len(boxes)) != 0:
            raise ValueError("the boxes do not match the refined grids, or a box does not fit its parent")
        self.boxes = [tuple(flat[6 * l:6 * l + 6]) for l in range(len(boxes))]
        self._sync_level1()
        return self

    def level(self, l: int):
        """Post-collision populations of level l, [Q][(nz,) ny, nx]."""
        sx, sy, sz = self.shape(l)
        f = np.zeros(self.Q * sx * sy * sz)
        self._lib.orc_mref_get(self._h, int(l), _dp(f))
        return f.reshape(self.Q, sy, sx) if self.D == 2 else f.reshape(self.Q, sz, sy, sx)

    def populations(self):
        """Post-collision populations of every level (coarse first); the
        covered nodes hold the restricted values."""
        return tuple(self.level(l) for l in range(self.levels))

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.orc_ref_destroy(self._h)
            self._h = None
