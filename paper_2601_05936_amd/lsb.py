"""Thin Python binding of liblsb.so (argument marshalling only).

Every step of the method runs in the HIP kernels behind the C ABI of
include/lsb.h, include/lsb_refine.h and include/lsb_refine2.h; this module only converts parameters, hands over torch device
memory (the caller-owned workspace) and stream handles, and wraps results.
It fails loudly when the built library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblsb.so")

LSB_OK, LSB_EINVAL, LSB_ENOMEM, LSB_EDEVICE, LSB_ESTATE, LSB_EUNSTABLE, LSB_EBAND = 0, -1, -2, -3, -4, -5, -6
D2Q9, D3Q19, D3Q27 = 0, 1, 2
F64, F32, F16DEV, BF16DEV = 0, 1, 2, 3


class LsbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lsb error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    """Mirror of lsb_params (include/lsb.h)."""
    _fields_ = [
        ("lattice", C.c_int), ("storage", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("bc", C.c_int * 6), ("wall_u", (C.c_double * 3) * 6),
        ("rho_phys", C.c_double * 2), ("tau", C.c_double * 2), ("accel", (C.c_double * 3) * 2),
        ("sigma", C.c_double), ("band", C.c_double), ("n_ext", C.c_int), ("ext_dtau", C.c_double),
        ("reinit_every", C.c_int), ("n_reinit", C.c_int), ("reinit_dtau", C.c_double),
        ("heaviside_eps", C.c_double), ("use_pb", C.c_int), ("pb0", C.c_double),
        ("init_hydrostatic", C.c_int), ("fp16_scale_log2", C.c_int), ("collision", C.c_int * 2),
    ]


class Integrals(C.Structure):
    _fields_ = [("mass", C.c_double * 2), ("volume_gas", C.c_double), ("centroid", C.c_double * 3),
                ("vel_b", C.c_double * 3), ("pb", C.c_double), ("umax", C.c_double), ("step", C.c_long)]


EXPORTS = [
    "lsb_create", "lsb_destroy", "lsb_workspace_bytes", "lsb_bind", "lsb_init", "lsb_step", "lsb_get_fields",
    "lsb_get_interface", "lsb_get_bubbles", "lsb_get_populations", "lsb_get_moments", "lsb_get_integrals", "lsb_get_integrals_static", "lsb_state_bytes",
    "lsb_save_state", "lsb_load_state", "lsb_step_count", "lsb_get_counts", "lsb_set_kernel_timing",
    "lsb_get_kernel_timing", "lsb_set_schedule", "lsb_adjoint_workspace_bytes", "lsb_adjoint_bind",
    "lsb_adjoint_record", "lsb_adjoint_seed_centroid", "lsb_adjoint_reverse", "lsb_adjoint_initial",
    "lsb_last_error",
    "lsb_ref_create", "lsb_ref_destroy", "lsb_ref_workspace_bytes", "lsb_ref_bind", "lsb_ref_init", "lsb_ref_step",
    "lsb_ref_get_populations", "lsb_ref_sensor", "lsb_ref_remesh", "lsb_ref_init_levels", "lsb_ref_get_level",
    "lsb_ref_sensor_levels", "lsb_ref_remesh_levels", "lsb_ref_create_tree", "lsb_ref_set_graphs",
    "lsb_ref_sensor_seeded",
    "lsb_ref2_create", "lsb_ref2_destroy", "lsb_ref2_workspace_bytes", "lsb_ref2_bind", "lsb_ref2_fine_shape",
    "lsb_ref2_fine", "lsb_ref2_init", "lsb_ref2_step", "lsb_ref2_step_count", "lsb_ref2_get_coarse",
    "lsb_ref2_get_box", "lsb_ref2_sensor", "lsb_ref2_remesh",
]


REF_MAX_LEVELS = 4  # LSB_REF_MAX_LEVELS


class RefParams(C.Structure):
    """Mirror of lsb_ref_params (include/lsb_refine.h)."""
    _fields_ = [("lattice", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("patch", C.c_int * 6),
                ("tau_c", C.c_double), ("max_extent", C.c_int * 3), ("levels", C.c_int),
                ("inner", (C.c_int * 6) * (REF_MAX_LEVELS - 2)),
                ("max_inner_extent", (C.c_int * 3) * (REF_MAX_LEVELS - 2))]
SCHED_SERIAL, SCHED_OVERLAP = 0, 1
MAX_BUBBLES = 64  # LSB_MAX_BUBBLES

_lib = None


def load() -> C.CDLL:
    """Load the built library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(or python paper_2601_05936_amd/build.py)")
    lib = C.CDLL(LIB_PATH)
    vp, dp, sz = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_size_t)
    P = C.POINTER(Params)
    lib.lsb_create.argtypes = [P, C.POINTER(vp)]
    lib.lsb_destroy.argtypes = [vp]
    lib.lsb_destroy.restype = None
    lib.lsb_workspace_bytes.argtypes = [vp, sz]
    lib.lsb_bind.argtypes = [vp, vp, C.c_size_t]
    lib.lsb_init.argtypes = [vp, vp, vp, vp, C.c_int, vp]
    lib.lsb_step.argtypes = [vp, C.c_int, C.c_int, vp]
    lib.lsb_get_fields.argtypes = [vp, vp, vp, vp, vp, C.c_int, vp]
    lib.lsb_get_interface.argtypes = [vp, vp, vp, vp, vp, C.c_int, vp]
    lib.lsb_get_populations.argtypes = [vp, vp, C.c_int, vp]
    lib.lsb_get_moments.argtypes = [vp, vp, C.c_int, vp]
    lib.lsb_get_integrals.argtypes = [vp, C.POINTER(Integrals), vp]
    lib.lsb_get_integrals_static.argtypes = [vp, vp, vp]
    lib.lsb_get_bubbles.argtypes = [vp, C.c_int, C.POINTER(C.c_int), vp, vp, C.c_int, vp]
    lib.lsb_state_bytes.argtypes = [vp, sz]
    lib.lsb_save_state.argtypes = [vp, vp, vp]
    lib.lsb_load_state.argtypes = [vp, vp, vp]
    lib.lsb_step_count.argtypes = [vp]
    lib.lsb_step_count.restype = C.c_long
    lib.lsb_get_counts.argtypes = [vp, C.POINTER(C.c_int), vp]
    lib.lsb_set_kernel_timing.argtypes = [vp, C.c_int]
    lib.lsb_get_kernel_timing.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_long)]
    lib.lsb_set_schedule.argtypes = [vp, C.c_int]
    lib.lsb_adjoint_workspace_bytes.argtypes = [vp, C.c_int, sz]
    lib.lsb_adjoint_bind.argtypes = [vp, vp, C.c_size_t, C.c_int]
    lib.lsb_adjoint_record.argtypes = [vp, C.c_int, vp]
    lib.lsb_adjoint_seed_centroid.argtypes = [vp, C.c_int, vp]
    lib.lsb_adjoint_reverse.argtypes = [vp, vp]
    lib.lsb_adjoint_initial.argtypes = [vp, vp, vp, C.c_int, vp, dp, vp]
    lib.lsb_last_error.restype = C.c_char_p
    R = C.POINTER(RefParams)
    lib.lsb_ref_create.argtypes = [R, C.POINTER(vp)]
    lib.lsb_ref_destroy.argtypes = [vp]
    lib.lsb_ref_destroy.restype = None
    lib.lsb_ref_workspace_bytes.argtypes = [vp, sz]
    lib.lsb_ref_bind.argtypes = [vp, vp, C.c_size_t]
    lib.lsb_ref_init.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.lsb_ref_step.argtypes = [vp, C.c_int, vp]
    lib.lsb_ref_get_populations.argtypes = [vp, vp, vp, vp]
    lib.lsb_ref_sensor.argtypes = [vp, vp, C.c_double, C.c_int, C.POINTER(C.c_int), vp]
    lib.lsb_ref_remesh.argtypes = [vp, C.POINTER(C.c_int), vp]
    lib.lsb_ref_init_levels.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), vp]
    lib.lsb_ref_get_level.argtypes = [vp, C.c_int, vp, vp]
    lib.lsb_ref_sensor_levels.argtypes = [vp, vp, C.c_double, C.POINTER(C.c_int), C.POINTER(C.c_int), vp]
    lib.lsb_ref_remesh_levels.argtypes = [vp, C.POINTER(C.c_int), C.c_int, vp]
    lib.lsb_ref_create_tree.argtypes = [R, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(vp)]
    lib.lsb_ref_set_graphs.argtypes = [vp, C.c_int]
    lib.lsb_ref_sensor_seeded.argtypes = [vp, vp, C.c_double, C.c_int, C.c_int, C.POINTER(C.c_int),
                                          C.POINTER(C.c_int), C.POINTER(C.c_int), vp]
    lib.lsb_ref2_create.argtypes = [P, C.POINTER(C.c_int), C.POINTER(vp)]
    lib.lsb_ref2_destroy.argtypes = [vp]
    lib.lsb_ref2_destroy.restype = None
    lib.lsb_ref2_workspace_bytes.argtypes = [vp, sz]
    lib.lsb_ref2_bind.argtypes = [vp, vp, C.c_size_t]
    lib.lsb_ref2_fine_shape.argtypes = [vp, C.POINTER(C.c_int)]
    lib.lsb_ref2_fine.argtypes = [vp, C.POINTER(vp)]
    lib.lsb_ref2_init.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.lsb_ref2_step.argtypes = [vp, C.c_int, vp]
    lib.lsb_ref2_step_count.argtypes = [vp]
    lib.lsb_ref2_step_count.restype = C.c_long
    lib.lsb_ref2_get_coarse.argtypes = [vp, vp, vp, vp]
    lib.lsb_ref2_get_box.argtypes = [vp, C.POINTER(C.c_int)]
    lib.lsb_ref2_sensor.argtypes = [vp, C.c_double, C.POINTER(C.c_int), vp]
    lib.lsb_ref2_remesh.argtypes = [vp, C.POINTER(C.c_int), vp]
    _lib = lib
    return lib


def to_params(p: dict) -> Params:
    s = Params()
    for k, _ in Params._fields_:
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


def _check(rc: int):
    if rc != LSB_OK:
        raise LsbError(rc, load().lsb_last_error().decode())


class Sim:
    """One simulation on one GPU.  Device memory is a torch uint8 tensor
    (the caller-owned workspace); calls run on torch's current stream."""

    def __init__(self, params: dict, device="cuda:0"):
        import torch
        self.torch = torch
        self.lib = load()
        self.p = dict(params)
        self.device = torch.device(device)
        self._cp = to_params(self.p)
        h = C.c_void_p()
        _check(self.lib.lsb_create(C.byref(self._cp), C.byref(h)))
        self.h = h
        nb = C.c_size_t()
        _check(self.lib.lsb_workspace_bytes(self.h, C.byref(nb)))
        self.workspace_bytes = nb.value
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        _check(self.lib.lsb_bind(self.h, C.c_void_p(self.ws.data_ptr()), nb.value))
        self.N = self.p["nx"] * self.p["ny"] * self.p["nz"]
        self.D = 2 if self.p["lattice"] == D2Q9 else 3
        self.Q = {D2Q9: 9, D3Q19: 19, D3Q27: 27}[self.p["lattice"]]
        self.shape = (self.p["nz"], self.p["ny"], self.p["nx"])

    @classmethod
    def _view(cls, handle: C.c_void_p, params: dict, owner, device):
        """A Sim over a plan owned by another handle (owner keeps it alive;
        the view never destroys it)."""
        import torch
        s = cls.__new__(cls)
        s.torch = torch
        s.lib = load()
        s.p = dict(params)
        s.device = torch.device(device)
        s.h = handle
        s._owner = owner
        s.N = s.p["nx"] * s.p["ny"] * s.p["nz"]
        s.D = 2 if s.p["lattice"] == D2Q9 else 3
        s.Q = {D2Q9: 9, D3Q19: 19, D3Q27: 27}[s.p["lattice"]]
        s.shape = (s.p["nz"], s.p["ny"], s.p["nx"])
        return s

    def __del__(self):
        if getattr(self, "_owner", None) is not None:
            return
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.lsb_destroy(self.h)
            self.h = None

    def stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _dev(self, a, n):
        if a is None:
            return None
        t = self.torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)) if isinstance(a, np.ndarray) \
            else a.reshape(-1).to(self.torch.float64)
        assert t.numel() == n, (t.numel(), n)
        return t.to(self.device).contiguous()

    def init(self, phi0, rho0=None, u0=None):
        """phi0 [N] signed distance; rho0 [N] or None; u0 [N,3] or None (numpy or torch)."""
        t_phi = self._dev(phi0, self.N)
        t_rho = self._dev(rho0, self.N)
        t_u = self._dev(u0, 3 * self.N)
        ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())  # noqa: E731
        _check(self.lib.lsb_init(self.h, ptr(t_phi), ptr(t_rho), ptr(t_u), 1, self.stream()))
        return self

    def step(self, n: int = 1, check_every: int = 0):
        _check(self.lib.lsb_step(self.h, int(n), int(check_every), self.stream()))

    @property
    def nstep(self) -> int:
        return self.lib.lsb_step_count(self.h)

    def _out(self, n, dtype):
        return self.torch.empty(n, dtype=dtype, device=self.device)

    def fields(self, as_numpy=True):
        t = self.torch
        rho, u, p = self._out(self.N, t.float64), self._out(self.N * self.D, t.float64), self._out(self.N, t.float64)
        ph = self._out(self.N, t.uint8)
        _check(self.lib.lsb_get_fields(self.h, C.c_void_p(rho.data_ptr()), C.c_void_p(u.data_ptr()),
                                       C.c_void_p(p.data_ptr()), C.c_void_p(ph.data_ptr()), 1, self.stream()))
        out = dict(rho=rho.view(self.shape), u=u.view(self.shape + (self.D,)), p=p.view(self.shape),
                   phase=ph.view(self.shape))
        return {k: v.cpu().numpy() for k, v in out.items()} if as_numpy else out

    def interface(self, as_numpy=True):
        t = self.torch
        phi, n, k = self._out(self.N, t.float64), self._out(self.N * self.D, t.float64), self._out(self.N, t.float64)
        tags = self._out(self.N, t.uint8)
        _check(self.lib.lsb_get_interface(self.h, C.c_void_p(phi.data_ptr()), C.c_void_p(n.data_ptr()),
                                          C.c_void_p(k.data_ptr()), C.c_void_p(tags.data_ptr()), 1, self.stream()))
        out = dict(phi=phi.view(self.shape), normal=n.view(self.shape + (self.D,)), kappa=k.view(self.shape),
                   tags=tags.view(self.shape))
        return {kk: v.cpu().numpy() for kk, v in out.items()} if as_numpy else out

    def populations(self, as_numpy=True):
        out = self._out(self.Q * self.N, self.torch.float64)
        _check(self.lib.lsb_get_populations(self.h, C.c_void_p(out.data_ptr()), 1, self.stream()))
        out = out.view((self.Q,) + self.shape)
        return out.cpu().numpy() if as_numpy else out

    def moments(self, as_numpy=True):
        out = self._out(10 * self.N, self.torch.float64)
        _check(self.lib.lsb_get_moments(self.h, C.c_void_p(out.data_ptr()), 1, self.stream()))
        out = out.view(self.shape + (10,))
        return out.cpu().numpy() if as_numpy else out

    def integrals(self) -> dict:
        I = Integrals()
        _check(self.lib.lsb_get_integrals(self.h, C.byref(I), self.stream()))
        return dict(mass=np.array(I.mass[:]), volume_gas=I.volume_gas, centroid=np.array(I.centroid[:]),
                    vel_b=np.array(I.vel_b[:]), pb=I.pb, umax=I.umax, step=I.step)

    def integrals_static(self, out):
        """lsb_get_integrals_static into `out`, a float64 device tensor of 16
        values (no allocation in the library, nothing synchronised)."""
        assert out.dtype == self.torch.float64 and out.is_cuda and out.numel() >= 16 and out.is_contiguous()
        _check(self.lib.lsb_get_integrals_static(self.h, C.c_void_p(out.data_ptr()), self.stream()))
        return out

    def bubbles(self, labels=False) -> dict:
        """Several-bubble mode (use_pb = 2): per bubble, numbered by its smallest
        cell, volume, centroid and gas pressure baseline; with labels, the
        bubble of every cell (-1 outside the Heaviside support)."""
        n = C.c_int()
        out = np.zeros(5 * MAX_BUBBLES)
        lab = np.zeros(self.N, dtype=np.int32) if labels else None
        _check(self.lib.lsb_get_bubbles(self.h, MAX_BUBBLES, C.byref(n), C.c_void_p(out.ctypes.data),
                                        None if lab is None else C.c_void_p(lab.ctypes.data), 0, self.stream()))
        b = out[:5 * n.value].reshape(-1, 5)
        res = dict(count=n.value, volume=b[:, 0].copy(), centroid=b[:, 1:4].copy(), pb=b[:, 4].copy())
        if labels:
            res["labels"] = lab.reshape(self.shape)
        return res

    def counts(self) -> dict:
        c = (C.c_int * 4)()
        _check(self.lib.lsb_get_counts(self.h, c, self.stream()))
        return dict(iface_cells=c[0], active_tiles=c[1], refilled=c[2], wall_cells=c[3])

    def set_schedule(self, schedule: int):
        """SCHED_SERIAL or SCHED_OVERLAP (bit-identical results)."""
        _check(self.lib.lsb_set_schedule(self.h, int(schedule)))
        return self

    def set_kernel_timing(self, enable: bool = True):
        _check(self.lib.lsb_set_kernel_timing(self.h, 1 if enable else 0))

    def kernel_timing(self):
        """(total ms, launches) of the bulk collide-stream kernel since enabling."""
        ms, n = C.c_double(), C.c_long()
        _check(self.lib.lsb_get_kernel_timing(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    # -- reverse mode (D2Q9, F64/F32 storage; the reinitialisation is
    # differentiated too, with its branches frozen) ----------------------
    def adjoint_bind(self, max_segment_steps: int):
        nb = C.c_size_t()
        _check(self.lib.lsb_adjoint_workspace_bytes(self.h, int(max_segment_steps), C.byref(nb)))
        self.adj_ws = self.torch.empty(nb.value, dtype=self.torch.uint8, device=self.device)
        _check(self.lib.lsb_adjoint_bind(self.h, C.c_void_p(self.adj_ws.data_ptr()), nb.value, int(max_segment_steps)))
        return self

    def adjoint_record(self, nsteps: int):
        _check(self.lib.lsb_adjoint_record(self.h, int(nsteps), self.stream()))

    def adjoint_seed_centroid(self, axis: int):
        _check(self.lib.lsb_adjoint_seed_centroid(self.h, int(axis), self.stream()))

    def adjoint_reverse(self):
        _check(self.lib.lsb_adjoint_reverse(self.h, self.stream()))

    def adjoint_initial(self, phi0, u0=None, rho0_given=False):
        """(dL/dphi0 as a float64 device tensor of N values, dL/dsigma)."""
        t_phi = self._dev(phi0, self.N)
        t_u = self._dev(u0, 3 * self.N)
        out = self._out(self.N, self.torch.float64)
        ds = C.c_double()
        _check(self.lib.lsb_adjoint_initial(self.h, C.c_void_p(t_phi.data_ptr()),
                                            None if t_u is None else C.c_void_p(t_u.data_ptr()),
                                            1 if rho0_given else 0, C.c_void_p(out.data_ptr()), C.byref(ds),
                                            self.stream()))
        return out.view(self.shape), ds.value

    def state_bytes(self) -> int:
        nb = C.c_size_t()
        _check(self.lib.lsb_state_bytes(self.h, C.byref(nb)))
        return nb.value

    def save_state(self):
        buf = self.torch.empty(self.state_bytes(), dtype=self.torch.uint8, device=self.device)
        _check(self.lib.lsb_save_state(self.h, C.c_void_p(buf.data_ptr()), self.stream()))
        return buf

    def load_state(self, buf):
        _check(self.lib.lsb_load_state(self.h, C.c_void_p(buf.data_ptr()), self.stream()))


class Refine:
    """Static refinement (BGK, FP64, ratio 2) on one GPU: lattice D2Q9, D3Q19
    or D3Q27; the coarse grid nx x ny (x nz), periodic, and a fine patch over
    the coarse nodes patch = (ia, ib, ja, jb[, ka, kb]); or nested patches, a
    list of such boxes (level 1 first, each in its parent level's node
    coordinates; two to four levels in all); or, with parents (one index per
    box: 0 for the coarse grid, else an earlier box counted from 1), a tree
    of up to 15 boxes.  Device memory is a torch
    uint8 tensor (the caller-owned workspace); calls run on torch's current
    stream."""

    def __init__(self, nx: int, ny: int, patch, tau_c: float, device="cuda:0", lattice: int = D2Q9, nz: int = 1,
                 max_extent=(0, 0, 0), max_inner_extent=(), parents=None):
        import torch
        self.torch = torch
        self.lib = load()
        self.device = torch.device(device)
        self.lattice = int(lattice)
        self.D, self.Q = (2, 9) if self.lattice == D2Q9 else (3, 19 if self.lattice == D3Q19 else 27)
        self.nx, self.ny, self.nz = int(nx), int(ny), (int(nz) if self.D == 3 else 1)
        boxes = [patch] if np.isscalar(patch[0]) else list(patch)
        self.boxes = []
        for bx in boxes:
            p = tuple(int(v) for v in bx) + (0, 0)
            self.boxes.append(p[:6] if self.D == 3 else p[:4] + (0, 0))
        self.levels = len(self.boxes) + 1
        self.parents = list(range(len(self.boxes))) if parents is None else [int(v) for v in parents]
        inner = ((C.c_int * 6) * (REF_MAX_LEVELS - 2))()
        for l, bx in enumerate(self.boxes[1:REF_MAX_LEVELS - 1] if parents is None else []):
            inner[l] = (C.c_int * 6)(*bx)
        mie = ((C.c_int * 3) * (REF_MAX_LEVELS - 2))()
        for l, e in enumerate(list(max_inner_extent)[:REF_MAX_LEVELS - 2]):
            mie[l] = (C.c_int * 3)(*[int(v) for v in e])
        self._cp = RefParams(self.lattice, self.nx, self.ny, self.nz, (C.c_int * 6)(*self.boxes[0]), float(tau_c),
                             (C.c_int * 3)(*[int(v) for v in max_extent]), self.levels if parents is None else 0,
                             inner, mie)
        self._sync_level1()
        h = C.c_void_p()
        if parents is None:
            _check(self.lib.lsb_ref_create(C.byref(self._cp), C.byref(h)))
        else:
            flat = [v for bx in self.boxes for v in bx]
            _check(self.lib.lsb_ref_create_tree(C.byref(self._cp), len(self.boxes),
                                                (C.c_int * len(self.parents))(*self.parents),
                                                (C.c_int * len(flat))(*flat), C.byref(h)))
        self.h = h
        nb = C.c_size_t()
        _check(self.lib.lsb_ref_workspace_bytes(self.h, C.byref(nb)))
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        _check(self.lib.lsb_ref_bind(self.h, C.c_void_p(self.ws.data_ptr()), nb.value))

    def _sync_level1(self):
        ia, ib, ja, jb, ka, kb = self.boxes[0]
        self.patch = self.boxes[0]
        self.mx, self.my, self.mz = 2 * (ib - ia), 2 * (jb - ja), 2 * (kb - ka)
        self.n_coarse = self.nx * self.ny * self.nz
        self.n_fine = (self.mx + 1) * (self.my + 1) * (self.mz + 1)

    def shape(self, level: int):
        """Nodes per axis (x, y, z) of a level."""
        if level == 0:
            return self.nx, self.ny, self.nz
        ia, ib, ja, jb, ka, kb = self.boxes[level - 1]
        return 2 * (ib - ia) + 1, 2 * (jb - ja) + 1, 2 * (kb - ka) + 1

    def n_level(self, level: int) -> int:
        return int(np.prod(self.shape(level)))

    def __del__(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.lsb_ref_destroy(self.h)
            self.h = None

    def stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _dev(self, a, n):
        t = self.torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)) if isinstance(a, np.ndarray) \
            else a.reshape(-1).to(self.torch.float64)
        assert t.numel() == n, (t.numel(), n)
        return t.to(self.device).contiguous()

    def init(self, rho_c, u_c, rho_f, u_f, *deeper):
        """rho [nodes], u [nodes, D] per level (numpy or torch): the coarse
        and level-1 arrays, then (rho, u) of each deeper level."""
        arrs = [rho_c, u_c, rho_f, u_f] + list(deeper)
        if len(arrs) != 2 * self.levels:
            raise ValueError("one (rho, u) pair per level expected")
        t = []
        for l in range(self.levels):
            n = self.n_level(l)
            t += [self._dev(arrs[2 * l], n), self._dev(arrs[2 * l + 1], self.D * n)]
        vp = C.c_void_p
        rho = (vp * self.levels)(*[t[2 * l].data_ptr() for l in range(self.levels)])
        u = (vp * self.levels)(*[t[2 * l + 1].data_ptr() for l in range(self.levels)])
        _check(self.lib.lsb_ref_init_levels(self.h, rho, u, self.stream()))
        self.torch.cuda.current_stream(self.device).synchronize()
        return self

    def step(self, n: int = 1):
        _check(self.lib.lsb_ref_step(self.h, int(n), self.stream()))
        return self

    def sensor(self, phi, d_ref: float, margin: int):
        """Patch box (6 ints) of the level-set sensor on the coarse level set
        phi [n_coarse] (numpy or torch); the current patch when no node is
        tagged."""
        t_phi = self._dev(phi, self.n_coarse)
        out = (C.c_int * 6)()
        _check(self.lib.lsb_ref_sensor(self.h, C.c_void_p(t_phi.data_ptr()), float(d_ref), int(margin), out,
                                       self.stream()))
        return tuple(out)

    def remesh(self, patch):
        """Re-mesh a two-level hierarchy onto patch (6 ints; ka, kb ignored in
        2D)."""
        p = (tuple(int(v) for v in patch) + (0, 0))[:6]
        _check(self.lib.lsb_ref_remesh(self.h, (C.c_int * 6)(*p), self.stream()))
        self.boxes[0] = p if self.D == 3 else p[:4] + (0, 0)
        self._sync_level1()
        return self

    def set_graphs(self, on: bool):
        """Coarse steps as HIP graph launches (default) or plain launches."""
        _check(self.lib.lsb_ref_set_graphs(self.h, 1 if on else 0))
        return self

    def sensor_levels(self, phi, d_ref: float, margins):
        """Boxes of every refined level (6 ints each, each in its parent's
        node coordinates) from the level-set sensor on the coarse level set
        phi [n_coarse], margins[l - 1] coarse nodes for level l; the current
        boxes when no node is tagged."""
        nl = self.levels - 1
        t_phi = self._dev(phi, self.n_coarse)
        out = (C.c_int * (6 * nl))()
        mg = (C.c_int * nl)(*[int(m) for m in margins])
        _check(self.lib.lsb_ref_sensor_levels(self.h, C.c_void_p(t_phi.data_ptr()), float(d_ref), mg, out,
                                              self.stream()))
        return [tuple(out[6 * l:6 * l + 6]) for l in range(nl)]

    def sensor_seeded(self, phi, d_ref: float, margin: int, seeds):
        """Boxes for a tree of root boxes (6 ints each) from the level-set
        sensor on the coarse level set phi [n_coarse]: tagged nodes go to
        their nearest seed (coarse nodes, (x, y[, z]) each), each seed's box
        grown by margin and clamped, boxes closer than one node merged."""
        sd = [tuple(int(v) for v in p) + (0,) * (3 - len(p)) for p in seeds]
        flat = [v for p in sd for v in p]
        t_phi = self._dev(phi, self.n_coarse)
        out = (C.c_int * (6 * len(sd)))()
        nb = C.c_int()
        _check(self.lib.lsb_ref_sensor_seeded(self.h, C.c_void_p(t_phi.data_ptr()), float(d_ref), int(margin), len(sd),
                                              (C.c_int * len(flat))(*flat), out, C.byref(nb), self.stream()))
        return [tuple(out[6 * k:6 * k + 6]) for k in range(nb.value)]

    def remesh_levels(self, boxes):
        """Re-mesh every refined level onto boxes (6 ints each, level 1
        first, each in its new parent's node coordinates), one box per
        refined grid (the seeded sensor returns fewer when boxes merge:
        that result needs a new tree)."""
        if len(boxes) != self.levels - 1:
            raise ValueError(f"{len(boxes)} boxes for {self.levels - 1} refined grids: the tree needs rebuilding")
        flat = []
        for bx in boxes:
            p = (tuple(int(v) for v in bx) + (0, 0))[:6]
            flat += list(p if self.D == 3 else p[:4] + (0, 0))
        _check(self.lib.lsb_ref_remesh_levels(self.h, (C.c_int * max(1, len(flat)))(*flat), len(boxes), self.stream()))
        self.boxes = [tuple(flat[6 * l:6 * l + 6]) for l in range(len(boxes))]
        self._sync_level1()
        return self

    def level(self, l: int, as_numpy=True):
        """Post-collision populations of level l, [Q][(nz,) ny, nx]."""
        t = self.torch
        sx, sy, sz = self.shape(l)
        f = t.empty(self.Q * sx * sy * sz, dtype=t.float64, device=self.device)
        _check(self.lib.lsb_ref_get_level(self.h, int(l), C.c_void_p(f.data_ptr()), self.stream()))
        f = f.reshape(self.Q, sy, sx) if self.D == 2 else f.reshape(self.Q, sz, sy, sx)
        return f.cpu().numpy() if as_numpy else f

    def populations(self, as_numpy=True):
        """Every level's post-collision populations, coarse first."""
        return tuple(self.level(l, as_numpy) for l in range(self.levels))


class TwoPhaseRefine:
    """The two-phase step on a two-level grid (include/lsb_refine2.h): a
    periodic coarse grid (params, coarse lattice units, each phase's BGK
    step) and one refined box over the coarse nodes box = (ia, ib, ja, jb[,
    ka, kb]) running the whole two-phase step at half spacing.  Device
    memory is a torch uint8 tensor (the caller-owned workspace); calls run
    on torch's current stream.  `fine` is a Sim view of the fine level (fine
    lattice units) for the queries."""

    def __init__(self, params: dict, box, device="cuda:0"):
        import torch
        self.torch = torch
        self.lib = load()
        self.p = dict(params)
        self.device = torch.device(device)
        self.D = 2 if self.p["lattice"] == D2Q9 else 3
        self.Q = {D2Q9: 9, D3Q19: 19, D3Q27: 27}[self.p["lattice"]]
        self.box = (tuple(int(v) for v in box) + (0, 0))[:6]
        self._cp = to_params(self.p)
        h = C.c_void_p()
        _check(self.lib.lsb_ref2_create(C.byref(self._cp), (C.c_int * 6)(*self.box), C.byref(h)))
        self.h = h
        nb = C.c_size_t()
        _check(self.lib.lsb_ref2_workspace_bytes(self.h, C.byref(nb)))
        self.workspace_bytes = nb.value
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        _check(self.lib.lsb_ref2_bind(self.h, C.c_void_p(self.ws.data_ptr()), nb.value))
        sh = (C.c_int * 3)()
        _check(self.lib.lsb_ref2_fine_shape(self.h, sh))
        fx, fy, fz = sh[0], sh[1], sh[2]
        self.fine_shape = (fz, fy, fx)
        self.coarse_shape = (self.p["nz"], self.p["ny"], self.p["nx"])
        self.n_coarse = self.p["nx"] * self.p["ny"] * self.p["nz"]
        self.n_fine = fx * fy * fz
        fp = dict(self.p, nx=fx, ny=fy, nz=fz, sigma=2.0 * self.p["sigma"],
                  tau=[2.0 * t - 0.5 for t in self.p["tau"]],
                  accel=[[0.5 * v for v in a] for a in self.p["accel"]])
        fh = C.c_void_p()
        _check(self.lib.lsb_ref2_fine(self.h, C.byref(fh)))
        self.fine = Sim._view(fh, fp, self, device)

    def __del__(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.lsb_ref2_destroy(self.h)
            self.h = None

    def stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _dev(self, a, n):
        t = self.torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)) if isinstance(a, np.ndarray) \
            else a.reshape(-1).to(self.torch.float64)
        assert t.numel() == n, (t.numel(), n)
        return t.to(self.device).contiguous()

    def init(self, phi_c, rho_c, u_c, phi_f, rho_f, u_f):
        """Coarse phi, rho [n_coarse] and u [n_coarse, 3]; fine phi (in fine
        cells), rho [n_fine] and u [n_fine, 3] (numpy or torch)."""
        nc, nf = self.n_coarse, self.n_fine
        t = [self._dev(phi_c, nc), self._dev(rho_c, nc), self._dev(u_c, 3 * nc),
             self._dev(phi_f, nf), self._dev(rho_f, nf), self._dev(u_f, 3 * nf)]
        _check(self.lib.lsb_ref2_init(self.h, *[C.c_void_p(x.data_ptr()) for x in t], self.stream()))
        self.torch.cuda.current_stream(self.device).synchronize()
        return self

    def step(self, n: int = 1):
        _check(self.lib.lsb_ref2_step(self.h, int(n), self.stream()))
        return self

    @property
    def nstep(self) -> int:
        return self.lib.lsb_ref2_step_count(self.h)

    @property
    def current_box(self):
        out = (C.c_int * 6)()
        _check(self.lib.lsb_ref2_get_box(self.h, out))
        return tuple(out)

    def sensor(self, d_ref: float):
        """The box (6 ints) that the level-set sensor moves the refined box to."""
        out = (C.c_int * 6)()
        _check(self.lib.lsb_ref2_sensor(self.h, float(d_ref), out, self.stream()))
        return tuple(out)

    def remesh(self, box):
        """Re-mesh onto a box of the same extents (6 ints; ka, kb ignored in 2D)."""
        b = (tuple(int(v) for v in box) + (0, 0))[:6]
        _check(self.lib.lsb_ref2_remesh(self.h, (C.c_int * 6)(*b), self.stream()))
        self.box = b
        return self

    def coarse(self, as_numpy=True):
        """(populations [Q, nz, ny, nx], phases [nz, ny, nx]) of the coarse grid
        (covered nodes hold the fine state restricted to the coarse level)."""
        t = self.torch
        pop = t.empty(self.Q * self.n_coarse, dtype=t.float64, device=self.device)
        ph = t.empty(self.n_coarse, dtype=t.uint8, device=self.device)
        _check(self.lib.lsb_ref2_get_coarse(self.h, C.c_void_p(pop.data_ptr()), C.c_void_p(ph.data_ptr()),
                                            self.stream()))
        pop, ph = pop.view((self.Q,) + self.coarse_shape), ph.view(self.coarse_shape)
        return (pop.cpu().numpy(), ph.cpu().numpy()) if as_numpy else (pop, ph)
