"""Python binding of libcrm (include/crm.h): argument marshalling only.

Every computation of the step runs in the HIP kernels of libcrm.so; this module
converts numpy arrays to the C ABI and back. PyTorch provides the device memory
(its caching allocator, through the allocator callbacks) and the stream.

There is no fallback: if libcrm.so has not been built, importing the binding
raises an ImportError.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # loads the HIP runtime that libcrm.so binds to

HERE = os.path.dirname(os.path.abspath(__file__))
# CRM_LIB_PATH selects another build of the same library (e.g. for A/B timing).
LIB_PATH = os.environ.get("CRM_LIB_PATH") or os.path.join(HERE, "libcrm.so")

CRM_ABI_VERSION = 4
STATUS = {0: "CRM_OK", -1: "CRM_E_INVALID", -2: "CRM_E_NOMEM", -3: "CRM_E_DEVICE",
          -4: "CRM_E_STATE", -5: "CRM_E_NONFINITE", -6: "CRM_E_UNSUPPORTED"}


class CrmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class crm_params(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("av_mode", C.c_uint32),
        ("dx", C.c_double), ("h", C.c_double), ("dt", C.c_double),
        ("gravity", C.c_double * 3),
        ("rho0", C.c_double), ("E", C.c_double), ("nu", C.c_double), ("mu_s", C.c_double),
        ("mu_2", C.c_double), ("I0", C.c_double), ("grain_d", C.c_double), ("cohesion", C.c_double),
        ("av_gamma", C.c_double), ("av_xi_over_h", C.c_double),
        ("domain_lo", C.c_double * 3), ("domain_hi", C.c_double * 3),
        ("ps_freq", C.c_uint32), ("active_domains", C.c_uint32),
        ("t_delay", C.c_double),
        ("grow_G", C.c_double), ("shrink_S", C.c_double),
        ("shrink_interval", C.c_uint32), ("pos_mode", C.c_uint32),
        ("bulk_coeff", C.c_double),
        ("kernel", C.c_uint32), ("activity_scan", C.c_uint32), ("skin", C.c_double),
        ("moved_cap", C.c_int64),
    ]


class crm_body_desc(C.Structure):
    _fields_ = [("n_markers", C.c_int64), ("marker_local", C.POINTER(C.c_float)),
                ("active_half", C.c_double * 3)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                          "python paper_2507_05643_amd/build.py")
    L = C.CDLL(LIB_PATH)
    vp, dp, fp = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_float)
    i32p, i64p, u32p, u8p = C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_uint32), C.POINTER(C.c_uint8)
    L.crm_init.restype = C.c_int
    L.crm_init.argtypes = [C.POINTER(crm_params), C.c_int64, dp, fp, fp, fp, C.c_int32,
                           C.POINTER(crm_body_desc), ALLOC_FN, FREE_FN, vp, vp, C.POINTER(vp)]
    L.crm_set_bodies.restype = C.c_int
    L.crm_set_bodies.argtypes = [vp, C.c_int32, dp, dp, dp, dp, dp, dp]
    L.crm_set_materials.restype = C.c_int
    L.crm_set_materials.argtypes = [vp, C.c_int32, dp, dp, dp, C.POINTER(C.c_uint16)]
    L.crm_step.restype = C.c_int
    L.crm_step.argtypes = [vp, C.c_int32]
    L.crm_step_noalloc.restype = C.c_int
    L.crm_step_noalloc.argtypes = [vp, C.c_int32]
    L.crm_record_forces.restype = C.c_int
    L.crm_record_forces.argtypes = [vp, dp, dp]
    L.crm_get_forces.restype = C.c_int
    L.crm_get_forces.argtypes = [vp, C.c_int32, dp, dp]
    L.crm_cosim_step.restype = C.c_int
    L.crm_cosim_step.argtypes = [vp, C.c_int32] + [vp] * 8   # raw addresses (see crm_cosim_step below)
    L.crm_get_state.restype = C.c_int
    L.crm_get_state.argtypes = [vp, dp, fp, fp, fp]
    L.crm_set_state.restype = C.c_int
    L.crm_set_state.argtypes = [vp, dp, fp, fp, fp]
    L.crm_get_counts.restype = C.c_int
    L.crm_get_counts.argtypes = [vp, i64p]
    L.crm_debug_export.restype = C.c_int
    L.crm_debug_export.argtypes = [vp, i32p, u32p, i32p, i64p, i32p, C.c_int64, u8p]
    L.crm_set_graph.restype = C.c_int
    L.crm_set_graph.argtypes = [vp, C.c_int32]
    L.crm_set_profiling.restype = C.c_int
    L.crm_set_profiling.argtypes = [vp, C.c_int32]
    L.crm_get_profile.restype = C.c_int
    L.crm_get_profile.argtypes = [vp, dp]
    L.crm_capacity_next.restype = C.c_int64
    L.crm_capacity_next.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_double, C.c_double, C.c_int64]
    L.crm_last_error.restype = C.c_char_p
    L.crm_last_error.argtypes = [vp]
    L.crm_destroy.restype = None
    L.crm_destroy.argtypes = [vp]
    L.crm_autotune.restype = C.c_int
    L.crm_autotune.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32)]
    L.crm_record.restype = C.c_int
    L.crm_record.argtypes = [vp, C.c_int32]
    L.crm_adjoint.restype = C.c_int
    L.crm_adjoint.argtypes = [vp, dp, fp, fp, fp, dp, dp, dp, fp, fp, fp, dp]
    L.crm_checkpoint_bytes.restype = C.c_int
    L.crm_checkpoint_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.crm_save_checkpoint.restype = C.c_int
    L.crm_save_checkpoint.argtypes = [vp, vp, C.c_size_t]
    L.crm_load_checkpoint.restype = C.c_int
    L.crm_load_checkpoint.argtypes = [vp, vp, C.c_size_t]
    return L


_lib = _load()

EXPORTED = ("crm_init", "crm_set_bodies", "crm_set_materials", "crm_step", "crm_get_forces", "crm_get_state",
            "crm_set_state", "crm_get_counts", "crm_debug_export", "crm_set_graph", "crm_set_profiling",
            "crm_get_profile", "crm_capacity_next", "crm_last_error", "crm_destroy", "crm_record",
            "crm_adjoint", "crm_autotune", "crm_cosim_step", "crm_checkpoint_bytes", "crm_save_checkpoint",
            "crm_load_checkpoint", "crm_step_noalloc", "crm_record_forces")

TILE_NONE, TILE_SMALL, TILE_LARGE = 0, 1, 2

PROFILE_CLASSES = ("rebuild", "place_markers", "bce_stage1", "soil_stage1", "bce_forces_stage2",
                   "soil_stage2", "body_reduce", "activity")


def lib():
    return _lib


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(C.POINTER(t))


def _check(ctx, st):
    if st != 0:
        raise CrmError(st, _lib.crm_last_error(ctx).decode())


def make_params(p: dict) -> crm_params:
    o = crm_params()
    o.abi_version = CRM_ABI_VERSION
    o.av_mode = int(p["av_mode"])
    o.dx, o.h, o.dt = float(p["dx"]), float(p["h"]), float(p["dt"])
    o.gravity[:] = [float(v) for v in p["gravity"]]
    for k in ("rho0", "E", "nu", "mu_s", "mu_2", "I0", "grain_d", "cohesion", "av_gamma",
              "av_xi_over_h", "t_delay", "grow_G", "shrink_S", "bulk_coeff"):
        setattr(o, k, float(p[k]))
    o.domain_lo[:] = [float(v) for v in p["domain_lo"]]
    o.domain_hi[:] = [float(v) for v in p["domain_hi"]]
    o.ps_freq = int(p["ps_freq"])
    o.active_domains = int(p["active_domains"])
    o.shrink_interval = int(p["shrink_interval"])
    o.pos_mode = int(p.get("pos_mode", 0))
    o.kernel = int(p.get("kernel", 0))
    o.skin = float(p.get("skin", 0.0))
    o.activity_scan = int(p.get("activity_scan", 0))
    o.moved_cap = int(p.get("moved_cap", 0))
    return o


class _TorchAllocator:
    """Allocator callbacks backed by torch's caching allocator."""

    def __init__(self, device: int):
        self.device = device

        def _alloc(nbytes, user, stream):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), self.device, stream or 0))
            except Exception:
                return None

        def _free(ptr, user, stream):
            try:
                torch.cuda.caching_allocator_delete(int(ptr))
            except Exception:
                pass

        self.alloc = ALLOC_FN(_alloc)
        self.free = FREE_FN(_free)


# ---- thin functions with the C names ----------------------------------------

def crm_init(params: dict, pos, vel=None, sigma=None, rho=None, bodies=(), device=None, stream=None,
             torch_allocator=True, allocator=None):
    """Create a context. bodies: sequence of (marker_local (m,3) float32, active_half (3,)).
    allocator: an object with ctypes callbacks .alloc (ALLOC_FN) and .free (FREE_FN)
    used in place of torch's caching allocator."""
    if not torch.cuda.is_available():
        raise RuntimeError("libcrm needs a HIP device")
    dev = torch.cuda.current_device() if device is None else int(device)
    torch.cuda.set_device(dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    P = make_params(params)
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    n = pos.shape[0]
    vel = None if vel is None else np.ascontiguousarray(vel, dtype=np.float32).reshape(n, 3)
    sigma = None if sigma is None else np.ascontiguousarray(sigma, dtype=np.float32).reshape(n, 6)
    rho = None if rho is None else np.ascontiguousarray(rho, dtype=np.float32).reshape(n)
    keep = []
    descs = (crm_body_desc * max(len(bodies), 1))()
    for b, (ml, half) in enumerate(bodies):
        ml = np.ascontiguousarray(ml, dtype=np.float32).reshape(-1, 3)
        keep.append(ml)
        descs[b].n_markers = ml.shape[0]
        descs[b].marker_local = ml.ctypes.data_as(C.POINTER(C.c_float))
        descs[b].active_half[:] = [float(v) for v in half]
    alloc = allocator if allocator is not None else (_TorchAllocator(dev) if torch_allocator else None)
    out = C.c_void_p()
    st = _lib.crm_init(C.byref(P), n, _ptr(pos, C.c_double), _ptr(vel, C.c_float), _ptr(sigma, C.c_float),
                       _ptr(rho, C.c_float), len(bodies), descs,
                       alloc.alloc if alloc else ALLOC_FN(), alloc.free if alloc else FREE_FN(),
                       None, C.c_void_p(stream), C.byref(out))
    _check(None, st)
    return out.value, alloc


def crm_set_bodies(ctx, pos, quat, linvel=None, angvel=None, linacc=None, angacc=None):
    arr = [None if a is None else np.ascontiguousarray(a, dtype=np.float64)
           for a in (pos, quat, linvel, angvel, linacc, angacc)]
    nb = 0 if arr[0] is None else arr[0].reshape(-1, 3).shape[0]
    _check(ctx, _lib.crm_set_bodies(ctx, nb, *[_ptr(a, C.c_double) for a in arr]))


def crm_set_materials(ctx, table, material):
    """table: (n_mat, 3) rows (mu_s, mu_2, cohesion); material: uint16 id per soil particle."""
    tab = np.ascontiguousarray(table, dtype=np.float64).reshape(-1, 3)
    cols = [np.ascontiguousarray(tab[:, k]) for k in range(3)]
    mat = np.ascontiguousarray(material, dtype=np.uint16)
    _check(ctx, _lib.crm_set_materials(ctx, tab.shape[0], *[_ptr(v, C.c_double) for v in cols],
                                       _ptr(mat, C.c_uint16)))


def crm_step(ctx, n_steps=1):
    _check(ctx, _lib.crm_step(ctx, int(n_steps)))


def crm_step_noalloc(ctx, n_steps=1):
    _check(ctx, _lib.crm_step_noalloc(ctx, int(n_steps)))


def crm_get_forces(ctx, nb):
    F = np.zeros((max(nb, 1), 3))
    T = np.zeros((max(nb, 1), 3))
    _check(ctx, _lib.crm_get_forces(ctx, nb, _ptr(F, C.c_double), _ptr(T, C.c_double)))
    return F[:nb], T[:nb]


def _addr(a):
    """Address of a float64 C-contiguous array (None for None), for the
    per-step exchange where ctypes pointer objects would dominate the call."""
    if a is None:
        return None
    if a.dtype != np.float64 or not a.flags.c_contiguous:
        raise TypeError("exchange arrays must be C-contiguous float64")
    return a.ctypes.data


def crm_cosim_step(ctx, nb, pos, quat, linvel, angvel, linacc, angacc, force, torque):
    """One exchange: body states in, one step, forces and torques out (into the
    given (nb, 3) float64 arrays)."""
    if pos.shape[0] != nb or force.shape[0] < nb or torque.shape[0] < nb:
        raise ValueError("array sizes differ from the body count")
    _check(ctx, _lib.crm_cosim_step(ctx, nb, _addr(pos), _addr(quat), _addr(linvel), _addr(angvel), _addr(linacc),
                                    _addr(angacc), _addr(force), _addr(torque)))


def crm_get_counts(ctx):
    out = np.zeros(10, dtype=np.int64)
    _check(ctx, _lib.crm_get_counts(ctx, _ptr(out, C.c_int64)))
    keys = ("n_total", "n_soil", "n_proc", "soil_rows", "marker_rows", "entries", "capacity",
            "steps", "cells", "rebuilds")
    return dict(zip(keys, (int(v) for v in out)))


def crm_get_state(ctx, n_total):
    pos = np.zeros((n_total, 3))
    vel = np.zeros((n_total, 3), dtype=np.float32)
    sig = np.zeros((n_total, 6), dtype=np.float32)
    rho = np.zeros(n_total, dtype=np.float32)
    _check(ctx, _lib.crm_get_state(ctx, _ptr(pos, C.c_double), _ptr(vel, C.c_float), _ptr(sig, C.c_float),
                                   _ptr(rho, C.c_float)))
    return dict(pos=pos, vel=vel, sigma=sig, rho=rho)


def crm_set_state(ctx, pos=None, vel=None, sigma=None, rho=None):
    a = [None if v is None else np.ascontiguousarray(v, dtype=t)
         for v, t in ((pos, np.float64), (vel, np.float32), (sigma, np.float32), (rho, np.float32))]
    _check(ctx, _lib.crm_set_state(ctx, _ptr(a[0], C.c_double), _ptr(a[1], C.c_float), _ptr(a[2], C.c_float),
                                   _ptr(a[3], C.c_float)))


def crm_debug_export(ctx):
    c = crm_get_counts(ctx)
    np_ = c["n_proc"]
    rows_n = c["soil_rows"] + c["marker_rows"]
    sid = np.zeros(max(np_, 1), dtype=np.int32)
    cs = np.zeros(c["cells"] + 1, dtype=np.uint32)
    rows = np.zeros(max(rows_n, 1), dtype=np.int32)
    off = np.zeros(rows_n + 1, dtype=np.int64)
    cap = max(c["entries"], 1)
    nbr = np.zeros(cap, dtype=np.int32)
    flags = np.zeros(c["n_total"], dtype=np.uint8)
    _check(ctx, _lib.crm_debug_export(ctx, _ptr(sid, C.c_int32), _ptr(cs, C.c_uint32), _ptr(rows, C.c_int32),
                                      _ptr(off, C.c_int64), _ptr(nbr, C.c_int32), cap, _ptr(flags, C.c_uint8)))
    return dict(sorted_ids=sid[:np_], cell_start=cs, rows=rows[:rows_n], off=off, nbr=nbr[: off[-1]],
                flags=flags)


def crm_autotune(ctx, config=-1):
    """config in (TILE_NONE, TILE_SMALL, TILE_LARGE) selects the soil-stage tile
    configuration; -1 times each on the current state and keeps the fastest.
    Returns the configuration in use."""
    out = C.c_int32(0)
    _check(ctx, _lib.crm_autotune(ctx, int(config), C.byref(out)))
    return int(out.value)


def crm_record(ctx, n_steps):
    _check(ctx, _lib.crm_record(ctx, int(n_steps)))


def crm_record_forces(ctx, n_steps, nb):
    """Per-step body forces and torques of the last crm_record: two (n_steps, nb, 3) arrays."""
    F = np.zeros((n_steps, max(nb, 1), 3))
    T = np.zeros((n_steps, max(nb, 1), 3))
    _check(ctx, _lib.crm_record_forces(ctx, _ptr(F, C.c_double), _ptr(T, C.c_double)))
    return F[:, :nb], T[:, :nb]


def crm_adjoint(ctx, n_soil, n_mat, lam_pos=None, lam_vel=None, lam_sigma=None, lam_rho=None, lam_force=None,
                lam_torque=None):
    """Vector-Jacobian product of the recorded run; returns dict(pos, vel, sigma, rho, params)
    with params = (dL/dE, dL/dnu, then dL/dmu_s, dL/dmu_2, dL/dcohesion per material)."""
    a = [None if v is None else np.ascontiguousarray(v, dtype=t)
         for v, t in ((lam_pos, np.float64), (lam_vel, np.float32), (lam_sigma, np.float32), (lam_rho, np.float32),
                      (lam_force, np.float64), (lam_torque, np.float64))]
    out = dict(pos=np.zeros((n_soil, 3)), vel=np.zeros((n_soil, 3), dtype=np.float32),
               sigma=np.zeros((n_soil, 6), dtype=np.float32), rho=np.zeros(n_soil, dtype=np.float32),
               params=np.zeros(2 + 3 * n_mat))
    _check(ctx, _lib.crm_adjoint(ctx, _ptr(a[0], C.c_double), _ptr(a[1], C.c_float), _ptr(a[2], C.c_float),
                                 _ptr(a[3], C.c_float), _ptr(a[4], C.c_double), _ptr(a[5], C.c_double),
                                 _ptr(out["pos"], C.c_double), _ptr(out["vel"], C.c_float),
                                 _ptr(out["sigma"], C.c_float), _ptr(out["rho"], C.c_float),
                                 _ptr(out["params"], C.c_double)))
    return out


def crm_save_checkpoint(ctx):
    """The context's checkpoint as bytes (see crm_save_checkpoint in crm.h)."""
    n = C.c_size_t(0)
    _check(ctx, _lib.crm_checkpoint_bytes(ctx, C.byref(n)))
    buf = (C.c_char * n.value)()
    _check(ctx, _lib.crm_save_checkpoint(ctx, C.cast(buf, C.c_void_p), n.value))
    return bytes(buf)


def crm_load_checkpoint(ctx, data):
    buf = C.create_string_buffer(bytes(data), len(data))
    _check(ctx, _lib.crm_load_checkpoint(ctx, C.cast(buf, C.c_void_p), len(data)))


def crm_set_graph(ctx, enable):
    _check(ctx, _lib.crm_set_graph(ctx, 1 if enable else 0))


PROF_CLASSES = 0x100


def crm_set_profiling(ctx, enable, classes=None):
    """enable: on/off; classes: names from PROFILE_CLASSES to time (default all)."""
    if not enable:
        v = 0
    elif classes is None:
        v = 1
    else:
        v = PROF_CLASSES
        for k in classes:
            v |= 1 << PROFILE_CLASSES.index(k)
    _check(ctx, _lib.crm_set_profiling(ctx, v))


def crm_get_profile(ctx):
    out = np.zeros(18)
    _check(ctx, _lib.crm_get_profile(ctx, _ptr(out, C.c_double)))
    at = [2 * i if i < 7 else 2 * i + 2 for i in range(len(PROFILE_CLASSES))]
    res = {k: dict(launches=int(out[a]), ms=float(out[a + 1])) for k, a in zip(PROFILE_CLASSES, at)}
    res["soil_pairs"] = int(out[14])
    res["marker_pairs"] = int(out[15])
    return res


def crm_capacity_next(cap, n, step, G=1.2, S=0.75, S_I=50):
    return int(_lib.crm_capacity_next(int(cap), int(n), int(step), float(G), float(S), int(S_I)))


def crm_last_error(ctx=None):
    return _lib.crm_last_error(ctx).decode()


def crm_destroy(ctx):
    _lib.crm_destroy(ctx)


# ---- convenience wrapper over a scene ----------------------------------------

class Simulation:
    """A libcrm context built from a scene (see ``scenes``)."""

    def __init__(self, scene, params=None, device=None, stream=None, torch_allocator=True, allocator=None):
        p = dict(scene.params if params is None else params)
        self.params = p
        self.n_soil = scene.n_soil
        self.nb = len(scene.bodies)
        bodies = [(b.markers, b.active_half) for b in scene.bodies]
        self.ctx, self._alloc = crm_init(p, scene.pos, scene.vel, scene.sigma, scene.rho, bodies,
                                         device=device, stream=stream, torch_allocator=torch_allocator,
                                         allocator=allocator)
        self.n_total = scene.n_total
        if self.nb:
            self.set_bodies(np.array([b.pos for b in scene.bodies]), np.array([b.quat for b in scene.bodies]),
                            np.array([b.linvel for b in scene.bodies]), np.array([b.angvel for b in scene.bodies]))

    def set_bodies(self, pos, quat, linvel=None, angvel=None, linacc=None, angacc=None):
        crm_set_bodies(self.ctx, pos, quat, linvel, angvel, linacc, angacc)

    def set_materials(self, table, material):
        crm_set_materials(self.ctx, table, material)
        self.n_mat = np.asarray(table).reshape(-1, 3).shape[0]

    def autotune(self, config=-1):
        return crm_autotune(self.ctx, config)

    def record(self, n):
        crm_record(self.ctx, n)
        self.rec_n = int(n)

    def record_forces(self):
        """Per-step body forces and torques of the last record: (n, nb, 3) each."""
        return crm_record_forces(self.ctx, self.rec_n, self.nb)

    def adjoint(self, **seeds):
        return crm_adjoint(self.ctx, self.n_soil, getattr(self, "n_mat", 1), **seeds)

    def step(self, n=1):
        crm_step(self.ctx, n)

    def forces(self):
        return crm_get_forces(self.ctx, self.nb)

    def cosim_step(self, pos, quat, linvel=None, angvel=None, linacc=None, angacc=None):
        """set_bodies + step(1) + forces() in one library call; returns views of
        (force, torque) buffers that the next call overwrites."""
        if not hasattr(self, "_xf"):
            self._xf = np.zeros((max(self.nb, 1), 3))
            self._xt = np.zeros((max(self.nb, 1), 3))
        crm_cosim_step(self.ctx, self.nb, pos, quat, linvel, angvel, linacc, angacc, self._xf, self._xt)
        return self._xf[:self.nb], self._xt[:self.nb]

    def state(self):
        return crm_get_state(self.ctx, self.n_total)

    def set_state(self, pos=None, vel=None, sigma=None, rho=None):
        crm_set_state(self.ctx, pos, vel, sigma, rho)

    def counts(self):
        return crm_get_counts(self.ctx)

    def export(self):
        return crm_debug_export(self.ctx)

    def save_checkpoint(self):
        return crm_save_checkpoint(self.ctx)

    def load_checkpoint(self, data):
        crm_load_checkpoint(self.ctx, data)

    def graph(self, enable=True):
        crm_set_graph(self.ctx, enable)

    def profiling(self, enable=True, classes=None):
        crm_set_profiling(self.ctx, enable, classes)

    def profile(self):
        return crm_get_profile(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            crm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- reverse mode as a torch.autograd.Function --------------------------------

class _Rollout(torch.autograd.Function):
    """forward: crm_record of n steps from the scene with the given material
    parameters and initial soil velocities; outputs the per-step body forces
    and torques (crm_record_forces) and the soil state at the end. backward:
    crm_adjoint with the outputs' gradients as seeds."""

    @staticmethod
    def forward(ctx, spec, E, nu, mu_s, mu_2, cohesion, vel0):
        scene, n_steps, device = spec
        p = dict(scene.params)
        for k, v in (("E", E), ("nu", nu), ("mu_s", mu_s), ("mu_2", mu_2), ("cohesion", cohesion)):
            p[k] = float(v)
        sim = Simulation(scene, params=p, device=device)
        try:
            if vel0 is not None:
                sim.set_state(vel=vel0.detach().to("cpu", torch.float32).numpy())
            sim.record(n_steps)
            F, T = sim.record_forces()
            st = sim.state()
        except Exception:
            sim.close()
            raise
        ctx.sim = sim
        ctx.n = scene.n_soil
        ctx.vel_like = vel0
        n = scene.n_soil
        outs = (torch.from_numpy(F.copy()), torch.from_numpy(T.copy()),
                torch.from_numpy(st["pos"][:n].copy()), torch.from_numpy(st["vel"][:n].copy()),
                torch.from_numpy(st["sigma"][:n].copy()), torch.from_numpy(st["rho"][:n].copy()))
        return outs

    @staticmethod
    def backward(ctx, gF, gT, gpos, gvel, gsig, grho):
        def npy(g, dt):
            return None if g is None else g.detach().to("cpu", dt).contiguous().numpy()
        sim = ctx.sim
        try:
            g = sim.adjoint(lam_pos=npy(gpos, torch.float64), lam_vel=npy(gvel, torch.float32),
                            lam_sigma=npy(gsig, torch.float32), lam_rho=npy(grho, torch.float32),
                            lam_force=npy(gF, torch.float64), lam_torque=npy(gT, torch.float64))
        finally:
            sim.close()
            ctx.sim = None
        prm = [torch.tensor(float(v), dtype=torch.float64) for v in g["params"][:5]]
        dvel = None
        if ctx.vel_like is not None:
            dvel = torch.from_numpy(g["vel"]).to(ctx.vel_like.device, ctx.vel_like.dtype)
        return (None, *prm, dvel)


def rollout(scene, n_steps, E, nu, mu_s, mu_2, cohesion, vel0=None, device=None):
    """Differentiable run of n_steps steps of `scene` (reverse mode of Sec. 2.3-2.5):
    returns (force, torque, pos, vel, sigma, rho) with force and torque the
    bodies' per-step values, shape (n_steps, nb, 3), and the soil state at the
    end. Gradients flow to the material parameters E, nu, mu_s, mu_2, cohesion
    (scalars or 0-d tensors; their values replace the scene's) and to the
    initial soil velocities vel0 ((n_soil, 3), None: the scene's). The run must
    not use active domains; the record keeps the state at every list rebuild
    (every ps_freq steps, the checkpoint interval of the reverse sweep)."""
    def t(v):
        return v if torch.is_tensor(v) else torch.tensor(float(v), dtype=torch.float64)
    return _Rollout.apply((scene, int(n_steps), device), t(E), t(nu), t(mu_s), t(mu_2), t(cohesion), vel0)
