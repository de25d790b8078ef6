"""ctypes wrapper of the FP64 CPU oracle (``crm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline of the benchmark, never by the product library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "crm_oracle.c")
LIB = os.path.join(HERE, "libcrm_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class OrcParams(C.Structure):
    _fields_ = [
        ("dx", C.c_double), ("h", C.c_double), ("dt", C.c_double),
        ("g", C.c_double * 3),
        ("rho0", C.c_double), ("E", C.c_double), ("nu", C.c_double), ("mu_s", C.c_double),
        ("mu_2", C.c_double), ("I0", C.c_double), ("grain_d", C.c_double), ("cohesion", C.c_double),
        ("av_gamma", C.c_double), ("av_xi_over_h", C.c_double),
        ("av_mode", C.c_int32), ("ps_freq", C.c_int32),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("periodic", C.c_int32 * 3),
        ("active_domains", C.c_int32),
        ("t_delay", C.c_double),
        ("grow_G", C.c_double), ("shrink_S", C.c_double),
        ("shrink_interval", C.c_int32),
        ("nbr_mode", C.c_int32),
        ("bulk_coeff", C.c_double),
        ("pos_mode", C.c_int32),
        ("kernel", C.c_int32),
    ]


def make_params(p: dict, nbr_mode: int = 0, periodic=(0, 0, 0)) -> OrcParams:
    o = OrcParams()
    o.dx, o.h, o.dt = p["dx"], p["h"], p["dt"]
    o.g[:] = list(p["gravity"])
    for k in ("rho0", "E", "nu", "mu_s", "mu_2", "I0", "grain_d", "cohesion",
              "av_gamma", "av_xi_over_h", "t_delay", "grow_G", "shrink_S", "bulk_coeff"):
        setattr(o, k, float(p[k]))
    o.av_mode = int(p["av_mode"])
    o.ps_freq = int(p["ps_freq"])
    o.lo[:] = list(p["domain_lo"])
    o.hi[:] = list(p["domain_hi"])
    o.periodic[:] = list(periodic)
    o.active_domains = int(p["active_domains"])
    o.shrink_interval = int(p["shrink_interval"])
    o.nbr_mode = int(nbr_mode)
    o.pos_mode = int(p.get("pos_mode", 0))
    o.kernel = int(p.get("kernel", 0))
    return o


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        i64p = C.POINTER(C.c_int64)
        i32p = C.POINTER(C.c_int32)
        u8p = C.POINTER(C.c_uint8)
        pp = C.POINTER(OrcParams)
        L.orc_W.restype = C.c_double
        L.orc_W.argtypes = [C.c_double, C.c_double]
        L.orc_dWdr.restype = C.c_double
        L.orc_dWdr.argtypes = [C.c_double, C.c_double]
        for name in ("orc_W_wendland", "orc_dWdr_wendland"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_double, C.c_double]
        L.orc_mu_I.restype = C.c_double
        L.orc_mu_I.argtypes = [pp, C.c_double, C.c_double]
        L.orc_return_map.restype = C.c_int
        L.orc_return_map.argtypes = [pp, dp, dp, dp]
        L.orc_capacity_next.restype = C.c_int64
        L.orc_capacity_next.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_double, C.c_double, C.c_int64]
        L.orc_neighbors_brute.restype = C.c_int64
        L.orc_neighbors_brute.argtypes = [pp, C.c_int64, i32p, dp, i64p, i32p, C.c_int64]
        L.orc_neighbors_cells.restype = C.c_int64
        L.orc_neighbors_cells.argtypes = [pp, C.c_int64, i32p, dp, i64p, i32p, C.c_int64]
        L.orc_grid_dims.restype = None
        L.orc_grid_dims.argtypes = [pp, i64p, dp]
        L.orc_sort_cells.restype = None
        L.orc_sort_cells.argtypes = [pp, C.c_int64, i32p, dp, i32p, i64p, C.c_int64, i64p, i64p]
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [pp, C.c_int64, dp, dp, dp, dp, C.c_int32, i64p, dp, dp]
        L.orc_destroy.restype = None
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_materials.restype = None
        L.orc_set_materials.argtypes = [C.c_void_p, C.c_int32, dp, i32p]
        L.orc_set_bodies.restype = None
        L.orc_set_bodies.argtypes = [C.c_void_p, C.c_int32, dp, dp, dp, dp, dp, dp]
        L.orc_step.restype = C.c_int
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_eval_rhs.restype = C.c_int
        L.orc_eval_rhs.argtypes = [C.c_void_p, dp, dp, dp, dp, dp, dp]
        L.orc_fluid_acc_from_body.restype = None
        L.orc_fluid_acc_from_body.argtypes = [C.c_void_p, C.c_int32, dp]
        for name in ("orc_n", "orc_n_proc", "orc_nbr_total", "orc_capacity", "orc_step_count"):
            getattr(L, name).restype = C.c_int64
            getattr(L, name).argtypes = [C.c_void_p]
        L.orc_mass.restype = C.c_double
        L.orc_mass.argtypes = [C.c_void_p]
        L.orc_get_state.restype = None
        L.orc_get_state.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_set_state.restype = None
        L.orc_set_state.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_get_forces.restype = None
        L.orc_get_forces.argtypes = [C.c_void_p, dp, dp]
        L.orc_return_map_ex.restype = C.c_int
        L.orc_return_map_ex.argtypes = [pp, dp, dp, dp, C.POINTER(C.c_int)]
        L.orc_get_branches.restype = None
        L.orc_get_branches.argtypes = [C.c_void_p, C.POINTER(C.c_int8), C.POINTER(C.c_int8)]
        L.orc_to_rep.restype = None
        L.orc_to_rep.argtypes = [pp, dp, i64p, dp]
        L.orc_get_flags.restype = None
        L.orc_get_flags.argtypes = [C.c_void_p, u8p]
        L.orc_get_lists.restype = None
        L.orc_get_lists.argtypes = [C.c_void_p, i32p, i64p, i32p]
        L.orc_positions.restype = None
        L.orc_positions.argtypes = [C.c_void_p, dp]
        L.orc_threads.restype = C.c_int
        L.orc_threads.argtypes = []
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t)) if a is not None else None


def _d(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def W(r, h, kernel=0):
    """Smoothing kernel: 0 cubic spline, 1 quintic Wendland."""
    f = lib().orc_W_wendland if kernel == 1 else lib().orc_W
    return f(float(r), float(h))


def dWdr(r, h, kernel=0):
    f = lib().orc_dWdr_wendland if kernel == 1 else lib().orc_dWdr
    return f(float(r), float(h))


def return_map(params: dict, s_star, s_n):
    P = make_params(params)
    a = np.ascontiguousarray(s_star, dtype=np.float64)
    b = np.ascontiguousarray(s_n, dtype=np.float64)
    out = np.zeros(6)
    br = lib().orc_return_map(C.byref(P), _p(a, C.c_double), _p(b, C.c_double), _p(out, C.c_double))
    return out, br


def return_map_ex(params: dict, s_star, s_n):
    """(corrected stress, branch, mu(I) case) of the return mapping; case 0: mu_s
    (no shear-rate increase), 1: mu_2 (p* <= 0), 2: the interior formula,
    -1: cut off at step 1."""
    P = make_params(params)
    a = np.ascontiguousarray(s_star, dtype=np.float64)
    b = np.ascontiguousarray(s_n, dtype=np.float64)
    out = np.zeros(6)
    mc = C.c_int(0)
    br = lib().orc_return_map_ex(C.byref(P), _p(a, C.c_double), _p(b, C.c_double), _p(out, C.c_double),
                                 C.byref(mc))
    return out, br, mc.value


def to_rep(params: dict, x):
    """Stored form of the position x (3,): (integer cell (3,), offset (3,)) for
    pos_mode 1, (0, FP32 coordinate) for pos_mode 0."""
    P = make_params(params)
    xx = np.ascontiguousarray(x, dtype=np.float64).reshape(3)
    c = np.zeros(3, dtype=np.int64)
    o = np.zeros(3)
    lib().orc_to_rep(C.byref(P), _p(xx, C.c_double), _p(c, C.c_int64), _p(o, C.c_double))
    return c, o


def mu_I(params: dict, gamma_dot, p):
    P = make_params(params)
    return lib().orc_mu_I(C.byref(P), float(gamma_dot), float(p))


def capacity_next(cap, n_ae, step, G=1.2, S=0.75, S_I=50):
    return lib().orc_capacity_next(int(cap), int(n_ae), int(step), float(G), float(S), int(S_I))


def neighbors(params: dict, x, ids=None, mode="brute", periodic=(0, 0, 0)):
    """Neighbour CSR of the set `ids` (default: all). Returns (off, nbr) with
    entries as particle ids in ascending order."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    n = x.shape[0]
    ids = np.arange(n, dtype=np.int32) if ids is None else np.ascontiguousarray(ids, dtype=np.int32)
    P = make_params(params, nbr_mode=1 if mode == "cells" else 0, periodic=periodic)
    off = np.zeros(ids.size + 1, dtype=np.int64)
    cap = 80 * (ids.size + 1)
    f = lib().orc_neighbors_cells if mode == "cells" else lib().orc_neighbors_brute
    while True:
        nbr = np.zeros(cap, dtype=np.int32)
        r = f(C.byref(P), ids.size, _p(ids, C.c_int32), _p(x, C.c_double), _p(off, C.c_int64),
              _p(nbr, C.c_int32), cap)
        if r >= 0:
            return off, nbr[:r].copy()
        cap *= 2


def grid_dims(params: dict):
    P = make_params(params)
    dims = np.zeros(3, dtype=np.int64)
    inv = np.zeros(1)
    lib().orc_grid_dims(C.byref(P), _p(dims, C.c_int64), _p(inv, C.c_double))
    return dims, float(inv[0])


def sort_cells(params: dict, x, ids=None):
    """(sorted_ids, sorted_keys, cell_start, cell_end) of Sec. 4.1 steps 1-3."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    ids = np.arange(x.shape[0], dtype=np.int32) if ids is None else np.ascontiguousarray(ids, dtype=np.int32)
    dims, _ = grid_dims(params)
    M = int(np.prod(dims))
    P = make_params(params)
    sid = np.zeros(ids.size, dtype=np.int32)
    skey = np.zeros(ids.size, dtype=np.int64)
    cs = np.zeros(M, dtype=np.int64)
    ce = np.zeros(M, dtype=np.int64)
    lib().orc_sort_cells(C.byref(P), ids.size, _p(ids, C.c_int32), _p(x, C.c_double),
                         _p(sid, C.c_int32), _p(skey, C.c_int64), M, _p(cs, C.c_int64), _p(ce, C.c_int64))
    return sid, skey, cs, ce


class Oracle:
    """FP64 oracle context over a scene (soil particles first, then the markers
    of each body in body order)."""

    def __init__(self, scene, nbr_mode="brute", periodic=(0, 0, 0), params=None):
        L = lib()
        p = dict(scene.params if params is None else params)
        self.params = p
        self.P = make_params(p, nbr_mode=1 if nbr_mode == "cells" else 0, periodic=periodic)
        pos = _d(scene.pos)
        vel = _d(scene.vel)
        sig = _d(scene.sigma)
        rho = _d(scene.rho)
        nb = len(scene.bodies)
        nm = np.array([b.markers.shape[0] for b in scene.bodies] or [0], dtype=np.int64)
        ml = (np.concatenate([b.markers for b in scene.bodies]).astype(np.float64)
              if nb else np.zeros((1, 3)))
        half = (np.array([b.active_half for b in scene.bodies], dtype=np.float64)
                if nb else np.zeros((1, 3)))
        self._keep = (pos, vel, sig, rho, nm, ml, half)
        dp = C.c_double
        self.ctx = L.orc_create(C.byref(self.P), scene.n_soil, _p(pos, dp), _p(vel, dp), _p(sig, dp),
                                _p(rho, dp), nb, _p(nm, C.c_int64), _p(ml, dp), _p(half, dp))
        self.n_soil = scene.n_soil
        self.nb = nb
        self.n = L.orc_n(self.ctx)
        if nb:
            self.set_bodies(np.array([b.pos for b in scene.bodies]), np.array([b.quat for b in scene.bodies]),
                            np.array([b.linvel for b in scene.bodies]), np.array([b.angvel for b in scene.bodies]))

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                lib().orc_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    def set_bodies(self, pos, quat, linvel=None, angvel=None, linacc=None, angacc=None):
        dp = C.c_double
        a = [_d(v) for v in (pos, quat, linvel, angvel, linacc, angacc)]
        lib().orc_set_bodies(self.ctx, self.nb, *[_p(v, dp) for v in a])

    def set_materials(self, table, material):
        """table: (n_mat, 3) rows (mu_s, mu_2, cohesion); material: id per soil particle."""
        tab = np.ascontiguousarray(table, dtype=np.float64).reshape(-1, 3)
        mat = np.ascontiguousarray(material, dtype=np.int32)
        lib().orc_set_materials(self.ctx, tab.shape[0], _p(tab, C.c_double), _p(mat, C.c_int32))

    def step(self, n=1):
        r = lib().orc_step(self.ctx, int(n))
        if r:
            raise RuntimeError("oracle step failed")

    def state(self):
        n = self.n
        x, u, s, r = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 6)), np.zeros(n)
        dp = C.c_double
        lib().orc_get_state(self.ctx, _p(x, dp), _p(u, dp), _p(s, dp), _p(r, dp))
        return dict(pos=x, vel=u, sigma=s, rho=r)

    def set_state(self, pos=None, vel=None, sigma=None, rho=None):
        dp = C.c_double
        a = [_d(v) for v in (pos, vel, sigma, rho)]
        lib().orc_set_state(self.ctx, *[_p(v, dp) for v in a])

    def forces(self):
        F, T = np.zeros((max(self.nb, 1), 3)), np.zeros((max(self.nb, 1), 3))
        lib().orc_get_forces(self.ctx, _p(F, C.c_double), _p(T, C.c_double))
        return F[: self.nb], T[: self.nb]

    def flags(self):
        f = np.zeros(self.n, dtype=np.uint8)
        lib().orc_get_flags(self.ctx, _p(f, C.c_uint8))
        return f

    def branches(self):
        """Per particle, the last step's return-mapping branch (0 not updated,
        1 tension cut-off, 3 admissible, 4 radial return) and mu(I) case
        (-1 cut off or not updated, 0 mu_s, 1 mu_2, 2 interior formula)."""
        br = np.zeros(self.n, dtype=np.int8)
        mc = np.zeros(self.n, dtype=np.int8)
        lib().orc_get_branches(self.ctx, _p(br, C.c_int8), _p(mc, C.c_int8))
        return br, mc

    def lists(self):
        L = lib()
        npr = L.orc_n_proc(self.ctx)
        tot = L.orc_nbr_total(self.ctx)
        proc = np.zeros(npr, dtype=np.int32)
        off = np.zeros(npr + 1, dtype=np.int64)
        nbr = np.zeros(max(tot, 1), dtype=np.int32)
        L.orc_get_lists(self.ctx, _p(proc, C.c_int32), _p(off, C.c_int64), _p(nbr, C.c_int32))
        return proc, off, nbr[:tot]

    def positions(self):
        x = np.zeros((self.n, 3))
        lib().orc_positions(self.ctx, _p(x, C.c_double))
        return x

    def eval_rhs(self):
        n = self.n
        out = dict(drho=np.zeros(n), du=np.zeros((n, 3)), ds=np.zeros((n, 6)),
                   mu=np.zeros((n, 3)), ms=np.zeros((n, 6)), mas=np.zeros((n, 3)))
        dp = C.c_double
        r = lib().orc_eval_rhs(self.ctx, *[_p(out[k], dp) for k in ("drho", "du", "ds", "mu", "ms", "mas")])
        if r:
            raise RuntimeError("oracle rhs failed")
        return out

    def fluid_acc_from_body(self, b):
        out = np.zeros((self.n, 3))
        lib().orc_fluid_acc_from_body(self.ctx, int(b), _p(out, C.c_double))
        return out

    @property
    def capacity(self):
        return lib().orc_capacity(self.ctx)

    @property
    def n_proc(self):
        return lib().orc_n_proc(self.ctx)

    @property
    def mass(self):
        return lib().orc_mass(self.ctx)

    @staticmethod
    def threads():
        return lib().orc_threads()
