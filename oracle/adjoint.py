"""Differentiable FP64 CRM step in plain PyTorch (CPU autograd): the oracle of
the reverse-mode (adjoint) sweep.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product library.

The step is the same map as the C oracle's (``crm_oracle.c``), written again
with tensor operations so that autograd gives its exact vector-Jacobian
product:

* Sec. 2.5.1, BCE: Adami velocity u_s = 2 u_body - sum u_f W / sum W and the
  extrapolated stress with the hydrostatic correction (g - a_s);
* Sec. 2.2, F2: L_i = sum_j V_j (u_j - u_i) (x) grad_i W_ij, drho/dt = -rho tr L;
* Sec. 2.2, F3: du/dt = (1/rho_i) sum_j V_j (s_i + s_j) . grad_i W_ij + g plus the
  artificial viscosity of eqs. artificial_viscosity_* (approaching pairs repel);
* eq. stress_rate_jaumann: ds/dt = Om s - s Om + 2G (D - tr D/3 I) + b K tr D I;
* Sec. 2.3: explicit midpoint rule on [x, u, s, rho];
* Sec. 2.4: the four-step return mapping with mu(I), tau^n from s_n;
* Sec. 2.5.1: body force and torque from the stage-2 marker accelerations.

Integer decisions (neighbour lists and their rebuild schedule, Alg. 1 and 2)
are the C oracle's, recorded step by step and held fixed; where the map has a
branch (unilateral viscosity, the return-mapping cases, mu(I) cases) the
derivative is that of the branch the particle takes. The parameters E and nu
enter through G = E / (2 (1 + nu)), K = E / (3 (1 - 2 nu)) and c_s = sqrt(K / rho0);
each material row holds (mu_s, mu_2, cohesion).

Only the non-periodic, all-active form is covered (no active domains).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from oracle.oracle import Oracle

DT = torch.float64


def _W(r, h, kernel=0):
    """Cubic spline, support 2h, 3-D normalisation 1/(pi h^3) (Sec. 4.1); or
    the quintic Wendland kernel a (1 - q/2)^4 (2q + 1), a = 21/(16 pi h^3)."""
    q = r / h
    if kernel == 1:
        t = torch.clamp(1.0 - 0.5 * q, min=0.0)
        return 21.0 / (16.0 * math.pi * h ** 3) * t ** 4 * (2.0 * q + 1.0)
    s = 1.0 / (math.pi * h ** 3)
    w1 = s * (1.0 - 1.5 * q * q + 0.75 * q * q * q)
    t = torch.clamp(2.0 - q, min=0.0)
    w2 = s * 0.25 * t * t * t
    return torch.where(q < 1.0, w1, w2)


def _dWdr(r, h, kernel=0):
    q = r / h
    if kernel == 1:
        t = torch.clamp(1.0 - 0.5 * q, min=0.0)
        return -5.0 * 21.0 / (16.0 * math.pi * h ** 3) * q * t ** 3 / h
    s = 1.0 / (math.pi * h ** 4)
    d1 = s * (-3.0 * q + 2.25 * q * q)
    t = torch.clamp(2.0 - q, min=0.0)
    d2 = s * (-0.75 * t * t)
    return torch.where(q < 1.0, d1, d2)


def _sym(s):
    """(n, 6) Voigt (xx, yy, zz, xy, xz, yz) -> (n, 3, 3)."""
    return torch.stack([torch.stack([s[:, 0], s[:, 3], s[:, 4]], -1),
                        torch.stack([s[:, 3], s[:, 1], s[:, 5]], -1),
                        torch.stack([s[:, 4], s[:, 5], s[:, 2]], -1)], -2)


def _voigt(m):
    return torch.stack([m[:, 0, 0], m[:, 1, 1], m[:, 2, 2], m[:, 0, 1], m[:, 0, 2], m[:, 1, 2]], -1)


def _safe_sqrt(v):
    """sqrt with a zero derivative where the argument is 0 (the equivalent shear
    stress of an isotropic tensor)."""
    pos = v > 0.0
    return torch.where(pos, torch.sqrt(torch.where(pos, v, torch.ones_like(v))), torch.zeros_like(v))


def _quat_R(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


class Recording:
    """A run of the C oracle whose per-step neighbour lists are kept for the
    differentiable replay. Bodies keep the scene's poses and velocities (they
    are frozen during a run of steps, as in the library)."""

    def __init__(self, scene, n_steps, params=None, materials=None, nbr_mode="cells"):
        p = dict(scene.params if params is None else params)
        if p.get("active_domains", 0):
            raise ValueError("the differentiable replay covers runs without active domains")
        self.scene, self.params, self.n_steps = scene, p, int(n_steps)
        orc = Oracle(scene, nbr_mode=nbr_mode, params=p)
        if materials is not None:
            orc.set_materials(*materials)
        self.x_markers = None
        self.lists = []
        for _ in range(self.n_steps):
            orc.step(1)
            self.lists.append(orc.lists())
        self.x_markers = orc.positions()[scene.n_soil:]
        self.final = orc.state()
        self.forces = orc.forces()
        self.n = orc.n
        self.m = orc.mass


class DiffStep:
    """Differentiable replay of a recorded run."""

    def __init__(self, rec: Recording, materials=None):
        sc, p = rec.scene, rec.params
        self.rec, self.p = rec, p
        self.ns, self.n = sc.n_soil, rec.n
        self.h, self.dt, self.m = p["h"], p["dt"], rec.m
        self.rho0 = p["rho0"]
        self.g = torch.tensor(p["gravity"], dtype=DT)
        self.xi2 = (p["av_xi_over_h"] * p["h"]) ** 2
        self.av_mode = int(p["av_mode"])
        self.bulk = float(p["bulk_coeff"])
        self.kernel = int(p.get("kernel", 0))
        body = np.full(self.n, -1, dtype=np.int64)
        k = self.ns
        for b, B in enumerate(sc.bodies):
            body[k:k + B.markers.shape[0]] = b
            k += B.markers.shape[0]
        self.body = body
        self.nb = len(sc.bodies)
        # marker kinematics from the frozen body state (Sec. 2.5.1)
        xm = rec.x_markers
        ub = np.zeros((self.n - self.ns, 3))
        asb = np.zeros((self.n - self.ns, 3))
        lever = np.zeros((self.n - self.ns, 3))
        for i in range(self.n - self.ns):
            B = sc.bodies[body[self.ns + i]]
            r = xm[i] - np.asarray(B.pos, dtype=np.float64)
            W = np.asarray(B.angvel, dtype=np.float64)
            wr = np.cross(W, r)
            ub[i] = np.asarray(B.linvel, dtype=np.float64) + wr
            asb[i] = np.cross(W, wr)
            lever[i] = r
        self.x_mark = torch.tensor(xm, dtype=DT)
        self.u_body = torch.tensor(ub, dtype=DT)
        self.a_body = torch.tensor(asb, dtype=DT)
        self.lever = torch.tensor(lever, dtype=DT)
        self.mark_body = torch.tensor(body[self.ns:], dtype=torch.int64)
        if materials is None:
            self.mat = torch.zeros(self.ns, dtype=torch.int64)
        else:
            self.mat = torch.tensor(np.asarray(materials[1], dtype=np.int64))
        self._pairs = {}

    # --- pair sets of one step's lists -------------------------------------
    def pairs(self, k):
        if k in self._pairs:
            return self._pairs[k]
        proc, off, nbr = self.rec.lists[k]
        rows = np.repeat(proc.astype(np.int64), np.diff(off))
        cols = nbr.astype(np.int64)
        keep = rows != cols
        rows, cols = rows[keep], cols[keep]
        soil_row = rows < self.ns
        # soil rows: all neighbours; marker rows: soil neighbours only
        fr, fc = rows[soil_row], cols[soil_row]
        mr, mc = rows[~soil_row], cols[~soil_row]
        ms = mc < self.ns
        out = (torch.tensor(fr), torch.tensor(fc), torch.tensor(mr[ms]), torch.tensor(mc[ms]))
        self._pairs[k] = out
        return out

    # --- pieces of the step -------------------------------------------------
    def _grad(self, d):
        r = torch.sqrt((d * d).sum(-1))
        return r, (_dWdr(r, self.h, self.kernel) / r)[:, None] * d

    def bce(self, x, u, s, rho, mr, mc):
        """Marker velocity and stress (Sec. 2.5.1) for all markers."""
        nm = self.n - self.ns
        i = mr - self.ns
        d = x[mr] - x[mc]
        r = torch.sqrt((d * d).sum(-1))
        w = _W(r, self.h, self.kernel)
        sw = torch.zeros(nm, dtype=DT).index_add(0, i, w)
        su = torch.zeros(nm, 3, dtype=DT).index_add(0, i, u[mc] * w[:, None])
        ss = torch.zeros(nm, 6, dtype=DT).index_add(0, i, s[mc] * w[:, None])
        sr = torch.zeros(nm, 3, dtype=DT).index_add(0, i, (rho[mc] * w)[:, None] * d)
        has = sw > 0.0
        sws = torch.where(has, sw, torch.ones_like(sw))
        gd = ((self.g[None, :] - self.a_body) * sr).sum(-1)
        us = torch.where(has[:, None], 2.0 * self.u_body - su / sws[:, None], self.u_body)
        iso = torch.zeros(nm, 6, dtype=DT)
        iso[:, :3] = 1.0
        sg = torch.where(has[:, None], (ss - gd[:, None] * iso) / sws[:, None], torch.zeros_like(ss))
        return us, sg

    def _pair_acc(self, x, u, s, rho, I, J, cs):
        """Momentum terms of the pairs (I, J): (V_j / rho_i) (s_i + s_j) . gradW + Pi."""
        d = x[I] - x[J]
        r, gw = self._grad(d)
        Vj = self.m / rho[J]
        ss = _sym(s[I] + s[J])
        acc = (Vj / rho[I])[:, None] * torch.einsum("nab,nb->na", ss, gw)
        if self.av_mode:
            v = u[I] - u[J]
            vr = (v * d).sum(-1)
            rbar = 0.5 * (rho[I] + rho[J])
            f = self.p["av_gamma"] * self.h * cs * (self.m / rbar) * vr / (r * r + self.xi2)
            if self.av_mode == 2:
                f = torch.where(vr < 0.0, f, torch.zeros_like(f))
            acc = acc + f[:, None] * gw
        return acc, d, gw, Vj

    def rhs(self, x, u, s, rho, fr, fc, G, K, cs):
        """Rates of the soil particles (ids 0..ns-1; all are active here)."""
        ns = self.ns
        acc, d, gw, Vj = self._pair_acc(x, u, s, rho, fr, fc, cs)
        du_ = u[fc] - u[fr]
        Lp = Vj[:, None, None] * du_[:, :, None] * gw[:, None, :]
        L = torch.zeros(ns, 3, 3, dtype=DT).index_add(0, fr, Lp)
        a = torch.zeros(ns, 3, dtype=DT).index_add(0, fr, acc) + self.g[None, :]
        trD = L[:, 0, 0] + L[:, 1, 1] + L[:, 2, 2]
        D = 0.5 * (L + L.transpose(1, 2))
        Om = 0.5 * (L - L.transpose(1, 2))
        S = _sym(s[:ns])
        eye = torch.eye(3, dtype=DT)[None]
        R = Om @ S - S @ Om + 2.0 * G * D + (self.bulk * K - 2.0 * G / 3.0) * trD[:, None, None] * eye
        return u[:ns], a, _voigt(R), -rho[:ns] * trD

    def marker_forces(self, x, u, s, rho, mr, mc, cs):
        acc, _, _, _ = self._pair_acc(x, u, s, rho, mr, mc, cs)
        nm = self.n - self.ns
        a = torch.zeros(nm, 3, dtype=DT).index_add(0, mr - self.ns, acc)
        f = self.m * a
        F = torch.zeros(self.nb, 3, dtype=DT).index_add(0, self.mark_body, f)
        T = torch.zeros(self.nb, 3, dtype=DT).index_add(0, self.mark_body, torch.cross(self.lever, f, dim=-1))
        return F, T

    def return_map(self, st, sn, G, mat_tab):
        """Sec. 2.4 with the particle's material row (mu_s, mu_2, cohesion)."""
        mu_s, mu_2, coh = mat_tab[self.mat, 0], mat_tab[self.mat, 1], mat_tab[self.mat, 2]

        def p_tb(v):
            p = -(v[:, 0] + v[:, 1] + v[:, 2]) / 3.0
            t = v[:, :3] + p[:, None]
            dd = (t * t).sum(-1) + 2.0 * (v[:, 3:] * v[:, 3:]).sum(-1)
            return p, _safe_sqrt(0.5 * dd)

        ps, tbs = p_tb(st)
        pn, tbn = p_tb(sn)
        gd = (tbs - tbn) / (G * self.dt)
        gpos = gd > 0.0
        ppos = ps > 0.0
        ok = gpos & ppos
        gd_s = torch.where(ok, gd, torch.ones_like(gd))
        ps_s = torch.where(ok, ps, torch.ones_like(ps))
        I = gd_s * self.p["grain_d"] * torch.sqrt(self.rho0 / ps_s)
        mu_I = mu_s + (mu_2 - mu_s) / (1.0 + self.p["I0"] / I)
        mu = torch.where(gpos, torch.where(ppos, mu_I, mu_2), mu_s)
        tmax = torch.clamp(mu * ps + coh, min=0.0)
        tbs_s = torch.where(tbs > 0.0, tbs, torch.ones_like(tbs))
        f = tmax / tbs_s
        rr = torch.cat([-ps[:, None] + f[:, None] * (st[:, :3] + ps[:, None]), f[:, None] * st[:, 3:]], -1)
        out = torch.where((tbs <= tmax)[:, None], st, rr)
        cut = ps < -coh / mu_s
        return torch.where(cut[:, None], torch.zeros_like(out), out)

    def step(self, k, x, u, s, rho, G, K, cs, mat_tab):
        """Step k of the recording; (x, u, s, rho) are the soil state (ns rows).
        Returns the new soil state and the stage-2 body force and torque."""
        fr, fc, mr, mc = self.pairs(k)
        ns, dt = self.ns, self.dt
        rho_m = torch.full((self.n - ns,), self.rho0, dtype=DT)

        def full(xs, us, ss, rs, um, sm):
            return (torch.cat([xs, self.x_mark]), torch.cat([us, um]), torch.cat([ss, sm]), torch.cat([rs, rho_m]))

        zu = torch.zeros(self.n - ns, 3, dtype=DT)
        zs = torch.zeros(self.n - ns, 6, dtype=DT)
        X, U, S, R = full(x, u, s, rho, zu, zs)
        um, sm = self.bce(X, U, S, R, mr, mc)
        X, U, S, R = full(x, u, s, rho, um, sm)
        dx, du, ds, dr = self.rhs(X, U, S, R, fr, fc, G, K, cs)
        h2 = 0.5 * dt
        xm, uq, sq, rq = x + h2 * dx, u + h2 * du, s + h2 * ds, rho + h2 * dr
        X, U, S, R = full(xm, uq, sq, rq, zu, zs)
        um, sm = self.bce(X, U, S, R, mr, mc)
        X, U, S, R = full(xm, uq, sq, rq, um, sm)
        F, T = self.marker_forces(X, U, S, R, mr, mc, cs)
        dx, du, ds, dr = self.rhs(X, U, S, R, fr, fc, G, K, cs)
        s_star = s + dt * ds
        s_new = self.return_map(s_star, s, G, mat_tab)
        return x + dt * dx, u + dt * du, s_new, rho + dt * dr, F, T

    def run(self, x0, u0, s0, rho0, E, nu, mat_tab):
        """All recorded steps from the soil state (x0, u0, s0, rho0). Returns the
        final soil state and the per-step body forces and torques."""
        G = E / (2.0 * (1.0 + nu))
        K = E / (3.0 * (1.0 - 2.0 * nu))
        cs = torch.sqrt(K / self.rho0)
        x, u, s, rho = x0, u0, s0, rho0
        Fs, Ts = [], []
        for k in range(self.rec.n_steps):
            x, u, s, rho, F, T = self.step(k, x, u, s, rho, G, K, cs, mat_tab)
            Fs.append(F)
            Ts.append(T)
        return x, u, s, rho, torch.stack(Fs) if Fs else None, torch.stack(Ts) if Ts else None


def initial_state(scene):
    """Soil state of a scene in FP64 (positions as the scene holds them)."""
    ns = scene.n_soil
    x = np.asarray(scene.pos, dtype=np.float64)
    u = np.zeros((ns, 3)) if scene.vel is None else np.asarray(scene.vel, dtype=np.float64)
    s = np.zeros((ns, 6)) if scene.sigma is None else np.asarray(scene.sigma, dtype=np.float64)
    r = (np.full(ns, scene.params["rho0"]) if scene.rho is None else np.asarray(scene.rho, dtype=np.float64))
    return x, u, s, r


def material_table(params, materials=None):
    if materials is None:
        return np.array([[params["mu_s"], params["mu_2"], params["cohesion"]]], dtype=np.float64)
    return np.asarray(materials[0], dtype=np.float64).reshape(-1, 3)


def loss_weights(seed, ns, n_steps, nb):
    """Seeded random weights of a linear functional of the final soil state and
    of the per-step body forces and torques (the adjoint's seeds)."""
    rng = np.random.default_rng(seed)
    return dict(x=rng.normal(size=(ns, 3)), u=rng.normal(size=(ns, 3)), s=rng.normal(size=(ns, 6)),
                rho=rng.normal(size=ns), F=rng.normal(size=(n_steps, nb, 3)), T=rng.normal(size=(n_steps, nb, 3)))


def gradient(rec: Recording, weights, materials=None):
    """Value and gradient of L = sum w . y_K + sum_k (wF . F_k + wT . T_k) with
    respect to the initial soil state, E, nu and the material table."""
    sc, p = rec.scene, rec.params
    x0, u0, s0, r0 = (torch.tensor(a, dtype=DT, requires_grad=True) for a in initial_state(sc))
    E = torch.tensor(p["E"], dtype=DT, requires_grad=True)
    nu = torch.tensor(p["nu"], dtype=DT, requires_grad=True)
    tab = torch.tensor(material_table(p, materials), requires_grad=True)
    ds = DiffStep(rec, materials)
    x, u, s, rho, F, T = ds.run(x0, u0, s0, r0, E, nu, tab)
    w = {k: torch.tensor(v, dtype=DT) for k, v in weights.items()}
    L = (w["x"] * x).sum() + (w["u"] * u).sum() + (w["s"] * s).sum() + (w["rho"] * rho).sum()
    if F is not None and ds.nb:
        L = L + (w["F"] * F).sum() + (w["T"] * T).sum()
    L.backward()
    return dict(L=float(L.detach()), x=x0.grad.numpy(), u=u0.grad.numpy(), s=s0.grad.numpy(), rho=r0.grad.numpy(),
                E=float(E.grad), nu=float(nu.grad), mat=tab.grad.numpy(),
                final=dict(pos=x.detach().numpy(), vel=u.detach().numpy(), sigma=s.detach().numpy(),
                           rho=rho.detach().numpy()))


def functional(scene, n_steps, weights, params=None, materials=None, state=None, nbr_mode="cells"):
    """The same functional evaluated by the C oracle alone (for finite differences)."""
    p = dict(scene.params if params is None else params)
    orc = Oracle(scene, nbr_mode=nbr_mode, params=p)
    if materials is not None:
        orc.set_materials(*materials)
    if state is not None:
        ns = scene.n_soil
        st = orc.state()
        x, u, s, r = st["pos"], st["vel"], st["sigma"], st["rho"]
        x[:ns], u[:ns], s[:ns], r[:ns] = state
        orc.set_state(x, u, s, r)
    L = 0.0
    for k in range(n_steps):
        orc.step(1)
        if len(scene.bodies):
            F, T = orc.forces()
            L += float((weights["F"][k] * F).sum() + (weights["T"][k] * T).sum())
    st = orc.state()
    ns = scene.n_soil
    L += float((weights["x"] * st["pos"][:ns]).sum() + (weights["u"] * st["vel"][:ns]).sum()
               + (weights["s"] * st["sigma"][:ns]).sum() + (weights["rho"] * st["rho"][:ns]).sum())
    return L
