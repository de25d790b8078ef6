"""Pins of the oracle's BCE extrapolation on moving, accelerating bodies
(Sec. 2.5.1: Adami velocity with the no-slip correction, and the stress
extrapolation with its (g - a_s) term).

The stress formula reproduces a linear isotropic field exactly when the field
is the hydrostatic one of the marker's own frame: with
sigma_f = rho0 ((g - a_s) . (x_top - x_f)) I around a marker of acceleration
a_s, every neighbour set gives sigma_s = rho0 ((g - a_s) . (x_top - x_s)) I.
A wrong sign of a_s, a_s left out, or a wrong composition of the rigid-body
acceleration a_s = A + alpha x r + w x (w x r) breaks the equality. Each body
here carries one marker, at a lever arm r from its origin, inside its own soil
block with its own field; a uniform soil velocity u0 gives the no-slip value
u_s = 2 (V + w x r) - u0 exactly.
"""
import numpy as np

from oracle.oracle import Oracle
from paper_2507_05643_amd import scenes
from paper_2507_05643_amd.scenes import Body, Scene

RHO0 = 1700.0
G_VEC = np.array([0.0, 0.0, -9.81])

# (linear acceleration A, angular acceleration alpha, angular velocity w, lever arm r)
CASES = [
    (np.array([1.5, -2.0, 3.5]), np.zeros(3), np.zeros(3), np.array([0.002, 0.001, -0.003])),
    (np.zeros(3), np.zeros(3), np.array([0.0, 4.0, 0.0]), np.array([0.03, 0.0, 0.01])),
    (np.array([0.2, 0.0, -1.0]), np.array([0.0, 0.0, 30.0]), np.array([1.0, -2.0, 0.5]),
     np.array([-0.02, 0.015, 0.01])),
]


def _scene():
    dx = 0.01
    blocks, bodies, fields = [], [], []
    for b, (A, al, w, r) in enumerate(CASES):
        origin = np.array([0.3 * b, 0.0, 0.0])
        p = scenes.lattice(6, 6, 6, dx, seed=b).astype(np.float64) + origin
        blocks.append(p)
        xs = origin + np.array([0.03, 0.03, 0.03])          # the marker, inside the block
        X = xs - r
        bodies.append(Body(markers=np.asarray([r], dtype=np.float32), pos=tuple(X)))
    pos = np.concatenate(blocks).astype(np.float32)
    params = dict(scenes.DEFAULT_PARAMS, dx=dx, h=1.2 * dx, domain_lo=(-0.1, -0.1, -0.1),
                  domain_hi=(1.0, 0.2, 0.2))
    return Scene("moving markers", params, pos, bodies=bodies)


def test_stress_and_velocity_extrapolation_on_accelerating_bodies():
    sc = _scene()
    ns = sc.n_soil
    u0 = np.array([0.05, -0.02, 0.01])
    X = np.array([b.pos for b in sc.bodies])
    V = np.array([[0.1, 0.0, -0.2], [0.0, 0.3, 0.0], [-0.1, 0.05, 0.0]])
    lin_acc = np.array([c[0] for c in CASES])
    ang_acc = np.array([c[1] for c in CASES])
    ang_vel = np.array([c[2] for c in CASES])
    o = Oracle(sc)
    o.set_bodies(X, np.tile([1.0, 0.0, 0.0, 0.0], (3, 1)), V, ang_vel, lin_acc, ang_acc)
    xm = o.positions()[ns:]
    x_soil = sc.pos.astype(np.float64)
    # per block, the hydrostatic field of its marker's frame
    x_top = np.array([0.0, 0.0, 0.2])
    sig = np.zeros((ns, 6))
    a_s = np.zeros((3, 3))
    for b, (A, al, w, r) in enumerate(CASES):
        rr = xm[b] - X[b]
        assert np.allclose(rr, r.astype(np.float32), atol=1e-9)
        a_s[b] = A + np.cross(al, rr) + np.cross(w, np.cross(w, rr))
        blk = slice(216 * b, 216 * (b + 1))
        phi = RHO0 * ((G_VEC - a_s[b]) @ (x_top[:, None] - x_soil[blk].T))
        sig[blk, 0] = sig[blk, 1] = sig[blk, 2] = phi
    o.set_state(vel=np.tile(u0, (ns, 1)), sigma=sig)
    r = o.eval_rhs()
    ms, mu = r["ms"][ns:], r["mu"][ns:]
    for b in range(3):
        want = RHO0 * ((G_VEC - a_s[b]) @ (x_top - xm[b]))
        scale = RHO0 * 9.81 * 0.2
        assert abs(ms[b, 0] - want) <= 1e-12 * scale, (b, ms[b], want)
        assert abs(ms[b, 1] - want) <= 1e-12 * scale and abs(ms[b, 2] - want) <= 1e-12 * scale
        assert np.abs(ms[b, 3:]).max() <= 1e-12 * scale
        ub = V[b] + np.cross(ang_vel[b], xm[b] - X[b])
        assert np.abs(mu[b] - (2.0 * ub - u0)).max() <= 1e-14
    # the gravity-only field (a_s ignored) is off by far more than the tolerance
    b = 0
    wrong = RHO0 * (G_VEC @ (x_top - xm[b]))
    assert abs(ms[b, 0] - wrong) > 1e-3 * RHO0 * 9.81 * 0.2
