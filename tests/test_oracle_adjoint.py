"""Pins of the adjoint's oracle (the FP64 autograd replay of ``oracle/adjoint.py``).

1. The replay is the same map as the C oracle: after several steps (with a list
   rebuild inside) the states and body forces agree to FP64 rounding.
2. Its gradient is the derivative of the C oracle's map: directional
   derivatives of a linear functional of the final state and of the per-step
   body forces match central differences of the C oracle alone, for every
   field of the initial state, E, nu and a material's mu_s, with plastic flow
   and unilateral viscosity on. The step is smooth away from branch switches
   (tension cut-off, yield, viscosity switch); a step of 1e-4 of each field's
   scale crosses none of them on this workload.
"""
import dataclasses

import numpy as np
import pytest

from oracle import adjoint as A
from oracle.oracle import Oracle
from paper_2507_05643_amd import scenes

K = 4


@pytest.fixture(scope="module", params=[0, 1], ids=["cubic", "wendland"])
def setup(request):
    sc = scenes.column(seed=0, n=8, ps_freq=2)
    sc.params["kernel"] = request.param
    o = Oracle(sc, nbr_mode="cells")
    o.step(30)
    st = o.state()
    ns = sc.n_soil
    # warm start: a settling column with non-zero velocity and stress
    sc = dataclasses.replace(sc, pos=st["pos"][:ns].copy(), vel=st["vel"][:ns].copy(),
                             sigma=st["sigma"][:ns].copy(), rho=st["rho"][:ns].copy())
    rec = A.Recording(sc, K)
    w = A.loss_weights(5, ns, K, len(sc.bodies))
    g = A.gradient(rec, w)
    return sc, rec, w, g


def test_replay_equals_c_oracle(setup):
    sc, rec, w, g = setup
    ns = sc.n_soil
    for k in ("pos", "vel", "sigma", "rho"):
        a, b = g["final"][k], rec.final[k][:ns]
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max(), k
    assert abs(g["L"] - A.functional(sc, K, w)) <= 1e-12 * abs(g["L"])


def _check(fd, ad, tol=1e-5):
    assert abs(fd - ad) <= tol * abs(ad), (fd, ad)


@pytest.mark.parametrize("field", ["x", "u", "s", "rho"])
def test_state_gradient_matches_central_differences(setup, field):
    sc, rec, w, g = setup
    x0, u0, s0, r0 = A.initial_state(sc)
    scale = dict(x=1e-5, u=1e-3 * np.abs(u0).max(), s=1e-3 * np.abs(s0).max(), rho=1.7)[field]
    i = ("x", "u", "s", "rho").index(field)
    d = np.random.default_rng(1 + i).normal(size=(x0, u0, s0, r0)[i].shape)
    eps = 1e-4 * scale

    def L_at(sgn):
        st = [x0.copy(), u0.copy(), s0.copy(), r0.copy()]
        st[i] = st[i] + sgn * eps * d
        return A.functional(sc, K, w, state=tuple(st))

    _check((L_at(1) - L_at(-1)) / (2 * eps), float((g[field] * d).sum()))


@pytest.mark.parametrize("name", ["E", "nu"])
def test_modulus_gradient_matches_central_differences(setup, name):
    sc, rec, w, g = setup
    p = sc.params
    eps = 1e-6 * p[name]

    def L_at(sgn):
        q = dict(p)
        q[name] = p[name] + sgn * eps
        return A.functional(sc, K, w, params=q)

    _check((L_at(1) - L_at(-1)) / (2 * eps), g[name])


def test_friction_gradient_matches_central_differences(setup):
    sc, rec, w, g = setup
    p = sc.params
    mat = np.zeros(sc.n_soil, dtype=np.int32)
    eps = 1e-6 * p["mu_s"]

    def L_at(sgn):
        tab = np.array([[p["mu_s"] + sgn * eps, p["mu_2"], p["cohesion"]]])
        return A.functional(sc, K, w, materials=(tab, mat))

    fd = (L_at(1) - L_at(-1)) / (2 * eps)
    assert abs(g["mat"][0, 0]) > 0.0      # plastic flow is active on this workload
    _check(fd, g["mat"][0, 0], tol=1e-4)


@pytest.fixture(scope="module")
def rate_setup():
    """A warm column with rate-dependent friction and cohesion (mu_s 0.7,
    mu_2 0.8, I0 0.08, d 3 mm, c = 100 Pa: the derivative in c is taken at
    c_0 = 100 Pa, where a relative step is well defined)."""
    sc = scenes.column(seed=4, n=8, ps_freq=2)
    sc.params.update(mu_s=0.7, mu_2=0.8, I0=0.08, grain_d=3.0e-3, cohesion=100.0)
    o = Oracle(sc, nbr_mode="cells")
    o.step(30)
    st = o.state()
    ns = sc.n_soil
    sc = dataclasses.replace(sc, pos=st["pos"][:ns].copy(), vel=st["vel"][:ns].copy(),
                             sigma=st["sigma"][:ns].copy(), rho=st["rho"][:ns].copy())
    rec = A.Recording(sc, K)
    w = A.loss_weights(3, ns, K, len(sc.bodies))
    g = A.gradient(rec, w)
    return sc, rec, w, g


@pytest.mark.parametrize("col,name", [(1, "mu_2"), (2, "cohesion")])
def test_rate_friction_and_cohesion_gradients_match_central_differences(rate_setup, col, name):
    sc, rec, w, g = rate_setup
    p = sc.params
    mat = np.zeros(sc.n_soil, dtype=np.int32)
    base = np.array([[p["mu_s"], p["mu_2"], p["cohesion"]]])
    eps = 1e-6 * base[0, col]

    def L_at(sgn):
        tab = base.copy()
        tab[0, col] += sgn * eps
        return A.functional(sc, K, w, materials=(tab, mat))

    fd = (L_at(1) - L_at(-1)) / (2 * eps)
    assert abs(g["mat"][0, col]) > 0.0, name     # the branch that carries it is taken
    _check(fd, g["mat"][0, col], tol=1e-4)
