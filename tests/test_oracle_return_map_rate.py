"""Pins of the shear-rate part of the oracle's return mapping (Sec. 2.4, eqs.
trial_quantities, muI, yieldsurf), with mu_2 != mu_s.

Each case is built by hand so that the expected stress follows from the
definitions alone: the pressure p* and equivalent shear stress of the trial
stress, the shear-rate estimate gamma_dot = (taubar* - taubar^n) / (G dt) with
G = E / (2 (1 + nu)) and taubar^n from the stress at the start of the step, the
inertial number I = gamma_dot d sqrt(rho0 / p*), mu(I) = mu_s + (mu_2 - mu_s) /
(I0 / I + 1), tau_max = mu p* + c and the radial return of the deviator. The
first case picks the grain size d so that I = I0 exactly, where mu(I) is the
mean of mu_s and mu_2: a factor 2 on G, taubar^n taken from the trial stress,
or the pressure of the start of the step in I all move mu away from that mean.
"""
import math

import numpy as np

from paper_2507_05643_amd import scenes

E, NU, DT, RHO0 = 1.0e6, 0.3, 2.5e-5, 1700.0
G = E / (2.0 * (1.0 + NU))


def _params(**over):
    p = dict(scenes.DEFAULT_PARAMS, E=E, nu=NU, dt=DT, rho0=RHO0, mu_s=0.7, mu_2=0.8, I0=0.08)
    p.update(over)
    return p


def _p_tb(s):
    s = np.asarray(s, dtype=np.float64)
    p = -(s[0] + s[1] + s[2]) / 3.0
    t = s[:3] + p
    return p, math.sqrt(0.5 * (float(t @ t) + 2.0 * float(s[3:] @ s[3:])))


def _radial(s_star, tmax):
    """-p* I + (tau_max / taubar*) dev(s*)."""
    p, tb = _p_tb(s_star)
    f = tmax / tb
    s = np.asarray(s_star, dtype=np.float64)
    out = np.empty(6)
    out[:3] = -p + f * (s[:3] + p)
    out[3:] = f * s[3:]
    return out


def test_rate_dependent_friction_at_I_equal_I0(orc):
    s_n = np.array([-1000.0, -1000.0, -1000.0, 100.0, 0.0, 0.0])        # p 1000, taubar 100
    s_star = np.array([-2000.0, -2000.0, -2000.0, 2000.0, 0.0, 0.0])    # p* 2000, taubar* 2000
    p_star, tb_star = _p_tb(s_star)
    _, tb_n = _p_tb(s_n)
    gd = (tb_star - tb_n) / (G * DT)
    d = 0.08 / (gd * math.sqrt(RHO0 / p_star))                          # I = I0
    c = 200.0
    p = _params(grain_d=d, cohesion=c)
    out, br, case = orc.return_map_ex(p, s_star, s_n)
    tmax = 0.5 * (0.7 + 0.8) * p_star + c                               # 1700 < 2000: yields
    assert br == 4 and case == 2
    want = _radial(s_star, tmax)
    assert np.abs(out - want).max() <= 1e-12 * np.abs(want).max()
    # the same state read with G doubled, or with taubar^n = taubar*, would not
    # give the mean friction
    I_2G = gd / 2 * d * math.sqrt(RHO0 / p_star)
    assert abs((0.7 + 0.1 * I_2G / (I_2G + 0.08)) - 0.75) > 1e-2


def test_shear_rate_scales_with_G_dt(orc):
    """Doubling E halves gamma_dot and so I: mu = mu_s + (mu_2 - mu_s) / 3."""
    s_n = np.array([-1000.0, -1000.0, -1000.0, 100.0, 0.0, 0.0])
    s_star = np.array([-2000.0, -2000.0, -2000.0, 2000.0, 0.0, 0.0])
    p_star, tb_star = _p_tb(s_star)
    _, tb_n = _p_tb(s_n)
    gd = (tb_star - tb_n) / (G * DT)
    d = 0.08 / (gd * math.sqrt(RHO0 / p_star))
    out, br, case = orc.return_map_ex(_params(grain_d=d, E=2.0 * E), s_star, s_n)
    mu = 0.7 + 0.1 * 0.5 / (0.5 + 1.0)                                   # I = I0 / 2
    assert br == 4 and case == 2
    want = _radial(s_star, mu * p_star)
    assert np.abs(out - want).max() <= 1e-12 * np.abs(want).max()


def test_tensile_trial_state_with_cohesion_takes_mu_2(orc):
    """p* < 0 above the cut-off p_cri = -c / mu_s with a rising shear stress:
    the I -> infinity limit mu_2 (reading of the undefined case)."""
    c = 500.0
    s_star = np.array([300.0, 300.0, 300.0, 400.0, 0.0, 0.0])           # p* -300 > -714.3
    s_n = np.zeros(6)
    out, br, case = orc.return_map_ex(_params(cohesion=c), s_star, s_n)
    p_star, _ = _p_tb(s_star)
    assert br == 4 and case == 1
    want = _radial(s_star, 0.8 * p_star + c)                             # 260 < 400
    assert np.abs(out - want).max() <= 1e-12 * np.abs(want).max()


def test_falling_shear_stress_takes_mu_s(orc):
    """gamma_dot < 0 is read as 0, where mu(I) = mu_s."""
    s_n = np.array([-1000.0, -1000.0, -1000.0, 1000.0, 0.0, 0.0])
    s_star = np.array([-1000.0, -1000.0, -1000.0, 900.0, 0.0, 0.0])
    out, br, case = orc.return_map_ex(_params(), s_star, s_n)
    assert br == 4 and case == 0
    want = _radial(s_star, 0.7 * 1000.0)
    assert np.abs(out - want).max() <= 1e-12 * np.abs(want).max()


def test_cut_off_reports_no_mu_case(orc):
    out, br, case = orc.return_map_ex(_params(cohesion=100.0), [200.0, 200.0, 200.0, 0, 0, 0], np.zeros(6))
    assert br == 1 and case == -1 and np.all(out == 0.0)
