"""The granular column settling under gravity in its no-slip marker box (the
16^3 column workload), run by the oracle far beyond the 100-step parity
window: 1,820 steps, about two periods of its slowest vertical oscillation.

1. Momentum balance, exact up to FP64 rounding: the soil's vertical momentum
   changes by the weight plus the force of the markers on the soil, and the
   body forces of Sec. 2.5.1 (the stage-2 marker accelerations of the step)
   are the reaction of that force. Over any window of steps [a, b),
       dt sum_k F_z^k = -W dt (b - a) - (P_z(b) - P_z(a)),
   with W = N_soil m g the soil's weight and P_z = sum m u_z.
2. The settled state: averaged over one full period of the residual
   oscillation (between sign changes of F_z + W) after the first 910 steps,
   the vertical force on the box is the soil's weight within 1 %.
"""
import numpy as np

from oracle.oracle import Oracle
from paper_2507_05643_amd import scenes

STEPS = 1820


def test_settled_column_carries_its_weight():
    sc = scenes.column(seed=0, ps_freq=10)
    o = Oracle(sc, nbr_mode="cells")
    ns, m, dt = sc.n_soil, o.mass, sc.params["dt"]
    W = ns * m * 9.81
    Fz = np.zeros(STEPS)
    Pz = np.zeros(STEPS + 1)
    for k in range(STEPS):
        o.step(1)
        Fz[k] = o.forces()[0][0, 2]
        Pz[k + 1] = m * o.state()["vel"][:ns, 2].sum()
    # 1. the discrete momentum balance, window by window
    for a, b in ((0, 100), (0, STEPS), (910, STEPS), (455, 1365)):
        lhs = dt * Fz[a:b].sum()
        rhs = -W * dt * (b - a) - (Pz[b] - Pz[a])
        assert abs(lhs - rhs) <= 1e-9 * W * dt * (b - a), (a, b, lhs, rhs)
    # 2. one full period of the residual oscillation after 910 steps
    f = Fz / W + 1.0
    s = np.sign(f[910:])
    z = 910 + np.nonzero(s[1:] != s[:-1])[0] + 1
    assert z.size >= 3, z
    a, b = z[-3], z[-1]                      # last complete period
    assert b - a > 300
    mean = Fz[a:b].mean() / W
    assert abs(mean + 1.0) <= 0.01, (a, b, mean)
    # the oscillation itself is far larger than that bar early on
    assert np.abs(f[:910]).max() > 0.3
