"""The workload generators and defaults use the constants the paper prints
(tests/golden/paper_constants.txt, each line citing its passage)."""
import math
import os

import numpy as np

from paper_2507_05643_amd import scenes

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")


def _load():
    out = {}
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = line.split()[:2]
        out[k] = float(v)
    return out


def test_defaults_match_paper():
    g = _load()
    p = scenes.DEFAULT_PARAMS
    assert p["grow_G"] == g["capacity_growth_G"]
    assert p["shrink_S"] == g["capacity_shrink_threshold_S"]
    assert p["shrink_interval"] == g["capacity_shrink_interval_SI"]
    assert p["av_gamma"] == g["wheel_av_gamma"] and p["av_mode"] == 2
    assert p["I0"] == g["mu_I_I0"]
    # h / d0 of the single-wheel row is the 1.2 used by every workload
    assert abs(g["wheel_h"] / g["wheel_d0"] - 1.2) < 1e-12


def test_marker_layers_cover_kernel_support():
    g = _load()
    n_layers = math.ceil(g["kernel_support_factor_K"] * 1.2)   # ceil(K h / d0)
    assert n_layers == 3
    sc = scenes.column(seed=0, n=6)
    z = np.unique(np.round(sc.bodies[0].markers[:, 2] / 0.01, 3))
    assert (z < 0).sum() == n_layers                            # floor layers
    sc = scenes.wheel_bin(seed=0, nx=20, ny=12, nz=6)
    assert sc.meta["omega"] == g["wheel_omega"]
    r = np.hypot(sc.bodies[1].markers[:, 0], sc.bodies[1].markers[:, 2])
    assert abs(r.max() - (g["wheel_radius"] + 0.01)) < 1e-6     # grouser tips
    assert abs(np.ptp(sc.bodies[1].markers[:, 1]) - g["wheel_width"]) < 1e-6
