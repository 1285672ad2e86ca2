"""The workloads' readings of the paper pinned to the values it prints (tests/golden/, each file
citing its section and table): the end time T = 0.32 implied by both level tables, the model
constants, and the Karhunen-Loeve parameters of the three experiments as the workloads take them.
The oracle's stochastic-dimension check against M = 66 is in tests/test_oracle_kl.py."""
import os

import numpy as np

import workloads as W
from workloads import tetshell

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    for ln in open(os.path.join(GOLDEN, name)):
        ln = ln.strip()
        if ln and not ln.startswith("#"):
            out.append(ln.split())
    return out


def _params():
    return {r[0]: [float(x) for x in r[1:]] for r in _rows("paper_parameters.txt")}


def test_level_tables_imply_the_end_time():
    """Every level of both tables takes T / dt time steps with T = 0.32 ms (reading A1); on the
    cube the spatial part is (1/h)^3 (the box has side 1): DOF = (1/h)^3 T / dt exactly."""
    for geo, l, dof, h, dt in _rows("paper_levels.txt"):
        steps = W.T_END / float(dt)
        assert abs(steps - round(steps)) < 1e-9 and round(steps) == 2 ** (int(l) + 1)
        space = int(dof) / round(steps)
        assert space == int(space)
        if geo == "cube":
            assert int(space) == round(1.0 / float(h)) ** 3


def test_model_constants_are_the_papers():
    p = _params()
    ph = W.physics(3)
    for k in ("alpha", "u_rest", "u_th", "u_peak"):
        assert ph[k] == p[k][0], k
    assert W.SIGMA_L == p["cube_mean_diffusion"][0] == p["ventricle_mean_diffusion"][0]
    assert W.SIGMA_T == p["heart_g"][0]


def test_workload_kl_parameters_follow_the_papers():
    """c2i: the cube's kernel, theta and M; c5i: the ventricle's (the shell has its size); c5v:
    the heart's theta and M = 3 x 45, sigma_KL scaled by the square of the size ratio (the
    shell's long axis 2 against the heart's box of about one unit; reading T8)."""
    p = _params()
    c2i, c5i, c5v = W.config("c2i")["kl"], W.config("c5i")["kl"], W.config("c5v")["kl"]
    assert (c2i["std"], c2i["corr_len"], c2i["n_modes"]) == (p["cube_theta"][0], p["cube_sigma_kl"][0],
                                                            p["cube_M"][0])
    assert c2i["kernel"] == c5i["kernel"] == c5v["kernel"] == "sqexp"
    assert (c5i["std"], c5i["corr_len"], c5i["n_modes"]) == (p["ventricle_theta"][0], p["ventricle_sigma_kl"][0],
                                                            p["ventricle_M"][0])
    assert c5v["std"] == p["heart_theta"][0] and c5v["components"] * c5v["n_modes"] == p["heart_M"][0]
    heart_extent = max(np.diff(np.reshape(p["heart_box"], (3, 2)), axis=1).ravel())
    assert abs(heart_extent - 1.07) < 0.01 and abs(tetshell.LONG_AXIS - 2.0) < 1e-12
    assert np.isclose(c5v["corr_len"], p["heart_sigma_kl"][0] * (tetshell.LONG_AXIS / 1.0) ** 2)
    ventricle = np.diff(np.reshape(p["ventricle_box"], (3, 2)), axis=1).ravel()
    assert (np.abs(ventricle - 2.0) <= 0.5).all()
    # the cube experiments run on the unit box, a translate of the paper's [-0.5, 0.5]^3
    lo, hi = np.reshape(p["cube_box"], (3, 2)).T
    assert np.allclose(hi - lo, 1.0) and W.config("c2i")["levels"][0]["hi"] == [1.0, 1.0, 1.0]
