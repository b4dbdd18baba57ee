"""Host-side grid rule of the library (Sec. IV) through the C ABI, no device
needed: the lossless spacing lambda_r / 20, its cap at the mean mesh edge,
and the strict refinement by the worst lossy/lossless bound ratio, checked
against the oracle's independent evaluation of eq. Ddef / LboundsD2."""
import numpy as np
import pytest

from oracle.bound import loss_ratio
from oracle import physics as ph


def _choose(*a, **k):
    from paper_2003_11679_amd.sie import grid_choose
    return grid_choose(*a, **k)


def test_lossless_spacing_is_lambda_over_20():
    # eps_r = 4 sphere of the sphere configuration at 150 MHz: lambda_r = 0.9993 m
    g = _choose(150e6, 4.0, 1.0, 0.0, 2.0, 0.151)
    lam = ph.C0 / 150e6 / 2.0
    assert abs(g["lambda_r"] - lam) < 1e-12 * lam
    assert g["loss_ratio"] == 1.0
    assert g["n"] == int(np.ceil(2.0 / (lam / 20.0))) + 3 == 44
    assert abs(g["h"] - 2.0 / (g["n"] - 3)) < 1e-15
    assert g["order"] == 2 and g["near_radius"] == 5


def test_losses_do_not_refine_the_default_rule():
    # Sec. IV: the grid of the lossless medium serves the lossy one
    # (the near-region boundary of the lambda_r / 20 grid with R = 5 sits at
    # theta_0 = pi / 2, next to the worst case of Sec. IV: loss factor
    # s = 2.894 at 1 GHz and eps_r = 4 means sigma = 0.644 S/m)
    a = _choose(1e9, 4.0, 1.0, 0.0, 0.06, 0.01)
    b = _choose(1e9, 4.0, 1.0, 0.644, 0.06, 0.01)
    c = _choose(1e9, 4.0, 1.0, 0.644, 0.06, 0.01, strict=True)
    assert a["n"] == b["n"] and 1.4 < b["loss_ratio"] <= 1.514
    assert c["n"] > b["n"] and c["h"] < b["h"]


def test_mean_edge_caps_the_spacing():
    # copper bar: lambda_r / 20 = 1.5 mm, far above the 0.56 um mesh edge
    g = _choose(10e9, 1.0, 1.0, 5.8e7, 100e-6, 0.5556e-6)
    assert g["h"] <= 0.5556e-6 * (1 + 1e-12)
    assert g["n"] == int(np.ceil(100e-6 / 0.5556e-6)) + 3


@pytest.mark.parametrize("sigma", [0.05, 0.5, 5.0, 50.0])
def test_strict_refinement_follows_the_bound_ratio(sigma):
    f, er, R = 200e6, 2.5, 5
    w = 2 * np.pi * f
    s = sigma / (w * ph.EPS0 * er)
    kr = w * np.sqrt(er) / ph.C0
    h0 = (2 * np.pi / kr) / 20.0
    # oracle: worst ratio of eq. Ddef beyond the near-region boundary
    th = kr * R * h0 * np.geomspace(1.0, 200.0, 4001)
    worst = float(np.max(loss_ratio(2, th, s)))
    g = _choose(f, er, 1.0, sigma, 1.0, 1.0, R, strict=True)
    assert abs(g["loss_ratio"] - worst) < 2e-3 * worst
    ref = 1.0 / (h0 / max(worst, 1.0) ** (1.0 / 3.0))
    assert g["n"] == int(np.ceil(ref)) + 3
    # the ratio stays within the worst case printed in Sec. IV
    assert g["loss_ratio"] <= 1.513 + 1e-3


def test_bad_arguments_are_refused():
    from paper_2003_11679_amd import SieError
    with pytest.raises(SieError):
        _choose(-1.0, 4.0, 1.0, 0.0, 1.0, 0.1)
    with pytest.raises(SieError):
        _choose(1e9, 4.0, 1.0, 0.0, 1.0, 0.1, near_radius=0)
