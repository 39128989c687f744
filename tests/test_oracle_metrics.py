"""Pins for the parity comparator (oracle/metrics.py) and for the target
subset of grid_kdtree.

Every GPU parity assertion ends in ``e_val`` / ``e_weights``, so these are
pinned on hand-built arrays whose answers are worked out by hand below, and
each plausible slip (a norm over the wrong axis, the norm taken from the
tested array, an inverted or all-false mask, a mean instead of a maximum)
is planted in a copy of the module and must fail at least one pin.
"""
import numpy as np
import pytest

import oracle
from oracle import grid as og
from oracle import metrics as om

from mutate import mutated

NAN = float("nan")

# Two channels, three targets; target 2 is empty (W = 0).
W3 = np.array([1.0, 2.0, 0.0])
R3 = np.array([[1.0, 2.0, NAN],
               [4.0, -8.0, NAN]])


def pin_e_val(m):
    # channel 0: target 1 off by 0.02, channel norm max(|1|, |2|) = 2 -> 0.01
    # channel 1: target 0 off by 0.04, channel norm max(|4|, |-8|) = 8 -> 0.005
    Rh = R3.copy()
    Rh[0, 1] += 0.02
    Rh[1, 0] -= 0.04
    assert m.e_val(Rh, R3, W3) == pytest.approx(0.01, rel=1e-12)
    # one bad channel: only channel 1, target 1 off by 0.8 -> 0.8 / 8 = 0.1
    Rh = R3.copy()
    Rh[1, 1] += 0.8
    assert m.e_val(Rh, R3, W3) == pytest.approx(0.1, rel=1e-12)
    # one bad target across both channels: target 0 off by 0.5 in each channel
    # -> max(0.5 / 2, 0.5 / 8) = 0.25
    Rh = R3.copy()
    Rh[:, 0] += 0.5
    assert m.e_val(Rh, R3, W3) == pytest.approx(0.25, rel=1e-12)
    # exact copy -> 0
    assert m.e_val(R3.copy(), R3, W3) == 0.0
    # a zero channel is compared in absolute terms (its norm counts as 1)
    R0 = np.array([[0.0, 0.0, NAN]])
    assert m.e_val(np.array([[0.0, 3e-7, NAN]]), R0, W3) == pytest.approx(3e-7, rel=1e-12)
    # cols: only targets 0 and 2 are compared; channel norms over those
    # targets (|1| and |4|), so target 1's error is not seen
    Rh = R3.copy()
    Rh[0, 1] += 5.0
    Rh[1, 0] += 0.2
    assert m.e_val(Rh, R3, W3, cols=[0, 2]) == pytest.approx(0.05, rel=1e-12)


def pin_e_val_masks(m):
    # NaN on a filled target in the tested array only -> mismatch
    Rh = R3.copy()
    Rh[0, 0] = NAN
    with pytest.raises(AssertionError):
        m.e_val(Rh, R3, W3)
    # a value where the oracle has no weight -> must be NaN there
    Rh = R3.copy()
    Rh[1, 2] = 0.0
    with pytest.raises(AssertionError):
        m.e_val(Rh, R3, W3)
    # every target empty: nothing to compare, but the tested array must be NaN
    Wz = np.zeros(3)
    Rn = np.full((2, 3), NAN)
    assert m.e_val(Rn, Rn, Wz) == 0.0
    with pytest.raises(AssertionError):
        m.e_val(np.zeros((2, 3)), Rn, Wz)


def pin_e_weights(m):
    W = np.array([2.0, 0.0, 4.0, 1.0])
    Wh = np.array([2.002, 0.0, 3.996, 1.0])
    # |2.002 - 2| / 2 = 1e-3, |3.996 - 4| / 4 = 1e-3, exact elsewhere
    assert m.e_weights(Wh, W) == pytest.approx(1e-3, rel=1e-9)
    Wh = np.array([2.0, 0.0, 4.0, 1.5])
    assert m.e_weights(Wh, W) == pytest.approx(0.5, rel=1e-12)
    # the relative error is taken against the oracle's weight, not the tested one
    assert m.e_weights(np.array([3.0, 0.0, 4.0, 1.0]), W) == pytest.approx(0.5, rel=1e-12)
    # weight where the oracle has none
    with pytest.raises(AssertionError):
        m.e_weights(np.array([2.0, 1e-9, 4.0, 1.0]), W)
    assert m.e_weights(np.zeros(3), np.zeros(3)) == 0.0


def pin_pointwise_rel(m):
    R = np.array([[10.0, 0.001, -5.0, 7.0]])
    W = np.array([1.0, 1.0, 1.0, 0.0])
    Rh = R + np.array([[0.1, 0.001, 0.05, 100.0]])
    # channel norm 10 (filled targets only); floors max(|R|, 1e-2) = 10, 0.01, 5
    got = m.pointwise_rel(Rh, R, W)
    np.testing.assert_allclose(got, [0.01, 0.1, 0.01], rtol=1e-12)
    assert m.pointwise_rel(R, R, np.zeros(4)).size == 0


PINS = [pin_e_val, pin_e_val_masks, pin_e_weights, pin_pointwise_rel]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_metric_pins(pin):
    pin(om)


def test_package_exports_the_pinned_functions():
    assert oracle.e_val is om.e_val
    assert oracle.e_weights is om.e_weights
    assert oracle.pointwise_rel is om.pointwise_rel


MUTATIONS = {
    "norm_over_all_channels": ("norm = np.abs(R[:, m]).max(axis=1)\n",
                               "norm = np.abs(R[:, m]).max()\n"),
    "diff_over_channels_axis": ("diff = np.abs(R_hat[:, m] - R[:, m]).max(axis=1)",
                                "diff = np.abs(R_hat[:, m] - R[:, m]).mean(axis=1)"),
    "norm_from_tested": ("norm = np.abs(R[:, m]).max(axis=1)\n",
                         "norm = np.abs(R_hat[:, m]).max(axis=1)\n"),
    "mask_inverted": ("    m = _mask(W)\n    if cols", "    m = ~_mask(W)\n    if cols"),
    "mask_all_false": ("return np.asarray(W, dtype=np.float64) > 0",
                       "return np.asarray(W, dtype=np.float64) > np.inf"),
    "no_empty_check": ("if not np.all(np.isnan(R_hat[:, ~m])):", "if False:"),
    "no_nan_check": ("if not np.array_equal(np.isnan(R_hat[:, m]), np.isnan(R[:, m])):",
                     "if False:"),
    "weights_rel_to_tested": ("(np.abs(W_hat[m] - W[m]) / W[m]).max()",
                              "(np.abs(W_hat[m] - W[m]) / W_hat[m]).max()"),
    "weights_mean": ("(np.abs(W_hat[m] - W[m]) / W[m]).max()",
                     "(np.abs(W_hat[m] - W[m]) / W[m]).mean()"),
    "weights_no_zero_check": ("if np.any(W_hat[~m] != 0):", "if False:"),
    "pointwise_floor_absolute": ("den = np.maximum(np.abs(R[:, m]), 1e-3 * norm)",
                                 "den = np.maximum(np.abs(R[:, m]), 1e-3)"),
    "pointwise_from_tested": ("den = np.maximum(np.abs(R[:, m]), 1e-3 * norm)",
                              "den = np.maximum(np.abs(R_hat[:, m]), 1e-3 * norm)"),
}


def _all_pins_pass(m):
    try:
        for pin in PINS:
            pin(m)
    except (AssertionError, pytest.fail.Exception):
        return False
    return True


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_metric_mistakes_fail_a_pin(name):
    old, new = MUTATIONS[name]
    assert _all_pins_pass(om)
    assert not _all_pins_pass(mutated(om, old, new)), f"planted mistake {name} passed every pin"


# ---------------------------------------------------------- grid_kdtree(targets=)

def test_kdtree_target_subset_equals_full_run():
    """A target subset gives exactly the full run's values on those targets
    and leaves every other target empty (NaN, W = 0, count 0)."""
    g = np.random.default_rng(11)
    lon = g.uniform(30.0, 30.6, 3000)
    lat = g.uniform(-20.3, -19.7, 3000)
    x = g.normal(size=(3000, 3))
    tl, tb = np.meshgrid(np.linspace(30.05, 30.55, 14), np.linspace(-20.25, -19.75, 11))
    tl, tb = tl.ravel(), tb.ravel()
    tb[5] = np.nan   # a target without coordinates stays empty in both runs
    kern = ("gauss2d", (3 / 60, 2 / 60, 25.0))
    full = og.grid_kdtree(lon, lat, x, tl, tb, kern, 9 / 60, block=37)
    sub = np.array([150, 3, 77, 5, 0, 101, 153], dtype=np.int64)
    part = og.grid_kdtree(lon, lat, x, tl, tb, kern, 9 / 60, block=2, targets=sub)
    other = np.setdiff1d(np.arange(tl.size), sub)
    np.testing.assert_array_equal(part["W"][sub], full["W"][sub])
    np.testing.assert_array_equal(part["count"][sub], full["count"][sub])
    np.testing.assert_array_equal(part["hash"][sub], full["hash"][sub])
    np.testing.assert_allclose(part["R"][:, sub], full["R"][:, sub], rtol=1e-13, atol=1e-15)
    assert np.all(part["W"][other] == 0) and np.all(part["count"][other] == 0)
    assert np.all(np.isnan(part["R"][:, other]))
    assert full["count"][sub[sub != 5]].min() > 0 and full["count"][5] == 0
    # and the full run agrees with brute force on the subset
    brute = og.grid_bruteforce(lon, lat, x, tl[sub], tb[sub], kern, 9 / 60)
    np.testing.assert_array_equal(brute["count"], full["count"][sub])
    np.testing.assert_allclose(brute["W"], full["W"][sub], rtol=1e-12)
