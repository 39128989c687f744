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
    "norm_over_all_channels": ("np.abs(R[:, m]).max(axis=1)\n",
                               "np.full(C, np.abs(R[:, m]).max())\n"),
    "diff_over_channels_axis": ("return np.abs(R_hat[:, m] - R[:, m]).max(axis=1)",
                                "return np.abs(R_hat[:, m] - R[:, m]).mean(axis=1)"),
    "norm_from_tested": ("np.abs(R[:, m]).max(axis=1)\n",
                         "np.abs(R_hat[:, m]).max(axis=1)\n"),
    "mask_inverted": ("    m = _mask(W)\n    if not np.array_equal",
                      "    m = ~_mask(W)\n    if not np.array_equal"),
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


def test_e_val_from_parts_of_blocks():
    """The pieces of disjoint blocks combine to e_val of the union (used to
    compare whole cubes block by block), including empty blocks and a zero
    channel."""
    g = np.random.default_rng(3)
    R = g.normal(size=(4, 300))
    R[2] = 0.0
    W = g.uniform(0.5, 2.0, 300)
    W[[5, 77, 250]] = 0.0
    R[:, W == 0] = np.nan
    Rh = R + g.normal(scale=1e-4, size=R.shape)
    Rh[:, W == 0] = np.nan
    whole = om.e_val(Rh, R, W)
    cuts = [0, 7, 7, 120, 299, 300]
    parts = [om.e_val_parts(Rh[:, a:b], R[:, a:b], W[a:b]) for a, b in zip(cuts[:-1], cuts[1:])]
    assert om.e_val_combine(parts) == whole
    with pytest.raises(AssertionError):
        Rbad = Rh.copy()
        Rbad[1, 3] = np.nan
        om.e_val_parts(Rbad, R, W)


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


# ------------------------------------------- targets_of / grid_workload glue

def _glue_workloads():
    import synth
    from oracle import healpix as oh
    g = np.random.default_rng(12)
    out = []
    # CAR at CRVAL2 = 0: pixel (x, y) centre is (CRVAL1 + CDELT1 (x + 1 - CRPIX1),
    # CDELT2 (y + 1 - CRPIX2)), row-major with x fastest
    wcs = synth.wcs_car(7, 5, 4.0, 3.0, 10.0, -0.5, 0.5)
    xs, ys = np.meshgrid(np.arange(7), np.arange(5))
    hand = ((10.0 - 0.5 * (xs + 1 - 4.0)).ravel(), (0.5 * (ys + 1 - 3.0)).ravel())
    lon = g.uniform(8.0, 12.5, 2500)
    lat = g.uniform(-1.5, 1.5, 2500)
    out.append((synth.Workload("car", lon, lat, g.normal(size=(2500, 2)), "f64",
                               {"kind": "wcs", "wcs": wcs}, ("gauss1d", (0.3,)), 0.9), hand))
    lon, lat = synth.uniform_sphere(g, 3000)
    for order in ("ring", "nested"):
        out.append((synth.Workload(f"hpx {order}", lon, lat, g.normal(size=(3000, 1)), "f64",
                                   {"kind": "healpix", "nside": 2, "order": order},
                                   ("gauss1d", (8.0,)), 24.0),
                    oh.centres(2, order)))
    tl, tb = g.uniform(40, 42, 30), g.uniform(-5, -3, 30)
    lon, lat = g.uniform(39.5, 42.5, 2000), g.uniform(-5.5, -2.5, 2000)
    out.append((synth.Workload("sl", lon, lat, g.normal(size=(2000, 3)), "f64",
                               {"kind": "sightlines", "lon": tl, "lat": tb},
                               ("gauss2d", (0.2, 0.1, 30.0)), 0.6), (tl, tb)))
    return out


def test_grid_workload_grids_onto_the_described_targets():
    """grid_workload (both methods, and with a target subset) equals brute
    force onto targets worked out independently of targets_of."""
    wls = _glue_workloads()
    ring, nest = wls[1][1], wls[2][1]
    assert not np.allclose(ring[0], nest[0])          # the order is honoured
    for wl, (tl, tb) in wls:
        ref = og.grid_bruteforce(wl.lon, wl.lat, wl.data, tl, tb, wl.kernel, wl.support)
        assert ref["count"].sum() > 0
        for res in (og.grid_workload(wl), og.grid_workload(wl, method="brute")):
            np.testing.assert_array_equal(res["count"], ref["count"])
            np.testing.assert_allclose(res["W"], ref["W"], rtol=1e-12, atol=1e-300)
            m = ref["W"] > 0
            np.testing.assert_allclose(res["R"][:, m], ref["R"][:, m], rtol=1e-10, atol=1e-12)
        sub = np.arange(0, len(tl), 3)
        part = og.grid_workload(wl, targets=sub)
        np.testing.assert_array_equal(part["count"][sub], ref["count"][sub])
        other = np.setdiff1d(np.arange(len(tl)), sub)
        assert np.all(part["count"][other] == 0)


GLUE_MUTATIONS = {
    "lon_lat_swapped": ("    tlon, tlat = targets_of(wl)\n", "    tlat, tlon = targets_of(wl)\n"),
    "order_ignored": ('healpix_centres(t["nside"], t.get("order", "ring"))',
                      'healpix_centres(t["nside"], "ring")'),
    "subset_ignored": ("                       targets=targets)", "                       targets=None)"),
    "brute_gets_kdtree": ('if method == "brute":', 'if method == "never":'),
}


@pytest.mark.parametrize("name", sorted(GLUE_MUTATIONS))
def test_planted_glue_mistakes_fail_the_pin(name):
    old, new = GLUE_MUTATIONS[name]
    bad = mutated(og, old, new)
    if name == "brute_gets_kdtree":
        # both methods give the same numbers, so the plant is seen in the
        # call it makes: brute force must not build a tree
        import scipy.spatial
        real = scipy.spatial.cKDTree
        try:
            def refuse(*a, **k):
                raise AssertionError("tree built")
            scipy.spatial.cKDTree = refuse
            wl = _glue_workloads()[0][0]
            og.grid_workload(wl, method="brute")
            with pytest.raises(AssertionError):
                bad.grid_workload(wl, method="brute")
        finally:
            scipy.spatial.cKDTree = real
        return
    with pytest.raises(AssertionError):
        _check_glue(bad)


def _check_glue(mod):
    for wl, (tl, tb) in _glue_workloads():
        ref = og.grid_bruteforce(wl.lon, wl.lat, wl.data, tl, tb, wl.kernel, wl.support)
        res = mod.grid_workload(wl)
        np.testing.assert_array_equal(res["count"], ref["count"])
        sub = np.arange(0, len(tl), 3)
        other = np.setdiff1d(np.arange(len(tl)), sub)
        assert np.all(mod.grid_workload(wl, targets=sub)["count"][other] == 0)
