"""Error measures for parity checks (test infrastructure).

The paper defines no error metric; these are the definitions every parity
test and the benchmark use:

* ``e_val``: max over channels c of ||R^_c - R_c||_inf / ||R_c||_inf over the
  targets with W > 0 (NaN masks must agree exactly).
* ``e_weights``: max over targets with W > 0 of |W^ - W| / W.
* ``pointwise_rel``: |R^ - R| / max(|R|, 1e-3 ||R_c||_inf), for percentiles.
"""
from __future__ import annotations

import numpy as np


def _mask(W):
    return np.asarray(W, dtype=np.float64) > 0


def e_val(R_hat, R, W, cols=None):
    """Channel-normalised max error; raises if the NaN masks differ.

    ``cols`` optionally restricts the comparison to those target columns
    (sampled outputs); the channel norm is then taken over the same columns
    unless the oracle's full-map norms are passed via ``R`` restricted the
    same way.
    """
    R_hat = np.asarray(R_hat, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    m = _mask(W)
    if cols is not None:
        R_hat, R, m = R_hat[:, cols], R[:, cols], m[cols]
    if not np.array_equal(np.isnan(R_hat[:, m]), np.isnan(R[:, m])):
        raise AssertionError("NaN mask mismatch on filled targets")
    if not np.all(np.isnan(R_hat[:, ~m])):
        raise AssertionError("empty targets must be NaN")
    if not m.any():
        return 0.0
    diff = np.abs(R_hat[:, m] - R[:, m]).max(axis=1)
    norm = np.abs(R[:, m]).max(axis=1)
    norm = np.where(norm > 0, norm, 1.0)
    return float((diff / norm).max())


def e_weights(W_hat, W):
    W_hat = np.asarray(W_hat, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    m = W > 0
    if np.any(W_hat[~m] != 0):
        raise AssertionError("weights must be zero where the oracle has none")
    if not m.any():
        return 0.0
    return float((np.abs(W_hat[m] - W[m]) / W[m]).max())


def pointwise_rel(R_hat, R, W):
    R_hat = np.asarray(R_hat, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    m = _mask(W)
    if not m.any():
        return np.zeros(0)
    norm = np.abs(R[:, m]).max(axis=1, keepdims=True)
    den = np.maximum(np.abs(R[:, m]), 1e-3 * norm)
    den = np.where(den > 0, den, 1.0)
    return (np.abs(R_hat[:, m] - R[:, m]) / den).ravel()
