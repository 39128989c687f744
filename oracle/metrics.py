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


def e_val_parts(R_hat, R, W):
    """The per-channel pieces of ``e_val`` on one block of targets: the
    largest |R^ - R| and the largest |R| over the block's filled targets
    (zeros if none is filled).  Raises if the NaN masks differ: filled
    targets must be NaN exactly where the oracle is, empty ones NaN always.
    ``e_val_combine`` of the pieces of disjoint blocks is ``e_val`` of their
    union."""
    R_hat = np.asarray(R_hat, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    m = _mask(W)
    if not np.array_equal(np.isnan(R_hat[:, m]), np.isnan(R[:, m])):
        raise AssertionError("NaN mask mismatch on filled targets")
    if not np.all(np.isnan(R_hat[:, ~m])):
        raise AssertionError("empty targets must be NaN")
    C = R.shape[0]
    if not m.any():
        return np.zeros(C), np.zeros(C)
    return np.abs(R_hat[:, m] - R[:, m]).max(axis=1), np.abs(R[:, m]).max(axis=1)


def e_val_combine(parts):
    """``e_val`` from the (diff, norm) pieces of disjoint blocks."""
    diff = np.max(np.stack([p[0] for p in parts]), axis=0)
    norm = np.max(np.stack([p[1] for p in parts]), axis=0)
    norm = np.where(norm > 0, norm, 1.0)
    return float((diff / norm).max()) if diff.size else 0.0


def e_val(R_hat, R, W, cols=None):
    """Channel-normalised max error; raises if the NaN masks differ.

    ``cols`` optionally restricts the comparison to those target columns
    (sampled outputs); the channel norm is then taken over the same columns.
    """
    R_hat = np.asarray(R_hat, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    if cols is not None:
        R_hat, R, W = R_hat[:, cols], R[:, cols], W[cols]
    return e_val_combine([e_val_parts(R_hat, R, W)])


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
