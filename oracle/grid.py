"""Convolution-based gridding, FP64 oracle (test infrastructure).

Follows Sect. 2.1 of the paper:

* Eq. (1)  S_t[c] = sum_n R_n[c] w(t, n)       (weighted data sum per channel)
* Eq. (2)  W_t    = sum_n w(t, n)              (weight map)
* Eq. (3)  R_t[c] = S_t[c] / W_t               (normalised map)

``grid_bruteforce`` is the serial algorithm of Sect. 2.1 taken literally:
zero S and W, loop over every input sample n and every target t, add
R_n w and w, divide at the end.  The only addition is the support cut: a
pair contributes iff its true angular distance d <= r_s (inclusive).  The
paper evaluates the kernel only inside the disk of radius r_d it queries
(Sect. 2.2 step 3b, Sect. 3.3) and states the kernel is negligible beyond;
taking the cut exactly makes the result independent of the HEALPix
resolution.

``grid_kdtree`` computes the same sums; it only replaces "every target"
by a superset found with ``scipy.spatial.cKDTree`` (chord radius slightly
larger than the support) followed by the same exact d <= r_s test.

Kernels (readings where the paper is silent):
* 'gauss1d', (sigma,): w = exp(-d^2 / (2 sigma^2))  (peak one; Listing 1
  uses 'gauss1d' with a sigma parameter; Eq. 3 makes the normalisation of
  w irrelevant for R).
* 'tapered_sinc', (sigma, b): w = exp(-d^2 / (2 sigma^2)) sin(pi d/b) / (pi d/b),
  the sin(ax)/ax kernel the paper names (Sect. 5, a = pi / b) under a
  Gaussian taper (reading: a finite support needs one).
* 'table', (dmax, w_0, ..., w_{n-1}): a radial profile of arbitrary shape
  (the abstract: a kernel of arbitrary shape), w_k at d = k dmax / (n - 1),
  linearly interpolated, zero beyond dmax.
* 'gauss2d', (sigma_maj, sigma_min, pa): elliptical Gaussian in true world
  coordinates (Sect. 2.1, Fig. 1).  With beta the bearing of the sample
  seen from the target (north through east) and pa the position angle of
  the major axis measured the same way:
      w = exp(-d^2/2 [cos^2(beta - pa)/sigma_maj^2 + sin^2(beta - pa)/sigma_min^2]).

Angles at the interface are degrees (Listing 1 passes degrees).  Data are
upcast to FP64 (exact for FP64/FP32/FP16/BF16).  Empty targets (W = 0) get
R = NaN (Eq. 3 is 0/0 there; the paper is silent).
"""
from __future__ import annotations

import numpy as np

from .sphere import vincenty, bearing, splitmix64, unit_vectors
from .wcs import wcs_targets
from .healpix import centres as healpix_centres

BAND_RAD = 1e-12   # samples this close to the support edge may go either way


def _validate(lon, lat):
    lon = np.asarray(lon, dtype=np.float64)
    lat = np.asarray(lat, dtype=np.float64)
    if lon.shape != lat.shape or lon.ndim != 1:
        raise ValueError("lon/lat must be 1-D arrays of equal length")
    if not (np.all(np.isfinite(lon)) and np.all(np.isfinite(lat))):
        raise ValueError("non-finite coordinate")
    if np.any(np.abs(lat) > 90.0):
        raise ValueError("|lat| > 90 deg")
    return np.mod(lon, 360.0), lat


def _as_f64_2d(data, n):
    try:
        import torch
        if isinstance(data, torch.Tensor):
            data = data.detach().to("cpu", torch.float64).numpy()
    except ImportError:  # pragma: no cover
        pass
    a = np.asarray(data, dtype=np.float64)
    if a.ndim == 1:
        a = a[:, None]
    if a.shape[0] != n:
        raise ValueError("data must be [N][C]")
    return a


def kernel_weight(kernel, d, tlon, tlat, slon, slat):
    """Kernel value for pairs at true distance d (radians).

    ``tlon, tlat`` target and ``slon, slat`` sample coordinates in radians
    (used only by the elliptical kernel, whose bearing is taken at the
    target).  Follows Sect. 2.1 (radially symmetric case) and Fig. 1 /
    Sect. 2.1 (elliptical case); see the module header for the formula.
    """
    kind, params = kernel
    if kind == "gauss1d":
        (sigma,) = params
        s = np.radians(sigma)
        return np.exp(-(d * d) / (2.0 * s * s))
    if kind == "gauss2d":
        smaj, smin, pa = params
        a, b, p = np.radians(smaj), np.radians(smin), np.radians(pa)
        beta = bearing(tlon, tlat, slon, slat)
        cb = np.cos(beta - p)
        sb = np.sin(beta - p)
        q = cb * cb / (a * a) + sb * sb / (b * b)
        return np.exp(-0.5 * d * d * q)
    if kind == "tapered_sinc":
        # the sin(ax)/ax kernel of Sect. 5 with a = pi / b, under a Gaussian
        # taper of width sigma so that a finite support suffices
        sigma, b = params
        s, bb = np.radians(sigma), np.radians(b)
        return np.exp(-(d * d) / (2.0 * s * s)) * np.sinc(d / bb)
    if kind == "table":
        # a radial profile of arbitrary shape (the abstract): values w_k at
        # d_k = k dmax / (n - 1), linear in between, zero beyond dmax
        dmax = np.radians(params[0])
        w = np.asarray(params[1:], dtype=np.float64)
        return np.interp(d, np.linspace(0.0, dmax, w.size), w, right=0.0)
    raise ValueError(f"unknown kernel {kind!r}")


def _finish(S, W):
    with np.errstate(invalid="ignore", divide="ignore"):
        R = S / W[None, :]
    R[:, W == 0] = np.nan
    return R


def grid_bruteforce(lon, lat, data, tlon, tlat, kernel, support):
    """All-pairs gridding following the serial loop of Sect. 2.1.

    Returns a dict with R [C][T] (NaN where W == 0), S [C][T], W [T],
    count [T] (number of samples with d <= r_s), hash [T] (sum mod 2^64 of
    splitmix64(n) over those samples, n = input index) and ``band``: an
    array of (t, n, d - r_s) rows for pairs within 1e-12 rad of the edge.
    Targets with NaN coordinates (outside a projection) stay empty.
    """
    lon, lat = _validate(lon, lat)
    n = lon.shape[0]
    X = _as_f64_2d(data, n)
    tlon = np.asarray(tlon, dtype=np.float64)
    tlat = np.asarray(tlat, dtype=np.float64)
    T = tlon.shape[0]
    C = X.shape[1]
    rs = np.radians(support)
    valid_t = np.isfinite(tlon) & np.isfinite(tlat)
    ta = np.radians(np.where(valid_t, tlon, 0.0))
    td = np.radians(np.where(valid_t, tlat, 0.0))
    sa, sd = np.radians(lon), np.radians(lat)
    # step 1: zero the maps
    S = np.zeros((C, T))
    W = np.zeros(T)
    count = np.zeros(T, dtype=np.int64)
    hsh = np.zeros(T, dtype=np.uint64)
    hn = splitmix64(np.arange(n, dtype=np.uint64))
    band = []
    # step 2: every sample, every target
    for k in range(n):
        d = vincenty(ta, td, sa[k], sd[k])
        edge = np.abs(d - rs) < BAND_RAD
        if edge.any():
            for t in np.nonzero(edge & valid_t)[0]:
                band.append((t, k, d[t] - rs))
        m = (d <= rs) & valid_t
        if not m.any():
            continue
        w = kernel_weight(kernel, d[m], ta[m], td[m], sa[k], sd[k])
        S[:, m] += X[k][:, None] * w[None, :]
        W[m] += w
        count[m] += 1
        with np.errstate(over="ignore"):
            hsh[m] += hn[k]
    # step 3: divide
    return {"R": _finish(S, W), "S": S, "W": W, "count": count, "hash": hsh,
            "band": np.array(band, dtype=np.float64).reshape(-1, 3)}


def _pairs_kdtree(tree, tv, rs):
    chord = 2.0 * np.sin(0.5 * rs) * (1.0 + 1e-9) + 1e-15
    lists = tree.query_ball_point(tv, chord, return_sorted=False)
    lens = np.fromiter((len(x) for x in lists), dtype=np.int64, count=len(lists))
    if lens.sum() == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    nid = np.concatenate([np.asarray(x, dtype=np.int64) for x in lists if len(x)])
    tid = np.repeat(np.arange(len(lists), dtype=np.int64), lens)
    return tid, nid


def neighbour_sets(lon, lat, tlon, tlat, support, block=4096):
    """Per-target neighbour statistics without data: count, hash and band.

    Same d <= r_s rule as ``grid_bruteforce``; candidates via cKDTree.
    """
    from scipy.spatial import cKDTree

    lon, lat = _validate(lon, lat)
    tlon = np.asarray(tlon, dtype=np.float64)
    tlat = np.asarray(tlat, dtype=np.float64)
    T = tlon.shape[0]
    rs = np.radians(support)
    tree = cKDTree(unit_vectors(lon, lat))
    valid_t = np.isfinite(tlon) & np.isfinite(tlat)
    count = np.zeros(T, dtype=np.int64)
    hsh = np.zeros(T, dtype=np.uint64)
    band = []
    sa, sd = np.radians(lon), np.radians(lat)
    for s in range(0, T, block):
        e = min(T, s + block)
        ok = np.nonzero(valid_t[s:e])[0] + s
        if ok.size == 0:
            continue
        tv = unit_vectors(tlon[ok], tlat[ok])
        tid, nid = _pairs_kdtree(tree, tv, rs)
        tg = ok[tid]
        d = vincenty(np.radians(tlon[tg]), np.radians(tlat[tg]), sa[nid], sd[nid])
        edge = np.abs(d - rs) < BAND_RAD
        for q in np.nonzero(edge)[0]:
            band.append((tg[q], nid[q], d[q] - rs))
        m = d <= rs
        np.add.at(count, tg[m], 1)
        with np.errstate(over="ignore"):
            np.add.at(hsh, tg[m], splitmix64(nid[m].astype(np.uint64)))
    return {"count": count, "hash": hsh,
            "band": np.array(band, dtype=np.float64).reshape(-1, 3)}


def grid_kdtree(lon, lat, data, tlon, tlat, kernel, support, block=4096,
                targets=None):
    """Same result as ``grid_bruteforce`` with cKDTree candidate search.

    ``targets`` (optional int array) restricts the computation to those
    target indices (the others stay empty); used to evaluate sampled
    outputs of full-size workloads.  Sums: FP64, one sparse product per
    block of targets (a library matmul as the summation step of Eq. 1).
    """
    from scipy.spatial import cKDTree
    from scipy.sparse import csr_matrix

    lon, lat = _validate(lon, lat)
    n = lon.shape[0]
    X = _as_f64_2d(data, n)
    tlon = np.asarray(tlon, dtype=np.float64)
    tlat = np.asarray(tlat, dtype=np.float64)
    T = tlon.shape[0]
    C = X.shape[1]
    rs = np.radians(support)
    tree = cKDTree(unit_vectors(lon, lat))
    valid_t = np.isfinite(tlon) & np.isfinite(tlat)
    sel = np.arange(T) if targets is None else np.asarray(targets, dtype=np.int64)
    sel = sel[valid_t[sel]]
    S = np.zeros((C, T))
    W = np.zeros(T)
    count = np.zeros(T, dtype=np.int64)
    hsh = np.zeros(T, dtype=np.uint64)
    sa, sd = np.radians(lon), np.radians(lat)
    for s in range(0, sel.shape[0], block):
        ok = sel[s:s + block]
        tv = unit_vectors(tlon[ok], tlat[ok])
        tid, nid = _pairs_kdtree(tree, tv, rs)
        if tid.size == 0:
            continue
        tg = ok[tid]
        ta, td = np.radians(tlon[tg]), np.radians(tlat[tg])
        d = vincenty(ta, td, sa[nid], sd[nid])
        m = d <= rs
        tid, nid, tg, d = tid[m], nid[m], tg[m], d[m]
        w = kernel_weight(kernel, d, ta[m], td[m], sa[nid], sd[nid])
        Wm = csr_matrix((w, (tid, nid)), shape=(ok.shape[0], n))
        S[:, ok] = (Wm @ X).T
        W[ok] = np.bincount(tid, weights=w, minlength=ok.shape[0])
        count[ok] = np.bincount(tid, minlength=ok.shape[0])
        hb = np.zeros(ok.shape[0], dtype=np.uint64)
        with np.errstate(over="ignore"):
            np.add.at(hb, tid, splitmix64(nid.astype(np.uint64)))
        hsh[ok] = hb
    return {"R": _finish(S, W), "S": S, "W": W, "count": count, "hash": hsh}


def targets_of(wl):
    """Target (lon, lat) arrays of a workload: WCS pixel centres, HEALPix
    pixel centres or sight lines."""
    t = wl.target
    if t["kind"] == "wcs":
        return wcs_targets(t["wcs"])
    if t["kind"] == "healpix":
        return healpix_centres(t["nside"], t.get("order", "ring"))
    return np.asarray(t["lon"], dtype=np.float64), np.asarray(t["lat"], dtype=np.float64)


def grid_workload(wl, method="kdtree", targets=None):
    """Grid a ``synth.Workload`` with the oracle; returns the result dict."""
    tlon, tlat = targets_of(wl)
    if method == "brute":
        return grid_bruteforce(wl.lon, wl.lat, wl.data, tlon, tlat, wl.kernel, wl.support)
    return grid_kdtree(wl.lon, wl.lat, wl.data, tlon, tlat, wl.kernel, wl.support,
                       targets=targets)
