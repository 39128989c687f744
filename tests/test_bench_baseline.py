"""The benchmark's CPU baseline: the oracle over bands of targets on forked
workers, each band compared with the result under test.  Checked here on
CPU with the oracle's own result standing in for a GPU cube, so that the
pooled comparison is known to reproduce the whole-cube one."""
import numpy as np
import torch

import bench
import oracle
import synth


def _job_and_reference(wl):
    tl, tb = oracle.targets_of(wl)
    data = wl.data.float().numpy() if isinstance(wl.data, torch.Tensor) else wl.data
    ref = oracle.grid_kdtree(wl.lon, wl.lat, np.asarray(data, np.float64), tl, tb, wl.kernel,
                             wl.support)
    nx, ny = wl.target["wcs"]["naxis1"], wl.target["wcs"]["naxis2"]
    return ref, nx, ny


def test_pooled_oracle_matches_whole_cube_comparison():
    wls = synth.config4(scale=0.02)[:4]
    jobs, truth_pairs, planted = [], 0, []
    for wl in wls:
        ref, nx, ny = _job_and_reference(wl)
        cube = torch.as_tensor(ref["R"]).reshape(wl.nchan, ny, nx).float()
        w = torch.as_tensor(ref["W"]).reshape(ny, nx).float()
        bad = cube.clone()
        y0, y1 = (3 * ny) // 8, max((5 * ny) // 8, (3 * ny) // 8 + 1)
        band = np.arange(y0 * nx, y1 * nx)
        # one bad value in the band, 1 % of that channel's band norm
        c = wl.nchan - 1
        rb = ref["R"][c, band]
        k = band[int(np.nanargmax(np.abs(rb)))]
        bad.reshape(wl.nchan, -1)[c, k] += 0.01 * float(np.nanmax(np.abs(rb)))
        planted.append(0.01)
        truth_pairs += int(ref["count"][band].sum())
        jobs.append(bench.oracle_job(wl, band, {"same": cube, "bad": bad},
                                     {"same": w, "bad": w}))
    cpu, errs = bench.cpu_baseline(jobs, "test", tasks_per_worker=2)
    assert cpu["kind"] == "oracle" and cpu["cores"] >= 1 and cpu["model"]
    assert f"{truth_pairs} pairs" in cpu["sample"]
    assert errs["e_val"]["same"] < 1e-6 and errs["e_W"]["same"] < 1e-6
    assert abs(errs["e_val"]["bad"] - 0.01) < 1e-4
    assert "mask_errors" not in errs


def test_pooled_oracle_reports_a_nan_mask_mismatch():
    wl = synth.config4(scale=0.02)[0]
    ref, nx, ny = _job_and_reference(wl)
    cube = torch.as_tensor(ref["R"]).reshape(wl.nchan, ny, nx).float()
    w = torch.as_tensor(ref["W"]).reshape(ny, nx).float()
    filled = np.nonzero(ref["W"] > 0)[0]
    cube.reshape(wl.nchan, -1)[0, int(filled[len(filled) // 2])] = float("nan")
    cpu, errs = bench.cpu_baseline([bench.oracle_job(wl, np.arange(nx * ny), {"x": cube},
                                                     {"x": w})], "test")
    assert errs.get("mask_errors")
