"""CPU oracle for convolution-based gridding (test infrastructure only).

This package is the plain, slow, obviously-correct FP64 reference that the
GPU path is checked against.  It is *test infrastructure*: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The product path (the C-ABI library and its Python binding)
never imports, links or calls anything here, and nothing here imports the
product path.

What it computes (Winkel, Floeer & Lenz 2016, "Cygrid", Sect. 2.1):

* Eq. (1): weighted sum  S_t[c] = sum_n R_n[c] w(t, n)
* Eq. (2): weight map    W_t    = sum_n w(t, n)
* Eq. (3): normalised    R_t[c] = S_t[c] / W_t

with the serial sample-outer loop of Sect. 2.1 (zero, accumulate, divide),
an exact inclusive support cut d <= r_s (the paper evaluates the kernel only
inside the queried disk of radius r_d, Sect. 3.3), true angular distances by
Vincenty's formula (Sect. 2.1 names Haversine and Vincenty), and the
elliptical Gaussian in true world coordinates of Sect. 2.1 / Fig. 1.

Modules
-------
``sphere``   unit vectors, Vincenty distance, bearing (spherical trigonometry)
``wcs``      FITS-WCS pixel -> world for CAR (non-oblique) and SIN
``healpix``  HEALPix pixel centres (RING and NESTED order) as map targets
``grid``     brute force (all pairs) and cKDTree-accelerated gridding,
             neighbour-set statistics
``metrics``  error measures used by the parity tests and the benchmark

Every function states the passage it follows.  Where the paper is silent the
reading taken is stated next to the code (support cut inclusive, empty
pixels NaN, peak-one Gaussian, bearing measured at the target).
"""

from .sphere import unit_vectors, vincenty, bearing, splitmix64  # noqa: F401
from .wcs import wcs_world, wcs_targets  # noqa: F401
from .healpix import ring_centres, nest_centres  # noqa: F401
from .grid import (grid_bruteforce, grid_kdtree, kernel_weight,  # noqa: F401
                   neighbour_sets, grid_workload, targets_of)
from .metrics import e_val, e_val_parts, e_val_combine, e_weights, pointwise_rel  # noqa: F401
