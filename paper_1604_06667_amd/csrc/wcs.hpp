// FITS-WCS pixel -> world for the target grids (Sect. 2: the targets of a
// WcsGrid are the world coordinates of the pixel centres of a FITS/WCS
// header; the projections are those of Calabretta & Greisen 2002, which the
// paper cites).  Four projections are provided:
//
//   CAR (non-oblique, CRVAL2 = 0): lon = CRVAL1 + x, lat = y,
//   SFL (Sanson-Flamsteed, non-oblique, CRVAL2 = 0; Listing 1 uses it):
//       x = phi cos theta, y = theta, so lat = y, lon = CRVAL1 + x / cos y,
//   SIN (zenithal orthographic) and ZEA (zenithal equal-area, Fig. 1), both
//       with LONPOLE = 180 deg: R = sqrt(x^2 + y^2), native phi =
//       atan2(x, -y), native theta = acos(R) (SIN) or 90 deg - 2 asin(R/2)
//       (ZEA), then the native -> celestial rotation with
//       (alpha_p, delta_p) = CRVAL, phi_p = 180 deg:
//         lat = asin(sin th sin dp + cos th cos dp cos(phi - phi_p))
//         lon = ap + atan2(-cos th sin(phi - phi_p),
//                          sin th cos dp - cos th sin dp cos(phi - phi_p)),
//
// with intermediate coordinates x = CDELT1 (i - CRPIX1),
// y = CDELT2 (j - CRPIX2) for 1-based pixel indices (i, j).  Degrees in,
// degrees out; a pixel without a world coordinate (SIN, R > 1; ZEA, R > 2;
// CAR and SFL, |lat| > 90; SFL, more than 180 deg from CRVAL1) returns false.
#pragma once

#include <math.h>
#include <stdint.h>

#include "healpix.hpp"

namespace cg {

enum { PROJ_CAR = 0, PROJ_SIN = 1, PROJ_SFL = 2, PROJ_ZEA = 3 };

struct WcsDev {
  int proj;
  int64_t naxis1, naxis2;
  double crpix1, crpix2, crval1, crval2, cdelt1, cdelt2;
};

CG_HD bool wcs_pix2world(const WcsDev& w, double i, double j, double* lon_deg, double* lat_deg) {
  const double d2r = hpx::kPi / 180.0;
  const double x = w.cdelt1 * (i - w.crpix1);
  const double y = w.cdelt2 * (j - w.crpix2);
  if (w.proj == PROJ_CAR) {
    if (fabs(y) > 90.0) return false;
    double lon = fmod(w.crval1 + x, 360.0);
    if (lon < 0.0) lon += 360.0;
    *lon_deg = lon;
    *lat_deg = y;
    return true;
  }
  if (w.proj == PROJ_SFL) {
    if (fabs(y) > 90.0) return false;
    const double dlon = x == 0.0 ? 0.0 : x / cos(y * d2r);
    if (!(fabs(dlon) <= 180.0)) return false;
    double lon = fmod(w.crval1 + dlon, 360.0);
    if (lon < 0.0) lon += 360.0;
    *lon_deg = lon;
    *lat_deg = y;
    return true;
  }
  // zenithal: SIN or ZEA
  const double r = sqrt(x * x + y * y) * d2r;
  const double phi = atan2(x * d2r, -y * d2r);
  double ct, st;                             // cos and sin of the native latitude
  if (w.proj == PROJ_ZEA) {
    if (r > 2.0) return false;
    // theta = 90 deg - 2 asin(R/2): sin theta = 1 - R^2/2, cos theta = R sqrt(1 - R^2/4)
    ct = r * sqrt((1.0 - 0.5 * r) * (1.0 + 0.5 * r));
    st = 1.0 - 0.5 * r * r;
  } else {
    if (r > 1.0) return false;
    ct = r;                                  // cos(theta) = R
    st = sqrt((1.0 - r) * (1.0 + r));
  }
  const double dp = w.crval2 * d2r;
  const double sdp = sin(dp), cdp = cos(dp);
  const double dphi = phi - hpx::kPi;
  const double cdphi = cos(dphi), sdphi = sin(dphi);
  double s = st * sdp + ct * cdp * cdphi;
  s = s > 1.0 ? 1.0 : (s < -1.0 ? -1.0 : s);
  const double lat = asin(s);
  double lon = w.crval1 * d2r + atan2(-ct * sdphi, st * cdp - ct * sdp * cdphi);
  lon = fmod(lon / d2r, 360.0);
  if (lon < 0.0) lon += 360.0;
  *lon_deg = lon;
  *lat_deg = lat / d2r;
  return true;
}

}  // namespace cg
