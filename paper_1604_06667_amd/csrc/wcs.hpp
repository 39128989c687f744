// FITS-WCS pixel -> world for the target grids (Sect. 2: the targets of a
// WcsGrid are the world coordinates of the pixel centres of a FITS/WCS
// header; the projections are those of Calabretta & Greisen 2002, which the
// paper cites).  Four projections are provided:
//
//   CAR (plate carree): native phi = x, theta = y,
//   SFL (Sanson-Flamsteed; Listing 1 uses it): x = phi cos theta,
//       y = theta, so theta = y, phi = x / cos y;
//       both cylindrical with the reference point at native (0, 0): with
//       CRVAL2 = 0, lon = CRVAL1 + phi and lat = theta; otherwise (oblique)
//       the native -> celestial rotation below with the default LONPOLE
//       (phi_p = 0 for CRVAL2 > 0, 180 deg for CRVAL2 < 0) and LATPOLE =
//       +90 deg, whose native pole lies at delta_p = 90 deg - |CRVAL2|,
//       alpha_p = CRVAL1 - 180 deg (CRVAL2 > 0) or CRVAL1 (CRVAL2 < 0)
//       (Calabretta & Greisen 2002, Sect. 2.4, where sin(phi_p - phi_0) = 0),
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
// CAR and SFL, |theta| > 90; SFL, |phi| > 180 deg) returns false.
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
  // oblique cylindrical (CAR, SFL with CRVAL2 != 0): celestial longitude
  // and latitude of the native pole and the native longitude of the
  // celestial pole, radians (wcs_set_pole)
  int oblique;
  double ap, dp, php;
};

// Fill the native pole of an oblique cylindrical projection (see above).
CG_HD void wcs_set_pole(WcsDev* w) {
  const double d2r = hpx::kPi / 180.0;
  w->oblique = (w->proj == PROJ_CAR || w->proj == PROJ_SFL) && w->crval2 != 0.0;
  w->dp = (90.0 - fabs(w->crval2)) * d2r;
  w->php = w->crval2 > 0.0 ? 0.0 : hpx::kPi;
  w->ap = (w->crval2 > 0.0 ? w->crval1 - 180.0 : w->crval1) * d2r;
}

// Native (phi, theta) -> celestial (degrees out), theta given by its cosine
// and sine: the spherical rotation with the native pole at (ap, dp) and the
// celestial pole at native longitude php.
CG_HD void native_to_world(double phi, double ct, double st, double ap, double dp, double php,
                           double* lon_deg, double* lat_deg) {
  const double d2r = hpx::kPi / 180.0;
  const double sdp = sin(dp), cdp = cos(dp);
  const double dphi = phi - php;
  const double cdphi = cos(dphi), sdphi = sin(dphi);
  double s = st * sdp + ct * cdp * cdphi;
  s = s > 1.0 ? 1.0 : (s < -1.0 ? -1.0 : s);
  const double lat = asin(s);
  double lon = ap + atan2(-ct * sdphi, st * cdp - ct * sdp * cdphi);
  lon = fmod(lon / d2r, 360.0);
  if (lon < 0.0) lon += 360.0;
  *lon_deg = lon;
  *lat_deg = lat / d2r;
}

CG_HD bool wcs_pix2world(const WcsDev& w, double i, double j, double* lon_deg, double* lat_deg) {
  const double d2r = hpx::kPi / 180.0;
  const double x = w.cdelt1 * (i - w.crpix1);
  const double y = w.cdelt2 * (j - w.crpix2);
  if (w.proj == PROJ_CAR) {
    if (fabs(y) > 90.0) return false;
    if (w.oblique) {
      native_to_world(x * d2r, cos(y * d2r), sin(y * d2r), w.ap, w.dp, w.php, lon_deg, lat_deg);
      return true;
    }
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
    if (w.oblique) {
      native_to_world(dlon * d2r, cos(y * d2r), sin(y * d2r), w.ap, w.dp, w.php, lon_deg, lat_deg);
      return true;
    }
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
  native_to_world(phi, ct, st, w.crval1 * d2r, w.crval2 * d2r, hpx::kPi, lon_deg, lat_deg);
  return true;
}

}  // namespace cg
