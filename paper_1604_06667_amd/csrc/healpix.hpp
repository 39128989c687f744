// HEALPix RING-scheme geometry used for the sample lookup table.
//
// The paper grids through an internal HEALPix grid (Sect. 2.2) and
// re-implements the HEALPix functions it needs (Sect. 3.2); the geometry
// below is written from the definitions in Gorski et al. (2005), the
// reference the paper cites for HEALPix:
//
//   * Npix = 12 nside^2 pixels in 4 nside - 1 iso-latitude rings.
//   * North polar cap, ring i < nside: 4 i pixels, centres at
//     z = 1 - i^2 / (3 nside^2), phi = (j + 1/2) pi / (2 i); first index 2 i (i - 1).
//   * Equatorial belt, nside <= i <= 3 nside: 4 nside pixels, centres at
//     z = 4/3 - 2 i / (3 nside), phi = (j + s/2) pi / (2 nside) with
//     s = 1 when i - nside is even and s = 0 otherwise;
//     first index 2 nside (nside - 1) + 4 nside (i - nside).
//   * South cap mirrors the north cap.
//
// Everything here is __host__ __device__ so that the CPU tests exercise the
// very code the kernels run.  FP64 throughout.
#pragma once

#include <stdint.h>
#include <math.h>

#ifdef __HIPCC__
#define CG_HD __host__ __device__ inline
#else
#define CG_HD inline
#endif

namespace cg {
namespace hpx {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;
constexpr double kHalfPi = 1.57079632679489661923;

CG_HD int64_t npix(int64_t nside) { return 12 * nside * nside; }
CG_HD int64_t nrings(int64_t nside) { return 4 * nside - 1; }

// Number of pixels in ring i (1 <= i <= 4 nside - 1).
CG_HD int64_t ring_npix(int64_t nside, int64_t i) {
  if (i < nside) return 4 * i;
  if (i <= 3 * nside) return 4 * nside;
  return 4 * (4 * nside - i);
}

// First RING index of ring i; ring_start(4 nside) = Npix is the end sentinel.
CG_HD int64_t ring_start(int64_t nside, int64_t i) {
  if (i <= nside) return 2 * i * (i - 1);
  if (i <= 3 * nside) return 2 * nside * (nside - 1) + 4 * nside * (i - nside);
  const int64_t ip = 4 * nside - i;
  return 12 * nside * nside - 2 * ip * (ip + 1);
}

// z of the centre of ring i; z(0) = 1 and z(4 nside) = -1 close the range.
CG_HD double ring_z(int64_t nside, int64_t i) {
  if (i <= 0) return 1.0;
  if (i >= 4 * nside) return -1.0;
  const double ns = (double)nside;
  if (i < nside) return 1.0 - (double)(i * i) / (3.0 * ns * ns);
  if (i <= 3 * nside) return 4.0 / 3.0 - 2.0 * (double)i / (3.0 * ns);
  const int64_t ip = 4 * nside - i;
  return -(1.0 - (double)(ip * ip) / (3.0 * ns * ns));
}

// Continuous ring coordinate of a latitude: the ring whose centre has this z
// (inverse of ring_z, monotone decreasing in z).
CG_HD double ring_of_z(int64_t nside, double z) {
  const double ns = (double)nside;
  if (z > 2.0 / 3.0) return ns * sqrt(3.0 * (1.0 - z));
  if (z < -2.0 / 3.0) return 4.0 * ns - ns * sqrt(3.0 * (1.0 + z));
  return ns * (2.0 - 1.5 * z);
}

// Angle -> RING index.  z = cos(theta) = sin(lat), st = sin(theta) = cos(lat)
// (passed separately so that near the poles 1 - |z| is not formed by
// cancellation), phi in [0, 2 pi).
CG_HD int64_t ang2pix_ring(int64_t nside, double z, double st, double phi) {
  const double za = fabs(z);
  double tt = phi * (2.0 / kPi);          // [0, 4)
  if (tt >= 4.0) tt -= 4.0;
  if (tt < 0.0) tt += 4.0;
  if (za <= 2.0 / 3.0) {
    const double t1 = (double)nside * (0.5 + tt);
    const double t2 = (double)nside * z * 0.75;
    const int64_t jp = (int64_t)floor(t1 - t2);   // index of the ascending edge line
    const int64_t jm = (int64_t)floor(t1 + t2);   // index of the descending edge line
    const int64_t ir = nside + 1 + jp - jm;       // ring counted from z = 2/3, 1..2 nside + 1
    const int64_t kshift = 1 - (ir & 1);
    int64_t ip = (jp + jm - nside + kshift + 1) / 2;
    const int64_t nl4 = 4 * nside;
    ip %= nl4;
    if (ip < 0) ip += nl4;
    return 2 * nside * (nside - 1) + (ir - 1) * nl4 + ip;
  }
  const double tp = tt - floor(tt);
  const double tmp = (double)nside * st * sqrt(3.0 / (1.0 + za));   // nside sqrt(3 (1 - |z|))
  const int64_t jp = (int64_t)(tp * tmp);
  const int64_t jm = (int64_t)((1.0 - tp) * tmp);
  int64_t ir = jp + jm + 1;                        // ring counted from the nearer pole
  if (ir > nside) ir = nside;
  int64_t ip = (int64_t)(tt * (double)ir);
  ip %= 4 * ir;
  if (ip < 0) ip += 4 * ir;
  if (z > 0.0) return 2 * ir * (ir - 1) + ip;
  return 12 * nside * nside - 2 * ir * (ir + 1) + ip;
}

CG_HD int64_t isqrt64(int64_t v) {
  int64_t r = (int64_t)sqrt((double)v);
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

// RING index -> (ring i, position j in ring).
CG_HD void pix2ring(int64_t nside, int64_t p, int64_t* ring, int64_t* j) {
  const int64_t ncap = 2 * nside * (nside - 1);
  const int64_t np = 12 * nside * nside;
  if (p < ncap) {
    int64_t i = (1 + isqrt64(1 + 2 * p)) / 2;
    while (2 * i * (i - 1) > p) --i;
    while (2 * (i + 1) * i <= p) ++i;
    *ring = i;
    *j = p - 2 * i * (i - 1);
  } else if (p < np - ncap) {
    const int64_t q = p - ncap;
    *ring = q / (4 * nside) + nside;
    *j = q % (4 * nside);
  } else {
    const int64_t q = np - p;                       // 1 .. ncap
    int64_t ip = (1 + isqrt64(2 * q - 1)) / 2;      // ring counted from the south pole
    while (2 * ip * (ip - 1) >= q) --ip;
    while (2 * ip * (ip + 1) < q) ++ip;
    *ring = 4 * nside - ip;
    *j = p - (np - 2 * ip * (ip + 1));
  }
}

// Centre of RING pixel p: z and phi.
CG_HD void pix2ang_ring(int64_t nside, int64_t p, double* z, double* phi) {
  int64_t i, j;
  pix2ring(nside, p, &i, &j);
  *z = ring_z(nside, i);
  double shift;
  int64_t n;
  if (i < nside) { n = 4 * i; shift = 0.5; }
  else if (i <= 3 * nside) { n = 4 * nside; shift = ((i - nside) & 1) ? 0.0 : 0.5; }
  else { n = 4 * (4 * nside - i); shift = 0.5; }
  *phi = ((double)j + shift) * kTwoPi / (double)n;
}

// ---------------------------------------------------------------------------
// Ring lookup for a spherical cap (the target-centric form of the paper's
// per-ring disk query shifted in longitude, Sect. 3.3 Eq. 4-5).
//
// For ring i, returns up to two inclusive RING-index ranges that contain
// every pixel of ring i holding a point within angular radius rho of the
// cap centre (cz = cos theta_c, cs = sin theta_c, cphi).  Properties used:
//   * a point whose pixel lies in ring i has z in [z(i+1), z(i-1)];
//   * within ring i, pixel j covers longitudes inside
//     [(j - 1/2), (j + 1)] * 2 pi / n_i (cap pixels: exactly [j, j+1));
//   * over a latitude band the half-width in longitude of the cap,
//     dphi(z) = acos((cos rho - z cz) / (sqrt(1 - z^2) cs)), is largest at
//     z* = cz / cos rho, so its maximum over [a, b] is dphi(clamp(z*, a, b)).
// One pixel of slack is added on each side.  Returns the number of ranges.
CG_HD int ring_cap_ranges(int64_t nside, int64_t i, double cz, double cs, double cphi,
                          double rho, int64_t lo[2], int64_t hi[2]) {
  const int64_t n = ring_npix(nside, i);
  const int64_t s0 = ring_start(nside, i);
  // latitude band of the cap (pole-containing caps reach z = +-1)
  const double thc = atan2(cs, cz);
  const double zmax = (thc - rho <= 0.0) ? 1.0 : cos(thc - rho);
  const double zmin = (thc + rho >= kPi) ? -1.0 : cos(thc + rho);
  const double eps = 1e-12;
  const double zl = ring_z(nside, i + 1) - eps;
  const double zh = ring_z(nside, i - 1) + eps;
  const double a = zl > zmin ? zl : zmin;
  const double b = zh < zmax ? zh : zmax;
  if (a > b) return 0;
  bool full = (rho >= kHalfPi);
  double dphi = kPi;
  if (!full) {
    const double crho = cos(rho);
    double zs = cz / crho;
    zs = zs < a ? a : (zs > b ? b : zs);
    const double sz = sqrt(fmax(0.0, (1.0 - zs) * (1.0 + zs)));
    const double den = sz * cs;
    if (den <= 0.0) {
      full = true;
    } else {
      const double arg = (crho - zs * cz) / den;
      if (arg <= -1.0) full = true;
      else dphi = (arg >= 1.0) ? 0.0 : acos(arg);
    }
  }
  if (!full) {
    const double scale = (double)n / kTwoPi;
    int64_t jl = (int64_t)floor((cphi - dphi) * scale) - 1;
    int64_t jh = (int64_t)floor((cphi + dphi) * scale) + 1;
    if (jh - jl + 1 >= n) {
      full = true;
    } else if (jl < 0) {
      if (jh < 0) { lo[0] = s0 + jl + n; hi[0] = s0 + jh + n; return 1; }
      lo[0] = s0; hi[0] = s0 + jh;
      lo[1] = s0 + jl + n; hi[1] = s0 + n - 1;
      return 2;
    } else if (jh >= n) {
      if (jl >= n) { lo[0] = s0 + jl - n; hi[0] = s0 + jh - n; return 1; }
      lo[0] = s0; hi[0] = s0 + jh - n;
      lo[1] = s0 + jl; hi[1] = s0 + n - 1;
      return 2;
    } else {
      lo[0] = s0 + jl; hi[0] = s0 + jh;
      return 1;
    }
  }
  lo[0] = s0; hi[0] = s0 + n - 1;
  return 1;
}

// One disk of angular radius rho around a point, prepared for the per-ring
// lookup (the quantities below depend only on the point and rho).
struct DiskPrep {
  double tz, ts;        // cos and sin of the colatitude of the centre
  double zmin, zmax;    // latitude band of the disk (z = cos theta)
  double crho, zstar;   // cos(rho); z at which the disk is widest in longitude
  int all;              // rho >= pi/2: every ring may be fully inside
};

CG_HD void disk_prepare(double tz, double ts, double rho, DiskPrep* d) {
  const double th = atan2(ts, tz);
  d->tz = tz;
  d->ts = ts;
  d->zmax = (th - rho <= 0.0) ? 1.0 : cos(th - rho);
  d->zmin = (th + rho >= kPi) ? -1.0 : cos(th + rho);
  d->crho = cos(rho);
  d->all = rho >= kHalfPi;
  d->zstar = d->all ? 0.0 : tz / d->crho;
}

// Half-width in longitude of the part of a latitude band [zl, zh] that can
// lie within the disk: the same bound as in ring_cap_ranges.  Returns 0 when
// the band misses the disk, 2 when the whole band may be inside (*dphi
// untouched), else 1 with the half-width in *dphi.
CG_HD int band_disk_halfwidth(double zl, double zh, const DiskPrep& d, double* dphi) {
  const double a = zl > d.zmin ? zl : d.zmin;
  const double b = zh < d.zmax ? zh : d.zmax;
  if (a > b) return 0;
  if (d.all) return 2;
  double zs = d.zstar;
  zs = zs < a ? a : (zs > b ? b : zs);
  const double sz = sqrt(fmax(0.0, (1.0 - zs) * (1.0 + zs)));
  const double den = sz * d.ts;
  if (den <= 0.0) return 2;
  const double arg = (d.crho - zs * d.tz) / den;
  if (arg <= -1.0) return 2;
  *dphi = (arg >= 1.0) ? 0.0 : acos(arg);
  return 1;
}

// Latitude band holding every point whose pixel lies in ring i, widened by
// 1e-12 for rounding.
CG_HD void ring_band(int64_t nside, int64_t i, double* zl, double* zh) {
  *zl = ring_z(nside, i + 1) - 1e-12;
  *zh = ring_z(nside, i - 1) + 1e-12;
}

CG_HD int ring_disk_halfwidth(int64_t nside, int64_t i, const DiskPrep& d, double* dphi) {
  double zl, zh;
  ring_band(nside, i, &zl, &zh);
  return band_disk_halfwidth(zl, zh, d, dphi);
}

// Longitude of a point relative to a reference longitude, in (-pi, pi].
CG_HD double rel_lon(double phi, double ref) {
  double r = phi - ref;
  if (r > kPi) r -= kTwoPi;
  if (r <= -kPi) r += kTwoPi;
  return r;
}

// Union over a set of disks of their longitude windows on ring i, as one
// window [*plo, *phi] (absolute longitudes, possibly outside [0, 2 pi)) or
// the whole ring (*full).  rel[k] is the centre longitude of disk k relative
// to ref.  Returns 0 when no disk meets the ring.  The tile kernel forms the
// same union with one ring per lane.
CG_HD int ring_union_window(int64_t nside, int64_t i, const DiskPrep* d, const double* rel,
                            int n, double ref, double* plo, double* phi, int* full) {
  double lo = 1e300, hi = -1e300;
  int any = 0, f = 0;
  for (int k = 0; k < n; ++k) {
    double w;
    const int r = ring_disk_halfwidth(nside, i, d[k], &w);
    if (r == 2) f = 1;
    if (r == 1) {
      any = 1;
      lo = fmin(lo, rel[k] - w);
      hi = fmax(hi, rel[k] + w);
    }
  }
  if (!any && !f) return 0;
  if (f || hi - lo >= kTwoPi) {
    *full = 1;
  } else {
    *full = 0;
    *plo = ref + lo;
    *phi = ref + hi;
  }
  return 1;
}

// Longitude offset, in pixel widths, of the first pixel centre of ring i:
// one half in the polar caps and on every other equatorial ring, else 0.
CG_HD double ring_phase(int64_t nside, int64_t i) {
  if (i < nside || i > 3 * nside) return 0.5;
  return ((i - nside) & 1) ? 0.0 : 0.5;
}

// Pixel ranges of ring i covering the longitude window [plo, phi] (plo may
// be negative and phi beyond 2 pi; phi - plo < 2 pi).  Pixel j of a ring
// with n pixels and phase s covers longitudes within
// [j + s - 1/2, j + s + 1/2] * 2 pi / n at every latitude of the ring (in the
// polar caps the pixel index is the floor of the scaled longitude; in the
// equatorial belt the pixel edges run diagonally between the vertices at the
// centre longitude +- half a pixel), so j is kept when that interval meets
// the window, with 1e-6 pixel of slack for rounding.  full != 0 selects the
// whole ring.
CG_HD int ring_window_ranges(int64_t nside, int64_t i, double plo, double phi, int full,
                             int64_t lo[2], int64_t hi[2]) {
  const int64_t n = ring_npix(nside, i);
  const int64_t s0 = ring_start(nside, i);
  if (!full) {
    const double scale = (double)n / kTwoPi;
    const double ph = ring_phase(nside, i);
    const int64_t jl = (int64_t)ceil(plo * scale - ph - 0.5 - 1e-6);
    const int64_t jh = (int64_t)floor(phi * scale - ph + 0.5 + 1e-6);
    if (jh - jl + 1 < n) {
      // bring jl into [0, n)
      int64_t sh = 0;
      if (jl < 0) sh = ((-jl) / n + 1) * n;
      else if (jl >= n) sh = -(jl / n) * n;
      const int64_t a = jl + sh, b = jh + sh;
      if (b < n) {
        lo[0] = s0 + a;
        hi[0] = s0 + b;
        return 1;
      }
      lo[0] = s0 + a;
      hi[0] = s0 + n - 1;
      lo[1] = s0;
      hi[1] = s0 + (b - n);
      return 2;
    }
  }
  lo[0] = s0;
  hi[0] = s0 + n - 1;
  return 1;
}

// Rings whose pixels can meet a cap of radius rho around colatitude thc:
// [first, last], clamped to [1, 4 nside - 1].  Conservative by two rings.
CG_HD void cap_ring_span(int64_t nside, double cz, double cs, double rho,
                         int64_t* first, int64_t* last) {
  const double thc = atan2(cs, cz);
  const double zmax = (thc - rho <= 0.0) ? 1.0 : cos(thc - rho);
  const double zmin = (thc + rho >= kPi) ? -1.0 : cos(thc + rho);
  int64_t f = (int64_t)floor(ring_of_z(nside, zmax)) - 2;
  int64_t l = (int64_t)ceil(ring_of_z(nside, zmin)) + 2;
  if (f < 1) f = 1;
  if (l > 4 * nside - 1) l = 4 * nside - 1;
  *first = f;
  *last = l;
}

// Ordering of sight-line targets along a space-filling curve, so that runs
// of consecutive targets are compact.  A point's base face and in-face cell
// (ix, iy) at a power-of-two nside follow Gorski et al. (2005), as for the
// NESTED scheme; within the face the cells are numbered along a Hilbert
// curve instead of the NESTED (Morton) one.  A run of a Hilbert curve is
// always one connected piece of the face, while a Morton run jumps between
// quadrants, so tiles of consecutive targets cover less sky and meet fewer
// candidate samples outside their targets' supports.
// Base face and in-face cell of a point (z = cos theta, st = sin theta).
CG_HD void ang2xyf(int64_t nside, double z, double st, double phi, int64_t* face_out,
                   int64_t* ix_out, int64_t* iy_out) {
  const double za = fabs(z);
  double tt = phi * (2.0 / kPi);
  if (tt >= 4.0) tt -= 4.0;
  if (tt < 0.0) tt += 4.0;
  int64_t face, ix, iy;
  if (za <= 2.0 / 3.0) {
    const double t1 = (double)nside * (0.5 + tt);
    const double t2 = (double)nside * z * 0.75;
    const int64_t jp = (int64_t)floor(t1 - t2);
    const int64_t jm = (int64_t)floor(t1 + t2);
    const int64_t ifp = jp / nside;
    const int64_t ifm = jm / nside;
    if (ifp == ifm) face = (ifp & 3) | 4;
    else if (ifp < ifm) face = ifp & 3;
    else face = (ifm & 3) + 8;
    ix = jm & (nside - 1);
    iy = nside - (jp & (nside - 1)) - 1;
  } else {
    int64_t ntt = (int64_t)tt;
    if (ntt > 3) ntt = 3;
    const double tp = tt - (double)ntt;
    const double tmp = (double)nside * st * sqrt(3.0 / (1.0 + za));
    int64_t jp = (int64_t)(tp * tmp);
    int64_t jm = (int64_t)((1.0 - tp) * tmp);
    if (jp > nside - 1) jp = nside - 1;
    if (jm > nside - 1) jm = nside - 1;
    if (z >= 0) { face = ntt; ix = nside - jm - 1; iy = nside - jp - 1; }
    else { face = ntt + 8; ix = jp; iy = jm; }
  }
  *face_out = face;
  *ix_out = ix;
  *iy_out = iy;
}

// Position of cell (x, y) of an n x n grid (n a power of two) along the
// Hilbert curve: from the top bit down, the quadrant holding the cell
// contributes its rank along the curve, and the cell's remaining
// coordinates are reflected or transposed into the orientation that
// quadrant's sub-curve has.
CG_HD uint64_t hilbert_index(int64_t n, int64_t x, int64_t y) {
  uint64_t d = 0;
  for (int64_t s = n / 2; s > 0; s /= 2) {
    const int64_t rx = (x & s) != 0, ry = (y & s) != 0;
    d += (uint64_t)s * (uint64_t)s * (uint64_t)((3 * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = n - 1 - x;
        y = n - 1 - y;
      }
      const int64_t t = x;
      x = y;
      y = t;
    }
  }
  return d;
}

// Sight-line ordering key: face * nside^2 + Hilbert position in the face.
CG_HD int64_t ang2hilbert(int64_t nside, double z, double st, double phi) {
  int64_t face, ix, iy;
  ang2xyf(nside, z, st, phi, &face, &ix, &iy);
  return face * nside * nside + (int64_t)hilbert_index(nside, ix, iy);
}

// ---------------------------------------------------------------------------
// Pixel centres as targets (a full HEALPix map gridded through the sight-line
// path; the paper's App. A.1 grids onto the nside = 512 pixel centres).

// The even bits of v packed together (one coordinate of a NESTED in-face
// index, whose bits interleave the two).
CG_HD uint64_t compact_bits(uint64_t v) {
  v &= 0x5555555555555555ull;
  v = (v | (v >> 1)) & 0x3333333333333333ull;
  v = (v | (v >> 2)) & 0x0F0F0F0F0F0F0F0Full;
  v = (v | (v >> 4)) & 0x00FF00FF00FF00FFull;
  v = (v | (v >> 8)) & 0x0000FFFF0000FFFFull;
  v = (v | (v >> 16)) & 0x00000000FFFFFFFFull;
  return v;
}

// NESTED index -> (ring i, 0-based position j in the ring).  Pixel p lies in
// base face f = p / nside^2 (face row f / 4: north, equator, south; column
// f % 4) at in-face position (ix, iy), the even and odd bits of p mod
// nside^2.  Its ring is (2 + row) nside - ix - iy - 1, and its position
// along the ring, counted in half pixels from longitude 0, is
// col2 nr + ix - iy + shift, where nr is the ring's pixel count / 4,
// col2 = 2 col (+1 off the equatorial row) is the face centre's longitude
// in units of pi / 4, and shift = 1 on rings whose first centre sits half
// a pixel east of longitude 0 (Gorski et al. 2005, Sect. 4).
CG_HD void nest2ring_ij(int64_t nside, int64_t p, int64_t* ring, int64_t* j) {
  const int64_t nn = nside * nside;
  const int64_t f = p / nn, loc = p - f * nn;
  const int64_t ix = (int64_t)compact_bits((uint64_t)loc);
  const int64_t iy = (int64_t)compact_bits((uint64_t)loc >> 1);
  const int64_t row = f >> 2, col = f & 3;
  const int64_t i = (2 + row) * nside - ix - iy - 1;
  int64_t nr, kshift;
  if (i < nside) { nr = i; kshift = 0; }
  else if (i > 3 * nside) { nr = 4 * nside - i; kshift = 0; }
  else { nr = nside; kshift = (i - nside) & 1; }
  const int64_t col2 = 2 * col + ((row & 1) ? 0 : 1);
  int64_t jp = (col2 * nr + ix - iy + 1 + kshift) / 2;   // 1-based
  if (jp > 4 * nr) jp -= 4 * nr;
  if (jp < 1) jp += 4 * nr;
  *ring = i;
  *j = jp - 1;
}

// Centre of pixel j (0-based) of ring i as (lon, lat) in degrees.  Cap rings
// form 1 - |z| = i^2 / (3 nside^2) directly, so that latitudes next to the
// poles keep full precision.
CG_HD void ring_pixel_centre(int64_t nside, int64_t i, int64_t j, double* lon_deg,
                             double* lat_deg) {
  const double ns = (double)nside;
  double z, st, phi;
  if (i < nside || i > 3 * nside) {
    const int64_t ic = i < nside ? i : 4 * nside - i;
    const double omz = (double)(ic * ic) / (3.0 * ns * ns);
    z = i < nside ? 1.0 - omz : omz - 1.0;
    st = sqrt(omz * (2.0 - omz));
    phi = ((double)j + 0.5) * kHalfPi / (double)ic;
  } else {
    z = (double)(2 * nside - i) * 2.0 / (3.0 * ns);
    st = sqrt((1.0 - z) * (1.0 + z));
    const double s = ((i - nside) & 1) ? 0.0 : 0.5;
    phi = ((double)j + s) * kHalfPi / ns;
  }
  *lon_deg = phi * (180.0 / kPi);
  *lat_deg = atan2(z, st) * (180.0 / kPi);
}

// Centre of pixel p of an nside map in RING (nested = false) or NESTED order.
CG_HD void pix_centre(int64_t nside, int64_t p, bool nested, double* lon_deg, double* lat_deg) {
  int64_t i, j;
  if (nested) nest2ring_ij(nside, p, &i, &j);
  else pix2ring(nside, p, &i, &j);
  ring_pixel_centre(nside, i, j, lon_deg, lat_deg);
}

// ---------------------------------------------------------------------------
// Query disks shifted along rings (Sect. 3.3, Eq. 4-5): the sample-centric
// lookup computes one disk per ring, around the ring's reference pixel, and
// moves it to every other pixel of the ring by integer index shifts.

// z and sin(theta) of the centre of ring i (0 and 4 nside give the poles);
// cap rings form 1 - |z| directly, as in ring_pixel_centre.
CG_HD void ring_zs(int64_t nside, int64_t i, double* z, double* st) {
  if (i <= 0 || i >= 4 * nside) {
    *z = i <= 0 ? 1.0 : -1.0;
    *st = 0.0;
    return;
  }
  const double ns = (double)nside;
  if (i < nside || i > 3 * nside) {
    const int64_t ic = i < nside ? i : 4 * nside - i;
    const double omz = (double)(ic * ic) / (3.0 * ns * ns);
    *z = i < nside ? 1.0 - omz : omz - 1.0;
    *st = sqrt(omz * (2.0 - omz));
  } else {
    *z = (double)(2 * nside - i) * 2.0 / (3.0 * ns);
    *st = sqrt((1.0 - *z) * (1.0 + *z));
  }
}

// Largest angular distance from the centre of a pixel of ring i to any point
// of that pixel.  Every such point lies in the latitude band
// [z(i+1), z(i-1)] within half a pixel width of the centre's longitude (the
// box used by ring_window_ranges); the distance grows with the longitude
// offset and, along a meridian, is largest at an end of the band, so the
// box's corners bound it.  Widened by a relative 1e-9 for rounding.
CG_HD double ring_pixel_radius(int64_t nside, int64_t i) {
  double z, st;
  ring_zs(nside, i, &z, &st);
  const double ch = cos(kPi / (double)ring_npix(nside, i));   // half a pixel width
  double m = 1.0;
  for (int e = -1; e <= 1; e += 2) {
    double z2, s2;
    ring_zs(nside, i + e, &z2, &s2);
    const double c = z * z2 + st * s2 * ch;
    m = c < m ? c : m;
  }
  m = m < -1.0 ? -1.0 : m;
  return acos(m) * (1.0 + 1e-9) + 1e-12;
}

// The reference pixel of ring i: the one whose centre is nearest longitude
// pi; on rings with a centre half a pixel either side of pi, the east one.
CG_HD int64_t ring_ref_pixel(int64_t nside, int64_t i) { return ring_npix(nside, i) / 2; }

// Eq. 4: the shift, in pixels of a ring of n2 pixels, that moves a point by
// k pixels of a ring of n1 pixels (an angle of k 2 pi / n1), rounded to the
// nearest integer with halves away from zero.  Exact integer arithmetic.
CG_HD int64_t disk_shift(int64_t k, int64_t n2, int64_t n1) {
  const int64_t num = k * n2;
  const int64_t a = num < 0 ? -num : num;
  const int64_t q = (2 * a + n1) / (2 * n1);
  return num < 0 ? -q : q;
}

// Query disk of the reference pixel of ring i, restricted to ring i2: the
// window [*lo, *hi] of pixel positions in ring i2 (unwrapped: it may start
// below 0 or end past the ring's last pixel) whose centres lie within
// rd = rs + R(i) + R(i2) + 1e-9 of the reference centre (R = ring_pixel_radius,
// so a sample and a target less than rs apart always have their pixels'
// centres within rd), widened by one pixel on each side so that it still
// holds the disk after the rounded shift of Eq. 4.  Returns 0 when the ring
// misses the disk, 1 for a window, 2 for the whole ring.
CG_HD int ref_disk_window(int64_t nside, int64_t i, int64_t i2, double rs, int64_t* lo,
                          int64_t* hi) {
  const int64_t n1 = ring_npix(nside, i), n2 = ring_npix(nside, i2);
  const double rd = rs + ring_pixel_radius(nside, i) + ring_pixel_radius(nside, i2) + 1e-9;
  if (rd >= kPi) return 2;
  double zc, sc, z, s;
  ring_zs(nside, i, &zc, &sc);
  ring_zs(nside, i2, &z, &s);
  const double den = sc * s;
  const double arg = (cos(rd) - zc * z) / den;
  if (arg > 1.0) return 0;
  if (arg <= -1.0) return 2;
  const double dphi = acos(arg);
  const double phc = ((double)ring_ref_pixel(nside, i) + ring_phase(nside, i)) * kTwoPi / (double)n1;
  const double scale = (double)n2 / kTwoPi, ph = ring_phase(nside, i2);
  const int64_t a = (int64_t)ceil((phc - dphi) * scale - ph) - 1;
  const int64_t b = (int64_t)floor((phc + dphi) * scale - ph) + 1;
  if (b - a + 1 >= n2) return 2;
  *lo = a;
  *hi = b;
  return 1;
}

// Eq. 5 applied to a window: the positions [lo, hi] of ring i2 moved by dp
// pixels, wrapped around the ring, as one or two RING index ranges
// [a[k], b[k]].  Requires hi - lo + 1 < the ring's pixel count.
CG_HD int shifted_window(int64_t nside, int64_t i2, int64_t lo, int64_t hi, int64_t dp,
                         int64_t a[2], int64_t b[2]) {
  const int64_t n = ring_npix(nside, i2), s0 = ring_start(nside, i2);
  int64_t x = (lo + dp) % n;
  if (x < 0) x += n;
  const int64_t y = x + (hi - lo);
  if (y < n) {
    a[0] = s0 + x;
    b[0] = s0 + y;
    return 1;
  }
  a[0] = s0 + x;
  b[0] = s0 + n - 1;
  a[1] = s0;
  b[1] = s0 + (y - n);
  return 2;
}

// Rings a shifted query disk can reach on either side of its own ring: the
// ring centres lie at least 2 / (3 nside) apart in colatitude (the belt's
// spacing; cap rings are further apart), so a disk of radius rd spans at
// most 1.5 rd nside + 1 rings each way.  Host-side helper.
inline int64_t disk_ring_reach(int64_t nside, double rs) {
  double rmax = 0.0;
  for (int64_t i = 1; i < 4 * nside; ++i) {
    const double r = ring_pixel_radius(nside, i);
    rmax = r > rmax ? r : rmax;
  }
  const double rd = rs + 2.0 * rmax + 1e-9;
  int64_t d = (int64_t)ceil(1.5 * rd * (double)nside) + 2;
  return d < 4 * nside ? d : 4 * nside;
}

}  // namespace hpx
}  // namespace cg
