// HEALPix RING-scheme geometry for host and device code (FP64).
//
// The paper pixelises the sphere with HEALPix (Sect. 3) and relies on the
// RING ordering, where pixels sit on iso-latitude rings, so that the part
// of a disc lying on one ring is an index interval (Sect. 3.2). The scheme
// (Gorski et al. 2005), for NSIDE = N:
//   rings i = 1 .. 4N-1, north to south;
//   polar caps (i < N, or 4N - i < N): 4k pixels with k = min(i, 4N - i),
//     1 - |z| = k^2 / (3 N^2), azimuths (j + 1/2) * 2 pi / (4k);
//   belt (N <= i <= 3N): 4N pixels, z = 4/3 - 2i / (3N), azimuths
//     (j + o) * 2 pi / (4N) with o = 1/2 when i - N is even, else 0.
// Pixel numbers count rings north to south and azimuth within a ring.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smart {

struct Ring {
  double z;      // cos(colatitude)
  double s;      // sin(colatitude), computed without cancellation
  int64_t first; // first pixel number of the ring
  int n;         // pixels on the ring
  int twice_o;   // 2 * azimuth offset in pixel steps (0 or 1)
};

__host__ __device__ inline Ring ring_info(int nside, int i) {
  Ring r;
  const int64_t N = nside;
  const double inv3nn = 1.0 / (3.0 * (double)N * (double)N);
  if (i < N) {
    const int64_t k = i;
    const double omz = (double)(k * k) * inv3nn;
    r.z = 1.0 - omz;
    r.s = sqrt(omz * (2.0 - omz));
    r.n = (int)(4 * k);
    r.first = 2 * k * (k - 1);
    r.twice_o = 1;
  } else if (i <= 3 * N) {
    r.z = (4.0 * (double)N - 2.0 * (double)i) / (3.0 * (double)N);
    r.s = sqrt((1.0 - r.z) * (1.0 + r.z));
    r.n = (int)(4 * N);
    r.first = 2 * N * (N - 1) + 4 * N * (int64_t)(i - N);
    r.twice_o = ((i - N) & 1) ? 0 : 1;
  } else {
    const int64_t k = 4 * N - i;
    const double omz = (double)(k * k) * inv3nn;
    r.z = -(1.0 - omz);
    r.s = sqrt(omz * (2.0 - omz));
    r.n = (int)(4 * k);
    r.first = 12 * N * N - 2 * k * (k + 1);
    r.twice_o = 1;
  }
  return r;
}

// Ring number (1..4N-1) and in-ring index of a RING pixel.
__host__ __device__ inline void pixel_ring(int nside, int64_t p, int* ring, int* j) {
  const int64_t N = nside;
  const int64_t ncap = 2 * N * (N - 1);
  const int64_t npix = 12 * N * N;
  if (p < ncap) {
    int64_t k = (int64_t)((1.0 + sqrt(1.0 + 2.0 * (double)p)) * 0.5);
    while (2 * k * (k - 1) > p) --k;
    while (2 * k * (k + 1) <= p) ++k;
    *ring = (int)k;
    *j = (int)(p - 2 * k * (k - 1));
  } else if (p < npix - ncap) {
    const int64_t q = p - ncap;
    *ring = (int)(q / (4 * N) + N);
    *j = (int)(q % (4 * N));
  } else {
    const int64_t q = npix - p;  // 1 .. ncap
    int64_t k = (int64_t)((1.0 + sqrt(2.0 * (double)q - 1.0)) * 0.5);
    while (2 * k * (k - 1) >= q) --k;
    while (2 * k * (k + 1) < q) ++k;
    *ring = (int)(4 * N - k);
    *j = (int)(p - (npix - 2 * k * (k + 1)));
  }
}

// Ring pixel containing the direction (z = sin dec, phi = ra), with
// one_minus_absz = 1 - |z| supplied accurately by the caller.
__host__ __device__ inline int64_t pixel_of(int nside, double z, double one_minus_absz, double phi) {
  const int64_t N = nside;
  const double two_pi = 6.283185307179586476925286766559;
  double tt = phi * (4.0 / two_pi);  // in units of pi/2
  tt = tt - 4.0 * floor(tt * 0.25);
  if (tt >= 4.0) tt = 0.0;
  const double za = fabs(z);
  if (za <= 2.0 / 3.0) {
    // belt: pixel edges are the lines phi' +- (3/4) z' = const
    const double a = (double)N * (0.5 + tt);
    const double b = (double)N * z * 0.75;
    const int64_t up = (int64_t)floor(a - b);
    const int64_t dn = (int64_t)floor(a + b);
    const int64_t ir = N + 1 + up - dn;  // 1 .. 2N+1, counted from z = 2/3
    const int64_t odd = ir & 1;
    int64_t ip = (up + dn - N + (1 - odd) + 1) >> 1;
    ip = ((ip % (4 * N)) + 4 * N) % (4 * N);
    return 2 * N * (N - 1) + (ir - 1) * 4 * N + ip;
  }
  // polar caps: edges are curves of constant (phi' mod 1) sqrt(3 (1-|z|))
  const double frac = tt - floor(tt);
  const double t = (double)N * sqrt(3.0 * one_minus_absz);
  const int64_t up = (int64_t)floor(frac * t);
  const int64_t dn = (int64_t)floor((1.0 - frac) * t);
  const int64_t k = up + dn + 1;  // ring counted from the nearest pole
  int64_t ip = (int64_t)floor(tt * (double)k);
  ip = ((ip % (4 * k)) + 4 * k) % (4 * k);
  if (z > 0) return 2 * k * (k - 1) + ip;
  return 12 * N * N - 2 * k * (k + 1) + ip;
}

// Continuous ring coordinate of a colatitude theta (radians): the ring
// number i at which the ring latitude formula reaches theta, increasing
// north to south. floor() of it bounds the rings a colatitude band touches.
__host__ __device__ inline double ring_coord(int nside, double theta) {
  const double N = nside;
  const double sqrt6 = 2.4494897427831781;
  const double theta_belt = 0.84106867056793033;  // acos(2/3)
  if (theta <= 0.0) return 0.0;
  if (theta >= 3.14159265358979323846) return 4.0 * N;
  if (theta < theta_belt) return N * sqrt6 * sin(0.5 * theta);            // 1 - z = 2 sin^2(theta/2)
  if (theta <= 3.14159265358979323846 - theta_belt) return N * (2.0 - 1.5 * cos(theta));
  return 4.0 * N - N * sqrt6 * cos(0.5 * theta);                         // 1 + z = 2 cos^2(theta/2)
}

// Rings [*lo, *hi] that may hold points within `radius` of a centre at
// colatitude theta (one ring of margin on each side; callers test exactly).
__host__ __device__ inline void ring_span(int nside, double theta, double radius, int* lo, int* hi) {
  const double a = ring_coord(nside, theta - radius);
  const double b = ring_coord(nside, theta + radius);
  int l = (int)floor(a);
  int h = (int)floor(b) + 1;
  if (l < 1) l = 1;
  if (h > 4 * nside - 1) h = 4 * nside - 1;
  *lo = l;
  *hi = h;
}

}  // namespace smart
