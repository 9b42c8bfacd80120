// Detection step (Sect. 6.1): the pixels of an aperture-mass map whose value
// is higher than those of their eight direct HEALPix neighbours, above a
// threshold (on the value, or on the value over a noise map).
//
// Neighbours. Each of the 12 base faces of the construction is a
// curvilinear square of N x N cells with continuous coordinates (alpha,
// beta) in [0, N)^2, (0, 0) at its northern corner, alpha growing to the
// south-east and beta to the south-west: in the belt the two edge-line
// coordinates of the point->pixel construction, Jp = N (1/2 + tt - 3z/4)
// and Jm = N (1/2 + tt + 3z/4) (tt = 2 phi / pi), shifted per face; in the
// caps tp t and (1 - tp) t with t = N sqrt(3 (1 - |z|)) and tp = tt mod 1,
// from the north pole for the northern faces and turned round for the
// southern ones. Every grid edge is shared by two cells, so the four edge
// neighbours are the pixels of points just across the middle of each edge
// (the face chart continued a little past the face). The neighbour across
// a corner is the common edge neighbour, other than the pixel itself, of
// the two edge neighbours beside that corner; if those two share an edge,
// only three pixels meet there (the 24 pixels at the eight corners where
// three faces meet have seven neighbours). A cell away from its face's
// border has all eight neighbours in its own face, the cells at (alpha +- 1,
// beta +- 1), which integer arithmetic finds (cell_pixel); only the cells on
// a face border take the chart probes.
//
// A pixel with a neighbour that is not in the map is not a detection, and
// "higher" is strict.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <string>

#include "hpx_ring.h"
#include "smart_internal.h"

namespace smart {

namespace {

constexpr double kProbe = 1e-6;  // distance of an edge probe beyond the edge, in cells

// Face and cell of a RING pixel, in integers: in the caps the quadrant
// and the position along the ring, in the belt the edge-line indices of the
// pixel centre, Jp - 1/2 = j + floor((i - N) / 2) and
// Jm - 1/2 = j + floor((3N - i) / 2).
__device__ inline void pixel_cell(int nside, int64_t p, int* face, int* ia, int* ib) {
  const int N = nside;
  int i, j;
  pixel_ring(N, p, &i, &j);
  if (i < N) {  // north cap: ring i has i cells per face, alpha + beta = i - 1
    const int g = j / i, q = j % i;
    *face = g;
    *ia = q;
    *ib = i - 1 - q;
  } else if (i <= 3 * N) {
    const int jp = j + ((i - N) >> 1);
    const int jm = j + ((3 * N - i) >> 1);
    const int fp = jp / N, fm = jm / N;
    *face = fp == fm ? 4 + (fp & 3) : (fp < fm ? (fp & 3) : 8 + (fm & 3));
    *ia = jp - fp * N;
    *ib = (fm + 1) * N - 1 - jm;
  } else {  // south cap: k = 4N - i cells per face on the ring
    const int k = 4 * N - i;
    const int g = j / k, q = j % k;
    *face = 8 + g;
    *ia = N - k + q;
    *ib = N - 1 - q;
  }
}

// The pixel at face coordinates (alpha, beta) of face f (slightly outside
// the face is fine): the chart's inverse, then the point->pixel map.
__device__ inline int64_t chart_pixel(int nside, int f, double al, double be) {
  const double N = (double)nside;
  const int g = f & 3, row = f >> 2;
  double z, omz, tt;
  const double s_n = al + be, s_s = 2.0 * N - al - be;
  if (row == 0 && s_n < N) {  // north cap
    tt = g + (s_n > 0.0 ? al / s_n : 0.0);
    omz = s_n * s_n / (3.0 * N * N);
    z = 1.0 - omz;
  } else if (row == 2 && s_s < N) {  // south cap
    tt = g + (s_s > 0.0 ? (N - be) / s_s : 0.0);
    omz = s_s * s_s / (3.0 * N * N);
    z = -(1.0 - omz);
  } else {  // belt form of any face
    const double off_p = (row == 2 ? g + 1 : g) * N;
    const double off_m = (row == 0 ? g + 2 : g + 1) * N;
    const double jp = al + off_p, jm = off_m - be;
    z = (jm - jp) / (1.5 * N);
    tt = (jp + jm) / (2.0 * N) - 0.5;
    omz = 1.0 - fabs(z);
  }
  tt -= 4.0 * floor(tt * 0.25);
  return pixel_of(nside, z, omz, tt * (0.5 * 3.141592653589793238462643383279502884));
}

// RING pixel of cell (a, b) of face f, 0 <= a, b < N: the integer form of
// chart_pixel at the cell's centre (the inverse of pixel_cell). North cap
// cells lie on ring a + b + 1 at position g i + a of the ring; south cap
// cells on ring 4N - k, k = 2N - 1 - a - b, at position g k + N - 1 - b; belt
// cells have edge-line indices j_p = a + off_p and j_m = off_m - b - 1, so
// their ring is 2N - (j_m - j_p) and their position j_p - (i - N) / 2
// (mod 4N).
__device__ inline int64_t cell_pixel(int nside, int f, int a, int b) {
  const int64_t N = nside;
  const int g = f & 3, row = f >> 2;
  if (row == 0 && a + b + 1 < nside) {
    const int64_t i = a + b + 1;
    return 2 * i * (i - 1) + g * i + a;
  }
  if (row == 2 && a + b >= nside) {
    const int64_t k = 2 * N - 1 - a - b;
    return 12 * N * N - 2 * k * (k + 1) + g * k + (N - 1 - b);
  }
  const int64_t off_p = (row == 2 ? g + 1 : g) * N, off_m = (row == 0 ? g + 2 : g + 1) * N;
  const int64_t jp = a + off_p, jm = off_m - b - 1;
  const int64_t i = 2 * N - (jm - jp);
  const int64_t j = (jp - ((i - N) >> 1)) & (4 * N - 1);  // 4N is a power of two
  return 2 * N * (N - 1) + 4 * N * (i - N) + j;
}

// Pixels across the four edges (alpha-, beta-, alpha+, beta+).
__device__ inline void edge_neighbours(int nside, int64_t p, int64_t e[4]) {
  int f, a, b;
  pixel_cell(nside, p, &f, &a, &b);
  e[0] = chart_pixel(nside, f, a - kProbe, b + 0.5);
  e[1] = chart_pixel(nside, f, a + 0.5, b - kProbe);
  e[2] = chart_pixel(nside, f, a + 1.0 + kProbe, b + 0.5);
  e[3] = chart_pixel(nside, f, a + 0.5, b + 1.0 + kProbe);
}

// Value of pixel q in the dense map, NaN when q is not in the map
__device__ inline double map_value(const double* dense, int64_t d0, int64_t dn, int64_t q) {
  const int64_t k = q - d0;
  return (k >= 0 && k < dn) ? dense[k] : __builtin_nan("");
}

__global__ void k_fill_nan(double* d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = __builtin_nan("");
}

__global__ void k_scatter_values(const int64_t* pix, const double* val, int64_t n, int64_t d0, double* dense) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dense[pix[i] - d0] = val[i];
}

// flags[i] = 1 when pixel pix[i] is a detection
__global__ void k_detect(int nside, const int64_t* pix, const double* val, const double* noise_sd, int64_t n,
                         double threshold, const double* dense, int64_t d0, int64_t dn, int* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t p = pix[i];
  const double v = val[i];
  int ok = v == v;  // not NaN
  if (noise_sd) {
    const double sd = noise_sd[i];
    ok = ok && sd > 0.0 && v / sd >= threshold;
  } else {
    ok = ok && v >= threshold;
  }
  int f, ca, cb;
  pixel_cell(nside, p, &f, &ca, &cb);
  if (ok && ca > 0 && cb > 0 && ca < nside - 1 && cb < nside - 1) {
    // inside its face: the eight neighbours are the cells around it
    for (int da = -1; da <= 1 && ok; ++da)
      for (int db = -1; db <= 1 && ok; ++db)
        if (da != 0 || db != 0) ok = v > map_value(dense, d0, dn, cell_pixel(nside, f, ca + da, cb + db));
    flags[i] = ok;
    return;
  }
  int64_t e[4];
  if (ok) {
    edge_neighbours(nside, p, e);
    for (int k = 0; k < 4 && ok; ++k) ok = v > map_value(dense, d0, dn, e[k]);  // false for NaN (absent)
  }
  if (ok) {
    int64_t ee[4][4];
    for (int k = 0; k < 4; ++k) edge_neighbours(nside, e[k], ee[k]);
    for (int k = 0; k < 4 && ok; ++k) {
      const int a = k, b = (k + 1) & 3;
      bool three = false;
      for (int m = 0; m < 4; ++m) three = three || ee[a][m] == e[b];
      if (three) continue;
      int64_t d = -1;
      for (int m = 0; m < 4 && d < 0; ++m) {
        const int64_t c = ee[a][m];
        if (c == p) continue;
        for (int l = 0; l < 4; ++l)
          if (ee[b][l] == c) d = c;
      }
      ok = d >= 0 && v > map_value(dense, d0, dn, d);
    }
  }
  flags[i] = ok;
}

unsigned grid_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

#define DCHK(x)                                                                 \
  do {                                                                          \
    hipError_t e_ = (x);                                                        \
    if (e_ != hipSuccess) {                                                     \
      release();                                                                \
      set_error(std::string("detection: ") + hipGetErrorString(e_) + " at " #x); \
      return SMART_EDEVICE;                                                     \
    }                                                                           \
  } while (0)

int detect_peaks(smart_ctx ctx, int nside, int64_t n, const int64_t* pix, const double* val, const double* noise_sd,
                 double threshold, int64_t* peaks, int64_t* n_peaks, hipStream_t st) {
  *n_peaks = 0;
  if (n == 0) return SMART_OK;
  int64_t ends[2] = {0, 0};
  double* dense = nullptr;
  int* flags = nullptr;
  int64_t* count = nullptr;
  auto release = [&]() {
    scratch_free(dense, st);
    scratch_free(flags, st);
    scratch_free(count, st);
    dense = nullptr;
    flags = nullptr;
    count = nullptr;
  };
  DCHK(hipMemcpyAsync(&ends[0], pix, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  DCHK(hipMemcpyAsync(&ends[1], pix + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  DCHK(hipStreamSynchronize(st));
  const int64_t d0 = ends[0], dn = ends[1] - ends[0] + 1;
  DCHK(scratch_alloc(&dense, sizeof(double) * dn, st));
  DCHK(scratch_alloc(&flags, sizeof(int) * n, st));
  DCHK(scratch_alloc(&count, sizeof(int64_t), st));
  hipLaunchKernelGGL(k_fill_nan, dim3(grid_of(dn)), dim3(kBlock), 0, st, dense, dn);
  hipLaunchKernelGGL(k_scatter_values, dim3(grid_of(n)), dim3(kBlock), 0, st, pix, val, n, d0, dense);
  hipLaunchKernelGGL(k_detect, dim3(grid_of(n)), dim3(kBlock), 0, st, nside, pix, val, noise_sd, n, threshold,
                     (const double*)dense, d0, dn, flags);
  DCHK(hipGetLastError());
  size_t tb = 0;
  DCHK(hipcub::DeviceSelect::Flagged(nullptr, tb, pix, flags, peaks, count, (int)n, st));
  if (ensure_temp(ctx, tb)) {
    release();
    return SMART_ENOMEM;
  }
  tb = ctx->temp_bytes;
  DCHK(hipcub::DeviceSelect::Flagged(ctx->d_temp, tb, pix, flags, peaks, count, (int)n, st));
  DCHK(hipMemcpyAsync(n_peaks, count, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  release();
  DCHK(hipStreamSynchronize(st));
  return SMART_OK;
}

}  // namespace smart
