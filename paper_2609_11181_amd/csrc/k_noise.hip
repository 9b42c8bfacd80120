// Shape-noise realisations of a pixel map (pixel variant).
//
// A realisation rotates each pixel's shear sum by a random spin-2 phase,
// G -> G exp(2 i pi u), u in [0, 1) supplied by the caller; the weights and
// the E2 sums are unchanged, so W, V and N of every aperture are too. This
// is the randomised-orientation noise map of the paper (Sect. 1; Sect. 5.3
// notes that the convergence route needs N such maps).
#include <hip/hip_runtime.h>

#include "smart_internal.h"

namespace smart {

namespace {

__global__ void k_rotate(const float4* map, const float* u, int64_t n, float4* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 g = map[i];
  float s, c;
  sincospif(2.0f * u[i], &s, &c);
  out[i] = make_float4(g.x * c - g.y * s, g.x * s + g.y * c, g.z, g.w);
}

}  // namespace

hipError_t launch_rotate_map(const float4* map, const float* u, int64_t n, float4* out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rotate, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, map, u, n, out);
  return hipGetLastError();
}

int noise_bf16x3(smart_plan plan, const float* d_u, int n_real, int norm, float* d_out, hipStream_t st) {
  (void)plan; (void)d_u; (void)n_real; (void)norm; (void)d_out; (void)st;
  set_error("split-BF16 noise batches are not available in this build");
  return SMART_EUNSUPPORTED;
}

}  // namespace smart
