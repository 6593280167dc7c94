// Depth-dependent average over a ring of the last volumes (Section 4.4, DDA), gfx950 wave64.
#include "nlos_internal.hpp"

namespace nlos {

// Lane groups of G lanes (G a power of two <= 64) take one voxel each, its depths d = g,
// g + G, ... on the group's lanes, so a wave covers 64 / G voxels and every access of a
// group is contiguous.  The new frame goes into its ring slot in the same pass; older
// frames whose weight at that depth is 0 are not read.  avg = sum_a w[d][a] v_{i-a} /
// sum_a w[d][a] over the count newest frames (a = 0: the new one), img = max over depth.
__global__ __launch_bounds__(256) void dda_push(const float* __restrict__ vol, float* __restrict__ ring,
                                                const float* __restrict__ w, long long nvox, int nd, int window,
                                                int slot, int count, int G, float* __restrict__ avg,
                                                float* __restrict__ img) {
  const int lane = threadIdx.x & 63;
  const int vpw = 64 / G;  // voxels per wave
  const int sub = lane / G, g = lane % G;
  const long long plane = nvox * nd;
  const long long wave = ((long long)blockIdx.x * 256 + threadIdx.x) >> 6;
  const long long nwaves = (long long)gridDim.x * 4;
  for (long long vb = wave * vpw; vb < nvox; vb += nwaves * vpw) {
    const long long v = vb + sub;
    float mx = -INFINITY;
    if (v < nvox) {
      for (int d = g; d < nd; d += G) {
        const long long off = v * nd + d;
        const float x = vol[off];
        ring[(long long)slot * plane + off] = x;
        const float* wd = w + (long long)d * window;
        float num = wd[0] * x, den = wd[0];
        for (int k = 1; k < count; ++k) {
          const float wk = wd[k];
          if (wk != 0.f) {
            int r = slot - k;
            if (r < 0) r += window;
            num += wk * ring[(long long)r * plane + off];
            den += wk;
          }
        }
        const float a = num / den;
        if (avg) avg[off] = a;
        mx = fmaxf(mx, a);
      }
    }
    if (img) {
      for (int o = G >> 1; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
      if (g == 0 && v < nvox) img[v] = mx;
    }
  }
}

hipError_t launch_dda(const float* vol, float* ring, const float* w, long long nvox, int nd, int window, int slot,
                      int count, float* avg, float* img, hipStream_t s) {
  if (nvox <= 0) return hipSuccess;
  if (nd < 1 || window < 1 || slot < 0 || slot >= window || count < 1 || count > window)
    return hipErrorInvalidValue;
  int G = 1;
  while (G < nd && G < 64) G <<= 1;
  const long long vpb = 4LL * (64 / G);  // voxels per block and trip
  long long blocks = (nvox + vpb - 1) / vpb;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(dda_push, dim3((unsigned)blocks), dim3(256), 0, s, vol, ring, w, nvox, nd, window, slot, count,
                     G, avg, img);
  return hipGetLastError();
}

}  // namespace nlos
