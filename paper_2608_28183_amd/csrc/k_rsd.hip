// Radial RSD propagation (Section 4.3 propagation sum, Listing 3 lookup,
// Algorithm 4 inner loop) for gfx950.
//
// One wave64 per Fourier pixel with one depth plane per lane: the radius,
// taper, interpolation indices, phasor and weight are wave-uniform (scalar
// registers) and each lane streams its depth's two radial-kernel samples per
// frequency, which are contiguous across lanes.  A block owns 64 consecutive
// pixels; results are staged through LDS so that the [d][pixel] output is
// written in 512-byte rows.
#include <hip/hip_fp16.h>

#include "nlos_internal.hpp"

namespace nlos {

template <bool FP16>
__device__ __forceinline__ float2 load_kr(const void* kr, long long i) {
  if constexpr (FP16) {
    const __half2 h = static_cast<const __half2*>(kr)[i];
    return __half22float2(h);
  } else {
    return static_cast<const float2*>(kr)[i];
  }
}

template <bool FP16>
__global__ __launch_bounds__(256) void rsd_propagate(RsdPropArgs a) {
  __shared__ float2 tile[64][65];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long long pix0 = (long long)blockIdx.x * 64;
  const long long npix = a.npix;
  const int Nf = a.Nf, Nd = a.Nd;
  for (int d0 = 0; d0 < Nd; d0 += 64) {
    const int d = d0 + lane;
    const bool dok = d < Nd;
    for (int k = 0; k < 16; ++k) {
      const int pl = wave * 16 + k;
      const long long pix = pix0 + pl;
      float2 acc = make_float2(0.f, 0.f);
      if (pix < npix) {
        const float rt = a.rho[pix];
        const float rc = a.rho_cut_bin;
        float aw;
        if (rt <= rc - 8.f) {
          aw = 1.f;
        } else if (rt < rc) {
          const float t = (rc - rt) * 0.125f;
          aw = t * t * (3.f - 2.f * t);
        } else {
          aw = 0.f;
        }
        if (aw > 0.f) {
          int i0 = (int)floorf(rt);
          i0 = i0 < 0 ? 0 : (i0 > a.last_base ? a.last_base : i0);
          const int i1 = i0 + 1 < a.cut_idx ? i0 + 1 : a.cut_idx;
          const float al = rt - (float)i0;
          const long long row0 = (long long)i0 * Nf * Nd + d;
          const long long row1 = (long long)i1 * Nf * Nd + d;
          for (int f = 0; f < Nf; ++f) {
            const float2 ph = a.Ph[(long long)f * npix + pix];
            const float2 wf = a.w[f];
            float2 pw;
            pw.x = (ph.x * wf.x - ph.y * wf.y) * aw;
            pw.y = (ph.x * wf.y + ph.y * wf.x) * aw;
            float2 k0 = make_float2(0.f, 0.f), k1 = make_float2(0.f, 0.f);
            if (dok) {
              k0 = load_kr<FP16>(a.Kr, row0 + (long long)f * Nd);
              k1 = load_kr<FP16>(a.Kr, row1 + (long long)f * Nd);
            }
            const float hx = fmaf(al, k1.x - k0.x, k0.x);
            const float hy = fmaf(al, k1.y - k0.y, k0.y);
            acc.x = fmaf(pw.x, hx, fmaf(-pw.y, hy, acc.x));
            acc.y = fmaf(pw.x, hy, fmaf(pw.y, hx, acc.y));
          }
        }
      }
      tile[lane][pl] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 64 * 64; i += 256) {
      const int dd = i >> 6, pp = i & 63;
      if (d0 + dd < Nd && pix0 + pp < npix) a.C[(long long)(d0 + dd) * npix + pix0 + pp] = tile[dd][pp];
    }
    __syncthreads();
  }
}

hipError_t launch_rsd_propagate(const RsdPropArgs& a, hipStream_t s) {
  dim3 grid((unsigned)((a.npix + 63) / 64));
  if (a.kernel_fp16)
    hipLaunchKernelGGL(rsd_propagate<true>, grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(rsd_propagate<false>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace nlos
