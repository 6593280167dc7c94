// Radial RSD propagation (Section 4.3 propagation sum, Listing 3 lookup, Algorithm 4
// inner loop) for gfx950.
//
//   C[pix][d] = sum_f w_f P^[pix][f] a(pix) lerp(K_r[., f, d], rho~(pix))
//             = sum_f (wa w_f P^) K_r[i0][f][d] + (wb w_f P^) K_r[i0+1][f][d]
//
// The plan sorts the pixels by their lower radial bin i0 and groups them into chunks of
// up to 64 that share i0.  One wave64 takes a chunk, one pixel per lane, and a slice of
// kDepths depths: the two kernel rows K_r[i0][f][d0..d0+kDepths) and K_r[i0+1][f][...]
// are the same for the whole wave, so they come in through the scalar unit and enter the
// FMAs as scalar operands, and each kernel value is loaded once per 64 pixels.  The
// lane's own phasor P^[pix][f] is read from its contiguous frequency row.  Every C
// element is produced by one lane in a fixed frequency order.
#include <hip/hip_fp16.h>

#include "nlos_internal.hpp"

namespace nlos {

constexpr int kGroupPix = 64;   // pixels per chunk (one per lane; matches the plan)
constexpr int kDepths = 8;      // depths per wave
constexpr int kWavesPerBlock = 4;

template <bool FP16>
__device__ __forceinline__ float2 load_kr(const void* __restrict__ kr, long long i) {
  if constexpr (FP16) {
    const __half2 h = static_cast<const __half2*>(kr)[i];
    return __half22float2(h);
  } else {
    return static_cast<const float2*>(kr)[i];
  }
}

// acc += pa K0 + pb K1 (complex), fixed operation order
__device__ __forceinline__ void cmac2(float2& acc, float2 pa, float2 k0, float2 pb, float2 k1) {
  acc.x = fmaf(pa.x, k0.x, fmaf(-pa.y, k0.y, fmaf(pb.x, k1.x, fmaf(-pb.y, k1.y, acc.x))));
  acc.y = fmaf(pa.x, k0.y, fmaf(pa.y, k0.x, fmaf(pb.x, k1.y, fmaf(pb.y, k1.x, acc.y))));
}

// One frequency f of the lane's pixel: tap-weighted phasors, then the ND depths of the
// wave's slice (kernel rows o0, o1 are wave-uniform).
template <bool FP16, int ND>
__device__ __forceinline__ void rsd_freq(float2* acc, float2 p, float2 wf, float wa, float wb, const void* kr,
                                         long long o0, long long o1) {
  const float2 pw = make_float2(p.x * wf.x - p.y * wf.y, p.x * wf.y + p.y * wf.x);
  const float2 pa = make_float2(pw.x * wa, pw.y * wa);
  const float2 pb = make_float2(pw.x * wb, pw.y * wb);
#pragma unroll
  for (int j = 0; j < ND; ++j) cmac2(acc[j], pa, load_kr<FP16>(kr, o0 + j), pb, load_kr<FP16>(kr, o1 + j));
}

template <bool FP16>
__global__ __launch_bounds__(256) void rsd_propagate(RsdPropArgs a) {
  const int lane = threadIdx.x & 63;
  // wave-uniform work index: chunk g, depth slice starting at d0
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nds = (a.Nd + kDepths - 1) / kDepths;
  const long long w = (long long)blockIdx.x * kWavesPerBlock + wib;
  if (w >= a.nchunks * nds) return;
  const long long g = w / nds;
  const int d0 = (int)(w % nds) * kDepths;
  const int Nf = a.Nf, Nd = a.Nd;
  const int i0 = a.chunk_i0[g];
  const int pix = a.chunk_pix[g * kGroupPix + lane];
  float2 acc[kDepths];
#pragma unroll
  for (int j = 0; j < kDepths; ++j) acc[j] = make_float2(0.f, 0.f);
  if (i0 >= 0) {
    const int i1 = i0 + 1 < a.cut_idx ? i0 + 1 : a.cut_idx;
    // unused slots have wa = wb = 0 and read pixel 0's row
    const float wa = a.chunk_wa[g * kGroupPix + lane];
    const float wb = a.chunk_wb[g * kGroupPix + lane];
    const float2* __restrict__ ph = a.Ph + (long long)(pix >= 0 ? pix : 0) * a.ph_stride;
    long long o0 = (long long)i0 * Nf * Nd + d0;
    long long o1 = (long long)i1 * Nf * Nd + d0;
    if (d0 + kDepths <= Nd) {
      int f = 0;
      // eight phasor loads in flight per lane
      for (; f + 8 <= Nf; f += 8) {
        float2 p[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) p[u] = ph[f + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          rsd_freq<FP16, kDepths>(acc, p[u], a.w[f + u], wa, wb, a.Kr, o0, o1);
          o0 += Nd;
          o1 += Nd;
        }
      }
      for (; f < Nf; ++f) {
        rsd_freq<FP16, kDepths>(acc, ph[f], a.w[f], wa, wb, a.Kr, o0, o1);
        o0 += Nd;
        o1 += Nd;
      }
    } else {
      // last, partial depth slice
      const int nd = Nd - d0;
      for (int f = 0; f < Nf; ++f) {
        const float2 p = ph[f], wf = a.w[f];
        const float2 pw = make_float2(p.x * wf.x - p.y * wf.y, p.x * wf.y + p.y * wf.x);
        const float2 pa = make_float2(pw.x * wa, pw.y * wa);
        const float2 pb = make_float2(pw.x * wb, pw.y * wb);
#pragma unroll
        for (int j = 0; j < kDepths; ++j)
          if (j < nd) cmac2(acc[j], pa, load_kr<FP16>(a.Kr, o0 + j), pb, load_kr<FP16>(a.Kr, o1 + j));
        o0 += Nd;
        o1 += Nd;
      }
    }
  }
  if (pix < 0) return;
  float2* out = a.C + (long long)pix * a.c_stride + d0;
#pragma unroll
  for (int j = 0; j < kDepths; ++j)
    if (d0 + j < Nd) out[j] = acc[j];
}

hipError_t launch_rsd_propagate(const RsdPropArgs& a, hipStream_t s) {
  const long long nds = (a.Nd + kDepths - 1) / kDepths;
  const long long waves = a.nchunks * nds;
  const long long blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  if (a.kernel_fp16)
    hipLaunchKernelGGL(rsd_propagate<true>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(rsd_propagate<false>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace nlos
