// Radial RSD propagation (Section 4.3 propagation sum, Listing 3 lookup, Algorithm 4
// inner loop) for gfx950.
//
//   C[pix][d] = sum_f w_f P^[pix][f] a(pix) lerp(K_r[., f, d], rho~(pix))
//             = sum_f (wa w_f P^) K_r[i0][f][d] + (wb w_f P^) K_r[i1][f][d]
//
// The pixels are pre-sorted by their lower radial bin i0 into chunks of up to 8 that
// share i0 (plan data), so one wave64 handles a chunk with one depth per lane: the two
// kernel rows K_r[i0][f][.], K_r[i1][f][.] are loaded once per frequency (512-byte
// rows across the lanes) and applied to all 8 pixels, whose tap-weighted phasors are
// staged in LDS and read as broadcasts.  Output rows C[pix][0..Nd) are written
// contiguously.  Every C element is produced by one lane in a fixed frequency order.
#include <hip/hip_fp16.h>

#include "nlos_internal.hpp"

namespace nlos {

constexpr int kChunkPix = 8;    // pixels per chunk (matches the plan's chunking)
constexpr int kFreqTile = 64;   // frequencies staged per LDS round
constexpr int kWaves = 4;       // waves (chunks) per block

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
  // per wave: tap-weighted phasors pa[j][f], pb[j][f] of one frequency tile
  __shared__ float2 sp[kWaves][2][kChunkPix][kFreqTile];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int Nf = a.Nf, Nd = a.Nd;
  const long long ngroups = (a.nchunks + kWaves - 1) / kWaves;
  for (long long g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const long long c = g * kWaves + wave;
    const bool cok = c < a.nchunks;
    const int i0 = cok ? a.chunk_i0[c] : -1;
    const int i1 = i0 + 1 < a.cut_idx ? i0 + 1 : a.cut_idx;
    int pix[kChunkPix];
    float wa[kChunkPix], wb[kChunkPix];
#pragma unroll
    for (int j = 0; j < kChunkPix; ++j) {
      pix[j] = cok ? a.chunk_pix[c * kChunkPix + j] : -1;
      wa[j] = cok ? a.chunk_wa[c * kChunkPix + j] : 0.f;
      wb[j] = cok ? a.chunk_wb[c * kChunkPix + j] : 0.f;
    }
    for (int d0 = 0; d0 < Nd; d0 += 64) {
      const int d = d0 + lane;
      const bool dok = d < Nd && i0 >= 0;
      float2 acc[kChunkPix];
#pragma unroll
      for (int j = 0; j < kChunkPix; ++j) acc[j] = make_float2(0.f, 0.f);
      for (int f0 = 0; f0 < Nf; f0 += kFreqTile) {
        // stage pa = wa w_f P^[pix][f], pb = wb w_f P^[pix][f] for this tile
        __syncthreads();
        const int f = f0 + lane;
        const bool fok = f < Nf && i0 >= 0;
        const float2 wf = fok ? a.w[f] : make_float2(0.f, 0.f);
#pragma unroll
        for (int j = 0; j < kChunkPix; ++j) {
          float2 ph = make_float2(0.f, 0.f);
          if (fok && pix[j] >= 0) ph = a.Ph[(long long)pix[j] * Nf + f];
          const float2 pw = make_float2(ph.x * wf.x - ph.y * wf.y, ph.x * wf.y + ph.y * wf.x);
          sp[wave][0][j][lane] = make_float2(pw.x * wa[j], pw.y * wa[j]);
          sp[wave][1][j][lane] = make_float2(pw.x * wb[j], pw.y * wb[j]);
        }
        __syncthreads();
        if (i0 >= 0) {
          const int nft = Nf - f0 < kFreqTile ? Nf - f0 : kFreqTile;
          const long long r0 = ((long long)i0 * Nf + f0) * Nd + d;
          const long long r1 = ((long long)i1 * Nf + f0) * Nd + d;
          for (int ff = 0; ff < nft; ++ff) {
            float2 k0 = make_float2(0.f, 0.f), k1 = make_float2(0.f, 0.f);
            if (dok) {
              k0 = load_kr<FP16>(a.Kr, r0 + (long long)ff * Nd);
              k1 = load_kr<FP16>(a.Kr, r1 + (long long)ff * Nd);
            }
#pragma unroll
            for (int j = 0; j < kChunkPix; ++j) {
              const float2 pa = sp[wave][0][j][ff];
              const float2 pb = sp[wave][1][j][ff];
              acc[j].x = fmaf(pa.x, k0.x, fmaf(-pa.y, k0.y, fmaf(pb.x, k1.x, fmaf(-pb.y, k1.y, acc[j].x))));
              acc[j].y = fmaf(pa.x, k0.y, fmaf(pa.y, k0.x, fmaf(pb.x, k1.y, fmaf(pb.y, k1.x, acc[j].y))));
            }
          }
        }
      }
      if (d < Nd) {
#pragma unroll
        for (int j = 0; j < kChunkPix; ++j)
          if (pix[j] >= 0) a.C[(long long)pix[j] * Nd + d] = acc[j];
      }
    }
  }
}

hipError_t launch_rsd_propagate(const RsdPropArgs& a, hipStream_t s) {
  const long long groups = (a.nchunks + kWaves - 1) / kWaves;
  const long long blocks = groups < 4096 ? groups : 4096;
  if (blocks <= 0) return hipSuccess;
  if (a.kernel_fp16)
    hipLaunchKernelGGL(rsd_propagate<true>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(rsd_propagate<false>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace nlos
