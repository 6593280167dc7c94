// Photon-event binning and small utility kernels (gfx950, wave64).
#include "nlos_internal.hpp"

namespace nlos {

__global__ __launch_bounds__(256) void fill_u32(uint32_t* __restrict__ p, size_t n, uint32_t v) {
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * 256;
  for (; i < n; i += stride) p[i] = v;
}

__global__ __launch_bounds__(256) void u32_to_f32(const uint32_t* __restrict__ in, float* __restrict__ out,
                                                  size_t n) {
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * 256;
  for (; i < n; i += stride) out[i] = (float)in[i];
}

hipError_t launch_u32_to_f32(const uint32_t* in, float* out, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(u32_to_f32, dim3((unsigned)blocks), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t value, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, value);
  return hipGetLastError();
}

// One event per lane, grid-stride over wave-sized chunks so that every lane of a
// wave takes the same trip count.  Lanes that target the same bin are merged for
// a few rounds (leader lane adds the popcount of its ballot); the remaining lanes
// add 1 each.  Integer atomics make the result exact and order independent.
__global__ __launch_bounds__(256) void bin_events(const uint2* __restrict__ ev, unsigned long long n,
                                                  uint32_t* __restrict__ hist,
                                                  unsigned long long* __restrict__ dropped, int npix,
                                                  int nt, uint32_t bin_ps, uint32_t t0) {
  const int lane = threadIdx.x & 63;
  const unsigned long long stride = (unsigned long long)gridDim.x * 256ull;
  unsigned int drop = 0;
  for (unsigned long long base = (unsigned long long)blockIdx.x * 256ull + (threadIdx.x & ~63u);
       base < n; base += stride) {
    const unsigned long long k = base + lane;
    long long key = -1;
    if (k < n) {
      const uint2 e = ev[k];
      const int pixel = (int)e.x;
      const uint32_t t = e.y;
      if (pixel >= 0 && pixel < npix && t >= t0) {
        const uint32_t b = (t - t0) / bin_ps;
        if (b < (uint32_t)nt) key = (long long)pixel * nt + b;
      }
      if (key < 0) ++drop;
    }
    bool pending = key >= 0;
#pragma unroll
    for (int round = 0; round < 4; ++round) {
      const unsigned long long m = __ballot(pending);
      if (m == 0ull) break;
      const int leader = __ffsll((long long)m) - 1;
      const long long lk = __shfl(key, leader);
      const bool same = pending && key == lk;
      const unsigned long long sm = __ballot(same);
      if (lane == leader) atomicAdd(hist + lk, (uint32_t)__popcll(sm));
      if (same) pending = false;
    }
    if (pending) atomicAdd(hist + key, 1u);
  }
  if (dropped != nullptr) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) drop += __shfl_xor(drop, off, 64);
    if (lane == 0 && drop != 0) atomicAdd(dropped, (unsigned long long)drop);
  }
}

hipError_t launch_bin(const void* events, unsigned long long n, uint32_t* hist,
                      unsigned long long* dropped, int npix, int nt, uint32_t bin_ps, uint32_t t0,
                      hipStream_t s) {
  if (n == 0) return hipSuccess;
  unsigned long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(bin_events, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<const uint2*>(events), n, hist, dropped, npix, nt, bin_ps, t0);
  return hipGetLastError();
}

// Phasors straight from photon records (Section 4.1, phasor binning; the paper's warp
// per photon becomes a wave64 per photon): a wave loads 64 events, then takes them one
// at a time, its lanes striding over the frequencies; lane f adds the unit phasor
// W_nt^(k_f b) of the event's bin b (from an LDS copy of the FP64-built table) to
// P[pixel][f] with hardware float atomics.  Float sums in arbitrary order: equal to the
// DFT of the histogram up to rounding.
__global__ __launch_bounds__(256) void phasor_bin(const uint2* __restrict__ ev, unsigned long long n,
                                                  float2* __restrict__ P, unsigned long long* __restrict__ dropped,
                                                  int npix, int nt, uint32_t bin_ps, uint32_t t0,
                                                  const float2* __restrict__ lut, const int* __restrict__ bins,
                                                  int nf) {
  __shared__ float2 slut[2048];
  for (int i = threadIdx.x; i < nt; i += 256) slut[i] = lut[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const unsigned long long stride = (unsigned long long)gridDim.x * 256ull;
  unsigned int drop = 0;
  for (unsigned long long base = (unsigned long long)blockIdx.x * 256ull + (threadIdx.x & ~63u);
       base < n; base += stride) {
    const unsigned long long k = base + lane;
    int pix = -1, b = 0;
    if (k < n) {
      const uint2 e = ev[k];
      const int pixel = (int)e.x;
      const uint32_t t = e.y;
      if (pixel >= 0 && pixel < npix && t >= t0) {
        const uint32_t bb = (t - t0) / bin_ps;
        if (bb < (uint32_t)nt) {
          pix = pixel;
          b = (int)bb;
        }
      }
      if (pix < 0) ++drop;
    }
    const unsigned long long valid = __ballot(pix >= 0);
    for (unsigned long long m = valid; m != 0ull; m &= m - 1ull) {
      const int j = __ffsll((long long)m) - 1;  // next valid event of the wave (uniform)
      const int pj = __shfl(pix, j), bj = __shfl(b, j);
      float2* row = P + (long long)pj * nf;
      for (int f = lane; f < nf; f += 64) {
        const float2 w = slut[(int)(((long long)bins[f] * bj) % nt)];
        unsafeAtomicAdd(&row[f].x, w.x);
        unsafeAtomicAdd(&row[f].y, w.y);
      }
    }
  }
  if (dropped != nullptr) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) drop += __shfl_xor(drop, off, 64);
    if (lane == 0 && drop != 0) atomicAdd(dropped, (unsigned long long)drop);
  }
}

hipError_t launch_phasor_bin(const void* events, unsigned long long n, float2* P, unsigned long long* dropped,
                             int npix, int nt, uint32_t bin_ps, uint32_t t0, const float2* lut, const int* bins,
                             int nf, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (nt < 1 || nt > 2048 || nf < 1) return hipErrorInvalidValue;
  unsigned long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(phasor_bin, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const uint2*>(events), n, P,
                     dropped, npix, nt, bin_ps, t0, lut, bins, nf);
  return hipGetLastError();
}

// Coherence-weighted merging (Section 4.4, Eq. 8-9) over the most recent `count` frames:
// S = sum f_j, A = sum |f_j| (oldest first), C = |S| / (eps + A), merged = C |S| / count.
// The new frame is stored into its ring slot in the same pass.
__global__ __launch_bounds__(256) void merge_frames(const float2* __restrict__ frame, float2* __restrict__ ring,
                                                    long long n, int window, int slot, int first, int count,
                                                    float eps, float* __restrict__ merged,
                                                    float* __restrict__ coherence) {
  for (long long v = (long long)blockIdx.x * 256 + threadIdx.x; v < n; v += (long long)gridDim.x * 256) {
    const float2 f = frame[v];
    ring[(long long)slot * n + v] = f;
    float2 S = make_float2(0.f, 0.f);
    float A = 0.f;
    for (int k = 0; k < count; ++k) {
      int r = first + k;
      if (r >= window) r -= window;
      const float2 g = (r == slot) ? f : ring[(long long)r * n + v];
      S.x += g.x;
      S.y += g.y;
      A += sqrtf(g.x * g.x + g.y * g.y);
    }
    const float s = sqrtf(S.x * S.x + S.y * S.y);
    const float C = s / (eps + A);
    merged[v] = C * s / (float)count;
    if (coherence) coherence[v] = C;
  }
}

hipError_t launch_merge(const float2* frame, float2* ring, long long n, int window, int slot, int first,
                        int count, float eps, float* merged, float* coherence, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (window < 1 || slot < 0 || slot >= window || first < 0 || first >= window || count < 1 || count > window)
    return hipErrorInvalidValue;
  long long blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(merge_frames, dim3((unsigned)blocks), dim3(256), 0, s, frame, ring, n, window, slot, first,
                     count, eps, merged, coherence);
  return hipGetLastError();
}

}  // namespace nlos
