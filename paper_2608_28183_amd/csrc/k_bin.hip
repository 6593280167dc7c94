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

// out[c][r] = in[r][c]: 32 x 32 tiles through LDS, both sides coalesced
__global__ __launch_bounds__(256) void transpose_f32(const float* __restrict__ in, float* __restrict__ out,
                                                     long long rows, int cols) {
  __shared__ float t[32][33];
  const long long r0 = (long long)blockIdx.y * 32;
  const int c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const long long r = r0 + k;
    const int c = c0 + tx;
    if (r < rows && c < cols) t[k][tx] = in[r * cols + c];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k;
    const long long r = r0 + tx;
    if (r < rows && c < cols) out[(long long)c * rows + r] = t[tx][k];
  }
}

hipError_t launch_transpose_f32(const float* in, float* out, long long rows, int cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const long long by = (rows + 31) / 32;
  if (by > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(transpose_f32, dim3((unsigned)((cols + 31) / 32), (unsigned)by), dim3(256), 0, s, in, out,
                     rows, cols);
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

// ---------------------------------------------------------------------------
// binning by pixel tiles
// ---------------------------------------------------------------------------
//
// The histogram (8 MiB at 64 x 64 x 512) is far larger than LDS, and device-scope atomics
// each reach the memory side, so the counters are privatised per tile of tp pixels (tp nt
// counters, at most 16 KB of LDS), in two passes with no global atomics:
// (1) each block takes a chunk of kBinChunk events and sorts it by tile in LDS (per-tile
//     counts, their scan, placement), then writes it back as runs of 16-bit codes
//     (pixel in tile) nt + bin, one run per tile, with the start of every run in a table
//     start[tile][chunk] (start[ntiles][chunk]: the chunk's valid events);
// (2) one block per tile gathers its runs from every chunk, histograms them in LDS and
//     writes the tile's rows with plain stores (all of them, so no clearing pass).
// Events are read once; all adds are integer adds, so the histogram is exact and does not
// depend on the order in which the LDS atomics land.

constexpr int kBinThreads = 256;
constexpr int kBinPerThread = 32;
constexpr int kBinChunk = kBinThreads * kBinPerThread;  // events per block in pass 1
// tp nt <= kBinTileWords (codes fit 16 bits).  At 64 x 64 x 512 with 1e7 events, tiles of
// 4096 words (512 tiles) measured 0.066 ms, of 8192 words 0.074 ms (the gather's time is
// its busiest tile's: fewer, larger tiles balance worse) and of 2048 words 0.080 ms.
constexpr int kBinTileWords = 4096;
constexpr int kBinMaxTiles = 8192;
constexpr int kBinGatherThreads = 1024;
constexpr int kBinGroup = 2048;  // chunks whose runs pass 2 gathers per round
constexpr int kBinBatch = 8;     // loads in flight per lane

// Quotient of a u32 by a divisor fixed for the launch: a multiply-high and two shifts with
// constants computed on the host (Granlund and Montgomery's division by invariant integers,
// the round-down form with the add fix-up), exact for every 32-bit dividend.
struct U32Div {
  uint32_t m;
  int s1, s2;
};
U32Div u32_div(uint32_t d) {
  int l = 0;
  while (l < 32 && (1ull << l) < d) ++l;
  U32Div r;
  r.m = (uint32_t)((((unsigned __int128)1 << 32) * ((1ull << l) - d)) / d + 1);
  r.s1 = l < 1 ? l : 1;
  r.s2 = l > 1 ? l - 1 : 0;
  return r;
}
__device__ __forceinline__ uint32_t u32_quot(uint32_t n, U32Div d) {
  const uint32_t t = __umulhi(n, d.m);
  return (t + ((n - t) >> d.s1)) >> d.s2;
}

// pixel of a valid event (-1 otherwise) and its bin
__device__ __forceinline__ int bin_event(uint2 e, int npix, int nt, U32Div bin_ps, uint32_t t0, int* b) {
  const int pixel = (int)e.x;
  if (pixel < 0 || pixel >= npix || e.y < t0) return -1;
  const uint32_t bb = u32_quot(e.y - t0, bin_ps);
  if (bb >= (uint32_t)nt) return -1;
  *b = (int)bb;
  return pixel;
}

// LDS atomic add of 1 per lane to cnt[key] (key < 0: none); returns the counter's value
// before this lane's add.  When every active lane of the wave has the same key (sorted
// events, a hot bin) one atomic adds them all; otherwise each lane adds its own (random
// keys rarely coincide within a wave, and the LDS resolves the few conflicts).  Every lane
// of the wave must call it.
__device__ __forceinline__ uint32_t lds_count(uint32_t* cnt, int key) {
  const int lane = threadIdx.x & 63;
  const unsigned long long act = __ballot(key >= 0);
  if (act == 0ull) return 0;
  const int leader = __ffsll((long long)act) - 1;
  const int lk = __shfl(key, leader);
  if (__ballot(key >= 0 && key == lk) == act) {
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(cnt + lk, (uint32_t)__popcll(act));
    base = __shfl(base, leader);
    return base + (uint32_t)__popcll(act & ((1ull << lane) - 1ull));
  }
  return key >= 0 ? atomicAdd(cnt + key, 1u) : 0u;
}

// In-place exclusive scan of a[0..m) in LDS by a block of NT threads, each taking a
// contiguous run; wsum holds NT / 64 words.  The caller synchronises before and after.
template <int NT>
__device__ __forceinline__ void block_exclusive_scan(uint32_t* a, int m, uint32_t* wsum) {
  const int per = (m + NT - 1) / NT;
  const int lo = threadIdx.x * per;
  const int hi = lo + per < m ? lo + per : m;
  uint32_t s = 0;
  for (int i = lo; i < hi; ++i) s += a[i];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = s;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint32_t run = x - s;
  for (int k = 0; k < w; ++k) run += wsum[k];
  for (int i = lo; i < hi; ++i) {
    const uint32_t v = a[i];
    a[i] = run;
    run += v;
  }
}

// Pass 1: chunk blockIdx.x -> runs[chunk][kBinChunk] (16-bit codes, sorted by tile) and
// start[tile][chunk]; invalid events are counted into *dropped.
__global__ __launch_bounds__(kBinThreads) void bin_chunk_sort(const uint2* __restrict__ ev, unsigned long long n,
                                                             int npix, int nt, U32Div bin_ps, uint32_t t0, int tp,
                                                             U32Div tp_div,
                                                             int ntiles, int nchunks, uint16_t* __restrict__ runs,
                                                             uint16_t* __restrict__ start,
                                                             unsigned long long* __restrict__ dropped) {
  extern __shared__ uint32_t sh[];
  uint32_t* cnt = sh;  // ntiles + 1 counters, then their exclusive scan
  uint16_t* sorted = reinterpret_cast<uint16_t*>(sh + ntiles + 1);  // kBinChunk codes
  __shared__ uint32_t wsum[kBinThreads / 64];
  for (int i = threadIdx.x; i <= ntiles; i += kBinThreads) cnt[i] = 0;
  __syncthreads();
  const unsigned long long beg = (unsigned long long)blockIdx.x * kBinChunk;
  uint32_t code[kBinPerThread];  // tile << 16 | (pixel in tile) nt + bin; ~0u: none
  uint32_t pos[kBinPerThread];   // place in the tile's run
  unsigned int drop = 0;
  constexpr int kLoads = 16;  // loads in flight per lane
#pragma unroll
  for (int r = 0; r < kBinPerThread; r += kLoads) {
    uint2 e[kLoads];
#pragma unroll
    for (int j = 0; j < kLoads; ++j) {
      const unsigned long long k = beg + (unsigned long long)(r + j) * kBinThreads + threadIdx.x;
      e[j] = k < n ? ev[k] : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int j = 0; j < kLoads; ++j) {
      const unsigned long long k = beg + (unsigned long long)(r + j) * kBinThreads + threadIdx.x;
      uint32_t c = ~0u;
      if (k < n) {
        int b = 0;
        const int px = bin_event(e[j], npix, nt, bin_ps, t0, &b);
        if (px >= 0) {
          const int tile = (int)u32_quot((uint32_t)px, tp_div);
          c = ((uint32_t)tile << 16) | (uint32_t)((px - tile * tp) * nt + b);
        } else {
          ++drop;
        }
      }
      code[r + j] = c;
      pos[r + j] = lds_count(cnt, c == ~0u ? -1 : (int)(c >> 16));
    }
  }
  __syncthreads();
  block_exclusive_scan<kBinThreads>(cnt, ntiles + 1, wsum);
  __syncthreads();
  for (int i = threadIdx.x; i <= ntiles; i += kBinThreads)
    start[(size_t)i * nchunks + blockIdx.x] = (uint16_t)cnt[i];
#pragma unroll
  for (int j = 0; j < kBinPerThread; ++j)
    if (code[j] != ~0u) sorted[cnt[code[j] >> 16] + pos[j]] = (uint16_t)(code[j] & 0xffffu);
  __syncthreads();
  const uint32_t nv = cnt[ntiles];
  uint16_t* out = runs + (size_t)blockIdx.x * kBinChunk;
  for (uint32_t i = threadIdx.x; i < nv; i += kBinThreads) out[i] = sorted[i];
  if (dropped != nullptr) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) drop += __shfl_xor(drop, off, 64);
    if ((threadIdx.x & 63) == 0 && drop != 0) atomicAdd(dropped, (unsigned long long)drop);
  }
}

// Pass 2: one block per tile.  Its runs from kBinGroup chunks at a time are laid end to
// end (exclusive scan of their lengths); lane i of the flat range finds its chunk by
// binary search and counts its code in the tile's LDS histogram.
__global__ __launch_bounds__(kBinGatherThreads) void bin_tile_gather(const uint16_t* __restrict__ runs,
                                                                    const uint16_t* __restrict__ start,
                                                                    int nchunks, int npix, int nt, int tp,
                                                                    uint32_t* __restrict__ hist, int accumulate) {
  extern __shared__ uint32_t h[];  // tp nt counters
  __shared__ uint32_t rbeg[kBinGroup];
  __shared__ uint32_t rpre[kBinGroup + 1];
  __shared__ uint32_t wsum[kBinGatherThreads / 64];
  const int t = blockIdx.x;
  const int words = tp * nt;
  for (int i = threadIdx.x; i < words; i += kBinGatherThreads) h[i] = 0;
  for (int c0 = 0; c0 < nchunks; c0 += kBinGroup) {
    const int g = nchunks - c0 < kBinGroup ? nchunks - c0 : kBinGroup;
    __syncthreads();  // h cleared, the previous round's readers of rbeg / rpre done
    for (int k = threadIdx.x; k < g; k += kBinGatherThreads) {
      const uint32_t b = start[(size_t)t * nchunks + c0 + k];
      rbeg[k] = b;
      rpre[k] = (uint32_t)start[(size_t)(t + 1) * nchunks + c0 + k] - b;
    }
    if (threadIdx.x == 0) rpre[g] = 0;
    __syncthreads();
    block_exclusive_scan<kBinGatherThreads>(rpre, g + 1, wsum);
    __syncthreads();
    const uint32_t total = rpre[g];
    int top = 1;  // largest power of two below g (g >= 1)
    while (2 * top < g) top <<= 1;
    // a batch covers kBinGatherThreads kBinBatch flat elements; wave w takes the 64 kBinBatch
    // of them from ew on, lane l element ew + 64 j + l at step j
    const int lane = threadIdx.x & 63;
    for (uint32_t b0 = 0; b0 < total; b0 += kBinGatherThreads * kBinBatch) {
      const uint32_t ew = b0 + (uint32_t)(threadIdx.x >> 6) * (64 * kBinBatch);
      // the chunk whose run holds element ew (the last k with rpre[k] <= ew): one search
      // per wave, on wave-uniform values
      int k = 0;
      for (int step = top; step > 0; step >>= 1) {
        const int m = k + step;
        if (m < g && (uint32_t)__builtin_amdgcn_readfirstlane((int)rpre[m]) <= ew) k = m;
      }
      uint32_t v[kBinBatch];
#pragma unroll
      for (int j = 0; j < kBinBatch; ++j) {
        const uint32_t i = ew + (uint32_t)(64 * j + lane);
        v[j] = 0xffffu;
        if (i < total) {
          // elements only grow with j: walk on to the run that holds i (rpre[g] = total > i
          // stops the walk at k = g - 1 at the latest)
          while (rpre[k + 1] <= i) ++k;
          v[j] = runs[(size_t)(c0 + k) * kBinChunk + rbeg[k] + (i - rpre[k])];
        }
      }
#pragma unroll
      for (int j = 0; j < kBinBatch; ++j) lds_count(h, v[j] == 0xffffu ? -1 : (int)v[j]);
    }
  }
  __syncthreads();
  const long long first = (long long)t * tp * nt;
  const long long last = (long long)npix * nt;
  for (int i = threadIdx.x; i < words && first + i < last; i += kBinGatherThreads) {
    uint32_t* g = hist + first + i;
    *g = accumulate ? *g + h[i] : h[i];
  }
}

// Tile layout of a binning job: tp pixels per tile (tp nt <= kBinTileWords), or false when
// the tiled path does not apply (then the per-event atomic kernel runs).
bool bin_tiles(int npix, int nt, unsigned long long n, int* tp, int* ntiles) {
  if (nt > kBinTileWords || n >= (1ull << 31)) return false;
  *tp = kBinTileWords / nt;
  if (*tp > npix) *tp = npix;
  *ntiles = (npix + *tp - 1) / *tp;
  return *ntiles <= kBinMaxTiles;
}

size_t bin_workspace_bytes(int npix, int nt, unsigned long long n) {
  int tp = 0, nti = 0;
  if (!bin_tiles(npix, nt, n, &tp, &nti)) return 0;
  const size_t nchunks = (size_t)((n + kBinChunk - 1) / kBinChunk);
  const size_t bytes = 2 * nchunks * kBinChunk + 2 * (size_t)(nti + 1) * nchunks;
  return bytes > 0 ? bytes : 256;  // never zero: zero means "not tiled"
}

hipError_t launch_bin_tiled(const void* events, unsigned long long n, uint32_t* hist, unsigned long long* dropped,
                            int npix, int nt, uint32_t bin_ps, uint32_t t0, int accumulate, void* ws, hipStream_t s) {
  int tp = 0, nti = 0;
  if (!bin_tiles(npix, nt, n, &tp, &nti)) return hipErrorInvalidValue;
  const int nchunks = (int)((n + kBinChunk - 1) / kBinChunk);
  uint16_t* runs = static_cast<uint16_t*>(ws);                // [chunk][kBinChunk]
  uint16_t* start = runs + (size_t)nchunks * kBinChunk;        // [tile][chunk], ntiles + 1 rows
  hipError_t e;
  if (nchunks > 0) {
    hipLaunchKernelGGL(bin_chunk_sort, dim3((unsigned)nchunks), dim3(kBinThreads),
                       (size_t)4 * (nti + 1) + (size_t)2 * kBinChunk, s, static_cast<const uint2*>(events), n, npix,
                       nt, u32_div(bin_ps), t0, tp, u32_div((uint32_t)tp), nti, nchunks, runs, start, dropped);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(bin_tile_gather, dim3((unsigned)nti), dim3(kBinGatherThreads), (size_t)4 * tp * nt, s, runs,
                     start, nchunks, npix, nt, tp, hist, accumulate);
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
