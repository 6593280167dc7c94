// General-length line passes (FP32): the strided and contiguous FFT passes and the f-k
// real x-FFT for lengths that are not powers of two.  The line transform itself is
// gen_fft (LDS-resident mixed-radix Stockham stages); the load and store modes follow
// the power-of-two passes of k_fft.hip and k_fk.hip one for one, so the host schedules
// and the workspace layouts are the same for every length.
#include "fft_general.hpp"
#include "nlos_internal.hpp"

namespace nlos {

namespace {

// At most kGenE samples per thread: a stage holds all butterflies of a thread in
// registers across the block barrier, at most kGenE + 15 values for radices up to 16.
constexpr int kGenE = 8;
constexpr int kGenMaxThreads = 1024;

// threads per line: ceil(n / kGenE)
int gen_line_threads(int n) { return (n + kGenE - 1) / kGenE; }

// columns per block of a strided pass: up to a 16-column (128-byte) row segment, within
// 64 KiB of LDS (the tile and the twiddle table) and 1024 threads
int gen_cols(int n) {
  int t = 16;
  while (t > 1 && ((long long)n * (t + 1) * (long long)sizeof(float2) > 65536 || t * gen_line_threads(n) > kGenMaxThreads))
    t >>= 1;
  return t;
}

int ilog2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

}  // namespace

// ---------------------------------------------------------------------------
// strided lines: tile of T adjacent columns, LDS [n][T]
// ---------------------------------------------------------------------------

// Tile of a block, XCD-aware: blocks b and b + 8 run on one XCD (blocks go round-robin
// over the 8 XCDs), so within each 16 blocks they take the tiles 2k and 2k + 1, whose
// 64-byte row segments share 128-byte lines, and the second finds the lines in that L2.
__device__ __forceinline__ int gen_tile() {
  const int b = blockIdx.x;
  return (gridDim.x % 16 == 0) ? ((b & ~15) | ((b & 7) << 1) | ((b >> 3) & 1)) : b;
}


template <int EMAX, bool INV, int ST>
__global__ __launch_bounds__(kGenMaxThreads) void gen_strided(StridedArgs a, GenPlan g, int lt) {
  extern __shared__ float2 glds[];
  const int n = g.n, T = 1 << lt, P = blockDim.x >> lt;
  const int tid = threadIdx.x;
  const int c = tid & (T - 1), p = tid >> lt;
  const long long plane = blockIdx.y;
  const int col = gen_tile() * T + c;
  const bool colok = col < a.ncols;
  const float2* in = static_cast<const float2*>(a.in) + plane * a.in_plane + (colok ? col : 0);
  // samples i = p + k P (k < EMAX cover the line): all loads in flight before any LDS write
  float2 x[EMAX];
  static_for<EMAX>([&](auto k_) {
    constexpr int k = decltype(k_)::value;
    const int i = p + k * P;
    x[k] = (colok && i < a.n_in) ? in[(long long)i * a.in_line] : make_float2(0.f, 0.f);
  });
  static_for<EMAX>([&](auto k_) {
    constexpr int k = decltype(k_)::value;
    const int i = p + k * P;
    if (i < n) glds[i * T + c] = x[k];
  });
  float2* twl = glds + n * T;
  gen_load_twiddles(twl, g);
  __syncthreads();
  gen_fft<EMAX, INV>(glds + c, T, g, twl, p, P);
  static_for<EMAX>([&](auto k_) {
    const int i = p + decltype(k_)::value * P;
    if (i >= a.n_out) return;
    const float2 v = glds[i * T + c];
    if constexpr (ST == ST_C64 || ST == ST_C64_SCALED) {
      if (colok)
        static_cast<float2*>(a.out)[plane * a.out_plane + (long long)i * a.out_line + col] =
            ST == ST_C64_SCALED ? cscale(v, a.oscale) : v;
    } else {  // ST_ABS_IMG: |v| * oscale, and the max over the tile's columns into img
      float m = colok ? sqrtf(v.x * v.x + v.y * v.y) * a.oscale : 0.f;
      if (a.out != nullptr && colok)
        static_cast<float*>(a.out)[plane * a.out_plane + (long long)i * a.out_line + col] = m;
      if (a.img != nullptr) {
        // the T lanes of one row are adjacent in the wave and take the same branches
        for (int off = 1; off < T; off <<= 1) m = fmaxf(m, __shfl_xor(m, off, T));
        if (c == 0)
          atomicMax(reinterpret_cast<unsigned int*>(a.img) + plane * a.img_plane + i, __float_as_uint(m));
      }
    }
  });
}

// ---------------------------------------------------------------------------
// contiguous lines: L lines per block, P threads per line (a power of two), LDS [L][n]
// ---------------------------------------------------------------------------

template <int EMAX, bool INV, int LD, int ST>
__global__ __launch_bounds__(kGenMaxThreads) void gen_contig(ContigArgs a, GenPlan g, int lp) {
  extern __shared__ float2 glds[];
  const int n = g.n, P = 1 << lp, L = blockDim.x >> lp;
  const int tid = threadIdx.x;
  const int l = tid >> lp, p = tid & (P - 1);
  const long long line = (long long)blockIdx.x * L + l;
  const bool lineok = line < a.nlines;
  float2* my = glds + l * n;
  float2 x[EMAX];
  static_for<EMAX>([&](auto k_) {
    constexpr int k = decltype(k_)::value;
    const int i = p + k * P;
    x[k] = make_float2(0.f, 0.f);
    if (lineok && i < a.n_in) {
      if constexpr (LD == CL_REAL)
        x[k].x = static_cast<const float*>(a.in)[line * a.in_line + i];
      else
        x[k] = static_cast<const float2*>(a.in)[line * a.in_line + i];
    }
  });
  static_for<EMAX>([&](auto k_) {
    constexpr int k = decltype(k_)::value;
    const int i = p + k * P;
    if (i < n) my[i] = x[k];
  });
  float2* twl = glds + L * n;
  gen_load_twiddles(twl, g);
  __syncthreads();
  gen_fft<EMAX, INV>(my, 1, g, twl, p, P);
  if constexpr (ST == CS_BINS) {
    const long long line0 = (long long)blockIdx.x * L;
    for (int k = tid; k < L * a.nbins; k += blockDim.x) {
      const int ll = k / a.nbins, f = k % a.nbins;
      if (line0 + ll < a.nlines)
        static_cast<float2*>(a.out)[(line0 + ll) * a.out_line + f] = glds[ll * n + a.bins[f]];
    }
  } else if constexpr (ST == CS_ABS2_MAX) {
    float m = 0.f;
    for (int i = p; i < a.n_out; i += P) {
      const float2 v = my[i];
      const float e = (v.x * v.x + v.y * v.y) * a.oscale;
      if (lineok && a.out != nullptr) static_cast<float*>(a.out)[line * a.out_line + i] = e;
      m = fmaxf(m, e);
    }
    if (a.img != nullptr) {
      const int W = P < 64 ? P : 64;  // lanes of one line within a wave
      for (int off = 1; off < W; off <<= 1) m = fmaxf(m, __shfl_xor(m, off, W));
      if (lineok && (p % W) == 0)
        atomicMax(reinterpret_cast<unsigned int*>(a.img) + line, __float_as_uint(m));
    }
  } else {
    if (!lineok) return;
    for (int i = p; i < a.n_out; i += P) {
      const float2 v = my[i];
      if constexpr (ST == CS_C64) {
        static_cast<float2*>(a.out)[line * a.out_line + i] = v;
      } else {  // CS_ABS_IMG
        const float m = sqrtf(v.x * v.x + v.y * v.y) * a.oscale;
        if (a.out != nullptr) static_cast<float*>(a.out)[line * a.out_line + i] = m;
        if (a.img != nullptr)
          atomicMax(reinterpret_cast<unsigned int*>(a.img) + (line % a.img_lines) * a.out_line + i,
                    __float_as_uint(m));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// f-k pass 1: real x-FFT of two t-columns per complex line (FP32 storage)
// ---------------------------------------------------------------------------

template <int EMAX>
__global__ __launch_bounds__(kGenMaxThreads) void gen_xr2c(FkXArgs a, GenPlan g, int lt) {
  extern __shared__ float2 glds[];
  const int n = g.n, T = 1 << lt, P = blockDim.x >> lt;
  const int tid = threadIdx.x;
  const int c = tid & (T - 1), p = tid >> lt;
  const long long y = blockIdx.y;
  const int t0 = 2 * (gen_tile() * T + c);  // real columns t0 and t0 + 1
  const bool colok = t0 < a.nt, has1 = t0 + 1 < a.nt;
  const float s0 = a.unscaled ? 1.f : float(t0) * a.tscale;
  const float s1 = a.unscaled ? 1.f : float(t0 + 1) * a.tscale;
  float2 x[EMAX];
  static_for<EMAX>([&](auto k_) {
    constexpr int k = decltype(k_)::value;
    const int i = p + k * P;
    x[k] = make_float2(0.f, 0.f);
    if (colok && i < a.nx) {
      const float* row = a.tau + (y * a.nx + i) * a.nt + t0;
      x[k].x = row[0];
      if (has1) x[k].y = row[1];
    }
  });
  static_for<EMAX>([&](auto k_) {
    constexpr int k = decltype(k_)::value;
    const int i = p + k * P;
    if (i < n) glds[i * T + c] = make_float2(x[k].x * s0, x[k].y * s1);
  });
  float2* twl = glds + n * T;
  gen_load_twiddles(twl, g);
  __syncthreads();
  gen_fft<EMAX, false>(glds + c, T, g, twl, p, P);
  if (!colok) return;
  float2* out = static_cast<float2*>(a.out) + y * a.out_plane + t0;
  for (int k = p; k <= n / 2; k += P) {
    const float2 zk = glds[k * T + c];
    const float2 zm = glds[(k == 0 ? 0 : n - k) * T + c];
    // A = (Z[k] + conj Z[-k]) / 2, B = (Z[k] - conj Z[-k]) / (2i)
    out[(long long)k * a.nt] = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
    if (has1) out[(long long)k * a.nt + 1] = make_float2(0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x));
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

bool gen_plan_radices(int n, GenPlan* g) {
  if (n < 2 || n > kGenMaxN || (n & 1)) return false;
  int m = n, k = 0;
  int e = 0;
  while (m % 2 == 0) { m /= 2; ++e; }
  int rad[kGenMaxStages + 8];
  while (e > 0) {  // the power-of-two part in radices 16, 8, 4, 2 (2^5 as 8 x 4)
    const int r = (e >= 4 && e != 5) ? 16 : e >= 3 ? 8 : e == 2 ? 4 : 2;
    rad[k++] = r;
    e -= ilog2i(r);
  }
  while (m % 9 == 0) {  // pairs of 3 as radix 9
    m /= 9;
    rad[k++] = 9;
  }
  for (int pr : {3, 5, 7, 11, 13})
    while (m % pr == 0) {
      m /= pr;
      rad[k++] = pr;
      if (k > kGenMaxStages) return false;
    }
  if (m != 1 || k > kGenMaxStages) return false;
  g->n = n;
  g->nstage = k;
  for (int i = 0; i < kGenMaxStages; ++i) g->radix[i] = i < k ? rad[i] : 1;
  return true;
}

namespace {

template <bool INV, int ST>
hipError_t gen_strided_st(const GenPlan& g, const StridedArgs& a, int nplanes, hipStream_t s) {
  const int T = gen_cols(g.n), P = gen_line_threads(g.n);
  const dim3 grid((a.ncols + T - 1) / T, nplanes);
  const size_t lds = (size_t)g.n * (T + 1) * sizeof(float2);
  hipLaunchKernelGGL((gen_strided<kGenE, INV, ST>), grid, dim3(T * P), lds, s, a, g, ilog2i(T));
  return hipGetLastError();
}

// contiguous lines: P = a power of two >= ceil(n / kGenE) threads per line, lines per
// block up to 256 threads
void gen_contig_shape(int n, int* lp, int* lines) {
  int l = 0;
  while ((1 << l) * kGenE < n) ++l;
  *lp = l;
  *lines = (1 << l) >= 256 ? 1 : 256 >> l;
}

template <bool INV, int LD, int ST>
hipError_t gen_contig_st(const GenPlan& g, const ContigArgs& a, hipStream_t s) {
  int lp, L;
  gen_contig_shape(g.n, &lp, &L);
  const long long blocks = (a.nlines + L - 1) / L;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const size_t lds = (size_t)(L + 1) * g.n * sizeof(float2);
  hipLaunchKernelGGL((gen_contig<kGenE, INV, LD, ST>), dim3((unsigned)blocks), dim3(L << lp), lds, s, a, g, lp);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gen_strided(const GenPlan& g, bool inverse, int st, const StridedArgs& a, int nplanes,
                              hipStream_t s) {
  if (a.ncols <= 0 || nplanes <= 0 || a.n_out > g.n) return hipErrorInvalidValue;
  switch (st) {
    case ST_C64: return inverse ? gen_strided_st<true, ST_C64>(g, a, nplanes, s)
                                : gen_strided_st<false, ST_C64>(g, a, nplanes, s);
    case ST_C64_SCALED: return inverse ? gen_strided_st<true, ST_C64_SCALED>(g, a, nplanes, s)
                                       : gen_strided_st<false, ST_C64_SCALED>(g, a, nplanes, s);
    case ST_ABS_IMG: return inverse ? gen_strided_st<true, ST_ABS_IMG>(g, a, nplanes, s)
                                    : gen_strided_st<false, ST_ABS_IMG>(g, a, nplanes, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gen_contig(const GenPlan& g, bool inverse, int ld, int st, const ContigArgs& a, hipStream_t s) {
  if (a.nlines <= 0 || a.n_out > g.n) return hipErrorInvalidValue;
  if (ld == CL_REAL && st == CS_BINS && !inverse) return gen_contig_st<false, CL_REAL, CS_BINS>(g, a, s);
  if (ld != CL_C64) return hipErrorInvalidValue;
  switch (st) {
    case CS_C64: return inverse ? gen_contig_st<true, CL_C64, CS_C64>(g, a, s)
                                : gen_contig_st<false, CL_C64, CS_C64>(g, a, s);
    case CS_ABS2_MAX: return inverse ? gen_contig_st<true, CL_C64, CS_ABS2_MAX>(g, a, s)
                                     : hipErrorInvalidValue;
    case CS_ABS_IMG: return inverse ? gen_contig_st<true, CL_C64, CS_ABS_IMG>(g, a, s)
                                    : hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gen_xr2c(const GenPlan& g, const FkXArgs& a, int ny, hipStream_t s) {
  if (ny <= 0 || a.nx > g.n || a.nt < 1) return hipErrorInvalidValue;
  const int T = gen_cols(g.n), P = gen_line_threads(g.n);
  const int pairs = (a.nt + 1) / 2;
  const dim3 grid((pairs + T - 1) / T, ny);
  const size_t lds = (size_t)g.n * (T + 1) * sizeof(float2);
  hipLaunchKernelGGL((gen_xr2c<kGenE>), grid, dim3(T * P), lds, s, a, g, ilog2i(T));
  return hipGetLastError();
}

}  // namespace nlos
