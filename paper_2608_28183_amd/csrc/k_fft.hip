// FFT pass kernels for f-k migration and RSD on gfx950.
//
// Two families, both built from the Stockham stages of fft_device.hpp:
//   strided_fft  -- lines along a strided axis (x or y of a [y][x][t] volume, y of
//                   a [plane][y][x] stack); a block owns T contiguous columns of
//                   one plane, so every global access is a T-wide contiguous run;
//   contig_fft   -- lines along the contiguous axis; a block owns L whole lines.
// The f-k specific passes (real-input x pass, paired column pass) are in k_fk.hip.
#include "fft_block.hpp"
#include "nlos_internal.hpp"
#include "prec.hpp"

namespace nlos {

// NT: non-temporal loads and stores of the FP32 complex lines (the f-k volumes)
template <int N, int E, int T_, bool INV, int LD, int ST, int SP = SP_F32, bool NT = false>
__global__ __launch_bounds__((StridedCfg<N, E, T_>::THREADS)) void strided_fft(StridedArgs a,
                                                                              const float2* __restrict__ tw) {
  using C = StridedCfg<N, E, T_>;
  using S = typename C::S;
  using ST_ = Stor<SP>;
  constexpr int T = C::T;
  constexpr int E_ = S::E;
  __shared__ float2 lds[C::LDS_ELEMS];
  const int tid = threadIdx.x;
  const int c = tid % T;
  const int p = tid / T;
  const long long plane = blockIdx.y;
  const int col = blockIdx.x * T + c;
  const bool colok = col < a.ncols;

  float2 v[E_];
  if constexpr (SP == SP_F32 || LD == LD_TAU_SCALED) {
    static_for<E / S::R0>([&](auto b_) {
      static_for<S::R0>([&](auto r_) {
        constexpr int b = decltype(b_)::value, r = decltype(r_)::value;
        const int n = stage_in_index<N, S::R0, E_>(p, b, r);
        float2 x = make_float2(0.f, 0.f);
        if (colok && n < a.n_in) {
          const long long i = plane * a.in_plane + (long long)n * a.in_line + col;
          if constexpr (LD == LD_TAU_SCALED) {
            x.x = static_cast<const float*>(a.in)[i] * (float(col) * a.tscale);
          } else if constexpr (NT) {
            x = ld_stream(static_cast<const float2*>(a.in) + i);
          } else {
            x = static_cast<const float2*>(a.in)[i];
          }
        }
        v[b * S::R0 + r] = x;
      });
    });
  } else {
    // four-byte storage: raw loads first, conversion after, so that all loads of the
    // thread are in flight together
    typename ST_::R raw[E_];
    // addresses relative to row p, so that row r P + p is a scalar multiple of in_line away
    const typename ST_::T* in = static_cast<const typename ST_::T*>(a.in) + plane * a.in_plane +
                                (colok ? col : 0) + (long long)p * a.in_line;
    load_first_stage<S>(raw, p, a.n_in, colok, ST_::zero(),
                        [&](int n) { return ST_::raw(in, (long long)(n - p) * a.in_line); });
    const int e = SP == SP_F16 ? -a.e_in[a.e_per_col && colok ? col : 0] : 0;
#pragma unroll
    for (int j = 0; j < E_; ++j) {
      v[j] = ST_::cvt(raw[j]);
      if constexpr (SP == SP_F16) v[j] = ldexp2(v[j], e);
    }
  }

  auto idx = [&](int n) { return n * C::LDS_W + c; };
  if constexpr (ST == ST_C64 && SP != SP_F32) {
    const int e = SP == SP_F16 ? a.e_out[a.e_per_col && colok ? col : 0] : 0;
    fft_run<S, INV, false>(v, p, lds, idx, tw, [&](int n, float2 val) {
      if (colok && n < a.n_out)
        ST_::st(static_cast<typename ST_::T*>(a.out), plane * a.out_plane + (long long)n * a.out_line + col,
                SP == SP_F16 ? ldexp2(val, e) : val);
    });
    return;
  }
  auto store = [&](int n, float2 val) {
    if constexpr (ST == ST_C64 || ST == ST_C64_SCALED) {
      if (colok && n < a.n_out)
      {
        const float2 w = ST == ST_C64_SCALED ? cscale(val, a.oscale) : val;
        float2* dst = static_cast<float2*>(a.out) + plane * a.out_plane + (long long)n * a.out_line + col;
        if constexpr (NT) {
          st_stream(dst, w);
        } else {
          *dst = w;
        }
      }
    } else {  // |v|^2 or |v| (times a.oscale) plus a max over this tile's columns into img
      float m = val.x * val.x + val.y * val.y;
      if constexpr (ST == ST_ABS_IMG) m = sqrtf(m);
      m = colok ? m * a.oscale : 0.f;
      if (a.out != nullptr && colok && n < a.n_out)
        static_cast<float*>(a.out)[plane * a.out_plane + (long long)n * a.out_line + col] = m;
      if (a.img != nullptr) {
#pragma unroll
        for (int off = 1; off < T; off <<= 1) m = fmaxf(m, __shfl_xor(m, off, T));
        if (c == 0 && n < a.n_out)
          atomicMax(reinterpret_cast<unsigned int*>(a.img) + plane * a.img_plane + n,
                    __float_as_uint(m));
      }
    }
  };
  fft_run<S, INV, false>(v, p, lds, idx, tw, store);
}

// FP32 complex lines along a strided axis with non-temporal loads and stores (the f-k y,
// inverse x and inverse y passes), as strided_fft<N, E, T, INV, LD_C64, ST_C64, SP_F32,
// true> computes them when n_in is N or N/2 (IN_HALF: the upper half is zero padding) and
// n_out is N or N/2 (OUT_HALF: the lower half is kept).  The blocks stay resident and
// walk (plane, column tile) items, item i then i + gridDim.x, ...: the next item's
// samples are loaded while the current item is transformed, and the stage twiddles stay
// in registers for the block's lifetime.  A column past ncols (in the last tile) stands
// in for the tile's first column: it reads that column, computes the same values and
// stores them to the same places, so every thread issues the same stores and the wait
// for the prefetched loads leaves the item's stores in flight.
template <int N, int E, int T_, bool INV, bool IN_HALF, bool OUT_HALF>
__global__ __launch_bounds__((StridedCfg<N, E, T_>::THREADS)) void strided_c64_stream(
    StridedArgs a, const float2* __restrict__ tw, int ntiles, int nitems) {
  using C = StridedCfg<N, E, T_>;
  using S = typename C::S;
  constexpr int T = C::T, E_ = S::E, P = S::P;
  constexpr int RL = S::NSTAGE == 1 ? S::R0 : (S::NSTAGE == 2 ? S::R1 : S::R2);  // last radix
  constexpr int NR = IN_HALF ? E_ / 2 : E_;  // nonzero inputs per thread
  static_assert(S::R0 == E_ && RL % 2 == 0, "first radix E, even last radix");
  __shared__ float2 lds[C::LDS_ELEMS];
  const int tid = threadIdx.x;
  const int c = tid % T;
  const int p = tid / T;
  TwRegs<S> twr;
  twr.load(p, tw);
  // the twiddles arrive before the first item's loads are issued: the waits of the loop
  // then count only that loop's own loads and stores
  __builtin_amdgcn_s_waitcnt(0);

  // the thread's column and plane offset of item it (a column past the end: the tile's first)
  auto column = [&](int it, int& plane) {
    plane = (unsigned)it / (unsigned)ntiles;
    const int col0 = (it - plane * ntiles) * T;
    return col0 + c < a.ncols ? col0 + c : col0;
  };
  float2 raw[NR];  // elements p + r P, r < NR, of the column
  auto fetch = [&](int it) {
    int plane;
    const int col = column(it, plane);
    const float2* in = static_cast<const float2*>(a.in) + plane * a.in_plane + col + (long long)p * a.in_line;
    static_for<NR>([&](auto r_) {
      constexpr int r = decltype(r_)::value;
      raw[r] = ld_stream(in + (long long)(r * P) * a.in_line);
    });
  };
  auto idx = [&](int n) { return n * C::LDS_W + c; };
  int it = blockIdx.x;
  if (it < nitems) fetch(it);
  // the first item's samples are needed at once; waiting here also leaves the loop's
  // own waits free of the loads issued before it
  __builtin_amdgcn_s_waitcnt(0);
  for (; it < nitems; it += gridDim.x) {
    float2 v[E_];
#pragma unroll
    for (int j = 0; j < NR; ++j) v[j] = raw[j];
#pragma unroll
    for (int j = NR; j < E_; ++j) v[j] = make_float2(0.f, 0.f);
    int plane;
    const int col = column(it, plane);
    if (it + (int)gridDim.x < nitems) fetch(it + gridDim.x);

    fft_stages<S, INV>(v, p, lds, idx, twr);
    // last stage: butterfly b of thread p holds outputs n = p + b P + r (N / RL); the
    // lower half is r < RL / 2
    float2* out = static_cast<float2*>(a.out) + plane * a.out_plane + col;
    static_for<E_ / RL>([&](auto b_) {
      static_for<RL>([&](auto r_) {
        constexpr int b = decltype(b_)::value, r = decltype(r_)::value;
        if constexpr (!OUT_HALF || r < RL / 2)
          st_stream(out + (long long)(p + b * P + r * (N / RL)) * a.out_line, v[b * RL + r]);
      });
    });
    __syncthreads();  // every read of this item's exchanges before the next item's writes
  }
}

// ---------------------------------------------------------------------------
// contiguous lines
// ---------------------------------------------------------------------------

// samples per thread of the contiguous passes (32 at 1024-point lines measured faster
// than 16 for the z-IFFT of the 256x256x512 f-k)
template <int N>
struct ContigTune {
  static constexpr int E = default_e(N);
};

// HALF: the line's upper half is zero padding (n_in = N/2) and only the lower half of the
// outputs is kept (n_out = N/2), both known at compile time, so the zero inputs fold out
// of the first radix stage and the unused outputs out of the last.
template <int N, bool INV, int LD, int ST, int SP = SP_F32, bool HALF = false>
__global__ __launch_bounds__((ContigCfg<N, ContigTune<N>::E>::THREADS)) void contig_fft(
    ContigArgs a, const float2* __restrict__ tw) {
  using C = ContigCfg<N, ContigTune<N>::E>;
  using S = typename C::S;
  constexpr int E = S::E, P = C::P;
  constexpr bool NEED_LDS = (S::NSTAGE > 1) || (ST == CS_BINS);
  // the |.|^2 pass uses LDS only for the exchange of its two-stage plans: real and
  // imaginary parts in turn, half the LDS, more lines resident per CU
  constexpr bool SPLIT = ST == CS_ABS2_MAX && S::NSTAGE == 2;
  __shared__ float2 lds[NEED_LDS ? (SPLIT ? (C::LDS_ELEMS + 1) / 2 : C::LDS_ELEMS) : 1];
  const int tid = threadIdx.x;
  const int l = tid / P;
  const int p = tid % P;
  const long long line = (long long)blockIdx.x * C::L + l;
  const bool lineok = line < a.nlines;
  float2 v[E];
  if constexpr (LD == CL_REAL || LD == CL_REAL_PAIR) {
    // real lines: raw loads first, branch-free (a missing line reads a present one and is
    // zeroed after), so that all of the thread's loads are in flight together
    static_assert(!HALF, "real lines are not zero-padded here");
    const bool oddok = LD == CL_REAL_PAIR && 2 * line + 1 < a.nreal;  // the pair's second line
    const float* f = static_cast<const float*>(a.in);
    const long long ra = lineok ? (LD == CL_REAL_PAIR ? 2 * line : line) : 0;
    const float* pa = f + ra * a.in_line;
    float xa[E], xb[E];
    load_first_stage<S>(xa, p, a.n_in, lineok, 0.f, [&](int n) { return pa[n]; });
    if constexpr (LD == CL_REAL_PAIR) {
      const float* pb = f + (oddok ? 2 * line + 1 : ra) * a.in_line;
      load_first_stage<S>(xb, p, a.n_in, oddok, 0.f, [&](int n) { return pb[n]; });
    }
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = make_float2(xa[j], LD == CL_REAL_PAIR ? xb[j] : 0.f);
  } else {
    // complex lines: raw loads first, branch-free (a line past the end reads line 0 and
    // is zeroed), conversion of four-byte storage after
    using ST_ = Stor<SP>;
    typename ST_::R raw[E];
    const typename ST_::T* in = static_cast<const typename ST_::T*>(a.in) + (lineok ? line : 0) * a.in_line;
    if constexpr (HALF) {
      static_assert(S::R0 == E, "first-stage radix equals the samples per thread");
      static_for<E / 2>([&](auto r_) {
        constexpr int r = decltype(r_)::value;
        raw[r] = ST_::raw(in, p + r * P);
        if (!lineok) raw[r] = ST_::zero();
      });
      static_for<E / 2>([&](auto r_) { raw[E / 2 + decltype(r_)::value] = ST_::zero(); });
    } else {
      load_first_stage<S>(raw, p, a.n_in, lineok, ST_::zero(), [&](int n) { return ST_::raw(in, n); });
    }
    const int e = SP == SP_F16 ? -*a.e_in : 0;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      v[j] = ST_::cvt(raw[j]);
      if constexpr (SP == SP_F16) v[j] = ldexp2(v[j], e);
    }
  }

  // a line's part of LDS: LSTRIDE complex values, or LSTRIDE floats when SPLIT
  float2* my = SPLIT ? reinterpret_cast<float2*>(reinterpret_cast<float*>(lds) + l * C::LSTRIDE)
                     : lds + (NEED_LDS ? l * C::LSTRIDE : 0);
  auto idx = [&](int n) { return swz(n); };
  if constexpr (ST == CS_BINS) {
    // natural-order spectrum into LDS, then gather the requested bins (four-byte output
    // for SP_F16 / SP_BF16, FP16 times 2^(*e_out))
    auto store = [&](int n, float2 val) { my[swz(n)] = val; };
    fft_run<S, INV, true>(v, p, my, idx, tw, store);
    __syncthreads();
    const long long line0 = (long long)blockIdx.x * C::L;
    const int eo = SP == SP_F16 ? *a.e_out : 0;
    auto put = [&](long long row, int f, float2 val) {
      if constexpr (SP == SP_F32) {
        static_cast<float2*>(a.out)[row * a.out_line + f] = val;
      } else {
        using SO = Stor<SP>;
        SO::st(static_cast<typename SO::T*>(a.out), row * a.out_line + f, SP == SP_F16 ? ldexp2(val, eo) : val);
      }
    };
    for (int k = tid; k < C::L * a.nbins; k += C::THREADS) {
      const int ll = k / a.nbins;
      const int f = k % a.nbins;
      const long long ln = line0 + ll;
      if (ln < a.nlines) {
        const int bin = a.bins[f];
        const float2 z = lds[ll * C::LSTRIDE + swz(bin)];
        if constexpr (LD == CL_REAL_PAIR) {
          // Z = X_a + i X_b for real lines a, b: X_a[k] = (Z[k] + conj Z[N-k]) / 2,
          // X_b[k] = (Z[k] - conj Z[N-k]) / 2i
          const float2 zm = lds[ll * C::LSTRIDE + swz((N - bin) & (N - 1))];
          put(2 * ln, f, make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y)));
          if (2 * ln + 1 < a.nreal) put(2 * ln + 1, f, make_float2(0.5f * (z.y + zm.y), 0.5f * (zm.x - z.x)));
        } else {
          put(ln, f, z);
        }
      }
    }
  } else if constexpr (ST == CS_ABS2_MAX) {
    // |v|^2 * oscale into out[line][n < n_out] and the max over the line into img[line]
    // (a line past the end holds zeros: it adds nothing to m and stores nothing)
    float m = 0.f;
    float* orow = a.out != nullptr ? static_cast<float*>(a.out) + (lineok ? line : 0) * a.out_line : nullptr;
    const bool wr = lineok && orow != nullptr;
    auto store = [&](int n, float2 val) {
      if (n >= (HALF ? N / 2 : a.n_out)) return;
      const float e = (val.x * val.x + val.y * val.y) * a.oscale;
      if (wr) orow[n] = e;
      m = fmaxf(m, e);
    };
    fft_run<S, INV, false, SPLIT>(v, p, my, idx, tw, store);
    if (a.img != nullptr) {
      constexpr int W = P < 64 ? P : 64;
#pragma unroll
      for (int off = 1; off < W; off <<= 1) m = fmaxf(m, __shfl_xor(m, off, W));
      if (lineok && (p % W) == 0)
        atomicMax(reinterpret_cast<unsigned int*>(a.img) + line, __float_as_uint(m));
    }
  } else {
    auto store = [&](int n, float2 val) {
      if (!lineok || n >= a.n_out) return;
      if constexpr (ST == CS_C64) {
        static_cast<float2*>(a.out)[line * a.out_line + n] = val;
      } else {  // |v| (times oscale) and max into img[line % img_lines][n]
        const float m = sqrtf(val.x * val.x + val.y * val.y) * a.oscale;
        if (a.out != nullptr) static_cast<float*>(a.out)[line * a.out_line + n] = m;
        if (a.img != nullptr)
          atomicMax(reinterpret_cast<unsigned int*>(a.img) + (line % a.img_lines) * a.out_line + n,
                    __float_as_uint(m));
      }
    };
    fft_run<S, INV, false>(v, p, my, idx, tw, store);
  }
}

// The FP32 z-IFFT of a zero-padded f-k volume (the upper half of every line is zero
// padding, the lower half of the outputs is kept), |.|^2 * oscale and the max over each
// line, as contig_fft<N, true, CL_C64, CS_ABS2_MAX, SP_F32, true> computes it, for two-
// and three-stage plans.  The blocks stay resident and walk groups of L lines (group g,
// then g + gridDim.x, ...): the next group's samples are loaded while the current group
// is transformed, and the inter-stage twiddles sit in LDS for the block's lifetime.  A line past
// the end (in the last group) stands in for the group's first line: it reads that line,
// so it computes the same values and stores them to the same places, and every thread
// issues the same stores, which lets the wait for the next group's loads leave this
// group's stores in flight.  a.out must not be null.
template <int N>
__global__ __launch_bounds__((ContigCfg<N, ContigTune<N>::E>::THREADS)) void zifft_abs2_stream(
    ContigArgs a, const float2* __restrict__ tw, long long ngroups) {
  using C = ContigCfg<N, ContigTune<N>::E>;
  using S = typename C::S;
  constexpr int E = S::E, P = C::P, L = C::L, R0 = S::R0, R1 = S::R1, R2 = S::R2;
  static_assert(S::NSTAGE == 2 || S::NSTAGE == 3, "two- or three-stage plans");
  constexpr int NW2 = S::NSTAGE == 3 ? (R2 - 1) * R0 * R1 : 1;
  __shared__ float xch[L * C::LSTRIDE];  // the exchange, one component at a time
  __shared__ float2 wt[R1 * R0];         // wt[r * R0 + j] = W_{R0 R1}^(j r)
  __shared__ float2 wt2[NW2];            // wt2[(r - 1) R0 R1 + j] = W_N^(j r) (three stages)
  const int tid = threadIdx.x;
  const int l = tid / P;
  const int p = tid % P;
  for (int k = tid; k < R1 * R0; k += C::THREADS) wt[k] = tw[(k % R0) * (k / R0) * (kTwiddleN / (R0 * R1))];
  if constexpr (S::NSTAGE == 3)
    for (int k = tid; k < NW2; k += C::THREADS)
      wt2[k] = tw[(k % (R0 * R1)) * (1 + k / (R0 * R1)) * (kTwiddleN / N)];

  const float2* in = static_cast<const float2*>(a.in);
  float2 raw[E / 2];  // elements p + r P (r < E/2) of the line: its nonzero half
  auto fetch = [&](long long g) {
    const long long line = g * L + l;
    const float2* row = in + (line < a.nlines ? line : g * L) * a.in_line;
    static_for<E / 2>([&](auto r_) { raw[decltype(r_)::value] = row[p + decltype(r_)::value * P]; });
  };
  float2* my = reinterpret_cast<float2*>(xch + l * C::LSTRIDE);
  auto idx = [&](int n) { return swz(n); };
  long long g = blockIdx.x;
  if (g < ngroups) fetch(g);
  for (; g < ngroups; g += gridDim.x) {
    float2 v[E];
#pragma unroll
    for (int j = 0; j < E / 2; ++j) v[j] = raw[j];
#pragma unroll
    for (int j = E / 2; j < E; ++j) v[j] = make_float2(0.f, 0.f);
    const long long line0 = g * L + l;
    const long long line = line0 < a.nlines ? line0 : g * L;
    if (g + gridDim.x < ngroups) fetch(g + gridDim.x);

    float m = 0.f;
    float* orow = static_cast<float*>(a.out) + line * a.out_line;
    auto store = [&](int n, float2 val) {
      if (n >= N / 2) return;
      const float e = (val.x * val.x + val.y * val.y) * a.oscale;
      orow[n] = e;
      m = fmaxf(m, e);
    };
    fft_run<S, true, false, true>(v, p, my, idx, TwLds<S>{wt, wt2}, store);
    if (a.img != nullptr) {
      constexpr int W = P < 64 ? P : 64;
#pragma unroll
      for (int off = 1; off < W; off <<= 1) m = fmaxf(m, __shfl_xor(m, off, W));
      if ((p % W) == 0) atomicMax(reinterpret_cast<unsigned int*>(a.img) + line, __float_as_uint(m));
    }
    __syncthreads();  // every read of this group's exchange before the next group's writes
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------


template <int N>
static hipError_t launch_zifft_stream(const ContigArgs& a, const float2* tw, hipStream_t s) {
  using C = ContigCfg<N, ContigTune<N>::E>;
  const long long ngroups = (a.nlines + C::L - 1) / C::L;
  const long long res = resident_blocks<zifft_abs2_stream<N>>(C::THREADS);
  const long long nb = res > 0 && res < ngroups ? res : ngroups;
  hipLaunchKernelGGL((zifft_abs2_stream<N>), dim3((unsigned)nb), dim3(C::THREADS), 0, s, a, tw, ngroups);
  return hipGetLastError();
}

// (samples per thread, columns per block) of the strided passes, from timing sweeps at
// 512-point lines (256x256x512 f-k): forward y pass E=16 T=16, inverse passes E=8 T=16;
// 256-point lines use 32 columns (256-byte rows).  With four-byte storage the 512-point
// passes double their columns so that a row segment stays 128 bytes (a whole cache line:
// 64-byte segments fetch every line twice); 256-point lines keep 32 columns, already
// 128 bytes at four bytes, since 64 would need 128 KB of LDS per block (one block per CU).
template <int N, bool INV, int LD, int ST, int SP = SP_F32>
struct StridedTune {
  static constexpr bool WIDE = SP != SP_F32;
  static constexpr int E = (N == 512) ? (INV && !WIDE ? 8 : 16) : default_e(N);
  static constexpr int T = (N == 512) ? (WIDE ? 32 : 16) : (N == 256 ? 32 : default_t(N));
};

template <int N, bool INV, int LD, int ST, int SP = SP_F32, bool NT = false,
          int E = StridedTune<N, INV, LD, ST, SP>::E, int T = StridedTune<N, INV, LD, ST, SP>::T>
static hipError_t launch_strided_n(const StridedArgs& a, int nplanes, const float2* tw,
                                   hipStream_t s) {
  using C = StridedCfg<N, E, T>;
  dim3 grid((a.ncols + C::T - 1) / C::T, nplanes);
  hipLaunchKernelGGL((strided_fft<N, E, T, INV, LD, ST, SP, NT>), grid, dim3(C::THREADS), 0, s, a, tw);
  return hipGetLastError();
}

template <bool INV, int LD, int ST, int SP = SP_F32, bool NT = false>
static hipError_t launch_strided_inv(int n, const StridedArgs& a, int nplanes, const float2* tw,
                                     hipStream_t s) {
  switch (n) {
    case 8: return launch_strided_n<8, INV, LD, ST, SP, NT>(a, nplanes, tw, s);
    case 16: return launch_strided_n<16, INV, LD, ST, SP, NT>(a, nplanes, tw, s);
    case 32: return launch_strided_n<32, INV, LD, ST, SP, NT>(a, nplanes, tw, s);
    case 64: return launch_strided_n<64, INV, LD, ST, SP, NT>(a, nplanes, tw, s);
    case 128: return launch_strided_n<128, INV, LD, ST, SP, NT>(a, nplanes, tw, s);
    case 256: return launch_strided_n<256, INV, LD, ST, SP, NT>(a, nplanes, tw, s);
    case 512: return launch_strided_n<512, INV, LD, ST, SP, NT>(a, nplanes, tw, s);
    case 1024: return launch_strided_n<1024, INV, LD, ST, SP, NT>(a, nplanes, tw, s);
    case 2048: return launch_strided_n<2048, INV, LD, ST, SP, NT>(a, nplanes, tw, s);
    default: return hipErrorInvalidValue;
  }
}

template <int N, bool INV, bool IN_HALF, bool OUT_HALF>
static hipError_t launch_strided_stream_n(const StridedArgs& a, int nplanes, const float2* tw, hipStream_t s) {
  using Tn = StridedTune<N, INV, LD_C64, ST_C64, SP_F32>;
  using C = StridedCfg<N, Tn::E, Tn::T>;
  const int ntiles = (a.ncols + C::T - 1) / C::T;
  const int nitems = ntiles * nplanes;
  auto k = strided_c64_stream<N, Tn::E, Tn::T, INV, IN_HALF, OUT_HALF>;
  const long long res = resident_blocks<strided_c64_stream<N, Tn::E, Tn::T, INV, IN_HALF, OUT_HALF>>(C::THREADS);
  const long long nb = res > 0 && res < nitems ? res : nitems;
  hipLaunchKernelGGL(k, dim3((unsigned)nb), dim3(C::THREADS), 0, s, a, tw, ntiles, nitems);
  return hipGetLastError();
}

// The streaming form of the FP32 f-k strided passes: forward with a zero-padded upper
// half, inverse with the lower half of the outputs kept, 256- and 512-point lines (1024
// would need 250 VGPRs).  Returns false (nothing launched) for other shapes, which
// strided_fft takes.
static bool launch_strided_stream(int n, bool inverse, const StridedArgs& a, int nplanes, const float2* tw,
                                  hipStream_t s, hipError_t& err) {
  if (a.ncols <= 0 || nplanes <= 0 || (long long)a.ncols * nplanes > (1LL << 30)) return false;
  const bool fwd_half = !inverse && 2 * a.n_in == n && a.n_out == n;
  const bool inv_half = inverse && a.n_in == n && 2 * a.n_out == n;
  if (!fwd_half && !inv_half) return false;
  switch (n) {
    case 256: err = inverse ? launch_strided_stream_n<256, true, false, true>(a, nplanes, tw, s)
                            : launch_strided_stream_n<256, false, true, false>(a, nplanes, tw, s); return true;
    case 512: err = inverse ? launch_strided_stream_n<512, true, false, true>(a, nplanes, tw, s)
                            : launch_strided_stream_n<512, false, true, false>(a, nplanes, tw, s); return true;
    default: return false;
  }
}

hipError_t launch_strided(int n, bool inverse, int ld, int st, const StridedArgs& a, int nplanes,
                          const float2* tw, hipStream_t s, int sp, bool stream) {
  hipError_t err = hipSuccess;
  if (stream && sp == SP_F32 && ld == LD_C64 && st == ST_C64 && launch_strided_stream(n, inverse, a, nplanes, tw, s, err))
    return err;
  if (stream && sp == SP_F32 && ld == LD_C64 && st == ST_C64)
    return inverse ? launch_strided_inv<true, LD_C64, ST_C64, SP_F32, true>(n, a, nplanes, tw, s)
                   : launch_strided_inv<false, LD_C64, ST_C64, SP_F32, true>(n, a, nplanes, tw, s);
  if (sp == SP_F16 && ld == LD_C64 && st == ST_C64)
    return inverse ? launch_strided_inv<true, LD_C64, ST_C64, SP_F16>(n, a, nplanes, tw, s)
                   : launch_strided_inv<false, LD_C64, ST_C64, SP_F16>(n, a, nplanes, tw, s);
  if (sp == SP_BF16 && ld == LD_C64 && st == ST_C64)
    return inverse ? launch_strided_inv<true, LD_C64, ST_C64, SP_BF16>(n, a, nplanes, tw, s)
                   : launch_strided_inv<false, LD_C64, ST_C64, SP_BF16>(n, a, nplanes, tw, s);
  // four-byte input, FP32 output (the last RSD pass: |I| or the complex field)
  if (sp == SP_F16 && inverse && ld == LD_C64 && st == ST_ABS_IMG)
    return launch_strided_inv<true, LD_C64, ST_ABS_IMG, SP_F16>(n, a, nplanes, tw, s);
  if (sp == SP_BF16 && inverse && ld == LD_C64 && st == ST_ABS_IMG)
    return launch_strided_inv<true, LD_C64, ST_ABS_IMG, SP_BF16>(n, a, nplanes, tw, s);
  if (sp == SP_F16 && inverse && ld == LD_C64 && st == ST_C64_SCALED)
    return launch_strided_inv<true, LD_C64, ST_C64_SCALED, SP_F16>(n, a, nplanes, tw, s);
  if (sp == SP_BF16 && inverse && ld == LD_C64 && st == ST_C64_SCALED)
    return launch_strided_inv<true, LD_C64, ST_C64_SCALED, SP_BF16>(n, a, nplanes, tw, s);
  if (sp != SP_F32) return hipErrorInvalidValue;
  if (!inverse && ld == LD_TAU_SCALED && st == ST_C64)
    return launch_strided_inv<false, LD_TAU_SCALED, ST_C64>(n, a, nplanes, tw, s);
  if (!inverse && ld == LD_C64 && st == ST_C64)
    return launch_strided_inv<false, LD_C64, ST_C64>(n, a, nplanes, tw, s);
  if (inverse && ld == LD_C64 && st == ST_C64)
    return launch_strided_inv<true, LD_C64, ST_C64>(n, a, nplanes, tw, s);
  if (inverse && ld == LD_C64 && st == ST_ABS2_IMG)
    return launch_strided_inv<true, LD_C64, ST_ABS2_IMG>(n, a, nplanes, tw, s);
  if (inverse && ld == LD_C64 && st == ST_ABS_IMG)
    return launch_strided_inv<true, LD_C64, ST_ABS_IMG>(n, a, nplanes, tw, s);
  if (inverse && ld == LD_C64 && st == ST_C64_SCALED)
    return launch_strided_inv<true, LD_C64, ST_C64_SCALED>(n, a, nplanes, tw, s);
  return hipErrorInvalidValue;
}

template <int N, bool INV, int LD, int ST, int SP = SP_F32, bool HALF = false>
static hipError_t launch_contig_n(const ContigArgs& a, const float2* tw, hipStream_t s) {
  using C = ContigCfg<N, ContigTune<N>::E>;
  dim3 grid((unsigned)((a.nlines + C::L - 1) / C::L));
  hipLaunchKernelGGL((contig_fft<N, INV, LD, ST, SP, HALF>), grid, dim3(C::THREADS), 0, s, a, tw);
  return hipGetLastError();
}

template <bool INV, int LD, int ST, int SP = SP_F32, bool HALF = false>
static hipError_t launch_contig_inv(int n, const ContigArgs& a, const float2* tw, hipStream_t s) {
  switch (n) {
    case 8: return launch_contig_n<8, INV, LD, ST, SP, HALF>(a, tw, s);
    case 16: return launch_contig_n<16, INV, LD, ST, SP, HALF>(a, tw, s);
    case 32: return launch_contig_n<32, INV, LD, ST, SP, HALF>(a, tw, s);
    case 64: return launch_contig_n<64, INV, LD, ST, SP, HALF>(a, tw, s);
    case 128: return launch_contig_n<128, INV, LD, ST, SP, HALF>(a, tw, s);
    case 256: return launch_contig_n<256, INV, LD, ST, SP, HALF>(a, tw, s);
    case 512: return launch_contig_n<512, INV, LD, ST, SP, HALF>(a, tw, s);
    case 1024: return launch_contig_n<1024, INV, LD, ST, SP, HALF>(a, tw, s);
    case 2048: return launch_contig_n<2048, INV, LD, ST, SP, HALF>(a, tw, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_contig(int n, bool inverse, int ld, int st, const ContigArgs& a, const float2* tw,
                         hipStream_t s, int sp) {
  // the f-k z pass of a padded volume: half the line in, half out
  const bool half = inverse && ld == CL_C64 && st == CS_ABS2_MAX && 2 * a.n_in == n && 2 * a.n_out == n;
  if (half) {
    if (sp == SP_F16) return launch_contig_inv<true, CL_C64, CS_ABS2_MAX, SP_F16, true>(n, a, tw, s);
    if (sp == SP_BF16) return launch_contig_inv<true, CL_C64, CS_ABS2_MAX, SP_BF16, true>(n, a, tw, s);
    if (sp == SP_F32 && n == 2048 && a.out != nullptr) return launch_zifft_stream<2048>(a, tw, s);
    if (sp == SP_F32 && n == 1024 && a.out != nullptr) return launch_zifft_stream<1024>(a, tw, s);
    if (sp == SP_F32 && n == 512 && a.out != nullptr) return launch_zifft_stream<512>(a, tw, s);
    if (sp == SP_F32) return launch_contig_inv<true, CL_C64, CS_ABS2_MAX, SP_F32, true>(n, a, tw, s);
  }
  if (sp == SP_F16 && inverse && ld == CL_C64 && st == CS_ABS2_MAX)
    return launch_contig_inv<true, CL_C64, CS_ABS2_MAX, SP_F16>(n, a, tw, s);
  if (sp == SP_BF16 && inverse && ld == CL_C64 && st == CS_ABS2_MAX)
    return launch_contig_inv<true, CL_C64, CS_ABS2_MAX, SP_BF16>(n, a, tw, s);
  // the RSD phasor pass: two real pixel lines per complex line, FP32 or four-byte output
  if (!inverse && ld == CL_REAL_PAIR && st == CS_BINS) {
    if (sp == SP_F16) return launch_contig_inv<false, CL_REAL_PAIR, CS_BINS, SP_F16>(n, a, tw, s);
    if (sp == SP_BF16) return launch_contig_inv<false, CL_REAL_PAIR, CS_BINS, SP_BF16>(n, a, tw, s);
    return launch_contig_inv<false, CL_REAL_PAIR, CS_BINS, SP_F32>(n, a, tw, s);
  }
  if (sp == SP_F16 && !inverse && ld == CL_REAL && st == CS_BINS)
    return launch_contig_inv<false, CL_REAL, CS_BINS, SP_F16>(n, a, tw, s);
  if (sp == SP_BF16 && !inverse && ld == CL_REAL && st == CS_BINS)
    return launch_contig_inv<false, CL_REAL, CS_BINS, SP_BF16>(n, a, tw, s);
  if (sp != SP_F32) return hipErrorInvalidValue;
  if (!inverse && ld == CL_REAL && st == CS_BINS)
    return launch_contig_inv<false, CL_REAL, CS_BINS>(n, a, tw, s);
  if (!inverse && ld == CL_C64 && st == CS_C64)
    return launch_contig_inv<false, CL_C64, CS_C64>(n, a, tw, s);
  if (inverse && ld == CL_C64 && st == CS_ABS_IMG)
    return launch_contig_inv<true, CL_C64, CS_ABS_IMG>(n, a, tw, s);
  if (inverse && ld == CL_C64 && st == CS_ABS2_MAX)
    return launch_contig_inv<true, CL_C64, CS_ABS2_MAX>(n, a, tw, s);
  if (inverse && ld == CL_C64 && st == CS_C64)
    return launch_contig_inv<true, CL_C64, CS_C64>(n, a, tw, s);
  return hipErrorInvalidValue;
}

}  // namespace nlos
