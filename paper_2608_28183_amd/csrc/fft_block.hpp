// Block-level FFT driver shared by the pass kernels: Stockham stages through LDS,
// tile shapes of the strided and contiguous families.
#pragma once

#include "fft_device.hpp"

namespace nlos {

// ---------------------------------------------------------------------------
// shared stage driver
// ---------------------------------------------------------------------------

template <int N, int R, int Ns, int E, class Idx>
__device__ __forceinline__ void write_lds(const float2* v, int p, float2* lds, Idx idx) {
  static_for<E / R>([&](auto b_) {
    static_for<R>([&](auto r_) {
      constexpr int b = decltype(b_)::value, r = decltype(r_)::value;
      lds[idx(stage_out_index<N, R, Ns, E>(p, b, r))] = v[b * R + r];
    });
  });
}

template <int N, int R, int E, class Idx>
__device__ __forceinline__ void read_lds(float2* v, int p, const float2* lds, Idx idx) {
  static_for<E / R>([&](auto b_) {
    static_for<R>([&](auto r_) {
      constexpr int b = decltype(b_)::value, r = decltype(r_)::value;
      v[b * R + r] = lds[idx(stage_in_index<N, R, E>(p, b, r))];
    });
  });
}

template <int N, int R, int Ns, int E, class Store>
__device__ __forceinline__ void emit(const float2* v, int p, Store store) {
  static_for<E / R>([&](auto b_) {
    static_for<R>([&](auto r_) {
      constexpr int b = decltype(b_)::value, r = decltype(r_)::value;
      store(stage_out_index<N, R, Ns, E>(p, b, r), v[b * R + r]);
    });
  });
}

// One component (C = 0: real parts, 1: imaginary parts) of write_lds / read_lds, through
// a float buffer: half the LDS of a complex exchange.
template <int N, int R, int Ns, int E, int C, class Idx>
__device__ __forceinline__ void write_lds_part(const float2* v, int p, float* lds, Idx idx) {
  static_for<E / R>([&](auto b_) {
    static_for<R>([&](auto r_) {
      constexpr int b = decltype(b_)::value, r = decltype(r_)::value;
      lds[idx(stage_out_index<N, R, Ns, E>(p, b, r))] = C == 0 ? v[b * R + r].x : v[b * R + r].y;
    });
  });
}

template <int N, int R, int E, class Idx>
__device__ __forceinline__ void read_lds_part(float* out, int p, const float* lds, Idx idx) {
  static_for<E / R>([&](auto b_) {
    static_for<R>([&](auto r_) {
      constexpr int b = decltype(b_)::value, r = decltype(r_)::value;
      out[b * R + r] = lds[idx(stage_in_index<N, R, E>(p, b, r))];
    });
  });
}

// Stage s (1 or 2) of plan S with twiddles from the global table or from registers.
template <class S, int STAGE, bool INV>
__device__ __forceinline__ void apply_stage(float2* v, int p, const float2* __restrict__ tw) {
  constexpr int N = S::R0 * S::R1 * S::R2;
  if constexpr (STAGE == 1) stage_compute<N, S::R1, S::R0, S::E, INV>(v, p, tw);
  else stage_compute<N, S::R2, S::R0 * S::R1, S::E, INV>(v, p, tw);
}
template <class S, int STAGE, bool INV>
__device__ __forceinline__ void apply_stage(float2* v, int, const TwRegs<S>& tw) {
  if constexpr (STAGE == 1) stage_compute_reg<S::R1, S::E, INV>(v, tw.w1);
  else stage_compute_reg<S::R2, S::E, INV>(v, tw.w2);
}

// Inter-stage twiddles from tables in LDS (short-latency reads in place of global ones).
// Stage 1 (span R0, radix R1): t[r * R0 + j] = W_{R0 R1}^(j r), r < R1, j < R0.
// Stage 2 of three-stage plans (span R0 R1, radix R2): t2[(r - 1) R0 R1 + j] = W_N^(j r),
// 1 <= r < R2, j < R0 R1.
template <class S>
struct TwLds {
  const float2* t;
  const float2* t2;
};
template <class S, int STAGE, bool INV>
__device__ __forceinline__ void apply_stage(float2* v, int p, const TwLds<S>& tw) {
  static_assert(S::NSTAGE >= 2 && STAGE <= S::NSTAGE - 1, "a stage after the first");
  constexpr int R = STAGE == 1 ? S::R1 : S::R2;
  constexpr int NS = STAGE == 1 ? S::R0 : S::R0 * S::R1;  // span of the stage
  constexpr int E = S::E, P = S::P;
  static_for<E / R>([&](auto b_) {
    constexpr int b = decltype(b_)::value;
    const int jm = (p + b * P) % NS;
    static_for<R - 1>([&](auto r_) {
      constexpr int r = decltype(r_)::value + 1;
      float2 w = STAGE == 1 ? tw.t[r * NS + jm] : tw.t2[(r - 1) * NS + jm];
      if (INV) w.y = -w.y;
      v[b * R + r] = cmul(v[b * R + r], w);
      // eight table reads in flight at a time, not all R - 1 (their registers on top of
      // the line's would cost occupancy)
      if constexpr (r % 8 == 0) __builtin_amdgcn_sched_barrier(0);
    });
    dft<R, INV>(v + b * R);
  });
}

// v holds the stage-0 inputs (element stage_in_index<N, R0, E>(p, b, r) at v[b*R0 + r]).
// Runs every stage; the last stage's outputs stay in v in the order emit_last visits.
// SPLIT (two- and three-stage plans): each exchange moves the real parts, then the
// imaginary parts, through a float buffer of half the size (lds is then a float array in
// disguise).
template <class S, bool INV, bool SPLIT = false, class Idx, class TW>
__device__ __forceinline__ void fft_stages(float2* v, int p, float2* lds, Idx idx, const TW& tw) {
  constexpr int N = S::R0 * S::R1 * S::R2;
  constexpr int E = S::E;
  stage_compute<N, S::R0, 1, E, INV>(v, p, nullptr);
  if constexpr (SPLIT) {
    static_assert(S::NSTAGE >= 2, "split exchange of multi-stage plans");
    float* f = reinterpret_cast<float*>(lds);
    {
      float re[E], im[E];
      write_lds_part<N, S::R0, 1, E, 0>(v, p, f, idx);
      __syncthreads();
      read_lds_part<N, S::R1, E>(re, p, f, idx);
      __syncthreads();
      write_lds_part<N, S::R0, 1, E, 1>(v, p, f, idx);
      __syncthreads();
      read_lds_part<N, S::R1, E>(im, p, f, idx);
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = make_float2(re[j], im[j]);
    }
    apply_stage<S, 1, INV>(v, p, tw);
    if constexpr (S::NSTAGE == 3) {
      float re[E], im[E];
      __syncthreads();  // every read of the first exchange before the second's writes
      write_lds_part<N, S::R1, S::R0, E, 0>(v, p, f, idx);
      __syncthreads();
      read_lds_part<N, S::R2, E>(re, p, f, idx);
      __syncthreads();
      write_lds_part<N, S::R1, S::R0, E, 1>(v, p, f, idx);
      __syncthreads();
      read_lds_part<N, S::R2, E>(im, p, f, idx);
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = make_float2(re[j], im[j]);
      apply_stage<S, 2, INV>(v, p, tw);
    }
    return;
  }
  if constexpr (S::NSTAGE >= 2) {
    write_lds<N, S::R0, 1, E>(v, p, lds, idx);
    __syncthreads();
    read_lds<N, S::R1, E>(v, p, lds, idx);
    if constexpr (S::NSTAGE == 2) {
      apply_stage<S, 1, INV>(v, p, tw);
    } else {
      __syncthreads();
      apply_stage<S, 1, INV>(v, p, tw);
      write_lds<N, S::R1, S::R0, E>(v, p, lds, idx);
      __syncthreads();
      read_lds<N, S::R2, E>(v, p, lds, idx);
      apply_stage<S, 2, INV>(v, p, tw);
    }
  }
}

// Calls store(n, value) for every output element held by thread p after fft_stages.
template <class S, class Store>
__device__ __forceinline__ void emit_last(const float2* v, int p, Store store) {
  constexpr int N = S::R0 * S::R1 * S::R2;
  constexpr int E = S::E;
  if constexpr (S::NSTAGE == 1) emit<N, S::R0, 1, E>(v, p, store);
  else if constexpr (S::NSTAGE == 2) emit<N, S::R1, S::R0, E>(v, p, store);
  else emit<N, S::R2, S::R0 * S::R1, E>(v, p, store);
}

// All stages, then store(n, value) for every output.  SYNC_BEFORE_STORE puts a
// barrier between the last LDS read and the stores (for stores into LDS).
template <class S, bool INV, bool SYNC_BEFORE_STORE, bool SPLIT = false, class Idx, class TW, class Store>
__device__ __forceinline__ void fft_run(float2* v, int p, float2* lds, Idx idx, const TW& tw,
                                        Store store) {
  fft_stages<S, INV, SPLIT>(v, p, lds, idx, tw);
  if constexpr (SYNC_BEFORE_STORE) __syncthreads();
  emit_last<S>(v, p, store);
}

// First-stage inputs of thread p without per-element branches: raw[r] = ld(n) for
// element n = p + r P of the line when n < n_in and ok, zero otherwise, so that all of
// the thread's loads are issued back to back.  The zero padding of a line is either
// absent (n_in >= N) or its upper half (n_in = N/2: exactly r >= E/2); other lengths
// load a clamped in-bounds element and select.  ld must accept any n in [0, n_in).
template <class S, class R, class Ld>
__device__ __forceinline__ void load_first_stage(R* raw, int p, int n_in, bool ok, R zero, Ld ld) {
  constexpr int N = S::R0 * S::R1 * S::R2, E = S::E, P = S::P;
  static_assert(S::R0 == E, "first-stage radix equals the samples per thread");
  if (n_in >= N) {
    static_for<E>([&](auto r_) { raw[decltype(r_)::value] = ld(p + decltype(r_)::value * P); });
  } else if (2 * n_in == N) {
    static_for<E / 2>([&](auto r_) { raw[decltype(r_)::value] = ld(p + decltype(r_)::value * P); });
    static_for<E / 2>([&](auto r_) { raw[E / 2 + decltype(r_)::value] = zero; });
  } else {
    static_for<E>([&](auto r_) {
      constexpr int r = decltype(r_)::value;
      const int n = p + r * P;
      const R x = ld(n < n_in ? n : 0);
      raw[r] = n < n_in ? x : zero;
    });
  }
  if (!ok) static_for<E>([&](auto r_) { raw[decltype(r_)::value] = zero; });
}

// ---------------------------------------------------------------------------
// strided-axis lines
// ---------------------------------------------------------------------------

// default columns per block for the strided passes: about 256 threads, 4..64 columns
constexpr int default_t(int n) {
  return (256 / (n / default_e(n)) < 4) ? 4 : ((256 / (n / default_e(n)) > 64) ? 64 : 256 / (n / default_e(n)));
}

template <int N, int E, int T_>
struct StridedCfg {
  using S = FftShape<N, E>;
  static constexpr int P = S::P;
  static constexpr int T = T_;
  static constexpr int THREADS = T * P;
  static constexpr int LDS_W = T + 1;
  static constexpr int LDS_ELEMS = S::NSTAGE > 1 ? N * LDS_W : 1;
};

template <int N, int E = default_e(N)>
struct ContigCfg {
  using S = FftShape<N, E>;
  static constexpr int P = S::P;
  static constexpr int L = 256 / P < 1 ? 1 : 256 / P;
  static constexpr int THREADS = L * P;
  static constexpr int LSTRIDE = N + (N >= 32 ? N / 32 : 1);
  static constexpr int LDS_ELEMS = L * LSTRIDE;
};

__device__ __forceinline__ int swz(int n) { return n + (n >> 5); }

}  // namespace nlos
