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

// v holds the stage-0 inputs (element stage_in_index<N, R0, E>(p, b, r) at v[b*R0 + r]).
// Runs every stage; outputs go through store(n, value).  When SYNC_BEFORE_STORE is
// set a barrier separates the last LDS read from the stores (for stores into LDS).
template <class S, bool INV, bool SYNC_BEFORE_STORE, class Idx, class TW, class Store>
__device__ __forceinline__ void fft_run(float2* v, int p, float2* lds, Idx idx, const TW& tw,
                                        Store store) {
  constexpr int N = S::R0 * S::R1 * S::R2;
  constexpr int E = S::E;
  stage_compute<N, S::R0, 1, E, INV>(v, p, nullptr);
  if constexpr (S::NSTAGE == 1) {
    if constexpr (SYNC_BEFORE_STORE) __syncthreads();
    emit<N, S::R0, 1, E>(v, p, store);
  } else {
    write_lds<N, S::R0, 1, E>(v, p, lds, idx);
    __syncthreads();
    read_lds<N, S::R1, E>(v, p, lds, idx);
    if constexpr (S::NSTAGE == 2) {
      apply_stage<S, 1, INV>(v, p, tw);
      if constexpr (SYNC_BEFORE_STORE) __syncthreads();
      emit<N, S::R1, S::R0, E>(v, p, store);
    } else {
      __syncthreads();
      apply_stage<S, 1, INV>(v, p, tw);
      write_lds<N, S::R1, S::R0, E>(v, p, lds, idx);
      __syncthreads();
      read_lds<N, S::R2, E>(v, p, lds, idx);
      apply_stage<S, 2, INV>(v, p, tw);
      if constexpr (SYNC_BEFORE_STORE) __syncthreads();
      emit<N, S::R2, S::R0 * S::R1, E>(v, p, store);
    }
  }
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
