// FFT pass kernels for f-k migration and RSD on gfx950.
//
// Two families, both built from the Stockham stages of fft_device.hpp:
//   strided_fft  -- lines along a strided axis (x or y of a [y][x][t] volume, y of
//                   a [plane][y][x] stack); a block owns T contiguous columns of
//                   one plane, so every global access is a T-wide contiguous run;
//   contig_fft   -- lines along the contiguous axis; a block owns L whole lines.
// fk_column is the contiguous f-k pass that runs, per (ky, kx) column, the
// forward t-FFT, the Stolt remap with its Jacobian (gathered from the LDS copy
// of the spectrum) and the inverse z-FFT, reading and writing only the nt
// samples that are non-zero on input and needed on output.
#include "fft_device.hpp"
#include "nlos_internal.hpp"

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

// v holds the stage-0 inputs (element stage_in_index<N, R0, E>(p, b, r) at v[b*R0 + r]).
// Runs every stage; outputs go through store(n, value).  When SYNC_BEFORE_STORE is
// set a barrier separates the last LDS read from the stores (for stores into LDS).
template <int N, bool INV, bool SYNC_BEFORE_STORE, class Idx, class Store>
__device__ __forceinline__ void fft_run(float2* v, int p, float2* lds, Idx idx,
                                        const float2* __restrict__ tw, Store store) {
  using S = FftShape<N>;
  constexpr int E = S::E;
  stage_compute<N, S::R0, 1, E, INV>(v, p, tw);
  if constexpr (S::NSTAGE == 1) {
    if constexpr (SYNC_BEFORE_STORE) __syncthreads();
    emit<N, S::R0, 1, E>(v, p, store);
  } else {
    write_lds<N, S::R0, 1, E>(v, p, lds, idx);
    __syncthreads();
    read_lds<N, S::R1, E>(v, p, lds, idx);
    if constexpr (S::NSTAGE == 2) {
      stage_compute<N, S::R1, S::R0, E, INV>(v, p, tw);
      if constexpr (SYNC_BEFORE_STORE) __syncthreads();
      emit<N, S::R1, S::R0, E>(v, p, store);
    } else {
      __syncthreads();
      stage_compute<N, S::R1, S::R0, E, INV>(v, p, tw);
      write_lds<N, S::R1, S::R0, E>(v, p, lds, idx);
      __syncthreads();
      read_lds<N, S::R2, E>(v, p, lds, idx);
      stage_compute<N, S::R2, S::R0 * S::R1, E, INV>(v, p, tw);
      if constexpr (SYNC_BEFORE_STORE) __syncthreads();
      emit<N, S::R2, S::R0 * S::R1, E>(v, p, store);
    }
  }
}

// ---------------------------------------------------------------------------
// strided-axis lines
// ---------------------------------------------------------------------------

template <int N>
struct StridedCfg {
  static constexpr int P = FftShape<N>::P;
  static constexpr int T0 = 256 / P < 4 ? 4 : (256 / P > 64 ? 64 : 256 / P);
  static constexpr int T = T0;
  static constexpr int THREADS = T * P;
  static constexpr int LDS_W = T + 1;
  static constexpr int LDS_ELEMS = FftShape<N>::NSTAGE > 1 ? N * LDS_W : 1;
};

template <int N, bool INV, int LD, int ST>
__global__ __launch_bounds__(StridedCfg<N>::THREADS) void strided_fft(StridedArgs a,
                                                                       const float2* __restrict__ tw) {
  using S = FftShape<N>;
  using C = StridedCfg<N>;
  constexpr int E = S::E, T = C::T;
  __shared__ float2 lds[C::LDS_ELEMS];
  const int tid = threadIdx.x;
  const int c = tid % T;
  const int p = tid / T;
  const long long plane = blockIdx.y;
  const int col = blockIdx.x * T + c;
  const bool colok = col < a.ncols;

  float2 v[E];
  static_for<E / S::R0>([&](auto b_) {
    static_for<S::R0>([&](auto r_) {
      constexpr int b = decltype(b_)::value, r = decltype(r_)::value;
      const int n = stage_in_index<N, S::R0, E>(p, b, r);
      float2 x = make_float2(0.f, 0.f);
      if (colok && n < a.n_in) {
        const long long i = plane * a.in_plane + (long long)n * a.in_line + col;
        if constexpr (LD == LD_TAU_SCALED) {
          x.x = static_cast<const float*>(a.in)[i] * (float(col) * a.tscale);
        } else {
          x = static_cast<const float2*>(a.in)[i];
        }
      }
      v[b * S::R0 + r] = x;
    });
  });

  auto idx = [&](int n) { return n * C::LDS_W + c; };
  auto store = [&](int n, float2 val) {
    if constexpr (ST == ST_C64) {
      if (colok && n < a.n_out)
        static_cast<float2*>(a.out)[plane * a.out_plane + (long long)n * a.out_line + col] = val;
    } else {  // |v|^2 (times a.oscale) plus a max over this tile's columns into img
      float m = colok ? (val.x * val.x + val.y * val.y) * a.oscale : 0.f;
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
  fft_run<N, INV, false>(v, p, lds, idx, tw, store);
}

// ---------------------------------------------------------------------------
// contiguous lines
// ---------------------------------------------------------------------------

template <int N>
struct ContigCfg {
  static constexpr int P = FftShape<N>::P;
  static constexpr int L = 256 / P < 1 ? 1 : 256 / P;
  static constexpr int THREADS = L * P;
  static constexpr int LSTRIDE = N + (N >= 32 ? N / 32 : 1);
  static constexpr int LDS_ELEMS = L * LSTRIDE;
};

__device__ __forceinline__ int swz(int n) { return n + (n >> 5); }

template <int N, bool INV, int LD, int ST>
__global__ __launch_bounds__(ContigCfg<N>::THREADS) void contig_fft(ContigArgs a,
                                                                     const float2* __restrict__ tw) {
  using S = FftShape<N>;
  using C = ContigCfg<N>;
  constexpr int E = S::E, P = C::P;
  constexpr bool NEED_LDS = (S::NSTAGE > 1) || (ST == CS_BINS);
  __shared__ float2 lds[NEED_LDS ? C::LDS_ELEMS : 1];
  const int tid = threadIdx.x;
  const int l = tid / P;
  const int p = tid % P;
  const long long line = (long long)blockIdx.x * C::L + l;
  const bool lineok = line < a.nlines;

  float2 v[E];
  static_for<E / S::R0>([&](auto b_) {
    static_for<S::R0>([&](auto r_) {
      constexpr int b = decltype(b_)::value, r = decltype(r_)::value;
      const int n = stage_in_index<N, S::R0, E>(p, b, r);
      float2 x = make_float2(0.f, 0.f);
      if (lineok && n < a.n_in) {
        const long long i = line * a.in_line + n;
        if constexpr (LD == CL_REAL) {
          x.x = static_cast<const float*>(a.in)[i];
        } else {
          x = static_cast<const float2*>(a.in)[i];
        }
      }
      v[b * S::R0 + r] = x;
    });
  });

  float2* my = lds + (NEED_LDS ? l * C::LSTRIDE : 0);
  auto idx = [&](int n) { return swz(n); };
  if constexpr (ST == CS_BINS) {
    // natural-order spectrum into LDS, then gather the requested bins
    auto store = [&](int n, float2 val) { my[swz(n)] = val; };
    fft_run<N, INV, true>(v, p, my, idx, tw, store);
    __syncthreads();
    const long long line0 = (long long)blockIdx.x * C::L;
    for (int k = tid; k < C::L * a.nbins; k += C::THREADS) {
      const int ll = k % C::L;
      const int f = k / C::L;
      const long long ln = line0 + ll;
      if (ln < a.nlines) {
        const int bin = a.bins[f];
        // pixel ln = y * row_in + x  ->  out[f][y][x] with row stride row_out
        const long long y = ln / a.row_in, x = ln % a.row_in;
        static_cast<float2*>(a.out)[(long long)f * a.out_fstride + y * a.row_out + x] =
            lds[ll * C::LSTRIDE + swz(bin)];
      }
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
    fft_run<N, INV, false>(v, p, my, idx, tw, store);
  }
}

// ---------------------------------------------------------------------------
// f-k column pass: t-FFT -> Stolt remap (+ Jacobian, normalisation) -> z-IFFT
// ---------------------------------------------------------------------------

template <int N>
__global__ __launch_bounds__(ContigCfg<N>::THREADS) void fk_column(FkColumnArgs a,
                                                                    const float2* __restrict__ tw) {
  using S = FftShape<N>;
  using C = ContigCfg<N>;
  constexpr int E = S::E, P = C::P, HALF = N / 2;
  __shared__ float2 lds[C::LDS_ELEMS];
  const int tid = threadIdx.x;
  const int l = tid / P;
  const int p = tid % P;
  const long long line = (long long)blockIdx.x * C::L + l;
  const bool lineok = line < a.ncols;
  float2* W = a.W;

  float2 v[E];
  static_for<E / S::R0>([&](auto b_) {
    static_for<S::R0>([&](auto r_) {
      constexpr int b = decltype(b_)::value, r = decltype(r_)::value;
      const int n = stage_in_index<N, S::R0, E>(p, b, r);
      float2 x = make_float2(0.f, 0.f);
      if (lineok && n < a.nt) x = W[line * a.nt + n];
      v[b * S::R0 + r] = x;
    });
  });
  float2* my = lds + l * C::LSTRIDE;
  auto idx = [&](int n) { return swz(n); };
  // forward transform along t; the spectrum stays in LDS in natural order
  fft_run<N, false, true>(v, p, my, idx, tw, [&](int n, float2 val) { my[swz(n)] = val; });
  __syncthreads();

  // Stolt: out(kz) = [0 < kz < N/2] (kz / q) lerp(S, q), q = sqrt(A + kz^2) in bins
  const long long ky = line / a.Mx, kx = line % a.Mx;
  const int kxs = kx < a.Mx / 2 ? int(kx) : int(kx) - a.Mx;
  const int kys = ky < a.My / 2 ? int(ky) : int(ky) - a.My;
  const double ax = a.sxk * kxs, ay = a.syk * kys;
  const double A = ax * ax + ay * ay;
  static_for<E / S::R0>([&](auto b_) {
    static_for<S::R0>([&](auto r_) {
      constexpr int b = decltype(b_)::value, r = decltype(r_)::value;
      const int kz = stage_in_index<N, S::R0, E>(p, b, r);
      float2 x = make_float2(0.f, 0.f);
      if (kz > 0 && kz < HALF) {
        const double q = sqrt(A + double(kz) * double(kz));
        if (q <= double(HALF - 1)) {
          const double fl = floor(q);
          const int i0 = int(fl);
          const int i1 = i0 + 1 < HALF ? i0 + 1 : HALF - 1;
          const float fr = float(q - fl);
          const float jac = float(double(kz) / q) * a.norm;
          const float2 s0 = my[swz(i0)], s1 = my[swz(i1)];
          x.x = fmaf(fr, s1.x - s0.x, s0.x) * jac;
          x.y = fmaf(fr, s1.y - s0.y, s0.y) * jac;
        }
      }
      v[b * S::R0 + r] = x;
    });
  });
  __syncthreads();
  // inverse transform along z; keep z < nt, written back in place
  fft_run<N, true, false>(v, p, my, idx, tw, [&](int n, float2 val) {
    if (lineok && n < a.nt) W[line * a.nt + n] = val;
  });
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <int N, bool INV, int LD, int ST>
static hipError_t launch_strided_n(const StridedArgs& a, int nplanes, const float2* tw,
                                   hipStream_t s) {
  using C = StridedCfg<N>;
  dim3 grid((a.ncols + C::T - 1) / C::T, nplanes);
  hipLaunchKernelGGL((strided_fft<N, INV, LD, ST>), grid, dim3(C::THREADS), 0, s, a, tw);
  return hipGetLastError();
}

template <bool INV, int LD, int ST>
static hipError_t launch_strided_inv(int n, const StridedArgs& a, int nplanes, const float2* tw,
                                     hipStream_t s) {
  switch (n) {
    case 8: return launch_strided_n<8, INV, LD, ST>(a, nplanes, tw, s);
    case 16: return launch_strided_n<16, INV, LD, ST>(a, nplanes, tw, s);
    case 32: return launch_strided_n<32, INV, LD, ST>(a, nplanes, tw, s);
    case 64: return launch_strided_n<64, INV, LD, ST>(a, nplanes, tw, s);
    case 128: return launch_strided_n<128, INV, LD, ST>(a, nplanes, tw, s);
    case 256: return launch_strided_n<256, INV, LD, ST>(a, nplanes, tw, s);
    case 512: return launch_strided_n<512, INV, LD, ST>(a, nplanes, tw, s);
    case 1024: return launch_strided_n<1024, INV, LD, ST>(a, nplanes, tw, s);
    case 2048: return launch_strided_n<2048, INV, LD, ST>(a, nplanes, tw, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_strided(int n, bool inverse, int ld, int st, const StridedArgs& a, int nplanes,
                          const float2* tw, hipStream_t s) {
  if (!inverse && ld == LD_TAU_SCALED && st == ST_C64)
    return launch_strided_inv<false, LD_TAU_SCALED, ST_C64>(n, a, nplanes, tw, s);
  if (!inverse && ld == LD_C64 && st == ST_C64)
    return launch_strided_inv<false, LD_C64, ST_C64>(n, a, nplanes, tw, s);
  if (inverse && ld == LD_C64 && st == ST_C64)
    return launch_strided_inv<true, LD_C64, ST_C64>(n, a, nplanes, tw, s);
  if (inverse && ld == LD_C64 && st == ST_ABS2_IMG)
    return launch_strided_inv<true, LD_C64, ST_ABS2_IMG>(n, a, nplanes, tw, s);
  return hipErrorInvalidValue;
}

template <int N, bool INV, int LD, int ST>
static hipError_t launch_contig_n(const ContigArgs& a, const float2* tw, hipStream_t s) {
  using C = ContigCfg<N>;
  dim3 grid((unsigned)((a.nlines + C::L - 1) / C::L));
  hipLaunchKernelGGL((contig_fft<N, INV, LD, ST>), grid, dim3(C::THREADS), 0, s, a, tw);
  return hipGetLastError();
}

template <bool INV, int LD, int ST>
static hipError_t launch_contig_inv(int n, const ContigArgs& a, const float2* tw, hipStream_t s) {
  switch (n) {
    case 8: return launch_contig_n<8, INV, LD, ST>(a, tw, s);
    case 16: return launch_contig_n<16, INV, LD, ST>(a, tw, s);
    case 32: return launch_contig_n<32, INV, LD, ST>(a, tw, s);
    case 64: return launch_contig_n<64, INV, LD, ST>(a, tw, s);
    case 128: return launch_contig_n<128, INV, LD, ST>(a, tw, s);
    case 256: return launch_contig_n<256, INV, LD, ST>(a, tw, s);
    case 512: return launch_contig_n<512, INV, LD, ST>(a, tw, s);
    case 1024: return launch_contig_n<1024, INV, LD, ST>(a, tw, s);
    case 2048: return launch_contig_n<2048, INV, LD, ST>(a, tw, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_contig(int n, bool inverse, int ld, int st, const ContigArgs& a, const float2* tw,
                         hipStream_t s) {
  if (!inverse && ld == CL_REAL && st == CS_BINS)
    return launch_contig_inv<false, CL_REAL, CS_BINS>(n, a, tw, s);
  if (!inverse && ld == CL_C64 && st == CS_C64)
    return launch_contig_inv<false, CL_C64, CS_C64>(n, a, tw, s);
  if (inverse && ld == CL_C64 && st == CS_ABS_IMG)
    return launch_contig_inv<true, CL_C64, CS_ABS_IMG>(n, a, tw, s);
  return hipErrorInvalidValue;
}

template <int N>
static hipError_t launch_fk_column_n(const FkColumnArgs& a, const float2* tw, hipStream_t s) {
  using C = ContigCfg<N>;
  dim3 grid((unsigned)((a.ncols + C::L - 1) / C::L));
  hipLaunchKernelGGL((fk_column<N>), grid, dim3(C::THREADS), 0, s, a, tw);
  return hipGetLastError();
}

hipError_t launch_fk_column(int n, const FkColumnArgs& a, const float2* tw, hipStream_t s) {
  switch (n) {
    case 8: return launch_fk_column_n<8>(a, tw, s);
    case 16: return launch_fk_column_n<16>(a, tw, s);
    case 32: return launch_fk_column_n<32>(a, tw, s);
    case 64: return launch_fk_column_n<64>(a, tw, s);
    case 128: return launch_fk_column_n<128>(a, tw, s);
    case 256: return launch_fk_column_n<256>(a, tw, s);
    case 512: return launch_fk_column_n<512>(a, tw, s);
    case 1024: return launch_fk_column_n<1024>(a, tw, s);
    case 2048: return launch_fk_column_n<2048>(a, tw, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace nlos
