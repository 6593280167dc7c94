// f-k passes that use the Hermitian symmetry of the real transient (gfx950).
//
// The scaled, padded transient g is real, so its 3D spectrum satisfies
// S(-kx, -ky, -w) = conj(S(kx, ky, w)).  Only the kx in [0, Mx/2] half is formed:
//   fk_xr2c        pass 1: x-FFT of tau * t/(nt-1), two real t-columns packed in one
//                  complex line (z = a + i b, A[k] = (Z[k] + conj Z[-k]) / 2,
//                  B[k] = (Z[k] - conj Z[-k]) / 2i), writes kx in [0, Mx/2];
//   fk_column_pair pass 3: one forward t-FFT of column (kx, ky) of the half spectrum
//                  serves the Stolt remap of output column (kx, ky) (w >= 0 half of
//                  the column) and of its mirror (-kx, -ky) (conjugated w <= 0 half);
//                  both share the Stolt coordinates, since sqrt(sx^2 X^2 + sy^2 Y^2 + Z^2)
//                  depends on X^2 and Y^2 only.  The remapped columns (kz in [0, Mt/2),
//                  the only non-zero half) are written out; the inverse transform along z
//                  runs last, after the y and x inverse passes have cropped the volume to
//                  ny x nx columns (the inverse 3D DFT is separable, so its axis order is
//                  free), which needs a quarter of the z transforms.
#include "fft_block.hpp"
#include "fft_general.hpp"
#include "fk_pairs.hpp"
#include "nlos_internal.hpp"
#include "prec.hpp"

namespace nlos {

// ---------------------------------------------------------------------------
// pass 1: real x-FFT with time scaling and zero padding
// ---------------------------------------------------------------------------

template <int N, int E, int T, int SP = SP_F32>
__global__ __launch_bounds__((StridedCfg<N, E, T>::THREADS)) void fk_xr2c(FkXArgs a,
                                                                          const float2* __restrict__ tw) {
  using C = StridedCfg<N, E, T>;
  using S = typename C::S;
  constexpr int P = S::P;
  __shared__ float2 lds[N * C::LDS_W];
  const int tid = threadIdx.x;
  const int c = tid % T;
  const int p = tid / T;
  const long long y = blockIdx.y;
  const int cc = blockIdx.x * T + c;        // complex line = real t-columns 2cc, 2cc+1
  const bool colok = 2 * cc < a.nt;
  const float s0 = a.unscaled ? 1.f : float(2 * cc) * a.tscale;
  const float s1 = a.unscaled ? 1.f : float(2 * cc + 1) * a.tscale;

  // all loads first (branch-free: the zero padding is the static upper half, or absent),
  // the t scaling after, so that the thread's loads are in flight together
  float2 v[S::E];
  const float2* row = reinterpret_cast<const float2*>(a.tau + y * a.nx * a.nt) + (colok ? cc : 0);
  const long long pitch = a.nt / 2;  // float2 elements between x samples
  load_first_stage<S>(v, p, a.nx, colok, make_float2(0.f, 0.f), [&](int n) { return row[(long long)n * pitch]; });
#pragma unroll
  for (int j = 0; j < S::E; ++j) v[j] = make_float2(v[j].x * s0, v[j].y * s1);
  auto idx = [&](int n) { return n * C::LDS_W + c; };
  fft_run<S, false, true>(v, p, lds, idx, tw, [&](int n, float2 val) { lds[idx(n)] = val; });
  __syncthreads();
  if constexpr (SP != SP_F32) {
    if (!colok) return;
    using ST_ = Stor<SP>;
    typename ST_::T* out = static_cast<typename ST_::T*>(a.out) + y * a.out_plane + 2 * cc;
    const float h = SP == SP_F16 ? ldexpf(0.5f, *a.e_out) : 0.5f;
    for (int k = p; k <= N / 2; k += P) {
      const float2 zk = lds[idx(k)];
      const float2 zm = lds[idx((N - k) & (N - 1))];
      ST_::st2(out, (long long)k * a.nt, make_float2(h * (zk.x + zm.x), h * (zk.y - zm.y)),
               make_float2(h * (zk.y + zm.y), h * (zm.x - zk.x)));
    }
    return;
  }
  if (!colok) return;
  float4* out = reinterpret_cast<float4*>(static_cast<float2*>(a.out) + y * a.out_plane + 2 * cc);
  for (int k = p; k <= N / 2; k += P) {
    const float2 zk = lds[idx(k)];
    const float2 zm = lds[idx((N - k) & (N - 1))];
    // A = (Z[k] + conj Z[-k]) / 2, B = (Z[k] - conj Z[-k]) / (2i)
    const float4 ab = make_float4(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y),
                                  0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x));
    st_stream(out + (long long)k * (a.nt / 2), ab);
  }
}

// ---------------------------------------------------------------------------
// pass 3: t-FFT -> Stolt remap for a column and its mirror -> two z-IFFTs
// ---------------------------------------------------------------------------

// Stolt sample kz (0 <= kz < Mt) of output column (kx, ky) and of its mirror (-kx, -ky)
// from the forward t-spectrum of column (kx, ky): q = sqrt(A + kz^2) in t-bin units
// (A = (sxk kx)^2 + (syk ky)^2, signed kx, ky), from a float square root refined by one
// FP64 Newton step; linear interpolation between bins floor(q) and floor(q) + 1 (the
// last bin at the top edge itself, zero beyond it), times the Jacobian kz / q and norm.
// The column reads bins +i (at(i)), its mirror the conjugates of bins -i (mir(i)); zero
// unless 0 < kz < Mt/2.
template <class At, class Mir>
__device__ __forceinline__ void stolt_pair(int kz, int half, double A, float norm, At at, Mir mir, float2& xa,
                                           float2& xb) {
  xa = make_float2(0.f, 0.f);
  xb = make_float2(0.f, 0.f);
  if (kz > 0 && kz < half) {
    const double q2 = A + double(kz * kz);
    const float qf = __builtin_amdgcn_sqrtf((float)q2);
    const float rq = __builtin_amdgcn_rcpf(qf);
    const double q0 = (double)qf;
    const double q = fma((double)(0.5f * rq), fma(-q0, q0, q2), q0);
    if (q <= double(half - 1)) {
      const double fl = floor(q);
      const int i0 = int(fl);
      const int i1 = i0 + 1 < half ? i0 + 1 : half - 1;
      const float fr = float(q - fl);
      const float jac = float(kz) * rq * norm;
      const float2 s0 = at(i0), s1 = at(i1);
      xa.x = fmaf(fr, s1.x - s0.x, s0.x) * jac;
      xa.y = fmaf(fr, s1.y - s0.y, s0.y) * jac;
      const float2 m0 = mir(i0), m1 = mir(i1);
      xb.x = fmaf(fr, m1.x - m0.x, m0.x) * jac;
      xb.y = -fmaf(fr, m1.y - m0.y, m0.y) * jac;
    }
  }
}

// The same remap from a natural-order spectrum sp[0..n] whose sp[n] repeats bin 0, so that
// both taps of the column (i0, i0 + 1) and of its mirror (n - 1 - i0, n - i0) are plain
// adjacent reads: at q = half - 1 exactly the weight of the second tap is zero.
__device__ __forceinline__ void stolt_pair_nat(int kz, int half, int n, double A, float norm, const float2* sp,
                                               float2& xa, float2& xb) {
  xa = make_float2(0.f, 0.f);
  xb = make_float2(0.f, 0.f);
  if (kz > 0 && kz < half) {
    const double q2 = A + double(kz * kz);
    const float qf = __builtin_amdgcn_sqrtf((float)q2);
    const float rq = __builtin_amdgcn_rcpf(qf);
    const double q0 = (double)qf;
    const double q = fma((double)(0.5f * rq), fma(-q0, q0, q2), q0);
    if (q <= double(half - 1)) {
      const double fl = floor(q);
      const int i0 = int(fl);
      const float fr = float(q - fl);
      const float jac = float(kz) * rq * norm;
      const float2 s0 = sp[i0], s1 = sp[i0 + 1];
      const float2 m1 = sp[n - 1 - i0], m0 = sp[n - i0];
      xa.x = fmaf(fr, s1.x - s0.x, s0.x) * jac;
      xa.y = fmaf(fr, s1.y - s0.y, s0.y) * jac;
      xb.x = fmaf(fr, m1.x - m0.x, m0.x) * jac;
      xb.y = -fmaf(fr, m1.y - m0.y, m0.y) * jac;
    }
  }
}

// PADDED: the column's upper half is the zero padding (nt = N/2), known at compile time,
// so the zero inputs fold out of the first radix stage.
template <int N, int E_ = default_e(N), int SP = SP_F32, bool TSCALE = false, bool PADDED = false>
__global__ __launch_bounds__((ContigCfg<N, E_>::THREADS)) void fk_column_pair(FkPairArgs a,
                                                                             const float2* __restrict__ tw) {
  using C = ContigCfg<N, E_>;
  using S = typename C::S;
  using ST_ = Stor<SP>;
  constexpr int E = S::E, P = C::P, HALF = N / 2;
  __shared__ float2 lds[C::LDS_ELEMS];
  const int tid = threadIdx.x;
  const int l = tid / P;
  const int p = tid % P;
  float2* my = lds + l * C::LSTRIDE;
  auto idx = [&](int n) { return swz(n); };
  const long long ngroups = (a.nwork + C::L - 1) / C::L;

  for (long long g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const long long w = g * C::L + l;
    const bool ok = w < a.nwork;
    const PairItem it = pair_item(ok ? w : 0, a.Mx, a.My);
    const long long src = (long long)it.ky * a.in_row + (long long)it.kx * a.nt;
    float2 v[E];
    {
      // raw loads first, conversion after, so that all loads of the column are in
      // flight together
      typename ST_::R raw[E];
      const typename ST_::T* in = static_cast<const typename ST_::T*>(a.in) + src;
      if constexpr (PADDED) {
        static_for<E / 2>([&](auto r_) {
          constexpr int r = decltype(r_)::value;
          raw[r] = ok ? ST_::raw(in, p + r * P) : ST_::zero();
        });
        static_for<E / 2>([&](auto r_) { raw[E / 2 + decltype(r_)::value] = ST_::zero(); });
      } else if constexpr (SP == SP_F32) {
        // per-element guards measured faster than the branch-free form for 8-byte loads
        static_for<E>([&](auto r_) {
          constexpr int r = decltype(r_)::value;
          const int n = p + r * P;
          raw[r] = (ok && n < a.nt) ? ld_stream(in + n) : ST_::zero();
        });
      } else {
        load_first_stage<S>(raw, p, a.nt, ok, ST_::zero(), [&](int n) { return ST_::raw(in, n); });
      }
      const int e = SP == SP_F16 ? -*a.e_in : 0;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        v[j] = ST_::cvt(raw[j]);
        if constexpr (SP == SP_F16) v[j] = ldexp2(v[j], e);
      }
      if constexpr (TSCALE) {  // separate instantiation: keeps the plain pass's registers
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = cscale(v[j], float(p + j * P) * a.tscale_in);
      }
    }
    __syncthreads();  // the previous item's last LDS reads are done
    // the spectrum in natural order (the line stride leaves room for the repeated bin 0)
    static_assert(C::LSTRIDE > N, "room for bin N");
    fft_run<S, false, true>(v, p, my, idx, tw, [&](int n, float2 val) {
      my[n] = val;
      if (n == 0) my[N] = val;
    });
    __syncthreads();

    // Stolt (shared by the pair): q = sqrt(A + kz^2) in t-bin units; lerp weight,
    // Jacobian kz/q, 1/(Mx My Mt).
    const int kxs = it.kx < a.Mx / 2 ? it.kx : it.kx - a.Mx;
    const int kys = it.ky < a.My / 2 ? it.ky : it.ky - a.My;
    const double ax = a.sxk * kxs, ay = a.syk * kys;
    const double A = ax * ax + ay * ay;
    // the remapped column and its mirror go straight to W3 (kz < nt; kz >= Mt/2 and
    // kz = 0 are zero)
    const long long dst = (long long)it.ky * a.out_row + (long long)it.kx * a.nt;
    const long long dst2 = (long long)it.ky2 * a.out_row + (long long)it.kx2 * a.nt;
    const bool ok2 = ok && it.has_mirror;
    const int ex = SP == SP_F16 ? *a.e_out : 0;
    typename ST_::T* outp = static_cast<typename ST_::T*>(a.out);
    // a rolled loop keeps the register footprint (and so the occupancy) of the remap low
#pragma unroll 2
    for (int kz = p; kz < a.nt; kz += P) {
      float2 xa, xb;
      stolt_pair_nat(kz, HALF, N, A, a.norm, my, xa, xb);
      if constexpr (SP == SP_F16) {
        xa = ldexp2(xa, ex);
        xb = ldexp2(xb, ex);
      }
      if (ok) ST_::st(outp, dst + kz, xa);
      if (ok2) ST_::st(outp, dst2 + kz, xb);
    }
  }
}

// The FP32 column pass of a padded volume (nt = N/2) for three-stage plans, as
// fk_column_pair<N, E, SP_F32> computes it, with resident blocks that load the next
// group's columns while they transform the current one; the inter-stage twiddles sit in
// LDS tables.  An item past the end (in the last group) stands in for the group's first
// item, and a column without a mirror stores its own remap twice, so every thread issues
// the same stores and the wait for the next group's loads leaves this group's stores in
// flight.
template <int N, int E_>
__global__ __launch_bounds__((ContigCfg<N, E_>::THREADS)) void fk_column_pair_stream(FkPairArgs a,
                                                                                    const float2* __restrict__ tw) {
  using C = ContigCfg<N, E_>;
  using S = typename C::S;
  constexpr int E = S::E, P = C::P, L = C::L, HALF = N / 2, R0 = S::R0, R1 = S::R1, R2 = S::R2;
  static_assert(S::NSTAGE == 3 && R0 == E && HALF % P == 0, "three-stage plans");
  __shared__ float2 lds[C::LDS_ELEMS];
  __shared__ float2 wt[R1 * R0];               // W_{R0 R1}^(j r)
  __shared__ float2 wt2[(R2 - 1) * R0 * R1];   // W_N^(j r), r >= 1
  const int tid = threadIdx.x;
  const int l = tid / P;
  const int p = tid % P;
  for (int k = tid; k < R1 * R0; k += C::THREADS) wt[k] = tw[(k % R0) * (k / R0) * (kTwiddleN / (R0 * R1))];
  for (int k = tid; k < (R2 - 1) * R0 * R1; k += C::THREADS)
    wt2[k] = tw[(k % (R0 * R1)) * (1 + k / (R0 * R1)) * (kTwiddleN / N)];
  float2* my = lds + l * C::LSTRIDE;
  auto idx = [&](int n) { return swz(n); };
  const long long ngroups = (a.nwork + L - 1) / L;
  const float2* in = static_cast<const float2*>(a.in);
  float2* outp = static_cast<float2*>(a.out);

  PairItem nit;
  float2 raw[E / 2];  // samples p + r P (r < E/2) of the column: its stored half
  auto fetch = [&](long long g) {
    const long long w = g * L + l;
    nit = pair_item(w < a.nwork ? w : g * L, a.Mx, a.My);
    const float2* col = in + (long long)nit.ky * a.in_row + (long long)nit.kx * a.nt;
    static_for<E / 2>([&](auto r_) {
      constexpr int r = decltype(r_)::value;
      raw[r] = ld_stream(col + p + r * P);
    });
  };
  if ((long long)blockIdx.x < ngroups) fetch(blockIdx.x);
  __builtin_amdgcn_s_waitcnt(0);  // tables and the first group before the loop
  for (long long g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const PairItem it = nit;
    float2 v[E];
#pragma unroll
    for (int j = 0; j < E / 2; ++j) v[j] = raw[j];
#pragma unroll
    for (int j = E / 2; j < E; ++j) v[j] = make_float2(0.f, 0.f);
    if (g + gridDim.x < ngroups) fetch(g + gridDim.x);
    __syncthreads();  // the previous item's LDS reads (and, first, the tables) are done
    // the spectrum in natural order (the line stride leaves room for the repeated bin 0)
    static_assert(C::LSTRIDE > N, "room for bin N");
    fft_run<S, false, true>(v, p, my, idx, TwLds<S>{wt, wt2}, [&](int n, float2 val) {
      my[n] = val;
      if (n == 0) my[N] = val;
    });
    __syncthreads();
    const int kxs = it.kx < a.Mx / 2 ? it.kx : it.kx - a.Mx;
    const int kys = it.ky < a.My / 2 ? it.ky : it.ky - a.My;
    const double ax = a.sxk * kxs, ay = a.syk * kys;
    const double A = ax * ax + ay * ay;
    const bool mir = it.has_mirror;
    float2* o1 = outp + (long long)it.ky * a.out_row + (long long)it.kx * a.nt;
    float2* o2 = mir ? outp + (long long)it.ky2 * a.out_row + (long long)it.kx2 * a.nt : o1;
#pragma unroll
    for (int i = 0; i < HALF / P; ++i) {
      const int kz = p + i * P;
      float2 xa, xb;
      stolt_pair_nat(kz, HALF, N, A, a.norm, my, xa, xb);
      o1[kz] = xa;
      o2[kz] = mir ? xb : xa;
    }
  }
}

// ---------------------------------------------------------------------------
// mixture of experts (Section 4.4): RSD phasors from the shared spatial spectrum
// ---------------------------------------------------------------------------
//
// The spatial DFT and the temporal DFT commute, so the RSD branch can take its phasors
// P^[ky][kx][f] from the spatial spectrum T[ky][kx][t] of the transient that the f-k
// branch also reads: one nt-point DFT per column at the selected bins.  The transient is
// real, so T(-kx, -ky, t) = conj T(kx, ky, t) and the mirror column's phasors are
// conj X[nt - k_f] of the same transform; only the kx <= Mx/2 half is stored.

template <int N>
__global__ __launch_bounds__((ContigCfg<N>::THREADS)) void moe_phasor_pair(MoePhasorArgs a,
                                                                          const float2* __restrict__ tw) {
  using C = ContigCfg<N>;
  using S = typename C::S;
  constexpr int E = S::E, P = C::P;
  __shared__ float2 lds[C::LDS_ELEMS];
  const int tid = threadIdx.x;
  const int l = tid / P;
  const int p = tid % P;
  float2* my = lds + l * C::LSTRIDE;
  auto idx = [&](int n) { return swz(n); };
  const long long w = (long long)blockIdx.x * C::L + l;
  const bool ok = w < a.nwork;
  const PairItem it = pair_item(ok ? w : 0, a.Mx, a.My);
  const float2* src = a.in + (long long)it.ky * a.in_row + (long long)it.kx * a.nt;
  float2 v[E];
  static_for<E>([&](auto r_) {
    constexpr int r = decltype(r_)::value;
    v[r] = src[p + r * P];  // the column has exactly N = nt samples
  });
  fft_run<S, false, true>(v, p, my, idx, tw, [&](int n, float2 val) { my[swz(n)] = val; });
  __syncthreads();
  if (!ok) return;
  float2* o1 = a.out + ((long long)it.ky * a.Mx + it.kx) * a.nbins;
  float2* o2 = a.out + ((long long)it.ky2 * a.Mx + it.kx2) * a.nbins;
  for (int f = p; f < a.nbins; f += P) {
    const int k = a.bins[f];
    o1[f] = my[swz(k)];
    if (it.has_mirror) {
      const float2 m = my[swz((N - k) & (N - 1))];
      o2[f] = make_float2(m.x, -m.y);
    }
  }
}

hipError_t launch_moe_phasor_pair(const MoePhasorArgs& a, const float2* tw, hipStream_t s) {
  auto go = [&](auto n_) -> hipError_t {
    constexpr int N = decltype(n_)::value;
    using C = ContigCfg<N>;
    const long long blocks = (a.nwork + C::L - 1) / C::L;
    hipLaunchKernelGGL((moe_phasor_pair<N>), dim3((unsigned)blocks), dim3(C::THREADS), 0, s, a, tw);
    return hipGetLastError();
  };
  switch (a.nt) {
    case 8: return go(std::integral_constant<int, 8>{});
    case 16: return go(std::integral_constant<int, 16>{});
    case 32: return go(std::integral_constant<int, 32>{});
    case 64: return go(std::integral_constant<int, 64>{});
    case 128: return go(std::integral_constant<int, 128>{});
    case 256: return go(std::integral_constant<int, 256>{});
    case 512: return go(std::integral_constant<int, 512>{});
    case 1024: return go(std::integral_constant<int, 1024>{});
    case 2048: return go(std::integral_constant<int, 2048>{});
    default: return hipErrorInvalidValue;
  }
}

// Eq. 10 on the two branch images in three grid passes: the two maxima, the mixture and
// its maximum, the normalisation.  Maxima of non-negative floats are taken with integer
// atomic max on their bit patterns, which is order independent, so the result is
// deterministic.  mx[0..2] (max F, max R, max m) must be zero on entry.
__global__ __launch_bounds__(256) void moe_maxima(const float* __restrict__ fk_img, const float* __restrict__ rsd_img,
                                                  int n, unsigned int* __restrict__ mx) {
  float mf = 0.f, mr = 0.f;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    mf = fmaxf(mf, fk_img[i]);
    mr = fmaxf(mr, rsd_img[i]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mf = fmaxf(mf, __shfl_xor(mf, off, 64));
    mr = fmaxf(mr, __shfl_xor(mr, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(mx, __float_as_uint(mf));
    atomicMax(mx + 1, __float_as_uint(mr));
  }
}

__global__ __launch_bounds__(256) void moe_product(const float* __restrict__ fk_img, const float* __restrict__ rsd_img,
                                                   float* __restrict__ img, int n, float beta, float eps,
                                                   unsigned int* __restrict__ mx) {
  const float mf = __uint_as_float(mx[0]), mr = __uint_as_float(mx[1]);
  const float sf = mf > 0.f ? 1.f / mf : 0.f, sr = mr > 0.f ? 1.f / mr : 0.f;
  float mm = 0.f;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const float m = fk_img[i] * sf * powf(rsd_img[i] * sr + eps, beta);
    img[i] = m;
    mm = fmaxf(mm, m);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mm = fmaxf(mm, __shfl_xor(mm, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(mx + 2, __float_as_uint(mm));
}

__global__ __launch_bounds__(256) void moe_normalise(float* __restrict__ img, int n, const unsigned int* __restrict__ mx) {
  const float mm = __uint_as_float(mx[2]);
  const float sm = mm > 0.f ? 1.f / mm : 0.f;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) img[i] *= sm;
}

hipError_t launch_moe_mix(const float* fk_img, const float* rsd_img, float* img, int n, float beta, float eps,
                          unsigned int* mx, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipError_t e = launch_fill_u32(mx, 3, 0u, s);
  if (e != hipSuccess) return e;
  const int blocks = std::min(256, (n + 255) / 256);
  hipLaunchKernelGGL(moe_maxima, dim3(blocks), dim3(256), 0, s, fk_img, rsd_img, n, mx);
  hipLaunchKernelGGL(moe_product, dim3(blocks), dim3(256), 0, s, fk_img, rsd_img, img, n, beta, eps, mx);
  hipLaunchKernelGGL(moe_normalise, dim3(blocks), dim3(256), 0, s, img, n, mx);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP16 storage scales (Section 4.2, data quantization: the input is scaled before the
// forward transform and the spectrum before the inverse one)
// ---------------------------------------------------------------------------
//
// Every forward intermediate is a partial DFT of g = tau t/(nt-1), so its magnitude is
// at most B = sum |g|; the Stolt output is at most B/(Mx My Mt) (a lerp of spectrum
// samples times Z/Z' <= 1 and the normalisation); each unnormalised inverse axis of
// length M multiplies the bound by M.  With B = f 2^k (f in [0.5, 1)), storing the
// forward intermediates times 2^(14-k) keeps them below 2^14 (binary16's largest
// finite value is 65504) and the later ones follow by exact powers of two.  B is summed
// in a fixed order, so the scales, and the result, are deterministic.

__device__ __forceinline__ float block_sum_256(float v, float* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void fk_l1_partial(const float2* __restrict__ tau, long long n2, int nt,
                                                     float tscale, float* __restrict__ partials) {
  __shared__ float red[4];
  float acc = 0.f;
  const long long stride = (long long)gridDim.x * 256;
  auto term = [&](long long i, float2 v) {
    const int t = (int)((2 * i) & (nt - 1));  // nt is an even power of two
    return fabsf(v.x) * float(t) + fabsf(v.y) * float(t + 1);
  };
  long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  // four loads in flight per thread
  for (; i + 3 * stride < n2; i += 4 * stride) {
    const float2 v0 = tau[i], v1 = tau[i + stride], v2 = tau[i + 2 * stride], v3 = tau[i + 3 * stride];
    acc += (term(i, v0) + term(i + stride, v1)) + (term(i + 2 * stride, v2) + term(i + 3 * stride, v3));
  }
  for (; i < n2; i += stride) acc += term(i, tau[i]);
  const float b = block_sum_256(acc * tscale, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

__global__ __launch_bounds__(256) void fk_scale_exponents(const float* __restrict__ partials, int np,
                                                          int* __restrict__ exps, int l_norm, int l_first_inv,
                                                          int l_second_inv) {
  __shared__ float red[4];
  float acc = 0.f;
  for (int j = threadIdx.x; j < np; j += 256) acc += partials[j];
  const float B = block_sum_256(acc, red);
  if (threadIdx.x == 0) {
    int k = 0;
    if (B > 0.f && B <= 3.0e38f) frexpf(B, &k);
    const int ef = (B > 0.f && B <= 3.0e38f) ? 14 - k : 0;
    // the inverse passes run x first (length Mx), then y (length My)
    exps[0] = ef;                        // W1, W2: bound B
    exps[1] = ef + l_norm;               // W3: bound B / (Mx My Mt)
    exps[2] = exps[1] - l_first_inv;     // W4 (after the x-IFFT): bound Mx B / (Mx My Mt)
    exps[3] = exps[2] - l_second_inv;    // W5 (after the y-IFFT): bound Mx My B / (Mx My Mt)
  }
}

hipError_t launch_fk_scales(const float* tau, long long n, int nt, float* partials, int* exps,
                            int l_norm, int l_first_inv, int l_second_inv, hipStream_t s) {
  if (n % 2 != 0 || (nt & (nt - 1)) != 0 || nt < 2) return hipErrorInvalidValue;
  const float tscale = (float)(1.0 / (double)(nt - 1));
  hipLaunchKernelGGL(fk_l1_partial, dim3(kScaleBlocks), dim3(256), 0, s,
                     reinterpret_cast<const float2*>(tau), n / 2, nt, tscale, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fk_scale_exponents, dim3(1), dim3(256), 0, s, partials, kScaleBlocks, exps, l_norm,
                     l_first_inv, l_second_inv);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

// The FP32 x pass as resident blocks that walk (y, tile of T column pairs) items, item i
// then i + gridDim.x, ...: the next item's samples load while the current item is
// transformed, the stage twiddles stay in registers.  IN_HALF: nx = N/2 (the upper half
// is the zero padding), else nx = N.  A column pair past nt/2 (in the last tile) stands in
// for the tile's first pair: it reads it, computes the same values and stores them to the
// same place, so every thread issues the same stores (the wait for the next item's loads
// then leaves the item's stores in flight).  Same results as fk_xr2c<N, E, T, SP_F32>.
template <int N, int E, int T, bool IN_HALF>
__global__ __launch_bounds__((StridedCfg<N, E, T>::THREADS)) void fk_xr2c_stream(FkXArgs a,
                                                                                 const float2* __restrict__ tw,
                                                                                 int ntiles, int nitems) {
  using C = StridedCfg<N, E, T>;
  using S = typename C::S;
  constexpr int P = S::P, E_ = S::E, NR = IN_HALF ? E_ / 2 : E_;
  static_assert(S::R0 == E_, "first radix E");
  __shared__ float2 lds[N * C::LDS_W];
  const int tid = threadIdx.x;
  const int c = tid % T;
  const int p = tid / T;
  TwRegs<S> twr;
  twr.load(p, tw);
  const int ncc = a.nt / 2;            // complex lines (real t-column pairs) per y
  const long long pitch = a.nt / 2;    // float2 elements between x samples
  auto pair = [&](int it, int& y) {
    y = (unsigned)it / (unsigned)ntiles;
    const int cc0 = (it - y * ntiles) * T;
    return cc0 + c < ncc ? cc0 + c : cc0;
  };
  float2 raw[NR];  // x samples p + r P, r < NR
  auto fetch = [&](int it) {
    int y;
    const int cc = pair(it, y);
    const float2* row = reinterpret_cast<const float2*>(a.tau + (long long)y * a.nx * a.nt) + cc;
    static_for<NR>([&](auto r_) {
      constexpr int r = decltype(r_)::value;
      raw[r] = row[(long long)(p + r * P) * pitch];
    });
  };
  auto idx = [&](int n) { return n * C::LDS_W + c; };
  int it = blockIdx.x;
  if (it < nitems) fetch(it);
  __builtin_amdgcn_s_waitcnt(0);  // twiddles and the first item before the loop
  for (; it < nitems; it += gridDim.x) {
    int y;
    const int cc = pair(it, y);
    const float s0 = a.unscaled ? 1.f : float(2 * cc) * a.tscale;
    const float s1 = a.unscaled ? 1.f : float(2 * cc + 1) * a.tscale;
    float2 v[E_];
#pragma unroll
    for (int j = 0; j < NR; ++j) v[j] = make_float2(raw[j].x * s0, raw[j].y * s1);
#pragma unroll
    for (int j = NR; j < E_; ++j) v[j] = make_float2(0.f, 0.f);
    if (it + (int)gridDim.x < nitems) fetch(it + gridDim.x);
    fft_run<S, false, true>(v, p, lds, idx, twr, [&](int n, float2 val) { lds[idx(n)] = val; });
    __syncthreads();
    float4* out = reinterpret_cast<float4*>(static_cast<float2*>(a.out) + (long long)y * a.out_plane + 2 * cc);
    // A = (Z[k] + conj Z[-k]) / 2, B = (Z[k] - conj Z[-k]) / (2i), k <= N/2: k = p + r P for
    // r < E/2, and k = N/2 on p = 0
    auto put = [&](int k) {
      const float2 zk = lds[idx(k)];
      const float2 zm = lds[idx((N - k) & (N - 1))];
      st_stream(out + (long long)k * (a.nt / 2), make_float4(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y),
                                                            0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x)));
    };
    static_for<E_ / 2>([&](auto r_) { put(p + decltype(r_)::value * P); });
    if (p == 0) put(N / 2);
    __syncthreads();  // this item's LDS reads before the next item's writes
  }
}

// samples per thread and real-column pairs per block of the x pass (timing sweep at
// 512-point lines: E=8, T=16)
template <int N>
struct XTune {
  static constexpr int E = (N == 512) ? 8 : default_e(N);
  static constexpr int T = (N == 512) ? 16 : (N == 256 ? 32 : default_t(N));
};

template <int N, int SP>
static hipError_t launch_xr2c_n(const FkXArgs& a, int ny, const float2* tw, hipStream_t s) {
  constexpr int E = XTune<N>::E, T = XTune<N>::T;
  using C = StridedCfg<N, E, T>;
  // (1024-point lines would need 235+ VGPRs in the streaming form: they keep fk_xr2c)
  if constexpr (SP == SP_F32 && (N == 256 || N == 512)) {
    const int ntiles = (a.nt / 2 + T - 1) / T;
    if ((a.nx == N || 2 * a.nx == N) && ntiles > 0 && ny > 0 && (long long)ntiles * ny < (1LL << 30)) {
      const int nitems = ntiles * ny;
      const bool half = 2 * a.nx == N;
      auto k = half ? fk_xr2c_stream<N, E, T, true> : fk_xr2c_stream<N, E, T, false>;
      const long long res = half ? resident_blocks<fk_xr2c_stream<N, E, T, true>>(C::THREADS)
                                 : resident_blocks<fk_xr2c_stream<N, E, T, false>>(C::THREADS);
      const long long nb = res > 0 && res < nitems ? res : nitems;
      hipLaunchKernelGGL(k, dim3((unsigned)nb), dim3(C::THREADS), 0, s, a, tw, ntiles, nitems);
      return hipGetLastError();
    }
  }
  dim3 grid((unsigned)((a.nt / 2 + T - 1) / T), (unsigned)ny);
  hipLaunchKernelGGL((fk_xr2c<N, E, T, SP>), grid, dim3(C::THREADS), 0, s, a, tw);
  return hipGetLastError();
}

template <int SP>
static hipError_t launch_xr2c_sp(int n, const FkXArgs& a, int ny, const float2* tw, hipStream_t s) {
  switch (n) {
    case 8: return launch_xr2c_n<8, SP>(a, ny, tw, s);
    case 16: return launch_xr2c_n<16, SP>(a, ny, tw, s);
    case 32: return launch_xr2c_n<32, SP>(a, ny, tw, s);
    case 64: return launch_xr2c_n<64, SP>(a, ny, tw, s);
    case 128: return launch_xr2c_n<128, SP>(a, ny, tw, s);
    case 256: return launch_xr2c_n<256, SP>(a, ny, tw, s);
    case 512: return launch_xr2c_n<512, SP>(a, ny, tw, s);
    case 1024: return launch_xr2c_n<1024, SP>(a, ny, tw, s);
    case 2048: return launch_xr2c_n<2048, SP>(a, ny, tw, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fk_xr2c(int n, const FkXArgs& a, int ny, const float2* tw, hipStream_t s, int sp) {
  if (sp == SP_F16) return launch_xr2c_sp<SP_F16>(n, a, ny, tw, s);
  if (sp == SP_BF16) return launch_xr2c_sp<SP_BF16>(n, a, ny, tw, s);
  return launch_xr2c_sp<SP_F32>(n, a, ny, tw, s);
}

// column pass: 16 samples per thread (64 threads per column) from timing sweeps at
// 1024-point columns; persistent blocks: 4096 for columns up to 1024 points (1-3 % faster
// than 2048 at 256x256x512 in every precision, 1024 slower), 2048 for 2048-point columns
// (4 % faster than 4096 at 128x128x1024)
constexpr long long column_blocks(int n) { return n >= 2048 ? 2048 : 4096; }

template <int N, int SP>
static hipError_t launch_pair_n(const FkPairArgs& a, const float2* tw, hipStream_t s) {
  constexpr int E = (N >= 1024) ? 16 : default_e(N);
  using C = ContigCfg<N, E>;
  const long long groups = (a.nwork + C::L - 1) / C::L;
  constexpr long long B = column_blocks(N);
  dim3 grid((unsigned)(groups < B ? groups : B));
  // padded volume, four-byte storage (FP32 keeps its guarded loads: the folded form
  // raised its registers from 157 to 173 and its occupancy from 3 to 2)
  const bool half = SP != SP_F32 && 2 * a.nt == N;
  if constexpr (SP == SP_F32 && FftShape<N, E>::NSTAGE == 3) {
    if (a.tscale_in == 0.f && 2 * a.nt == N) {
      const long long res = resident_blocks<fk_column_pair_stream<N, E>>(C::THREADS);
      const long long nb = res > 0 && res < groups ? res : groups;
      hipLaunchKernelGGL((fk_column_pair_stream<N, E>), dim3((unsigned)nb), dim3(C::THREADS), 0, s, a, tw);
      return hipGetLastError();
    }
  }
  if (SP == SP_F32 && a.tscale_in != 0.f)
    hipLaunchKernelGGL((fk_column_pair<N, E, SP_F32, true>), grid, dim3(C::THREADS), 0, s, a, tw);
  else if (a.tscale_in != 0.f)
    return hipErrorInvalidValue;  // input scaling is built for FP32 storage only
  else if (half)
    hipLaunchKernelGGL((fk_column_pair<N, E, SP, false, true>), grid, dim3(C::THREADS), 0, s, a, tw);
  else
    hipLaunchKernelGGL((fk_column_pair<N, E, SP>), grid, dim3(C::THREADS), 0, s, a, tw);
  return hipGetLastError();
}

template <int SP>
static hipError_t launch_pair_sp(int n, const FkPairArgs& a, const float2* tw, hipStream_t s) {
  switch (n) {
    case 8: return launch_pair_n<8, SP>(a, tw, s);
    case 16: return launch_pair_n<16, SP>(a, tw, s);
    case 32: return launch_pair_n<32, SP>(a, tw, s);
    case 64: return launch_pair_n<64, SP>(a, tw, s);
    case 128: return launch_pair_n<128, SP>(a, tw, s);
    case 256: return launch_pair_n<256, SP>(a, tw, s);
    case 512: return launch_pair_n<512, SP>(a, tw, s);
    case 1024: return launch_pair_n<1024, SP>(a, tw, s);
    case 2048: return launch_pair_n<2048, SP>(a, tw, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fk_column_pair(int n, const FkPairArgs& a, const float2* tw, hipStream_t s, int sp) {
  if (sp == SP_F16) return launch_pair_sp<SP_F16>(n, a, tw, s);
  if (sp == SP_BF16) return launch_pair_sp<SP_BF16>(n, a, tw, s);
  return launch_pair_sp<SP_F32>(n, a, tw, s);
}

// ---------------------------------------------------------------------------
// pass 3 for general Mt (FP32): the same column pairs and Stolt remap, the t-FFT in LDS
// ---------------------------------------------------------------------------

template <int EMAX>
__global__ __launch_bounds__(512) void gen_column_pair(FkPairArgs a, GenPlan g, int lp) {
  extern __shared__ float2 glds[];
  const int N = g.n, half = N / 2, P = 1 << lp, L = blockDim.x >> lp;
  const int tid = threadIdx.x;
  const int l = tid >> lp, p = tid & (P - 1);
  float2* my = glds + l * N;
  float2* twl = glds + L * N;
  gen_load_twiddles(twl, g);  // read after the first barrier of the loop
  const long long ngroups = (a.nwork + L - 1) / L;
  for (long long grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const long long w = grp * L + l;
    const bool ok = w < a.nwork;
    const PairItem it = pair_item(ok ? w : 0, a.Mx, a.My);
    const float2* in = static_cast<const float2*>(a.in) + (long long)it.ky * a.in_row + (long long)it.kx * a.nt;
    float2 x[EMAX];  // all loads in flight before any LDS write (EMAX * P >= N)
    static_for<EMAX>([&](auto k_) {
      constexpr int k = decltype(k_)::value;
      const int i = p + k * P;
      x[k] = (ok && i < a.nt) ? in[i] : make_float2(0.f, 0.f);
    });
    __syncthreads();  // the previous item's last LDS reads are done
    static_for<EMAX>([&](auto k_) {
      constexpr int k = decltype(k_)::value;
      const int i = p + k * P;
      if (i < N) my[i] = x[k];
    });
    __syncthreads();
    gen_fft<EMAX, false>(my, 1, g, twl, p, P);
    const int kxs = it.kx < a.Mx / 2 ? it.kx : it.kx - a.Mx;
    const int kys = it.ky < a.My / 2 ? it.ky : it.ky - a.My;
    const double ax = a.sxk * kxs, ay = a.syk * kys;
    const double A = ax * ax + ay * ay;
    float2* out = static_cast<float2*>(a.out);
    const long long dst = (long long)it.ky * a.out_row + (long long)it.kx * a.nt;
    const long long dst2 = (long long)it.ky2 * a.out_row + (long long)it.kx2 * a.nt;
    const bool ok2 = ok && it.has_mirror;
    for (int kz = p; kz < a.nt; kz += P) {
      float2 xa, xb;
      stolt_pair(
          kz, half, A, a.norm, [&](int i) { return my[i]; }, [&](int i) { return my[i == 0 ? 0 : N - i]; }, xa,
          xb);
      if (ok) out[dst + kz] = xa;
      if (ok2) out[dst2 + kz] = xb;
    }
  }
}

hipError_t launch_gen_column_pair(const GenPlan& g, const FkPairArgs& a, hipStream_t s) {
  if (a.nwork <= 0 || a.nt > g.n || a.tscale_in != 0.f) return hipErrorInvalidValue;
  int lp = 0;  // threads per column: a power of two with at most 8 samples per thread
  while ((8 << lp) < g.n) ++lp;
  if ((1 << lp) > 512) return hipErrorInvalidValue;
  const int L = (1 << lp) >= 256 ? 1 : 256 >> lp;
  const long long groups = (a.nwork + L - 1) / L;
  const unsigned grid = (unsigned)(groups < 8192 ? groups : 8192);
  const size_t lds = (size_t)(L + 1) * g.n * sizeof(float2);
  hipLaunchKernelGGL((gen_column_pair<8>), dim3(grid), dim3(L << lp), lds, s, a, g, lp);
  return hipGetLastError();
}

}  // namespace nlos
