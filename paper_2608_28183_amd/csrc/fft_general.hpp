// General-length line FFTs held in LDS (gfx950, FP32).
//
// Lengths n whose prime factors are 2, 3, 5, 7, 11 and 13 (the office-scene grids of
// the paper's Table 4 pad to 720 x 520 and to time axes of 750, 1500 or 3000 samples)
// run as Stockham stages over radices from {2, 3, 4, 5, 7, 8, 9, 11, 13, 16}, chosen on the
// host (GenPlan).  A line lives in LDS for the whole transform; each stage reads all of
// its butterfly inputs into registers, waits for the block, and writes the outputs back
// in place, so no second buffer is needed.  Butterfly j of a stage with radix R and span
// Ns reads x[j + r n/R], multiplies by W_{Ns R}^{(j mod Ns) r} = W_n^{(j mod Ns) r n/(Ns R)}
// from a table of W_n^k built in FP64 on the host, runs an R-point DFT in registers and
// writes y[(j / Ns) Ns R + (j mod Ns) + r Ns].
//
// Power-of-two lengths keep the register-resident kernels; these serve the rest.
#pragma once

#include <hip/hip_runtime.h>

#include "fft_device.hpp"
#include "nlos_internal.hpp"

namespace nlos {

// R-point DFT of an odd prime R in registers, natural order in and out.  Inputs n and
// R - n are folded first: X[k] = v0 + sum_n s_n cos(2 pi n k / R) -+ i sum_n d_n sin(...)
// with s_n = v[n] + v[R-n], d_n = v[n] - v[R-n] (n = 1 .. (R-1)/2), and X[R-k] takes the
// other sign of the sine sum.  Constants are FP64 values rounded once to FP32.
template <int R, bool INV>
__device__ __forceinline__ void dft_prime(float2* v) {
  constexpr int H = (R - 1) / 2;
  float2 s[H + 1], d[H + 1];
  float2 sum = v[0];
  static_for<H>([&](auto n_) {
    constexpr int n = decltype(n_)::value + 1;
    s[n] = cadd(v[n], v[R - n]);
    d[n] = csub(v[n], v[R - n]);
    sum = cadd(sum, s[n]);
  });
  const float2 v0 = v[0];
  v[0] = sum;
  static_for<H>([&](auto k_) {
    constexpr int k = decltype(k_)::value + 1;
    float2 re = v0, im = make_float2(0.f, 0.f);
    static_for<H>([&](auto n_) {
      constexpr int n = decltype(n_)::value + 1;
      constexpr float c = float(cx_cospi2((long)n * k, R, false));
      constexpr float sn = float(cx_cospi2((long)n * k, R, true));
      re.x = fmaf(c, s[n].x, re.x);
      re.y = fmaf(c, s[n].y, re.y);
      im.x = fmaf(sn, d[n].x, im.x);
      im.y = fmaf(sn, d[n].y, im.y);
    });
    // forward: X[k] = re - i im, X[R-k] = re + i im; inverse the other way round
    const float2 minus = make_float2(re.x + im.y, re.y - im.x);
    const float2 plus = make_float2(re.x - im.y, re.y + im.x);
    v[k] = INV ? plus : minus;
    v[R - k] = INV ? minus : plus;
  });
}

template <int R, bool INV>
__device__ __forceinline__ void dft_any(float2* v);

// Four-step split R = N1 N2 (n = r + N1 j, k = s + N2 q): N1 DFTs of length N2 over j,
// twiddles W_R^{r s}, N2 DFTs of length N1 over r.
template <int R, int N1, bool INV>
__device__ __forceinline__ void dft_split(float2* v) {
  constexpr int N2 = R / N1;
  float2 t[R];
  static_for<N1>([&](auto r_) {
    constexpr int r = decltype(r_)::value;
    float2 u[N2];
    static_for<N2>([&](auto j_) { u[decltype(j_)::value] = v[r + N1 * decltype(j_)::value]; });
    dft_any<N2, INV>(u);
    static_for<N2>([&](auto s_) {
      constexpr int s = decltype(s_)::value;
      t[r * N2 + s] = twc<R, r * s, INV>(u[s]);
    });
  });
  static_for<N2>([&](auto s_) {
    constexpr int s = decltype(s_)::value;
    float2 u[N1];
    static_for<N1>([&](auto r_) { u[decltype(r_)::value] = t[decltype(r_)::value * N2 + s]; });
    dft_any<N1, INV>(u);
    static_for<N1>([&](auto q_) { v[s + N2 * decltype(q_)::value] = u[decltype(q_)::value]; });
  });
}

template <int R, bool INV>
__device__ __forceinline__ void dft_any(float2* v) {
  if constexpr (R == 3 || R == 5 || R == 7 || R == 11 || R == 13) {
    dft_prime<R, INV>(v);
  } else if constexpr (R == 9) {
    dft_split<9, 3, INV>(v);
  } else {
    dft<R, INV>(v);
  }
}

// LDS pointers typed as such (address space 3): the stages are not inlined, and through
// a plain pointer their accesses would compile to flat instructions instead of ds_ ones.
typedef float nlos_v2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) nlos_v2 lds_v2;
__device__ __forceinline__ lds_v2* as_lds(float2* p) { return (lds_v2*)p; }
__device__ __forceinline__ const lds_v2* as_lds(const float2* p) { return (const lds_v2*)p; }

// One stage on a line at base[i * ls], i < n, shared by P threads (thread p).  Every
// thread of the block calls it (it synchronises the block); Q bounds the butterflies per
// thread, so Q * P >= n / R must hold.  Not inlined: each radix then gets its own register
// allocation instead of the union over the dispatch in gen_fft.
template <int R, int Q, bool INV>
__device__ __attribute__((noinline)) void gen_stage(lds_v2* base, int ls, int n, int ns, int p, int P,
                                                   const lds_v2* tw) {
  const int nb = n / R;
  float2 v[Q][R];
  static_for<Q>([&](auto q_) {
    constexpr int q = decltype(q_)::value;
    const int j = p + q * P;
    if (j < nb) {
      static_for<R>([&](auto r_) {
        constexpr int r = decltype(r_)::value;
        const nlos_v2 t = base[(j + r * nb) * ls];
        v[q][r] = make_float2(t.x, t.y);
      });
    }
  });
  __syncthreads();
  const int step = n / (ns * R);
  static_for<Q>([&](auto q_) {
    constexpr int q = decltype(q_)::value;
    const int j = p + q * P;
    if (j < nb) {
      const int jm = j % ns;
      if (ns > 1) {
        static_for<R - 1>([&](auto r_) {
          constexpr int r = decltype(r_)::value + 1;
          const nlos_v2 t = tw[jm * r * step];
          const float2 w = make_float2(t.x, INV ? -t.y : t.y);
          v[q][r] = cmul(v[q][r], w);
        });
      }
      dft_any<R, INV>(v[q]);
      const int o = (j - jm) * R + jm;
      static_for<R>([&](auto r_) {
        constexpr int r = decltype(r_)::value;
        base[(o + r * ns) * ls] = nlos_v2{v[q][r].x, v[q][r].y};
      });
    }
  });
  __syncthreads();
}

constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// The block's copy of the twiddle table in LDS (read before the first stage's barrier):
// a stage then waits on LDS, not on a gather from L2.
__device__ __forceinline__ void gen_load_twiddles(float2* twl, const GenPlan& g) {
  for (int k = threadIdx.x; k < g.n; k += blockDim.x) twl[k] = g.tw[k];
}

// Whole transform of the line at base[i * ls] in place, natural order in and out
// (unnormalised both ways).  EMAX bounds the samples per thread: EMAX * P >= g.n.  tw is
// the block's LDS copy of g.tw (gen_load_twiddles).
template <int EMAX, bool INV>
__device__ __forceinline__ void gen_fft(float2* line, int ls, const GenPlan& g, const float2* twl, int p, int P) {
  lds_v2* base = as_lds(line);
  const lds_v2* tw = as_lds(twl);
  int ns = 1;
  for (int s = 0; s < g.nstage; ++s) {
    const int R = g.radix[s];
    switch (R) {
      case 2: gen_stage<2, cdiv(EMAX, 2), INV>(base, ls, g.n, ns, p, P, tw); break;
      case 3: gen_stage<3, cdiv(EMAX, 3), INV>(base, ls, g.n, ns, p, P, tw); break;
      case 4: gen_stage<4, cdiv(EMAX, 4), INV>(base, ls, g.n, ns, p, P, tw); break;
      case 5: gen_stage<5, cdiv(EMAX, 5), INV>(base, ls, g.n, ns, p, P, tw); break;
      case 7: gen_stage<7, cdiv(EMAX, 7), INV>(base, ls, g.n, ns, p, P, tw); break;
      case 8: gen_stage<8, cdiv(EMAX, 8), INV>(base, ls, g.n, ns, p, P, tw); break;
      case 9: gen_stage<9, cdiv(EMAX, 9), INV>(base, ls, g.n, ns, p, P, tw); break;
      case 16: gen_stage<16, cdiv(EMAX, 16), INV>(base, ls, g.n, ns, p, P, tw); break;
      case 11: gen_stage<11, cdiv(EMAX, 11), INV>(base, ls, g.n, ns, p, P, tw); break;
      case 13: gen_stage<13, cdiv(EMAX, 13), INV>(base, ls, g.n, ns, p, P, tw); break;
      default: break;  // the host plans only the radices above
    }
    ns *= R;
  }
}

}  // namespace nlos
