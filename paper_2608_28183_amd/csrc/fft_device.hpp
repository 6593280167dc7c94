// Device-side FFT building blocks for gfx950 (wave64).
//
// A line of N complex samples is transformed by P cooperating threads, each
// holding E = N / P samples in registers.  The transform is a sequence of
// Stockham autosort stages (radix R_s, span Ns = product of earlier radices):
// butterfly j reads x[j + r N/R], multiplies by W_{Ns R}^{(j mod Ns) r}, runs an
// R-point DFT in registers and writes y[(j / Ns) Ns R + (j mod Ns) + r Ns].
// The first stage can read global memory directly and the last stage writes
// natural-order results directly, so a two-stage transform exchanges data
// through LDS once.
//
// R-point register DFTs are generated at compile time (four-step split into
// smaller DFTs, twiddles folded to constants computed in double precision by
// constexpr code).  Inter-stage twiddles come from a table of W_2048^k built in
// FP64 on the host.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace nlos {

constexpr int kTwiddleN = 2048;  // length of the device twiddle table W_2048^k

// ---------------------------------------------------------------------------
// compile-time helpers
// ---------------------------------------------------------------------------

template <int... Is, class F>
__device__ __forceinline__ void static_for_impl(std::integer_sequence<int, Is...>, F&& f) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(std::make_integer_sequence<int, N>{}, f);
}

constexpr double cx_pi = 3.14159265358979323846264338327950288;

// Taylor series on |x| <= pi/4 (terms up to x^25): error far below double epsilon.
constexpr double cx_sin_small(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int n = 1; n < 13; ++n) {
    term *= -x2 / double((2 * n) * (2 * n + 1));
    sum += term;
  }
  return sum;
}
constexpr double cx_cos_small(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int n = 1; n < 13; ++n) {
    term *= -x2 / double((2 * n - 1) * (2 * n));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi k / n with exact integer octant reduction.
constexpr double cx_cospi2(long k, long n, bool want_sin) {
  k %= n;
  if (k < 0) k += n;
  long q = (4 * k) / n;             // quadrant
  long rem = 4 * k - q * n;         // angle within quadrant = (pi/2) rem / n
  double c = 0.0, s = 0.0;
  if (2 * rem <= n) {
    double a = 0.5 * cx_pi * double(rem) / double(n);
    c = cx_cos_small(a);
    s = cx_sin_small(a);
  } else {
    double a = 0.5 * cx_pi * double(n - rem) / double(n);
    c = cx_sin_small(a);
    s = cx_cos_small(a);
  }
  double cc = c, ss = s;  // rotate by q quarter turns
  if (q == 1) { cc = -s; ss = c; }
  if (q == 2) { cc = -c; ss = -s; }
  if (q == 3) { cc = s; ss = -c; }
  return want_sin ? ss : cc;
}

// ---------------------------------------------------------------------------
// complex arithmetic on float2
// ---------------------------------------------------------------------------

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// Non-temporal (streaming) global accesses for volumes that are read or written once per
// pass and are far larger than the caches: they keep such lines from displacing the
// ones the next pass can still reuse.
__device__ __forceinline__ float2 ld_stream(const float2* p) {
  return make_float2(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
}
__device__ __forceinline__ void st_stream(float2* p, float2 v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}
typedef float nlos_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void st_stream(float4* p, float4 v) {
  const nlos_f4 w = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(w, reinterpret_cast<nlos_f4*>(p));
}
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 rot90(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// a * W_N^K where W_N = exp(-2 pi i / N) (forward) or its conjugate (inverse).
template <int N, int K, bool INV>
__device__ __forceinline__ float2 twc(float2 a) {
  constexpr int k = ((K % N) + N) % N;
  if constexpr (k == 0) {
    return a;
  } else if constexpr (2 * k == N) {
    return make_float2(-a.x, -a.y);
  } else if constexpr (4 * k == N) {
    return rot90<INV>(a);
  } else if constexpr (4 * k == 3 * N) {
    return rot90<!INV>(a);
  } else if constexpr (8 * k == N || 8 * k == 3 * N || 8 * k == 5 * N || 8 * k == 7 * N) {
    // (+-1 +- i)/sqrt(2): two adds and two multiplies
    constexpr float h = 0.70710678118654752440f;
    constexpr double cd = cx_cospi2(k, N, false);
    constexpr double sd = (INV ? 1.0 : -1.0) * cx_cospi2(k, N, true);
    constexpr float c = cd > 0 ? h : -h;
    constexpr float s = sd > 0 ? h : -h;
    // (a.x + i a.y)(c + i s)
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
  } else {
    constexpr float c = float(cx_cospi2(k, N, false));
    constexpr float s = float((INV ? 1.0 : -1.0) * cx_cospi2(k, N, true));
    return cmul(a, make_float2(c, s));
  }
}

// In-place R-point DFT on registers v[0..R), natural order in and out.
template <int R, bool INV>
__device__ __forceinline__ void dft(float2* v) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    float2 b0 = cadd(v[1], v[3]), b1 = rot90<INV>(csub(v[1], v[3]));
    v[0] = cadd(a0, b0);
    v[2] = csub(a0, b0);
    v[1] = cadd(a1, b1);
    v[3] = csub(a1, b1);
  } else {
    // four-step split R = N1 * N2: n = r + N1 j, k = s + N2 q
    constexpr int N1 = (R == 8) ? 2 : (R == 16) ? 4 : (R == 32) ? 4 : 8;
    constexpr int N2 = R / N1;
    float2 t[R];
    static_for<N1>([&](auto r_) {
      constexpr int r = decltype(r_)::value;
      float2 u[N2];
      static_for<N2>([&](auto j_) { u[decltype(j_)::value] = v[r + N1 * decltype(j_)::value]; });
      dft<N2, INV>(u);
      static_for<N2>([&](auto s_) {
        constexpr int s = decltype(s_)::value;
        t[r * N2 + s] = twc<R, r * s, INV>(u[s]);
      });
    });
    static_for<N2>([&](auto s_) {
      constexpr int s = decltype(s_)::value;
      float2 u[N1];
      static_for<N1>([&](auto r_) { u[decltype(r_)::value] = t[decltype(r_)::value * N2 + s]; });
      dft<N1, INV>(u);
      static_for<N1>([&](auto q_) { v[s + N2 * decltype(q_)::value] = u[decltype(q_)::value]; });
    });
  }
}

// ---------------------------------------------------------------------------
// radix plans: N = R0 * R1 * R2, each radix divides E (samples per thread)
// ---------------------------------------------------------------------------

// default samples per thread for a line length
constexpr int default_e(int n) {
  return n <= 16 ? n : (n == 32 || n == 64) ? 8 : (n <= 256) ? 16 : 32;
}

template <int N, int E_ = default_e(N)>
struct FftShape {
  static constexpr int E = E_ < N ? E_ : N;
  static constexpr int R0 = E;
  static constexpr int R1 = (N / R0) < E ? (N / R0) : E;
  static constexpr int R2 = N / (R0 * R1);
  static constexpr int P = N / E;
  static constexpr int NSTAGE = (R1 == 1) ? 1 : (R2 == 1 ? 2 : 3);
  static_assert(R0 * R1 * R2 == N, "radices must multiply to N");
  static_assert(E % R1 == 0 && E % R2 == 0 && R2 <= E, "radix must divide E");
};

// Element indices touched by thread p in a stage of radix R:
// butterfly b (0 <= b < E/R) is j = p + b P and reads x[j + r N/R].
template <int N, int R, int E>
__device__ __forceinline__ int stage_in_index(int p, int b, int r) {
  constexpr int P = N / E;
  return p + b * P + r * (N / R);
}
template <int N, int R, int Ns, int E>
__device__ __forceinline__ int stage_out_index(int p, int b, int r) {
  constexpr int P = N / E;
  const int j = p + b * P;
  return (j / Ns) * Ns * R + (j % Ns) + r * Ns;
}

// Twiddle + butterflies of one stage on registers v[b * R + r].
template <int N, int R, int Ns, int E, bool INV>
__device__ __forceinline__ void stage_compute(float2* v, int p, const float2* __restrict__ tw) {
  constexpr int P = N / E;
  static_for<E / R>([&](auto b_) {
    constexpr int b = decltype(b_)::value;
    if constexpr (Ns > 1) {
      const int jm = (p + b * P) % Ns;
      constexpr int step = kTwiddleN / (Ns * R);
      static_for<R - 1>([&](auto r_) {
        constexpr int r = decltype(r_)::value + 1;
        float2 w = tw[jm * r * step];
        if (INV) w.y = -w.y;
        v[b * R + r] = cmul(v[b * R + r], w);
      });
    }
    dft<R, INV>(v + b * R);
  });
}

// Inter-stage twiddles of thread p kept in registers (loaded once, reused for
// every line the thread transforms): stage 1 (span R0, radix R1) and stage 2
// (span R0 R1, radix R2); entry b * (R - 1) + r - 1 is W_{Ns R}^{((p + b P) mod Ns) r}.
template <class S>
struct TwRegs {
  static constexpr int N = S::R0 * S::R1 * S::R2;
  static constexpr int E = S::E, P = S::P;
  static constexpr int C1 = S::NSTAGE >= 2 ? (E / S::R1) * (S::R1 - 1) : 0;
  static constexpr int C2 = S::NSTAGE >= 3 ? (E / S::R2) * (S::R2 - 1) : 0;
  float2 w1[C1 > 0 ? C1 : 1];
  float2 w2[C2 > 0 ? C2 : 1];

  __device__ __forceinline__ void load(int p, const float2* __restrict__ tw) {
    if constexpr (C1 > 0) {
      constexpr int R = S::R1, Ns = S::R0, step = kTwiddleN / (Ns * R);
      static_for<E / R>([&](auto b_) {
        constexpr int b = decltype(b_)::value;
        const int jm = (p + b * P) % Ns;
        static_for<R - 1>([&](auto r_) {
          constexpr int r = decltype(r_)::value + 1;
          w1[b * (R - 1) + r - 1] = tw[jm * r * step];
        });
      });
    }
    if constexpr (C2 > 0) {
      constexpr int R = S::R2, Ns = S::R0 * S::R1, step = kTwiddleN / (Ns * R);
      static_for<E / R>([&](auto b_) {
        constexpr int b = decltype(b_)::value;
        const int jm = (p + b * P) % Ns;
        static_for<R - 1>([&](auto r_) {
          constexpr int r = decltype(r_)::value + 1;
          w2[b * (R - 1) + r - 1] = tw[jm * r * step];
        });
      });
    }
  }
};

// Stage with twiddles from registers w[b * (R - 1) + r - 1].
template <int R, int E, bool INV>
__device__ __forceinline__ void stage_compute_reg(float2* v, const float2* w) {
  static_for<E / R>([&](auto b_) {
    constexpr int b = decltype(b_)::value;
    static_for<R - 1>([&](auto r_) {
      constexpr int r = decltype(r_)::value + 1;
      float2 t = w[b * (R - 1) + r - 1];
      if (INV) t.y = -t.y;
      v[b * R + r] = cmul(v[b * R + r], t);
    });
    dft<R, INV>(v + b * R);
  });
}

}  // namespace nlos
