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
#include "nlos_internal.hpp"

namespace nlos {

// ---------------------------------------------------------------------------
// pass 1: real x-FFT with time scaling and zero padding
// ---------------------------------------------------------------------------

template <int N, int E, int T>
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
  const float s0 = float(2 * cc) * a.tscale, s1 = float(2 * cc + 1) * a.tscale;

  float2 v[S::E];
  static_for<S::E / S::R0>([&](auto b_) {
    static_for<S::R0>([&](auto r_) {
      constexpr int b = decltype(b_)::value, r = decltype(r_)::value;
      const int n = stage_in_index<N, S::R0, S::E>(p, b, r);
      float2 x = make_float2(0.f, 0.f);
      if (colok && n < a.nx) {
        const float2 t2 = *reinterpret_cast<const float2*>(a.tau + (y * a.nx + n) * a.nt + 2 * cc);
        x = make_float2(t2.x * s0, t2.y * s1);
      }
      v[b * S::R0 + r] = x;
    });
  });
  auto idx = [&](int n) { return n * C::LDS_W + c; };
  fft_run<S, false, true>(v, p, lds, idx, tw, [&](int n, float2 val) { lds[idx(n)] = val; });
  __syncthreads();
  if (!colok) return;
  float4* out = reinterpret_cast<float4*>(a.out + y * a.out_plane + 2 * cc);
  for (int k = p; k <= N / 2; k += P) {
    const float2 zk = lds[idx(k)];
    const float2 zm = lds[idx((N - k) & (N - 1))];
    // A = (Z[k] + conj Z[-k]) / 2, B = (Z[k] - conj Z[-k]) / (2i)
    const float4 ab = make_float4(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y),
                                  0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x));
    out[(long long)k * (a.nt / 2)] = ab;
  }
}

// ---------------------------------------------------------------------------
// pass 3: t-FFT -> Stolt remap for a column and its mirror -> two z-IFFTs
// ---------------------------------------------------------------------------

// Work item w -> input column (kx, ky) of the half spectrum and its mirror (kx2, ky2).
// Columns 1 <= kx < Mx/2 pair with (Mx - kx, -ky); on the planes kx = 0 and kx = Mx/2
// the mirror stays on the plane, so only ky in [0, My/2] is taken there, and ky = 0,
// My/2 are their own mirrors.
struct PairItem {
  int kx, ky, kx2, ky2;
  bool has_mirror;
};

__device__ __forceinline__ PairItem pair_item(long long w, int Mx, int My) {
  PairItem it;
  const long long nmain = (long long)(Mx / 2 - 1) * My;
  if (w < nmain) {
    it.kx = 1 + int(w / My);
    it.ky = int(w % My);
    it.kx2 = Mx - it.kx;
    it.ky2 = (My - it.ky) & (My - 1);
    it.has_mirror = true;
  } else {
    const int half = My / 2 + 1;
    const int w2 = int(w - nmain);
    it.kx = (w2 < half) ? 0 : Mx / 2;
    it.ky = w2 % half;
    it.kx2 = it.kx;
    it.ky2 = (My - it.ky) & (My - 1);
    it.has_mirror = (it.ky != 0) && (it.ky != My / 2);
  }
  return it;
}

template <int N, int E_ = default_e(N)>
__global__ __launch_bounds__((ContigCfg<N, E_>::THREADS)) void fk_column_pair(FkPairArgs a,
                                                                             const float2* __restrict__ tw) {
  using C = ContigCfg<N, E_>;
  using S = typename C::S;
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
    const float2* src = a.in + (long long)it.ky * a.in_row + (long long)it.kx * a.nt;

    float2 v[E];
    static_for<E / S::R0>([&](auto b_) {
      static_for<S::R0>([&](auto r_) {
        constexpr int b = decltype(b_)::value, r = decltype(r_)::value;
        const int n = stage_in_index<N, S::R0, E>(p, b, r);
        float2 x = make_float2(0.f, 0.f);
        if (ok && n < a.nt) x = src[n];
        v[b * S::R0 + r] = x;
      });
    });
    __syncthreads();  // the previous item's last LDS reads are done
    fft_run<S, false, true>(v, p, my, idx, tw, [&](int n, float2 val) { my[swz(n)] = val; });
    __syncthreads();

    // Stolt (shared by the pair): q = sqrt(A + kz^2) in t-bin units from a float square
    // root refined by one FP64 Newton step; lerp weight, Jacobian kz/q, 1/(Mx My Mt).
    const int kxs = it.kx < a.Mx / 2 ? it.kx : it.kx - a.Mx;
    const int kys = it.ky < a.My / 2 ? it.ky : it.ky - a.My;
    const double ax = a.sxk * kxs, ay = a.syk * kys;
    const double A = ax * ax + ay * ay;
    // the remapped column and its mirror go straight to W3 (kz < nt; kz >= Mt/2 and
    // kz = 0 are zero)
    float2* dst = a.out + (long long)it.ky * a.out_row + (long long)it.kx * a.nt;
    float2* dst2 = a.out + (long long)it.ky2 * a.out_row + (long long)it.kx2 * a.nt;
    const bool ok2 = ok && it.has_mirror;
    static_for<E / S::R0>([&](auto b_) {
      static_for<S::R0>([&](auto r_) {
        constexpr int b = decltype(b_)::value, r = decltype(r_)::value;
        const int kz = stage_in_index<N, S::R0, E>(p, b, r);
        if (kz < a.nt) {
          float2 xa = make_float2(0.f, 0.f), xb = make_float2(0.f, 0.f);
          if (kz > 0 && kz < HALF) {
            const double q2 = A + double(kz * kz);
            const float qf = __builtin_amdgcn_sqrtf((float)q2);
            const float rq = __builtin_amdgcn_rcpf(qf);
            const double q0 = (double)qf;
            const double q = fma((double)(0.5f * rq), fma(-q0, q0, q2), q0);
            if (q <= double(HALF - 1)) {
              const double fl = floor(q);
              const int i0 = int(fl);
              const int i1 = i0 + 1 < HALF ? i0 + 1 : HALF - 1;
              const float fr = float(q - fl);
              const float jac = float(kz) * rq * a.norm;
              // column (kx, ky): samples i0, i1 of the w >= 0 half
              const float2 s0 = my[swz(i0)], s1 = my[swz(i1)];
              xa.x = fmaf(fr, s1.x - s0.x, s0.x) * jac;
              xa.y = fmaf(fr, s1.y - s0.y, s0.y) * jac;
              // mirror (-kx, -ky): conj of samples -i0, -i1 (mod N)
              const float2 m0 = my[swz((N - i0) & (N - 1))], m1 = my[swz((N - i1) & (N - 1))];
              xb.x = fmaf(fr, m1.x - m0.x, m0.x) * jac;
              xb.y = -fmaf(fr, m1.y - m0.y, m0.y) * jac;
            }
          }
          if (ok) dst[kz] = xa;
          if (ok2) dst2[kz] = xb;
        }
      });
    });
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

// samples per thread and real-column pairs per block of the x pass (timing sweep at
// 512-point lines: E=8, T=16)
template <int N>
struct XTune {
  static constexpr int E = (N == 512) ? 8 : default_e(N);
  static constexpr int T = (N == 512) ? 16 : (N == 256 ? 32 : default_t(N));
};

template <int N>
static hipError_t launch_xr2c_n(const FkXArgs& a, int ny, const float2* tw, hipStream_t s) {
  constexpr int E = XTune<N>::E, T = XTune<N>::T;
  using C = StridedCfg<N, E, T>;
  dim3 grid((unsigned)((a.nt / 2 + T - 1) / T), (unsigned)ny);
  hipLaunchKernelGGL((fk_xr2c<N, E, T>), grid, dim3(C::THREADS), 0, s, a, tw);
  return hipGetLastError();
}

hipError_t launch_fk_xr2c(int n, const FkXArgs& a, int ny, const float2* tw, hipStream_t s) {
  switch (n) {
    case 8: return launch_xr2c_n<8>(a, ny, tw, s);
    case 16: return launch_xr2c_n<16>(a, ny, tw, s);
    case 32: return launch_xr2c_n<32>(a, ny, tw, s);
    case 64: return launch_xr2c_n<64>(a, ny, tw, s);
    case 128: return launch_xr2c_n<128>(a, ny, tw, s);
    case 256: return launch_xr2c_n<256>(a, ny, tw, s);
    case 512: return launch_xr2c_n<512>(a, ny, tw, s);
    case 1024: return launch_xr2c_n<1024>(a, ny, tw, s);
    case 2048: return launch_xr2c_n<2048>(a, ny, tw, s);
    default: return hipErrorInvalidValue;
  }
}

// column pass: 16 samples per thread (64 threads per column) from timing sweeps at
// 1024-point columns; persistent blocks, a few per CU
constexpr long long kColumnBlocks = 2048;

template <int N>
static hipError_t launch_pair_n(const FkPairArgs& a, const float2* tw, hipStream_t s) {
  constexpr int E = (N >= 1024) ? 16 : default_e(N);
  using C = ContigCfg<N, E>;
  const long long groups = (a.nwork + C::L - 1) / C::L;
  dim3 grid((unsigned)(groups < kColumnBlocks ? groups : kColumnBlocks));
  hipLaunchKernelGGL((fk_column_pair<N, E>), grid, dim3(C::THREADS), 0, s, a, tw);
  return hipGetLastError();
}

hipError_t launch_fk_column_pair(int n, const FkPairArgs& a, const float2* tw, hipStream_t s) {
  switch (n) {
    case 8: return launch_pair_n<8>(a, tw, s);
    case 16: return launch_pair_n<16>(a, tw, s);
    case 32: return launch_pair_n<32>(a, tw, s);
    case 64: return launch_pair_n<64>(a, tw, s);
    case 128: return launch_pair_n<128>(a, tw, s);
    case 256: return launch_pair_n<256>(a, tw, s);
    case 512: return launch_pair_n<512>(a, tw, s);
    case 1024: return launch_pair_n<1024>(a, tw, s);
    case 2048: return launch_pair_n<2048>(a, tw, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace nlos
