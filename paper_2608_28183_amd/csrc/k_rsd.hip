// Radial RSD propagation (Section 4.3 propagation sum, Listing 3 lookup, Algorithm 4
// inner loop) for gfx950.
//
//   C[pix][d] = sum_f w_f P^[pix][f] a(pix) lerp(K_r[., f, d], rho~(pix))
//             = sum_f (wa w_f P^) K_r[i0][f][d] + (wb w_f P^) K_r[i0+1][f][d]
//
// The plan sorts the pixels by their lower radial bin i0 and groups them into chunks of
// up to 64 that share i0.  One wave64 takes a chunk, one pixel per lane, and a slice of
// kDepths depths: the two kernel rows K_r[i0][f][d0..d0+kDepths) and K_r[i0+1][f][...]
// are the same for the whole wave, so they come in through the scalar unit and enter the
// FMAs as scalar operands, and each kernel value is loaded once per 64 pixels.  The
// lane's own phasor P^[pix][f] is read from its contiguous frequency row.  Every C
// element is produced by one lane in a fixed frequency order.
#include <hip/hip_fp16.h>

#include <type_traits>

#include "mfma_fft.hpp"
#include "nlos_internal.hpp"

namespace nlos {

constexpr int kGroupPix = 64;   // pixels per chunk (one per lane; matches the plan)
constexpr int kDepths = 8;      // depths per wave
constexpr int kWavesPerBlock = 4;

template <int SP>
__device__ __forceinline__ float2 load_kr(const void* __restrict__ kr, long long i) {
  if constexpr (SP == SP_F32) {
    return static_cast<const float2*>(kr)[i];
  } else {
    return Mfma<SP>::unpack(static_cast<const unsigned int*>(kr)[i]);
  }
}

// acc += pa K0 + pb K1 (complex), fixed operation order
__device__ __forceinline__ void cmac2(float2& acc, float2 pa, float2 k0, float2 pb, float2 k1) {
  acc.x = fmaf(pa.x, k0.x, fmaf(-pa.y, k0.y, fmaf(pb.x, k1.x, fmaf(-pb.y, k1.y, acc.x))));
  acc.y = fmaf(pa.x, k0.y, fmaf(pa.y, k0.x, fmaf(pb.x, k1.y, fmaf(pb.y, k1.x, acc.y))));
}

// One frequency f of the lane's pixel: tap-weighted phasors, then the ND depths of the
// wave's slice (kernel rows o0, o1 are wave-uniform).
template <int SP, int ND>
__device__ __forceinline__ void rsd_freq(float2* acc, float2 p, float2 wf, float wa, float wb, const void* kr,
                                         long long o0, long long o1) {
  const float2 pw = make_float2(p.x * wf.x - p.y * wf.y, p.x * wf.y + p.y * wf.x);
  const float2 pa = make_float2(pw.x * wa, pw.y * wa);
  const float2 pb = make_float2(pw.x * wb, pw.y * wb);
#pragma unroll
  for (int j = 0; j < ND; ++j) cmac2(acc[j], pa, load_kr<SP>(kr, o0 + j), pb, load_kr<SP>(kr, o1 + j));
}

template <int SP>
__global__ __launch_bounds__(256) void rsd_propagate(RsdPropArgs a) {
  const int lane = threadIdx.x & 63;
  // wave-uniform work index: chunk g, depth slice starting at d0
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nds = (a.Nd + kDepths - 1) / kDepths;
  const long long w = (long long)blockIdx.x * kWavesPerBlock + wib;
  if (w >= a.nchunks * nds) return;
  const long long g = w / nds;
  const int d0 = (int)(w % nds) * kDepths;
  const int Nf = a.Nf, Nd = a.Nd;
  const int i0 = a.chunk_i0[g];
  const int pix = a.chunk_pix[g * kGroupPix + lane];
  float2 acc[kDepths];
#pragma unroll
  for (int j = 0; j < kDepths; ++j) acc[j] = make_float2(0.f, 0.f);
  if (i0 >= 0) {
    const int i1 = i0 + 1 < a.cut_idx ? i0 + 1 : a.cut_idx;
    // unused slots have wa = wb = 0 and read pixel 0's row
    const float wa = a.chunk_wa[g * kGroupPix + lane];
    const float wb = a.chunk_wb[g * kGroupPix + lane];
    const float2* __restrict__ ph = static_cast<const float2*>(a.Ph) + (long long)(pix >= 0 ? pix : 0) * a.ph_stride;
    long long o0 = (long long)i0 * Nf * Nd + d0;
    long long o1 = (long long)i1 * Nf * Nd + d0;
    if (d0 + kDepths <= Nd) {
      int f = 0;
      // eight phasor loads in flight per lane
      for (; f + 8 <= Nf; f += 8) {
        float2 p[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) p[u] = ph[f + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          rsd_freq<SP, kDepths>(acc, p[u], a.w[f + u], wa, wb, a.Kr, o0, o1);
          o0 += Nd;
          o1 += Nd;
        }
      }
      for (; f < Nf; ++f) {
        rsd_freq<SP, kDepths>(acc, ph[f], a.w[f], wa, wb, a.Kr, o0, o1);
        o0 += Nd;
        o1 += Nd;
      }
    } else {
      // last, partial depth slice
      const int nd = Nd - d0;
      for (int f = 0; f < Nf; ++f) {
        const float2 p = ph[f], wf = a.w[f];
        const float2 pw = make_float2(p.x * wf.x - p.y * wf.y, p.x * wf.y + p.y * wf.x);
        const float2 pa = make_float2(pw.x * wa, pw.y * wa);
        const float2 pb = make_float2(pw.x * wb, pw.y * wb);
#pragma unroll
        for (int j = 0; j < kDepths; ++j)
          if (j < nd) cmac2(acc[j], pa, load_kr<SP>(a.Kr, o0 + j), pb, load_kr<SP>(a.Kr, o1 + j));
        o0 += Nd;
        o1 += Nd;
      }
    }
  }
  if (pix < 0) return;
  float2* out = static_cast<float2*>(a.C) + (long long)pix * a.c_stride + d0;
#pragma unroll
  for (int j = 0; j < kDepths; ++j)
    if (d0 + j < Nd) out[j] = acc[j];
}

// ---------------------------------------------------------------------------
// matrix-core propagation (FP16 / BF16 radial kernel)
// ---------------------------------------------------------------------------
//
// For one chunk the sum is a complex matrix product: rows = the chunk's 64 pixels, the
// contraction runs over (frequency, tap) with the tap-weighted phasors A[p][f, tap] =
// w_f P^[p][f] (wa | wb)[p] on one side and the kernel rows K_r[i0 | i1][f][d] on the
// other, columns = depths.  As a real product on (re, im) pairs it maps onto
// v_mfma_f32_32x32x16 (FP32 accumulate): one 16-wide K step covers 4 frequencies x 2
// taps x (re, im), lane l holding frequencies 4s + 2(l/32) + {0, 1}.  B comes straight
// from the stored kernel pairs: (re, -im) for the real part of the output, (im, re) for
// the imaginary part.  A is rounded to the kernel's format after scaling by a power of two
// 2^e chosen per chunk from the largest |w_f P^| (wa | wb) of its pixels (a first pass
// over their rows), so that every component stays below 2^14; the FP32 result is
// multiplied by 2^-e.  A wave takes one chunk and DT 32-depth tiles.  DATA4: P^ and C are
// stored in the kernel's four-byte format too (FP16 P^ times 2^e_ph, FP16 C at depth d
// written times 2^e_c[d]); the chunk scale is then chosen on the stored values and the
// exponents are folded into one final ldexp.

template <int SP, int DT, bool DATA4>
__global__ __launch_bounds__(256) void rsd_propagate_mfma(RsdPropArgs a) {
  using M = Mfma<SP>;
  const int lane = threadIdx.x & 63;
  const int hl = lane >> 5, c32 = lane & 31;
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nds = (a.Nd + 32 * DT - 1) / (32 * DT);
  const long long w = (long long)blockIdx.x * kWavesPerBlock + wib;
  if (w >= a.nchunks * nds) return;
  const long long g = w / nds;
  const int d0 = (int)(w % nds) * 32 * DT;
  const int Nf = a.Nf, Nd = a.Nd;
  const int i0 = a.chunk_i0[g];
  // the lane's own pixel (first pass, stores) and the two rows it feeds into A
  const int pix = a.chunk_pix[g * kGroupPix + lane];
  const int pr0 = a.chunk_pix[g * kGroupPix + c32], pr1 = a.chunk_pix[g * kGroupPix + 32 + c32];
  mf_acc acc[2][DT][2];  // [row tile][depth tile][re | im]
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int q = 0; q < DT; ++q)
#pragma unroll
      for (int o = 0; o < 2; ++o)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[r][q][o][v] = 0.f;
  int out_exp = 0;  // C = acc 2^out_exp (before its own storage scale)
  if (i0 >= 0) {
    const int i1 = i0 + 1 < a.cut_idx ? i0 + 1 : a.cut_idx;
    // pass 1: the largest component of w_f P^ times the larger tap weight
    float m = 0.f;
    {
      const float tw = fmaxf(a.chunk_wa[g * kGroupPix + lane], a.chunk_wb[g * kGroupPix + lane]);
      const long long row = (long long)(pix >= 0 ? pix : 0) * a.ph_stride;
      constexpr int U = 16;  // loads in flight per lane (unconditional, clamped indices:
                             // a repeated last frequency does not change the maximum)
      for (int f0 = 0; f0 < Nf; f0 += U) {
        float2 p[U], wf[U];
        if constexpr (DATA4) {
          unsigned int raw[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int f = min(f0 + u, Nf - 1);
            raw[u] = static_cast<const unsigned int*>(a.Ph)[row + f];
            wf[u] = a.w[f];
          }
#pragma unroll
          for (int u = 0; u < U; ++u) p[u] = M::unpack(raw[u]);
        } else {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int f = min(f0 + u, Nf - 1);
            p[u] = static_cast<const float2*>(a.Ph)[row + f];
            wf[u] = a.w[f];
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const float re = p[u].x * wf[u].x - p[u].y * wf[u].y, im = p[u].x * wf[u].y + p[u].y * wf[u].x;
          m = fmaxf(m, fmaxf(fabsf(re), fabsf(im)));
        }
      }
      m *= tw;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    }
    int ex = 0;
    if (m > 0.f) (void)frexpf(m, &ex);  // m < 2^ex
    // clamped so that the scaled tap weights (<= 1) and 2^-e stay finite normal floats
    const int e = min(max(14 - ex, -100), 100);
    out_exp = -e;
    const float wa0 = ldexpf(a.chunk_wa[g * kGroupPix + c32], e), wb0 = ldexpf(a.chunk_wb[g * kGroupPix + c32], e);
    const float wa1 = ldexpf(a.chunk_wa[g * kGroupPix + 32 + c32], e);
    const float wb1 = ldexpf(a.chunk_wb[g * kGroupPix + 32 + c32], e);
    const long long row0 = (long long)(pr0 >= 0 ? pr0 : 0) * a.ph_stride;
    const long long row1 = (long long)(pr1 >= 0 ? pr1 : 0) * a.ph_stride;
    // the phasors of rows 0 and 1 at frequency f, loaded as stored
    using PRaw = typename std::conditional<DATA4, unsigned int, float2>::type;
    auto ldp = [&](long long row, int f) { return static_cast<const PRaw*>(a.Ph)[row + f]; };
    auto cvp = [&](PRaw r) {
      if constexpr (DATA4) return M::unpack(r);
      else return r;
    };
    const unsigned int* kr = static_cast<const unsigned int*>(a.Kr);
    const long long k0 = (long long)i0 * Nf * Nd, k1 = (long long)i1 * Nf * Nd;
    // one K step: this lane's frequencies fa = f0, fb = f0 + 1.  Every load is
    // unconditional, from clamped (valid) indices, so that the loads of several steps stay
    // in flight: a frequency beyond Nf is zeroed by its multiplier ma / mb on w_f P^ (its
    // A entries are then 0, whatever kernel value it meets), and a depth beyond Nd only
    // feeds output columns that are never stored.
    struct Step {
      float2 wfa, wfb;
      PRaw pa0, pb0, pa1, pb1;
      float ma, mb;
      unsigned int kv[DT][4];  // [depth tile][K0a, K1a, K0b, K1b]
    };
    auto load = [&](int f0) {
      Step t;
      const int fa = min(f0, Nf - 1), fb = min(f0 + 1, Nf - 1);
      t.ma = f0 < Nf ? 1.f : 0.f;
      t.mb = f0 + 1 < Nf ? 1.f : 0.f;
      t.wfa = a.w[fa];
      t.wfb = a.w[fb];
      t.pa0 = ldp(row0, fa);
      t.pb0 = ldp(row0, fb);
      t.pa1 = ldp(row1, fa);
      t.pb1 = ldp(row1, fb);
#pragma unroll
      for (int q = 0; q < DT; ++q) {
        const int d = min(d0 + 32 * q + c32, Nd - 1);
        t.kv[q][0] = kr[k0 + (long long)fa * Nd + d];
        t.kv[q][1] = kr[k1 + (long long)fa * Nd + d];
        t.kv[q][2] = kr[k0 + (long long)fb * Nd + d];
        t.kv[q][3] = kr[k1 + (long long)fb * Nd + d];
      }
      return t;
    };
    auto cm = [](float2 p, float2 wf) { return make_float2(p.x * wf.x - p.y * wf.y, p.x * wf.y + p.y * wf.x); };
    auto step = [&](const Step& t) {
      const float2 wa_ = make_float2(t.wfa.x * t.ma, t.wfa.y * t.ma), wb_ = make_float2(t.wfb.x * t.mb, t.wfb.y * t.mb);
      const float2 za0 = cm(cvp(t.pa0), wa_), zb0 = cm(cvp(t.pb0), wb_), za1 = cm(cvp(t.pa1), wa_),
                   zb1 = cm(cvp(t.pb1), wb_);
      mf_u4 A[2];
      A[0] = mf_u4{M::pack(za0.x * wa0, za0.y * wa0), M::pack(za0.x * wb0, za0.y * wb0),
                   M::pack(zb0.x * wa0, zb0.y * wa0), M::pack(zb0.x * wb0, zb0.y * wb0)};
      A[1] = mf_u4{M::pack(za1.x * wa1, za1.y * wa1), M::pack(za1.x * wb1, za1.y * wb1),
                   M::pack(zb1.x * wa1, zb1.y * wa1), M::pack(zb1.x * wb1, zb1.y * wb1)};
#pragma unroll
      for (int q = 0; q < DT; ++q) {
        // (re, -im): flip the sign of the upper half; (im, re): swap the halves
        const unsigned int* kq = t.kv[q];
        const mf_u4 Bre = mf_u4{kq[0] ^ 0x80000000u, kq[1] ^ 0x80000000u, kq[2] ^ 0x80000000u, kq[3] ^ 0x80000000u};
        const mf_u4 Bim = mf_u4{(kq[0] >> 16) | (kq[0] << 16), (kq[1] >> 16) | (kq[1] << 16),
                                (kq[2] >> 16) | (kq[2] << 16), (kq[3] >> 16) | (kq[3] << 16)};
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          acc[r][q][0] = M::mma(A[r], Bre, acc[r][q][0]);
          acc[r][q][1] = M::mma(A[r], Bim, acc[r][q][1]);
        }
      }
    };
    // K steps s = 0 .. ns-1 (frequencies 4s + 2hl + {0, 1}); the loads of step s + 4 are
    // issued right after step s is consumed, so four steps of loads are in flight
    const int ns = (Nf + 3) / 4;
    const int fl = 2 * hl;
    Step b0 = load(fl), b1 = load(fl + 4), b2 = load(fl + 8), b3 = load(fl + 12);
    for (int s0 = 0; s0 < ns; s0 += 4) {
      step(b0);
      b0 = load(fl + 4 * (s0 + 4));
      if (s0 + 1 < ns) step(b1);
      b1 = load(fl + 4 * (s0 + 5));
      if (s0 + 2 < ns) step(b2);
      b2 = load(fl + 4 * (s0 + 6));
      if (s0 + 3 < ns) step(b3);
      b3 = load(fl + 4 * (s0 + 7));
    }
  }
  // D lane layout: rows 8(v/4) + 4 hl + v%4 of the tile, column c32
  int qexp[DT];  // final exponent per depth tile column: the chunk scale, and for FP16
                 // data the stored P^ scale (undone) and C's storage scale at that depth
#pragma unroll
  for (int q = 0; q < DT; ++q) {
    const int d = min(d0 + 32 * q + c32, Nd - 1);
    qexp[q] = out_exp;
    if constexpr (DATA4 && SP == SP_F16) qexp[q] += a.e_c[d] - a.e_ph[0];
  }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int row = 32 * r + 8 * (v >> 2) + 4 * hl + (v & 3);
      const int pp = __shfl(pix, row, 64);
#pragma unroll
      for (int q = 0; q < DT; ++q) {
        const int d = d0 + 32 * q + c32;
        if (pp >= 0 && d < Nd) {
          const float re = ldexpf(acc[r][q][0][v], qexp[q]), im = ldexpf(acc[r][q][1][v], qexp[q]);
          const long long o = (long long)pp * a.c_stride + d;
          if constexpr (DATA4) static_cast<unsigned int*>(a.C)[o] = M::pack(re, im);
          else static_cast<float2*>(a.C)[o] = make_float2(re, im);
        }
      }
    }
}

// FP32 kernels on the matrix cores: the same product on v_mfma_f32_32x32x2f32 (FP32
// operands, FP32 accumulation).  A K step is one (frequency, tap): lane l holds part
// l/32 (re or im) of the tap-weighted phasor of its row, and the kernel value of its depth
// column as (re, -im) for the real part of the output and (im, re) for the imaginary part,
// the half l/32 selecting the entry.  A wave takes one chunk and DT 32-depth tiles; the
// loads of four frequencies ahead are in flight (unconditional, clamped indices as above).
typedef float rsd_f16v __attribute__((ext_vector_type(16)));

template <int DT>
__global__ __launch_bounds__(256) void rsd_propagate_mfma32(RsdPropArgs a) {
  const int lane = threadIdx.x & 63;
  const int hl = lane >> 5, c32 = lane & 31;
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nds = (a.Nd + 32 * DT - 1) / (32 * DT);
  const long long w = (long long)blockIdx.x * kWavesPerBlock + wib;
  if (w >= a.nchunks * nds) return;
  const long long g = w / nds;
  const int d0 = (int)(w % nds) * 32 * DT;
  const int Nf = a.Nf, Nd = a.Nd;
  const int i0 = a.chunk_i0[g];
  const int pix = a.chunk_pix[g * kGroupPix + lane];
  const int pr0 = a.chunk_pix[g * kGroupPix + c32], pr1 = a.chunk_pix[g * kGroupPix + 32 + c32];
  rsd_f16v acc[2][DT][2];  // [row tile][depth tile][re | im]
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int q = 0; q < DT; ++q)
#pragma unroll
      for (int o = 0; o < 2; ++o)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[r][q][o][v] = 0.f;
  if (i0 >= 0) {
    const int i1 = i0 + 1 < a.cut_idx ? i0 + 1 : a.cut_idx;
    const float wa0 = a.chunk_wa[g * kGroupPix + c32], wb0 = a.chunk_wb[g * kGroupPix + c32];
    const float wa1 = a.chunk_wa[g * kGroupPix + 32 + c32], wb1 = a.chunk_wb[g * kGroupPix + 32 + c32];
    const float2* ph = static_cast<const float2*>(a.Ph);
    const long long row0 = (long long)(pr0 >= 0 ? pr0 : 0) * a.ph_stride;
    const long long row1 = (long long)(pr1 >= 0 ? pr1 : 0) * a.ph_stride;
    const float2* kr = static_cast<const float2*>(a.Kr);
    const long long k0 = (long long)i0 * Nf * Nd, k1 = (long long)i1 * Nf * Nd;
    struct Step {
      float2 wf, p0, p1;
      float m;
      float2 kv[DT][2];  // [depth tile][tap]
    };
    auto load = [&](int f) {
      Step t;
      const int fc = min(f, Nf - 1);
      t.m = f < Nf ? 1.f : 0.f;
      t.wf = a.w[fc];
      t.p0 = ph[row0 + fc];
      t.p1 = ph[row1 + fc];
#pragma unroll
      for (int q = 0; q < DT; ++q) {
        const int d = min(d0 + 32 * q + c32, Nd - 1);
        t.kv[q][0] = kr[k0 + (long long)fc * Nd + d];
        t.kv[q][1] = kr[k1 + (long long)fc * Nd + d];
      }
      return t;
    };
    auto step = [&](const Step& t) {
      const float2 wf = make_float2(t.wf.x * t.m, t.wf.y * t.m);
      const float2 z0 = make_float2(t.p0.x * wf.x - t.p0.y * wf.y, t.p0.x * wf.y + t.p0.y * wf.x);
      const float2 z1 = make_float2(t.p1.x * wf.x - t.p1.y * wf.y, t.p1.x * wf.y + t.p1.y * wf.x);
      const float c0 = hl ? z0.y : z0.x, c1 = hl ? z1.y : z1.x;
      const float A[2][2] = {{wa0 * c0, wb0 * c0}, {wa1 * c1, wb1 * c1}};  // [row tile][tap]
#pragma unroll
      for (int q = 0; q < DT; ++q)
#pragma unroll
        for (int tap = 0; tap < 2; ++tap) {
          const float2 K = t.kv[q][tap];
          const float bre = hl ? -K.y : K.x, bim = hl ? K.x : K.y;
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            acc[r][q][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[r][tap], bre, acc[r][q][0], 0, 0, 0);
            acc[r][q][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[r][tap], bim, acc[r][q][1], 0, 0, 0);
          }
        }
    };
    Step b0 = load(0), b1 = load(1), b2 = load(2), b3 = load(3);
    for (int f0 = 0; f0 < Nf; f0 += 4) {
      step(b0);
      b0 = load(f0 + 4);
      if (f0 + 1 < Nf) step(b1);
      b1 = load(f0 + 5);
      if (f0 + 2 < Nf) step(b2);
      b2 = load(f0 + 6);
      if (f0 + 3 < Nf) step(b3);
      b3 = load(f0 + 7);
    }
  }
  // D lane layout: rows 8(v/4) + 4 hl + v%4 of the tile, column c32
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int row = 32 * r + 8 * (v >> 2) + 4 * hl + (v & 3);
      const int pp = __shfl(pix, row, 64);
#pragma unroll
      for (int q = 0; q < DT; ++q) {
        const int d = d0 + 32 * q + c32;
        if (pp >= 0 && d < Nd)
          static_cast<float2*>(a.C)[(long long)pp * a.c_stride + d] = make_float2(acc[r][q][0][v], acc[r][q][1][v]);
      }
    }
}

// ---------------------------------------------------------------------------
// FP16 storage scales of the RSD intermediates
// ---------------------------------------------------------------------------
//
// L = sum |tau| bounds every phasor |P[f]| (a DFT of one pixel's line), and so also the x
// and y DFTs of the padded phasor planes (sums over pixels).  The propagated plane at
// depth d is bounded by L kappa_d with kappa_d = sum_f |w_f| max_i |K_r[i][f][d]| (the
// tap weights are at most 1), and its unnormalised y-IFFT by My L kappa_d.  Each is stored
// times 2^(14 - k) with bound = f 2^k, f in [0.5, 1), so stored magnitudes stay below
// 2^14: one exponent for P, X and P^, one per depth plane for C and for D.  L is summed in
// a fixed order, so the scales, and the results, are deterministic.

__global__ __launch_bounds__(256) void rsd_l1_partial(const float2* __restrict__ tau, long long n2,
                                                      float* __restrict__ partials) {
  __shared__ float red[4];
  float acc = 0.f;
  const long long stride = (long long)gridDim.x * 256;
  long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  for (; i + 3 * stride < n2; i += 4 * stride) {  // four loads in flight per thread
    const float2 v0 = tau[i], v1 = tau[i + stride], v2 = tau[i + 2 * stride], v3 = tau[i + 3 * stride];
    acc += ((fabsf(v0.x) + fabsf(v0.y)) + (fabsf(v1.x) + fabsf(v1.y))) +
           ((fabsf(v2.x) + fabsf(v2.y)) + (fabsf(v3.x) + fabsf(v3.y)));
  }
  for (; i < n2; i += stride) acc += fabsf(tau[i].x) + fabsf(tau[i].y);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__device__ __forceinline__ int rsd_storage_exponent(float bound) {
  if (!(bound > 0.f) || !(bound <= 3.0e38f)) return 0;
  int k = 0;
  (void)frexpf(bound, &k);
  return min(max(14 - k, -120), 120);
}

__global__ __launch_bounds__(256) void rsd_scale_exponents(const float* __restrict__ partials, int np,
                                                           const float* __restrict__ kappa, int nd, int l_my,
                                                           int* __restrict__ exps) {
  __shared__ float red[4];
  float acc = 0.f;
  for (int j = threadIdx.x; j < np; j += 256) acc += partials[j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  const float L = (red[0] + red[1]) + (red[2] + red[3]);
  if (threadIdx.x == 0) exps[0] = rsd_storage_exponent(L);
  for (int d = threadIdx.x; d < nd; d += 256) {
    const int ec = rsd_storage_exponent(L * kappa[d]);
    exps[1 + d] = ec;
    exps[1 + nd + d] = ec - l_my;
  }
}

hipError_t launch_rsd_scales(const float* tau, long long n, float* partials, const float* kappa, int nd, int l_my,
                             int* exps, hipStream_t s) {
  if (n % 2 != 0 || nd < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rsd_l1_partial, dim3(kScaleBlocks), dim3(256), 0, s, reinterpret_cast<const float2*>(tau),
                     n / 2, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rsd_scale_exponents, dim3(1), dim3(256), 0, s, partials, kScaleBlocks, kappa, nd, l_my, exps);
  return hipGetLastError();
}

hipError_t launch_rsd_propagate(const RsdPropArgs& a, hipStream_t s) {
  if (a.data_sp != SP_F32 && (a.data_sp != a.kernel_sp || !a.mfma)) return hipErrorInvalidValue;
  if (a.mfma && (a.kernel_sp == SP_F16 || a.kernel_sp == SP_BF16)) {
    // FP16 / BF16: two depth tiles per wave by default (0.079 against 0.114 ms with one);
    // a.mfma == 2 asks for the other tiling
    const int dt = (a.mfma == 2 || a.Nd <= 32) ? 1 : 2;
    const long long waves = a.nchunks * ((a.Nd + 32 * dt - 1) / (32 * dt));
    const long long blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks);
    const bool d4 = a.data_sp != SP_F32;
#define NLOS_PROP(SPV, DTV, D4V) hipLaunchKernelGGL((rsd_propagate_mfma<SPV, DTV, D4V>), grid, dim3(256), 0, s, a)
    if (a.kernel_sp == SP_F16) {
      if (d4) { if (dt == 1) NLOS_PROP(SP_F16, 1, true); else NLOS_PROP(SP_F16, 2, true); }
      else { if (dt == 1) NLOS_PROP(SP_F16, 1, false); else NLOS_PROP(SP_F16, 2, false); }
    } else {
      if (d4) { if (dt == 1) NLOS_PROP(SP_BF16, 1, true); else NLOS_PROP(SP_BF16, 2, true); }
      else { if (dt == 1) NLOS_PROP(SP_BF16, 1, false); else NLOS_PROP(SP_BF16, 2, false); }
    }
#undef NLOS_PROP
    return hipGetLastError();
  }
  if (a.mfma && a.kernel_sp == SP_F32) {
    // FP32: one depth tile per wave by default (two waves per SIMD: 0.133 against 0.165 ms
    // with two tiles at 128 x 128 x 1024, 64 depths); a.mfma == 2 asks for the other tiling
    const int dt = (a.mfma == 2 && a.Nd > 32) ? 2 : 1;
    const long long waves = a.nchunks * ((a.Nd + 32 * dt - 1) / (32 * dt));
    const long long blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    if (dt == 1) hipLaunchKernelGGL(rsd_propagate_mfma32<1>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(rsd_propagate_mfma32<2>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  const long long nds = (a.Nd + kDepths - 1) / kDepths;
  const long long waves = a.nchunks * nds;
  const long long blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  if (a.kernel_sp == SP_F16)
    hipLaunchKernelGGL(rsd_propagate<SP_F16>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  else if (a.kernel_sp == SP_BF16)
    hipLaunchKernelGGL(rsd_propagate<SP_BF16>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(rsd_propagate<SP_F32>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace nlos
