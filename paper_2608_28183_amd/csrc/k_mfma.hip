// f-k passes of the four-byte storage path with their DFT stages on the matrix cores.
//
// Every line transform is split in two (N = N1 N2, input n = n1 + N1 n2, output
// k = k2 + N2 k1):  Y[n1][k2] = sum_n2 x[n1 + N1 n2] W_N2^(n2 k2), the twiddle
// W_N^(n1 k2), then X[k2 + N2 k1] = sum_n1 W_N1^(n1 k1) Y[n1][k2].  Both inner sums are
// matrix products of a constant DFT matrix (FP64-built operands, binary16 or bfloat16)
// with the stored four-byte values, accumulated in FP32; the twiddle is an FP32 complex
// multiply before the intermediate is rounded back to the storage format.
//   strided_fft_mfma  lines along a strided axis (y, x; columns contiguous), the 32
//                     columns of a tile being the batch of both products; Y goes
//                     through LDS between them;
//   fk_column_pair_mfma  the paired column pass of 1024-point columns: the t-FFT in
//                     registers (the batch of the first product is n1 and of the second
//                     k2, which leaves each lane holding exactly the values its second
//                     product needs), the spectrum in LDS, the Stolt remap of the
//                     column and its mirror;
//   zfft_abs2_mfma    the z-IFFT of the cropped 1024-point columns, |Psi|^2 and the
//                     max over depth.
// FP16 scaling: stored values carry the power-of-two factor of their intermediate.  The
// forward passes keep it (every partial DFT of the scaled transient is below 2^14); the
// inverse passes use DFT matrices scaled by 1/N2 and 1/N1 (exact), so that their
// outputs carry the factor of the next intermediate, 2^-log2(N) times the input's; BF16
// is unscaled.
#include "fft_device.hpp"
#include "fk_pairs.hpp"
#include "mfma_fft.hpp"
#include "prec.hpp"

namespace nlos {

__device__ __forceinline__ unsigned int ld_u32_nt(const unsigned int* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_u32_nt(unsigned int* p, unsigned int v) { __builtin_nontemporal_store(v, p); }

// Orders one wave's LDS accesses on either side (a spectrum written by some lanes and
// read by others of the same wave).
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// strided lines: N = 16 N1 points (N1 = 16 or 32), tiles of 32 columns, 8 waves
// ---------------------------------------------------------------------------

constexpr int kMfT = 32;   // columns per tile
constexpr int kMfW = 8;    // waves per block

// One tile (32 columns of one plane) per block.  The inputs n_in and outputs n_out are N
// or N/2 (zero padding, crop) and the column count a multiple of 32 (checked on the host),
// so no load or store needs a guard.
template <int N, bool INV, int SP>
__global__ __launch_bounds__(64 * kMfW) void strided_fft_mfma(StridedArgs a, const mf_u4* __restrict__ t1,
                                                              const mf_u4* __restrict__ t3,
                                                              const float2* __restrict__ tw, int tiles_x) {
  constexpr int N2 = 16, N1 = N / 16;
  constexpr int KS3 = N1 / 8, MB3 = N1 / 16;   // K steps and output blocks of the second product
  constexpr int IT1 = N1 / kMfW, IT3 = N2 / kMfW;
  static_assert(N1 == 16 || N1 == 32, "N = 256 or 512");
  using M = Mfma<SP>;
  __shared__ unsigned int ybuf[N * kMfT];  // Y'[n1][k2][column], four-byte complex
  __shared__ float2 twl[N];                // W_N^m
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = lane & 31, hl = lane >> 5;
  const long long plane = blockIdx.x / tiles_x;
  const int c0 = (blockIdx.x % tiles_x) * kMfT;
  for (int m = threadIdx.x; m < N; m += 64 * kMfW) twl[m] = tw[m * (kTwiddleN / N)];
  // inputs n2 >= 8 (n >= N/2) are all zero padding when n_in = N/2: one K step
  const bool upper = a.n_in > N / 2;
  // row n = n1 + N1 n2 of this lane: n2 = 8 q + 4 hl + r, n1 = wv + 8 it; the lane part
  // of the offset is (4 N1 hl) rows + its column, the rest is uniform
  const unsigned int* in = static_cast<const unsigned int*>(a.in) + plane * a.in_plane + c0;
  const long long lin = (long long)(4 * N1 * hl) * a.in_line + col;
  unsigned int raw[IT1][2][4];
#pragma unroll
  for (int it = 0; it < IT1; ++it)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const unsigned int* row = in + (long long)((wv + kMfW * it) + N1 * (8 * q + r)) * a.in_line;
        raw[it][q][r] = (q == 0 || upper) ? ld_u32_nt(row + lin) : 0u;
      }
  const mf_u4 A1[2] = {t1[lane], t1[64 + lane]};
  mf_u4 A3[MB3][KS3];
#pragma unroll
  for (int b = 0; b < MB3; ++b)
#pragma unroll
    for (int q = 0; q < KS3; ++q) A3[b][q] = t3[(b * KS3 + q) * 64 + lane];
  __syncthreads();  // twl
  // first product and twiddle -> ybuf
#pragma unroll
  for (int it = 0; it < IT1; ++it) {
    const int n1 = wv + kMfW * it;
    mf_acc d = {};
    d = M::mma(A1[0], mf_u4{raw[it][0][0], raw[it][0][1], raw[it][0][2], raw[it][0][3]}, d);
    if (upper) d = M::mma(A1[1], mf_u4{raw[it][1][0], raw[it][1][1], raw[it][1][2], raw[it][1][3]}, d);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k2 = mf_out_index(j, hl);
      const float2 y = mf_cmul<INV>(mf_out(d, j), twl[(n1 * k2) & (N - 1)]);
      ybuf[(n1 * N2 + k2) * kMfT + col] = M::pack(y.x, y.y);
    }
  }
  __syncthreads();
  // second product: this wave's k2, outputs n = k2 + N2 k1 < n_out
  unsigned int* out = static_cast<unsigned int*>(a.out) + plane * a.out_plane + c0;
  const long long lout = (long long)(N2 * 4 * hl) * a.out_line + col;
#pragma unroll
  for (int it = 0; it < IT3; ++it) {
    const int k2 = wv + kMfW * it;
    mf_u4 B[KS3];
#pragma unroll
    for (int q = 0; q < KS3; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) B[q][r] = ybuf[((8 * q + 4 * hl + r) * N2 + k2) * kMfT + col];
#pragma unroll
    for (int b = 0; b < MB3; ++b) {
      if (16 * b * N2 >= a.n_out) continue;  // a cropped output block (uniform)
      mf_acc d = {};
#pragma unroll
      for (int q = 0; q < KS3; ++q) d = M::mma(A3[b][q], B[q], d);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        // n = k2 + N2 (16 b + (j < 4 ? 0 : 8) + (j & 3)) + N2 4 hl
        const int nu = k2 + N2 * (16 * b + (j < 4 ? 0 : 8) + (j & 3));
        if (nu + N2 * 4 * hl < a.n_out) st_u32_nt(out + (long long)nu * a.out_line + lout, M::pack(d[j], d[j + 8]));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 1024-point columns: N1 = N2 = 32, one column per wave
// ---------------------------------------------------------------------------

constexpr int kColN = 1024;

// Lane (j = l % 32, hl = l / 32) of a 1024-point line transform computes Y[n1][k2 = j] for
// n1 = 8 (v / 4) + 4 hl + v % 4 (v < 16) in the first product (rows n1, data as the A
// operand) and X[j + 32 k1] in the second (data as B), so its twiddles W_1024^(n1 j) are
// fixed: a block-shared LDS table tl[v][lane].
__device__ __forceinline__ void col1024_twiddles(float2* tl, const float2* twt, bool inverse) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x, j = lane & 31, hl = lane >> 5;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int n1 = 8 * (v / 4) + 4 * hl + (v % 4);
      float2 w = twt[2 * ((n1 * j) & (kColN - 1))];  // W_1024^m = W_2048^(2m)
      if (inverse) w.y = -w.y;
      tl[v * 64 + lane] = w;
    }
  }
}

// First product and twiddle of one line whose inputs n < 512 are raw[q][r] =
// x[j + 32 (8 q + 4 hl + r)] (four-byte values), giving the second product's B operands.
// B1[c][q]: part c of the outputs, K step q (the upper 512 inputs are zero).
template <int SP>
__device__ __forceinline__ void col1024_first(const mf_u4 (&B1)[2][2], const float2* tl, int lane,
                                              const unsigned int (&raw)[2][4], mf_u4 (&B3)[4]) {
  using M = Mfma<SP>;
  const mf_u4 a0 = {raw[0][0], raw[0][1], raw[0][2], raw[0][3]};
  const mf_u4 a1 = {raw[1][0], raw[1][1], raw[1][2], raw[1][3]};
  mf_acc re = {}, im = {};
  re = M::mma(a0, B1[0][0], re);
  re = M::mma(a1, B1[0][1], re);
  im = M::mma(a0, B1[1][0], im);
  im = M::mma(a1, B1[1][1], im);
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const float2 y = mf_cmul<false>(make_float2(re[v], im[v]), tl[v * 64 + lane]);
    B3[v / 4][v % 4] = M::pack(y.x, y.y);
  }
}

__device__ __forceinline__ void load_b1(mf_u4 (&B1)[2][2], const mf_u4* tb1, int lane) {
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int q = 0; q < 2; ++q) B1[c][q] = tb1[(c * 4 + q) * 64 + lane];
}

// Two work items (column pairs) per wave and iteration: the loads of both are in flight
// before the first is transformed.
template <int SP>
__global__ __launch_bounds__(256) void fk_column_pair_mfma(FkPairArgs a, const mf_u4* __restrict__ tb1,
                                                           const mf_u4* __restrict__ ta3,
                                                           const float2* __restrict__ twt, float oscale) {
  constexpr int N = kColN, HALF = N / 2;
  using M = Mfma<SP>;
  __shared__ float2 spec[4][N + 2];  // a wave's column spectrum, natural order; bin N repeats bin 0
  __shared__ float2 tl[16 * 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j = lane & 31, hl = lane >> 5;
  col1024_twiddles(tl, twt, false);
  mf_u4 B1[2][2];
  load_b1(B1, tb1, lane);
  mf_u4 A3[2][4];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int q = 0; q < 4; ++q) A3[b][q] = ta3[(b * 4 + q) * 64 + lane];
  __syncthreads();
  float2* my = spec[wv];
  const unsigned int* inb = static_cast<const unsigned int*>(a.in);
  unsigned int* outb = static_cast<unsigned int*>(a.out);
  const long long ngroups = (a.nwork + 7) / 8;
  // The next group's columns are loaded while this group is transformed.  An item past
  // the end (in the last group) stands in for the group's first item: it reads that
  // column, computes the same values and stores them to the same places, so that every
  // wave issues the same loads and stores and the wait for the next group's loads leaves
  // this group's stores in flight.
  PairItem nitem[2];
  unsigned int nraw[2][2][4];
  auto fetch = [&](long long g) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const long long w = g * 8 + 4 * u + wv;
      nitem[u] = pair_item(w < a.nwork ? w : g * 8, a.Mx, a.My);
      const unsigned int* in = inb + (long long)nitem[u].ky * a.in_row + (long long)nitem[u].kx * a.nt + j;
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) nraw[u][q][r] = ld_u32_nt(in + 32 * (8 * q + 4 * hl + r));
    }
  };
  if ((long long)blockIdx.x < ngroups) fetch(blockIdx.x);
  // the tables and the first group arrive before the loop, whose one wait per group then
  // counts only the loop's own loads and stores
  __builtin_amdgcn_s_waitcnt(0);
  for (long long g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const PairItem item[2] = {nitem[0], nitem[1]};
    unsigned int raw[2][2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) raw[u][q][r] = nraw[u][q][r];
    if (g + gridDim.x < ngroups) fetch(g + gridDim.x);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      mf_u4 B3[4];
      col1024_first<SP>(B1, tl, lane, raw[u], B3);
      wave_lds_fence();  // the previous spectrum's LDS reads come first
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        mf_acc d = {};
#pragma unroll
        for (int q = 0; q < 4; ++q) d = M::mma(A3[b][q], B3[q], d);
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
          const int n = j + 32 * (16 * b + mf_out_index(jj, hl));
          my[n] = mf_out(d, jj);
          if (n == 0) my[N] = mf_out(d, jj);
        }
      }
      wave_lds_fence();
      // Stolt remap of the column (w >= 0 half) and of its mirror (conjugated w <= 0
      // half), sharing q = sqrt(A + kz^2) in t-bin units (FP32); zero beyond the last
      // frequency sample, the last sample itself at q = HALF - 1; Jacobian kz / q times
      // the output scale
      const PairItem& it = item[u];
      const int kxs = it.kx < a.Mx / 2 ? it.kx : it.kx - a.Mx;
      const int kys = it.ky < a.My / 2 ? it.ky : it.ky - a.My;
      const double ax = a.sxk * kxs, ay = a.syk * kys;
      const double Ad = ax * ax + ay * ay;
      const float A = (float)Ad;
      // the last kz inside the frequency grid, q = sqrt(A + kz^2) <= HALF - 1, decided in FP64
      // once per column as in the FP64 definition (an FP32 q^2 can flip it for tiny A)
      const double rem = double((HALF - 1) * (HALF - 1)) - Ad;
      int kzmax = rem < 0.0 ? -1 : (int)sqrt(rem);
      if (kzmax >= 0 && double(kzmax) * kzmax > rem) --kzmax;
      if (double(kzmax + 1) * (kzmax + 1) <= rem) ++kzmax;
      // a column without a mirror (its own mirror) stores its own remap twice
      const bool mir = it.has_mirror;
      unsigned int* o1 = outb + (long long)it.ky * a.out_row + (long long)it.kx * a.nt + lane;
      unsigned int* o2 = mir ? outb + (long long)it.ky2 * a.out_row + (long long)it.kx2 * a.nt + lane : o1;
#pragma unroll
      for (int i = 0; i < HALF / 64; ++i) {
        const float kz = (float)(lane + 64 * i);
        const float q2 = fmaf(kz, kz, A);
        const float rq = __builtin_amdgcn_rsqf(q2);
        const float qv = q2 * rq;
        // q is clamped to HALF - 1 (a NaN, kz = 0 at kx = ky = 0, also gives HALF - 1, with a
        // zero Jacobian)
        const int kzi = lane + 64 * i;
        const bool inside = kzi > 0 && kzi <= kzmax;
        const float qc = fminf(qv, (float)(HALF - 1));
        const float fl = floorf(qc);
        const int i0 = (int)fl;
        const float fr = qc - fl;
        const float jac = inside ? kz * oscale * rq : 0.f;
        const float2 s0 = my[i0], s1 = my[i0 + 1];
        const float2 m1 = my[N - 1 - i0], m0 = my[N - i0];
        const float ar = fmaf(fr, s1.x - s0.x, s0.x) * jac, ai = fmaf(fr, s1.y - s0.y, s0.y) * jac;
        const float br = fmaf(fr, m1.x - m0.x, m0.x) * jac, bi = -fmaf(fr, m1.y - m0.y, m0.y) * jac;
        const unsigned int pa = M::pack(ar, ai);
        st_u32_nt(o1 + 64 * i, pa);
        st_u32_nt(o2 + 64 * i, mir ? M::pack(br, bi) : pa);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// z-IFFT of 1024-point columns (512 stored samples, 512 outputs kept), |.|^2, max
// ---------------------------------------------------------------------------

// VOL: the volume is written (a.out not null).  A line past the end (in the last group)
// stands in for the group's first line, as in fk_column_pair_mfma.
template <int SP, bool VOL>
__global__ __launch_bounds__(256, 3) void zfft_abs2_mfma(ContigArgs a, const mf_u4* __restrict__ tb1,
                                                      const mf_u4* __restrict__ ta3,
                                                      const float2* __restrict__ twt) {
  using M = Mfma<SP>;
  __shared__ float2 tl[16 * 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j = lane & 31, hl = lane >> 5;
  col1024_twiddles(tl, twt, true);
  mf_u4 B1[2][2];
  load_b1(B1, tb1, lane);
  mf_u4 A3[4];  // output block 0: z = j + 32 k1, k1 < 16
#pragma unroll
  for (int q = 0; q < 4; ++q) A3[q] = ta3[q * 64 + lane];
  // the first product is scaled by 1/32 (FP16 range); FP16 values carry 2^e_in
  const int e = SP == SP_F16 ? *a.e_in : 0;
  const float sc = ldexpf(32.f, -e);
  __syncthreads();
  const unsigned int* inb = static_cast<const unsigned int*>(a.in);
  float* vol = static_cast<float*>(a.out);
  const long long ngroups = (a.nlines + 7) / 8;
  // the next group's lines are loaded while this group is transformed
  unsigned int nraw[2][2][4];
  auto fetch = [&](long long g) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const long long ln = g * 8 + 4 * u + wv;
      const unsigned int* in = inb + (ln < a.nlines ? ln : g * 8) * a.in_line + j;
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) nraw[u][q][r] = ld_u32_nt(in + 32 * (8 * q + 4 * hl + r));
    }
  };
  if ((long long)blockIdx.x < ngroups) fetch(blockIdx.x);
  __builtin_amdgcn_s_waitcnt(0);  // tables and the first group before the loop
  for (long long g = blockIdx.x; g < ngroups; g += gridDim.x) {
    unsigned int raw[2][2][4];
    long long line[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      line[u] = g * 8 + 4 * u + wv < a.nlines ? g * 8 + 4 * u + wv : g * 8;
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) raw[u][q][r] = nraw[u][q][r];
    }
    if (g + gridDim.x < ngroups) fetch(g + gridDim.x);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      mf_u4 B3[4];
      col1024_first<SP>(B1, tl, lane, raw[u], B3);
      mf_acc d = {};
#pragma unroll
      for (int q = 0; q < 4; ++q) d = M::mma(A3[q], B3[q], d);
      float mx = 0.f;
      float* vrow = VOL ? vol + line[u] * a.out_line + j : nullptr;
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        const float re = d[jj] * sc, im = d[jj + 8] * sc;
        const float v = (re * re + im * im) * a.oscale;
        mx = fmaxf(mx, v);
        if constexpr (VOL) vrow[32 * mf_out_index(jj, hl)] = v;
      }
      if (a.img != nullptr) {
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
        if (lane == 0) atomicMax(reinterpret_cast<unsigned int*>(a.img) + line[u], __float_as_uint(mx));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

bool mfma_strided_ok(int n, int sp, const StridedArgs& a) {
  return sp != SP_F32 && (n == 256 || n == 512) && a.ncols > 0 && a.ncols % kMfT == 0 &&
         (a.n_in == n || 2 * a.n_in == n) && (a.n_out == n || 2 * a.n_out == n);
}

hipError_t launch_strided_mfma(int n, bool inverse, const StridedArgs& a, int nplanes, const MfmaTables& t,
                               const float2* tw, hipStream_t s, int sp) {
  if (!mfma_strided_ok(n, sp, a)) return hipErrorInvalidValue;
  const int bf = sp == SP_BF16 ? 1 : 0;
  const int scaled = (inverse && sp == SP_F16) ? 1 : 0;  // FP16 inverse: outputs carry 2^-log2(N) more
  const mf_u4* t1 = static_cast<const mf_u4*>(t.a16[inverse][scaled][bf]);
  const mf_u4* t3 = static_cast<const mf_u4*>(n == 512 ? t.a32[inverse][scaled][bf] : t.a16[inverse][scaled][bf]);
  const int tiles_x = a.ncols / kMfT;
  const dim3 grid((unsigned)((long long)tiles_x * nplanes));
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(64 * kMfW), 0, s, a, t1, t3, tw, tiles_x);
    return hipGetLastError();
  };
  if (n == 512) {
    if (sp == SP_F16) return inverse ? go(strided_fft_mfma<512, true, SP_F16>) : go(strided_fft_mfma<512, false, SP_F16>);
    return inverse ? go(strided_fft_mfma<512, true, SP_BF16>) : go(strided_fft_mfma<512, false, SP_BF16>);
  }
  if (sp == SP_F16) return inverse ? go(strided_fft_mfma<256, true, SP_F16>) : go(strided_fft_mfma<256, false, SP_F16>);
  return inverse ? go(strided_fft_mfma<256, true, SP_BF16>) : go(strided_fft_mfma<256, false, SP_BF16>);
}

bool mfma_column_ok(int mt, int nt, int sp, const FkPairArgs& a) {
  return sp != SP_F32 && mt == kColN && nt == kColN / 2 && a.tscale_in == 0.f;
}

hipError_t launch_fk_column_pair_mfma(const FkPairArgs& a, const MfmaTables& t, const float2* tw, float oscale,
                                      hipStream_t s, int sp) {
  const int bf = sp == SP_BF16 ? 1 : 0;
  const mf_u4* tb1 = static_cast<const mf_u4*>(t.b32[0][0][bf]);
  const mf_u4* ta3 = static_cast<const mf_u4*>(t.a32[0][0][bf]);
  const long long groups = (a.nwork + 7) / 8;
  const unsigned grid = (unsigned)(groups < 2048 ? groups : 2048);
  if (sp == SP_F16)
    hipLaunchKernelGGL(fk_column_pair_mfma<SP_F16>, dim3(grid), dim3(256), 0, s, a, tb1, ta3, tw, oscale);
  else
    hipLaunchKernelGGL(fk_column_pair_mfma<SP_BF16>, dim3(grid), dim3(256), 0, s, a, tb1, ta3, tw, oscale);
  return hipGetLastError();
}

bool mfma_zfft_ok(int mt, int sp, const ContigArgs& a) {
  return sp != SP_F32 && mt == kColN && a.n_in == kColN / 2 && a.n_out == kColN / 2;
}

hipError_t launch_zfft_abs2_mfma(const ContigArgs& a, const MfmaTables& t, const float2* tw, hipStream_t s, int sp) {
  const int bf = sp == SP_BF16 ? 1 : 0;
  const mf_u4* tb1 = static_cast<const mf_u4*>(t.b32[1][1][bf]);   // inverse, scaled by 1/32
  const mf_u4* ta3 = static_cast<const mf_u4*>(t.a32[1][0][bf]);   // inverse, unscaled, block 0
  const long long blocks = (a.nlines + 7) / 8;
  const unsigned grid = (unsigned)(blocks < 2048 ? blocks : 2048);
  auto k = sp == SP_F16 ? (a.out ? zfft_abs2_mfma<SP_F16, true> : zfft_abs2_mfma<SP_F16, false>)
                        : (a.out ? zfft_abs2_mfma<SP_BF16, true> : zfft_abs2_mfma<SP_BF16, false>);
  hipLaunchKernelGGL(k, dim3(grid), dim3(256), 0, s, a, tb1, ta3, tw);
  return hipGetLastError();
}

}  // namespace nlos
