// Internal declarations shared by the host API (nlos_api.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstddef>
#include <cstdint>

namespace nlos {

// Blocks of kernel K (launched with `threads` threads) resident on the whole current
// device at once, CUs times blocks per CU from the occupancy query, cached per kernel and
// device; 0 if the runtime cannot tell.  Sizes the grids of the kernels whose blocks stay
// resident and walk work items.
template <auto K>
inline long long resident_blocks(int threads) {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 0;
  if (dev < 64) {
    const int v = cache[dev].load(std::memory_order_relaxed);
    if (v > 0) return v;
  }
  int cus = 0, per = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, K, threads, 0) != hipSuccess || cus <= 0 || per <= 0)
    return 0;
  if (dev < 64) cache[dev].store(cus * per, std::memory_order_relaxed);
  return (long long)cus * per;
}

// storage precision of complex intermediates (float2, __half2, __hip_bfloat162)
enum { SP_F32 = 0, SP_F16 = 1, SP_BF16 = 2 };

// strided_fft load / store modes
enum { LD_C64 = 0, LD_TAU_SCALED = 1 };
enum { ST_C64 = 0, ST_ABS2_IMG = 1, ST_ABS_IMG = 2, ST_C64_SCALED = 3 };
// contig_fft load / store modes
// CL_REAL_PAIR: line ln is two real lines, 2 ln (real part) and 2 ln + 1 (imaginary part,
// zero beyond nreal), split again by the CS_BINS store
enum { CL_C64 = 0, CL_REAL = 1, CL_REAL_PAIR = 2 };
enum { CS_C64 = 0, CS_ABS_IMG = 1, CS_BINS = 2, CS_ABS2_MAX = 3 };

// Lines along a strided axis.  Element n of line `col` in plane `plane` is at
// in[plane * in_plane + n * in_line + col]; n < n_in are read (the rest are the
// zero padding), n < n_out are written.
struct StridedArgs {
  const void* in;
  void* out;
  long long in_plane, in_line;
  long long out_plane, out_line;
  int ncols, n_in, n_out;
  float tscale;        // LD_TAU_SCALED: the sample in column t is scaled by t * tscale
  float oscale;        // ST_ABS2_IMG: |v|^2 * oscale; ST_ABS_IMG: |v| * oscale; ST_C64_SCALED: v * oscale
  float* img;          // ST_ABS*_IMG: img[plane * img_plane + n] = max over columns (may be null)
  long long img_plane;
  // four-byte storage (SP_F16 / SP_BF16): an FP16 input holds value * 2^(*e_in) and an
  // FP16 output is written as value * 2^(*e_out); BF16 is unscaled.  e_per_col: one
  // exponent per column instead, e_in[col] / e_out[col] (per-plane scales)
  const int* e_in;
  const int* e_out;
  int e_per_col;
};

// Lines along the contiguous axis: line `ln` is in[ln * in_line + n], n < n_in.
struct ContigArgs {
  const void* in;
  void* out;
  long long nlines, in_line, out_line;
  int n_in, n_out;
  float oscale;        // CS_ABS_IMG: output = |v| * oscale; CS_ABS2_MAX: |v|^2 * oscale
  float* img;          // CS_ABS_IMG: img[(ln % img_lines) * out_line + n] = max over lines;
                       // CS_ABS2_MAX: img[ln] = max over the line
  long long img_lines;
  const int* bins;     // CS_BINS: out[ln * out_line + f] = X[bins[f]], f < nbins
  int nbins;
  const int* e_in;     // FP16 input: holds value * 2^(*e_in)
  const int* e_out;    // CS_BINS with FP16 output: written as value * 2^(*e_out)
  long long nreal;     // CL_REAL_PAIR: number of real input lines (nlines = ceil(nreal / 2))
};

// f-k pass 1: tau[ny][nx][nt] (float) -> half spectrum out[ny][Mx/2 + 1][nt] with
// plane (y) stride out_plane, two real t-columns per complex line.
struct FkXArgs {
  const float* tau;
  void* out;           // float2 or four-byte complex
  long long out_plane;
  int nx, nt;
  float tscale;        // 1 / (nt - 1)
  const int* e_out;    // FP16 output: written as value * 2^(*e_out)
  int unscaled;        // 1: plain x-FFT of tau (no t/(nt-1) factor, which then comes later)
};

// f-k pass 3: input half spectrum in[ky][kx <= Mx/2][nt] (row stride in_row), output full
// spectrum columns out[ky][kx][nt] (row stride out_row); nwork paired work items.
struct FkPairArgs {
  const void* in;      // float2 or four-byte complex
  void* out;
  long long in_row, out_row, nwork;
  int nt, Mx, My;
  double sxk, syk;     // Stolt coordinate per signed kx, ky in units of the t bins
  float norm;          // 1 / (Mx My Mt)
  const int* e_in;     // FP16: input holds value * 2^(*e_in), output is written
  const int* e_out;    // as value * 2^(*e_out)
  float tscale_in;     // non-zero: input sample t is first multiplied by t * tscale_in
};

// Mixture of experts, phasors from the shared spatial half spectrum: for each column
// pair of in[ky][kx <= Mx/2][nt] (row stride in_row), the nt-point DFT of the column
// gives out[ky * Mx + kx][f] = X[bins[f]] and, for the mirror column (-kx, -ky) of the
// real input, out[.][f] = conj X[nt - bins[f]].
struct MoePhasorArgs {
  const float2* in;
  float2* out;         // [My * Mx][nbins]
  long long in_row, nwork;
  int nt, Mx, My, nbins;
  const int* bins;
};

// One rounding to nearest even of v to binary16 / bfloat16 (host), as stored bits.
uint16_t to_f16_bits(double v);
uint16_t to_bf16_bits(double v);

// Radial propagation over chunks of pixels that share the lower radial bin.
struct RsdPropArgs {
  const void* Ph;          // [npix][Nf] spectra of the padded phasor planes (float2, or
                           // four-byte pairs when data_sp != SP_F32)
  const void* Kr;          // [Nrho][Nf][Nd] radial kernel, float2 or (re, im) FP16 / BF16 pairs
  const float2* w;         // [Nf] complex frequency weights
  void* C;                 // [npix][Nd] propagated spectra (float2 or four-byte pairs)
  const int* chunk_i0;     // [nchunks] lower radial bin (-1: all-zero chunk)
  const int* chunk_pix;    // [nchunks][64] pixel index or -1
  const float* chunk_wa;   // [nchunks][64] a (1 - alpha), 0 in unused slots
  const float* chunk_wb;   // [nchunks][64] a alpha, 0 in unused slots
  long long nchunks;
  int Nf, Nd;
  int ph_stride, c_stride;  // elements between the pixel rows of Ph and of C
  int cut_idx;
  int kernel_sp;           // SP_F32, SP_F16 or SP_BF16: storage of Kr
  int data_sp;             // storage of Ph and C (four-byte forms: matrix cores, data_sp ==
                           // kernel_sp); FP16 Ph holds value * 2^e_ph[0], FP16 C[.][d] is
                           // written as value * 2^e_c[d]
  const int* e_ph;
  const int* e_c;
  int mfma;                // propagation on the matrix cores: 0 no (FP32 FMAs), 1 yes, 2 yes
                           // with the other depth tiling (FP32: two 32-depth tiles per wave,
                           // FP16 / BF16: one)
};

// stream: non-temporal loads and stores (FP32 LD_C64 -> ST_C64 only; ignored otherwise)
hipError_t launch_strided(int n, bool inverse, int ld, int st, const StridedArgs& a, int nplanes,
                          const float2* tw, hipStream_t s, int sp = 0, bool stream = false);
hipError_t launch_contig(int n, bool inverse, int ld, int st, const ContigArgs& a,
                         const float2* tw, hipStream_t s, int sp = 0);
hipError_t launch_fk_xr2c(int n, const FkXArgs& a, int ny, const float2* tw, hipStream_t s, int sp = 0);
hipError_t launch_fk_column_pair(int n, const FkPairArgs& a, const float2* tw, hipStream_t s, int sp = 0);

// General-length lines (FP32 only): n even, n <= kGenMaxN, prime factors 2, 3, 5, 7, 11,
// 13; the radices of the Stockham stages and a table of W_n^k (k < n, FP64-generated).
constexpr int kGenMaxStages = 12;
constexpr int kGenMaxN = 4096;
struct GenPlan {
  int n, nstage;
  int radix[kGenMaxStages];
  const float2* tw;  // device, W_n^k = exp(-2 pi i k / n), k in [0, n)
};
// host: radix plan of n (tw left null); false when n is not supported
bool gen_plan_radices(int n, GenPlan* g);
// the same passes as launch_strided (LD_C64 with ST_C64, ST_C64_SCALED or ST_ABS_IMG),
// launch_contig (CL_C64 or CL_REAL with CS_C64, CS_ABS2_MAX, CS_BINS or CS_ABS_IMG),
// launch_fk_xr2c and launch_fk_column_pair (no input t-scaling), for lines of length g.n
hipError_t launch_gen_strided(const GenPlan& g, bool inverse, int st, const StridedArgs& a, int nplanes,
                              hipStream_t s);
hipError_t launch_gen_contig(const GenPlan& g, bool inverse, int ld, int st, const ContigArgs& a, hipStream_t s);
hipError_t launch_gen_xr2c(const GenPlan& g, const FkXArgs& a, int ny, hipStream_t s);
hipError_t launch_gen_column_pair(const GenPlan& g, const FkPairArgs& a, hipStream_t s);
hipError_t launch_moe_phasor_pair(const MoePhasorArgs& a, const float2* tw, hipStream_t s);
// coherence-weighted merging over a ring of `window` complex frames of n values:
// writes `frame` into ring slot `slot`, then sums the `count` most recent frames (ring
// slots first, first + 1, ... mod window, oldest first)
hipError_t launch_merge(const float2* frame, float2* ring, long long n, int window, int slot, int first,
                        int count, float eps, float* merged, float* coherence, hipStream_t s);
// Depth-dependent average: stores vol (nvox x nd, depth fastest) into ring slot `slot` and
// averages the `count` newest frames with weights w[nd][window] (avg, img nullable).
hipError_t launch_dda(const float* vol, float* ring, const float* w, long long nvox, int nd, int window, int slot,
                      int count, float* avg, float* img, hipStream_t s);
// img = max-normalised fk_img * (max-normalised rsd_img + eps)^beta, max-normalised
// (images of n pixels; mx: 3 words of device scratch)
hipError_t launch_moe_mix(const float* fk_img, const float* rsd_img, float* img, int n, float beta,
                          float eps, unsigned int* mx, hipStream_t s);

// FP16 storage scales of the f-k intermediates from the bound B = sum |tau| t/(nt-1)
// (nt a power of two): partials[kScaleBlocks] scratch, exps[4] = the exponents of
// W1/W2, W3, W4, W5; l_norm = log2(Mx My Mt), l_first_inv / l_second_inv = log2 of the
// length of the first (x, Mx) and second (y, My) inverse pass.
constexpr int kScaleBlocks = 1024;
hipError_t launch_fk_scales(const float* tau, long long n, int nt, float* partials, int* exps,
                            int l_norm, int l_first_inv, int l_second_inv, hipStream_t s);
hipError_t launch_rsd_propagate(const RsdPropArgs& a, hipStream_t s);
// FP16 storage scales of the RSD intermediates from L = sum |tau| (n values, n even):
// exps[0] for P, X and P^ (bound L), exps[1 + d] for C at depth d (bound L kappa[d]) and
// exps[1 + nd + d] for D (bound My L kappa[d], l_my = log2 My); partials[kScaleBlocks].
hipError_t launch_rsd_scales(const float* tau, long long n, float* partials, const float* kappa, int nd, int l_my,
                             int* exps, hipStream_t s);

// Constant operands of the matrix-core DFT stages (mfma_fft.hpp), per context, indexed
// [inverse][scaled by 1/R][0 binary16, 1 bfloat16]; 64 lanes x 16 bytes per operand.
//   a16: radix-16 DFT matrix as the A operand (outputs along rows), 2 operands (K steps);
//   a32: radix 32 as A, 8 operands: output block b (outputs 16 b..16 b + 15), K step q at b * 4 + q;
//   b32: radix 32 as the B operand (outputs along columns), 8 operands: part c (0 re,
//        1 im) of outputs 0..31, K step q at c * 4 + q.
struct MfmaTables {
  const void* a16[2][2][2];
  const void* a32[2][2][2];
  const void* b32[2][2][2];
};
hipError_t mfma_tables_create(int device, void** d_buf, MfmaTables* t);

// Matrix-core passes of the four-byte f-k storage (k_mfma.hip) and the shapes they take:
// strided lines of 256 or 512 points over a multiple of 32 columns with n_in, n_out in
// {N/2, N}; 1024-point columns with 512 stored samples.  FP16 inverse strided passes
// return values carrying 2^-log2(N) times their input's factor (the next intermediate's).
bool mfma_strided_ok(int n, int sp, const StridedArgs& a);
hipError_t launch_strided_mfma(int n, bool inverse, const StridedArgs& a, int nplanes, const MfmaTables& t,
                               const float2* tw, hipStream_t s, int sp);
bool mfma_column_ok(int mt, int nt, int sp, const FkPairArgs& a);
// oscale: 1/(Mx My Mt) times 2^(e_out - e_in) (FP16: 1; BF16: 1/(Mx My Mt))
hipError_t launch_fk_column_pair_mfma(const FkPairArgs& a, const MfmaTables& t, const float2* tw, float oscale,
                                      hipStream_t s, int sp);
bool mfma_zfft_ok(int mt, int sp, const ContigArgs& a);
hipError_t launch_zfft_abs2_mfma(const ContigArgs& a, const MfmaTables& t, const float2* tw, hipStream_t s, int sp);

// Every device allocation of the library goes through dev_alloc and every host allocation
// point calls host_alloc_point (it throws std::bad_alloc, caught at the C boundary), so
// that nlos_debug_fail_allocations can make the next allocations fail.
hipError_t dev_alloc(void** p, size_t bytes);
void host_alloc_point();

// Static device scratch of the allocation-free entry points (k_scratch.hip): its size,
// and its device address on `device` (looked up once per device with that device
// current, then cached; the array's name itself is never passed to a kernel).
constexpr size_t kStaticScratchBytes = size_t(128) << 20;
hipError_t static_scratch_address(int device, void** out);
hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t value, hipStream_t s);
// out[c][r] = in[r][c] for r < rows, c < cols (float)
hipError_t launch_transpose_f32(const float* in, float* out, long long rows, int cols, hipStream_t s);
hipError_t launch_u32_to_f32(const uint32_t* in, float* out, size_t n, hipStream_t s);
hipError_t launch_bin(const void* events, unsigned long long n, uint32_t* hist,
                      unsigned long long* dropped, int npix, int nt, uint32_t bin_ps, uint32_t t0,
                      hipStream_t s);
// Binning by pixel tiles (each chunk sorted by tile into runs, then one LDS histogram per
// tile gathered from every chunk's run) into workspace ws of
// bin_workspace_bytes (0: the tiled path does not apply to this shape); every bin of hist is
// written (added to when accumulate), so no clearing pass is needed.
size_t bin_workspace_bytes(int npix, int nt, unsigned long long n);
hipError_t launch_bin_tiled(const void* events, unsigned long long n, uint32_t* hist, unsigned long long* dropped,
                            int npix, int nt, uint32_t bin_ps, uint32_t t0, int accumulate, void* ws, hipStream_t s);
// P[pixel][f] += W_nt^(bins[f] b) per valid event (nt <= 2048, lut = W_nt^m, m < nt)
hipError_t launch_phasor_bin(const void* events, unsigned long long n, float2* P, unsigned long long* dropped,
                             int npix, int nt, uint32_t bin_ps, uint32_t t0, const float2* lut, const int* bins,
                             int nf, hipStream_t s);

}  // namespace nlos
