/*
 * nlos.h -- C ABI of the MI355X NLOS reconstruction library (libnlos.so).
 *
 * Three operations of wave-based non-line-of-sight reconstruction, after
 * López-Ruiz & Royo, "Memory-efficient GPU pipelines for real-time
 * non-line-of-sight reconstruction":
 *   nlos_bin  -- photon events -> transient histogram (Section 4.1, photon binner)
 *   nlos_fk   -- f-k migration of a confocal transient (Section 3.1 Eq. 1-2,
 *                Section 4.2, Algorithms 1-2 of the supplementary material)
 *   nlos_rsd  -- phasor-field RSD with the radial kernel (Section 4.3 Eq. 4-7,
 *                supplementary sampling rules, Listing 3, Algorithm 4)
 *
 * Conventions shared by every entry point
 *   - Only plain C types cross this interface.  Pointers named d_* are device
 *     (HBM) pointers on the context's device; every other pointer is host memory.
 *   - The caller owns every buffer it passes (inputs, outputs, workspace) and
 *     keeps it alive until the stream work completes.  Plans own their device
 *     tables; a context owns its workspace pool and its twiddle table.
 *   - Every call returns an nlos_status and never throws.  Arguments are
 *     validated on the host before anything is enqueued; on an error nothing is
 *     enqueued and nlos_last_error() describes the failure.
 *   - Compute calls are asynchronous: they enqueue kernels on the context's HIP
 *     stream and return.  A context is not thread safe; use one per host thread.
 *   - Volumes are row-major with the last index contiguous.  A transient is
 *     tau[ny][nx][nt] (time contiguous, scan point y*nx + x).  Complex values are
 *     interleaved (re, im).  Results are deterministic: the same inputs give
 *     bitwise-equal outputs, also when other work runs concurrently.
 */
#ifndef NLOS_H
#define NLOS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NLOS_OK = 0,
  NLOS_ERR_INVALID_ARG = 1,   /* null pointer, non-positive size, bad enum, value out of range */
  NLOS_ERR_UNSUPPORTED = 2,   /* valid request outside what the library implements */
  NLOS_ERR_OUT_OF_MEMORY = 3, /* device allocation failed, or workspace too small */
  NLOS_ERR_DEVICE = 4,        /* HIP runtime or launch failure */
  NLOS_ERR_INTERNAL = 5
} nlos_status;

typedef enum { NLOS_FP32 = 0, NLOS_FP16 = 1, NLOS_BF16 = 2 } nlos_precision;

typedef struct nlos_ctx nlos_ctx;
typedef struct nlos_fk_plan nlos_fk_plan;
typedef struct nlos_rsd_plan nlos_rsd_plan;
typedef struct nlos_moe_plan nlos_moe_plan;
typedef struct nlos_phasor_plan nlos_phasor_plan;
typedef struct nlos_merge nlos_merge;
typedef struct nlos_dda nlos_dda;
typedef struct nlos_graph nlos_graph;

/* ------------------------------------------------------------------------ */
/* Context                                                                   */
/* ------------------------------------------------------------------------ */

/* Binds HIP device `device` and stream `hip_stream` (a hipStream_t; NULL means
 * the null stream), uploads the FP64-generated twiddle table.  *out is set on
 * NLOS_OK only.  NLOS_ERR_DEVICE if the device cannot be used. */
nlos_status nlos_create(int device, void *hip_stream, nlos_ctx **out);
/* Frees the context's pool and tables (waits for its stream first).  NULL is a no-op. */
nlos_status nlos_destroy(nlos_ctx *ctx);
/* Waits for the work already enqueued on the current stream (the context's
 * workspace pool is ordered by it), then later calls on ctx enqueue on hip_stream. */
nlos_status nlos_set_stream(nlos_ctx *ctx, void *hip_stream);
/* Static text for a status code. */
const char *nlos_status_string(nlos_status s);
/* Detail of the last failure on ctx ("" if none); valid until the next call on ctx. */
const char *nlos_last_error(const nlos_ctx *ctx);
/* Library ABI version (major * 100 + minor). */
int nlos_version(void);

/* Per-pass timing, a profiling aid.  While enabled, every kernel launch of
 * nlos_bin / nlos_fk / nlos_rsd on ctx is bracketed by two HIP events on the
 * context's stream (the only cost is the two event records per launch). */
typedef enum {
  NLOS_PASS_FILL = 0,          /* zero fill of an output (histogram, image) */
  NLOS_PASS_BIN = 1,           /* event binning */
  NLOS_PASS_FK_X = 2,          /* f-k pass 1: x-FFT with time scaling and zero padding */
  NLOS_PASS_FK_Y = 3,          /* f-k pass 2: y-FFT */
  NLOS_PASS_FK_COLUMN = 4,     /* f-k pass 3: t-FFT and Stolt remap per column */
  NLOS_PASS_FK_YI = 5,         /* f-k pass 5: y-IFFT */
  NLOS_PASS_FK_XI = 6,         /* f-k pass 4: x-IFFT (runs before the y-IFFT) */
  NLOS_PASS_RSD_PHASOR = 7,    /* RSD: temporal DFT to the selected frequencies */
  NLOS_PASS_RSD_X = 8,         /* RSD: x-FFT of the padded phasor planes */
  NLOS_PASS_RSD_Y = 9,         /* RSD: y-FFT */
  NLOS_PASS_RSD_PROPAGATE = 10,/* RSD: radial-kernel propagation */
  NLOS_PASS_RSD_YI = 11,       /* RSD: y-IFFT per depth */
  NLOS_PASS_RSD_XI = 12,       /* RSD: x-IFFT, |.|, max over depth */
  NLOS_PASS_FK_ZI = 13,        /* f-k pass 6: z-IFFT, |.|^2, max over depth */
  NLOS_PASS_FK_SCALE = 14,     /* f-k FP16 storage scales from the input bound */
  NLOS_PASS_MOE_PHASOR = 15,   /* mixture of experts: RSD phasors from the shared spectrum */
  NLOS_PASS_MOE_MIX = 16,      /* mixture of experts: Eq. 10 on the branch images */
  NLOS_PASS_PHASOR_BIN = 17,   /* phasors straight from photon records */
  NLOS_PASS_MERGE = 18,        /* coherence-weighted temporal merging */
  NLOS_PASS_DDA = 19,          /* depth-dependent temporal average */
  NLOS_PASS_RSD_SCALE = 20,    /* RSD FP16 storage scales from the input bound */
  NLOS_PASS_COUNT = 21
} nlos_pass;

/* Turns per-pass timing on (1) or off (0) for later calls on ctx. */
nlos_status nlos_timing_enable(nlos_ctx *ctx, int enable);
/* Waits for the context's stream, then writes, for every pass p < n (n at most
 * NLOS_PASS_COUNT), the total milliseconds and the number of launches recorded
 * since the previous read into ms[p] and count[p], and clears the record. */
nlos_status nlos_timing_read(nlos_ctx *ctx, double *ms, int *count, int n);
/* Static name of a pass ("fk_column", ...), or "?" when out of range. */
const char *nlos_pass_name(int pass);

/* ------------------------------------------------------------------------ */
/* Photon-event binning (Section 4.1: GPU histogramming of photon records)   */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t pixel;   /* scan point y*nx + x */
  uint32_t t_ps;   /* arrival time, picoseconds from the laser hitting the wall point */
} nlos_event;

typedef struct {
  int nx, ny, nt;     /* histogram shape [ny][nx][nt], each >= 1 */
  uint32_t bin_ps;    /* bin width, >= 1 */
  uint32_t t0_ps;     /* time of the left edge of bin 0 */
  int accumulate;     /* 0: d_hist is overwritten; 1: counts are added to it */
} nlos_bin_desc;

/* Host-only validation of a binning descriptor. */
nlos_status nlos_bin_check(const nlos_bin_desc *desc);

/* Histogram n_events events (AoS, 8 bytes each) into d_hist[ny][nx][nt] (uint32,
 * time contiguous).  An event is valid iff 0 <= pixel < nx*ny, t_ps >= t0_ps and
 * b = (t_ps - t0_ps) / bin_ps < nt (integer division, left-closed bins); it adds 1
 * to d_hist[pixel][b].  Invalid events add 1 to *d_dropped (a device uint64,
 * optional: NULL skips the count; it is zeroed first unless accumulate = 1).
 * n_events may be 0.  Counts wrap modulo 2^32 per bin.  Bit-exact and order
 * independent. */
nlos_status nlos_bin(nlos_ctx *ctx, const nlos_bin_desc *desc, const nlos_event *d_events,
                     uint64_t n_events, uint32_t *d_hist, unsigned long long *d_dropped);

/* Converts n binned counts (uint32, e.g. the output of nlos_bin) to float32
 * transient samples, d_tau[i] = (float)d_hist[i], so that a binned histogram can
 * feed nlos_fk / nlos_rsd.  Buffers may not overlap. */
nlos_status nlos_counts_to_float(nlos_ctx *ctx, const uint32_t *d_hist, float *d_tau, uint64_t n);

/* Phasors straight from photon records (Section 4.1, phasor binning, Listing 1): the
 * plan holds the table exp(-2 pi i m / nt) (FP64-built, nt <= 2048, else
 * NLOS_ERR_UNSUPPORTED) and the n_freq DFT bins freq_bin[f] in [0, nt) (host array,
 * copied).  Validation of desc as for nlos_bin. */
nlos_status nlos_phasor_plan_create(nlos_ctx *ctx, const nlos_bin_desc *desc, int n_freq, const int *freq_bin,
                                    nlos_phasor_plan **out);
nlos_status nlos_phasor_plan_destroy(nlos_phasor_plan *plan);
/* Every valid event (as in nlos_bin) in bin b of its pixel adds
 * exp(-2 pi i freq_bin[f] b / nt) to d_phasor[pixel][f] (float re, im pairs,
 * [ny][nx][n_freq], 8-byte aligned; zeroed first unless desc->accumulate), which is the
 * DFT at those bins of the histogram nlos_bin would build, up to rounding: hardware
 * float atomics, one wave per event with its lanes over the frequencies, so the order of
 * the sums (and the last bits) varies from run to run.  Dropped events are counted as
 * in nlos_bin.  Feeds nlos_rsd_from_phasors. */
nlos_status nlos_phasor_bin(nlos_ctx *ctx, const nlos_phasor_plan *plan, const nlos_event *d_events,
                            uint64_t n_events, float *d_phasor, unsigned long long *d_dropped);

/* ------------------------------------------------------------------------ */
/* f-k migration (Section 4.2; Algorithms 1-2)                               */
/* ------------------------------------------------------------------------ */

typedef struct {
  int nx, ny, nt;          /* transient shape [ny][nx][nt] */
  double wall_w_m;         /* scanned wall extent along x (m); dx = wall_w_m / nx */
  double wall_h_m;         /* along y (m); dy = wall_h_m / ny */
  double bin_ps;           /* time-bin width (ps) */
  int pad;                 /* 1 (no padding) or 2 (x2 zero padding on every axis) */
  nlos_precision prec;     /* storage of the complex intermediates (Section 4.2, data
                            quantization); arithmetic is FP32 in every case.
                            NLOS_FP32: 8-byte complex values.  NLOS_BF16: 4-byte, stored
                            as is (FP32's exponent range).  NLOS_FP16: 4-byte, each
                            intermediate stored times a power of two computed on the
                            device from the bound B = sum |tau| t/(nt-1) on its
                            magnitude (forward: B, Stolt output: B/(Mx My Mt), times M
                            per inverse axis), so stored values stay below 2^14;
                            requires a finite B */
} nlos_fk_desc;

/* Host-only validation: dims >= 1, nt >= 2, pad in {1, 2}, positive finite geometry;
 * each of pad*nx, pad*ny and pad*nt either a power of two in [8, 2048] or an even
 * length in [8, 4096] whose prime factors are 2, 3, 5, 7, 11 and 13 (the grids of the
 * paper's Table 4, e.g. 360 x 260 x 512 padded to 720 x 520 x 1024), else
 * NLOS_ERR_UNSUPPORTED.  Grids with any such general length run on FP32 storage only
 * (NLOS_FP16 / NLOS_BF16 there: NLOS_ERR_UNSUPPORTED); results meet the same FP32
 * accuracy as power-of-two grids. */
nlos_status nlos_fk_check(const nlos_fk_desc *desc);
/* Exact device workspace one nlos_fk call with a plan of this descriptor needs (host
 * only, no plan required): about half the FP32 figure for NLOS_FP16 / NLOS_BF16 (FP16 adds
 * 4.3 KB of scale scratch). */
nlos_status nlos_fk_desc_workspace_bytes(const nlos_fk_desc *desc, size_t *bytes);
nlos_status nlos_fk_plan_create(nlos_ctx *ctx, const nlos_fk_desc *desc, nlos_fk_plan **out);
nlos_status nlos_fk_plan_destroy(nlos_fk_plan *plan);
/* Exact device workspace one nlos_fk call on plan needs (host only; the same figure as
 * nlos_fk_desc_workspace_bytes of the plan's descriptor).  This is the size the serving
 * loop admits requests against. */
nlos_status nlos_fk_workspace_bytes(const nlos_fk_plan *plan, size_t *bytes);

/* f-k migration of d_tau[ny][nx][nt] (float32 counts):
 *   g = tau * t/(nt-1), zero-padded to My x Mx x Mt (M = pad * n);
 *   unnormalised 3D DFT; Stolt remap out = [Z>0] (Z/Z') lerp_w(S, Z') with
 *   Z' = sqrt(sx^2 X^2 + sy^2 Y^2 + Z^2), sx = c dt / (2 dx), sy = c dt / (2 dy),
 *   X, Y, Z the signed frequencies normalised to [-1, 1), zero beyond the last
 *   frequency sample; inverse 3D DFT normalised by 1/(Mx My Mt).
 * Writes d_vol[ny][nx][nt] = |Psi|^2 on the unpadded grid and d_img[ny][nx] =
 * max over depth of d_vol; either output may be NULL (not both).  d_ws is
 * 256-byte aligned device workspace of ws_bytes >= nlos_fk_workspace_bytes(plan)
 * (NULL: the context pool is used and grown as needed; misaligned:
 * NLOS_ERR_INVALID_ARG; too small: NLOS_ERR_OUT_OF_MEMORY).  d_tau must be 8-byte
 * aligned.  Inputs are not modified. */
nlos_status nlos_fk(nlos_ctx *ctx, const nlos_fk_plan *plan, const float *d_tau, float *d_vol,
                    float *d_img, void *d_ws, size_t ws_bytes);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): nlos_fk with the same arguments and
 * results (the same kernels and pass sequence, bitwise-equal outputs), whose workspace
 * is the library's static device scratch instead of a caller or pool buffer.  The call
 * allocates nothing and frees nothing.  The scratch is one file-scope device array of
 * NLOS_STATIC_SCRATCH_BYTES per GPU, held from the library's first use on that GPU
 * (nlos_create) until the process ends; its device address is looked up once per device.
 * Plans whose workspace (nlos_fk_workspace_bytes) exceeds it return NLOS_ERR_UNSUPPORTED
 * before anything is enqueued: 128 MiB holds e.g. 64 x 64 x 512 padded x2 in FP32 and
 * 128 x 128 x 256 padded x2 in FP16/BF16.  Every call on a GPU shares that GPU's array and
 * leaves its last contents there (nothing in it needs clearing between calls): calls that
 * overlap on one GPU -- from two streams, contexts or threads -- race and give undefined
 * results; order them (one stream, or events).  Per-pass timing does not cover it. */
#define NLOS_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
nlos_status nlos_fk_noalloc(nlos_ctx *ctx, const nlos_fk_plan *plan, const float *d_tau, float *d_vol,
                            float *d_img);

/* ------------------------------------------------------------------------ */
/* Phasor-field RSD with the radial kernel (Section 4.3; Algorithm 4)        */
/* ------------------------------------------------------------------------ */

typedef struct {
  int nx, ny, nt;          /* transient shape [ny][nx][nt] */
  double dx_m, dy_m;       /* wall sample spacing (m) */
  double bin_ps;           /* time-bin width (ps) */
  int pad;                 /* 1 or 2: the 2D FFT grid is My x Mx = pad*ny x pad*nx */
  int n_freq;              /* number of temporal frequencies, >= 1 */
  const int32_t *freq_bin; /* host [n_freq]: DFT bins of nt, each in [1, nt/2 - 1] */
  const float *w;          /* host [2*n_freq]: complex frequency weights (re, im) */
  int n_depth;             /* number of depth planes, in [1, 4096] */
  double depth0_m;         /* depth of plane 0 (m) */
  double depth_step_m;     /* spacing of the depth planes (m) */
  int sigma_s, sigma_t;    /* modality: (2, 0) confocal, (1, 1) non-confocal */
  double delta_m;          /* calibration offset of the optical path (m) */
  nlos_precision data_prec;   /* storage of the complex intermediates P, X, P^, C, D:
                                 NLOS_FP32 (8-byte complex) or NLOS_FP16 / NLOS_BF16
                                 (4-byte; needs kernel_prec == data_prec and power-of-two
                                 pad*nx, pad*ny, nt; FP16 values are stored times exact
                                 powers of two computed on the device from L = sum |tau|:
                                 one for P, X, P^ and one per depth plane for C and D,
                                 from the plan's per-depth kernel bound) */
  nlos_precision kernel_prec; /* storage of the radial kernel K_r: NLOS_FP32, or NLOS_FP16 /
                                 NLOS_BF16 (rounded once), whose propagation runs on the
                                 matrix cores with FP32 accumulation */
  int vol_depth_major;        /* layout of nlos_rsd's d_vol: 0 [ny][nx][n_depth] (depth
                                 contiguous, like the time axis of the transient); 1
                                 [n_depth][ny][nx] (a stack of depth planes), written by one
                                 more pass over the volume */
} nlos_rsd_desc;

/* Radial sampling of the supplementary material: r_max, rho_max, ring count
 * N_r (power of two >= ceil(2 sigma_s r_max / lambda_min) + 1, at least 2),
 * radius count N_rho (power of two >= ceil(2 r_max rho_max) + 1), ring spacing,
 * sampling rate f_s = (N_r - 1)/r_max, cutoff min(rho_max, f_s/2) and its bin
 * coordinate, and the clamped lookup bounds of Listing 3. */
typedef struct {
  double r_max, rho_max, lambda_min, dr, f_s, rho_cut, rho_cut_bin;
  int n_r_min, n_r, n_rho_min, n_rho, cut_idx, last_base;
} nlos_rsd_geometry;

/* Host-only validation: dims >= 1, pad in {1, 2}; pad*nx, pad*ny and nt each a power
 * of two in [8, 2048] or an even length in [8, 4096] with prime factors 2, 3, 5, 7, 11,
 * 13 (else NLOS_ERR_UNSUPPORTED); frequency bins in range, positive spacings, n_depth
 * in [1, 4096], sigma_s in {1, 2}; FP16 / BF16 data as stated at data_prec (else
 * NLOS_ERR_UNSUPPORTED). */
nlos_status nlos_rsd_check(const nlos_rsd_desc *desc);
/* Host-only: the radial sampling geometry of desc. */
nlos_status nlos_rsd_geometry_get(const nlos_rsd_desc *desc, nlos_rsd_geometry *out);
/* Host-only: builds the radial kernel of Eq. 6 in FP64 exactly as a plan does and
 * stores it as float (re, im) into out[n_rho][n_freq][n_depth][2]; n_floats must
 * be at least 2 * n_rho * n_freq * n_depth. */
nlos_status nlos_rsd_kernel_host(const nlos_rsd_desc *desc, float *out, size_t n_floats);
/* Exact device workspace one nlos_rsd call with a plan of this descriptor needs (host
 * only, no plan required). */
nlos_status nlos_rsd_desc_workspace_bytes(const nlos_rsd_desc *desc, size_t *bytes);
/* Builds K_r (Eq. 4-6, FP64 on the host, stored per kernel_prec), the pixel lookup
 * (radius map -> taper, interpolation bins and weights of Listing 3, pixels grouped by
 * radial bin) and the frequency tables, and uploads them to HBM. */
nlos_status nlos_rsd_plan_create(nlos_ctx *ctx, const nlos_rsd_desc *desc, nlos_rsd_plan **out);
nlos_status nlos_rsd_plan_destroy(nlos_rsd_plan *plan);
/* Exact device workspace one nlos_rsd call on plan needs (host only). */
nlos_status nlos_rsd_workspace_bytes(const nlos_rsd_plan *plan, size_t *bytes);

/* Radial RSD of d_tau[ny][nx][nt] (float32):
 *   P[f] = sum_t tau e^{-2 pi i k_f t / nt};  P^ = DFT2(P padded top-left);
 *   C[d](u,v) = sum_f w_f P^[f](u,v) a(rho) lerp(K_r[., f, d], rho(u,v)) with the
 *   smoothstep taper a over the last 8 radial bins below the cutoff;
 *   I[d] = IDFT2(C[d]) normalised by 1/(Mx My).
 * Writes d_vol = |I| on the unpadded grid, [ny][nx][n_depth] (depth contiguous, like the
 * time axis of the transient) or, with desc->vol_depth_major, [n_depth][ny][nx], and
 * d_img[ny][nx] = max over depth; either may be NULL (not both).  Workspace as for nlos_fk.
 * FP16 data plans need d_tau 8-byte aligned (NLOS_ERR_INVALID_ARG otherwise). */
nlos_status nlos_rsd(nlos_ctx *ctx, const nlos_rsd_plan *plan, const float *d_tau, float *d_vol,
                     float *d_img, void *d_ws, size_t ws_bytes);
/* nlos_rsd from phasors already at the plan's frequencies: d_phasor[ny][nx][n_freq]
 * complex (float re, im; e.g. from nlos_phasor_bin with the same bins), read only.  FP32
 * data plans only (NLOS_ERR_UNSUPPORTED otherwise: the FP16 scales are bounds of the
 * transient). */
nlos_status nlos_rsd_from_phasors(nlos_ctx *ctx, const nlos_rsd_plan *plan, const float *d_phasor, float *d_vol,
                                  float *d_img, void *d_ws, size_t ws_bytes);

/* ------------------------------------------------------------------------ */
/* Mixture of experts of f-k and RSD (Section 4.4, Eq. 10)                   */
/* ------------------------------------------------------------------------ */

/* Host-only validation: both descriptors valid, describing the same transient and grid
 * (nx, ny, nt, pad, bin_ps equal; dx_m = wall_w_m / nx, dy_m = wall_h_m / ny to 1e-9
 * relative), FP32 intermediates (kernel_prec may be FP16), power-of-two padded sizes
 * (else NLOS_ERR_UNSUPPORTED), beta >= 0, eps > 0. */
nlos_status nlos_moe_check(const nlos_fk_desc *fk, const nlos_rsd_desc *rsd, double beta, double eps);
/* Exact device workspace of one nlos_moe call: the f-k and RSD workspaces plus two
 * images (host only). */
nlos_status nlos_moe_workspace_bytes(const nlos_fk_desc *fk, const nlos_rsd_desc *rsd, size_t *bytes);
/* Builds both branch plans (see nlos_fk_plan_create, nlos_rsd_plan_create).
 * shared_spectrum = 1 selects the paper's schedule: both branches read one spatial
 * spectrum of the transient and run concurrently on two streams.  0 runs the two
 * complete reconstructions one after the other on the context stream; it reads the
 * 4-byte transient for the RSD phasors instead of the padded complex half spectrum and
 * measured 1-3 % faster at 128x128x1024 and 256x256x512. */
nlos_status nlos_moe_plan_create(nlos_ctx *ctx, const nlos_fk_desc *fk, const nlos_rsd_desc *rsd, double beta,
                                 double eps, int shared_spectrum, nlos_moe_plan **out);
nlos_status nlos_moe_plan_destroy(nlos_moe_plan *plan);

/* Both reconstructions of d_tau[ny][nx][nt], then the mixture.  With a shared spectrum
 * the RSD branch runs on a second stream of the context (created on first use, default
 * priority), joined before the mixture, and the x and y DFTs of the
 * zero-padded transient run once: the RSD branch takes its phasors from that spectrum
 * (temporal DFT at the plan's bins, the mirror columns from the Hermitian symmetry of
 * the real input) and the f-k branch applies t/(nt-1) as it loads the spectrum's
 * columns.  Writes
 *   d_img[ny][nx]     = m / max m,  m = (F / max F) * (R / max R + eps)^beta,
 *   d_img_fk[ny][nx]  = F, the f-k image (max over depth of |Psi|^2; nullable),
 *   d_img_rsd[ny][nx] = R, the RSD image (max over depth of |I|; nullable);
 * an all-zero image stays zero.  Workspace as for nlos_fk. */
nlos_status nlos_moe(nlos_ctx *ctx, const nlos_moe_plan *plan, const float *d_tau, float *d_img,
                     float *d_img_fk, float *d_img_rsd, void *d_ws, size_t ws_bytes);

/* ------------------------------------------------------------------------ */
/* Complex fields and coherence-weighted temporal merging (Section 4.4,      */
/* Eq. 8-9)                                                                  */
/* ------------------------------------------------------------------------ */

/* nlos_fk without the magnitude: d_psi[ny][nx][nt] = Psi (complex, float re, im pairs,
 * 8-byte aligned), the field whose |.|^2 nlos_fk returns.  FP32 plans only
 * (NLOS_ERR_UNSUPPORTED otherwise).  Workspace as for nlos_fk. */
nlos_status nlos_fk_complex(nlos_ctx *ctx, const nlos_fk_plan *plan, const float *d_tau, float *d_psi,
                            void *d_ws, size_t ws_bytes);
/* nlos_rsd without the magnitude: d_field[ny][nx][n_depth] = I (complex), the field
 * whose |.| nlos_rsd returns. */
nlos_status nlos_rsd_complex(nlos_ctx *ctx, const nlos_rsd_plan *plan, const float *d_tau, float *d_field,
                             void *d_ws, size_t ws_bytes);

/* Merging state over a window of up to `window` (1..64) complex frames of n_values
 * each (device ring buffer of window * n_values * 8 bytes, owned by the state). */
nlos_status nlos_merge_create(nlos_ctx *ctx, uint64_t n_values, int window, double eps, nlos_merge **out);
nlos_status nlos_merge_destroy(nlos_merge *merge);
/* Forgets the frames pushed so far (host only). */
nlos_status nlos_merge_reset(nlos_merge *merge);
/* Adds frame i (complex, n_values) and, over the W = min(i + 1, window) most recent
 * frames f_j, writes
 *   d_coherence = C = |sum f_j| / (eps + sum |f_j|)   (0 <= C < 1; nullable),
 *   d_merged    = C |sum f_j| / W,
 * the sums taken oldest first.  Calls on one state are ordered by the context's stream;
 * a state must not be pushed from two streams at once. */
nlos_status nlos_merge_push(nlos_ctx *ctx, nlos_merge *merge, const float *d_frame, float *d_merged,
                            float *d_coherence);

/* ------------------------------------------------------------------------ */
/* Depth-dependent average of the last N_w volumes (Section 4.4, DDA)        */
/* ------------------------------------------------------------------------ */

/* The library's default weight table (host only; the paper leaves the weights open):
 * weights[d * window + a] = 1 for a < n_d and 0 otherwise, a counting frames back from the
 * newest, with n_d = 1 + floor((window - 1) d / (n_depth - 1) + 1/2) at depth index d
 * (n_d = window when n_depth = 1): the nearest plane keeps only the newest frame, the
 * farthest averages all window frames, since farther planes return less light.
 * n_depth >= 1, 1 <= window <= 64, weights holds n_depth * window floats. */
nlos_status nlos_dda_default_weights(int n_depth, int window, float *weights);
/* DDA state over volumes of n_vox voxels x n_depth depths, depth fastest ([n_vox][n_depth]:
 * the default layout of nlos_fk, whose depth axis is nt, and of nlos_rsd): a device ring of
 * `window` (1..64) volumes, window * n_vox * n_depth * 4 bytes owned by the state, and a
 * device copy of the host table weights[n_depth][window] (read at creation; entries finite
 * and >= 0, weights[d * window] > 0 for every d, else NLOS_ERR_INVALID_ARG). */
nlos_status nlos_dda_create(nlos_ctx *ctx, uint64_t n_vox, int n_depth, int window, const float *weights,
                            nlos_dda **out);
nlos_status nlos_dda_destroy(nlos_dda *dda);
/* Forgets the frames pushed so far (host only). */
nlos_status nlos_dda_reset(nlos_dda *dda);
/* Adds frame i, d_vol[n_vox][n_depth] (read only), and over the m = min(i + 1, window)
 * newest frames v_{i-a}, a < m, writes
 *   d_avg[v][d] = sum_a W[d][a] v_{i-a}[v][d] / sum_a W[d][a]   (nullable),
 *   d_img[v]    = max over d of d_avg[v][d]                      (nullable; not both NULL).
 * All pointers 4-byte aligned device memory; d_vol must not overlap the outputs.  Calls on
 * one state are ordered by the context's stream; a state must not be pushed from two
 * streams at once. */
nlos_status nlos_dda_push(nlos_ctx *ctx, nlos_dda *dda, const float *d_vol, float *d_avg, float *d_img);

/* Graph replay (the paper records each frame's launch sequence into a graph and replays
 * it, Section 2.2, and measures the gain in its ablations, Section 5.2): captures one
 * nlos_fk (nlos_rsd) call with these exact buffers -- same argument
 * meaning, layout and workspace rules, except that d_ws is required (no pool) -- into an
 * instantiated HIP graph owned by *out; nothing runs at creation.  nlos_graph_launch
 * replays it on the context's current stream: the same kernels on the same pointers, so
 * results are bitwise equal to the eager call on the same inputs.  The buffers must stay
 * allocated while the graph lives; new inputs are written into d_tau between replays
 * (stream-ordered), and replays on one workspace must not overlap (same stream, or
 * ordered by events).  Per-pass timing does not cover replays.  A graph belongs to the
 * device it was created on. */
nlos_status nlos_fk_graph_create(nlos_ctx *ctx, const nlos_fk_plan *plan, const float *d_tau, float *d_vol,
                                 float *d_img, void *d_ws, size_t ws_bytes, nlos_graph **out);
nlos_status nlos_rsd_graph_create(nlos_ctx *ctx, const nlos_rsd_plan *plan, const float *d_tau, float *d_vol,
                                  float *d_img, void *d_ws, size_t ws_bytes, nlos_graph **out);
nlos_status nlos_graph_launch(nlos_ctx *ctx, const nlos_graph *graph);
nlos_status nlos_graph_destroy(nlos_graph *graph);

#ifdef __cplusplus
}
#endif

#endif /* NLOS_H */
