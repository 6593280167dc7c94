// Host side of libnlos: contexts, plans, validation, plan-time tables and the
// pass schedules of nlos_bin / nlos_fk / nlos_rsd.  See include/nlos.h.
#include "nlos.h"
#include "nlos_debug.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "nlos_internal.hpp"
#include "rsd_host.hpp"

using nlos::ContigArgs;
using nlos::FkPairArgs;
using nlos::FkXArgs;
using nlos::StridedArgs;

namespace nlos {

std::atomic<int> g_fail_allocs{0};
namespace {
bool take_injected_failure() {
  int n = g_fail_allocs.load();
  while (n > 0)
    if (g_fail_allocs.compare_exchange_weak(n, n - 1)) return true;
  return false;
}
}  // namespace

hipError_t dev_alloc(void** p, size_t bytes) {
  if (take_injected_failure()) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

void host_alloc_point() {
  if (take_injected_failure()) throw std::bad_alloc();
}

}  // namespace nlos

namespace {

constexpr double kC = 299792458.0;
thread_local std::string g_err;  // failures without a context

bool is_pow2_in(long long n, long long lo, long long hi) {
  return n >= lo && n <= hi && (n & (n - 1)) == 0;
}

// A padded FFT length runs on the power-of-two kernels (8 .. 2048) or on the general
// mixed-radix ones (even, 8 .. 4096, prime factors 2, 3, 5, 7, 11, 13; FP32 only).
bool is_general_len(long long n) {
  nlos::GenPlan g;
  return !is_pow2_in(n, 8, 2048) && n >= 8 && n <= nlos::kGenMaxN && nlos::gen_plan_radices((int)n, &g);
}
bool fk_all_pow2(const nlos_fk_desc* d) {
  const long long p = d->pad;
  return is_pow2_in(p * d->nx, 8, 2048) && is_pow2_in(p * d->ny, 8, 2048) && is_pow2_in(p * d->nt, 8, 2048);
}

// Radix plans of the axes that run on the general kernels (use[i]) and their W_m^k =
// exp(-2 pi i k / m) tables (FP64 with exact octant reduction, stored as float), in one
// device allocation *d_tw (null when no axis needs one).
hipError_t gen_tables(int device, const int* m, const bool* use, nlos::GenPlan* const* g, int naxes,
                      float2** d_tw) {
  std::vector<float2> tw;
  std::vector<size_t> off(naxes, 0);
  for (int i = 0; i < naxes; ++i) {
    if (!use[i]) continue;
    if (!nlos::gen_plan_radices(m[i], g[i])) return hipErrorInvalidValue;
    off[i] = tw.size();
    for (int k = 0; k < m[i]; ++k) {
      double cs, sn;
      nlos::cos_sin_2pi_frac(k, m[i], &cs, &sn);
      tw.push_back(make_float2((float)cs, (float)-sn));
    }
  }
  *d_tw = nullptr;
  if (tw.empty()) return hipSuccess;
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = nlos::dev_alloc((void**)d_tw, tw.size() * sizeof(float2));
  if (e != hipSuccess) return e;
  if ((e = hipMemcpy(*d_tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess) {
    (void)hipFree(*d_tw);
    *d_tw = nullptr;
    return e;
  }
  for (int i = 0; i < naxes; ++i)
    if (use[i]) g[i]->tw = *d_tw + off[i];
  return hipSuccess;
}

// Elements between consecutive y (or ky) rows of the f-k intermediates: Mx * nt plus
// 256 bytes, so that the y passes, which step through rows, do not hit the same
// memory channels at a power-of-two stride.  es is the bytes per complex element.
size_t fk_row_stride(size_t Mx, size_t nt, size_t es) { return Mx * nt + 256 / es; }

// log2 of a power of two (0 for n <= 1)
int ilog2(int n) {
  int k = 0;
  while ((1 << (k + 1)) <= n) ++k;
  return k;
}

size_t fk_elem_bytes(nlos_precision p) { return p == NLOS_FP32 ? 8 : 4; }
int fk_sp(nlos_precision p) { return p == NLOS_FP16 ? nlos::SP_F16 : p == NLOS_BF16 ? nlos::SP_BF16 : nlos::SP_F32; }

// f-k workspace (complex elements of es bytes): region A holds W1 [ny][Mx/2+1][nt] and
// W2 [My][Mx/2+1][nt] (half spectra, row stride rs_half), later W4 [My][nx][nt] (row
// stride nx nt + 256 bytes);
// region B holds W3 [My][Mx][nt] (rs_full), later W5 [ny][nx][nt].  FP16 appends the
// scale scratch: kScaleBlocks partial sums and the four storage exponents.
struct FkLayout {
  size_t es, rs_half, rs_full, w2_off, b_off, total;  // elements
  size_t scale_off;                                   // bytes (FP16 only)
  size_t bytes;
};
FkLayout fk_layout(const nlos_fk_desc* d) {
  const size_t Mx = (size_t)d->pad * d->nx, My = (size_t)d->pad * d->ny, nt = d->nt, ny = d->ny;
  FkLayout L{};
  L.es = fk_elem_bytes(d->prec);
  L.rs_half = fk_row_stride(Mx / 2 + 1, nt, L.es);
  L.rs_full = fk_row_stride(Mx, nt, L.es);
  L.w2_off = ny * L.rs_half;
  // region A also holds the [My][nx][nt] x-IFFT output W4 (never the largest tenant for
  // pad 1 or 2, but bounded here all the same)
  const size_t a = std::max({(ny + My) * L.rs_half, ny * L.rs_full,
                             My * fk_row_stride((size_t)d->nx, nt, L.es)});
  const size_t align = 256 / L.es;
  L.b_off = (a + align - 1) / align * align;
  L.total = L.b_off + My * L.rs_full;
  L.bytes = L.total * L.es;
  if (d->prec == NLOS_FP16) {
    L.scale_off = (L.bytes + 255) / 256 * 256;
    L.bytes = L.scale_off + 4 * nlos::kScaleBlocks + 256;
  }
  return L;
}

}  // namespace

struct TimedLaunch {
  int pass;
  hipEvent_t start, stop;
};

struct nlos_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  float2* d_tw = nullptr;     // W_2048^k, FP64-generated, stored FP32
  void* pool = nullptr;       // workspace when the caller passes none
  size_t pool_bytes = 0;
  std::string err;
  bool timing = false;
  std::vector<TimedLaunch> recs;      // launches recorded since the last read
  std::vector<hipEvent_t> spare;      // recycled events
  hipStream_t aux = nullptr;          // second stream of the mixture of experts
  hipEvent_t fork[3] = {nullptr, nullptr, nullptr};
  void* scratch = nullptr;            // this device's static scratch (nlos_fk_noalloc)
  void* d_mfma = nullptr;             // matrix-core DFT operands (FP64-built)
  nlos::MfmaTables mt{};
  bool mfma = true;                   // four-byte f-k passes on the matrix cores
  int rsd_mfma = 1;                   // RSD propagation on the matrix cores (0 no: FP32 FMAs; 2 the
                                      // other depth tiling)
};

struct nlos_fk_plan {
  nlos_fk_desc d{};
  int device = 0;
  int Mx = 0, My = 0, Mt = 0;
  double sxk = 0, syk = 0;
  float norm = 0.f;
  // general (not power-of-two) axis lengths: radix plans and their W_M^k tables, which
  // live in d_gtw.  gen_xr2c: the x pass runs on the general kernel, also for a
  // power-of-two Mx when nt is odd (the tuned kernel packs t-column pairs as float2).
  bool gen_x = false, gen_y = false, gen_t = false, gen_xr2c = false;
  nlos::GenPlan gx{}, gy{}, gt{};
  float2* d_gtw = nullptr;
};

struct nlos_rsd_plan {
  nlos_rsd_desc d{};
  int device = 0;
  int Mx = 0, My = 0;
  nlos::RsdGeometry g{};
  void* d_kr = nullptr;       // [Nrho][Nf][Nd] float2 or (re, im) FP16 / BF16 pairs
  float* d_kappa = nullptr;   // [Nd] sum_f |w_f| max_i |K_r[i][f][d]| (four-byte data: scales)
  float2* d_w = nullptr;      // [Nf]
  int* d_bins = nullptr;      // [Nf]
  int* d_chunk_i0 = nullptr;  // pixel chunks sharing a radial bin (rsd_build_chunks)
  int* d_chunk_pix = nullptr;
  float* d_chunk_wa = nullptr;
  float* d_chunk_wb = nullptr;
  long long nchunks = 0;
  // general (not power-of-two) lengths of the x, y and phasor t transforms: radix plans
  // and W_m^k tables (in d_gtw)
  bool gen_x = false, gen_y = false, gen_t = false;
  nlos::GenPlan gx{}, gy{}, gt{};
  float2* d_gtw = nullptr;
};

static nlos_status fail(nlos_ctx* ctx, nlos_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  g_err = buf;
  return s;
}

#define HIP_TRY(ctx, call)                                                                   \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail((ctx), e_ == hipErrorOutOfMemory ? NLOS_ERR_OUT_OF_MEMORY : NLOS_ERR_DEVICE, \
                  "%s: %s", #call, hipGetErrorString(e_));                                    \
  } while (0)

// Runs launch() and, when timing is on, brackets it with events on the stream.
template <class F>
static hipError_t timed_on(nlos_ctx* ctx, hipStream_t stream, int pass, F launch);
template <class F>
static hipError_t timed(nlos_ctx* ctx, int pass, F launch) {
  return timed_on(ctx, ctx->stream, pass, launch);
}

// Runs launch() and, when timing is on, brackets it with events on `stream`.
template <class F>
static hipError_t timed_on(nlos_ctx* ctx, hipStream_t stream, int pass, F launch) {
  if (!ctx->timing) return launch();
  hipEvent_t ev[2];
  for (auto& e : ev) {
    if (!ctx->spare.empty()) {
      e = ctx->spare.back();
      ctx->spare.pop_back();
    } else {
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
    }
  }
  hipError_t r = hipEventRecord(ev[0], stream);
  if (r == hipSuccess) r = launch();
  if (r == hipSuccess) r = hipEventRecord(ev[1], stream);
  if (r != hipSuccess) {
    ctx->spare.push_back(ev[0]);
    ctx->spare.push_back(ev[1]);
    return r;
  }
  ctx->recs.push_back({pass, ev[0], ev[1]});
  return hipSuccess;
}

static const char* const kPassNames[NLOS_PASS_COUNT] = {
    "fill", "bin", "fk_x", "fk_y", "fk_column", "fk_yi", "fk_xi",
    "rsd_phasor", "rsd_x", "rsd_y", "rsd_propagate", "rsd_yi", "rsd_xi", "fk_zi", "fk_scale",
    "moe_phasor", "moe_mix", "phasor_bin", "merge", "dda", "rsd_scale"};

extern "C" {

void nlos_debug_fail_allocations(int n) { nlos::g_fail_allocs.store(n > 0 ? n : 0); }

int nlos_version(void) { return 100; }

const char* nlos_pass_name(int pass) {
  return (pass >= 0 && pass < NLOS_PASS_COUNT) ? kPassNames[pass] : "?";
}

nlos_status nlos_timing_enable(nlos_ctx* ctx, int enable) {
  if (!ctx) return fail(nullptr, NLOS_ERR_INVALID_ARG, "nlos_timing_enable: ctx is NULL");
  ctx->timing = enable != 0;
  return NLOS_OK;
}

nlos_status nlos_timing_read(nlos_ctx* ctx, double* ms, int* count, int n) {
  if (!ctx || !ms || !count || n < 0 || n > NLOS_PASS_COUNT)
    return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_timing_read: bad arguments");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (int p = 0; p < n; ++p) {
    ms[p] = 0.0;
    count[p] = 0;
  }
  nlos_status st = NLOS_OK;
  for (const TimedLaunch& t : ctx->recs) {
    float e = 0.f;
    if (hipEventElapsedTime(&e, t.start, t.stop) != hipSuccess) st = NLOS_ERR_DEVICE;
    if (t.pass < n) {
      ms[t.pass] += e;
      count[t.pass] += 1;
    }
    ctx->spare.push_back(t.start);
    ctx->spare.push_back(t.stop);
  }
  ctx->recs.clear();
  if (st != NLOS_OK) return fail(ctx, st, "nlos_timing_read: hipEventElapsedTime failed");
  return NLOS_OK;
}

const char* nlos_status_string(nlos_status s) {
  switch (s) {
    case NLOS_OK: return "NLOS_OK";
    case NLOS_ERR_INVALID_ARG: return "NLOS_ERR_INVALID_ARG";
    case NLOS_ERR_UNSUPPORTED: return "NLOS_ERR_UNSUPPORTED";
    case NLOS_ERR_OUT_OF_MEMORY: return "NLOS_ERR_OUT_OF_MEMORY";
    case NLOS_ERR_DEVICE: return "NLOS_ERR_DEVICE";
    case NLOS_ERR_INTERNAL: return "NLOS_ERR_INTERNAL";
  }
  return "NLOS_ERR_UNKNOWN";
}

const char* nlos_last_error(const nlos_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------

nlos_status nlos_create(int device, void* hip_stream, nlos_ctx** out) {
  try {
    if (!out) return fail(nullptr, NLOS_ERR_INVALID_ARG, "nlos_create: out is NULL");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
      return fail(nullptr, NLOS_ERR_DEVICE, "nlos_create: no HIP device");
    if (device < 0 || device >= count)
      return fail(nullptr, NLOS_ERR_INVALID_ARG, "nlos_create: device %d of %d", device, count);
    if (hipSetDevice(device) != hipSuccess)
      return fail(nullptr, NLOS_ERR_DEVICE, "nlos_create: hipSetDevice(%d) failed", device);
    nlos::host_alloc_point();
    nlos_ctx* c = new (std::nothrow) nlos_ctx();
    if (!c) return fail(nullptr, NLOS_ERR_OUT_OF_MEMORY, "nlos_create: host allocation");
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    // the static scratch's device address on this device (looked up once per device)
    const hipError_t se = nlos::static_scratch_address(device, &c->scratch);
    if (se != hipSuccess) {
      delete c;
      return fail(nullptr, NLOS_ERR_DEVICE, "nlos_create: static scratch address: %s", hipGetErrorString(se));
    }
    // W_2048^k = exp(-2 pi i k / 2048) in double with exact octant reduction, stored as float
    std::vector<float2> tw(nlos::kTwiddleTableN);
    for (int k = 0; k < nlos::kTwiddleTableN; ++k) {
      double cs, sn;
      nlos::cos_sin_2pi_frac(k, nlos::kTwiddleTableN, &cs, &sn);
      tw[k] = make_float2((float)cs, (float)-sn);
    }
    if (nlos::dev_alloc((void**)&c->d_tw, tw.size() * sizeof(float2)) != hipSuccess) {
      delete c;
      return fail(nullptr, NLOS_ERR_OUT_OF_MEMORY, "nlos_create: twiddle table allocation");
    }
    if (hipMemcpy(c->d_tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(c->d_tw);
      delete c;
      return fail(nullptr, NLOS_ERR_DEVICE, "nlos_create: twiddle upload failed");
    }
    const hipError_t me = nlos::mfma_tables_create(device, &c->d_mfma, &c->mt);
    if (me != hipSuccess) {
      (void)hipFree(c->d_tw);
      delete c;
      return fail(nullptr, me == hipErrorOutOfMemory ? NLOS_ERR_OUT_OF_MEMORY : NLOS_ERR_DEVICE,
                  "nlos_create: matrix-core operand tables: %s", hipGetErrorString(me));
    }
    const char* mf = std::getenv("NLOS_FK_MFMA");
    c->mfma = !(mf && mf[0] == '0');
    const char* rm = std::getenv("NLOS_RSD_MFMA");
    c->rsd_mfma = (rm && (rm[0] == '0' || rm[0] == '2')) ? rm[0] - '0' : 1;
    *out = c;
    return NLOS_OK;
  } catch (const std::bad_alloc&) {
    return fail(nullptr, NLOS_ERR_OUT_OF_MEMORY, "nlos_create: host allocation failed");
  }
}

nlos_status nlos_destroy(nlos_ctx* ctx) {
  if (!ctx) return NLOS_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->pool) (void)hipFree(ctx->pool);
  if (ctx->d_tw) (void)hipFree(ctx->d_tw);
  if (ctx->d_mfma) (void)hipFree(ctx->d_mfma);
  for (auto& t : ctx->recs) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  for (auto& e : ctx->spare) (void)hipEventDestroy(e);
  if (ctx->aux) {
    (void)hipStreamSynchronize(ctx->aux);
    (void)hipStreamDestroy(ctx->aux);
  }
  for (auto& e : ctx->fork)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
  return NLOS_OK;
}

nlos_status nlos_set_stream(nlos_ctx* ctx, void* hip_stream) {
  if (!ctx) return fail(nullptr, NLOS_ERR_INVALID_ARG, "nlos_set_stream: ctx is NULL");
  // the context's pool is ordered by its stream: drain the old one
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (ctx->aux) HIP_TRY(ctx, hipStreamSynchronize(ctx->aux));
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return NLOS_OK;
}

static nlos_status get_workspace(nlos_ctx* ctx, void* d_ws, size_t ws_bytes, size_t need, void** out) {
  if (d_ws) {
    if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0)
      return fail(ctx, NLOS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
      return fail(ctx, NLOS_ERR_OUT_OF_MEMORY, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    *out = d_ws;
    return NLOS_OK;
  }
  if (ctx->pool_bytes < need) {
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->pool) HIP_TRY(ctx, hipFree(ctx->pool));
    ctx->pool = nullptr;
    ctx->pool_bytes = 0;
    HIP_TRY(ctx, nlos::dev_alloc((void**)&ctx->pool, need));
    ctx->pool_bytes = need;
  }
  *out = ctx->pool;
  return NLOS_OK;
}

// ---------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------

nlos_status nlos_bin_check(const nlos_bin_desc* d) {
  if (!d) return fail(nullptr, NLOS_ERR_INVALID_ARG, "bin: desc is NULL");
  if (d->nx < 1 || d->ny < 1 || d->nt < 1)
    return fail(nullptr, NLOS_ERR_INVALID_ARG, "bin: dims must be >= 1 (%d %d %d)", d->nx, d->ny, d->nt);
  if ((long long)d->nx * d->ny > 0x7fffffffLL ||
      (long long)d->nx * d->ny * (long long)d->nt > (1LL << 40))
    return fail(nullptr, NLOS_ERR_UNSUPPORTED, "bin: histogram too large");
  if (d->bin_ps < 1) return fail(nullptr, NLOS_ERR_INVALID_ARG, "bin: bin_ps must be >= 1");
  if (d->accumulate != 0 && d->accumulate != 1)
    return fail(nullptr, NLOS_ERR_INVALID_ARG, "bin: accumulate must be 0 or 1");
  return NLOS_OK;
}

nlos_status nlos_bin(nlos_ctx* ctx, const nlos_bin_desc* d, const nlos_event* d_events,
                     uint64_t n_events, uint32_t* d_hist, unsigned long long* d_dropped) {
  if (!ctx) return fail(nullptr, NLOS_ERR_INVALID_ARG, "nlos_bin: ctx is NULL");
  nlos_status st = nlos_bin_check(d);
  if (st != NLOS_OK) return fail(ctx, st, "%s", g_err.c_str());
  if (!d_hist) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_bin: d_hist is NULL");
  if (n_events > 0 && !d_events) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_bin: d_events is NULL");
  if (reinterpret_cast<uintptr_t>(d_events) % 8 != 0)
    return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_bin: d_events must be 8-byte aligned");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const size_t nbins = (size_t)d->nx * d->ny * d->nt;
  const int npix = d->nx * d->ny;
  const size_t wsb = nlos::bin_workspace_bytes(npix, d->nt, n_events);
  if (wsb > 0) {
    // tiled path: its workspace comes from the context pool (stream ordered)
    void* ws = nullptr;
    nlos_status st2 = get_workspace(ctx, nullptr, 0, wsb, &ws);
    if (st2 != NLOS_OK) return st2;
    if (d_dropped && !d->accumulate)
      HIP_TRY(ctx, timed(ctx, NLOS_PASS_FILL, [&] {
        return nlos::launch_fill_u32(reinterpret_cast<uint32_t*>(d_dropped), 2, 0u, ctx->stream);
      }));
    HIP_TRY(ctx, timed(ctx, NLOS_PASS_BIN, [&] {
      return nlos::launch_bin_tiled(d_events, n_events, d_hist, d_dropped, npix, d->nt, d->bin_ps, d->t0_ps,
                                    d->accumulate, ws, ctx->stream);
    }));
    return NLOS_OK;
  }
  if (!d->accumulate) {
    HIP_TRY(ctx, timed(ctx, NLOS_PASS_FILL, [&] { return nlos::launch_fill_u32(d_hist, nbins, 0u, ctx->stream); }));
    if (d_dropped)
      HIP_TRY(ctx, timed(ctx, NLOS_PASS_FILL, [&] {
        return nlos::launch_fill_u32(reinterpret_cast<uint32_t*>(d_dropped), 2, 0u, ctx->stream);
      }));
  }
  HIP_TRY(ctx, timed(ctx, NLOS_PASS_BIN, [&] {
    return nlos::launch_bin(d_events, n_events, d_hist, d_dropped, d->nx * d->ny, d->nt, d->bin_ps,
                            d->t0_ps, ctx->stream);
  }));
  return NLOS_OK;
}

nlos_status nlos_counts_to_float(nlos_ctx* ctx, const uint32_t* d_hist, float* d_tau, uint64_t n) {
  if (!ctx) return fail(nullptr, NLOS_ERR_INVALID_ARG, "nlos_counts_to_float: ctx is NULL");
  if (n > 0 && (!d_hist || !d_tau)) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_counts_to_float: NULL buffer");
  if (n > 0 && (const void*)d_hist < (const void*)(d_tau + n) && (const void*)d_tau < (const void*)(d_hist + n))
    return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_counts_to_float: buffers overlap");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, timed(ctx, NLOS_PASS_FILL, [&] { return nlos::launch_u32_to_f32(d_hist, d_tau, n, ctx->stream); }));
  return NLOS_OK;
}

// ---------------------------------------------------------------------------
// phasor binning (Section 4.1)
// ---------------------------------------------------------------------------

struct nlos_phasor_plan {
  nlos_bin_desc d{};
  int device = 0;
  int nf = 0;
  float2* d_lut = nullptr;  // W_nt^m, m < nt (FP64-generated)
  int* d_bins = nullptr;
};

nlos_status nlos_phasor_plan_destroy(nlos_phasor_plan* p) {
  if (!p) return NLOS_OK;
  (void)hipSetDevice(p->device);
  if (p->d_lut) (void)hipFree(p->d_lut);
  if (p->d_bins) (void)hipFree(p->d_bins);
  delete p;
  return NLOS_OK;
}

nlos_status nlos_phasor_plan_create(nlos_ctx* ctx, const nlos_bin_desc* d, int n_freq, const int* freq_bin,
                                    nlos_phasor_plan** out) {
  try {
    if (!ctx || !out) return fail(ctx, NLOS_ERR_INVALID_ARG, "phasor_plan_create: NULL argument");
    nlos_status st = nlos_bin_check(d);
    if (st != NLOS_OK) return fail(ctx, st, "%s", g_err.c_str());
    if (d->nt > 2048) return fail(ctx, NLOS_ERR_UNSUPPORTED, "phasor_plan_create: nt must be <= 2048");
    if (n_freq < 1 || !freq_bin) return fail(ctx, NLOS_ERR_INVALID_ARG, "phasor_plan_create: need n_freq >= 1 and freq_bin");
    for (int f = 0; f < n_freq; ++f)
      if (freq_bin[f] < 0 || freq_bin[f] >= d->nt)
        return fail(ctx, NLOS_ERR_INVALID_ARG, "phasor_plan_create: freq_bin[%d] = %d outside [0, nt)", f, freq_bin[f]);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    nlos_phasor_plan* p = new (std::nothrow) nlos_phasor_plan();
    if (!p) return fail(ctx, NLOS_ERR_OUT_OF_MEMORY, "phasor_plan_create: host allocation");
    p->d = *d;
    p->device = ctx->device;
    p->nf = n_freq;
    std::vector<float2> lut(d->nt);
    for (int m = 0; m < d->nt; ++m) {
      double c, sn;
      nlos::cos_sin_2pi_frac(m, d->nt, &c, &sn);
      lut[m] = make_float2((float)c, (float)-sn);  // exp(-2 pi i m / nt)
    }
    hipError_t e = nlos::dev_alloc((void**)&p->d_lut, lut.size() * sizeof(float2));
    if (e == hipSuccess) e = nlos::dev_alloc((void**)&p->d_bins, n_freq * sizeof(int));
    if (e == hipSuccess) e = hipMemcpy(p->d_lut, lut.data(), lut.size() * sizeof(float2), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_bins, freq_bin, n_freq * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      nlos_phasor_plan_destroy(p);
      return fail(ctx, NLOS_ERR_DEVICE, "phasor_plan_create: %s", hipGetErrorString(e));
    }
    *out = p;
    return NLOS_OK;
  } catch (const std::bad_alloc&) {
    return fail(ctx, NLOS_ERR_OUT_OF_MEMORY, "nlos_phasor_plan_create: host allocation failed");
  }
}

nlos_status nlos_phasor_bin(nlos_ctx* ctx, const nlos_phasor_plan* p, const nlos_event* d_events, uint64_t n_events,
                            float* d_phasor, unsigned long long* d_dropped) {
  if (!ctx || !p) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_phasor_bin: ctx or plan is NULL");
  if (!d_phasor) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_phasor_bin: d_phasor is NULL");
  if (n_events > 0 && !d_events) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_phasor_bin: d_events is NULL");
  if (reinterpret_cast<uintptr_t>(d_events) % 8 != 0 || reinterpret_cast<uintptr_t>(d_phasor) % 8 != 0)
    return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_phasor_bin: d_events and d_phasor must be 8-byte aligned");
  if (p->device != ctx->device) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_phasor_bin: plan of another device");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const nlos_bin_desc& d = p->d;
  const size_t nval = 2 * (size_t)d.nx * d.ny * p->nf;
  if (!d.accumulate) {
    HIP_TRY(ctx, timed(ctx, NLOS_PASS_FILL, [&] { return nlos::launch_fill_u32(reinterpret_cast<uint32_t*>(d_phasor), nval, 0u, ctx->stream); }));
    if (d_dropped)
      HIP_TRY(ctx, timed(ctx, NLOS_PASS_FILL, [&] {
        return nlos::launch_fill_u32(reinterpret_cast<uint32_t*>(d_dropped), 2, 0u, ctx->stream);
      }));
  }
  HIP_TRY(ctx, timed(ctx, NLOS_PASS_PHASOR_BIN, [&] {
    return nlos::launch_phasor_bin(d_events, n_events, reinterpret_cast<float2*>(d_phasor), d_dropped, d.nx * d.ny,
                                   d.nt, d.bin_ps, d.t0_ps, p->d_lut, p->d_bins, p->nf, ctx->stream);
  }));
  return NLOS_OK;
}

// ---------------------------------------------------------------------------
// f-k
// ---------------------------------------------------------------------------

nlos_status nlos_fk_check(const nlos_fk_desc* d) {
  if (!d) return fail(nullptr, NLOS_ERR_INVALID_ARG, "fk: desc is NULL");
  if (d->nx < 1 || d->ny < 1 || d->nt < 2)
    return fail(nullptr, NLOS_ERR_INVALID_ARG, "fk: need nx, ny >= 1 and nt >= 2 (%d %d %d)", d->nx,
                d->ny, d->nt);
  if (d->pad != 1 && d->pad != 2) return fail(nullptr, NLOS_ERR_INVALID_ARG, "fk: pad must be 1 or 2");
  if (!(d->wall_w_m > 0) || !(d->wall_h_m > 0) || !(d->bin_ps > 0) || !std::isfinite(d->wall_w_m) ||
      !std::isfinite(d->wall_h_m) || !std::isfinite(d->bin_ps))
    return fail(nullptr, NLOS_ERR_INVALID_ARG, "fk: wall size and bin width must be positive");
  if (d->prec != NLOS_FP32 && d->prec != NLOS_FP16 && d->prec != NLOS_BF16)
    return fail(nullptr, NLOS_ERR_INVALID_ARG, "fk: bad precision %d", (int)d->prec);
  const long long p = d->pad;
  if (fk_all_pow2(d)) return NLOS_OK;
  for (long long m : {p * d->nx, p * d->ny, p * d->nt})
    if (!is_pow2_in(m, 8, 2048) && !is_general_len(m))
      return fail(nullptr, NLOS_ERR_UNSUPPORTED,
                  "fk: padded sizes %lld x %lld x %lld must be powers of two in [8, 2048] or even lengths "
                  "in [8, 4096] with prime factors 2, 3, 5, 7, 11, 13",
                  p * d->ny, p * d->nx, p * d->nt);
  if (d->prec != NLOS_FP32)
    return fail(nullptr, NLOS_ERR_UNSUPPORTED,
                "fk: FP16 / BF16 storage needs power-of-two padded sizes (%lld x %lld x %lld)", p * d->ny,
                p * d->nx, p * d->nt);
  return NLOS_OK;
}

nlos_status nlos_fk_desc_workspace_bytes(const nlos_fk_desc* d, size_t* bytes) {
  nlos_status st = nlos_fk_check(d);
  if (st != NLOS_OK) return st;
  if (!bytes) return fail(nullptr, NLOS_ERR_INVALID_ARG, "fk: bytes is NULL");
  *bytes = fk_layout(d).bytes;
  return NLOS_OK;
}

nlos_status nlos_fk_plan_create(nlos_ctx* ctx, const nlos_fk_desc* d, nlos_fk_plan** out) {
  try {
    if (!ctx || !out) return fail(ctx, NLOS_ERR_INVALID_ARG, "fk_plan_create: NULL argument");
    nlos_status st = nlos_fk_check(d);
    if (st != NLOS_OK) return fail(ctx, st, "%s", g_err.c_str());
    nlos::host_alloc_point();
    nlos_fk_plan* p = new (std::nothrow) nlos_fk_plan();
    if (!p) return fail(ctx, NLOS_ERR_OUT_OF_MEMORY, "fk_plan_create: host allocation");
    p->d = *d;
    p->device = ctx->device;
    p->Mx = d->pad * d->nx;
    p->My = d->pad * d->ny;
    p->Mt = d->pad * d->nt;
    const double c_dt = kC * d->bin_ps * 1e-12;
    const double sx = c_dt / (2.0 * (d->wall_w_m / d->nx));
    const double sy = c_dt / (2.0 * (d->wall_h_m / d->ny));
    p->sxk = sx * (double)p->Mt / (double)p->Mx;
    p->syk = sy * (double)p->Mt / (double)p->My;
    p->norm = (float)(1.0 / ((double)p->Mx * (double)p->My * (double)p->Mt));
    // general axis lengths (the x pass also for odd nt: see gen_xr2c)
    p->gen_x = !is_pow2_in(p->Mx, 8, 2048);
    p->gen_y = !is_pow2_in(p->My, 8, 2048);
    p->gen_t = !is_pow2_in(p->Mt, 8, 2048);
    p->gen_xr2c = p->gen_x || (d->nt & 1) != 0;
    const int m[3] = {p->Mx, p->My, p->Mt};
    const bool use[3] = {p->gen_xr2c, p->gen_y, p->gen_t};
    nlos::GenPlan* const g[3] = {&p->gx, &p->gy, &p->gt};
    const hipError_t e = gen_tables(ctx->device, m, use, g, 3, &p->d_gtw);
    if (e != hipSuccess) {
      delete p;
      return fail(ctx, e == hipErrorOutOfMemory ? NLOS_ERR_OUT_OF_MEMORY : NLOS_ERR_DEVICE,
                  "fk_plan_create: general-length twiddle tables: %s", hipGetErrorString(e));
    }
    *out = p;
    return NLOS_OK;
  } catch (const std::bad_alloc&) {
    return fail(ctx, NLOS_ERR_OUT_OF_MEMORY, "nlos_fk_plan_create: host allocation failed");
  }
}

nlos_status nlos_fk_workspace_bytes(const nlos_fk_plan* p, size_t* bytes) {
  if (!p || !bytes) return fail(nullptr, NLOS_ERR_INVALID_ARG, "nlos_fk_workspace_bytes: NULL argument");
  *bytes = fk_layout(&p->d).bytes;
  return NLOS_OK;
}

nlos_status nlos_fk_plan_destroy(nlos_fk_plan* p) {
  if (!p) return NLOS_OK;
  if (p->d_gtw) {
    (void)hipSetDevice(p->device);
    (void)hipFree(p->d_gtw);
  }
  delete p;
  return NLOS_OK;
}

// The f-k pass sequence on stream s with workspace ws (validated by the caller).
static nlos_status fk_run(nlos_ctx* ctx, const nlos_fk_plan* p, hipStream_t s, const float* d_tau, float* d_vol,
                          float* d_img, void* ws, float2* d_psi = nullptr) {
  const nlos_fk_desc& d = p->d;
  const long long nx = d.nx, ny = d.ny, nt = d.nt, Mx = p->Mx, My = p->My;
  const FkLayout L = fk_layout(&d);
  const int sp = fk_sp(d.prec);
  char* base = static_cast<char*>(ws);
  void* W1 = base;                          // [ny][Mx/2+1][nt] half spectrum after the x pass
  void* W2 = base + L.w2_off * L.es;        // [My][Mx/2+1][nt] half spectrum after the y pass
  void* W3 = base + L.b_off * L.es;         // [My][Mx][nt] after the column pass
  void* W4 = base;                          // [My][nx][nt] after the x-IFFT (W1, W2 are dead)
  void* W5 = W3;                            // [ny][nx][nt] after the x-IFFT (W3 is dead)
  // FP16 storage exponents: [0] W1 and W2, [1] W3, [2] W4, [3] W5
  int* ex = nullptr;
  float* partials = nullptr;
  if (sp == nlos::SP_F16) {
    partials = reinterpret_cast<float*>(base + L.scale_off);
    ex = reinterpret_cast<int*>(base + L.scale_off + 4 * nlos::kScaleBlocks);
  }
  const long long RH = (long long)L.rs_half, RF = (long long)L.rs_full;
  const float2* tw = ctx->d_tw;
  if (d_img)
    HIP_TRY(ctx, timed_on(ctx, s, NLOS_PASS_FILL, [&] {
      return nlos::launch_fill_u32(reinterpret_cast<uint32_t*>(d_img), (size_t)nx * ny, 0u, s);
    }));

  if (ex) {
    // FP16: power-of-two storage scales from the bound sum |tau| t/(nt-1)
    // W4 follows the x-IFFT (its bound gains Mx), W5 the y-IFFT as well
    const int l_my = ilog2((int)My), l_mx = ilog2((int)Mx), l_norm = l_my + l_mx + ilog2(p->Mt);
    HIP_TRY(ctx, timed_on(ctx, s, NLOS_PASS_FK_SCALE, [&] {
      return nlos::launch_fk_scales(d_tau, ny * nx * nt, (int)nt, partials, ex, l_norm, /*first inverse*/ l_mx,
                                    /*second inverse*/ l_my, s);
    }));
  }
  // pass 1: x-FFT of tau * t/(nt-1), zero padded to Mx, kx in [0, Mx/2]
  FkXArgs x{};
  x.tau = d_tau; x.out = W1; x.out_plane = RH; x.nx = (int)nx; x.nt = (int)nt;
  x.tscale = (float)(1.0 / (double)(nt - 1));
  x.e_out = ex;
  HIP_TRY(ctx, timed_on(ctx, s, NLOS_PASS_FK_X, [&] {
    return p->gen_xr2c ? nlos::launch_gen_xr2c(p->gx, x, (int)ny, s) : nlos::launch_fk_xr2c((int)Mx, x, (int)ny, tw, s, sp);
  }));
  // pass 2: y-FFT of the Mx/2 + 1 planes, zero padded to My
  StridedArgs a{};
  a.in = W1; a.out = W2;
  a.in_plane = nt; a.in_line = RH; a.out_plane = nt; a.out_line = RH;
  a.ncols = (int)nt; a.n_in = (int)ny; a.n_out = (int)My;
  a.e_in = ex; a.e_out = ex;
  const bool mf = ctx->mfma && sp != nlos::SP_F32;
  HIP_TRY(ctx, timed_on(ctx, s, NLOS_PASS_FK_Y, [&] {
    if (mf && nlos::mfma_strided_ok((int)My, sp, a))
      return nlos::launch_strided_mfma((int)My, false, a, (int)(Mx / 2 + 1), ctx->mt, tw, s, sp);
    return p->gen_y ? nlos::launch_gen_strided(p->gy, false, nlos::ST_C64, a, (int)(Mx / 2 + 1), s)
                    : nlos::launch_strided((int)My, false, nlos::LD_C64, nlos::ST_C64, a, (int)(Mx / 2 + 1), tw, s, sp, true);
  }));
  // pass 3: per column of the half spectrum: t-FFT, Stolt + Jacobian + 1/(Mx My Mt) for the
  // column and its mirror; the remapped spectra (kz < nt) go to W3
  FkPairArgs c{};
  c.in = W2; c.out = W3; c.in_row = RH; c.out_row = RF;
  c.nwork = (Mx / 2 - 1) * My + 2 * (My / 2 + 1);
  c.nt = (int)nt; c.Mx = (int)Mx; c.My = (int)My;
  c.sxk = p->sxk; c.syk = p->syk; c.norm = p->norm;
  c.e_in = ex; c.e_out = ex ? ex + 1 : nullptr;
  HIP_TRY(ctx, timed_on(ctx, s, NLOS_PASS_FK_COLUMN, [&] {
    // FP16 stores the remapped spectrum times 2^(e_in + log2(Mx My Mt)): the 1/(Mx My Mt)
    // and the exponent change cancel
    if (mf && nlos::mfma_column_ok(p->Mt, (int)nt, sp, c))
      return nlos::launch_fk_column_pair_mfma(c, ctx->mt, tw, sp == nlos::SP_F16 ? 1.0f : p->norm, s, sp);
    return p->gen_t ? nlos::launch_gen_column_pair(p->gt, c, s) : nlos::launch_fk_column_pair(p->Mt, c, tw, s, sp);
  }));
  // The x-IFFT runs first: it walks W3's rows 4 KB apart, which runs faster than the
  // y-IFFT's 2 MB strides on the larger of the two inverse volumes (same bytes)
  const long long RX = (long long)fk_row_stride((size_t)nx, (size_t)nt, L.es);
  // pass 4: x-IFFT of W3, keep x < nx -> W4 [My][nx][nt] (row stride RX)
  a = StridedArgs{};
  a.in = W3; a.out = W4;
  a.in_plane = RF; a.in_line = nt; a.out_plane = RX; a.out_line = nt;
  a.ncols = (int)nt; a.n_in = (int)Mx; a.n_out = (int)nx;
  a.e_in = ex ? ex + 1 : nullptr; a.e_out = ex ? ex + 2 : nullptr;
  HIP_TRY(ctx, timed_on(ctx, s, NLOS_PASS_FK_XI, [&] {
    if (mf && nlos::mfma_strided_ok((int)Mx, sp, a))
      return nlos::launch_strided_mfma((int)Mx, true, a, (int)My, ctx->mt, tw, s, sp);
    return p->gen_x ? nlos::launch_gen_strided(p->gx, true, nlos::ST_C64, a, (int)My, s)
                    : nlos::launch_strided((int)Mx, true, nlos::LD_C64, nlos::ST_C64, a, (int)My, tw, s, sp, true);
  }));
  // pass 5: y-IFFT, keep y < ny -> W5 [ny][nx][nt]
  a = StridedArgs{};
  a.in = W4; a.out = W5;
  a.in_plane = nt; a.in_line = RX; a.out_plane = nt; a.out_line = nx * nt;
  a.ncols = (int)nt; a.n_in = (int)My; a.n_out = (int)ny;
  a.e_in = ex ? ex + 2 : nullptr; a.e_out = ex ? ex + 3 : nullptr;
  HIP_TRY(ctx, timed_on(ctx, s, NLOS_PASS_FK_YI, [&] {
    if (mf && nlos::mfma_strided_ok((int)My, sp, a))
      return nlos::launch_strided_mfma((int)My, true, a, (int)nx, ctx->mt, tw, s, sp);
    return p->gen_y ? nlos::launch_gen_strided(p->gy, true, nlos::ST_C64, a, (int)nx, s)
                    : nlos::launch_strided((int)My, true, nlos::LD_C64, nlos::ST_C64, a, (int)nx, tw, s, sp, true);
  }));
  // pass 6: z-IFFT of each (y, x) line (kz < nt stored, zero padded to Mt), keep z < nt,
  // |Psi|^2 and the max over depth
  ContigArgs z{};
  z.in = W5; z.out = d_vol; z.nlines = ny * nx; z.in_line = nt; z.out_line = nt;
  z.n_in = (int)nt; z.n_out = (int)nt; z.oscale = 1.0f; z.img = d_img;
  z.e_in = ex ? ex + 3 : nullptr;
  if (d_psi) {  // the complex field Psi itself (FP32 path)
    z.out = d_psi; z.img = nullptr;
    HIP_TRY(ctx, timed_on(ctx, s, NLOS_PASS_FK_ZI, [&] {
      return p->gen_t ? nlos::launch_gen_contig(p->gt, true, nlos::CL_C64, nlos::CS_C64, z, s)
                      : nlos::launch_contig(p->Mt, true, nlos::CL_C64, nlos::CS_C64, z, tw, s);
    }));
    return NLOS_OK;
  }
  HIP_TRY(ctx, timed_on(ctx, s, NLOS_PASS_FK_ZI, [&] {
    if (mf && nlos::mfma_zfft_ok(p->Mt, sp, z)) return nlos::launch_zfft_abs2_mfma(z, ctx->mt, tw, s, sp);
    return p->gen_t ? nlos::launch_gen_contig(p->gt, true, nlos::CL_C64, nlos::CS_ABS2_MAX, z, s)
                    : nlos::launch_contig(p->Mt, true, nlos::CL_C64, nlos::CS_ABS2_MAX, z, tw, s, sp);
  }));
  return NLOS_OK;
}

nlos_status nlos_fk(nlos_ctx* ctx, const nlos_fk_plan* p, const float* d_tau, float* d_vol, float* d_img,
                    void* d_ws, size_t ws_bytes) {
  if (!ctx || !p) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_fk: ctx or plan is NULL");
  if (!d_tau) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_fk: d_tau is NULL");
  if (reinterpret_cast<uintptr_t>(d_tau) % 8 != 0)
    return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_fk: d_tau must be 8-byte aligned");
  if (!d_vol && !d_img) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_fk: d_vol and d_img are both NULL");
  if (p->device != ctx->device) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_fk: plan of another device");
  const nlos_fk_desc& d = p->d;
  size_t need = 0;
  nlos_status st = nlos_fk_desc_workspace_bytes(&d, &need);
  if (st != NLOS_OK) return fail(ctx, st, "%s", g_err.c_str());
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  void* ws = nullptr;
  st = get_workspace(ctx, d_ws, ws_bytes, need, &ws);
  if (st != NLOS_OK) return st;
  return fk_run(ctx, p, ctx->stream, d_tau, d_vol, d_img, ws);
}

nlos_status nlos_fk_noalloc(nlos_ctx* ctx, const nlos_fk_plan* p, const float* d_tau, float* d_vol, float* d_img) {
  if (!ctx || !p) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_fk_noalloc: ctx or plan is NULL");
  if (!d_tau) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_fk_noalloc: d_tau is NULL");
  if (reinterpret_cast<uintptr_t>(d_tau) % 8 != 0)
    return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_fk_noalloc: d_tau must be 8-byte aligned");
  if (!d_vol && !d_img) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_fk_noalloc: d_vol and d_img are both NULL");
  if (p->device != ctx->device) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_fk_noalloc: plan of another device");
  size_t need = 0;
  nlos_status st = nlos_fk_desc_workspace_bytes(&p->d, &need);
  if (st != NLOS_OK) return fail(ctx, st, "%s", g_err.c_str());
  if (need > nlos::kStaticScratchBytes)
    return fail(ctx, NLOS_ERR_UNSUPPORTED,
                "nlos_fk_noalloc: this reconstruction needs %zu bytes of workspace, more than the %zu bytes of "
                "static scratch (use nlos_fk)",
                need, nlos::kStaticScratchBytes);
  if (!ctx->scratch) return fail(ctx, NLOS_ERR_DEVICE, "nlos_fk_noalloc: no static scratch on device %d", ctx->device);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  // per-pass timing would create HIP events: it is suspended for this call
  const bool timing = ctx->timing;
  ctx->timing = false;
  st = fk_run(ctx, p, ctx->stream, d_tau, d_vol, d_img, ctx->scratch);
  ctx->timing = timing;
  return st;
}

// ---------------------------------------------------------------------------
// RSD
// ---------------------------------------------------------------------------

// RSD workspace (complex elements), frequency / depth contiguous, rows of Nf (Nd) values
// at a stride of Nfs (Nds), rounded up to 16:
//   A: phasors P [ny][nx][Nfs], later the y-IFFT output D [ny][Mx][Nds]
//   B: x-FFT output [ny][Mx][Nfs], later the propagated spectra C [My][Mx][Nds]
//   E: y-FFT output P^ [My][Mx][Nfs]
struct RsdLayout {
  size_t b_off, e_off, total;  // complex elements of es bytes
  size_t nfs, nds;  // row strides (elements) of the frequency and depth contiguous arrays
  size_t es;        // 8 (FP32 data) or 4 (FP16 / BF16 data)
  size_t scale_off; // bytes: FP16 scale scratch (kScaleBlocks partial sums, 1 + 2 Nd exponents)
  size_t bytes;     // the whole workspace
};
// Rows of Nf frequencies or Nd depths are padded to a multiple of 16 complex values (128
// bytes at FP32), so that the column tiles of the strided passes cover whole cache lines.
// The last pass writes |I| (float) depth contiguous into region B when the caller asks
// for a depth-major volume: ny nx Nd floats fit in My Mx Nds elements of either size.
static RsdLayout rsd_layout(const nlos_rsd_desc* d) {
  const size_t Mx = (size_t)d->pad * d->nx, My = (size_t)d->pad * d->ny;
  auto up = [](size_t n) { return (n + 31) / 32 * 32; };
  auto up16 = [](size_t n) { return (n + 15) / 16 * 16; };
  const size_t nf = up16(d->n_freq), nd = up16(d->n_depth), ny = d->ny, nx = d->nx;
  RsdLayout L;
  L.nfs = nf;
  L.nds = nd;
  L.es = d->data_prec == NLOS_FP32 ? 8 : 4;
  const size_t a = up(std::max(ny * nx * nf, ny * Mx * nd));
  const size_t b = up(std::max(ny * Mx * nf, My * Mx * nd));
  L.b_off = a;
  L.e_off = a + b;
  L.total = a + b + My * Mx * nf;
  L.scale_off = (L.total * L.es + 255) / 256 * 256;
  L.bytes = d->data_prec == NLOS_FP16 ? L.scale_off + 4 * (size_t)nlos::kScaleBlocks + 4 * (1 + 2 * (size_t)d->n_depth)
                                      : L.total * L.es;
  return L;
}

static nlos::RsdInputs rsd_inputs(const nlos_rsd_desc* d) {
  nlos::RsdInputs in;
  in.nx = d->nx; in.ny = d->ny; in.nt = d->nt; in.pad = d->pad;
  in.dx = d->dx_m; in.dy = d->dy_m; in.c_dt = kC * d->bin_ps * 1e-12;
  in.n_freq = d->n_freq; in.freq_bin = d->freq_bin;
  in.n_depth = d->n_depth; in.depth0 = d->depth0_m; in.depth_step = d->depth_step_m;
  in.sigma_s = d->sigma_s; in.sigma_t = d->sigma_t; in.delta = d->delta_m;
  return in;
}

nlos_status nlos_rsd_check(const nlos_rsd_desc* d) {
  if (!d) return fail(nullptr, NLOS_ERR_INVALID_ARG, "rsd: desc is NULL");
  if (d->nx < 1 || d->ny < 1 || d->nt < 1)
    return fail(nullptr, NLOS_ERR_INVALID_ARG, "rsd: dims must be >= 1");
  if (d->pad != 1 && d->pad != 2) return fail(nullptr, NLOS_ERR_INVALID_ARG, "rsd: pad must be 1 or 2");
  if (!(d->dx_m > 0) || !(d->dy_m > 0) || !(d->bin_ps > 0) || !std::isfinite(d->dx_m) ||
      !std::isfinite(d->dy_m) || !std::isfinite(d->bin_ps))
    return fail(nullptr, NLOS_ERR_INVALID_ARG, "rsd: spacings must be positive");
  if (d->n_freq < 1 || !d->freq_bin || !d->w)
    return fail(nullptr, NLOS_ERR_INVALID_ARG, "rsd: need n_freq >= 1, freq_bin and w");
  if (d->n_depth < 1 || d->n_depth > 4096)
    return fail(nullptr, NLOS_ERR_INVALID_ARG, "rsd: n_depth must be in [1, 4096]");
  if (!std::isfinite(d->depth0_m) || !std::isfinite(d->depth_step_m) || !std::isfinite(d->delta_m))
    return fail(nullptr, NLOS_ERR_INVALID_ARG, "rsd: depth grid must be finite");
  if (d->sigma_s != 1 && d->sigma_s != 2) return fail(nullptr, NLOS_ERR_INVALID_ARG, "rsd: sigma_s must be 1 or 2");
  if (d->sigma_t < 0 || d->sigma_t > 2) return fail(nullptr, NLOS_ERR_INVALID_ARG, "rsd: sigma_t must be 0, 1 or 2");
  if (d->vol_depth_major != 0 && d->vol_depth_major != 1)
    return fail(nullptr, NLOS_ERR_INVALID_ARG, "rsd: vol_depth_major must be 0 or 1");
  if (d->data_prec < NLOS_FP32 || d->data_prec > NLOS_BF16 || d->kernel_prec < NLOS_FP32 ||
      d->kernel_prec > NLOS_BF16)
    return fail(nullptr, NLOS_ERR_INVALID_ARG, "rsd: bad precision");
  const long long p = d->pad;
  for (long long m : {p * d->nx, p * d->ny, (long long)d->nt})
    if (!is_pow2_in(m, 8, 2048) && !is_general_len(m))
      return fail(nullptr, NLOS_ERR_UNSUPPORTED,
                  "rsd: pad*nx, pad*ny and nt must be powers of two in [8, 2048] or even lengths in "
                  "[8, 4096] with prime factors 2, 3, 5, 7, 11, 13");
  for (int f = 0; f < d->n_freq; ++f)
    if (d->freq_bin[f] < 1 || d->freq_bin[f] > d->nt / 2 - 1)
      return fail(nullptr, NLOS_ERR_INVALID_ARG, "rsd: freq_bin[%d] = %d outside [1, nt/2 - 1]", f,
                  d->freq_bin[f]);
  for (int f = 0; f < 2 * d->n_freq; ++f)
    if (!std::isfinite(d->w[f])) return fail(nullptr, NLOS_ERR_INVALID_ARG, "rsd: w is not finite");
  if (d->data_prec != NLOS_FP32) {
    // four-byte intermediates: the power-of-two passes and the matrix-core propagation
    // with a kernel stored in the same format
    if (d->kernel_prec != d->data_prec)
      return fail(nullptr, NLOS_ERR_UNSUPPORTED, "rsd: FP16 / BF16 data needs kernel_prec equal to data_prec");
    for (long long m : {p * d->nx, p * d->ny, (long long)d->nt})
      if (!is_pow2_in(m, 8, 2048))
        return fail(nullptr, NLOS_ERR_UNSUPPORTED, "rsd: FP16 / BF16 data needs power-of-two pad*nx, pad*ny and nt");
  }
  return NLOS_OK;
}

nlos_status nlos_rsd_geometry_get(const nlos_rsd_desc* d, nlos_rsd_geometry* out) {
  try {
    nlos_status st = nlos_rsd_check(d);
    if (st != NLOS_OK) return st;
    if (!out) return fail(nullptr, NLOS_ERR_INVALID_ARG, "rsd_geometry_get: out is NULL");
    const nlos::RsdGeometry g = nlos::rsd_geometry(rsd_inputs(d));
    out->r_max = g.r_max; out->rho_max = g.rho_max; out->lambda_min = g.lambda_min; out->dr = g.dr;
    out->f_s = g.f_s; out->rho_cut = g.rho_cut; out->rho_cut_bin = g.rho_cut_bin;
    out->n_r_min = g.n_r_min; out->n_r = g.n_r; out->n_rho_min = g.n_rho_min; out->n_rho = g.n_rho;
    out->cut_idx = g.cut_idx; out->last_base = g.last_base;
    return NLOS_OK;
  } catch (const std::bad_alloc&) {
    return fail(nullptr, NLOS_ERR_OUT_OF_MEMORY, "nlos_rsd_geometry_get: host allocation failed");
  }
}

nlos_status nlos_rsd_kernel_host(const nlos_rsd_desc* d, float* out, size_t n_floats) {
  try {
    nlos_status st = nlos_rsd_check(d);
    if (st != NLOS_OK) return st;
    if (!out) return fail(nullptr, NLOS_ERR_INVALID_ARG, "rsd_kernel_host: out is NULL");
    const nlos::RsdInputs in = rsd_inputs(d);
    const nlos::RsdGeometry g = nlos::rsd_geometry(in);
    const size_t need = 2ull * g.n_rho * d->n_freq * d->n_depth;
    nlos::host_alloc_point();
    if (n_floats < need) return fail(nullptr, NLOS_ERR_INVALID_ARG, "rsd_kernel_host: need %zu floats", need);
    std::vector<double> re, im;
    nlos::rsd_radial_kernel(in, g, re, im);
    for (size_t i = 0; i < re.size(); ++i) {
      out[2 * i] = (float)re[i];
      out[2 * i + 1] = (float)im[i];
    }
    return NLOS_OK;
  } catch (const std::bad_alloc&) {
    return fail(nullptr, NLOS_ERR_OUT_OF_MEMORY, "nlos_rsd_kernel_host: host allocation failed");
  }
}

nlos_status nlos_rsd_desc_workspace_bytes(const nlos_rsd_desc* d, size_t* bytes) {
  nlos_status st = nlos_rsd_check(d);
  if (st != NLOS_OK) return st;
  if (!bytes) return fail(nullptr, NLOS_ERR_INVALID_ARG, "rsd: bytes is NULL");
  *bytes = rsd_layout(d).bytes;
  return NLOS_OK;
}

nlos_status nlos_rsd_workspace_bytes(const nlos_rsd_plan* p, size_t* bytes) {
  if (!p || !bytes) return fail(nullptr, NLOS_ERR_INVALID_ARG, "nlos_rsd_workspace_bytes: NULL argument");
  *bytes = rsd_layout(&p->d).bytes;
  return NLOS_OK;
}

nlos_status nlos_rsd_plan_destroy(nlos_rsd_plan* p) {
  if (!p) return NLOS_OK;
  (void)hipSetDevice(p->device);
  if (p->d_kr) (void)hipFree(p->d_kr);
  if (p->d_kappa) (void)hipFree(p->d_kappa);
  if (p->d_chunk_i0) (void)hipFree(p->d_chunk_i0);
  if (p->d_chunk_pix) (void)hipFree(p->d_chunk_pix);
  if (p->d_chunk_wa) (void)hipFree(p->d_chunk_wa);
  if (p->d_chunk_wb) (void)hipFree(p->d_chunk_wb);
  if (p->d_w) (void)hipFree(p->d_w);
  if (p->d_bins) (void)hipFree(p->d_bins);
  if (p->d_gtw) (void)hipFree(p->d_gtw);
  delete p;
  return NLOS_OK;
}

nlos_status nlos_rsd_plan_create(nlos_ctx* ctx, const nlos_rsd_desc* d, nlos_rsd_plan** out) {
  nlos_rsd_plan* p = nullptr;
  try {
    if (!ctx || !out) return fail(ctx, NLOS_ERR_INVALID_ARG, "rsd_plan_create: NULL argument");
    nlos_status st = nlos_rsd_check(d);
    if (st != NLOS_OK) return fail(ctx, st, "%s", g_err.c_str());
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    nlos::host_alloc_point();
    p = new (std::nothrow) nlos_rsd_plan();
    if (!p) return fail(ctx, NLOS_ERR_OUT_OF_MEMORY, "rsd_plan_create: host allocation");
    p->d = *d;
    p->d.freq_bin = nullptr;  // host arrays are copied to the device below
    p->d.w = nullptr;
    p->device = ctx->device;
    p->Mx = d->pad * d->nx;
    p->My = d->pad * d->ny;
    const nlos::RsdInputs in = rsd_inputs(d);
    p->g = nlos::rsd_geometry(in);
    std::vector<double> kre, kim;
    nlos::rsd_radial_kernel(in, p->g, kre, kim);
    nlos::RsdChunks ch;
    nlos::rsd_build_chunks(in, p->g, ch);
    const size_t nk = kre.size();
    auto cleanup = [&](nlos_status s, const char* what, hipError_t e) {
      nlos_rsd_plan_destroy(p);
      return fail(ctx, e == hipErrorOutOfMemory ? NLOS_ERR_OUT_OF_MEMORY : s, "rsd_plan_create: %s: %s", what,
                  hipGetErrorString(e));
    };
    hipError_t e;
    if (d->kernel_prec == NLOS_FP16 || d->kernel_prec == NLOS_BF16) {
      // FP64 accumulation, a single rounding (to nearest even) to binary16 or bfloat16 on
      // store; (re, im) pairs, re in the lower half
      std::vector<uint16_t> kh(2 * nk);
      const bool bf = d->kernel_prec == NLOS_BF16;
      for (size_t i = 0; i < nk; ++i) {
        kh[2 * i] = bf ? nlos::to_bf16_bits(kre[i]) : nlos::to_f16_bits(kre[i]);
        kh[2 * i + 1] = bf ? nlos::to_bf16_bits(kim[i]) : nlos::to_f16_bits(kim[i]);
      }
      if ((e = nlos::dev_alloc((void**)&p->d_kr, nk * 4)) != hipSuccess) return cleanup(NLOS_ERR_DEVICE, "K_r", e);
      if ((e = hipMemcpy(p->d_kr, kh.data(), nk * 4, hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup(NLOS_ERR_DEVICE, "K_r upload", e);
    } else {
      std::vector<float2> kf(nk);
      for (size_t i = 0; i < nk; ++i) kf[i] = make_float2((float)kre[i], (float)kim[i]);
      if ((e = nlos::dev_alloc((void**)&p->d_kr, nk * sizeof(float2))) != hipSuccess) return cleanup(NLOS_ERR_DEVICE, "K_r", e);
      if ((e = hipMemcpy(p->d_kr, kf.data(), nk * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup(NLOS_ERR_DEVICE, "K_r upload", e);
    }
    if (d->data_prec != NLOS_FP32) {
      // kappa_d = sum_f |w_f| max_i |K_r[i][f][d]|: with L = sum |tau| it bounds the
      // propagated plane at depth d (FP16 storage scales)
      const int Nf = d->n_freq, Nd = d->n_depth;
      const size_t nrho = nk / ((size_t)Nf * Nd);
      std::vector<float> kappa(Nd);
      for (int dd = 0; dd < Nd; ++dd) {
        double sum = 0.0;
        for (int f = 0; f < Nf; ++f) {
          double mx = 0.0;
          for (size_t i = 0; i < nrho; ++i) {
            const size_t o = (i * Nf + f) * Nd + dd;
            mx = std::max(mx, std::hypot(kre[o], kim[o]));
          }
          sum += std::hypot((double)d->w[2 * f], (double)d->w[2 * f + 1]) * mx;
        }
        kappa[dd] = (float)sum;
      }
      if ((e = nlos::dev_alloc((void**)&p->d_kappa, Nd * sizeof(float))) != hipSuccess)
        return cleanup(NLOS_ERR_DEVICE, "kappa", e);
      if ((e = hipMemcpy(p->d_kappa, kappa.data(), Nd * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup(NLOS_ERR_DEVICE, "kappa upload", e);
    }
    p->nchunks = ch.count();
    auto upload = [&](void** dst, const void* src, size_t bytes) -> hipError_t {
      hipError_t r = nlos::dev_alloc((void**)dst, bytes);
      if (r == hipSuccess) r = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
      return r;
    };
    if ((e = upload((void**)&p->d_chunk_i0, ch.i0.data(), ch.i0.size() * sizeof(int))) != hipSuccess ||
        (e = upload((void**)&p->d_chunk_pix, ch.pix.data(), ch.pix.size() * sizeof(int))) != hipSuccess ||
        (e = upload((void**)&p->d_chunk_wa, ch.wa.data(), ch.wa.size() * sizeof(float))) != hipSuccess ||
        (e = upload((void**)&p->d_chunk_wb, ch.wb.data(), ch.wb.size() * sizeof(float))) != hipSuccess)
      return cleanup(NLOS_ERR_DEVICE, "pixel chunks", e);
    std::vector<float2> w(d->n_freq);
    for (int f = 0; f < d->n_freq; ++f) w[f] = make_float2(d->w[2 * f], d->w[2 * f + 1]);
    if ((e = nlos::dev_alloc((void**)&p->d_w, w.size() * sizeof(float2))) != hipSuccess) return cleanup(NLOS_ERR_DEVICE, "w", e);
    if ((e = hipMemcpy(p->d_w, w.data(), w.size() * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess)
      return cleanup(NLOS_ERR_DEVICE, "w upload", e);
    std::vector<int> bins(d->freq_bin, d->freq_bin + d->n_freq);
    if ((e = nlos::dev_alloc((void**)&p->d_bins, bins.size() * sizeof(int))) != hipSuccess) return cleanup(NLOS_ERR_DEVICE, "bins", e);
    if ((e = hipMemcpy(p->d_bins, bins.data(), bins.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
      return cleanup(NLOS_ERR_DEVICE, "bins upload", e);
    p->gen_x = !is_pow2_in(p->Mx, 8, 2048);
    p->gen_y = !is_pow2_in(p->My, 8, 2048);
    p->gen_t = !is_pow2_in(d->nt, 8, 2048);
    const int m[3] = {p->Mx, p->My, d->nt};
    const bool use[3] = {p->gen_x, p->gen_y, p->gen_t};
    nlos::GenPlan* const g[3] = {&p->gx, &p->gy, &p->gt};
    if ((e = gen_tables(ctx->device, m, use, g, 3, &p->d_gtw)) != hipSuccess)
      return cleanup(NLOS_ERR_DEVICE, "general-length twiddle tables", e);
    *out = p;
    return NLOS_OK;
  } catch (const std::bad_alloc&) {
    nlos_rsd_plan_destroy(p);
    return fail(ctx, NLOS_ERR_OUT_OF_MEMORY, "nlos_rsd_plan_create: host allocation failed");
  }
}

// The RSD pass sequence on stream s with workspace ws (validated by the caller).
static nlos_status rsd_run(nlos_ctx* ctx, const nlos_rsd_plan* p, hipStream_t s, const float* d_tau, float* d_vol,
                           float* d_img, void* ws, const float2* d_phasor = nullptr, float2* d_field = nullptr) {
  const nlos_rsd_desc& d = p->d;
  const long long nx = d.nx, ny = d.ny, nt = d.nt, Mx = p->Mx, My = p->My;
  const long long Nf = d.n_freq, Nd = d.n_depth;
  const RsdLayout L = rsd_layout(&d);
  const int sp = fk_sp(d.data_prec);  // storage of the complex intermediates
  char* base = static_cast<char*>(ws);
  const size_t es = L.es;
  // frequency rows hold Nf values in a stride of Nfs, depth rows Nd in Nds
  const long long Nfs = (long long)L.nfs, Nds = (long long)L.nds;
  void* P = base;                   // [ny][nx][Nfs]
  void* X = base + L.b_off * es;    // [ny][Mx][Nfs]
  void* Ph = base + L.e_off * es;   // [My][Mx][Nfs]
  void* C = base + L.b_off * es;    // [My][Mx][Nds]
  void* D = base;                   // [ny][Mx][Nds]
  const float2* tw = ctx->d_tw;
  if (d_img)
    HIP_TRY(ctx, timed_on(ctx, s, NLOS_PASS_FILL, [&] {
      return nlos::launch_fill_u32(reinterpret_cast<uint32_t*>(d_img), (size_t)nx * ny, 0u, s);
    }));
  // FP16 storage exponents: [0] P, X, P^; [1 + d] C at depth d; [1 + Nd + d] D at depth d
  int* ex = nullptr;
  if (sp == nlos::SP_F16) {
    float* partials = reinterpret_cast<float*>(base + L.scale_off);
    ex = reinterpret_cast<int*>(base + L.scale_off + 4 * (size_t)nlos::kScaleBlocks);
    HIP_TRY(ctx, timed_on(ctx, s, NLOS_PASS_RSD_SCALE, [&] {
      return nlos::launch_rsd_scales(d_tau, ny * nx * nt, partials, p->d_kappa, (int)Nd, ilog2((int)My), ex, s);
    }));
  }
  const int* e_pc = ex ? ex + 1 : nullptr;            // per depth: C
  const int* e_pd = ex ? ex + 1 + Nd : nullptr;       // per depth: D

  // 1. phasors: t-FFT of each pixel, bins k_f -> P[y][x][f] (or the caller's phasors)
  if (!d_phasor) {
    ContigArgs c{};
    c.in = d_tau; c.out = P; c.nlines = ny * nx; c.in_line = nt; c.out_line = Nfs; c.n_in = (int)nt;
    c.n_out = (int)nt; c.bins = p->d_bins; c.nbins = (int)Nf; c.e_out = ex;
    if (!p->gen_t) {  // two real pixel lines per complex transform
      c.nreal = ny * nx;
      c.nlines = (ny * nx + 1) / 2;
    }
    HIP_TRY(ctx, timed_on(ctx, s, NLOS_PASS_RSD_PHASOR, [&] {
      return p->gen_t ? nlos::launch_gen_contig(p->gt, false, nlos::CL_REAL, nlos::CS_BINS, c, s)
                      : nlos::launch_contig((int)nt, false, nlos::CL_REAL_PAIR, nlos::CS_BINS, c, tw, s, sp);
    }));
  }
  // 2. x-FFT of the top-left padded planes: lines along x, columns f
  StridedArgs a{};
  const long long Pin = d_phasor ? Nf : Nfs;  // the caller's phasors are [ny][nx][Nf]
  a.in = d_phasor ? static_cast<const void*>(d_phasor) : P; a.out = X; a.in_plane = nx * Pin; a.in_line = Pin;
  a.out_plane = Mx * Nfs; a.out_line = Nfs; a.ncols = (int)Nf; a.n_in = (int)nx; a.n_out = (int)Mx;
  a.e_in = ex; a.e_out = ex;
  HIP_TRY(ctx, timed_on(ctx, s, NLOS_PASS_RSD_X, [&] {
    return p->gen_x ? nlos::launch_gen_strided(p->gx, false, nlos::ST_C64, a, (int)ny, s)
                    : nlos::launch_strided((int)Mx, false, nlos::LD_C64, nlos::ST_C64, a, (int)ny, tw, s, sp);
  }));
  // 3. y-FFT: planes kx, lines along y -> P^[ky][kx][f]
  a = StridedArgs{};
  a.in = X; a.out = Ph; a.in_plane = Nfs; a.in_line = Mx * Nfs; a.out_plane = Nfs; a.out_line = Mx * Nfs;
  a.ncols = (int)Nf; a.n_in = (int)ny; a.n_out = (int)My; a.e_in = ex; a.e_out = ex;
  HIP_TRY(ctx, timed_on(ctx, s, NLOS_PASS_RSD_Y, [&] {
    return p->gen_y ? nlos::launch_gen_strided(p->gy, false, nlos::ST_C64, a, (int)Mx, s)
                    : nlos::launch_strided((int)My, false, nlos::LD_C64, nlos::ST_C64, a, (int)Mx, tw, s, sp);
  }));
  // 4. radial propagation over pixel chunks: P^ -> C[pix][d]
  nlos::RsdPropArgs r{};
  r.Ph = Ph; r.Kr = p->d_kr; r.w = p->d_w; r.C = C;
  r.chunk_i0 = p->d_chunk_i0; r.chunk_pix = p->d_chunk_pix; r.chunk_wa = p->d_chunk_wa;
  r.chunk_wb = p->d_chunk_wb; r.nchunks = p->nchunks;
  r.Nf = (int)Nf; r.Nd = (int)Nd; r.ph_stride = (int)Nfs; r.c_stride = (int)Nds;
  r.cut_idx = p->g.cut_idx; r.kernel_sp = fk_sp(d.kernel_prec);
  // four-byte data exist only on the matrix cores
  r.mfma = sp != nlos::SP_F32 && ctx->rsd_mfma == 0 ? 1 : ctx->rsd_mfma;
  r.data_sp = sp; r.e_ph = ex; r.e_c = e_pc;
  HIP_TRY(ctx, timed_on(ctx, s, NLOS_PASS_RSD_PROPAGATE, [&] { return nlos::launch_rsd_propagate(r, s); }));
  // 5. y-IFFT per depth column, keep y < ny: C -> D[y][kx][d] (FP16: per-depth exponents)
  a = StridedArgs{};
  a.in = C; a.out = D; a.in_plane = Nds; a.in_line = Mx * Nds; a.out_plane = Nds; a.out_line = Mx * Nds;
  a.ncols = (int)Nd; a.n_in = (int)My; a.n_out = (int)ny; a.e_in = e_pc; a.e_out = e_pd; a.e_per_col = 1;
  HIP_TRY(ctx, timed_on(ctx, s, NLOS_PASS_RSD_YI, [&] {
    return p->gen_y ? nlos::launch_gen_strided(p->gy, true, nlos::ST_C64, a, (int)Mx, s)
                    : nlos::launch_strided((int)My, true, nlos::LD_C64, nlos::ST_C64, a, (int)Mx, tw, s, sp);
  }));
  // 6. x-IFFT, keep x < nx, |I| / (Mx My) -> vol[y][x][d], max over depth -> img
  a = StridedArgs{};
  a.in = D; a.out = d_vol; a.in_plane = Mx * Nds; a.in_line = Nds; a.out_plane = nx * Nd; a.out_line = Nd;
  a.ncols = (int)Nd; a.n_in = (int)Mx; a.n_out = (int)nx; a.e_in = e_pd; a.e_per_col = 1;
  a.oscale = (float)(1.0 / ((double)Mx * (double)My)); a.img = d_img; a.img_plane = nx;
  if (d_field) {  // the complex field I itself
    a.out = d_field; a.img = nullptr;
    HIP_TRY(ctx, timed_on(ctx, s, NLOS_PASS_RSD_XI, [&] {
      return p->gen_x ? nlos::launch_gen_strided(p->gx, true, nlos::ST_C64_SCALED, a, (int)ny, s)
                      : nlos::launch_strided((int)Mx, true, nlos::LD_C64, nlos::ST_C64_SCALED, a, (int)ny, tw, s, sp);
    }));
    return NLOS_OK;
  }
  // depth-major volume: |I| lands depth contiguous in region B (C is dead), then one
  // transpose pass writes d_vol[n_depth][ny][nx]
  const bool depth_major = d.vol_depth_major && d_vol != nullptr;
  float* vtmp = reinterpret_cast<float*>(base + L.b_off * es);
  if (depth_major) a.out = vtmp;
  HIP_TRY(ctx, timed_on(ctx, s, NLOS_PASS_RSD_XI, [&] {
    return p->gen_x ? nlos::launch_gen_strided(p->gx, true, nlos::ST_ABS_IMG, a, (int)ny, s)
                    : nlos::launch_strided((int)Mx, true, nlos::LD_C64, nlos::ST_ABS_IMG, a, (int)ny, tw, s, sp);
  }));
  if (depth_major)
    HIP_TRY(ctx, timed_on(ctx, s, NLOS_PASS_FILL, [&] {
      return nlos::launch_transpose_f32(vtmp, d_vol, ny * nx, (int)Nd, s);
    }));
  return NLOS_OK;
}

nlos_status nlos_rsd(nlos_ctx* ctx, const nlos_rsd_plan* p, const float* d_tau, float* d_vol, float* d_img,
                     void* d_ws, size_t ws_bytes) {
  if (!ctx || !p) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd: ctx or plan is NULL");
  if (!d_tau) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd: d_tau is NULL");
  if (p->d.data_prec == NLOS_FP16 && reinterpret_cast<uintptr_t>(d_tau) % 8 != 0)
    return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd: d_tau must be 8-byte aligned for FP16 data");
  if (!d_vol && !d_img) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd: d_vol and d_img are both NULL");
  if (p->device != ctx->device) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd: plan of another device");
  const RsdLayout L = rsd_layout(&p->d);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  void* ws = nullptr;
  nlos_status st = get_workspace(ctx, d_ws, ws_bytes, L.bytes, &ws);
  if (st != NLOS_OK) return st;
  return rsd_run(ctx, p, ctx->stream, d_tau, d_vol, d_img, ws);
}

nlos_status nlos_rsd_from_phasors(nlos_ctx* ctx, const nlos_rsd_plan* p, const float* d_phasor, float* d_vol,
                                  float* d_img, void* d_ws, size_t ws_bytes) {
  if (!ctx || !p) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd_from_phasors: ctx or plan is NULL");
  if (!d_phasor) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd_from_phasors: d_phasor is NULL");
  if (reinterpret_cast<uintptr_t>(d_phasor) % 8 != 0)
    return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd_from_phasors: d_phasor must be 8-byte aligned");
  if (!d_vol && !d_img) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd_from_phasors: d_vol and d_img are both NULL");
  if (p->device != ctx->device) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd_from_phasors: plan of another device");
  if (p->d.data_prec != NLOS_FP32)
    return fail(ctx, NLOS_ERR_UNSUPPORTED, "nlos_rsd_from_phasors: FP32 data plans only (the FP16 scales come from "
                                           "the transient)");
  const RsdLayout L = rsd_layout(&p->d);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  void* ws = nullptr;
  nlos_status st = get_workspace(ctx, d_ws, ws_bytes, L.bytes, &ws);
  if (st != NLOS_OK) return st;
  return rsd_run(ctx, p, ctx->stream, nullptr, d_vol, d_img, ws, reinterpret_cast<const float2*>(d_phasor));
}

nlos_status nlos_fk_complex(nlos_ctx* ctx, const nlos_fk_plan* p, const float* d_tau, float* d_psi, void* d_ws,
                            size_t ws_bytes) {
  if (!ctx || !p) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_fk_complex: ctx or plan is NULL");
  if (!d_tau || !d_psi) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_fk_complex: d_tau and d_psi are required");
  if (reinterpret_cast<uintptr_t>(d_tau) % 8 != 0 || reinterpret_cast<uintptr_t>(d_psi) % 8 != 0)
    return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_fk_complex: d_tau and d_psi must be 8-byte aligned");
  if (p->d.prec != NLOS_FP32) return fail(ctx, NLOS_ERR_UNSUPPORTED, "nlos_fk_complex: FP32 plans only");
  if (p->device != ctx->device) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_fk_complex: plan of another device");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  void* ws = nullptr;
  nlos_status st = get_workspace(ctx, d_ws, ws_bytes, fk_layout(&p->d).bytes, &ws);
  if (st != NLOS_OK) return st;
  return fk_run(ctx, p, ctx->stream, d_tau, nullptr, nullptr, ws, reinterpret_cast<float2*>(d_psi));
}

nlos_status nlos_rsd_complex(nlos_ctx* ctx, const nlos_rsd_plan* p, const float* d_tau, float* d_field, void* d_ws,
                             size_t ws_bytes) {
  if (!ctx || !p) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd_complex: ctx or plan is NULL");
  if (!d_tau || !d_field) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd_complex: d_tau and d_field are required");
  if (reinterpret_cast<uintptr_t>(d_field) % 8 != 0)
    return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd_complex: d_field must be 8-byte aligned");
  if (p->device != ctx->device) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd_complex: plan of another device");
  if (p->d.data_prec == NLOS_FP16 && reinterpret_cast<uintptr_t>(d_tau) % 8 != 0)
    return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd_complex: d_tau must be 8-byte aligned for FP16 data");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  void* ws = nullptr;
  nlos_status st = get_workspace(ctx, d_ws, ws_bytes, rsd_layout(&p->d).bytes, &ws);
  if (st != NLOS_OK) return st;
  return rsd_run(ctx, p, ctx->stream, d_tau, nullptr, nullptr, ws, nullptr, reinterpret_cast<float2*>(d_field));
}

// ---------------------------------------------------------------------------
// graph replay: one reconstruction with fixed buffers as an instantiated HIP graph
// ---------------------------------------------------------------------------

struct nlos_graph {
  int device = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// Captures run(stream) on a private default-priority stream and instantiates it.  Per-pass
// timing is suspended during the capture, so the graph holds the kernel launches only.
extern "C++" {
template <class Run>
static nlos_status capture_graph(nlos_ctx* ctx, const char* who, Run run, nlos_graph** out) {
  hipStream_t cs = nullptr;
  HIP_TRY(ctx, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  const bool timing = ctx->timing;
  ctx->timing = false;
  nlos_status st = NLOS_OK;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = run(cs);
    const hipError_t e_end = hipStreamEndCapture(cs, &g);
    if (st == NLOS_OK) e = e_end;
  }
  ctx->timing = timing;
  nlos_graph* gr = nullptr;
  if (st == NLOS_OK && e == hipSuccess) {
    gr = new (std::nothrow) nlos_graph();
    if (!gr) {
      st = fail(ctx, NLOS_ERR_OUT_OF_MEMORY, "%s: host allocation", who);
    } else {
      gr->device = ctx->device;
      gr->graph = g;
      e = hipGraphInstantiate(&gr->exec, g, nullptr, nullptr, 0);
    }
  }
  (void)hipStreamDestroy(cs);
  if (st != NLOS_OK || e != hipSuccess) {
    if (gr && gr->exec) (void)hipGraphExecDestroy(gr->exec);
    delete gr;
    if (g) (void)hipGraphDestroy(g);
    if (st != NLOS_OK) return st;
    return fail(ctx, e == hipErrorOutOfMemory ? NLOS_ERR_OUT_OF_MEMORY : NLOS_ERR_DEVICE, "%s: graph capture: %s",
                who, hipGetErrorString(e));
  }
  *out = gr;
  return NLOS_OK;
}
}  // extern "C++"

nlos_status nlos_fk_graph_create(nlos_ctx* ctx, const nlos_fk_plan* p, const float* d_tau, float* d_vol,
                                 float* d_img, void* d_ws, size_t ws_bytes, nlos_graph** out) {
  if (!ctx || !p || !out) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_fk_graph_create: NULL argument");
  if (!d_tau || !d_ws) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_fk_graph_create: d_tau and d_ws are required");
  if (reinterpret_cast<uintptr_t>(d_tau) % 8 != 0)
    return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_fk_graph_create: d_tau must be 8-byte aligned");
  if (!d_vol && !d_img) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_fk_graph_create: d_vol and d_img are both NULL");
  if (p->device != ctx->device) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_fk_graph_create: plan of another device");
  size_t need = 0;
  nlos_status st = nlos_fk_desc_workspace_bytes(&p->d, &need);
  if (st != NLOS_OK) return fail(ctx, st, "%s", g_err.c_str());
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  void* ws = nullptr;
  if ((st = get_workspace(ctx, d_ws, ws_bytes, need, &ws)) != NLOS_OK) return st;
  return capture_graph(
      ctx, "nlos_fk_graph_create", [&](hipStream_t cs) { return fk_run(ctx, p, cs, d_tau, d_vol, d_img, ws); }, out);
}

nlos_status nlos_rsd_graph_create(nlos_ctx* ctx, const nlos_rsd_plan* p, const float* d_tau, float* d_vol,
                                  float* d_img, void* d_ws, size_t ws_bytes, nlos_graph** out) {
  if (!ctx || !p || !out) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd_graph_create: NULL argument");
  if (!d_tau || !d_ws) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd_graph_create: d_tau and d_ws are required");
  if (p->d.data_prec == NLOS_FP16 && reinterpret_cast<uintptr_t>(d_tau) % 8 != 0)
    return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd_graph_create: d_tau must be 8-byte aligned for FP16 data");
  if (!d_vol && !d_img) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd_graph_create: d_vol and d_img are both NULL");
  if (p->device != ctx->device) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_rsd_graph_create: plan of another device");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  void* ws = nullptr;
  nlos_status st = get_workspace(ctx, d_ws, ws_bytes, rsd_layout(&p->d).bytes, &ws);
  if (st != NLOS_OK) return st;
  return capture_graph(
      ctx, "nlos_rsd_graph_create", [&](hipStream_t cs) { return rsd_run(ctx, p, cs, d_tau, d_vol, d_img, ws); }, out);
}

nlos_status nlos_graph_launch(nlos_ctx* ctx, const nlos_graph* g) {
  if (!ctx || !g) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_graph_launch: ctx or graph is NULL");
  if (g->device != ctx->device) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_graph_launch: graph of another device");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipGraphLaunch(g->exec, ctx->stream));
  return NLOS_OK;
}

nlos_status nlos_graph_destroy(nlos_graph* g) {
  if (!g) return NLOS_OK;
  (void)hipSetDevice(g->device);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return NLOS_OK;
}

// ---------------------------------------------------------------------------
// coherence-weighted temporal merging (Section 4.4, Eq. 8-9)
// ---------------------------------------------------------------------------

struct nlos_merge {
  int device = 0;
  long long n = 0;
  int window = 0;
  float eps = 0.f;
  long long pushed = 0;      // frames since the last reset
  float2* ring = nullptr;    // [window][n]
};

nlos_status nlos_merge_create(nlos_ctx* ctx, uint64_t n_values, int window, double eps, nlos_merge** out) {
  if (!ctx || !out) return fail(ctx, NLOS_ERR_INVALID_ARG, "merge_create: NULL argument");
  if (n_values == 0 || window < 1 || window > 64 || !(eps > 0.0) || !std::isfinite(eps))
    return fail(ctx, NLOS_ERR_INVALID_ARG, "merge_create: need n_values >= 1, window in [1, 64], eps > 0");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  nlos_merge* m = new (std::nothrow) nlos_merge();
  if (!m) return fail(ctx, NLOS_ERR_OUT_OF_MEMORY, "merge_create: host allocation");
  m->device = ctx->device;
  m->n = (long long)n_values;
  m->window = window;
  m->eps = (float)eps;
  hipError_t e = nlos::dev_alloc((void**)&m->ring, (size_t)window * n_values * sizeof(float2));
  if (e != hipSuccess) {
    delete m;
    return fail(ctx, e == hipErrorOutOfMemory ? NLOS_ERR_OUT_OF_MEMORY : NLOS_ERR_DEVICE, "merge_create: %s",
                hipGetErrorString(e));
  }
  *out = m;
  return NLOS_OK;
}

nlos_status nlos_merge_destroy(nlos_merge* m) {
  if (!m) return NLOS_OK;
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  if (m->ring) (void)hipFree(m->ring);
  delete m;
  return NLOS_OK;
}

nlos_status nlos_merge_reset(nlos_merge* m) {
  if (!m) return fail(nullptr, NLOS_ERR_INVALID_ARG, "merge_reset: NULL");
  m->pushed = 0;
  return NLOS_OK;
}

nlos_status nlos_merge_push(nlos_ctx* ctx, nlos_merge* m, const float* d_frame, float* d_merged, float* d_coherence) {
  if (!ctx || !m) return fail(ctx, NLOS_ERR_INVALID_ARG, "merge_push: ctx or merge is NULL");
  if (!d_frame || !d_merged) return fail(ctx, NLOS_ERR_INVALID_ARG, "merge_push: d_frame and d_merged are required");
  if (reinterpret_cast<uintptr_t>(d_frame) % 8 != 0)
    return fail(ctx, NLOS_ERR_INVALID_ARG, "merge_push: d_frame must be 8-byte aligned");
  if (m->device != ctx->device) return fail(ctx, NLOS_ERR_INVALID_ARG, "merge_push: state of another device");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const int slot = (int)(m->pushed % m->window);
  const int count = (int)std::min<long long>(m->pushed + 1, m->window);
  const int first = (int)((m->pushed + 1 - count) % m->window);
  HIP_TRY(ctx, timed(ctx, NLOS_PASS_MERGE, [&] {
    return nlos::launch_merge(reinterpret_cast<const float2*>(d_frame), m->ring, m->n, m->window, slot, first, count,
                              m->eps, d_merged, d_coherence, ctx->stream);
  }));
  ++m->pushed;
  return NLOS_OK;
}

// ---------------------------------------------------------------------------
// depth-dependent average (Section 4.4, DDA)
// ---------------------------------------------------------------------------

struct nlos_dda {
  int device = 0;
  long long nvox = 0;
  int nd = 0;
  int window = 0;
  long long pushed = 0;    // frames since the last reset
  float* ring = nullptr;   // [window][nvox][nd]
  float* w = nullptr;      // [nd][window]
};

nlos_status nlos_dda_default_weights(int n_depth, int window, float* weights) {
  if (n_depth < 1 || window < 1 || window > 64 || !weights)
    return fail(nullptr, NLOS_ERR_INVALID_ARG, "dda_default_weights: need n_depth >= 1, window in [1, 64]");
  for (int d = 0; d < n_depth; ++d) {
    // n_d = 1 + floor((window - 1) d / (n_depth - 1) + 1/2), in integers
    const long long nd = n_depth == 1 ? window
                                      : 1 + (2LL * (window - 1) * d + (n_depth - 1)) / (2LL * (n_depth - 1));
    for (int a = 0; a < window; ++a) weights[(size_t)d * window + a] = a < nd ? 1.f : 0.f;
  }
  return NLOS_OK;
}

nlos_status nlos_dda_create(nlos_ctx* ctx, uint64_t n_vox, int n_depth, int window, const float* weights,
                            nlos_dda** out) {
  try {
    if (!ctx || !out || !weights) return fail(ctx, NLOS_ERR_INVALID_ARG, "dda_create: NULL argument");
    if (n_vox == 0 || n_depth < 1 || window < 1 || window > 64)
      return fail(ctx, NLOS_ERR_INVALID_ARG, "dda_create: need n_vox >= 1, n_depth >= 1, window in [1, 64]");
    if (n_vox > (1ull << 40) / (uint64_t)n_depth)
      return fail(ctx, NLOS_ERR_UNSUPPORTED, "dda_create: volume too large");
    for (int d = 0; d < n_depth; ++d)
      for (int a = 0; a < window; ++a) {
        const float v = weights[(size_t)d * window + a];
        if (!std::isfinite(v) || v < 0.f || (a == 0 && !(v > 0.f)))
          return fail(ctx, NLOS_ERR_INVALID_ARG,
                      "dda_create: weights must be finite and >= 0, with weights[d][0] > 0 (d %d, a %d: %g)", d, a,
                      (double)v);
      }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    nlos::host_alloc_point();
    nlos_dda* m = new (std::nothrow) nlos_dda();
    if (!m) return fail(ctx, NLOS_ERR_OUT_OF_MEMORY, "dda_create: host allocation");
    m->device = ctx->device;
    m->nvox = (long long)n_vox;
    m->nd = n_depth;
    m->window = window;
    const size_t wbytes = (size_t)n_depth * window * sizeof(float);
    hipError_t e = nlos::dev_alloc((void**)&m->ring, (size_t)window * n_vox * n_depth * sizeof(float));
    if (e == hipSuccess) e = nlos::dev_alloc((void**)&m->w, wbytes);
    if (e == hipSuccess) e = hipMemcpy(m->w, weights, wbytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      nlos_dda_destroy(m);
      return fail(ctx, e == hipErrorOutOfMemory ? NLOS_ERR_OUT_OF_MEMORY : NLOS_ERR_DEVICE, "dda_create: %s",
                  hipGetErrorString(e));
    }
    *out = m;
    return NLOS_OK;
  } catch (const std::bad_alloc&) {
    return fail(ctx, NLOS_ERR_OUT_OF_MEMORY, "nlos_dda_create: host allocation failed");
  }
}

nlos_status nlos_dda_destroy(nlos_dda* m) {
  if (!m) return NLOS_OK;
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  if (m->ring) (void)hipFree(m->ring);
  if (m->w) (void)hipFree(m->w);
  delete m;
  return NLOS_OK;
}

nlos_status nlos_dda_reset(nlos_dda* m) {
  if (!m) return fail(nullptr, NLOS_ERR_INVALID_ARG, "dda_reset: NULL");
  m->pushed = 0;
  return NLOS_OK;
}

nlos_status nlos_dda_push(nlos_ctx* ctx, nlos_dda* m, const float* d_vol, float* d_avg, float* d_img) {
  if (!ctx || !m) return fail(ctx, NLOS_ERR_INVALID_ARG, "dda_push: ctx or state is NULL");
  if (!d_vol) return fail(ctx, NLOS_ERR_INVALID_ARG, "dda_push: d_vol is NULL");
  if (!d_avg && !d_img) return fail(ctx, NLOS_ERR_INVALID_ARG, "dda_push: d_avg and d_img are both NULL");
  if (reinterpret_cast<uintptr_t>(d_vol) % 4 != 0 || reinterpret_cast<uintptr_t>(d_avg) % 4 != 0 ||
      reinterpret_cast<uintptr_t>(d_img) % 4 != 0)
    return fail(ctx, NLOS_ERR_INVALID_ARG, "dda_push: buffers must be 4-byte aligned");
  if (m->device != ctx->device) return fail(ctx, NLOS_ERR_INVALID_ARG, "dda_push: state of another device");
  const size_t nv = (size_t)m->nvox * m->nd;
  const char* vb = reinterpret_cast<const char*>(d_vol);
  const char* ve = vb + nv * sizeof(float);
  auto overlaps = [&](const void* p, size_t n) {
    const char* b = static_cast<const char*>(p);
    return p != nullptr && b < ve && vb < b + n * sizeof(float);
  };
  if (overlaps(d_avg, nv) || overlaps(d_img, (size_t)m->nvox))
    return fail(ctx, NLOS_ERR_INVALID_ARG, "dda_push: d_vol overlaps an output");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const int slot = (int)(m->pushed % m->window);
  const int count = (int)std::min<long long>(m->pushed + 1, m->window);
  HIP_TRY(ctx, timed(ctx, NLOS_PASS_DDA, [&] {
    return nlos::launch_dda(d_vol, m->ring, m->w, m->nvox, m->nd, m->window, slot, count, d_avg, d_img,
                            ctx->stream);
  }));
  ++m->pushed;
  return NLOS_OK;
}

// ---------------------------------------------------------------------------
// mixture of experts (Section 4.4, Eq. 10)
// ---------------------------------------------------------------------------

struct nlos_moe_plan {
  nlos_fk_plan* fk = nullptr;
  nlos_rsd_plan* rsd = nullptr;
  float beta = 0.3f, eps = 1e-6f;
  int shared = 0;  // 1: both branches read one shared spatial spectrum
  int device = 0;
};

static bool close_rel(double a, double b) { return std::fabs(a - b) <= 1e-9 * std::max(std::fabs(a), std::fabs(b)); }

nlos_status nlos_moe_check(const nlos_fk_desc* fk, const nlos_rsd_desc* rsd, double beta, double eps) {
  nlos_status st = nlos_fk_check(fk);
  if (st != NLOS_OK) return st;
  st = nlos_rsd_check(rsd);
  if (st != NLOS_OK) return st;
  if (fk->nx != rsd->nx || fk->ny != rsd->ny || fk->nt != rsd->nt || fk->pad != rsd->pad ||
      !close_rel(fk->bin_ps, rsd->bin_ps) || !close_rel(fk->wall_w_m / fk->nx, rsd->dx_m) ||
      !close_rel(fk->wall_h_m / fk->ny, rsd->dy_m))
    return fail(nullptr, NLOS_ERR_INVALID_ARG,
                "moe: the f-k and RSD descriptors must describe the same transient and grid");
  if (fk->prec != NLOS_FP32 || rsd->data_prec != NLOS_FP32)
    return fail(nullptr, NLOS_ERR_UNSUPPORTED, "moe: FP32 intermediates only");
  if (!fk_all_pow2(fk))
    return fail(nullptr, NLOS_ERR_UNSUPPORTED, "moe: power-of-two padded sizes only");
  if (!(beta >= 0.0) || !std::isfinite(beta) || !(eps > 0.0) || !std::isfinite(eps))
    return fail(nullptr, NLOS_ERR_INVALID_ARG, "moe: need beta >= 0 and eps > 0, finite");
  return NLOS_OK;
}

// MoE workspace: the f-k workspace (its W2 is the shared spatial spectrum), the RSD
// workspace (P^, C, D) and the two branch images.
struct MoeLayout {
  size_t rsd_off, img_off, bytes;
};
static MoeLayout moe_layout(const nlos_fk_desc* fk, const nlos_rsd_desc* rsd) {
  MoeLayout L;
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  L.rsd_off = up(fk_layout(fk).bytes);
  L.img_off = L.rsd_off + up(rsd_layout(rsd).bytes);
  L.bytes = L.img_off + up(2 * sizeof(float) * (size_t)fk->nx * fk->ny) + 256;  // + 3 maxima
  return L;
}

nlos_status nlos_moe_workspace_bytes(const nlos_fk_desc* fk, const nlos_rsd_desc* rsd, size_t* bytes) {
  nlos_status st = nlos_moe_check(fk, rsd, 0.3, 1e-6);
  if (st != NLOS_OK) return st;
  if (!bytes) return fail(nullptr, NLOS_ERR_INVALID_ARG, "moe: bytes is NULL");
  *bytes = moe_layout(fk, rsd).bytes;
  return NLOS_OK;
}

nlos_status nlos_moe_plan_create(nlos_ctx* ctx, const nlos_fk_desc* fk, const nlos_rsd_desc* rsd, double beta,
                                 double eps, int shared_spectrum, nlos_moe_plan** out) {
  if (!ctx || !out) return fail(ctx, NLOS_ERR_INVALID_ARG, "moe_plan_create: NULL argument");
  nlos_status st = nlos_moe_check(fk, rsd, beta, eps);
  if (st != NLOS_OK) return fail(ctx, st, "%s", g_err.c_str());
  nlos_moe_plan* p = new (std::nothrow) nlos_moe_plan();
  if (!p) return fail(ctx, NLOS_ERR_OUT_OF_MEMORY, "moe_plan_create: host allocation");
  p->device = ctx->device;
  p->beta = (float)beta;
  p->eps = (float)eps;
  p->shared = shared_spectrum ? 1 : 0;
  st = nlos_fk_plan_create(ctx, fk, &p->fk);
  if (st == NLOS_OK) st = nlos_rsd_plan_create(ctx, rsd, &p->rsd);
  if (st != NLOS_OK) {
    nlos_fk_plan_destroy(p->fk);
    delete p;
    return st;
  }
  *out = p;
  return NLOS_OK;
}

nlos_status nlos_moe_plan_destroy(nlos_moe_plan* p) {
  if (!p) return NLOS_OK;
  nlos_fk_plan_destroy(p->fk);
  nlos_rsd_plan_destroy(p->rsd);
  delete p;
  return NLOS_OK;
}

nlos_status nlos_moe(nlos_ctx* ctx, const nlos_moe_plan* p, const float* d_tau, float* d_img, float* d_img_fk,
                     float* d_img_rsd, void* d_ws, size_t ws_bytes) {
  if (!ctx || !p) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_moe: ctx or plan is NULL");
  if (!d_tau || !d_img) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_moe: d_tau and d_img are required");
  if (reinterpret_cast<uintptr_t>(d_tau) % 8 != 0)
    return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_moe: d_tau must be 8-byte aligned");
  if (p->device != ctx->device) return fail(ctx, NLOS_ERR_INVALID_ARG, "nlos_moe: plan of another device");
  const nlos_fk_desc& fd = p->fk->d;
  const nlos_rsd_desc& rd = p->rsd->d;
  const MoeLayout ML = moe_layout(&fd, &rd);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  void* ws = nullptr;
  nlos_status st = get_workspace(ctx, d_ws, ws_bytes, ML.bytes, &ws);
  if (st != NLOS_OK) return st;
  const long long nx = fd.nx, ny = fd.ny, nt = fd.nt, Mx = p->fk->Mx, My = p->fk->My;
  const long long Nf = rd.n_freq, Nd = rd.n_depth;
  const FkLayout L = fk_layout(&fd);
  const RsdLayout R = rsd_layout(&rd);
  char* base = static_cast<char*>(ws);
  float2* W1 = reinterpret_cast<float2*>(base);
  float2* W2 = W1 + L.w2_off;          // shared spatial half spectrum [My][Mx/2+1][nt]
  float2* W3 = W1 + L.b_off;
  float2* W4 = W1;
  float2* W5 = W3;
  float2* rbase = reinterpret_cast<float2*>(base + ML.rsd_off);
  float2* Ph = rbase + R.e_off;        // [My][Mx][Nf]
  float2* Cr = rbase + R.b_off;        // [My][Mx][Nd]
  float2* Dr = rbase;                  // [ny][Mx][Nd]
  float* scratch = reinterpret_cast<float*>(base + ML.img_off);  // two images
  unsigned int* mx = reinterpret_cast<unsigned int*>(base + ML.bytes - 256);
  float* img_fk = d_img_fk ? d_img_fk : scratch;
  float* img_rsd = d_img_rsd ? d_img_rsd : scratch + nx * ny;
  const long long RH = (long long)L.rs_half, RF = (long long)L.rs_full;
  hipStream_t s0 = ctx->stream, s1 = ctx->aux;
  const float2* tw = ctx->d_tw;
  if (!p->shared) {
    // the two complete reconstructions one after the other on the context stream (each
    // fills the device by itself: overlapping the independent branches on two streams
    // measured slower than this order)
    nlos_status st1 = rsd_run(ctx, p->rsd, s0, d_tau, nullptr, img_rsd, base + ML.rsd_off);
    if (st1 != NLOS_OK) return st1;
    st1 = fk_run(ctx, p->fk, s0, d_tau, nullptr, img_fk, base);
    if (st1 != NLOS_OK) return st1;
    HIP_TRY(ctx, timed(ctx, NLOS_PASS_MOE_MIX, [&] {
      return nlos::launch_moe_mix(img_fk, img_rsd, d_img, (int)(nx * ny), p->beta, p->eps, mx, s0);
    }));
    return NLOS_OK;
  }
  if (!ctx->aux) {
    HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));  // default priority
    for (auto& e : ctx->fork) HIP_TRY(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    s1 = ctx->aux;
  }
  HIP_TRY(ctx, timed(ctx, NLOS_PASS_FILL, [&] {
    hipError_t e = nlos::launch_fill_u32(reinterpret_cast<uint32_t*>(img_fk), (size_t)nx * ny, 0u, s0);
    return e != hipSuccess ? e : nlos::launch_fill_u32(reinterpret_cast<uint32_t*>(img_rsd), (size_t)nx * ny, 0u, s0);
  }));
  // shared: x and y FFTs of the (unscaled) transient -> W2
  FkXArgs x{};
  x.tau = d_tau; x.out = W1; x.out_plane = RH; x.nx = (int)nx; x.nt = (int)nt;
  x.tscale = (float)(1.0 / (double)(nt - 1)); x.unscaled = 1;
  HIP_TRY(ctx, timed(ctx, NLOS_PASS_FK_X, [&] { return nlos::launch_fk_xr2c((int)Mx, x, (int)ny, tw, s0); }));
  StridedArgs a{};
  a.in = W1; a.out = W2;
  a.in_plane = nt; a.in_line = RH; a.out_plane = nt; a.out_line = RH;
  a.ncols = (int)nt; a.n_in = (int)ny; a.n_out = (int)My;
  HIP_TRY(ctx, timed(ctx, NLOS_PASS_FK_Y, [&] { return nlos::launch_strided((int)My, false, nlos::LD_C64, nlos::ST_C64, a, (int)(Mx / 2 + 1), tw, s0, nlos::SP_F32, true); }));
  // fork: the RSD branch on the second stream
  HIP_TRY(ctx, hipEventRecord(ctx->fork[0], s0));
  HIP_TRY(ctx, hipStreamWaitEvent(s1, ctx->fork[0], 0));
  const long long nwork = (Mx / 2 - 1) * My + 2 * (My / 2 + 1);
  nlos::MoePhasorArgs ph{};
  ph.in = W2; ph.out = Ph; ph.in_row = RH; ph.nwork = nwork; ph.nt = (int)nt; ph.Mx = (int)Mx; ph.My = (int)My;
  ph.nbins = (int)Nf; ph.bins = p->rsd->d_bins;
  HIP_TRY(ctx, timed_on(ctx, s1, NLOS_PASS_MOE_PHASOR, [&] { return nlos::launch_moe_phasor_pair(ph, tw, s1); }));
  HIP_TRY(ctx, hipEventRecord(ctx->fork[1], s1));  // W2 no longer read by the RSD branch
  nlos::RsdPropArgs r{};
  r.Ph = Ph; r.Kr = p->rsd->d_kr; r.w = p->rsd->d_w; r.C = Cr;
  r.chunk_i0 = p->rsd->d_chunk_i0; r.chunk_pix = p->rsd->d_chunk_pix; r.chunk_wa = p->rsd->d_chunk_wa;
  r.chunk_wb = p->rsd->d_chunk_wb; r.nchunks = p->rsd->nchunks;
  r.Nf = (int)Nf; r.Nd = (int)Nd; r.ph_stride = (int)Nf; r.c_stride = (int)Nd;
  r.cut_idx = p->rsd->g.cut_idx; r.kernel_sp = fk_sp(rd.kernel_prec); r.mfma = ctx->rsd_mfma;
  HIP_TRY(ctx, timed_on(ctx, s1, NLOS_PASS_RSD_PROPAGATE, [&] { return nlos::launch_rsd_propagate(r, s1); }));
  a = StridedArgs{};
  a.in = Cr; a.out = Dr; a.in_plane = Nd; a.in_line = Mx * Nd; a.out_plane = Nd; a.out_line = Mx * Nd;
  a.ncols = (int)Nd; a.n_in = (int)My; a.n_out = (int)ny;
  HIP_TRY(ctx, timed_on(ctx, s1, NLOS_PASS_RSD_YI, [&] { return nlos::launch_strided((int)My, true, nlos::LD_C64, nlos::ST_C64, a, (int)Mx, tw, s1); }));
  a = StridedArgs{};
  a.in = Dr; a.out = nullptr; a.in_plane = Mx * Nd; a.in_line = Nd; a.out_plane = nx * Nd; a.out_line = Nd;
  a.ncols = (int)Nd; a.n_in = (int)Mx; a.n_out = (int)nx;
  a.oscale = (float)(1.0 / ((double)Mx * (double)My)); a.img = img_rsd; a.img_plane = nx;
  HIP_TRY(ctx, timed_on(ctx, s1, NLOS_PASS_RSD_XI, [&] { return nlos::launch_strided((int)Mx, true, nlos::LD_C64, nlos::ST_ABS_IMG, a, (int)ny, tw, s1); }));
  HIP_TRY(ctx, hipEventRecord(ctx->fork[2], s1));
  // f-k branch on the context stream: the t/(nt-1) scaling is applied as the columns load
  FkPairArgs c{};
  c.in = W2; c.out = W3; c.in_row = RH; c.out_row = RF; c.nwork = nwork;
  c.nt = (int)nt; c.Mx = (int)Mx; c.My = (int)My;
  c.sxk = p->fk->sxk; c.syk = p->fk->syk; c.norm = p->fk->norm;
  c.tscale_in = (float)(1.0 / (double)(nt - 1));
  HIP_TRY(ctx, timed(ctx, NLOS_PASS_FK_COLUMN, [&] { return nlos::launch_fk_column_pair(p->fk->Mt, c, tw, s0); }));
  HIP_TRY(ctx, hipStreamWaitEvent(s0, ctx->fork[1], 0));  // W4 overwrites W2
  a = StridedArgs{};
  a.in = W3; a.out = W4;
  a.in_plane = nt; a.in_line = RF; a.out_plane = nt; a.out_line = RF;
  a.ncols = (int)nt; a.n_in = (int)My; a.n_out = (int)ny;
  HIP_TRY(ctx, timed(ctx, NLOS_PASS_FK_YI, [&] { return nlos::launch_strided((int)My, true, nlos::LD_C64, nlos::ST_C64, a, (int)Mx, tw, s0, nlos::SP_F32, true); }));
  a = StridedArgs{};
  a.in = W4; a.out = W5;
  a.in_plane = RF; a.in_line = nt; a.out_plane = nx * nt; a.out_line = nt;
  a.ncols = (int)nt; a.n_in = (int)Mx; a.n_out = (int)nx;
  HIP_TRY(ctx, timed(ctx, NLOS_PASS_FK_XI, [&] { return nlos::launch_strided((int)Mx, true, nlos::LD_C64, nlos::ST_C64, a, (int)ny, tw, s0, nlos::SP_F32, true); }));
  ContigArgs z{};
  z.in = W5; z.out = nullptr; z.nlines = ny * nx; z.in_line = nt; z.out_line = nt;
  z.n_in = (int)nt; z.n_out = (int)nt; z.oscale = 1.0f; z.img = img_fk;
  HIP_TRY(ctx, timed(ctx, NLOS_PASS_FK_ZI, [&] { return nlos::launch_contig(p->fk->Mt, true, nlos::CL_C64, nlos::CS_ABS2_MAX, z, tw, s0); }));
  // join and mix (Eq. 10)
  HIP_TRY(ctx, hipStreamWaitEvent(s0, ctx->fork[2], 0));
  HIP_TRY(ctx, timed(ctx, NLOS_PASS_MOE_MIX, [&] {
    return nlos::launch_moe_mix(img_fk, img_rsd, d_img, (int)(nx * ny), p->beta, p->eps, mx, s0);
  }));
  return NLOS_OK;
}

}  // extern "C"
