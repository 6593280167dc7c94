// Constant DFT-matrix operands of the matrix-core FFT stages (see mfma_fft.hpp), built
// on the host in FP64 with the angles reduced exactly in integers, then rounded once to
// binary16 or bfloat16.  Each operand is 64 lanes x 8 values.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "nlos_internal.hpp"
#include "rsd_host.hpp"

namespace nlos {

uint16_t to_f16_bits(double v) {
  const _Float16 h = (_Float16)v;  // one rounding, to nearest even
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}

uint16_t to_bf16_bits(double v) {
  const float f = (float)v;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}

namespace {

// Entry (c, k; n, cin) of the real form of F[k][n] = scale exp(-+2 pi i k n / R):
// output part c (0 re, 1 im) of complex output k, input part cin of complex input n.
double entry(int R, bool inverse, double scale, int c, int k, int n, int cin) {
  double cs, sn;
  cos_sin_2pi_frac((long long)k * n % R, R, &cs, &sn);
  const double fr = scale * cs, fi = (inverse ? 1.0 : -1.0) * scale * sn;
  if (c == 0) return cin == 0 ? fr : -fi;
  return cin == 0 ? fi : fr;
}

// Appends one operand: lane l holds K values 8 (l / 32) + s of K step q, s = 0..7, i.e.
// complex input n = 8 q + 4 (l / 32) + s / 2, part s % 2; (c, k) = out(l % 32).
template <class Out>
void operand(std::vector<uint16_t>& dst, int R, bool inverse, double scale, int q, bool bf16, Out out) {
  for (int l = 0; l < 64; ++l) {
    int c = 0, k = 0;
    out(l % 32, &c, &k);
    for (int s = 0; s < 8; ++s) {
      const int n = 8 * q + 4 * (l / 32) + s / 2;
      const double v = entry(R, inverse, scale, c, k, n, s % 2);
      dst.push_back(bf16 ? to_bf16_bits(v) : to_f16_bits(v));
    }
  }
}

}  // namespace

hipError_t mfma_tables_create(int device, void** d_buf, MfmaTables* t) {
  std::vector<uint16_t> h;
  struct Pending {
    const void** slot;
    size_t off;
  };
  std::vector<Pending> pend;
  for (int inv = 0; inv < 2; ++inv)
    for (int sc = 0; sc < 2; ++sc)
      for (int bf = 0; bf < 2; ++bf) {
        // A-const radix 16 and 32: rows are outputs, a 32-row block holds outputs
        // 16 b .. 16 b + 15 (rows 0..15 real parts, 16..31 imaginary parts)
        for (int R : {16, 32}) {
          pend.push_back({R == 16 ? &t->a16[inv][sc][bf] : &t->a32[inv][sc][bf], h.size()});
          const double scale = sc ? 1.0 / R : 1.0;
          for (int b = 0; b < R / 16; ++b)
            for (int q = 0; q < R / 8; ++q)
              operand(h, R, inv, scale, q, bf, [&](int row, int* c, int* k) {
                *c = row / 16;
                *k = 16 * b + row % 16;
              });
        }
        // B-const radix 32: columns are outputs, block c holds part c of outputs 0..31
        pend.push_back({&t->b32[inv][sc][bf], h.size()});
        for (int c = 0; c < 2; ++c)
          for (int q = 0; q < 4; ++q)
            operand(h, 32, inv, sc ? 1.0 / 32 : 1.0, q, bf, [&](int col, int* cc, int* k) {
              *cc = c;
              *k = col;
            });
      }
  *d_buf = nullptr;
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = dev_alloc(d_buf, h.size() * sizeof(uint16_t));
  if (e != hipSuccess) return e;
  e = hipMemcpy(*d_buf, h.data(), h.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(*d_buf);
    *d_buf = nullptr;
    return e;
  }
  for (const Pending& p : pend) *p.slot = static_cast<const uint16_t*>(*d_buf) + p.off;
  return hipSuccess;
}

}  // namespace nlos
