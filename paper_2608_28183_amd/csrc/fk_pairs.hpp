// Work items of the paired f-k column pass (shared by its FP32 and matrix-core forms).
#pragma once

#include <hip/hip_runtime.h>

namespace nlos {

// Work item w -> input column (kx, ky) of the half spectrum and its mirror (kx2, ky2).
// Columns 1 <= kx < Mx/2 pair with (Mx - kx, -ky); on the planes kx = 0 and kx = Mx/2
// the mirror stays on the plane, so only ky in [0, My/2] is taken there, and ky = 0,
// My/2 are their own mirrors.
struct PairItem {
  int kx, ky, kx2, ky2;
  bool has_mirror;
};

// The work counts stay below 2^24 (Mx, My <= 4096): 32-bit unsigned arithmetic, not the
// much longer 64-bit division.
__device__ __forceinline__ PairItem pair_item(long long w64, int Mx, int My) {
  PairItem it;
  const unsigned w = (unsigned)w64, my = (unsigned)My;
  const unsigned nmain = (unsigned)(Mx / 2 - 1) * my;
  if (w < nmain) {
    it.kx = 1 + int(w / my);
    it.ky = int(w % my);
    it.kx2 = Mx - it.kx;
    it.ky2 = it.ky == 0 ? 0 : My - it.ky;
    it.has_mirror = true;
  } else {
    const unsigned half = my / 2 + 1;
    const unsigned w2 = w - nmain;
    it.kx = (w2 < half) ? 0 : Mx / 2;
    it.ky = int(w2 % half);
    it.kx2 = it.kx;
    it.ky2 = it.ky == 0 ? 0 : My - it.ky;
    it.has_mirror = (it.ky != 0) && (it.ky != My / 2);
  }
  return it;
}

}  // namespace nlos
