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

__device__ __forceinline__ PairItem pair_item(long long w, int Mx, int My) {
  PairItem it;
  const long long nmain = (long long)(Mx / 2 - 1) * My;
  if (w < nmain) {
    it.kx = 1 + int(w / My);
    it.ky = int(w % My);
    it.kx2 = Mx - it.kx;
    it.ky2 = it.ky == 0 ? 0 : My - it.ky;
    it.has_mirror = true;
  } else {
    const int half = My / 2 + 1;
    const int w2 = int(w - nmain);
    it.kx = (w2 < half) ? 0 : Mx / 2;
    it.ky = w2 % half;
    it.kx2 = it.kx;
    it.ky2 = it.ky == 0 ? 0 : My - it.ky;
    it.has_mirror = (it.ky != 0) && (it.ky != My / 2);
  }
  return it;
}

}  // namespace nlos
