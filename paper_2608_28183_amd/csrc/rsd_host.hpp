// Plan-time host math for the radial RSD, in FP64: the radial sampling rules of
// the supplementary material, the radial kernel K_r of Eq. 4-6 and the
// pixel-to-radius map; also the FP64 twiddle generator.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace nlos {

constexpr int kTwiddleTableN = 2048;

// cos and sin of 2 pi k / n, with the angle reduced to the first octant in
// exact integer arithmetic before calling std::cos / std::sin.
void cos_sin_2pi_frac(long long k, long long n, double* c, double* s);

struct RsdInputs {
  int nx, ny, nt, pad;
  double dx, dy, c_dt;
  int n_freq;
  const int32_t* freq_bin;
  int n_depth;
  double depth0, depth_step;
  int sigma_s, sigma_t;
  double delta;
};

struct RsdGeometry {
  double r_max, rho_max, lambda_min, dr, f_s, rho_cut, rho_cut_bin;
  int n_r_min, n_r, n_rho_min, n_rho, cut_idx, last_base;
};

RsdGeometry rsd_geometry(const RsdInputs& in);
// K_r[i][f][d] (re, im) for i < n_rho, f < n_freq, d < n_depth.
void rsd_radial_kernel(const RsdInputs& in, const RsdGeometry& g, std::vector<double>& re,
                       std::vector<double>& im);
// rho~(u, v) in bin units on the My x Mx grid, signed FFT indices (FP64).
void rsd_radius_map(const RsdInputs& in, const RsdGeometry& g, std::vector<double>& rho);

// Pixel lookup of Listing 3 grouped for the propagation kernel.  Each Fourier pixel
// with a positive taper weight a gets i0 = clamp(floor(rho~), 0, lastBase),
// alpha = rho~ - i0 and the two tap weights wa = a (1 - alpha), wb = a alpha (the
// second tap is row min(i0 + 1, cutIdx)).  Pixels are sorted by i0 and cut into
// chunks of at most kChunk pixels with one i0; pixels with a = 0 form chunks with
// i0 = -1 (their spectrum is zero).  Slot j of chunk c is pix[c * kChunk + j]
// (-1 when unused).
constexpr int kChunk = 64;
struct RsdChunks {
  std::vector<int> i0;
  std::vector<int> pix;
  std::vector<float> wa, wb;
  int count() const { return (int)i0.size(); }
};
void rsd_build_chunks(const RsdInputs& in, const RsdGeometry& g, RsdChunks& out);

}  // namespace nlos
