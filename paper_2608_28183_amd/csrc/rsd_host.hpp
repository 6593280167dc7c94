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
// rho~(u, v) in bin units on the My x Mx grid, signed FFT indices.
void rsd_radius_map(const RsdInputs& in, const RsdGeometry& g, std::vector<float>& rho);

}  // namespace nlos
