// Plan-time host math for the radial RSD (FP64).  See rsd_host.hpp.
#include "rsd_host.hpp"

#include <algorithm>
#include <cmath>
#include <thread>

namespace nlos {

namespace {
constexpr double kPi = 3.14159265358979323846264338327950288;

// ceil of a quantity that is an integer in exact arithmetic must not be bumped
// up by the rounding of the products that form it: 1e-9 relative tolerance.
long long ceil_tol(double x) { return (long long)std::ceil(x - 1e-9 * std::fabs(x)); }

long long pow2_at_least(long long n) {
  long long p = 1;
  while (p < n) p <<= 1;
  return p;
}

template <class F>
void parallel_for(long long n, F f) {
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 64 || nth == 1) {
    for (long long i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nth; ++t)
    th.emplace_back([=] {
      for (long long i = t; i < n; i += nth) f(i);
    });
  for (auto& x : th) x.join();
}
}  // namespace

void cos_sin_2pi_frac(long long k, long long n, double* c, double* s) {
  k %= n;
  if (k < 0) k += n;
  // angle = 2 pi k / n = (pi / 4) * (8 k / n): octant o and remainder within it
  const long long o = (8 * k) / n;
  const long long rem = 8 * k - o * n;  // remaining angle (pi/4) rem / n
  double base_c, base_s;
  // angle within the octant pair: theta = (pi/4) (o + rem/n)
  // use symmetric reduction: for odd octants measure from the next multiple of pi/4
  const double frac = double(rem) / double(n);
  double t;
  if (o % 2 == 0) {
    t = 0.25 * kPi * frac;  // in [0, pi/4)
  } else {
    t = 0.25 * kPi * (1.0 - frac);  // distance back from (o+1) pi/4
  }
  const double ct = std::cos(t), st = std::sin(t);
  // quadrant q = o / 2; within quadrant, angle a = (pi/2)(o%2) + sign * t
  const long long q = o / 2;
  if (o % 2 == 0) {
    base_c = ct;
    base_s = st;
  } else {  // a = pi/2 - t
    base_c = st;
    base_s = ct;
  }
  double cc = base_c, ss = base_s;
  switch (q) {
    case 1: cc = -base_s; ss = base_c; break;
    case 2: cc = -base_c; ss = -base_s; break;
    case 3: cc = base_s; ss = -base_c; break;
    default: break;
  }
  *c = cc;
  *s = ss;
}

RsdGeometry rsd_geometry(const RsdInputs& in) {
  RsdGeometry g{};
  const int Mx = in.pad * in.nx, My = in.pad * in.ny;
  g.r_max = std::sqrt((0.5 * Mx * in.dx) * (0.5 * Mx * in.dx) + (0.5 * My * in.dy) * (0.5 * My * in.dy));
  g.rho_max = std::sqrt((0.5 / in.dx) * (0.5 / in.dx) + (0.5 / in.dy) * (0.5 / in.dy));
  int kmax = 1;
  for (int f = 0; f < in.n_freq; ++f) kmax = std::max(kmax, (int)in.freq_bin[f]);
  // shortest reconstructed wavelength: 2 pi / kappa_max with kappa = 2 pi k / (nt c dt)
  g.lambda_min = (double)in.nt * in.c_dt / (double)kmax;
  g.n_r_min = (int)(ceil_tol(2.0 * in.sigma_s * g.r_max / g.lambda_min) + 1);
  g.n_r = (int)std::max(2LL, pow2_at_least(g.n_r_min));
  g.dr = g.r_max / (g.n_r - 1);
  g.n_rho_min = (int)(ceil_tol(2.0 * g.r_max * g.rho_max) + 1);
  g.n_rho = (int)pow2_at_least(g.n_rho_min);
  g.f_s = (g.n_r - 1) / g.r_max;
  g.rho_cut = std::min(g.rho_max, 0.5 * g.f_s);
  g.rho_cut_bin = g.rho_cut * (g.n_rho - 1) / g.rho_max;
  g.cut_idx = std::min(g.n_rho - 1, (int)std::ceil(g.rho_cut_bin));
  g.last_base = std::max(0, std::min(g.cut_idx - 1, g.n_rho - 2));
  return g;
}

void rsd_radial_kernel(const RsdInputs& in, const RsdGeometry& g, std::vector<double>& re,
                       std::vector<double>& im) {
  const int NR = g.n_r, NP = g.n_rho, NF = in.n_freq, ND = in.n_depth;
  // ring radii, trapezoid weights and ring basis B(r_j, rho_i) = 2 pi r_j J0(2 pi r_j rho_i)
  std::vector<double> r(NR), q(NR, g.dr);
  for (int j = 0; j < NR; ++j) r[j] = j * g.dr;
  q[0] = q[NR - 1] = 0.5 * g.dr;
  std::vector<double> B((size_t)NP * NR);
  parallel_for(NP, [&](long long i) {
    const double rho = (double)i * g.rho_max / (double)(NP - 1);
    for (int j = 0; j < NR; ++j) B[(size_t)i * NR + j] = 2.0 * kPi * r[j] * std::cyl_bessel_j(0.0, 2.0 * kPi * r[j] * rho);
  });
  // ring coefficients q_j A(r_j, d, f), A = exp(i sigma_s kappa sqrt(r^2 + d^2))
  const size_t FD = (size_t)NF * ND;
  std::vector<double> Are(FD * NR), Aim(FD * NR), Pre(FD), Pim(FD);
  parallel_for((long long)FD, [&](long long fd) {
    const int f = (int)(fd / ND), d = (int)(fd % ND);
    const double kappa = 2.0 * kPi * in.freq_bin[f] / ((double)in.nt * in.c_dt);
    const double depth = in.depth0 + d * in.depth_step;
    for (int j = 0; j < NR; ++j) {
      const double ph = in.sigma_s * kappa * std::sqrt(r[j] * r[j] + depth * depth);
      Are[fd * NR + j] = q[j] * std::cos(ph);
      Aim[fd * NR + j] = q[j] * std::sin(ph);
    }
    const double m = kappa * (in.sigma_t * depth + in.delta);  // modality phase, applied after the sum
    Pre[fd] = std::cos(m);
    Pim[fd] = std::sin(m);
  });
  re.assign((size_t)NP * FD, 0.0);
  im.assign((size_t)NP * FD, 0.0);
  parallel_for(NP, [&](long long i) {
    if ((double)i > g.rho_cut_bin + 1e-9) return;  // beyond the cutoff: zero
    const double* b = &B[(size_t)i * NR];
    for (size_t fd = 0; fd < FD; ++fd) {
      const double* ar = &Are[fd * NR];
      const double* ai = &Aim[fd * NR];
      double sr = 0.0, si = 0.0;
      for (int j = 0; j < NR; ++j) {
        sr += b[j] * ar[j];
        si += b[j] * ai[j];
      }
      re[(size_t)i * FD + fd] = sr * Pre[fd] - si * Pim[fd];
      im[(size_t)i * FD + fd] = sr * Pim[fd] + si * Pre[fd];
    }
  });
}

void rsd_radius_map(const RsdInputs& in, const RsdGeometry& g, std::vector<double>& rho) {
  const int Mx = in.pad * in.nx, My = in.pad * in.ny;
  rho.resize((size_t)My * Mx);
  for (int u = 0; u < My; ++u) {
    const int us = u < My / 2 ? u : u - My;
    const double fu = us / (My * in.dy);
    for (int v = 0; v < Mx; ++v) {
      const int vs = v < Mx / 2 ? v : v - Mx;
      const double fv = vs / (Mx * in.dx);
      rho[(size_t)u * Mx + v] = std::sqrt(fu * fu + fv * fv) * (g.n_rho - 1) / g.rho_max;
    }
  }
}

void rsd_build_chunks(const RsdInputs& in, const RsdGeometry& g, RsdChunks& out) {
  std::vector<double> rho;
  rsd_radius_map(in, g, rho);
  const int npix = (int)rho.size();
  struct Tap {
    int i0, pix;
    float wa, wb;
  };
  std::vector<Tap> active;
  std::vector<int> inactive;
  active.reserve(npix);
  const double rc = g.rho_cut_bin;
  for (int p = 0; p < npix; ++p) {
    const double rt = rho[p];
    double a;  // smoothstep taper over the last 8 bins below the cutoff
    if (rt <= rc - 8.0) {
      a = 1.0;
    } else if (rt < rc) {
      const double t = (rc - rt) / 8.0;
      a = t * t * (3.0 - 2.0 * t);
    } else {
      a = 0.0;
    }
    if (!(a > 0.0)) {
      inactive.push_back(p);
      continue;
    }
    int i0 = (int)std::floor(rt);
    i0 = std::max(0, std::min(i0, g.last_base));
    const double al = rt - i0;
    active.push_back({i0, p, (float)(a * (1.0 - al)), (float)(a * al)});
  }
  std::stable_sort(active.begin(), active.end(), [](const Tap& x, const Tap& y) { return x.i0 < y.i0; });
  out.i0.clear();
  out.pix.clear();
  out.wa.clear();
  out.wb.clear();
  auto open_chunk = [&](int i0) {
    out.i0.push_back(i0);
    for (int j = 0; j < kChunk; ++j) {
      out.pix.push_back(-1);
      out.wa.push_back(0.f);
      out.wb.push_back(0.f);
    }
  };
  int fill = kChunk;
  for (const Tap& t : active) {
    if (fill == kChunk || out.i0.back() != t.i0) {
      open_chunk(t.i0);
      fill = 0;
    }
    const size_t s = (out.i0.size() - 1) * kChunk + fill;
    out.pix[s] = t.pix;
    out.wa[s] = t.wa;
    out.wb[s] = t.wb;
    ++fill;
  }
  fill = kChunk;
  for (int p : inactive) {
    if (fill == kChunk) {
      open_chunk(-1);
      fill = 0;
    }
    out.pix[(out.i0.size() - 1) * kChunk + fill] = p;
    ++fill;
  }
}

}  // namespace nlos
