// ov_host.cpp -- host-only logic of libov.so: parameter validation, the limits of
// the momentum-space kernels, the analytic free spectrum of |H_W| and the CG iteration
// bound on H_W^2.  No HIP: built by the host compiler, and under ASan/UBSan by the tests.
#include "ov_host.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace ov {

// Iterations CG on H_W^2 needs, in the worst case, to bring every shifted
// residual |zeta_k| |r| below tol |src|: Chebyshev bound with kappa =
// (smax/smin)^2 and the sqrt(kappa) factor between error and residual norms.
int cg_bound(double smin, double smax, double tol) {
  const double kap = (smax / smin) * (smax / smin);
  const double sk = std::sqrt(kap);
  const double q = (sk - 1.0) / (sk + 1.0);
  if (q <= 0.0) return 2;
  return (int)std::ceil(std::log(2.0 * sk / tol) / std::log(1.0 / q));
}

bool fft_ok(const ov_params* p, std::string& why) {
  const int X = p->dims[0], Y = p->dims[1], Z = p->dims[2], T = p->dims[3];
  if (X > 64 || Y > 64 || Z > 64 || T > 64 || X * Y > 1024 || X * Z > 1024) {
    why = "momentum-space kernels need every extent <= 64, X*Y <= 1024 and X*Z <= 1024";
    return false;
  }
  return true;
}

ov_status validate(const ov_params* p, std::string& err) {
  for (int d = 0; d < 4; ++d)
    if (p->dims[d] < 2 || (p->dims[d] & 1)) {
      err = "every extent must be even and >= 2";
      return OV_ERR_INVALID_ARG;
    }
  const long long V = (long long)p->dims[0] * p->dims[1] * p->dims[2] * p->dims[3];
  if (V > (1LL << 28)) {
    err = "lattice too large";
    return OV_ERR_INVALID_ARG;
  }
  if (p->bc_t != 1 && p->bc_t != -1) {
    err = "bc_t must be +1 or -1";
    return OV_ERR_INVALID_ARG;
  }
  if (p->n_poles < 1 || p->n_poles > HOST_MAXP) {
    err = "n_poles must be in 1..32";
    return OV_ERR_INVALID_ARG;
  }
  if (!(p->lambda_min > 0) || !(p->lambda_max > p->lambda_min)) {
    err = "need 0 < lambda_min < lambda_max";
    return OV_ERR_INVALID_ARG;
  }
  if (!(p->inner_tol > 0) || !(p->outer_tol > 0) || !(p->truth_tol > 0) ||
      !(p->mixed_inner_tol > 0) || p->reliable_delta < 0 || p->reliable_delta >= 1) {
    err = "tolerances must be positive (0 <= reliable_delta < 1)";
    return OV_ERR_INVALID_ARG;
  }
  if (p->inner_relax < 0 || !(p->inner_tol_max > 0) || p->inner_tol_max >= 1) {
    err = "need inner_relax >= 0 and 0 < inner_tol_max < 1";
    return OV_ERR_INVALID_ARG;
  }
  if (p->max_inner < 4 || p->max_outer < 1) {
    err = "max_inner >= 4 and max_outer >= 1 required";
    return OV_ERR_INVALID_ARG;
  }
  // the field arrives through the C ABI and may hold any integer: read it as one (loading
  // an out-of-range value as the C++ enum type is undefined)
  int precision = 0;
  std::memcpy(&precision, &p->precision, sizeof precision);
  if (precision != OV_FP64 && precision != OV_MIXED) {
    err = "precision must be OV_FP64 or OV_MIXED";
    return OV_ERR_INVALID_ARG;
  }
  if (!(p->truth_relax > 0) || p->truth_relax > 1) {
    err = "need 0 < truth_relax <= 1";
    return OV_ERR_INVALID_ARG;
  }
  if (!(p->shift_pc_cutoff >= 0.0) || !std::isfinite(p->shift_pc_cutoff)) {
    err = "shift_pc_cutoff must be finite and >= 0";
    return OV_ERR_INVALID_ARG;
  }
  if (p->pc_mass != 0 && p->pc_mass != 1) {
    err = "pc_mass must be 0 or 1";
    return OV_ERR_INVALID_ARG;
  }
  if (p->inner_form != 0 && p->inner_form != 1) {
    err = "inner_form must be 0 or 1";
    return OV_ERR_INVALID_ARG;
  }
  if (p->precondition != 0 && p->precondition != 1) {
    err = "precondition must be 0 or 1";
    return OV_ERR_INVALID_ARG;
  }
  if (p->precondition && !fft_ok(p, err)) {
    err += " (set precondition = 0 for larger lattices)";
    return OV_ERR_INVALID_ARG;
  }
  if (p->dirac < OV_DIRAC_OVERLAP_MS || p->dirac > OV_DIRAC_DSLASH) {
    err = "dirac must be one of OV_DIRAC_*";
    return OV_ERR_INVALID_ARG;
  }
  if (p->dirac != OV_DIRAC_OVERLAP_MS && !fft_ok(p, err)) return OV_ERR_INVALID_ARG;
  if (p->dirac == OV_DIRAC_DSLASH && p->bc_t != -1) {
    err = "Dslash needs antiperiodic time (1 - D/2 is singular at the doublers otherwise)";
    return OV_ERR_INVALID_ARG;
  }
  return OV_OK;
}

// free |H_W| spectrum on the lattice: s(p)^2 = sum sin^2 p + (M0' )^2 with
// the Wilson mass term 4 - M0 - sum cos p (antiperiodic time: p_t = (2n+1) pi/T)
void free_spectrum(const ov_params* p, double& smin, double& smax) {
  smin = 1e300;
  smax = 0;
  std::vector<double> cx[4], sx[4];
  for (int d = 0; d < 4; ++d) {
    const int L = p->dims[d];
    for (int n = 0; n < L; ++n) {
      double ph = 2.0 * M_PI * n / L;
      if (d == 3 && p->bc_t < 0) ph += M_PI / L;
      cx[d].push_back(std::cos(ph));
      sx[d].push_back(std::sin(ph) * std::sin(ph));
    }
  }
  for (size_t a = 0; a < cx[0].size(); ++a)
    for (size_t b = 0; b < cx[1].size(); ++b)
      for (size_t c = 0; c < cx[2].size(); ++c)
        for (size_t d = 0; d < cx[3].size(); ++d) {
          const double w = 4.0 - p->M0 - (cx[0][a] + cx[1][b] + cx[2][c] + cx[3][d]);
          const double s2 = sx[0][a] + sx[1][b] + sx[2][c] + sx[3][d] + w * w;
          const double s = std::sqrt(s2);
          smin = std::min(smin, s);
          smax = std::max(smax, s);
        }
}

}  // namespace ov
