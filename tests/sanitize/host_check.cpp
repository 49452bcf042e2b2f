// Host-only functions of libov.so (parameter validation, the free spectrum, the CG bound,
// the Zolotarev generator) driven under AddressSanitizer / UndefinedBehaviorSanitizer.
// Prints "host_check ok" and exits 0 when every check holds.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "ov_host.hpp"

static int fails = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++fails;                                                          \
    }                                                                   \
  } while (0)

static ov_params base() {
  ov_params p;
  std::memset(&p, 0, sizeof p);
  p.dims[0] = p.dims[1] = p.dims[2] = p.dims[3] = 4;
  p.bc_t = -1;
  p.M0 = 1.0;
  p.m_re = 0.05;
  p.g_re = 0.3;
  p.n_poles = 20;
  p.lambda_min = 1e-3;
  p.lambda_max = 8.0;
  p.inner_tol = 1e-12;
  p.outer_tol = 1e-10;
  p.truth_tol = 1e-13;
  p.mixed_inner_tol = 1e-6;
  p.reliable_delta = 3e-4;
  p.max_inner = 400;
  p.max_outer = 2000;
  p.precision = OV_MIXED;
  p.inner_relax = 3e-4;
  p.inner_tol_max = 1e-2;
  p.precondition = 1;
  p.truth_relax = 0.01;
  p.inner_form = 1;
  p.pc_mass = 1;
  return p;
}

int main() {
  std::string err;
  ov_params p = base();
  CHECK(ov::validate(&p, err) == OV_OK);
  struct Bad {
    void (*set)(ov_params&);
  } bad[] = {
      {[](ov_params& q) { q.dims[0] = 3; }},       {[](ov_params& q) { q.dims[3] = 0; }},
      {[](ov_params& q) { q.n_poles = 0; }},       {[](ov_params& q) { q.n_poles = 33; }},
      {[](ov_params& q) { q.lambda_min = 9.0; }},  {[](ov_params& q) { q.bc_t = 0; }},
      {[](ov_params& q) { q.inner_tol = 0.0; }},   {[](ov_params& q) { q.reliable_delta = 1.0; }},
      {[](ov_params& q) { q.inner_tol_max = 1.0; }}, {[](ov_params& q) { q.max_inner = 3; }},
      {[](ov_params& q) { q.max_outer = 0; }},     {[](ov_params& q) { q.precision = (ov_precision)7; }},
      {[](ov_params& q) { q.truth_relax = 0.0; }}, {[](ov_params& q) { q.pc_mass = 2; }},
      {[](ov_params& q) { q.inner_form = 2; }},    {[](ov_params& q) { q.precondition = 2; }},
      {[](ov_params& q) { q.dims[0] = 128; }},     {[](ov_params& q) { q.dirac = 9; }},
      {[](ov_params& q) { q.dirac = OV_DIRAC_DSLASH; q.bc_t = 1; }},
  };
  for (auto& b : bad) {
    ov_params q = base();
    b.set(q);
    err.clear();
    CHECK(ov::validate(&q, err) == OV_ERR_INVALID_ARG && !err.empty());
  }
  // a lattice beyond the momentum-space limits is fine without the preconditioner
  {
    ov_params q = base();
    q.dims[0] = 128;
    q.precondition = 0;
    CHECK(ov::validate(&q, err) == OV_OK);
    CHECK(!ov::fft_ok(&q, err));
  }
  // free |H_W| at M0 = 1: every momentum inside [1, 7), the extremes reached on large lattices
  const int lat[][4] = {{2, 2, 2, 2}, {4, 4, 4, 4}, {2, 4, 6, 8}, {8, 8, 8, 16}};
  for (auto& d : lat)
    for (int bc : {-1, 1}) {
      ov_params q = base();
      for (int k = 0; k < 4; ++k) q.dims[k] = d[k];
      q.bc_t = bc;
      double smin = 0, smax = 0;
      ov::free_spectrum(&q, smin, smax);
      CHECK(smin >= 1.0 - 1e-12 && smax < 7.0 + 1e-12 && smin <= smax);
    }
  // CG bound: grows as the tolerance tightens and as the spectrum widens
  CHECK(ov::cg_bound(1.0, 7.0, 1e-12) > ov::cg_bound(1.0, 7.0, 1e-6));
  CHECK(ov::cg_bound(1.0, 7.0, 1e-8) > ov::cg_bound(1.0, 3.0, 1e-8));
  CHECK(ov::cg_bound(1.0, 1.0, 1e-8) == 2);
  // Zolotarev: every pole count on the workloads' intervals
  const double iv[][2] = {{0.01, 8.0}, {1e-3, 8.0}, {1e-4, 8.0}, {1.0, 7.0}, {0.5, 2.0}};
  for (auto& I : iv)
    for (int n = 1; n <= ov::HOST_MAXP; ++n) {
      double a[ov::HOST_MAXP], b[ov::HOST_MAXP], delta = -1;
      const int rc = ov::zolotarev_coeffs(n, I[0], I[1], a, b, &delta);
      CHECK(rc == 0);
      CHECK(delta >= 0.0 && delta < 1.0);
      for (int k = 0; k < n; ++k) CHECK(std::isfinite(a[k]) && a[k] > 0 && b[k] > 0);
    }
  double a[4], b[4], delta;
  CHECK(ov::zolotarev_coeffs(4, 2.0, 1.0, a, b, &delta) != 0);  // empty interval
  if (fails) {
    std::fprintf(stderr, "host_check: %d failures\n", fails);
    return 1;
  }
  std::printf("host_check ok\n");
  return 0;
}
