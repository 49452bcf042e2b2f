// ov_zolotarev.cpp -- Zolotarev optimal rational approximation of sign(x).
//
//   sign(x) ~ x sum_{k=1..n} a_k / (x^2 + b_k),   lmin <= |x| <= lmax,
//
// the best uniform approximation of type (2n-1, 2n) (Zolotarev; in the form of
// Chiu et al., PRD 66 (2002) 114502, and van den Eshof et al., CPC 146 (2002) 203).
// With b = (lmax/lmin)^2, parameter m = 1 - 1/b and K = K(m):
//   c_l = sn^2(u_l|m) / cn^2(u_l|m),  u_l = l K / (2n),  l = 1 .. 2n-1,
//   R(Y) = d0 prod_{l<n} (Y + c_{2l}) / prod_{l<=n} (Y + c_{2l-1}),  Y = x^2/lmin^2,
//   sign(x) ~ (x/lmin) R(Y),   d0 = 2/(max f + min f),  delta = (max f - min f)/(max f + min f)
// where f is the un-normalised product on the interval.
//
// Jacobi functions by the descending Landen transformation (Abramowitz &
// Stegun 16.12, 17.5) in long double.  Only arguments u <= K/2 are evaluated:
// the remaining c_l follow from c_l c_{2n-l} = b (the reflection u -> K - u).
#include <cmath>
#include <vector>

namespace ov {

namespace {

using ld = long double;

// sn, cn, dn of parameter m = 1 - m1 (m1 given so that m1 ~ 1e-10 is exact).
struct Landen {
  std::vector<ld> mu;  // sqrt of the successive parameters
  ld K;
  explicit Landen(ld m1) {
    // k'_0 = sqrt(m1); k_{j+1} = (1 - k'_j) / (1 + k'_j);  k'_{j+1} = sqrt(1 - k_{j+1}^2)
    ld kp = sqrtl(m1);
    ld prodK = 1.0L;
    for (int it = 0; it < 40; ++it) {
      const ld k1 = (1.0L - kp) / (1.0L + kp);  // sqrt(mu)
      mu.push_back(k1);
      prodK *= (1.0L + k1);
      if (k1 < 1e-22L) break;
      // k'_{j+1} = sqrt(1 - k1^2) = 2 sqrt(kp) / (1 + kp), exact without cancellation
      kp = 2.0L * sqrtl(kp) / (1.0L + kp);
    }
    K = 1.5707963267948966192313216916397514L * prodK;
  }
  void eval(ld u, ld& sn, ld& cn, ld& dn) const {
    // descend: v_{j+1} = v_j / (1 + sqrt(mu_j))
    std::vector<ld> v(mu.size() + 1);
    v[0] = u;
    for (size_t j = 0; j < mu.size(); ++j) v[j + 1] = v[j] / (1.0L + mu[j]);
    // bottom: parameter ~ 0
    ld s = sinl(v.back()), c = cosl(v.back()), d = 1.0L;
    for (size_t jj = mu.size(); jj-- > 0;) {
      const ld q = mu[jj];
      const ld den = 1.0L + q * s * s;
      const ld s1 = (1.0L + q) * s / den;
      const ld c1 = c * d / den;
      const ld d1 = (1.0L - q * s * s) / den;
      s = s1; c = c1; d = d1;
    }
    sn = s; cn = c; dn = d;
  }
};

ld prod_f(ld x, ld lmin, int n, const std::vector<ld>& c) {
  const ld t = x / lmin, Y = t * t;
  ld num = t, den = 1.0L;
  for (int l = 1; l < n; ++l) num *= (Y + c[2 * l]);
  for (int l = 1; l <= n; ++l) den *= (Y + c[2 * l - 1]);
  return num / den;
}

// extremum of prod_f on [lo, hi] by golden-section search in log x
ld extremum(ld lo, ld hi, ld lmin, int n, const std::vector<ld>& c, bool maximise) {
  const ld r = 0.6180339887498948482045868343656381L;
  ld a = logl(lo), b = logl(hi);
  ld x1 = b - r * (b - a), x2 = a + r * (b - a);
  ld f1 = prod_f(expl(x1), lmin, n, c), f2 = prod_f(expl(x2), lmin, n, c);
  while (b - a > 1e-16L * (1.0L + fabsl(a))) {
    const bool keep_left = maximise ? (f1 >= f2) : (f1 <= f2);
    if (keep_left) {
      b = x2; x2 = x1; f2 = f1;
      x1 = b - r * (b - a);
      f1 = prod_f(expl(x1), lmin, n, c);
    } else {
      a = x1; x1 = x2; f1 = f2;
      x2 = a + r * (b - a);
      f2 = prod_f(expl(x2), lmin, n, c);
    }
  }
  return prod_f(expl(0.5L * (a + b)), lmin, n, c);
}

}  // namespace

// Returns 0 on success.
int zolotarev_coeffs(int n, double lmin_d, double lmax_d, double* a, double* b, double* delta) {
  if (n < 1 || !(lmin_d > 0.0) || !(lmax_d > lmin_d)) return 1;
  const ld lmin = lmin_d, lmax = lmax_d;
  const ld bb = (lmax / lmin) * (lmax / lmin);
  Landen el(1.0L / bb);
  std::vector<ld> c(2 * n + 1, 0.0L);
  for (int l = 1; l <= n; ++l) {
    ld sn, cn, dn;
    el.eval(el.K * (ld)l / (ld)(2 * n), sn, cn, dn);
    c[l] = (sn / cn) * (sn / cn);
  }
  for (int l = n + 1; l <= 2 * n - 1; ++l) c[l] = bb / c[2 * n - l];

  // extremes of the un-normalised approximant over [lmin, lmax]
  const int M = 6000;
  std::vector<ld> xs(M + 1), fs(M + 1);
  const ld la = logl(lmin), lb = logl(lmax);
  for (int i = 0; i <= M; ++i) {
    xs[i] = expl(la + (lb - la) * (ld)i / (ld)M);
    fs[i] = prod_f(xs[i], lmin, n, c);
  }
  ld fmax = fs[0] > fs[M] ? fs[0] : fs[M];
  ld fmin = fs[0] < fs[M] ? fs[0] : fs[M];
  for (int i = 1; i < M; ++i) {
    if (fs[i] > fs[i - 1] && fs[i] >= fs[i + 1]) {
      const ld v = extremum(xs[i - 1], xs[i + 1], lmin, n, c, true);
      if (v > fmax) fmax = v;
    } else if (fs[i] < fs[i - 1] && fs[i] <= fs[i + 1]) {
      const ld v = extremum(xs[i - 1], xs[i + 1], lmin, n, c, false);
      if (v < fmin) fmin = v;
    }
  }
  const ld d0 = 2.0L / (fmax + fmin);
  if (delta) *delta = (double)((fmax - fmin) / (fmax + fmin));

  // residues of R at Y = -c_{2k-1}
  for (int k = 1; k <= n; ++k) {
    const ld pole = c[2 * k - 1];
    ld num = 1.0L, den = 1.0L;
    for (int l = 1; l < n; ++l) num *= (c[2 * l] - pole);
    for (int l = 1; l <= n; ++l)
      if (l != k) den *= (c[2 * l - 1] - pole);
    a[k - 1] = (double)(d0 * (num / den) * lmin);
    b[k - 1] = (double)(pole * lmin * lmin);
  }
  return 0;
}

}  // namespace ov
