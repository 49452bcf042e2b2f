// CPU check of the fixed-length line transforms of the momentum-space kernels
// (LineFft, the compile-time twiddle table): every length the kernels are instantiated
// for, both signs, both precisions, against a direct DFT in long double.  Built by hipcc
// for the host only; prints the worst relative errors and "line_fft ok".
#include <cmath>
#include <complex>
#include <cstdio>

#include "ov_kernels.hpp"

using namespace ov;
using cld = std::complex<long double>;

template <class R, int N, int SGN>
double worst_rel() {
  c2<R> a[N];
  cld in[N];
  unsigned s = 2654435761u * (unsigned)(N + 7) + (SGN > 0 ? 1u : 0u);
  for (int j = 0; j < N; ++j) {
    s = s * 1664525u + 1013904223u;
    const double re = (double)(s >> 8) / 16777216.0 - 0.5;
    s = s * 1664525u + 1013904223u;
    const double im = (double)(s >> 8) / 16777216.0 - 0.5;
    a[j] = c2<R>{(R)re, (R)im};
    in[j] = cld((long double)(R)re, (long double)(R)im);
  }
  LineFft<R, N, SGN>::run(a);
  const long double pi = 3.141592653589793238462643383279503L;
  long double err = 0, nrm = 0;
  for (int k = 0; k < N; ++k) {
    cld acc = 0;
    for (int j = 0; j < N; ++j)
      acc += in[j] * std::polar(1.0L, (long double)SGN * 2 * pi * (long double)((j * k) % N) / N);
    err = std::max(err, std::abs(acc - cld(a[k].x, a[k].y)));
    nrm = std::max(nrm, std::abs(acc));
  }
  return (double)(err / nrm);
}

int fails = 0;

template <int N>
void lengths() {
  const double e64 = std::max(worst_rel<double, N, -1>(), worst_rel<double, N, 1>());
  const double e32 = std::max(worst_rel<float, N, -1>(), worst_rel<float, N, 1>());
  std::printf("N=%2d fp64 %.2e fp32 %.2e\n", N, e64, e32);
  if (!(e64 < 1e-14) || !(e32 < 5e-7)) ++fails;
}

int main() {
  lengths<1>();
  lengths<2>();
  lengths<3>();
  lengths<4>();
  lengths<6>();
  lengths<8>();
  lengths<12>();
  lengths<16>();
  lengths<24>();
  lengths<32>();
  lengths<48>();
  lengths<64>();
  // the compile-time cos / sin against the library's, on every angle 2 pi j / n the
  // tables hold (and their periodic images)
  double worst = 0;
  for (int n = 1; n <= 64; ++n)
    for (int j = -n; j < 2 * n; ++j) {
      const CS v = ce_cossin(j, n);
      const long double th = 2 * 3.141592653589793238462643383279503L * (long double)j / n;
      worst = std::max(worst, (double)(std::fabs(v.c - std::cos(th)) + std::fabs(v.s - std::sin(th))));
    }
  std::printf("twiddles %.2e\n", worst);
  if (!(worst < 1e-15)) ++fails;
  if (fails) {
    std::printf("line_fft FAILED (%d)\n", fails);
    return 1;
  }
  std::printf("line_fft ok\n");
  return 0;
}
