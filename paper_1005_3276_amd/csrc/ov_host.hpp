// ov_host.hpp -- host-only functions of libov.so (ov_host.cpp, ov_zolotarev.cpp).
#pragma once
#include <string>

#include "../../include/ov.h"

namespace ov {

constexpr int HOST_MAXP = 32;  // poles (the kernels' MAXP)

// Worst-case CG iterations on H_W^2 (spectrum [smin^2, smax^2]) for the shifted
// residuals to reach tol (Chebyshev bound).
int cg_bound(double smin, double smax, double tol);
// The momentum-space kernels' lattice limits; why receives the reason when false.
bool fft_ok(const ov_params* p, std::string& why);
// OV_OK or OV_ERR_INVALID_ARG with the reason in err.
ov_status validate(const ov_params* p, std::string& err);
// Range of the free |H_W| over the lattice momenta (antiperiodic time: p_t = (2n+1) pi/T).
void free_spectrum(const ov_params* p, double& smin, double& smax);
// Zolotarev coefficients of sign(x) ~ x sum_k a_k/(x^2 + b_k) on [lmin, lmax]; 0 on success.
int zolotarev_coeffs(int n, double lmin, double lmax, double* a, double* b, double* delta);

}  // namespace ov
