// Host-only numerics shared by the Newton driver and the advected-operator
// build (host_math.cpp); no HIP types.
#pragma once

#include <complex>

#include "../../include/sp.h"

namespace sp {

// Solution operator of the advected tau system of one mode, column-major
// 3(N+1) x 3(N-1) (see sp_advected_mode_operator). False if singular.
bool adv_mode_operator(int N, double kx, double kz, double re, double inv_dt,
                       std::complex<double>* S);

// The hookstep y minimising ||g[0..k-1] - R y|| over ||y|| <= delta, given the
// unconstrained minimiser yN (R k x k upper triangular, column-major, leading
// dimension ld). Returns the Lagrange multiplier mu (0: yN fits).
double hook_solve(const double* R, int ld, const double* g, int k, const double* yN,
                  double delta, double* y);

// ||g[0..k-1] - R y||^2 + g[k]^2, the GMRES model's squared residual at y.
double model_res2(const double* R, int ld, const double* g, int k, const double* y);

}  // namespace sp
