// Driver of the library's host-only numerics (host_math.cpp) for the sanitizer
// test: the hookstep subproblem (sp_hook_step) and the advected per-mode
// operator (sp_advected_mode_operator) on valid and invalid arguments. Exit
// status 0 when every check holds; the sanitizers abort on any memory or
// undefined-behaviour error.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "sp.h"

static int fail(const char* what) {
  std::fprintf(stderr, "check failed: %s\n", what);
  return 1;
}

int main() {
  std::mt19937_64 rng(1234);
  std::normal_distribution<double> nd;
  for (int k : {1, 2, 5, 17, 40}) {
    const int ld = k + 3;
    std::vector<double> R((size_t)ld * k, 0.0), g(k + 1), y(k);
    for (int j = 0; j < k; ++j)
      for (int i = 0; i <= j; ++i) R[(size_t)j * ld + i] = nd(rng) + (i == j ? 3.0 : 0.0);
    for (auto& v : g) v = nd(rng);
    for (double delta : {1e-3, 0.1, 1.0, 1e3}) {
      double mu = -1, res = -1;
      if (sp_hook_step(R.data(), ld, g.data(), k, delta, y.data(), &mu, &res) != SP_OK)
        return fail("sp_hook_step status");
      double ny = 0;
      for (double v : y) ny += v * v;
      ny = std::sqrt(ny);
      if (!(mu >= 0) || !std::isfinite(res) || !(ny <= delta * (1 + 1e-9)))
        return fail("sp_hook_step result");
    }
    double mu, res;
    if (sp_hook_step(nullptr, ld, g.data(), k, 1.0, y.data(), &mu, &res) != SP_ERR_INVALID ||
        sp_hook_step(R.data(), k - 1, g.data(), k, 1.0, y.data(), &mu, &res) != SP_ERR_INVALID ||
        sp_hook_step(R.data(), ld, g.data(), k, 0.0, y.data(), &mu, &res) != SP_ERR_INVALID)
      return fail("sp_hook_step invalid arguments");
    R[0] = 0.0;
    if (sp_hook_step(R.data(), ld, g.data(), k, 1.0, y.data(), &mu, &res) != SP_ERR_INVALID)
      return fail("sp_hook_step zero diagonal");
  }
  for (int N : {4, 8, 16}) {
    std::vector<double> S((size_t)18 * (N - 1) * (N + 1), NAN);
    if (sp_advected_mode_operator(N, 1.14, 2.5, 400.0, 0.01, S.data()) != SP_OK)
      return fail("sp_advected_mode_operator status");
    for (double v : S)
      if (!std::isfinite(v)) return fail("sp_advected_mode_operator finite");
    if (sp_advected_mode_operator(N, 0.0, 0.0, 400.0, 0.01, S.data()) != SP_ERR_INVALID ||
        sp_advected_mode_operator(N, 1.0, 0.0, -1.0, 0.01, S.data()) != SP_ERR_INVALID ||
        sp_advected_mode_operator(3, 1.0, 0.0, 400.0, 0.01, S.data()) != SP_ERR_INVALID ||
        sp_advected_mode_operator(N, 1.0, 0.0, 400.0, 0.01, nullptr) != SP_ERR_INVALID)
      return fail("sp_advected_mode_operator invalid arguments");
  }
  std::puts("host numerics: all checks passed");
  return 0;
}
