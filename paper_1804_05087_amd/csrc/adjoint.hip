// Vector-Jacobian products (placeholder until the adjoint kernels land).
#include <hip/hip_runtime.h>

#include "sp_internal.h"

namespace sp {
sp_status vjp_lin(sp_plan* p, int op, const double2* w, double2* out) {
  (void)op; (void)w; (void)out;
  return set_error(p, SP_ERR_INVALID, "vjp not available");
}
}  // namespace sp

using namespace sp;

extern "C" sp_status sp_vjp_lin(sp_plan* p, int32_t op, const double* w, double* out) {
  if (!p) return SP_ERR_INVALID;
  return vjp_lin(p, op, (const double2*)w, (double2*)out);
}

extern "C" sp_status sp_vjp(sp_plan* p, int32_t op, const double* u, const double* w, double* out) {
  if (!p) return SP_ERR_INVALID;
  sp_status s = sp_linearize(p, u);
  if (s) return s;
  return sp_vjp_lin(p, op, w, out);
}
