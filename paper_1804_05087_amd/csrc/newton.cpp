// Host Newton-GMRES driver (paper Sec. 2, eqs. linear, biglin, Kspace).
//
// Newton: U <- U - du with J_r(U) du = r(U), r = (Phi_dt(U) - U)/dt.
// GMRES: unrestarted, x0 = 0, Arnoldi with classical Gram-Schmidt applied
// twice (CGS2) on the device, the Hessenberg column read back once per
// iteration, Givens rotations and the least-squares solve on the host.
// The residual, its norm and the orthogonalisation are FP64; the Jacobian
// actions use the plan's precision.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "sp_internal.h"

using namespace sp;

#define SP_TRY_HIP(expr, what)                 \
  do {                                         \
    sp_status _s = hip_check(p, (expr), what); \
    if (_s != SP_OK) return _s;                \
  } while (0)
#define SP_TRY(expr)              \
  do {                            \
    sp_status _s = (expr);        \
    if (_s != SP_OK) return _s;   \
  } while (0)

namespace {

size_t canon_bytes(const sp_plan* p) {
  return (size_t)3 * p->d.nx * p->d.nzh * p->d.ny * sizeof(double2);
}
size_t align256(size_t b) { return (b + 255) / 256 * 256; }

size_t ws_bytes_for(const sp_plan* p, int K) {
  size_t b = 0;
  b += align256((size_t)(K + 1) * canon_bytes(p));         // Krylov basis
  b += align256(canon_bytes(p));                           // w
  b += align256(canon_bytes(p));                           // scratch field
  b += align256((size_t)(K + 1) * kMultidotBlocks * sizeof(double));  // partials
  b += 3 * align256((size_t)(K + 2) * sizeof(double));     // h1, h2, y
  return b;
}

struct Workspace {
  double2* V;
  double2* w;
  double2* s;
  double* partial;
  double* h1;
  double* h2;
  double* y;
};

Workspace carve(sp_plan* p, int K) {
  Workspace W;
  char* c = (char*)p->ws;
  W.V = (double2*)c;
  c += align256((size_t)(K + 1) * canon_bytes(p));
  W.w = (double2*)c;
  c += align256(canon_bytes(p));
  W.s = (double2*)c;
  c += align256(canon_bytes(p));
  W.partial = (double*)c;
  c += align256((size_t)(K + 1) * kMultidotBlocks * sizeof(double));
  W.h1 = (double*)c;
  c += align256((size_t)(K + 2) * sizeof(double));
  W.h2 = (double*)c;
  c += align256((size_t)(K + 2) * sizeof(double));
  W.y = (double*)c;
  return W;
}

}  // namespace

extern "C" sp_status sp_plan_workspace_bytes(const sp_plan* p, int32_t max_krylov, size_t* bytes) {
  if (!p || !bytes || max_krylov < 1) return SP_ERR_INVALID;
  *bytes = ws_bytes_for(p, max_krylov);
  return SP_OK;
}

extern "C" sp_status sp_plan_set_workspace(sp_plan* p, void* dev_ptr, size_t bytes) {
  if (!p) return SP_ERR_INVALID;
  if (!dev_ptr || ((uintptr_t)dev_ptr % 256) != 0)
    return set_error(p, SP_ERR_INVALID, "workspace must be a non-null 256-byte aligned pointer");
  if (p->ws && p->ws_owned) (void)hipFree(p->ws);
  p->ws = dev_ptr;
  p->ws_bytes = bytes;
  p->ws_owned = false;
  return SP_OK;
}

namespace {

// <a, b> in the packed product, read back to the host (synchronises).
sp_status dot_host(sp_plan* p, const double2* a, const double2* b, double* partial, double* dev_out,
                   double* host_out) {
  SP_TRY_HIP(launch_multidot(p, a, 1, b, partial, dev_out, nullptr), "dot");
  SP_TRY_HIP(hipMemcpyAsync(host_out, dev_out, sizeof(double), hipMemcpyDeviceToHost, p->stream),
             "copy dot");
  SP_TRY_HIP(hipStreamSynchronize(p->stream), "sync");
  return SP_OK;
}

}  // namespace

extern "C" sp_status sp_newton_gmres(sp_plan* p, double* u_inout, const sp_newton_opts* o,
                                     sp_newton_report* rep) {
  if (!p) return SP_ERR_INVALID;
  if (!u_inout || !o || !rep) return set_error(p, SP_ERR_INVALID, "null argument");
  if (o->max_newton < 0 || o->max_newton > 64)
    return set_error(p, SP_ERR_INVALID, "max_newton must be in [0, 64]");
  if (o->max_krylov < 1) return set_error(p, SP_ERR_INVALID, "max_krylov must be >= 1");
  if (!(o->gmres_rtol >= 0) || !(o->newton_tol >= 0))
    return set_error(p, SP_ERR_INVALID, "tolerances must be >= 0");
  if (o->jvp_mode != 0 && o->jvp_mode != 1) return set_error(p, SP_ERR_INVALID, "bad jvp_mode");
  if (o->jvp_mode == 1 && !(o->fd_eps > 0)) return set_error(p, SP_ERR_INVALID, "fd_eps must be > 0");
  const int K = o->max_krylov;
  const size_t need = ws_bytes_for(p, K);
  if (!p->ws || p->ws_bytes < need) {
    if (p->ws && !p->ws_owned)
      return set_error(p, SP_ERR_INVALID, "supplied workspace is smaller than required");
    if (p->ws) (void)hipFree(p->ws);
    p->ws = nullptr;
    hipError_t e = hipMalloc(&p->ws, need);
    if (e != hipSuccess) {
      p->ws = nullptr;
      p->ws_bytes = 0;
      return set_error(p, SP_ERR_NOMEM, "cannot allocate the Krylov workspace");
    }
    p->ws_bytes = need;
    p->ws_owned = true;
  }
  std::memset(rep, 0, sizeof(*rep));
  Workspace W = carve(p, K);
  const size_t canon = canon_bytes(p);
  double2* U = (double2*)u_inout;
  double2* r = p->t3;

  double* hbuf = nullptr;  // pinned: h1[K+2] h2[K+2] hn[1]
  SP_TRY_HIP(hipHostMalloc((void**)&hbuf, (2 * (K + 2) + 2) * sizeof(double)), "hipHostMalloc");
  struct Free {
    double* b;
    ~Free() { (void)hipHostFree(b); }
  } guard{hbuf};
  double* hh1 = hbuf;
  double* hh2 = hbuf + (K + 2);
  double* hn = hbuf + 2 * (K + 2);

  std::vector<double> H((size_t)(K + 1) * K), cs(K), sn(K), gv(K + 1), yv(K);
  auto Hat = [&](int i, int k) -> double& { return H[(size_t)i * K + k]; };
  const auto t0 = std::chrono::steady_clock::now();
  sp_status result = SP_ERR_NOT_CONVERGED;
  for (int it = 0; it <= o->max_newton; ++it) {
    double rn = 0.0;
    SP_TRY(residual_into(p, U, r));
    rep->total_actions += 1;
    SP_TRY(host_norm_of(p, r, &rn));
    rep->res_norm[it] = rn;
    if (rn < o->newton_tol) {
      result = SP_OK;
      rep->converged = 1;
      break;
    }
    if (it == o->max_newton) break;
    double unorm = 0.0;
    if (o->jvp_mode == 0) {
      SP_TRY(linearize(p, U));
    } else {
      double u2 = 0.0;
      SP_TRY(dot_host(p, U, U, W.partial, W.h1, &u2));
      unorm = std::sqrt(u2);
    }
    double b2 = 0.0;
    SP_TRY(dot_host(p, r, r, W.partial, W.h1, &b2));
    const double beta = std::sqrt(b2);
    if (!std::isfinite(beta)) return set_error(p, SP_ERR_NONFINITE, "residual is not finite");
    SP_TRY_HIP(launch_scale(p, r, 1.0 / beta, W.V), "scale");
    SP_TRY_HIP(launch_hermitian(p, W.V), "hermitian");
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int kd = 0;
    double relres = 1.0;
    for (int k = 0; k < K; ++k) {
      double2* vk = W.V + (size_t)k * (canon / sizeof(double2));
      if (o->jvp_mode == 0) {
        SP_TRY(jvp_lin(p, SP_OP_RESIDUAL, vk, W.w));
      } else {
        const double eps = o->fd_eps * (unorm > 0 ? unorm : 1.0);
        SP_TRY_HIP(launch_axpby(p, U, 1.0, vk, eps, W.s, canon / sizeof(double2)), "axpby");
        SP_TRY(residual_into(p, W.s, W.w));
        SP_TRY_HIP(launch_axpby(p, W.w, 1.0 / eps, r, -1.0 / eps, W.w, canon / sizeof(double2)),
                   "axpby");
      }
      rep->total_actions += 1;
      SP_TRY_HIP(launch_hermitian(p, W.w), "hermitian");
      // CGS2
      SP_TRY_HIP(launch_multidot(p, W.V, k + 1, W.w, W.partial, W.h1, nullptr), "multidot");
      SP_TRY_HIP(launch_multiaxpy(p, W.V, k + 1, W.h1, -1.0, 1.0, W.w), "multiaxpy");
      SP_TRY_HIP(launch_multidot(p, W.V, k + 1, W.w, W.partial, W.h2, nullptr), "multidot");
      SP_TRY_HIP(launch_multiaxpy(p, W.V, k + 1, W.h2, -1.0, 1.0, W.w), "multiaxpy");
      SP_TRY_HIP(launch_multidot(p, W.w, 1, W.w, W.partial, W.y, nullptr), "norm");
      SP_TRY_HIP(hipMemcpyAsync(hh1, W.h1, (k + 1) * sizeof(double), hipMemcpyDeviceToHost,
                                p->stream),
                 "copy h1");
      SP_TRY_HIP(hipMemcpyAsync(hh2, W.h2, (k + 1) * sizeof(double), hipMemcpyDeviceToHost,
                                p->stream),
                 "copy h2");
      SP_TRY_HIP(hipMemcpyAsync(hn, W.y, sizeof(double), hipMemcpyDeviceToHost, p->stream),
                 "copy hn");
      SP_TRY_HIP(hipStreamSynchronize(p->stream), "sync");
      for (int i = 0; i <= k; ++i) Hat(i, k) = hh1[i] + hh2[i];
      const double hk1 = std::sqrt(hn[0] > 0 ? hn[0] : 0.0);
      if (!std::isfinite(hk1)) return set_error(p, SP_ERR_NONFINITE, "Arnoldi norm not finite");
      Hat(k + 1, k) = hk1;
      if (hk1 > 0 && k + 1 < K + 1)
        SP_TRY_HIP(launch_scale(p, W.w, 1.0 / hk1, W.V + (size_t)(k + 1) * (canon / sizeof(double2))),
                   "scale");
      for (int i = 0; i < k; ++i) {
        const double t = cs[i] * Hat(i, k) + sn[i] * Hat(i + 1, k);
        Hat(i + 1, k) = -sn[i] * Hat(i, k) + cs[i] * Hat(i + 1, k);
        Hat(i, k) = t;
      }
      const double dd = std::hypot(Hat(k, k), Hat(k + 1, k));
      cs[k] = Hat(k, k) / dd;
      sn[k] = Hat(k + 1, k) / dd;
      Hat(k, k) = dd;
      Hat(k + 1, k) = 0.0;
      gv[k + 1] = -sn[k] * gv[k];
      gv[k] = cs[k] * gv[k];
      kd = k + 1;
      relres = std::fabs(gv[k + 1]) / beta;
      if (std::fabs(gv[k + 1]) <= o->gmres_rtol * beta || hk1 == 0.0) break;
    }
    for (int i = kd - 1; i >= 0; --i) {
      double s = gv[i];
      for (int j = i + 1; j < kd; ++j) s -= Hat(i, j) * yv[j];
      yv[i] = s / Hat(i, i);
    }
    SP_TRY_HIP(hipMemcpyAsync(W.y, yv.data(), kd * sizeof(double), hipMemcpyHostToDevice,
                              p->stream),
               "upload y");
    SP_TRY_HIP(launch_multiaxpy(p, W.V, kd, W.y, -1.0, 1.0, U), "update");
    SP_TRY_HIP(hipStreamSynchronize(p->stream), "sync");
    rep->krylov[it] = kd;
    rep->gmres_relres[it] = relres;
    rep->total_krylov += kd;
    rep->newton_iters = it + 1;
  }
  rep->seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (result != SP_OK) set_error(p, SP_ERR_NOT_CONVERGED, "Newton did not reach newton_tol");
  return result;
}
