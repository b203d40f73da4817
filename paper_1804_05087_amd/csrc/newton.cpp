// Host Newton-GMRES driver (paper Sec. 2, eqs. linear, biglin, Kspace).
//
// Newton: U <- U - du with J_r(U) du = r(U), r = (Phi_dt(U) - U)/dt.
// GMRES: unrestarted, x0 = 0, Givens rotations and the least-squares solve on
// the host. The residual, its norm, the GMRES scalars and every sum of the
// orthogonalisation are FP64; the Jacobian actions use the plan's precision
// and the basis is stored in FP64 or (krylov_fp32) FP32, in the compact layout
// (only the entries of the packed real vector space: no Nyquist entries, the
// m_z = 0 plane at m_x >= 0 only), 8 % smaller than a canonical field at
// 48x65x48, which is what every pass of the orthogonalisation streams.
//
// Arnoldi orthogonalisation: classical Gram-Schmidt with the second
// (re-orthogonalising) pass delayed by one iteration, so every iteration reads
// the basis twice instead of four times (the delayed CGS2 of Swirydowicz,
// Langou et al., "Low synchronization Gram-Schmidt and GMRES algorithms").
// Iteration j holds u_j, the first-pass-orthogonalised candidate for q_j, and
// its image w = A u_j. One fused reduction gives a = Q^T u_j, b = Q^T w,
// u_j^T u_j and u_j^T w (Q = q_0..q_{j-1}); then
//   gamma_j = sqrt(u_j^T u_j - a^T a),  q_j = (u_j - Q a) / gamma_j,
//   column j-1 of H: h_{j-1} + a, subdiagonal gamma_j (u_j = A q_{j-1} - Q h_{j-1}),
//   A q_j = (w - A Q a) / gamma_j with A Q a = Q_{j+1} H a (Arnoldi relation),
//   h_j = Q_{j+1}^T A q_j  from b, u_j^T w and H a,
//   u_{j+1} = A q_j - Q_{j+1} h_j = w / gamma_j - Q_{j+1} (H a / gamma_j + h_j),
// and one fused pass over Q writes q_j and u_{j+1}. The GMRES residual of the
// j-dimensional space is known once column j-1 is complete, one iteration
// after the Jacobian action that produced it.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "host_math.h"
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
size_t compact_bytes(const sp_plan* p) {
  return (size_t)compact_map(p->d).len * sizeof(double2);
}
size_t align256(size_t b) { return (b + 255) / 256 * 256; }

size_t ws_bytes_for(const sp_plan* p, int K) {
  size_t b = 0;
  b += align256((size_t)(K + 1) * compact_bytes(p));       // Krylov basis (compact)
  b += align256(canon_bytes(p));                           // w
  b += align256(canon_bytes(p));                           // scratch field
  b += align256(canon_bytes(p));                           // u_j, canonical FP64
  b += align256((size_t)2 * (K + 1) * multidot_blocks(p) * sizeof(double));  // partials
  b += 3 * align256((size_t)2 * (K + 2) * sizeof(double));  // dots, a|c, y
  b += align256((size_t)(K + 1) * K * sizeof(double));      // Hessenberg matrix
  b += align256((size_t)(K + 2) * sizeof(double));          // provisional column
  b += align256((size_t)(K + 2) * sizeof(double));          // H a
  b += align256(sizeof(double));                            // 1 / gamma
  b += align256((size_t)2 * (K + 5) * sizeof(double));      // two host records
  return b;
}

struct Workspace {
  double2* V;
  double2* w;
  double2* s;
  double2* u;
  double* partial;
  double* h1;
  double* h2;
  double* y;
  double* H;      // (K+1) x K, row-major
  double* hprev;  // K+2
  double* ha;     // K+2
  double* ig;     // 1
  double* rec;    // 2 (K+5)
};

Workspace carve(sp_plan* p, int K) {
  Workspace W;
  char* c = (char*)p->ws;
  W.V = (double2*)c;
  c += align256((size_t)(K + 1) * compact_bytes(p));
  W.w = (double2*)c;
  c += align256(canon_bytes(p));
  W.s = (double2*)c;
  c += align256(canon_bytes(p));
  W.u = (double2*)c;
  c += align256(canon_bytes(p));
  W.partial = (double*)c;
  c += align256((size_t)2 * (K + 1) * multidot_blocks(p) * sizeof(double));
  W.h1 = (double*)c;
  c += align256((size_t)2 * (K + 2) * sizeof(double));
  W.h2 = (double*)c;
  c += align256((size_t)2 * (K + 2) * sizeof(double));
  W.y = (double*)c;
  c += align256((size_t)2 * (K + 2) * sizeof(double));
  W.H = (double*)c;
  c += align256((size_t)(K + 1) * K * sizeof(double));
  W.hprev = (double*)c;
  c += align256((size_t)(K + 2) * sizeof(double));
  W.ha = (double*)c;
  c += align256((size_t)(K + 2) * sizeof(double));
  W.ig = (double*)c;
  c += align256(sizeof(double));
  W.rec = (double*)c;
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

namespace {

sp_status check_newton_opts(sp_plan* p, const sp_newton_opts* o) {
  if (o->max_newton < 0 || o->max_newton > 64)
    return set_error(p, SP_ERR_INVALID, "max_newton must be in [0, 64]");
  if (o->max_krylov < 1) return set_error(p, SP_ERR_INVALID, "max_krylov must be >= 1");
  if (!(o->gmres_rtol >= 0) || !(o->newton_tol >= 0))
    return set_error(p, SP_ERR_INVALID, "tolerances must be >= 0");
  if (o->jvp_mode != 0 && o->jvp_mode != 1) return set_error(p, SP_ERR_INVALID, "bad jvp_mode");
  if (o->jvp_mode == 1 && !(o->fd_eps > 0)) return set_error(p, SP_ERR_INVALID, "fd_eps must be > 0");
  if (o->krylov_fp32 != 0 && o->krylov_fp32 != 1)
    return set_error(p, SP_ERR_INVALID, "krylov_fp32 must be 0 or 1");
  return SP_OK;
}

sp_status ensure_workspace(sp_plan* p, int K) {
  const size_t need = ws_bytes_for(p, K);
  if (p->ws && p->ws_bytes >= need) return SP_OK;
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
  return SP_OK;
}

// Unrestarted GMRES on J_r du = r from du = 0 with delayed CGS2 Arnoldi. After
// solve(): the first kd basis slots of W.V hold q_0..q_{kd-1} (compact,
// orthonormal in the packed product), R the Givens-rotated Hessenberg matrix (upper
// triangular kd x kd, column-major with leading dimension K+1), g the rotated
// right-hand side (g[kd] the least-squares residual), beta = ||r||.
//
// Each Arnoldi iteration runs on the device from end to end: the Jacobian
// action, the fused projections, the coefficients (launch_arnoldi_coef) and the
// update pass. The host only reads each iteration's Hessenberg column back
// (a small record copied to pinned memory) and applies the Givens rotations
// and the stop test one iteration behind the device, so the device never waits
// for it. When the test stops the solve at iteration j, iteration j + 1 has
// already been queued; its work writes only basis slots j + 1 and above and
// the Jacobian action's buffers, none of which the solution uses, and its
// action is counted.
struct Gmres {
  sp_plan* p;
  const sp_newton_opts* o;
  int K;
  Workspace W;
  size_t canon, nc, nk;
  double* hrec = nullptr;  // pinned: two records of K+5 doubles
  hipEvent_t ev[2] = {nullptr, nullptr};
  std::vector<double> H, R, cs, sn, g;
  int kd = 0;
  double beta = 0.0, relres = 1.0;
  // slot j of the basis holds q_j (u_j while iteration j runs), in FP64 (W.V)
  // or FP32 (Vf, the same memory); W.u holds u_j as a canonical FP64 field,
  // the input of the Jacobian action
  const bool f32;
  float2* Vf;

  Gmres(sp_plan* p_, const sp_newton_opts* o_)
      : p(p_), o(o_), K(o_->max_krylov), W(carve(p_, o_->max_krylov)),
        canon(canon_bytes(p_)), nc(canon_bytes(p_) / sizeof(double2)),
        nk((size_t)compact_map(p_->d).len),
        H((size_t)(K + 1) * K), R((size_t)(K + 1) * K), cs(K), sn(K), g(K + 1),
        f32(o_->krylov_fp32 != 0), Vf((float2*)W.V) {}
  ~Gmres() {
    // the queued work may still use the pinned records
    if (hrec || ev[0] || ev[1]) (void)hipStreamSynchronize(p->stream);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (hrec) (void)hipHostFree(hrec);
  }
  sp_status init() {
    SP_TRY_HIP(hipHostMalloc((void**)&hrec, 2 * (K + 5) * sizeof(double)), "hipHostMalloc");
    for (hipEvent_t& e : ev)
      SP_TRY_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    return SP_OK;
  }
  double& Hat(int i, int k) { return H[(size_t)k * (K + 1) + i]; }
  double& Rat(int i, int k) { return R[(size_t)k * (K + 1) + i]; }

  // Queues iteration j: u_j -> w = J u_j (none at j = K, which only completes
  // column K-1), the dots of q_0..q_{j-1} and u_j with u_j and w, the
  // coefficients, the update pass (q_j into slot j, u_{j+1} into slot j+1 and
  // W.u), and the copy of the record to pinned slot j % 2.
  sp_status enqueue(int j, const double2* U, const double2* r, double unorm, int* actions) {
    double2* uj = W.u;
    double* d_dots = W.h1;  // 2 (K + 2) doubles
    double* d_ac = W.h2;    // a[0..K+1] then c[0..K+1]
    const bool last = (j == K);
    if (!last) {
      if (o->jvp_mode == 0) {
        SP_TRY(jvp_lin(p, SP_OP_RESIDUAL, uj, W.w));
      } else {
        // finite difference along u_j / ||u_j||, scaled back by ||u_j||
        double uu = 0.0;
        SP_TRY(dot_host(p, uj, uj, W.partial, W.h1, &uu));
        const double un = std::sqrt(uu > 0 ? uu : 1.0);
        const double eps = o->fd_eps * (unorm > 0 ? unorm : 1.0) / un;
        SP_TRY_HIP(launch_axpby(p, U, 1.0, uj, eps, W.s, nc), "axpby");
        SP_TRY(residual_into(p, W.s, W.w));
        SP_TRY_HIP(launch_axpby(p, W.w, 1.0 / eps, r, -1.0 / eps, W.w, nc), "axpby");
      }
      *actions += 1;
      // the exact residual JVP already writes the Hermitian form
      if (o->jvp_mode != 0) SP_TRY_HIP(launch_hermitian(p, W.w), "hermitian");
    }
    if (f32)
      SP_TRY_HIP(launch_krylov_multidot2(p, Vf, j + 1, uj, last ? uj : W.w, W.partial, d_dots),
                 "multidot");
    else
      SP_TRY_HIP(launch_krylov_multidot2(p, W.V, j + 1, uj, last ? uj : W.w, W.partial, d_dots),
                 "multidot");
    double* rec = W.rec + (size_t)(j & 1) * (K + 5);
    SP_TRY_HIP(launch_arnoldi_coef(p, j, K, K + 2, d_dots, W.H, W.hprev, W.ha, d_ac, W.ig, rec),
               "arnoldi coefficients");
    if (!last) {
      if (f32)
        SP_TRY_HIP(launch_dcgs2_update(p, Vf, j, d_ac, d_ac + (K + 2), W.ig, W.w,
                                       Vf + (size_t)(j + 1) * nk, W.u),
                   "dcgs2 update");
      else
        SP_TRY_HIP(launch_dcgs2_update(p, W.V, j, d_ac, d_ac + (K + 2), W.ig, W.w,
                                       W.V + (size_t)(j + 1) * nk, W.u),
                   "dcgs2 update");
    }
    SP_TRY_HIP(hipMemcpyAsync(hrec + (size_t)(j & 1) * (K + 5), rec, (5 + j) * sizeof(double),
                              hipMemcpyDeviceToHost, p->stream),
               "copy record");
    SP_TRY_HIP(hipEventRecord(ev[j & 1], p->stream), "record event");
    return SP_OK;
  }

  // Waits for iteration j's record, completes column j-1 of the host's H,
  // rotates it and tests convergence of the j-dimensional space.
  sp_status take(int j, bool* stop) {
    SP_TRY_HIP(hipEventSynchronize(ev[j & 1]), "sync");
    const double* rc = hrec + (size_t)(j & 1) * (K + 5);
    const double gamma = rc[0];
    if (!std::isfinite(rc[1])) return set_error(p, SP_ERR_NONFINITE, "Arnoldi norm not finite");
    *stop = false;
    if (j == 0) {
      beta = gamma;
      if (!(beta > 0)) return set_error(p, SP_ERR_NONFINITE, "zero or non-finite residual");
      g[0] = beta;
      return SP_OK;
    }
    const int k = j - 1;
    for (int i = 0; i <= j; ++i) Hat(i, k) = rc[4 + i];
    for (int i = 0; i <= j; ++i) Rat(i, k) = Hat(i, k);
    for (int i = 0; i < k; ++i) {
      const double t = cs[i] * Rat(i, k) + sn[i] * Rat(i + 1, k);
      Rat(i + 1, k) = -sn[i] * Rat(i, k) + cs[i] * Rat(i + 1, k);
      Rat(i, k) = t;
    }
    const double dd = std::hypot(Rat(k, k), Rat(k + 1, k));
    cs[k] = Rat(k, k) / dd;
    sn[k] = Rat(k + 1, k) / dd;
    Rat(k, k) = dd;
    Rat(k + 1, k) = 0.0;
    g[k + 1] = -sn[k] * g[k];
    g[k] = cs[k] * g[k];
    kd = j;
    relres = std::fabs(g[k + 1]) / beta;
    *stop = std::fabs(g[k + 1]) <= o->gmres_rtol * beta || !(gamma > 0) || j == K;
    return SP_OK;
  }

  // U the linearisation point (its base state must be cached for the exact
  // JVP), r = r(U); unorm = ||U|| for the finite-difference mode.
  sp_status solve(const double2* U, const double2* r, double unorm, int* actions) {
    // u_0 = r (unnormalised; gamma_0 = ||r|| comes out of the first reduction)
    SP_TRY_HIP(hipMemcpyAsync(W.u, r, canon, hipMemcpyDeviceToDevice, p->stream), "copy r");
    SP_TRY_HIP(launch_hermitian(p, W.u), "hermitian");
    if (f32)
      SP_TRY_HIP(launch_compact(p, W.u, Vf), "compact r");
    else
      SP_TRY_HIP(launch_compact(p, W.u, W.V), "compact r");
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(R.begin(), R.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    beta = 0.0;
    kd = 0;
    relres = 1.0;
    // iteration j is queued before iteration j-1's record is taken
    bool stop = false;
    for (int j = 0; j <= K + 1 && !stop; ++j) {
      if (j <= K) SP_TRY(enqueue(j, U, r, unorm, actions));
      if (j > 0) SP_TRY(take(j - 1, &stop));
    }
    return SP_OK;
  }

  // the least-squares minimiser: R y = g[0..kd-1]
  void newton_step(double* y) {
    for (int i = kd - 1; i >= 0; --i) {
      double s2 = g[i];
      for (int j2 = i + 1; j2 < kd; ++j2) s2 -= Rat(i, j2) * y[j2];
      y[i] = s2 / Rat(i, i);
    }
  }

  // target <- target - Q y (y on the host)
  sp_status apply(const double* y, double2* target) {
    SP_TRY_HIP(hipMemcpyAsync(W.y, y, kd * sizeof(double), hipMemcpyHostToDevice, p->stream),
               "upload y");
    if (f32)
      SP_TRY_HIP(launch_krylov_multiaxpy(p, Vf, kd, W.y, -1.0, 1.0, target), "update");
    else
      SP_TRY_HIP(launch_krylov_multiaxpy(p, W.V, kd, W.y, -1.0, 1.0, target), "update");
    return SP_OK;
  }
};

double norm2(const double* v, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += v[i] * v[i];
  return std::sqrt(s);
}

}  // namespace

extern "C" sp_status sp_symmetrize(sp_plan* p, double* field) {
  if (!p) return SP_ERR_INVALID;
  if (!field) return set_error(p, SP_ERR_INVALID, "null field");
  SP_TRY_HIP(launch_symmetrize(p, (double2*)field), "symmetrize");
  return SP_OK;
}

extern "C" sp_status sp_plan_set_symmetry(sp_plan* p, int32_t on) {
  if (!p) return SP_ERR_INVALID;
  p->symmetric = (on != 0);
  return SP_OK;
}

extern "C" sp_status sp_newton_gmres(sp_plan* p, double* u_inout, const sp_newton_opts* o,
                                     sp_newton_report* rep) {
  if (!p) return SP_ERR_INVALID;
  if (!u_inout || !o || !rep) return set_error(p, SP_ERR_INVALID, "null argument");
  SP_TRY(check_newton_opts(p, o));
  SP_TRY(ensure_workspace(p, o->max_krylov));
  std::memset(rep, 0, sizeof(*rep));
  Gmres G(p, o);
  SP_TRY(G.init());
  double2* U = (double2*)u_inout;
  double2* r = p->t3;
  std::vector<double> yv(o->max_krylov);
  const auto t0 = std::chrono::steady_clock::now();
  sp_status result = SP_ERR_NOT_CONVERGED;
  for (int it = 0; it <= o->max_newton; ++it) {
    double rn = 0.0;
    if (p->symmetric) SP_TRY_HIP(launch_symmetrize(p, U), "symmetrize U");
    SP_TRY(residual_into(p, U, r));
    rep->total_actions += 1;
    if (p->symmetric) SP_TRY_HIP(launch_symmetrize(p, r), "symmetrize r");
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
      SP_TRY(dot_host(p, U, U, G.W.partial, G.W.h1, &u2));
      unorm = std::sqrt(u2);
    }
    int actions = 0;
    SP_TRY(G.solve(U, r, unorm, &actions));
    rep->total_actions += actions;
    G.newton_step(yv.data());
    SP_TRY(G.apply(yv.data(), U));
    SP_TRY_HIP(hipStreamSynchronize(p->stream), "sync");
    rep->krylov[it] = G.kd;
    rep->gmres_relres[it] = G.relres;
    rep->total_krylov += G.kd;
    rep->newton_iters = it + 1;
  }
  rep->seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (result != SP_OK) set_error(p, SP_ERR_NOT_CONVERGED, "Newton did not reach newton_tol");
  return result;
}

extern "C" sp_status sp_newton_hookstep(sp_plan* p, double* u_inout, const sp_newton_opts* o,
                                        const sp_hook_opts* h, sp_newton_report* rep,
                                        sp_hook_report* hrep) {
  if (!p) return SP_ERR_INVALID;
  if (!u_inout || !o || !h || !rep) return set_error(p, SP_ERR_INVALID, "null argument");
  SP_TRY(check_newton_opts(p, o));
  if (h->max_trials < 1) return set_error(p, SP_ERR_INVALID, "max_trials must be >= 1");
  if (!(h->delta_min > 0) || !(h->delta_max >= h->delta_min) || std::isnan(h->delta_init))
    return set_error(p, SP_ERR_INVALID, "need 0 < delta_min <= delta_max");
  SP_TRY(ensure_workspace(p, o->max_krylov));
  std::memset(rep, 0, sizeof(*rep));
  if (hrep) std::memset(hrep, 0, sizeof(*hrep));
  Gmres G(p, o);
  SP_TRY(G.init());
  const int K = o->max_krylov;
  double2* U = (double2*)u_inout;
  double2* r = p->t3;
  double2* Uc = G.W.s;  // candidate state
  double2* rc = G.W.w;  // its residual
  std::vector<double> yN(K), y(K);
  double delta = std::min(h->delta_init, h->delta_max);
  const auto t0 = std::chrono::steady_clock::now();
  sp_status result = SP_ERR_NOT_CONVERGED;
  const char* why = "Newton did not reach newton_tol";
  if (p->symmetric) SP_TRY_HIP(launch_symmetrize(p, U), "symmetrize U");
  SP_TRY(residual_into(p, U, r));
  rep->total_actions += 1;
  for (int it = 0; it <= o->max_newton; ++it) {
    double rn = 0.0;
    if (p->symmetric) {  // keep the state and the Krylov space in the subspace
      SP_TRY_HIP(launch_symmetrize(p, U), "symmetrize U");
      SP_TRY_HIP(launch_symmetrize(p, r), "symmetrize r");
    }
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
      SP_TRY(dot_host(p, U, U, G.W.partial, G.W.h1, &u2));
      unorm = std::sqrt(u2);
    }
    int actions = 0;
    SP_TRY(G.solve(U, r, unorm, &actions));
    rep->total_actions += actions;
    rep->krylov[it] = G.kd;
    rep->gmres_relres[it] = G.relres;
    rep->total_krylov += G.kd;
    rep->newton_iters = it + 1;
    const int k = G.kd;
    G.newton_step(yN.data());
    if (!(delta > 0)) delta = std::min(norm2(yN.data(), k), h->delta_max);
    const double b2 = G.beta * G.beta;
    bool accepted = false;
    for (int trial = 1; trial <= h->max_trials; ++trial) {
      const double mu = hook_solve(G.R.data(), K + 1, G.g.data(), k, yN.data(), delta, y.data());
      const double ny = norm2(y.data(), k);
      const double pred = b2 - model_res2(G.R.data(), K + 1, G.g.data(), k, y.data());
      SP_TRY_HIP(hipMemcpyAsync(Uc, U, G.canon, hipMemcpyDeviceToDevice, p->stream), "copy U");
      SP_TRY(G.apply(y.data(), Uc));
      SP_TRY(residual_into(p, Uc, rc));
      rep->total_actions += 1;
      SP_TRY_HIP(launch_hermitian(p, rc), "hermitian");
      double rc2 = 0.0;
      SP_TRY(dot_host(p, rc, rc, G.W.partial, G.W.h1, &rc2));
      const double rho = pred > 0 ? (b2 - rc2) / pred : -HUGE_VAL;
      if (!(rho >= 0.01)) {  // also rejects a non-finite candidate
        delta = 0.5 * std::min(delta, ny);
        if (delta < h->delta_min) {
          why = "hookstep: trust radius fell below delta_min";
          break;
        }
        continue;
      }
      accepted = true;
      if (hrep) {
        hrep->trials[it] = trial;
        hrep->delta[it] = delta;
        hrep->mu[it] = mu;
        hrep->step_norm[it] = ny;
        hrep->rho[it] = rho;
      }
      SP_TRY_HIP(hipMemcpyAsync(U, Uc, G.canon, hipMemcpyDeviceToDevice, p->stream), "accept U");
      SP_TRY_HIP(hipMemcpyAsync(r, rc, G.canon, hipMemcpyDeviceToDevice, p->stream), "accept r");
      if (rho < 0.25)
        delta = 0.5 * ny;
      else if (rho > 0.75 && mu > 0)
        delta = std::min(2.0 * delta, h->delta_max);
      break;
    }
    if (!accepted) {
      if (std::strcmp(why, "Newton did not reach newton_tol") == 0)
        why = "hookstep: max_trials candidates rejected";
      // report the residual of the unchanged state as the last entry
      rep->res_norm[it + 1] = rn;
      break;
    }
  }
  SP_TRY_HIP(hipStreamSynchronize(p->stream), "sync");
  rep->seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (result != SP_OK) set_error(p, SP_ERR_NOT_CONVERGED, why);
  return result;
}
