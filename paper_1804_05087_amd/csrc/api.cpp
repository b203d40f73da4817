// C ABI entry points: stream-ordered compositions of the kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "sp_internal.h"

using namespace sp;

#define SP_TRY_HIP(expr, what)                                  \
  do {                                                          \
    sp_status _s = hip_check(p, (expr), what);                  \
    if (_s != SP_OK) return _s;                                 \
  } while (0)

static size_t canon_count(const sp_plan* p) {
  return (size_t)3 * p->d.nx * p->d.nzh * p->d.ny;
}

namespace sp {

// a2-a5: N(u) (or its linearisation, mode 1) into p->nv (y-valued spectral).
static sp_status nonlinear_to_nv(sp_plan* p, const double2* u, int mode, bool fp32) {
  SP_TRY_HIP(launch_synth_y(p, u, fp32), "synth_y");
  if (!zline_fuses_x_inverse(p, fp32, 5)) SP_TRY_HIP(launch_fft_x_inv(p, fp32), "fft_x_inv");
  SP_TRY_HIP(launch_z_product(p, mode, fp32), "z_product");
  SP_TRY_HIP(launch_fft_x_fwd(p, fp32), "fft_x_fwd");
  return SP_OK;
}

sp_status host_norm_of(sp_plan* p, const double2* a, double* out) {
  int nb = 0;
  SP_TRY_HIP(launch_norm_partial(p, a, p->partial, &nb), "norm_partial");
  SP_TRY_HIP(hipMemcpyAsync(p->h_partial, p->partial, nb * sizeof(double), hipMemcpyDeviceToHost,
                            p->stream),
             "copy partials");
  SP_TRY_HIP(hipStreamSynchronize(p->stream), "sync");
  double s = 0.0;
  for (int i = 0; i < nb; ++i) s += p->h_partial[i];
  *out = std::sqrt(s);
  if (!std::isfinite(*out)) return set_error(p, SP_ERR_NONFINITE, "norm is not finite");
  return SP_OK;
}

sp_status befe_into(sp_plan* p, const double2* u, double2* out, bool fp32) {
  if (p->advect && u == out) {  // the advected step reads u after the solve writes out
    SP_TRY_HIP(hipMemcpyAsync(p->adv_x, u, canon_count(p) * sizeof(double2),
                              hipMemcpyDeviceToDevice, p->stream),
               "copy u");
    u = p->adv_x;
  }
  sp_status s = nonlinear_to_nv(p, u, 0, fp32);
  if (s) return s;
  if (p->advect) {
    SP_TRY_HIP(launch_analysis_rhs(p, u, p->d.inv_dt, p->g, fp32), "analysis_rhs");
    SP_TRY_HIP(launch_stokes_solve(p, p->g, out, 1), "stokes_solve (mean mode)");
    SP_TRY_HIP(launch_adv_apply(p, p->g, u, out, fp32), "advected solve");
    return SP_OK;
  }
  SP_TRY_HIP(launch_analysis_solve(p, u, p->d.inv_dt, out, 1, fp32), "analysis+solve");
  return SP_OK;
}

// r = (Phi_dt^n(u) - u) / (n dt) with n = p->nsteps (n = 1: the Stokes
// operator); the intermediate states ping-pong between t1 and t2.
static sp_status check_scheme(sp_plan* p) {
  if (p->scheme == 1 && (p->precision == SP_MIXED || p->advect))
    return set_error(p, SP_ERR_INVALID,
                     "the SBDF2 operator needs FP64 actions and the Stokes implicit operator");
  return SP_OK;
}

static size_t nv_count(const sp_plan* p) {
  return (size_t)3 * p->d.ny * p->d.nzm * p->d.nx;
}

// One SBDF2 step (scheme 1) with implicit step tau = the plan's dt:
//   out = (I - tau L)^{-1} [ (4 uk - ukm1) / 3 + tau (2 N_k - N_{k-1}) ],
// mode 0: the step (N the nonlinear term, the walls' velocities); mode 1: its
// linearisation about the cached base (N the linearised product, homogeneous
// walls). N_{k-1} is carried in y-values in nv_prev; first: N_{k-1} = N_k.
static sp_status sbdf2_step(sp_plan* p, const double2* uk, const double2* ukm1, double2* out,
                            int mode, bool first) {
  sp_status s = nonlinear_to_nv(p, uk, mode, false);
  if (s) return s;
  const size_t m = nv_count(p);
  double2* nv = reinterpret_cast<double2*>(p->nv);
  if (first)
    SP_TRY_HIP(hipMemcpyAsync(p->nv_prev, nv, m * sizeof(double2), hipMemcpyDeviceToDevice,
                              p->stream),
               "copy N");
  SP_TRY_HIP(launch_sbdf2_combine(p, nv, p->nv_prev, m), "combine N");
  SP_TRY_HIP(launch_axpby(p, uk, 4.0 / 3.0, ukm1, -1.0 / 3.0, p->sb_x, canon_count(p)),
             "combine u");
  SP_TRY_HIP(launch_analysis_solve(p, p->sb_x, p->d.inv_dt, out, mode == 0 ? 1 : 0, false),
             "analysis+solve");
  return SP_OK;
}

// the one of t1, t2, sb_u that is neither a nor b
static double2* third_buffer(sp_plan* p, const double2* a, const double2* b) {
  double2* c[3] = {p->t1, p->t2, p->sb_u};
  for (double2* x : c)
    if (x != a && x != b) return x;
  return nullptr;
}

// 1 / T of the residual operator: T = n dt (BEFE) or n 3 dt / 2 (SBDF2)
static double inv_horizon(const sp_plan* p) {
  return p->d.inv_dt / (p->nsteps * (p->scheme == 1 ? 1.5 : 1.0));
}

sp_status residual_into(sp_plan* p, const double2* u, double2* r) {
  const int n = p->nsteps;
  if (p->scheme == 1) {
    sp_status s = check_scheme(p);
    if (s) return s;
    const double2* prev = u;
    const double2* cur = u;
    for (int k = 0; k < n; ++k) {
      double2* nxt = third_buffer(p, prev, cur);
      s = sbdf2_step(p, cur, prev, nxt, 0, k == 0);
      if (s) return s;
      prev = cur;
      cur = nxt;
    }
    const double iT = inv_horizon(p);
    SP_TRY_HIP(launch_axpby(p, cur, iT, u, -iT, r, canon_count(p)), "axpby");
    return SP_OK;
  }
  const double2* x = u;
  for (int k = 0; k < n; ++k) {
    double2* dst = (k & 1) ? p->t2 : p->t1;
    sp_status s = befe_into(p, x, dst, false);
    if (s) return s;
    x = dst;
  }
  const double iT = p->d.inv_dt / n;
  SP_TRY_HIP(launch_axpby(p, x, iT, u, -iT, r, canon_count(p)), "axpby");
  return SP_OK;
}

// the cached physical U, Omega of one state (the base of the linearised product)
static sp_status cache_base(sp_plan* p, const double2* u) {
  const bool fp32 = (p->precision == SP_MIXED);
  SP_TRY_HIP(launch_synth_y(p, u, fp32), "synth_y");
  if (!zline_fuses_x_inverse(p, fp32, 5)) SP_TRY_HIP(launch_fft_x_inv(p, fp32), "fft_x_inv");
  SP_TRY_HIP(launch_z_product(p, 2, fp32), "z_product(base)");
  return SP_OK;
}

// Base state at u; for nsteps > 1 also the trajectory U_k = Phi_dt^k(u),
// k < nsteps, for the chain rule of the multi-step operator.
sp_status linearize(sp_plan* p, const double2* u) {
  p->base_valid = false;
  p->traj_valid = false;
  sp_status s = check_scheme(p);
  if (s) return s;
  s = cache_base(p, u);
  if (s) return s;
  p->base_valid = true;
  p->base_step = 0;
  if (p->nsteps > 1) {
    const size_t nc = canon_count(p);
    SP_TRY_HIP(hipMemcpyAsync(p->traj, u, nc * sizeof(double2), hipMemcpyDeviceToDevice,
                              p->stream),
               "copy U_0");
    for (int k = 0; k + 1 < p->nsteps; ++k) {
      double2* cur = p->traj + (size_t)k * nc;
      if (p->scheme == 1)
        s = sbdf2_step(p, cur, p->traj + (size_t)(k > 0 ? k - 1 : 0) * nc, cur + nc, 0, k == 0);
      else
        s = befe_into(p, cur, cur + nc, false);
      if (s) return s;
    }
    p->traj_valid = true;
  }
  return SP_OK;
}

// make the cached base the state U_k of the trajectory (k = 0: the
// linearisation point itself)
sp_status base_at(sp_plan* p, int k) {
  if (p->base_step == k) return SP_OK;
  if (!p->traj_valid) return set_error(p, SP_ERR_INVALID, "no trajectory: call sp_linearize");
  sp_status s = cache_base(p, p->traj + (size_t)k * canon_count(p));
  if (s) return s;
  p->base_step = k;
  return SP_OK;
}

// one linearised BEFE step about the cached base: J_Phi du
static sp_status jvp_phi_step(sp_plan* p, const double2* du, double2* out) {
  const bool fp32 = (p->precision == SP_MIXED);
  sp_status s = nonlinear_to_nv(p, du, 1, fp32);
  if (s) return s;
  if (p->advect) {
    SP_TRY_HIP(launch_analysis_rhs(p, du, p->d.inv_dt, p->g, fp32), "analysis_rhs");
    SP_TRY_HIP(launch_stokes_solve(p, p->g, out, 0), "stokes_solve (mean mode)");
    SP_TRY_HIP(launch_adv_apply(p, p->g, du, out, fp32), "advected solve");
    return SP_OK;
  }
  SP_TRY_HIP(launch_analysis_solve(p, du, p->d.inv_dt, out, 0, fp32), "analysis+solve");
  return SP_OK;
}

sp_status jvp_lin(sp_plan* p, int op, const double2* du, double2* out) {
  if (!p->base_valid) return set_error(p, SP_ERR_INVALID, "no base state: call sp_linearize");
  if (op != SP_OP_PHI && p->scheme == 1) {
    // chain rule of the SBDF2 steps along the trajectory, with du_{-1} = du_0 = du
    sp_status s = check_scheme(p);
    if (s) return s;
    const double2* prev = du;
    const double2* cur = du;
    for (int k = 0; k < p->nsteps; ++k) {
      s = base_at(p, k);
      if (s) return s;
      double2* nxt = third_buffer(p, prev, cur);
      s = sbdf2_step(p, cur, prev, nxt, 1, k == 0);
      if (s) return s;
      prev = cur;
      cur = nxt;
    }
    const double iT = inv_horizon(p);
    SP_TRY_HIP(launch_axpby_herm(p, cur, iT, du, -iT, out), "axpby");
    return SP_OK;
  }
  const int n = (op == SP_OP_PHI) ? 1 : p->nsteps;
  if (n == 1 && op != SP_OP_PHI && !p->advect) {
    // (J_Phi du - du) / dt formed by the solve itself, in the Hermitian form
    sp_status s = base_at(p, 0);
    if (s) return s;
    const bool fp32 = (p->precision == SP_MIXED);
    s = nonlinear_to_nv(p, du, 1, fp32);
    if (s) return s;
    SP_TRY_HIP(launch_analysis_solve_res(p, du, p->d.inv_dt, p->d.inv_dt, -p->d.inv_dt, out, fp32),
               "analysis+solve (residual form)");
    return SP_OK;
  }
  if (n == 1) {
    sp_status s = base_at(p, 0);
    if (s) return s;
    double2* dst = (op == SP_OP_PHI) ? out : p->t2;
    s = jvp_phi_step(p, du, dst);
    if (s) return s;
    if (op != SP_OP_PHI)
      SP_TRY_HIP(launch_axpby_herm(p, p->t2, p->d.inv_dt, du, -p->d.inv_dt, out), "axpby");
    return SP_OK;
  }
  // chain rule along the trajectory: v_{k+1} = J_Phi(U_k) v_k
  const double2* v = du;
  for (int k = 0; k < n; ++k) {
    sp_status s = base_at(p, k);
    if (s) return s;
    double2* dst = (k & 1) ? p->t2 : p->t1;
    s = jvp_phi_step(p, v, dst);
    if (s) return s;
    v = dst;
  }
  const double iT = p->d.inv_dt / n;
  SP_TRY_HIP(launch_axpby_herm(p, v, iT, du, -iT, out), "axpby");
  return SP_OK;
}

}  // namespace sp

#define CHECK_PLAN()                      \
  do {                                    \
    if (!p) return SP_ERR_INVALID;        \
  } while (0)
#define CHECK_PTR(x)                                                     \
  do {                                                                   \
    if (!(x)) return set_error(p, SP_ERR_INVALID, "null pointer: " #x); \
  } while (0)

extern "C" sp_status sp_nonlinear(sp_plan* p, const double* u, double* out) {
  CHECK_PLAN();
  CHECK_PTR(u);
  CHECK_PTR(out);
  if (u == out) return set_error(p, SP_ERR_INVALID, "sp_nonlinear: out aliases u");
  sp_status s = nonlinear_to_nv(p, (const double2*)u, 0, false);
  if (s) return s;
  SP_TRY_HIP(launch_analysis_rhs(p, nullptr, 0.0, (double2*)out, false), "analysis_rhs");
  return SP_OK;
}

extern "C" sp_status sp_stokes_solve(sp_plan* p, const double* g, double* out,
                                     int32_t inhomogeneous) {
  CHECK_PLAN();
  CHECK_PTR(g);
  CHECK_PTR(out);
  const double2* src = (const double2*)g;
  if (g == out) {
    SP_TRY_HIP(hipMemcpyAsync(p->g, g, canon_count(p) * sizeof(double2), hipMemcpyDeviceToDevice,
                              p->stream),
               "copy g");
    src = p->g;
  }
  SP_TRY_HIP(launch_stokes_solve(p, src, (double2*)out, inhomogeneous ? 1 : 0), "stokes_solve");
  return SP_OK;
}

extern "C" sp_status sp_befe_step(sp_plan* p, const double* u, double* out) {
  CHECK_PLAN();
  CHECK_PTR(u);
  CHECK_PTR(out);
  return befe_into(p, (const double2*)u, (double2*)out, p->precision == SP_MIXED);
}

extern "C" sp_status sp_residual(sp_plan* p, const double* u, double* r_out, double* host_norm) {
  CHECK_PLAN();
  CHECK_PTR(u);
  CHECK_PTR(r_out);
  if (u == r_out) return set_error(p, SP_ERR_INVALID, "sp_residual: r_out aliases u");
  sp_status s = residual_into(p, (const double2*)u, (double2*)r_out);
  if (s) return s;
  if (host_norm) return host_norm_of(p, (const double2*)r_out, host_norm);
  return SP_OK;
}

extern "C" sp_status sp_norm(sp_plan* p, const double* a, double* host_norm) {
  CHECK_PLAN();
  CHECK_PTR(a);
  CHECK_PTR(host_norm);
  return host_norm_of(p, (const double2*)a, host_norm);
}

extern "C" sp_status sp_plan_set_steps(sp_plan* p, int32_t nsteps) {
  CHECK_PLAN();
  if (nsteps < 1 || nsteps > 100000)
    return set_error(p, SP_ERR_INVALID, "nsteps must be in [1, 100000]");
  sp_status s = hip_check(p, hipStreamSynchronize(p->stream), "sync");
  if (s) return s;
  if (p->traj) (void)hipFree(p->traj);
  p->traj = nullptr;
  p->traj_valid = false;
  p->base_valid = false;
  p->nsteps = 1;
  if (nsteps > 1) {
    const size_t bytes = (size_t)nsteps * canon_count(p) * sizeof(double2);
    if (hipMalloc((void**)&p->traj, bytes) != hipSuccess) {
      p->traj = nullptr;
      return set_error(p, SP_ERR_NOMEM, "cannot allocate the trajectory");
    }
  }
  p->nsteps = nsteps;
  return SP_OK;
}

extern "C" sp_status sp_plan_set_scheme(sp_plan* p, int32_t scheme) {
  CHECK_PLAN();
  if (scheme != 0 && scheme != 1) return set_error(p, SP_ERR_INVALID, "scheme must be 0 or 1");
  sp_status s = hip_check(p, hipStreamSynchronize(p->stream), "sync");
  if (s) return s;
  if (scheme == 1 && !p->sb_u) {
    const size_t cb = canon_count(p) * sizeof(double2);
    if (hipMalloc((void**)&p->sb_u, cb) != hipSuccess ||
        hipMalloc((void**)&p->sb_x, cb) != hipSuccess ||
        hipMalloc((void**)&p->nv_prev, nv_count(p) * sizeof(double2)) != hipSuccess) {
      (void)hipGetLastError();
      if (p->sb_u) (void)hipFree(p->sb_u);
      if (p->sb_x) (void)hipFree(p->sb_x);
      if (p->nv_prev) (void)hipFree(p->nv_prev);
      p->sb_u = p->sb_x = p->nv_prev = nullptr;
      return set_error(p, SP_ERR_NOMEM, "cannot allocate the SBDF2 scratch");
    }
  }
  p->scheme = scheme;
  p->base_valid = false;
  p->traj_valid = false;
  return SP_OK;
}

extern "C" sp_status sp_plan_set_advection(sp_plan* p, int32_t on) {
  CHECK_PLAN();
  sp_status s = hip_check(p, hipStreamSynchronize(p->stream), "sync");
  if (s) return s;
  p->base_valid = false;
  p->traj_valid = false;
  if (!on) {
    p->advect = false;
    return SP_OK;
  }
  if (on != 1 && on != 2) return set_error(p, SP_ERR_INVALID, "advection must be 0, 1 or 2");
  p->adv_host = (on == 2);
  s = build_advection(p);
  if (s) return s;
  p->advect = true;
  return SP_OK;
}

extern "C" sp_status sp_linearize(sp_plan* p, const double* u) {
  CHECK_PLAN();
  CHECK_PTR(u);
  return linearize(p, (const double2*)u);
}

extern "C" sp_status sp_jvp_lin(sp_plan* p, int32_t op, const double* du, double* out) {
  CHECK_PLAN();
  CHECK_PTR(du);
  CHECK_PTR(out);
  if (op != SP_OP_PHI && op != SP_OP_RESIDUAL) return set_error(p, SP_ERR_INVALID, "bad op");
  if (du == out) return set_error(p, SP_ERR_INVALID, "sp_jvp: out aliases du");
  return jvp_lin(p, op, (const double2*)du, (double2*)out);
}

extern "C" sp_status sp_jvp(sp_plan* p, int32_t op, const double* u, const double* du,
                            double* out) {
  CHECK_PLAN();
  CHECK_PTR(u);
  if (du == out) return set_error(p, SP_ERR_INVALID, "sp_jvp: out aliases du");
  sp_status s = sp_linearize(p, u);
  if (s) return s;
  return sp_jvp_lin(p, op, du, out);
}

extern "C" sp_status sp_pack(sp_plan* p, const double* canonical, double* packed) {
  CHECK_PLAN();
  CHECK_PTR(canonical);
  CHECK_PTR(packed);
  SP_TRY_HIP(launch_pack(p, (const double2*)canonical, packed), "pack");
  return SP_OK;
}

extern "C" sp_status sp_unpack(sp_plan* p, const double* packed, double* canonical) {
  CHECK_PLAN();
  CHECK_PTR(canonical);
  CHECK_PTR(packed);
  SP_TRY_HIP(launch_unpack(p, packed, (double2*)canonical), "unpack");
  return SP_OK;
}

// ---- batched calls ----------------------------------------------------------------
// Member i of a batch runs the unchanged pipeline on buffer set i mod S and its
// stream, S = nstreams: while a member's launches are issued the plan's
// intermediate pointers and stream point at its set (kernels take pointers and
// the stream at launch), so up to S members execute concurrently. The sets'
// streams wait for the plan's stream before the batch, and the plan's stream
// waits for them after it.
static sp_status ensure_batch(sp_plan* p, int nstreams) {
  if (!p->bstart && hipEventCreateWithFlags(&p->bstart, hipEventDisableTiming) != hipSuccess) {
    p->bstart = nullptr;
    return set_error(p, SP_ERR_HIP, "cannot create the batch event");
  }
  const Dims& d = p->d;
  const size_t cz = sizeof(double2), canon = canon_count(p) * cz;
  const size_t sizes[7] = {(size_t)6 * d.ny * d.nzm * d.nx * cz, (size_t)6 * d.ny * d.px * d.nzm * cz,
                           (size_t)3 * d.ny * d.px * d.nzm * cz, (size_t)3 * d.ny * d.nzm * d.nx * cz,
                           canon, canon, canon};
  size_t total = 0;
  for (size_t b : sizes) total += (b + 255) / 256 * 256;
  while ((int)p->bsets.size() < nstreams) {
    BatchSet b;
    if (hipMalloc(&b.mem, total) != hipSuccess) {
      (void)hipGetLastError();
      return set_error(p, SP_ERR_NOMEM, "cannot allocate the intermediates of a batch member");
    }
    if (hipStreamCreateWithFlags(&b.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      if (b.s) (void)hipStreamDestroy(b.s);
      (void)hipFree(b.mem);
      return set_error(p, SP_ERR_HIP, "cannot create the stream of a batch member");
    }
    void** dst[7] = {&b.yv, &b.xp, &b.np, &b.nv, (void**)&b.g, (void**)&b.t1, (void**)&b.t2};
    size_t off = 0;
    for (int k = 0; k < 7; ++k) {
      *dst[k] = (char*)b.mem + off;
      off += (sizes[k] + 255) / 256 * 256;
    }
    p->bsets.push_back(b);
  }
  return SP_OK;
}

// Points the plan at one buffer set for the launches issued in its scope.
struct BatchView {
  sp_plan* p;
  void *yv, *xp, *np, *nv;
  double2 *g, *t1, *t2;
  hipStream_t s;
  BatchView(sp_plan* p_, const BatchSet& b)
      : p(p_), yv(p_->yv), xp(p_->xp), np(p_->np), nv(p_->nv), g(p_->g), t1(p_->t1), t2(p_->t2),
        s(p_->stream) {
    p->yv = b.yv;
    p->xp = b.xp;
    p->np = b.np;
    p->nv = b.nv;
    p->g = b.g;
    p->t1 = b.t1;
    p->t2 = b.t2;
    p->stream = b.s;
  }
  ~BatchView() {
    p->yv = yv;
    p->xp = xp;
    p->np = np;
    p->nv = nv;
    p->g = g;
    p->t1 = t1;
    p->t2 = t2;
    p->stream = s;
  }
};

template <typename F>
static sp_status run_batch(sp_plan* p, int count, int nstreams, F member) {
  if (count == 0) return SP_OK;
  const int S = nstreams < count ? nstreams : count;
  sp_status s = ensure_batch(p, S);
  if (s) return s;
  SP_TRY_HIP(hipEventRecord(p->bstart, p->stream), "record batch start");
  for (int b = 0; b < S; ++b)
    SP_TRY_HIP(hipStreamWaitEvent(p->bsets[b].s, p->bstart, 0), "batch wait");
  for (int i = 0; i < count && s == SP_OK; ++i) {
    BatchView v(p, p->bsets[i % S]);
    s = member(i);
  }
  for (int b = 0; b < S; ++b) {  // join even after an error: no member is left running
    SP_TRY_HIP(hipEventRecord(p->bsets[b].done, p->bsets[b].s), "record batch end");
    SP_TRY_HIP(hipStreamWaitEvent(p->stream, p->bsets[b].done, 0), "batch join");
  }
  return s;
}

extern "C" sp_status sp_jacobian_columns(sp_plan* p, int32_t op, int64_t first, int64_t count,
                                        double* J, int64_t ld) {
  CHECK_PLAN();
  if (count > 0) CHECK_PTR(J);
  if (op != SP_OP_PHI && op != SP_OP_RESIDUAL) return set_error(p, SP_ERR_INVALID, "bad op");
  const Dims& d = p->d;
  const int64_t n = (int64_t)3 * d.ny * (d.nx - 1) * (2 * (d.nzh - 1) - 1);
  if (first < 0 || count < 0 || first > n || count > n - first || ld < n)
    return set_error(p, SP_ERR_INVALID, "columns out of range or ld < packed length");
  if (!p->base_valid) return set_error(p, SP_ERR_INVALID, "no base state: call sp_linearize");
  if (count == 0) return SP_OK;
  if (!p->jc_e) {
    const size_t cb = canon_count(p) * sizeof(double2);
    if (hipMalloc((void**)&p->jc_e, (size_t)n * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&p->jc_in, cb) != hipSuccess ||
        hipMalloc((void**)&p->jc_out, cb) != hipSuccess) {
      (void)hipGetLastError();
      if (p->jc_e) (void)hipFree(p->jc_e);
      if (p->jc_in) (void)hipFree(p->jc_in);
      if (p->jc_out) (void)hipFree(p->jc_out);
      p->jc_e = nullptr;
      p->jc_in = p->jc_out = nullptr;
      return set_error(p, SP_ERR_NOMEM, "cannot allocate the Jacobian column buffers");
    }
    SP_TRY_HIP(launch_fill(p, p->jc_e, (size_t)n, 0.0), "zero unit vector");
  }
  // one-step operators (whose base state the members only read) spread the
  // columns over 3 streams with their own buffers; the multi-step chain
  // re-caches the base per step, so it runs them one after another
  const bool one_step = (op == SP_OP_PHI || (p->nsteps == 1 && p->scheme == 0)) && !p->advect;
  if (one_step && count >= 8) {
    if (p->base_step != 0) {
      sp_status s = base_at(p, 0);
      if (s) return s;
    }
    const int S = 3;  // with the plan's stream: the 4 hardware queues of a process
    sp_status s = ensure_batch(p, S);
    if (s) return s;
    for (int b = 0; b < S; ++b) {
      BatchSet& bs = p->bsets[b];
      if (bs.e) continue;
      const size_t cb = canon_count(p) * sizeof(double2);
      if (hipMalloc((void**)&bs.e, (size_t)n * sizeof(double)) != hipSuccess ||
          hipMalloc((void**)&bs.fin, cb) != hipSuccess ||
          hipMalloc((void**)&bs.fout, cb) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(p, SP_ERR_NOMEM, "cannot allocate the Jacobian column buffers");
      }
      SP_TRY_HIP(launch_fill(p, bs.e, (size_t)n, 0.0), "zero unit vector");
    }
    return run_batch(p, (int)count, S, [&](int c) -> sp_status {
      BatchSet& bs = p->bsets[c % S];
      const size_t i = (size_t)(first + c);
      SP_TRY_HIP(launch_set_entry(p, bs.e, i, 1.0), "unit vector");
      SP_TRY_HIP(launch_unpack(p, bs.e, bs.fin), "unpack");
      SP_TRY_HIP(launch_set_entry(p, bs.e, i, 0.0), "unit vector");
      sp_status st = jvp_lin(p, op, bs.fin, bs.fout);
      if (st) return st;
      SP_TRY_HIP(launch_pack(p, bs.fout, J + (size_t)c * (size_t)ld), "pack");
      return SP_OK;
    });
  }
  for (int64_t c = 0; c < count; ++c) {
    const size_t i = (size_t)(first + c);
    SP_TRY_HIP(launch_set_entry(p, p->jc_e, i, 1.0), "unit vector");
    SP_TRY_HIP(launch_unpack(p, p->jc_e, p->jc_in), "unpack");
    SP_TRY_HIP(launch_set_entry(p, p->jc_e, i, 0.0), "unit vector");
    sp_status s = jvp_lin(p, op, p->jc_in, p->jc_out);
    if (s) return s;
    SP_TRY_HIP(launch_pack(p, p->jc_out, J + (size_t)c * (size_t)ld), "pack");
  }
  return SP_OK;
}

static sp_status check_batch_args(sp_plan* p, int32_t count, int32_t nstreams, const double* a,
                                  const double* out) {
  if (count < 0 || nstreams < 1 || nstreams > 8)
    return set_error(p, SP_ERR_INVALID, "count must be >= 0 and nstreams in [1, 8]");
  if (count > 0 && (!a || !out)) return set_error(p, SP_ERR_INVALID, "null pointer");
  const size_t bytes = canon_count(p) * sizeof(double2) * (size_t)count;
  const char *ab = (const char*)a, *ob = (const char*)out;
  if (count > 0 && ab < ob + bytes && ob < ab + bytes)
    return set_error(p, SP_ERR_INVALID, "out overlaps the input batch");
  if (p->advect)
    return set_error(p, SP_ERR_INVALID, "batched calls need the Stokes implicit operator");
  return SP_OK;
}

extern "C" sp_status sp_befe_step_batch(sp_plan* p, int32_t count, int32_t nstreams,
                                        const double* u, double* out) {
  CHECK_PLAN();
  sp_status s = check_batch_args(p, count, nstreams, u, out);
  if (s) return s;
  const size_t nc = canon_count(p);
  const bool fp32 = (p->precision == SP_MIXED);
  return run_batch(p, count, nstreams, [&](int i) {
    return befe_into(p, (const double2*)u + i * nc, (double2*)out + i * nc, fp32);
  });
}

extern "C" sp_status sp_jvp_lin_batch(sp_plan* p, int32_t op, int32_t count, int32_t nstreams,
                                      const double* du, double* out) {
  CHECK_PLAN();
  if (op != SP_OP_PHI && op != SP_OP_RESIDUAL) return set_error(p, SP_ERR_INVALID, "bad op");
  sp_status s = check_batch_args(p, count, nstreams, du, out);
  if (s) return s;
  if (!p->base_valid) return set_error(p, SP_ERR_INVALID, "no base state: call sp_linearize");
  if (op == SP_OP_RESIDUAL && (p->nsteps > 1 || p->scheme != 0))
    return set_error(p, SP_ERR_INVALID, "batched residual actions need the one-step operator");
  if (p->base_step != 0) {
    s = base_at(p, 0);
    if (s) return s;
  }
  const size_t nc = canon_count(p);
  return run_batch(p, count, nstreams, [&](int i) {
    return jvp_lin(p, op, (const double2*)du + i * nc, (double2*)out + i * nc);
  });
}

extern "C" sp_status sp_profile_enable(sp_plan* p, int32_t on) {
  CHECK_PLAN();
  p->prof.on = (on != 0);
  return SP_OK;
}

extern "C" sp_status sp_profile_read(sp_plan* p, int32_t n_max, char* names, int64_t* counts,
                                     double* total_ms, int32_t* n_out, int32_t reset) {
  CHECK_PLAN();
  CHECK_PTR(n_out);
  SP_TRY_HIP(hipStreamSynchronize(p->stream), "sync");
  p->prof.collect();
  int n = 0;
  for (int k = 0; k < KID_COUNT; ++k) {
    if (p->prof.count[k] == 0) continue;
    if (n < n_max) {
      if (names) {
        std::strncpy(names + 32 * n, kernel_name(k), 31);
        names[32 * n + 31] = 0;
      }
      if (counts) counts[n] = p->prof.count[k];
      if (total_ms) total_ms[n] = p->prof.ms[k];
    }
    ++n;
  }
  *n_out = n < n_max ? n : n_max;
  if (reset) p->prof.reset();
  return SP_OK;
}

extern "C" sp_status sp_time_stage(sp_plan* p, int32_t stage, const double* u, double* out,
                                   int32_t reps, double* avg_us) {
  CHECK_PLAN();
  CHECK_PTR(u);
  CHECK_PTR(out);
  CHECK_PTR(avg_us);
  if (u == out) return set_error(p, SP_ERR_INVALID, "sp_time_stage: out aliases u");
  if (stage < SP_STAGE_SYNTH || stage > SP_STAGE_SOLVE)
    return set_error(p, SP_ERR_INVALID, "sp_time_stage: unknown stage");
  if (reps < 1 || reps > 100000) return set_error(p, SP_ERR_INVALID, "sp_time_stage: bad reps");
  const bool fp32 = (p->precision == SP_MIXED);
  const double2* uu = (const double2*)u;
  double2* oo = (double2*)out;
  sp_status s = befe_into(p, uu, oo, fp32);
  if (s) return s;
  if (stage == SP_STAGE_XINV && zline_fuses_x_inverse(p, fp32, 5)) {  // no launch of its own
    *avg_us = 0.0;
    return SP_OK;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  SP_TRY_HIP(hipEventCreate(&e0), "event");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return set_error(p, SP_ERR_HIP, "event");
  }
  hipError_t e = hipEventRecord(e0, p->stream);
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    switch (stage) {
      case SP_STAGE_SYNTH: e = launch_synth_y(p, uu, fp32); break;
      case SP_STAGE_XINV: e = launch_fft_x_inv(p, fp32); break;
      case SP_STAGE_ZLINE: e = launch_z_product(p, 0, fp32); break;
      case SP_STAGE_XFWD: e = launch_fft_x_fwd(p, fp32); break;
      default: e = launch_analysis_solve(p, uu, p->d.inv_dt, oo, 1, fp32); break;
    }
  }
  if (e == hipSuccess) e = hipEventRecord(e1, p->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_check(p, e, "sp_time_stage");
  *avg_us = 1000.0 * ms / reps;
  return SP_OK;
}
