// Plan creation: validation, host FP64 precompute of the operator data
// (Chebyshev matrices, FFT twiddles, per-mode tau factorisations and
// influence matrices) and device allocation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "solve_core.h"
#include "sp_internal.h"

namespace sp {

sp_status set_error(sp_plan* p, sp_status s, const std::string& msg) {
  if (p) p->last_error = msg;
  return s;
}

sp_status hip_check(sp_plan* p, hipError_t e, const char* what) {
  if (e == hipSuccess) return SP_OK;
  return set_error(p, SP_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

static bool factor_fft(int P, FFTPlan1D& pl) {
  pl.P = P;
  pl.nrad = 0;
  int r = P;
  while (r % 4 == 0 && pl.nrad < 12) {
    pl.rad[pl.nrad++] = 4;
    r /= 4;
  }
  if (r % 2 == 0 && pl.nrad < 12) {
    pl.rad[pl.nrad++] = 2;
    r /= 2;
  }
  while (r % 3 == 0 && pl.nrad < 12) {
    pl.rad[pl.nrad++] = 3;
    r /= 3;
  }
  return r == 1;
}

// exp(-2 pi i q / P), q = 0..P-1, from the host libm in long double.
static std::vector<double> twiddles(int P) {
  std::vector<double> t(2 * P);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int q = 0; q < P; ++q) {
    long double a = 2.0L * pi * (long double)q / (long double)P;
    t[2 * q] = (double)cosl(a);
    t[2 * q + 1] = (double)(-sinl(a));
  }
  return t;
}

// Host FP64 Chebyshev matrices on the Gauss-Lobatto grid y_j = cos(pi j / N).
static void cheb_matrices(int N, std::vector<double>& T, std::vector<double>& TD,
                          std::vector<double>& Tinv, std::vector<double>& G) {
  const int n1 = N + 1;
  const long double pi = 3.141592653589793238462643383279502884L;
  std::vector<long double> Tl(n1 * n1);
  T.assign(n1 * n1, 0.0);
  Tinv.assign(n1 * n1, 0.0);
  for (int j = 0; j < n1; ++j)
    for (int n = 0; n < n1; ++n) {
      const int a = (j * n) % (2 * N);
      Tl[j * n1 + n] = cosl(pi * (long double)a / (long double)N);
      T[j * n1 + n] = (double)Tl[j * n1 + n];
    }
  // D[n][m] = (2/c_n) m for m > n, m + n odd
  std::vector<long double> D(n1 * n1, 0.0L);
  for (int n = 0; n < n1; ++n)
    for (int m = n + 1; m < n1; ++m)
      if ((m + n) % 2 == 1) D[n * n1 + m] = (n == 0 ? 1.0L : 2.0L) * m;
  TD.assign(n1 * n1, 0.0);
  for (int j = 0; j < n1; ++j)
    for (int m = 0; m < n1; ++m) {
      long double s = 0.0L;
      for (int n = 0; n < m; ++n) s += Tl[j * n1 + n] * D[n * n1 + m];
      TD[j * n1 + m] = (double)s;
    }
  for (int n = 0; n < n1; ++n)
    for (int j = 0; j < n1; ++j) {
      const long double cn = (n == 0 || n == N) ? 2.0L : 1.0L;
      const long double cj = (j == 0 || j == N) ? 2.0L : 1.0L;
      Tinv[n * n1 + j] = (double)(2.0L / ((long double)N * cn * cj) * Tl[j * n1 + n]);
    }
  G.assign(n1 * n1, 0.0);
  for (int n = 0; n < n1; ++n)
    for (int m = 0; m < n1; ++m)
      if ((n + m) % 2 == 0) {
        const double s = (double)(n + m), d = (double)(n - m);
        G[n * n1 + m] = 1.0 / (1.0 - s * s) + 1.0 / (1.0 - d * d);
      }
}

// Influence solutions of one parity class (v of parity pv) for one mode:
// returns v_delta, v_b (parity pv entries) and the 2x2 influence matrix.
static void influence_class(int N, double k, double lam, const double* helm, const double* pois,
                            const double* hw, int pv, double* vdel, double* vb, double Mout[4]) {
  const int n1 = N + 1;
  const int po = 1 - pv;
  SweepView H(helm, n1), Pq(pois, n1);
  std::vector<double> r(n1, 0.0), P(n1, 0.0), DP(n1, 0.0), v(n1, 0.0), w(n1, 0.0);
  const int m = (N % 2 == pv) ? N : N - 1;
  double ell[2][2];
  for (int b = 0; b < 2; ++b) {
    std::fill(r.begin(), r.end(), 0.0);
    std::fill(P.begin(), P.end(), 0.0);
    std::fill(DP.begin(), DP.end(), 0.0);
    std::fill(v.begin(), v.end(), 0.0);
    double beta = 0.0;
    if (b == 0) {
      beta = 1.0;  // Dirichlet value of the parity-po part of P
    } else {
      // forcing -D T_m: (D T_m)_n = (2/c_n) m for n < m, n + m odd
      for (int n = 0; n < m; ++n)
        if ((n + m) % 2 == 1) r[n] = -(n == 0 ? 1.0 : 2.0) * m;
    }
    sweep_solve<double>(Pq, hw, N, po, r.data(), beta, P.data(), w.data());
    deriv_parity<double>(N, po, P.data(), DP.data());
    sweep_solve<double>(H, hw, N, pv, DP.data(), 0.0, v.data(), w.data());
    double la = 0.0;
    for (int n = pv; n <= N; n += 2) la += (double)n * n * v[n];
    double lb = lam * v[m];
    if (m == N - 1) lb += 2.0 * N * P[N];
    ell[0][b] = la;
    ell[1][b] = lb;
    double* dst = (b == 0) ? vdel : vb;
    for (int n = pv; n <= N; n += 2) dst[n] = v[n];
  }
  // rows: (D v(1) condition, tau definition); columns: (delta, b)
  const double M00 = ell[0][0], M01 = ell[0][1], M10 = ell[1][0], M11 = 1.0 + ell[1][1];
  const double det = M00 * M11 - M01 * M10;
  Mout[0] = M11 / det;
  Mout[1] = -M01 / det;
  Mout[2] = -M10 / det;
  Mout[3] = M00 / det;
  (void)k;
}

// The record's sweep block (inv_den, Q, inv_sum) from a full factorisation
// block (inv_den, cc, q, Q, inv_sum) of sweep_factor.
static void compact_sweep(const double* full, int n1, double* out) {
  for (int n = 0; n < n1; ++n) {
    out[n] = full[n];               // inv_den
    out[n1 + n] = full[3 * n1 + n];  // Q
  }
  out[2 * n1] = full[4 * n1];
  out[2 * n1 + 1] = full[4 * n1 + 1];
}

sp_status build_mode_data(sp_plan* p) {
  const Dims& d = p->d;
  const int N = d.N;
  const int n1 = N + 1;
  ModeLayout L{n1};
  const int stride = L.stride();
  const int nmodes = d.nx * d.nzh;
  std::vector<double> hw(3 * n1);
  rhs_weights(N, hw.data());
  std::vector<double> rec((size_t)nmodes * stride, 0.0);
  std::vector<double> hfull(4 * n1 + 2), pfull(4 * n1 + 2);
  for (int i = 0; i < d.nx; ++i)
    for (int j = 0; j < d.nzh; ++j) {
      if (i == d.nx / 2 || j == d.nzh - 1) continue;
      double* r = rec.data() + (size_t)(i * d.nzh + j) * stride;
      const int mxv = (i < d.nx / 2) ? i : i - d.nx;
      const double kx = d.alpha * mxv, kz = d.gamma * j;
      const double k2 = kx * kx + kz * kz;
      const double lam = k2 + d.re * d.inv_dt;
      // full factorisations (inv_den, cc, q, Q, inv_sum) for the host's own
      // influence solutions; the record keeps inv_den, Q and inv_sum
      sweep_factor(N, lam, hfull.data());
      compact_sweep(hfull.data(), n1, r + L.helm());
      if (i == 0 && j == 0) continue;
      sweep_factor(N, k2, pfull.data());
      compact_sweep(pfull.data(), n1, r + L.pois());
      const double k = std::sqrt(k2);
      for (int pv = 0; pv < 2; ++pv)
        influence_class(N, k, lam, hfull.data(), pfull.data(), hw.data(), pv, r + L.vdel(),
                        r + L.vb(), r + L.minv() + 4 * pv);
    }
  for (double x : rec)
    if (!std::isfinite(x))
      return set_error(p, SP_ERR_INVALID, "non-finite per-mode solve data (dt or Re out of range)");
  sp_status s;
  if (!p->d_mode) {
    s = hip_check(p, hipMalloc(&p->d_mode, rec.size() * sizeof(double)), "hipMalloc(mode data)");
    if (s) return s;
  }
  if (!p->d_hw) {
    s = hip_check(p, hipMalloc(&p->d_hw, hw.size() * sizeof(double)), "hipMalloc(hw)");
    if (s) return s;
  }
  s = hip_check(p, hipMemcpy(p->d_mode, rec.data(), rec.size() * sizeof(double),
                             hipMemcpyHostToDevice),
                "upload mode data");
  if (s) return s;
  s = hip_check(p, hipMemcpy(p->d_hw, hw.data(), hw.size() * sizeof(double), hipMemcpyHostToDevice),
                "upload hw");
  if (s) return s;
  {
    // the solve kernels stage record + weights with solve_record_loads(E)
    // doubles per lane (E = elements per lane and parity chain, at most 5)
    int E = solve_lanes_per_chain(p->d.ny);
    if (E > 5) E = 5;
    if (stride + 3 * p->d.ny > 64 * solve_record_loads(E))
      return set_error(p, SP_ERR_SHAPE, "mode record does not fit the solve kernels' loads");
  }
  p->mode_stride = stride;
  return SP_OK;
}

static sp_status upload(sp_plan* p, void** dst, const void* src, size_t bytes, const char* what) {
  sp_status s = hip_check(p, hipMalloc(dst, bytes), what);
  if (s) return s;
  return hip_check(p, hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice), what);
}

template <typename F, typename D>
static std::vector<F> convert(const std::vector<D>& v) {
  std::vector<F> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = (F)v[i];
  return o;
}

static void free_plan(sp_plan* p) {
  void* ptrs[] = {p->d_T,   p->d_TD,  p->d_Tinv, p->d_G,    p->d_hw,   p->d_mode, p->d_twx,
                  p->d_twz, p->f_twx, p->f_twz,  p->f_T,    p->f_TD,   p->f_Tinv, p->d_scratch,
                  p->d_yfrag, p->f_yfrag, p->d_tinv_th, p->f_tinv_th};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (p->h_partial) (void)hipHostFree(p->h_partial);
  p->prof.release();
  for (auto& b : p->bsets) {
    if (b.s) (void)hipStreamSynchronize(b.s);
    if (b.mem) (void)hipFree(b.mem);
    if (b.e) (void)hipFree(b.e);
    if (b.fin) (void)hipFree(b.fin);
    if (b.fout) (void)hipFree(b.fout);
    if (b.s) (void)hipStreamDestroy(b.s);
    if (b.done) (void)hipEventDestroy(b.done);
  }
  p->bsets.clear();
  if (p->bstart) (void)hipEventDestroy(p->bstart);
  if (p->ws && p->ws_owned) (void)hipFree(p->ws);
  if (p->traj) (void)hipFree(p->traj);
  if (p->d_adv) (void)hipFree(p->d_adv);
  if (p->f_adv) (void)hipFree(p->f_adv);
  if (p->adv_x) (void)hipFree(p->adv_x);
  if (p->sb_u) (void)hipFree(p->sb_u);
  if (p->sb_x) (void)hipFree(p->sb_x);
  if (p->nv_prev) (void)hipFree(p->nv_prev);
  if (p->jc_e) (void)hipFree(p->jc_e);
  if (p->jc_in) (void)hipFree(p->jc_in);
  if (p->jc_out) (void)hipFree(p->jc_out);
}

}  // namespace sp

using namespace sp;

static bool is_23_smooth(int P) {
  if (P <= 0) return false;
  while (P % 2 == 0) P /= 2;
  while (P % 3 == 0) P /= 3;
  return P == 1;
}

extern "C" sp_status sp_plan_create(const sp_params* prm, void* hip_stream, sp_plan** out) {
  if (!prm || !out) return SP_ERR_INVALID;
  *out = nullptr;
  const sp_params& q = *prm;
  if (q.nx < 4 || q.nz < 4 || (q.nx % 2) || (q.nz % 2)) return SP_ERR_SHAPE;
  if (q.ny < 5 || q.ny > 129) return SP_ERR_SHAPE;
  if (!is_23_smooth(3 * q.nx / 2) || !is_23_smooth(3 * q.nz / 2)) return SP_ERR_SHAPE;
  if (!(q.lx > 0) || !(q.lz > 0) || !std::isfinite(q.lx) || !std::isfinite(q.lz))
    return SP_ERR_INVALID;
  if (!(q.re > 0) || !std::isfinite(q.re)) return SP_ERR_INVALID;
  if (!(q.dt > 0) || !std::isfinite(q.dt)) return SP_ERR_INVALID;
  if (!std::isfinite(q.wall_upper) || !std::isfinite(q.wall_lower)) return SP_ERR_INVALID;
  if (q.precision != SP_FP64 && q.precision != SP_MIXED) return SP_ERR_INVALID;

  sp_plan* p = new (std::nothrow) sp_plan();
  if (!p) return SP_ERR_NOMEM;
  p->prm = q;
  p->stream = (hipStream_t)hip_stream;
  p->precision = q.precision;
  {
    // the device the plan works on: the library's per-device set-up runs here
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
      (void)hipGetLastError();
      delete p;
      return SP_ERR_HIP;
    }
    p->device = dev;
    noalloc_setup(dev);
  }
  Dims& d = p->d;
  d.nx = q.nx;
  d.ny = q.ny;
  d.nz = q.nz;
  d.N = q.ny - 1;
  d.nzh = q.nz / 2 + 1;
  d.nzm = q.nz / 2;
  d.px = 3 * q.nx / 2;
  d.pz = 3 * q.nz / 2;
  const double pi = 3.14159265358979323846;
  d.alpha = 2.0 * pi / q.lx;
  d.gamma = 2.0 * pi / q.lz;
  d.re = q.re;
  d.dt = q.dt;
  d.inv_dt = 1.0 / q.dt;
  d.wall_upper = q.wall_upper;
  d.wall_lower = q.wall_lower;
  factor_fft(d.px, p->fx);
  factor_fft(d.pz, p->fz);

  sp_status s = SP_OK;
  std::vector<double> T, TD, Tinv, G;
  cheb_matrices(d.N, T, TD, Tinv, G);
  const size_t mb = T.size() * sizeof(double);
  auto fail = [&](sp_status st) {
    free_plan(p);
    delete p;
    return st;
  };
  if ((s = upload(p, (void**)&p->d_T, T.data(), mb, "upload T"))) return fail(s);
  if ((s = upload(p, (void**)&p->d_TD, TD.data(), mb, "upload TD"))) return fail(s);
  if ((s = upload(p, (void**)&p->d_Tinv, Tinv.data(), mb, "upload Tinv"))) return fail(s);
  if ((s = upload(p, (void**)&p->d_G, G.data(), mb, "upload G"))) return fail(s);
  {
    auto fT = convert<float>(T), fTD = convert<float>(TD), fTi = convert<float>(Tinv);
    const size_t fb = fT.size() * sizeof(float);
    if ((s = upload(p, (void**)&p->f_T, fT.data(), fb, "upload fT"))) return fail(s);
    if ((s = upload(p, (void**)&p->f_TD, fTD.data(), fb, "upload fTD"))) return fail(s);
    if ((s = upload(p, (void**)&p->f_Tinv, fTi.data(), fb, "upload fTinv"))) return fail(s);
  }
  {
    const int jh = (d.ny - 1) / 2 + 1;
    std::vector<double> th((size_t)jh * d.ny);
    for (int j = 0; j < jh; ++j)
      for (int n = 0; n < d.ny; ++n) th[(size_t)j * d.ny + n] = Tinv[(size_t)n * d.ny + j];
    if ((s = upload(p, (void**)&p->d_tinv_th, th.data(), th.size() * sizeof(double), "tinv_th")))
      return fail(s);
    auto fth = convert<float>(th);
    if ((s = upload(p, (void**)&p->f_tinv_th, fth.data(), fth.size() * sizeof(float), "ftinv_th")))
      return fail(s);
  }
  {
    // MFMA fragment tables of the six y-contraction matrices: every 16-row tile
    // including a last partial one (rows past ny and columns past ny zero)
    const int ny = d.ny, nt = (ny + 15) / 16, ks = ycontract_ks(ny);
    const size_t per = std::max<size_t>((size_t)nt * ks * 64, 64);
    std::vector<double> fr((size_t)YM_COUNT * per, 0.0);
    auto elem = [&](int m, int r, int c) -> double {
      switch (m) {
        case YM_T: return T[(size_t)r * ny + c];
        case YM_TD: return TD[(size_t)r * ny + c];
        case YM_TINV_T: return Tinv[(size_t)c * ny + r];
        case YM_TINV: return Tinv[(size_t)r * ny + c];
        case YM_T_T: return T[(size_t)c * ny + r];
        default: return TD[(size_t)c * ny + r];
      }
    };
    for (int m = 0; m < YM_COUNT; ++m)
      for (int t = 0; t < nt; ++t)
        for (int st = 0; st < ks; ++st)
          for (int l = 0; l < 64; ++l) {
            const int r = 16 * t + l % 16, c = 4 * st + l / 16;
            if (r < ny && c < ny) fr[m * per + ((size_t)t * ks + st) * 64 + l] = elem(m, r, c);
          }
    p->yfrag_stride = per;
    if ((s = upload(p, (void**)&p->d_yfrag, fr.data(), fr.size() * sizeof(double), "yfrag")))
      return fail(s);
    auto ff = convert<float>(fr);
    if ((s = upload(p, (void**)&p->f_yfrag, ff.data(), ff.size() * sizeof(float), "fyfrag")))
      return fail(s);
  }
  {
    auto tx = twiddles(d.px), tz = twiddles(d.pz);
    if ((s = upload(p, (void**)&p->d_twx, tx.data(), tx.size() * sizeof(double), "twx")))
      return fail(s);
    if ((s = upload(p, (void**)&p->d_twz, tz.data(), tz.size() * sizeof(double), "twz")))
      return fail(s);
    auto fx = convert<float>(tx), fz = convert<float>(tz);
    if ((s = upload(p, (void**)&p->f_twx, fx.data(), fx.size() * sizeof(float), "ftwx")))
      return fail(s);
    if ((s = upload(p, (void**)&p->f_twz, fz.data(), fz.size() * sizeof(float), "ftwz")))
      return fail(s);
  }
  if ((s = build_mode_data(p))) return fail(s);
  // scratch: one allocation carved into 256-byte aligned pieces
  const size_t cz = sizeof(double2);
  const size_t canon = (size_t)3 * d.nx * d.nzh * d.ny * cz;
  struct Piece {
    void** dst;
    size_t bytes;
  };
  p->npartial = 1024;
  Piece pieces[] = {
      {&p->yv, (size_t)6 * d.ny * d.nzm * d.nx * cz},
      {&p->xp, (size_t)6 * d.ny * d.px * d.nzm * cz},
      {&p->np, (size_t)3 * d.ny * d.px * d.nzm * cz},
      {&p->nv, (size_t)3 * d.ny * d.nzm * d.nx * cz},
      {(void**)&p->g, canon},
      {(void**)&p->t1, canon},
      {(void**)&p->t2, canon},
      {(void**)&p->t3, canon},
      {(void**)&p->base, (size_t)6 * d.ny * d.px * d.pz * sizeof(double)},
      {(void**)&p->base32, (size_t)6 * d.ny * d.px * d.pz * sizeof(float)},
      {(void**)&p->partial, (size_t)p->npartial * sizeof(double)},
  };
  size_t total = 0;
  for (auto& pc : pieces) total += (pc.bytes + 255) / 256 * 256;
  if ((s = hip_check(p, hipMalloc(&p->d_scratch, total), "hipMalloc(scratch)"))) return fail(s);
  p->scratch_bytes = total;
  size_t off = 0;
  for (auto& pc : pieces) {
    *pc.dst = (char*)p->d_scratch + off;
    off += (pc.bytes + 255) / 256 * 256;
  }
  if ((s = hip_check(p, hipHostMalloc((void**)&p->h_partial, p->npartial * sizeof(double)),
                     "hipHostMalloc")))
    return fail(s);
  *out = p;
  return SP_OK;
}

extern "C" sp_status sp_plan_destroy(sp_plan* p) {
  if (!p) return SP_ERR_INVALID;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  else (void)hipDeviceSynchronize();
  free_plan(p);
  delete p;
  return SP_OK;
}

extern "C" sp_status sp_plan_set_dt(sp_plan* p, double dt) {
  if (!p) return SP_ERR_INVALID;
  if (!(dt > 0) || !std::isfinite(dt)) return set_error(p, SP_ERR_INVALID, "dt must be > 0");
  sp_status s = hip_check(p, p->stream ? hipStreamSynchronize(p->stream) : hipDeviceSynchronize(),
                          "sync");
  if (s) return s;
  p->prm.dt = dt;
  p->d.dt = dt;
  p->d.inv_dt = 1.0 / dt;
  p->base_valid = false;
  p->traj_valid = false;
  sp_status bs = build_mode_data(p);
  if (bs == SP_OK && p->advect) bs = build_advection(p);
  return bs;
}

extern "C" sp_status sp_plan_set_precision(sp_plan* p, int32_t precision) {
  if (!p) return SP_ERR_INVALID;
  if (precision != SP_FP64 && precision != SP_MIXED)
    return set_error(p, SP_ERR_INVALID, "precision must be SP_FP64 or SP_MIXED");
  if (precision != p->precision) p->base_valid = false;
  p->precision = precision;
  p->prm.precision = precision;
  return SP_OK;
}

extern "C" sp_status sp_state_shape(const sp_plan* p, int64_t shape4[4], int64_t* packed_n) {
  if (!p || !shape4) return SP_ERR_INVALID;
  shape4[0] = 3;
  shape4[1] = p->d.nx;
  shape4[2] = p->d.nzh;
  shape4[3] = p->d.ny;
  if (packed_n) *packed_n = (int64_t)3 * p->d.ny * (p->d.nx - 1) * (p->d.nz - 1);
  return SP_OK;
}

extern "C" const char* sp_status_string(sp_status s) {
  switch (s) {
    case SP_OK: return "ok";
    case SP_ERR_INVALID: return "invalid argument";
    case SP_ERR_SHAPE: return "unsupported grid shape";
    case SP_ERR_HIP: return "HIP runtime error";
    case SP_ERR_NOMEM: return "out of memory";
    case SP_ERR_NOT_CONVERGED: return "not converged";
    case SP_ERR_NONFINITE: return "non-finite value";
  }
  return "unknown status";
}

extern "C" const char* sp_last_error(const sp_plan* p) {
  if (!p) return "null plan";
  return p->last_error.c_str();
}
