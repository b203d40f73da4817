// Internal definitions shared by the host code and the kernels of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/sp.h"
#include "prof.h"

namespace sp {

// Per-mode record of the implicit-solve data (doubles), for one Fourier mode.
// Offsets in units of doubles; n1 = N + 1.
//   [0      , 2 n1 + 2) Helmholtz (D^2 - lam) sweep data, lam = k^2 + Re/dt
//   [2n1 + 2, 4 n1 + 4) Poisson   (D^2 - k^2) sweep data (unused for (0,0))
//   [4n1 + 4, 5 n1 + 4) influence basis v_delta (even n: class 0, odd n: class 1)
//   [5n1 + 4, 6 n1 + 4) influence basis v_b
//   [6n1 + 4, 6 n1 + 12) 2x2 inverse influence matrices of class 0 and class 1
// Each sweep block: inv_den[n1], Q[n1], inv_sum_q[2]. The other two arrays of
// the factorisation follow from the operator parameter and the right-hand-side
// weights (solve_core.h): cc_n = -lam w3_n, q_n = lam w1_n inv_den_n.
struct ModeLayout {
  int n1;
  __host__ __device__ int helm() const { return 0; }
  __host__ __device__ int pois() const { return 2 * n1 + 2; }
  __host__ __device__ int vdel() const { return 4 * n1 + 4; }
  __host__ __device__ int vb() const { return 5 * n1 + 4; }
  __host__ __device__ int minv() const { return 6 * n1 + 4; }
  __host__ __device__ int stride() const { return ((6 * n1 + 12) + 1) / 2 * 2; }
};

// Doubles each of the 64 lanes of the per-mode solve kernels loads to stage one
// mode record and the three weight rows (stride + 3 ny = 9 ny + 12 values),
// for E elements per lane and parity chain: enough up to ny = 32 E, the
// largest (even) ny with E elements per lane.
__host__ __device__ constexpr int solve_record_loads(int E) { return (288 * E + 12 + 63) / 64; }

struct FFTPlan1D {
  int P = 0;
  int nrad = 0;
  int rad[12] = {0};
};

// The y-contractions (Chebyshev synthesis/analysis and their adjoints) run as
// 16x16x4 MFMAs: ny rows split into ny/16 full tiles (the rest on the vector
// unit) and the ny-long sums into ycontract_ks(ny) steps of 4.
enum YMatId { YM_T = 0, YM_TD, YM_TINV_T, YM_TINV, YM_T_T, YM_TD_T, YM_COUNT };
inline int ycontract_ks(int ny) {
  const int k = (ny + 3) / 4;
  return k <= 5 ? 5 : k <= 9 ? 9 : k <= 17 ? 17 : k <= 25 ? 25 : 33;
}

struct Dims {
  int nx, ny, nz, N, nzh, nzm, px, pz;
  double alpha, gamma, re, dt, inv_dt, wall_upper, wall_lower;
};

// Compact storage of a Krylov vector: the canonical entries of the packed real
// vector space, as one contiguous run of canonical entries per (component,
// m_x):
//   m_x in [0, nx/2):   m_z in [0, nzh - 1)  (the m_z = 0 plane keeps +m_x only)
//   m_x = nx/2:         none (x Nyquist)
//   m_x in (nx/2, nx):  m_z in [1, nzh - 1)
// with all ny coefficients each. For fields in the Hermitian form (m_z = 0
// entry at -m_x the conjugate of the one at +m_x, Nyquist entries zero) the
// packed product is the plain sum of a.re b.re + a.im b.im over the compact
// entries: each m_z = 0 pair appears once with weight 1 instead of twice
// with weight 1/2.
struct CMap {
  int nx, ny, nzh;
  int h;    // nx / 2
  int r1;   // run length for m_x < nx/2: (nzh - 1) ny
  int r2;   // run length for m_x > nx/2: (nzh - 2) ny
  int lc;   // entries per component
  int len;  // 3 lc
  // canonical index of compact entry k; *mirror = canonical index of its
  // conjugate partner (m_z = 0, 0 < m_x < nx/2) or -1
  __host__ __device__ int canon(int k, int* mirror) const {
    const int c = k / lc;
    int r = k - c * lc;
    if (r < h * r1) {
      const int mx = r / r1;
      const int off = r - mx * r1;  // kz * ny + n
      *mirror = (off < ny && mx > 0) ? ((c * nx + (nx - mx)) * nzh) * ny + off : -1;
      return ((c * nx + mx) * nzh) * ny + off;
    }
    r -= h * r1;
    const int q = r / r2;
    const int off = r - q * r2;
    *mirror = -1;
    return ((c * nx + h + 1 + q) * nzh + 1) * ny + off;
  }
};
inline CMap compact_map(const Dims& d) {
  CMap m;
  m.nx = d.nx;
  m.ny = d.ny;
  m.nzh = d.nzh;
  m.h = d.nx / 2;
  m.r1 = (d.nzh - 1) * d.ny;
  m.r2 = (d.nzh - 2) * d.ny;
  m.lc = m.h * m.r1 + (m.h - 1) * m.r2;
  m.len = 3 * m.lc;
  return m;
}

// Intermediates and stream of one member of a batched call (see api.cpp).
struct BatchSet {
  void* mem = nullptr;
  void* yv = nullptr;
  void* xp = nullptr;
  void* np = nullptr;
  void* nv = nullptr;
  double2* g = nullptr;
  double2* t1 = nullptr;
  double2* t2 = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t done = nullptr;
  // dense Jacobian columns: packed unit vector, its field and the action
  double* e = nullptr;
  double2* fin = nullptr;
  double2* fout = nullptr;
};

}  // namespace sp

struct sp_plan {
  sp_params prm;
  sp::Dims d;
  hipStream_t stream = nullptr;
  int device = -1;  // current device when the plan was created
  int precision = SP_FP64;
  std::string last_error;

  // constant operator data (device)
  double* d_T = nullptr;      // [ny][ny] synthesis T[j][n] = T_n(y_j)
  double* d_TD = nullptr;     // [ny][ny] T . D (values of d/dy)
  double* d_Tinv = nullptr;   // [ny][ny] analysis
  double* d_G = nullptr;      // [ny][ny] Gram matrix int T_n T_m
  double* d_hw = nullptr;     // [3][ny] Helmholtz right-hand-side weights
  double* d_mode = nullptr;   // per-mode solve records
  int mode_stride = 0;
  double2* d_twx = nullptr;   // [px] exp(-2 pi i k / px)
  double2* d_twz = nullptr;   // [pz]
  float2* f_twx = nullptr;
  float2* f_twz = nullptr;
  float* f_T = nullptr;
  float* f_TD = nullptr;
  float* f_Tinv = nullptr;
  // y-contraction matrices in MFMA fragment order (sp::YMatId), zero padded:
  // frag[m][t][s][l] = M_m(16 t + l % 16, 4 s + l / 16), t < ny / 16, s < ycontract_ks(ny)
  // Tinv transposed over the folded half: th[j][n] = Tinv[n][j], j <= N/2 (fused analysis)
  double* d_tinv_th = nullptr;
  float* f_tinv_th = nullptr;
  double* d_yfrag = nullptr;
  float* f_yfrag = nullptr;
  size_t yfrag_stride = 0;    // elements per matrix
  sp::FFTPlan1D fx, fz;

  // scratch (device)
  void* d_scratch = nullptr;
  size_t scratch_bytes = 0;
  void* yv = nullptr;         // [6][ny][nzm][nx] complex (real type of the path)
  void* xp = nullptr;         // [6][ny][px][nzm] complex
  void* np = nullptr;         // [3][ny][px][nzm] complex
  void* nv = nullptr;         // [3][ny][nzm][nx] complex
  double2* g = nullptr;       // canonical rhs
  double2* t1 = nullptr;      // canonical temporaries
  double2* t2 = nullptr;
  double2* t3 = nullptr;
  double* base = nullptr;     // [6][ny][px][pz] physical U, Omega (FP64)
  float* base32 = nullptr;    // same, FP32 copy for the mixed path
  double* partial = nullptr;  // reduction partials
  double* h_partial = nullptr;  // pinned host mirror
  int npartial = 0;
  bool base_valid = false;
  // residual operator: nsteps BEFE steps of dt (1: Stokes operator, T = dt;
  // > 1: time-integration operator, T = nsteps dt) and, for nsteps > 1, the
  // trajectory U_0 .. U_{nsteps-1} of the linearisation point (device)
  int nsteps = 1;
  // integrator of the residual operator: 0 = BEFE steps of dt, 1 = SBDF2 with
  // implicit step tau = dt (time step 3 dt / 2); scratch of the SBDF2 steps
  int scheme = 0;
  double2* sb_u = nullptr;
  double2* sb_x = nullptr;
  double2* nv_prev = nullptr;
  double2* traj = nullptr;
  bool traj_valid = false;
  int base_step = 0;  // trajectory index of the cached base state
  // laminar advection in the implicit operator: per-mode dense solution
  // operators [mode][3(N-1)][3 ny] (device) and an input copy for aliasing
  bool symmetric = false;  // Newton drivers confined to the shift-reflect subspace
  bool advect = false;
  bool adv_host = false;  // build the advected operators on the host (reference) or the device
  double2* d_adv = nullptr;
  float2* f_adv = nullptr;  // FP32 copy of d_adv for the mixed-precision path
  double2* adv_x = nullptr;
  // batched calls: one buffer set and stream per concurrent member
  std::vector<sp::BatchSet> bsets;
  hipEvent_t bstart = nullptr;
  // dense Jacobian columns: a packed unit vector and its field in and out
  double* jc_e = nullptr;
  double2* jc_in = nullptr;
  double2* jc_out = nullptr;

  sp::Profiler prof;

  // Krylov workspace
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;
};

namespace sp {

// scratch-free Phi (noalloc.hip): per-device set-up of the file-scope scratch
// array (called by sp_plan_create with the plan's device current) and the
// bytes of intermediates one evaluation on grid d needs there
void noalloc_setup(int device);
size_t noalloc_bytes_needed(const Dims& d);

// host helpers (plan.cpp)
sp_status set_error(sp_plan* p, sp_status s, const std::string& msg);
sp_status hip_check(sp_plan* p, hipError_t e, const char* what);
sp_status build_mode_data(sp_plan* p);
// elements per lane of a 16-lane row covering one parity chain (kernels.hip)
int solve_lanes_per_chain(int ny);

// kernel launchers (kernels.hip); all enqueue on p->stream
hipError_t launch_synth_y(sp_plan* p, const double2* u, bool fp32);
hipError_t launch_fft_x_inv(sp_plan* p, bool fp32);
// mode 0: u x omega ; 1: linearised du x Omega + U x dw (needs base) ;
// 2: store U, Omega into base (no product) ; 3: adjoint (see kernels.hip)
hipError_t launch_z_product(sp_plan* p, int mode, bool fp32);
// true when the z-line kernels take the inverse x transforms themselves,
// reading nfields y-valued fields (5: launch_z_product, from p->yv; 3:
// launch_adj_z, from p->nv), so that no separate inverse x launch precedes them
bool zline_fuses_x_inverse(const sp_plan* p, bool fp32, int nfields);
hipError_t launch_fft_x_fwd(sp_plan* p, bool fp32);
// which = 0: forward synthesis table into p->yv; 1: Tinv^T on 3 components into out
hipError_t launch_synth_tab(sp_plan* p, const double2* u, int which, void* out, bool fp32);
hipError_t launch_fft_x_inv_gen(sp_plan* p, const void* in, void* out, int nfields, int plain,
                                bool fp32);
hipError_t launch_fft_x_fwd_gen(sp_plan* p, const void* in, void* out, int nfields, bool fp32);
// adjoint kernels (adjoint.hip)
hipError_t launch_stokes_solve_adj(sp_plan* p, const double2* w, double2* out);
hipError_t launch_adj_z(sp_plan* p, bool fp32);
// transposed synthesis of the six adjoint fields p->yv, finished as
// out = fa s (. + a x) + fb w with s = 1/2 on the (0,0) mode (x, w may be NULL)
hipError_t launch_adj_synth(sp_plan* p, const double2* x, double a, double fa, double fb,
                            const double2* w, double2* out, bool fp32);
hipError_t launch_analysis_rhs(sp_plan* p, const double2* x, double a, double2* g, bool fp32);
hipError_t launch_stokes_solve(sp_plan* p, const double2* g, double2* out, int inhomogeneous);
// y-valued product fields p->nv -> Chebyshev analysis + xa * x -> solve, one kernel
hipError_t launch_analysis_solve(sp_plan* p, const double2* x, double xa, double2* out,
                                 int inhomogeneous, bool fp32);
// the same with homogeneous walls in the residual form out = oa S + ob x, written
// in the Hermitian form (m_z = 0 plane exactly Hermitian, Nyquist entries zero)
hipError_t launch_analysis_solve_res(sp_plan* p, const double2* x, double xa, double oa, double ob,
                                     double2* out, bool fp32);
// out = a x + b y with the m_z = 0 plane made exactly Hermitian and Nyquist
// entries zero (out must not alias x or y)
hipError_t launch_axpby_herm(sp_plan* p, const double2* x, double a, const double2* y, double b,
                             double2* out);
hipError_t launch_axpby(sp_plan* p, const double2* x, double a, const double2* y, double b,
                        double2* out, size_t n);
hipError_t launch_norm_partial(sp_plan* p, const double2* a, double* partial, int* nblocks);
hipError_t launch_pack(sp_plan* p, const double2* c, double* packed);
hipError_t launch_unpack(sp_plan* p, const double* packed, double2* c);

// GMRES BLAS (blas.hip)
hipError_t launch_multidot(sp_plan* p, const double2* V, int nvec, const double2* w,
                           double* partial, double* out, int* nb_out);
// Krylov basis kernels (compact vectors, see CMap; T = double2 or float2, sums
// in FP64):
// out[2 v + r] = <V_v, w_r> for r = 0, 1 with w_r canonical fields in the
// Hermitian form (partial: 2 nvec multidot_blocks(p) doubles)
hipError_t launch_krylov_multidot2(sp_plan* p, const double2* V, int nvec, const double2* w0,
                                   const double2* w1, double* partial, double* out);
hipError_t launch_krylov_multidot2(sp_plan* p, const float2* V, int nvec, const double2* w0,
                                   const double2* w1, double* partial, double* out);
// w (canonical) = beta w + alpha sum_v h[v] V_v on the entries the compact
// layout holds and their mirrors
hipError_t launch_krylov_multiaxpy(sp_plan* p, const double2* V, int nvec, const double* h,
                                   double alpha, double beta, double2* w);
hipError_t launch_krylov_multiaxpy(sp_plan* p, const float2* V, int nvec, const double* h,
                                   double alpha, double beta, double2* w);
// V_j <- (V_j - sum_{i<j} a_i V_i) inv_gamma ; unew <- w inv_gamma - sum_{i<j} c_i V_i - c_j V_j,
// w canonical; u64 (canonical) receives the stored unew in FP64; inv_gamma is
// read from device memory
hipError_t launch_dcgs2_update(sp_plan* p, double2* V, int j, const double* a, const double* c,
                              const double* inv_gamma, const double2* w, double2* unew,
                              double2* u64);
hipError_t launch_dcgs2_update(sp_plan* p, float2* V, int j, const double* a, const double* c,
                              const double* inv_gamma, const double2* w, float2* unew,
                              double2* u64);
// The coefficients of Arnoldi iteration j on the device (blas.hip): from the
// dots of launch_krylov_multidot2, the row-major Hessenberg matrix H (row
// stride ld) and the provisional column hprev (both updated), writes a and c
// (ac[i], ac[cst + i]), 1/gamma and the host record rec (gamma, the squared
// norm, j, -, then column j-1 of H); Ha is scratch (j doubles).
hipError_t launch_arnoldi_coef(sp_plan* p, int j, int ld, int cst, const double* dots, double* H,
                              double* hprev, double* Ha, double* ac, double* inv_gamma,
                              double* rec);
// dst (compact) = src (canonical, Hermitian form); the FP32 form also writes the
// rounded values back into src
hipError_t launch_compact(sp_plan* p, double2* src, double2* dst);
hipError_t launch_compact(sp_plan* p, double2* src, float2* dst);
hipError_t launch_scale(sp_plan* p, const double2* y, double s, double2* x);
hipError_t launch_hermitian(sp_plan* p, double2* a);
hipError_t launch_symmetrize(sp_plan* p, double2* a);
// a[i] = v for i in [0, n) (fill) or for the single index i (set)
hipError_t launch_fill(sp_plan* p, double* a, size_t n, double v);
// nv <- 2 nv - prev, prev <- nv (the SBDF2 extrapolation of the nonlinear term)
hipError_t launch_sbdf2_combine(sp_plan* p, double2* nv, double2* prev, size_t n);
hipError_t launch_set_entry(sp_plan* p, double* a, size_t i, double v);
// element chunks of launch_multidot (1024 consecutive complex entries each); the
// partial buffer passed to it holds nvec * multidot_blocks(p) doubles
int multidot_blocks(const sp_plan* p);

// compositions (api.cpp)
sp_status host_norm_of(sp_plan* p, const double2* a, double* out);
sp_status befe_into(sp_plan* p, const double2* u, double2* out, bool fp32);
sp_status residual_into(sp_plan* p, const double2* u, double2* r);
sp_status linearize(sp_plan* p, const double2* u);
sp_status base_at(sp_plan* p, int k);
sp_status build_advection(sp_plan* p);
// fp32: use the FP32 copy of the operators (the mixed-precision path)
hipError_t launch_adv_apply(sp_plan* p, const double2* g, const double2* x, double2* out,
                            bool fp32);
sp_status jvp_lin(sp_plan* p, int op, const double2* du, double2* out);
sp_status vjp_lin(sp_plan* p, int op, const double2* w, double2* out);

}  // namespace sp
