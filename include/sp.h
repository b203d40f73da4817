/*
 * sp.h -- C ABI of the MI355X Stokes-preconditioned BEFE library.
 *
 * The library evaluates one large Backwards-Euler / Forwards-Euler step of
 * plane Couette flow,
 *
 *     Phi_dt(u) = (I - dt L)^{-1} (u + dt N(u)),        (paper Sec. 2, eq. befe)
 *
 * with L = (1/Re) Laplacian, N(u) = u x curl(u) (the advective term; its
 * gradient part is absorbed by the pressure), the no-slip walls, the
 * incompressibility constraint and the pressure carried inside the implicit
 * solve (Sec. 2, after eq. befe; Sec. 3.2: exact direct inversion, divergence
 * free to machine accuracy by the influence-matrix technique). The root of the
 * Stokes-preconditioned operator G = B_T - I (Sec. 2, eq. Gstokes) is sought by
 * Newton's method (eqs. linear, biglin) with unrestarted GMRES (eq. Kspace).
 *
 * Discretisation (Sec. 3.2): Fourier in x and z, Chebyshev in y on the
 * Gauss-Lobatto grid y_j = cos(pi j / N), N = ny - 1; products are formed on
 * the 3/2-padded grid (3nx/2) x ny x (3nz/2). The per-mode implicit solve is
 * the Chebyshev-tau system with momentum imposed on T_0..T_{N-2}, no-slip
 * walls and continuity on every coefficient T_0..T_N.
 *
 * FIELD LAYOUT (every field argument, "canonical layout"):
 *   device pointer to interleaved complex128 (re, im) numbers, C order
 *   [3][nx][nz/2+1][ny]: velocity component, Fourier index i in x (m_x = i
 *   for i < nx/2, i - nx otherwise), m_z = 0..nz/2, Chebyshev coefficient n.
 *   Inputs must be zero at the Nyquist indices (i = nx/2, m_z = nz/2), have a
 *   Hermitian m_z = 0 plane (entry at -m_x = conjugate of the one at +m_x) and a
 *   real (0,0) mode; outputs have the same form up to rounding.
 *   The full step works on the total velocity; laminar Couette flow u = y e_x
 *   is its fixed point. Linearised and adjoint steps use homogeneous walls.
 *
 * OWNERSHIP: the caller owns every field buffer (e.g. torch tensors). The plan
 * owns its precomputed operator data and internal scratch (device memory it
 * allocates at creation) and, unless a workspace is supplied, the Krylov
 * basis of sp_newton_gmres. Output buffers must not alias inputs unless stated.
 *
 * STREAMS: a plan is bound to one HIP stream (given at creation, NULL = the
 * null stream). Every call is enqueued on it and returns without waiting,
 * except where "synchronises" is stated. A plan is not thread safe.
 *
 * ERRORS: every call returns an sp_status. Parameters are validated on the
 * host before any HIP call; HIP failures return SP_ERR_HIP; a per-plan message
 * is available from sp_last_error. Nothing throws across the ABI.
 */
#ifndef SP_H
#define SP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SP_OK = 0,
  SP_ERR_INVALID = -1,       /* bad parameter or NULL pointer                */
  SP_ERR_SHAPE = -2,         /* grid not supported by the kernels            */
  SP_ERR_HIP = -3,           /* a HIP runtime call failed                    */
  SP_ERR_NOMEM = -4,         /* device allocation failed                      */
  SP_ERR_NOT_CONVERGED = -5, /* Newton stopped before the tolerance          */
  SP_ERR_NONFINITE = -6      /* a residual norm was NaN or Inf               */
} sp_status;

/* Arithmetic of sp_befe_step and of the Jacobian actions (sp_jvp / sp_vjp and
 * the GMRES matvecs). SP_MIXED: transforms, products and y-contractions in
 * FP32 with FP32 accumulation; the implicit per-mode solves stay FP64. The
 * Newton residual (sp_residual) and the GMRES orthogonalisation are always
 * FP64. */
typedef enum { SP_FP64 = 0, SP_MIXED = 1 } sp_precision;

/* Which Jacobian: of Phi_dt, or of r = (Phi_dt(u) - u)/dt (= G^Stokes/T). */
typedef enum { SP_OP_PHI = 0, SP_OP_RESIDUAL = 1 } sp_op;

typedef struct {
  int32_t nx, ny, nz;          /* nx, nz even >= 4 with 3nx/2, 3nz/2 of the form
                                  2^a 3^b; 5 <= ny <= 129                     */
  double lx, lz;               /* periodic box lengths (> 0); y in [-1, 1]     */
  double re;                   /* Reynolds number, L = (1/Re) Laplacian (> 0)  */
  double dt;                   /* BEFE step = T of G^Stokes_T (> 0, finite)    */
  double wall_upper, wall_lower; /* wall velocities in x at y = +1 / -1       */
  int32_t precision;           /* sp_precision of the Jacobian actions         */
} sp_params;

typedef struct sp_plan sp_plan;

/* Validates *params, precomputes the per-mode solve data (Chebyshev-tau
 * factorisations and influence matrices for this Re and dt), uploads it and
 * allocates scratch. hip_stream: a hipStream_t or NULL. Synchronises. */
sp_status sp_plan_create(const sp_params* params, void* hip_stream, sp_plan** out);
sp_status sp_plan_destroy(sp_plan* plan);
/* Recomputes the per-mode data for a new dt (> 0). Synchronises. */
sp_status sp_plan_set_dt(sp_plan* plan, double dt);
/* Selects the precision of subsequent Jacobian actions. */
sp_status sp_plan_set_precision(sp_plan* plan, int32_t precision);
/* Number n of BEFE steps of the plan's dt composing the residual operator
 * (Sec. 2, eqs. Gstokes and Gint). n = 1 (the default): r = (Phi_dt(U) - U)/dt,
 * the Stokes-preconditioned operator with T = dt. n > 1: the time-integration
 * operator r = (Phi_dt^n(U) - U)/T with T = n dt, BEFE as the integrator. It
 * governs sp_residual, the SP_OP_RESIDUAL Jacobian actions (sp_jvp, sp_jvp_lin:
 * the chain rule along the trajectory U_k = Phi_dt^k(U), k < n, which
 * sp_linearize computes and keeps) and the Newton drivers; SP_OP_PHI actions and
 * sp_befe_step stay one step, and the SP_OP_RESIDUAL VJP of an n > 1 operator is
 * not provided (SP_ERR_INVALID). n in [1, 100000]; n > 1 allocates the
 * trajectory, n canonical fields (SP_ERR_NOMEM if that fails). Synchronises. */
sp_status sp_plan_set_steps(sp_plan* plan, int32_t nsteps);
/* Integrator of the residual operator of sp_plan_set_steps (Sec. 2: G^int
 * allows any scheme). scheme = 0 (the default): BEFE steps of the plan's dt.
 * scheme = 1: SBDF2 (second-order semi-implicit backward differences with the
 * nonlinear term extrapolated as 2 N_k - N_{k-1}) with time step 3 dt / 2, so
 * that each step is one solve of the plan's (I - dt L):
 *   u_{k+1} = (I - dt L)^{-1} [ (4 u_k - u_{k-1}) / 3 + dt (2 N(u_k) - N(u_{k-1})) ],
 * started with u_{-1} = u_0 = U (the first step is then a BEFE step of dt, and
 * the equilibria stay the roots). The residual becomes (u_n - U) / T with
 * T = n 3 dt / 2, its Jacobian actions the chain rule of these steps along the
 * trajectory (du_{-1} = du_0 = du). SBDF2 needs FP64 actions and the Stokes
 * implicit operator (SP_ERR_INVALID from the residual, linearisation and
 * Jacobian calls otherwise); sp_befe_step and SP_OP_PHI actions stay one BEFE
 * step. The first switch to 1 allocates two canonical fields and one y-valued
 * nonlinear term (SP_ERR_NOMEM if that fails). Invalidates the base state.
 * Synchronises. */
sp_status sp_plan_set_scheme(sp_plan* plan, int32_t scheme);
/* Laminar advection in the implicit operator (the remedy proposed in Sec. 3.6):
 * with on != 0 every BEFE step of the plan (sp_befe_step, sp_residual, the
 * Jacobian actions and the Newton drivers) becomes
 *   (I - dt (L + M)) Phi~(U) = U + dt (N(U) - M U),
 *   M u = -(U_lam . grad) u - (u . grad) U_lam,  U_lam = y e_x,
 * which has the same roots as the Stokes step. Per Fourier mode
 * M u = -(i k_x y u + v, i k_x y v, i k_x y w); the tau systems lose the parity
 * splitting, so the plan builds each mode's dense solution operator and keeps
 * 3 (N-1) x 3 (N+1) complex entries per mode on the device (0.74 GB at
 * 48x65x48), plus an FP32 copy (half that) that the mixed-precision steps and
 * Jacobian actions read, with FP64 sums. on = 1 builds them on the device (one workgroup per mode: LU
 * with partial pivoting and two refinement passes with double-double
 * residuals; up to 4 GiB of temporary device scratch); on = 2 builds them on
 * the host instead (LU, long-double refinement, up to 16 threads; the
 * reference construction, seconds at 48x65x48). sp_plan_set_dt rebuilds them
 * the same way. The VJP is not provided for this operator (SP_ERR_INVALID);
 * sp_stokes_solve stays the Stokes solve. on = 0 restores the Stokes step (the
 * operators stay allocated); other values are SP_ERR_INVALID. Synchronises. */
sp_status sp_plan_set_advection(sp_plan* plan, int32_t on);
/* The per-mode computation of sp_plan_set_advection alone, on the host (no
 * plan, no device work): the solution operator of the advected tau system of
 * one mode (k_x, k_z) != (0, 0) with N+1 Chebyshev coefficients, written to
 * S_out as 3(N-1) x 3(N+1) complex values (interleaved re, im), column-major:
 * entry (row, col) at 2 (col 3(N+1) + row); col = c (N-1) + n for the
 * right-hand-side coefficient n <= N-2 of component c, row = c (N+1) + n for
 * the velocity coefficient. The caller owns S_out (18 (N-1)(N+1) doubles).
 * SP_ERR_INVALID on bad arguments or a singular system. */
sp_status sp_advected_mode_operator(int32_t N, double kx, double kz, double re, double inv_dt,
                                    double* S_out);
/* shape4 = {3, nx, nz/2+1, ny}; packed_n = 3 ny (nx-1)(nz-1). */
sp_status sp_state_shape(const sp_plan* plan, int64_t shape4[4], int64_t* packed_n);
/* Device bytes of a Krylov workspace for sp_newton_gmres with max_krylov. */
sp_status sp_plan_workspace_bytes(const sp_plan* plan, int32_t max_krylov, size_t* bytes);
/* Supplies that workspace (caller-owned device memory, 256-byte aligned). The
 * plan keeps the pointer until it is replaced or the plan destroyed. */
sp_status sp_plan_set_workspace(sp_plan* plan, void* dev_ptr, size_t bytes);

/* N(u): the dealiased advective term u x curl(u) as Chebyshev coefficients
 * (Sec. 3.2, pseudospectral product). out must not alias u. */
sp_status sp_nonlinear(sp_plan* plan, const double* u, double* out);

/* The implicit solve: out = S(g), the velocity solving
 * (1/Re) Lap phi - phi/dt - grad p = -g, div phi = 0, with the wall velocities
 * when inhomogeneous != 0 and zero walls otherwise (Sec. 2, after eq. befe;
 * Sec. 3.2). The two highest Chebyshev coefficients of g are not used
 * (tau method). out may alias g. */
sp_status sp_stokes_solve(sp_plan* plan, const double* g, double* out, int32_t inhomogeneous);

/* Phi_dt(u) (Sec. 2, eq. befe) in the plan's precision (SP_MIXED: FP32
 * transforms, products and y-contractions; FP64 implicit solve). out may
 * alias u. */
sp_status sp_befe_step(sp_plan* plan, const double* u, double* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): Phi_dt(u)
 * exactly as sp_befe_step computes it (same kernels, same result), with the
 * intermediates of the transforms in a fixed array of the library's own device
 * memory instead of the plan's scratch. The array holds 32 MiB per device and
 * stays allocated until the process ends; its address is looked up while the
 * first plan on a device is created, and this call allocates nothing.
 * SP_ERR_SHAPE if the grid's intermediates exceed 32 MiB (48x65x48 needs
 * 27 MB), SP_ERR_INVALID for the advected step (sp_plan_set_advection) or NULL
 * pointers, SP_ERR_HIP if the array's address could not be obtained. Every call
 * on one device uses the same array: calls that overlap on one device (other
 * streams or plans) race, and the caller must order them. out may alias u. */
sp_status sp_befe_step_noalloc(sp_plan* plan, const double* u, double* out);

/* r = (Phi_dt(u) - u)/dt, FP64. If host_norm != NULL, synchronises and stores
 * the volume-normalised L2 norm sqrt((1/V) int |r|^2 dV) there (returns
 * SP_ERR_NONFINITE if it is NaN/Inf). r_out must not alias u. */
sp_status sp_residual(sp_plan* plan, const double* u, double* r_out, double* host_norm);

/* Volume-normalised L2 norm of a field. Synchronises. */
sp_status sp_norm(sp_plan* plan, const double* a, double* host_norm);

/* Caches the base state u (and its vorticity) used by the *_lin calls below
 * (the linearisation point U of Sec. 2, eq. linear). */
sp_status sp_linearize(sp_plan* plan, const double* u);

/* Jacobian-vector product about the cached base state: the exact
 * linearisation N_U(du) = du x Omega + U x curl(du) with homogeneous walls
 * (Sec. 2, after eq. factor2). SP_OP_PHI: J_Phi du; SP_OP_RESIDUAL:
 * (J_Phi du - du)/dt, written with the m_z = 0 plane exactly Hermitian (entry
 * -m_x taken as the conjugate of entry m_x) and Nyquist entries zero, the form
 * the packed vectors represent. out must not alias du. */
sp_status sp_jvp_lin(sp_plan* plan, int32_t op, const double* du, double* out);
/* sp_linearize(u) followed by sp_jvp_lin. */
sp_status sp_jvp(sp_plan* plan, int32_t op, const double* u, const double* du, double* out);

/* Vector-Jacobian product about the cached base state: the adjoint of the
 * JVP in the packed Euclidean inner product (the product of the packed real
 * vectors of sp_pack). out must not alias w. */
sp_status sp_vjp_lin(sp_plan* plan, int32_t op, const double* w, double* out);
sp_status sp_vjp(sp_plan* plan, int32_t op, const double* u, const double* w, double* out);

/* Canonical layout <-> packed real float64 vector of length 3 ny (nx-1)(nz-1):
 * for each component c and Chebyshev index n: the (0,0) mode (real part), the
 * m_z = 0 modes m_x = 1..nx/2-1 as (re, im), then for m_z = 1..nz/2-1 every
 * non-Nyquist m_x in FFT order as (re, im). sp_unpack writes the Hermitian
 * m_z = 0 plane and zero Nyquist entries. */
sp_status sp_pack(sp_plan* plan, const double* canonical, double* packed);
sp_status sp_unpack(sp_plan* plan, const double* packed, double* canonical);

/* Batched evaluations for throughput (independent states: seeds, sweeps,
 * Jacobian columns): count canonical fields stored one after another in u
 * (du) and out. sp_befe_step_batch: out_i = Phi_dt(u_i) as sp_befe_step;
 * sp_jvp_lin_batch: out_i = the Jacobian action of sp_jvp_lin on du_i about
 * the cached base state (SP_OP_RESIDUAL only for the one-step operator). Up to
 * nstreams (1..8) members run concurrently (3 fill, with the plan's own
 * stream, the 4 hardware queues a process gets by default), each with its own intermediates
 * (about 10 canonical fields) and stream, allocated on first use and kept
 * until sp_plan_destroy; the plan's stream waits for all members before the
 * call returns its work, so results are ordered like those of single calls and
 * equal to them bit for bit. SP_ERR_INVALID for count < 0, nstreams outside
 * [1, 8], overlapping in and out, the advected operator, or (JVP) no base
 * state or a multi-step residual operator. */
sp_status sp_befe_step_batch(sp_plan* plan, int32_t count, int32_t nstreams, const double* u,
                             double* out);
sp_status sp_jvp_lin_batch(sp_plan* plan, int32_t op, int32_t count, int32_t nstreams,
                           const double* du, double* out);

/* Columns first .. first+count-1 of the dense Jacobian in the packed real
 * basis, the matrix whose eigenvalues give the spectra of Sec. 3.5: column i is
 * pack(J unpack(e_i)) with J the Jacobian action of sp_jvp_lin for op about
 * the cached base state (sp_linearize first), written to J + (i - first) ld
 * (device, float64; ld >= packed_n, the caller owns J; J may be NULL when
 * count = 0, which does nothing). Each column is formed
 * on the device (unit vector, unpack, Jacobian action, pack) without host
 * synchronisation. For the one-step operators (SP_OP_PHI, or SP_OP_RESIDUAL
 * with one BEFE step, no laminar advection) and count >= 8 the columns are
 * spread over 3 concurrent members as in sp_jvp_lin_batch, each with its own
 * unit vector and fields; the multi-step chain forms them one after another.
 * The plan's stream waits for all of them. Buffers are allocated on first use
 * and kept until sp_plan_destroy (SP_ERR_NOMEM if that fails). SP_ERR_INVALID for a bad
 * op, a range outside [0, packed_n), ld < packed_n or no base state. */
sp_status sp_jacobian_columns(sp_plan* plan, int32_t op, int64_t first, int64_t count, double* J,
                              int64_t ld);

typedef struct {
  int32_t max_newton;   /* Newton steps (<= 64)                                 */
  int32_t max_krylov;   /* GMRES iterations per Newton step (unrestarted)       */
  double gmres_rtol;    /* stop GMRES when its residual <= rtol * ||r||          */
  double newton_tol;    /* stop Newton when the L2 norm of r < newton_tol        */
  int32_t jvp_mode;     /* 0: exact JVP; 1: finite difference [G(U+eps u)-G(U)]/eps */
  double fd_eps;        /* relative step of jvp_mode 1 (eps = fd_eps ||U||/||u||)  */
  int32_t krylov_fp32;  /* 0: Krylov basis stored in FP64; 1: stored in FP32,
                           halving the orthogonalisation's memory traffic (the
                           dot products, GMRES scalars, residual and Newton
                           update stay FP64; the basis vectors and the GMRES
                           residual estimate are then accurate to about 1e-7
                           relative, so gmres_rtol should be >= 1e-6)        */
} sp_newton_opts;

/* total_actions counts the residual evaluations and the Jacobian actions
 * performed. The device runs one Arnoldi iteration ahead of the host's stop
 * test, so a GMRES solve that stops before max_krylov performs two actions
 * beyond its last basis direction; one that runs to max_krylov performs none. */
typedef struct {
  int32_t converged, newton_iters, total_krylov, total_actions;
  double seconds;
  double res_norm[65];       /* L2 norm of r before each Newton step           */
  int32_t krylov[64];        /* GMRES iterations of each Newton step           */
  double gmres_relres[64];   /* final GMRES relative residual of each step      */
} sp_newton_report;

/* Newton-GMRES on r(U) = (Phi_dt(U) - U)/dt = 0 (Sec. 2): U <- U - du with
 * J_r du = r solved by unrestarted GMRES (x0 = 0, classical Gram-Schmidt with
 * reorthogonalisation, Givens rotations) in the packed Euclidean product. The
 * Arnoldi iterations run on the device without a host round trip; the host
 * applies the rotations and the stop test one iteration behind.
 * u_inout: initial guess in, final iterate out. Synchronises. Returns SP_OK on
 * convergence, SP_ERR_NOT_CONVERGED otherwise (report filled either way). */
sp_status sp_newton_gmres(sp_plan* plan, double* u_inout, const sp_newton_opts* opts,
                          sp_newton_report* report);

typedef struct {
  int32_t max_trials;  /* candidate steps per Newton iteration (>= 1)            */
  double delta_init;   /* first trust radius; <= 0: length of the first Newton step */
  double delta_min;    /* give up when a rejection takes the radius below (> 0)  */
  double delta_max;    /* upper limit of the radius (>= delta_min)                */
} sp_hook_opts;

typedef struct {
  int32_t trials[64];    /* candidates evaluated in each accepted Newton step    */
  double delta[64];      /* trust radius the accepted step was computed with      */
  double mu[64];         /* its Lagrange multiplier (0: the unconstrained step)   */
  double step_norm[64];  /* its length ||y|| in the packed Euclidean norm          */
  double rho[64];        /* actual / predicted decrease of ||r||^2                 */
} sp_hook_report;

/* Newton-GMRES with the hookstep (Sec. 3.2: the step is kept inside a trusted
 * region of validity of the linearisation, after Viswanath 2007). Each Newton
 * iteration runs GMRES as sp_newton_gmres does, then takes du = Q y with y
 * minimising the GMRES model ||beta e_1 - Hbar y|| subject to ||y|| <= delta
 * (Q the orthonormal Krylov basis, so ||du|| = ||y|| in the packed Euclidean
 * norm). The candidate U - du is evaluated; with rho the ratio of the actual
 * to the predicted decrease of ||r||^2 (packed Euclidean), a candidate with
 * rho < 0.01 is rejected and delta set to half of min(delta, ||y||); an
 * accepted step halves delta (to ||y|| / 2) when rho < 0.25 and doubles it (up
 * to delta_max) when rho > 0.75 and the constraint was active. A rejected
 * candidate costs one Phi evaluation and no new Krylov work. Stops with
 * SP_ERR_NOT_CONVERGED when max_trials candidates in a row are rejected or the
 * radius falls below delta_min. Arguments as for sp_newton_gmres; hook_report
 * may be NULL. The residual of an accepted candidate is reused by the next
 * iteration, so total_actions counts every Phi and JVP evaluation once. */
sp_status sp_newton_hookstep(sp_plan* plan, double* u_inout, const sp_newton_opts* opts,
                             const sp_hook_opts* hook, sp_newton_report* report,
                             sp_hook_report* hook_report);

/* Projection onto the fields invariant under the shift-reflect group of plane
 * Couette flow that contains EQ1 (Sec. 3.3), {1, s1, s2, s1 s2} with
 *   s1 [u, v, w](x, y, z) = [u, v, -w](x + Lx/2, y, -z),
 *   s2 [u, v, w](x, y, z) = [-u, -v, w](-x + Lx/2, -y, z + Lz/2):
 * field <- (field + s1 field + s2 field + s1 s2 field) / 4, in place, on the
 * device (canonical layout; Hermitian and Nyquist conventions preserved).
 * Phi_dt commutes with the group, so invariant fields stay invariant. */
sp_status sp_symmetrize(sp_plan* plan, double* field);
/* on != 0: the Newton drivers project the state and each residual with
 * sp_symmetrize, so that the search (and its Krylov spaces) stays in the
 * invariant subspace, which excludes the continuous translations. */
sp_status sp_plan_set_symmetry(sp_plan* plan, int32_t on);

/* The hookstep subproblem alone, on the host (no plan, no device work): R is
 * the k x k upper-triangular Givens-rotated GMRES matrix (column-major, leading
 * dimension ld >= k, nonzero diagonal), g the k+1 rotated right-hand side.
 * Writes y[k] minimising ||g[0..k-1] - R y||^2 + g[k]^2 over ||y|| <= delta
 * (delta > 0), its Lagrange multiplier *mu (0 when the unconstrained minimiser
 * fits) and the model residual norm *model_res. SP_ERR_INVALID on bad
 * arguments. This is the computation sp_newton_hookstep performs per trial. */
sp_status sp_hook_step(const double* R, int32_t ld, const double* g, int32_t k, double delta,
                       double* y, double* mu, double* model_res);

/* Per-kernel timing (tracing aid): when on != 0, every kernel the plan launches
 * is bracketed by HIP events on the plan's stream, which adds a small gap
 * between launches; leave it off for throughput measurements. */
sp_status sp_profile_enable(sp_plan* plan, int32_t on);
/* Synchronises, then writes for each kernel that ran since the last reset its
 * name (names: n_max slots of 32 chars, NUL terminated), launch count and
 * summed duration in ms; *n_out = number of kernels written. Clears the
 * counters if reset != 0. */
sp_status sp_profile_read(sp_plan* plan, int32_t n_max, char* names, int64_t* counts,
                          double* total_ms, int32_t* n_out, int32_t reset);

/* Stage timing (measurement aid). Evaluates Phi_dt(u) into out once, then
 * launches the kernel of one stage of that evaluation reps times back to back
 * on the plan's stream, between two HIP events, on the scratch state the
 * evaluation left (each stage reads its input buffer and writes its output
 * buffer, so repeated launches recompute the same result). Synchronises and
 * writes the average duration per launch in microseconds to *avg_us. On
 * return out holds Phi_dt(u). stage: SP_STAGE_*; reps in [1, 100000]; u and
 * out as for sp_befe_step, out must not alias u. Uses the plan's precision.
 * Where the z-line kernel takes the inverse x transforms itself (it reads the
 * y-valued fields; chosen per grid and precision), SP_STAGE_XINV launches
 * nothing and writes 0 to *avg_us, and SP_STAGE_ZLINE covers both stages. */
typedef enum {
  SP_STAGE_SYNTH = 0, /* y-synthesis of u, du/dy, v, w, dw/dy (Sec. 3.2) */
  SP_STAGE_XINV = 1,  /* curl factors, 3/2 padding, inverse x FFT */
  SP_STAGE_ZLINE = 2, /* [inverse x FFT,] inverse z FFT, u x omega, forward z FFT */
  SP_STAGE_XFWD = 3,  /* forward x FFT, truncation */
  SP_STAGE_SOLVE = 4  /* Chebyshev analysis + u/dt + per-mode implicit solve */
} sp_stage;
sp_status sp_time_stage(sp_plan* plan, int32_t stage, const double* u, double* out, int32_t reps,
                        double* avg_us);

const char* sp_status_string(sp_status s);
const char* sp_last_error(const sp_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* SP_H */
