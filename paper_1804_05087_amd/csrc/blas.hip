// Device BLAS-1/2 for GMRES on canonical fields in the packed Euclidean
// inner product: <a, b> = sum over stored entries of w (a.re b.re + a.im b.im),
// w = 1 for m_z > 0 and for the (0,0) mode, 1/2 for the other m_z = 0 modes
// (each stored twice, at +m_x and -m_x), 0 at Nyquist entries.
#include <hip/hip_runtime.h>

#include "sp_internal.h"

namespace sp {

// partial[(v * NR + r) * nb + chunk] = a chunk's share of <V_v, w_r>,
// v = 0..nvec-1, r < NR (one or two right-hand vectors). Block (chunk, g) owns
// 256 * ept consecutive entries of V's layout and the vectors 32 g .. 32 g + 31:
// each thread keeps its weighted entries of the w_r in registers (weights
// computed once), streams the vectors a group at a time, and the sums are
// reduced with wave shuffles and LDS.
// Layouts of V: CanonLayout (canonical fields, the packed product's weights)
// or CompactLayout (the Krylov basis: compact vectors, every weight 1; the w_r
// are canonical fields gathered through the map).
// The Krylov basis is stored in FP64 (double2) or, to halve the traffic of the
// orthogonalisation, in FP32 (float2); every sum is accumulated in FP64.
// Basis entries are read with nontemporal loads: a pass streams far more than
// the caches hold and reads each entry once, so the hint keeps the stream from
// evicting the cached operands (measured at 48x65x48 with 600 vectors: a GMRES
// solve 6.6 % faster with the FP64 basis, 3 % with the FP32 one).
typedef double basis_d2 __attribute__((ext_vector_type(2)));
typedef float basis_f2 __attribute__((ext_vector_type(2)));
__device__ inline double2 ld_basis(const double2* V, size_t i) {
  const basis_d2 x = __builtin_nontemporal_load(reinterpret_cast<const basis_d2*>(V + i));
  return make_double2(x.x, x.y);
}
__device__ inline double2 ld_basis(const float2* V, size_t i) {
  const basis_f2 f = __builtin_nontemporal_load(reinterpret_cast<const basis_f2*>(V + i));
  return make_double2(f.x, f.y);
}
__device__ inline double2 st_basis(double2* V, size_t i, double x, double y) {
  V[i] = make_double2(x, y);
  return make_double2(x, y);
}
// returns the stored (rounded) value
__device__ inline double2 st_basis(float2* V, size_t i, double x, double y) {
  const float2 f = make_float2((float)x, (float)y);
  V[i] = f;
  return make_double2(f.x, f.y);
}

// Entry t of a canonical field: itself, with the packed product's weight.
struct CanonLayout {
  int n, nx, ny, nzh;
  __device__ int size() const { return n; }
  __device__ int canon(int t, double* wt) const {
    const int j = (t / ny) % nzh;
    const int m = (t / (ny * nzh)) % nx;
    *wt = (m == nx / 2 || j == nzh - 1) ? 0.0 : (j > 0 ? 1.0 : (m == 0 ? 1.0 : 0.5));
    return t;
  }
};
// Entry t of a compact vector: its canonical index, weight 1.
struct CompactLayout {
  CMap m;
  __device__ int size() const { return m.len; }
  __device__ int canon(int t, double* wt) const {
    int mir;
    *wt = 1.0;
    return m.canon(t, &mir);
  }
};

// Launch shape per basis precision (measured at 48x65x48 with 24-200 vectors:
// an FP32 basis streams fastest with four vectors per group and eight entries
// per thread, an FP64 one with eight and four).
template <typename T>
struct DotShape {
  static constexpr int group = 8, ept = 4;
};
template <>
struct DotShape<float2> {
  static constexpr int group = 4, ept = 8;
};
constexpr int kDotVecs = 32;

template <int NR, typename T, class Layout>
__global__ void __launch_bounds__(256)
    k_multidot(const T* __restrict__ V, int nvec, const double2* __restrict__ w0,
               const double2* __restrict__ w1, double* __restrict__ partial, Layout L) {
  constexpr int kDotGroup = DotShape<T>::group;
  constexpr int kDotEPT = DotShape<T>::ept;
  __shared__ double red[4][kDotGroup * NR];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int n = L.size();
  const int t0 = blockIdx.x * 256 * kDotEPT + threadIdx.x;
  double wr[NR][kDotEPT], wi[NR][kDotEPT];
  int tc[kDotEPT];
#pragma unroll
  for (int i = 0; i < kDotEPT; ++i) {
    const int t = t0 + 256 * i;
    tc[i] = t < n ? t : n - 1;
    double wt;
    const int ci = L.canon(tc[i], &wt);
    if (t >= n) wt = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double2 x = (r == 0 ? w0 : w1)[ci];
      wr[r][i] = wt * x.x;
      wi[r][i] = wt * x.y;
    }
  }
  const int vbeg = blockIdx.y * kDotVecs;
  const int vend = min(nvec, vbeg + kDotVecs);
  for (int v0 = vbeg; v0 < vend; v0 += kDotGroup) {
    double acc[kDotGroup * NR];
#pragma unroll
    for (int q = 0; q < kDotGroup; ++q) {
      const int v = (v0 + q < vend) ? v0 + q : vend - 1;  // clamped; extra sums are dropped
      const T* Vv = V + (size_t)v * n;
      double2 av[kDotEPT];
#pragma unroll
      for (int i = 0; i < kDotEPT; ++i) av[i] = ld_basis(Vv, tc[i]);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < kDotEPT; ++i) s += av[i].x * wr[r][i] + av[i].y * wi[r][i];
        acc[q * NR + r] = s;
      }
    }
#pragma unroll
    for (int q = 0; q < kDotGroup * NR; ++q) {
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) acc[q] += __shfl_xor(acc[q], d);
    }
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < kDotGroup * NR; ++q) red[wid][q] = acc[q];
    }
    __syncthreads();
    const int q = threadIdx.x;
    if (q < kDotGroup * NR && v0 + q / NR < vend)
      partial[((size_t)v0 * NR + q) * gridDim.x + blockIdx.x] =
          red[0][q] + red[1][q] + red[2][q] + red[3][q];
    __syncthreads();
  }
}

// out[v] = sum_b partial[v * nb + b] (+ add[v] if add != NULL); one block per v.
__global__ void __launch_bounds__(256)
    k_reduce_rows(const double* __restrict__ partial, int nb, double* __restrict__ out) {
  __shared__ double red[256];
  const int v = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += partial[(size_t)v * nb + b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = red[0];
}

// w = beta * w + alpha * sum_v h[v] V_v (h in device memory) on the compact
// basis: entry t adds to its canonical entry of w and, conjugated, to the
// mirror entry (-m_x) of the m_z = 0 plane; w's other entries are untouched.
// One compact entry per thread; the vector loop is unrolled by eight so eight
// loads are in flight.
template <typename T>
__global__ void __launch_bounds__(256)
    k_multiaxpy(const T* __restrict__ V, int nvec, const double* __restrict__ h,
                double alpha, double beta, double2* __restrict__ w, CMap m) {
  const int n = m.len;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  double rx = 0.0, ry = 0.0;
  int v = 0;
  for (; v + 8 <= nvec; v += 8) {
    double2 a[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = ld_basis(V, (size_t)(v + q) * n + t);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double c = h[v + q];
      rx += c * a[q].x;
      ry += c * a[q].y;
    }
  }
  for (; v < nvec; ++v) {
    const double c = h[v];
    const double2 a = ld_basis(V, (size_t)v * n + t);
    rx += c * a.x;
    ry += c * a.y;
  }
  int mir;
  const int ci = m.canon(t, &mir);
  const double2 o = w[ci];
  w[ci] = make_double2(beta * o.x + alpha * rx, beta * o.y + alpha * ry);
  if (mir >= 0) {
    const double2 om = w[mir];
    w[mir] = make_double2(beta * om.x + alpha * rx, beta * om.y - alpha * ry);
  }
}

// The coefficients of one delayed-CGS2 Arnoldi step (newton.cpp), formed on the
// device so that the step's update pass does not wait for the host. Iteration j
// has dots[2 i + r] = <q_i, u_j> (r = 0) and <q_i, w> (r = 1) for i < j, then
// <u_j, u_j> and <u_j, w> (w = J u_j); a_i = dots[2 i], b_i = dots[2 i + 1].
// u_j's norm after the projection is gamma = sqrt(<u_j, u_j> - sum a_i^2); the
// Hessenberg column j-1 is completed as hprev + a (rows < j) and gamma (row j),
// hprev being the provisional column the previous iteration formed before u_j
// was reorthogonalised. With q_j = (u_j - Q a) / gamma and J Q = Q H,
//   J q_j = (w - Q (H a)) / gamma,
// so the next provisional column is hprev_i = (b_i - (H a)_i) / gamma (i < j),
// hprev_j = ((<u_j, w> - a.b) / gamma - (H a)_j) / gamma, and the update
// coefficients are c_i = (H a)_i / gamma + hprev_i (i <= j).
// H is kept row-major on the device (H[l ld + i] = H(l, i)), so that a row of
// H a is one contiguous run.

// Ha[l] = (H a)_l for l < j: the completed columns i <= j - 2 (rows l <= i + 1)
// plus column j - 1 = hprev + a. One wave per row.
__global__ void __launch_bounds__(256)
    k_arnoldi_ha(int j, int ld, const double* __restrict__ dots, const double* __restrict__ H,
                 const double* __restrict__ hprev, double* __restrict__ Ha) {
  const int l = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (l >= j) return;  // uniform per wave
  double s = 0.0;
  for (int i = (l > 0 ? l - 1 : 0) + lane; i <= j - 2; i += 64)
    s += H[(size_t)l * ld + i] * dots[2 * i];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
  if (lane == 0) Ha[l] = s + (hprev[l] + dots[2 * l]) * dots[2 * (j - 1)];
}

// One block: gamma, column j - 1 of H (device H and the host record), the new
// provisional column, a and c for the update pass (ac[i] = a_i, ac[cst + i] =
// c_i) and 1 / gamma. rec[0] = gamma, rec[1] = <u_j, u_j> - sum a_i^2 (its
// finiteness is the host's check), rec[2] = j, rec[4 + i] = H(i, j - 1) for
// i <= j (j > 0).
constexpr int kCoefThreads = 1024;
__global__ void __launch_bounds__(kCoefThreads)
    k_arnoldi_coef(int j, int ld, int cst, const double* __restrict__ dots, double* __restrict__ H,
                   double* __restrict__ hprev, const double* __restrict__ Ha,
                   double* __restrict__ ac, double* __restrict__ inv_gamma,
                   double* __restrict__ rec) {
  __shared__ double red[2][kCoefThreads / 64];
  const int t = threadIdx.x;
  double saa = 0.0, sab = 0.0;
  for (int i = t; i < j; i += kCoefThreads) {
    const double ai = dots[2 * i], bi = dots[2 * i + 1];
    saa += ai * ai;
    sab += ai * bi;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    saa += __shfl_xor(saa, d);
    sab += __shfl_xor(sab, d);
  }
  if ((t & 63) == 0) {
    red[0][t >> 6] = saa;
    red[1][t >> 6] = sab;
  }
  __syncthreads();
  double aa = 0.0, ab = 0.0;
#pragma unroll
  for (int q = 0; q < kCoefThreads / 64; ++q) {
    aa += red[0][q];
    ab += red[1][q];
  }
  const double g2 = dots[2 * j] - aa;
  const double gamma = g2 > 0.0 ? sqrt(g2) : 0.0;
  const double ig = 1.0 / gamma;  // infinite at a breakdown, where the host stops
  const double haj = j > 0 ? gamma * dots[2 * (j - 1)] : 0.0;  // (H a)_j
  for (int i = t; i < j; i += kCoefThreads) {
    const double ai = dots[2 * i], bi = dots[2 * i + 1];
    const double hc = hprev[i] + ai;
    H[(size_t)i * ld + (j - 1)] = hc;
    rec[4 + i] = hc;
    const double hai = Ha[i];
    const double hp = (bi - hai) * ig;
    hprev[i] = hp;
    ac[i] = ai;
    ac[cst + i] = hai * ig + hp;
  }
  if (t == 0) {
    if (j > 0) {
      H[(size_t)j * ld + (j - 1)] = gamma;
      rec[4 + j] = gamma;
    }
    const double hp = ((dots[2 * j + 1] - ab) * ig - haj) * ig;
    hprev[j] = hp;
    ac[cst + j] = haj * ig + hp;
    inv_gamma[0] = ig;
    rec[0] = gamma;
    rec[1] = g2;
    rec[2] = (double)j;
    rec[3] = 0.0;
  }
}

// One pass of the delayed-reorthogonalisation Arnoldi step (newton.cpp) on the
// compact basis:
//   q    = (u - sum_{i<j} a_i V_i) * inv_gamma            (written over u = V_j)
//   unew = w * inv_gamma - sum_{i<j} c_i V_i - c_j q
// Each V_i is read once for both sums; w is canonical (gathered through the
// map). q and unew are stored in the basis precision and c_j multiplies the
// stored q; u64 receives the stored unew as a canonical FP64 field (mirror
// entries conjugated; its Nyquist entries are never written and stay zero),
// the input of the next Jacobian action, so that the action and the basis see
// the same vector.
template <typename T>
__global__ void __launch_bounds__(256)
    k_dcgs2_update(T* V, int j, const double* __restrict__ a, const double* __restrict__ c,
                   const double* __restrict__ inv_gamma_p, const double2* __restrict__ w, T* unew,
                   double2* __restrict__ u64, CMap m) {
  const int n = m.len;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const double inv_gamma = inv_gamma_p[0];
  double ax = 0.0, ay = 0.0, cx = 0.0, cy = 0.0;
  int i = 0;
  for (; i + 8 <= j; i += 8) {
    double2 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = ld_basis(V, (size_t)(i + q) * n + t);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double ai = a[i + q], ci = c[i + q];
      ax += ai * v[q].x;
      ay += ai * v[q].y;
      cx += ci * v[q].x;
      cy += ci * v[q].y;
    }
  }
  for (; i < j; ++i) {
    const double2 v = ld_basis(V, (size_t)i * n + t);
    ax += a[i] * v.x;
    ay += a[i] * v.y;
    cx += c[i] * v.x;
    cy += c[i] * v.y;
  }
  int mir;
  const int cidx = m.canon(t, &mir);
  const double2 u = ld_basis(V, (size_t)j * n + t);
  const double2 q = st_basis(V, (size_t)j * n + t, (u.x - ax) * inv_gamma, (u.y - ay) * inv_gamma);
  const double2 wv = w[cidx];
  const double cj = c[j];
  const double2 un =
      st_basis(unew, t, wv.x * inv_gamma - cx - cj * q.x, wv.y * inv_gamma - cy - cj * q.y);
  u64[cidx] = un;
  if (mir >= 0) u64[mir] = make_double2(un.x, -un.y);
}

// dst (compact) = src (canonical, in the Hermitian form); with write_back the
// stored (possibly rounded) values replace src's entries and mirrors, so that
// src is the FP64 image of what the basis holds.
template <typename T>
__global__ void __launch_bounds__(256)
    k_compact(double2* src, T* __restrict__ dst, CMap m, int write_back) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= m.len) return;
  int mir;
  const int ci = m.canon(t, &mir);
  const double2 v = src[ci];
  const double2 s = st_basis(dst, t, v.x, v.y);
  if (write_back) {
    src[ci] = s;
    if (mir >= 0) src[mir] = make_double2(s.x, -s.y);
  }
}

// x = s * y
__global__ void k_scale(const double2* __restrict__ y, double s, double2* __restrict__ x,
                        size_t n) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
       t += (size_t)gridDim.x * blockDim.x)
    x[t] = make_double2(s * y[t].x, s * y[t].y);
}

// Makes the m_z = 0 plane exactly Hermitian (entry at -m_x := conjugate of the
// one at +m_x, (0,0) real) and zeroes Nyquist entries, so that Krylov vectors
// stay in the real vector space the packed product is defined on.
__global__ void k_hermitian(double2* __restrict__ a, int nx, int ny, int nzh) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = 3 * nx * ny;  // (component, i, n) in the m_z = 0 plane
  if (t < total) {
    const int n = t % ny;
    const int i = (t / ny) % nx;
    const int c = t / (ny * nx);
    const size_t o = (((size_t)c * nx + i) * nzh + 0) * ny + n;
    if (i == 0) {
      a[o].y = 0.0;
    } else if (i == nx / 2) {
      a[o] = make_double2(0.0, 0.0);
    } else if (i < nx / 2) {
      const size_t om = (((size_t)c * nx + (nx - i)) * nzh + 0) * ny + n;
      a[om] = make_double2(a[o].x, -a[o].y);
    }
  }
  // Nyquist m_z column
  if (t < 3 * nx * ny) {
    const int n = t % ny;
    const int i = (t / ny) % nx;
    const int c = t / (ny * nx);
    a[(((size_t)c * nx + i) * nzh + (nzh - 1)) * ny + n] = make_double2(0.0, 0.0);
  }
}

static int nblocks_for(size_t n) {
  size_t b = (n + 255) / 256;
  if (b > 1024) b = 1024;
  return (int)b;
}

// element chunks of the FP64 shape over a canonical field; the compact layout
// and the FP32 shape have fewer
int multidot_blocks(const sp_plan* p) {
  const int n = 3 * p->d.nx * p->d.nzh * p->d.ny;
  constexpr int e = DotShape<double2>::ept;
  return (n + 256 * e - 1) / (256 * e);
}

template <typename T, class Layout>
static hipError_t multidot_impl(sp_plan* p, const T* V, int n, Layout L, int nvec,
                                const double2* w0, const double2* w1, int nr, double* partial,
                                double* out) {
  constexpr int ept = DotShape<T>::ept;
  static_assert(ept >= DotShape<double2>::ept, "the partial buffer holds multidot_blocks chunks");
  const int nb = (n + 256 * ept - 1) / (256 * ept);
  SP_PROF_BEGIN(p, KID_MULTIDOT);
  const dim3 grid(nb, (nvec + kDotVecs - 1) / kDotVecs);
  if (nr == 1)
    hipLaunchKernelGGL((k_multidot<1, T, Layout>), grid, dim3(256), 0, p->stream, V, nvec, w0, w0,
                       partial, L);
  else
    hipLaunchKernelGGL((k_multidot<2, T, Layout>), grid, dim3(256), 0, p->stream, V, nvec, w0, w1,
                       partial, L);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_rows, dim3(nr * nvec), dim3(256), 0, p->stream, partial, nb, out);
  SP_PROF_END(p, KID_MULTIDOT);
  return hipGetLastError();
}

hipError_t launch_multidot(sp_plan* p, const double2* V, int nvec, const double2* w,
                           double* partial, double* out, int* nb_out) {
  if (nb_out) *nb_out = multidot_blocks(p);
  const int n = 3 * p->d.nx * p->d.nzh * p->d.ny;
  const CanonLayout L{n, p->d.nx, p->d.ny, p->d.nzh};
  return multidot_impl(p, V, n, L, nvec, w, w, 1, partial, out);
}

template <typename T>
static hipError_t kmultidot2(sp_plan* p, const T* V, int nvec, const double2* w0,
                             const double2* w1, double* partial, double* out) {
  const CompactLayout L{compact_map(p->d)};
  return multidot_impl(p, V, L.m.len, L, nvec, w0, w1, 2, partial, out);
}
hipError_t launch_krylov_multidot2(sp_plan* p, const double2* V, int nvec, const double2* w0,
                                   const double2* w1, double* partial, double* out) {
  return kmultidot2(p, V, nvec, w0, w1, partial, out);
}
hipError_t launch_krylov_multidot2(sp_plan* p, const float2* V, int nvec, const double2* w0,
                                   const double2* w1, double* partial, double* out) {
  return kmultidot2(p, V, nvec, w0, w1, partial, out);
}

template <typename T>
static hipError_t multiaxpy_impl(sp_plan* p, const T* V, int nvec, const double* h, double alpha,
                                 double beta, double2* w) {
  const CMap m = compact_map(p->d);
  SP_PROF_BEGIN(p, KID_MULTIAXPY);
  hipLaunchKernelGGL(k_multiaxpy<T>, dim3((m.len + 255) / 256), dim3(256), 0, p->stream, V, nvec,
                     h, alpha, beta, w, m);
  SP_PROF_END(p, KID_MULTIAXPY);
  return hipGetLastError();
}
hipError_t launch_krylov_multiaxpy(sp_plan* p, const double2* V, int nvec, const double* h,
                                   double alpha, double beta, double2* w) {
  return multiaxpy_impl(p, V, nvec, h, alpha, beta, w);
}
hipError_t launch_krylov_multiaxpy(sp_plan* p, const float2* V, int nvec, const double* h,
                                   double alpha, double beta, double2* w) {
  return multiaxpy_impl(p, V, nvec, h, alpha, beta, w);
}

template <typename T>
static hipError_t dcgs2_impl(sp_plan* p, T* V, int j, const double* a, const double* c,
                             const double* inv_gamma, const double2* w, T* unew, double2* u64) {
  const CMap m = compact_map(p->d);
  SP_PROF_BEGIN(p, KID_MULTIAXPY);
  hipLaunchKernelGGL(k_dcgs2_update<T>, dim3((m.len + 255) / 256), dim3(256), 0, p->stream, V, j,
                     a, c, inv_gamma, w, unew, u64, m);
  SP_PROF_END(p, KID_MULTIAXPY);
  return hipGetLastError();
}
hipError_t launch_dcgs2_update(sp_plan* p, double2* V, int j, const double* a, const double* c,
                              const double* inv_gamma, const double2* w, double2* unew,
                              double2* u64) {
  return dcgs2_impl(p, V, j, a, c, inv_gamma, w, unew, u64);
}
hipError_t launch_dcgs2_update(sp_plan* p, float2* V, int j, const double* a, const double* c,
                              const double* inv_gamma, const double2* w, float2* unew,
                              double2* u64) {
  return dcgs2_impl(p, V, j, a, c, inv_gamma, w, unew, u64);
}

hipError_t launch_arnoldi_coef(sp_plan* p, int j, int ld, int cst, const double* dots, double* H,
                              double* hprev, double* Ha, double* ac, double* inv_gamma,
                              double* rec) {
  SP_PROF_BEGIN(p, KID_MULTIAXPY);
  if (j > 0) {
    hipLaunchKernelGGL(k_arnoldi_ha, dim3((j + 3) / 4), dim3(256), 0, p->stream, j, ld, dots, H,
                       hprev, Ha);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_arnoldi_coef, dim3(1), dim3(kCoefThreads), 0, p->stream, j, ld, cst, dots,
                     H, hprev, Ha, ac, inv_gamma, rec);
  SP_PROF_END(p, KID_MULTIAXPY);
  return hipGetLastError();
}

template <typename T>
static hipError_t compact_impl(sp_plan* p, double2* src, T* dst, int write_back) {
  const CMap m = compact_map(p->d);
  SP_PROF_BEGIN(p, KID_SCALE);
  hipLaunchKernelGGL(k_compact<T>, dim3((m.len + 255) / 256), dim3(256), 0, p->stream, src, dst,
                     m, write_back);
  SP_PROF_END(p, KID_SCALE);
  return hipGetLastError();
}
hipError_t launch_compact(sp_plan* p, double2* src, double2* dst) {
  return compact_impl(p, src, dst, 0);
}
hipError_t launch_compact(sp_plan* p, double2* src, float2* dst) {
  return compact_impl(p, src, dst, 1);
}

// out = a x + b y on a canonical field, written in the form the packed real
// vector represents: the m_z = 0 plane exactly Hermitian (entry -m_x is the
// conjugate of entry m_x, the (0, 0) mode real) and every Nyquist entry zero.
// Entry -m_x of the m_z = 0 plane is computed from the inputs' entry m_x, so
// out must not alias x or y.
__global__ void k_axpby_herm(const double2* __restrict__ x, double a,
                             const double2* __restrict__ y, double b, double2* __restrict__ out,
                             int nx, int ny, int nzh) {
  const int n_all = 3 * nx * nzh * ny;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n_all; t += gridDim.x * blockDim.x) {
    const int j = (t / ny) % nzh;
    const int i = (t / (ny * nzh)) % nx;
    if (i == nx / 2 || j == nzh - 1) {
      out[t] = make_double2(0.0, 0.0);
      continue;
    }
    const bool mirror = (j == 0 && i > nx / 2);
    const int src = mirror ? t + (nx - 2 * i) * nzh * ny : t;  // entry (nx - i, 0, n)
    const double2 X = x[src], Y = y[src];
    double re = a * X.x + b * Y.x;
    double im = a * X.y + b * Y.y;
    if (j == 0 && i == 0) im = 0.0;
    out[t] = make_double2(re, mirror ? -im : im);
  }
}

hipError_t launch_axpby_herm(sp_plan* p, const double2* x, double a, const double2* y, double b,
                             double2* out) {
  const auto& d = p->d;
  const int n = 3 * d.nx * d.nzh * d.ny;
  int blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  SP_PROF_BEGIN(p, KID_AXPBY);
  hipLaunchKernelGGL(k_axpby_herm, dim3(blocks), dim3(256), 0, p->stream, x, a, y, b, out, d.nx,
                     d.ny, d.nzh);
  SP_PROF_END(p, KID_AXPBY);
  return hipGetLastError();
}

// In-place projection onto the fields invariant under the shift-reflect group
// {1, s1, s2, s1 s2} of plane Couette flow,
//   s1 [u, v, w](x, y, z) = [u, v, -w](x + Lx/2, y, -z),
//   s2 [u, v, w](x, y, z) = [-u, -v, w](-x + Lx/2, -y, z + Lz/2),
// P = (1 + s1 + s2 + s1 s2) / 4. On coefficients of mode (m_x, m_z, n) of
// component c, with A = a(m_x) and B = a(-m_x):
//   s1 a(m_x) = (-1)^m_x z_c conj(B),  s2 a(m_x) = r_c (-1)^(m_x + m_z + n) B,
//   s1 s2 a(m_x) = z_c r_c (-1)^(m_z + n) conj(A),
// z = (1, 1, -1), r = (-1, -1, 1). One thread owns the pair (m_x, -m_x) for one
// (c, m_z, n) and writes both; the x Nyquist column stays as it is (zero).
__global__ void k_symmetrize(double2* __restrict__ a, int nx, int ny, int nzh) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int hx = nx / 2;
  const int total = 3 * hx * nzh * ny;  // i = 0 .. nx/2 - 1 (partner nx - i)
  if (t >= total) return;
  const int n = t % ny;
  const int j = (t / ny) % nzh;
  const int i = (t / (ny * nzh)) % hx;
  const int c = t / (ny * nzh * hx);
  const int in = (nx - i) % nx;
  const size_t ia = (((size_t)c * nx + i) * nzh + j) * ny + n;
  const size_t ib = (((size_t)c * nx + in) * nzh + j) * ny + n;
  const double2 A = a[ia], B = a[ib];
  const double z = (c == 2) ? -1.0 : 1.0;
  const double r = (c == 2) ? 1.0 : -1.0;
  const double sx = (i & 1) ? -1.0 : 1.0;        // (-1)^m_x (the same for -m_x)
  const double szn = ((j + n) & 1) ? -1.0 : 1.0;  // (-1)^(m_z + n)
  // P a(m_x)
  const double2 pa = make_double2(0.25 * (A.x + sx * z * B.x + r * sx * szn * B.x + z * r * szn * A.x),
                                  0.25 * (A.y - sx * z * B.y + r * sx * szn * B.y - z * r * szn * A.y));
  // P a(-m_x): the same with A and B exchanged
  const double2 pb = make_double2(0.25 * (B.x + sx * z * A.x + r * sx * szn * A.x + z * r * szn * B.x),
                                  0.25 * (B.y - sx * z * A.y + r * sx * szn * A.y - z * r * szn * B.y));
  a[ia] = pa;
  if (in != i) a[ib] = pb;
}

__global__ void k_fill(double* __restrict__ a, size_t n, double v) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
       t += (size_t)gridDim.x * blockDim.x)
    a[t] = v;
}

hipError_t launch_fill(sp_plan* p, double* a, size_t n, double v) {
  SP_PROF_BEGIN(p, KID_SCALE);
  hipLaunchKernelGGL(k_fill, dim3(nblocks_for(n)), dim3(256), 0, p->stream, a, n, v);
  SP_PROF_END(p, KID_SCALE);
  return hipGetLastError();
}

__global__ void k_sbdf2_combine(double2* __restrict__ nv, double2* __restrict__ prev, size_t n) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
       t += (size_t)gridDim.x * blockDim.x) {
    const double2 a = nv[t], b = prev[t];
    nv[t] = make_double2(2.0 * a.x - b.x, 2.0 * a.y - b.y);
    prev[t] = a;
  }
}

hipError_t launch_sbdf2_combine(sp_plan* p, double2* nv, double2* prev, size_t n) {
  SP_PROF_BEGIN(p, KID_AXPBY);
  hipLaunchKernelGGL(k_sbdf2_combine, dim3(nblocks_for(n)), dim3(256), 0, p->stream, nv, prev, n);
  SP_PROF_END(p, KID_AXPBY);
  return hipGetLastError();
}

hipError_t launch_set_entry(sp_plan* p, double* a, size_t i, double v) {
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, p->stream, a + i, (size_t)1, v);
  return hipGetLastError();
}

hipError_t launch_symmetrize(sp_plan* p, double2* a) {
  const int total = 3 * (p->d.nx / 2) * p->d.nzh * p->d.ny;
  SP_PROF_BEGIN(p, KID_SCALE);
  hipLaunchKernelGGL(k_symmetrize, dim3((total + 255) / 256), dim3(256), 0, p->stream, a,
                     p->d.nx, p->d.ny, p->d.nzh);
  SP_PROF_END(p, KID_SCALE);
  return hipGetLastError();
}

hipError_t launch_hermitian(sp_plan* p, double2* a) {
  const int total = 3 * p->d.nx * p->d.ny;
  SP_PROF_BEGIN(p, KID_SCALE);
  hipLaunchKernelGGL(k_hermitian, dim3((total + 255) / 256), dim3(256), 0, p->stream, a, p->d.nx,
                     p->d.ny, p->d.nzh);
  SP_PROF_END(p, KID_SCALE);
  return hipGetLastError();
}

hipError_t launch_scale(sp_plan* p, const double2* y, double s, double2* x) {
  const size_t n = (size_t)3 * p->d.nx * p->d.nzh * p->d.ny;
  SP_PROF_BEGIN(p, KID_SCALE);
  hipLaunchKernelGGL(k_scale, dim3(nblocks_for(n)), dim3(256), 0, p->stream, y, s, x, n);
  SP_PROF_END(p, KID_SCALE);
  return hipGetLastError();
}

}  // namespace sp
