// Device BLAS-1/2 for GMRES on canonical fields in the packed Euclidean
// inner product: <a, b> = sum over stored entries of w (a.re b.re + a.im b.im),
// w = 1 for m_z > 0 and for the (0,0) mode, 1/2 for the other m_z = 0 modes
// (each stored twice, at +m_x and -m_x), 0 at Nyquist entries.
#include <hip/hip_runtime.h>

#include "sp_internal.h"

namespace sp {

__device__ inline double packed_weight(size_t t, int nx, int ny, int nzh) {
  const int j = (int)((t / ny) % nzh);
  const int i = (int)((t / ((size_t)ny * nzh)) % nx);
  if (i == nx / 2 || j == nzh - 1) return 0.0;
  if (j > 0) return 1.0;
  return (i == 0) ? 1.0 : 0.5;
}

// partial[v * nb + block] = block's share of <V_v, w>, v = 0..nvec-1.
// V is nvec contiguous canonical vectors of n complex entries. Vectors are
// taken eight at a time: each thread streams its grid-strided entries of w
// once per group, then the eight sums are reduced with wave shuffles.
constexpr int kDotGroup = 8;

__global__ void __launch_bounds__(256)
    k_multidot(const double2* __restrict__ V, int nvec, const double2* __restrict__ w,
               double* __restrict__ partial, size_t n, int nx, int ny, int nzh) {
  __shared__ double red[4][kDotGroup];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (int v0 = 0; v0 < nvec; v0 += kDotGroup) {
    const int nv = (nvec - v0 < kDotGroup) ? nvec - v0 : kDotGroup;
    double acc[kDotGroup];
#pragma unroll
    for (int q = 0; q < kDotGroup; ++q) acc[q] = 0.0;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
      const double wt = packed_weight(t, nx, ny, nzh);
      const double2 x = w[t];
      const double wr = wt * x.x, wi = wt * x.y;
#pragma unroll
      for (int q = 0; q < kDotGroup; ++q) {
        if (q < nv) {
          const double2 a = V[(size_t)(v0 + q) * n + t];
          acc[q] += a.x * wr + a.y * wi;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kDotGroup; ++q) {
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) acc[q] += __shfl_xor(acc[q], d);
    }
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < kDotGroup; ++q) red[wid][q] = acc[q];
    }
    __syncthreads();
    if (threadIdx.x < nv)
      partial[(size_t)(v0 + threadIdx.x) * gridDim.x + blockIdx.x] =
          red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
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

// w = beta * w + alpha * sum_v h[v] V_v   (h in device memory)
__global__ void __launch_bounds__(256)
    k_multiaxpy(const double2* __restrict__ V, int nvec, const double* __restrict__ h,
                double alpha, double beta, double2* __restrict__ w, size_t n) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
       t += (size_t)gridDim.x * blockDim.x) {
    double rx = 0.0, ry = 0.0;
    for (int v = 0; v < nvec; ++v) {
      const double c = h[v];
      const double2 a = V[(size_t)v * n + t];
      rx += c * a.x;
      ry += c * a.y;
    }
    const double2 o = w[t];
    w[t] = make_double2(beta * o.x + alpha * rx, beta * o.y + alpha * ry);
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

hipError_t launch_multidot(sp_plan* p, const double2* V, int nvec, const double2* w,
                           double* partial, double* out, int* nb_out) {
  const size_t n = (size_t)3 * p->d.nx * p->d.nzh * p->d.ny;
  int nb = nblocks_for(n);
  if (nb > 256) nb = 256;
  SP_PROF_BEGIN(p, KID_MULTIDOT);
  hipLaunchKernelGGL(k_multidot, dim3(nb), dim3(256), 0, p->stream, V, nvec, w, partial, n, p->d.nx,
                     p->d.ny, p->d.nzh);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_rows, dim3(nvec), dim3(256), 0, p->stream, partial, nb, out);
  SP_PROF_END(p, KID_MULTIDOT);
  if (nb_out) *nb_out = nb;
  return hipGetLastError();
}

hipError_t launch_multiaxpy(sp_plan* p, const double2* V, int nvec, const double* h, double alpha,
                            double beta, double2* w) {
  const size_t n = (size_t)3 * p->d.nx * p->d.nzh * p->d.ny;
  SP_PROF_BEGIN(p, KID_MULTIAXPY);
  hipLaunchKernelGGL(k_multiaxpy, dim3(nblocks_for(n)), dim3(256), 0, p->stream, V, nvec, h, alpha,
                     beta, w, n);
  SP_PROF_END(p, KID_MULTIAXPY);
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
