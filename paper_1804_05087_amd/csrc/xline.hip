// x-line kernels with register-resident FFTs (paper Sec. 3.2: 3/2 zero
// padding in x). Same four-step split as the z-line kernels: a line of length
// P = P1 * P2 is transformed by P2 threads holding P1 values each, one
// exchange through LDS, then P1 threads holding P2 values each.
//
//   k_xinv_reg  y-valued spectral fields [f][y][kz][mx] (nx modes, FFT order)
//               -> zero padded to P = 3 nx / 2 -> inverse FFT -> [f][y][x][kz]
//   k_xfwd_reg  [f][y][x][kz] -> forward FFT -> truncated to nx modes (Nyquist
//               zero) -> [f][y][kz][mx]
// Block: (y, field, chunk of kc z-modes); a thread of the second step writes
// its physical points for consecutive kz, so stores to the x-major layout are
// contiguous across lanes.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "sp_internal.h"

namespace sp {

// Logical block (y, field, z-chunk) of an x-line grid (hardware grid
// (ny, nfields, chunks)), reordered by xcd_order with the field fastest and
// then the chunk: the blocks of one (y, chunk), which read the same spectral
// lines for different output fields, share an L2.
struct XBlk {
  int y, f, ch;
};
__device__ inline XBlk xline_block() {
  const int gy = gridDim.x, gf = gridDim.y, gc = gridDim.z;
  const int b = blockIdx.x + gy * (blockIdx.y + gf * blockIdx.z);
  const int l = xcd_order(b, gy * gf * gc);
  return XBlk{l / (gf * gc), l % gf, (l / gf) % gc};
}

// plain == 0: output field f of (u, v, w, omega_x, omega_y, omega_z) from the
// five y-valued fields (u, du/dy, v, w, dw/dy) with i k_x, i k_z; plain != 0:
// output field f is input field f.
template <typename R, int P1, int P2>
__global__ void __launch_bounds__(128)
    k_xinv_reg(const typename V2<R>::T* __restrict__ yv, typename V2<R>::T* __restrict__ xp,
               const typename V2<R>::T* __restrict__ tw, int nx, int ny, int nzm, int kc, R alpha,
               R gamma, int plain) {
  using C = typename V2<R>::T;
  constexpr int P = P1 * P2;
  constexpr int S1 = P1 + 1;
  extern __shared__ unsigned char smem_raw[];
  C* twl = reinterpret_cast<C*>(smem_raw);
  C* ex = twl + P;  // [kc][P2][S1]
  const XBlk bk = xline_block();
  const int y = bk.y;
  const int f = bk.f;
  const int kz0 = bk.ch * kc;
  const int nl = min(kc, nzm - kz0);
  for (int t = threadIdx.x; t < P; t += blockDim.x) twl[t] = tw[t];
  __syncthreads();
  const size_t fs = (size_t)ny * nzm * nx;
  const int h = nx / 2;
  // step 1: task (l, n2), values at padded positions pos = P2 n1 + n2
  for (int task = threadIdx.x; task < kc * P2; task += blockDim.x) {
    const int l = task / P2;
    const int n2 = task - l * P2;
    if (l < nl) {
      const int kz = kz0 + l;
      const C* src = yv + ((size_t)y * nzm + kz) * nx;
      const R kzv = gamma * (R)kz;
      C v[P1];
#pragma unroll
      for (int n1 = 0; n1 < P1; ++n1) {
        const int pos = P2 * n1 + n2;
        const bool lo = pos < h;
        const bool hi = pos > P - h;
        const int i = lo ? pos : (hi ? pos - P + nx : 0);
        const R keep = (lo || hi) ? (R)1 : (R)0;
        const R kxv = alpha * (R)(lo ? i : i - nx);
        C val;
        if (plain) {
          val = src[f * fs + i];
        } else if (f == 0) {
          val = src[i];
        } else if (f == 1) {
          val = src[2 * fs + i];
        } else if (f == 2) {
          val = src[3 * fs + i];
        } else if (f == 3) {  // dw/dy - i kz v
          val = csub(src[4 * fs + i], sidot(cscale(src[2 * fs + i], kzv), (R)1));
        } else if (f == 4) {  // i kz u - i kx w
          val = sidot(csub(cscale(src[i], kzv), cscale(src[3 * fs + i], kxv)), (R)1);
        } else {  // i kx v - du/dy
          val = csub(sidot(cscale(src[2 * fs + i], kxv), (R)1), src[fs + i]);
        }
        v[n1] = cscale(val, keep);
      }
      dft_reg<P1, P, C, R>(v, (R)1, twl);
      C* e = ex + (l * P2 + n2) * S1;
#pragma unroll
      for (int k1 = 0; k1 < P1; ++k1)
        e[k1] = (k1 == 0 || n2 == 0) ? v[k1] : cmul(v[k1], wpow<P, P, C, R>(n2 * k1, (R)1, twl));
    }
  }
  __syncthreads();
  // step 2: task (k1, l), physical points x = k1 + P1 k2
  C* dst = xp + ((size_t)f * ny + y) * P * nzm + kz0;
  for (int task = threadIdx.x; task < P1 * kc; task += blockDim.x) {
    const int k1 = task / kc;
    const int l = task - k1 * kc;
    if (l < nl) {
      C t[P2];
      const C* e = ex + l * P2 * S1 + k1;
#pragma unroll
      for (int n2 = 0; n2 < P2; ++n2) t[n2] = e[n2 * S1];
      dft_reg<P2, P, C, R>(t, (R)1, twl);
#pragma unroll
      for (int k2 = 0; k2 < P2; ++k2) dst[(size_t)(k1 + P1 * k2) * nzm + l] = t[k2];
    }
  }
}

template <typename R, int P1, int P2>
__global__ void __launch_bounds__(128)
    k_xfwd_reg(const typename V2<R>::T* __restrict__ np, typename V2<R>::T* __restrict__ nv,
               const typename V2<R>::T* __restrict__ tw, int nx, int ny, int nzm, int kc) {
  using C = typename V2<R>::T;
  constexpr int P = P1 * P2;
  constexpr int S1 = P1 + 1;
  extern __shared__ unsigned char smem_raw[];
  C* twl = reinterpret_cast<C*>(smem_raw);
  C* ex = twl + P;  // [kc][P2][S1]
  const XBlk bk = xline_block();
  const int y = bk.y;
  const int c = bk.f;
  const int kz0 = bk.ch * kc;
  const int nl = min(kc, nzm - kz0);
  for (int t = threadIdx.x; t < P; t += blockDim.x) twl[t] = tw[t];
  __syncthreads();
  const int h = nx / 2;
  // step 1: task (n1, l); points x = n1 + P1 n2, m = P2 m1 + m2
  const C* src = np + ((size_t)c * ny + y) * P * nzm + kz0;
  for (int task = threadIdx.x; task < P1 * kc; task += blockDim.x) {
    const int n1 = task / kc;
    const int l = task - n1 * kc;
    if (l < nl) {
      C t[P2];
#pragma unroll
      for (int n2 = 0; n2 < P2; ++n2) t[n2] = src[(size_t)(n1 + P1 * n2) * nzm + l];
      dft_reg<P2, P, C, R>(t, (R)-1, twl);
      C* e = ex + l * P2 * S1 + n1;
#pragma unroll
      for (int m2 = 0; m2 < P2; ++m2)
        e[m2 * S1] = (m2 == 0 || n1 == 0) ? t[m2] : cmul(t[m2], wpow<P, P, C, R>(n1 * m2, (R)-1, twl));
    }
  }
  __syncthreads();
  // step 2: task (l, m2); keep |m_x| < nx / 2
  for (int task = threadIdx.x; task < kc * P2; task += blockDim.x) {
    const int l = task / P2;
    const int m2 = task - l * P2;
    if (l < nl) {
      C v[P1];
      const C* e = ex + (l * P2 + m2) * S1;
#pragma unroll
      for (int n1 = 0; n1 < P1; ++n1) v[n1] = e[n1];
      dft_reg<P1, P, C, R>(v, (R)-1, twl);
      C* dst = nv + (((size_t)c * ny + y) * nzm + kz0 + l) * nx;
#pragma unroll
      for (int m1 = 0; m1 < P1; ++m1) {
        const int pos = P2 * m1 + m2;
        if (pos < h)
          dst[pos] = v[m1];
        else if (pos > P - h)
          dst[pos - P + nx] = v[m1];
      }
      if (m2 == 0) dst[h] = mk((R)0, (R)0);
    }
  }
}

// ----------------------------------- launchers -----------------------------------

hipError_t launch_fft_x_inv_lds(sp_plan* p, const void* in, void* out, int nfields, int plain,
                                bool fp32);
hipError_t launch_fft_x_fwd_lds(sp_plan* p, const void* in, void* out, int nfields, bool fp32);

// z-modes per block: the fewest chunks that give the grid at least 512 blocks
// (and at least 4 modes per chunk) and keep the exchange buffer within 64 KiB
// of LDS, split evenly; a chunk is widened to a whole number of 128-byte cache
// lines (8 FP64 or 16 FP32 complex values) when that keeps the same even split,
// so that chunks of the x-physical rows [x][kz] start on line boundaries
static int xline_chunk(const Dims& d, int nfields, bool fp32, int P1, int P2) {
  const int lw = fp32 ? 16 : 8;
  const size_t el = fp32 ? sizeof(float2) : sizeof(double2);
  const long per = (long)d.ny * nfields;
  const int nmax = d.nzm / 4 > 1 ? d.nzm / 4 : 1;
  auto lds = [&](int kc) { return ((size_t)d.px + (size_t)kc * P2 * (P1 + 1)) * el; };
  int nch = 1;
  while (nch < d.nzm &&
         ((nch < nmax && per * nch < 512) || lds((d.nzm + nch - 1) / nch) > 65536))
    ++nch;
  int kc = (d.nzm + nch - 1) / nch;
  const int ka = (kc + lw - 1) / lw * lw;
  if (d.nzm % ka == 0 && d.nzm / ka == nch) kc = ka;
  return kc;
}

hipError_t launch_fft_x_inv_gen(sp_plan* p, const void* in, void* out, int nfields, int plain,
                                bool fp32) {
  const Dims& d = p->d;
  const int P1 = reg_fft_split(d.px);
  if (P1 == 0) return launch_fft_x_inv_lds(p, in, out, nfields, plain, fp32);
  const int P2 = d.px / P1;
  const int kc = xline_chunk(d, nfields, fp32, P1, P2);
  const dim3 grid(d.ny, nfields, (d.nzm + kc - 1) / kc);
  const size_t el = fp32 ? sizeof(float2) : sizeof(double2);
  const size_t sh = ((size_t)d.px + (size_t)kc * P2 * (P1 + 1)) * el;
  SP_PROF_BEGIN(p, KID_FFT_X_INV);
#define XI(A, B)                                                                                \
  if (fp32)                                                                                     \
    hipLaunchKernelGGL((k_xinv_reg<float, A, B>), grid, dim3(128), sh, p->stream,               \
                       (const float2*)in, (float2*)out, p->f_twx, d.nx, d.ny, d.nzm, kc,        \
                       (float)d.alpha, (float)d.gamma, plain);                                  \
  else                                                                                          \
    hipLaunchKernelGGL((k_xinv_reg<double, A, B>), grid, dim3(128), sh, p->stream,              \
                       (const double2*)in, (double2*)out, p->d_twx, d.nx, d.ny, d.nzm, kc,      \
                       d.alpha, d.gamma, plain)
  SP_REG_FFT_DISPATCH(d.px, XI)
#undef XI
  SP_PROF_END(p, KID_FFT_X_INV);
  return hipGetLastError();
}

hipError_t launch_fft_x_fwd_gen(sp_plan* p, const void* in, void* out, int nfields, bool fp32) {
  const Dims& d = p->d;
  const int P1 = reg_fft_split(d.px);
  if (P1 == 0) return launch_fft_x_fwd_lds(p, in, out, nfields, fp32);
  const int P2 = d.px / P1;
  const int kc = xline_chunk(d, nfields, fp32, P1, P2);
  const dim3 grid(d.ny, nfields, (d.nzm + kc - 1) / kc);
  const size_t el = fp32 ? sizeof(float2) : sizeof(double2);
  const size_t sh = ((size_t)d.px + (size_t)kc * P2 * (P1 + 1)) * el;
  SP_PROF_BEGIN(p, KID_FFT_X_FWD);
#define XF(A, B)                                                                                 \
  if (fp32)                                                                                      \
    hipLaunchKernelGGL((k_xfwd_reg<float, A, B>), grid, dim3(128), sh, p->stream,                \
                       (const float2*)in, (float2*)out, p->f_twx, d.nx, d.ny, d.nzm, kc);        \
  else                                                                                           \
    hipLaunchKernelGGL((k_xfwd_reg<double, A, B>), grid, dim3(128), sh, p->stream,               \
                       (const double2*)in, (double2*)out, p->d_twx, d.nx, d.ny, d.nzm, kc)
  SP_REG_FFT_DISPATCH(d.px, XF)
#undef XF
  SP_PROF_END(p, KID_FFT_X_FWD);
  return hipGetLastError();
}

hipError_t launch_fft_x_inv(sp_plan* p, bool fp32) {
  return launch_fft_x_inv_gen(p, p->yv, p->xp, 6, 0, fp32);
}

hipError_t launch_fft_x_fwd(sp_plan* p, bool fp32) {
  return launch_fft_x_fwd_gen(p, p->np, p->nv, 3, fp32);
}

}  // namespace sp
