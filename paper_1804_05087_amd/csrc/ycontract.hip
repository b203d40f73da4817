// Dense y-contractions on the matrix cores (v_mfma_*_16x16x4).
//
// Every Chebyshev transform of the step is a small dense matrix (ny x ny)
// applied to the ny-long y-columns of all 2 * nx * (nz/2) real columns of a
// field (paper Sec. 3.2: coefficients <-> values at the Gauss-Lobatto points):
//
//   k_ysynth_mfma  coefficients -> y-values:  out_f[y][col] = sum_n M_f[y][n] u_c[n][col]
//                  (synthesis with T and T.D; adjoint of the analysis with Tinv^T)
//   k_ycoef_mfma   y-values -> coefficients:  out_c[col][n] = sum_t sum_j M_t[n][j] Y_t[j][col]
//                  (analysis with Tinv)
//   k_adjsynth_mfma  the same form for the adjoint of the synthesis (T^T, (T.D)^T
//                  applied to curl-combined adjoint fields), operand staged in LDS
//
// A column is (kz, mx, re|im) with kz < nz/2, i.e. q = kz * nx + mx and
// col = 2q + re|im, which is the contiguous order of the y-valued layout
// [field][y][kz][mx]. Matrices are read through (row stride, column stride),
// so transposes cost nothing.
//
// Fragment layout of the 16x16x4 MFMA (one block, 64 lanes; l = lane),
// measured on gfx950:
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l, register i holds D[r][l % 16] with
//                r = 4 (l / 16) + i for f32 and r = (l / 16) + 4 i for f64.
// In k_ycoef_mfma a wave owns 16 real columns (8 modes) and one 16-row tile
// of the output, the block's four waves 32 consecutive modes, and rows beyond
// the last full tile (ny = 2^k + 1 leaves one) are finished on the vector unit
// with a 4-lane reduction; in k_ysynth_mfma a wave owns 16 modes (their real
// and imaginary columns as two MFMA column groups), the block's four waves 64,
// and the last, partial row tile goes through the MFMA like the others (its
// padded rows are zero).
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "sp_internal.h"

namespace sp {

template <typename R>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static constexpr bool kRegMajor = true;
  static __device__ inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output row held by register i of a lane in k-phase kq (= lane / 16)
  static __device__ inline int drow(int kq, int i) { return kq + 4 * i; }
};
template <>
struct Mfma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static constexpr bool kRegMajor = false;
  static __device__ inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int drow(int kq, int i) { return 4 * kq + i; }
};

template <typename R>
__device__ inline R sum_kphase(R v) {
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// One contraction matrix: its MFMA fragment table (every 16-row tile, the
// last one partial when 16 does not divide ny; zero padded beyond ny rows and
// columns) and the plain matrix with (row, column) strides.
template <typename R>
struct YMat {
  const R* frag;  // [ceil(ny / 16)][KS][64]
  const R* full;
  int rs, cs;     // element (r, c) at full[r * rs + c * cs]
};

// Synthesis work list: entry g applies matrix mat[g] to component comp[g] and
// writes y-valued field field[g] (one grid z index per entry).
template <typename R>
struct SynthSpec {
  int n;
  int comp[5];
  int field[5];
  YMat<R> mat[5];
};

// Logical (x, y, z) block of a contraction grid: the hardware index is
// reordered by xcd_order with the y index (output row tile) fastest, so the
// blocks that read the same columns for different row tiles share an L2.
struct Blk3 {
  int x, y, z;
};
__device__ inline Blk3 ycontract_block() {
  const int gx = gridDim.x, gy = gridDim.y;
  const int b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int l = xcd_order(b, gx * gy * (int)gridDim.z);
  const int rest = l / gy;
  return Blk3{rest % gx, l % gy, rest / gx};
}

// Synthesis: a wave owns 16 modes (kz * nx + mx = q0 .. q0 + 15), one 16-row
// tile of the output (the last tile may be partial: its padded rows are zero
// in the table and are not stored) and one work-list entry (matrix, component,
// field), so that every wave is one load -> MFMA -> store chain. Each lane
// loads one complex coefficient (16 bytes) per k-step and feeds its real part
// to one MFMA column group and its imaginary part to a second, so the two
// groups share every A fragment, a lane issues one load per two output values,
// and each output row of the wave is one contiguous run of 16 complex values
// (stored as pairs). Loads use clamped addresses and are masked after (a 0/1
// factor rather than a select keeps the compiler from sinking each load into
// a branch of its own).
template <typename R, int KS>
__global__ void __launch_bounds__(256)
    k_ysynth_mfma(const double2* __restrict__ u, SynthSpec<R> spec, R* __restrict__ out,
                   int nx, int ny, int nzh, int nzm) {
  using MF = Mfma<R>;
  using C = typename V2<R>::T;
  const int lane = threadIdx.x & 63;
  const int kq = lane >> 4;
  const int nq = nzm * nx;
  const Blk3 bk = ycontract_block();
  const int g = bk.z;
  const int t = bk.y;
  const int q0 = (bk.x * 4 + (threadIdx.x >> 6)) * 16;
  const int q = q0 + (lane & 15);
  const bool qv = q < nq;
  const size_t fstride = (size_t)ny * nq * 2;
  const YMat<R> M = spec.mat[g];
  R a[KS], br[KS], bi[KS];
  {
    const R* fa = M.frag + (size_t)t * KS * 64 + lane;
#pragma unroll
    for (int s = 0; s < KS; ++s) a[s] = fa[s * 64];
    const int qc = qv ? q : nq - 1;
    const int kz = qc / nx;
    const int mx = qc - kz * nx;
    const double2* src = u + (((size_t)spec.comp[g] * nx + mx) * nzh + kz) * ny;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int n = 4 * s + kq;
      const double2 v = src[n < ny ? n : ny - 1];
      const R m = (R)((qv && n < ny) ? 1 : 0);
      br[s] = (R)v.x * m;
      bi[s] = (R)v.y * m;
    }
  }
  // issue every load before the first MFMA waits on one: with one or two
  // waves per SIMD nothing else hides their latency (left alone, the
  // scheduler interleaves them with the MFMAs and keeps about ten in flight)
  typename MF::acc_t accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    accr = MF::mma(a[s], br[s], accr);
    acci = MF::mma(a[s], bi[s], acci);
  }
  if (qv) {
    R* o = out + (size_t)spec.field[g] * fstride + 2 * (size_t)q;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int y = 16 * t + MF::drow(kq, i);
      if (y < ny) {
        C v;
        v.x = accr[i];
        v.y = acci[i];
        *reinterpret_cast<C*>(o + (size_t)y * nq * 2) = v;
      }
    }
  }
}

// Loaders of the A operand of k_ycoef_mfma: the real part (ri = 0) or
// imaginary part (ri = 1) of term t of component c at y-index j, mode q.
template <typename R>
struct AnalysisLoad {
  const typename V2<R>::T* nv;  // [3][ny][nzm][nx]
  int ny, nq;
  __device__ R operator()(int, int c, int j, int q, int, int, int ri) const {
    const R* p = reinterpret_cast<const R*>(nv);
    return p[(((size_t)c * ny + j) * nq + q) * 2 + ri];
  }
};

// Adjoint of the synthesis followed by the curl combination: six y-valued
// adjoint fields F (u, v, w, omega_x, omega_y, omega_z) fold into
//   c = 0:  T^T (F0 - i kz F4) - (T.D)^T F5
//   c = 1:  T^T (F1 + i kz F3 - i kx F5)
//   c = 2:  T^T (F2 + i kx F4) + (T.D)^T F3
// (term 0 goes with T^T, term 1 with (T.D)^T); the x Nyquist column is zero.
template <typename R>
struct AdjSynthLoad {
  const typename V2<R>::T* F;  // [6][ny][nzm][nx]
  int nx, ny, nq;
  R alpha, gamma;
  // the combined value of term t, component c at y index j, mode q = (kz, mx)
  // (zero in the x Nyquist column)
  __device__ typename V2<R>::T value(int term, int c, int j, int q, int kz, int mx) const {
    using C = typename V2<R>::T;
    const size_t fs = (size_t)ny * nq;
    const size_t off = (size_t)j * nq + q;
    const int mxv = (mx < nx / 2) ? mx : mx - nx;
    const R kxv = alpha * (R)mxv;
    const R kzv = gamma * (R)kz;
    C v;
    if (term == 0) {
      if (c == 0) {
        v = csub(F[off], sidot(cscale(F[4 * fs + off], kzv), (R)1));
      } else if (c == 1) {
        v = cadd(F[fs + off],
                 sidot(csub(cscale(F[3 * fs + off], kzv), cscale(F[5 * fs + off], kxv)), (R)1));
      } else {
        v = cadd(F[2 * fs + off], sidot(cscale(F[4 * fs + off], kxv), (R)1));
      }
    } else {
      v = (c == 0) ? cscale(F[5 * fs + off], (R)-1) : F[3 * fs + off];
    }
    return (mx == nx / 2) ? mk((R)0, (R)0) : v;
  }
};

// out[c][mx][kz][n] = sum_t sum_j M_t(n, j) Y_t[j][(kz, mx)] + xa * x[c][mx][kz][n]
// for kz < nz/2 (x may be NULL); the z Nyquist rows kz = nz/2 get xa * x (or
// zero) from the blocks past the first nqb column blocks. nterm[c] terms for
// component c = the logical z block index.
template <typename R, int KS, class Load>
__global__ void __launch_bounds__(256)
    k_ycoef_mfma(Load load, int nterm0, int nterm1, int nterm2, YMat<R> M0, YMat<R> M1,
                 const double2* __restrict__ x, double xa, double2* __restrict__ out, int nx,
                 int ny, int nzh, int nzm, int nqb) {
  using MF = Mfma<R>;
  const Blk3 bk = ycontract_block();
  if (bk.x >= nqb) {  // block-uniform
    const int e = (bk.x - nqb) * 256 + (int)threadIdx.x;
    if (bk.y == 0 && e < nx * ny) {
      const int mx = e / ny;
      const int n = e - mx * ny;
      const size_t o = (((size_t)bk.z * nx + mx) * nzh + (nzh - 1)) * ny + n;
      double2 v = make_double2(0.0, 0.0);
      if (x != nullptr) v = make_double2(xa * x[o].x, xa * x[o].y);
      out[o] = v;
    }
    return;
  }
  const int lane = threadIdx.x & 63;
  const int kq = lane >> 4;
  const int nq = nzm * nx;
  const int c = bk.z;
  const int nterm = (c == 0) ? nterm0 : (c == 1 ? nterm1 : nterm2);
  const int q0 = (bk.x * 4 + (threadIdx.x >> 6)) * 8;
  // A fragments: this lane's column (mode qa, part ra) at j = 4 s + kq; indexes
  // clamped into range, values past the range zeroed after the load
  const int qa = q0 + ((lane & 15) >> 1);
  const int ra = lane & 1;
  const bool qav = qa < nq;
  const int qcl = qav ? qa : nq - 1;
  const int kza = qcl / nx;
  const int mxa = qcl - kza * nx;
  const int nt = ny >> 4;
  const int ty = (int)gridDim.y;  // row tiles of the launch
  R a[2][KS];
#pragma unroll
  for (int tm = 0; tm < 2; ++tm) {
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int j = 4 * s + kq;
      const R v = (tm < nterm) ? load(tm, c, j < ny ? j : ny - 1, qcl, kza, mxa, ra) : (R)0;
      a[tm][s] = v * (R)((qav && j < ny) ? 1 : 0);  // a mask, not a select (see k_ysynth_mfma)
    }
  }
  {
  const int t = bk.y;
  const bool tile = t < nt;
  const bool tail = (t == ty - 1) && (16 * nt < ny);
  if (tile) {
    const int n = 16 * t + (lane & 15);
    typename MF::acc_t acc = {0, 0, 0, 0};
#pragma unroll
    for (int tm = 0; tm < 2; ++tm) {
      if (tm < nterm) {
        const R* fb = (tm ? M1.frag : M0.frag) + (size_t)t * KS * 64 + lane;
        R bm[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) bm[s] = fb[s * 64];
#pragma unroll
        for (int s = 0; s < KS; ++s) acc = MF::mma(a[tm][s], bm[s], acc);
      }
    }
    // D row r is data column 2 q0 + r. f32 (r = 4 kq + i): registers (0, 1) and
    // (2, 3) are (re, im) of modes q0 + 2 kq + {0, 1}. f64 (r = kq + 4 i): the
    // lane holds one part of modes q0 + kq / 2 + 2 i; the other part sits in
    // lane ^ 16, and the pair (kq even, kq odd) writes i = 0, 1 and i = 2, 3.
    R pre[2], pim[2];
    int qd2[2];
    if constexpr (MF::kRegMajor) {
      R other[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) other[i] = __shfl_xor(acc[i], 16, 64);
      const int e = kq & 1;
#pragma unroll
      for (int pr = 0; pr < 2; ++pr) {
        const int i = 2 * e + pr;
        pre[pr] = e ? other[i] : acc[i];
        pim[pr] = e ? acc[i] : other[i];
        qd2[pr] = q0 + (kq >> 1) + 2 * i;
      }
    } else {
#pragma unroll
      for (int pr = 0; pr < 2; ++pr) {
        pre[pr] = acc[2 * pr];
        pim[pr] = acc[2 * pr + 1];
        qd2[pr] = q0 + 2 * kq + pr;
      }
    }
#pragma unroll
    for (int pr = 0; pr < 2; ++pr) {
      const int qd = qd2[pr];
      if (qd < nq) {
        const int kz = qd / nx;
        const int mx = qd - kz * nx;
        const size_t o = (((size_t)c * nx + mx) * nzh + kz) * ny + n;
        double re = (double)pre[pr], im = (double)pim[pr];
        if (x != nullptr) {
          const double2 xv = x[o];
          re += xa * xv.x;
          im += xa * xv.y;
        }
        out[o] = make_double2(re, im);
      }
    }
  }
  if (tail) {
    for (int n = 16 * nt; n < ny; ++n) {
      R part = 0;
#pragma unroll
      for (int tm = 0; tm < 2; ++tm) {
        if (tm < nterm) {
          const YMat<R> M = tm ? M1 : M0;
          const R* mrow = M.full + (size_t)n * M.rs;
          R mv[KS];
#pragma unroll
          for (int s = 0; s < KS; ++s) {
            const int j = 4 * s + kq;
            mv[s] = mrow[(size_t)(j < ny ? j : ny - 1) * M.cs];
          }
#pragma unroll
          for (int s = 0; s < KS; ++s) part += a[tm][s] * mv[s];  // a = 0 past ny
        }
      }
      part = sum_kphase(part);
      if (kq == 0 && qav) {
        const size_t o = (((size_t)c * nx + mxa) * nzh + kza) * ny + n;
        double v = (double)part;
        if (x != nullptr) v += xa * reinterpret_cast<const double*>(x + o)[ra];
        reinterpret_cast<double*>(out + o)[ra] = v;
      }
    }
  }
  }
}

// The transposed synthesis with its operand staged in LDS: a block owns 8 modes
// (16 real columns) of output component c. Its threads gather the curl-combined
// operand of those columns (AdjSynthLoad, every y index and term) once into
// LDS; wave t then computes output row tile t from it, the last tile partial
// (the tables' rows past ny are zero; those rows are not stored). So every
// operand element is gathered once, as with all tiles in one wave, while the
// tiles run on separate waves. Blocks past the ncb column blocks write the z
// Nyquist rows. Every entry is finished as
//   out = fa s (sum + xa x) + fb w,  s = 1/2 on the (0,0) mode and 1 elsewhere
// (x and w may be NULL: zero), the end of the VJP.
template <typename R, int KS>
__global__ void __launch_bounds__(640)
    k_adjsynth_mfma(AdjSynthLoad<R> ld, YMat<R> M0, YMat<R> M1, const double2* __restrict__ x,
                    double xa, double fa, double fb, const double2* __restrict__ w,
                    double2* __restrict__ out, int nx, int ny, int nzh, int nzm, int ncb) {
  using MF = Mfma<R>;
  using C = typename V2<R>::T;
  __shared__ R ys[2][4 * KS][16];
  const Blk3 bk = ycontract_block();
  const int c = bk.z;
  if (bk.x >= ncb) {  // block-uniform
    const int e = (bk.x - ncb) * (int)blockDim.x + (int)threadIdx.x;
    if (e < nx * ny) {
      const int mx = e / ny;
      const int n = e - mx * ny;
      const size_t o = (((size_t)c * nx + mx) * nzh + (nzh - 1)) * ny + n;
      double2 v = make_double2(0.0, 0.0);
      if (x != nullptr) v = make_double2(xa * x[o].x, xa * x[o].y);
      v = make_double2(fa * v.x, fa * v.y);
      if (w != nullptr) v = make_double2(v.x + fb * w[o].x, v.y + fb * w[o].y);
      out[o] = v;
    }
    return;
  }
  const int nq = nzm * nx;
  const int q0 = bk.x * 8;
  const int nterm = (c == 1) ? 1 : 2;
  for (int e = threadIdx.x; e < nterm * 4 * KS * 8; e += blockDim.x) {
    const int m = e & 7;
    const int rest = e >> 3;
    const int j = rest % (4 * KS);
    const int tm = rest / (4 * KS);
    const int q = q0 + m;
    C v = mk((R)0, (R)0);
    if (j < ny && q < nq) {
      const int kz = q / nx;
      v = ld.value(tm, c, j, q, kz, q - kz * nx);
    }
    ys[tm][j][2 * m] = v.x;
    ys[tm][j][2 * m + 1] = v.y;
  }
  __syncthreads();
  const int t = threadIdx.x >> 6;  // row tile (blockDim = 64 * row tiles)
  const int lane = threadIdx.x & 63;
  const int kq = lane >> 4;
  typename MF::acc_t acc = {0, 0, 0, 0};
  for (int tm = 0; tm < nterm; ++tm) {
    const R* fb = (tm ? M1.frag : M0.frag) + (size_t)t * KS * 64 + lane;
    R bm[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) bm[s] = fb[s * 64];
#pragma unroll
    for (int s = 0; s < KS; ++s) acc = MF::mma(ys[tm][4 * s + kq][lane & 15], bm[s], acc);
  }
  // D row r is data column 2 q0 + r (see k_ycoef_mfma)
  R pre[2], pim[2];
  int qd2[2];
  if constexpr (MF::kRegMajor) {
    R other[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) other[i] = __shfl_xor(acc[i], 16, 64);
    const int e = kq & 1;
#pragma unroll
    for (int pr = 0; pr < 2; ++pr) {
      const int i = 2 * e + pr;
      pre[pr] = e ? other[i] : acc[i];
      pim[pr] = e ? acc[i] : other[i];
      qd2[pr] = q0 + (kq >> 1) + 2 * i;
    }
  } else {
#pragma unroll
    for (int pr = 0; pr < 2; ++pr) {
      pre[pr] = acc[2 * pr];
      pim[pr] = acc[2 * pr + 1];
      qd2[pr] = q0 + 2 * kq + pr;
    }
  }
  const int n = 16 * t + (lane & 15);
#pragma unroll
  for (int pr = 0; pr < 2; ++pr) {
    const int qd = qd2[pr];
    if (qd < nq && n < ny) {
      const int kz = qd / nx;
      const int mx = qd - kz * nx;
      const size_t o = (((size_t)c * nx + mx) * nzh + kz) * ny + n;
      double re = (double)pre[pr], im = (double)pim[pr];
      if (x != nullptr) {
        const double2 xv = x[o];
        re += xa * xv.x;
        im += xa * xv.y;
      }
      const double sa = (qd == 0) ? 0.5 * fa : fa;  // qd = 0: the (0,0) mode
      re *= sa;
      im *= sa;
      if (w != nullptr) {
        const double2 wv = w[o];
        re += fb * wv.x;
        im += fb * wv.y;
      }
      out[o] = make_double2(re, im);
    }
  }
}

// ----------------------------------- launchers -----------------------------------

#define SP_KS_DISPATCH(ny, LAUNCH)             \
  do {                                         \
    switch (ycontract_ks(ny)) {                \
      case 5: LAUNCH(5); break;                \
      case 9: LAUNCH(9); break;                \
      case 17: LAUNCH(17); break;              \
      case 25: LAUNCH(25); break;              \
      default: LAUNCH(33); break;              \
    }                                          \
  } while (0)

template <typename R>
static YMat<R> ymat(const sp_plan* p, int id) {
  const int ny = p->d.ny;
  const bool f = sizeof(R) == sizeof(float);
  const R* frag = (const R*)(f ? (const void*)p->f_yfrag : (const void*)p->d_yfrag) +
                  (size_t)id * p->yfrag_stride;
  const R* T = (const R*)(f ? (const void*)p->f_T : (const void*)p->d_T);
  const R* TD = (const R*)(f ? (const void*)p->f_TD : (const void*)p->d_TD);
  const R* Ti = (const R*)(f ? (const void*)p->f_Tinv : (const void*)p->d_Tinv);
  switch (id) {
    case YM_T: return {frag, T, ny, 1};
    case YM_TD: return {frag, TD, ny, 1};
    case YM_TINV_T: return {frag, Ti, 1, ny};
    case YM_TINV: return {frag, Ti, ny, 1};
    case YM_T_T: return {frag, T, 1, ny};
    default: return {frag, TD, 1, ny};
  }
}

template <typename R>
static SynthSpec<R> synth_spec(const sp_plan* p, int which) {
  SynthSpec<R> sp{};
  if (which == 0) {  // forward: fields u, du/dy, v, w, dw/dy
    const int comp[5] = {0, 0, 1, 2, 2};
    const int mat[5] = {YM_T, YM_TD, YM_T, YM_T, YM_TD};
    sp.n = 5;
    for (int g = 0; g < 5; ++g) {
      sp.comp[g] = comp[g];
      sp.field[g] = g;
      sp.mat[g] = ymat<R>(p, mat[g]);
    }
  } else {  // adjoint of the analysis: Tinv^T on each component
    sp.n = 3;
    for (int g = 0; g < 3; ++g) {
      sp.comp[g] = g;
      sp.field[g] = g;
      sp.mat[g] = ymat<R>(p, YM_TINV_T);
    }
  }
  return sp;
}

static dim3 ycontract_grid(const Dims& d) {
  const int nq = d.nzm * d.nx;
  const int nt = d.ny / 16;
  return dim3((nq + 31) / 32, nt > 0 ? nt : 1, 3);
}

// k_ycoef_mfma grid: the column blocks plus the blocks of the z Nyquist rows
static dim3 ycoef_grid(const Dims& d, int* nqb) {
  dim3 g = ycontract_grid(d);
  *nqb = (int)g.x;
  g.x += (d.nx * d.ny + 255) / 256;
  return g;
}

hipError_t launch_synth_tab(sp_plan* p, const double2* u, int which, void* out, bool fp32) {
  const Dims& d = p->d;
  // 64 modes per block, every 16-row tile, one work-list entry per z index
  const SynthSpec<double> sp64 = synth_spec<double>(p, which);
  const dim3 grid((d.nzm * d.nx + 63) / 64, (d.ny + 15) / 16, sp64.n);
  SP_PROF_BEGIN(p, KID_SYNTH_Y);
  if (fp32) {
    const SynthSpec<float> sp = synth_spec<float>(p, which);
#define L32(KS)                                                                                  \
  hipLaunchKernelGGL((k_ysynth_mfma<float, KS>), grid, dim3(256), 0, p->stream, u, sp,          \
                     (float*)out, d.nx, d.ny, d.nzh, d.nzm)
    SP_KS_DISPATCH(d.ny, L32);
#undef L32
  } else {
    const SynthSpec<double>& sp = sp64;
#define L64(KS)                                                                                  \
  hipLaunchKernelGGL((k_ysynth_mfma<double, KS>), grid, dim3(256), 0, p->stream, u, sp,         \
                     (double*)out, d.nx, d.ny, d.nzh, d.nzm)
    SP_KS_DISPATCH(d.ny, L64);
#undef L64
  }
  SP_PROF_END(p, KID_SYNTH_Y);
  return hipGetLastError();
}

hipError_t launch_synth_y(sp_plan* p, const double2* u, bool fp32) {
  return launch_synth_tab(p, u, 0, p->yv, fp32);
}

hipError_t launch_analysis_rhs(sp_plan* p, const double2* x, double a, double2* g, bool fp32) {
  const Dims& d = p->d;
  const int nq = d.nzm * d.nx;
  int nqb;
  const dim3 grid = ycoef_grid(d, &nqb);
  SP_PROF_BEGIN(p, KID_ANALYSIS);
  if (fp32) {
    const YMat<float> m = ymat<float>(p, YM_TINV);
    const AnalysisLoad<float> ld{(const float2*)p->nv, d.ny, nq};
#define L32(KS)                                                                                \
  hipLaunchKernelGGL((k_ycoef_mfma<float, KS, AnalysisLoad<float>>), grid, dim3(256), 0,        \
                     p->stream, ld, 1, 1, 1, m, m, x, a, g, d.nx, d.ny, d.nzh, d.nzm, nqb)
    SP_KS_DISPATCH(d.ny, L32);
#undef L32
  } else {
    const YMat<double> m = ymat<double>(p, YM_TINV);
    const AnalysisLoad<double> ld{(const double2*)p->nv, d.ny, nq};
#define L64(KS)                                                                                \
  hipLaunchKernelGGL((k_ycoef_mfma<double, KS, AnalysisLoad<double>>), grid, dim3(256), 0,      \
                     p->stream, ld, 1, 1, 1, m, m, x, a, g, d.nx, d.ny, d.nzh, d.nzm, nqb)
    SP_KS_DISPATCH(d.ny, L64);
#undef L64
  }
  SP_PROF_END(p, KID_ANALYSIS);
  return hipGetLastError();
}

hipError_t launch_adj_synth(sp_plan* p, const double2* x, double a, double fa, double fb,
                            const double2* w, double2* out, bool fp32) {
  const Dims& d = p->d;
  const int nq = d.nzm * d.nx;
  const int ntile = (d.ny + 15) / 16;
  const int nthr = 64 * ntile;
  const int ncb = (nq + 7) / 8;
  const dim3 grid(ncb + (d.nx * d.ny + nthr - 1) / nthr, 1, 3);
  SP_PROF_BEGIN(p, KID_ADJ_SYNTH);
  if (fp32) {
    const AdjSynthLoad<float> ld{(const float2*)p->yv, d.nx, d.ny, nq, (float)d.alpha,
                                 (float)d.gamma};
    const YMat<float> m0 = ymat<float>(p, YM_T_T), m1 = ymat<float>(p, YM_TD_T);
#define L32(KS)                                                                                \
  hipLaunchKernelGGL((k_adjsynth_mfma<float, KS>), grid, dim3(nthr), 0, p->stream, ld, m0, m1,  \
                     x, a, fa, fb, w, out, d.nx, d.ny, d.nzh, d.nzm, ncb)
    SP_KS_DISPATCH(d.ny, L32);
#undef L32
  } else {
    const AdjSynthLoad<double> ld{(const double2*)p->yv, d.nx, d.ny, nq, d.alpha, d.gamma};
    const YMat<double> m0 = ymat<double>(p, YM_T_T), m1 = ymat<double>(p, YM_TD_T);
#define L64(KS)                                                                                \
  hipLaunchKernelGGL((k_adjsynth_mfma<double, KS>), grid, dim3(nthr), 0, p->stream, ld, m0, m1, \
                     x, a, fa, fb, w, out, d.nx, d.ny, d.nzh, d.nzm, ncb)
    SP_KS_DISPATCH(d.ny, L64);
#undef L64
  }
  SP_PROF_END(p, KID_ADJ_SYNTH);
  return hipGetLastError();
}

}  // namespace sp
