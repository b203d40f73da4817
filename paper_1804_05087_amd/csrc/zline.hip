// z-line kernels with register-resident FFTs (paper Sec. 3.2: products on the
// 3/2-padded physical grid, transforms in z).
//
// A z-line of length P = P1 * P2 is transformed in two steps with a single
// exchange through LDS (the "four-step" split of a DFT):
//   n = P2 n1 + n2, k = k1 + P1 k2:
//   X[k1 + P1 k2] = sum_n2 W_P2^(n2 k2) [ W_P^(n2 k1) sum_n1 x[P2 n1 + n2] W_P1^(n1 k1) ].
// Step 1 (one thread per n2) keeps P1 values in registers, step 2 (one thread
// per k1) keeps P2 values in registers. The inverse transform therefore ends
// with each thread holding the physical points z = k1 + P1 k2 of its lines,
// where the pointwise product is taken, and the forward transform starts from
// the same registers with the mirrored split (n = k1 + P1 k2, m = P2 m1 + m2).
//
// Lines are packed pairs of real fields (a + i b): the inverse input is the
// Hermitian extension of both spectra, and the forward output is unpacked with
// A[m] = (C[m] + conj C[P - m]) / 2, B[m] = (C[m] - conj C[P - m]) / (2i).
// Block: XL x-lines of one y-plane.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.h"
#include "sp_internal.h"

namespace sp {

// ------------------------------- pointwise stages -------------------------------
// in[i]: packed physical values of input line i at one point; out[f]: packed
// values of forward line f. bo: offset of the point in a base field.

template <typename R>
struct OpCross {  // n = u x omega; in = (u + i v, w + i ox, oy + i oz); out = (nx + i ny, nz)
  static constexpr int NI = 3, NF = 2;
  static constexpr bool kBase = false;  // reads no base state
  template <typename C>
  __device__ void operator()(const C (&in)[3], C (&out)[2], const R*, size_t, size_t) const {
    const R u = in[0].x, v = in[0].y, w = in[1].x, ox = in[1].y, oy = in[2].x, oz = in[2].y;
    out[0] = mk(v * oz - w * oy, w * ox - u * oz);
    out[1] = mk(u * oy - v * ox, (R)0);
  }
};

template <typename R>
struct OpCrossLin {  // n = du x Omega + U x domega with (U, Omega) from base
  static constexpr int NI = 3, NF = 2;
  static constexpr bool kBase = true;
  template <typename C>
  __device__ void operator()(const C (&in)[3], C (&out)[2], const R* base, size_t bs,
                             size_t bo) const {
    const R u = in[0].x, v = in[0].y, w = in[1].x, ox = in[1].y, oy = in[2].x, oz = in[2].y;
    const R U = base[bo], V = base[bs + bo], W = base[2 * bs + bo];
    const R OX = base[3 * bs + bo], OY = base[4 * bs + bo], OZ = base[5 * bs + bo];
    out[0] = mk((v * OZ - w * OY) + (V * oz - W * oy), (w * OX - u * OZ) + (W * ox - U * oz));
    out[1] = mk((u * OY - v * OX) + (U * oy - V * ox), (R)0);
  }
};

template <typename R>
struct OpStoreBase {  // cache U, Omega of the base state; no forward transform
  static constexpr int NI = 3, NF = 0;
  static constexpr bool kBase = true;
};

template <typename R>
struct OpAdjCross {  // in = (lam_x + i lam_y, lam_z); out = adjoint of the linearised product
  static constexpr int NI = 2, NF = 3;
  static constexpr bool kBase = true;
  template <typename C>
  __device__ void operator()(const C (&in)[2], C (&out)[3], const R* base, size_t bs,
                             size_t bo) const {
    const R lx = in[0].x, ly = in[0].y, lz = in[1].x;
    const R U = base[bo], V = base[bs + bo], W = base[2 * bs + bo];
    const R OX = base[3 * bs + bo], OY = base[4 * bs + bo], OZ = base[5 * bs + bo];
    out[0] = mk(OY * lz - OZ * ly, OZ * lx - OX * lz);  // (du_x, du_y)
    out[1] = mk(OX * ly - OY * lx, ly * W - lz * V);    // (du_z, dom_x)
    out[2] = mk(lz * U - lx * W, lx * V - ly * U);      // (dom_y, dom_z)
  }
};

// Field indices of the packed lines: input line i is (fin_a[i], fin_b[i]),
// forward line f is unpacked into (fout_a[f], fout_b[f]); b < 0 marks a line
// whose imaginary part is zero (input: no partner; output: no unpacking).
struct ZLineMap {
  int fin_a[3], fin_b[3];
  int fout_a[3], fout_b[3];
};

template <typename R, int P1, int P2, int XL, class Op>
__global__ void __launch_bounds__(256)
    k_zline(const typename V2<R>::T* in, typename V2<R>::T* out,  // may alias (in place)
            R* __restrict__ base, const typename V2<R>::T* __restrict__ tw, ZLineMap map, int ny,
            int px, int nzm, R scale) {
  using C = typename V2<R>::T;
  constexpr int P = P1 * P2;
  constexpr int NI = Op::NI;
  constexpr int NF = Op::NF;
  constexpr int S1 = P1 + 1;  // padded row of the exchange buffers
  // operators with a base state and no more output than input lines take the
  // pointwise stage one physical point per task, writing the products in place
  // over their input slots (the others keep one task per (line, k1), which
  // for base-state operators reads the base once per point)
  constexpr bool kSplit = Op::kBase && NF > 0 && NF <= NI;
  constexpr int LS = NI;  // line slots per x-line in the exchange block
  constexpr int E1 = (XL * LS * P2 * S1 > XL * NF * P) ? XL * LS * P2 * S1 : XL * NF * P;
  __shared__ C twl[P];
  __shared__ C ex1[E1];                          // inverse exchange, then forward output
  __shared__ C ex2[NF > 0 ? XL * NF * P2 * S1 : 1];  // forward exchange
  const int y = blockIdx.x;
  const int x0 = blockIdx.y * XL;
  const int nxl = min(XL, px - x0);
  const int tid = threadIdx.x;
  const size_t fs = (size_t)ny * px * nzm;
  const size_t lo = ((size_t)y * px + x0) * nzm;  // first line of the block in a field
  for (int t = tid; t < P; t += 256) twl[t] = tw[t];
  __syncthreads();

  // step 1 of the inverse transforms: task (xl, line i, n2)
  for (int task = tid; task < XL * NI * P2; task += 256) {
    const int n2 = task % P2;
    const int li = task / P2;  // xl * NI + i
    const int i = li % NI;
    const int xl = li / NI;
    if (xl < nxl) {
      const C* fa = in + (size_t)map.fin_a[i] * fs + lo + (size_t)xl * nzm;
      const int fb = map.fin_b[i];
      const C* fbp = in + (size_t)(fb < 0 ? map.fin_a[i] : fb) * fs + lo + (size_t)xl * nzm;
      const R bk = (fb < 0) ? (R)0 : (R)1;
      C v[P1];
#pragma unroll
      for (int n1 = 0; n1 < P1; ++n1) {
        const int m = P2 * n1 + n2;
        // Hermitian extension: m < nzm direct, m > P - nzm mirrored, else zero;
        // masks multiply loaded values so the loads stay unconditional
        const bool lo_half = m < nzm;
        const bool hi_half = m > P - nzm;
        const int mm = lo_half ? m : (hi_half ? P - m : 0);
        const C a = fa[mm];
        const C b = fbp[mm];
        const R keep = (lo_half || hi_half) ? (R)1 : (R)0;
        const R cj = (m == 0) ? (R)0 : (lo_half ? (R)1 : (R)-1);  // sign of the imaginary part
        const R ar = a.x * keep, ai = a.y * cj * keep;
        const R br = b.x * keep * bk, bi = b.y * cj * keep * bk;
        v[n1] = mk(ar - bi, ai + br);
      }
      dft_reg<P1, P, C, R>(v, (R)1, twl);
      C* e = ex1 + ((xl * LS + i) * P2 + n2) * S1;
#pragma unroll
      for (int k1 = 0; k1 < P1; ++k1)
        e[k1] = (k1 == 0 || n2 == 0) ? v[k1] : cmul(v[k1], wpow<P, P, C, R>(n2 * k1, (R)1, twl));
    }
  }
  __syncthreads();

  // step 2 of the inverse transforms, in place: task (xl, line i, k1); column
  // k1 of the exchange block then holds the physical points z = k1 + P1 k2
  const size_t bs = (size_t)ny * px * P;
  for (int task = tid; task < XL * NI * P1; task += 256) {
    const int k1 = task % P1;
    const int li = task / P1;  // xl * NI + i
    const int xl = li / NI;
    const int il = li - xl * NI;
    if (xl < nxl) {
      C* e = ex1 + ((xl * LS + il) * P2) * S1 + k1;
      C ph[P2];
#pragma unroll
      for (int n2 = 0; n2 < P2; ++n2) ph[n2] = e[n2 * S1];
      dft_reg<P2, P, C, R>(ph, (R)1, twl);
      if constexpr (NF == 0) {  // the base state: packed line i holds fields 2i, 2i + 1
        const int i = li % NI;
        const size_t bo0 = ((size_t)y * px + x0 + xl) * P + k1;
#pragma unroll
        for (int k2 = 0; k2 < P2; ++k2) {
          const size_t bo = bo0 + (size_t)P1 * k2;
          base[(size_t)(2 * i) * bs + bo] = ph[k2].x;
          base[(size_t)(2 * i + 1) * bs + bo] = ph[k2].y;
        }
      } else {
#pragma unroll
        for (int k2 = 0; k2 < P2; ++k2) e[k2 * S1] = ph[k2];
      }
    }
  }
  if constexpr (kSplit) {
    __syncthreads();
    // the pointwise stage, split: task (xl, k1, k2), one
    // physical point z = k1 + P1 k2 each, so that every wave reads base values
    // (consecutive tasks read consecutive z); the products go in place over the
    // point's input slots (slot f < NF of the x-line's LS slots)
    for (int task = tid; task < XL * P1 * P2; task += 256) {
      const int k1 = task % P1;
      const int k2 = (task / P1) % P2;
      const int xl = task / (P1 * P2);
      if (xl < nxl) {
        C pin[NI], pout[NF];
#pragma unroll
        for (int i = 0; i < NI; ++i) pin[i] = ex1[((xl * LS + i) * P2 + k2) * S1 + k1];
        const Op op{};
        op(pin, pout, base, bs, ((size_t)y * px + x0 + xl) * P + k1 + (size_t)P1 * k2);
#pragma unroll
        for (int f = 0; f < NF; ++f) ex1[((xl * LS + f) * P2 + k2) * S1 + k1] = pout[f];
      }
    }
    __syncthreads();
    // step 1 of the forward transforms: task (xl, k1, forward line f), f slowest
    for (int task = tid; task < XL * P1 * NF; task += 256) {
      const int f = task / (XL * P1);
      const int k1 = task % P1;
      const int xl = (task / P1) % XL;
      if (xl < nxl) {
        C fw[P2];
#pragma unroll
        for (int k2 = 0; k2 < P2; ++k2) fw[k2] = ex1[((xl * LS + f) * P2 + k2) * S1 + k1];
        dft_reg<P2, P, C, R>(fw, (R)-1, twl);
        C* e = ex2 + ((xl * NF + f) * P2) * S1 + k1;
#pragma unroll
        for (int m2 = 0; m2 < P2; ++m2)
          e[m2 * S1] = (m2 == 0 || k1 == 0) ? fw[m2]
                                            : cmul(fw[m2], wpow<P, P, C, R>(k1 * m2, (R)-1, twl));
      }
    }
  }
  if constexpr (NF > 0 && !kSplit) {
    __syncthreads();
    // the pointwise stage and step 1 of the forward transforms: task (xl, k1,
    // forward line f) for operators that read no base state, f slowest (with
    // XL * P1 a multiple of 64 it is uniform over a wave), else (xl, k1) with
    // every f in one task, so the base state is read once per point
    constexpr int NFT = Op::kBase ? 1 : NF;  // forward lines per task split
    for (int task = tid; task < XL * P1 * NFT; task += 256) {
      const int fsel = task / (XL * P1);
      const int k1 = task % P1;
      const int xl = (task / P1) % XL;
      if (xl < nxl) {
        const size_t bo0 = ((size_t)y * px + x0 + xl) * P + k1;
        // forward lines F0 .. F0 + NFL - 1 (compile-time, so pout stays in registers)
        auto run = [&](auto f0) {
          constexpr int F0 = decltype(f0)::value;
          constexpr int NFL = Op::kBase ? NF : 1;
          C fw[NFL][P2];
          const Op op{};
#pragma unroll
          for (int k2 = 0; k2 < P2; ++k2) {
            C pin[NI], pout[NF];
#pragma unroll
            for (int i = 0; i < NI; ++i) pin[i] = ex1[((xl * NI + i) * P2 + k2) * S1 + k1];
            op(pin, pout, base, bs, bo0 + (size_t)P1 * k2);
#pragma unroll
            for (int q = 0; q < NFL; ++q) fw[q][k2] = pout[F0 + q];
          }
#pragma unroll
          for (int q = 0; q < NFL; ++q) {
            dft_reg<P2, P, C, R>(fw[q], (R)-1, twl);
            C* e = ex2 + ((xl * NF + F0 + q) * P2) * S1 + k1;
#pragma unroll
            for (int m2 = 0; m2 < P2; ++m2)
              e[m2 * S1] = (m2 == 0 || k1 == 0)
                               ? fw[q][m2]
                               : cmul(fw[q][m2], wpow<P, P, C, R>(k1 * m2, (R)-1, twl));
          }
        };
        if constexpr (Op::kBase) {
          run(std::integral_constant<int, 0>{});
        } else {
          if (fsel == 0) run(std::integral_constant<int, 0>{});
          if constexpr (NF > 1) {
            if (fsel == 1) run(std::integral_constant<int, 1>{});
          }
          if constexpr (NF > 2) {
            if (fsel == 2) run(std::integral_constant<int, 2>{});
          }
        }
      }
    }
  }
  if constexpr (NF > 0) {
    __syncthreads();
    // step 2 of the forward transforms: task (xl, line f, m2), outputs m = P2 m1 + m2
    for (int task = tid; task < XL * NF * P2; task += 256) {
      const int m2 = task % P2;
      const int lf = task / P2;
      const int xl = lf / NF;
      if (xl < nxl) {
        const C* e = ex2 + (lf * P2 + m2) * S1;
        C v[P1];
#pragma unroll
        for (int n1 = 0; n1 < P1; ++n1) v[n1] = e[n1];
        dft_reg<P1, P, C, R>(v, (R)-1, twl);
        C* o = ex1 + lf * P;
#pragma unroll
        for (int m1 = 0; m1 < P1; ++m1) o[P2 * m1 + m2] = v[m1];
      }
    }
    __syncthreads();
    // unpack, scale and store the kept modes m < nzm: task (xl, line f, m)
    for (int task = tid; task < XL * NF * nzm; task += 256) {
      const int m = task % nzm;
      const int lf = task / nzm;
      const int f = lf % NF;
      const int xl = lf / NF;
      if (xl < nxl) {
        const C* o = ex1 + lf * P;
        const C a = o[m];
        const size_t off = lo + (size_t)xl * nzm + m;
        if (map.fout_b[f] < 0) {
          out[(size_t)map.fout_a[f] * fs + off] = cscale(a, scale);
        } else {
          const C am = conjc(o[(P - m) % P]);
          const C s1 = cscale(cadd(a, am), (R)0.5 * scale);
          const C d = csub(a, am);
          out[(size_t)map.fout_a[f] * fs + off] = s1;
          out[(size_t)map.fout_b[f] * fs + off] = mk(d.y * (R)0.5 * scale, -d.x * (R)0.5 * scale);
        }
      }
    }
  }
}

// ----------------------------------- launchers -----------------------------------

hipError_t launch_z_product_lds(sp_plan* p, int mode, bool fp32);
hipError_t launch_adj_z_lds(sp_plan* p, bool fp32);

constexpr int kZXL = 8;

template <typename R, class Op>
static void zline_launch(sp_plan* p, const void* in, void* out, R* base, const void* tw,
                         const ZLineMap& map, double scale) {
  const Dims& d = p->d;
  using C = typename V2<R>::T;
  dim3 grid(d.ny, (d.px + kZXL - 1) / kZXL);
  const C* ci = (const C*)in;
  C* co = (C*)out;
  const C* ct = (const C*)tw;
#define ZL(A, B)                                                                              \
  hipLaunchKernelGGL((k_zline<R, A, B, kZXL, Op>), grid, dim3(256), 0, p->stream, ci, co, base, \
                     ct, map, d.ny, d.px, d.nzm, (R)scale)
  SP_REG_FFT_DISPATCH(d.pz, ZL)
#undef ZL
}

hipError_t launch_z_product(sp_plan* p, int mode, bool fp32) {
  const Dims& d = p->d;
  if (reg_fft_split(d.pz) == 0) return launch_z_product_lds(p, mode, fp32);
  const double scale = 1.0 / ((double)d.px * d.pz);
  const ZLineMap map{{0, 2, 4}, {1, 3, 5}, {0, 2, -1}, {1, -1, -1}};
  SP_PROF_BEGIN(p, KID_Z_PRODUCT);
  if (fp32) {
    if (mode == 0)
      zline_launch<float, OpCross<float>>(p, p->xp, p->np, p->base32, p->f_twz, map, scale);
    else if (mode == 1)
      zline_launch<float, OpCrossLin<float>>(p, p->xp, p->np, p->base32, p->f_twz, map, scale);
    else
      zline_launch<float, OpStoreBase<float>>(p, p->xp, p->np, p->base32, p->f_twz, map, scale);
  } else {
    if (mode == 0)
      zline_launch<double, OpCross<double>>(p, p->xp, p->np, p->base, p->d_twz, map, scale);
    else if (mode == 1)
      zline_launch<double, OpCrossLin<double>>(p, p->xp, p->np, p->base, p->d_twz, map, scale);
    else
      zline_launch<double, OpStoreBase<double>>(p, p->xp, p->np, p->base, p->d_twz, map, scale);
  }
  SP_PROF_END(p, KID_Z_PRODUCT);
  return hipGetLastError();
}

hipError_t launch_adj_z(sp_plan* p, bool fp32) {
  const Dims& d = p->d;
  if (reg_fft_split(d.pz) == 0) return launch_adj_z_lds(p, fp32);
  const double scale = 1.0 / ((double)d.px * d.pz);
  const ZLineMap map{{0, 2, -1}, {1, -1, -1}, {0, 2, 4}, {1, 3, 5}};
  SP_PROF_BEGIN(p, KID_ADJ_Z);
  if (fp32)
    zline_launch<float, OpAdjCross<float>>(p, p->xp, p->xp, p->base32, p->f_twz, map, scale);
  else
    zline_launch<double, OpAdjCross<double>>(p, p->xp, p->xp, p->base, p->d_twz, map, scale);
  SP_PROF_END(p, KID_ADJ_Z);
  return hipGetLastError();
}

}  // namespace sp
