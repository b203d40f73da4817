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
//
// With XF the kernel also takes the inverse x transforms (3/2 padding in x)
// that feed its lines, from the y-valued spectral fields [f][y][kz][mx]: the
// block's lines are x = a + Q j (j < XL, Q = px / XL), for which
//   X(a + Q j) = sum_r W_XL^(-r j) g_r,  g_r = sum_{m = r mod XL} c_m exp(2 pi i m a / px),
// so each block forms XL partial sums per (field, kz) and one XL-point DFT,
// and the x-physical fields never leave the block.
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
  static constexpr int kXIn = 5;        // XF: y-valued fields in (curl-combined to six)
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
  static constexpr int kXIn = 5;
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
  static constexpr int kXIn = 5;
  static constexpr bool kBase = true;
};

template <typename R>
struct OpAdjCross {  // in = (lam_x + i lam_y, lam_z); out = adjoint of the linearised product
  static constexpr int NI = 2, NF = 3;
  static constexpr int kXIn = 3;  // XF: the three fields as they are
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

// XF: in = y-valued fields [f][y][kz][mx]: for Op::kXIn == 5 the five fields
// (u, du/dy, v, w, dw/dy), from which the six curl-combined fields of the
// x-lines are formed (the line map pairs fields (0, 1), (2, 3), (4, 5)); for
// kXIn == 3 three fields taken as they are (pairs (0, 1), (2)). Requires
// nx % 16 == 0 (so px % XL == 0), nzm == P / 3 and a 1-D grid of
// ny * (px / XL) blocks; in and out do not alias.
// Otherwise in = the x-physical fields [f][y][x][kz] (out may alias it) and
// the grid is (ny, ceil(px / XL)).
template <typename R, int P1, int P2, int XL, class Op, bool XF = false>
__global__ void __launch_bounds__(256)
    k_zline(const typename V2<R>::T* in, typename V2<R>::T* out,
            R* __restrict__ base, const typename V2<R>::T* __restrict__ tw, ZLineMap map, int ny,
            int px, int nzm, R scale, const typename V2<R>::T* __restrict__ twx = nullptr,
            int nx = 0, R alpha = 0, R gamma = 0) {
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
  constexpr int NXF = Op::kXIn == 5 ? 6 : Op::kXIn;  // x-physical fields formed by XF
  constexpr int E2F = NF > 0 ? XL * NF * P2 * S1 : 1;
  constexpr int E2X = XF ? XL * NXF * (P / 3) : 1;
  static_assert(!XF || (XL == 8 && 2 * NI >= NXF && E1 >= NXF * (P / 3) * (XL + 1)),
                "XF: eight lines of packed pairs; partial sums fit the exchange block");
  __shared__ C twl[P];
  __shared__ C ex1[E1];  // inverse exchange, then forward output (XF: first the partial sums)
  __shared__ C ex2[E2F > E2X ? E2F : E2X];  // forward exchange (XF: first the x-physical lines)
  const int tid = threadIdx.x;
  int y, x0, xq, nxl;  // line xl of the block is x = x0 + xq * xl
  if constexpr (XF) {
    const int nq = px / XL;
    const int l = xcd_order(blockIdx.x, gridDim.x);  // the blocks of one y-plane share an L2
    y = l / nq;
    x0 = l - y * nq;
    xq = nq;
    nxl = XL;
  } else {
    y = blockIdx.x;
    x0 = blockIdx.y * XL;
    xq = 1;
    nxl = min(XL, px - x0);
  }
  // kept z modes per line: P / 3 for XF (checked by the launcher), so that the
  // Hermitian extension's masks fold at compile time where they are uniform
  const int nzk = XF ? P / 3 : nzm;
  const size_t fs = (size_t)ny * px * nzk;
  // offset of line xl in a field of the x-physical layout (in units of nzm)
  auto line_of = [&](int xl) { return (size_t)y * px + x0 + (size_t)xq * xl; };
  for (int t = tid; t < P; t += 256) twl[t] = tw[t];
  if constexpr (XF) {
    // Partial sums g_r of the NXF x-line fields: task (kz, r), over the kept
    // padded positions m = r mod XL. With nx a multiple of 16 these are, for
    // t < nx/16, m = r + XL t (mode i = m) in the low half and m = nx + r + XL t
    // (mode i = m - nx/2) in the high half, except the empty position m = nx;
    // taken in pairs with unconditional loads (the empty one loads mode nx/2
    // and is weighted 0) so that each pair's loads are in flight together.
    // The curl combination is linear, so the sums run over the input fields
    // (A_k = sum w s_k) and, for the two curl terms with a factor i k_x, over
    // k_x w s_k (B_2, B_3); the six fields are formed from them once.
    C* gl = ex1;  // [NXF][nzm][XL + 1]
    const size_t fsy = (size_t)ny * nzk * nx;
    const int h = nx / 2;
    const int h8 = nx / (2 * XL);
    const int dq = (XL * x0) % px;  // step of the twiddle index m a mod px per t
    for (int task = tid; task < nzk * XL; task += 256) {
      const int r = task % XL;
      const int kz = task / XL;
      const C* src = in + ((size_t)y * nzk + kz) * nx;
      constexpr int NA = Op::kXIn;
      C A[NA], B2 = mk((R)0, (R)0), B3 = mk((R)0, (R)0);
#pragma unroll
      for (int k = 0; k < NA; ++k) A[k] = mk((R)0, (R)0);
      int q[2] = {(r * x0) % px, ((nx + r) * x0) % px};
      for (int t = 0; t < h8; ++t) {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          const int pos = (half ? nx : 0) + r + XL * t;
          const int i = half ? pos - h : pos;
          C sk[NA];
#pragma unroll
          for (int k = 0; k < NA; ++k) sk[k] = src[k * fsy + i];
          // exp(2 pi i m a / px), zero at the empty position
          const R keep = (half && pos == nx) ? (R)0 : (R)1;
          const C w = cscale(conjc(twx[q[half]]), keep);
#pragma unroll
          for (int k = 0; k < NA; ++k) A[k] = cadd(A[k], cmul(sk[k], w));
          if constexpr (NA == 5) {
            const R kxv = alpha * (R)(half ? i - nx : i);
            const C wk = cscale(w, kxv);
            B2 = cadd(B2, cmul(sk[2], wk));
            B3 = cadd(B3, cmul(sk[3], wk));
          }
          q[half] += dq;
          q[half] -= (q[half] >= px) ? px : 0;
        }
      }
      C g[NXF];
      if constexpr (NA == 5) {
        const R kzv = gamma * (R)kz;
        g[0] = A[0];                                             // u
        g[1] = A[2];                                             // v
        g[2] = A[3];                                             // w
        g[3] = csub(A[4], sidot(cscale(A[2], kzv), (R)1));       // dw/dy - i kz v
        g[4] = sidot(csub(cscale(A[0], kzv), B3), (R)1);         // i kz u - i kx w
        g[5] = csub(sidot(B2, (R)1), A[1]);                      // i kx v - du/dy
      } else {
#pragma unroll
        for (int f = 0; f < NXF; ++f) g[f] = A[f];
      }
#pragma unroll
      for (int f = 0; f < NXF; ++f) gl[(f * nzk + kz) * (XL + 1) + r] = g[f];
    }
    __syncthreads();
    // XL-point inverse DFT over r: task (field, kz) -> the block's XL lines
    C* xs = ex2;  // [XL][NXF][nzm]
    for (int task = tid; task < NXF * nzk; task += 256) {
      const int kz = task % nzk;
      const int f = task / nzk;
      C v[XL];
#pragma unroll
      for (int r = 0; r < XL; ++r) v[r] = gl[(f * nzk + kz) * (XL + 1) + r];
      dft_reg<XL, P, C, R>(v, (R)1, twl);
#pragma unroll
      for (int j = 0; j < XL; ++j) xs[(j * NXF + f) * nzk + kz] = v[j];
    }
  }
  __syncthreads();

  // step 1 of the inverse transforms: task (xl, line i, n2)
  for (int task = tid; task < XL * NI * P2; task += 256) {
    const int n2 = task % P2;
    const int li = task / P2;  // xl * NI + i
    const int i = li % NI;
    const int xl = li / NI;
    if (xl < nxl) {
      const int fb = map.fin_b[i];
      const int fbi = fb < 0 ? map.fin_a[i] : fb;
      const C* fa;
      const C* fbp;
      if constexpr (XF) {
        fa = ex2 + (xl * NXF + map.fin_a[i]) * nzk;
        fbp = ex2 + (xl * NXF + fbi) * nzk;
      } else {
        fa = in + (size_t)map.fin_a[i] * fs + line_of(xl) * nzk;
        fbp = in + (size_t)fbi * fs + line_of(xl) * nzk;
      }
      const R bk = (fb < 0) ? (R)0 : (R)1;
      C v[P1];
#pragma unroll
      for (int n1 = 0; n1 < P1; ++n1) {
        const int m = P2 * n1 + n2;
        // Hermitian extension: m < nzm direct, m > P - nzm mirrored, else zero;
        // masks multiply loaded values so the loads stay unconditional
        const bool lo_half = m < nzk;
        const bool hi_half = m > P - nzk;
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
        const size_t bo0 = line_of(xl) * P + k1;
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
        op(pin, pout, base, bs, line_of(xl) * P + k1 + (size_t)P1 * k2);
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
        const size_t bo0 = line_of(xl) * P + k1;
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
    for (int task = tid; task < XL * NF * nzk; task += 256) {
      const int m = task % nzk;
      const int lf = task / nzk;
      const int f = lf % NF;
      const int xl = lf / NF;
      if (xl < nxl) {
        const C* o = ex1 + lf * P;
        const C a = o[m];
        const size_t off = line_of(xl) * nzk + m;
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

template <typename R, class Op, bool XF = false>
static void zline_launch(sp_plan* p, const void* in, void* out, R* base, const void* tw,
                         const ZLineMap& map, double scale, const void* twx = nullptr) {
  const Dims& d = p->d;
  using C = typename V2<R>::T;
  const dim3 grid = XF ? dim3(d.ny * (d.px / kZXL)) : dim3(d.ny, (d.px + kZXL - 1) / kZXL);
  const C* ci = (const C*)in;
  C* co = (C*)out;
  const C* ct = (const C*)tw;
  const C* cx = (const C*)twx;
#define ZL(A, B)                                                                              \
  hipLaunchKernelGGL((k_zline<R, A, B, kZXL, Op, XF>), grid, dim3(256), 0, p->stream, ci, co,  \
                     base, ct, map, d.ny, d.px, d.nzm, (R)scale, cx, d.nx, (R)d.alpha,        \
                     (R)d.gamma)
  SP_REG_FFT_DISPATCH(d.pz, ZL)
#undef ZL
}

// Every block of the fused kernel reads its whole y-plane of the y-valued
// fields, so one plane is read px / kZXL times. Measured on MI355X, forward
// (five fields): fused is faster while those reads stay within one XCD's
// 4 MiB L2 (48x65x48 in FP64 and FP32: 0.8 and 0.4 MiB per plane; 96x97x96
// in FP32: 3.2 MiB) and slower beyond (96x97x96 in FP64: 6.3 MiB per plane,
// 146 us against 57 + 61 us for the two kernels). The adjoint kernel (three
// fields) holds two waves per SIMD instead of three and hides less of that
// latency: fused it was 6-10 % faster at 48x65x48 (0.5 and 0.2 MiB) and 1-2 %
// slower at 96x97x96 (3.8 and 1.9 MiB), so its bound is 1 MiB.
bool zline_fuses_x_inverse(const sp_plan* p, bool fp32, int nfields) {
  const Dims& d = p->d;
  if (reg_fft_split(d.pz) == 0 || d.nx % (2 * kZXL) != 0 || 3 * d.nzm != d.pz) return false;
  const size_t plane =
      (size_t)nfields * d.nzm * d.nx * (fp32 ? sizeof(float2) : sizeof(double2));
  const size_t bound = (nfields == 5 ? (size_t)4 : (size_t)1) << 20;
  return (size_t)(d.px / kZXL) * plane <= bound;
}

hipError_t launch_z_product(sp_plan* p, int mode, bool fp32) {
  const Dims& d = p->d;
  if (reg_fft_split(d.pz) == 0) return launch_z_product_lds(p, mode, fp32);
  const double scale = 1.0 / ((double)d.px * d.pz);
  const ZLineMap map{{0, 2, 4}, {1, 3, 5}, {0, 2, -1}, {1, -1, -1}};
  SP_PROF_BEGIN(p, KID_Z_PRODUCT);
  // fused: the y-valued fields in, the inverse x transforms taken in the kernel
  auto run = [&](auto xf) {
    constexpr bool XF = decltype(xf)::value;
    const void* in = XF ? p->yv : p->xp;
    if (fp32) {
      if (mode == 0)
        zline_launch<float, OpCross<float>, XF>(p, in, p->np, p->base32, p->f_twz, map, scale,
                                                p->f_twx);
      else if (mode == 1)
        zline_launch<float, OpCrossLin<float>, XF>(p, in, p->np, p->base32, p->f_twz, map,
                                                   scale, p->f_twx);
      else
        zline_launch<float, OpStoreBase<float>, XF>(p, in, p->np, p->base32, p->f_twz, map,
                                                    scale, p->f_twx);
    } else {
      if (mode == 0)
        zline_launch<double, OpCross<double>, XF>(p, in, p->np, p->base, p->d_twz, map, scale,
                                                  p->d_twx);
      else if (mode == 1)
        zline_launch<double, OpCrossLin<double>, XF>(p, in, p->np, p->base, p->d_twz, map,
                                                     scale, p->d_twx);
      else
        zline_launch<double, OpStoreBase<double>, XF>(p, in, p->np, p->base, p->d_twz, map,
                                                      scale, p->d_twx);
    }
  };
  if (zline_fuses_x_inverse(p, fp32, 5))
    run(std::true_type{});
  else
    run(std::false_type{});
  SP_PROF_END(p, KID_Z_PRODUCT);
  return hipGetLastError();
}

hipError_t launch_adj_z(sp_plan* p, bool fp32) {
  const Dims& d = p->d;
  if (reg_fft_split(d.pz) == 0) return launch_adj_z_lds(p, fp32);
  const double scale = 1.0 / ((double)d.px * d.pz);
  const ZLineMap map{{0, 2, -1}, {1, -1, -1}, {0, 2, 4}, {1, 3, 5}};
  SP_PROF_BEGIN(p, KID_ADJ_Z);
  // fused: the three y-valued fields in p->nv, the inverse x transforms taken
  // in the kernel; else the x-physical fields in p->xp, transformed in place
  auto run = [&](auto xf) {
    constexpr bool XF = decltype(xf)::value;
    const void* in = XF ? p->nv : p->xp;
    if (fp32)
      zline_launch<float, OpAdjCross<float>, XF>(p, in, p->xp, p->base32, p->f_twz, map, scale,
                                                 p->f_twx);
    else
      zline_launch<double, OpAdjCross<double>, XF>(p, in, p->xp, p->base, p->d_twz, map, scale,
                                                   p->d_twx);
  };
  if (zline_fuses_x_inverse(p, fp32, 3))
    run(std::true_type{});
  else
    run(std::false_type{});
  SP_PROF_END(p, KID_ADJ_Z);
  return hipGetLastError();
}

}  // namespace sp
