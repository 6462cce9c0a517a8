// Stockham auto-sort FFT staged in LDS, radices 2, 3, 4, 5, 6, 8, 9 and 10, for gfx950.
//
// A workgroup transforms C interleaved sequences of length n held in LDS as
// buf[m*C + c] (m in [0, n), c in [0, C)).  Each Stockham pass of radix R with stride Ns
// (the product of the radices already applied) reads, for butterfly j,
//     v[r] = buf[(j + r*n/R)*C + c],  r = 0..R-1,
// multiplies v[r] by W_{Ns*R}^{r*(j mod Ns)}, applies the length-R DFT and writes
//     buf[((j - j mod Ns)*R + j mod Ns + r*Ns)*C + c] = v[r].
// After the last pass the output is in natural order.  Every thread keeps its
// butterflies in registers between the read and the write half of a pass, so one LDS
// buffer suffices (two barriers per pass).  E bounds the values one thread holds.
// Forward transforms use W = exp(-2 pi i/R); the inverse (INV = true) uses the
// conjugate and is unnormalised.
#pragma once

#include "common.hpp"

namespace wct {

template <typename T>
struct FftConst;
template <>
struct FftConst<float> {
  static constexpr float s3 = 0.86602540378443864676f;   // sin(2 pi / 3)
  static constexpr float c51 = 0.30901699437494742410f;  // cos(2 pi / 5)
  static constexpr float c52 = -0.80901699437494742410f; // cos(4 pi / 5)
  static constexpr float s51 = 0.95105651629515357212f;  // sin(2 pi / 5)
  static constexpr float s52 = 0.58778525229247312917f;  // sin(4 pi / 5)
  static constexpr float r2 = 0.70710678118654752440f;   // 1 / sqrt(2)
};
template <>
struct FftConst<double> {
  static constexpr double s3 = 0.86602540378443864676;
  static constexpr double c51 = 0.30901699437494742410;
  static constexpr double c52 = -0.80901699437494742410;
  static constexpr double s51 = 0.95105651629515357212;
  static constexpr double s52 = 0.58778525229247312917;
  static constexpr double r2 = 0.70710678118654752440;
};

// -i*a for the forward sign, +i*a for the inverse.
template <typename T, bool INV>
__host__ __device__ __forceinline__ cx<T> rot(cx<T> a) {
  return INV ? mk(-a.y, a.x) : mk(a.y, -a.x);
}

template <typename T, bool INV>
__host__ __device__ __forceinline__ void dft2(cx<T>* v) {
  cx<T> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <typename T, bool INV>
__host__ __device__ __forceinline__ void dft3(cx<T>* v) {
  cx<T> t = v[1] + v[2];
  cx<T> m = v[0] - scale(t, T(0.5));
  cx<T> d = scale(rot<T, INV>(v[1] - v[2]), FftConst<T>::s3);
  v[0] = v[0] + t;
  v[1] = m + d;
  v[2] = m - d;
}

template <typename T, bool INV>
__host__ __device__ __forceinline__ void dft4(cx<T>* v) {
  cx<T> t0 = v[0] + v[2], t1 = v[0] - v[2];
  cx<T> t2 = v[1] + v[3], t3 = rot<T, INV>(v[1] - v[3]);
  v[0] = t0 + t2;
  v[2] = t0 - t2;
  v[1] = t1 + t3;
  v[3] = t1 - t3;
}

template <typename T, bool INV>
__host__ __device__ __forceinline__ void dft5(cx<T>* v) {
  using K = FftConst<T>;
  cx<T> t1 = v[1] + v[4], t2 = v[2] + v[3];
  cx<T> t3 = v[1] - v[4], t4 = v[2] - v[3];
  cx<T> p1 = v[0] + scale(t1, K::c51) + scale(t2, K::c52);
  cx<T> p2 = v[0] + scale(t1, K::c52) + scale(t2, K::c51);
  cx<T> q1 = rot<T, INV>(scale(t3, K::s51) + scale(t4, K::s52));
  cx<T> q2 = rot<T, INV>(scale(t3, K::s52) - scale(t4, K::s51));
  v[0] = v[0] + t1 + t2;
  v[1] = p1 + q1;
  v[4] = p1 - q1;
  v[2] = p2 + q2;
  v[3] = p2 - q2;
}

template <typename T, bool INV>
__host__ __device__ __forceinline__ void dft8(cx<T>* v) {
  using K = FftConst<T>;
  cx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<T, INV>(e);
  dft4<T, INV>(o);
  // twiddles W8^k (forward) or W8^-k (inverse) on o[1..3]
  cx<T> o1, o3;
  if (!INV) {
    o1 = mk((o[1].x + o[1].y) * K::r2, (o[1].y - o[1].x) * K::r2);
    o3 = mk((o[3].y - o[3].x) * K::r2, -(o[3].x + o[3].y) * K::r2);
  } else {
    o1 = mk((o[1].x - o[1].y) * K::r2, (o[1].x + o[1].y) * K::r2);
    o3 = mk(-(o[3].x + o[3].y) * K::r2, (o[3].x - o[3].y) * K::r2);
  }
  cx<T> o2 = rot<T, INV>(o[2]);
  v[0] = e[0] + o[0];
  v[4] = e[0] - o[0];
  v[1] = e[1] + o1;
  v[5] = e[1] - o1;
  v[2] = e[2] + o2;
  v[6] = e[2] - o2;
  v[3] = e[3] + o3;
  v[7] = e[3] - o3;
}

// exp(-2 pi i m / N) for the composite codelets (N = 6, 9, 10), 22-digit literals.
template <int N>
struct WTab;
template <>
struct WTab<6> {
  static constexpr double re[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
  static constexpr double im[6] = {0.0, -8.660254037844386467637e-1, -8.660254037844386467637e-1, 0.0,
                                   8.660254037844386467637e-1, 8.660254037844386467637e-1};
};
template <>
struct WTab<9> {
  static constexpr double re[9] = {1.0, 7.660444431189780352024e-1, 1.736481776669303488517e-1, -0.5,
                                   -9.396926207859083840541e-1, -9.396926207859083840541e-1, -0.5,
                                   1.736481776669303488517e-1, 7.660444431189780352024e-1};
  static constexpr double im[9] = {0.0, -6.427876096865393263226e-1, -9.848077530122080593667e-1,
                                   -8.660254037844386467637e-1, -3.420201433256687330441e-1,
                                   3.420201433256687330441e-1, 8.660254037844386467637e-1,
                                   9.848077530122080593667e-1, 6.427876096865393263226e-1};
};
template <>
struct WTab<10> {
  static constexpr double re[10] = {1.0, 8.090169943749474241023e-1, 3.090169943749474241023e-1,
                                    -3.090169943749474241023e-1, -8.090169943749474241023e-1, -1.0,
                                    -8.090169943749474241023e-1, -3.090169943749474241023e-1,
                                    3.090169943749474241023e-1, 8.090169943749474241023e-1};
  static constexpr double im[10] = {0.0, -5.877852522924731291687e-1, -9.510565162951535721164e-1,
                                    -9.510565162951535721164e-1, -5.877852522924731291687e-1, 0.0,
                                    5.877852522924731291687e-1, 9.510565162951535721164e-1,
                                    9.510565162951535721164e-1, 5.877852522924731291687e-1};
};
// a * W_N^m (forward) or a * W_N^-m (inverse) for a compile-time m after unrolling.
template <typename T, bool INV, int N>
__host__ __device__ __forceinline__ cx<T> wmul(cx<T> a, int m) {
  m %= N;
  if (m == 0) return a;
  if (4 * m == N) return rot<T, INV>(a);
  if (2 * m == N) return mk(-a.x, -a.y);
  if (4 * m == 3 * N) return rot<T, !INV>(a);
  const T c = (T)WTab<N>::re[m];
  const T s = INV ? -(T)WTab<N>::im[m] : (T)WTab<N>::im[m];
  return mk(a.x * c - a.y * s, a.x * s + a.y * c);
}

template <int R, typename T, bool INV>
__host__ __device__ __forceinline__ void dftR(cx<T>* v);

// Length R1*R2 DFT: R2 DFTs of length R1 on x[R2 n1 + n2], twiddles W_N^{n2 k1},
// R1 DFTs of length R2, output X[k1 + R1 k2].
template <typename T, bool INV, int R1, int R2>
__host__ __device__ __forceinline__ void dft_comp(cx<T>* v) {
  constexpr int N = R1 * R2;
  cx<T> y[R2][R1];
#pragma unroll
  for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) y[n2][n1] = v[R2 * n1 + n2];
    dftR<R1, T, INV>(y[n2]);
#pragma unroll
    for (int k1 = 1; k1 < R1; ++k1)
      if (n2 > 0) y[n2][k1] = wmul<T, INV, N>(y[n2][k1], n2 * k1);
  }
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    cx<T> t[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) t[n2] = y[n2][k1];
    dftR<R2, T, INV>(t);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = t[k2];
  }
}

template <int R, typename T, bool INV>
__host__ __device__ __forceinline__ void dftR(cx<T>* v) {
  if constexpr (R == 2) dft2<T, INV>(v);
  else if constexpr (R == 3) dft3<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v);
  else if constexpr (R == 5) dft5<T, INV>(v);
  else if constexpr (R == 6) dft_comp<T, INV, 3, 2>(v);
  else if constexpr (R == 8) dft8<T, INV>(v);
  else if constexpr (R == 9) dft_comp<T, INV, 3, 3>(v);
  else dft_comp<T, INV, 5, 2>(v);  // 10
}

// Butterfly idx of a Stockham pass (radix R, stride Ns) over C interleaved sequences:
// the load half and the twiddle + DFT + store half.  Shared by the device pass and the
// host check of the transforms.
template <int R, typename T, int C>
__host__ __device__ __forceinline__ void bf_load(const cx<T>* buf, int idx, int nr, cx<T>* v) {
  const int c = idx % C, j = idx / C;
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = buf[(j + r * nr) * C + c];
}
template <int R, typename T, bool INV, int C>
__host__ __device__ __forceinline__ void bf_store(cx<T>* buf, int idx, int Ns, const cx<T>* __restrict__ tw,
                                                  cx<T>* v) {
  const int c = idx % C, j = idx / C;
  const int k = j % Ns;
  if (Ns > 1) {
    const cx<T>* w = tw + k * (R - 1);
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = INV ? cmulc(v[r], w[r - 1]) : cmul(v[r], w[r - 1]);
  }
  dftR<R, T, INV>(v);
  const int base = (j - k) * R + k;
#pragma unroll
  for (int r = 0; r < R; ++r) buf[(base + r * Ns) * C + c] = v[r];
}

// One Stockham pass over C interleaved sequences of length n in LDS.
template <int R, typename T, bool INV, int C, int E>
__device__ __forceinline__ void stockham_pass(cx<T>* buf, int n, int Ns, const cx<T>* __restrict__ tw) {
  constexpr int MAXB = (E + R - 1) / R;
  const int nr = n / R;
  const int nbf = nr * C;
  cx<T> v[MAXB][R];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    if (idx < nbf) bf_load<R, T, C>(buf, idx, nr, v[q]);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    if (idx < nbf) bf_store<R, T, INV, C>(buf, idx, Ns, tw, v[q]);
  }
  __syncthreads();
}

// Full transform; every thread of the block must call it, and the block must have at
// least n*C/E threads (E = elements a thread holds).  `tw` is the length's
// twiddle table (per pass p, W_{Ns*R}^{r*k} at tw_off[p] + k*(R-1) + r-1).
template <typename T, bool INV, int C, int E>
__device__ __forceinline__ void fft_lds(cx<T>* buf, const FftPlan& plan, const cx<T>* __restrict__ tw) {
  int Ns = 1;
  for (int p = 0; p < plan.npass; ++p) {
    const int R = plan.radix[p];
    const cx<T>* twp = tw + plan.tw_off[p];
    switch (R) {
      case 2: stockham_pass<2, T, INV, C, E>(buf, plan.n, Ns, twp); break;
      case 3: stockham_pass<3, T, INV, C, E>(buf, plan.n, Ns, twp); break;
      case 4: stockham_pass<4, T, INV, C, E>(buf, plan.n, Ns, twp); break;
      case 5: stockham_pass<5, T, INV, C, E>(buf, plan.n, Ns, twp); break;
      case 6: stockham_pass<6, T, INV, C, E>(buf, plan.n, Ns, twp); break;
      case 8: stockham_pass<8, T, INV, C, E>(buf, plan.n, Ns, twp); break;
      case 9: stockham_pass<9, T, INV, C, E>(buf, plan.n, Ns, twp); break;
      default: stockham_pass<10, T, INV, C, E>(buf, plan.n, Ns, twp); break;
    }
    Ns *= R;
  }
}

}  // namespace wct
