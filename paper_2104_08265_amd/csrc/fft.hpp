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

// cos and sin of 2 pi m / n, evaluated at compile time: the angle is reduced exactly to
// a quarter turn and then to [0, pi/4], where short Taylor series are accurate to the
// last bit of a double.
constexpr double ct_sin_small(double a) {
  const double a2 = a * a;
  double t = a, s = a;
  for (int k = 1; k <= 12; ++k) {
    t = -t * a2 / (double)((2 * k) * (2 * k + 1));
    s += t;
  }
  return s;
}
constexpr double ct_cos_small(double a) {
  const double a2 = a * a;
  double t = 1.0, s = 1.0;
  for (int k = 1; k <= 12; ++k) {
    t = -t * a2 / (double)((2 * k - 1) * (2 * k));
    s += t;
  }
  return s;
}
struct CtCis {
  double c, s;
};
constexpr CtCis ct_cis(long m, long n) {
  m %= n;
  if (m < 0) m += n;
  const long q = (4 * m) / n;  // quarter turn
  const long r = 4 * m - q * n;  // angle within it: (pi/2) r / n
  constexpr double kHalfPi = 1.5707963267948966;
  double c = 0, s = 0;
  if (2 * r <= n) {
    const double a = kHalfPi * ((double)r / (double)n);
    c = ct_cos_small(a);
    s = ct_sin_small(a);
  } else {
    const double a = kHalfPi * ((double)(n - r) / (double)n);
    c = ct_sin_small(a);
    s = ct_cos_small(a);
  }
  if (q == 0) return CtCis{c, s};
  if (q == 1) return CtCis{-s, c};
  if (q == 2) return CtCis{-c, -s};
  return CtCis{s, -c};
}

// exp(-2 pi i m / N), m < N, for the composite codelets.
template <int N>
struct WTabData {
  double re[N], im[N];
};
template <int N>
constexpr WTabData<N> make_wtab() {
  WTabData<N> d{};
  for (int m = 0; m < N; ++m) {
    const CtCis e = ct_cis(m, N);
    d.re[m] = e.c;
    d.im[m] = -e.s;
  }
  return d;
}
template <int N>
struct WTab {
  static constexpr WTabData<N> d = make_wtab<N>();
};
// a * W_N^m (forward) or a * W_N^-m (inverse) for a compile-time m after unrolling.
template <typename T, bool INV, int N>
__host__ __device__ __forceinline__ cx<T> wmul(cx<T> a, int m) {
  m %= N;
  if (m == 0) return a;
  if (4 * m == N) return rot<T, INV>(a);
  if (2 * m == N) return mk(-a.x, -a.y);
  if (4 * m == 3 * N) return rot<T, !INV>(a);
  const T c = (T)WTab<N>::d.re[m];
  const T s = INV ? -(T)WTab<N>::d.im[m] : (T)WTab<N>::d.im[m];
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

// Split of a composite radix R = R1 * R2: the largest of 10, 9, 8, 5, 4, 3, 2 below R
// that divides it.
constexpr int comp_split(int R) {
  constexpr int c[7] = {10, 9, 8, 5, 4, 3, 2};
  for (int k = 0; k < 7; ++k)
    if (c[k] < R && R % c[k] == 0) return c[k];
  return 0;
}

template <int R, typename T, bool INV>
__host__ __device__ __forceinline__ void dftR(cx<T>* v) {
  if constexpr (R == 2) dft2<T, INV>(v);
  else if constexpr (R == 3) dft3<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v);
  else if constexpr (R == 5) dft5<T, INV>(v);
  else if constexpr (R == 8) dft8<T, INV>(v);
  else {
    static_assert(comp_split(R) > 0, "radix must be a product of 2, 3 and 5");
    dft_comp<T, INV, comp_split(R), R / comp_split(R)>(v);
  }
}

// Butterfly idx of a Stockham pass (radix R, stride Ns) over C interleaved sequences:
// the load half, the twiddle load and the twiddle + DFT + store half.  Shared by the
// device pass and the host check of the transforms.
template <int R, typename T, int C>
__host__ __device__ __forceinline__ void bf_load(const cx<T>* buf, int idx, int nr, cx<T>* v) {
  const int c = idx % C, j = idx / C;
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = buf[(j + r * nr) * C + c];
}
template <int R, typename T, int C>
__host__ __device__ __forceinline__ void bf_twiddles(int idx, int Ns, const cx<T>* __restrict__ tw, cx<T>* w) {
  const int k = (idx / C) % Ns;
  const cx<T>* p = tw + k * (R - 1);
#pragma unroll
  for (int r = 0; r < R - 1; ++r) w[r] = p[r];
}
template <int R, typename T, bool INV, int C>
__host__ __device__ __forceinline__ void bf_store(cx<T>* buf, int idx, int Ns, const cx<T>* w, cx<T>* v) {
  const int c = idx % C, j = idx / C;
  const int k = j % Ns;
  if (Ns > 1) {
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = INV ? cmulc(v[r], w[r - 1]) : cmul(v[r], w[r - 1]);
  }
  dftR<R, T, INV>(v);
  const int base = (j - k) * R + k;
#pragma unroll
  for (int r = 0; r < R; ++r) buf[(base + r * Ns) * C + c] = v[r];
}

// One Stockham pass over C interleaved sequences of length n in LDS.  The twiddles do
// not depend on the LDS contents; with TWPF they are requested before the barrier (at
// the cost of holding them across it).
template <int R, typename T, bool INV, int C, int E, bool TWPF>
__device__ __forceinline__ void stockham_pass(cx<T>* buf, int n, int Ns, const cx<T>* __restrict__ tw) {
  constexpr int MAXB = (E + R - 1) / R;
  const int nr = n / R;
  const int nbf = nr * C;
  cx<T> v[MAXB][R];
  cx<T> w[MAXB][R - 1];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    if (idx < nbf) {
      if (TWPF && Ns > 1) bf_twiddles<R, T, C>(idx, Ns, tw, w[q]);
      bf_load<R, T, C>(buf, idx, nr, v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    if (idx < nbf) {
      if (!TWPF && Ns > 1) bf_twiddles<R, T, C>(idx, Ns, tw, w[q]);
      bf_store<R, T, INV, C>(buf, idx, Ns, w[q], v[q]);
    }
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
      case 2: stockham_pass<2, T, INV, C, E, (C == 1)>(buf, plan.n, Ns, twp); break;
      case 3: stockham_pass<3, T, INV, C, E, (C == 1)>(buf, plan.n, Ns, twp); break;
      case 4: stockham_pass<4, T, INV, C, E, (C == 1)>(buf, plan.n, Ns, twp); break;
      case 5: stockham_pass<5, T, INV, C, E, (C == 1)>(buf, plan.n, Ns, twp); break;
      case 6: stockham_pass<6, T, INV, C, E, (C == 1)>(buf, plan.n, Ns, twp); break;
      case 8: stockham_pass<8, T, INV, C, E, (C == 1)>(buf, plan.n, Ns, twp); break;
      case 9: stockham_pass<9, T, INV, C, E, (C == 1)>(buf, plan.n, Ns, twp); break;
      default: stockham_pass<10, T, INV, C, E, (C == 1)>(buf, plan.n, Ns, twp); break;
    }
    Ns *= R;
  }
}

// ---------------------------------------------------------------------------
// Compile-time plans.  For the transform lengths of the shipped geometries the radix
// sequence, the thread count and the interleave are template parameters: strides,
// twiddle offsets and divisions fold into constants, LDS addresses into instruction
// offsets, and each thread's butterflies of a pass are a fixed unrolled set.  The
// butterflies are the runtime pass's (same codelets, same index formulas), with the
// twiddle table laid out as build_fft lays it out for the same radices.
// ---------------------------------------------------------------------------
template <int R, typename T, int C, int NR>
__host__ __device__ __forceinline__ void bfc_load(const cx<T>* buf, int idx, cx<T>* v) {
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = buf[idx + r * NR * C];
}
template <int R, typename T, int C, int NS>
__host__ __device__ __forceinline__ void bfc_twiddles(int idx, const cx<T>* __restrict__ tw, cx<T>* w) {
  const int k = (idx / C) % NS;
  const cx<T>* p = tw + k * (R - 1);
#pragma unroll
  for (int r = 0; r < R - 1; ++r) w[r] = p[r];
}
// Same twiddles from one table entry, W^k, and its powers by squaring and multiplying
// (depth <= log2 R products; relative error grows to about R rounding errors of the
// entry).  Holds one value across the barrier instead of R - 1.
template <int R, typename T, int C, int NS>
__host__ __device__ __forceinline__ void bfc_twiddles_pow(int idx, const cx<T>* __restrict__ tw, cx<T>* w) {
  const int k = (idx / C) % NS;
  w[0] = tw[k * (R - 1)];
#pragma unroll
  for (int r = 2; r < R; ++r) w[r - 1] = (r % 2 == 0) ? cmul(w[r / 2 - 1], w[r / 2 - 1]) : cmul(w[r - 2], w[0]);
}
template <int R, typename T, bool INV, int C, int NS>
__host__ __device__ __forceinline__ void bfc_store(cx<T>* buf, int idx, const cx<T>* w, cx<T>* v) {
  const int c = idx % C, j = idx / C;
  const int k = j % NS;
  if constexpr (NS > 1) {
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = INV ? cmulc(v[r], w[r - 1]) : cmul(v[r], w[r - 1]);
  }
  dftR<R, T, INV>(v);
  const int base = ((j - k) * R + k) * C + c;
#pragma unroll
  for (int r = 0; r < R; ++r) buf[base + r * NS * C] = v[r];
}

// Twiddle policy of the compiled passes: row transforms (C = 1) request the table
// entries before the barrier; column transforms, which hold many values per thread,
// load one entry per butterfly after it and form the powers.
template <typename T, bool INV, int C, int NT, int N, int R, int NS>
__device__ __forceinline__ void ct_pass(cx<T>* buf, const cx<T>* __restrict__ tw) {
  constexpr bool TWPF = C == 1;
  constexpr int NR = N / R, NB = NR * C, MB = (NB + NT - 1) / NT;
  constexpr bool FULL = NB % NT == 0;
  cx<T> v[MB][R];
  cx<T> w[MB][R - 1];
#pragma unroll
  for (int q = 0; q < MB; ++q) {
    const int idx = (int)threadIdx.x + q * NT;
    if (FULL || idx < NB) {
      if constexpr (TWPF && NS > 1) bfc_twiddles<R, T, C, NS>(idx, tw, w[q]);
      bfc_load<R, T, C, NR>(buf, idx, v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MB; ++q) {
    const int idx = (int)threadIdx.x + q * NT;
    if (FULL || idx < NB) {
      if constexpr (!TWPF && NS > 1) bfc_twiddles_pow<R, T, C, NS>(idx, tw, w[q]);
      bfc_store<R, T, INV, C, NS>(buf, idx, w[q], v[q]);
    }
  }
  __syncthreads();
}

template <typename T, bool INV, int C, int NT, int N, int NS, int TWO, int R, int... Rest>
__device__ __forceinline__ void ct_fft(cx<T>* buf, const cx<T>* __restrict__ tw) {
  ct_pass<T, INV, C, NT, N, R, NS>(buf, tw + TWO);
  if constexpr (sizeof...(Rest) > 0) ct_fft<T, INV, C, NT, N, NS * R, TWO + NS * (R - 1), Rest...>(buf, tw);
}

// Chains with register input and output.  The first pass (stride 1) needs no twiddles
// and reads, for butterfly idx, the elements idx + r (N/R0) C; a caller that holds
// exactly those values in registers skips the LDS write and read before it.  The last
// pass (stride N/RL) writes every output back to the position it read it from, so its
// results can stay in the registers that held its inputs.
template <typename T, bool INV, int C, int NT, int N, int R, int NS>
__device__ __forceinline__ void ct_last_to_regs(cx<T>* buf, const cx<T>* __restrict__ tw, cx<T>* out) {
  constexpr int NR = N / R, NB = NR * C, MB = (NB + NT - 1) / NT;
  constexpr bool FULL = NB % NT == 0;
  constexpr bool TWPF = C == 1;
  cx<T> w[MB][R - 1];
#pragma unroll
  for (int q = 0; q < MB; ++q) {
    const int idx = (int)threadIdx.x + q * NT;
    if (FULL || idx < NB) {
      if constexpr (TWPF && NS > 1) bfc_twiddles<R, T, C, NS>(idx, tw, w[q]);
      bfc_load<R, T, C, NR>(buf, idx, &out[q * R]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MB; ++q) {
    const int idx = (int)threadIdx.x + q * NT;
    if (FULL || idx < NB) {
      if constexpr (!TWPF && NS > 1) bfc_twiddles_pow<R, T, C, NS>(idx, tw, w[q]);
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r)
          out[q * R + r] = INV ? cmulc(out[q * R + r], w[q][r - 1]) : cmul(out[q * R + r], w[q][r - 1]);
      }
      dftR<R, T, INV>(&out[q * R]);
    }
  }
}

template <typename T, bool INV, int C, int NT, int N, bool OREG, int NS, int TWO, int R, int... Rest>
__device__ __forceinline__ void ct_rest(cx<T>* buf, const cx<T>* __restrict__ tw, cx<T>* out) {
  if constexpr (sizeof...(Rest) == 0) {
    if constexpr (OREG) ct_last_to_regs<T, INV, C, NT, N, R, NS>(buf, tw + TWO, out);
    else ct_pass<T, INV, C, NT, N, R, NS>(buf, tw + TWO);
  } else {
    ct_pass<T, INV, C, NT, N, R, NS>(buf, tw + TWO);
    ct_rest<T, INV, C, NT, N, OREG, NS * R, TWO + NS * (R - 1), Rest...>(buf, tw, out);
  }
}

// in: first-pass inputs (consumed); out: last-pass outputs (OREG) or natural order in
// LDS.  hook() runs once the inputs are no longer needed (to start the next loads).
template <typename T, bool INV, int C, int NT, int N, bool OREG, typename Hook, int R0, int... Rest>
__device__ __forceinline__ void ct_chain(cx<T>* buf, const cx<T>* __restrict__ tw, cx<T>* in, cx<T>* out,
                                         Hook& hook) {
  constexpr int NB = (N / R0) * C, MB = (NB + NT - 1) / NT;
  constexpr bool FULL = NB % NT == 0;
  if constexpr (sizeof...(Rest) == 0) {
#pragma unroll
    for (int q = 0; q < MB; ++q) {
      const int idx = (int)threadIdx.x + q * NT;
      if (FULL || idx < NB) {
        if constexpr (OREG) {
          dftR<R0, T, INV>(&in[q * R0]);
#pragma unroll
          for (int r = 0; r < R0; ++r) out[q * R0 + r] = in[q * R0 + r];
        } else {
          bfc_store<R0, T, INV, C, 1>(buf, idx, nullptr, &in[q * R0]);
        }
      }
    }
    hook();
    if constexpr (!OREG) __syncthreads();
  } else {
#pragma unroll
    for (int q = 0; q < MB; ++q) {
      const int idx = (int)threadIdx.x + q * NT;
      if (FULL || idx < NB) bfc_store<R0, T, INV, C, 1>(buf, idx, nullptr, &in[q * R0]);
    }
    hook();
    __syncthreads();
    ct_rest<T, INV, C, NT, N, OREG, R0, R0 - 1, Rest...>(buf, tw, out);
  }
}

template <int... Rs>
struct IntList {};
template <typename L, typename A = IntList<>>
struct RevList;
template <int R, int... Rs, int... A>
struct RevList<IntList<R, Rs...>, IntList<A...>> {
  using type = typename RevList<IntList<Rs...>, IntList<R, A...>>::type;
};
template <int... A>
struct RevList<IntList<>, IntList<A...>> {
  using type = IntList<A...>;
};
template <int... Rs>
constexpr int first_of() {
  constexpr int r[] = {Rs...};
  return r[0];
}
template <int... Rs>
constexpr int last_of() {
  constexpr int r[] = {Rs...};
  return r[sizeof...(Rs) - 1];
}

// Transform policies the kernels are written against.
//  RtFft: runtime plan (any 2,3,5-smooth length), E values per thread, any block size.
//  CtFft: compile-time plan with radices Rs..., exactly NT threads per block, registers
//         budgeted for MINW waves per SIMD; besides the
//         LDS-to-LDS run() it offers the register-input chains rr() and rl().
template <typename T, int C, int E_>
struct RtFft {
  static constexpr int E = E_;
  static constexpr int kBound = LaunchBound<T, E_>::value;
  FftPlan p;
  __device__ __forceinline__ int n() const { return p.n; }
  __device__ __forceinline__ int nthr() const { return (int)blockDim.x; }
  template <bool INV>
  __device__ __forceinline__ void run(cx<T>* buf, const cx<T>* __restrict__ tw) const {
    fft_lds<T, INV, C, E_>(buf, p, tw);
  }
};
template <typename T, int C, int NT, int MINW, typename L>
struct CtFftOf;
template <typename T, int C, int NT, int MINW, int... Rs>
struct CtFft {
  static constexpr int N = (1 * ... * Rs);
  static constexpr int CI = C;  // interleaved sequences
  static constexpr int E = (N * C + NT - 1) / NT;
  static constexpr int kBound = NT;
  static constexpr int kThreads = NT;
  // waves per SIMD the register allocation must allow (chosen per variant so that the
  // blocks the LDS admits also fit in the register file)
  static constexpr int kMinWaves = MINW;
  static constexpr int R0 = first_of<Rs...>(), RL = last_of<Rs...>();
  static constexpr int NB0 = (N / R0) * C, NBL = (N / RL) * C;  // butterflies of the first / last pass
  static constexpr int MB0 = (NB0 + NT - 1) / NT, MBL = (NBL + NT - 1) / NT;
  static constexpr int IN = MB0 * R0, OUT = MBL * RL;  // register values per thread
  // same radices in reverse order: its first pass reads what this one's last pass leaves
  using Reverse = typename CtFftOf<T, C, NT, MINW, typename RevList<IntList<Rs...>>::type>::type;
  __device__ __forceinline__ constexpr int n() const { return N; }
  __device__ __forceinline__ constexpr int nthr() const { return NT; }
  // element held in register slot (q, r): first-pass and last-pass arrangement
  __device__ __forceinline__ static int in_elem(int q, int r) { return (int)threadIdx.x + q * NT + r * NB0; }
  // the same minus the thread index: a compile-time constant after unrolling
  __host__ __device__ __forceinline__ static constexpr int in_off(int q, int r) { return q * NT + r * NB0; }
  __host__ __device__ __forceinline__ static constexpr int out_off(int q, int r) { return q * NT + r * NBL; }
  __device__ __forceinline__ static bool in_ok(int q) { return NB0 % NT == 0 || (int)threadIdx.x + q * NT < NB0; }
  __device__ __forceinline__ static int out_elem(int q, int r) { return (int)threadIdx.x + q * NT + r * NBL; }
  __device__ __forceinline__ static bool out_ok(int q) { return NBL % NT == 0 || (int)threadIdx.x + q * NT < NBL; }
  template <bool INV>
  __device__ __forceinline__ void run(cx<T>* buf, const cx<T>* __restrict__ tw) const {
    ct_fft<T, INV, C, NT, N, 1, 0, Rs...>(buf, tw);
  }
  template <bool INV, typename Hook>
  __device__ __forceinline__ static void rr(cx<T>* buf, const cx<T>* __restrict__ tw, cx<T>* in, cx<T>* out,
                                            Hook&& hook) {
    ct_chain<T, INV, C, NT, N, true, Hook, Rs...>(buf, tw, in, out, hook);
  }
  template <bool INV, typename Hook>
  __device__ __forceinline__ static void rl(cx<T>* buf, const cx<T>* __restrict__ tw, cx<T>* in, Hook&& hook) {
    ct_chain<T, INV, C, NT, N, false, Hook, Rs...>(buf, tw, in, nullptr, hook);
  }
};
template <typename T, int C, int NT, int MINW, int... Rs>
struct CtFftOf<T, C, NT, MINW, IntList<Rs...>> {
  using type = CtFft<T, C, NT, MINW, Rs...>;
};

}  // namespace wct
