// Pre-calculated response spectrum (arXiv:2104.08265 Eq. 2: R(omega_t, omega_x) is
// computed once, in the frequency domain, before any event is simulated).
//
// For phase i, tick frequency w_t in [0, F) and wire frequency w_w in [0, L_w):
//   Rt[k][i][w_t] = sum_tau R[k][i][tau] exp(-2 pi i tau w_t / L_t)
//   R~_i(w_w, w_t) = (1 / (L_w L_t)) sum_{k=-K..K} Rt[k][i][w_t] exp(+2 pi i k w_w / L_w)
// (the +k sign because the wire sum is a correlation: wire w sees impact rows of
// wires w+k).  Both sums are evaluated directly in FP64 with exact integer reduction
// of the phase (the table holds exp(-2 pi i m / L) for m in [0, L)); R~ is stored in
// the plan dtype in the column-chunk layout [chunk][i][w_w][C] the column pass reads.
#include "kernels.hpp"

namespace wct {

__global__ void k_resp_tick(const double* __restrict__ R, int nk, int I, int TR, int lt, int F,
                            const cx<double>* __restrict__ tw_lt, cx<double>* __restrict__ out) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nk * I * F) return;
  const int w = (int)(idx % F);
  const int64_t ki = idx / F;
  const double* r = R + ki * TR;
  double ax = 0.0, ay = 0.0;
  for (int tau = 0; tau < TR; ++tau) {
    const cx<double> e = tw_lt[(int)(((int64_t)tau * w) % lt)];
    ax += r[tau] * e.x;
    ay += r[tau] * e.y;
  }
  out[idx] = mk(ax, ay);
}

template <typename T>
__global__ void k_resp_wire(const cx<double>* __restrict__ rt, int K, int I, int F, int lw, int lt, int nchunk,
                            const cx<double>* __restrict__ tw_lw, cx<T>* __restrict__ rtil) {
  const int64_t total = (int64_t)nchunk * I * lw * kChunk;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= total) return;
  // layout [chunk][i][w_w][C]
  const int cc = (int)(idx % kChunk);
  int64_t rest = idx / kChunk;
  const int ww = (int)(rest % lw);
  rest /= lw;
  const int i = (int)(rest % I);
  const int ch = (int)(rest / I);
  const int wt = ch * kChunk + cc;
  double ax = 0.0, ay = 0.0;
  if (wt < F) {
    for (int k = -K; k <= K; ++k) {
      const cx<double> a = rt[((int64_t)(k + K) * I + i) * F + wt];
      int m = (int)(((int64_t)k * ww) % lw);
      if (m < 0) m += lw;
      const cx<double> e = conj(tw_lw[m]);  // exp(+2 pi i k w_w / L_w)
      ax += a.x * e.x - a.y * e.y;
      ay += a.x * e.y + a.y * e.x;
    }
    const double s = 1.0 / ((double)lw * (double)lt);
    ax *= s;
    ay *= s;
  }
  rtil[idx] = mk((T)ax, (T)ay);
}

// Coefficients of the direct wire pass: R^_t[k][i](w_t) / L_t in the layout
// [w_t (padded to the chunks)][i][k + K], zero for w_t >= F.
template <typename T>
__global__ void k_resp_tick_pack(const cx<double>* __restrict__ rt, int K, int I, int F, int fpad, int lt,
                                 cx<T>* __restrict__ out) {
  const int nk = 2 * K + 1;
  const int64_t total = (int64_t)fpad * I * nk;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int kk = (int)(idx % nk);
  const int64_t rest = idx / nk;
  const int i = (int)(rest % I);
  const int wt = (int)(rest / I);
  cx<double> a = mk(0.0, 0.0);
  if (wt < F) {
    a = rt[((int64_t)kk * I + i) * F + wt];
    const double s = 1.0 / (double)lt;
    a = mk(a.x * s, a.y * s);
  }
  out[idx] = mk((T)a.x, (T)a.y);
}

template <typename T>
hipError_t launch_resp_tick_pack(const cx<double>* rt, int K, int I, int F, int fpad, int lt, cx<T>* rtick,
                                 hipStream_t st) {
  const int64_t n = (int64_t)fpad * I * (2 * K + 1);
  hipLaunchKernelGGL((k_resp_tick_pack<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rt, K, I, F, fpad, lt,
                     rtick);
  return hipGetLastError();
}
template hipError_t launch_resp_tick_pack<float>(const cx<double>*, int, int, int, int, int, cx<float>*, hipStream_t);
template hipError_t launch_resp_tick_pack<double>(const cx<double>*, int, int, int, int, int, cx<double>*,
                                                  hipStream_t);

hipError_t launch_resp_tick(const double* R, int nk, int I, int TR, int lt, int F, const cx<double>* tw_lt,
                            cx<double>* out, hipStream_t st) {
  const int64_t n = (int64_t)nk * I * F;
  hipLaunchKernelGGL(k_resp_tick, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, R, nk, I, TR, lt, F, tw_lt,
                     out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_resp_wire(const cx<double>* rt, int K, int I, int F, int lw, int lt, int nchunk,
                            const cx<double>* tw_lw, cx<T>* rtil, hipStream_t st) {
  const int64_t n = (int64_t)nchunk * I * lw * kChunk;
  hipLaunchKernelGGL((k_resp_wire<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rt, K, I, F, lw, lt,
                     nchunk, tw_lw, rtil);
  return hipGetLastError();
}

template hipError_t launch_resp_wire<float>(const cx<double>*, int, int, int, int, int, int, const cx<double>*,
                                            cx<float>*, hipStream_t);
template hipError_t launch_resp_wire<double>(const cx<double>*, int, int, int, int, int, int, const cx<double>*,
                                             cx<double>*, hipStream_t);

}  // namespace wct
