// Drift, diffusion, attenuation and projection of ionisation clouds onto the wire planes
// (Fig. 2: the clouds drift to the readout and spread along and across the drift;
// Sec. 2.1.1: the raster takes each cloud's Gaussian at the plane).  One thread per
// deposition computes, in FP64 in the order written,
//   t_d = x / v;  sigma_L = sqrt(sigma_L0^2 + 2 D_L t_d);  sigma_T = sqrt(sigma_T0^2 + 2 D_T t_d);
//   Q = q exp(-t_d / tau)  (tau <= 0: Q = q);  Q = 0 unless x >= 0 and every input is finite;
// and writes one row per plane k (plane-major, row k n + j):
//   t = (t0 + t_d + d_k) / T_tick,  p = (z cos th_k + y sin th_k) / P_k + o_k,
//   sigma_t = sigma_L / (v T_tick),  sigma_p = sigma_T / P_k,
// rounded to the plan dtype.  The cosines and sines of the plane angles are computed once
// on the host.  HBM-bound: 7 values read and 5 n_planes values (plus 3 n_planes ints)
// written per deposition, coalesced.  This file is compiled with contraction off.
#include "kernels.hpp"

namespace wct {

template <typename T>
__global__ void __launch_bounds__(256) k_drift(DriftIn<T> in, DriftArgs a, DriftOut<T> out) {
  const int64_t n = in.n;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const double x = (double)in.x[j], y = (double)in.y[j], z = (double)in.z[j];
    const double t0 = (double)in.t0[j], q = (double)in.q[j];
    const double sl0 = (double)in.sl0[j], st0 = (double)in.st0[j];
    const bool ok = x >= 0.0 && isfinite(x) && isfinite(y) && isfinite(z) && isfinite(t0) && isfinite(q) &&
                    isfinite(sl0) && isfinite(st0);
    const double td = (ok ? x : 0.0) / a.speed;
    const double sl = sqrt(sl0 * sl0 + 2.0 * a.dl * td);
    const double st = sqrt(st0 * st0 + 2.0 * a.dt * td);
    double Q = a.lifetime > 0.0 ? q * exp(-td / a.lifetime) : q;
    Q = ok ? Q : 0.0;
    const int32_t ev = in.event ? in.event[j] : 0;
    const int32_t id = in.depo_id ? in.depo_id[j] : (int32_t)j;
    const double sig_t = sl / (a.speed * a.tick);
    for (int k = 0; k < a.n_planes; ++k) {
      const int64_t r = (int64_t)k * n + j;
      out.q[r] = (T)Q;
      out.t[r] = (T)((t0 + td + a.toff[k]) / a.tick);
      out.p[r] = (T)((z * a.cth[k] + y * a.sth[k]) / a.pitch[k] + a.woff[k]);
      out.st[r] = (T)sig_t;
      out.sp[r] = (T)(st / a.pitch[k]);
      out.plane[r] = k;
      out.event[r] = ev;
      out.depo_id[r] = id;
    }
  }
}

template <typename T>
hipError_t launch_drift(const DriftIn<T>& in, const DriftArgs& a, const DriftOut<T>& out, int n_cu, hipStream_t st) {
  if (in.n <= 0) return hipSuccess;
  int64_t blocks = (in.n + 255) / 256;
  if (blocks > (int64_t)n_cu * 16) blocks = (int64_t)n_cu * 16;
  hipLaunchKernelGGL(k_drift<T>, dim3((unsigned)blocks), dim3(256), 0, st, in, a, out);
  return hipGetLastError();
}

template hipError_t launch_drift<float>(const DriftIn<float>&, const DriftArgs&, const DriftOut<float>&, int,
                                        hipStream_t);
template hipError_t launch_drift<double>(const DriftIn<double>&, const DriftArgs&, const DriftOut<double>&, int,
                                         hipStream_t);

}  // namespace wct
