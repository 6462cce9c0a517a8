// Per-row gradient gather for the differentiable mode.
//
// Given H = dL/dS (the convolution's adjoint applied to dL/dM), the raster
// S = sum_j Q_j A_j (x) B_j gives, for row j with window cells (b, k),
//   g_Q       = sum H A_b B_k
//   g_t       = Q sum H A_b dB_k/dt          g_sigma_t = Q sum H A_b dB_k/dsigma_t
//   g_p       = Q I sum H dA_b/du B_k       g_sigma_p = Q I sum H dA_b/dsigma_u B_k
// with u = I p, sigma_u = I sigma_p.  For a cell with edges e_lo = max(k, lo),
// e_hi = min(k+1, hi) and z = (e - mu) / sigma, the clipped integral
// w = Phi(z_hi) - Phi(z_lo) has
//   dw/dmu    = -(phi(z_hi) [hi edge free] - phi(z_lo) [lo edge free]) / sigma
//   dw/dsigma = -(z_hi phi(z_hi) [free] - z_lo phi(z_lo) [free]) / sigma,
// an edge clipped to the truncation window (mu +- nsigma sigma) being fixed in z.
// One wave per row; cells are visited in chunks so any window size is handled, and
// the five sums are accumulated in FP64 and reduced across the wave.
#include "kernels.hpp"

namespace wct {

namespace {

struct AxisD {
  double w, dmu, dsig;
};

__device__ __forceinline__ AxisD axis_d(int k, double mu, double sigma, double lo, double hi) {
  const double kf = (double)k;
  const bool clo = kf < lo, chi = kf + 1.0 > hi;
  const double elo = clo ? lo : kf, ehi = chi ? hi : kf + 1.0;
  const double zlo = (elo - mu) / sigma, zhi = (ehi - mu) / sigma;
  constexpr double inv_sqrt2pi = 0.39894228040143267794;
  const double plo = clo ? 0.0 : inv_sqrt2pi * exp(-0.5 * zlo * zlo);
  const double phi = chi ? 0.0 : inv_sqrt2pi * exp(-0.5 * zhi * zhi);
  AxisD a;
  a.w = 0.5 * (erf(zhi * 0.70710678118654752440) - erf(zlo * 0.70710678118654752440));
  a.dmu = -(phi - plo) / sigma;
  a.dsig = -(zhi * phi - zlo * plo) / sigma;
  return a;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace

template <typename T>
__global__ void __launch_bounds__(256) k_grad_gather(DepoView<T> d, RasterGeom g, double nsigma,
                                                     const T* __restrict__ H, T* __restrict__ gq, T* __restrict__ gt,
                                                     T* __restrict__ gp, T* __restrict__ gst,
                                                     T* __restrict__ gsp) {
  constexpr int CB = 64, CK = 64;
  __shared__ AxisD s_a[4][CB];
  __shared__ AxisD s_b[4][CK];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 4 + wv;
  if (j >= d.n) return;
  const int pl_i = d.plane ? d.plane[j] : 0;
  const int ev_id = d.event ? d.event[j] : 0;
  const int ev = ev_id - g.event_base;
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0;
  double q = 0;
  int I = 1;
  bool ok = pl_i >= 0 && pl_i < g.n_planes && ev_id >= 0 && ev >= 0 && ev < g.n_events;
  if (ok) {
    const PlaneGeom& pl = g.pl[pl_i];
    I = pl.I;
    q = (double)d.q[j];
    const double t = (double)d.t[j], p = (double)d.p[j];
    const double st = (double)d.st[j], sp = (double)d.sp[j];
    ok = q >= 0.0 && st > 0.0 && sp > 0.0 && isfinite(q) && isfinite(t) && isfinite(p) && isfinite(st) &&
         isfinite(sp);
    if (ok) {
      const double u = (double)pl.I * p, su = (double)pl.I * sp;
      const double hu = nsigma * su, ht = nsigma * st;
      const double ulo = u - hu, uhi = u + hu, tlo = t - ht, thi = t + ht;
      const int b0 = (int)fmax(floor(ulo), 0.0), b1 = (int)fmin(ceil(uhi), (double)pl.nb);
      const int k0 = (int)fmax(floor(tlo), 0.0), k1 = (int)fmin(ceil(thi), (double)pl.nt);
      const T* h = H + (int64_t)ev * g.grid_ev_stride + pl.grid_off;
      for (int cb = b0; cb < b1; cb += CB)
        for (int ck = k0; ck < k1; ck += CK) {
          const int nbr = min(CB, b1 - cb), nkr = min(CK, k1 - ck);
          if (lane < nbr) s_a[wv][lane] = axis_d(cb + lane, u, su, ulo, uhi);
          if (lane < nkr) s_b[wv][lane] = axis_d(ck + lane, t, st, tlo, thi);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          for (int x = lane; x < nbr * nkr; x += 64) {
            const int bi = x / nkr, ki = x - (x / nkr) * nkr;
            const double hv = (double)h[(int64_t)(cb + bi) * pl.nt + ck + ki];
            const AxisD A = s_a[wv][bi], B = s_b[wv][ki];
            s0 += hv * A.w * B.w;
            s1 += hv * A.w * B.dmu;
            s2 += hv * A.w * B.dsig;
            s3 += hv * A.dmu * B.w;
            s4 += hv * A.dsig * B.w;
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  s3 = wave_sum(s3);
  s4 = wave_sum(s4);
  if (lane == 0) {
    gq[j] = (T)s0;
    gt[j] = (T)(q * s1);
    gst[j] = (T)(q * s2);
    gp[j] = (T)(q * I * s3);
    gsp[j] = (T)(q * I * s4);
  }
}

template <typename T>
hipError_t launch_grad_gather(const DepoView<T>& d, const RasterGeom& g, double nsigma, const T* H, T* gq, T* gt,
                              T* gp, T* gst, T* gsp, hipStream_t st) {
  if (d.n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((d.n + 3) / 4);
  hipLaunchKernelGGL((k_grad_gather<T>), dim3(blocks), dim3(256), 0, st, d, g, nsigma, H, gq, gt, gp, gst, gsp);
  return hipGetLastError();
}

template hipError_t launch_grad_gather<float>(const DepoView<float>&, const RasterGeom&, double, const float*, float*,
                                              float*, float*, float*, float*, hipStream_t);
template hipError_t launch_grad_gather<double>(const DepoView<double>&, const RasterGeom&, double, const double*,
                                               double*, double*, double*, double*, double*, hipStream_t);

}  // namespace wct
