// ADC digitisation of the waveform (Eq. 1: M is a measurement such as an ADC value,
// Sec. 2): per plane, code = min(max(floor(M g + b + 1/2), 0), c_max), a non-number
// giving 0, computed in the plan's type with one rounding per operation: the product and
// the two sums are rounded one by one (this file is compiled with contraction off; the
// round-to-nearest intrinsics alone are plain operations that may be fused).
//
// HBM-bound: each sample is read once (4 or 8 bytes) and its code written once (2
// bytes).  A thread handles 4 consecutive samples per step (one 16- or 32-byte load, one
// 8-byte store) when the plane's rows allow it; grid-stride over the plane's samples of
// every event of the call.
#include "kernels.hpp"

namespace wct {

__device__ __forceinline__ float adc_step(float m, float g, float b, float cmax) {
  float t = __fmul_rn(m, g);
  t = __fadd_rn(t, b);
  t = __fadd_rn(t, 0.5f);
  const float x = floorf(t);
  return x >= 0.f ? (x <= cmax ? x : cmax) : 0.f;
}
__device__ __forceinline__ double adc_step(double m, double g, double b, double cmax) {
  double t = __dmul_rn(m, g);
  t = __dadd_rn(t, b);
  t = __dadd_rn(t, 0.5);
  const double x = floor(t);
  return x >= 0.0 ? (x <= cmax ? x : cmax) : 0.0;
}

template <typename T, bool VEC>
__global__ void __launch_bounds__(256) k_digitize(const T* __restrict__ wave, int64_t ev_stride, int64_t n,
                                                  int n_events, T gain, T base, T cmax,
                                                  uint16_t* __restrict__ out) {
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int ev = 0; ev < n_events; ++ev) {
    const T* w = wave + ev * ev_stride;
    uint16_t* o = out + ev * ev_stride;
    if (VEC) {  // n, ev_stride and the plane offset are multiples of 4
      for (int64_t q = g0; q < n / 4; q += nthreads) {
        typedef T V4 __attribute__((ext_vector_type(4)));
        const V4 m = *reinterpret_cast<const V4*>(w + 4 * q);
        ushort4 c;
        c.x = (uint16_t)adc_step(m.x, gain, base, cmax);
        c.y = (uint16_t)adc_step(m.y, gain, base, cmax);
        c.z = (uint16_t)adc_step(m.z, gain, base, cmax);
        c.w = (uint16_t)adc_step(m.w, gain, base, cmax);
        *reinterpret_cast<ushort4*>(o + 4 * q) = c;
      }
    } else {
      for (int64_t q = g0; q < n; q += nthreads) o[q] = (uint16_t)adc_step(w[q], gain, base, cmax);
    }
  }
}

template <typename T>
hipError_t launch_digitize(const T* wave, int64_t ev_stride, int64_t n, int n_events, double gain, double base,
                           int max_code, uint16_t* out, int n_cu, hipStream_t st) {
  if (n <= 0 || n_events <= 0) return hipSuccess;
  const bool vec = n % 4 == 0 && ev_stride % 4 == 0 && reinterpret_cast<uintptr_t>(wave) % (4 * sizeof(T)) == 0 &&
                   reinterpret_cast<uintptr_t>(out) % 8 == 0;
  const int64_t work = vec ? n / 4 : n;
  int64_t blocks = (work + 255) / 256;
  const int64_t cap = (int64_t)n_cu * 8;  // a few waves of 256-thread blocks per CU, grid-stride beyond
  if (blocks > cap) blocks = cap;
  if (vec)
    hipLaunchKernelGGL((k_digitize<T, true>), dim3((unsigned)blocks), dim3(256), 0, st, wave, ev_stride, n, n_events,
                       (T)gain, (T)base, (T)max_code, out);
  else
    hipLaunchKernelGGL((k_digitize<T, false>), dim3((unsigned)blocks), dim3(256), 0, st, wave, ev_stride, n,
                       n_events, (T)gain, (T)base, (T)max_code, out);
  return hipGetLastError();
}

template hipError_t launch_digitize<float>(const float*, int64_t, int64_t, int, double, double, int, uint16_t*, int,
                                           hipStream_t);
template hipError_t launch_digitize<double>(const double*, int64_t, int64_t, int, double, double, int, uint16_t*,
                                            int, hipStream_t);

}  // namespace wct
