// Throughput probes (include/wct_probe.h).  Atomic adds: the on-device analog of the paper's
// atomic_add unit test and scaling figure for the scatter-add (arXiv:2104.08265 Sec. 5,
// Fig. 5).  They measure what the raster's two accumulation paths can reach on this
// chip: float adds into LDS (the privatised raster tiles) and float adds into device
// memory performed at L2 (crowded tiles, wide rows).  Both kernels use conflict-free
// addresses (a wave's 64 lanes hit 64 consecutive floats), so the rates are the peaks the
// raster's counts are compared against.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "wct_probe.h"

namespace {

thread_local std::string g_probe_err;

int probe_fail(int code, const char* what, hipError_t e) {
  g_probe_err = std::string(what) + (e != hipSuccess ? std::string(": ") + hipGetErrorString(e) : std::string());
  return code;
}

constexpr int kProbeThreads = 256;
constexpr int kProbeLds = 8192;  // floats of LDS per block
constexpr int kProbeUnroll = 8;

// iters rounds of kProbeUnroll LDS adds per thread; the result is unused (ds_add_f32
// without return), as in the raster tile.
__global__ void __launch_bounds__(kProbeThreads) k_probe_lds_add(float* __restrict__ out, int iters) {
  __shared__ float s[kProbeLds];
  for (int x = threadIdx.x; x < kProbeLds; x += kProbeThreads) s[x] = 0.f;
  __syncthreads();
  const int t = threadIdx.x;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) atomicAdd(&s[(t + (i * kProbeUnroll + u) * kProbeThreads) & (kProbeLds - 1)], 1.0f);
  }
  __syncthreads();
  out[(size_t)blockIdx.x * kProbeThreads + t] = s[t];
}

// iters rounds of kProbeUnroll device-memory adds per thread over a buffer of n floats
// (n a multiple of the grid's thread count): each wave adds into 64 consecutive floats.
__global__ void __launch_bounds__(kProbeThreads) k_probe_global_add(float* __restrict__ buf, int64_t n, int iters) {
  const int64_t nthreads = (int64_t)gridDim.x * kProbeThreads;
  const int64_t g = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) atomicAdd(&buf[(g + (int64_t)(i * kProbeUnroll + u) * nthreads) % n], 1.0f);
  }
}

// Instruction issue-rate probes: kProbeChains independent chains per thread, iters rounds.
// KIND 0: FP32 FMA with both multiplicands in vector registers; 1: FP32 FMA whose
// multiplier is a kernel argument (a scalar register, as the direct wire pass's
// coefficients are); 2: FP64 FMA, vector operands; 3: 32 x 32 -> 64-bit multiply-add
// with a scalar multiplier (the Philox product).  One 8-byte result per thread keeps
// the chains live.
constexpr int kProbeChains = 16;

template <int KIND>
__global__ void __launch_bounds__(kProbeThreads) k_probe_issue(uint64_t* __restrict__ out, int iters, float kf,
                                                               uint32_t ku) {
  const int t = threadIdx.x;
  uint64_t res = 0;
  if (KIND == 0 || KIND == 1) {
    float c[kProbeChains], x[kProbeChains], y[kProbeChains];
    for (int i = 0; i < kProbeChains; ++i) {
      c[i] = (float)(t + i);
      x[i] = 0.5f + 0.001f * (float)(t + i);
      y[i] = kf + 0.01f * (float)i + 1e-7f * (float)t;  // per lane: a vector register
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int i = 0; i < kProbeChains; ++i) c[i] = __builtin_fmaf(KIND == 0 ? y[i] : kf, x[i], c[i]);
    }
    float acc = 0.f;
    for (int i = 0; i < kProbeChains; ++i) acc += c[i];
    res = (uint64_t)__float_as_uint(acc);
  } else if (KIND == 2) {
    double c[kProbeChains], x[kProbeChains], y[kProbeChains];
    for (int i = 0; i < kProbeChains; ++i) {
      c[i] = (double)(t + i);
      x[i] = 0.5 + 0.001 * (double)(t + i);
      y[i] = (double)kf + 0.01 * (double)i + 1e-9 * (double)t;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int i = 0; i < kProbeChains; ++i) c[i] = __builtin_fma(y[i], x[i], c[i]);
    }
    double acc = 0.0;
    for (int i = 0; i < kProbeChains; ++i) acc += c[i];
    res = (uint64_t)__double_as_longlong(acc);
  } else {
    uint64_t c[kProbeChains];
    for (int i = 0; i < kProbeChains; ++i) c[i] = (uint64_t)(t * kProbeChains + i);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int i = 0; i < kProbeChains; ++i) c[i] = (uint64_t)ku * (uint32_t)c[i] + c[i];
    }
    for (int i = 0; i < kProbeChains; ++i) res ^= c[i];
  }
  out[(size_t)blockIdx.x * kProbeThreads + t] = res;
}

}  // namespace

extern "C" {

int wct_probe_issue_rate(int32_t kind, int32_t blocks, int32_t iters, void* buf, int64_t buf_bytes,
                         double* ops_per_s, void* stream) {
  g_probe_err.clear();
  if (!ops_per_s || !buf || blocks < 1 || iters < 1 || kind < 0 || kind > 3)
    return probe_fail(-1, "wct_probe_issue_rate: bad argument", hipSuccess);
  const int64_t nthreads = (int64_t)blocks * kProbeThreads;
  if (buf_bytes < nthreads * (int64_t)sizeof(uint64_t))
    return probe_fail(-1, "wct_probe_issue_rate: buffer below blocks x 256 x 8 bytes", hipSuccess);
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint64_t* out = static_cast<uint64_t*>(buf);
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  auto launch = [&]() {
    const dim3 g(blocks), t(kProbeThreads);
    if (kind == 0) hipLaunchKernelGGL(k_probe_issue<0>, g, t, 0, st, out, iters, 0.999f, 0xD2511F53u);
    if (kind == 1) hipLaunchKernelGGL(k_probe_issue<1>, g, t, 0, st, out, iters, 0.999f, 0xD2511F53u);
    if (kind == 2) hipLaunchKernelGGL(k_probe_issue<2>, g, t, 0, st, out, iters, 0.999f, 0xD2511F53u);
    if (kind == 3) hipLaunchKernelGGL(k_probe_issue<3>, g, t, 0, st, out, iters, 0.999f, 0xD2511F53u);
    return hipGetLastError();
  };
  if (e == hipSuccess) e = launch();  // warm-up
  if (e == hipSuccess) e = hipEventRecord(a, st);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, st);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (e != hipSuccess) return probe_fail(-3, "wct_probe_issue_rate", e);
  *ops_per_s = (double)nthreads * iters * kProbeChains / (ms * 1e-3);
  return 0;
}

int wct_probe_atomic_add(int32_t where, int32_t blocks, int32_t iters, float* buf, int64_t buf_elems,
                         double* adds_per_s, void* stream) {
  g_probe_err.clear();
  if (!adds_per_s || !buf || blocks < 1 || iters < 1 || (where != 0 && where != 1))
    return probe_fail(-1, "wct_probe_atomic_add: bad argument", hipSuccess);
  const int64_t nthreads = (int64_t)blocks * kProbeThreads;
  if (where == 0 && buf_elems < nthreads) return probe_fail(-1, "wct_probe_atomic_add: buffer below blocks x 256", hipSuccess);
  if (where == 1 && (buf_elems < nthreads || buf_elems % nthreads != 0))
    return probe_fail(-1, "wct_probe_atomic_add: buffer not a multiple of blocks x 256", hipSuccess);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  auto launch = [&]() {
    if (where == 0)
      hipLaunchKernelGGL(k_probe_lds_add, dim3(blocks), dim3(kProbeThreads), 0, st, buf, iters);
    else
      hipLaunchKernelGGL(k_probe_global_add, dim3(blocks), dim3(kProbeThreads), 0, st, buf, buf_elems, iters);
    return hipGetLastError();
  };
  if (e == hipSuccess) e = launch();  // warm-up
  if (e == hipSuccess) e = hipEventRecord(a, st);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, st);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (e != hipSuccess) return probe_fail(-3, "wct_probe_atomic_add", e);
  *adds_per_s = (double)nthreads * iters * kProbeUnroll / (ms * 1e-3);
  return 0;
}

const char* wct_probe_last_error(void) { return g_probe_err.c_str(); }

}  // extern "C"
