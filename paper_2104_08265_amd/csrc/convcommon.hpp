// Helpers shared by the transform kernels (conv.hip: runtime plans; conv_ct.hip:
// compiled plans).
#pragma once

#include <type_traits>

#include "fft.hpp"
#include "fftvariants.hpp"
#include "kernels.hpp"

namespace wct {

// [lo, hi) of a row from its recorded span (kSpanBase - lo, hi); the whole row [0, nt)
// without spans.  A row no window reached has hi = 0: an empty span.
__device__ __forceinline__ int2 row_span(const int2* __restrict__ span, int64_t idx, int nt) {
  if (!span) return make_int2(0, nt);
  const int2 s = span[idx];
  return make_int2(kSpanBase - s.x, s.y);
}

// Blocks are dispatched to the 8 XCDs round-robin; map them so that consecutive
// logical indices share an XCD (and its L2).
__device__ __forceinline__ int xcd_remap(int b, int nblk) {
  const int q = nblk >> 3, r = nblk & 7;
  const int xcd = b & 7, pos = b >> 3;
  return xcd < r ? xcd * (q + 1) + pos : r * (q + 1) + (xcd - r) * q + pos;
}

// Column-pass block -> (chunk, event).  Events vary fastest and consecutive logical
// blocks share an XCD, so the blocks of one chunk, which read the same slice of R~, run
// together on one L2.
__device__ __forceinline__ void colpass_block(int n_events, int& ch, int& ev) {
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  ch = L / n_events;
  ev = L - ch * n_events;
}
// The same with NSUB blocks per (chunk, event), each taking one part of the chunk's
// frequencies (the parts of a chunk vary fastest).
__device__ __forceinline__ void colpass_block_sub(int n_events, int nsub, int& ch, int& ev, int& h) {
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int rest = L / nsub;
  h = L - rest * nsub;
  ch = rest / n_events;
  ev = rest - ch * n_events;
}

// 16-byte vector of the real type (4 floats or 2 doubles) for row loads: a clang vector,
// so register arrays of it stay in registers.
template <typename T>
struct Vec16 {
  static constexpr int n = 16 / sizeof(T);
  typedef T type __attribute__((ext_vector_type(16 / sizeof(T))));
};

// Noise value amp[k] * Z[k] of frequency k (of M + 1) for wire w of `event` (see NoiseArgs):
// u1 = 1 - (53-bit uniform of words 0-1) in (0, 1], u2 = uniform of words 2-3,
// r = sqrt(-2 ln u1), theta = 2 pi u2; Z = r e^{i theta} / sqrt(2), or r cos(theta) at
// k = 0 and k = M.  The transcendental functions run in the plan's precision.
__device__ __forceinline__ void sincospi_t(float x, float* s, float* c) { sincospif(x, s, c); }
__device__ __forceinline__ void sincospi_t(double x, double* s, double* c) { sincospi(x, s, c); }
template <typename T>
__device__ __forceinline__ cx<T> noise_at(const NoiseArgs<T>& nz, int k, int M, uint32_t wire, uint32_t event) {
  const Philox4 ph = philox4x32_10((uint32_t)k, wire, event, (nz.plane << 24) | kNoiseStreamBit, nz.key0, nz.key1);
  const T u1 = (T)(1.0 - uniform53(ph.w0, ph.w1));
  const T u2 = (T)uniform53(ph.w2, ph.w3);
  const T r = sqrt(T(-2) * log(u1));
  T s, c;
  sincospi_t(T(2) * u2, &s, &c);
  const T a = nz.amp[k] * r;
  if (k == 0 || k == M) return mk(a * c, T(0));
  const T h = a * T(0.70710678118654752);
  return mk(h * c, h * s);
}

// Complex value as a clang 2-vector for register arrays (aggregates there can end up in
// scratch memory).
template <typename T>
using cv2 = T __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ cv2<T> to_v(cx<T> a) {
  cv2<T> r;
  r.x = a.x;
  r.y = a.y;
  return r;
}
template <typename T>
__device__ __forceinline__ cx<T> from_v(cv2<T> a) { return mk(a.x, a.y); }

// Persistent grid: as many workgroups as fit on the device at once (LDS and waves).
inline int persistent_blocks(int n_cu, size_t lds, int threads, int work) {
  int per_cu = (int)((160 * 1024) / (lds > 0 ? lds : 1));
  const int waves = (threads + 63) / 64;
  if (per_cu * waves > 32) per_cu = 32 / waves;
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 8) per_cu = 8;
  const int g = n_cu * per_cu;
  return work < g ? work : g;
}


// Launchers of the compiled-plan kernels (conv_ct.hip), selected by plan.variant.
template <typename T>
hipError_t launch_rows_r2c_ct(const T* src, int64_t src_ev_stride, cx<T>* dst, int64_t dst_ev_stride, int nt,
                              int nphase, int nper, int nchunk, int n_events, const FftPlan& plan, const cx<T>* tw,
                              const cx<T>* post, int n_cu, hipStream_t st, const int2* span, int64_t span_ev,
                              const WireTiles& wt);
template <typename T>
hipError_t launch_colpass_ct(const cx<T>* shat, int64_t shat_ev_stride, const cx<T>* rtil, cx<T>* mhat,
                             int64_t mhat_ev_stride, int nw, int nphase, int nchunk, int n_events,
                             const FftPlan& plan, const cx<T>* tw, const cx<T>* tw_rev, hipStream_t st);
template <typename T>
hipError_t launch_colpass_adj_ct(const cx<T>* ghat, int64_t ghat_ev_stride, const cx<T>* rtil, cx<T>* hhat,
                                 int64_t hhat_ev_stride, int nw, int nphase, int nchunk, int n_events,
                                 const FftPlan& plan, const cx<T>* tw, const cx<T>* tw_rev, hipStream_t st);
template <typename T>
hipError_t launch_rows_c2r_ct(const cx<T>* src, int64_t src_ev_stride, T* dst, int64_t dst_ev_stride, int nt,
                              bool tiled, int nphase, int nper, int nchunk, int n_events, const FftPlan& plan,
                              const cx<T>* tw, const cx<T>* post, hipStream_t st, const NoiseArgs<T>& nz,
                              const WireLive& wl);
void conv_ct_init_kernels();

}  // namespace wct
