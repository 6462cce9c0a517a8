// Internal types shared by the HIP kernels and the host orchestration of libwct.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace wct {

// Complex value in plain (re, im) layout; 8 bytes in FP32, 16 in FP64.
template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T a, T b) {
  cx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> conj(cx<T> a) { return mk(a.x, -a.y); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return mk(a.x * s, a.y * s); }

// Transform plan of one length: Stockham passes with their radices and the offsets of
// their twiddles in the length's twiddle table.  Passed to kernels by value.
constexpr int kMaxPass = 16;
struct FftPlan {
  int n;
  int variant;  // index of a compiled variant with this plan, or -1 (runtime plan)
  int npass;
  int radix[kMaxPass];
  int tw_off[kMaxPass];
};

// Register budget of the LDS transforms: E = complex values one thread holds.  The
// kernels are instantiated for several E and the launcher picks the smallest E whose
// thread count fits the block; the bound keeps E values of accumulators plus one
// Stockham pass in registers without spilling.
template <typename T, int E>
struct LaunchBound {
  static constexpr int value = (E <= 8 && sizeof(T) == 4) ? 1024 : 512;
};

// Layout constants of the frequency-domain work arrays.
constexpr int kChunk = 4;  // tick frequencies per column chunk (C)

// Everything a kernel needs about one plane.
struct PlaneGeom {
  int nw, nt, I, K, TR;
  int lw, lt, M, F;   // L_w, L_t, M = L_t/2, F = M + 1
  int nchunk;         // ceil(F / kChunk)
  int nb;             // I * N_w
  int64_t grid_off;   // element offset of the plane within an event's grid
  int64_t wave_off;   // element offset within an event's waveform
  int64_t shat_off;   // complex offset within an event's S-hat work array
  int64_t mhat_off;   // complex offset within an event's M-hat work array
  int64_t tile_off;   // raster tile index offset within an event
  int64_t row_off;    // impact-row offset of the plane within an event (row flags)
  int ntr, ntc;       // raster tiles along rows and ticks
};

}  // namespace wct
