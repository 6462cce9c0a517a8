// Transform variants compiled with their plan as template parameters (see CtFft in
// fft.hpp).  One line per variant: X(kind, real type, threads per block, minimum waves
// per SIMD the registers must allow, radices...).
//  kind 0: tick rows, one sequence per block (passes A and C);
//  kind 1: wire columns, the kChunk tick frequencies of a chunk interleaved in a block;
//  kind 2: wire columns, half a chunk per block (kChunk / 2 interleaved sequences): half
//          the LDS and registers, twice the blocks.
// A plan uses the first variant whose kind, type and length match (listed fastest
// first as measured on MI355X; the tuner may pick another); lengths without a variant
// run the runtime plan.  The radices of a variant
// are its Stockham passes in order; its twiddle table is built by build_fft for them.
#pragma once

#define WCT_FFT_VARIANTS(X)                  \
  /* tick half-lengths: 5000 (9600 ticks), 3125 (6000), 625 (1024) */ \
  X(0, float, 500, 4, 5, 10, 10, 10)         \
  X(0, float, 250, 1, 5, 10, 10, 10)         \
  X(0, float, 250, 1, 25, 20, 10)            \
  X(0, float, 640, 4, 5, 5, 5, 5, 5)         \
  X(0, float, 320, 4, 5, 5, 5, 5, 5)         \
  X(0, float, 128, 1, 25, 25, 5)             \
  X(0, float, 128, 4, 5, 5, 5, 5)            \
  X(0, double, 128, 4, 5, 5, 5, 5)           \
  /* wire lengths: 2430, 3600 (2400 / 3456 wires), 810, 972 (800 / 960), 270 (256) */ \
  X(1, float, 648, 3, 9, 9, 10, 3)           \
  X(1, float, 540, 3, 9, 9, 5, 6)            \
  X(1, float, 384, 3, 27, 9, 10)             \
  X(1, float, 720, 3, 10, 9, 8, 5)           \
  X(1, float, 800, 4, 10, 10, 9, 4)          \
  X(1, float, 180, 2, 9, 9, 10)              \
  X(1, float, 360, 4, 9, 9, 10)              \
  X(1, float, 216, 2, 9, 9, 12)              \
  X(1, float, 128, 2, 9, 5, 6)               \
  X(1, double, 128, 2, 9, 5, 6)              \
  X(2, float, 540, 5, 9, 9, 10, 3)           \
  X(2, float, 320, 3, 9, 9, 10, 3)           \
  X(2, float, 480, 4, 10, 10, 9, 4)          \
  X(2, float, 360, 3, 10, 9, 8, 5)

namespace wct {

// Host-side description of a compiled variant.
struct FftVariantDesc {
  int kind;      // 0 rows, 1 columns (whole chunks), 2 columns (half chunks)
  int dbl;       // 0 float, 1 double
  int threads;   // threads per block
  int n;         // transform length
  int npass;
  int radix[8];
};

template <typename... A>
constexpr int wct_count_args(A...) { return (int)sizeof...(A); }
template <typename... A>
constexpr int wct_prod_args(A... a) { return (1 * ... * a); }

#define WCT_VARIANT_DESC(K, TT, NT, MW, ...) \
  FftVariantDesc{K, sizeof(TT) == 8, NT, wct_prod_args(__VA_ARGS__), wct_count_args(__VA_ARGS__), {__VA_ARGS__}},
inline const FftVariantDesc* fft_variants(int* count) {
  static const FftVariantDesc v[] = {WCT_FFT_VARIANTS(WCT_VARIANT_DESC)};
  *count = (int)(sizeof(v) / sizeof(v[0]));
  return v;
}
#undef WCT_VARIANT_DESC

}  // namespace wct
