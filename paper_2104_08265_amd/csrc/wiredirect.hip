// Pass B as direct sums along wires, an alternative to the wire transforms of conv.hip /
// conv_ct.hip for responses 2K+1 = 21 wires wide (arXiv:2104.08265 Eq. 1; Eq. 2 with the
// tick axis transformed only).  With the response's tick spectrum R^_t[k][i](w_t) (plan
// data, scaled by 1/L_t for the inverse tick transform of pass C),
//
//   M^(w, w_t) = sum_{k=-K..K} sum_{i<I} R^_t[k][i](w_t) S^(I (w + k) + i, w_t),
//
// rows outside the grid being zero: along wires the signal is a correlation with 2K+1
// taps per phase, which the column transforms evaluate through a length-L_w transform
// pair and a product with the full 2D spectrum R~; here it is summed as it stands.
// Work per output: (2K+1) I complex products (FP32: 840 FMAs), against the transforms'
// 10 forward and one inverse transform per (frequency, wire column) plus the read of R~
// (10 complex per output); the direct sum reads only S^ and 21 I coefficients per
// frequency.
#include "convcommon.hpp"

namespace wct {

namespace {

constexpr int kDirectK = kDirectHalfWires;  // response half-width the kernel is compiled for
constexpr int kDirectWL = 8;                // output wires per lane
constexpr int kDirectWT = 64 * kDirectWL;   // output wires per block
static_assert(kDirectWT == kDirectTileWires, "tile flags and blocks share their wires");
constexpr int kDirectSpan = kDirectWT + 2 * kDirectK;  // S^ wires staged per phase
// LDS stride of one frequency's staged wires: one pad element every kDirectWL wires, so
// that lanes reading wires kDirectWL apart hit distinct banks
constexpr int kDirectPstr = kDirectSpan + kDirectSpan / kDirectWL + 1;

}  // namespace

// One block: kChunk tick frequencies (one per wave, so a wave's coefficients are
// uniform: scalar loads) x kDirectWT consecutive wires of one (chunk, event).  Phases are
// staged through LDS in two buffers: the next phase's global loads are in flight while
// the current one is summed.
template <typename T>
__global__ void __launch_bounds__(64 * kChunk) k_colpass_direct(const cx<T>* __restrict__ shat, int64_t shat_ev_stride,
                                                               const cx<T>* __restrict__ rtick, cx<T>* __restrict__ mhat,
                                                               int64_t mhat_ev_stride, int nw, int nphase, int nchunk,
                                                               int ntile, int n_events, WireTiles wt) {
  constexpr int K = kDirectK, NK = 2 * K + 1, WL = kDirectWL, WT = kDirectWT;
  constexpr int SPAN = kDirectSpan, PSTR = kDirectPstr, C = kChunk;
  constexpr int CPV = 16 / (int)sizeof(cx<T>);  // complex values per 16-byte load
  constexpr int VPW = C / CPV;                  // 16-byte loads per staged wire
  constexpr int NE = SPAN * VPW, NPT = (NE + 64 * C - 1) / (64 * C);
  using V = typename Vec16<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);  // [2][C][PSTR]
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = L % ntile, rest = L / ntile;
  const int ev = rest % n_events, ch = rest / n_events;
  const int w0 = tile * WT;
  const int tid = (int)threadIdx.x, lane = tid & 63;
  const int f = __builtin_amdgcn_readfirstlane(tid >> 6);  // this wave's frequency in the chunk
  if (wt.live && !wt.live[ev * wt.ev_stride + tile]) {  // no row reaches the tile: M^ = 0
    cx<T>* dst = mhat + ev * mhat_ev_stride;
    for (int o = 0; o < WL; ++o) {
      const int w = w0 + WL * lane + o;
      if (w < nw) dst[(int64_t)w * (nchunk * C) + ch * C + f] = mk(T(0), T(0));
    }
    return;
  }
  const cx<T>* src = shat + ev * shat_ev_stride + (int64_t)ch * nphase * nw * C;
  // the row flags of the staged wires (rows of wires w0 - K .. w0 + WT + K), one bit each
  constexpr int kBitWords = (SPAN * 10 + 31) / 32 + 2;  // up to 10 phases
  __shared__ uint32_t s_bits[kBitWords];
  const int r_lo = max(0, w0 - K) * nphase, wd0 = r_lo >> 5;
  const bool bits = wt.rowbits != nullptr && nphase <= 10;
  if (bits) {
    const int r_hi = min(nw, w0 + WT + K) * nphase, wd1 = (r_hi + 31) >> 5;
    for (int x = tid; x < wd1 - wd0; x += 64 * C) s_bits[x] = wt.rowbits[ev * wt.bits_ev + wd0 + x];
    __syncthreads();
  }
  auto row_live = [&](int w, int i) {
    if (!bits) return true;
    const int r = w * nphase + i;
    return ((s_bits[(r >> 5) - wd0] >> (r & 31)) & 1u) != 0;
  };

  V stage[NPT];
  auto load = [&](int i) {
    const cx<T>* s = src + (int64_t)i * nw * C;
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
      const int e = tid + u * 64 * C;
      const int w = w0 - K + e / VPW;
      V v = {};
      if (e < NE && w >= 0 && w < nw && row_live(w, i)) v = *reinterpret_cast<const V*>(s + (int64_t)w * C + (e % VPW) * CPV);
      stage[u] = v;
    }
  };
  auto store = [&](int b) {
    cx<T>* d = lds + b * C * PSTR;
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
      const int e = tid + u * 64 * C;
      if (e < NE) {
        const int x = e / VPW, f0 = (e % VPW) * CPV;
#pragma unroll
        for (int q = 0; q < CPV; ++q) d[(f0 + q) * PSTR + x + x / WL] = mk(stage[u][2 * q], stage[u][2 * q + 1]);
      }
    }
  };

  T ax[WL], ay[WL];
#pragma unroll
  for (int o = 0; o < WL; ++o) ax[o] = ay[o] = T(0);
  load(0);
  store(0);
  __syncthreads();
  for (int i = 0; i < nphase; ++i) {
    if (i + 1 < nphase) load(i + 1);
    const cx<T>* coef = rtick + ((int64_t)(ch * C + f) * nphase + i) * NK;  // uniform: scalar loads
    cx<T> r[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) r[k] = coef[k];
    // staged wire x = WL lane + j (j < WL + 2K) sits at (WL + 1) lane + j + j / WL
    const cx<T>* s = lds + (i & 1) * C * PSTR + f * PSTR + (WL + 1) * lane;
#pragma unroll
    for (int j = 0; j < WL + 2 * K; ++j) {
      const cx<T> v = s[j + j / WL];
#pragma unroll
      for (int o = 0; o < WL; ++o) {
        if (j - o < 0 || j - o > 2 * K) continue;  // output wire w0 + WL lane + o, tap k = j - o - K
        const cx<T> c = r[j - o];
        ax[o] = fma(c.x, v.x, ax[o]);
        ax[o] = fma(-c.y, v.y, ax[o]);
        ay[o] = fma(c.x, v.y, ay[o]);
        ay[o] = fma(c.y, v.x, ay[o]);
      }
    }
    if (i + 1 < nphase) store((i + 1) & 1);
    __syncthreads();
  }
  cx<T>* dst = mhat + ev * mhat_ev_stride;
  const int fpad = nchunk * C;
#pragma unroll
  for (int o = 0; o < WL; ++o) {
    const int w = w0 + WL * lane + o;
    if (w < nw) dst[(int64_t)w * fpad + ch * C + f] = mk(ax[o], ay[o]);  // [w][fpad]
  }
}

// Adjoint of the direct pass: H^(I c + i, w_t) = sum_k conj(R^_t[k][i](w_t)) G^(c - k, w_t)
// (the correlation's transpose; G^ rows outside the wires are zero).  One staged window
// of G^ serves all I phases: each lane keeps its 8 + 2K values in registers and runs the
// 21 taps once per phase with that phase's coefficients.
template <typename T>
__global__ void __launch_bounds__(64 * kChunk) k_colpass_adj_direct(const cx<T>* __restrict__ ghat,
                                                                   int64_t ghat_ev_stride,
                                                                   const cx<T>* __restrict__ rtick,
                                                                   cx<T>* __restrict__ hhat, int64_t hhat_ev_stride,
                                                                   int nw, int nphase, int nchunk, int ntile,
                                                                   int n_events) {
  constexpr int K = kDirectK, NK = 2 * K + 1, WL = kDirectWL, WT = kDirectWT;
  constexpr int SPAN = kDirectSpan, PSTR = kDirectPstr, C = kChunk;
  constexpr int CPV = 16 / (int)sizeof(cx<T>);
  constexpr int VPW = C / CPV;
  constexpr int NE = SPAN * VPW;
  using V = typename Vec16<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);  // [C][PSTR]
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = L % ntile, rest = L / ntile;
  const int ev = rest % n_events, ch = rest / n_events;
  const int w0 = tile * WT;
  const int tid = (int)threadIdx.x, lane = tid & 63;
  const int f = __builtin_amdgcn_readfirstlane(tid >> 6);
  const cx<T>* src = ghat + ev * ghat_ev_stride + (int64_t)ch * nw * C;  // [chunk][wire][C]
  for (int e = tid; e < NE; e += 64 * C) {
    const int w = w0 - K + e / VPW;
    V v = {};
    if (w >= 0 && w < nw) v = *reinterpret_cast<const V*>(src + (int64_t)w * C + (e % VPW) * CPV);
    const int x = e / VPW, f0 = (e % VPW) * CPV;
#pragma unroll
    for (int q = 0; q < CPV; ++q) lds[(f0 + q) * PSTR + x + x / WL] = mk(v[2 * q], v[2 * q + 1]);
  }
  __syncthreads();
  // G^ of wires w0 + WL lane - K + j, j < WL + 2K
  cx<T> g[WL + 2 * K];
  const cx<T>* s = lds + f * PSTR + (WL + 1) * lane;
#pragma unroll
  for (int j = 0; j < WL + 2 * K; ++j) g[j] = s[j + j / WL];
  cx<T>* dst = hhat + ev * hhat_ev_stride + (int64_t)ch * nphase * nw * C;  // [chunk][i][wire][C]
  for (int i = 0; i < nphase; ++i) {
    const cx<T>* coef = rtick + ((int64_t)(ch * C + f) * nphase + i) * NK;  // uniform: scalar loads
    cx<T> r[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) r[k] = coef[k];
#pragma unroll
    for (int o = 0; o < WL; ++o) {
      // output wire c = w0 + WL lane + o takes G^(c - k) = g[o + K - k], k = -K..K
      T ax = T(0), ay = T(0);
#pragma unroll
      for (int kk = 0; kk < NK; ++kk) {
        const cx<T> c = r[kk], v = g[o + 2 * K - kk];  // conj(c) * v
        ax = fma(c.x, v.x, ax);
        ax = fma(c.y, v.y, ax);
        ay = fma(c.x, v.y, ay);
        ay = fma(-c.y, v.x, ay);
      }
      const int w = w0 + WL * lane + o;
      if (w < nw) dst[((int64_t)i * nw + w) * C + f] = mk(ax, ay);
    }
  }
}

namespace {
template <typename T>
size_t direct_lds() {
  return sizeof(cx<T>) * 2 * kChunk * kDirectPstr;
}
}  // namespace

bool colpass_direct_fits(int K) { return K == kDirectK; }

// Dynamic LDS above the default 64 KB for the direct kernels (on the current device).
void wiredirect_init_kernels() {
  const int lim = 160 * 1024 - 1024;
  (void)hipFuncSetAttribute((const void*)k_colpass_direct<float>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void*)k_colpass_direct<double>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void*)k_colpass_adj_direct<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lim);
  (void)hipFuncSetAttribute((const void*)k_colpass_adj_direct<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lim);
}

template <typename T>
hipError_t launch_colpass_direct(const cx<T>* shat, int64_t shat_ev_stride, const cx<T>* rtick, cx<T>* mhat,
                                 int64_t mhat_ev_stride, int nw, int nphase, int nchunk, int n_events, hipStream_t st,
                                 const WireTiles& wt) {
  static_assert(kChunk == 4, "one wave per frequency of a chunk");
  const int ntile = (nw + kDirectWT - 1) / kDirectWT;
  const int64_t nblk = (int64_t)nchunk * n_events * ntile;
  if (nblk <= 0) return hipSuccess;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  const size_t lds = direct_lds<T>();  // FP64: above 64 KB, allowed by wiredirect_init_kernels
  hipLaunchKernelGGL((k_colpass_direct<T>), dim3((unsigned)nblk), dim3(64 * kChunk), lds, st, shat, shat_ev_stride,
                     rtick, mhat, mhat_ev_stride, nw, nphase, nchunk, ntile, n_events, wt);
  return hipGetLastError();
}

// One block per (event, tile): whether any impact row of the tile's wires, halo included,
// holds a window (span hi != 0).
__global__ void __launch_bounds__(256) k_wire_tiles(WireTileGeom g, const int2* __restrict__ span,
                                                     uint8_t* __restrict__ live) {
  const int ev = blockIdx.x / g.tiles_ev;
  int t = blockIdx.x - ev * g.tiles_ev;
  int p = 0;
  while (p + 1 < g.n_planes && t >= g.tile_off[p + 1]) ++p;
  t -= g.tile_off[p];
  const int wlo = max(0, t * kDirectWT - kDirectK), whi = min(g.nw[p], (t + 1) * kDirectWT + kDirectK);
  const int2* f = span + (int64_t)ev * g.rows_ev + g.row_off[p];
  int any = 0;
  for (int r = wlo * g.I[p] + (int)threadIdx.x; r < whi * g.I[p]; r += 256) any |= f[r].y != 0;
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) live[blockIdx.x] = (uint8_t)(any != 0);
}

// One thread per (event, wire): whether any impact row of wires w - K .. w + K (inside
// the plane) holds a window (span hi != 0).
__global__ void __launch_bounds__(256) k_wire_live(WireTileGeom g, int64_t n, const int2* __restrict__ span,
                                                    uint8_t* __restrict__ live) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const int ev = (int)(x / g.wires_ev);
    int w = (int)(x - (int64_t)ev * g.wires_ev);
    int p = 0;
    while (p + 1 < g.n_planes && w >= g.wire_off[p + 1]) ++p;
    w -= g.wire_off[p];
    const int wlo = max(0, w - g.K[p]), whi = min(g.nw[p], w + g.K[p] + 1);
    const int2* f = span + (int64_t)ev * g.rows_ev + g.row_off[p];
    int any = 0;
    for (int r = wlo * g.I[p]; r < whi * g.I[p] && !any; ++r) any = f[r].y != 0;
    live[x] = (uint8_t)any;
  }
}

// One thread per (event, 32-row word): bit j set when row 32 word + j of the plane holds a
// window (span hi != 0).
__global__ void __launch_bounds__(256) k_row_bits(WireTileGeom g, int64_t n, const int2* __restrict__ span,
                                                   uint32_t* __restrict__ bits) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const int ev = (int)(x / g.bits_ev);
    int wd = (int)(x - (int64_t)ev * g.bits_ev);
    int p = 0;
    while (p + 1 < g.n_planes && wd >= g.bit_off[p + 1]) ++p;
    wd -= g.bit_off[p];
    const int nb = g.nw[p] * g.I[p];
    const int2* f = span + (int64_t)ev * g.rows_ev + g.row_off[p];
    uint32_t v = 0;
    for (int j = 0; j < 32; ++j) {
      const int r = wd * 32 + j;
      if (r < nb && f[r].y != 0) v |= 1u << j;
    }
    bits[x] = v;
  }
}

hipError_t launch_row_bits(const WireTileGeom& g, int n_events, const int2* span, uint32_t* bits, hipStream_t st) {
  const int64_t n = (int64_t)n_events * g.bits_ev;
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  hipLaunchKernelGGL(k_row_bits, dim3((unsigned)blocks), dim3(256), 0, st, g, n, span, bits);
  return hipGetLastError();
}

hipError_t launch_wire_live(const WireTileGeom& g, int n_events, const int2* span, uint8_t* live, hipStream_t st) {
  const int64_t n = (int64_t)n_events * g.wires_ev;
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  hipLaunchKernelGGL(k_wire_live, dim3((unsigned)blocks), dim3(256), 0, st, g, n, span, live);
  return hipGetLastError();
}

hipError_t launch_wire_tiles(const WireTileGeom& g, int n_events, const int2* span, uint8_t* live, hipStream_t st) {
  if (n_events <= 0 || g.tiles_ev <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_wire_tiles, dim3((unsigned)(n_events * g.tiles_ev)), dim3(256), 0, st, g, span, live);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_colpass_adj_direct(const cx<T>* ghat, int64_t ghat_ev_stride, const cx<T>* rtick, cx<T>* hhat,
                                     int64_t hhat_ev_stride, int nw, int nphase, int nchunk, int n_events,
                                     hipStream_t st) {
  const int ntile = (nw + kDirectWT - 1) / kDirectWT;
  const int64_t nblk = (int64_t)nchunk * n_events * ntile;
  if (nblk <= 0) return hipSuccess;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  const size_t lds = direct_lds<T>() / 2;  // one buffer
  hipLaunchKernelGGL((k_colpass_adj_direct<T>), dim3((unsigned)nblk), dim3(64 * kChunk), lds, st, ghat,
                     ghat_ev_stride, rtick, hhat, hhat_ev_stride, nw, nphase, nchunk, ntile, n_events);
  return hipGetLastError();
}

template hipError_t launch_colpass_adj_direct<float>(const cx<float>*, int64_t, const cx<float>*, cx<float>*, int64_t,
                                                     int, int, int, int, hipStream_t);
template hipError_t launch_colpass_adj_direct<double>(const cx<double>*, int64_t, const cx<double>*, cx<double>*,
                                                      int64_t, int, int, int, int, hipStream_t);
template hipError_t launch_colpass_direct<float>(const cx<float>*, int64_t, const cx<float>*, cx<float>*, int64_t, int,
                                                 int, int, int, hipStream_t, const WireTiles&);
template hipError_t launch_colpass_direct<double>(const cx<double>*, int64_t, const cx<double>*, cx<double>*, int64_t,
                                                  int, int, int, int, hipStream_t, const WireTiles&);

}  // namespace wct
