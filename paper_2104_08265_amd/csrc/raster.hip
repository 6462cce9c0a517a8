// Rasterisation and scatter adding of depositions (arXiv:2104.08265 Sec. 2.1.1):
// every depo-plane row becomes a patch of clipped Gaussian bin integrals Q*A_b*B_k
// (or binomial electron counts, Sec. 4.3.1) that is added into its plane's grid.
//
// Scatter adding goes through LDS-privatised tiles of TH x TW cells:
//  1. k_count    - each row counts the tiles its window overlaps (<= 4; wider rows go
//                  to a separate list handled in 64 x 64 chunks with global atomics, k_big)
//                  and keeps the value each increment returns, its slot in that tile's
//                  row list; optionally it marks the impact rows its window reaches;
//  2. scan       - exclusive prefix sums give each tile its slice of a row list and
//                  a number of work items (ceil(rows / kRowsPerItem); 0 for an empty tile);
//  3. k_fill     - rows are written into their tiles' slices at their slots (plain stores);
//  4. k_tile     - a persistent kernel takes, in step, a work item and a group of
//                  kZeroGroup consecutive tiles from two atomic queues; a work item
//                  accumulates its rows' in-tile sub-patches with LDS atomics and then
//                  writes the tile: plain stores when the tile has one item, global atomic
//                  adds when a crowded tile was split across items (those tiles are cleared
//                  first by k_zero_split); a group's tiles that no row touches are cleared
//                  with plain stores, so the grid needs no separate clearing.
// Window bounds are formed in FP64 exactly as the oracle forms them, so both sides
// agree on which cells a row touches; fluctuated counts use the deterministic
// Philox + binomial chain of fluct.hpp (this file is compiled with contraction off).
#include <type_traits>

#include "kernels.hpp"

namespace wct {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct RowWin {
  double q, u, su, t, st;
  double ulo, uhi, tlo, thi;
  int b0, b1, k0, k1;  // cell ranges clipped to the grid, [b0, b1) x [k0, k1)
  int plane, event;  // event: slot in this call's grids (id - event_base)
  int key_event;     // event id (fluctuation counter word 2)
  bool ok;
};

__device__ __forceinline__ int clamp_idx(double v) {
  v = fmin(fmax(v, -1.0e9), 1.0e9);
  return (int)v;
}

template <typename T>
__device__ __forceinline__ RowWin row_window(const DepoView<T>& d, int64_t j, const RasterGeom& g, double nsigma) {
  RowWin w;
  w.plane = d.plane ? d.plane[j] : 0;
  w.key_event = d.event ? d.event[j] : 0;
  w.event = w.key_event - g.event_base;
  w.ok = w.plane >= 0 && w.plane < g.n_planes && w.key_event >= 0 && w.event >= 0 && w.event < g.n_events;
  if (!w.ok) return w;
  const PlaneGeom& pl = g.pl[w.plane];
  w.q = (double)d.q[j];
  const double p = (double)d.p[j];
  const double sp = (double)d.sp[j];
  w.t = (double)d.t[j];
  w.st = (double)d.st[j];
  w.ok = (w.q >= 0.0) && (w.st > 0.0) && (sp > 0.0) && isfinite(w.q) && isfinite(w.t) && isfinite(p) &&
         isfinite(w.st) && isfinite(sp);
  if (!w.ok) return w;
  w.u = (double)pl.I * p;
  w.su = (double)pl.I * sp;
  const double hu = nsigma * w.su;
  w.ulo = w.u - hu;
  w.uhi = w.u + hu;
  const double ht = nsigma * w.st;
  w.tlo = w.t - ht;
  w.thi = w.t + ht;
  w.b0 = max(clamp_idx(floor(w.ulo)), 0);
  w.b1 = min(clamp_idx(ceil(w.uhi)), pl.nb);
  w.k0 = max(clamp_idx(floor(w.tlo)), 0);
  w.k1 = min(clamp_idx(ceil(w.thi)), pl.nt);
  w.ok = w.b0 < w.b1 && w.k0 < w.k1;
  return w;
}

__device__ __forceinline__ int find_plane(const RasterGeom& g, int tin) {
  int p = 0;
  for (int k = 1; k < g.n_planes; ++k)
    if (tin >= g.pl[k].tile_off) p = k;
  return p;
}

// Erf at the cell edges of [k0, k1) for a window (lo, hi) around mu: edge 0 = max(k0, lo),
// edge n = min(k1, hi), interior edges the integers between.  A cell's weight (the
// Gaussian's integral over its part inside the window) is then 0.5 (e[x+1] - e[x]),
// computed from the same doubles the oracle uses, with one erf per edge.
// Both axes of a patch share one pass over the lanes: the impact edges [b0, b1] first,
// then the tick edges [k0, k1] (a short tick window would leave most lanes idle in a
// pass of its own).
template <int MODE>
__device__ __forceinline__ void edge_fill2(double* __restrict__ ea, int b0, int b1, double mua, double siga,
                                           double loa, double hia, double* __restrict__ eb, int k0, int k1,
                                           double mub, double sigb, double lob, double hib, int lane) {
  const int na = b1 - b0, nb = k1 - k0;
  const double s2a = siga * kSqrt2, s2b = sigb * kSqrt2;
  for (int x = lane; x <= na + 1 + nb; x += 64) {
    const bool a = x <= na;
    const int i = a ? x : x - (na + 1), n = a ? na : nb, c0 = a ? b0 : k0, c1 = a ? b1 : k1;
    const double lo = a ? loa : lob, hi = a ? hia : hib, mu = a ? mua : mub, s2 = a ? s2a : s2b;
    const double edge = i == 0 ? fmax((double)c0, lo) : (i == n ? fmin((double)c1, hi) : (double)(c0 + i));
    const double v = MODE != kModeMean ? det_erf((edge - mu) / s2) : erf((edge - mu) / s2);
    (a ? ea : eb)[i] = v;
  }
}
__device__ __forceinline__ double edge_weight(const double* e, int x) { return 0.5 * (e[x + 1] - e[x]); }

// x / d for 0 <= x < 2^22 without an integer divide (float reciprocal, then corrected).
__device__ __forceinline__ int div_small(int x, int d, float rd) {
  int q = (int)((float)x * rd);
  if (q * d > x) --q;
  else if ((q + 1) * d <= x) ++q;
  return q;
}

// Cells whose count needs the full sampler wait in per-wave queues, one per regime of the
// sampler (inversion, chop-down), so that a batch of 64 runs one regime's code with all
// lanes instead of every wave diverging over both.  Cells whose count follows from the
// cheap tests (p = 0, p = 1, or the exact zero bound) never enter them.
//
// A queue lives in registers: position e (< 128) is held by lane e & 63 in slot e >> 6.
// A push moves each new entry to its lane with one ds_permute per 32-bit word; a run
// takes slot 0 (positions 0..63) and slot 1 moves down.  The queues are emptied at the
// end of every row's sub-patch, so a batch shares the row's electron count N (a
// wave-uniform value: the sampler's power loop then runs under scalar control).

__device__ __forceinline__ int lanes_below(uint64_t mask, int lane) {
  return __popcll(mask & ((1ull << lane) - 1ull));
}

__device__ __forceinline__ uint32_t lo32(double v) { return (uint32_t)__double_as_longlong(v); }
__device__ __forceinline__ uint32_t hi32(double v) { return (uint32_t)((uint64_t)__double_as_longlong(v) >> 32); }
__device__ __forceinline__ double mkd(uint32_t lo, uint32_t hi) {
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ uint32_t permute_to(int lane_dst, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_ds_permute(lane_dst << 2, (int)v);
}

struct RegQueue {
  double p0, u0, p1, u1;  // probability and uniform of the entries in slot 0 / slot 1
  uint32_t d0, d1;        // their tile offsets
  int n;                  // entries (wave-uniform)
};

__device__ __forceinline__ void rq_push(RegQueue& q, bool need, double p, double u, uint32_t dst, int lane) {
  const uint64_t mask = __ballot(need);
  const int cnt = __popcll(mask);
  if (cnt == 0) return;
  // new entries go to positions n .. n+cnt-1; the other lanes fill the rest of the
  // rotation so that every lane sends and receives exactly one value
  const int below = lanes_below(mask, lane);
  const int t = need ? below : cnt + (lane - below);
  const int to = (q.n + t) & 63;
  const double rp = mkd(permute_to(to, lo32(p)), permute_to(to, hi32(p)));
  const double ru = mkd(permute_to(to, lo32(u)), permute_to(to, hi32(u)));
  const uint32_t rd = permute_to(to, dst);
  const int off = (lane - q.n) & 63;
  if (off < cnt) {
    if (((q.n + off) >> 6) == 0) {
      q.p0 = rp;
      q.u0 = ru;
      q.d0 = rd;
    } else {
      q.p1 = rp;
      q.u1 = ru;
      q.d1 = rd;
    }
  }
  q.n += cnt;
}

// Samples slot 0 (lanes below `take`) with regime REGIME, then moves slot 1 down.
template <typename T, int REGIME, typename Add>
__device__ __forceinline__ void rq_run(RegQueue& q, int take, int N, double lfN, int lane, const DetTablesSmall& tb,
                                       const double* __restrict__ lf, Add add) {
  if (lane < take) {
    const int k = binom_regime_draw<REGIME>(N, lfN, q.p0, q.u0, tb, lf);
    if (k) add(q.d0, (T)k);
  }
  q.p0 = q.p1;
  q.u0 = q.u1;
  q.d0 = q.d1;
  q.n -= take;
}

// The chop-down queue may outlive a row: the tile kernel keeps one per wave for a whole
// work item, so that its batches fill up across rows.  Its entries then carry their
// row's electron count in the bits of the offset above kDstBits (tile offsets are below
// 2^13); a count of 0 there stands for `rowN`, the count of the row being rasterised,
// which is how rows with 2^19 or more electrons (and the wide-row kernel, whose offsets
// need all the bits) enqueue: such a row empties the queue when it ends.
constexpr int kDstBits = 13;
constexpr int kPackN = 1 << (32 - kDstBits);

template <typename T, typename Add>
__device__ __forceinline__ void rq_run_chop(RegQueue& q, int take, int rowN, bool packed, int lane,
                                            const DetTablesSmall& tb, const double* __restrict__ lf, Add add) {
  if (lane < take) {
    const uint32_t e = q.d0;
    const int fieldN = packed ? (int)(e >> kDstBits) : 0;
    const int N = fieldN ? fieldN : rowN;
    const uint32_t d = packed ? (e & ((1u << kDstBits) - 1u)) : e;
    const int k = binom_regime_draw<1>(N, lfact_of(N, lf, tb), q.p0, q.u0, tb, lf);
    if (k) add(d, (T)k);
  }
  q.p0 = q.p1;
  q.u0 = q.u1;
  q.d0 = q.d1;
  q.n -= take;
}

// A cell's outcome of the cheap tests: added at once, queued for its regime, or nothing.
// `tagN` is what the chop-down entry carries (the row's count, or 0 for `rowN`).
template <typename T, typename Add>
__device__ __forceinline__ void cell_route(RegQueue& qi, RegQueue& qc, bool packed, int tagN, int quick,
                                           double p, double u, int N, double lfN, uint32_t dst, int lane,
                                           const DetTablesSmall& tb, const double* __restrict__ lf, Add add) {
  if (quick > 0) add(dst, (T)quick);
  rq_push(qi, quick == -1, p, u, dst, lane);
  if (qi.n >= 64) rq_run<T, 0>(qi, 64, N, lfN, lane, tb, lf, add);
  rq_push(qc, quick == -2, p, u, packed ? dst | ((uint32_t)tagN << kDstBits) : dst, lane);
  if (qc.n >= 64) rq_run_chop<T>(qc, 64, N, packed, lane, tb, lf, add);
}

// One wave rasterises the cells [b0, b1) x [k0, k1) of a row; `dst(b, k)` names a cell and
// `add(dst, value)` accumulates a nonzero contribution.  Fluctuated cells are drawn in
// tick pairs: cells (b, 2m), (b, 2m+1) share one Philox4x32-10 block (counter
// b*ceil(N_t/2) + m), words 0-1 for the even tick and 2-3 for the odd one.
// PACKED: `qc` is the caller's chop-down queue of a whole work item (entries carry their
// count; the caller empties it at the item's end); otherwise it is emptied here.
template <typename T, int MODE, bool PACKED, typename Dst, typename Add>
__device__ __forceinline__ void patch_cells(const RowWin& w, int b0, int b1, int k0, int k1, int nt, uint32_t did,
                                            uint32_t ev, uint32_t plane, uint32_t key0, uint32_t key1,
                                            double* __restrict__ ea, double* __restrict__ eb,
                                            const DetTablesSmall& tb, const double* __restrict__ lf, int lane, Dst dst,
                                            Add add, RegQueue& qc) {
  const int nbr = b1 - b0, nkr = k1 - k0;
  edge_fill2<MODE>(ea, b0, b1, w.u, w.su, w.ulo, w.uhi, eb, k0, k1, w.t, w.st, w.tlo, w.thi, lane);
  wave_sync();
  if (MODE == kModeNormal) {
    // each cell's count from its own normal: no search, no queue
    const int N = __builtin_amdgcn_readfirstlane((int)floor(fmin(w.q + 0.5, 2147483647.0)));
    if (N > 0) {
      const int j0 = k0 >> 1, np = ((k1 - 1) >> 1) - j0 + 1;
      const uint32_t half_nt = (uint32_t)((nt + 1) >> 1);
      const float rd = 1.0f / (float)np;
      for (int x = lane; x < nbr * np; x += 64) {
        const int bi = div_small(x, np, rd), pj = x - bi * np;
        const int b = b0 + bi, m = j0 + pj;
        const Philox4 ph = philox4x32_10((uint32_t)b * half_nt + (uint32_t)m, did, ev, plane << 24, key0, key1);
        double ze, zo;
        box_muller_pair(ph, &ze, &zo);
        const double a = edge_weight(ea, bi);
        const int ke = 2 * m, ko = 2 * m + 1;
        if (ke >= k0) {
          const int n = normal_count(N, a * edge_weight(eb, ke - k0), ze);
          if (n > 0) add(dst(b, ke), (T)n);
        }
        if (ko < k1) {
          const int n = normal_count(N, a * edge_weight(eb, ko - k0), zo);
          if (n > 0) add(dst(b, ko), (T)n);
        }
      }
    }
  } else if (MODE == kModeMean) {
    const float rd = 1.0f / (float)nkr;
    for (int x = lane; x < nbr * nkr; x += 64) {
      const int bi = div_small(x, nkr, rd), ki = x - bi * nkr;
      add(dst(b0 + bi, k0 + ki), (T)(w.q * (edge_weight(ea, bi) * edge_weight(eb, ki))));
    }
  } else {
    // the row's electron count, wave-uniform (counts are 32-bit: charges from 2^31 - 1
    // electrons up draw as 2^31 - 1)
    const int N = __builtin_amdgcn_readfirstlane((int)floor(fmin(w.q + 0.5, 2147483647.0)));
    if (N > 0) {
      const double lfN = lfact_of(N, lf, tb);
      const int tagN = N < kPackN ? N : 0;  // 0: the entry stands for this row's count
      RegQueue qi;
      qi.n = 0;
      const int j0 = k0 >> 1, np = ((k1 - 1) >> 1) - j0 + 1;
      const uint32_t half_nt = (uint32_t)((nt + 1) >> 1);
      const float rd = 1.0f / (float)np;
      const int total = nbr * np;
      for (int base = 0; base < total; base += 64) {
        const int x = base + lane;
        int quick_e = 0, quick_o = 0;
        double pe = 0.0, po = 0.0, ue = 0.0, uo = 0.0;
        uint32_t de = 0, dodd = 0;
        if (x < total) {
          const int bi = div_small(x, np, rd), pj = x - bi * np;
          const int b = b0 + bi, m = j0 + pj;
          const Philox4 ph = philox4x32_10((uint32_t)b * half_nt + (uint32_t)m, did, ev, plane << 24, key0, key1);
          const double a = edge_weight(ea, bi);
          const int ke = 2 * m, ko = 2 * m + 1;
          if (ke >= k0) {
            pe = a * edge_weight(eb, ke - k0);
            ue = uniform53(ph.w0, ph.w1);
            de = dst(b, ke);
            quick_e = binom_quick(N, pe, ue);
          }
          if (ko < k1) {
            po = a * edge_weight(eb, ko - k0);
            uo = uniform53(ph.w2, ph.w3);
            dodd = dst(b, ko);
            quick_o = binom_quick(N, po, uo);
          }
        }
        cell_route<T>(qi, qc, PACKED, tagN, quick_e, pe, ue, N, lfN, de, lane, tb, lf, add);
        cell_route<T>(qi, qc, PACKED, tagN, quick_o, po, uo, N, lfN, dodd, lane, tb, lf, add);
      }
      if (qi.n > 0) rq_run<T, 0>(qi, qi.n, N, lfN, lane, tb, lf, add);
      // entries that stand for this row's count cannot outlive it
      if ((!PACKED || tagN == 0) && qc.n > 0) rq_run_chop<T>(qc, qc.n, N, PACKED, lane, tb, lf, add);
    }
  }
  wave_sync();
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// 1. tiles per row ---------------------------------------------------------
// A row's slot in a tile's row list is the tile counter's value before its increment,
// kept in rank[4 j + n] (n-th tile of row j, rows of tiles outer), so the list fill
// needs no second pass of atomics.  The block first counts its rows per tile in an LDS
// table (open addressing: 2048 slots for at most 4 x 256 tiles, so every probe sequence
// ends at a free or matching slot) and then makes one global atomic add per distinct
// tile: rows of a shower or a track that share tiles no longer queue on one counter.
constexpr int kCountBlock = 256;
constexpr int kCountSlots = 2048;
template <typename T, int TH, int TW>
__global__ void __launch_bounds__(kCountBlock) k_count(DepoView<T> d, RasterGeom g, double nsigma,
                                                       int32_t* __restrict__ counts, int32_t* __restrict__ rank,
                                                       int32_t* __restrict__ big, int32_t* __restrict__ ctrl,
                                                       int2* __restrict__ span, int2* __restrict__ hull) {
  static_assert(kCountSlots > 4 * kCountBlock && (kCountSlots & (kCountSlots - 1)) == 0, "count table size");
  __shared__ int32_t s_key[kCountSlots];  // tile index, -1 = free
  __shared__ int32_t s_cnt[kCountSlots];  // rows of this block in the tile, then their first slot
  __shared__ int32_t s_pack[4 * kCountBlock];  // per (thread, n): table slot | (rank in the block) << 11
  for (int e = threadIdx.x; e < kCountSlots; e += kCountBlock) {
    s_key[e] = -1;
    s_cnt[e] = 0;
  }
  __syncthreads();
  const int64_t j = blockIdx.x * (int64_t)kCountBlock + threadIdx.x;
  int nt = 0;
  if (j < d.n) {
    const RowWin w = row_window(d, j, g, nsigma);
    if (w.ok) {
      const PlaneGeom& pl = g.pl[w.plane];
      const int tr0 = w.b0 / TH, tr1 = (w.b1 - 1) / TH, tc0 = w.k0 / TW, tc1 = (w.k1 - 1) / TW;
      const bool wide = (tr1 - tr0 + 1) * (tc1 - tc0 + 1) > 4;
      if (span) {
        // The impact rows this window reaches are marked (span hi >= 1); they get their
        // band's tile hull afterwards (k_band_spans).  Test first, so that neighbouring
        // depositions do not contend.  A wide row, which no tile counts, widens the hulls
        // of its bands itself (these rows are few).
        int2* f = span + (int64_t)w.event * g.rows_ev + pl.row_off;
        for (int b = w.b0; b < w.b1; ++b)
          if (f[b].y == 0) atomicMax(&f[b].y, 1);
        if (wide) {
          int bands_ev = 0;
          for (int q = 0; q < g.n_planes; ++q) bands_ev += g.pl[q].ntr;
          int2* h = hull + (int64_t)w.event * bands_ev + bands_before(g, w.plane);
          for (int tr = tr0; tr <= tr1; ++tr) {
            atomicMax(&h[tr].x, kSpanBase - tc0);
            atomicMax(&h[tr].y, tc1 + 1);
          }
        }
      }
      if (wide) {
        big[atomicAdd(&ctrl[kCtrlNBig], 1)] = (int32_t)j;
      } else {
        const int64_t base = (int64_t)w.event * g.ntiles_ev + pl.tile_off;
        for (int tr = tr0; tr <= tr1; ++tr)
          for (int tc = tc0; tc <= tc1; ++tc) {
            const int32_t key = (int32_t)(base + (int64_t)tr * pl.ntc + tc);
            uint32_t h = ((uint32_t)key * 2654435761u) >> 21;  // 11 bits
            for (int probe = 0; probe < kCountSlots; ++probe) {
              const int32_t old = atomicCAS(&s_key[h], -1, key);
              if (old == -1 || old == key) break;
              h = (h + 1) & (kCountSlots - 1);
            }
            const int loc = atomicAdd(&s_cnt[h], 1);
            s_pack[4 * threadIdx.x + nt++] = (int32_t)h | (loc << 11);
          }
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kCountSlots; e += kCountBlock) {
    const int c = s_cnt[e];
    if (c > 0) s_cnt[e] = atomicAdd(&counts[s_key[e]], c);
  }
  __syncthreads();
  for (int n = 0; n < nt; ++n) {
    const int32_t pk = s_pack[4 * threadIdx.x + n];
    rank[4 * j + n] = s_cnt[pk & (kCountSlots - 1)] + (pk >> 11);
  }
}

// 1b. row tick spans from the tiles (wct_simulate) -----------------------------
// One block per band of TH impact rows (one tile row of a plane): the band's tiles that
// some row reaches (a tile row's count, or a wide row's window) form the hull of tile
// columns [lo, hi]; ticks [TW lo, TW (hi + 1)) hold every nonzero cell of the band, so the
// band's marked rows take that span.  The hull is kept ({2^30 - lo, hi + 1}) for the tile
// kernel, which clears only the empty tiles inside it: the row transform reads nothing
// else.  Rows no window reached keep {0, 0}.
template <int TH, int TW>
__global__ void __launch_bounds__(256) k_band_spans(RasterGeom g, const int32_t* __restrict__ counts,
                                                     int bands_ev, int2* __restrict__ span, int2* __restrict__ hull) {
  __shared__ int s_lo[4], s_hi[4];
  const int ev = blockIdx.x / bands_ev;
  int bin = blockIdx.x - ev * bands_ev;
  int p = 0;
  while (p + 1 < g.n_planes && bin >= g.pl[p].ntr) bin -= g.pl[p++].ntr;
  const PlaneGeom& pl = g.pl[p];
  const int tr = bin;
  const int32_t* cnt = counts + (int64_t)ev * g.ntiles_ev + pl.tile_off + (int64_t)tr * pl.ntc;
  int lo = INT_MAX, hi = -1;
  for (int tc = threadIdx.x; tc < pl.ntc; tc += 256)
    if (cnt[tc] > 0) {
      lo = min(lo, tc);
      hi = max(hi, tc);
    }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = min(lo, __shfl_xor(lo, o, 64));
    hi = max(hi, __shfl_xor(hi, o, 64));
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_lo[wv] = lo;
    s_hi[wv] = hi;
  }
  __syncthreads();
  lo = min(min(s_lo[0], s_lo[1]), min(s_lo[2], s_lo[3]));
  hi = max(max(s_hi[0], s_hi[1]), max(s_hi[2], s_hi[3]));
  int2* hb = hull + blockIdx.x;  // [event][band]: blockIdx.x = ev * bands_ev + band
  const int2 wide = *hb;         // the wide rows' tile columns, {2^30 - lo, hi + 1} or {0, 0}
  if (wide.y > 0) {
    lo = min(lo, kSpanBase - wide.x);
    hi = max(hi, wide.y - 1);
  }
  __syncthreads();  // every thread has read the wide rows' hull
  if (threadIdx.x == 0) *hb = hi >= 0 ? make_int2(kSpanBase - lo, hi + 1) : make_int2(0, 0);
  const int klo = hi >= 0 ? lo * TW : 0, khi = hi >= 0 ? min((hi + 1) * TW, pl.nt) : 0;
  int2* f = span + (int64_t)ev * g.rows_ev + pl.row_off;
  const int b1 = min((tr + 1) * TH, pl.nb);
  for (int b = tr * TH + threadIdx.x; b < b1; b += 256)
    if (f[b].y != 0) f[b] = make_int2(kSpanBase - klo, khi);
}

// 2. scan of (rows, items) per tile -------------------------------------------
// Tiles no row touches get no work item: the tile kernel clears them in groups.
__device__ __forceinline__ int items_of(int c) { return (c + kRowsPerItem - 1) / kRowsPerItem; }

// Inclusive block scan of int2 over 1024 threads (16 waves of 64).
__device__ int2 block_scan_incl(int2 v, int2* s_wave) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int ax = __shfl_up(v.x, o, 64), ay = __shfl_up(v.y, o, 64);
    if (lane >= o) {
      v.x += ax;
      v.y += ay;
    }
  }
  if (lane == 63) s_wave[wv] = v;
  __syncthreads();
  if (wv == 0) {
    const int nw = blockDim.x >> 6;
    int2 t = lane < nw ? s_wave[lane] : make_int2(0, 0);
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int ax = __shfl_up(t.x, o, 64), ay = __shfl_up(t.y, o, 64);
      if (lane >= o) {
        t.x += ax;
        t.y += ay;
      }
    }
    if (lane < nw) s_wave[lane] = t;
  }
  __syncthreads();
  if (wv > 0) {
    v.x += s_wave[wv - 1].x;
    v.y += s_wave[wv - 1].y;
  }
  return v;
}

__global__ void __launch_bounds__(1024) k_scan_local(const int32_t* __restrict__ counts, int64_t n,
                                                     int2* __restrict__ blocks) {
  __shared__ int2 s_wave[16];
  const int64_t base = (int64_t)blockIdx.x * kScanPerBlock + threadIdx.x * 4;
  int2 s = make_int2(0, 0);
  for (int e = 0; e < 4; ++e)
    if (base + e < n) {
      const int c = counts[base + e];
      s.x += c;
      s.y += items_of(c);
    }
  const int2 incl = block_scan_incl(s, s_wave);
  if (threadIdx.x == blockDim.x - 1) blocks[blockIdx.x] = incl;
}

__global__ void __launch_bounds__(1024) k_scan_blocks(int2* __restrict__ blocks, int nblocks,
                                                      int32_t* __restrict__ ctrl) {
  __shared__ int2 s_wave[16];
  __shared__ int2 s_carry;
  if (threadIdx.x == 0) s_carry = make_int2(0, 0);
  __syncthreads();
  for (int b0 = 0; b0 < nblocks; b0 += blockDim.x) {
    const int b = b0 + threadIdx.x;
    const int2 v = b < nblocks ? blocks[b] : make_int2(0, 0);
    const int2 incl = block_scan_incl(v, s_wave);
    const int2 carry = s_carry;
    if (b < nblocks) blocks[b] = make_int2(carry.x + incl.x - v.x, carry.y + incl.y - v.y);  // exclusive
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) s_carry = make_int2(carry.x + incl.x, carry.y + incl.y);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    ctrl[kCtrlTotal] = s_carry.x;
    ctrl[kCtrlNItems] = s_carry.y;
  }
}

__global__ void __launch_bounds__(1024) k_scan_apply(const int32_t* __restrict__ counts, int64_t n,
                                                     const int2* __restrict__ blocks, int32_t* __restrict__ offs,
                                                     int32_t* __restrict__ item_off) {
  __shared__ int2 s_wave[16];
  const int64_t base = (int64_t)blockIdx.x * kScanPerBlock + threadIdx.x * 4;
  int c[4];
  int2 s = make_int2(0, 0);
  for (int e = 0; e < 4; ++e) {
    c[e] = base + e < n ? counts[base + e] : 0;
    s.x += c[e];
    s.y += base + e < n ? items_of(c[e]) : 0;
  }
  const int2 incl = block_scan_incl(s, s_wave);
  const int2 bo = blocks[blockIdx.x];
  int2 run = make_int2(bo.x + incl.x - s.x, bo.y + incl.y - s.y);
  for (int e = 0; e < 4; ++e) {
    const int64_t t = base + e;
    if (t < n) {
      offs[t] = run.x;
      item_off[t] = run.y;
      run.x += c[e];
      run.y += items_of(c[e]);
      if (t == n - 1) {
        offs[n] = run.x;
        item_off[n] = run.y;
      }
    }
  }
}

// 3. rows into tile slices; 4a. item -> tile map; 4b. clear split tiles -------
template <typename T, int TH, int TW>
__global__ void k_fill(DepoView<T> d, RasterGeom g, double nsigma, const int32_t* __restrict__ offs,
                       const int32_t* __restrict__ rank, int32_t* __restrict__ list) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= d.n) return;
  const RowWin w = row_window(d, j, g, nsigma);
  if (!w.ok) return;
  const PlaneGeom& pl = g.pl[w.plane];
  const int tr0 = w.b0 / TH, tr1 = (w.b1 - 1) / TH, tc0 = w.k0 / TW, tc1 = (w.k1 - 1) / TW;
  if ((tr1 - tr0 + 1) * (tc1 - tc0 + 1) > 4) return;
  const int64_t base = (int64_t)w.event * g.ntiles_ev + pl.tile_off;
  int n = 0;
  for (int tr = tr0; tr <= tr1; ++tr)
    for (int tc = tc0; tc <= tc1; ++tc) {
      const int64_t t = base + (int64_t)tr * pl.ntc + tc;
      list[offs[t] + rank[4 * j + n++]] = (int32_t)j;
    }
}

__global__ void k_items(const int32_t* __restrict__ item_off, int64_t ntiles, int32_t* __restrict__ items) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  for (int k = item_off[t]; k < item_off[t + 1]; ++k) items[k] = (int32_t)t;
}

// Writes zeros over tile t of the grid with the block's threads: 16-byte stores when the
// tile's rows start on 16-byte boundaries, element stores otherwise.
template <typename T, int TH, int TW>
__device__ __forceinline__ void zero_tile(const RasterGeom& g, int64_t t, T* __restrict__ grid) {
  constexpr int V = 16 / (int)sizeof(T);
  static_assert(TW % V == 0, "tile width must be a whole number of 16-byte vectors");
  const int ev = (int)(t / g.ntiles_ev);
  const int tin = (int)(t - (int64_t)ev * g.ntiles_ev);
  const PlaneGeom& pl = g.pl[find_plane(g, tin)];
  const int tl = tin - pl.tile_off;
  const int tr = tl / pl.ntc, tc = tl - (tl / pl.ntc) * pl.ntc;
  const int tb0 = tr * TH, tk0 = tc * TW;
  const int th = min(TH, pl.nb - tb0), tw = min(TW, pl.nt - tk0);
  T* gp = grid + (int64_t)ev * g.grid_ev_stride + pl.grid_off + (int64_t)tb0 * pl.nt + tk0;
  if (tw == TW && pl.nt % V == 0 && (reinterpret_cast<uintptr_t>(gp) & 15) == 0) {
    constexpr int VR = TW / V;  // vectors per tile row
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int x = threadIdx.x; x < th * VR; x += blockDim.x) {
      const int r = x / VR, c = x - (x / VR) * VR;
      *reinterpret_cast<float4*>(gp + (int64_t)r * pl.nt + c * V) = z;
    }
  } else {
    for (int x = threadIdx.x; x < th * TW; x += blockDim.x) {
      const int r = x / TW, c = x - (x / TW) * TW;
      if (c < tw) gp[(int64_t)r * pl.nt + c] = T(0);
    }
  }
}

// Tiles that several work items accumulate into start from zero.
template <typename T, int TH, int TW>
__global__ void k_zero_split(RasterGeom g, const int32_t* __restrict__ counts, int64_t ntiles, T* __restrict__ grid) {
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x)
    if (counts[t] > kRowsPerItem) zero_tile<T, TH, TW>(g, t, grid);
}

// 4. persistent tile kernel -------------------------------------------------
// Blocks take work from two queues in step: a tile work item (rows of one tile, added
// in LDS and written out) and a group of kZeroGroup consecutive tiles, of which those no
// row touches are cleared.  The clearing stores (HBM-bound) then overlap the arithmetic
// of the rows instead of costing work items of their own.
template <typename T, int MODE, int TH, int TW, int OCC>
__global__ void __launch_bounds__(256, OCC) k_tile(DepoView<T> d, RasterGeom g, double nsigma, uint64_t seed,
                                              T* __restrict__ grid, const int32_t* __restrict__ list,
                                              const int32_t* __restrict__ offs, const int32_t* __restrict__ items,
                                              const int32_t* __restrict__ item_off, const int32_t* __restrict__ counts,
                                              int64_t ntiles, int32_t* __restrict__ ctrl,
                                              const DetTables* __restrict__ tables, const double* __restrict__ lf,
                                              const int2* __restrict__ hull) {
  constexpr int NWAVE = 4;
  static_assert(TH * TW <= (1 << kDstBits), "tile offsets must fit below the packed electron count");
  __shared__ T tile[TH * TW];
  __shared__ double s_ea[NWAVE][TH + 1];
  __shared__ double s_eb[NWAVE][TW + 1];
  __shared__ DetTablesSmall s_tb;
  __shared__ int s_item, s_zero, s_row;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (MODE == kModeBinomial) {
    for (int x = threadIdx.x; x < 129; x += blockDim.x) s_tb.inv[x] = tables->inv[x];
    for (int x = threadIdx.x; x < 19; x += blockDim.x) s_tb.fact[x] = tables->fact[x];
  }
  const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
  const int nzero = (int)((ntiles + kZeroGroup - 1) / kZeroGroup);
  bool more_items = true, more_zero = true;  // block-uniform
  for (;;) {
    if (threadIdx.x == 0) {
      s_item = more_items ? atomicAdd(&ctrl[kCtrlHead], 1) : INT_MAX;
      s_zero = more_zero ? atomicAdd(&ctrl[kCtrlHeadZero], 1) : INT_MAX;
    }
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);  // block-uniform: keep it scalar
    const int zg = __builtin_amdgcn_readfirstlane(s_zero);
    more_items = item < ctrl[kCtrlNItems];
    more_zero = zg < nzero;
    if (!more_items && !more_zero) break;
    __syncthreads();  // every thread has read s_item and s_zero
    // the group is cleared after the item, so that its stores drain while the other
    // blocks of the CU compute
    // With band hulls (wct_simulate), an empty tile outside its band's hull is left as it
    // is: the row transform reads only inside the hulls.  The group's tiles are walked with
    // their band and column stepped along (a band's hull is read once).
    auto clear_group = [&]() {
      if (!more_zero) return;
      const int64_t t0 = (int64_t)zg * kZeroGroup, z1 = min(t0 + kZeroGroup, ntiles);
      if (!hull) {
        for (int64_t t = t0; t < z1; ++t)
          if (counts[t] == 0) zero_tile<T, TH, TW>(g, t, grid);
        return;
      }
      int ev = 0, p = 0, tr = 0, tc = 0;
      int2 h = make_int2(0, 0);
      auto locate = [&](int64_t t) {  // band, column and hull of tile t
        ev = (int)(t / g.ntiles_ev);
        const int tin = (int)(t - (int64_t)ev * g.ntiles_ev);
        p = find_plane(g, tin);
        const int tl = tin - (int)g.pl[p].tile_off;
        tr = tl / g.pl[p].ntc;
        tc = tl - tr * g.pl[p].ntc;
        h = hull[(int64_t)ev * bands_before(g, g.n_planes) + bands_before(g, p) + tr];
      };
      locate(t0);
      for (int64_t t = t0; t < z1; ++t) {
        if (counts[t] == 0 && h.y > 0 && tc >= kSpanBase - h.x && tc < h.y) zero_tile<T, TH, TW>(g, t, grid);
        if (++tc == g.pl[p].ntc) {  // next band (of this plane, or the next plane or event)
          if (tr + 1 < g.pl[p].ntr) {
            tc = 0;
            ++tr;
            h = hull[(int64_t)ev * bands_before(g, g.n_planes) + bands_before(g, p) + tr];
          } else if (t + 1 < z1) {
            locate(t + 1);
          }
        }
      }
    };
    if (!more_items) {
      clear_group();
      continue;
    }
    const int t = items[item];
    const int chunk = item - item_off[t];
    const bool owned = (item_off[t + 1] - item_off[t]) == 1;
    const int ev = t / g.ntiles_ev;
    const int tin = t - ev * g.ntiles_ev;
    const int pi = find_plane(g, tin);
    const PlaneGeom& pl = g.pl[pi];
    const int tl = tin - pl.tile_off;
    const int tr = tl / pl.ntc, tc = tl - (tl / pl.ntc) * pl.ntc;
    const int tb0 = tr * TH, tk0 = tc * TW;
    const int th = min(TH, pl.nb - tb0), tw = min(TW, pl.nt - tk0);
    const int r0 = offs[t] + chunk * kRowsPerItem;
    const int r1 = min(offs[t] + (chunk + 1) * kRowsPerItem, offs[t + 1]);
    for (int x = threadIdx.x; x < TH * TW; x += blockDim.x) tile[x] = T(0);
    if (threadIdx.x == 0) s_row = r0;
    __syncthreads();
    auto dst = [&](int b, int k) { return (uint32_t)((b - tb0) * TW + (k - tk0)); };
    auto add = [&](uint32_t o, T v) { atomicAdd(&tile[o], v); };
    // the waves claim rows one at a time, so that they finish the item together
    auto claim = [&]() {
      int r = 0;
      if (lane == 0) r = atomicAdd(&s_row, 1);
      return __builtin_amdgcn_readfirstlane(r);
    };
    RegQueue qc;  // this wave's chop-down queue for the item
    qc.n = 0;
    for (int r = claim(); r < r1; r = claim()) {
      // the row is wave-uniform: a scalar index makes its parameters scalar loads and registers
      const int64_t j = __builtin_amdgcn_readfirstlane(list[r]);
      const RowWin w = row_window(d, j, g, nsigma);
      const int bb0 = max(w.b0, tb0), bb1 = min(w.b1, tb0 + th);
      const int kk0 = max(w.k0, tk0), kk1 = min(w.k1, tk0 + tw);
      if (!w.ok || bb0 >= bb1 || kk0 >= kk1) continue;
      const uint32_t did = d.depo_id ? (uint32_t)d.depo_id[j] : (uint32_t)j;
      patch_cells<T, MODE, true>(w, bb0, bb1, kk0, kk1, pl.nt, did, (uint32_t)w.key_event, (uint32_t)pi, key0, key1,
                                  s_ea[wv], s_eb[wv], s_tb, lf, lane, dst, add, qc);
    }
    if (MODE == kModeBinomial && qc.n > 0) rq_run_chop<T>(qc, qc.n, 0, true, lane, s_tb, lf, add);
    __syncthreads();
    T* gp = grid + (int64_t)ev * g.grid_ev_stride + pl.grid_off;
    for (int x = threadIdx.x; x < th * TW; x += blockDim.x) {
      const int rr = x / TW, c = x - (x / TW) * TW;
      if (c < tw) {
        T* dst = gp + (int64_t)(tb0 + rr) * pl.nt + tk0 + c;
        if (owned)
          *dst = tile[x];
        else if (tile[x] != T(0))
          atomicAdd(dst, tile[x]);
      }
    }
    __syncthreads();
    clear_group();
  }
}

// 5. rows wider than 4 tiles: 64 x 64 chunks per wave, straight to global atomics ------
template <typename T, int MODE>
__global__ void __launch_bounds__(256, 3) k_big(DepoView<T> d, RasterGeom g, double nsigma, uint64_t seed,
                                             T* __restrict__ grid, const int32_t* __restrict__ big,
                                             const int32_t* __restrict__ ctrl, const DetTables* __restrict__ tables,
                                             const double* __restrict__ lf) {
  constexpr int NWAVE = 4, CB = 64, CK = 64;
  __shared__ double s_ea[NWAVE][CB + 1];
  __shared__ double s_eb[NWAVE][CK + 1];
  __shared__ DetTablesSmall s_tb;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (MODE == kModeBinomial) {
    for (int x = threadIdx.x; x < 129; x += blockDim.x) s_tb.inv[x] = tables->inv[x];
    for (int x = threadIdx.x; x < 19; x += blockDim.x) s_tb.fact[x] = tables->fact[x];
    __syncthreads();
  }
  const int nbig = ctrl[kCtrlNBig];
  const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
  for (int r = blockIdx.x; r < nbig; r += gridDim.x) {
    const int64_t j = __builtin_amdgcn_readfirstlane(big[r]);
    const RowWin w = row_window(d, j, g, nsigma);
    if (!w.ok) continue;
    const PlaneGeom& pl = g.pl[w.plane];
    T* gp = grid + (int64_t)w.event * g.grid_ev_stride + pl.grid_off;
    const uint32_t did = d.depo_id ? (uint32_t)d.depo_id[j] : (uint32_t)j;
    const int kstart = w.k0 & ~1;  // chunks start on even ticks: a Philox pair never straddles two
    const int ncb = (w.b1 - w.b0 + CB - 1) / CB, nck = (w.k1 - kstart + CK - 1) / CK;
    const int nt = pl.nt;
    auto dst = [&](int b, int k) { return (uint32_t)((int64_t)b * nt + k); };
    auto add = [&](uint32_t o, T v) { atomicAdd(gp + o, v); };
    for (int c = wv; c < ncb * nck; c += NWAVE) {
      const int cb = c / nck, ck = c - (c / nck) * nck;
      const int b0 = w.b0 + cb * CB, b1 = min(b0 + CB, w.b1);
      const int k0 = max(kstart + ck * CK, w.k0), k1 = min(kstart + (ck + 1) * CK, w.k1);
      RegQueue qc;
      qc.n = 0;
      patch_cells<T, MODE, false>(w, b0, b1, k0, k1, pl.nt, did, (uint32_t)w.key_event, (uint32_t)w.plane, key0, key1,
                                   s_ea[wv], s_eb[wv], s_tb, lf, lane, dst, add, qc);
    }
  }
}

// ---------------------------------------------------------------------------
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

#define WCT_CHECK_LAUNCH()                  \
  do {                                      \
    hipError_t e_ = hipGetLastError();      \
    if (e_ != hipSuccess) return e_;        \
  } while (0)

template <typename T, int TH, int TW, int OCC>
hipError_t launch_raster_tiles(const DepoView<T>& d, const RasterGeom& g, double nsigma, int mode, uint64_t seed,
                               T* grid, const RasterWs& ws, const DetTables* tables, const double* lfact, int n_cu,
                               hipStream_t st, ProfHook* prof) {
  const int64_t nt = ws.ntiles;
  if (nt >= INT32_MAX) return hipErrorInvalidValue;  // tile indices and list offsets are int32
  if (prof) prof->begin("raster_bin", st);
  // control words and counts are contiguous
  hipError_t e = launch_fill_i32(ws.ctrl, kCtrlWords + nt, 0, st);
  if (e != hipSuccess) return e;
  const int bands_ev = bands_before(g, g.n_planes);
  if (ws.span && !ws.hull) return hipErrorInvalidValue;  // spans come with band hulls
  if (ws.span) {
    e = launch_fill_i32(reinterpret_cast<int32_t*>(ws.hull), 2 * (int64_t)g.n_events * bands_ev, 0, st);
    if (e != hipSuccess) return e;
    e = launch_fill_i32(reinterpret_cast<int32_t*>(ws.span), 2 * g.n_events * g.rows_ev, 0, st);
    if (e != hipSuccess) return e;
  }
  const unsigned rblocks = (unsigned)((d.n + 255) / 256);
  if (d.n > 0) {
    hipLaunchKernelGGL((k_count<T, TH, TW>), dim3((unsigned)((d.n + kCountBlock - 1) / kCountBlock)),
                       dim3(kCountBlock), 0, st, d, g, nsigma, ws.counts, ws.rank, ws.big, ws.ctrl, ws.span,
                       ws.hull);
    WCT_CHECK_LAUNCH();
  }
  if (ws.span) {
    hipLaunchKernelGGL((k_band_spans<TH, TW>), dim3((unsigned)(g.n_events * bands_ev)), dim3(256), 0, st, g,
                       ws.counts, bands_ev, ws.span, ws.hull);
    WCT_CHECK_LAUNCH();
  }
  const int nsb = (int)((nt + kScanPerBlock - 1) / kScanPerBlock);
  int2* blocks = reinterpret_cast<int2*>(ws.blocks);
  hipLaunchKernelGGL(k_scan_local, dim3(nsb), dim3(1024), 0, st, ws.counts, nt, blocks);
  WCT_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, blocks, nsb, ws.ctrl);
  WCT_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_scan_apply, dim3(nsb), dim3(1024), 0, st, ws.counts, nt, blocks, ws.offs, ws.item_off);
  WCT_CHECK_LAUNCH();
  if (d.n > 0) {
    hipLaunchKernelGGL((k_fill<T, TH, TW>), dim3(rblocks), dim3(256), 0, st, d, g, nsigma, ws.offs, ws.rank,
                       ws.list);
    WCT_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_items, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, ws.item_off, nt, ws.items);
  WCT_CHECK_LAUNCH();
  hipLaunchKernelGGL((k_zero_split<T, TH, TW>), dim3(1024), dim3(256), 0, st, g, ws.counts, nt, grid);
  WCT_CHECK_LAUNCH();
  if (prof) prof->end(st);
  const unsigned pblocks = (unsigned)(n_cu * OCC);  // the blocks that fit a CU at once (LDS, registers)
  static const char* const kTileName[3] = {"raster_tile_mean", "raster_tile_fluct", "raster_tile_normal"};
  if (prof) prof->begin(kTileName[mode], st);
#define WCT_TILE_LAUNCH(M)                                                                                        \
  hipLaunchKernelGGL((k_tile<T, M, TH, TW, OCC>), dim3(pblocks), dim3(256), 0, st, d, g, nsigma, seed, grid, ws.list, \
                     ws.offs, ws.items, ws.item_off, ws.counts, nt, ws.ctrl, tables, lfact, ws.hull)
  if (mode == kModeBinomial)
    WCT_TILE_LAUNCH(kModeBinomial);
  else if (mode == kModeNormal)
    WCT_TILE_LAUNCH(kModeNormal);
  else
    WCT_TILE_LAUNCH(kModeMean);
#undef WCT_TILE_LAUNCH
  WCT_CHECK_LAUNCH();
  if (prof) prof->end(st);
  if (prof) prof->begin("raster_wide_rows", st);
#define WCT_BIG_LAUNCH(M)                                                                                      \
  hipLaunchKernelGGL((k_big<T, M>), dim3(256), dim3(256), 0, st, d, g, nsigma, seed, grid, ws.big, ws.ctrl, tables, \
                     lfact)
  if (mode == kModeBinomial)
    WCT_BIG_LAUNCH(kModeBinomial);
  else if (mode == kModeNormal)
    WCT_BIG_LAUNCH(kModeNormal);
  else
    WCT_BIG_LAUNCH(kModeMean);
#undef WCT_BIG_LAUNCH
  WCT_CHECK_LAUNCH();
  if (prof) prof->end(st);
  return hipSuccess;
}

template <typename T>
hipError_t launch_raster(const DepoView<T>& d, const RasterGeom& g, double nsigma, int mode, uint64_t seed,
                         T* grid, const RasterWs& ws, const DetTables* tables, const double* lfact, int n_cu,
                         hipStream_t st, ProfHook* prof, int tile) {
  if (mode < kModeMean || mode > kModeNormal) return hipErrorInvalidValue;
  int id = 0;  // index among the variants of type T
  hipError_t e = hipErrorInvalidValue;
#define WCT_TILE_CASE(TT, TH_, TW_, OCC)                                                                    \
  if constexpr (std::is_same<T, TT>::value) {                                                              \
    if (id++ == tile)                                                                                      \
      e = launch_raster_tiles<T, TH_, TW_, OCC>(d, g, nsigma, mode, seed, grid, ws, tables, lfact, n_cu,      \
                                                st, prof);                                                  \
  }
  WCT_TILE_VARIANTS(WCT_TILE_CASE)
#undef WCT_TILE_CASE
  return e;
}

template hipError_t launch_raster<float>(const DepoView<float>&, const RasterGeom&, double, int, uint64_t, float*,
                                         const RasterWs&, const DetTables*, const double*, int, hipStream_t,
                                         ProfHook*, int);
template hipError_t launch_raster<double>(const DepoView<double>&, const RasterGeom&, double, int, uint64_t, double*,
                                          const RasterWs&, const DetTables*, const double*, int, hipStream_t,
                                          ProfHook*, int);

// ln(n!) table for the chop-down sampler, filled with the sampler's own det_lfact.
__global__ void k_lfact_table(double* __restrict__ out, int n, const DetTables* __restrict__ tables) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = det_lfact((int64_t)i, *tables);
}
hipError_t launch_lfact_table(double* out, int n, const DetTables* tables, hipStream_t st) {
  hipLaunchKernelGGL(k_lfact_table, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, out, n, tables);
  return hipGetLastError();
}

}  // namespace wct
