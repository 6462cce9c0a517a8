// The transform passes of conv.hip for the compiled plans of fftvariants.hpp.
//
// Same arithmetic, same layouts and same results as the runtime-plan kernels; the
// difference is where values live between HBM and the transform.  A compiled plan
// knows which elements each thread's first-pass butterflies read, so the kernels load
// those straight from HBM into registers (no LDS staging), and its last pass leaves its
// outputs in registers in a fixed arrangement:
//   pass A:  HBM -> registers -> passes -> LDS -> post-twiddle -> HBM;
//   pass B:  per phase HBM -> registers -> passes -> registers, multiplied by R~_i and
//            summed in registers; the inverse transform runs with the radices reversed,
//            so its first pass reads exactly the sums each thread holds, and its last pass
//            writes HBM from registers;
//   pass C:  pre-twiddle HBM -> registers -> passes -> registers -> HBM.
#include "convcommon.hpp"

namespace wct {

// A thread's first-pass inputs of the half-length transform of a row of nt reals:
// complex sample m is (x[2m], x[2m+1]), zero past the row's end and outside the row's
// span [sp.x, sp.y) (where the row holds zeros, so those are not read from HBM).  The
// choice between 2-vector and element loads is made once for all of them (it is uniform),
// so the loads of a thread issue back to back with no branch between them; an index
// outside reads the span's first element (a cached line) and the zero is selected
// afterwards.
template <typename F, typename T>
__device__ __forceinline__ void load_row_inputs(const T* __restrict__ s, int nt, bool v2, int2 sp, cx<T>* in) {
  constexpr int R0 = F::R0;
  const int hi = sp.y < nt ? sp.y : nt;
  const int lo = sp.x < hi ? sp.x : 0;  // an empty span (a row of a pair no window reached) reads index 0
  if (v2) {  // even row length, 8-byte aligned rows
    const int m0 = lo >> 1;
#pragma unroll
    for (int q = 0; q < F::MB0; ++q) {
      if (!F::in_ok(q)) continue;
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const int m = F::in_elem(q, r);
        const bool ok = 2 * m + 2 > lo && 2 * m < hi;
        const cv2<T> p = *reinterpret_cast<const cv2<T>*>(s + 2 * (ok ? m : m0));
        in[q * R0 + r] = ok ? mk(p.x, p.y) : mk(T(0), T(0));
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < F::MB0; ++q) {
      if (!F::in_ok(q)) continue;
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const int m = F::in_elem(q, r);
        const bool ok0 = 2 * m >= lo && 2 * m < hi, ok1 = 2 * m + 1 >= lo && 2 * m + 1 < hi;
        const T a = s[ok0 ? 2 * m : lo], b = s[ok1 ? 2 * m + 1 : lo];
        in[q * R0 + r] = mk(ok0 ? a : T(0), ok1 ? b : T(0));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Pass A (compiled plan).  Persistent over rows; the next row's first-pass inputs are
// requested as soon as the current row's first pass has consumed its registers.
// ---------------------------------------------------------------------------
template <typename T, int C, typename F>
__global__ void __launch_bounds__(F::kThreads, F::kMinWaves) k_rows_r2c_ct(const T* __restrict__ src, int64_t src_ev_stride,
                                                             cx<T>* __restrict__ dst, int64_t dst_ev_stride, int nt,
                                                             int nphase, int nper, int nchunk, int n_events,
                                                             const cx<T>* __restrict__ tw,
                                                             const cx<T>* __restrict__ post,
                                                             const int2* __restrict__ span, int64_t span_ev) {
  constexpr int M = F::N, NT = F::kThreads, R0 = F::R0;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* z = reinterpret_cast<cx<T>*>(smem_raw);
  const int rows = nphase * nper;
  const int total = rows * n_events;
  // sample pairs (x[2m], x[2m+1]) are one 2-vector load when rows allow it
  const bool v2 = (nt % 2) == 0 && (reinterpret_cast<uintptr_t>(src) % (2 * sizeof(T))) == 0 &&
                  (src_ev_stride % 2) == 0;
  cx<T> in[F::IN];
  auto row_of = [&](int L, int& ev, int& i, int& c) {
    ev = L / rows;
    const int rin = L - ev * rows;
    i = rin / nper;
    c = rin - i * nper;
  };
  auto load = [&](int L) {
    int ev, i, c;
    row_of(L, ev, i, c);
    // with row spans a row is read only inside its span (a row no window reached: none of it)
    const int64_t row = (int64_t)c * nphase + i;
    load_row_inputs<F>(src + ev * src_ev_stride + row * nt, nt, v2, row_span(span, ev * span_ev + row, nt), in);
  };
  int L = xcd_remap(blockIdx.x, gridDim.x);
  if (L < total) load(L);
  while (L < total) {
    const int Ln = L + gridDim.x;
    int ev, i, c;
    row_of(L, ev, i, c);
    F::template rl<false>(z, tw, in, [&]() {
      if (Ln < total) load(Ln);
    });
    cx<T>* out = dst + ev * dst_ev_stride;
    constexpr int fpad = (M + 1 + C - 1) / C * C;  // nchunk * C (checked by the launcher)
    // frequency k goes to [k / C][i][c][k % C]; with NT a multiple of C a thread keeps
    // k % C and advances by NT / C chunks per step
    const int64_t cstride = (int64_t)nphase * nper * C;
    cx<T>* o = out + ((int64_t)i * nper + c) * C;
    auto post_twiddle = [&](int k, cx<T> pw) {
      cx<T> X = mk(T(0), T(0));
      if (k <= M) {
        const cx<T> A = z[k == M ? 0 : k];
        const cx<T> B = conj(z[k == 0 ? 0 : M - k]);
        const cx<T> Ev = scale(A + B, T(0.5));
        const cx<T> D = scale(A - B, T(0.5));
        const cx<T> O = mk(D.y, -D.x);  // (A - B) / (2i)
        X = Ev + cmul(pw, O);
      }
      return X;
    };
    auto post_at = [&](int k) { return k <= M ? post[k] : mk(T(0), T(0)); };
    cx<T> pw = post_at(threadIdx.x);  // the table entry is loaded a loop trip ahead
#pragma unroll 1
    for (int k = threadIdx.x; k < fpad; k += NT) {
      const cx<T> pn = post_at(k + NT);
      o[(int64_t)(k / C) * cstride + k % C] = post_twiddle(k, pw);
      pw = pn;
    }
    __syncthreads();
    L = Ln;
  }
}

// Pass A over row pairs (wires c, c + 1 of one phase, c even; needs an even wire count):
// the first row's spectrum waits in LDS while the second is transformed, then both are
// written together, so each chunk of C frequencies goes out as 2C contiguous values
// (64 bytes in FP32) instead of two separate C-value pieces.  LDS: the transform buffer
// plus one staged spectrum.
template <typename T, int C, typename F>
__global__ void __launch_bounds__(F::kThreads, F::kMinWaves) k_rows_r2c_pair_ct(const T* __restrict__ src,
                                                                  int64_t src_ev_stride, cx<T>* __restrict__ dst,
                                                                  int64_t dst_ev_stride, int nt, int nphase, int nper,
                                                                  int nchunk, int n_events,
                                                                  const cx<T>* __restrict__ tw,
                                                                  const cx<T>* __restrict__ post,
                                                                  const int2* __restrict__ span, int64_t span_ev,
                                                                  WireTiles wt) {
  constexpr int M = F::N, NT = F::kThreads, R0 = F::R0;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* z = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* stg = z + M;  // the pair's first spectrum, [fpad]
  const int rows = nphase * nper;
  const int pairs = rows / 2 * n_events;
  // M + 1 frequencies padded to whole chunks (the launcher checks nchunk * C == FPAD)
  constexpr int FPAD = (M + 1 + C - 1) / C * C;
  constexpr int fpad = FPAD;
  const bool v2 = (nt % 2) == 0 && (reinterpret_cast<uintptr_t>(src) % (2 * sizeof(T))) == 0 &&
                  (src_ev_stride % 2) == 0;
  cx<T> in[F::IN];
  // row r (0 or 1) of pair P: event, phase, wire
  auto row_of = [&](int P, int r, int& ev, int& i, int& c) {
    const int L = 2 * P + r;
    ev = L / rows;
    const int rin = L - ev * rows;
    i = rin / nper;
    c = rin - i * nper;
  };
  auto load = [&](int P, int r) {
    int ev, i, c;
    row_of(P, r, ev, i, c);
    const int64_t row = (int64_t)c * nphase + i;
    load_row_inputs<F>(src + ev * src_ev_stride + row * nt, nt, v2, row_span(span, ev * span_ev + row, nt), in);
  };
  // pw = post[k], loaded by the caller a loop trip ahead (its latency then overlaps a trip)
  auto post_twiddle = [&](int k, cx<T> pw) {
    cx<T> X = mk(T(0), T(0));
    if (k <= M) {
      const cx<T> A = z[k == M ? 0 : k];
      const cx<T> B = conj(z[k == 0 ? 0 : M - k]);
      const cx<T> Ev = scale(A + B, T(0.5));
      const cx<T> D = scale(A - B, T(0.5));
      const cx<T> O = mk(D.y, -D.x);  // (A - B) / (2i)
      X = Ev + cmul(pw, O);
    }
    return X;
  };
  auto post_at = [&](int k) { return k <= M ? post[k] : mk(T(0), T(0)); };
  // With row spans (span != NULL), a pair whose two rows no window reached is neither
  // loaded nor transformed: its zero spectrum is written directly.  Without them every pair
  // is transformed (one kernel serves both: the test of `span` is uniform).  Each wave reads the spans of its
  // block's next kSpan pairs at once (lane j: the pair j iterations on) and keeps the
  // answers as a ballot mask, so the per-pair test is a bit of a scalar register.  kSpan is
  // the lane count of the block's last wave, which is partial when NT is not a multiple of 64.
  constexpr int kSpan = NT % 64 == 0 ? 64 : NT % 64;
  auto pair_live = [&](int Q) {
    int ev, i, c;
    row_of(Q, 0, ev, i, c);
    const int2* f = span + ev * span_ev;
    return (f[(int64_t)c * nphase + i].y | f[(int64_t)(c + 1) * nphase + i].y) != 0;
  };
  // Whether a dead pair's zero spectrum is read: with row flags the direct column pass
  // takes such rows as zeros, so it is never written; with tile flags alone only a live
  // tile reads S^ (wires [t W - K, t W + W + K) of tile t), so a dead pair that no live
  // tile covers is not written.
  auto pair_read = [&](int Q) -> bool {
    if (wt.rowbits) return false;  // the direct pass reads the rows no window reached as zeros
    if (!wt.live) return true;
    int ev, i, c;
    row_of(Q, 0, ev, i, c);
    const uint8_t* tl = wt.live + ev * wt.ev_stride;
    constexpr int W = kDirectTileWires, K = kDirectHalfWires;
    const int thi = min(wt.ntile - 1, (c + 1 + K) / W);
    bool r = false;
    for (int t = max(0, thi - 2); t <= thi; ++t) r |= (t * W - K <= c + 1) && (c < t * W + W + K) && tl[t] != 0;
    return r;
  };
  unsigned long long mask = 0;
  int left = 0;  // unused bits of mask
  auto live_at = [&](int Q) -> bool {  // called once per iteration, in order; Q: its pair
    if (!span) {
      return true;
    } else {
      if (left == 0) {
        const int lane = threadIdx.x & 63;
        const int Ql = Q + lane * (int)gridDim.x;
        mask = __ballot(lane < kSpan && Ql < pairs && pair_live(Ql));
        left = kSpan;
      }
      const bool b = mask & 1ull;
      mask >>= 1;
      --left;
      return b;
    }
  };
  int P = xcd_remap(blockIdx.x, gridDim.x);
  bool liveP = P < pairs && live_at(P);
  if (liveP) load(P, 0);
  while (P < pairs) {
    const int Pn = P + gridDim.x;
    const bool liveN = Pn < pairs && live_at(Pn);
    int ev, i, c;
    row_of(P, 0, ev, i, c);
    // chunk q of the pair: [q][i][c .. c + 1][C], 2C contiguous values
    cx<T>* o = dst + ev * dst_ev_stride + ((int64_t)i * nper + c) * C;
    const int64_t cstride = (int64_t)nphase * nper * C;
    {
      if (!liveP) {
        if (liveN) load(Pn, 0);
        if (pair_read(P))
          for (int x = threadIdx.x; x < 2 * fpad; x += NT) {
            const int q = x / (2 * C), e = x - q * (2 * C);
            o[(int64_t)q * cstride + e] = mk(T(0), T(0));
          }
        P = Pn;
        liveP = liveN;
        continue;
      }
    }
    F::template rl<false>(z, tw, in, [&]() { load(P, 1); });
    {
      cx<T> pw = post_at(threadIdx.x);
#pragma unroll 1
      for (int k = threadIdx.x; k < FPAD; k += NT) {
        const cx<T> pn = post_at(k + NT);
        stg[k] = post_twiddle(k, pw);
        pw = pn;
      }
    }
    __syncthreads();
    F::template rl<false>(z, tw, in, [&]() {
      if (liveN) load(Pn, 0);
    });
    {
      // entry x of the pair's output: chunk q = x / 2C, position e = x % 2C (e < C: first row)
      auto k_of = [&](int x) {
        const int q = x / (2 * C), e = x - q * (2 * C);
        return q * C + (e < C ? e : e - C);
      };
      cx<T> pw = post_at(k_of(threadIdx.x));
#pragma unroll 1
      for (int x = threadIdx.x; x < 2 * FPAD; x += NT) {
        const cx<T> pn = x + NT < 2 * FPAD ? post_at(k_of(x + NT)) : mk(T(0), T(0));
        const int q = x / (2 * C), e = x - q * (2 * C);
        const int k = q * C + (e < C ? e : e - C);
        o[(int64_t)q * cstride + e] = e < C ? stg[k] : post_twiddle(k, pw);
        pw = pn;
      }
    }
    __syncthreads();
    P = Pn;
    liveP = liveN;
  }
}

// ---------------------------------------------------------------------------
// Pass B (compiled plan): phase transforms along wires, product with R~_i and phase
// sum in registers, inverse transform with the reversed plan.
// ---------------------------------------------------------------------------
template <typename T, int C, typename F>
__global__ void __launch_bounds__(F::kThreads, F::kMinWaves) k_colpass_ct(const cx<T>* __restrict__ shat, int64_t shat_ev_stride,
                                                            const cx<T>* __restrict__ rtil, cx<T>* __restrict__ mhat,
                                                            int64_t mhat_ev_stride, int nw, int nphase, int nchunk, int n_events,
                                                            const cx<T>* __restrict__ tw,
                                                            const cx<T>* __restrict__ tw_rev) {
  using FI = typename F::Reverse;
  constexpr int CI = F::CI, NSUB = C / CI;
  constexpr int NE = F::N * C, R0 = F::R0, RL = F::RL;  // NE: one phase of R~ (whole chunk)
  static_assert(FI::R0 == RL && FI::IN == F::OUT, "the reversed plan must start where the forward one ends");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int nin = nw * CI;  // elements of this block's sequences inside the grid
  int ch, ev, h;
  colpass_block_sub(n_events, NSUB, ch, ev, h);
  // element tid + K of the block (wire (tid + K) / CI, sequence (tid + K) % CI) in the
  // chunk layout [wire][C]: with NT and every K multiples of CI this is a per-thread base
  // plus a compile-time offset
  static_assert(F::kThreads % CI == 0 && F::NB0 % CI == 0 && F::NBL % CI == 0, "layout offsets");
  const int tid = (int)threadIdx.x;
  const int abase = (tid / CI) * C + h * CI + tid % CI;
  auto at = [&](int K) { return abase + (K / CI) * C; };
  const cx<T>* src = shat + ev * shat_ev_stride + (int64_t)ch * nphase * nw * C;
  const cx<T>* rt = rtil + (int64_t)ch * nphase * NE;
  cx<T> in[F::IN], out[F::OUT], acc[F::OUT];
#pragma unroll
  for (int u = 0; u < F::OUT; ++u) acc[u] = mk(T(0), T(0));
  auto load = [&](const cx<T>* s) {
#pragma unroll
    for (int q = 0; q < F::MB0; ++q) {
      if (!F::in_ok(q)) continue;
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const int K = F::in_off(q, r);
        in[q * R0 + r] = tid + K < nin ? s[at(K)] : mk(T(0), T(0));
      }
    }
  };
  for (int i = 0; i < nphase; ++i) {
    load(src + (int64_t)i * nw * C);
    F::template rr<false>(buf, tw, in, out, []() {});
    const cx<T>* r = rt + (int64_t)i * NE;
#pragma unroll
    for (int q = 0; q < F::MBL; ++q) {
      if (!F::out_ok(q)) continue;
#pragma unroll
      for (int rr = 0; rr < RL; ++rr)
        acc[q * RL + rr] = acc[q * RL + rr] + cmul(out[q * RL + rr], r[at(F::out_off(q, rr))]);
    }
    // keep the next phase's loads behind this product (register budget)
    __builtin_amdgcn_sched_barrier(0);
  }
  cx<T> res[FI::OUT];
  FI::template rr<true>(buf, tw_rev, acc, res, []() {});
  cx<T>* dst = mhat + ev * mhat_ev_stride;
  const int fpad = nchunk * C;
#pragma unroll
  for (int q = 0; q < FI::MBL; ++q) {
    if (!FI::out_ok(q)) continue;
#pragma unroll
    for (int r = 0; r < FI::RL; ++r) {
      const int e = FI::out_elem(q, r);
      if (e < nin) dst[(int64_t)(e / CI) * fpad + ch * C + h * CI + (e % CI)] = res[q * FI::RL + r];  // [w][fpad]
    }
  }
}

// ---------------------------------------------------------------------------
// Pass B adjoint (compiled plan): one forward transform of dL/dM-hat, then per phase
// conj(R~_i) and an inverse transform with the reversed plan, written from registers.
// ---------------------------------------------------------------------------
template <typename T, int C, typename F>
__global__ void __launch_bounds__(F::kThreads, F::kMinWaves) k_colpass_adj_ct(const cx<T>* __restrict__ ghat,
                                                                int64_t ghat_ev_stride,
                                                                const cx<T>* __restrict__ rtil,
                                                                cx<T>* __restrict__ hhat, int64_t hhat_ev_stride,
                                                                int nw, int nphase, int nchunk, int n_events,
                                                                const cx<T>* __restrict__ tw,
                                                                const cx<T>* __restrict__ tw_rev) {
  using FI = typename F::Reverse;
  constexpr int CI = F::CI, NSUB = C / CI;
  constexpr int NE = F::N * C, R0 = F::R0, RL = F::RL;
  static_assert(FI::R0 == RL && FI::IN == F::OUT, "the reversed plan must start where the forward one ends");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int nin = nw * CI;
  int ch, ev, h;
  colpass_block_sub(n_events, NSUB, ch, ev, h);
  static_assert(F::kThreads % CI == 0 && F::NB0 % CI == 0 && F::NBL % CI == 0, "layout offsets");
  const int tid = (int)threadIdx.x;
  const int abase = (tid / CI) * C + h * CI + tid % CI;
  auto at = [&](int K) { return abase + (K / CI) * C; };
  const cx<T>* s = ghat + ev * ghat_ev_stride + (int64_t)ch * nw * C;
  cx<T> in[F::IN], g[F::OUT];
#pragma unroll
  for (int q = 0; q < F::MB0; ++q) {
    if (!F::in_ok(q)) continue;
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int K = F::in_off(q, r);
      in[q * R0 + r] = tid + K < nin ? s[at(K)] : mk(T(0), T(0));
    }
  }
  F::template rr<false>(buf, tw, in, g, []() {});
  const cx<T>* rt = rtil + (int64_t)ch * nphase * NE;
  cx<T>* dst = hhat + ev * hhat_ev_stride + (int64_t)ch * nphase * nw * C;
  for (int i = 0; i < nphase; ++i) {
    const cx<T>* r = rt + (int64_t)i * NE;
    cx<T> hv[FI::IN], res[FI::OUT];
#pragma unroll
    for (int q = 0; q < F::MBL; ++q) {
      if (!F::out_ok(q)) continue;
#pragma unroll
      for (int rr = 0; rr < RL; ++rr) hv[q * RL + rr] = cmulc(g[q * RL + rr], r[at(F::out_off(q, rr))]);
    }
    FI::template rr<true>(buf, tw_rev, hv, res, []() {});
    cx<T>* d = dst + (int64_t)i * nw * C;
#pragma unroll
    for (int q = 0; q < FI::MBL; ++q) {
      if (!FI::out_ok(q)) continue;
#pragma unroll
      for (int r2 = 0; r2 < FI::RL; ++r2) {
        const int K = FI::out_off(q, r2);
        if (tid + K < nin) d[at(K)] = res[q * FI::RL + r2];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Pass C (compiled plan): pre-twiddled half spectrum -> registers -> real row.
// ---------------------------------------------------------------------------
template <typename T, int C, bool TILED, typename F, bool NOISE>
__global__ void __launch_bounds__(F::kThreads, F::kMinWaves) k_rows_c2r_ct(const cx<T>* __restrict__ src, int64_t src_ev_stride,
                                                             T* __restrict__ dst, int64_t dst_ev_stride, int nt,
                                                             int nphase, int nper, int nchunk,
                                                             const cx<T>* __restrict__ tw,
                                                             const cx<T>* __restrict__ post, NoiseArgs<T> nz,
                                                             WireLive wl) {
  constexpr int M = F::N, R0 = F::R0, RL = F::RL;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* z = reinterpret_cast<cx<T>*>(smem_raw);
  const int L = TILED ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  if (!TILED && !NOISE && wl.live && !wl.live[(int64_t)blockIdx.y * wl.ev_stride + L]) {
    // no window reaches this wire within the response's reach: its waveform is zero
    T* o = dst + blockIdx.y * dst_ev_stride + (int64_t)L * nt;
    for (int x = threadIdx.x; x < nt; x += blockDim.x) o[x] = T(0);
    return;
  }
  const int i = L / nper, c = L - (L / nper) * nper;
  const int64_t row = TILED ? (int64_t)c * nphase + i : (int64_t)L;
  const cx<T>* inp = src + blockIdx.y * src_ev_stride;
  const int fpad = nchunk * C;
  auto X = [&](int k) -> cx<T> {
    if (TILED) return inp[(((int64_t)(k / C) * nphase + i) * nper + c) * C + (k % C)];
    cx<T> v = inp[(int64_t)L * fpad + k];
    if constexpr (NOISE) v = v + noise_at(nz, k, M, (uint32_t)L, (uint32_t)(nz.event_base + (int)blockIdx.y));
    return v;
  };
  cx<T> in[F::IN], out[F::OUT];
#pragma unroll
  for (int q = 0; q < F::MB0; ++q) {
    if (!F::in_ok(q)) continue;
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int k = F::in_elem(q, r);
      const cx<T> A = X(k);
      const cx<T> B = conj(X(M - k));
      const cx<T> Ev = A + B;
      const cx<T> O = cmulc(A - B, post[k]);        // (A - B) * W_L^-k
      in[q * R0 + r] = mk(Ev.x - O.y, Ev.y + O.x);  // Ev + i*O
    }
  }
  F::template rr<true>(z, tw, in, out, []() {});
  T* o = dst + blockIdx.y * dst_ev_stride + row * nt;
  const bool v2 = (nt % 2) == 0 && (reinterpret_cast<uintptr_t>(dst) % (2 * sizeof(T))) == 0 &&
                  (dst_ev_stride % 2) == 0;
#pragma unroll
  for (int q = 0; q < F::MBL; ++q) {
    if (!F::out_ok(q)) continue;
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int m = F::out_elem(q, r);
      const cx<T> v = out[q * RL + r];
      if (v2) {
        if (2 * m < nt) {
          cv2<T> p;
          p.x = v.x;
          p.y = v.y;
          *reinterpret_cast<cv2<T>*>(o + 2 * m) = p;
        }
      } else {
        if (2 * m < nt) o[2 * m] = v.x;
        if (2 * m + 1 < nt) o[2 * m + 1] = v.y;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// Calls fn(policy) for compiled variant `v` of kind KIND and type T.
template <typename T, int KIND, typename Fn>
static hipError_t with_variant(int v, Fn&& fn) {
  constexpr int CI = KIND == 0 ? 1 : (KIND == 1 ? kChunk : kChunk / 2);
  bool done = false;
  int id = 0;
#define WCT_VARIANT_CASE(K, TT, NT, MW, ...)                   \
  if constexpr (K == KIND && std::is_same<T, TT>::value) {     \
    if (id == v) {                                             \
      fn(CtFft<T, CI, NT, MW, __VA_ARGS__>{});                 \
      done = true;                                             \
    }                                                          \
  }                                                            \
  ++id;
  WCT_FFT_VARIANTS(WCT_VARIANT_CASE)
#undef WCT_VARIANT_CASE
  return done ? hipSuccess : hipErrorInvalidValue;
}

// Wire-transform variants: kind 1 (whole chunks) and kind 2 (half chunks).
template <typename T, typename Fn>
static hipError_t with_wire_variant(int v, Fn&& fn) {
  int cnt = 0;
  const FftVariantDesc* d = fft_variants(&cnt);
  if (v < 0 || v >= cnt) return hipErrorInvalidValue;
  return d[v].kind == 2 ? with_variant<T, 2>(v, fn) : with_variant<T, 1>(v, fn);
}

template <typename T, int KIND, typename Fn>
static void for_all_variants(Fn&& fn) {
  constexpr int CI = KIND == 0 ? 1 : (KIND == 1 ? kChunk : kChunk / 2);
#define WCT_VARIANT_ALL(K, TT, NT, MW, ...) \
  if constexpr (K == KIND && std::is_same<T, TT>::value) fn(CtFft<T, CI, NT, MW, __VA_ARGS__>{});
  WCT_FFT_VARIANTS(WCT_VARIANT_ALL)
#undef WCT_VARIANT_ALL
}

template <typename T>
hipError_t launch_rows_r2c_ct(const T* src, int64_t src_ev_stride, cx<T>* dst, int64_t dst_ev_stride, int nt,
                              int nphase, int nper, int nchunk, int n_events, const FftPlan& plan, const cx<T>* tw,
                              const cx<T>* post, int n_cu, hipStream_t st, const int2* span, int64_t span_ev,
                              const WireTiles& wt) {
  const size_t lds = sizeof(cx<T>) * plan.n;
  const size_t lds_pair = lds + sizeof(cx<T>) * nchunk * kChunk;
  const int total = nphase * nper * n_events;
  // wire pairs when the wires pair up and the staged spectrum fits beside the buffer
  const bool pair = nper % 2 == 0 && lds_pair <= 160 * 1024;
  if (nchunk * kChunk != (plan.n + 1 + kChunk - 1) / kChunk * kChunk) return hipErrorInvalidValue;
  const hipError_t e = with_variant<T, 0>(plan.variant, [&](auto f) {
    using F = decltype(f);
    const dim3 pgrid(persistent_blocks(n_cu, lds_pair, F::kThreads, total / 2));
    if (pair)
      hipLaunchKernelGGL((k_rows_r2c_pair_ct<T, kChunk, F>), pgrid, dim3(F::kThreads), lds_pair, st, src,
                         src_ev_stride, dst, dst_ev_stride, nt, nphase, nper, nchunk, n_events, tw, post, span,
                         span_ev, wt);
    else
      hipLaunchKernelGGL((k_rows_r2c_ct<T, kChunk, F>), dim3(persistent_blocks(n_cu, lds, F::kThreads, total)),
                         dim3(F::kThreads), lds, st, src, src_ev_stride, dst, dst_ev_stride, nt, nphase, nper, nchunk,
                         n_events, tw, post, span, span_ev);
  });
  return e != hipSuccess ? e : hipGetLastError();
}

template <typename T>
hipError_t launch_colpass_ct(const cx<T>* shat, int64_t shat_ev_stride, const cx<T>* rtil, cx<T>* mhat,
                             int64_t mhat_ev_stride, int nw, int nphase, int nchunk, int n_events,
                             const FftPlan& plan, const cx<T>* tw, const cx<T>* tw_rev, hipStream_t st) {
  const hipError_t e = with_wire_variant<T>(plan.variant, [&](auto f) {
    using F = decltype(f);
    const size_t lds = sizeof(cx<T>) * plan.n * F::CI;
    hipLaunchKernelGGL((k_colpass_ct<T, kChunk, F>), dim3(nchunk * n_events * (kChunk / F::CI)), dim3(F::kThreads),
                       lds, st, shat,
                       shat_ev_stride, rtil, mhat, mhat_ev_stride, nw, nphase, nchunk, n_events, tw, tw_rev);
  });
  return e != hipSuccess ? e : hipGetLastError();
}

template <typename T>
hipError_t launch_colpass_adj_ct(const cx<T>* ghat, int64_t ghat_ev_stride, const cx<T>* rtil, cx<T>* hhat,
                                 int64_t hhat_ev_stride, int nw, int nphase, int nchunk, int n_events,
                                 const FftPlan& plan, const cx<T>* tw, const cx<T>* tw_rev, hipStream_t st) {
  const hipError_t e = with_wire_variant<T>(plan.variant, [&](auto f) {
    using F = decltype(f);
    const size_t lds = sizeof(cx<T>) * plan.n * F::CI;
    hipLaunchKernelGGL((k_colpass_adj_ct<T, kChunk, F>), dim3(nchunk * n_events * (kChunk / F::CI)),
                       dim3(F::kThreads), lds, st,
                       ghat, ghat_ev_stride, rtil, hhat, hhat_ev_stride, nw, nphase, nchunk, n_events, tw, tw_rev);
  });
  return e != hipSuccess ? e : hipGetLastError();
}

template <typename T>
hipError_t launch_rows_c2r_ct(const cx<T>* src, int64_t src_ev_stride, T* dst, int64_t dst_ev_stride, int nt,
                              bool tiled, int nphase, int nper, int nchunk, int n_events, const FftPlan& plan,
                              const cx<T>* tw, const cx<T>* post, hipStream_t st, const NoiseArgs<T>& nz,
                              const WireLive& wl) {
  const size_t lds = sizeof(cx<T>) * plan.n;
  const dim3 grid(nphase * nper, n_events);
  const hipError_t e = with_variant<T, 0>(plan.variant, [&](auto f) {
    using F = decltype(f);
    if (tiled)
      hipLaunchKernelGGL((k_rows_c2r_ct<T, kChunk, true, F, false>), grid, dim3(F::kThreads), lds, st, src,
                         src_ev_stride, dst, dst_ev_stride, nt, nphase, nper, nchunk, tw, post, nz, wl);
    else if (nz.amp)
      hipLaunchKernelGGL((k_rows_c2r_ct<T, kChunk, false, F, true>), grid, dim3(F::kThreads), lds, st, src,
                         src_ev_stride, dst, dst_ev_stride, nt, nphase, nper, nchunk, tw, post, nz, wl);
    else
      hipLaunchKernelGGL((k_rows_c2r_ct<T, kChunk, false, F, false>), grid, dim3(F::kThreads), lds, st, src,
                         src_ev_stride, dst, dst_ev_stride, nt, nphase, nper, nchunk, tw, post, nz, wl);
  });
  return e != hipSuccess ? e : hipGetLastError();
}

template <typename T>
static void raise_lds_limits_ct() {
  const int lim = 160 * 1024;
  for_all_variants<T, 0>([&](auto f) {
    using F = decltype(f);
    (void)hipFuncSetAttribute((const void*)k_rows_r2c_ct<T, kChunk, F>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              lim);
    (void)hipFuncSetAttribute((const void*)k_rows_r2c_pair_ct<T, kChunk, F>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)k_rows_c2r_ct<T, kChunk, true, F, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)k_rows_c2r_ct<T, kChunk, false, F, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)k_rows_c2r_ct<T, kChunk, false, F, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  });
  auto wire = [&](auto f) {
    using F = decltype(f);
    (void)hipFuncSetAttribute((const void*)k_colpass_ct<T, kChunk, F>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              lim);
    (void)hipFuncSetAttribute((const void*)k_colpass_adj_ct<T, kChunk, F>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  };
  for_all_variants<T, 1>(wire);
  for_all_variants<T, 2>(wire);
}

void conv_ct_init_kernels() {
  raise_lds_limits_ct<float>();
  raise_lds_limits_ct<double>();
}

#define WCT_INST(T)                                                                                              \
  template hipError_t launch_rows_r2c_ct<T>(const T*, int64_t, cx<T>*, int64_t, int, int, int, int, int,         \
                                            const FftPlan&, const cx<T>*, const cx<T>*, int, hipStream_t,       \
                                            const int2*, int64_t, const WireTiles&);                            \
  template hipError_t launch_colpass_ct<T>(const cx<T>*, int64_t, const cx<T>*, cx<T>*, int64_t, int, int, int,  \
                                           int, const FftPlan&, const cx<T>*, const cx<T>*, hipStream_t);        \
  template hipError_t launch_colpass_adj_ct<T>(const cx<T>*, int64_t, const cx<T>*, cx<T>*, int64_t, int, int,   \
                                               int, int, const FftPlan&, const cx<T>*, const cx<T>*,             \
                                               hipStream_t);                                                     \
  template hipError_t launch_rows_c2r_ct<T>(const cx<T>*, int64_t, T*, int64_t, int, bool, int, int, int, int,   \
                                            const FftPlan&, const cx<T>*, const cx<T>*, hipStream_t,            \
                                            const NoiseArgs<T>&, const WireLive&);
WCT_INST(float)
WCT_INST(double)
#undef WCT_INST

}  // namespace wct
