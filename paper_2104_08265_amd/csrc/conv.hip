// FFT convolution of charge grids with the wire response (Eq. 2 of arXiv:2104.08265):
// transform S, multiply by the pre-computed response spectrum, transform back.
//
// Pass A  (k_rows_r2c):  every impact row of S, zero-padded from N_t to L_t = 2M ticks,
//                         is transformed real-to-complex through one length-M complex
//                         transform (even/odd samples packed as re/im) and a post-twiddle;
//                         the F = M+1 tick frequencies go to S-hat in the column-chunk
//                         layout [chunk][phase i][wire c][C].
// Pass B  (k_colpass):    per chunk of C tick frequencies: for every phase i, the N_w
//                         values of rows I*c+i are transformed along wires (length L_w,
//                         zero padded), multiplied by the phase's spectrum R~_i and summed
//                         over i in registers (the impact-to-wire reduction); the sum is
//                         transformed back along wires and the N_w wires are kept.
// Pass C  (k_rows_c2r):  every wire's F frequencies are transformed complex-to-real back
//                         to L_t ticks and cropped to N_t.
// The 1/(L_w L_t) normalisation is folded into R~ at plan time.
//
// The backward (adjoint) variants reuse the passes: rows of dL/dM through pass A, a
// column pass that transforms once and applies conj(R~_i) per phase, and pass C over
// the I*N_w impact rows of the column-chunk layout.
#include "convcommon.hpp"

namespace wct {

// ---------------------------------------------------------------------------
// Pass A: real rows -> half spectra, column-chunk layout.  Persistent: a workgroup
// walks rows L = first + k * gridDim.x; the next row is loaded into registers while the
// current one is transformed, so HBM reads overlap the LDS work.  With row spans (FLAGS:
// the raster's tick span per impact row, [event][row], row = wire * nphase + phase), a
// row no deposition window reached is neither loaded nor transformed: its zero spectrum
// is written directly; the other rows are read only inside their spans (16-byte pieces
// outside hold zeros: they are taken as zero without a load from HBM).  Each wave reads
// whether its block's next rows are reached at once, one per lane, and keeps the answers
// as a ballot mask.
// ---------------------------------------------------------------------------
template <typename T, int C, typename F, bool FLAGS>
__global__ void __launch_bounds__(F::kBound) k_rows_r2c(const T* __restrict__ src, int64_t src_ev_stride,
                                                   cx<T>* __restrict__ dst, int64_t dst_ev_stride, int nt,
                                                   int nphase, int nper, int nchunk, int n_events, F f,
                                                   const cx<T>* __restrict__ tw,
                                                   const cx<T>* __restrict__ post,
                                                   const int2* __restrict__ span, int64_t span_ev) {
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::n;
  constexpr int PF = (2 * F::E + VN - 1) / VN;  // 16-byte loads per thread: a row has <= 2 E reals per thread
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* z = reinterpret_cast<cx<T>*>(smem_raw);
  T* zr = reinterpret_cast<T*>(smem_raw);
  V* zv = reinterpret_cast<V*>(smem_raw);
  const int M = f.n();
  const int nthr = f.nthr();
  const int rows = nphase * nper;
  const int total = rows * n_events;
  // Rows whose length or base is not a multiple of 16 bytes are read with scalar loads
  // and without prefetch.
  const bool vec = (nt % VN) == 0 && (reinterpret_cast<uintptr_t>(src) % 16) == 0 && (src_ev_stride % VN) == 0;
  const int ntv = vec ? nt / VN : 0;
  V pre[PF];
  // lanes of the block's last wave (partial when the block is not a multiple of 64)
  const int wspan = blockDim.x % 64 == 0 ? 64 : (int)(blockDim.x % 64);
  unsigned long long mask = 0;
  int left = 0;  // unused bits of mask
  auto live_at = [&](int Q) -> bool {  // called once per iteration, in order; Q: its row
    if constexpr (!FLAGS) {
      return true;
    } else {
      if (left == 0) {
        const int lane = threadIdx.x & 63;
        const int Ql = Q + lane * (int)gridDim.x;
        bool l = false;
        if (lane < wspan && Ql < total) {
          const int ev = Ql / rows, rin = Ql - (Ql / rows) * rows;
          const int i = rin / nper, c = rin - (rin / nper) * nper;
          l = span[ev * span_ev + (int64_t)c * nphase + i].y != 0;
        }
        mask = __ballot(l);
        left = wspan;
      }
      const bool b = mask & 1ull;
      mask >>= 1;
      --left;
      return b;
    }
  };
  // 16-byte pieces u of row Q inside the row and its span; the others are zero (their
  // loads are clamped to the span's first piece, a cached line, and the value dropped):
  // unconditional loads keep pre[] in registers
  auto prefetch = [&](int Q) {
    const int ev = Q / rows, rin = Q - (Q / rows) * rows;
    const int i = rin / nper, c = rin - (rin / nper) * nper;
    const int2 sp = row_span(FLAGS ? span : nullptr, ev * span_ev + (int64_t)c * nphase + i, nt);
    const int u0 = sp.x < sp.y ? sp.x / VN : 0;  // < ntv: a nonempty span lies inside [0, nt)
    const V* s = reinterpret_cast<const V*>(src + ev * src_ev_stride + ((int64_t)c * nphase + i) * nt);
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int u = threadIdx.x + q * nthr;
      const bool ok = u < ntv && (u + 1) * VN > sp.x && u * VN < sp.y;
      const V v = s[ok ? u : u0];
      pre[q] = ok ? v : (V)(T(0));
    }
  };
  int L = xcd_remap(blockIdx.x, gridDim.x);
  bool liveL = L < total && live_at(L);
  if (vec && liveL) prefetch(L);
  const int fpad = nchunk * C;
  while (L < total) {
    const int ev = L / rows, rin = L - (L / rows) * rows;
    const int i = rin / nper, c = rin - (rin / nper) * nper;
    const int Ln = L + gridDim.x;
    const bool liveN = Ln < total && live_at(Ln);
    cx<T>* out = dst + ev * dst_ev_stride;
    if constexpr (FLAGS) {
      if (!liveL) {
        if (vec && liveN) prefetch(Ln);
        for (int k = threadIdx.x; k < fpad; k += nthr) {
          const int ch = k / C, cc = k - (k / C) * C;
          out[(((int64_t)ch * nphase + i) * nper + c) * C + cc] = mk(T(0), T(0));
        }
        L = Ln;
        liveL = liveN;
        continue;
      }
    }
    if (vec) {
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int u = threadIdx.x + q * nthr;
        if (u < ntv) zv[u] = pre[q];
      }
      for (int u = ntv * VN + threadIdx.x; u < 2 * M; u += nthr) zr[u] = T(0);
    } else {
      const T* s = src + ev * src_ev_stride + ((int64_t)c * nphase + i) * nt;
      const int2 sp = row_span(FLAGS ? span : nullptr, ev * span_ev + (int64_t)c * nphase + i, nt);
      for (int u = threadIdx.x; u < 2 * M; u += nthr) zr[u] = (u < nt && u >= sp.x && u < sp.y) ? s[u] : T(0);
    }
    __syncthreads();
    if (vec && liveN) prefetch(Ln);  // next row in flight during this row's transform
    f.template run<false>(z, tw);
    for (int k = threadIdx.x; k < fpad; k += nthr) {
      cx<T> X = mk(T(0), T(0));
      if (k <= M) {
        const cx<T> A = z[k == M ? 0 : k];
        const cx<T> B = conj(z[k == 0 ? 0 : M - k]);
        const cx<T> Ev = scale(A + B, T(0.5));
        const cx<T> D = scale(A - B, T(0.5));
        const cx<T> O = mk(D.y, -D.x);  // (A - B) / (2i)
        X = Ev + cmul(post[k], O);
      }
      const int ch = k / C, cc = k - (k / C) * C;
      out[(((int64_t)ch * nphase + i) * nper + c) * C + cc] = X;
    }
    __syncthreads();
    L = Ln;
    liveL = liveN;
  }
}

// ---------------------------------------------------------------------------
// Pass B (forward): transforms along wires per phase, spectrum product, phase sum.
// The next phase's S-hat block and the current phase's spectrum are loaded into
// registers while the current phase is transformed (PF, for small register budgets E).
// ---------------------------------------------------------------------------
template <typename T, int C, typename F, bool PF>
__global__ void __launch_bounds__(F::kBound) k_colpass(const cx<T>* __restrict__ shat, int64_t shat_ev_stride,
                                                  const cx<T>* __restrict__ rtil, cx<T>* __restrict__ mhat,
                                                  int64_t mhat_ev_stride, int nw, int nphase, int nchunk, int n_events,
                                                  F f, const cx<T>* __restrict__ tw) {
  constexpr int E = F::E;
  const int nthr = f.nthr();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int lw = f.n();
  const int ne = lw * C;
  const int nin = nw * C;
  int ch, ev;
  colpass_block(n_events, ch, ev);
  constexpr bool PFS = PF;
  cv2<T> acc[E], rreg[PF ? E : 1], sreg[PFS ? E : 1];
#pragma unroll
  for (int q = 0; q < E; ++q) acc[q] = to_v(mk(T(0), T(0)));
  const cx<T>* src = shat + ev * shat_ev_stride + (int64_t)ch * nphase * nin;
  const cx<T>* rt = rtil + (int64_t)ch * nphase * ne;
  if (PFS) {
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int idx = threadIdx.x + q * nthr;
      sreg[PFS ? q : 0] = to_v(idx < nin ? src[idx] : mk(T(0), T(0)));
    }
  }
  for (int i = 0; i < nphase; ++i) {
    const cx<T>* s = src + (int64_t)i * nin;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int idx = threadIdx.x + q * nthr;
      if (idx < ne) buf[idx] = PFS ? from_v(sreg[PFS ? q : 0]) : (idx < nin ? s[idx] : mk(T(0), T(0)));
    }
    __syncthreads();
    // this phase's spectrum and the next phase's data in flight during the transform
    const cx<T>* r = rt + (int64_t)i * ne;
    if (PF) {
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int idx = threadIdx.x + q * nthr;
        rreg[PF ? q : 0] = to_v(r[idx < ne ? idx : 0]);
      }
    }
    if (PFS && i + 1 < nphase) {
      const cx<T>* sn = s + nin;
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int idx = threadIdx.x + q * nthr;
        sreg[PFS ? q : 0] = to_v(idx < nin ? sn[idx] : mk(T(0), T(0)));
      }
    }
    f.template run<false>(buf, tw);
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int idx = threadIdx.x + q * nthr;
      if (idx < ne) acc[q] = acc[q] + to_v(cmul(buf[idx], PF ? from_v(rreg[PF ? q : 0]) : r[idx]));
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int idx = threadIdx.x + q * nthr;
    if (idx < ne) buf[idx] = from_v(acc[q]);
  }
  __syncthreads();
  f.template run<true>(buf, tw);
  cx<T>* dst = mhat + ev * mhat_ev_stride;
  const int fpad = nchunk * C;
  for (int idx = threadIdx.x; idx < nin; idx += nthr) {
    const int w = idx / C, cc = idx - (idx / C) * C;
    dst[(int64_t)w * fpad + ch * C + cc] = buf[idx];
  }
}

// ---------------------------------------------------------------------------
// Pass B (adjoint): one transform of dL/dM-hat along wires, conj(R~_i) per phase,
// inverse transform per phase into the column-chunk layout
// ---------------------------------------------------------------------------
template <typename T, int C, typename F>
__global__ void __launch_bounds__(F::kBound) k_colpass_adj(const cx<T>* __restrict__ ghat, int64_t ghat_ev_stride,
                                                      const cx<T>* __restrict__ rtil, cx<T>* __restrict__ hhat,
                                                      int64_t hhat_ev_stride, int nw, int nphase, int nchunk, int n_events,
                                                      F f, const cx<T>* __restrict__ tw) {
  constexpr int E = F::E;
  const int nthr = f.nthr();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int lw = f.n();
  const int ne = lw * C;
  const int nin = nw * C;
  int ch, ev;
  colpass_block(n_events, ch, ev);
  const cx<T>* s = ghat + ev * ghat_ev_stride + (int64_t)ch * nin;
  for (int idx = threadIdx.x; idx < ne; idx += nthr) buf[idx] = idx < nin ? s[idx] : mk(T(0), T(0));
  __syncthreads();
  f.template run<false>(buf, tw);
  cv2<T> g[E];
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int idx = threadIdx.x + q * nthr;
    g[q] = to_v(buf[idx < ne ? idx : 0]);
  }
  __syncthreads();
  const cx<T>* rt = rtil + (int64_t)ch * nphase * ne;
  cx<T>* dst = hhat + ev * hhat_ev_stride + (int64_t)ch * nphase * nin;
  for (int i = 0; i < nphase; ++i) {
    const cx<T>* r = rt + (int64_t)i * ne;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int idx = threadIdx.x + q * nthr;
      if (idx < ne) buf[idx] = cmulc(from_v(g[q]), r[idx]);
    }
    __syncthreads();
    f.template run<true>(buf, tw);
    cx<T>* d = dst + (int64_t)i * nin;
    for (int idx = threadIdx.x; idx < nin; idx += nthr) d[idx] = buf[idx];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Pass C: half spectra -> real rows.  Input either wire-major rows [w][fpad]
// (TILED = false) or the column-chunk layout [chunk][phase][c][C] (TILED = true).
// ---------------------------------------------------------------------------
template <typename T, int C, bool TILED, typename F, bool NOISE>
__global__ void __launch_bounds__(F::kBound) k_rows_c2r(const cx<T>* __restrict__ src, int64_t src_ev_stride,
                                                   T* __restrict__ dst, int64_t dst_ev_stride, int nt,
                                                   int nphase, int nper, int nchunk, F f,
                                                   const cx<T>* __restrict__ tw,
                                                   const cx<T>* __restrict__ post, NoiseArgs<T> nz, WireLive wl) {
  const int nthr = f.nthr();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* z = reinterpret_cast<cx<T>*>(smem_raw);
  T* zr = reinterpret_cast<T*>(smem_raw);
  const int M = f.n();
  const int L = TILED ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  if (!TILED && !NOISE && wl.live && !wl.live[(int64_t)blockIdx.y * wl.ev_stride + L]) {
    // no window reaches this wire within the response's reach: its waveform is zero
    T* o = dst + blockIdx.y * dst_ev_stride + (int64_t)L * nt;
    for (int x = threadIdx.x; x < nt; x += blockDim.x) o[x] = T(0);
    return;
  }
  const int i = L / nper, c = L - (L / nper) * nper;
  const int64_t row = TILED ? (int64_t)c * nphase + i : (int64_t)L;
  const cx<T>* in = src + blockIdx.y * src_ev_stride;
  const int fpad = nchunk * C;
  auto X = [&](int k) -> cx<T> {
    if (TILED) return in[(((int64_t)(k / C) * nphase + i) * nper + c) * C + (k % C)];
    cx<T> v = in[(int64_t)L * fpad + k];
    if constexpr (NOISE) v = v + noise_at(nz, k, M, (uint32_t)L, (uint32_t)(nz.event_base + (int)blockIdx.y));
    return v;
  };
  for (int k = threadIdx.x; k < M; k += nthr) {
    const cx<T> A = X(k);
    const cx<T> B = conj(X(M - k));
    const cx<T> Ev = A + B;
    const cx<T> O = cmulc(A - B, post[k]);  // (A - B) * W_L^-k
    z[k] = mk(Ev.x - O.y, Ev.y + O.x);      // Ev + i*O
  }
  __syncthreads();
  f.template run<true>(z, tw);
  T* out = dst + blockIdx.y * dst_ev_stride + row * nt;
  for (int n = threadIdx.x; n < nt; n += nthr) out[n] = zr[n];
}

// ---------------------------------------------------------------------------
// host launchers: the plan's compiled variant, or the runtime plan with the smallest
// register budget E whose block fits
// ---------------------------------------------------------------------------
template <typename T>
static int pick_e(int elems) {
  const int cands[4] = {8, 16, 24, 32};
  const int ncand = sizeof(T) == 4 ? 4 : 2;
  for (int k = 0; k < ncand; ++k) {
    const int e = cands[k];
    const int bound = e <= 8 ? LaunchBound<T, 8>::value : LaunchBound<T, 16>::value;  // mirrors the kernels
    if ((elems + e - 1) / e <= bound) return e;
  }
  return 0;
}
static int threads_for(int elems, int e) {
  int t = (elems + e - 1) / e;
  t = ((t + 63) / 64) * 64;
  return t < 64 ? 64 : t;
}

template <typename T>
bool conv_fits(int elems) { return pick_e<T>(elems) > 0; }
template bool conv_fits<float>(int);
template bool conv_fits<double>(int);

// Column passes keep the next phase and the spectrum in registers when E is small.
template <typename T, typename F>
constexpr bool colpass_prefetch() { return sizeof(T) == 4 ? (F::E > 8 && F::E <= 16) : F::E <= 8; }

// Calls fn(policy, threads) with the runtime plan and the smallest register budget E
// whose block fits (KIND 0: rows, 1: columns).
template <typename T, int KIND, typename Fn>
static hipError_t with_fft(const FftPlan& plan, Fn&& fn) {
  constexpr int CI = KIND == 0 ? 1 : kChunk;
  const int elems = plan.n * CI;
  switch (pick_e<T>(elems)) {
    case 8: fn(RtFft<T, CI, 8>{plan}, threads_for(elems, 8)); return hipSuccess;
    case 16: fn(RtFft<T, CI, 16>{plan}, threads_for(elems, 16)); return hipSuccess;
    case 24:
      if constexpr (sizeof(T) == 4) {
        fn(RtFft<T, CI, 24>{plan}, threads_for(elems, 24));
        return hipSuccess;
      }
      break;
    case 32:
      if constexpr (sizeof(T) == 4) {
        fn(RtFft<T, CI, 32>{plan}, threads_for(elems, 32));
        return hipSuccess;
      }
      break;
    default: break;
  }
  return hipErrorInvalidValue;
}

// Every runtime policy of one kind and type (for per-kernel set-up).
template <typename T, int KIND, typename Fn>
static void for_all_fft(Fn&& fn) {
  constexpr int CI = KIND == 0 ? 1 : kChunk;
  fn(RtFft<T, CI, 8>{});
  fn(RtFft<T, CI, 16>{});
  if constexpr (sizeof(T) == 4) {
    fn(RtFft<T, CI, 24>{});
    fn(RtFft<T, CI, 32>{});
  }
}

template <typename T>
hipError_t launch_rows_r2c(const T* src, int64_t src_ev_stride, cx<T>* dst, int64_t dst_ev_stride, int nt, int nphase,
                           int nper, int nchunk, int n_events, const FftPlan& plan, const cx<T>* tw,
                           const cx<T>* post, int n_cu, hipStream_t st, const int2* span, int64_t span_ev,
                           const WireTiles& wt) {
  if (plan.variant >= 0)
    return launch_rows_r2c_ct<T>(src, src_ev_stride, dst, dst_ev_stride, nt, nphase, nper, nchunk, n_events, plan, tw,
                                 post, n_cu, st, span, span_ev, wt);
  const size_t lds = sizeof(cx<T>) * plan.n;
  const int total = nphase * nper * n_events;
  const hipError_t e = with_fft<T, 0>(plan, [&](auto f, int thr) {
    using F = decltype(f);
    const dim3 grid(persistent_blocks(n_cu, lds, thr, total));
    if (span)
      hipLaunchKernelGGL((k_rows_r2c<T, kChunk, F, true>), grid, dim3(thr), lds, st, src, src_ev_stride, dst,
                         dst_ev_stride, nt, nphase, nper, nchunk, n_events, f, tw, post, span, span_ev);
    else
      hipLaunchKernelGGL((k_rows_r2c<T, kChunk, F, false>), grid, dim3(thr), lds, st, src, src_ev_stride, dst,
                         dst_ev_stride, nt, nphase, nper, nchunk, n_events, f, tw, post, span, span_ev);
  });
  return e != hipSuccess ? e : hipGetLastError();
}

template <typename T>
hipError_t launch_colpass(const cx<T>* shat, int64_t shat_ev_stride, const cx<T>* rtil, cx<T>* mhat,
                          int64_t mhat_ev_stride, int nw, int nphase, int nchunk, int n_events, const FftPlan& plan,
                          const cx<T>* tw, const cx<T>* tw_rev, hipStream_t st) {
  if (plan.variant >= 0)
    return launch_colpass_ct<T>(shat, shat_ev_stride, rtil, mhat, mhat_ev_stride, nw, nphase, nchunk, n_events, plan,
                                tw, tw_rev, st);
  const size_t lds = sizeof(cx<T>) * plan.n * kChunk;
  const dim3 grid(nchunk * n_events);
  const hipError_t e = with_fft<T, 1>(plan, [&](auto f, int thr) {
    using F = decltype(f);
    hipLaunchKernelGGL((k_colpass<T, kChunk, F, colpass_prefetch<T, F>()>), grid, dim3(thr), lds, st, shat,
                       shat_ev_stride, rtil, mhat, mhat_ev_stride, nw, nphase, nchunk, n_events, f, tw);
  });
  return e != hipSuccess ? e : hipGetLastError();
}

template <typename T>
hipError_t launch_colpass_adj(const cx<T>* ghat, int64_t ghat_ev_stride, const cx<T>* rtil, cx<T>* hhat,
                              int64_t hhat_ev_stride, int nw, int nphase, int nchunk, int n_events,
                              const FftPlan& plan, const cx<T>* tw, const cx<T>* tw_rev, hipStream_t st) {
  if (plan.variant >= 0)
    return launch_colpass_adj_ct<T>(ghat, ghat_ev_stride, rtil, hhat, hhat_ev_stride, nw, nphase, nchunk, n_events,
                                    plan, tw, tw_rev, st);
  const size_t lds = sizeof(cx<T>) * plan.n * kChunk;
  const dim3 grid(nchunk * n_events);
  const hipError_t e = with_fft<T, 1>(plan, [&](auto f, int thr) {
    using F = decltype(f);
    hipLaunchKernelGGL((k_colpass_adj<T, kChunk, F>), grid, dim3(thr), lds, st, ghat, ghat_ev_stride, rtil, hhat,
                       hhat_ev_stride, nw, nphase, nchunk, n_events, f, tw);
  });
  return e != hipSuccess ? e : hipGetLastError();
}

template <typename T>
hipError_t launch_rows_c2r(const cx<T>* src, int64_t src_ev_stride, T* dst, int64_t dst_ev_stride, int nt,
                           bool tiled, int nphase, int nper, int nchunk, int n_events, const FftPlan& plan,
                           const cx<T>* tw, const cx<T>* post, hipStream_t st, const NoiseArgs<T>& nz,
                           const WireLive& wl) {
  if (tiled && nz.amp) return hipErrorInvalidValue;  // noise belongs to the forward's waveform rows
  if (tiled && wl.live) return hipErrorInvalidValue;  // wire flags belong to the forward's waveform rows
  if (plan.variant >= 0)
    return launch_rows_c2r_ct<T>(src, src_ev_stride, dst, dst_ev_stride, nt, tiled, nphase, nper, nchunk, n_events,
                                 plan, tw, post, st, nz, wl);
  const size_t lds = sizeof(cx<T>) * plan.n;
  const dim3 grid(nphase * nper, n_events);
  const hipError_t e = with_fft<T, 0>(plan, [&](auto f, int thr) {
    using F = decltype(f);
    if (tiled)
      hipLaunchKernelGGL((k_rows_c2r<T, kChunk, true, F, false>), grid, dim3(thr), lds, st, src, src_ev_stride, dst,
                         dst_ev_stride, nt, nphase, nper, nchunk, f, tw, post, nz, wl);
    else if (nz.amp)
      hipLaunchKernelGGL((k_rows_c2r<T, kChunk, false, F, true>), grid, dim3(thr), lds, st, src, src_ev_stride,
                         dst, dst_ev_stride, nt, nphase, nper, nchunk, f, tw, post, nz, wl);
    else
      hipLaunchKernelGGL((k_rows_c2r<T, kChunk, false, F, false>), grid, dim3(thr), lds, st, src, src_ev_stride,
                         dst, dst_ev_stride, nt, nphase, nper, nchunk, f, tw, post, nz, wl);
  });
  return e != hipSuccess ? e : hipGetLastError();
}

template <typename T>
static void raise_lds_limits() {
  const int lim = 160 * 1024;
  for_all_fft<T, 0>([&](auto f) {
    using F = decltype(f);
    (void)hipFuncSetAttribute((const void*)k_rows_r2c<T, kChunk, F, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              lim);
    (void)hipFuncSetAttribute((const void*)k_rows_r2c<T, kChunk, F, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)k_rows_c2r<T, kChunk, true, F, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)k_rows_c2r<T, kChunk, false, F, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)k_rows_c2r<T, kChunk, false, F, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  });
  for_all_fft<T, 1>([&](auto f) {
    using F = decltype(f);
    (void)hipFuncSetAttribute((const void*)k_colpass<T, kChunk, F, colpass_prefetch<T, F>()>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)k_colpass_adj<T, kChunk, F>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              lim);
  });
}

void conv_init_kernels() {
  raise_lds_limits<float>();
  raise_lds_limits<double>();
  conv_ct_init_kernels();
  wiredirect_init_kernels();
}

#define WCT_INST(T)                                                                                            \
  template hipError_t launch_rows_r2c<T>(const T*, int64_t, cx<T>*, int64_t, int, int, int, int, int,          \
                                         const FftPlan&, const cx<T>*, const cx<T>*, int, hipStream_t,        \
                                         const int2*, int64_t, const WireTiles&); \
  template hipError_t launch_colpass<T>(const cx<T>*, int64_t, const cx<T>*, cx<T>*, int64_t, int, int, int,   \
                                        int, const FftPlan&, const cx<T>*, const cx<T>*, hipStream_t);         \
  template hipError_t launch_colpass_adj<T>(const cx<T>*, int64_t, const cx<T>*, cx<T>*, int64_t, int, int,    \
                                            int, int, const FftPlan&, const cx<T>*, const cx<T>*, hipStream_t);\
  template hipError_t launch_rows_c2r<T>(const cx<T>*, int64_t, T*, int64_t, int, bool, int, int, int, int,    \
                                         const FftPlan&, const cx<T>*, const cx<T>*, hipStream_t,              \
                                         const NoiseArgs<T>&, const WireLive&);
WCT_INST(float)
WCT_INST(double)
#undef WCT_INST

}  // namespace wct
