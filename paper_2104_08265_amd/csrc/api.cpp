// C ABI of libwct.so (declared in include/wct.h): plans, workspace carving, argument
// validation and the launch sequences of the raster, convolution and gradient paths.
#include <cerrno>
#include <cmath>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "fftplan.hpp"
#include "fftvariants.hpp"
#include "kernels.hpp"
#include "wct.h"

using namespace wct;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? WCT_E_NOMEM : WCT_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                       \
  do {                                            \
    hipError_t e__ = (expr);                      \
    if (e__ != hipSuccess) return hip_fail(e__, what); \
  } while (0)

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

bool smooth235(int64_t n) {
  if (n < 1) return false;
  for (int f : {2, 3, 5})
    while (n % f == 0) n /= f;
  return n == 1;
}
int64_t next_smooth(int64_t n) {
  if (n < 1) n = 1;
  while (!smooth235(n)) ++n;
  return n;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bump allocator over a caller-provided workspace (base == nullptr only sizes).
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  void* take(size_t bytes) {
    off = align_up(off, 256);
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

// Kernel timing: events recorded around launch groups while enabled, folded into
// per-name totals when read.
struct Profiler final : ProfHook {
  struct Rec {
    std::string name;
    hipEvent_t a = nullptr, b = nullptr;
  };
  bool on = false;
  std::vector<Rec> pending;
  std::map<std::string, std::pair<double, int64_t>> acc;
  void begin(const char* name, hipStream_t st) override {
    Rec r;
    r.name = name;
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return;
    (void)hipEventRecord(r.a, st);
    pending.push_back(r);
  }
  void end(hipStream_t st) override {
    if (!pending.empty()) (void)hipEventRecord(pending.back().b, st);
  }
  hipError_t collect() {
    hipError_t err = hipSuccess;
    for (Rec& r : pending) {
      float ms = 0.f;
      hipError_t e = hipEventSynchronize(r.b);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
      if (e == hipSuccess) {
        auto& v = acc[r.name];
        v.first += ms;
        v.second += 1;
      } else {
        err = e;
      }
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    pending.clear();
    return err;
  }
};

// Scratch of wct_raster_noalloc: the raster's tile counters, row lists and work items
// for callers that cannot allocate.  Each device holds its own copy from the library's
// first use on it until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: its device address comes from hipGetSymbolAddress, taken
// once per device with that device current and kept in g_scratch.
static_assert(WCT_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");
static __device__ __align__(256) char scratch[WCT_NOALLOC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
std::vector<void*> g_scratch;  // device address of `scratch`, by device ordinal

// The device address of `scratch` on device `dev` (which must be current).
int scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1, nullptr);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return WCT_OK;
}

}  // namespace

struct wct_plan {
  Profiler prof;
  int dtype = WCT_F32;
  int device = 0;
  int n_planes = 0;
  int max_events = 1;
  int n_cu = 256;
  size_t esize = 4;  // bytes of one real value
  std::vector<PlaneGeom> geom;
  std::vector<FftPlan> fp_t, fp_w;
  std::vector<void*> tw_t, post_t, tw_w, tw_w_rev, rtil;
  std::vector<void*> rtick;      // direct wire pass coefficients, [F padded][I][2K+1]
  std::vector<void*> rt64;       // FP64 tick spectrum of the response, [2K+1][I][F]: R~ is built
                                 // from it when a wire transform plan is first selected
  std::vector<int> wire_direct;  // wire pass (forward and adjoint) as direct sums, else fp_w
  DetTables* d_tables = nullptr;
  double* d_lfact = nullptr;  // ln(n!), n < kLfactTable, for the chop-down sampler
  void* scratch = nullptr;    // this device's static scratch (wct_raster_noalloc)
  std::vector<void*> noise_amp;  // per plane: amplitude spectrum / L_t, [F] in plan dtype (or null)
  std::vector<double> adc_gain, adc_base;  // per plane: ADC gain and pedestal (wct_plan_set_adc)
  std::vector<int> adc_max;                // per plane: largest ADC code
  std::vector<void*> allocs;
  int64_t grid_elems = 0, wave_elems = 0, shat_elems = 0, mhat_elems = 0;
  int64_t rows_ev = 0;  // impact rows per event, all planes
  int ntiles_ev = 0;
  int tile = 0;         // raster tile variant: index among the variants of the plan's dtype
  int tile_global = 0;  // the same variant's index in the whole list (wct_tile_variant_info)

  // wct_simulate_graph: instantiated graphs by call key, and the stream they are captured on
  std::map<std::string, hipGraphExec_t> graphs;
  hipStream_t cap_stream = nullptr;

  // wct_plan_create's device memory cap (WCT_PLAN_MEM_CAP; 0: none), what dalloc has
  // handed out, and whether the cap refused an allocation
  size_t mem_cap = 0, mem_used = 0;
  bool cap_hit = false;

  void* dalloc(size_t bytes, hipError_t* e) {
    void* p = nullptr;
    if (bytes == 0) bytes = 1;
    if (mem_cap && bytes > mem_cap - (mem_used < mem_cap ? mem_used : mem_cap)) {
      cap_hit = true;
      *e = hipErrorOutOfMemory;
      return nullptr;
    }
    *e = hipMalloc(&p, bytes);
    if (*e == hipSuccess) {
      allocs.push_back(p);
      mem_used += bytes;
    }
    return p;
  }
  // Graphs hold the plan's choices (transform plans, tile shape, noise spectra) and
  // buffers as kernel arguments: a set-up call that changes them drops them first.
  void drop_graphs() {
    if (graphs.empty()) return;
    (void)hipDeviceSynchronize();  // a replay may still run
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
  }
  ~wct_plan() {
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (void* p : allocs) (void)hipFree(p);
  }
};

namespace {

ProfHook* hook(wct_plan* P) { return P->prof.on ? &P->prof : nullptr; }

// Brackets one launch with profiler events when timing is enabled.
#define PROF_LAUNCH(P, name, st, expr, what)         \
  do {                                              \
    ProfHook* h__ = hook(P);                        \
    if (h__) h__->begin(name, st);                  \
    hipError_t e__ = (expr);                        \
    if (h__) h__->end(st);                          \
    if (e__ != hipSuccess) return hip_fail(e__, what); \
  } while (0)

RasterGeom raster_geom(const wct_plan* P, int n_events, int event_base) {
  RasterGeom g;
  std::memset(&g, 0, sizeof(g));
  g.n_planes = P->n_planes;
  g.n_events = n_events;
  g.event_base = event_base;
  g.ntiles_ev = P->ntiles_ev;
  g.grid_ev_stride = P->grid_elems;
  g.rows_ev = P->rows_ev;
  for (int p = 0; p < P->n_planes; ++p) g.pl[p] = P->geom[p];
  return g;
}

// Raster tiles of variant v (index in the whole list): tiles per plane and their offsets.
int set_tiles(wct_plan* P, int v) {
  int nvar = 0;
  const TileVariantDesc* tv = tile_variants(&nvar);
  if (v < 0 || v >= nvar || tv[v].dbl != (int)(P->dtype == WCT_F64))
    return fail(WCT_E_INVALID, "tile variant %d does not exist for this plan's dtype", v);
  int64_t toff = 0;
  std::vector<PlaneGeom> g = P->geom;
  for (PlaneGeom& G : g) {
    G.tile_off = toff;
    G.ntr = (G.nb + tv[v].th - 1) / tv[v].th;
    G.ntc = (G.nt + tv[v].tw - 1) / tv[v].tw;
    toff += (int64_t)G.ntr * G.ntc;
  }
  if (toff * (int64_t)P->max_events > 0x3fffffffLL)
    return fail(WCT_E_UNSUPPORTED, "too many raster tiles (%lld per event)", (long long)toff);
  P->geom = g;
  P->ntiles_ev = (int)toff;
  P->tile_global = v;
  int local = 0;
  for (int k = 0; k < v; ++k) local += tv[k].dbl == tv[v].dbl;
  P->tile = local;
  return WCT_OK;
}

// Workspace layouts ---------------------------------------------------------------
RasterWs carve_raster(const wct_plan* P, Carver& cv, int n_events, int64_t n_rows) {
  RasterWs w;
  w.ntiles = (int64_t)n_events * P->ntiles_ev;
  const int64_t nrow = n_rows > 0 ? n_rows : 1;
  w.max_items = w.ntiles + (4 * nrow + kRowsPerItem - 1) / kRowsPerItem + 1;
  const int64_t nsb = (w.ntiles + kScanPerBlock - 1) / kScanPerBlock;
  w.ctrl = static_cast<int32_t*>(cv.take(sizeof(int32_t) * (kCtrlWords + w.ntiles)));
  w.counts = w.ctrl ? w.ctrl + kCtrlWords : nullptr;
  w.rank = static_cast<int32_t*>(cv.take(sizeof(int32_t) * 4 * nrow));
  w.offs = static_cast<int32_t*>(cv.take(sizeof(int32_t) * (w.ntiles + 1)));
  w.item_off = static_cast<int32_t*>(cv.take(sizeof(int32_t) * (w.ntiles + 1)));
  w.items = static_cast<int32_t*>(cv.take(sizeof(int32_t) * w.max_items));
  w.list = static_cast<int32_t*>(cv.take(sizeof(int32_t) * 4 * nrow));
  w.big = static_cast<int32_t*>(cv.take(sizeof(int32_t) * nrow));
  w.blocks = static_cast<int32_t*>(cv.take(sizeof(int32_t) * 2 * (nsb > 0 ? nsb : 1)));
  return w;
}

struct ConvWs {
  void* shat;
  void* mhat;
};
ConvWs carve_conv(const wct_plan* P, Carver& cv, int n_events) {
  ConvWs c;
  c.shat = cv.take(2 * P->esize * (size_t)n_events * P->shat_elems);
  c.mhat = cv.take(2 * P->esize * (size_t)n_events * P->mhat_elems);
  return c;
}

// Bands of raster tile rows per event, all planes (the current tile variant's TH).
int64_t bands_ev(const wct_plan* P) {
  int64_t b = 0;
  for (const PlaneGeom& G : P->geom) b += G.ntr;
  return b;
}

// Tiles of the direct column pass per event (all planes) and each plane's first tile.
WireTileGeom wire_tile_geom(const wct_plan* P) {
  WireTileGeom g;
  std::memset(&g, 0, sizeof(g));
  g.n_planes = P->n_planes;
  g.rows_ev = P->rows_ev;
  for (int p = 0; p < P->n_planes; ++p) {
    const PlaneGeom& G = P->geom[p];
    g.nw[p] = G.nw;
    g.I[p] = G.I;
    g.K[p] = G.K;
    g.row_off[p] = G.row_off;
    g.tile_off[p] = g.tiles_ev;
    g.tiles_ev += (G.nw + kDirectTileWires - 1) / kDirectTileWires;
    g.wire_off[p] = g.wires_ev;
    g.wires_ev += G.nw;
  }
  g.tile_off[P->n_planes] = g.tiles_ev;
  g.wire_off[P->n_planes] = g.wires_ev;
  for (int p = 0; p < P->n_planes; ++p) {
    g.bit_off[p] = g.bits_ev;
    g.bits_ev += (P->geom[p].nw * P->geom[p].I + 31) / 32;
  }
  g.bit_off[P->n_planes] = g.bits_ev;
  return g;
}

size_t ws_bytes(const wct_plan* P, int op, int n_events, int64_t n_rows) {
  if (op == WCT_OP_RASTER) {
    Carver cv(nullptr);
    carve_raster(P, cv, n_events, n_rows);
    return align_up(cv.off, 256);
  }
  if (op == WCT_OP_CONVOLVE) {
    Carver cv(nullptr);
    carve_conv(P, cv, n_events);
    return align_up(cv.off, 256);
  }
  if (op == WCT_OP_SIMULATE) {
    Carver a(nullptr);
    a.take(P->esize * (size_t)n_events * P->grid_elems);
    const size_t head = align_up(a.off, 256);
    Carver r(nullptr), c(nullptr);
    carve_raster(P, r, n_events, n_rows);
    carve_conv(P, c, n_events);
    // the row spans, band hulls, tile flags and wire flags go last, so the grid and the
    // transform buffers keep their places
    const WireTileGeom tg = wire_tile_geom(P);
    return head + align_up(r.off > c.off ? r.off : c.off, 256) + align_up(sizeof(int2) * n_events * P->rows_ev, 256) +
           align_up(sizeof(int2) * n_events * bands_ev(P), 256) + align_up((size_t)n_events * tg.tiles_ev, 256) +
           align_up((size_t)n_events * tg.wires_ev, 256) + align_up(sizeof(uint32_t) * n_events * tg.bits_ev, 256);
  }
  if (op == WCT_OP_BACKWARD) {
    Carver a(nullptr);
    a.take(P->esize * (size_t)n_events * P->grid_elems);        // H = dL/dS
    a.take(2 * P->esize * (size_t)n_events * P->mhat_elems);    // dL/dM-hat
    a.take(2 * P->esize * (size_t)n_events * P->shat_elems);    // dL/dS-hat
    return align_up(a.off, 256);
  }
  return 0;
}

// Validation -----------------------------------------------------------------------
// batched: n_events may exceed max_events (wct_simulate processes sub-batches)
int check_opts(const wct_plan* P, const wct_opts* o, bool need_nsigma, bool batched = false) {
  if (!o) return fail(WCT_E_INVALID, "opts is NULL");
  if (o->n_events < 1 || (!batched && o->n_events > P->max_events))
    return fail(WCT_E_INVALID, "n_events %d outside [1, %d]", o->n_events, P->max_events);
  if (o->event_base < 0 || (int64_t)o->event_base + o->n_events > 0x7fffffffLL)
    return fail(WCT_E_INVALID, "event window [%d, %d + %d) out of range", o->event_base, o->event_base, o->n_events);
  if (o->noise != 0 && o->noise != 1) return fail(WCT_E_INVALID, "noise must be 0 or 1");
  if (need_nsigma && !(o->nsigma > 0.0 && o->nsigma <= 8.0))
    return fail(WCT_E_INVALID, "nsigma %g outside (0, 8]", o->nsigma);
  if (o->fluctuate < kModeMean || o->fluctuate > kModeNormal) return fail(WCT_E_INVALID, "fluctuate must be 0, 1 or 2");
  if (o->fluctuate && o->nsigma > 4.2)
    return fail(WCT_E_INVALID, "fluctuation needs nsigma <= 4.2 (the erf series range), got %g", o->nsigma);
  return WCT_OK;
}

int check_depos(const wct_depos* d) {
  if (!d) return fail(WCT_E_INVALID, "depos is NULL");
  if (d->n < 0 || d->n > 0x7fffffffLL) return fail(WCT_E_INVALID, "depos.n %lld out of range", (long long)d->n);
  if (d->n > 0 && (!d->q || !d->t || !d->p || !d->sigma_t || !d->sigma_p))
    return fail(WCT_E_INVALID, "depos float arrays must not be NULL");
  return WCT_OK;
}

template <typename T>
DepoView<T> view(const wct_depos* d) {
  DepoView<T> v;
  v.n = d->n;
  v.q = static_cast<const T*>(d->q);
  v.t = static_cast<const T*>(d->t);
  v.p = static_cast<const T*>(d->p);
  v.st = static_cast<const T*>(d->sigma_t);
  v.sp = static_cast<const T*>(d->sigma_p);
  v.plane = d->plane;
  v.event = d->event;
  v.depo_id = d->depo_id;
  return v;
}

// Launch sequences -------------------------------------------------------------------
template <typename T>
int run_raster(wct_plan* P, const wct_depos* d, const wct_opts* o, T* grid, Carver& cv, hipStream_t st,
               int2* span = nullptr, int2* hull = nullptr) {
  const RasterGeom g = raster_geom(P, o->n_events, o->event_base);
  RasterWs ws = carve_raster(P, cv, o->n_events, d->n);
  ws.span = span;
  ws.hull = hull;
  HIP_TRY(launch_raster<T>(view<T>(d), g, o->nsigma, o->fluctuate, o->seed, grid, ws, P->d_tables, P->d_lfact,
                           P->n_cu, st, hook(P), P->tile),
          "raster launch");
  return WCT_OK;
}


// span (optional): the raster's row tick spans of these events; the row transform then
// skips the work (not the zero output) of rows, or row pairs, that no window reached, and
// reads the others only inside their spans.  tiles (optional, with span): room for the
// direct column pass's tile flags of these events; a plane on the direct pass then skips
// the tiles no row reaches (zero M^ without reading S^), and its row transform does not
// write the zero spectra that only such tiles would read.  wires (optional, with tiles):
// room for the per-wire flags; on a plane of the direct column pass without noise, the
// inverse row transform writes the zero waveform of a wire no window reaches within the
// response's reach (its M^ is exactly zero there) without transforming it.
template <typename T>
int run_convolve(wct_plan* P, const T* grid, int n_events, T* wave, Carver& cv, hipStream_t st,
                 const int2* span = nullptr, const wct_opts* noise = nullptr, uint8_t* tiles = nullptr,
                 uint8_t* wires = nullptr, uint32_t* rbits = nullptr) {
  const ConvWs c = carve_conv(P, cv, n_events);
  cx<T>* shat = static_cast<cx<T>*>(c.shat);
  cx<T>* mhat = static_cast<cx<T>*>(c.mhat);
  const WireTileGeom tg = wire_tile_geom(P);
  const bool flags = span && tiles;
  if (flags) HIP_TRY(launch_wire_tiles(tg, n_events, span, tiles, st), "tile flag launch");
  if (flags && wires) HIP_TRY(launch_wire_live(tg, n_events, span, wires, st), "wire flag launch");
  if (flags && rbits) HIP_TRY(launch_row_bits(tg, n_events, span, rbits, st), "row flag launch");
  for (int p = 0; p < P->n_planes; ++p) {
    const PlaneGeom& G = P->geom[p];
    const cx<T>* tw_t = static_cast<const cx<T>*>(P->tw_t[p]);
    const cx<T>* post = static_cast<const cx<T>*>(P->post_t[p]);
    const cx<T>* tw_w = static_cast<const cx<T>*>(P->tw_w[p]);
    const cx<T>* tw_wr = static_cast<const cx<T>*>(P->tw_w_rev[p]);
    const int2* lv = span ? span + G.row_off : nullptr;
    WireTiles wt;
    if (flags && P->wire_direct[p]) {
      wt.live = tiles + tg.tile_off[p];
      wt.ev_stride = tg.tiles_ev;
      wt.ntile = tg.tile_off[p + 1] - tg.tile_off[p];
      if (rbits && G.I <= 10) {
        wt.rowbits = rbits + tg.bit_off[p];
        wt.bits_ev = tg.bits_ev;
      }
    }
    PROF_LAUNCH(P, "rows_r2c", st,
                launch_rows_r2c<T>(grid + G.grid_off, P->grid_elems, shat + G.shat_off, P->shat_elems, G.nt, G.I,
                                   G.nw, G.nchunk, n_events, P->fp_t[p], tw_t, post, P->n_cu, st, lv, P->rows_ev, wt),
                "row transform launch");
    if (P->wire_direct[p])
      PROF_LAUNCH(P, "colpass", st,
                  launch_colpass_direct<T>(shat + G.shat_off, P->shat_elems, static_cast<const cx<T>*>(P->rtick[p]),
                                           mhat + G.mhat_off, P->mhat_elems, G.nw, G.I, G.nchunk, n_events, st, wt),
                  "column pass launch");
    else
      PROF_LAUNCH(P, "colpass", st,
                  launch_colpass<T>(shat + G.shat_off, P->shat_elems, static_cast<const cx<T>*>(P->rtil[p]),
                                    mhat + G.mhat_off, P->mhat_elems, G.nw, G.I, G.nchunk, n_events, P->fp_w[p], tw_w,
                                    tw_wr, st),
                  "column pass launch");
    NoiseArgs<T> nz;  // Eq. 1's noise term, added to the half spectra before the inverse
    if (noise && noise->noise && P->noise_amp[p]) {
      nz.amp = static_cast<const T*>(P->noise_amp[p]);
      nz.key0 = (uint32_t)noise->seed;
      nz.key1 = (uint32_t)(noise->seed >> 32);
      nz.plane = (uint32_t)p;
      nz.event_base = noise->event_base;
    }
    WireLive wl;
    if (flags && wires && P->wire_direct[p] && !nz.amp) {
      wl.live = wires + tg.wire_off[p];
      wl.ev_stride = tg.wires_ev;
    }
    PROF_LAUNCH(P, "rows_c2r", st,
                launch_rows_c2r<T>(mhat + G.mhat_off, P->mhat_elems, wave + G.wave_off, P->wave_elems, G.nt, false,
                                   1, G.nw, G.nchunk, n_events, P->fp_t[p], tw_t, post, st, nz, wl),
                "inverse row transform launch");
  }
  return WCT_OK;
}

template <typename T>
int run_backward(wct_plan* P, const wct_depos* d, const wct_opts* o, const T* gw, T* gq, T* gt, T* gp, T* gst,
                 T* gsp, Carver& cv, hipStream_t st) {
  const int ne = o->n_events;
  T* H = static_cast<T*>(cv.take(P->esize * (size_t)ne * P->grid_elems));
  cx<T>* ghat = static_cast<cx<T>*>(cv.take(2 * P->esize * (size_t)ne * P->mhat_elems));
  cx<T>* hhat = static_cast<cx<T>*>(cv.take(2 * P->esize * (size_t)ne * P->shat_elems));
  for (int p = 0; p < P->n_planes; ++p) {
    const PlaneGeom& G = P->geom[p];
    const cx<T>* tw_t = static_cast<const cx<T>*>(P->tw_t[p]);
    const cx<T>* post = static_cast<const cx<T>*>(P->post_t[p]);
    const cx<T>* tw_w = static_cast<const cx<T>*>(P->tw_w[p]);
    const cx<T>* tw_wr = static_cast<const cx<T>*>(P->tw_w_rev[p]);
    PROF_LAUNCH(P, "adj_rows_r2c", st,
                launch_rows_r2c<T>(gw + G.wave_off, P->wave_elems, ghat + G.mhat_off, P->mhat_elems, G.nt, 1, G.nw,
                                   G.nchunk, ne, P->fp_t[p], tw_t, post, P->n_cu, st),
                "adjoint row transform launch");
    if (P->wire_direct[p])
      PROF_LAUNCH(P, "adj_colpass", st,
                  launch_colpass_adj_direct<T>(ghat + G.mhat_off, P->mhat_elems,
                                               static_cast<const cx<T>*>(P->rtick[p]), hhat + G.shat_off,
                                               P->shat_elems, G.nw, G.I, G.nchunk, ne, st),
                  "adjoint column pass launch");
    else
      PROF_LAUNCH(P, "adj_colpass", st,
                  launch_colpass_adj<T>(ghat + G.mhat_off, P->mhat_elems, static_cast<const cx<T>*>(P->rtil[p]),
                                        hhat + G.shat_off, P->shat_elems, G.nw, G.I, G.nchunk, ne, P->fp_w[p], tw_w,
                                        tw_wr, st),
                  "adjoint column pass launch");
    PROF_LAUNCH(P, "adj_rows_c2r", st,
                launch_rows_c2r<T>(hhat + G.shat_off, P->shat_elems, H + G.grid_off, P->grid_elems, G.nt, true, G.I,
                                   G.nw, G.nchunk, ne, P->fp_t[p], tw_t, post, st),
                "adjoint inverse row transform launch");
  }
  PROF_LAUNCH(P, "grad_gather", st,
              launch_grad_gather<T>(view<T>(d), raster_geom(P, ne, o->event_base), o->nsigma, H, gq, gt, gp, gst, gsp, st),
              "gradient gather launch");
  return WCT_OK;
}

// Plan creation ------------------------------------------------------------------------
template <typename T>
int upload_table(wct_plan* P, const std::vector<cx<double>>& h, void** out) {
  std::vector<cx<T>> v(h.size());
  for (size_t i = 0; i < h.size(); ++i) v[i] = mk((T)h[i].x, (T)h[i].y);
  hipError_t e;
  void* d = P->dalloc(sizeof(cx<T>) * v.size(), &e);
  if (e != hipSuccess) return fail(WCT_E_NOMEM, "hipMalloc of a twiddle table failed: %s", hipGetErrorString(e));
  HIP_TRY(hipMemcpy(d, v.data(), sizeof(cx<T>) * v.size(), hipMemcpyHostToDevice), "twiddle upload");
  *out = d;
  return WCT_OK;
}

// Whether a compiled variant of kind `vkind` can run a plane's transforms of `kind`
// (0 ticks, 1 wires): wire transforms take whole-chunk (1) or half-chunk (2) variants.
bool kind_fits(int vkind, int kind) { return kind == 0 ? vkind == 0 : (vkind == 1 || vkind == 2); }

// First compiled variant of a kind, precision and length, or -1.
int find_variant(int kind, bool dbl, int n) {
  int cnt = 0;
  const FftVariantDesc* v = fft_variants(&cnt);
  for (int i = 0; i < cnt; ++i)
    if (kind_fits(v[i].kind, kind) && v[i].dbl == (int)dbl && v[i].n == n) return i;
  return -1;
}

void free_table(wct_plan* P, void* d) {
  if (!d) return;
  for (size_t i = 0; i < P->allocs.size(); ++i)
    if (P->allocs[i] == d) {
      (void)hipFree(d);
      P->allocs.erase(P->allocs.begin() + i);
      return;
    }
}

// R~ of plane p (the wire transforms' 2D spectrum, 1/(L_w L_t) folded in), built from the
// plan's FP64 tick spectrum the first time a wire transform plan is selected: a plan
// that only runs the direct wire sums never holds it (3.4 GB on the three-plane
// geometry).  A set-up step: allocates and synchronises.
template <typename T>
int ensure_rtil(wct_plan* P, int p) {
  if (P->rtil[p]) return WCT_OK;
  const PlaneGeom& G = P->geom[p];
  std::vector<cx<double>> tlw(G.lw);
  for (int m = 0; m < G.lw; ++m) tlw[m] = wexp(m, G.lw);
  cx<double>* dtlw = nullptr;
  hipError_t e = hipMalloc(&dtlw, sizeof(cx<double>) * G.lw);
  void* rtil = nullptr;
  if (e == hipSuccess) rtil = P->dalloc(sizeof(cx<T>) * (size_t)G.nchunk * G.I * G.lw * kChunk, &e);
  if (e == hipSuccess) e = hipMemcpy(dtlw, tlw.data(), sizeof(cx<double>) * G.lw, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = launch_resp_wire<T>(static_cast<const cx<double>*>(P->rt64[p]), G.K, G.I, G.F, G.lw, G.lt, G.nchunk, dtlw,
                            static_cast<cx<T>*>(rtil), nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  (void)hipFree(dtlw);
  if (e != hipSuccess) {
    free_table(P, rtil);
    return hip_fail(e, "wire transform spectrum");
  }
  P->rtil[p] = rtil;
  return WCT_OK;
}

// (Re)builds the transform plan and twiddle tables of plane p along ticks (kind 0) or
// wires (kind 1): compiled variant v, or the runtime plan (v < 0).  Column variants
// also get the table of their radices reversed (the inverse transform's plan).
template <typename T>
int set_fft(wct_plan* P, int p, int kind, int v) {
  const PlaneGeom& G = P->geom[p];
  if (v == WCT_WIRE_DIRECT) {
    if (kind != 1) return fail(WCT_E_INVALID, "the direct sum applies to the wire pass (kind 1) only");
    if (!colpass_direct_fits(G.K))
      return fail(WCT_E_UNSUPPORTED, "plane %d: direct wire pass needs a response of 21 wires (K = 10), K = %d", p,
                  G.K);
    P->wire_direct[p] = 1;
    return WCT_OK;
  }
  if (v < 0) v = -1;
  const int n = kind == 0 ? G.M : G.lw;
  FftPlan fp;
  std::vector<cx<double>> tw, twr;
  if (v >= 0) {
    int cnt = 0;
    const FftVariantDesc* vd = fft_variants(&cnt);
    if (v >= cnt || !kind_fits(vd[v].kind, kind) || vd[v].dbl != (int)(sizeof(T) == 8) || vd[v].n != n)
      return fail(WCT_E_INVALID, "transform variant %d does not apply to plane %d kind %d (length %d)", v, p, kind,
                  n);
    if (!build_fft_variant(vd[v], v, fp, tw)) return fail(WCT_E_INVALID, "transform variant %d: bad plan", v);
    std::vector<int> rad(vd[v].radix, vd[v].radix + vd[v].npass);
    std::reverse(rad.begin(), rad.end());
    FftPlan fr;
    if (kind != 0 && !build_fft_radices(n, rad, fr, twr))
      return fail(WCT_E_INVALID, "transform variant %d: bad reversed plan", v);
  } else if (!build_fft(n, 0, fp, tw)) {
    return fail(WCT_E_UNSUPPORTED, "plane %d: length %d not 2,3,5-smooth", p, n);
  }
  void* d = nullptr;
  int rc = upload_table<T>(P, tw, &d);
  if (rc) return rc;
  void* dr = d;
  if (!twr.empty()) {
    rc = upload_table<T>(P, twr, &dr);
    if (rc) return rc;
  }
  if (kind == 0) {
    free_table(P, P->tw_t[p]);
    P->fp_t[p] = fp;
    P->tw_t[p] = d;
  } else {
    if (P->tw_w_rev[p] != P->tw_w[p]) free_table(P, P->tw_w_rev[p]);
    free_table(P, P->tw_w[p]);
    P->fp_w[p] = fp;
    P->tw_w[p] = d;
    P->tw_w_rev[p] = dr;
    if ((size_t)p < P->rtil.size()) {  // set after plan creation: the transforms run now
      P->wire_direct[p] = 0;
      return ensure_rtil<T>(P, p);
    }
  }
  return WCT_OK;
}

template <typename T>
int plan_tables(wct_plan* P, const wct_plan_desc* desc) {
  const size_t lds_max = 160 * 1024;
  for (int p = 0; p < P->n_planes; ++p) {
    PlaneGeom& G = P->geom[p];
    if ((size_t)G.M * sizeof(cx<T>) > lds_max || !conv_fits<T>(G.M))
      return fail(WCT_E_UNSUPPORTED, "plane %d: tick transform length %d exceeds the LDS-resident limit", p, G.lt);
    if ((size_t)G.lw * kChunk * sizeof(cx<T>) > lds_max || !conv_fits<T>(G.lw * kChunk))
      return fail(WCT_E_UNSUPPORTED, "plane %d: wire transform length %d exceeds the LDS-resident limit", p, G.lw);
    P->fp_t.emplace_back();
    P->fp_w.emplace_back();
    P->tw_t.push_back(nullptr);
    P->tw_w.push_back(nullptr);
    P->tw_w_rev.push_back(nullptr);
    P->wire_direct.push_back(0);
    int rc = set_fft<T>(P, p, 0, find_variant(0, sizeof(T) == 8, G.M));
    if (rc) return rc;
    rc = set_fft<T>(P, p, 1, find_variant(1, sizeof(T) == 8, G.lw));
    if (rc) return rc;
    // the wire pass (forward and adjoint) defaults to the direct sums where the response
    // allows them (about twice as fast as the transform pair on MI355X)
    if (colpass_direct_fits(G.K)) P->wire_direct[p] = 1;
    std::vector<cx<double>> post(G.M + 1);
    for (int k = 0; k <= G.M; ++k) post[k] = wexp(k, G.lt);
    void* d = nullptr;
    rc = upload_table<T>(P, post, &d);
    if (rc) return rc;
    P->post_t.push_back(d);

    // response spectrum, FP64 on the device, stored in the plan dtype
    const wct_plane_desc& pd = desc->planes[p];
    const int nk = 2 * G.K + 1;
    const size_t nr = (size_t)nk * G.I * G.TR;
    std::vector<double> R(nr);
    for (size_t i = 0; i < nr; ++i) R[i] = (double)static_cast<const T*>(pd.response)[i];
    std::vector<cx<double>> tlt(G.lt);
    for (int m = 0; m < G.lt; ++m) tlt[m] = wexp(m, G.lt);
    double* dR = nullptr;
    cx<double>* dtlt = nullptr;
    hipError_t e = hipMalloc(&dR, sizeof(double) * nr);
    if (e == hipSuccess) e = hipMalloc(&dtlt, sizeof(cx<double>) * G.lt);
    void* drt = nullptr;
    void* rtick = nullptr;
    if (e == hipSuccess) drt = P->dalloc(sizeof(cx<double>) * (size_t)nk * G.I * G.F, &e);
    if (e == hipSuccess) rtick = P->dalloc(sizeof(cx<T>) * (size_t)G.nchunk * kChunk * G.I * nk, &e);
    if (e == hipSuccess) e = hipMemcpy(dR, R.data(), sizeof(double) * nr, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dtlt, tlt.data(), sizeof(cx<double>) * G.lt, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_resp_tick(dR, nk, G.I, G.TR, G.lt, G.F, dtlt, static_cast<cx<double>*>(drt), nullptr);
    if (e == hipSuccess)
      e = launch_resp_tick_pack<T>(static_cast<cx<double>*>(drt), G.K, G.I, G.F, G.nchunk * kChunk, G.lt,
                                   static_cast<cx<T>*>(rtick), nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    (void)hipFree(dR);
    (void)hipFree(dtlt);
    if (e != hipSuccess) return hip_fail(e, "response spectrum");
    P->rt64.push_back(drt);
    P->rtick.push_back(rtick);
    P->rtil.push_back(nullptr);
    // the 2D spectrum of the wire transforms only where they run
    if (!P->wire_direct[p] && (rc = ensure_rtil<T>(P, p))) return rc;
  }
  return WCT_OK;
}

// Fraction by which a raster tile variant must beat the one kept so far to replace it.
constexpr float kTileMargin = 0.015f;

// Position of variant v in a candidate list (v is in it).
size_t best_at(const std::vector<int>& cand, int v) {
  size_t i = 0;
  while (cand[i] != v) ++i;
  return i;
}

// Timing of the tuners' candidates: the candidates run in turn for kRounds rounds of kReps
// back-to-back runs each; the first round only warms up (clocks ramp, caches fill), and a
// candidate's time is its fastest later round.  Taking turns keeps a slow start of the
// device, or load from elsewhere, from favouring the candidates timed last.
template <typename SetF, typename RunF>
int time_round_robin(const std::vector<int>& cand, SetF set_variant, RunF run_once, hipStream_t st,
                     std::vector<float>* ms_out) {
  constexpr int kRounds = 4, kReps = 3;
  ms_out->assign(cand.size(), 0.f);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  int rc = e == hipSuccess ? WCT_OK : fail(WCT_E_DEVICE, "event create: %s", hipGetErrorString(e));
  for (int round = 0; round < kRounds && rc == WCT_OK; ++round) {
    for (size_t c = 0; c < cand.size() && rc == WCT_OK; ++c) {
      if ((rc = set_variant(cand[c]))) break;
      if (hipEventRecord(e0, st) != hipSuccess) rc = fail(WCT_E_DEVICE, "event record");
      for (int rep = 0; rep < kReps && rc == WCT_OK; ++rep) rc = run_once();
      float ms = 0.f;
      if (rc == WCT_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = fail(WCT_E_DEVICE, "timing the tuner's candidates failed");
      if (rc == WCT_OK && round > 0 && (round == 1 || ms < (*ms_out)[c])) (*ms_out)[c] = ms;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return rc;
}

// Autotuning of the transform variants -------------------------------------------------
// Cache file: one line per (geometry, dtype, kind) with the chosen variant's threads and
// radices ("runtime" for the runtime plan), e.g.
//   wct-fft f32 2400 9600 10 10 200 kind 1 -> 540 9 9 5 6
std::string tune_key(const wct_plan* P, int p, int kind) {
  const PlaneGeom& G = P->geom[p];
  char b[160];
  std::snprintf(b, sizeof(b), "wct-fft %s %d %d %d %d %d kind %d", P->dtype == WCT_F32 ? "f32" : "f64", G.nw, G.nt,
                G.I, G.K, G.TR, kind);
  return b;
}
std::string variant_text(int v) {
  if (v == WCT_WIRE_DIRECT) return "direct";
  if (v < 0) return "runtime";
  int cnt = 0;
  const FftVariantDesc* d = fft_variants(&cnt);
  std::string s = (d[v].kind == 2 ? "half " : "") + std::to_string(d[v].threads);
  for (int k = 0; k < d[v].npass; ++k) s += " " + std::to_string(d[v].radix[k]);
  return s;
}
std::map<std::string, std::string> read_tune_cache(const char* path) {
  std::map<std::string, std::string> m;
  if (!path) return m;
  FILE* f = std::fopen(path, "r");
  if (!f) return m;
  char line[512];
  while (std::fgets(line, sizeof(line), f)) {
    std::string l(line);
    while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
    const size_t a = l.find(" -> ");
    if (a != std::string::npos) m[l.substr(0, a)] = l.substr(a + 4);
  }
  std::fclose(f);
  return m;
}

template <typename T>
int run_tune(wct_plan* P, int n_events, const char* cache_path, void* ws, hipStream_t st) {
  Carver cv(ws);
  T* grid = static_cast<T*>(cv.take(P->esize * (size_t)n_events * P->grid_elems));
  T* wave = static_cast<T*>(cv.take(P->esize * (size_t)n_events * P->wave_elems));
  const size_t conv_off = align_up(cv.off, 256);
  // every cell nonzero (0x3ff00000 in each 32-bit word: 1.875f, or about 1.0 as a
  // double), so that no row transform is skipped as empty while timing
  HIP_TRY(launch_fill_i32(reinterpret_cast<int32_t*>(grid), (int64_t)(P->esize / 4) * n_events * P->grid_elems,
                          0x3ff00000, st),
          "tune grid fill");
  auto cache = read_tune_cache(cache_path);
  auto run_once = [&]() -> int {
    Carver cc(static_cast<char*>(ws) + conv_off);
    return run_convolve<T>(P, grid, n_events, wave, cc, st);
  };
  int cnt = 0;
  const FftVariantDesc* vd = fft_variants(&cnt);
  std::string appended;
  int rc = WCT_OK;
  for (int p = 0; p < P->n_planes && rc == WCT_OK; ++p) {
    for (int kind = 0; kind < 2 && rc == WCT_OK; ++kind) {
      const int n = kind == 0 ? P->geom[p].M : P->geom[p].lw;
      std::vector<int> cand;
      for (int v = 0; v < cnt; ++v)
        if (kind_fits(vd[v].kind, kind) && vd[v].dbl == (int)(sizeof(T) == 8) && vd[v].n == n) cand.push_back(v);
      cand.push_back(-1);
      if (kind == 1 && colpass_direct_fits(P->geom[p].K)) cand.push_back(WCT_WIRE_DIRECT);
      const std::string key = tune_key(P, p, kind);
      auto it = cache.find(key);
      constexpr int kNone = -1000;
      int best = kNone, best_fft = kNone;  // best_fft: the transform plan the adjoint keeps
      if (it != cache.end())
        for (int v : cand)
          if (variant_text(v) == it->second) best = v;
      if (best == kNone) {
        std::vector<float> ms;
        if ((rc = time_round_robin(cand, [&](int v) { return set_fft<T>(P, p, kind, v); }, run_once, st, &ms))) break;
        for (size_t c = 0; c < cand.size(); ++c) {
          if (best == kNone || ms[c] < ms[best_at(cand, best)]) best = cand[c];
          if (cand[c] != WCT_WIRE_DIRECT && (best_fft == kNone || ms[c] < ms[best_at(cand, best_fft)]))
            best_fft = cand[c];
        }
        appended += key + " -> " + variant_text(best) + "\n";
        cache[key] = variant_text(best);  // planes of the same geometry take the same choice
      }
      // with the direct sums chosen, the plane keeps the fastest transform plan timed
      // (or, from the cache, its current one) for a later set_fft of -1 or a variant
      if (best == WCT_WIRE_DIRECT && best_fft != kNone) rc = set_fft<T>(P, p, kind, best_fft);
      if (rc == WCT_OK) rc = set_fft<T>(P, p, kind, best);
    }
  }
  if (rc) return rc;
  if (cache_path && !appended.empty()) {
    FILE* f = std::fopen(cache_path, "a");
    if (!f) return fail(WCT_E_INVALID, "cannot append to tune cache %s", cache_path);
    std::fputs(appended.c_str(), f);
    std::fclose(f);
  }
  return WCT_OK;
}

size_t tune_ws_bytes(const wct_plan* P, int n_events) {
  Carver a(nullptr);
  a.take(P->esize * (size_t)n_events * P->grid_elems);
  a.take(P->esize * (size_t)n_events * P->wave_elems);
  return align_up(a.off, 256) + ws_bytes(P, WCT_OP_CONVOLVE, n_events, 0);
}

// Autotuning of the raster tile ---------------------------------------------------------
// Cache line per (dtype, plane geometries, mean or fluctuated raster), e.g.
//   wct-tile f32 3 2400 9600 10 2400 9600 10 3456 9600 10 fluct 1 -> 128 64 4
std::string tile_key(const wct_plan* P, int fluctuate) {
  std::string k = std::string("wct-tile ") + (P->dtype == WCT_F32 ? "f32" : "f64") + " " + std::to_string(P->n_planes);
  for (const PlaneGeom& G : P->geom) k += " " + std::to_string(G.nw) + " " + std::to_string(G.nt) + " " + std::to_string(G.I);
  return k + " fluct " + std::to_string(fluctuate);
}
std::string tile_text(int v) {
  int n = 0;
  const TileVariantDesc* tv = tile_variants(&n);
  return std::to_string(tv[v].th) + " " + std::to_string(tv[v].tw) + " " + std::to_string(tv[v].blocks_per_cu);
}
// Workspace of the raster tuner: the grid of n_events events plus the largest raster
// workspace over the tile variants of the plan's dtype.
size_t tune_raster_ws_bytes(wct_plan* P, int n_events, int64_t n_rows) {
  const int keep = P->tile_global;
  int nvar = 0;
  const TileVariantDesc* tv = tile_variants(&nvar);
  size_t most = 0;
  for (int v = 0; v < nvar; ++v) {
    if (tv[v].dbl != (int)(P->dtype == WCT_F64) || set_tiles(P, v)) continue;
    const size_t b = ws_bytes(P, WCT_OP_RASTER, n_events, n_rows);
    most = b > most ? b : most;
  }
  (void)set_tiles(P, keep);
  return align_up(P->esize * (size_t)n_events * P->grid_elems, 256) + most;
}

template <typename T>
int run_tune_raster(wct_plan* P, const wct_depos* d, const wct_opts* o, const char* cache_path, void* ws,
                    hipStream_t st) {
  auto cache = read_tune_cache(cache_path);
  const std::string key = tile_key(P, o->fluctuate);
  int nvar = 0;
  const TileVariantDesc* tv = tile_variants(&nvar);
  std::vector<int> cand;
  for (int v = 0; v < nvar; ++v)
    if (tv[v].dbl == (int)(sizeof(T) == 8)) cand.push_back(v);
  auto it = cache.find(key);
  if (it != cache.end())
    for (int v : cand)
      if (tile_text(v) == it->second) return set_tiles(P, v);
  T* grid = static_cast<T*>(ws);
  char* rws = static_cast<char*>(ws) + align_up(P->esize * (size_t)o->n_events * P->grid_elems, 256);
  std::vector<float> ms;
  int rc = time_round_robin(cand, [&](int v) { return set_tiles(P, v); },
                            [&]() -> int {
                              Carver cv(rws);
                              return run_raster<T>(P, d, o, grid, cv, st);
                            },
                            st, &ms);
  if (rc) return rc;
  // a later variant replaces the one kept so far only when clearly faster: the first
  // (the plan's default) wins ties within the timing noise of a few percent
  int best = cand[0];
  for (size_t c = 1; c < cand.size(); ++c)
    if (ms[c] < (1.0f - kTileMargin) * ms[best_at(cand, best)]) best = cand[c];
  if ((rc = set_tiles(P, best))) return rc;
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "a");
    if (!f) return fail(WCT_E_INVALID, "cannot append to tune cache %s", cache_path);
    std::fputs((key + " -> " + tile_text(best) + "\n").c_str(), f);
    std::fclose(f);
  }
  return WCT_OK;
}

}  // namespace

// A named range (roctx) around each call that enqueues work, so that a trace with markers
// (rocprofv3 --marker-trace) groups the kernels under the call that launched them.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

extern "C" {

int wct_abi_version(void) { return WCT_ABI_VERSION; }
int wct_fluct_spec_version(void) { return WCT_FLUCT_SPEC_VERSION; }
const char* wct_last_error(void) { return g_err.c_str(); }

int wct_plan_create(const wct_plan_desc* desc, wct_plan** out) {
  TraceRange trace_range("wct_plan_create");
  g_err.clear();
  if (!out) return fail(WCT_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!desc) return fail(WCT_E_INVALID, "desc is NULL");
  if (desc->dtype != WCT_F32 && desc->dtype != WCT_F64) return fail(WCT_E_INVALID, "dtype %d", desc->dtype);
  if (desc->n_planes < 1 || desc->n_planes > kMaxPlanes)
    return fail(WCT_E_INVALID, "n_planes %d outside [1, %d]", desc->n_planes, kMaxPlanes);
  if (!desc->planes) return fail(WCT_E_INVALID, "planes is NULL");
  if (desc->max_events < 1) return fail(WCT_E_INVALID, "max_events %d < 1", desc->max_events);
  size_t mem_cap = 0;
  if (const char* cs = std::getenv("WCT_PLAN_MEM_CAP")) {
    char* end = nullptr;
    errno = 0;
    const unsigned long long v = std::strtoull(cs, &end, 10);
    if (end == cs || *end != '\0' || errno != 0 || cs[0] == '-')
      return fail(WCT_E_INVALID, "WCT_PLAN_MEM_CAP=\"%s\" is not a byte count", cs);
    mem_cap = (size_t)v;
  }

  wct_plan* P = new wct_plan();
  P->dtype = desc->dtype;
  P->device = desc->device;
  P->n_planes = desc->n_planes;
  P->max_events = desc->max_events;
  P->esize = desc->dtype == WCT_F32 ? 4 : 8;
  int64_t goff = 0, woff = 0, soff = 0, moff = 0, roff = 0;
  for (int p = 0; p < P->n_planes; ++p) {
    const wct_plane_desc& pd = desc->planes[p];
    if (pd.n_wires < 1 || pd.n_ticks < 1 || pd.n_impacts < 1 || pd.half_wires < 0 || pd.resp_ticks < 1 ||
        !pd.response) {
      delete P;
      return fail(WCT_E_INVALID, "plane %d: bad geometry or NULL response", p);
    }
    PlaneGeom G;
    std::memset(&G, 0, sizeof(G));
    G.nw = pd.n_wires;
    G.nt = pd.n_ticks;
    G.I = pd.n_impacts;
    G.K = pd.half_wires;
    G.TR = pd.resp_ticks;
    G.nb = G.I * G.nw;
    const int64_t nbt = (int64_t)G.nb * G.nt;
    if ((int64_t)G.nb > 0x7fffffff / 2 || nbt >= (1LL << 32)) {
      delete P;
      return fail(WCT_E_UNSUPPORTED, "plane %d: grid of %lld cells exceeds 2^32", p, (long long)nbt);
    }
    G.lw = (int)next_smooth((int64_t)G.nw + G.K);
    G.lt = 2 * (int)next_smooth(((int64_t)G.nt + G.TR - 1 + 1) / 2);
    G.M = G.lt / 2;
    G.F = G.M + 1;
    G.nchunk = (G.F + kChunk - 1) / kChunk;
    G.grid_off = goff;
    G.wave_off = woff;
    G.shat_off = soff;
    G.mhat_off = moff;
    G.row_off = roff;
    goff += nbt;
    woff += (int64_t)G.nw * G.nt;
    soff += (int64_t)G.nchunk * kChunk * G.nb;
    moff += (int64_t)G.nw * G.nchunk * kChunk;
    roff += G.nb;
    P->geom.push_back(G);
  }
  P->noise_amp.assign(P->n_planes, nullptr);
  P->adc_gain.assign(P->n_planes, 1.0);
  P->adc_base.assign(P->n_planes, 0.0);
  P->adc_max.assign(P->n_planes, 65535);
  P->rows_ev = roff;
  P->grid_elems = goff;
  P->wave_elems = woff;
  P->shat_elems = soff;
  P->mhat_elems = moff;
  {
    // the per-event buffers of max_events events (grid, both spectra twice over, rows'
    // records) must stay far from the size_t range of the workspace arithmetic
    const double per_ev = (double)P->esize * (double)(goff + woff + 4 * soff + 4 * moff) + 64.0 * (double)roff;
    if ((double)P->max_events * per_ev > 0x1p60) {
      delete P;
      return fail(WCT_E_UNSUPPORTED, "max_events %d x %.3g bytes of buffers per event exceeds 2^60 bytes",
                  desc->max_events, per_ev);
    }
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    delete P;
    return fail(WCT_E_DEVICE, "no HIP device available");
  }
  if (desc->device < 0 || desc->device >= ndev) {
    delete P;
    return fail(WCT_E_INVALID, "device %d of %d", desc->device, ndev);
  }
  int tile0 = -1, nvar = 0;  // the first tile variant of the dtype
  const TileVariantDesc* tv = tile_variants(&nvar);
  for (int v = 0; v < nvar && tile0 < 0; ++v)
    if (tv[v].dbl == (int)(P->dtype == WCT_F64)) tile0 = v;
  if (int rc0 = set_tiles(P, tile0)) {
    delete P;
    return rc0;
  }

  DeviceGuard dg(P->device);
  if (!dg.ok) {
    delete P;
    return fail(WCT_E_DEVICE, "hipSetDevice(%d) failed", desc->device);
  }
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, P->device) == hipSuccess && ncu > 0)
    P->n_cu = ncu;
  conv_init_kernels();
  int rc = scratch_address(P->device, &P->scratch);
  if (rc) {
    delete P;
    return rc;
  }
  P->mem_cap = mem_cap;
  // a refusal by the cap reports as such, whichever allocation it met
  auto capped = [&](int code) {
    if (P->cap_hit)
      code = fail(WCT_E_NOMEM, "the plan's device tables need more than WCT_PLAN_MEM_CAP = %zu bytes", mem_cap);
    delete P;
    return code;
  };
  rc = P->dtype == WCT_F32 ? plan_tables<float>(P, desc) : plan_tables<double>(P, desc);
  if (rc) return capped(rc);
  DetTables tb;
  std::memset(&tb, 0, sizeof(tb));
  for (int j = 1; j < 256; ++j) tb.inv[j] = 1.0 / (double)j;
  double f = 1.0;
  for (int j = 0; j <= 18; ++j) {
    if (j > 0) f *= (double)j;
    tb.fact[j] = f;
    if (j <= 16) tb.inv_fact[j] = 1.0 / f;
  }
  hipError_t e;
  P->d_tables = static_cast<DetTables*>(P->dalloc(sizeof(DetTables), &e));
  if (e != hipSuccess) return capped(fail(WCT_E_NOMEM, "hipMalloc failed: %s", hipGetErrorString(e)));
  e = hipMemcpy(P->d_tables, &tb, sizeof(tb), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    delete P;
    return hip_fail(e, "table upload");
  }
  P->d_lfact = static_cast<double*>(P->dalloc(sizeof(double) * kLfactTable, &e));
  if (e == hipSuccess) e = launch_lfact_table(P->d_lfact, kLfactTable, P->d_tables, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return capped(hip_fail(e, "log-factorial table"));
  P->mem_cap = 0;  // the cap is plan creation's: later set-up calls allocate freely
  *out = P;
  return WCT_OK;
}

void wct_plan_destroy(wct_plan* plan) {
  if (!plan) return;
  DeviceGuard dg(plan->device);
  (void)hipDeviceSynchronize();
  delete plan;
}

int64_t wct_grid_elems(const wct_plan* plan) { return plan ? plan->grid_elems : -1; }
int64_t wct_wave_elems(const wct_plan* plan) { return plan ? plan->wave_elems : -1; }

int wct_plane_info(const wct_plan* plan, int32_t plane, int64_t out[10]) {
  g_err.clear();
  if (!plan || !out) return fail(WCT_E_INVALID, "NULL argument");
  if (plane < 0 || plane >= plan->n_planes) return fail(WCT_E_INVALID, "plane %d of %d", plane, plan->n_planes);
  const PlaneGeom& G = plan->geom[plane];
  const int64_t v[10] = {G.nw, G.nt, G.I, G.K, G.TR, G.lw, G.lt, G.F, G.grid_off, G.wave_off};
  for (int i = 0; i < 10; ++i) out[i] = v[i];
  return WCT_OK;
}

size_t wct_workspace_bytes(const wct_plan* plan, int32_t op, int32_t n_events, int64_t n_rows) {
  if (!plan || n_events < 1 || n_rows < 0) return 0;
  if (op == WCT_OP_SIMULATE && n_events > plan->max_events) n_events = plan->max_events;  // sub-batched
  if (n_events > plan->max_events) return 0;
  return ws_bytes(plan, op, n_events, n_rows);
}

int wct_raster(wct_plan* plan, const wct_depos* depos, const wct_opts* opts, void* grid, void* ws, size_t ws_size,
               void* stream) {
  TraceRange trace_range("wct_raster");
  g_err.clear();
  if (!plan) return fail(WCT_E_INVALID, "plan is NULL");
  int rc = check_opts(plan, opts, true);
  if (rc) return rc;
  if ((rc = check_depos(depos))) return rc;
  if (!grid) return fail(WCT_E_INVALID, "grid is NULL");
  const size_t need = ws_bytes(plan, WCT_OP_RASTER, opts->n_events, depos->n);
  if (!ws || ws_size < need) return fail(WCT_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_size, need);
  DeviceGuard dg(plan->device);
  if (!dg.ok) return fail(WCT_E_DEVICE, "hipSetDevice(%d) failed", plan->device);
  Carver cv(ws);
  hipStream_t st = static_cast<hipStream_t>(stream);
  return plan->dtype == WCT_F32 ? run_raster<float>(plan, depos, opts, static_cast<float*>(grid), cv, st)
                                : run_raster<double>(plan, depos, opts, static_cast<double*>(grid), cv, st);
}

int wct_plan_set_noise(wct_plan* plan, int32_t plane, const double* amp, int64_t n) {
  g_err.clear();
  if (!plan) return fail(WCT_E_INVALID, "plan is NULL");
  plan->drop_graphs();
  if (plane < 0 || plane >= plan->n_planes) return fail(WCT_E_INVALID, "plane %d of %d", plane, plan->n_planes);
  const PlaneGeom& G = plan->geom[plane];
  if (!amp) {  // no noise on this plane (the buffer stays with the plan)
    if (plan->noise_amp[plane]) {
      DeviceGuard dg(plan->device);
      (void)hipDeviceSynchronize();  // queued work may still read it
    }
    plan->noise_amp[plane] = nullptr;
    return WCT_OK;
  }
  if (n != G.F) return fail(WCT_E_INVALID, "noise spectrum of %lld values, the plane has %d frequencies", (long long)n, G.F);
  for (int64_t k = 0; k < n; ++k)
    if (!(amp[k] >= 0.0) || !std::isfinite(amp[k]))
      return fail(WCT_E_INVALID, "noise amplitude %lld is negative or not finite", (long long)k);
  DeviceGuard dg(plan->device);
  if (!dg.ok) return fail(WCT_E_DEVICE, "hipSetDevice(%d) failed", plan->device);
  hipError_t e = hipDeviceSynchronize();  // queued work may still read the old values
  if (e != hipSuccess) return hip_fail(e, "synchronise before the noise upload");
  void* d = plan->noise_amp[plane];
  if (!d) {
    d = plan->dalloc(plan->esize * (size_t)n, &e);
    if (e != hipSuccess) return fail(WCT_E_NOMEM, "hipMalloc of a noise spectrum failed: %s", hipGetErrorString(e));
  }
  // the inverse row transform is unnormalised: store A[k] / L_t
  if (plan->dtype == WCT_F32) {
    std::vector<float> v(n);
    for (int64_t k = 0; k < n; ++k) v[k] = (float)(amp[k] / (double)G.lt);
    e = hipMemcpy(d, v.data(), sizeof(float) * n, hipMemcpyHostToDevice);
  } else {
    std::vector<double> v(n);
    for (int64_t k = 0; k < n; ++k) v[k] = amp[k] / (double)G.lt;
    e = hipMemcpy(d, v.data(), sizeof(double) * n, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_fail(e, "noise spectrum upload");
  plan->noise_amp[plane] = d;
  return WCT_OK;
}

int wct_raster_noalloc(wct_plan* plan, const wct_depos* depos, const wct_opts* opts, void* grid, void* stream) {
  g_err.clear();
  if (!plan) return fail(WCT_E_INVALID, "plan is NULL");
  int rc = check_opts(plan, opts, true);
  if (rc) return rc;
  if ((rc = check_depos(depos))) return rc;
  if (!grid) return fail(WCT_E_INVALID, "grid is NULL");
  const size_t need = ws_bytes(plan, WCT_OP_RASTER, opts->n_events, depos->n);
  if (need > (size_t)WCT_NOALLOC_SCRATCH_BYTES)
    return fail(WCT_E_WORKSPACE, "wct_raster_noalloc: %lld rows x %d events need %zu bytes of scratch, above its %zu",
                (long long)depos->n, opts->n_events, need, (size_t)WCT_NOALLOC_SCRATCH_BYTES);
  if (!plan->scratch) return fail(WCT_E_DEVICE, "wct_raster_noalloc: no scratch address for device %d", plan->device);
  DeviceGuard dg(plan->device);
  if (!dg.ok) return fail(WCT_E_DEVICE, "hipSetDevice(%d) failed", plan->device);
  Carver cv(plan->scratch);  // the kernels get the device address, never `scratch` itself
  hipStream_t st = static_cast<hipStream_t>(stream);
  return plan->dtype == WCT_F32 ? run_raster<float>(plan, depos, opts, static_cast<float*>(grid), cv, st)
                                : run_raster<double>(plan, depos, opts, static_cast<double*>(grid), cv, st);
}

static_assert(kMaxPlanes == WCT_MAX_PLANES, "plane limit of the kernels and of the ABI");

int wct_drift(const wct_plan* plan, const wct_depos3d* in, const wct_drift_params* prm, const wct_depos_out* out,
              void* stream) {
  TraceRange trace_range("wct_drift");
  g_err.clear();
  if (!plan || !in || !prm || !out) return fail(WCT_E_INVALID, "NULL argument");
  if (in->n < 0) return fail(WCT_E_INVALID, "n = %lld < 0", (long long)in->n);
  if (in->n > 0 && (!in->x || !in->y || !in->z || !in->t0 || !in->q || !in->sigma_l || !in->sigma_t))
    return fail(WCT_E_INVALID, "a deposition array is NULL");
  if (in->n > 0 && (!out->q || !out->t || !out->p || !out->sigma_t || !out->sigma_p || !out->plane || !out->event ||
                    !out->depo_id))
    return fail(WCT_E_INVALID, "a row array is NULL");
  if (!(prm->drift_speed > 0.0) || !std::isfinite(prm->drift_speed) || !(prm->tick > 0.0) ||
      !std::isfinite(prm->tick))
    return fail(WCT_E_INVALID, "drift speed and tick must be positive and finite");
  if (!(prm->diffusion_l >= 0.0) || !(prm->diffusion_t >= 0.0) || !std::isfinite(prm->diffusion_l) ||
      !std::isfinite(prm->diffusion_t) || !std::isfinite(prm->lifetime))
    return fail(WCT_E_INVALID, "diffusion constants must be finite and >= 0, the lifetime finite");
  DriftArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n_planes = plan->n_planes;
  a.speed = prm->drift_speed;
  a.dl = prm->diffusion_l;
  a.dt = prm->diffusion_t;
  a.lifetime = prm->lifetime;
  a.tick = prm->tick;
  for (int k = 0; k < plan->n_planes; ++k) {
    if (!std::isfinite(prm->angle[k]) || !(prm->pitch[k] > 0.0) || !std::isfinite(prm->pitch[k]) ||
        !std::isfinite(prm->wire_offset[k]) || !std::isfinite(prm->time_offset[k]))
      return fail(WCT_E_INVALID, "plane %d: angle, offsets finite and pitch > 0 required", k);
    a.cth[k] = std::cos(prm->angle[k]);
    a.sth[k] = std::sin(prm->angle[k]);
    a.pitch[k] = prm->pitch[k];
    a.woff[k] = prm->wire_offset[k];
    a.toff[k] = prm->time_offset[k];
  }
  DeviceGuard dg(plan->device);
  if (!dg.ok) return fail(WCT_E_DEVICE, "hipSetDevice(%d) failed", plan->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (plan->dtype == WCT_F32) {
    using T = float;
    DriftIn<T> di{in->n, (const T*)in->x, (const T*)in->y, (const T*)in->z, (const T*)in->t0, (const T*)in->q,
                  (const T*)in->sigma_l, (const T*)in->sigma_t, in->event, in->depo_id};
    DriftOut<T> o{(T*)out->q, (T*)out->t, (T*)out->p, (T*)out->sigma_t, (T*)out->sigma_p, out->plane, out->event,
                  out->depo_id};
    e = launch_drift<T>(di, a, o, plan->n_cu, st);
  } else {
    using T = double;
    DriftIn<T> di{in->n, (const T*)in->x, (const T*)in->y, (const T*)in->z, (const T*)in->t0, (const T*)in->q,
                  (const T*)in->sigma_l, (const T*)in->sigma_t, in->event, in->depo_id};
    DriftOut<T> o{(T*)out->q, (T*)out->t, (T*)out->p, (T*)out->sigma_t, (T*)out->sigma_p, out->plane, out->event,
                  out->depo_id};
    e = launch_drift<T>(di, a, o, plan->n_cu, st);
  }
  if (e != hipSuccess) return hip_fail(e, "drift launch");
  return WCT_OK;
}

int wct_plan_set_adc(wct_plan* plan, int32_t plane, double gain, double baseline, int32_t max_code) {
  g_err.clear();
  if (!plan) return fail(WCT_E_INVALID, "plan is NULL");
  if (plane < 0 || plane >= plan->n_planes) return fail(WCT_E_INVALID, "plane %d of %d", plane, plan->n_planes);
  if (!std::isfinite(gain) || !std::isfinite(baseline)) return fail(WCT_E_INVALID, "ADC gain and pedestal must be finite");
  if (max_code < 1 || max_code > 65535) return fail(WCT_E_INVALID, "largest ADC code %d outside [1, 65535]", max_code);
  plan->adc_gain[plane] = gain;
  plan->adc_base[plane] = baseline;
  plan->adc_max[plane] = max_code;
  return WCT_OK;
}

int wct_digitize(const wct_plan* plan, const void* wave, int32_t n_events, uint16_t* adc, void* stream) {
  TraceRange trace_range("wct_digitize");
  g_err.clear();
  if (!plan) return fail(WCT_E_INVALID, "plan is NULL");
  if (n_events < 1) return fail(WCT_E_INVALID, "n_events %d < 1", n_events);
  if (!wave || !adc) return fail(WCT_E_INVALID, "wave or adc is NULL");
  DeviceGuard dg(plan->device);
  if (!dg.ok) return fail(WCT_E_DEVICE, "hipSetDevice(%d) failed", plan->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int p = 0; p < plan->n_planes; ++p) {
    const PlaneGeom& G = plan->geom[p];
    const int64_t n = (int64_t)G.nw * G.nt;
    hipError_t e;
    if (plan->dtype == WCT_F32)
      e = launch_digitize<float>(static_cast<const float*>(wave) + G.wave_off, plan->wave_elems, n, n_events,
                                 plan->adc_gain[p], plan->adc_base[p], plan->adc_max[p], adc + G.wave_off, plan->n_cu,
                                 st);
    else
      e = launch_digitize<double>(static_cast<const double*>(wave) + G.wave_off, plan->wave_elems, n, n_events,
                                  plan->adc_gain[p], plan->adc_base[p], plan->adc_max[p], adc + G.wave_off,
                                  plan->n_cu, st);
    if (e != hipSuccess) return hip_fail(e, "digitize launch");
  }
  return WCT_OK;
}

int wct_convolve(wct_plan* plan, const void* grid, int32_t n_events, void* wave, void* ws, size_t ws_size,
                 void* stream) {
  TraceRange trace_range("wct_convolve");
  g_err.clear();
  if (!plan) return fail(WCT_E_INVALID, "plan is NULL");
  if (n_events < 1 || n_events > plan->max_events)
    return fail(WCT_E_INVALID, "n_events %d outside [1, %d]", n_events, plan->max_events);
  if (!grid || !wave) return fail(WCT_E_INVALID, "grid or wave is NULL");
  const size_t need = ws_bytes(plan, WCT_OP_CONVOLVE, n_events, 0);
  if (!ws || ws_size < need) return fail(WCT_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_size, need);
  DeviceGuard dg(plan->device);
  if (!dg.ok) return fail(WCT_E_DEVICE, "hipSetDevice(%d) failed", plan->device);
  Carver cv(ws);
  hipStream_t st = static_cast<hipStream_t>(stream);
  return plan->dtype == WCT_F32
             ? run_convolve<float>(plan, static_cast<const float*>(grid), n_events, static_cast<float*>(wave), cv, st)
             : run_convolve<double>(plan, static_cast<const double*>(grid), n_events, static_cast<double*>(wave), cv,
                                    st);
}

// Graphs kept per plan by wct_simulate_graph before the cache is emptied.
static constexpr size_t kMaxGraphs = 32;

// The launches of wct_simulate on stream st (arguments checked; `need` workspace bytes).
static int simulate_enqueue(wct_plan* plan, const wct_depos* depos, const wct_opts* opts, void* wave, void* ws, size_t need,
                            hipStream_t st) {
  int rc = WCT_OK;
  const int batch = opts->n_events < plan->max_events ? opts->n_events : plan->max_events;
  Carver head(ws);
  void* grid = head.take(plan->esize * (size_t)batch * plan->grid_elems);
  const size_t rest = align_up(head.off, 256);
  // the tail of the workspace: row spans, band hulls, tile flags, wire flags
  const WireTileGeom tg = wire_tile_geom(plan);
  const size_t wire_bytes = align_up((size_t)batch * tg.wires_ev, 256) +
                            align_up(sizeof(uint32_t) * (size_t)batch * tg.bits_ev, 256);
  const size_t tile_bytes = align_up((size_t)batch * tg.tiles_ev, 256);
  const size_t hull_bytes = align_up(sizeof(int2) * (size_t)batch * bands_ev(plan), 256);
  char* tail = static_cast<char*>(ws) + need;
  uint8_t* wires = reinterpret_cast<uint8_t*>(tail - wire_bytes);  // then the row words
  uint32_t* rbits = reinterpret_cast<uint32_t*>(tail - wire_bytes + align_up((size_t)batch * tg.wires_ev, 256));
  uint8_t* tiles = reinterpret_cast<uint8_t*>(tail - wire_bytes - tile_bytes);
  int2* hull = reinterpret_cast<int2*>(tail - wire_bytes - tile_bytes - hull_bytes);
  int2* span = reinterpret_cast<int2*>(tail - wire_bytes - tile_bytes - hull_bytes -
                                       align_up(sizeof(int2) * (size_t)batch * plan->rows_ev, 256));
  // sub-batches of up to max_events events: raster into the workspace grid, then the
  // transform passes write the sub-batch's slots of `wave`
  for (int e0 = 0; e0 < opts->n_events; e0 += batch) {
    wct_opts sub = *opts;
    sub.n_events = opts->n_events - e0 < batch ? opts->n_events - e0 : batch;
    sub.event_base = opts->event_base + e0;
    Carver cr(static_cast<char*>(ws) + rest), cc(static_cast<char*>(ws) + rest);
    char* w = static_cast<char*>(wave) + plan->esize * (size_t)e0 * plan->wave_elems;
    if (plan->dtype == WCT_F32) {
      if ((rc = run_raster<float>(plan, depos, &sub, static_cast<float*>(grid), cr, st, span, hull))) return rc;
      rc = run_convolve<float>(plan, static_cast<const float*>(grid), sub.n_events, reinterpret_cast<float*>(w), cc,
                               st, span, &sub, tiles, wires, rbits);
    } else {
      if ((rc = run_raster<double>(plan, depos, &sub, static_cast<double*>(grid), cr, st, span, hull))) return rc;
      rc = run_convolve<double>(plan, static_cast<const double*>(grid), sub.n_events, reinterpret_cast<double*>(w),
                                cc, st, span, &sub, tiles, wires, rbits);
    }
    if (rc) return rc;
  }
  return WCT_OK;
}

int wct_simulate(wct_plan* plan, const wct_depos* depos, const wct_opts* opts, void* wave, void* ws, size_t ws_size,
                 void* stream) {
  TraceRange trace_range("wct_simulate");
  g_err.clear();
  if (!plan) return fail(WCT_E_INVALID, "plan is NULL");
  int rc = check_opts(plan, opts, true, true);
  if (rc) return rc;
  if ((rc = check_depos(depos))) return rc;
  if (!wave) return fail(WCT_E_INVALID, "wave is NULL");
  const int batch = opts->n_events < plan->max_events ? opts->n_events : plan->max_events;
  const size_t need = ws_bytes(plan, WCT_OP_SIMULATE, batch, depos->n);
  if (!ws || ws_size < need) return fail(WCT_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_size, need);
  DeviceGuard dg(plan->device);
  if (!dg.ok) return fail(WCT_E_DEVICE, "hipSetDevice(%d) failed", plan->device);
  return simulate_enqueue(plan, depos, opts, wave, ws, need, static_cast<hipStream_t>(stream));
}

int wct_simulate_graph(wct_plan* plan, const wct_depos* depos, const wct_opts* opts, void* wave, void* ws,
                       size_t ws_size, void* stream) {
  TraceRange trace_range("wct_simulate_graph");
  g_err.clear();
  if (!plan) return fail(WCT_E_INVALID, "plan is NULL");
  int rc = check_opts(plan, opts, true, true);
  if (rc) return rc;
  if ((rc = check_depos(depos))) return rc;
  if (!wave) return fail(WCT_E_INVALID, "wave is NULL");
  if (plan->prof.on) return fail(WCT_E_INVALID, "wct_simulate_graph: kernel timing is on (graphs hold no timing events)");
  const int batch = opts->n_events < plan->max_events ? opts->n_events : plan->max_events;
  const size_t need = ws_bytes(plan, WCT_OP_SIMULATE, batch, depos->n);
  if (!ws || ws_size < need) return fail(WCT_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_size, need);
  DeviceGuard dg(plan->device);
  if (!dg.ok) return fail(WCT_E_DEVICE, "hipSetDevice(%d) failed", plan->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the key: every argument the launches take by value
  char key[512];
  std::snprintf(key, sizeof(key), "%p %p %p %p %p %p %p %p %lld|%a %d %d %llu %d %d|%p %p %zu", depos->q, depos->t,
                depos->p, depos->sigma_t, depos->sigma_p, (const void*)depos->plane, (const void*)depos->event,
                (const void*)depos->depo_id, (long long)depos->n, opts->nsigma, opts->fluctuate, opts->n_events,
                (unsigned long long)opts->seed, opts->event_base, opts->noise, wave, ws, need);
  auto it = plan->graphs.find(key);
  if (it == plan->graphs.end()) {
    if (plan->graphs.size() >= kMaxGraphs) plan->drop_graphs();
    hipError_t e = hipSuccess;
    if (!plan->cap_stream) e = hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    e = hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "begin capture");
    rc = simulate_enqueue(plan, depos, opts, wave, ws, need, plan->cap_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(plan->cap_stream, &graph);
    if (rc == WCT_OK && e != hipSuccess) rc = hip_fail(e, "end capture");
    hipGraphExec_t exec = nullptr;
    if (rc == WCT_OK) {
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (e != hipSuccess) rc = hip_fail(e, "graph instantiate");
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (rc) return rc;
    it = plan->graphs.emplace(key, exec).first;
  }
  const hipError_t e = hipGraphLaunch(it->second, st);
  return e == hipSuccess ? WCT_OK : hip_fail(e, "graph launch");
}

int wct_simulate_backward(wct_plan* plan, const wct_depos* depos, const wct_opts* opts, const void* grad_wave,
                          void* g_q, void* g_t, void* g_p, void* g_sigma_t, void* g_sigma_p, void* ws, size_t ws_size,
                          void* stream) {
  TraceRange trace_range("wct_simulate_backward");
  g_err.clear();
  if (!plan) return fail(WCT_E_INVALID, "plan is NULL");
  int rc = check_opts(plan, opts, true);
  if (rc) return rc;
  if (opts->fluctuate) return fail(WCT_E_INVALID, "the backward pass requires fluctuate = 0");
  if ((rc = check_depos(depos))) return rc;
  if (!grad_wave) return fail(WCT_E_INVALID, "grad_wave is NULL");
  if (depos->n > 0 && (!g_q || !g_t || !g_p || !g_sigma_t || !g_sigma_p))
    return fail(WCT_E_INVALID, "gradient outputs must not be NULL");
  const size_t need = ws_bytes(plan, WCT_OP_BACKWARD, opts->n_events, depos->n);
  if (!ws || ws_size < need) return fail(WCT_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_size, need);
  DeviceGuard dg(plan->device);
  if (!dg.ok) return fail(WCT_E_DEVICE, "hipSetDevice(%d) failed", plan->device);
  Carver cv(ws);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (plan->dtype == WCT_F32)
    return run_backward<float>(plan, depos, opts, static_cast<const float*>(grad_wave), static_cast<float*>(g_q),
                               static_cast<float*>(g_t), static_cast<float*>(g_p), static_cast<float*>(g_sigma_t),
                               static_cast<float*>(g_sigma_p), cv, st);
  return run_backward<double>(plan, depos, opts, static_cast<const double*>(grad_wave), static_cast<double*>(g_q),
                              static_cast<double*>(g_t), static_cast<double*>(g_p), static_cast<double*>(g_sigma_t),
                              static_cast<double*>(g_sigma_p), cv, st);
}

int wct_fft_variant_count(void) {
  int cnt = 0;
  (void)fft_variants(&cnt);
  return cnt;
}

int wct_fft_variant_info(int32_t idx, int32_t* out) {
  g_err.clear();
  int cnt = 0;
  const FftVariantDesc* v = fft_variants(&cnt);
  if (!out) return fail(WCT_E_INVALID, "out is NULL");
  if (idx < 0 || idx >= cnt) return fail(WCT_E_INVALID, "variant index %d out of range [0, %d)", idx, cnt);
  std::memset(out, 0, sizeof(int32_t) * 12);
  out[0] = v[idx].kind;
  out[1] = v[idx].dbl;
  out[2] = v[idx].threads;
  out[3] = v[idx].n;
  out[4] = v[idx].npass;
  for (int k = 0; k < v[idx].npass && k < 7; ++k) out[5 + k] = v[idx].radix[k];
  return WCT_OK;
}

int wct_plan_get_fft(const wct_plan* plan, int32_t plane, int32_t kind, int32_t* variant) {
  g_err.clear();
  if (!plan || !variant) return fail(WCT_E_INVALID, "plan or variant is NULL");
  if (plane < 0 || plane >= plan->n_planes || (kind != 0 && kind != 1))
    return fail(WCT_E_INVALID, "plane %d / kind %d out of range", plane, kind);
  *variant = kind == 0 ? plan->fp_t[plane].variant
                      : (plan->wire_direct[plane] ? WCT_WIRE_DIRECT : plan->fp_w[plane].variant);
  return WCT_OK;
}

int wct_plan_set_fft(wct_plan* plan, int32_t plane, int32_t kind, int32_t variant) {
  g_err.clear();
  if (!plan) return fail(WCT_E_INVALID, "plan is NULL");
  plan->drop_graphs();
  if (plane < 0 || plane >= plan->n_planes || (kind != 0 && kind != 1))
    return fail(WCT_E_INVALID, "plane %d / kind %d out of range", plane, kind);
  DeviceGuard dg(plan->device);
  const hipError_t e = hipDeviceSynchronize();  // tables may be in use by queued work
  if (e != hipSuccess) return hip_fail(e, "synchronise before replacing twiddle tables");
  return plan->dtype == WCT_F32 ? set_fft<float>(plan, plane, kind, variant)
                                : set_fft<double>(plan, plane, kind, variant);
}

size_t wct_tune_workspace_bytes(const wct_plan* plan, int32_t n_events) {
  if (!plan || n_events < 1 || n_events > plan->max_events) return 0;
  return tune_ws_bytes(plan, n_events);
}

int wct_plan_tune(wct_plan* plan, int32_t n_events, const char* cache_path, void* ws, size_t ws_size, void* stream) {
  TraceRange trace_range("wct_plan_tune");
  g_err.clear();
  if (!plan) return fail(WCT_E_INVALID, "plan is NULL");
  plan->drop_graphs();
  if (n_events < 1 || n_events > plan->max_events)
    return fail(WCT_E_INVALID, "n_events %d outside [1, %d]", n_events, plan->max_events);
  const size_t need = tune_ws_bytes(plan, n_events);
  if (!ws || ws_size < need) return fail(WCT_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_size, need);
  DeviceGuard dg(plan->device);
  if (!dg.ok) return fail(WCT_E_DEVICE, "hipSetDevice(%d) failed", plan->device);
  const bool prof = plan->prof.on;
  plan->prof.on = false;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int rc = plan->dtype == WCT_F32 ? run_tune<float>(plan, n_events, cache_path, ws, st)
                                        : run_tune<double>(plan, n_events, cache_path, ws, st);
  plan->prof.on = prof;
  return rc;
}

int wct_tile_variant_count(void) {
  int n = 0;
  (void)tile_variants(&n);
  return n;
}

int wct_tile_variant_info(int32_t idx, int32_t* out) {
  int n = 0;
  const TileVariantDesc* tv = tile_variants(&n);
  if (idx < 0 || idx >= n || !out) return fail(WCT_E_INVALID, "tile variant %d of %d", idx, n);
  out[0] = tv[idx].dbl;
  out[1] = tv[idx].th;
  out[2] = tv[idx].tw;
  out[3] = tv[idx].blocks_per_cu;
  return WCT_OK;
}

int wct_plan_get_tile(const wct_plan* plan, int32_t* variant) {
  g_err.clear();
  if (!plan || !variant) return fail(WCT_E_INVALID, "NULL argument");
  *variant = plan->tile_global;
  return WCT_OK;
}

int wct_plan_set_tile(wct_plan* plan, int32_t variant) {
  g_err.clear();
  if (!plan) return fail(WCT_E_INVALID, "plan is NULL");
  plan->drop_graphs();
  return set_tiles(plan, variant);
}

size_t wct_tune_raster_workspace_bytes(wct_plan* plan, int32_t n_events, int64_t n_rows) {
  if (!plan || n_events < 1 || n_events > plan->max_events || n_rows < 0) return 0;
  return tune_raster_ws_bytes(plan, n_events, n_rows);
}

int wct_plan_tune_raster(wct_plan* plan, const wct_depos* depos, const wct_opts* opts, const char* cache_path,
                         void* ws, size_t ws_size, void* stream) {
  TraceRange trace_range("wct_plan_tune_raster");
  g_err.clear();
  if (!plan) return fail(WCT_E_INVALID, "plan is NULL");
  plan->drop_graphs();
  int rc = check_opts(plan, opts, true);
  if (rc) return rc;
  if ((rc = check_depos(depos))) return rc;
  const size_t need = tune_raster_ws_bytes(plan, opts->n_events, depos->n);
  if (!ws || ws_size < need) return fail(WCT_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_size, need);
  DeviceGuard dg(plan->device);
  if (!dg.ok) return fail(WCT_E_DEVICE, "hipSetDevice(%d) failed", plan->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  return plan->dtype == WCT_F32 ? run_tune_raster<float>(plan, depos, opts, cache_path, ws, st)
                                : run_tune_raster<double>(plan, depos, opts, cache_path, ws, st);
}

int wct_profile_enable(wct_plan* plan, int32_t enable) {
  g_err.clear();
  if (!plan) return fail(WCT_E_INVALID, "plan is NULL");
  plan->prof.on = enable != 0;
  return WCT_OK;
}

int wct_profile_reset(wct_plan* plan) {
  g_err.clear();
  if (!plan) return fail(WCT_E_INVALID, "plan is NULL");
  DeviceGuard dg(plan->device);
  const hipError_t e = plan->prof.collect();
  plan->prof.acc.clear();
  if (e != hipSuccess) return hip_fail(e, "profiler events");
  return WCT_OK;
}

int wct_profile_count(wct_plan* plan) {
  g_err.clear();
  if (!plan) return fail(WCT_E_INVALID, "plan is NULL");
  DeviceGuard dg(plan->device);
  const hipError_t e = plan->prof.collect();
  if (e != hipSuccess) return hip_fail(e, "profiler events");
  return (int)plan->prof.acc.size();
}

int wct_profile_get(wct_plan* plan, int32_t idx, char* name, size_t name_len, double* total_ms, int64_t* launches) {
  g_err.clear();
  if (!plan || !name || name_len == 0 || !total_ms || !launches) return fail(WCT_E_INVALID, "NULL argument");
  if (idx < 0 || idx >= (int32_t)plan->prof.acc.size()) return fail(WCT_E_INVALID, "profile index %d", idx);
  auto it = plan->prof.acc.begin();
  std::advance(it, idx);
  std::snprintf(name, name_len, "%s", it->first.c_str());
  *total_ms = it->second.first;
  *launches = it->second.second;
  return WCT_OK;
}

}  // extern "C"
