// Host-side launchers of the HIP kernels (one translation unit per kernel family).
#pragma once

#include "common.hpp"
#include "fluct.hpp"

namespace wct {

constexpr int kMaxPlanes = 8;

// Depo-plane rows as the kernels read them.
template <typename T>
struct DepoView {
  int64_t n;
  const T *q, *t, *p, *st, *sp;
  const int32_t *plane, *event, *depo_id;
};

// Geometry of all planes of a plan, passed to the raster and gradient kernels by value.
struct RasterGeom {
  int n_planes;
  int n_events;
  int event_base;          // rows of events [event_base, event_base + n_events) are used
  int ntiles_ev;           // raster tiles per event
  int64_t grid_ev_stride;  // grid elements per event
  int64_t rows_ev;         // impact rows per event (all planes)
  PlaneGeom pl[kMaxPlanes];
};

// Control words at the head of the raster workspace.
enum RasterCtrl {
  kCtrlHead = 0,    // work-queue head of the tile kernel
  kCtrlNItems = 1,  // number of tile work items
  kCtrlNBig = 2,    // rows whose window covers more than 4 tiles
  kCtrlTotal = 3,   // total (row, tile) pairs
  kCtrlHeadZero = 4,  // queue head of the groups of tiles the tile kernel clears
  kCtrlWords = 64
};
constexpr int kRowsPerItem = 256;  // rows one tile work item processes at most
constexpr int kZeroGroup = 16;     // tiles per clearing item of the tile kernel
constexpr int kScanPerBlock = 4096;

// Raster tile variants: X(real type, TH rows, TW ticks, tile-kernel blocks per CU).
// Tall tiles: a window of up to 129 impact rows (sigma_p <= 2 pitches at 3 sigma) spans
// at most 2 tile rows, so typical rows take the tile path.  TW is even (the tick pairs that
// share a Philox block never straddle two tiles) and a multiple of 16 bytes (tiles are
// cleared with 16-byte stores); TH * TW <= 2^13 (tile offsets beside the packed electron
// count of the chop-down queue).  Smaller tiles take less LDS, so more blocks share a CU,
// but more rows straddle tiles.  The first variant of a type is a plan's default; the
// raster tuner (wct_plan_tune_raster) times them on an event's rows.
#define WCT_TILE_VARIANTS(X) \
  X(float, 128, 48, 5)      \
  X(float, 128, 64, 4)      \
  X(float, 128, 32, 6)      \
  X(float, 256, 32, 3)      \
  X(double, 64, 64, 4)      \
  X(double, 64, 32, 6)

struct TileVariantDesc {
  int dbl;  // 0 float, 1 double
  int th, tw;
  int blocks_per_cu;
};
#define WCT_TILE_DESC(TT, TH_, TW_, OCC) TileVariantDesc{sizeof(TT) == 8, TH_, TW_, OCC},
inline const TileVariantDesc* tile_variants(int* count) {
  static const TileVariantDesc v[] = {WCT_TILE_VARIANTS(WCT_TILE_DESC)};
  *count = (int)(sizeof(v) / sizeof(v[0]));
  return v;
}
#undef WCT_TILE_DESC

struct RasterWs {
  int32_t* ctrl;      // kCtrlWords
  int32_t* counts;    // [ntiles]
  int32_t* rank;      // [4 n]: a row's slot in the row list of each tile it touches
  int32_t* offs;      // [ntiles + 1]
  int32_t* item_off;  // [ntiles + 1]
  int32_t* items;     // [max_items]
  int32_t* list;      // [4 n]
  int32_t* big;       // [n]
  int32_t* blocks;    // [2 * nscan_blocks]
  int64_t ntiles;
  int64_t max_items;
  int2* span = nullptr;  // optional [event][rows_ev] tick spans of the rows (row_span)
  int2* hull = nullptr;  // with span: [event][bands] tile-column hull of each band of TH rows
};

// Bands of TH impact rows (tile rows) per event over all planes, and plane p's first band.
__host__ __device__ inline int bands_before(const RasterGeom& g, int p) {
  int b = 0;
  for (int q = 0; q < p; ++q) b += g.pl[q].ntr;
  return b;
}

// Tick span of an impact row as the raster records it: {kSpanBase - lo, hi}, both
// raised by atomic max from zero, where [lo, hi) is the union hull of the tick windows of
// the depositions that reach the row; {0, 0} when none does.  The row's samples outside
// [lo, hi) are zero, so the row transform reads only inside it.
constexpr int kSpanBase = 1 << 30;

// Noise of Eq. 1's N term, added to the half spectra of the inverse row transform (pass
// C of the forward): frequency k of wire w in event `event_base + slot` receives
// amp[k] * Z[k], with Z the Box-Muller complex normal of the Philox4x32-10 block of counter
// (k, w, event, plane << 24 | kNoiseStreamBit) under the run's key (real at k = 0 and
// k = L_t / 2).  amp holds the plane's amplitude spectrum divided by L_t (the inverse
// transform is unnormalised), in the plan dtype.
constexpr uint32_t kNoiseStreamBit = 1u << 23;
template <typename T>
struct NoiseArgs {
  const T* amp = nullptr;  // [L_t / 2 + 1]; nullptr: no noise
  uint32_t key0 = 0, key1 = 0;
  uint32_t plane = 0;
  int event_base = 0;
};

// Optional kernel timing: begin/end bracket a launch group with events on the stream.
struct ProfHook {
  virtual void begin(const char* name, hipStream_t st) = 0;
  virtual void end(hipStream_t st) = 0;
  virtual ~ProfHook() = default;
};

// raster.hip
// Raster modes (the fluctuate option): the mean charge, binomial electron counts, or the
// binomial's normal approximation with Box-Muller normals.
constexpr int kModeMean = 0, kModeBinomial = 1, kModeNormal = 2;
// lfact: ln(n!) for n < kLfactTable (launch_lfact_table), or NULL (evaluated per cell).
// tile: index into WCT_TILE_VARIANTS (of type T); the geometry g was built for it.
template <typename T>
hipError_t launch_raster(const DepoView<T>& d, const RasterGeom& g, double nsigma, int mode, uint64_t seed,
                         T* grid, const RasterWs& ws, const DetTables* tables, const double* lfact, int n_cu,
                         hipStream_t st, ProfHook* prof, int tile);
hipError_t launch_lfact_table(double* out, int n, const DetTables* tables, hipStream_t st);

// drift.hip: 3D depositions -> depo-plane rows (plane-major, n_planes * n rows).
template <typename T>
struct DriftIn {
  int64_t n;
  const T *x, *y, *z, *t0, *q, *sl0, *st0;
  const int32_t *event, *depo_id;  // may be null (0, and the deposition index)
};
struct DriftArgs {
  int n_planes;
  double speed, dl, dt, lifetime, tick;
  double cth[kMaxPlanes], sth[kMaxPlanes], pitch[kMaxPlanes], woff[kMaxPlanes], toff[kMaxPlanes];
};
template <typename T>
struct DriftOut {
  T *q, *t, *p, *st, *sp;
  int32_t *plane, *event, *depo_id;
};
template <typename T>
hipError_t launch_drift(const DriftIn<T>& in, const DriftArgs& a, const DriftOut<T>& out, int n_cu, hipStream_t st);

// adc.hip: codes of n samples per event (event stride ev_stride, in samples, for both the
// waveform and the codes) of one plane.
template <typename T>
hipError_t launch_digitize(const T* wave, int64_t ev_stride, int64_t n, int n_events, double gain, double base,
                           int max_code, uint16_t* out, int n_cu, hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);

// conv.hip.  A plan with variant >= 0 runs the compiled-plan kernels; the column passes
// of those take a second twiddle table for the same radices in reverse order (tw_rev).
// Rows are read with 16-byte loads (and the next row prefetched) when their length and base allow it.
// Tiles of the direct column pass (kDirectTileWires output wires each, reading the S^ rows
// of kDirectHalfWires more wires on either side) that some window's rows reach, and the
// rows themselves (one bit each), as wct_simulate records them: a tile no row reaches
// writes a zero M^ without reading S^, a live tile takes the rows no window reached as
// zeros without reading them, so pass A writes no spectrum for a row pair no window reached.
constexpr int kDirectTileWires = 512, kDirectHalfWires = 10;
struct WireTiles {
  const uint8_t* live = nullptr;  // [event][tile] of this plane (ev_stride apart); nullptr: all
  int64_t ev_stride = 0;
  int ntile = 0;
  const uint32_t* rowbits = nullptr;  // [event][bits_ev words] from this plane's first word:
  int64_t bits_ev = 0;                // bit r of the plane set when row r holds a window
};
// Wires whose output some window reaches (a row of wires w - K .. w + K holds one), as
// wct_simulate records them: the inverse row transform writes the zero waveform of any
// other wire without reading or transforming its spectrum (which is exactly zero there).
struct WireLive {
  const uint8_t* live = nullptr;  // [event][wire] of this plane (ev_stride apart); nullptr: all
  int64_t ev_stride = 0;
};

// span (optional, [event][span_ev] row tick spans of this plane): the runtime kernel
// and the wire-pair kernel neither load nor transform a row (pair) no window reached and
// write its zero spectrum directly, and read a row only inside its span; the compiled
// single-row kernel (odd wire counts) reads and transforms every row whole.
template <typename T>
hipError_t launch_rows_r2c(const T* src, int64_t src_ev_stride, cx<T>* dst, int64_t dst_ev_stride, int nt, int nphase,
                           int nper, int nchunk, int n_events, const FftPlan& plan, const cx<T>* tw,
                           const cx<T>* post, int n_cu, hipStream_t st, const int2* span = nullptr,
                           int64_t span_ev = 0, const WireTiles& wt = WireTiles());
template <typename T>
hipError_t launch_colpass(const cx<T>* shat, int64_t shat_ev_stride, const cx<T>* rtil, cx<T>* mhat,
                          int64_t mhat_ev_stride, int nw, int nphase, int nchunk, int n_events, const FftPlan& plan,
                          const cx<T>* tw, const cx<T>* tw_rev, hipStream_t st);
// wiredirect.hip: pass B as direct sums over the response's 2K+1 wires (K = 10 only)
bool colpass_direct_fits(int K);
void wiredirect_init_kernels();
// wt (optional): the plane's tile flags; a tile no row reaches writes zeros.
template <typename T>
hipError_t launch_colpass_direct(const cx<T>* shat, int64_t shat_ev_stride, const cx<T>* rtick, cx<T>* mhat,
                                 int64_t mhat_ev_stride, int nw, int nphase, int nchunk, int n_events, hipStream_t st,
                                 const WireTiles& wt = WireTiles());
// The direct pass's tile flags of every plane and event from the row spans: plane p's
// tiles start at tile_off[p] of an event's tiles_ev.
struct WireTileGeom {
  int n_planes, tiles_ev, wires_ev;
  int64_t rows_ev;
  int nw[kMaxPlanes], I[kMaxPlanes], K[kMaxPlanes], tile_off[kMaxPlanes + 1], wire_off[kMaxPlanes + 1];
  int64_t row_off[kMaxPlanes];
  int bits_ev, bit_off[kMaxPlanes + 1];  // 32-row words of the row flags per event, per plane
};
hipError_t launch_row_bits(const WireTileGeom& g, int n_events, const int2* span, uint32_t* bits, hipStream_t st);
hipError_t launch_wire_tiles(const WireTileGeom& g, int n_events, const int2* span, uint8_t* live, hipStream_t st);
// The per-wire flags of WireLive for every plane and event ([event][wires_ev], plane p's
// wires from wire_off[p]).
hipError_t launch_wire_live(const WireTileGeom& g, int n_events, const int2* span, uint8_t* live, hipStream_t st);
template <typename T>
hipError_t launch_colpass_adj_direct(const cx<T>* ghat, int64_t ghat_ev_stride, const cx<T>* rtick, cx<T>* hhat,
                                     int64_t hhat_ev_stride, int nw, int nphase, int nchunk, int n_events,
                                     hipStream_t st);
template <typename T>
hipError_t launch_colpass_adj(const cx<T>* ghat, int64_t ghat_ev_stride, const cx<T>* rtil, cx<T>* hhat,
                              int64_t hhat_ev_stride, int nw, int nphase, int nchunk, int n_events,
                              const FftPlan& plan, const cx<T>* tw, const cx<T>* tw_rev, hipStream_t st);
template <typename T>
hipError_t launch_rows_c2r(const cx<T>* src, int64_t src_ev_stride, T* dst, int64_t dst_ev_stride, int nt,
                           bool tiled, int nphase, int nper, int nchunk, int n_events, const FftPlan& plan,
                           const cx<T>* tw, const cx<T>* post, hipStream_t st,
                           const NoiseArgs<T>& noise = NoiseArgs<T>(), const WireLive& wl = WireLive());
template <typename T>
bool conv_fits(int elems);  // a transform of `elems` complex values fits one block
void conv_init_kernels();

// plan.hip
hipError_t launch_resp_tick(const double* R, int nk, int I, int TR, int lt, int F, const cx<double>* tw_lt,
                            cx<double>* out, hipStream_t st);
template <typename T>
hipError_t launch_resp_wire(const cx<double>* rt, int K, int I, int F, int lw, int lt, int nchunk,
                            const cx<double>* tw_lw, cx<T>* rtil, hipStream_t st);
template <typename T>
hipError_t launch_resp_tick_pack(const cx<double>* rt, int K, int I, int F, int fpad, int lt, cx<T>* rtick,
                                 hipStream_t st);

// grad.hip
template <typename T>
hipError_t launch_grad_gather(const DepoView<T>& d, const RasterGeom& g, double nsigma, const T* H, T* gq, T* gt,
                              T* gp, T* gst, T* gsp, hipStream_t st);

}  // namespace wct
