/*
 * wct.h - C ABI of libwct.so: LArTPC signal simulation on AMD MI355X (gfx950).
 *
 * Implements the signal part of the paper's Eq. 1,
 *     M(t, x) = (R (*) S)(t, x),
 * evaluated as in its Eq. 2 (transform S, multiply by the pre-computed response
 * spectrum, transform back), where S is built by rasterising every energy
 * deposition into a small patch and scatter-adding the patches into a large grid
 * (Sec. 2.1.1 "rasterization" and "scatter adding"), optionally with binomial
 * fluctuation of the electron counts (Sec. 4.3.1, Table 2).
 *   Reference: H. Yu et al., "Evaluation of Portable Acceleration Solutions for LArTPC
 *   Simulation Using Wire-Cell Toolkit", arXiv:2104.08265.
 *
 * Discretisation.  A plane has N_w wires, N_t ticks and I impact rows per wire pitch;
 * the charge grid S of a plane is [N_b = I*N_w][N_t] (impact row major, ticks
 * contiguous).  Time t is in ticks (tick k covers [k, k+1)); the pitch coordinate p
 * is in wire pitches from the plane's low edge (wire w at p = w + 1/2, impact row b
 * covers [b/I, (b+1)/I)).  The response R[k][i][tau] (k = -K..K stored at k+K,
 * i in [0, I), tau in [0, T_R)) is the signal on wire w from unit charge in impact row
 * I*(w+k)+i, tau ticks after arrival.  Then
 *     M[w][t] = sum_{k,i,tau} R[k][i][tau] * S[I*(w+k)+i][t-tau],
 * S taken as 0 outside the grid (linear, causal convolution cropped to the grid).
 *
 * Memory.  Every pointer argument of the run calls is a DEVICE pointer unless it is
 * marked HOST.  The caller owns depositions, grids, waveforms, gradients and the
 * workspace; the plan owns only its response spectra and twiddle tables (the 2D
 * spectrum the wire transforms use, I L_w F complex values per plane, only once a
 * plane's wire pass is set to a transform plan).  Outputs are
 * overwritten, never accumulated.  Grids and waveforms of one event pack the planes
 * back to back (offsets from wct_plane_info); events follow one another.
 *
 * Streams and errors.  Run calls enqueue work on `stream` (a hipStream_t, NULL = the
 * null stream) and return without synchronising.  Every call returns WCT_OK or a
 * negative WCT_E_* code; wct_last_error() then describes it.  Invalid arguments are
 * detected on the host before anything is enqueued.  Faults inside kernels surface at
 * the caller's next synchronisation, as HIP specifies.  Only wct_plan_create and the
 * set-up calls wct_plan_set_fft and wct_plan_tune allocate device memory or
 * synchronise.  One plan must
 * not be used by two threads at once; separate plans are independent.
 */
#ifndef WCT_H
#define WCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WCT_ABI_VERSION 8
/* Version of the fluctuation draw stream (counter layout + sampler).  Bumped whenever a
 * change would alter any fluctuated count for the same inputs and seed. */
#define WCT_FLUCT_SPEC_VERSION 2

typedef struct wct_plan wct_plan;

enum wct_dtype { WCT_F32 = 0, WCT_F64 = 1 };

enum wct_status {
  WCT_OK = 0,
  WCT_E_INVALID = -1,     /* bad argument (NULL, size, range, dtype, option)          */
  WCT_E_WORKSPACE = -2,   /* workspace smaller than wct_workspace_bytes() asks for     */
  WCT_E_DEVICE = -3,      /* a HIP runtime call failed (text in wct_last_error)        */
  WCT_E_UNSUPPORTED = -4, /* geometry the kernels do not handle (e.g. FFT length)      */
  WCT_E_NOMEM = -5        /* device allocation failed, or passed WCT_PLAN_MEM_CAP       */
};

enum wct_op { WCT_OP_RASTER = 0, WCT_OP_CONVOLVE = 1, WCT_OP_SIMULATE = 2, WCT_OP_BACKWARD = 3 };

/* One readout plane. */
typedef struct {
  int32_t n_wires;      /* N_w >= 1 */
  int32_t n_ticks;      /* N_t >= 1 */
  int32_t n_impacts;    /* I >= 1, impact rows per wire pitch */
  int32_t half_wires;   /* K >= 0: the response spans wires -K..K */
  int32_t resp_ticks;   /* T_R >= 1 */
  const void* response; /* HOST [2K+1][I][T_R] row-major in the plan dtype; copied */
} wct_plane_desc;

typedef struct {
  int32_t dtype;                /* WCT_F32 or WCT_F64: grids, waveforms, depo floats */
  int32_t n_planes;             /* >= 1 */
  const wct_plane_desc* planes; /* HOST [n_planes] */
  int32_t max_events;           /* largest n_events any run call will pass (>= 1) */
  int32_t device;               /* HIP device ordinal the plan and its calls use */
} wct_plan_desc;

/* Depo-plane rows: one row per (deposition, plane) projection, structure of arrays.
 * Float arrays are in the plan dtype. */
typedef struct {
  int64_t n;              /* number of rows, >= 0 */
  const void* q;          /* [n] charge, electrons, >= 0 */
  const void* t;          /* [n] arrival time, ticks */
  const void* p;          /* [n] pitch coordinate, wire pitches */
  const void* sigma_t;    /* [n] longitudinal width, ticks, > 0 */
  const void* sigma_p;    /* [n] transverse width, wire pitches, > 0 */
  const int32_t* plane;   /* [n] plane index in [0, n_planes) */
  const int32_t* event;   /* [n] event id >= 0 (NULL: all 0); see wct_opts.event_base */
  const int32_t* depo_id; /* [n] deposition id (fluctuation counter word 1) */
} wct_depos;

/* Event window.  A call simulates the events event_base .. event_base + n_events - 1:
 * rows whose event id lies in that range are used, the others ignored (gradients of
 * ignored rows are written as 0).  Event e fills output slot e - event_base, while its
 * fluctuation draws are keyed by e itself, so an event gets the same counts whether it
 * is simulated alone or inside a batch. */
typedef struct {
  double nsigma;      /* truncation half-width of the Gaussian patch in sigmas, (0, 8] */
  int32_t fluctuate;  /* 0: mean charge; 1: binomial electron counts; 2: their normal
                         approximation with Box-Muller normals (1 and 2 need nsigma <= 4.2;
                         electron counts are 32-bit: a charge of 2^31 - 1 or more draws
                         as 2^31 - 1 electrons) */
  int32_t n_events;   /* events in this call: 1..max_events (wct_simulate: any >= 1) */
  uint64_t seed;      /* fluctuation key (Philox4x32-10 key words: low, high 32 bits) */
  int32_t event_base; /* first event id of the window, >= 0 */
  int32_t noise;      /* wct_simulate: 1 adds each plane's noise (wct_plan_set_noise) to the
                         waveforms, 0 none; the other calls ignore it.  0 or 1. */
} wct_opts;

/* Geometry of a plane as planned: out[0..9] = N_w, N_t, I, K, T_R, L_w, L_t, F,
 * grid offset (elements within an event), waveform offset (elements within an event).
 * L_w >= N_w + K and L_t >= N_t + T_R - 1 are the 2,3,5-smooth transform lengths,
 * F = L_t/2 + 1 the number of tick frequencies kept. */
int wct_plane_info(const wct_plan* plan, int32_t plane, int64_t out[10]);

/* Build a plan: validates the geometry, copies the responses and pre-computes, on the
 * device, the response spectrum of every plane (Eq. 2 takes the response in the
 * frequency domain, transformed once ahead of the per-event work).  Allocates device
 * memory and synchronises (as does wct_plan_set_fft; no run call does).  On failure
 * *out is NULL and nothing stays allocated.
 * Errors: WCT_E_INVALID for a bad description; WCT_E_UNSUPPORTED for a plane grid of
 * 2^32 cells or more, or when max_events events' buffers (grid, spectra, waveforms,
 * row records) would exceed 2^60 bytes; WCT_E_DEVICE without a HIP device; WCT_E_NOMEM
 * when a device allocation fails.  The environment variable WCT_PLAN_MEM_CAP (a
 * decimal byte count, read by each call) caps the device memory the plan's own tables
 * may take while it is built: a plan that needs more fails with WCT_E_NOMEM before the
 * allocation that would pass the cap (a value that is not a byte count: WCT_E_INVALID).
 * The geometry checks come before any device call, so they answer without a GPU. */
int wct_plan_create(const wct_plan_desc* desc, wct_plan** out);
void wct_plan_destroy(wct_plan* plan); /* NULL is a no-op; synchronises the device */

/* Elements of one event's packed grid (sum over planes of I*N_w*N_t) and waveform
 * (sum over planes of N_w*N_t).  -1 on a NULL plan. */
int64_t wct_grid_elems(const wct_plan* plan);
int64_t wct_wave_elems(const wct_plan* plan);

/* Workspace bytes a run call needs for `n_events` events and `n_rows` depo rows
 * (n_rows is ignored by WCT_OP_CONVOLVE).  0 on invalid arguments. */
size_t wct_workspace_bytes(const wct_plan* plan, int32_t op, int32_t n_events, int64_t n_rows);

/* Rasterisation + scatter adding (Sec. 2.1.1): grid[event][planes packed][N_b][N_t]
 * receives, for every row, Q * A_b * B_k on the cells of its truncated window, where
 * A_b, B_k are the Gaussian's integrals over the parts of impact row b and tick k that
 * lie inside mu +- nsigma*sigma (u = I*p, sigma_u = I*sigma_p on the impact axis).
 * Cells outside the grid are dropped.  With fluctuate = 1 each cell instead receives an
 * independent Binomial(floor(Q+1/2), A_b*B_k) count drawn from Philox4x32-10 with key
 * `seed`; cells (b, 2m) and (b, 2m+1) share the counter (b*ceil(N_t/2) + m, depo_id,
 * event, plane << 24), the even tick taking words 0-1 and the odd tick words 2-3; the
 * sampler is that of WCT_FLUCT_SPEC_VERSION (bit-reproducible, independent of
 * scheduling and batching; `event` is the row's event id).  With fluctuate = 2 (the
 * Kokkos port's Box-Muller normals, Sec. 4.3.1) a cell with N electrons and probability
 * p receives min(max(floor(N p + sqrt(N p (1 - p)) z + 1/2), 0), N): the cells (b, 2m),
 * (b, 2m+1) take z = r cos(2 pi u2) and r sin(2 pi u2) of the same Philox block, with
 * r = sqrt(-2 ln u1), u1 = 1 - (the even tick's uniform), u2 = the odd tick's uniform;
 * sqrt, ln, cos and sin are evaluated with IEEE +, -, *, / only, so these counts too are
 * bit-reproducible.  Rows with sigma <= 0,
 * Q < 0 or non-finite values contribute nothing.  The whole grid of every event of the
 * window is overwritten. */
int wct_raster(wct_plan* plan, const wct_depos* depos, const wct_opts* opts, void* grid, void* ws,
               size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): wct_raster without a caller workspace.
 * The raster's scratch (tile counters, per-tile row lists, work items, the wide-row list)
 * lives instead in a static device array of WCT_NOALLOC_SCRATCH_BYTES that each device the
 * library runs on holds from its first plan there until the process ends.  Same grid,
 * same counts and the same kernels as wct_raster.  The call allocates nothing and does
 * not synchronise; it needs wct_workspace_bytes(plan, WCT_OP_RASTER, n_events, depos->n)
 * <= WCT_NOALLOC_SCRATCH_BYTES (about 3.5 million rows on the three-plane 2400/2400/3456 x
 * 9600 geometry), else it returns WCT_E_WORKSPACE before enqueuing anything.  Every call on
 * one device shares that device's array (it keeps the last call's contents; the counters
 * that must start at zero are cleared by a kernel at the start of each call): calls that
 * may overlap in time on one device (several streams or threads) race, and the caller must
 * order them. */
#define WCT_NOALLOC_SCRATCH_BYTES (128u << 20)
int wct_raster_noalloc(wct_plan* plan, const wct_depos* depos, const wct_opts* opts, void* grid, void* stream);

/* Noise (the additive term N of Eq. 1, M = R (*) S + N; Sec. 2 notes it is cheaper to
 * simulate than the signal).  Sets plane `plane`'s amplitude spectrum: amp (HOST) holds
 * A[k] >= 0 for the n = F = L_t/2 + 1 frequencies of the plane's tick transform
 * (wct_plane_info), or is NULL to remove the plane's noise.  With opts.noise = 1,
 * wct_simulate then adds to every wire w of event e
 *     n[t] = irfft(A * Z, L_t)[t],  t < N_t,
 * (irfft: the inverse real transform with the 1/L_t factor) where Z[k] is a complex
 * normal: the Philox4x32-10 block of counter (k, w, e, plane << 24 | 2^23) under key
 * `seed` gives u1 = 1 - (53-bit uniform of words 0-1), u2 = (uniform of words 2-3),
 * r = sqrt(-2 ln u1), theta = 2 pi u2, and Z = r e^{i theta} / sqrt(2), or r cos(theta)
 * at k = 0 and k = L_t/2.  The noise is added in the frequency domain just before the
 * inverse row transform (no extra pass over the waveforms); a batch gives each event the
 * noise it gets alone.  A set-up call: allocates on first use and synchronises. */
int wct_plan_set_noise(wct_plan* plan, int32_t plane, const double* amp, int64_t n);

/* Drift of 3D depositions to the readout (Fig. 2: ionisation clouds drift to the wire
 * planes, spreading along and across the drift; Sec. 2.1.1: the raster takes each
 * cloud's Gaussian at the plane).  Readout planes at x = 0, uniform drift along -x. */
#define WCT_MAX_PLANES 8
typedef struct {
  int64_t n;                /* depositions, >= 0 */
  const void* x;            /* [n] distance to the readout planes along the drift, cm */
  const void* y;            /* [n] cm */
  const void* z;            /* [n] cm */
  const void* t0;           /* [n] deposition time, us */
  const void* q;            /* [n] ionisation electrons */
  const void* sigma_l;      /* [n] initial extent along the drift, cm (>= 0) */
  const void* sigma_t;      /* [n] initial extent across the drift, cm (>= 0) */
  const int32_t* event;     /* [n] event id, or NULL (all 0) */
  const int32_t* depo_id;   /* [n] deposition id, or NULL (the index j) */
} wct_depos3d;
typedef struct {
  double drift_speed;                    /* v, cm/us, > 0 */
  double diffusion_l, diffusion_t;       /* D_L, D_T, cm^2/us, >= 0 */
  double lifetime;                       /* electron lifetime tau, us; <= 0: no attenuation */
  double tick;                           /* T_tick, us per tick, > 0 */
  double angle[WCT_MAX_PLANES];          /* plane k: angle theta_k (radians) of its wire normal in (y, z) */
  double pitch[WCT_MAX_PLANES];          /* P_k, cm, > 0 */
  double wire_offset[WCT_MAX_PLANES];    /* o_k: pitch coordinate of y = z = 0, pitches */
  double time_offset[WCT_MAX_PLANES];    /* d_k: time added at plane k, us */
} wct_drift_params;
typedef struct {
  void* q; void* t; void* p; void* sigma_t; void* sigma_p; /* [n_planes * n], plan dtype */
  int32_t* plane; int32_t* event; int32_t* depo_id;         /* [n_planes * n] */
} wct_depos_out;
/* wct_drift (DEVICE arrays; inputs in the plan dtype) writes, for deposition j and plane
 * k, row k n + j of `out`:
 *   t_d = x / v,  sigma_L^2 = sigma_l^2 + 2 D_L t_d,  sigma_T^2 = sigma_t^2 + 2 D_T t_d,
 *   q' = q exp(-t_d / tau) (q without a lifetime), 0 unless x >= 0 and all inputs finite,
 *   t = (t0 + t_d + d_k) / T_tick,  p = (z cos theta_k + y sin theta_k) / P_k + o_k,
 *   sigma_t = sigma_L / (v T_tick),  sigma_p = sigma_T / P_k,
 * with plane k, the deposition's event and id: the rows wct_raster / wct_simulate take
 * (a row of zero width is dropped there).  Evaluated in FP64 and rounded to the plan
 * dtype.  A run call: enqueued on `stream`, no workspace, no synchronisation.  Invalid
 * parameters return WCT_E_INVALID before anything is enqueued. */
int wct_drift(const wct_plan* plan, const wct_depos3d* in, const wct_drift_params* prm, const wct_depos_out* out,
              void* stream);

/* ADC digitisation (Eq. 1, Sec. 2: M is a measurement such as an ADC value).
 * wct_plan_set_adc sets plane `plane`'s converter: gain (counts per unit of M), baseline
 * (the pedestal, counts; both finite) and max_code in [1, 65535] (2^bits - 1); a plan
 * starts with gain 1, baseline 0, max_code 65535 on every plane.  wct_digitize writes
 *     adc = min(max(floor(M * gain + baseline + 1/2), 0), max_code)
 * (0 where M is not a number) for every sample of n_events events of `wave` (DEVICE,
 * plan dtype, the layout wct_convolve writes) to `adc` (DEVICE, uint16, same layout and
 * element count).  The arithmetic is in the plan's dtype, gain and baseline rounded to it,
 * one rounding per operation in the order written.  A run call: enqueued on `stream`, no
 * workspace, no synchronisation. */
int wct_plan_set_adc(wct_plan* plan, int32_t plane, double gain, double baseline, int32_t max_code);
int wct_digitize(const wct_plan* plan, const void* wave, int32_t n_events, uint16_t* adc, void* stream);

/* Convolution by FFT (Eq. 2): wave[event][planes packed][N_w][N_t] = R (*) grid for
 * n_events events.  Row transforms along ticks (real-to-complex, length L_t), column
 * transforms along impact rows per phase (length L_w), the product with the
 * pre-computed spectrum summed over the I phases, and the inverse transforms. */
int wct_convolve(wct_plan* plan, const void* grid, int32_t n_events, void* wave, void* ws, size_t ws_bytes,
                 void* stream);

/* wct_raster followed by wct_convolve, the grid living in the workspace.  n_events may
 * exceed the plan's max_events: the events are then processed in consecutive
 * sub-batches of max_events (one persistent raster launch and one set of batched
 * transform passes per sub-batch), with the workspace of max_events events
 * (wct_workspace_bytes(plan, WCT_OP_SIMULATE, n, rows) caps n at max_events).
 * The raster also records which impact rows (and the tick span of each), which column
 * tiles and which wires any window reaches; the transform passes then skip the work on
 * the rest (rows not transformed, tiles and rows of the direct wire pass taken as zero,
 * wires without noise written as zero waveforms), which changes no result: the waveform
 * equals that of wct_raster followed by wct_convolve. */
int wct_simulate(wct_plan* plan, const wct_depos* depos, const wct_opts* opts, void* wave, void* ws,
                 size_t ws_bytes, void* stream);

/* wct_simulate replayed from a HIP graph, for callers that repeat the same call and want
 * one launch instead of one per kernel (the launches of a whole event take a few hundred
 * microseconds to enqueue one by one).  Same arguments, result and errors as
 * wct_simulate.  The first call with a given set of arguments (every pointer in depos,
 * depos->n, every field of opts, wave, ws, the needed workspace size) captures the
 * launches on a stream the plan owns and keeps the instantiated graph; later calls with
 * the same arguments launch it on `stream`.  The graph reads the buffers the pointers
 * name when it runs, so the data behind them may change between calls; new pointers,
 * sizes or options (a new seed, say) capture a new graph.  The plan keeps at most 32
 * graphs (the cache is emptied when full) and drops them in every set-up call that
 * changes what its launches take (wct_plan_set_noise, wct_plan_set_fft, wct_plan_tune,
 * wct_plan_set_tile, wct_plan_tune_raster) and in wct_plan_destroy; those calls
 * synchronise the device first.  WCT_E_INVALID while kernel timing is on.  Calls on one
 * plan are not thread safe; two replays of one graph on different streams race on the
 * same workspace like two wct_simulate calls would. */
int wct_simulate_graph(wct_plan* plan, const wct_depos* depos, const wct_opts* opts, void* wave, void* ws,
                       size_t ws_bytes, void* stream);

/* Gradients of a scalar loss with respect to each row's (Q, t, p, sigma_t, sigma_p),
 * given grad_wave = dL/dwave (same layout as wave).  Uses the convolution's adjoint
 * (correlation with the conjugate spectrum) and the Gaussian-pdf derivatives of the
 * clipped bin integrals; the charge grid is recomputed, never stored.  Requires
 * fluctuate = 0.  Each g_* is [n] in the plan dtype, overwritten. */
int wct_simulate_backward(wct_plan* plan, const wct_depos* depos, const wct_opts* opts, const void* grad_wave,
                          void* g_q, void* g_t, void* g_p, void* g_sigma_t, void* g_sigma_p, void* ws,
                          size_t ws_bytes, void* stream);

/* Kernel timing.  While enabled, each kernel (or launch group) a run call enqueues is
 * bracketed by HIP events on the call's stream.  wct_profile_count synchronises on the
 * recorded events and returns the number of distinct kernel names seen since the last
 * reset; wct_profile_get(idx) reports a name (HOST buffer of name_len bytes), its summed
 * device milliseconds and its number of launches.  Enabling creates events per launch:
 * a measurement mode, not for production calls. */
int wct_profile_enable(wct_plan* plan, int32_t enable);
int wct_profile_reset(wct_plan* plan);
int wct_profile_count(wct_plan* plan);
int wct_profile_get(wct_plan* plan, int32_t idx, char* name, size_t name_len, double* total_ms, int64_t* launches);

/* Transform variants.  The Stockham transforms of Eq. 2 along ticks (kind 0: passes A
 * and C, half-length complex transforms of length L_t/2) and along wires (kind 1:
 * pass B, length L_w) run either a runtime plan (any 2,3,5-smooth length) or one of the
 * plans compiled into the library, whose radices and block size are fixed at build
 * time.  A plan starts with the first compiled variant that matches each length, or
 * the runtime plan when none does (the forward wire pass: see WCT_WIRE_DIRECT below); every choice computes the same transform (results
 * differ by floating-point rounding only).
 * wct_fft_variant_info(idx, out[12]) fills out = {kind, is_double, threads per block,
 * length, number of passes, radices[0..6] (0-padded)} (HOST buffer); kind 2 is a wire
 * transform that takes half of a chunk's tick frequencies per block (it serves kind 1).
 * wct_plan_get_fft reports a plane's current choice (-1 = runtime plan);
 * wct_plan_set_fft selects one: -1 or a variant of that kind, dtype and length, else
 * WCT_E_INVALID.  set_fft allocates the new twiddle tables and synchronises the device;
 * it is a set-up call (for example for an autotuner), not a run call.
 * Kind 1 also takes WCT_WIRE_DIRECT: the wire pass (forward, and the adjoint of
 * wct_simulate_backward) as direct sums over the response's 2K+1 wires in the
 * tick-frequency domain (Eq. 1 with only the tick axis transformed; needs K = 10, else
 * WCT_E_UNSUPPORTED), the same convolution up to rounding; get_fft then reports
 * WCT_WIRE_DIRECT, and a later -1 or variant index returns to a transform plan.  A new
 * plan starts with the direct sum wherever it applies. */
#define WCT_WIRE_DIRECT (-2)
int wct_fft_variant_count(void);
int wct_fft_variant_info(int32_t idx, int32_t* out);
int wct_plan_get_fft(const wct_plan* plan, int32_t plane, int32_t kind, int32_t* variant);
int wct_plan_set_fft(wct_plan* plan, int32_t plane, int32_t kind, int32_t variant);

/* Autotuning of the transform variants: for every plane and kind, times the
 * convolution of n_events events of constant charge (HIP events on `stream`) with each
 * applicable compiled variant and with the runtime plan (wires: and the direct sum), and
 * keeps the fastest.  The candidates take turns: four rounds of three runs each, the
 * first round a warm-up, a candidate's time its fastest later round.  cache_path (HOST string, NULL = none) names a text file of earlier choices:
 * lines "wct-fft <dtype> <N_w> <N_t> <I> <K> <T_R> kind <k> -> <threads> <radices...>"
 * (or "-> runtime", "-> direct"); choices found there for this library's variants are applied
 * without timing, new ones are appended.  ws: wct_tune_workspace_bytes(plan, n_events)
 * bytes (grid, waveform and convolution workspace).  A set-up call: allocates twiddle
 * tables and synchronises. */
size_t wct_tune_workspace_bytes(const wct_plan* plan, int32_t n_events);
int wct_plan_tune(wct_plan* plan, int32_t n_events, const char* cache_path, void* ws, size_t ws_bytes, void* stream);

/* Raster tile variants.  The raster accumulates each tile of TH impact rows x TW ticks in
 * LDS (Sec. 2.1.1 scatter adding through privatised tiles); the library compiles a few
 * shapes per dtype.  wct_tile_variant_info(idx, out[4]) fills out = {is_double, TH, TW,
 * tile-kernel blocks per CU} (HOST buffer).  A plan starts on the first variant of its
 * dtype; wct_plan_set_tile selects another (an index of the whole list, of the plan's
 * dtype, else WCT_E_INVALID) and wct_plan_get_tile reports it.  Every variant gives the
 * same grid (fluctuated: bit for bit).  The raster workspace depends on the variant:
 * query wct_workspace_bytes after a change.  Set-up calls: not for use while run calls on
 * the plan are queued with a workspace sized for another variant. */
int wct_tile_variant_count(void);
int wct_tile_variant_info(int32_t idx, int32_t* out);
int wct_plan_get_tile(const wct_plan* plan, int32_t* variant);
int wct_plan_set_tile(wct_plan* plan, int32_t variant);

/* Autotuning of the raster tile: times wct_raster of `depos` with `opts` (HIP events on
 * `stream`; turns as in wct_plan_tune) for every tile variant of the plan's dtype and
 * keeps the fastest (a variant replaces an earlier one only when more than 1.5% faster,
 * so the list's first, the plan's default, wins ties within the timing noise).  cache_path (HOST, NULL = none): the same text file as
 * wct_plan_tune, lines "wct-tile <dtype> <n_planes> (<N_w> <N_t> <I>)... fluct <0|1> ->
 * <TH> <TW> <blocks>"; a choice found there is applied without timing, a new one is
 * appended.  ws: wct_tune_raster_workspace_bytes(plan, opts->n_events, depos->n) bytes
 * (a grid and the largest raster workspace).  A set-up call: synchronises. */
size_t wct_tune_raster_workspace_bytes(wct_plan* plan, int32_t n_events, int64_t n_rows);
int wct_plan_tune_raster(wct_plan* plan, const wct_depos* depos, const wct_opts* opts, const char* cache_path,
                         void* ws, size_t ws_bytes, void* stream);

/* Thread-local text of the last error on this thread ("" if none). */
const char* wct_last_error(void);

int wct_abi_version(void);          /* WCT_ABI_VERSION */
int wct_fluct_spec_version(void);   /* WCT_FLUCT_SPEC_VERSION */

#ifdef __cplusplus
}
#endif

#endif /* WCT_H */
