/*
 * wct_probe.h - throughput probes of libwct.so (measurement calls, not part of the
 * simulation path).
 *
 * The paper plans the scatter-add of rasterised patches as atomic adds and shows a
 * unit test and a thread-scaling figure for it (arXiv:2104.08265 Sec. 5, Fig. 5).  On
 * MI355X the raster accumulates in LDS-privatised tiles and falls back to device-memory
 * atomics only for crowded tiles and wide rows; these probes measure the peak rate of
 * both kinds of float atomic add on the device, so that the raster's own atomic counts
 * (rocprofv3 SQ_INSTS_LDS_ATOMIC, TCC_ATOMIC) can be read as fractions of them.  An
 * instruction-rate probe gives the same reference for the arithmetic the raster's
 * sampler and the direct wire pass issue.
 */
#ifndef WCT_PROBE_H
#define WCT_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Float atomic-add throughput.  where = 0: adds into LDS (each block of 256 threads adds
 * into its own 32 KB of LDS; `buf` receives one value per thread, buf_elems >= blocks*256);
 * where = 1: adds into device memory `buf` of buf_elems floats (a multiple of blocks*256,
 * overwritten with counts; its size decides whether the adds stay in L2).  Each of the
 * blocks*256 threads makes iters*8 adds, a wave's 64 lanes to 64 consecutive floats (no
 * bank or line conflicts).  Launches once to warm up and once timed with HIP events on
 * `stream`, synchronises, and writes the adds per second (lane operations) to *adds_per_s
 * (HOST).  Returns 0, -1 on bad arguments, -3 on a HIP error (text in
 * wct_probe_last_error). */
int wct_probe_atomic_add(int32_t where, int32_t blocks, int32_t iters, float* buf, int64_t buf_elems,
                         double* adds_per_s, void* stream);
/* Instruction issue rate: kind 0 = FP32 FMA with vector-register operands, 1 = FP32 FMA
 * with a scalar-register multiplier, 2 = FP64 FMA, 3 = 32 x 32 -> 64-bit integer
 * multiply-add with a scalar multiplier (v_mad_u64_u32, the Philox product).  Each of the
 * blocks*256 threads runs 16 independent chains of iters operations; `buf` (device,
 * buf_bytes >= blocks*256*8) receives one 8-byte value per thread.  Launches once to warm
 * up and once timed with HIP events on `stream`, synchronises, and writes the operations
 * per second (lane operations) to *ops_per_s (HOST).  These are the rates the raster's
 * and the direct wire pass's instruction mixes are read against.  Returns 0, -1 on bad
 * arguments, -3 on a HIP error (text in wct_probe_last_error). */
int wct_probe_issue_rate(int32_t kind, int32_t blocks, int32_t iters, void* buf, int64_t buf_bytes,
                         double* ops_per_s, void* stream);
const char* wct_probe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WCT_PROBE_H */
