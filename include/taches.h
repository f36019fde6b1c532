/*
 * taches.h — C-ABI of the streaming taches convolution library (libtaches.so)
 * for AMD MI355X (gfx950).
 *
 * The method (Millot & Pelé, AES 2008, Section 3.2, Eq. 4): every input
 * sample x[m] adds its "tache" x[m] * h[n - m], a scaled and delayed copy of
 * the impulse response h, to the output; the output is the sum of all
 * taches.  The buffer form (Section 4.2, algorithm TachesAlgorithm) consumes
 * the input block by block and keeps the not-yet-emitted part of the sum in
 * a circular residue, so each output sample is ready as soon as its own
 * input sample has been consumed.  The impulse response may be replaced
 * while running; the new one is used for the next samples (Abstract;
 * Section 6).  Outputs continue for L-1 samples after the last input
 * (temporal overflow, Section 4.1): drain them by processing zero blocks or
 * by passing x = NULL to taches_process_blocks.
 *
 * Semantics implemented (exactly, up to floating-point summation order):
 *   y[c][n] = sum over m <= n of x[c][m] * h_{b(m)}[n - m]
 * where b(m) is the block that holds input sample m and h_b is the IR that
 * was active for block b (the last one set before that block; taps outside
 * [0, L_b) are zero).  Taches already started keep the IR that made them.
 *
 * Conventions for every call:
 *   - Sizes are counts of float samples.  Multichannel buffers are planar:
 *     x[c * B + i] for channel c, sample i of the block (c < channels).
 *   - "host" pointers are ordinary CPU memory owned by the caller; "device"
 *     pointers are GPU memory (e.g. from PyTorch) owned by the caller, on the
 *     stream's device.  The library owns all device memory it allocates (the
 *     circular tail, IR slots, staging); taches_close frees it.
 *   - Return value: TACHES_OK (0) or a negative status.  On error nothing is
 *     written to the caller's output and taches_last_error() returns a
 *     message (thread-local, valid until the next failing call on the same
 *     thread).  No call throws across the ABI.
 *   - A handle is not thread-safe; distinct handles may be used from
 *     distinct threads.  All device work of a handle is ordered on one HIP
 *     stream (its own, or the one given with taches_set_hip_stream).
 */
#ifndef TACHES_H
#define TACHES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define TACHES_OK 0
#define TACHES_EINVAL (-1)  /* bad size, NULL pointer, bad slot or config   */
#define TACHES_ENOIR (-2)   /* process before any IR was set                */
#define TACHES_ENOMEM (-3)  /* device/host allocation or HBM budget failure */
#define TACHES_EDEVICE (-4) /* a HIP call failed                            */
#define TACHES_EBUSY (-5)   /* pool: stream attached elsewhere / slots full */

/* ---- precision of the contraction -------------------------------------- */
#define TACHES_PREC_FP32 0       /* FP32 multiply-add on the vector ALUs      */
#define TACHES_PREC_SPLIT_BF16 1 /* hi+lo BF16 on MFMA, FP32 accumulation     */

/* ---- type of the circular tail accumulator ----------------------------- */
#define TACHES_TAIL_AUTO 0 /* FP64 when L >= 2^18 or L/min(B,256) > 1024 */
#define TACHES_TAIL_FP32 1
#define TACHES_TAIL_FP64 2

typedef struct taches_stream taches_stream;
typedef struct taches_pool taches_pool;

typedef struct taches_config {
  int32_t block_size;          /* B >= 1: samples per channel per block      */
  int32_t max_ir_len;          /* Lmax >= 1: longest IR this stream accepts  */
  int32_t channels;            /* C >= 1: channels sharing the IR            */
  int32_t max_blocks_per_call; /* >= 1: largest n_blocks of process_blocks   */
  int32_t precision;           /* TACHES_PREC_*                              */
  int32_t tail;                /* TACHES_TAIL_*                              */
  int32_t ir_slots;            /* >= 2: device IR slots (for IR schedules)   */
  int32_t device;              /* HIP device ordinal                         */
} taches_config;

/* Fill *cfg with defaults: channels 1, one block per call, FP32, AUTO tail,
 * 2 IR slots, device 0. */
void taches_config_default(taches_config* cfg, int32_t block_size, int32_t max_ir_len);

/* ---- stream lifetime --------------------------------------------------- */

/* Open a mono FP32 stream (the paper's TachesAlgorithm(pe, h, Nb) with Nb =
 * block_size, Section 4.2).  Allocates the circular tail of
 * >= max_ir_len - 1 + block_size slots on device 0 and clears it.
 * Returns NULL on failure (see taches_last_error). */
taches_stream* taches_open(int32_t block_size, int32_t max_ir_len);

/* Same with every option.  The tail holds max_ir_len - 1 +
 * block_size * max_blocks_per_call slots per channel (FP32 or FP64). */
taches_stream* taches_open_ex(const taches_config* cfg);

/* Wait for the handle's work, free all its device and host memory.  NULL is
 * a no-op.  Returns TACHES_EBUSY if the stream is attached to a pool. */
int taches_close(taches_stream* s);

/* Message of the last failure on this thread ("" if none). */
const char* taches_last_error(void);

/* Order all later device work of this handle on `hip_stream`, a
 * hipStream_t such as torch.cuda.current_stream().cuda_stream.  NULL is
 * HIP's null (default) stream, as in the HIP API.  A handle starts on a
 * non-blocking stream of its own.  Work already enqueued is first waited for. */
int taches_set_hip_stream(taches_stream* s, void* hip_stream);

/* Block the host until all device work of the handle is done. */
int taches_synchronize(taches_stream* s);

/* ---- a1: impulse response staging -------------------------------------- */

/* Queue h[0..L) (host, FP32) as the IR for the next block (Abstract,
 * Section 6): it becomes active at the first block of the next process
 * call; blocks already processed keep their taches.  Several calls before
 * one block: the last wins.  1 <= L <= max_ir_len, else TACHES_EINVAL.
 * h is copied before return; the caller may reuse it at once. */
int taches_set_ir(taches_stream* s, const float* h, int32_t L);

/* Same with h on the device (stream-ordered copy; keep h alive until the
 * handle's stream has passed this point). */
int taches_set_ir_device(taches_stream* s, const float* h_dev, int32_t L);

/* Sample-accurate swap (the IR may change "even sample by sample", Section
 * 6): like taches_set_ir, but the new IR takes over at sample `offset`
 * (0 <= offset < B) of the next processed block; that block's samples
 * before `offset` keep the current IR's taches, and its later samples and
 * all later blocks use the new one.  offset 0 is taches_set_ir.  h on the
 * device if h_on_device is nonzero.  TACHES_EINVAL for an offset out of
 * range, or an offset > 0 on a SPLIT_BF16 stream (not supported there); the
 * next process call returns TACHES_ENOIR if no IR is active for the samples
 * before `offset`. */
int taches_set_ir_at(taches_stream* s, const float* h, int32_t L, int32_t offset, int32_t h_on_device);

/* As taches_set_ir_at with a device IR, without copying it: the stream reads
 * h_dev[0..L) in place from sample `offset` of the next processed block on.
 * The caller keeps those L floats unchanged and allocated until a later IR
 * has taken over and every block enqueued with this one has completed (for
 * a stream attached to a pool: until the pool's queued steps are done).
 * TACHES_EINVAL on a SPLIT_BF16 stream (its MFMA path needs the BF16 split
 * of a copy) and for the sizes taches_set_ir_at refuses. */
int taches_set_ir_ref(taches_stream* s, const float* h_dev, int32_t L, int32_t offset);

/* Load h[0..L) into IR slot `slot` (0 <= slot < ir_slots) for use by an IR
 * schedule of taches_process_blocks.  h_on_device selects host or device
 * memory for h.  Loading the active slot is allowed: the copy is ordered
 * after the work already enqueued, so earlier blocks keep the old IR. */
int taches_load_ir_slot(taches_stream* s, int32_t slot, const float* h, int32_t L,
                        int32_t h_on_device);

/* ---- a2..a4: process blocks -------------------------------------------- */

/* One block, host buffers, blocking: x[C*B] in, y[C*B] out.  y[c*B+i] is
 * the output for the same sample time as x[c*B+i] and already holds that
 * sample's own tache (zero algorithmic latency, Sections 4.1-4.2). */
int taches_process(taches_stream* s, const float* x, float* y);

/* One block, device buffers, asynchronous on the handle's stream. */
int taches_process_async(taches_stream* s, const float* x_dev, float* y_dev);

/* n_blocks consecutive blocks in one launch, device buffers, asynchronous.
 * x_dev: [C][n_blocks*B] planar (channel stride n_blocks*B), or NULL for
 * zero input (drains the temporal overflow); y_dev: same shape.
 * ir_slot_of_block: host array of n_blocks entries or NULL; entry b >= 0
 * makes that IR slot active from block b on, -1 keeps the current IR.  A
 * pending taches_set_ir applies before block 0.  The result equals n_blocks
 * calls of taches_process_async bit for bit. */
int taches_process_blocks(taches_stream* s, const float* x_dev, float* y_dev, int32_t n_blocks,
                          const int32_t* ir_slot_of_block);

/* taches_process_blocks with sample-accurate swaps: offset_of_block (host,
 * n_blocks entries, or NULL for all 0) gives, for every block b with
 * ir_slot_of_block[b] >= 0, the sample of block b (0 <= offset < B) from
 * which that slot takes over.  Equals the same schedule applied block by
 * block with taches_set_ir_at, bit for bit.  TACHES_EINVAL if offsets are
 * given without a schedule, an offset is out of range, or the stream is
 * SPLIT_BF16 and an offset is > 0. */
int taches_process_blocks_at(taches_stream* s, const float* x_dev, float* y_dev, int32_t n_blocks,
                             const int32_t* ir_slot_of_block, const int32_t* offset_of_block);

/* ---- off-line mode ---------------------------------------------------------
 *
 * Whole-signal convolution, the paper's measured setting (files convolved
 * off-line, Section 5.1): y = x * h for `channels` channels sharing h, one
 * launch of the same kernels over all blocks plus the temporal overflow.
 * x_dev: [channels][nx] planar device buffer; h_dev: nh device taps;
 * y_dev: [channels][nx + nh - 1] planar device buffer (written in full).
 * precision: TACHES_PREC_FP32 or TACHES_PREC_SPLIT_BF16.  role_swap != 0
 * with one channel and nh > nx exchanges the roles of input and IR (Section
 * 3.2, Fig. 6): the shorter operand becomes the IR, so min(nx, nh) taches
 * of max(nx, nh) taps are scattered; the result is the same convolution up
 * to rounding order.  Runs on
 * hip_stream (NULL = HIP's null stream) of `device`, allocates its work
 * buffers itself and returns when y is written.  TACHES_EINVAL for NULL
 * buffers or bad sizes, TACHES_ENOMEM, TACHES_EDEVICE. */
int taches_convolve(const float* x_dev, int64_t nx, int32_t channels, const float* h_dev, int32_t nh, float* y_dev,
                    int32_t precision, int32_t role_swap, int32_t device, void* hip_stream);

/* taches_convolve for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  FP32 precision; same operands, role exchange and result as
 * taches_convolve with TACHES_PREC_FP32, bit for bit.  Its work memory (the
 * zero-padded input and the tail the kernel clears as it emits; nothing in
 * it needs clearing between calls) is a fixed 64 MiB array in the library's
 * device code, held on every device the library runs on until the process
 * ends: the call needs
 *   align256(4 * channels * ceil(ns / 256) * 256) + w * channels * (nx + nh - 1)
 * bytes of it (ns = the signal operand's length after any role exchange,
 * w = 8 when the longer-lived operand, the IR, has >= 2^18 taps, else 4),
 * and returns TACHES_EINVAL when that exceeds 64 MiB.  Allocates nothing
 * (no hipMalloc, hipFree or allocating library call) and does not wait:
 * the work is enqueued on hip_stream (NULL = HIP's null stream) of `device`
 * and y_dev is written once that stream has run it; keep x_dev, h_dev and
 * y_dev alive until then.  Every call on one device shares the one array:
 * calls that may overlap on a device (on different HIP streams, or from
 * different threads without ordering) race and give wrong results; calls
 * ordered on one HIP stream are safe.  TACHES_EINVAL for NULL buffers, bad
 * sizes or a device ordinal >= 64, TACHES_EDEVICE on a HIP error. */
int taches_convolve_noalloc(const float* x_dev, int64_t nx, int32_t channels, const float* h_dev, int32_t nh,
                            float* y_dev, int32_t role_swap, int32_t device, void* hip_stream);

/* ---- state ------------------------------------------------------------- */

typedef struct taches_info {
  int32_t block_size, max_ir_len, channels, max_blocks_per_call;
  int32_t precision;
  int32_t tail_fp64;     /* 1 if the tail accumulator is FP64 */
  int32_t ring_slots;    /* circular tail length per channel */
  int32_t head;          /* slot of the next output sample */
  int32_t live;          /* slots after head that may hold pending sums */
  int32_t active_len;    /* length of the active IR, 0 = none */
  int64_t blocks_done;   /* blocks processed since open */
  int64_t device_bytes;  /* device memory owned by the handle */
  int32_t tile_r, tile_w;/* last gather tile config used */
} taches_info;

int taches_get_info(const taches_stream* s, taches_info* out);

/* Device timing of calls (measurement).  While timing is on, every
 * taches_process* call records a pair of HIP events on the stream right
 * before and right after its kernel launches, so host-side work before the
 * launch is not counted; the last 4096 recorded calls are kept.
 * taches_call_times waits for the recorded calls, writes the device time in
 * ms of the last min(n, recorded) of them, oldest first, to ms_out, clears
 * the record and returns how many it wrote (negative: error code).  Calls on
 * a stream attached to a pool are not recorded (taches_pool_info reports the
 * batched launch). */
int taches_set_timing(taches_stream* s, int32_t on);
int taches_call_times(taches_stream* s, double* ms_out, int32_t n);

/* Device bytes a stream with this config would own (for HBM admission). */
int64_t taches_bytes_for(const taches_config* cfg);

/* 1 if a stream opened with this config keeps an FP64 tail, 0 for FP32
 * (TACHES_TAIL_AUTO resolved from block_size and max_ir_len: one output
 * receives about max_ir_len / min(block_size, 256) chunk sums, and more
 * than 1024 of them, or an IR of >= 2^18 taps, take FP64); TACHES_EINVAL for
 * an invalid config.  Lets a caller that opens streams with a larger
 * max_ir_len than the IRs it will load pick the tail from the IR length. */
int taches_tail_is_fp64(const taches_config* cfg);

/* Copy the pending sums for the next n output samples of channel c into
 * out[0..n) (host, FP64).  Synchronizes the handle.  Slot k is what the
 * tail holds for output head+k: the residue of Section 4.2 in output order. */
int taches_read_tail(taches_stream* s, int32_t channel, double* out, int32_t n);

/* Return the stream to its state right after open (empty tail, no IR)
 * without freeing memory or enqueuing device work: the tail counts as empty
 * (no slot is read before it is written again).  For reusing a stream for
 * a new input. */
int taches_reset(taches_stream* s);

/* Force the gather tile shape (R outputs per lane in {4, 8, 12, 14, 16}, W waves
 * per output tile in {1, 2, 4}); 0, 0 = automatic choice per call.  A forced
 * shape keeps the automatic choice of launch order (the order in which
 * output tiles are handed to workgroups).  Results do not depend on either. */
int taches_set_tile(taches_stream* s, int32_t r, int32_t w);

/* ---- a6/a7: pools — many streams advanced by one batched launch ----------
 *
 * A pool admits streams up to a stream count and an HBM byte budget (the
 * sum of the attached streams' device_bytes).  taches_pool_step advances a
 * set of attached streams by n_blocks[i] blocks each in one persistent
 * launch: the host cuts every stream's call into work items (output tiles,
 * or runs of consecutive tiles when tiles are many) and lists them in the
 * order the resident workgroups take them from a shared counter: stream
 * order for many similar items, largest first otherwise.  Each stream's
 * result is bit-identical to processing it alone, whatever workgroup
 * computes which tile.  While attached, a stream's
 * device work runs on the pool's HIP stream; taches_set_ir and
 * taches_load_ir_slot stay usable (a pending IR applies at the stream's next
 * step); taches_process* and taches_close return TACHES_EBUSY. */

/* NULL on failure.  max_streams in [1, 2^20], hbm_budget_bytes >= 0. */
taches_pool* taches_pool_create(int32_t max_streams, int64_t hbm_budget_bytes, int32_t device);

/* TACHES_EBUSY while streams are attached.  NULL is a no-op. */
int taches_pool_destroy(taches_pool* p);

/* Admit a stream: TACHES_EBUSY if the pool is full or the stream is already
 * in a pool, TACHES_ENOMEM if its device bytes exceed the remaining budget.
 * Does not wait: the pool's later work is ordered after the work queued on
 * the stream's HIP stream. */
int taches_pool_attach(taches_pool* p, taches_stream* s);

/* Release the stream's slot and bytes.  Does not wait: later work on the
 * stream's own HIP stream is ordered after the pool's queued steps, which
 * may still use the stream's tail and IR slots. */
int taches_pool_detach(taches_pool* p, taches_stream* s);

/* Advance n attached streams (each listed once): stream i processes
 * n_blocks[i] blocks, input x_dev[i] ([C][n_blocks*B] device, or NULL /
 * x_dev == NULL for zero input), output y_dev[i] (same shape).  Device
 * buffers must stay alive until the pool's HIP stream has run the step.
 * On error no stream is advanced. */
int taches_pool_step(taches_pool* p, int32_t n, taches_stream* const* streams, const float* const* x_dev,
                     float* const* y_dev, const int32_t* n_blocks);

/* taches_pool_step with explicit channel strides (in floats): channel c of
 * stream i reads x_dev[i] + c * x_cstride[i] and writes y_dev[i] +
 * c * y_cstride[i], n_blocks[i] * B samples each, so the buffers can be
 * slices of larger planar arrays (e.g. blocks k..k+n-1 of a whole-signal
 * buffer).  A NULL stride array, or a 0 entry, means packed channels
 * (stride n_blocks[i] * B).  Multichannel strides shorter than
 * n_blocks[i] * B are TACHES_EINVAL.  Same ownership and errors as
 * taches_pool_step. */
int taches_pool_step_strided(taches_pool* p, int32_t n, taches_stream* const* streams, const float* const* x_dev,
                             const int64_t* x_cstride, float* const* y_dev, const int64_t* y_cstride,
                             const int32_t* n_blocks);

/* HIP stream for the pool and its attached streams (NULL = HIP's null
 * stream).  Work already enqueued is first waited for. */
int taches_pool_set_hip_stream(taches_pool* p, void* hip_stream);

/* HIP stream for the host-to-device copy of each step's work table
 * (nullptr, the default: the pool's stream, inside its captured graph).
 * With a copy stream, the copy of step k + 1's table can run while step
 * k's kernel does; the pool's stream waits for each copy through an event.
 * The caller keeps the stream alive while it is set; setting another one
 * first waits for the current one. */
int taches_pool_set_copy_stream(taches_pool* p, void* hip_stream);

/* Per-lane tile of the batched kernel (4, 8, 12, 16; 0 = automatic). */
int taches_pool_set_tile(taches_pool* p, int32_t r);

/* Run each step as a replay of a captured hipGraph (table copy + kernel);
 * the graph is captured again when the tile or workgroup count changes. */
int taches_pool_use_graph(taches_pool* p, int32_t on);

int taches_pool_synchronize(taches_pool* p);

typedef struct taches_pool_info {
  int32_t attached, max_streams;
  int64_t budget_bytes, used_bytes;
  int32_t last_items;       /* work items of the last step */
  int32_t last_workgroups;  /* persistent workgroups of the last step */
  int32_t last_r;           /* per-lane tile of the last step */
  int32_t pad_;
  int64_t graph_replays;
  double last_plan_ms;      /* host time to plan the last step */
  double last_imbalance;    /* estimated busiest workgroup's work / mean work
                               (workgroups take work items from a queue) */
  double last_device_ms;    /* device time of the last step's batched launch
                               (table copy + kernel); -1 until it has run */
  double device_ms_total;   /* device time of all batched launches found
                               complete so far (steps run without waiting) */
  int64_t graph_captures;   /* graphs captured (one per tile, FP64-tail mix and
                               workgroup count class; again after the table grows) */
} taches_pool_info;

int taches_pool_get_info(const taches_pool* p, taches_pool_info* out);

/* ---- a7: serving tick — real-time streams of a pool, one call per tick ----
 *
 * A server drives attached streams of one pool in real time (continuous
 * batching for low-latency real-time use with changing IRs, Section 6).  A
 * registered stream delivers one block of B samples per channel every
 * B / fs seconds from its start time; after its n_in input blocks, its
 * temporal overflow (Section 4.1) is drained with zero-input blocks paced
 * the same way, up to n_total blocks.  taches_server_tick takes every block
 * whose last sample has arrived by the server clock, over all registered
 * streams (at most max_blocks_per_step per stream), and runs them as one
 * pool step: the arrived input is gathered from each stream's host buffer
 * into pinned memory and copied to the device in one transfer; after the
 * pool step one launch writes every output block (for a two-segment stream,
 * with the rest segment's ring added) to mapped, coherent pinned host
 * memory, and the outputs are copied to the stream's host buffer (if any)
 * when the step completes (during the next tick or flush).  An IR change scheduled at time
 * t (seconds from the stream's start) applies to the first block that
 * starts at or after t (the IR is replaced for the next samples, Abstract
 * and Section 6).  Latency of a block = the time its step's output launch
 * completed (outputs in host memory; a device event recorded after it,
 * placed on the server clock) minus the arrival time of its last sample; the deadline is one
 * block period.  The server does not own streams: register an
 * attached stream, and detach it after its tag is reported finished.  A
 * server is not thread-safe.  After TACHES_EDEVICE from a tick, destroy the
 * server and its pool. */

typedef struct taches_server taches_server;

typedef struct taches_server_tick_info {
  int32_t streams;  /* streams advanced (0: no block was due, nothing ran) */
  int32_t pad_;
  int64_t blocks;   /* blocks processed */
  double now_s;     /* server clock when the tick started */
  double done_s;    /* server clock when the tick returned (the previous step completed) */
  double host_ms;   /* host work before the first transfer (ranges, IR changes, input gather) */
  double step_ms;   /* the whole tick */
  double next_due_s;/* server clock at which the next block of a registered
                       stream is complete (HUGE_VAL if none is registered) */
} taches_server_tick_info;

typedef struct taches_server_stats {
  int64_t ticks;                  /* ticks that ran a step */
  int64_t blocks;                 /* blocks processed */
  int64_t macs;                   /* direct-equivalent MACs of the input blocks */
  int64_t max_blocks_in_a_range;  /* most blocks of one stream in one step */
  int64_t bytes_in, bytes_out;    /* input bytes copied to the device, output bytes written to host memory */
  double busy_s;                  /* summed duration of the ticks that ran a step, split into: */
  double gather_s;                /*   ranges, IR changes and input gather on the host */
  double launch_s;                /*   input copy and pool step enqueued (step planning included) */
  double wait_s;                  /*   waiting for the device (step and output launch) */
  double scatter_s;               /*   outputs to the streams' host buffers, latency records */
  int32_t streams;                /* streams registered and not finished */
  int32_t pad_;
  int64_t recorded;               /* blocks with a latency record, whose latencies split into: */
  double pickup_s;                /*   summed time from a block's arrival to the start of its tick */
  double service_s;               /*   summed time from the start of its tick to its outputs in host memory */
  double device_s;                /* summed device time of the completed steps, input copy to output launch */
} taches_server_stats;

/* NULL on failure.  fs > 0 (samples per second), max_blocks_per_step >= 1
 * (every registered stream must accept that many blocks per call); blocks
 * whose last sample arrives before warmup_s (server clock) are not
 * recorded.  The server clock starts at 0 when the server is created. */
taches_server* taches_server_create(taches_pool* pool, double fs, int32_t max_blocks_per_step, double warmup_s);

/* Waits for the pool's queued work and frees the staging.  NULL is a no-op. */
int taches_server_destroy(taches_server* sv);

/* Seconds since taches_server_create (steady clock); -1 for NULL. */
double taches_server_clock(const taches_server* sv);

/* Register stream s (attached to the server's pool, its IR for the first
 * block already set) under `tag` (unique per server).  start_s: server-clock
 * time of its first sample.  x_host: [C][x_cstride] host input, n_in_blocks
 * * B samples per channel (caller-owned, alive until the stream finishes).
 * y_host: [C][y_cstride] host output of n_total_blocks * B samples per
 * channel, or NULL to discard the outputs after their transfer.
 * n_swaps IR changes: ascending times swap_times_s (seconds from the
 * stream's start), device IRs swap_ir_dev[i] of swap_len[i] taps (alive
 * until the stream is reported finished: an FP32 stream reads them in
 * place, taches_set_ir_ref; a split-BF16 stream copies each when it
 * applies).  TACHES_EINVAL for bad sizes or a duplicate tag. */
int taches_server_add(taches_server* sv, taches_stream* s, int64_t tag, double start_s, int64_t n_in_blocks,
                      int64_t n_total_blocks, const float* x_host, int64_t x_cstride, float* y_host, int64_t y_cstride,
                      int32_t n_swaps, const double* swap_times_s, const float* const* swap_ir_dev,
                      const int32_t* swap_len);

/* Register a stream served in two segments of its IR (Eq. (1) is linear in
 * h): `head` (block B, capacity >= head_len) convolves with h[0, H), H =
 * head_len, and is advanced every tick as in taches_server_add; `rest`
 * (block Br, a multiple of B with Br <= H) convolves with h[H, L) and is
 * advanced once per Br samples, its outputs z kept on the device in the
 * ring z_dev [C][z_len] (caller-owned, z_len a multiple of Br and at least
 * 2 Br, alive until the stream finishes; contents need no initialisation);
 * the result is
 * y[n] = y_head[n] + z[n - H] (FP32 add), written to y_host as in
 * taches_server_add.  Both streams must be attached to the server's pool,
 * FP32 precision, with the same channel count; `head` must take
 * max_blocks_per_step blocks per call, `rest` at least one.  The library
 * loads the two segments of ir_dev [ir_len] (H < ir_len <= H + rest
 * capacity) as the initial IR, and of each change's IR (swap_len[i] in the
 * same range) when it applies, reading them in place (taches_set_ir_ref:
 * ir_dev and the change IRs stay allocated until the stream finishes): the rest segment takes over at the same
 * input sample as the head (an IR change inside a rest block), so two
 * changes applying inside one rest block are refused, the initial IR
 * counting as a change at sample 0.  A tick runs a head
 * block once the rest blocks whose outputs it needs are enqueued (their
 * last sample arrives no later than the head block's), and holds rest
 * blocks while their outputs would overwrite ring entries not yet added.
 * Latency records and outputs are the head's; rest blocks have none.
 * TACHES_EINVAL for sizes or streams outside these rules. */
int taches_server_add_segmented(taches_server* sv, taches_stream* head, taches_stream* rest, int32_t head_len,
                                float* z_dev, int32_t z_len, int64_t tag, double start_s, int64_t n_in_blocks,
                                int64_t n_total_blocks, const float* x_host, int64_t x_cstride, float* y_host,
                                int64_t y_cstride, const float* ir_dev, int32_t ir_len, int32_t n_swaps,
                                const double* swap_times_s, const float* const* swap_ir_dev, const int32_t* swap_len);

/* One tick at the current server clock: if any block is due, enqueues its
 * step (input copy, pool step, output launch) on the pool's stream; then waits
 * for the previous tick's step, hands its outputs to the host buffers and
 * records its latencies (so the host prepares step k + 1 while the device
 * runs step k).  Fills *out (may be NULL).  A stream whose last block has
 * been enqueued no longer takes part; it is reported by
 * taches_server_take_finished once that step has completed. */
int taches_server_tick(taches_server* sv, taches_server_tick_info* out);

/* Wait for the step in flight (if any) and complete it as a tick would. */
int taches_server_flush(taches_server* sv);

/* Tags of streams that finished since the last call (at most cap, oldest
 * first); returns how many were written. */
int taches_server_take_finished(taches_server* sv, int64_t* tags, int32_t cap);

/* Recorded block latencies (seconds) and their block sizes since the last
 * call (at most cap, oldest first); returns how many were written. */
int taches_server_take_latencies(taches_server* sv, float* latency_s, int32_t* block_size, int32_t cap);

/* Next block of a registered (or finished) stream, and the blocks at which
 * its IR changes took effect (at most cap written); returns the number of
 * changes applied so far. */
int taches_server_stream_state(taches_server* sv, int64_t tag, int64_t* next_block, int64_t* swap_blocks, int32_t cap);

int taches_server_get_stats(const taches_server* sv, taches_server_stats* out);

/* ---- diagnostics -----------------------------------------------------------
 *
 * FP32 fused-multiply-add rate (TFLOP/s, 2 FLOP per FMA) that independent
 * unpacked v_fmac_f32 chains reach on `device`, with no memory traffic: the
 * issue ceiling of the FP32 gather kernels, which are built without packed
 * FP32 instructions (the published vector peak counts packed FP32).  Runs
 * for about 20 ms.  TACHES_EDEVICE on a HIP error. */
int taches_fp32_fma_ceiling(int32_t device, double* tflops_out);

#ifdef __cplusplus
}
#endif

#endif /* TACHES_H */
