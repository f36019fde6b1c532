// Host runtime and C-ABI of libtaches: stream handles, IR slots, the
// circular tail, call planning and kernel launches.
#include <algorithm>
#include <array>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "taches.h"
#include "taches_internal.h"

using taches::BlockIR;
using taches::GatherCall;

// Work memory of taches_convolve_noalloc on each device (see below).
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

// Message of the last failure on this thread: a fixed buffer, so that
// reporting an error allocates nothing.
constexpr size_t kErrLen = 512;
thread_local char g_err[kErrLen] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, kErrLen, fmt, ap);
  va_end(ap);
  return code;
}

// Keeps the current error message across cleanup calls that may fail.
struct ErrKeep {
  char msg[kErrLen];
  ErrKeep() { std::memcpy(msg, g_err, kErrLen); }
  ~ErrKeep() { std::memcpy(g_err, msg, kErrLen); }
};

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(TACHES_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Tail accumulator type: FP64 when the IR is long (L >= 2^18) or when one
// output would receive more than 1024 chunk additions in FP32 (measured on
// flat white-noise IRs: up to 1024 additions the FP32 tail stays below
// 7.3e-6 * RMS of the FP64 result, at 2048 it reaches 1.04e-5).
bool want_fp64(const taches_config& c) {
  if (c.tail == TACHES_TAIL_FP64) return true;
  if (c.tail == TACHES_TAIL_FP32) return false;
  const int64_t chunk = std::min<int64_t>(c.block_size, taches::CHUNK_MAX);
  return c.max_ir_len >= (1 << 18) || (int64_t)c.max_ir_len > 1024 * chunk;
}

int64_t ring_slots_for(const taches_config& c) {
  return round_up((int64_t)c.max_ir_len - 1 + (int64_t)c.block_size * c.max_blocks_per_call, 64);
}

bool is_split(const taches_config& c) { return c.precision == TACHES_PREC_SPLIT_BF16; }

// Per-call table (device, filled per call when needed): one BlockIR per block
// when the IR changes between blocks; when an IR takes over inside a block,
// one BlockIR per slot followed by the chunk table: the first chunk of each
// block [n_blocks + 1], then {first sample, length, slot} per chunk (a block
// cut by a swap has at most one chunk more than ceil(B / CHUNK_MAX)).
int64_t max_chunks_per_call(const taches_config& c) {
  return (int64_t)c.max_blocks_per_call * ((c.block_size + taches::CHUNK_MAX - 1) / taches::CHUNK_MAX + 1);
}

int64_t irtab_bytes(const taches_config& c) {
  const int64_t per_block = (int64_t)c.max_blocks_per_call * (int64_t)sizeof(BlockIR);
  const int64_t chunked = (int64_t)c.ir_slots * (int64_t)sizeof(BlockIR) +
                          4 * ((int64_t)c.max_blocks_per_call + 1 + 3 * max_chunks_per_call(c));
  return std::max(per_block, chunked);
}

// channels stored per tail slot: the split path pads to its MFMA width
int64_t ring_channels(const taches_config& c) { return is_split(c) ? taches::split_cpad(c.channels) : c.channels; }

int64_t chunks_per_block(const taches_config& c) { return (c.block_size + taches::CHUNK_MAX - 1) / taches::CHUNK_MAX; }

// bytes of one split input staging buffer (hi or lo) for the largest call
int64_t xs_bytes(const taches_config& c) {
  return is_split(c) ? (int64_t)c.max_blocks_per_call * chunks_per_block(c) * 32 * ring_channels(c) * 8 * 2 : 0;
}

int validate(const taches_config* c) {
  if (!c) return fail(TACHES_EINVAL, "config is NULL");
  if (c->block_size < 1 || c->max_ir_len < 1 || c->channels < 1 || c->max_blocks_per_call < 1)
    return fail(TACHES_EINVAL, "block_size, max_ir_len, channels and max_blocks_per_call must be >= 1");
  if (c->precision != TACHES_PREC_FP32 && c->precision != TACHES_PREC_SPLIT_BF16)
    return fail(TACHES_EINVAL, "unknown precision %d", c->precision);
  if (c->tail < TACHES_TAIL_AUTO || c->tail > TACHES_TAIL_FP64) return fail(TACHES_EINVAL, "unknown tail %d", c->tail);
  if (c->ir_slots < 2 || c->ir_slots > 64) return fail(TACHES_EINVAL, "ir_slots must be in [2, 64]");
  const int64_t S = (int64_t)c->block_size * c->max_blocks_per_call;
  if (S + c->max_ir_len >= (int64_t)1 << 30) return fail(TACHES_EINVAL, "block_size * max_blocks_per_call + max_ir_len too large");
  if ((int64_t)c->channels * ring_slots_for(*c) >= (int64_t)1 << 34) return fail(TACHES_EINVAL, "tail too large");
  if (c->precision == TACHES_PREC_SPLIT_BF16 && (c->channels < 1 || c->channels > 64))
    return fail(TACHES_EINVAL, "split-BF16 path needs 1 <= channels <= 64");
  return TACHES_OK;
}

struct IrSlot {
  float* h = nullptr;       // device, Lmax taps
  const float* ref = nullptr;   // the caller's device IR, read in place instead of h (FP32 only)
  uint16_t* hi = nullptr;   // device BF16 hi copy (split precision)
  uint16_t* lo = nullptr;   // device BF16 lo copy
  int L = 0;
  float* staging = nullptr; // pinned host copy source
  hipEvent_t ev = nullptr;  // completes when the last copy out of staging is done
  bool ev_pending = false;
};

}  // namespace

struct taches_stream {
  taches_config cfg{};
  bool tail_fp64 = false;
  int Rcap = 0;
  void* ring = nullptr;
  std::vector<IrSlot> slots;
  int active = -1, pending = -1;
  int pending_off = 0;                            // sample of the next block where `pending` takes over
  int head = 0, live = 0;
  int64_t blocks_done = 0;
  hipStream_t own = nullptr, stream = nullptr;
  float *x_pin = nullptr, *y_pin = nullptr, *x_dev = nullptr, *y_dev = nullptr;
  BlockIR *irtab_dev = nullptr, *irtab_pin = nullptr;
  hipEvent_t irtab_ev = nullptr;
  bool irtab_pending = false;
  std::vector<unsigned char> irtab_new, irtab_dev_copy;   // table being built; what irtab_dev holds
  bool timing = false;                            // record events around each call's kernels
  std::vector<hipEvent_t> tev;                    // [2 * kTimedCalls] start/end pairs (ring)
  int64_t timed = 0;                              // calls recorded since the last read
  int force_r = 0, force_w = 0, last_r = 0, last_w = 0;
  int64_t device_bytes = 0;
  taches_pool* pool = nullptr;
  hipStream_t stream_before_pool = nullptr;
  uint16_t *xs_hi = nullptr, *xs_lo = nullptr;  // split path: per-call input fragments
  int cpad = 0;                                 // channels per tail slot (split path)
  int64_t plan_key[4] = {-1, -1, -1, -1};        // last planned call shape and its tile plan
  int plan_val[3] = {0, 0, 0};
  uint64_t step_mark = 0;                         // pool step that last listed the stream
};

namespace {

void free_stream(taches_stream* s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  (void)hipFree(s->ring);
  for (auto& sl : s->slots) {
    (void)hipFree(sl.h);
    (void)hipFree(sl.hi);
    (void)hipFree(sl.lo);
    (void)hipHostFree(sl.staging);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
  }
  (void)hipFree(s->x_dev);
  (void)hipFree(s->y_dev);
  (void)hipHostFree(s->x_pin);
  (void)hipHostFree(s->y_pin);
  (void)hipFree(s->irtab_dev);
  (void)hipHostFree(s->irtab_pin);
  (void)hipFree(s->xs_hi);
  (void)hipFree(s->xs_lo);
  if (s->irtab_ev) (void)hipEventDestroy(s->irtab_ev);
  for (hipEvent_t ev : s->tev)
    if (ev) (void)hipEventDestroy(ev);
  if (s->own) (void)hipStreamDestroy(s->own);
  delete s;
}

template <typename T>
int dev_alloc(taches_stream* s, T** p, size_t bytes) {
  hipError_t e = hipMalloc((void**)p, bytes);
  if (e != hipSuccess) return fail(TACHES_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  s->device_bytes += (int64_t)bytes;
  return TACHES_OK;
}

template <typename T>
int host_alloc(T** p, size_t bytes) {
  hipError_t e = hipHostMalloc((void**)p, bytes, hipHostMallocDefault);
  if (e != hipSuccess) return fail(TACHES_ENOMEM, "hipHostMalloc(%zu): %s", bytes, hipGetErrorString(e));
  return TACHES_OK;
}

int stream_init(taches_stream* s) {
  const taches_config& c = s->cfg;
  HIPCHK(hipSetDevice(c.device));
  HIPCHK(hipStreamCreateWithFlags(&s->own, hipStreamNonBlocking));
  s->stream = s->own;
  s->tail_fp64 = want_fp64(c);
  s->Rcap = (int)ring_slots_for(c);
  s->cpad = (int)ring_channels(c);
  const size_t esz = s->tail_fp64 ? 8 : 4;
  const size_t ring_bytes = (size_t)s->cpad * s->Rcap * esz;
  int rc;
  if ((rc = dev_alloc(s, &s->ring, ring_bytes))) return rc;
  HIPCHK(hipMemsetAsync(s->ring, 0, ring_bytes, s->stream));
  s->slots.resize(c.ir_slots);
  for (auto& sl : s->slots) {
    if ((rc = dev_alloc(s, &sl.h, (size_t)c.max_ir_len * 4))) return rc;
    if (c.precision == TACHES_PREC_SPLIT_BF16) {
      if ((rc = dev_alloc(s, &sl.hi, (size_t)c.max_ir_len * 2))) return rc;
      if ((rc = dev_alloc(s, &sl.lo, (size_t)c.max_ir_len * 2))) return rc;
    }
    HIPCHK(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
  }
  const size_t blk = (size_t)c.channels * c.block_size * 4;
  if ((rc = dev_alloc(s, &s->x_dev, blk))) return rc;
  if ((rc = dev_alloc(s, &s->y_dev, blk))) return rc;
  const size_t tab = (size_t)irtab_bytes(c);
  if ((rc = dev_alloc(s, &s->irtab_dev, tab))) return rc;
  HIPCHK(hipEventCreateWithFlags(&s->irtab_ev, hipEventDisableTiming));
  if (is_split(c)) {
    if ((rc = dev_alloc(s, &s->xs_hi, (size_t)xs_bytes(c)))) return rc;
    if ((rc = dev_alloc(s, &s->xs_lo, (size_t)xs_bytes(c)))) return rc;
  }
  HIPCHK(hipStreamSynchronize(s->stream));
  return TACHES_OK;
}

int load_slot(taches_stream* s, int slot, const float* h, int L, bool on_device) {
  IrSlot& sl = s->slots[slot];
  sl.ref = nullptr;
  if (on_device) {
    HIPCHK(hipMemcpyAsync(sl.h, h, (size_t)L * 4, hipMemcpyDeviceToDevice, s->stream));
  } else {
    if (!sl.staging) {  // pinned staging is allocated on first use
      int rc = host_alloc(&sl.staging, (size_t)s->cfg.max_ir_len * 4);
      if (rc != TACHES_OK) return rc;
    }
    if (sl.ev_pending) {
      HIPCHK(hipEventSynchronize(sl.ev));
      sl.ev_pending = false;
    }
    std::memcpy(sl.staging, h, (size_t)L * 4);
    HIPCHK(hipMemcpyAsync(sl.h, sl.staging, (size_t)L * 4, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipEventRecord(sl.ev, s->stream));
    sl.ev_pending = true;
  }
  if (s->cfg.precision == TACHES_PREC_SPLIT_BF16) {
    hipError_t e = taches::launch_split_bf16(sl.h, sl.hi, sl.lo, L, s->stream);
    if (e != hipSuccess) return fail(TACHES_EDEVICE, "IR split: %s", hipGetErrorString(e));
  }
  sl.L = L;
  return TACHES_OK;
}

// Tile shape (r outputs per lane, w waves per tile) and tile order.  The
// estimate simulates the dispatch: workgroup i (in launch order) goes to XCD
// i % 8 and, within it, round-robin over its 32 CUs; a CU's time is the FMA
// work of its tiles divided by the SIMDs it keeps busy; the launch takes as
// long as its busiest CU.  Work per tile is
// the number of input samples that reach it.  Longer per-lane tiles need
// fewer LDS reads per FMA (eff_r) and fewer than two waves per SIMD expose
// latency.
struct TilePlan {
  int r = 4, w = 1, order = 0;
};

// CU loads of one tile shape and launch order (the same for every W): the
// FMA work of the tiles each CU receives, and their number.
constexpr int kCUs = 256;
typedef std::array<double, kCUs> CuLoad;
typedef std::array<int, kCUs> CuCount;

void plan_loads(int64_t S, int64_t n_out, int64_t lmax, int channels, int r, int order, CuLoad& cu, CuCount& cnt) {
  const int64_t T = 64 * r;
  const int64_t nt = (n_out + T - 1) / T;
  cu.fill(0.0);
  cnt.fill(0);
  const int64_t total = nt * channels;
  const int64_t mid = (nt - 1) / 2;
  const int64_t q = nt >> 3, rem = nt & 7;
  for (int64_t id = 0; id < total; ++id) {
    const int64_t ci = id % nt;  // launch index within one channel
    int64_t t;
    if (order == 0) {
      const int64_t x = ci & 7, k = ci >> 3;
      t = x * q + std::min(x, rem) + k;
    } else if (order == 1) {
      t = (ci & 1) ? mid + ((ci + 1) >> 1) : mid - (ci >> 1);
    } else {
      t = ci;
    }
    const int64_t n0 = t * T;
    const int64_t lo = std::max<int64_t>(0, n0 - (lmax - 1));
    const int64_t hi = std::min<int64_t>(S, n0 + T);
    const double work = (double)std::max<int64_t>(hi - lo, 0) * T + 64.0 * T;  // + staging/tail io
    const int c = (int)((id & 7) * 32 + (id >> 3) % 32);
    cu[c] += work;
    cnt[c] += 1;
  }
}

// Estimated time of the launch with w waves per tile: its busiest CU.
// Measured efficiencies with every CU full: longer per-lane tiles need
// fewer LDS reads per FMA (eff_r); waves that share a tile work on adjacent
// chunks whose IR windows overlap, one-wave tiles each stream their own
// window (eff_w).
double plan_cost(const CuLoad& cu, const CuCount& cnt, int r, int w) {
  static const double eff_r[17] = {0, 0, 0, 0, 0.85, 0, 0, 0, 0.92, 0, 0, 0, 0.95, 0, 0.885, 0, 0.97};
  const double eff_w = w == 4 ? 1.0 : w == 2 ? 0.92 : 0.845;
  double worst = 0.0;
  for (size_t i = 0; i < cu.size(); ++i) {
    const double waves = (double)cnt[i] * w;
    const double simds = std::min(4.0, waves);
    double t = simds > 0 ? cu[i] / simds : 0.0;
    if (waves < 8.0) t /= 0.9;  // fewer than two waves per SIMD
    worst = std::max(worst, t);
  }
  return worst / (eff_r[r] * eff_w);
}

// Plans by call shape, shared by all streams of the process (a stream also
// keeps its last plan): a call shape seen before is not simulated again.
std::mutex g_plan_mu;
std::map<std::array<int64_t, 6>, TilePlan> g_plans;

// The estimate for one call shape (no caching, no allocation).  force =
// R * 8 + W for a forced shape (which still gets the launch order the
// estimate prefers for it), 0 for the automatic choice.
TilePlan plan_tile(int force, int channels, int64_t S, int64_t n_out, int64_t lmax, int chunks_per_tile) {
  TilePlan best;
  static const int rs_auto[5] = {16, 14, 12, 8, 4};
  static const int ws_auto[3] = {1, 2, 4};
  const int rs_forced[1] = {force >> 3}, ws_forced[1] = {force & 7};
  const int* rs = force ? rs_forced : rs_auto;
  const int* ws = force ? ws_forced : ws_auto;
  const int nr = force ? 1 : 5, nw = force ? 1 : 3;
  double best_cost = 1e300;
  CuLoad cu[3];
  CuCount cnt[3];
  for (int ir = 0; ir < nr; ++ir) {
    const int r = rs[ir];
    for (int order = 0; order < 3; ++order) plan_loads(S, n_out, lmax, channels, r, order, cu[order], cnt[order]);
    for (int iw = 0; iw < nw; ++iw) {
      const int w = ws[iw];
      if (!force && w > 1 && chunks_per_tile < 2 * w) continue;
      for (int order = 0; order < 3; ++order) {
        const double c = plan_cost(cu[order], cnt[order], r, w);
        if (c < best_cost * 0.999) {
          best_cost = c;
          best.r = r;
          best.w = w;
          best.order = order;
        }
      }
    }
  }
  return best;
}

TilePlan pick_tile(const taches_stream* s, int64_t S, int64_t n_out, int64_t lmax, int chunks_per_tile) {
  const int force = s->force_r ? s->force_r * 8 + (s->force_w ? s->force_w : 1) : 0;
  const std::array<int64_t, 6> key = {S, n_out, lmax, s->cfg.channels, chunks_per_tile, force};
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) return it->second;
  }
  const TilePlan best = plan_tile(force, s->cfg.channels, S, n_out, lmax, chunks_per_tile);
  std::lock_guard<std::mutex> lk(g_plan_mu);
  if (g_plans.size() >= 4096) g_plans.clear();
  g_plans[key] = best;
  return best;
}

// A planned call: the kernel descriptor plus the stream state to commit once
// the call is enqueued.
struct CallPlan {
  GatherCall g{};
  int next_active = -1;
  int64_t S = 0, n_out = 0;
  int n_blocks = 0;
};

// Validate a call and build its descriptor.  Uploads the per-block IR table
// when the IR changes inside the call (and the chunk table when an IR takes
// over inside a block).  Nothing is launched.
// Channel strides of 0 mean packed channels (stride n_blocks * B).
// sched[b] >= 0: slot set before block b, taking over at sample offs[b] of
// it (offs NULL: at its start).
int plan_call(taches_stream* s, const float* x_dev, int64_t x_cstride, float* y_dev, int64_t y_cstride, int n_blocks,
              const int32_t* sched, const int32_t* offs, CallPlan* out) {
  const taches_config& c = s->cfg;
  if (n_blocks < 1 || n_blocks > c.max_blocks_per_call)
    return fail(TACHES_EINVAL, "n_blocks %d outside [1, %d]", n_blocks, c.max_blocks_per_call);
  if (!y_dev) return fail(TACHES_EINVAL, "y is NULL");
  const int B = c.block_size;
  {
    const int64_t S = (int64_t)n_blocks * B;
    if (x_cstride == 0) x_cstride = S;
    if (y_cstride == 0) y_cstride = S;
    if (c.channels > 1 && (x_cstride < S || y_cstride < S))
      return fail(TACHES_EINVAL, "channel stride (x %lld, y %lld) shorter than the call's %lld samples",
                  (long long)x_cstride, (long long)y_cstride, (long long)S);
  }
  if (sched) {
    for (int b = 0; b < n_blocks; ++b) {
      const int k = sched[b];
      if (k < -1 || k >= c.ir_slots) return fail(TACHES_EINVAL, "schedule entry %d: slot %d", b, k);
      if (k >= 0 && s->slots[k].L == 0) return fail(TACHES_ENOIR, "schedule entry %d: slot %d holds no IR", b, k);
      if (k >= 0 && offs && (offs[b] < 0 || offs[b] >= B))
        return fail(TACHES_EINVAL, "schedule entry %d: offset %d outside [0, %d)", b, offs[b], B);
    }
  }
  // IR set before block b (a pending set_ir applies to block 0 unless the
  // schedule sets it) and the sample of the block it takes over at
  auto entry = [&](int b, int* k, int* off) {
    *k = -1;
    *off = 0;
    if (sched && sched[b] >= 0) {
      *k = sched[b];
      *off = offs ? offs[b] : 0;
    } else if (b == 0 && s->pending >= 0) {
      *k = s->pending;
      *off = s->pending_off;
    }
  };
  // resolve every block: IR ir0 from its start, and ir1 from sample `off` on
  // when an IR takes over inside the block
  const int64_t S = (int64_t)n_blocks * B;
  bool uniform = true, intra = false;
  int first_slot = -1, Lmax_call = 0;
  int64_t ext = 0;
  int cur = s->active;
  for (int b = 0; b < n_blocks; ++b) {
    int k, off;
    entry(b, &k, &off);
    int ir0 = cur, ir1 = -1;
    if (k >= 0 && off == 0) ir0 = k;
    if (k >= 0 && off > 0) ir1 = k;
    if (k >= 0) cur = k;
    if (x_dev && ir0 < 0) return fail(TACHES_ENOIR, "no impulse response set for block %d", b);
    if (b == 0) first_slot = ir0;
    if (ir0 != first_slot || ir1 >= 0) uniform = false;
    if (ir1 >= 0) intra = true;
    if (x_dev) {
      const int L0 = s->slots[ir0].L;
      Lmax_call = std::max(Lmax_call, L0);
      ext = std::max<int64_t>(ext, (int64_t)b * B + (ir1 >= 0 ? off : B) + L0 - 1);
      if (ir1 >= 0) {
        const int L1 = s->slots[ir1].L;
        Lmax_call = std::max(Lmax_call, L1);
        ext = std::max<int64_t>(ext, (int64_t)b * B + B + L1 - 1);
      }
    }
    if (!sched && b == 0 && n_blocks > 1) {
      // no schedule: blocks 1 .. n-1 all use `cur`
      if (x_dev) {
        const int L = s->slots[cur].L;
        Lmax_call = std::max(Lmax_call, L);
        ext = std::max<int64_t>(ext, S + L - 1);
      }
      if (cur != first_slot) uniform = false;
      break;
    }
  }
  if (intra && x_dev && is_split(c))
    return fail(TACHES_EINVAL, "an IR taking over inside a block needs FP32 precision");
  const int64_t n_out = std::max<int64_t>(std::max<int64_t>(S, s->live), ext);
  if (n_out > s->Rcap) return fail(TACHES_EINVAL, "call needs %lld tail slots, ring has %d", (long long)n_out, s->Rcap);

  GatherCall& g = out->g;
  g = GatherCall{};
  g.x = x_dev;
  g.y = y_dev;
  g.ring = s->ring;
  g.x_cstride = x_cstride;
  g.y_cstride = y_cstride;
  g.ring_cstride = s->Rcap;
  g.S = (int32_t)S;
  g.B = B;
  g.n_blocks = n_blocks;
  g.cpb = (B + taches::CHUNK_MAX - 1) / taches::CHUNK_MAX;
  g.Rcap = s->Rcap;
  g.head = s->head;
  g.live_in = s->live;
  g.n_out = (int32_t)n_out;
  g.Lmax_call = std::max(Lmax_call, 1);
  g.channels = c.channels;
  g.xs_hi = s->xs_hi;
  g.xs_lo = s->xs_lo;
  g.cpad = s->cpad;
  auto ir_of = [&](int k) {
    BlockIR ir{};
    if (k >= 0) {
      ir.h = s->slots[k].ref ? s->slots[k].ref : s->slots[k].h;
      ir.h_hi = s->slots[k].hi;
      ir.h_lo = s->slots[k].lo;
      ir.L = s->slots[k].L;
    }
    return ir;
  };
  if (!x_dev || uniform) {
    g.irs = nullptr;
    g.ir0 = ir_of(first_slot);
  } else {
    // The table is built on the host and uploaded only when it differs from
    // what the device copy already holds (a call that repeats the previous
    // call's schedule and slots reuses it): the upload is a host-to-device
    // transfer the kernel has to wait for.
    std::vector<unsigned char>& tb = s->irtab_new;
    tb.resize((size_t)irtab_bytes(c));
    BlockIR* tab = reinterpret_cast<BlockIR*>(tb.data());
    size_t bytes;
    if (!intra) {
      int k = s->active;
      for (int b = 0; b < n_blocks; ++b) {
        int e, off;
        entry(b, &e, &off);
        if (e >= 0) k = e;
        tab[b] = ir_of(k);
      }
      bytes = (size_t)n_blocks * sizeof(BlockIR);
    } else {
      // slot table, then the chunk table: each IR segment of a block is cut
      // into ceil(len / CHUNK_MAX) near-equal chunks (a block without a swap
      // inside gets exactly the chunks of the regular geometry)
      for (int k = 0; k < c.ir_slots; ++k) tab[k] = ir_of(k);
      int32_t* bc0 = reinterpret_cast<int32_t*>(tab + c.ir_slots);
      int32_t* cd = bc0 + (n_blocks + 1);
      int nc = 0;
      auto cut = [&](int b, int a, int e, int k) {
        const int n = (e - a + taches::CHUNK_MAX - 1) / taches::CHUNK_MAX;
        for (int i = 0; i < n; ++i) {
          const int lo = b * B + a + (i * (e - a)) / n;
          const int hi = b * B + a + ((i + 1) * (e - a)) / n;
          cd[3 * nc] = lo;
          cd[3 * nc + 1] = hi - lo;
          cd[3 * nc + 2] = k;
          ++nc;
        }
      };
      int k = s->active;
      for (int b = 0; b < n_blocks; ++b) {
        int e, off;
        entry(b, &e, &off);
        bc0[b] = nc;
        if (e >= 0 && off > 0) {
          cut(b, 0, off, k);
          cut(b, off, B, e);
        } else {
          if (e >= 0) k = e;
          cut(b, 0, B, k);
        }
        if (e >= 0) k = e;
      }
      bc0[n_blocks] = nc;
      bytes = (size_t)c.ir_slots * sizeof(BlockIR) + 4 * ((size_t)n_blocks + 1 + 3 * (size_t)nc);
      g.ctab = reinterpret_cast<const int32_t*>(s->irtab_dev + c.ir_slots);
    }
    const bool same = s->irtab_dev_copy.size() == bytes && std::memcmp(s->irtab_dev_copy.data(), tb.data(), bytes) == 0;
    if (!same) {
      if (!s->irtab_pin) {
        int rc = host_alloc(&s->irtab_pin, (size_t)irtab_bytes(c));
        if (rc != TACHES_OK) return rc;
      }
      if (s->irtab_pending) {   // the pinned copy may still be in flight
        HIPCHK(hipEventSynchronize(s->irtab_ev));
        s->irtab_pending = false;
      }
      std::memcpy(s->irtab_pin, tb.data(), bytes);
      HIPCHK(hipMemcpyAsync(s->irtab_dev, s->irtab_pin, bytes, hipMemcpyHostToDevice, s->stream));
      HIPCHK(hipEventRecord(s->irtab_ev, s->stream));
      s->irtab_pending = true;
      s->irtab_dev_copy.assign(tb.begin(), tb.begin() + bytes);
    }
    g.irs = s->irtab_dev;
  }
  out->next_active = cur;
  out->S = S;
  out->n_out = n_out;
  out->n_blocks = n_blocks;
  return TACHES_OK;
}

void commit_call(taches_stream* s, const CallPlan& p) {
  s->active = p.next_active;
  s->pending = -1;
  s->pending_off = 0;
  s->head = (int)((s->head + p.S) % s->Rcap);
  s->live = (int)(p.n_out - p.S);
  s->blocks_done += p.n_blocks;
}

constexpr int kTimedCalls = 4096;

// Event pair of the next timed call (nullptrs when timing is off).
void timed_events(taches_stream* s, hipEvent_t* e0, hipEvent_t* e1) {
  *e0 = *e1 = nullptr;
  if (!s->timing || s->tev.empty()) return;
  const int k = (int)(s->timed % kTimedCalls);
  *e0 = s->tev[2 * k];
  *e1 = s->tev[2 * k + 1];
}

// Launch one planned call on the stream's own kernels.
int launch_call(taches_stream* s, CallPlan& p) {
  GatherCall& g = p.g;
  hipEvent_t e0, e1;
  timed_events(s, &e0, &e1);
  if (s->cfg.precision == TACHES_PREC_SPLIT_BF16) {
    if (e0) HIPCHK(hipEventRecord(e0, s->stream));
    hipError_t e = taches::launch_toeplitz(g, s->tail_fp64, s->stream);
    if (e != hipSuccess) return fail(TACHES_EDEVICE, "toeplitz launch: %s", hipGetErrorString(e));
    if (e1) {
      HIPCHK(hipEventRecord(e1, s->stream));
      ++s->timed;
    }
    s->last_r = 0;
    s->last_w = 0;
    return TACHES_OK;
  }
  const int B = g.B;
  const bool has_x = g.x != nullptr;
  const int span_blocks = (int)std::min<int64_t>(g.n_blocks, (64 * 16 + g.Lmax_call - 1 + B - 1) / B + 1);
  const int64_t key[4] = {p.S, p.n_out, has_x ? g.Lmax_call : 1, (int64_t)s->force_r * 8 + s->force_w};
  TilePlan plan;
  if (std::equal(key, key + 4, s->plan_key)) {
    plan.r = s->plan_val[0];
    plan.w = s->plan_val[1];
    plan.order = s->plan_val[2];
  } else {
    plan = pick_tile(s, p.S, p.n_out, has_x ? g.Lmax_call : 1, has_x ? span_blocks * g.cpb : 0);
    std::copy(key, key + 4, s->plan_key);
    s->plan_val[0] = plan.r;
    s->plan_val[1] = plan.w;
    s->plan_val[2] = plan.order;
  }
  g.tile_order = plan.order;
  if (e0) HIPCHK(hipEventRecord(e0, s->stream));
  hipError_t e = taches::launch_gather(g, s->tail_fp64, plan.r, plan.w, s->stream);
  if (e != hipSuccess) return fail(TACHES_EDEVICE, "gather launch: %s", hipGetErrorString(e));
  if (e1) {
    HIPCHK(hipEventRecord(e1, s->stream));
    ++s->timed;
  }
  s->last_r = plan.r;
  s->last_w = plan.w;
  return TACHES_OK;
}

int process_common(taches_stream* s, const float* x_dev, float* y_dev, int n_blocks, const int32_t* sched,
                   const int32_t* offs = nullptr) {
  if (s->pool) return fail(TACHES_EBUSY, "stream is attached to a pool; use taches_pool_step");
  CallPlan p;
  int rc = plan_call(s, x_dev, 0, y_dev, 0, n_blocks, sched, offs, &p);
  if (rc != TACHES_OK) return rc;
  rc = launch_call(s, p);
  if (rc != TACHES_OK) return rc;
  commit_call(s, p);
  return TACHES_OK;
}

// ---- work memory of taches_convolve_noalloc ----
// One fixed array per device, set aside when the code object is loaded on
// that device and held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol): the device address comes from hipGetSymbolAddress, once per
// device, and is kept in g_scratch_dev.
constexpr int kMaxDevices = 64;
void* g_scratch_dev[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Zero-padded copy of planar signals: dst[c][i] = src[c][i] for i < ns, 0
// for ns <= i < nd.
__global__ __launch_bounds__(256) void k_pad_copy(const float* __restrict__ src, int64_t ns, float* __restrict__ dst,
                                                  int64_t nd, int channels) {
  const int64_t total = nd * channels;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = t / nd, i = t - c * nd;
    dst[t] = i < ns ? src[c * ns + i] : 0.f;
  }
}

}  // namespace

extern "C" {

void taches_config_default(taches_config* cfg, int32_t block_size, int32_t max_ir_len) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof *cfg);
  cfg->block_size = block_size;
  cfg->max_ir_len = max_ir_len;
  cfg->channels = 1;
  cfg->max_blocks_per_call = 1;
  cfg->precision = TACHES_PREC_FP32;
  cfg->tail = TACHES_TAIL_AUTO;
  cfg->ir_slots = 2;
  cfg->device = 0;
}

const char* taches_last_error(void) { return g_err; }

taches_stream* taches_open_ex(const taches_config* cfg) {
  if (validate(cfg) != TACHES_OK) return nullptr;
  taches_stream* s = new (std::nothrow) taches_stream();
  if (!s) {
    fail(TACHES_ENOMEM, "out of host memory");
    return nullptr;
  }
  s->cfg = *cfg;
  if (stream_init(s) != TACHES_OK) {
    ErrKeep keep;
    free_stream(s);
    return nullptr;
  }
  return s;
}

taches_stream* taches_open(int32_t block_size, int32_t max_ir_len) {
  taches_config c;
  taches_config_default(&c, block_size, max_ir_len);
  return taches_open_ex(&c);
}

int taches_close(taches_stream* s) {
  if (!s) return TACHES_OK;
  if (s->pool) return fail(TACHES_EBUSY, "stream is attached to a pool");
  free_stream(s);
  return TACHES_OK;
}

int taches_set_hip_stream(taches_stream* s, void* hip_stream) {
  if (!s) return fail(TACHES_EINVAL, "stream is NULL");
  if (s->pool) return fail(TACHES_EBUSY, "stream is attached to a pool; it runs on the pool's HIP stream");
  hipStream_t next = (hipStream_t)hip_stream;  // NULL: HIP's null stream
  if (next != s->stream) {
    HIPCHK(hipStreamSynchronize(s->stream));
    s->stream = next;
  }
  return TACHES_OK;
}

int taches_synchronize(taches_stream* s) {
  if (!s) return fail(TACHES_EINVAL, "stream is NULL");
  HIPCHK(hipStreamSynchronize(s->stream));
  return TACHES_OK;
}

static int set_ir_common(taches_stream* s, const float* h, int32_t L, bool on_device, int32_t offset = 0) {
  if (!s) return fail(TACHES_EINVAL, "stream is NULL");
  if (!h) return fail(TACHES_EINVAL, "h is NULL");
  if (L < 1 || L > s->cfg.max_ir_len) return fail(TACHES_EINVAL, "L=%d outside [1, %d]", L, s->cfg.max_ir_len);
  if (offset < 0 || offset >= s->cfg.block_size)
    return fail(TACHES_EINVAL, "offset %d outside [0, %d)", offset, s->cfg.block_size);
  if (offset > 0 && is_split(s->cfg))
    return fail(TACHES_EINVAL, "an IR taking over inside a block needs FP32 precision");
  int slot = s->pending;
  if (slot < 0) {
    for (int k = 0; k < (int)s->slots.size(); ++k)
      if (k != s->active) {
        slot = k;
        break;
      }
  }
  int rc = load_slot(s, slot, h, L, on_device);
  if (rc != TACHES_OK) return rc;
  s->pending = slot;
  s->pending_off = offset;
  return TACHES_OK;
}

int taches_set_ir(taches_stream* s, const float* h, int32_t L) { return set_ir_common(s, h, L, false); }

int taches_set_ir_ref(taches_stream* s, const float* h_dev, int32_t L, int32_t offset) {
  if (!s) return fail(TACHES_EINVAL, "stream is NULL");
  if (!h_dev) return fail(TACHES_EINVAL, "h is NULL");
  if (is_split(s->cfg)) return fail(TACHES_EINVAL, "an IR read in place needs FP32 precision");
  if (L < 1 || L > s->cfg.max_ir_len) return fail(TACHES_EINVAL, "L=%d outside [1, %d]", L, s->cfg.max_ir_len);
  if (offset < 0 || offset >= s->cfg.block_size)
    return fail(TACHES_EINVAL, "offset %d outside [0, %d)", offset, s->cfg.block_size);
  // the same slot choice as a copy; only the pointer changes on the host,
  // so calls already planned keep reading what they were planned with
  int slot = s->pending;
  if (slot < 0) {
    for (int k = 0; k < (int)s->slots.size(); ++k)
      if (k != s->active) {
        slot = k;
        break;
      }
  }
  IrSlot& sl = s->slots[slot];
  sl.ref = h_dev;
  sl.L = L;
  s->pending = slot;
  s->pending_off = offset;
  return TACHES_OK;
}

int taches_set_ir_at(taches_stream* s, const float* h, int32_t L, int32_t offset, int32_t h_on_device) {
  return set_ir_common(s, h, L, h_on_device != 0, offset);
}

int taches_set_ir_device(taches_stream* s, const float* h_dev, int32_t L) { return set_ir_common(s, h_dev, L, true); }

int taches_load_ir_slot(taches_stream* s, int32_t slot, const float* h, int32_t L, int32_t h_on_device) {
  if (!s) return fail(TACHES_EINVAL, "stream is NULL");
  if (slot < 0 || slot >= (int)s->slots.size()) return fail(TACHES_EINVAL, "slot %d outside [0, %zu)", slot, s->slots.size());
  if (!h) return fail(TACHES_EINVAL, "h is NULL");
  if (L < 1 || L > s->cfg.max_ir_len) return fail(TACHES_EINVAL, "L=%d outside [1, %d]", L, s->cfg.max_ir_len);
  if (slot == s->pending) {
    s->pending = -1;
    s->pending_off = 0;
  }
  return load_slot(s, slot, h, L, h_on_device != 0);
}

int taches_process(taches_stream* s, const float* x, float* y) {
  if (!s) return fail(TACHES_EINVAL, "stream is NULL");
  if (!x || !y) return fail(TACHES_EINVAL, "x or y is NULL");
  const size_t n = (size_t)s->cfg.channels * s->cfg.block_size;
  if (!s->x_pin) {
    int rc = host_alloc(&s->x_pin, n * 4);
    if (rc == TACHES_OK) rc = host_alloc(&s->y_pin, n * 4);
    if (rc != TACHES_OK) return rc;
  }
  std::memcpy(s->x_pin, x, n * 4);
  HIPCHK(hipMemcpyAsync(s->x_dev, s->x_pin, n * 4, hipMemcpyHostToDevice, s->stream));
  int rc = process_common(s, s->x_dev, s->y_dev, 1, nullptr);
  if (rc != TACHES_OK) {
    (void)hipStreamSynchronize(s->stream);
    return rc;
  }
  HIPCHK(hipMemcpyAsync(s->y_pin, s->y_dev, n * 4, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  std::memcpy(y, s->y_pin, n * 4);
  return TACHES_OK;
}

int taches_process_async(taches_stream* s, const float* x_dev, float* y_dev) {
  if (!s) return fail(TACHES_EINVAL, "stream is NULL");
  if (!x_dev) return fail(TACHES_EINVAL, "x is NULL");
  return process_common(s, x_dev, y_dev, 1, nullptr);
}

int taches_process_blocks(taches_stream* s, const float* x_dev, float* y_dev, int32_t n_blocks,
                          const int32_t* ir_slot_of_block) {
  if (!s) return fail(TACHES_EINVAL, "stream is NULL");
  return process_common(s, x_dev, y_dev, n_blocks, ir_slot_of_block);
}

int taches_convolve(const float* x_dev, int64_t nx, int32_t channels, const float* h_dev, int32_t nh, float* y_dev,
                    int32_t precision, int32_t role_swap, int32_t device, void* hip_stream) {
  if (!x_dev || !h_dev || !y_dev) return fail(TACHES_EINVAL, "NULL buffer");
  if (nx < 1 || nh < 1 || channels < 1) return fail(TACHES_EINVAL, "nx, nh and channels must be >= 1");
  // exchanging the roles (Section 3.2, Fig. 6) needs one channel: with C
  // channels sharing h, x would become C different IRs
  const bool swap = role_swap != 0 && channels == 1 && (int64_t)nh > nx;
  const float* sig = swap ? h_dev : x_dev;
  const float* ir = swap ? x_dev : h_dev;
  const int64_t ns = swap ? nh : nx;
  const int64_t L = swap ? nx : nh;
  const int64_t n_out = nx + nh - 1;
  const int B = 256;
  // the input blocks in one call, then the temporal overflow drained with
  // zero input in a second (no input samples to walk)
  const int64_t n_in = (ns + B - 1) / B;
  const int64_t n_drain = (n_out - n_in * B + B - 1) / B;   // may be <= 0
  const int64_t nblk = n_in + std::max<int64_t>(n_drain, 0);
  if (nblk > INT32_MAX || L > INT32_MAX) return fail(TACHES_EINVAL, "signal too long");
  taches_config cfg;
  taches_config_default(&cfg, B, (int32_t)L);
  cfg.channels = channels;
  cfg.max_blocks_per_call = (int32_t)std::max<int64_t>(n_in, n_drain);
  cfg.precision = precision;
  cfg.device = device;
  if (validate(&cfg) != TACHES_OK) return TACHES_EINVAL;
  taches_stream* s = taches_open_ex(&cfg);
  if (!s) return TACHES_ENOMEM;
  int rc = taches_set_hip_stream(s, hip_stream);
  float *xp = nullptr, *yp = nullptr;
  const size_t xrow = (size_t)n_in * B * 4, yrow = (size_t)nblk * B * 4;
  if (rc == TACHES_OK) rc = set_ir_common(s, ir, (int32_t)L, true);
  if (rc == TACHES_OK && hipMalloc((void**)&xp, xrow * channels) != hipSuccess) rc = fail(TACHES_ENOMEM, "input buffer");
  if (rc == TACHES_OK && hipMalloc((void**)&yp, yrow * channels) != hipSuccess) rc = fail(TACHES_ENOMEM, "output buffer");
  if (rc == TACHES_OK) {
    // zero-padded input [C][n_in*B]; the output is cut back to nx + nh - 1
    hipError_t e = hipMemsetAsync(xp, 0, xrow * channels, s->stream);
    if (e == hipSuccess)
      e = hipMemcpy2DAsync(xp, xrow, sig, (size_t)ns * 4, (size_t)ns * 4, channels, hipMemcpyDeviceToDevice, s->stream);
    if (e != hipSuccess) rc = fail(TACHES_EDEVICE, "input copy: %s", hipGetErrorString(e));
  }
  // the input call writes [C][n_in*B] into a packed buffer, the drain its
  // [C][n_drain*B]; both are then copied out channel by channel
  float* yd = yp + (size_t)channels * n_in * B;
  if (rc == TACHES_OK) rc = process_common(s, xp, yp, (int)n_in, nullptr);
  if (rc == TACHES_OK && n_drain > 0) rc = process_common(s, nullptr, yd, (int)n_drain, nullptr);
  if (rc == TACHES_OK) {
    const int64_t first = std::min<int64_t>(n_in * B, n_out);
    hipError_t e = hipMemcpy2DAsync(y_dev, (size_t)n_out * 4, yp, xrow, (size_t)first * 4, channels,
                                    hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess && n_out > first)
      e = hipMemcpy2DAsync(y_dev + first, (size_t)n_out * 4, yd, (size_t)n_drain * B * 4, (size_t)(n_out - first) * 4,
                           channels, hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) rc = fail(TACHES_EDEVICE, "output copy: %s", hipGetErrorString(e));
  }
  (void)hipStreamSynchronize(s->stream);
  (void)hipFree(xp);
  (void)hipFree(yp);
  {
    ErrKeep keep;
    (void)taches_close(s);
  }
  return rc;
}

int taches_convolve_noalloc(const float* x_dev, int64_t nx, int32_t channels, const float* h_dev, int32_t nh,
                            float* y_dev, int32_t role_swap, int32_t device, void* hip_stream) {
  if (!x_dev || !h_dev || !y_dev) return fail(TACHES_EINVAL, "NULL buffer");
  if (nx < 1 || nh < 1 || channels < 1) return fail(TACHES_EINVAL, "nx, nh and channels must be >= 1");
  if (device < 0 || device >= kMaxDevices) return fail(TACHES_EINVAL, "device %d outside [0, %d)", device, kMaxDevices);
  // the same operands, block size, chunks and tail type as taches_convolve,
  // so both give the same bits
  const bool swap = role_swap != 0 && channels == 1 && (int64_t)nh > nx;
  const float* sig = swap ? h_dev : x_dev;
  const float* ir = swap ? x_dev : h_dev;
  const int64_t ns = swap ? nh : nx;
  const int64_t L = swap ? nx : nh;
  const int64_t n_out = nx + nh - 1;
  const int B = 256;
  const int64_t n_in = (ns + B - 1) / B;
  const int64_t S_in = n_in * B;
  if (S_in + L >= ((int64_t)1 << 30)) return fail(TACHES_EINVAL, "signal too long");
  taches_config cfg;
  taches_config_default(&cfg, B, (int32_t)L);
  const bool fp64 = want_fp64(cfg);
  // work memory: the zero-padded input [C][S_in] (FP32) and a tail of
  // [C][n_out] slots that the kernel clears as it emits (every output of the
  // single call is emitted, none is kept)
  const size_t x_bytes = (size_t)round_up((int64_t)channels * S_in * 4, 256);
  const size_t need = x_bytes + (size_t)channels * (size_t)n_out * (fp64 ? 8 : 4);
  if ((int64_t)channels * n_out > ((int64_t)1 << 32) || need > kNoallocScratchBytes)
    return fail(TACHES_EINVAL, "needs %zu bytes of work memory, the limit is %zu", need, kNoallocScratchBytes);
  int prev = -1;
  HIPCHK(hipGetDevice(&prev));
  if (prev != device) HIPCHK(hipSetDevice(device));
  int rc = TACHES_OK;
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        rc = fail(TACHES_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      else
        g_scratch_dev[device] = ptr;
    }
    base = static_cast<unsigned char*>(g_scratch_dev[device]);
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  float* xp = reinterpret_cast<float*>(base);
  if (rc == TACHES_OK) {
    const int64_t total = (int64_t)channels * S_in;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_pad_copy, dim3(blocks), dim3(256), 0, st, sig, ns, xp, S_in, channels);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) rc = fail(TACHES_EDEVICE, "input copy: %s", hipGetErrorString(e));
  }
  if (rc == TACHES_OK) {
    GatherCall g{};
    g.x = xp;
    g.y = y_dev;
    g.ring = base + x_bytes;
    g.irs = nullptr;
    g.ir0.h = ir;
    g.ir0.L = (int32_t)L;
    g.x_cstride = S_in;
    g.y_cstride = n_out;
    g.ring_cstride = n_out;
    g.S = (int32_t)n_out;          // every output is emitted by this call
    g.B = B;
    g.n_blocks = (int32_t)n_in;
    g.cpb = (B + taches::CHUNK_MAX - 1) / taches::CHUNK_MAX;
    g.Rcap = (int32_t)n_out;
    g.head = 0;
    g.live_in = 0;
    g.n_out = (int32_t)n_out;
    g.Lmax_call = (int32_t)L;
    g.channels = channels;
    g.cpad = channels;
    const int span_blocks = (int)std::min<int64_t>(n_in, (64 * 16 + L - 1 + B - 1) / B + 1);
    const TilePlan plan = plan_tile(0, channels, S_in, n_out, L, span_blocks * g.cpb);
    g.tile_order = plan.order;
    const hipError_t e = taches::launch_gather(g, fp64, plan.r, plan.w, st);
    if (e != hipSuccess) rc = fail(TACHES_EDEVICE, "gather launch: %s", hipGetErrorString(e));
  }
  if (prev != device) {
    ErrKeep keep;
    (void)hipSetDevice(prev);
  }
  return rc;
}

int taches_process_blocks_at(taches_stream* s, const float* x_dev, float* y_dev, int32_t n_blocks,
                             const int32_t* ir_slot_of_block, const int32_t* offset_of_block) {
  if (!s) return fail(TACHES_EINVAL, "stream is NULL");
  if (offset_of_block && !ir_slot_of_block) return fail(TACHES_EINVAL, "offsets given without a schedule");
  return process_common(s, x_dev, y_dev, n_blocks, ir_slot_of_block, offset_of_block);
}

int taches_set_timing(taches_stream* s, int32_t on) {
  if (!s) return fail(TACHES_EINVAL, "stream is NULL");
  if (on && s->tev.empty()) {
    HIPCHK(hipSetDevice(s->cfg.device));
    s->tev.assign(2 * kTimedCalls, nullptr);
    for (hipEvent_t& ev : s->tev) {
      hipError_t e = hipEventCreate(&ev);
      if (e != hipSuccess) return fail(TACHES_EDEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    }
  }
  s->timing = on != 0;
  return TACHES_OK;
}

int taches_call_times(taches_stream* s, double* ms_out, int32_t n) {
  if (!s || (!ms_out && n > 0)) return fail(TACHES_EINVAL, "NULL argument");
  if (n < 0) return fail(TACHES_EINVAL, "n = %d", n);
  const int64_t have = std::min<int64_t>(s->timed, kTimedCalls);
  const int64_t m = std::min<int64_t>(have, n);
  for (int64_t i = 0; i < m; ++i) {
    const int k = (int)((s->timed - m + i) % kTimedCalls);
    HIPCHK(hipEventSynchronize(s->tev[2 * k + 1]));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, s->tev[2 * k], s->tev[2 * k + 1]));
    ms_out[i] = ms;
  }
  s->timed = 0;
  return (int)m;
}

int taches_get_info(const taches_stream* s, taches_info* out) {
  if (!s || !out) return fail(TACHES_EINVAL, "NULL argument");
  std::memset(out, 0, sizeof *out);
  out->block_size = s->cfg.block_size;
  out->max_ir_len = s->cfg.max_ir_len;
  out->channels = s->cfg.channels;
  out->max_blocks_per_call = s->cfg.max_blocks_per_call;
  out->precision = s->cfg.precision;
  out->tail_fp64 = s->tail_fp64 ? 1 : 0;
  out->ring_slots = s->Rcap;
  out->head = s->head;
  out->live = s->live;
  out->active_len = s->active >= 0 ? s->slots[s->active].L : 0;
  out->blocks_done = s->blocks_done;
  out->device_bytes = s->device_bytes;
  out->tile_r = s->last_r;
  out->tile_w = s->last_w;
  return TACHES_OK;
}

int64_t taches_bytes_for(const taches_config* cfg) {
  if (validate(cfg) != TACHES_OK) return -1;
  const int64_t esz = want_fp64(*cfg) ? 8 : 4;
  int64_t b = ring_channels(*cfg) * ring_slots_for(*cfg) * esz;
  b += 2 * xs_bytes(*cfg);
  b += (int64_t)cfg->ir_slots * cfg->max_ir_len * (cfg->precision == TACHES_PREC_SPLIT_BF16 ? 8 : 4);
  b += 2 * (int64_t)cfg->channels * cfg->block_size * 4;
  b += irtab_bytes(*cfg);
  return b;
}

int taches_tail_is_fp64(const taches_config* cfg) {
  if (!cfg) return fail(TACHES_EINVAL, "config is NULL");
  if (validate(cfg) != TACHES_OK) return TACHES_EINVAL;
  return want_fp64(*cfg) ? 1 : 0;
}

int taches_read_tail(taches_stream* s, int32_t channel, double* out, int32_t n) {
  if (!s || !out) return fail(TACHES_EINVAL, "NULL argument");
  if (channel < 0 || channel >= s->cfg.channels) return fail(TACHES_EINVAL, "channel %d out of range", channel);
  if (n < 0 || n > s->Rcap) return fail(TACHES_EINVAL, "n=%d outside [0, %d]", n, s->Rcap);
  HIPCHK(hipStreamSynchronize(s->stream));
  const size_t esz = s->tail_fp64 ? 8 : 4;
  const unsigned char* base = (const unsigned char*)s->ring;
  std::vector<unsigned char> buf((size_t)n * esz);
  if (is_split(s->cfg)) {
    // [slot][cpad]: strided copy of one channel column
    for (int k = 0; k < n;) {
      const int slot = (s->head + k) % s->Rcap;
      const int run = std::min(n - k, s->Rcap - slot);
      HIPCHK(hipMemcpy2D(buf.data() + (size_t)k * esz, esz, base + ((size_t)slot * s->cpad + channel) * esz,
                         (size_t)s->cpad * esz, esz, run, hipMemcpyDeviceToHost));
      k += run;
    }
  } else {
    const int first = std::min(n, s->Rcap - s->head);
    const int64_t coff = (int64_t)channel * s->Rcap;
    if (first > 0)
      HIPCHK(hipMemcpy(buf.data(), base + (coff + s->head) * esz, (size_t)first * esz, hipMemcpyDeviceToHost));
    if (n > first)
      HIPCHK(hipMemcpy(buf.data() + (size_t)first * esz, base + coff * esz, (size_t)(n - first) * esz,
                       hipMemcpyDeviceToHost));
  }
  for (int k = 0; k < n; ++k) {
    if (k >= s->live) {   // no pending sums past `live` (the slots may hold stale values)
      out[k] = 0.0;
    } else if (s->tail_fp64) {
      double v;
      std::memcpy(&v, buf.data() + (size_t)k * 8, 8);
      out[k] = v;
    } else {
      float v;
      std::memcpy(&v, buf.data() + (size_t)k * 4, 4);
      out[k] = v;
    }
  }
  return TACHES_OK;
}

int taches_reset(taches_stream* s) {
  if (!s) return fail(TACHES_EINVAL, "stream is NULL");
  // The ring is not cleared: with live = 0 no kernel reads a slot before
  // writing it (slots past `live` count as zero, and emitted slots are
  // cleared as they are read), and taches_read_tail reports zeros there.
  for (auto& sl : s->slots) {
    sl.L = 0;
    sl.ref = nullptr;
  }
  s->active = s->pending = -1;
  s->head = s->live = 0;
  s->blocks_done = 0;
  return TACHES_OK;
}

int taches_set_tile(taches_stream* s, int32_t r, int32_t w) {
  if (!s) return fail(TACHES_EINVAL, "stream is NULL");
  if (r == 0 && w == 0) {
    s->force_r = s->force_w = 0;
    return TACHES_OK;
  }
  if ((r != 4 && r != 8 && r != 12 && r != 14 && r != 16) || (w != 1 && w != 2 && w != 4))
    return fail(TACHES_EINVAL, "tile (%d, %d) not in {4,8,12,14,16} x {1,2,4}", r, w);
  s->force_r = r;
  s->force_w = w;
  return TACHES_OK;
}

}  // extern "C"

// ===========================================================================
// Pools: many streams advanced by one batched launch.
// ===========================================================================

using taches::WorkItem;

// One unit of a batched step's plan: a work item and its estimated work.
struct PoolItem {
  WorkItem w;
  int64_t work;
};

struct taches_pool {
  int max_streams = 0;
  int64_t budget = 0, used = 0;
  int device = 0;
  std::vector<taches_stream*> attached;
  hipStream_t own = nullptr, stream = nullptr, capture = nullptr;
  // one packed table: [header][calls][fp64 flags][items][counter], pinned and device.
  // Two pinned buffers are used in turn, so the host can build a step's
  // table while the previous step (and its copy) is still queued.
  unsigned char* tab_pin[2] = {nullptr, nullptr};
  unsigned char* tab_dev[2] = {nullptr, nullptr};   // device copies, used in turn like the pinned ones
  // stream of the table copies (nullptr: the pool's stream); the pool's
  // stream waits for each copy through tab_copied
  hipStream_t copy = nullptr;
  hipEvent_t tab_copied = nullptr;
  size_t tab_cap = 0;
  hipEvent_t tab_free[2] = {nullptr, nullptr};
  bool tab_pending[2] = {false, false};
  int tab_cur = 0;
  hipEvent_t detach_ev = nullptr, attach_ev = nullptr;
  int force_r = 0;
  bool use_graph = false;
  // captured [table copy -> batched kernel], one per (tile r, FP64 tails
  // present, launched workgroups rounded up to 256 * 2^k): steps of similar
  // shape replay the same graph
  struct Graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t copy_node = nullptr;
    int nwg = 0;
    size_t cap = 0;
  };
  static constexpr int kGraphs = 4 * 2 * 8 * 2 * 2;   // ... x table buffer x copy inside or outside
  Graph graphs[kGraphs];
  int64_t captures = 0;
  int64_t replays = 0;
  int last_items = 0, last_wg = 0, last_r = 0;
  double last_plan_ms = 0.0;
  // estimate of the last step's busiest workgroup over the mean; with few
  // items per workgroup it is played out on request (taches_pool_get_info),
  // off the step's path
  mutable double last_imbalance = 0.0;
  mutable bool imbalance_pending = false;
  int64_t last_total_work = 0;
  uint64_t steps = 0;                             // step counter (duplicate detection)
  // device time of the batched launches: a ring of event pairs; completed
  // launches are added to dev_ms_total when they are found complete
  static constexpr int kRing = 8;
  hipEvent_t ev_beg[kRing] = {}, ev_end[kRing] = {};
  mutable bool ev_pending[kRing] = {};
  mutable double dev_ms_total = 0.0;
  int ev_next = 0, ev_last = -1;
  // per-step planning buffers, kept from step to step so that a step
  // allocates no host memory once the pool has seen its largest step
  std::vector<CallPlan> plans;
  std::vector<int> gather_ids, split_ids[4];
  std::vector<const GatherCall*> gcalls;
  std::vector<char> enqueued;
  std::vector<PoolItem> items;
  std::vector<uint32_t> order;
  std::vector<uint16_t> keys;
  mutable std::vector<int64_t> heap;
};

namespace {

void drop_graph(taches_pool::Graph& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g = taches_pool::Graph{};
}

void pool_drop_graph(taches_pool* p) {
  for (taches_pool::Graph& g : p->graphs) drop_graph(g);
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Indices of `items` in decreasing work, to within 1/8: one counting pass
// on a key made of the work's binary exponent and the three bits after its
// leading one (works in the same eighth of an octave share a bucket and
// keep their list order).  Largest-first dealing by the work queue needs no
// finer order.
template <typename ItemT, typename WorkOf>
void order_by_work_desc(const std::vector<ItemT>& items, std::vector<uint32_t>& order, std::vector<uint16_t>& keys,
                        WorkOf work_of) {
  constexpr int kKeys = 64 * 8;
  const size_t n = items.size();
  keys.resize(n);
  order.resize(n);
  uint32_t cnt[kKeys + 1] = {};
  for (size_t i = 0; i < n; ++i) {
    const uint64_t w = (uint64_t)std::max<int64_t>(1, work_of(items[i]));
    const int e = 63 - __builtin_clzll(w);
    const int m = (int)((e >= 3 ? (w >> (e - 3)) : (w << (3 - e))) & 7);
    const int key = (63 - e) * 8 + (7 - m);   // ascending key = descending work
    keys[i] = (uint16_t)key;
    cnt[key + 1] += 1;
  }
  for (int k = 0; k < kKeys; ++k) cnt[k + 1] += cnt[k];
  for (size_t i = 0; i < n; ++i) order[cnt[keys[i]]++] = (uint32_t)i;
}

// Add the device time of every completed launch of the ring to the total
// (wait: block until each pending launch has completed).
int pool_account(const taches_pool* p, bool wait) {
  for (int k = 0; k < taches_pool::kRing; ++k) {
    if (!p->ev_pending[k]) continue;
    if (wait) HIPCHK(hipEventSynchronize(p->ev_end[k]));
    else if (hipEventQuery(p->ev_end[k]) != hipSuccess) continue;
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, p->ev_beg[k], p->ev_end[k]));
    p->dev_ms_total += ms;
    p->ev_pending[k] = false;
  }
  return TACHES_OK;
}

int pool_reserve(taches_pool* p, size_t bytes) {
  if (bytes <= p->tab_cap) return TACHES_OK;
  for (int k = 0; k < 2; ++k)
    if (p->tab_pending[k]) {
      HIPCHK(hipEventSynchronize(p->tab_free[k]));
      p->tab_pending[k] = false;
    }
  HIPCHK(hipStreamSynchronize(p->stream));
  pool_drop_graph(p);
  for (int k = 0; k < 2; ++k) {
    (void)hipHostFree(p->tab_pin[k]);
    p->tab_pin[k] = nullptr;
  }
  for (int k = 0; k < 2; ++k) {
    (void)hipFree(p->tab_dev[k]);
    p->tab_dev[k] = nullptr;
  }
  p->tab_cap = 0;
  // grow by 2x, at least 4 MB: a reallocation waits for the pool's stream
  // and drops the captured graphs, so a growing load should meet few of them
  const size_t cap = align256(std::max<size_t>(2 * bytes, size_t(4) << 20));
  for (int k = 0; k < 2; ++k) {
    hipError_t e = hipHostMalloc((void**)&p->tab_pin[k], cap, hipHostMallocDefault);
    if (e != hipSuccess) return fail(TACHES_ENOMEM, "pool table (host): %s", hipGetErrorString(e));
  }
  for (int k = 0; k < 2; ++k) {
    hipError_t e = hipMalloc((void**)&p->tab_dev[k], cap);
    if (e != hipSuccess) return fail(TACHES_ENOMEM, "pool table (device): %s", hipGetErrorString(e));
  }
  p->tab_cap = cap;
  return TACHES_OK;
}

// Tile shape of a batched launch: the same per-lane tile for every stream.
// Longer tiles need fewer LDS reads per FMA and pay each tile's fixed costs
// (descriptor, tail read and write) over more outputs.  The largest one is
// taken that leaves about four items per resident workgroup, or at least
// one when every tile is light (at most 4096 input samples reach a tile of
// 1024 outputs: a few microseconds of one wave, so the work queue balances
// the step whatever their number, as in serving steps); smaller tiles
// otherwise keep steps of heavy tiles balanced.
int pool_pick_r(const taches_pool* p, const std::vector<const GatherCall*>& calls, bool mixed) {
  if (p->force_r) return p->force_r;
  static const int rs[4] = {16, 12, 8, 4};
  constexpr int64_t kLightTile = 1024LL * 4096;   // multiply-adds
  for (int r : rs) {
    const int64_t T = 64 * r;
    const int64_t wg = 256LL * taches::gather_batched_waves_per_cu(r, mixed);
    int64_t items = 0, heaviest = 0;
    for (const GatherCall* g : calls) {
      items += (int64_t)g->channels * ((g->n_out + T - 1) / T);
      if (g->x) heaviest = std::max(heaviest, T * std::min<int64_t>(g->S, T + g->Lmax_call - 1));
    }
    if (items >= 4 * wg || (items >= wg && heaviest <= kLightTile)) return r;
  }
  return 4;
}

}  // namespace

extern "C" {

taches_pool* taches_pool_create(int32_t max_streams, int64_t hbm_budget_bytes, int32_t device) {
  if (max_streams < 1 || max_streams > (1 << 20) || hbm_budget_bytes < 0) {
    fail(TACHES_EINVAL, "max_streams must be in [1, 2^20] and the budget >= 0");
    return nullptr;
  }
  taches_pool* p = new (std::nothrow) taches_pool();
  if (!p) {
    fail(TACHES_ENOMEM, "out of host memory");
    return nullptr;
  }
  p->max_streams = max_streams;
  p->budget = hbm_budget_bytes;
  p->device = device;
  bool ok = hipSetDevice(device) == hipSuccess && hipStreamCreateWithFlags(&p->own, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&p->tab_free[0], hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&p->tab_free[1], hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&p->detach_ev, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&p->attach_ev, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&p->tab_copied, hipEventDisableTiming) == hipSuccess;
  for (int k = 0; ok && k < taches_pool::kRing; ++k)
    ok = hipEventCreate(&p->ev_beg[k]) == hipSuccess && hipEventCreate(&p->ev_end[k]) == hipSuccess;
  if (!ok) {
    fail(TACHES_EDEVICE, "pool stream/event creation failed");
    if (p->own) (void)hipStreamDestroy(p->own);
    if (p->capture) (void)hipStreamDestroy(p->capture);
    for (hipEvent_t ev : {p->tab_free[0], p->tab_free[1], p->detach_ev, p->attach_ev, p->tab_copied})
      if (ev) (void)hipEventDestroy(ev);
    for (int k = 0; k < taches_pool::kRing; ++k) {
      if (p->ev_beg[k]) (void)hipEventDestroy(p->ev_beg[k]);
      if (p->ev_end[k]) (void)hipEventDestroy(p->ev_end[k]);
    }
    delete p;
    return nullptr;
  }
  p->stream = p->own;
  return p;
}

int taches_pool_destroy(taches_pool* p) {
  if (!p) return TACHES_OK;
  if (!p->attached.empty()) return fail(TACHES_EBUSY, "pool still has %zu attached streams", p->attached.size());
  (void)hipStreamSynchronize(p->stream);
  pool_drop_graph(p);
  for (int k = 0; k < 2; ++k) (void)hipHostFree(p->tab_pin[k]);
  for (int k = 0; k < 2; ++k) (void)hipFree(p->tab_dev[k]);
  for (hipEvent_t ev : {p->tab_free[0], p->tab_free[1], p->detach_ev, p->attach_ev, p->tab_copied})
    if (ev) (void)hipEventDestroy(ev);
  for (int k = 0; k < taches_pool::kRing; ++k) {
    (void)hipEventDestroy(p->ev_beg[k]);
    (void)hipEventDestroy(p->ev_end[k]);
  }
  (void)hipStreamDestroy(p->own);
  (void)hipStreamDestroy(p->capture);
  delete p;
  return TACHES_OK;
}

int taches_pool_set_hip_stream(taches_pool* p, void* hip_stream) {
  if (!p) return fail(TACHES_EINVAL, "pool is NULL");
  hipStream_t next = (hipStream_t)hip_stream;
  if (next != p->stream) {
    HIPCHK(hipStreamSynchronize(p->stream));
    p->stream = next;
    for (taches_stream* s : p->attached) s->stream = next;
  }
  return TACHES_OK;
}

int taches_pool_set_copy_stream(taches_pool* p, void* hip_stream) {
  if (!p) return fail(TACHES_EINVAL, "pool is NULL");
  hipStream_t next = (hipStream_t)hip_stream;
  if (next != p->copy) {
    if (p->copy) HIPCHK(hipStreamSynchronize(p->copy));
    p->copy = next;
  }
  return TACHES_OK;
}

int taches_pool_attach(taches_pool* p, taches_stream* s) {
  if (!p || !s) return fail(TACHES_EINVAL, "NULL argument");
  if (s->pool) return fail(TACHES_EBUSY, "stream already attached to a pool");
  if ((int)p->attached.size() >= p->max_streams) return fail(TACHES_EBUSY, "pool has no free slot (%d streams)", p->max_streams);
  if (s->cfg.device != p->device) return fail(TACHES_EINVAL, "stream and pool are on different devices");
  if (p->used + s->device_bytes > p->budget)
    return fail(TACHES_ENOMEM, "HBM budget: %lld + %lld bytes exceed %lld", (long long)p->used, (long long)s->device_bytes,
                (long long)p->budget);
  if (s->stream != p->stream) {
    // the pool's later work waits for what is queued on the stream's HIP
    // stream (initialisation, reset, IR copies); the host does not wait
    HIPCHK(hipEventRecord(p->attach_ev, s->stream));
    HIPCHK(hipStreamWaitEvent(p->stream, p->attach_ev, 0));
  }
  s->stream_before_pool = s->stream;
  s->stream = p->stream;
  s->pool = p;
  p->used += s->device_bytes;
  p->attached.push_back(s);
  return TACHES_OK;
}

int taches_pool_detach(taches_pool* p, taches_stream* s) {
  if (!p || !s) return fail(TACHES_EINVAL, "NULL argument");
  if (s->pool != p) return fail(TACHES_EINVAL, "stream is not attached to this pool");
  // later work on the stream's own HIP stream waits for the pool's queued
  // steps (which may still use the stream's tail and IR slots)
  HIPCHK(hipEventRecord(p->detach_ev, p->stream));
  HIPCHK(hipStreamWaitEvent(s->stream_before_pool, p->detach_ev, 0));
  p->attached.erase(std::find(p->attached.begin(), p->attached.end(), s));
  p->used -= s->device_bytes;
  s->pool = nullptr;
  s->stream = s->stream_before_pool;
  return TACHES_OK;
}

int taches_pool_set_tile(taches_pool* p, int32_t r) {
  if (!p) return fail(TACHES_EINVAL, "pool is NULL");
  if (r != 0 && r != 4 && r != 8 && r != 12 && r != 16) return fail(TACHES_EINVAL, "r=%d not in {0,4,8,12,16}", r);
  p->force_r = r;
  return TACHES_OK;
}

int taches_pool_use_graph(taches_pool* p, int32_t on) {
  if (!p) return fail(TACHES_EINVAL, "pool is NULL");
  p->use_graph = on != 0;
  return TACHES_OK;
}

int taches_pool_synchronize(taches_pool* p) {
  if (!p) return fail(TACHES_EINVAL, "pool is NULL");
  HIPCHK(hipStreamSynchronize(p->stream));
  return TACHES_OK;
}

int taches_pool_get_info(const taches_pool* p, taches_pool_info* out) {
  if (!p || !out) return fail(TACHES_EINVAL, "NULL argument");
  std::memset(out, 0, sizeof *out);
  out->attached = (int32_t)p->attached.size();
  out->max_streams = p->max_streams;
  out->budget_bytes = p->budget;
  out->used_bytes = p->used;
  out->last_items = p->last_items;
  out->last_workgroups = p->last_wg;
  out->last_r = p->last_r;
  out->graph_replays = p->replays;
  out->graph_captures = p->captures;
  out->last_plan_ms = p->last_plan_ms;
  if (p->imbalance_pending) {
    // the last step's list played out on the estimated works: each item
    // goes to the least loaded workgroup (a min-heap of workgroup loads)
    std::vector<int64_t>& heap = p->heap;
    heap.assign(std::max(1, p->last_wg), 0);
    for (uint32_t i : p->order) {
      heap[0] += p->items[i].work;
      size_t j = 0;
      for (;;) {
        const size_t l = 2 * j + 1, r = l + 1;
        size_t m = j;
        if (l < heap.size() && heap[l] < heap[m]) m = l;
        if (r < heap.size() && heap[r] < heap[m]) m = r;
        if (m == j) break;
        std::swap(heap[j], heap[m]);
        j = m;
      }
    }
    const double mean = (double)p->last_total_work / (double)heap.size();
    const int64_t mx = *std::max_element(heap.begin(), heap.end());
    p->last_imbalance = mean > 0 ? (double)mx / mean : 1.0;
    p->imbalance_pending = false;
  }
  out->last_imbalance = p->last_imbalance;
  out->last_device_ms = -1.0;
  float ms = 0.f;
  if (p->ev_last >= 0 && hipEventQuery(p->ev_end[p->ev_last]) == hipSuccess &&
      hipEventElapsedTime(&ms, p->ev_beg[p->ev_last], p->ev_end[p->ev_last]) == hipSuccess)
    out->last_device_ms = ms;
  int rc = pool_account(p, false);
  if (rc != TACHES_OK) return rc;
  out->device_ms_total = p->dev_ms_total;
  return TACHES_OK;
}

int taches_fp32_fma_ceiling(int32_t device, double* tflops_out) {
  if (!tflops_out) return fail(TACHES_EINVAL, "NULL argument");
  hipError_t e = taches::measure_fmac_ceiling(device, tflops_out);
  if (e != hipSuccess) return fail(TACHES_EDEVICE, "fma ceiling: %s", hipGetErrorString(e));
  return TACHES_OK;
}

int taches_pool_step(taches_pool* p, int32_t n, taches_stream* const* streams, const float* const* x_dev,
                     float* const* y_dev, const int32_t* n_blocks) {
  return taches_pool_step_strided(p, n, streams, x_dev, nullptr, y_dev, nullptr, n_blocks);
}

int taches_pool_step_strided(taches_pool* p, int32_t n, taches_stream* const* streams, const float* const* x_dev,
                             const int64_t* x_cstride, float* const* y_dev, const int64_t* y_cstride,
                             const int32_t* n_blocks) {
  if (!p) return fail(TACHES_EINVAL, "pool is NULL");
  if (n < 0 || (n > 0 && (!streams || !y_dev || !n_blocks))) return fail(TACHES_EINVAL, "bad step arguments");
  if (n == 0) return TACHES_OK;
  const auto t0 = std::chrono::steady_clock::now();
  const uint64_t mark = ++p->steps;
  p->ev_last = -1;
  for (int i = 0; i < n; ++i) {
    if (!streams[i] || streams[i]->pool != p) return fail(TACHES_EINVAL, "stream %d is not attached to this pool", i);
    if (streams[i]->step_mark == mark) return fail(TACHES_EINVAL, "stream listed twice in one step");
    streams[i]->step_mark = mark;
  }
  // plan every call (validation first: an error leaves every stream untouched)
  std::vector<CallPlan>& plans = p->plans;
  if ((int)plans.size() < n) plans.resize(n);
  for (int i = 0; i < n; ++i) {
    int rc = plan_call(streams[i], x_dev ? x_dev[i] : nullptr, x_cstride ? x_cstride[i] : 0, y_dev[i],
                       y_cstride ? y_cstride[i] : 0, n_blocks[i], nullptr, nullptr, &plans[i]);
    if (rc != TACHES_OK) return rc;
  }
  // Every fallible host step (planning, table packing, table buffers, graph
  // capture) comes before the first launch.  Once work is enqueued, every
  // stream whose kernels are on the device is committed, also when a later
  // launch fails, so the host state (head, live tail) always matches the
  // device's.  FP32 streams share one persistent gather launch; split-BF16
  // streams share one split-input launch and one Toeplitz MFMA launch per
  // class (tail type, padded channel count), after the gather launch.
  std::vector<int>& gather_ids = p->gather_ids;
  std::vector<const GatherCall*>& gcalls = p->gcalls;
  std::vector<int>* split_ids = p->split_ids;   // class = 2 * tail_fp64 + (cpad > 32)
  gather_ids.clear();
  gcalls.clear();
  for (int k = 0; k < 4; ++k) split_ids[k].clear();
  for (int i = 0; i < n; ++i) {
    taches_stream* s = streams[i];
    if (s->cfg.precision == TACHES_PREC_SPLIT_BF16) {
      split_ids[2 * (s->tail_fp64 ? 1 : 0) + (s->cpad > 32 ? 1 : 0)].push_back(i);
    } else {
      gather_ids.push_back(i);
      gcalls.push_back(&plans[i].g);
    }
  }
  std::vector<char>& enqueued = p->enqueued;
  enqueued.assign(n, 0);
  auto finish = [&](int rc) {
    for (int i = 0; i < n; ++i)
      if (enqueued[i]) commit_call(streams[i], plans[i]);
    return rc;
  };
  const bool has_gather = !gather_ids.empty();
  // ---- gather planning: work items over the resident workgroups ----
  typedef PoolItem Item;
  std::vector<Item>& items = p->items;
  items.clear();
  p->imbalance_pending = false;
  int nwg = 0, r = 0;
  bool mixed = false;   // some gather stream keeps an FP64 tail
  const int ng = (int)gather_ids.size();
  if (has_gather) {
    for (int i : gather_ids) mixed |= streams[i]->tail_fp64;
    r = pool_pick_r(p, gcalls, mixed);
    const int64_t T = 64 * r;
    // work items: runs of consecutive output tiles of one channel of one
    // call, with their FMA count (plus the tail read/write)
    auto tile_work = [T](const GatherCall& g, int64_t t) {
      const int64_t n0 = t * T;
      int64_t work = 4 * T;
      if (g.x) {
        const int64_t lo = std::max<int64_t>(0, n0 - (g.Lmax_call - 1));
        const int64_t hi = std::min<int64_t>(g.S, n0 + T);
        work += std::max<int64_t>(hi - lo, 0) * T;
      }
      return work;
    };
    // Tiles [flat_lo, flat_hi) of a call are reached by all its S input
    // samples (or, without input, all tiles): their work is the same.  The
    // work of the others rises or falls by T per tile at the two ends.
    auto flat_range = [T](const GatherCall& g, int64_t nt, int64_t* lo, int64_t* hi) {
      if (!g.x) {
        *lo = 0;
        *hi = nt;
        return;
      }
      *lo = std::max<int64_t>(0, (g.S + T - 1) / T - 1);                 // (t + 1) T >= S
      *hi = std::min<int64_t>(nt, (int64_t)(g.Lmax_call - 1) / T + 1);   // t T <= Lmax - 1
      if (*hi < *lo) *hi = *lo;
    };
    const int per_cu = taches::gather_batched_waves_per_cu(r, mixed);
    const int64_t wg_max = 256LL * per_cu;
    int64_t n_tiles = 0, tiles_work = 0, tile_max = 1;
    for (int k = 0; k < ng; ++k) {
      const GatherCall& g = plans[gather_ids[k]].g;
      const int64_t nt = (g.n_out + T - 1) / T;
      n_tiles += nt * g.channels;
      int64_t lo, hi;
      flat_range(g, nt, &lo, &hi);
      int64_t sum = 0;
      for (int64_t t = 0; t < lo; ++t) sum += tile_work(g, t);
      for (int64_t t = hi; t < nt; ++t) sum += tile_work(g, t);
      if (hi > lo) sum += (hi - lo) * tile_work(g, lo);
      tiles_work += sum * g.channels;
      for (int64_t t : {(int64_t)0, lo, hi - 1, hi, nt - 1})
        if (t >= 0 && t < nt) tile_max = std::max(tile_max, tile_work(g, t));
    }
    // With many small tiles (more than 32 per resident workgroup, as in a
    // step of one or a few blocks per stream, which touches every tail slot
    // of every stream), consecutive tiles are merged into items of about
    // 1/8 of a workgroup's share, so the table, its planning and the
    // kernel's per-item work shrink; otherwise one item per tile.
    const int64_t span_work = n_tiles > 32 * wg_max ? std::max(tile_max, tiles_work / (8 * wg_max)) : 0;
    items.reserve(span_work ? (size_t)(tiles_work / span_work + ng * 2 + 16) : (size_t)n_tiles);
    for (int k = 0; k < ng; ++k) {
      const GatherCall& g = plans[gather_ids[k]].g;
      const int64_t nt = (g.n_out + T - 1) / T;
      int64_t flo, fhi;
      flat_range(g, nt, &flo, &fhi);
      // equal tiles of the flat range: as many per item as fit in span_work
      const int64_t w_flat = fhi > flo ? tile_work(g, flo) : 1;
      const int64_t m_flat = span_work ? std::max<int64_t>(1, std::min<int64_t>(span_work / w_flat, 65535)) : 1;
      for (int c = 0; c < g.channels; ++c) {
        int64_t t = 0;
        while (t < nt) {
          if (span_work && t >= flo && t < fhi) {
            const int64_t m = std::min<int64_t>(m_flat, fhi - t);
            items.push_back({WorkItem{k, c, (int32_t)t, (int32_t)m}, w_flat * m});
            t += m;
            continue;
          }
          int64_t t1 = t + 1, w = tile_work(g, t);
          if (span_work) {
            while (t1 < nt && t1 - t < 65535) {
              const int64_t w1 = tile_work(g, t1);
              if (w + w1 > span_work) break;
              w += w1;
              ++t1;
            }
          }
          items.push_back({WorkItem{k, c, (int32_t)t, (int32_t)(t1 - t)}, w});
          t = t1;
        }
      }
    }
    // persistent workgroups (one wave each): as many as stay resident, but
    // no more than leave each at least the largest item's work
    int64_t total_work = 0, max_work = 1;
    for (const Item& it : items) {
      total_work += it.work;
      max_work = std::max(max_work, it.work);
    }
    const int64_t by_work = std::max<int64_t>(1, total_work / max_work);
    nwg = (int)std::max<int64_t>(std::min<int64_t>(256, (int64_t)items.size()),
                                           std::min<int64_t>(256LL * per_cu, by_work));
    // launched workgroups rounded up to 256 * 2^k (at most the resident
    // maximum), so that steps of similar size replay one captured graph; the
    // extra workgroups find the queue empty and leave
    {
      int64_t b = 256;
      while (b < nwg && b < wg_max) b *= 2;
      nwg = (int)std::min<int64_t>(b, wg_max);
    }
    // Workgroups take the items from a shared counter in list order.  With
    // merged runs or many small items, the list stays in stream and tile
    // order (neighbouring tiles share IR windows and inputs in L2);
    // otherwise it is sorted largest first, so the queue hands out the
    // heaviest items while every workgroup is still busy and the small
    // ones fill the end (greedy largest-first: no workgroup ends more
    // than one item after the mean).
    const size_t n_items = items.size();
    std::vector<uint32_t>& order = p->order;
    const bool in_order = (span_work > 0 && n_items >= 8 * (size_t)nwg) ||
                          (total_work >= 8 * max_work * (int64_t)nwg && n_items >= 16 * (size_t)nwg);
    if (in_order) {
      order.resize(n_items);
      for (size_t k = 0; k < n_items; ++k) order[k] = (uint32_t)k;
    } else {
      order_by_work_desc(items, order, p->keys, [](const Item& it) { return it.work; });
    }
    // reported estimate of the busiest workgroup's work over the mean: the
    // greedy bound (mean + largest item) / mean when items are many (at
    // least 8 per workgroup), else the queue played out on the estimated
    // works, on request
    const double mean = (double)total_work / nwg;
    p->last_total_work = total_work;
    p->imbalance_pending = !(in_order || n_items >= 8 * (size_t)nwg);
    if (!p->imbalance_pending) p->last_imbalance = mean > 0 ? (mean + (double)max_work) / mean : 1.0;
  }
  // ---- split classes: calls, tile and fragment prefix sums ----
  const int mt = taches::toeplitz_rows_per_tile();
  taches::ToeplitzBatch sb[4];
  int64_t split_tiles = 0;
  for (int k = 0; k < 4; ++k) {
    sb[k] = taches::ToeplitzBatch{};
    sb[k].n_calls = (int32_t)split_ids[k].size();
    for (int i : split_ids[k]) {
      const GatherCall& g = plans[i].g;
      sb[k].n_tiles += (g.n_out + mt - 1) / mt;
      if (g.x) sb[k].n_frags += (int64_t)g.n_blocks * g.cpb * 32 * g.cpad;
    }
    split_tiles += sb[k].n_tiles;
  }
  if (split_tiles > INT32_MAX) return fail(TACHES_EINVAL, "step too large: %lld Toeplitz tiles", (long long)split_tiles);
  // ---- table layout: [gather: header, calls, fp64 flags, items, counter]
  // [per split class: calls, tile starts (int32), fragment starts (int64)] ----
  size_t off_calls = 0, off_fp64 = 0, off_items = 0, off_next = 0, bytes = 0;
  if (has_gather) {
    off_calls = align256(sizeof(taches::BatchHeader));
    off_fp64 = align256(off_calls + sizeof(GatherCall) * ng);
    off_items = align256(off_fp64 + sizeof(int32_t) * ng);
    off_next = align256(off_items + sizeof(WorkItem) * items.size());
    bytes = align256(off_next + sizeof(int32_t));
  }
  for (int k = 0; k < 4; ++k) {
    if (!sb[k].n_calls) continue;
    sb[k].off_calls = (int64_t)bytes;
    sb[k].off_tiles = (int64_t)align256(bytes + sizeof(GatherCall) * sb[k].n_calls);
    sb[k].off_frags = (int64_t)align256(sb[k].off_tiles + sizeof(int32_t) * (sb[k].n_calls + 1));
    bytes = align256(sb[k].off_frags + sizeof(int64_t) * (sb[k].n_calls + 1));
  }
  int rc = pool_reserve(p, bytes);
  if (rc != TACHES_OK) return rc;
  const int cur = p->tab_cur;
  unsigned char* pin = p->tab_pin[cur];
  if (p->tab_pending[cur]) {   // the step before the previous one read this buffer
    HIPCHK(hipEventSynchronize(p->tab_free[cur]));
    p->tab_pending[cur] = false;
  }
  if (has_gather) {
    taches::BatchHeader* hd = (taches::BatchHeader*)pin;
    hd->off_calls = (int32_t)off_calls;
    hd->off_fp64 = (int32_t)off_fp64;
    hd->off_items = (int32_t)off_items;
    hd->off_next = (int32_t)off_next;
    hd->n_items = (int32_t)items.size();
    hd->pad_ = 0;
    GatherCall* calls = (GatherCall*)(pin + off_calls);
    int32_t* fp64 = (int32_t*)(pin + off_fp64);
    WorkItem* wit = (WorkItem*)(pin + off_items);
    for (int k = 0; k < ng; ++k) {
      calls[k] = plans[gather_ids[k]].g;
      calls[k].tile_order = 2;
      fp64[k] = streams[gather_ids[k]]->tail_fp64 ? 1 : 0;
    }
    const std::vector<uint32_t>& order = p->order;
    for (size_t k = 0; k < items.size(); ++k) wit[k] = items[order[k]].w;
    *(int32_t*)(pin + off_next) = 0;   // items taken: reset by every table copy
  }
  for (int k = 0; k < 4; ++k) {
    if (!sb[k].n_calls) continue;
    GatherCall* calls = (GatherCall*)(pin + sb[k].off_calls);
    int32_t* ts = (int32_t*)(pin + sb[k].off_tiles);
    int64_t* fs = (int64_t*)(pin + sb[k].off_frags);
    ts[0] = 0;
    fs[0] = 0;
    for (int j = 0; j < sb[k].n_calls; ++j) {
      const GatherCall& g = plans[split_ids[k][j]].g;
      calls[j] = g;
      ts[j + 1] = ts[j] + (g.n_out + mt - 1) / mt;
      fs[j + 1] = fs[j] + (g.x ? (int64_t)g.n_blocks * g.cpb * 32 * g.cpad : 0);
    }
  }
  const auto t1 = std::chrono::steady_clock::now();
  p->last_plan_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  const int ev = p->ev_next;
  if (p->ev_pending[ev]) {
    HIPCHK(hipEventSynchronize(p->ev_end[ev]));
    int rc2 = pool_account(p, false);
    if (rc2 != TACHES_OK) return rc2;
  }
  unsigned char* dev = p->tab_dev[cur];
  const bool sep = p->copy != nullptr;   // table copy on the copy stream, outside the graph
  taches_pool::Graph* pg = nullptr;
  if (has_gather && p->use_graph) {
    int b = 0;
    while ((256 << b) < nwg && b < 7) ++b;
    pg = &p->graphs[(((((r / 4 - 1) * 2 + (mixed ? 1 : 0)) * 8 + b) * 2 + cur) * 2) + (sep ? 1 : 0)];
    if (!pg->exec || pg->nwg != nwg || pg->cap != p->tab_cap) {
      drop_graph(*pg);
      HIPCHK(hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal));
      hipError_t e1 = sep ? hipSuccess : hipMemcpyAsync(dev, pin, p->tab_cap, hipMemcpyHostToDevice, p->capture);
      hipError_t e2 = taches::launch_gather_batched(dev, nwg, r, mixed, p->capture);
      hipError_t e3 = hipStreamEndCapture(p->capture, &pg->graph);
      if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
        return fail(TACHES_EDEVICE, "graph capture failed: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2 != hipSuccess ? e2 : e3));
      HIPCHK(hipGraphInstantiate(&pg->exec, pg->graph, nullptr, nullptr, 0));
      size_t nn = 0;
      HIPCHK(hipGraphGetNodes(pg->graph, nullptr, &nn));
      std::vector<hipGraphNode_t> nodes(nn);
      HIPCHK(hipGraphGetNodes(pg->graph, nodes.data(), &nn));
      for (auto nd : nodes) {
        hipGraphNodeType ty;
        HIPCHK(hipGraphNodeGetType(nd, &ty));
        if (ty == hipGraphNodeTypeMemcpy) pg->copy_node = nd;
      }
      pg->nwg = nwg;
      pg->cap = p->tab_cap;
      p->captures += 1;
    }
  }
  bool replay = false;
  if (pg && pg->exec)
    replay = sep || (pg->copy_node && hipGraphExecMemcpyNodeSetParams1D(pg->exec, pg->copy_node, dev, pin, bytes,
                                                                        hipMemcpyHostToDevice) == hipSuccess);
  // ---- enqueue: from here on, failures commit what was enqueued ----
  hipError_t e = hipSuccess;
  if (sep) {
    e = hipMemcpyAsync(dev, pin, bytes, hipMemcpyHostToDevice, p->copy);
    if (e == hipSuccess) e = hipEventRecord(p->tab_copied, p->copy);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->stream, p->tab_copied, 0);
  }
  if (e == hipSuccess) e = hipEventRecord(p->ev_beg[ev], p->stream);
  if (e == hipSuccess) {
    if (replay) {
      e = hipGraphLaunch(pg->exec, p->stream);
      if (e == hipSuccess) p->replays += 1;
    } else {
      if (!sep) e = hipMemcpyAsync(dev, pin, bytes, hipMemcpyHostToDevice, p->stream);
      if (e == hipSuccess && has_gather) e = taches::launch_gather_batched(dev, nwg, r, mixed, p->stream);
    }
  }
  if (e != hipSuccess) return finish(fail(TACHES_EDEVICE, "batched launch: %s", hipGetErrorString(e)));
  for (int i : gather_ids) enqueued[i] = 1;
  for (int k = 0; k < 4; ++k) {
    if (!sb[k].n_calls) continue;
    e = taches::launch_toeplitz_batched(dev, sb[k], (k & 2) != 0, (k & 1) != 0, p->stream);
    if (e != hipSuccess) return finish(fail(TACHES_EDEVICE, "batched Toeplitz launch: %s", hipGetErrorString(e)));
    for (int i : split_ids[k]) {
      enqueued[i] = 1;
      streams[i]->last_r = 0;
      streams[i]->last_w = 0;
    }
  }
  p->ev_pending[ev] = hipEventRecord(p->ev_end[ev], p->stream) == hipSuccess;
  p->ev_last = p->ev_pending[ev] ? ev : -1;
  p->ev_next = (ev + 1) % taches_pool::kRing;
  p->tab_pending[cur] = hipEventRecord(p->tab_free[cur], p->stream) == hipSuccess;
  if (!p->tab_pending[cur]) {
    // without the event the pinned table cannot be reused safely: wait here
    (void)hipStreamSynchronize(p->stream);
  }
  p->tab_cur = cur ^ 1;
  p->last_items = (int)items.size();
  p->last_wg = nwg;
  p->last_r = r;
  for (int k = 0; k < ng; ++k) {
    streams[gather_ids[k]]->last_r = r;
    streams[gather_ids[k]]->last_w = 1;
  }
  return finish(TACHES_OK);
}

}  // extern "C"

namespace taches {

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, kErrLen, fmt, ap);
  va_end(ap);
  return code;
}

hipStream_t pool_stream(const taches_pool* p) { return p->stream; }

bool stream_in_pool(const taches_stream* s, const taches_pool* p) { return s->pool == p; }

}  // namespace taches
