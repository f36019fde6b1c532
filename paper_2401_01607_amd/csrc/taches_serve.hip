// Serving tick of libtaches: real-time streams of a pool advanced by one
// library call per tick.
//
// Each registered stream delivers one block of B samples per channel every
// B / fs seconds from its start time (real-time pacing); after its input,
// the temporal overflow (L - 1 samples, Section 4.1) is drained with
// zero-input blocks paced the same way.  A tick takes every block whose
// last sample has arrived by the tick's clock reading, over all streams,
// and runs them as one pool step: the arrived input is gathered from each
// stream's host buffer into pinned memory, copied to the device in one
// transfer and processed by the pool's batched launch; one more launch
// writes every output block to mapped, coherent pinned host memory, from
// where it is handed to the stream's host buffer.
// An IR change scheduled at time t of a stream applies to its first block
// that starts at or after t (the IR is replaced "for next samples",
// Abstract and Section 6): a step's range of blocks ends before such a
// block, which starts the next range.
//
// A stream may be served in two segments of its IR (linearity of Eq. (1)):
// the head h[0, H) on a stream of block B advanced every tick, and the rest
// h[H, L) on a second stream of block Br = K * B (Br <= H), whose output z
// enters the result H samples later, y[n] = y_head[n] + z[n - H].  The rest
// stream keeps the long tail and is advanced once per Br samples instead of
// once per tick, so a tick reads and writes H + B tail slots of the stream
// instead of L + B.  Its outputs stay on the device in a ring [C][Z] owned
// by the caller (the pool step writes them there in place); after the pool
// step, one launch adds the ring into the head outputs while it writes every
// output block to the mapped host staging.  A head block is run only once
// the rest blocks it needs have been enqueued (by arrival they always have: their last sample comes no later
// than the head block's, as Br <= H), and rest blocks wait while their
// outputs would overwrite ring entries not yet added.
//
// Ticks overlap with the device: a tick enqueues its step (input copy, pool
// step, output launch) and then waits for the previous tick's step, so the
// host gathers and plans step k + 1 while the device runs step k, and the
// device always has the next step queued.  Latency of a block = the time
// its outputs are in host memory (the completion event recorded after the
// output launch, placed on the host clock) minus the arrival time of the block's last
// sample; the deadline is one block period.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "taches.h"
#include "taches_internal.h"

namespace {

struct ServeStream {
  taches_stream* s = nullptr;
  int64_t tag = 0;
  double start_s = 0.0;
  int32_t B = 0, C = 0;
  int64_t n_in = 0, n_total = 0, next = 0;
  const float* x = nullptr;
  int64_t x_cs = 0;
  float* y = nullptr;
  int64_t y_cs = 0;
  std::vector<double> swap_t;
  std::vector<const float*> swap_h;
  std::vector<int32_t> swap_L;
  size_t swap_next = 0;
  std::vector<int64_t> swap_blocks;   // block index at which each applied swap took effect
  bool in_place = false;              // FP32: IRs are read in place (taches_set_ir_ref), not copied
  // two-segment streams (rs != nullptr): the rest segment h[H, L)
  taches_stream* rs = nullptr;
  int32_t H = 0, Br = 0, r_cap = 1;
  int64_t r_in = 0, r_total = 0, r_next = 0;
  float* z = nullptr;                 // device ring [C][Z] of the rest segment's outputs
  int32_t Z = 0;
  std::vector<int64_t> swap_s;        // input sample at which each IR change applies (within the input)
  size_t r_swap_next = 0;
};

// First block k of a stream with start time k * B / fs >= t (k >= k_min).
int64_t first_block_at(double t, int32_t B, double fs, int64_t k_min) {
  int64_t k = (int64_t)std::ceil(t * fs / B - 1e-9);
  k = std::max(k, k_min);
  while (k > k_min && (double)((k - 1) * B) / fs >= t) --k;
  while ((double)(k * B) / fs < t) ++k;
  return k;
}

// The outputs of one range of a step, from the device staging (C rows of
// len) to the host staging (the same layout, pinned and mapped for the
// device); for a two-segment stream, ring entries p0, p0 + 1, ... (mod Z) of
// the rows of z are added from output `skip` on (outputs before sample H
// get nothing).
struct OutOp {
  const float* y;
  float* out;
  const float* z;   // nullptr: a stream served whole
  int32_t len, C, Z, p0, skip, pad_;
};

// One workgroup per range: the ring add and the write to host memory in one pass.
__global__ __launch_bounds__(256) void k_out(const OutOp* __restrict__ ops) {
  const OutOp o = ops[blockIdx.x];
  for (int c = 0; c < o.C; ++c) {
    const float* y = o.y + (int64_t)c * o.len;
    float* out = o.out + (int64_t)c * o.len;
    const float* z = o.z ? o.z + (int64_t)c * o.Z : nullptr;
    for (int i = threadIdx.x; i < o.len; i += blockDim.x) {
      float v = y[i];
      if (z && i >= o.skip) {
        int pos = o.p0 + (i - o.skip);
        if (pos >= o.Z) pos -= o.Z;
        v += z[pos];
      }
      out[i] = v;
    }
  }
}

}  // namespace

// One block range of a step in flight: what completing the step needs.
struct FlightRange {
  int64_t tag;
  float* y;
  int64_t y_cs;
  int32_t C, B;
  int64_t k0;
  int32_t n;
  int64_t yoff;
  double start_s;
  double tick_s;   // server clock at the start of the tick that enqueued the range
  bool last;   // the stream's last block: it finishes when this step completes
};

struct Flight {
  bool active = false;
  int buf = 0;        // pinned buffer pair used
  int ev = 0;         // completion event (after the output launch)
  std::vector<FlightRange> ranges;
};

struct taches_server {
  taches_pool* pool = nullptr;
  double fs = 48000.0;
  int32_t max_blocks = 1;
  double warmup_s = 0.0;
  std::chrono::steady_clock::time_point t0;
  std::vector<ServeStream> st;
  // staging of one step's input and output blocks: two pinned pairs used in
  // turn (a step's input copy may still be queued while the next gathers;
  // its outputs are read after the next step is enqueued); one device pair
  // (copies and steps are ordered on the pool's stream)
  float* x_pin[2] = {nullptr, nullptr};
  float* y_pin[2] = {nullptr, nullptr};      // mapped and coherent: written by k_out
  float* y_pin_dev[2] = {nullptr, nullptr};  // their device addresses
  size_t pin_cap = 0;     // floats per buffer
  float* x_dev = nullptr;
  float* y_dev = nullptr;
  size_t dev_cap = 0;
  // completion events (a ring: the previous completed one is the time
  // reference for the next), and the host time of the last completed one
  static constexpr int kEv = 4;
  hipEvent_t ev[kEv] = {};
  hipEvent_t ev_beg[kEv] = {};   // a step's start on the device (before its input copy)
  int ev_next = 0;
  int ref_ev = -1;
  double ref_t = 0.0;
  hipEvent_t anchor = nullptr;
  Flight fl;
  int tick_buf = 0;
  // per-tick argument arrays of the pool step (kept to avoid reallocation)
  std::vector<taches_stream*> a_s;
  std::vector<const float*> a_x;
  std::vector<float*> a_y;
  std::vector<int64_t> a_xcs, a_ycs;   // channel strides of the pool step's input and output
  std::vector<int32_t> a_n;
  std::vector<int32_t> a_idx;
  std::vector<int64_t> a_k0, a_xoff, a_yoff;
  std::vector<char> a_rest;          // range of a rest segment (outputs stay on the device)
  std::vector<int64_t> r_end;        // per registered stream: rest blocks enqueued after this tick
  // records
  std::vector<float> lat_s;
  std::vector<int32_t> lat_B;
  std::vector<int64_t> finished;     // tags not yet taken by the caller
  std::vector<ServeStream> done;     // records of finished streams (state queries)
  taches_server_stats stats{};
};

namespace {

double clock_s(const taches_server* sv) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - sv->t0).count();
}

ServeStream* find_tag(taches_server* sv, int64_t tag, bool with_done = false) {
  for (ServeStream& r : sv->st)
    if (r.tag == tag) return &r;
  if (with_done)
    for (ServeStream& r : sv->done)
      if (r.tag == tag) return &r;
  return nullptr;
}

// Larger staging (called with no step in flight).
int grow(taches_server* sv, size_t floats) {
  // capacity grows in large steps (at least 16 M floats, then 4x): a larger
  // staging costs pinned allocations and frees, which stall the tick
  constexpr size_t kMinFloats = size_t(1) << 24;
  if (floats > sv->pin_cap) {
    const size_t cap = std::max({floats, 4 * sv->pin_cap, kMinFloats});
    for (int k = 0; k < 2; ++k) {
      (void)hipHostFree(sv->x_pin[k]);
      (void)hipHostFree(sv->y_pin[k]);
      sv->x_pin[k] = sv->y_pin[k] = nullptr;
    }
    sv->pin_cap = 0;
    for (int k = 0; k < 2; ++k) {
      sv->y_pin_dev[k] = nullptr;
      if (hipHostMalloc((void**)&sv->x_pin[k], cap * 4, hipHostMallocDefault) != hipSuccess ||
          hipHostMalloc((void**)&sv->y_pin[k], cap * 4, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
          hipHostGetDevicePointer((void**)&sv->y_pin_dev[k], sv->y_pin[k], 0) != hipSuccess)
        return taches::set_error(TACHES_ENOMEM, "serving: pinned staging of %zu floats", cap);
    }
    sv->pin_cap = cap;
  }
  if (floats > sv->dev_cap) {
    const size_t cap = std::max({floats, 4 * sv->dev_cap, kMinFloats});
    (void)hipFree(sv->x_dev);
    (void)hipFree(sv->y_dev);
    sv->x_dev = sv->y_dev = nullptr;
    sv->dev_cap = 0;
    if (hipMalloc((void**)&sv->x_dev, cap * 4) != hipSuccess || hipMalloc((void**)&sv->y_dev, cap * 4) != hipSuccess)
      return taches::set_error(TACHES_ENOMEM, "serving: device staging of %zu floats", cap);
    sv->dev_cap = cap;
  }
  return TACHES_OK;
}

// Wait for the step in flight, place its completion on the host clock, hand
// its outputs to the streams' host buffers, record its block latencies and
// report streams whose last block it held.
int complete_flight(taches_server* sv) {
  Flight& f = sv->fl;
  if (!f.active) return TACHES_OK;
  const double t0 = clock_s(sv);
  hipError_t e = hipEventSynchronize(sv->ev[f.ev]);
  if (e != hipSuccess) return taches::set_error(TACHES_EDEVICE, "serving: wait: %s", hipGetErrorString(e));
  const double t1 = clock_s(sv);
  float ms = 0.f;
  double done = t1;
  if (sv->ref_ev >= 0 && hipEventElapsedTime(&ms, sv->ev[sv->ref_ev], sv->ev[f.ev]) == hipSuccess)
    done = std::min(t1, sv->ref_t + (double)ms * 1e-3);
  sv->ref_ev = f.ev;
  sv->ref_t = done;
  if (hipEventElapsedTime(&ms, sv->ev_beg[f.ev], sv->ev[f.ev]) == hipSuccess) sv->stats.device_s += (double)ms * 1e-3;
  const double fs = sv->fs;
  for (const FlightRange& q : f.ranges) {
    if (q.y) {
      const size_t row = (size_t)q.n * q.B;
      const float* src = sv->y_pin[f.buf] + q.yoff;
      for (int c = 0; c < q.C; ++c) std::memcpy(q.y + c * q.y_cs + q.k0 * q.B, src + c * row, row * 4);
    }
    const double per = (double)q.B / fs;
    for (int32_t k = 0; k < q.n; ++k) {
      const double arrival = q.start_s + (double)(q.k0 + k + 1) * per;
      if (arrival < sv->warmup_s) continue;
      sv->lat_s.push_back((float)(done - arrival));
      sv->lat_B.push_back(q.B);
      sv->stats.recorded += 1;
      sv->stats.pickup_s += q.tick_s - arrival;
      sv->stats.service_s += done - q.tick_s;
    }
    if (q.last) sv->finished.push_back(q.tag);
  }
  f.active = false;
  f.ranges.clear();
  sv->stats.wait_s += t1 - t0;
  sv->stats.scatter_s += clock_s(sv) - t1;
  return TACHES_OK;
}

// With nothing in flight, tie a fresh event on the pool's (idle) stream to
// the host clock: the time reference for the next completion.
int anchor_clock(taches_server* sv, hipStream_t hs) {
  const int k = sv->ev_next;
  sv->ev_next = (sv->ev_next + 1) % taches_server::kEv;
  hipError_t e = hipEventRecord(sv->ev[k], hs);
  if (e == hipSuccess) e = hipEventSynchronize(sv->ev[k]);
  if (e != hipSuccess) return taches::set_error(TACHES_EDEVICE, "serving: clock anchor: %s", hipGetErrorString(e));
  sv->ref_ev = k;
  sv->ref_t = clock_s(sv);
  return TACHES_OK;
}

}  // namespace

extern "C" {

taches_server* taches_server_create(taches_pool* pool, double fs, int32_t max_blocks_per_step, double warmup_s) {
  if (!pool || !(fs > 0.0) || max_blocks_per_step < 1) {
    taches::set_error(TACHES_EINVAL, "serving: bad pool, sample rate or block limit");
    return nullptr;
  }
  taches_server* sv = new taches_server;
  sv->pool = pool;
  sv->fs = fs;
  sv->max_blocks = max_blocks_per_step;
  sv->warmup_s = warmup_s;
  sv->t0 = std::chrono::steady_clock::now();
  for (int k = 0; k < taches_server::kEv; ++k) {
    if (hipEventCreate(&sv->ev[k]) != hipSuccess || hipEventCreate(&sv->ev_beg[k]) != hipSuccess) {
      taches::set_error(TACHES_EDEVICE, "serving: event creation failed");
      for (int j = 0; j <= k; ++j)
        for (hipEvent_t e : {sv->ev[j], sv->ev_beg[j]})
          if (e) (void)hipEventDestroy(e);
      delete sv;
      return nullptr;
    }
  }
  return sv;
}

int taches_server_destroy(taches_server* sv) {
  if (!sv) return TACHES_OK;
  (void)taches_pool_synchronize(sv->pool);
  for (int k = 0; k < 2; ++k) {
    (void)hipHostFree(sv->x_pin[k]);
    (void)hipHostFree(sv->y_pin[k]);
  }
  (void)hipFree(sv->x_dev);
  (void)hipFree(sv->y_dev);
  for (int k = 0; k < taches_server::kEv; ++k)
    for (hipEvent_t e : {sv->ev[k], sv->ev_beg[k]})
      if (e) (void)hipEventDestroy(e);
  delete sv;
  return TACHES_OK;
}

int taches_server_flush(taches_server* sv) {
  if (!sv) return taches::set_error(TACHES_EINVAL, "server is NULL");
  return complete_flight(sv);
}

double taches_server_clock(const taches_server* sv) { return sv ? clock_s(sv) : -1.0; }

namespace {

// Checks shared by both registrations; fills the record of a one-segment
// stream.
int fill_record(taches_server* sv, taches_stream* s, int64_t tag, double start_s, int64_t n_in_blocks,
                int64_t n_total_blocks, const float* x_host, int64_t x_cstride, float* y_host, int64_t y_cstride,
                int32_t n_swaps, const double* swap_times_s, const float* const* swap_ir_dev, const int32_t* swap_len,
                int32_t swap_len_min, int32_t swap_len_max, ServeStream* out, taches_info* inf) {
  if (!sv || !s) return taches::set_error(TACHES_EINVAL, "serving: NULL server or stream");
  int rc = taches_get_info(s, inf);
  if (rc != TACHES_OK) return rc;
  if (!taches::stream_in_pool(s, sv->pool)) return taches::set_error(TACHES_EINVAL, "serving: stream not attached to the pool");
  if (find_tag(sv, tag, true)) return taches::set_error(TACHES_EINVAL, "serving: tag %lld already registered", (long long)tag);
  if (n_in_blocks < 1 || n_total_blocks < n_in_blocks) return taches::set_error(TACHES_EINVAL, "serving: block counts");
  if (sv->max_blocks > inf->max_blocks_per_call)
    return taches::set_error(TACHES_EINVAL, "serving: stream takes %d blocks per call, the server %d",
                             inf->max_blocks_per_call, sv->max_blocks);
  const int64_t need = n_in_blocks * inf->block_size;
  if (!x_host || x_cstride < need)
    return taches::set_error(TACHES_EINVAL, "serving: input buffer shorter than the input blocks");
  if (y_host && y_cstride < n_total_blocks * inf->block_size)
    return taches::set_error(TACHES_EINVAL, "serving: output buffer shorter than the stream");
  if (n_swaps < 0 || (n_swaps > 0 && (!swap_times_s || !swap_ir_dev || !swap_len)))
    return taches::set_error(TACHES_EINVAL, "serving: swap arrays");
  if (swap_len_max <= 0) swap_len_max = inf->max_ir_len;
  for (int i = 0; i < n_swaps; ++i) {
    if (!swap_ir_dev[i] || swap_len[i] < swap_len_min || swap_len[i] > swap_len_max)
      return taches::set_error(TACHES_EINVAL, "serving: swap %d IR", i);
    if (i > 0 && swap_times_s[i] < swap_times_s[i - 1])
      return taches::set_error(TACHES_EINVAL, "serving: swap times not ascending");
  }
  ServeStream& r = *out;
  r.s = s;
  r.in_place = inf->precision == TACHES_PREC_FP32;
  r.tag = tag;
  r.start_s = start_s;
  r.B = inf->block_size;
  r.C = inf->channels;
  r.n_in = n_in_blocks;
  r.n_total = n_total_blocks;
  r.x = x_host;
  r.x_cs = x_cstride;
  r.y = y_host;
  r.y_cs = y_cstride;
  r.swap_t.assign(swap_times_s, swap_times_s + n_swaps);
  r.swap_h.assign(swap_ir_dev, swap_ir_dev + n_swaps);
  r.swap_L.assign(swap_len, swap_len + n_swaps);
  return TACHES_OK;
}

}  // namespace

int taches_server_add(taches_server* sv, taches_stream* s, int64_t tag, double start_s, int64_t n_in_blocks,
                      int64_t n_total_blocks, const float* x_host, int64_t x_cstride, float* y_host, int64_t y_cstride,
                      int32_t n_swaps, const double* swap_times_s, const float* const* swap_ir_dev,
                      const int32_t* swap_len) {
  ServeStream r;
  taches_info inf;
  int rc = fill_record(sv, s, tag, start_s, n_in_blocks, n_total_blocks, x_host, x_cstride, y_host, y_cstride, n_swaps,
                       swap_times_s, swap_ir_dev, swap_len, 1, 0, &r, &inf);
  if (rc != TACHES_OK) return rc;
  sv->st.push_back(std::move(r));
  return TACHES_OK;
}

int taches_server_add_segmented(taches_server* sv, taches_stream* head, taches_stream* rest, int32_t head_len,
                                float* z_dev, int32_t z_len, int64_t tag, double start_s, int64_t n_in_blocks,
                                int64_t n_total_blocks, const float* x_host, int64_t x_cstride, float* y_host,
                                int64_t y_cstride, const float* ir_dev, int32_t ir_len, int32_t n_swaps,
                                const double* swap_times_s, const float* const* swap_ir_dev, const int32_t* swap_len) {
  if (!sv || !head || !rest || !ir_dev || !z_dev)
    return taches::set_error(TACHES_EINVAL, "serving: NULL server, stream, IR or ring");
  taches_info ri, hi0;
  int rc = taches_get_info(rest, &ri);
  if (rc == TACHES_OK) rc = taches_get_info(head, &hi0);
  if (rc != TACHES_OK) return rc;
  if (!taches::stream_in_pool(rest, sv->pool)) return taches::set_error(TACHES_EINVAL, "serving: rest stream not attached to the pool");
  if (hi0.precision != TACHES_PREC_FP32 || ri.precision != TACHES_PREC_FP32)
    return taches::set_error(TACHES_EINVAL, "serving: two-segment streams need FP32 precision");
  const int32_t H = head_len, Br = ri.block_size;
  const int32_t lmin = H + 1, lmax = std::min<int64_t>((int64_t)H + ri.max_ir_len, INT32_MAX);
  ServeStream r;
  taches_info hi;
  rc = fill_record(sv, head, tag, start_s, n_in_blocks, n_total_blocks, x_host, x_cstride, y_host, y_cstride, n_swaps,
                   swap_times_s, swap_ir_dev, swap_len, lmin, lmax, &r, &hi);
  if (rc != TACHES_OK) return rc;
  if (ri.channels != hi.channels) return taches::set_error(TACHES_EINVAL, "serving: head and rest channel counts differ");
  if (Br % hi.block_size != 0 || H < Br || H > hi.max_ir_len)
    return taches::set_error(TACHES_EINVAL, "serving: segments need B | Br <= H <= head capacity (B %d, Br %d, H %d)",
                             hi.block_size, Br, H);
  if (ir_len < lmin || ir_len > lmax) return taches::set_error(TACHES_EINVAL, "serving: IR of %d taps for H = %d", ir_len, H);
  if (z_len < 2 * Br || z_len % Br != 0)
    return taches::set_error(TACHES_EINVAL, "serving: ring of %d entries: not a multiple of Br = %d of at least 2 Br",
                             z_len, Br);
  const int32_t B = hi.block_size;
  // input sample at which each change applies (the head's rule: the first
  // block starting at or after its time); changes after the input never apply
  // (the initial IR counts as a change at sample 0: a rest block takes one
  // IR from its start and at most one change inside)
  std::vector<int64_t> ss;
  int64_t prev = 0;
  for (int i = 0; i < n_swaps; ++i) {
    const int64_t k = first_block_at(swap_times_s[i], B, sv->fs, 0);
    if (k >= n_in_blocks) break;
    const int64_t smp = k * B;
    if (smp != prev && smp / Br == prev / Br)
      return taches::set_error(TACHES_EINVAL, "serving: two IR changes inside one rest block of %d samples", Br);
    ss.push_back(smp);
    prev = smp;
  }
  rc = taches_set_ir_ref(head, ir_dev, H, 0);
  if (rc == TACHES_OK) rc = taches_set_ir_ref(rest, ir_dev + H, ir_len - H, 0);
  if (rc != TACHES_OK) return rc;
  r.rs = rest;
  r.H = H;
  r.Br = Br;
  r.r_cap = std::max(1, std::min(sv->max_blocks, ri.max_blocks_per_call));
  r.r_in = (n_in_blocks * B + Br - 1) / Br;
  r.r_total = std::max(r.r_in, (n_total_blocks * B - H + Br - 1) / Br);
  r.z = z_dev;
  r.Z = z_len;
  r.swap_s = std::move(ss);
  sv->st.push_back(std::move(r));
  return TACHES_OK;
}

int taches_server_tick(taches_server* sv, taches_server_tick_info* out) {
  if (!sv) return taches::set_error(TACHES_EINVAL, "server is NULL");
  taches_server_tick_info info{};
  const double now = clock_s(sv);
  info.now_s = now;
  const double fs = sv->fs;
  // ---- ranges: every arrived block of each stream, in order ----
  sv->a_s.clear();
  sv->a_n.clear();
  sv->a_idx.clear();
  sv->a_k0.clear();
  sv->a_xoff.clear();
  sv->a_yoff.clear();
  sv->a_rest.clear();
  sv->r_end.assign(sv->st.size(), 0);
  size_t xf = 0, yf = 0;   // input floats; head output floats
  auto push_range = [&](taches_stream* s, int32_t n, size_t i, int64_t k0, bool in, size_t len, bool rest) {
    sv->a_s.push_back(s);
    sv->a_n.push_back(n);
    sv->a_idx.push_back((int32_t)i);
    sv->a_k0.push_back(k0);
    sv->a_xoff.push_back(in ? (int64_t)xf : -1);
    if (in) xf += len;
    sv->a_yoff.push_back(rest ? -1 : (int64_t)yf);   // rest outputs go straight into the ring
    if (!rest) yf += len;
    sv->a_rest.push_back(rest ? 1 : 0);
  };
  for (size_t i = 0; i < sv->st.size(); ++i) {
    ServeStream& r = sv->st[i];
    // rest segment first: a head block runs once the rest blocks it needs are enqueued
    if (r.rs) {
      int64_t rend = r.r_next;
      if (r.r_next < r.r_total) {
        int64_t arr = (int64_t)std::floor((now - r.start_s) * fs / r.Br);
        arr = std::min(std::max<int64_t>(arr, 0), r.r_total);
        // ring entries below `consumed` have been added by enqueued steps
        const int64_t consumed = std::max<int64_t>(0, r.next * r.B - r.H);
        const int64_t j0 = r.r_next;
        int64_t end = std::min(std::min(arr, j0 + r.r_cap), (consumed + r.Z) / r.Br);
        const int64_t zb = r.Z / r.Br;   // rest blocks per ring: a range is written in place, unwrapped
        end = std::min(end, (j0 / zb + 1) * zb);
        if (end > j0) {
          const bool in = j0 < r.r_in;
          if (in) {
            // changes applying inside or at the start of block j0
            while (r.r_swap_next < r.swap_s.size() && r.swap_s[r.r_swap_next] < (j0 + 1) * r.Br) {
              const size_t q = r.r_swap_next;
              const int64_t off = std::max<int64_t>(0, r.swap_s[q] - j0 * r.Br);
              const float* h = r.swap_h[q] + r.H;
              const int32_t L = r.swap_L[q] - r.H;
              int rc = taches_set_ir_ref(r.rs, h, L, (int32_t)off);
              if (rc != TACHES_OK) return rc;
              ++r.r_swap_next;
            }
            end = std::min(end, r.r_in);
            if (r.r_swap_next < r.swap_s.size()) end = std::min(end, r.swap_s[r.r_swap_next] / r.Br);
          }
          push_range(r.rs, (int32_t)(end - j0), i, j0, in, (size_t)r.C * (end - j0) * r.Br, true);
          rend = end;
        }
      }
      sv->r_end[i] = rend;
    }
    int64_t arrived = (int64_t)std::floor((now - r.start_s) * fs / r.B);
    arrived = std::min(std::max<int64_t>(arrived, 0), r.n_total);
    if (r.rs) arrived = std::min(arrived, (sv->r_end[i] * r.Br + r.H) / r.B);
    if (arrived <= r.next) continue;
    const int64_t k0 = r.next;
    const bool is_in = k0 < r.n_in;
    // IR changes due by the start of this range's first block apply to it
    if (is_in) {
      while (r.swap_next < r.swap_t.size() && r.swap_t[r.swap_next] <= (double)(k0 * r.B) / fs) {
        const int32_t L = r.rs ? r.H : r.swap_L[r.swap_next];
        int rc = r.in_place ? taches_set_ir_ref(r.s, r.swap_h[r.swap_next], L, 0)
                            : taches_set_ir_device(r.s, r.swap_h[r.swap_next], L);
        if (rc != TACHES_OK) return rc;
        r.swap_blocks.push_back(k0);
        ++r.swap_next;
      }
    }
    int64_t end = std::min<int64_t>(arrived, k0 + sv->max_blocks);
    if (is_in) {
      end = std::min(end, r.n_in);
      if (r.swap_next < r.swap_t.size()) end = std::min(end, first_block_at(r.swap_t[r.swap_next], r.B, fs, k0 + 1));
    }
    push_range(r.s, (int32_t)(end - k0), i, k0, is_in, (size_t)r.C * (end - k0) * r.B, false);
  }
  const size_t m = sv->a_s.size();
  auto next_due = [&]() {
    double t = HUGE_VAL;
    for (const ServeStream& r : sv->st) t = std::min(t, r.start_s + (double)((r.next + 1) * r.B) / fs);
    return t;
  };
  if (m == 0) {
    // nothing new: finish the step in flight (its outputs are due)
    int rc = complete_flight(sv);
    if (rc != TACHES_OK) return rc;
    info.next_due_s = next_due();
    if (out) *out = info;
    return TACHES_OK;
  }
  // one output operation per head range: the ring add (two-segment streams)
  // and the copy into the mapped host staging
  size_t n_ops = 0;
  for (size_t j = 0; j < m; ++j) n_ops += sv->a_rest[j] ? 0 : 1;
  const size_t ops_off = (xf * 4 + 255) & ~(size_t)255;   // bytes: the ops follow the input
  const size_t x_floats = n_ops ? (ops_off + n_ops * sizeof(OutOp) + 3) / 4 : xf;
  const size_t y_floats = yf;
  const hipStream_t hs = taches::pool_stream(sv->pool);
  int rc = TACHES_OK;
  if (std::max(x_floats, y_floats) > std::min(sv->pin_cap, sv->dev_cap)) {
    rc = complete_flight(sv);   // staging in use by the step in flight
    if (rc == TACHES_OK) rc = grow(sv, std::max(x_floats, y_floats));
    if (rc != TACHES_OK) return rc;
  }
  const int buf = sv->tick_buf;
  // ---- gather the arrived input into pinned memory ----
  for (size_t j = 0; j < m; ++j) {
    if (sv->a_xoff[j] < 0) continue;
    const ServeStream& r = sv->st[sv->a_idx[j]];
    const int32_t Bj = sv->a_rest[j] ? r.Br : r.B;
    const int64_t row = (int64_t)sv->a_n[j] * Bj;
    const int64_t s0 = sv->a_k0[j] * Bj;
    // a rest block may reach past the input: zeros there
    const int64_t avail = std::min(row, std::max<int64_t>(0, r.n_in * r.B - s0));
    float* dst = sv->x_pin[buf] + sv->a_xoff[j];
    for (int c = 0; c < r.C; ++c) {
      std::memcpy(dst + c * row, r.x + c * r.x_cs + s0, (size_t)avail * 4);
      if (avail < row) std::memset(dst + c * row + avail, 0, (size_t)(row - avail) * 4);
    }
  }
  if (n_ops) {
    OutOp* o = reinterpret_cast<OutOp*>(reinterpret_cast<unsigned char*>(sv->x_pin[buf]) + ops_off);
    size_t q = 0;
    for (size_t j = 0; j < m; ++j) {
      if (sv->a_rest[j]) continue;
      const ServeStream& r = sv->st[sv->a_idx[j]];
      const int32_t len = sv->a_n[j] * r.B;
      OutOp op{sv->y_dev + sv->a_yoff[j], sv->y_pin_dev[buf] + sv->a_yoff[j], nullptr, len, r.C, 1, 0, len, 0};
      if (r.rs) {
        // ring index of the first output that gets a rest output (outputs
        // before sample H get none)
        const int64_t skip = std::min<int64_t>(len, std::max<int64_t>(0, r.H - sv->a_k0[j] * r.B));
        if (skip < len) {
          op.z = r.z;
          op.Z = r.Z;
          op.skip = (int32_t)skip;
          op.p0 = (int32_t)((sv->a_k0[j] * r.B + skip - r.H) % r.Z);
        }
      }
      o[q++] = op;
    }
  }
  // pool step arguments: head ranges read and write the staging (packed
  // channels); rest ranges read the staging and write into the ring
  sv->a_x.resize(m);
  sv->a_y.resize(m);
  sv->a_xcs.resize(m);
  sv->a_ycs.resize(m);
  for (size_t j = 0; j < m; ++j) {
    const ServeStream& r = sv->st[sv->a_idx[j]];
    sv->a_x[j] = sv->a_xoff[j] >= 0 ? sv->x_dev + sv->a_xoff[j] : nullptr;
    sv->a_xcs[j] = 0;
    if (sv->a_rest[j]) {
      sv->a_y[j] = r.z + (sv->a_k0[j] * r.Br) % r.Z;
      sv->a_ycs[j] = r.Z;
    } else {
      sv->a_y[j] = sv->y_dev + sv->a_yoff[j];
      sv->a_ycs[j] = 0;
    }
  }
  if (!sv->fl.active) {
    rc = anchor_clock(sv, hs);
    if (rc != TACHES_OK) return rc;
  }
  const double t_launch = clock_s(sv);
  const int evk = sv->ev_next;
  {
    hipError_t e = hipEventRecord(sv->ev_beg[evk], hs);
    if (e == hipSuccess && x_floats > 0)
      e = hipMemcpyAsync(sv->x_dev, sv->x_pin[buf], x_floats * 4, hipMemcpyHostToDevice, hs);
    if (e != hipSuccess) return taches::set_error(TACHES_EDEVICE, "serving: input copy: %s", hipGetErrorString(e));
  }
  rc = taches_pool_step_strided(sv->pool, (int32_t)m, sv->a_s.data(), sv->a_x.data(), sv->a_xcs.data(),
                                sv->a_y.data(), sv->a_ycs.data(), sv->a_n.data());
  if (rc != TACHES_OK) return rc;
  // the step is committed on the host: from here on, state advances even if
  // a later call reports an error
  for (size_t j = 0; j < m; ++j) {
    ServeStream& r = sv->st[sv->a_idx[j]];
    (sv->a_rest[j] ? r.r_next : r.next) = sv->a_k0[j] + sv->a_n[j];
  }
  sv->ev_next = (evk + 1) % taches_server::kEv;
  {
    hipError_t e = hipSuccess;
    if (n_ops) {
      const OutOp* dops = reinterpret_cast<const OutOp*>(reinterpret_cast<unsigned char*>(sv->x_dev) + ops_off);
      hipLaunchKernelGGL(k_out, dim3((unsigned)n_ops), dim3(256), 0, hs, dops);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(sv->ev[evk], hs);
    if (e != hipSuccess) return taches::set_error(TACHES_EDEVICE, "serving: output pass: %s", hipGetErrorString(e));
  }
  const double t_queued = clock_s(sv);
  // ---- the new step's book-keeping; finished streams leave the server ----
  Flight nf;
  nf.active = true;
  nf.buf = buf;
  nf.ev = evk;
  nf.ranges.reserve(m);
  int64_t blocks = 0, macs = 0, max_n = 0;
  int32_t heads = 0;
  for (size_t j = 0; j < m; ++j) {
    const ServeStream& r = sv->st[sv->a_idx[j]];
    const int32_t n = sv->a_n[j];
    const bool rest = sv->a_rest[j] != 0;
    if ((rest ? sv->a_k0[j] < r.r_in : sv->a_k0[j] < r.n_in)) {
      taches_info inf;
      if (taches_get_info(rest ? r.rs : r.s, &inf) == TACHES_OK)
        macs += (int64_t)n * (rest ? r.Br : r.B) * inf.active_len * r.C;
    }
    if (rest) continue;
    ++heads;
    blocks += n;
    max_n = std::max<int64_t>(max_n, n);
    nf.ranges.push_back(FlightRange{r.tag, r.y, r.y_cs, r.C, r.B, sv->a_k0[j], n, sv->a_yoff[j], r.start_s, now,
                                    sv->a_k0[j] + n >= r.n_total});
  }
  for (size_t i = sv->st.size(); i-- > 0;) {
    if (sv->st[i].next >= sv->st[i].n_total) {
      sv->done.push_back(std::move(sv->st[i]));
      sv->st[i] = std::move(sv->st.back());
      sv->st.pop_back();
    }
  }
  // ---- then wait for the previous step (the device works on this one) ----
  rc = complete_flight(sv);
  sv->fl = std::move(nf);
  sv->tick_buf ^= 1;
  if (rc != TACHES_OK) return rc;
  const double done = clock_s(sv);
  info.next_due_s = next_due();
  info.streams = heads;
  info.blocks = blocks;
  info.done_s = done;
  info.host_ms = (t_launch - now) * 1e3;
  info.step_ms = (done - now) * 1e3;
  sv->stats.ticks += 1;
  sv->stats.blocks += blocks;
  sv->stats.macs += macs;
  sv->stats.busy_s += done - now;
  sv->stats.gather_s += t_launch - now;
  sv->stats.launch_s += t_queued - t_launch;
  sv->stats.max_blocks_in_a_range = std::max(sv->stats.max_blocks_in_a_range, max_n);
  sv->stats.bytes_in += (int64_t)x_floats * 4;
  sv->stats.bytes_out += (int64_t)yf * 4;
  if (out) *out = info;
  return TACHES_OK;
}

int taches_server_take_finished(taches_server* sv, int64_t* tags, int32_t cap) {
  if (!sv || (cap > 0 && !tags) || cap < 0) return taches::set_error(TACHES_EINVAL, "bad arguments");
  const int32_t n = (int32_t)std::min<size_t>(cap, sv->finished.size());
  std::copy(sv->finished.begin(), sv->finished.begin() + n, tags);
  sv->finished.erase(sv->finished.begin(), sv->finished.begin() + n);
  return n;
}

int taches_server_take_latencies(taches_server* sv, float* latency_s, int32_t* block_size, int32_t cap) {
  if (!sv || cap < 0 || (cap > 0 && (!latency_s || !block_size))) return taches::set_error(TACHES_EINVAL, "bad arguments");
  const int32_t n = (int32_t)std::min<size_t>(cap, sv->lat_s.size());
  std::copy(sv->lat_s.begin(), sv->lat_s.begin() + n, latency_s);
  std::copy(sv->lat_B.begin(), sv->lat_B.begin() + n, block_size);
  sv->lat_s.erase(sv->lat_s.begin(), sv->lat_s.begin() + n);
  sv->lat_B.erase(sv->lat_B.begin(), sv->lat_B.begin() + n);
  return n;
}

int taches_server_stream_state(taches_server* sv, int64_t tag, int64_t* next_block, int64_t* swap_blocks, int32_t cap) {
  if (!sv || !next_block || cap < 0 || (cap > 0 && !swap_blocks)) return taches::set_error(TACHES_EINVAL, "bad arguments");
  const ServeStream* r = find_tag(sv, tag, true);
  if (!r) return taches::set_error(TACHES_EINVAL, "serving: tag %lld not registered", (long long)tag);
  *next_block = r->next;
  const int32_t n = (int32_t)std::min<size_t>(cap, r->swap_blocks.size());
  std::copy(r->swap_blocks.begin(), r->swap_blocks.begin() + n, swap_blocks);
  return (int)r->swap_blocks.size();
}

int taches_server_get_stats(const taches_server* sv, taches_server_stats* out) {
  if (!sv || !out) return taches::set_error(TACHES_EINVAL, "bad arguments");
  *out = sv->stats;
  out->streams = (int32_t)sv->st.size();
  return TACHES_OK;
}

}  // extern "C"
