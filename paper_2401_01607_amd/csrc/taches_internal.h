// Internal declarations shared by the runtime and the kernels of libtaches.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "taches.h"

namespace taches {

// Longest run of input samples whose products are summed in FP32 before the
// sum is added to the tail accumulator.  Each block is cut into
// ceil(B / CHUNK_MAX) chunks of near-equal length; chunk boundaries depend
// only on B, so a block gives the same partial sums whether it is processed
// alone or inside a multi-block call.
constexpr int CHUNK_MAX = 256;

// IR of one block: device pointer to L FP32 taps (plus BF16 hi/lo copies for
// the split path).
struct BlockIR {
  const float* h;
  const uint16_t* h_hi;
  const uint16_t* h_lo;
  int32_t L;
  int32_t pad_;
};

// Device memory reached through pointers loaded from memory (call tables,
// per-block IR tables) would otherwise be accessed with flat instructions,
// which also count against the LDS wait counter: every LDS wait of a kernel's
// inner loop would then wait for its global prefetches too.  The kernels
// therefore access global memory through global-address-space pointers.
#define GLB __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const GLB T* gr(const T* p) { return (const GLB T*)p; }
template <typename T>
__device__ __forceinline__ GLB T* gw(T* p) { return (GLB T*)p; }
__device__ __forceinline__ BlockIR load_ir(const BlockIR* tab, int i) {
  const GLB BlockIR* e = gr(tab) + i;
  BlockIR r;
  r.h = e->h;
  r.h_hi = e->h_hi;
  r.h_lo = e->h_lo;
  r.L = e->L;
  r.pad_ = 0;
  return r;
}

// One stream-call of the gather kernels: n_blocks blocks of one stream.
//  Outputs n in [0, n_out) are computed relative to the slot at `head`:
//    acc(n) = tail(n) [if n < live_in] + the partial sums of every chunk of
//             this call that reaches n, added in chunk order;
//  n < S:  y[n] = acc(n) (rounded to FP32) and the slot is cleared;
//  n >= S: the slot keeps acc(n) for later calls.
struct GatherCall {
  const float* x;        // [C][x_cstride] planar input, nullptr = all zero
  float* y;              // [C][y_cstride] planar output
  void* ring;            // [C][ring_cstride] tail (float or double)
  const BlockIR* irs;    // per-block IR table (device), nullptr = ir0 for all;
                         // with ctab: one entry per IR slot
  const int32_t* ctab;   // chunk table (device) when an IR takes over inside a
                         // block, nullptr = regular chunks: first chunk of each
                         // block [n_blocks + 1], then {first sample, length,
                         // slot} per chunk
  BlockIR ir0;
  int64_t x_cstride, y_cstride, ring_cstride;
  int32_t S;             // input samples of the call = n_blocks * B
  int32_t B;             // block size
  int32_t n_blocks;
  int32_t cpb;           // chunks per block
  int32_t Rcap;          // ring slots
  int32_t head;          // ring slot of output n = 0
  int32_t live_in;       // slots (from head) holding pending sums
  int32_t n_out;         // outputs to produce (>= S)
  int32_t Lmax_call;     // longest IR used by the call's blocks
  int32_t channels;
  // split-BF16 path only: per-chunk hi/lo input fragments and padded channels
  uint16_t* xs_hi;
  uint16_t* xs_lo;
  int32_t cpad;
  int32_t tile_order;    // gather path: 0 = XCD-grouped, 1 = center-out, 2 = launch order
};

// One unit of batched work: output tiles tile .. tile+count-1 of one channel
// of one call.
struct WorkItem {
  int32_t call;    // index into the GatherCall table
  int32_t channel;
  int32_t tile;    // first output tile (tile size fixed by the kernel's R)
  int32_t count;   // number of consecutive tiles
};

// Kernel launchers (k_gather.hip).  r in {4, 8, 12, 16}, w in {1, 2, 4}.
hipError_t launch_gather(const GatherCall& call, bool tail_fp64, int r, int w, hipStream_t st);
// Packed table of a batched launch: this header, then the sub-tables at the
// given byte offsets (GatherCall[n_calls], int32 tail-is-FP64[n_calls],
// WorkItem[n_items] in the order workgroups take them, and an int32 counter
// of items taken, 0 in the table the host copies in).
struct BatchHeader {
  int32_t off_calls, off_fp64, off_items, off_next;
  int32_t n_items, pad_;
};
// mixed: some calls of the table keep an FP64 tail.
hipError_t launch_gather_batched(unsigned char* table_dev, int n_wg, int r, bool mixed, hipStream_t st);

inline int tile_outputs(int r) { return 64 * r; }

// Resident one-wave workgroups per CU of the batched gather kernel.
int gather_batched_waves_per_cu(int r, bool mixed);

// IR staging for the split-BF16 path (k_toeplitz.hip): hi = RN_bf16(h),
// lo = RN_bf16(h - hi), bit patterns stored as uint16.
hipError_t launch_split_bf16(const float* h, uint16_t* hi, uint16_t* lo, int L, hipStream_t st);

// Multichannel split-BF16 Toeplitz-block MFMA (k_toeplitz.hip).  The tail of
// a split stream is laid out [slot][cpad] (channel fastest).
hipError_t launch_toeplitz(const GatherCall& call, bool tail_fp64, hipStream_t st);
bool split_supported(const taches_config& cfg);
int split_cpad(int channels);

// Split-BF16 streams of one pool step that share a kernel class (tail type,
// padded channel count): their calls and prefix sums in the pool table.
struct ToeplitzBatch {
  int64_t off_calls;   // GatherCall[n_calls]
  int64_t off_tiles;   // int32 tile_start[n_calls + 1]: first output tile of each call
  int64_t off_frags;   // int64 frag_start[n_calls + 1]: first input fragment of each call
  int64_t n_tiles;     // tile_start[n_calls]
  int64_t n_frags;     // frag_start[n_calls]
  int32_t n_calls;
  int32_t pad_;
};
// Output rows of one Toeplitz workgroup tile.
int toeplitz_rows_per_tile();
// The split-input launch (if any input) and the Toeplitz launch of one class.
hipError_t launch_toeplitz_batched(const unsigned char* table_dev, const ToeplitzBatch& b, bool tail_fp64, bool wide,
                                   hipStream_t st);

// Runtime services for the serving tick (taches_runtime.hip): set the
// thread's error message and return `code`; the HIP stream a pool's steps
// run on; whether a stream is attached to a pool.
int set_error(int code, const char* fmt, ...);
hipStream_t pool_stream(const taches_pool* p);
bool stream_in_pool(const taches_stream* s, const taches_pool* p);

// FP32 FMA issue ceiling of the device (k_diag.hip): TFLOP/s reached by
// independent v_fmac_f32 chains.
hipError_t measure_fmac_ceiling(int device, double* tflops);

}  // namespace taches
