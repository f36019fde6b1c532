// Split-BF16 path for channels that share one impulse response.
//
// For a tile of output slots n and a chunk of input samples m the taches of
// all channels c form one dense contraction:
//   P[n][c] = sum_m A[n][m] * X[m][c],   A[n][m] = h[n - m]  (Toeplitz in h),
// which runs on the MFMA units (v_mfma_f32_32x32x16_bf16).  FP32 values are
// split as v = hi + lo with hi = RN_bf16(v), lo = RN_bf16(v - hi); the
// product is taken as A_hi X_hi + A_hi X_lo + A_lo X_hi (the A_lo X_lo term,
// below 2^-16 |A||X|, is dropped) with FP32 accumulation inside the chunk.
// Each chunk's FP32 partial is then added to the tail accumulator (FP64 for
// long IRs) in chunk order, as on the FP32 gather path.  The paper points at
// GPUs for the per-channel matrix form and names precision as the key factor
// (Section 4.2); this extends its requantization count (Sections 5.3-5.5)
// to a measured error against an FP64 reference.
//
// Data layout:
//  - IR: FP32 taps plus BF16 hi/lo copies (split once per set_ir).
//  - Input: per call, every chunk of every channel is split into hi/lo and
//    stored as [chunk][k-group of 8 samples][channel (padded)][8] BF16 so a
//    lane's MFMA B fragment (8 consecutive samples of one channel) is one
//    aligned 16-byte load and 32 lanes read 512 contiguous bytes.
//  - Tail: [slot][channel (padded)], so the 32 lanes of an MFMA result
//    column group write contiguous memory.
//  - LDS: the IR window a tile needs, reversed, in 8 copies shifted by one
//    element each: the A fragment of a lane (8 taps, descending) is then
//    one aligned 16-byte read from the copy that matches its alignment.  The
//    window is loaded into registers one chunk ahead, stored once, and the
//    shifted copies are built from it inside LDS.
#include <algorithm>

#include "taches_internal.h"

namespace taches {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int MT = 128;                    // output slots per workgroup (MT / 32 waves x 32 rows)
constexpr int NT = 2 * MT;                 // threads per workgroup
constexpr int KC = CHUNK_MAX;              // longest chunk (samples)
constexpr int CP_LEN = MT + KC + 16;       // elements per shifted copy (>= MT + KC + 7)
constexpr int REV_LEN = CP_LEN + 16;       // reversed window staged once per chunk
constexpr int REV_PER_THREAD = (REV_LEN + NT - 1) / NT;
static_assert(CP_LEN % 8 == 0 && 2 * (CP_LEN / 8) <= NT, "copy-building needs one group per thread");

// Round an FP32 value to the nearest BF16 (ties to even); returns the bits.
__device__ __forceinline__ uint16_t bf16_rn(float v) {
  uint32_t u = __float_as_uint(v);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__global__ void k_split_bf16(const float* __restrict__ h, uint16_t* __restrict__ hi, uint16_t* __restrict__ lo, int L) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < L; i += gridDim.x * blockDim.x) {
    const float v = h[i];
    const uint16_t a = bf16_rn(v);
    hi[i] = a;
    lo[i] = bf16_rn(v - bf16_to_f(a));
  }
}

__device__ __forceinline__ void chunk_span(const GatherCall& d, int ck, int& m_lo, int& len, int& b) {
  b = ck / d.cpb;
  const int i = ck - b * d.cpb;
  m_lo = b * d.B + (i * d.B) / d.cpb;
  len = b * d.B + ((i + 1) * d.B) / d.cpb - m_lo;
}

// Fragment t of a call's input, t = (chunk * 32 + k-group of 8 samples) *
// cpad + padded channel: split the 8 samples into hi/lo BF16 and store them
// as one 16-byte fragment each.
__device__ __forceinline__ void split_fragment(const GatherCall& d, int64_t t) {
  const int cpad = d.cpad;
  {
    const int c = (int)(t % cpad);
    const int kg = (int)((t / cpad) % 32);
    const int ck = (int)(t / ((int64_t)cpad * 32));
    int m_lo, len, b;
    chunk_span(d, ck, m_lo, len, b);
    uint16_t hv[8], lv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int s = kg * 8 + j;
      float v = 0.f;
      if (c < d.channels && s < len) v = gr(d.x)[(int64_t)c * d.x_cstride + m_lo + s];
      hv[j] = bf16_rn(v);
      lv[j] = bf16_rn(v - bf16_to_f(hv[j]));
    }
    u32x4 ph, pl;
    ph.x = hv[0] | ((uint32_t)hv[1] << 16); ph.y = hv[2] | ((uint32_t)hv[3] << 16);
    ph.z = hv[4] | ((uint32_t)hv[5] << 16); ph.w = hv[6] | ((uint32_t)hv[7] << 16);
    pl.x = lv[0] | ((uint32_t)lv[1] << 16); pl.y = lv[2] | ((uint32_t)lv[3] << 16);
    pl.z = lv[4] | ((uint32_t)lv[5] << 16); pl.w = lv[6] | ((uint32_t)lv[7] << 16);
    *reinterpret_cast<GLB u32x4*>(gw(d.xs_hi) + t * 8) = ph;
    *reinterpret_cast<GLB u32x4*>(gw(d.xs_lo) + t * 8) = pl;
  }
}

// One thread per fragment of one call.
__global__ __launch_bounds__(256) void k_split_input(GatherCall d, int n_chunks) {
  const int64_t total = (int64_t)n_chunks * 32 * d.cpad;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x)
    split_fragment(d, t);
}

// Index k with start[k] <= v < start[k + 1] (start ascending, start[0] = 0).
template <typename T>
__device__ __forceinline__ int find_call(const T* start, int n, int64_t v) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((int64_t)gr(start)[mid] <= v) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Every input fragment of the calls of one pool-step class.
__global__ __launch_bounds__(256) void k_split_input_batched(const GatherCall* calls, const int64_t* frag_start,
                                                              int n_calls) {
  const int64_t total = gr(frag_start)[n_calls];
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int k = find_call(frag_start, n_calls, t);
    const GatherCall d = calls[k];
    split_fragment(d, t - gr(frag_start)[k]);
  }
}

// Launch order of the output tiles of one call: the middle tile first, then
// alternately right and left of it.  Tile work follows the number of input
// samples that reach the tile, which rises from the first tile, is flat
// where every sample reaches and falls to the last, so this order launches
// the heaviest tiles first and leaves the light ones to fill the end.
// Workgroups go to the 8 XCDs round-robin in launch order, so every XCD
// gets the same mix of heavy and light tiles (giving each XCD a contiguous
// range of tiles instead left the XCDs that held the middle of the output
// with 1.75 times the mean work in a 64-channel call of 2^18 taps), and the
// tiles running together on one XCD are near each other, so they read
// nearly the same input chunks through its L2.
__device__ __forceinline__ int center_out(int id, int n) {
  const int mid = (n - 1) >> 1;
  return (id & 1) ? mid + ((id + 1) >> 1) : mid - (id >> 1);
}

// A thread's share of one chunk's reversed IR window (hi and lo halves).
struct RevPrefetch {
  uint16_t hi[REV_PER_THREAD], lo[REV_PER_THREAD];
};

__device__ __forceinline__ void rev_load(const BlockIR& ir, int top, int tid, RevPrefetch& pf) {
#pragma unroll
  for (int j = 0; j < REV_PER_THREAD; ++j) {
    const int hidx = top - (tid + NT * j);
    const bool ok = tid + NT * j < REV_LEN && hidx >= 0 && hidx < ir.L;
    pf.hi[j] = ok ? gr(ir.h_hi)[hidx] : (uint16_t)0;
    pf.lo[j] = ok ? gr(ir.h_lo)[hidx] : (uint16_t)0;
  }
}

// Wave layout: the workgroup's MT x cpad result is cut into 4 wave tiles of
// NM*32 rows x NN*32 channels.  Every K-step a wave reads NM A fragments
// (LDS) and NN pairs of B fragments (global, hi and lo) and issues 3*NM*NN
// MFMAs, so taller wave tiles (NM = 2) halve the global B traffic per MFMA.
template <typename TailT, int NM, int NN>
__device__ __forceinline__ void toeplitz_tile(const GatherCall& d, const int tile) {
  __shared__ __attribute__((aligned(16))) uint16_t cp_hi[8 * CP_LEN];
  __shared__ __attribute__((aligned(16))) uint16_t cp_lo[8 * CP_LEN];
  __shared__ __attribute__((aligned(16))) uint16_t rev_hi[REV_LEN];
  __shared__ __attribute__((aligned(16))) uint16_t rev_lo[REV_LEN];
  const int tid = threadIdx.x;
  const int l = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i = l & 31;   // row within the wave's 32-row MFMA tile (A) / column (B, D)
  const int kg = l >> 5;  // k-group of 8 within a 16-deep K-step
  const int n0 = tile * MT;
  const int cpad = d.cpad;
  GLB TailT* ring = gw(reinterpret_cast<TailT*>(d.ring));
  // this wave's tile: rows r0 .. r0 + 32*NM - 1, channels c0 .. c0 + 32*NN - 1
  constexpr int WN = 64 / (32 * NN) > 0 ? 64 / (32 * NN) : 1;   // wave columns for 64 channels
  const int wn = (cpad == 64) ? w % WN : 0;
  const int wm = (cpad == 64) ? w / WN : w;
  const int r0 = 32 * NM * wm;
  const int c0 = 32 * NN * wn;
  // accumulators: NM x NN 32x32 result tiles; lane l holds column l%32 and
  // rows 8*(q/4) + 4*(l/32) + q%4 of each tile
  TailT acc[NM][NN][16];
#pragma unroll
  for (int mt = 0; mt < NM; ++mt)
#pragma unroll
    for (int nt = 0; nt < NN; ++nt)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int n = n0 + r0 + 32 * mt + 8 * (q >> 2) + 4 * kg + (q & 3);
        const int c = c0 + 32 * nt + i;
        TailT v = 0;
        if (n < d.live_in && c < cpad) {
          int slot = d.head + n;
          if (slot >= d.Rcap) slot -= d.Rcap;
          v = ring[(int64_t)slot * cpad + c];
        }
        acc[mt][nt][q] = v;
      }

  RevPrefetch pf;
  bool pf_valid = false;
  int pf_ck = -1;
  // B fragments (8 samples of channel c0 + 32*nt + i, k-group 2t + kg) go
  // through a ring of three register buffers, two K-steps ahead; the first
  // two K-steps of a chunk are loaded during the previous chunk's tail
  struct BF {
    bf16x8 h[NN], l[NN];
  };
  BF bf[3];
  int b_pre = -1;   // chunk whose K-steps 0 and 1 are already in bf[0], bf[1]
  auto load_b_at = [&](int chunk, int t, BF& f) {
    const int64_t xo = (((int64_t)chunk * 32 + 2 * t + kg) * cpad + c0 + i) * 8;
#pragma unroll
    for (int nt = 0; nt < NN; ++nt) {
      f.h[nt] = *reinterpret_cast<const GLB bf16x8*>(gr(d.xs_hi) + xo + nt * 32 * 8);
      f.l[nt] = *reinterpret_cast<const GLB bf16x8*>(gr(d.xs_lo) + xo + nt * 32 * 8);
    }
  };
  if (d.x != nullptr) {
    const int lo = n0 - (d.Lmax_call - 1);
    const int b_first = lo <= 0 ? 0 : lo / d.B;
    const int b_last = min(d.n_blocks - 1, (n0 + MT - 1) / d.B);
    const int c_first = b_first * d.cpb;
    const int nch = b_first <= b_last ? (b_last - b_first + 1) * d.cpb : 0;
    for (int k = 0; k < nch; ++k) {
      const int ck = c_first + k;
      int m_lo, len, b;
      chunk_span(d, ck, m_lo, len, b);
      const BlockIR ir = d.irs ? load_ir(d.irs, b) : d.ir0;
      if (len <= 0 || m_lo > n0 + MT - 1 || m_lo + len + ir.L - 2 < n0) continue;  // uniform
      const int chp = (len + 15) & ~15;
      __syncthreads();  // the previous chunk's reads of the copies are done
      // 1) the reversed window rev[u] = h[n0 - m_lo + MT - 1 - u] (hi and lo),
      //    loaded into registers one chunk earlier (or now, for the first)
      if (!pf_valid || pf_ck != ck) rev_load(ir, n0 - m_lo + MT - 1, tid, pf);
#pragma unroll
      for (int j = 0; j < REV_PER_THREAD; ++j) {
        const int u = tid + NT * j;
        if (u < REV_LEN) {
          rev_hi[u] = pf.hi[j];
          rev_lo[u] = pf.lo[j];
        }
      }
      __syncthreads();
      // 2) eight copies shifted by s = 0..7: cp_s[v] = rev[v + s]; one thread
      //    per 8-element group reads 16 elements and writes 8 aligned groups
      if (tid < 2 * (CP_LEN / 8)) {
        const bool lo_set = tid >= CP_LEN / 8;
        const int v0 = 8 * (lo_set ? tid - CP_LEN / 8 : tid);
        const uint16_t* src = lo_set ? rev_lo : rev_hi;
        uint16_t* dst = lo_set ? cp_lo : cp_hi;
        const uint4 a = *reinterpret_cast<const uint4*>(src + v0);
        const uint4 b = *reinterpret_cast<const uint4*>(src + v0 + 8);
        const uint32_t dw[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int sh = 0; sh < 8; ++sh) {
          uint32_t o[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            if (sh % 2 == 0) {
              o[k] = dw[sh / 2 + k];
            } else {
              const int m = (sh - 1) / 2 + k;
              o[k] = (dw[m] >> 16) | (dw[m + 1] << 16);
            }
          }
          *reinterpret_cast<uint4*>(dst + sh * CP_LEN + v0) = make_uint4(o[0], o[1], o[2], o[3]);
        }
      }
      __syncthreads();
      // 3) the next reaching chunk: its window is prefetched into registers
      //    after this chunk's last B loads are issued (the load counter is
      //    in order, so earlier it would delay this chunk's first K-steps)
      pf_valid = false;
      int nx_ck = -1, nx_top = 0, nx_len = 0;
      BlockIR nx_ir{};
      for (int k2 = k + 1; k2 < nch; ++k2) {
        int m2, len2, b2;
        chunk_span(d, c_first + k2, m2, len2, b2);
        const BlockIR ir2 = d.irs ? load_ir(d.irs, b2) : d.ir0;
        if (len2 <= 0 || m2 > n0 + MT - 1 || m2 + len2 + ir2.L - 2 < n0) continue;
        nx_ck = c_first + k2;
        nx_top = n0 - m2 + MT - 1;
        nx_len = len2;
        nx_ir = ir2;
        break;
      }
      auto prefetch_next = [&]() {
        if (nx_ck >= 0) {
          rev_load(nx_ir, nx_top, tid, pf);
          pf_ck = nx_ck;
          pf_valid = true;
        }
      };
      f32x16 p[NM][NN];
#pragma unroll
      for (int mt = 0; mt < NM; ++mt)
#pragma unroll
        for (int nt = 0; nt < NN; ++nt) p[mt][nt] = f32x16{};
      const int ksteps = chp >> 4;
      auto load_b = [&](int t, BF& f) { load_b_at(ck, t, f); };
      // A fragments: taps for rows n0+r0+32mt+i and samples m_lo+16t+8kg+j
      struct AF {
        bf16x8 h[NM], l[NM];
      };
      auto load_a = [&](int t, AF& af) {
#pragma unroll
        for (int mt = 0; mt < NM; ++mt) {
          const int a = MT - 1 - r0 - 32 * mt - i + 16 * t + 8 * kg;
          const int aoff = (a & 7) * CP_LEN + (a & ~7);
          af.h[mt] = *reinterpret_cast<const bf16x8*>(cp_hi + aoff);
          af.l[mt] = *reinterpret_cast<const bf16x8*>(cp_lo + aoff);
        }
      };
      auto mfmas = [&](const AF& af, const BF& f) {
#pragma unroll
        for (int mt = 0; mt < NM; ++mt)
#pragma unroll
          for (int nt = 0; nt < NN; ++nt) {
            p[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af.h[mt], f.h[nt], p[mt][nt], 0, 0, 0);
            p[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af.h[mt], f.l[nt], p[mt][nt], 0, 0, 0);
            p[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af.l[mt], f.h[nt], p[mt][nt], 0, 0, 0);
          }
      };
      auto kstep = [&](int t, const BF& f) {
        AF af;
        load_a(t, af);
        mfmas(af, f);
      };
      if (ksteps == KC / 16) {
        // The scheduling barriers keep each K-step's loads ahead of the
        // previous steps' MFMAs: without them the compiler sinks every load
        // to just before its first use and each K-step waits for memory.
        if (b_pre != ck) {
          load_b(0, bf[0]);
          load_b(1, bf[1]);
        }
        if constexpr (NM == 2) {
          // A is Toeplitz: the fragment of the lower 32-row tile at K-step t
          // is the upper tile's fragment of K-step t - 2 (32 rows down = 32
          // samples later).  Only the upper tile's fragments come from LDS
          // (one K-step ahead), kept in a four-slot ring; the lower tile
          // reads LDS for K-steps 0 and 1 only.
          struct A1 {
            bf16x8 h, l;
          };
          auto load_a0 = [&](int t, int mt, A1& f) {
            const int a = MT - 1 - r0 - 32 * mt - i + 16 * t + 8 * kg;
            const int aoff = (a & 7) * CP_LEN + (a & ~7);
            f.h = *reinterpret_cast<const bf16x8*>(cp_hi + aoff);
            f.l = *reinterpret_cast<const bf16x8*>(cp_lo + aoff);
          };
          A1 up[4], low01[2];
          load_a0(0, 0, up[0]);
          load_a0(0, 1, low01[0]);
#pragma unroll
          for (int t = 0; t < KC / 16; ++t) {
            if (t + 2 < KC / 16) load_b(t + 2, bf[(t + 2) % 3]);
            if (t == KC / 16 - 3) prefetch_next();
            if (t + 1 < KC / 16) load_a0(t + 1, 0, up[(t + 1) % 4]);
            if (t + 1 < 2) load_a0(t + 1, 1, low01[t + 1]);
            __builtin_amdgcn_sched_barrier(0);
            AF af;
            af.h[0] = up[t % 4].h;
            af.l[0] = up[t % 4].l;
            af.h[1] = t < 2 ? low01[t < 2 ? t : 0].h : up[(t + 2) % 4].h;
            af.l[1] = t < 2 ? low01[t < 2 ? t : 0].l : up[(t + 2) % 4].l;
            mfmas(af, bf[t % 3]);
            __builtin_amdgcn_sched_barrier(0);
          }
        } else {
          // A fragments come from LDS one K-step ahead (two-slot ring)
          AF af[2];
          load_a(0, af[0]);
#pragma unroll
          for (int t = 0; t < KC / 16; ++t) {
            if (t + 2 < KC / 16) load_b(t + 2, bf[(t + 2) % 3]);
            if (t == KC / 16 - 3) prefetch_next();
            if (t + 1 < KC / 16) load_a(t + 1, af[(t + 1) % 2]);
            __builtin_amdgcn_sched_barrier(0);
            mfmas(af[t % 2], bf[t % 3]);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      } else {
        for (int t = 0; t < ksteps; ++t) {
          load_b(t, bf[0]);
          kstep(t, bf[0]);
        }
        prefetch_next();
      }
      // the next chunk's first two K-steps fly during the fold and staging
      b_pre = -1;
      if (nx_ck >= 0 && nx_len == KC) {
        load_b_at(nx_ck, 0, bf[0]);
        load_b_at(nx_ck, 1, bf[1]);
        b_pre = nx_ck;
      }
#pragma unroll
      for (int mt = 0; mt < NM; ++mt)
#pragma unroll
        for (int nt = 0; nt < NN; ++nt)
#pragma unroll
          for (int q = 0; q < 16; ++q) acc[mt][nt][q] += (TailT)p[mt][nt][q];
    }
  }

#pragma unroll
  for (int mt = 0; mt < NM; ++mt)
#pragma unroll
    for (int nt = 0; nt < NN; ++nt)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int n = n0 + r0 + 32 * mt + 8 * (q >> 2) + 4 * kg + (q & 3);
        const int c = c0 + 32 * nt + i;
        if (n < d.n_out && c < cpad) {
          int slot = d.head + n;
          if (slot >= d.Rcap) slot -= d.Rcap;
          if (n < d.S) {
            if (c < d.channels) gw(d.y)[(int64_t)c * d.y_cstride + n] = (float)acc[mt][nt][q];
            ring[(int64_t)slot * cpad + c] = (TailT)0;
          } else {
            ring[(int64_t)slot * cpad + c] = acc[mt][nt][q];
          }
        }
      }
}

template <typename TailT, int NM, int NN>
__global__ __launch_bounds__(NT) void k_toeplitz(GatherCall d, int n_tiles) {
  toeplitz_tile<TailT, NM, NN>(d, center_out(blockIdx.x, n_tiles));
}

// The calls of one pool-step class: workgroup i takes tile i - tile_start[k]
// of call k (tile_start: prefix sums of the calls' tile counts), in launch
// order, so consecutive tiles (and calls) go to different XCDs.
template <typename TailT, int NM, int NN>
__global__ __launch_bounds__(NT) void k_toeplitz_batched(const GatherCall* calls, const int32_t* tile_start,
                                                         int n_calls) {
  const int id = blockIdx.x;
  const int k = find_call(tile_start, n_calls, id);
  const GatherCall d = calls[k];
  toeplitz_tile<TailT, NM, NN>(d, id - gr(tile_start)[k]);
}

template <typename TailT, int NM, int NN>
hipError_t launch_batched_class(const unsigned char* tab, const ToeplitzBatch& b, hipStream_t st) {
  const GatherCall* calls = reinterpret_cast<const GatherCall*>(tab + b.off_calls);
  if (b.n_frags > 0) {
    const int blocks = (int)std::min<int64_t>((b.n_frags + 255) / 256, 4096);
    hipLaunchKernelGGL(k_split_input_batched, dim3(blocks), dim3(256), 0, st, calls,
                       reinterpret_cast<const int64_t*>(tab + b.off_frags), b.n_calls);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (b.n_tiles > 0)
    hipLaunchKernelGGL((k_toeplitz_batched<TailT, NM, NN>), dim3((unsigned)b.n_tiles), dim3(NT), 0, st, calls,
                       reinterpret_cast<const int32_t*>(tab + b.off_tiles), b.n_calls);
  return hipGetLastError();
}

}  // namespace

int toeplitz_rows_per_tile() { return MT; }

hipError_t launch_toeplitz_batched(const unsigned char* table_dev, const ToeplitzBatch& b, bool tail_fp64, bool wide,
                                   hipStream_t st) {
  if (b.n_calls <= 0) return hipSuccess;
  if (tail_fp64)
    return wide ? launch_batched_class<double, 2, 1>(table_dev, b, st) : launch_batched_class<double, 1, 1>(table_dev, b, st);
  return wide ? launch_batched_class<float, 2, 1>(table_dev, b, st) : launch_batched_class<float, 1, 1>(table_dev, b, st);
}

hipError_t launch_split_bf16(const float* h, uint16_t* hi, uint16_t* lo, int L, hipStream_t st) {
  if (L <= 0) return hipSuccess;
  const int blocks = (L + 255) / 256 < 1024 ? (L + 255) / 256 : 1024;
  hipLaunchKernelGGL(k_split_bf16, dim3(blocks), dim3(256), 0, st, h, hi, lo, L);
  return hipGetLastError();
}

bool split_supported(const taches_config& cfg) { return cfg.channels >= 1 && cfg.channels <= 64; }

int split_cpad(int channels) { return channels <= 32 ? 32 : 64; }

hipError_t launch_toeplitz(const GatherCall& call, bool tail_fp64, hipStream_t st) {
  if (call.n_out <= 0) return hipSuccess;
  if (call.x) {
    const int n_chunks = call.n_blocks * call.cpb;
    const int64_t total = (int64_t)n_chunks * 32 * call.cpad;
    const int blocks = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_split_input, dim3(blocks), dim3(256), 0, st, call, n_chunks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int n_tiles = (call.n_out + MT - 1) / MT;
  // 32 channels: one 32x32 tile per wave; 64 channels: 64 rows x 32 channels
  // per wave (each B fragment then feeds twice as many MFMAs: the vector
  // memory traffic of the B fragments is what bounds this loop)
  const bool wide = call.cpad > 32;
  if (tail_fp64) {
    if (wide)
      hipLaunchKernelGGL((k_toeplitz<double, 2, 1>), dim3(n_tiles), dim3(NT), 0, st, call, n_tiles);
    else
      hipLaunchKernelGGL((k_toeplitz<double, 1, 1>), dim3(n_tiles), dim3(NT), 0, st, call, n_tiles);
  } else {
    if (wide)
      hipLaunchKernelGGL((k_toeplitz<float, 2, 1>), dim3(n_tiles), dim3(NT), 0, st, call, n_tiles);
    else
      hipLaunchKernelGGL((k_toeplitz<float, 1, 1>), dim3(n_tiles), dim3(NT), 0, st, call, n_tiles);
  }
  return hipGetLastError();
}

}  // namespace taches
