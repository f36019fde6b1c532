// Gather kernels for the taches convolution on gfx950 (FP32 vector ALUs).
//
// The paper's buffer form (Section 4.2) scatters each input sample's tache
// e0 * h into a circular residue.  On the GPU the same sums are regrouped by
// output slot: a wave owns 64*R consecutive output slots (R per lane) and
// walks the input samples that reach them, so every slot has exactly one
// writer and no atomics are needed.
//
// Summation order (fixed, independent of tiling and of how blocks are
// grouped into calls): the input is cut into chunks (each block into
// ceil(B/CHUNK_MAX) near-equal pieces).  For one output n and one chunk, the
// products x[m]*h[n-m] are accumulated with fused multiply-adds in
// increasing m, starting from 0 (the per-MAC requantization of Section 5.5,
// one rounding per MAC).  The chunk sums are then added to the tail value of
// slot n in chunk order, in the tail's type (FP32, or FP64 for long IRs).
//
// Data movement per chunk and tile: the T + len - 1 taps of h that the tile
// needs and the chunk's len input samples are staged in LDS (per wave).  A
// lane keeps two R-tap windows of h in registers; for each group of R input
// samples it loads one new window (R/4 ds_read_b128) and the group's R
// input samples (uniform ds_read_b128 broadcasts), then issues R*R FMAs.
// The LDS copy of h pads every R-float row so that the lanes' 16-byte
// window reads fall in distinct banks.
#include "taches_internal.h"

namespace taches {
namespace {

template <int R>
struct Geo {
  static_assert(R % 4 == 0, "R must be a multiple of 4");
  static constexpr int T = 64 * R;                           // outputs per wave tile
  static constexpr int LP = (CHUNK_MAX + R - 1) / R * R;     // longest padded chunk
  static constexpr int NW = T + LP;                          // staged taps (max)
  // padded floats per R-tap window row: a multiple of 4 with an odd number of
  // 16-byte units, so the 16-byte reads of consecutive lanes hit distinct banks
  static constexpr int ROW = ((R + 4) / 4) % 2 == 1 ? R + 4 : R + 8;
  static constexpr int HF = (NW / R) * ROW;                  // LDS floats for h
  static constexpr int WF = HF + LP;                         // + input samples
};

template <int R>
__device__ __forceinline__ int hphys(int i) {
  return (int)(((unsigned)i / R) * Geo<R>::ROW + ((unsigned)i % R));
}

// Map the launch order of workgroups to tiles so that consecutive tiles run
// on the same XCD (workgroups are dispatched to the 8 XCDs round-robin):
// neighbouring tiles share most of their IR window and input samples, which
// then stay in one XCD's L2.
__device__ __forceinline__ int xcd_remap(int id, int n) {
  const int x = id & 7;
  const int k = id >> 3;
  const int q = n >> 3, rem = n & 7;
  return x * q + (x < rem ? x : rem) + k;
}

// Load the R taps of one window; `src` points at its first padded float.
template <int R>
__device__ __forceinline__ void load_win(const float* src, float (&v)[R]) {
#pragma unroll
  for (int j = 0; j < R; j += 4) {
    const float4 q = *reinterpret_cast<const float4*>(src + j);
    v[j] = q.x;
    v[j + 1] = q.y;
    v[j + 2] = q.z;
    v[j + 3] = q.w;
  }
}

template <int R>
__device__ __forceinline__ void load_x(const float* xs, int s0, float (&v)[R]) {
#pragma unroll
  for (int j = 0; j < R; j += 4) {
    const float4 q = *reinterpret_cast<const float4*>(xs + s0 + j);
    v[j] = q.x;
    v[j + 1] = q.y;
    v[j + 2] = q.z;
    v[j + 3] = q.w;
  }
}

// One group of R input samples: for each sample t (in order) and each of
// the lane's R outputs r, p[r] += x[t] * h[(lane window) + r - t].
// A holds the window of taps (r - t + R - 1) in [0, R), Bw those in [R, 2R-1).
template <int R>
__device__ __forceinline__ void fma_group(const float (&xv)[R], const float (&A)[R],
                                          const float (&Bw)[R], float (&p)[R]) {
#pragma unroll
  for (int t = 0; t < R; ++t) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int idx = r - t + R - 1;
      const float hv = idx < R ? A[idx] : Bw[idx - R];
      p[r] = __builtin_fmaf(xv[t], hv, p[r]);
    }
  }
}

// Partial sums of one staged chunk for the lane's R outputs.
//   hs[i] = h[base + i], base = n0 - m_lo - len_pad + 1; xs[s] = x[m_lo + s].
//   Output n0 + lane*R + r, sample s = g*R + t uses
//   hs[lane*R + (G - 1 - g)*R + (r - t + R - 1)], G = len_pad / R, i.e. the
//   window pair starting at padded row lane + G - 1 - g.
template <int R>
__device__ __forceinline__ void chunk_compute(const float* hs, const float* xs, int lane,
                                              int len_pad, float (&p)[R]) {
  constexpr int ROW = Geo<R>::ROW;
  const int G = len_pad / R;   // wave-uniform
  const float* wl = hs + lane * ROW;
  float X[R], Y[R], xv[R];
  load_win<R>(wl + (G - 1) * ROW, X);
  load_win<R>(wl + G * ROW, Y);
  int g = 0;
  for (; g + 2 <= G; g += 2) {
    load_x<R>(xs, g * R, xv);
    fma_group<R>(xv, X, Y, p);                                 // group g:   A = X, B = Y
    load_win<R>(wl + (G - 2 - g) * ROW, Y);
    load_x<R>(xs, (g + 1) * R, xv);
    fma_group<R>(xv, Y, X, p);                                 // group g+1: A = Y, B = X
    // window of group g+2 (a harmless in-bounds read when the loop ends)
    load_win<R>(wl + max(G - 3 - g, -lane) * ROW, X);
  }
  if (g < G) {
    load_x<R>(xs, g * R, xv);
    fma_group<R>(xv, X, Y, p);
  }
}

struct ChunkGeo {
  int m_lo, len, len_pad;
  BlockIR ir;
  bool reaches;
};

template <int R>
__device__ __forceinline__ ChunkGeo chunk_geo(const GatherCall& d, int ck, int n0) {
  ChunkGeo g;
  const int b = ck / d.cpb;
  const int i = ck - b * d.cpb;
  g.m_lo = b * d.B + (i * d.B) / d.cpb;
  const int m_hi = b * d.B + ((i + 1) * d.B) / d.cpb;
  g.len = m_hi - g.m_lo;
  g.len_pad = (g.len + R - 1) / R * R;
  g.ir = d.irs ? d.irs[b] : d.ir0;
  // the chunk's taches cover outputs [m_lo, m_hi - 1 + L - 1]
  g.reaches = g.len > 0 && g.m_lo <= n0 + Geo<R>::T - 1 && m_hi + g.ir.L - 2 >= n0;
  return g;
}

template <int R>
__device__ __forceinline__ void chunk_stage(const ChunkGeo& g, const float* __restrict__ xc, int n0,
                                            float* hs, float* xs, int lane) {
  const int base = n0 - g.m_lo - g.len_pad + 1;
  const int NW = Geo<R>::T + g.len_pad;
  const float* __restrict__ h = g.ir.h;
  const int L = g.ir.L;
  for (int i = lane; i < NW; i += 64) {
    const int j = base + i;
    const float v = (j >= 0 && j < L) ? h[j] : 0.f;
    hs[hphys<R>(i)] = v;
  }
  for (int s = lane; s < g.len_pad; s += 64) xs[s] = s < g.len ? xc[g.m_lo + s] : 0.f;
}

// One output tile of one channel of one call.  W waves share the tile; wave
// w handles chunks w, w+W, ... of each round and the partial sums are added
// to the accumulators in chunk order after every round.
template <int R, int W, typename TailT>
__device__ __forceinline__ void gather_tile(const GatherCall& d, int c, int tile, float* lds) {
  constexpr int T = Geo<R>::T;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  float* hs = lds + w * Geo<R>::WF;
  float* xs = hs + Geo<R>::HF;
  float* pbuf = lds + W * Geo<R>::WF;  // [W][64][R], used when W > 1

  const int n0 = tile * T;
  const int nb = n0 + lane * R;
  TailT* ring = reinterpret_cast<TailT*>(d.ring) + (int64_t)c * d.ring_cstride;

  TailT acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int n = nb + r;
    TailT v = 0;
    if (n < d.live_in) {
      int slot = d.head + n;
      if (slot >= d.Rcap) slot -= d.Rcap;
      v = ring[slot];
    }
    acc[r] = v;
  }

  if (d.x != nullptr) {
    const float* __restrict__ xc = d.x + (int64_t)c * d.x_cstride;
    const int lo = n0 - (d.Lmax_call - 1);
    const int b_first = lo <= 0 ? 0 : lo / d.B;
    const int b_last = min(d.n_blocks - 1, (n0 + T - 1) / d.B);
    const int c_first = b_first * d.cpb;
    const int nch = b_first <= b_last ? (b_last - b_first + 1) * d.cpb : 0;
    for (int base = 0; base < nch; base += W) {
      const int k = base + w;
      float p[R];
#pragma unroll
      for (int r = 0; r < R; ++r) p[r] = 0.f;
      ChunkGeo g;
      g.reaches = false;
      if (k < nch) {
        g = chunk_geo<R>(d, c_first + k, n0);
        if (g.reaches) chunk_stage<R>(g, xc, n0, hs, xs, lane);
      }
      __syncthreads();
      if (g.reaches) chunk_compute<R>(hs, xs, lane, g.len_pad, p);
      if constexpr (W == 1) {
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] += (TailT)p[r];
      } else {
        float* mine = pbuf + (w * 64 + lane) * R;
#pragma unroll
        for (int r = 0; r < R; r += 4) *reinterpret_cast<float4*>(mine + r) = make_float4(p[r], p[r + 1], p[r + 2], p[r + 3]);
        __syncthreads();
        const int nv = min(W, nch - base);
        for (int v = 0; v < nv; ++v) {
          const float* src = pbuf + (v * 64 + lane) * R;
#pragma unroll
          for (int r = 0; r < R; r += 4) {
            const float4 q = *reinterpret_cast<const float4*>(src + r);
            acc[r] += (TailT)q.x;
            acc[r + 1] += (TailT)q.y;
            acc[r + 2] += (TailT)q.z;
            acc[r + 3] += (TailT)q.w;
          }
        }
        __syncthreads();
      }
    }
  }

  if (w == 0) {
    float* yc = d.y + (int64_t)c * d.y_cstride;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int n = nb + r;
      if (n < d.n_out) {
        int slot = d.head + n;
        if (slot >= d.Rcap) slot -= d.Rcap;
        if (n < d.S) {
          yc[n] = (float)acc[r];
          ring[slot] = (TailT)0;
        } else {
          ring[slot] = acc[r];
        }
      }
    }
  }
}

template <int R, int W, typename TailT>
__global__ __launch_bounds__(64 * W) void k_gather(GatherCall d, int n_tiles) {
  __shared__ __attribute__((aligned(16))) float lds[W * Geo<R>::WF + (W > 1 ? W * 64 * R : 0)];
  const int tile = xcd_remap(blockIdx.x, n_tiles);
  gather_tile<R, W, TailT>(d, blockIdx.y, tile, lds);
}

// Batched: workgroup b walks work items [wg_begin[b], wg_begin[b+1]) of a
// host-built list (largest items first, balanced over workgroups).  Each
// call's tail type is chosen per stream.
template <int R>
__global__ __launch_bounds__(64) void k_gather_batched(const GatherCall* __restrict__ calls,
                                                       const WorkItem* __restrict__ items,
                                                       const int32_t* __restrict__ wg_begin,
                                                       const int32_t* __restrict__ call_fp64) {
  __shared__ __attribute__((aligned(16))) float lds[Geo<R>::WF];
  const int b = blockIdx.x;
  const int it0 = wg_begin[b], it1 = wg_begin[b + 1];
  for (int it = it0; it < it1; ++it) {
    const WorkItem wi = items[it];
    const GatherCall d = calls[wi.call];
    if (call_fp64[wi.call])
      gather_tile<R, 1, double>(d, wi.channel, wi.tile, lds);
    else
      gather_tile<R, 1, float>(d, wi.channel, wi.tile, lds);
    __syncthreads();
  }
}

template <int R, int W>
hipError_t launch_rw(const GatherCall& call, bool fp64, hipStream_t st) {
  const int n_tiles = (call.n_out + Geo<R>::T - 1) / Geo<R>::T;
  dim3 grid(n_tiles, call.channels);
  if (fp64)
    hipLaunchKernelGGL((k_gather<R, W, double>), grid, dim3(64 * W), 0, st, call, n_tiles);
  else
    hipLaunchKernelGGL((k_gather<R, W, float>), grid, dim3(64 * W), 0, st, call, n_tiles);
  return hipGetLastError();
}

template <int R>
hipError_t launch_r(const GatherCall& call, bool fp64, int w, hipStream_t st) {
  switch (w) {
    case 1: return launch_rw<R, 1>(call, fp64, st);
    case 2: return launch_rw<R, 2>(call, fp64, st);
    case 4: return launch_rw<R, 4>(call, fp64, st);
    default: return hipErrorInvalidValue;
  }
}

template <int R>
hipError_t launch_batched_r(const GatherCall* calls_dev, const WorkItem* items_dev, const int32_t* wg_begin_dev,
                            const int32_t* call_fp64_dev, int n_wg, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_batched<R>, dim3(n_wg), dim3(64), 0, st, calls_dev, items_dev, wg_begin_dev,
                     call_fp64_dev);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gather(const GatherCall& call, bool tail_fp64, int r, int w, hipStream_t st) {
  if (call.n_out <= 0 || call.channels <= 0) return hipSuccess;
  switch (r) {
    case 4: return launch_r<4>(call, tail_fp64, w, st);
    case 8: return launch_r<8>(call, tail_fp64, w, st);
    case 12: return launch_r<12>(call, tail_fp64, w, st);
    case 16: return launch_r<16>(call, tail_fp64, w, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gather_batched(const GatherCall* calls_dev, const WorkItem* items_dev,
                                 const int32_t* wg_begin_dev, const int32_t* call_fp64_dev, int n_wg,
                                 int r, hipStream_t st) {
  if (n_wg <= 0) return hipSuccess;
  switch (r) {
    case 4: return launch_batched_r<4>(calls_dev, items_dev, wg_begin_dev, call_fp64_dev, n_wg, st);
    case 8: return launch_batched_r<8>(calls_dev, items_dev, wg_begin_dev, call_fp64_dev, n_wg, st);
    case 12: return launch_batched_r<12>(calls_dev, items_dev, wg_begin_dev, call_fp64_dev, n_wg, st);
    case 16: return launch_batched_r<16>(calls_dev, items_dev, wg_begin_dev, call_fp64_dev, n_wg, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace taches
