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
// needs and the chunk's len input samples are staged in LDS (per wave),
// loaded into registers one chunk ahead.  A
// lane keeps two R-tap windows of h in registers; for each group of R input
// samples it loads one new window (ds_read_b128, plus one ds_read_b64 when
// R is not a multiple of 4) and the group's R input samples (uniform
// broadcasts of the same widths), then issues R*R FMAs.  R is even.  The LDS
// copy of h pads every R-float row so that the lanes' 16-byte window reads
// fall in distinct banks; each group of R input samples starts on a 16-byte
// boundary.
#include <algorithm>

#include "taches_internal.h"

namespace taches {
namespace {

// All LDS data lives in one dynamic array indexed by 32-bit float offsets.
extern __shared__ __attribute__((aligned(16))) float g_lds[];
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef float vf4u __attribute__((ext_vector_type(4))) __attribute__((aligned(4)));


typedef float vf2 __attribute__((ext_vector_type(2)));
typedef float vf2u __attribute__((ext_vector_type(2))) __attribute__((aligned(4)));

__device__ __forceinline__ vf4 lds_read4(int off) { return *reinterpret_cast<const vf4*>(&g_lds[off]); }
__device__ __forceinline__ void lds_write4(int off, vf4 v) { *reinterpret_cast<vf4*>(&g_lds[off]) = v; }
__device__ __forceinline__ vf2 lds_read2(int off) { return *reinterpret_cast<const vf2*>(&g_lds[off]); }
__device__ __forceinline__ void lds_write2(int off, vf2 v) { *reinterpret_cast<vf2*>(&g_lds[off]) = v; }

template <int R>
struct Geo {
  static_assert(R % 2 == 0 && R >= 4, "R must be even");
  static constexpr int T = 64 * R;                           // outputs per wave tile
  static constexpr int LP = (CHUNK_MAX + R - 1) / R * R;     // longest padded chunk
  static constexpr int NW = T + LP;                          // staged taps (max)
  static constexpr int R4 = (R + 3) / 4 * 4;                 // R rounded up to 16 bytes
  // floats per R-tap window row in LDS: an odd number of 16-byte units, so
  // the 16-byte reads of consecutive lanes hit distinct banks
  static constexpr int ROW = (R4 / 4) % 2 == 1 ? R4 : R4 + 4;
  static constexpr int HF = (NW / R) * ROW;                  // LDS floats for h
  static constexpr int XG = R4;                              // LDS floats per group of R samples
  static constexpr int WF = HF + (LP / R) * XG;              // + input samples
};

// R consecutive floats of LDS starting at a 16-byte-aligned offset.
template <int R>
__device__ __forceinline__ void lds_read_row(int off, float (&v)[R]) {
#pragma unroll
  for (int j = 0; j < R; j += 4) {
    if (j + 4 <= R) {
      const vf4 q = lds_read4(off + j);
      v[j] = q.x;
      v[j + 1] = q.y;
      v[j + 2] = q.z;
      v[j + 3] = q.w;
    } else {
      const vf2 q = lds_read2(off + j);
      v[j] = q.x;
      v[j + 1] = q.y;
    }
  }
}

template <int R>
__device__ __forceinline__ void lds_write_row(int off, const float (&v)[R]) {
#pragma unroll
  for (int j = 0; j < R; j += 4) {
    if (j + 4 <= R)
      lds_write4(off + j, vf4{v[j], v[j + 1], v[j + 2], v[j + 3]});
    else
      lds_write2(off + j, vf2{v[j], v[j + 1]});
  }
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

// Center-out order: the middle tile first, then alternately right and left
// of it.  In a call that spans many blocks the tiles near both ends of the
// output range reach fewer input samples; launching them last lets the
// workgroup dispatcher hand the light tiles to the CUs that already hold
// heavy ones.
__device__ __forceinline__ int center_out(int id, int n) {
  const int mid = (n - 1) >> 1;
  return (id & 1) ? mid + ((id + 1) >> 1) : mid - (id >> 1);
}

// Load the R taps of one window; `src` points at its first padded float.
template <int R>
__device__ __forceinline__ void load_win(int src, float (&v)[R]) { lds_read_row<R>(src, v); }

// The R input samples of group g.
template <int R>
__device__ __forceinline__ void load_x(int xs, int g, float (&v)[R]) { lds_read_row<R>(xs + g * Geo<R>::XG, v); }

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
//   Only groups [g0, g1) are summed (a run of several chunks staged together
//   is computed one chunk at a time).
template <int R>
__device__ __forceinline__ void chunk_compute(int hs, int xs, int lane, int G, int g0, int g1, float (&p)[R]) {
  constexpr int ROW = Geo<R>::ROW;
  const int wl = hs + lane * ROW;
  float X[R], Y[R], xv[R];
  load_win<R>(wl + (G - 1 - g0) * ROW, X);
  load_win<R>(wl + (G - g0) * ROW, Y);
  int g = g0;
  for (; g + 2 <= g1; g += 2) {
    load_x<R>(xs, g, xv);
    fma_group<R>(xv, X, Y, p);                                 // group g:   A = X, B = Y
    load_win<R>(wl + (G - 2 - g) * ROW, Y);
    load_x<R>(xs, g + 1, xv);
    fma_group<R>(xv, Y, X, p);                                 // group g+1: A = Y, B = X
    // window of group g+2 (a harmless in-bounds read when the loop ends)
    load_win<R>(hs + max(lane + G - 3 - g, 0) * ROW, X);
  }
  if (g < g1) {
    load_x<R>(xs, g, xv);
    fma_group<R>(xv, X, Y, p);
  }
}

// Samples staged together in one wave's LDS region: chunk `ck` alone, or
// (one-wave tiles) a run of `nsub` consecutive whole blocks of B samples.
struct ChunkGeo {
  int m_lo, len, len_pad;
  int ck, nsub;
  BlockIR ir;
  bool reaches;
  uint32_t nz;     // bit j: block j of the unit (or the single chunk, bit 0) has a nonzero sample
};

// Where chunk ck lies and which IR it uses: the part of a chunk's geometry
// that comes from memory (the per-block IR table, or the chunk table).
struct ChunkDesc {
  int m_lo, len;
  BlockIR ir;
};

__device__ __forceinline__ ChunkDesc chunk_desc(const GatherCall& d, int ck) {
  ChunkDesc c;
  if (d.ctab) {
    // an IR takes over inside some block: chunks come from the table
    const GLB int32_t* cd = gr(d.ctab) + (d.n_blocks + 1) + 3 * ck;
    c.m_lo = cd[0];
    c.len = cd[1];
    c.ir = load_ir(d.irs, cd[2]);
  } else {
    const int b = ck / d.cpb;
    const int i = ck - b * d.cpb;
    c.m_lo = b * d.B + (i * d.B) / d.cpb;
    c.len = b * d.B + ((i + 1) * d.B) / d.cpb - c.m_lo;
    c.ir = d.irs ? load_ir(d.irs, b) : d.ir0;
  }
  return c;
}

template <int R>
__device__ __forceinline__ ChunkGeo chunk_geo(const ChunkDesc& c, int ck, int n0) {
  ChunkGeo g;
  g.m_lo = c.m_lo;
  g.len = c.len;
  g.ir = c.ir;
  const int m_hi = g.m_lo + g.len;
  g.len_pad = (g.len + R - 1) / R * R;
  // the chunk's taches cover outputs [m_lo, m_hi - 1 + L - 1]
  g.reaches = g.len > 0 && g.m_lo <= n0 + Geo<R>::T - 1 && m_hi + g.ir.L - 2 >= n0;
  g.ck = ck;
  g.nsub = 1;
  g.nz = ~0u;
  return g;
}

// The staging unit that starts at chunk ck (one-wave tiles).  When whole
// blocks are short (kmax = CHUNK_MAX / B > 1, one chunk per block, B a
// multiple of R), up to kmax consecutive blocks that use the same IR are
// staged as one unit: one IR window of T + kmax*B - 1 taps serves them all,
// so short blocks no longer pay a full staging round each.  Their partial
// sums are still formed and added to the tail one block at a time.
template <int R>
__device__ __forceinline__ ChunkGeo unit_geo(const GatherCall& d, int ck, int ck_end, int kmax, int n0) {
  ChunkGeo g;
  if (ck >= ck_end) {
    g.m_lo = g.len = g.len_pad = 0;
    g.ck = ck;
    g.nsub = 0;
    g.reaches = false;
    g.nz = 0u;
    return g;
  }
  if (kmax == 1) return chunk_geo<R>(chunk_desc(d, ck), ck, n0);
  g.ir = d.irs ? load_ir(d.irs, ck) : d.ir0;
  int e = min(ck + kmax, ck_end);
  if (d.irs) {
    for (int b = ck + 1; b < e; ++b) {
      const GLB BlockIR* o = gr(d.irs) + b;
      if (o->h != g.ir.h || o->L != g.ir.L) {
        e = b;
        break;
      }
    }
  }
  g.ck = ck;
  g.nsub = e - ck;
  g.nz = ~0u;
  g.m_lo = ck * d.B;
  g.len = g.nsub * d.B;
  g.len_pad = g.len;
  g.reaches = g.m_lo <= n0 + Geo<R>::T - 1 && g.m_lo + g.len + g.ir.L - 2 >= n0;
  return g;
}

// 16- and 8-byte loads from a 4-byte-aligned global address.
__device__ __forceinline__ vf4u load4(const GLB float* p) { return *reinterpret_cast<const GLB vf4u*>(p); }
__device__ __forceinline__ vf2u load2(const GLB float* p) { return *reinterpret_cast<const GLB vf2u*>(p); }

// One chunk's staged data on its way from global memory to LDS: each lane
// holds two R-tap rows of the IR window (rows lane and lane + 64) and up to
// XPL input samples.  Loading it one round ahead hides the global-memory
// latency behind the FMAs of the current chunk.
template <int R>
struct Prefetch {
  static constexpr int XPL = (Geo<R>::LP + 63) / 64;
  float hrow[2][R];
  float xv[XPL];
};

// Row r of the staged window holds taps base + r*R .. base + r*R + R - 1,
// base = n0 - m_lo - len_pad + 1; taps outside [0, L) are zero.
template <int R>
__device__ __forceinline__ void chunk_load(const ChunkGeo& g, const GLB float* __restrict__ xc, int n0, int lane,
                                           Prefetch<R>& pf) {
  const int base = n0 - g.m_lo - g.len_pad + 1;
  const int rows = (Geo<R>::T + g.len_pad) / R;
  const GLB float* __restrict__ h = gr(g.ir.h);
  const int L = g.ir.L;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int row = lane + 64 * k;
    const int j0 = base + row * R;
    if (row < rows && j0 >= 0 && j0 + R <= L) {
#pragma unroll
      for (int e = 0; e < R; e += 4) {
        if (e + 4 <= R) {
          const vf4u q = load4(h + j0 + e);
          pf.hrow[k][e] = q.x;
          pf.hrow[k][e + 1] = q.y;
          pf.hrow[k][e + 2] = q.z;
          pf.hrow[k][e + 3] = q.w;
        } else {
          const vf2u q = load2(h + j0 + e);
          pf.hrow[k][e] = q.x;
          pf.hrow[k][e + 1] = q.y;
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < R; ++e) {
        const int j = j0 + e;
        pf.hrow[k][e] = (row < rows && j >= 0 && j < L) ? h[j] : 0.f;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < Prefetch<R>::XPL; ++k) {
    const int s = lane + 64 * k;
    pf.xv[k] = s < g.len ? xc[g.m_lo + s] : 0.f;
  }
}

// Exact-zero bypass (the paper skips the tache of a zero input sample,
// Section 3.2): while its samples are stored, the wave records which blocks
// of the unit hold a nonzero sample.  A chunk of zeros adds only zero
// products, so skipping its multiply-adds and its addition to the tail
// leaves every output unchanged (up to the sign of an exact zero).
template <int R>
__device__ __forceinline__ uint32_t nonzero_blocks(const ChunkGeo& g, int lane, const Prefetch<R>& pf, int B) {
  if (g.nsub <= 1) {
    bool any = false;
#pragma unroll
    for (int k = 0; k < Prefetch<R>::XPL; ++k) any |= (lane + 64 * k < g.len) && pf.xv[k] != 0.f;
    return __any(any) ? 1u : 0u;
  }
  uint32_t m = 0;
  for (int j = 0; j < g.nsub; ++j) {
    bool any = false;
#pragma unroll
    for (int k = 0; k < Prefetch<R>::XPL; ++k) {
      const int s = lane + 64 * k;
      any |= s >= j * B && s < (j + 1) * B && pf.xv[k] != 0.f;
    }
    if (__any(any)) m |= 1u << j;
  }
  return m;
}

template <int R>
__device__ __forceinline__ void chunk_store(const ChunkGeo& g, int lane, const Prefetch<R>& pf, int hs, int xs) {
  const int rows = (Geo<R>::T + g.len_pad) / R;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int row = lane + 64 * k;
    if (row < rows) lds_write_row<R>(hs + row * Geo<R>::ROW, pf.hrow[k]);
  }
#pragma unroll
  for (int k = 0; k < Prefetch<R>::XPL; ++k) {
    const int s = lane + 64 * k;
    if (s < g.len_pad) {
      if constexpr (Geo<R>::XG == R)
        g_lds[xs + s] = pf.xv[k];
      else
        g_lds[xs + (s / R) * Geo<R>::XG + s % R] = pf.xv[k];
    }
  }
}

// One-wave tiles: a lane's run of tail slots moves as 16-byte vectors when it
// neither wraps around the ring nor crosses the live, emitted or written
// boundary (every lane but a few at those boundaries); the others move value
// by value.  In short calls (a few blocks per stream, as in serving steps)
// the tail traffic dominates the tile.  Multi-wave tiles own a few outputs
// per lane and keep the value-by-value form, which schedules better there.
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4))) __attribute__((aligned(4)));
  static constexpr int N = 4;
};
template <>
struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2))) __attribute__((aligned(8)));
  static constexpr int N = 2;
};

template <typename T, int Q>
__device__ __forceinline__ void load_run(const GLB T* p, T (&v)[Q]) {
  constexpr int N = Vec16<T>::N;
  if constexpr (Q % N == 0) {
#pragma unroll
    for (int k = 0; k < Q / N; ++k) {
      const typename Vec16<T>::type u = *reinterpret_cast<const GLB typename Vec16<T>::type*>(p + k * N);
#pragma unroll
      for (int j = 0; j < N; ++j) v[k * N + j] = u[j];
    }
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = p[q];
  }
}

template <typename T, int Q>
__device__ __forceinline__ void store_run(GLB T* p, const T (&v)[Q]) {
  constexpr int N = Vec16<T>::N;
  if constexpr (Q % N == 0) {
#pragma unroll
    for (int k = 0; k < Q / N; ++k) {
      typename Vec16<T>::type u;
#pragma unroll
      for (int j = 0; j < N; ++j) u[j] = v[k * N + j];
      *reinterpret_cast<GLB typename Vec16<T>::type*>(p + k * N) = u;
    }
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) p[q] = v[q];
  }
}

// One output tile of one channel of one call.  W waves share the tile; wave
// w handles chunks w, w+W, ... of each round and the partial sums are added
// to the accumulators in chunk order after every round.  Each wave keeps the
// accumulators of its share of a lane's R outputs (outputs
// floor(w*R/W) .. floor((w+1)*R/W) - 1) and adds only those partial sums,
// then writes those outputs.
template <int R, int W, typename TailT>
__device__ __forceinline__ void gather_tile(const GatherCall& d, int c, int tile) {
  constexpr int T = Geo<R>::T;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int hs = w * Geo<R>::WF;           // LDS float offsets of this wave's region
  const int xs = hs + Geo<R>::HF;
  const int pbuf = W * Geo<R>::WF;         // [W][64][R4], used when W > 1

  const int n0 = tile * T;
  constexpr int QM = (R + W - 1) / W;      // most accumulators a wave owns per lane
  constexpr bool EVEN = R % W == 0;
  const int q0 = (w * R) / W;              // the first of this wave's
  const int qn = EVEN ? QM : ((w + 1) * R) / W - q0;   // and their number (wave-uniform)
  const int nq = n0 + lane * R + q0;
  GLB TailT* ring = gw(reinterpret_cast<TailT*>(d.ring)) + (int64_t)c * d.ring_cstride;

  // slot of the lane's first output (its run is contiguous unless it wraps)
  int s0 = d.head + nq;
  if (s0 >= d.Rcap) s0 -= d.Rcap;
  TailT acc[QM];
  if (W == 1 && qn == QM && nq + QM <= d.live_in && s0 + QM <= d.Rcap) {
    load_run<TailT, QM>(ring + s0, acc);
  } else {
#pragma unroll
    for (int q = 0; q < QM; ++q) {
      const int n = nq + q;
      TailT v = 0;
      if (q < qn && n < d.live_in) {
        int slot = d.head + n;
        if (slot >= d.Rcap) slot -= d.Rcap;
        v = ring[slot];
      }
      acc[q] = v;
    }
  }

  if (d.x != nullptr) {
    const GLB float* __restrict__ xc = gr(d.x) + (int64_t)c * d.x_cstride;
    const int lo = n0 - (d.Lmax_call - 1);
    const int b_first = lo <= 0 ? 0 : lo / d.B;
    const int b_last = min(d.n_blocks - 1, (n0 + T - 1) / d.B);
    int c_first = b_first * d.cpb;
    int nch = b_first <= b_last ? (b_last - b_first + 1) * d.cpb : 0;
    if (d.ctab && b_first <= b_last) {
      c_first = gr(d.ctab)[b_first];
      nch = gr(d.ctab)[b_last + 1] - c_first;
    }
    // `gc` is staged in LDS, `gn` (the wave's next unit) is in registers.
    // A wave's LDS region is private and LDS operations of one wave complete
    // in program order, so storing `gn` after computing `gc` needs no
    // barrier.
    Prefetch<R> pf;
    if constexpr (W == 1) {
      const int kmax = (!d.ctab && d.cpb == 1 && d.B % R == 0) ? max(1, CHUNK_MAX / d.B) : 1;
      const int c_end = c_first + nch;
      ChunkGeo gc = unit_geo<R>(d, c_first, c_end, kmax, n0);
      if (gc.reaches) {
        chunk_load<R>(gc, xc, n0, lane, pf);
        gc.nz = nonzero_blocks<R>(gc, lane, pf, d.B);
        chunk_store<R>(gc, lane, pf, hs, xs);
      }
      ChunkGeo gn = unit_geo<R>(d, gc.ck + gc.nsub, c_end, kmax, n0);
      if (gn.reaches) chunk_load<R>(gn, xc, n0, lane, pf);
      while (gc.nsub > 0) {
        if (gc.reaches) {
          const int G = gc.len_pad / R;
          const int gs = G / gc.nsub;        // groups per block (all of G for a single chunk)
          const int L = gc.ir.L;
          for (int j = 0; j < gc.nsub; ++j) {
            const int m0 = gc.m_lo + j * d.B;
            if (gc.nsub > 1 && !(m0 <= n0 + T - 1 && m0 + d.B + L - 2 >= n0)) continue;
            if (!((gc.nz >> j) & 1u)) continue;
            float p[R];
#pragma unroll
            for (int r = 0; r < R; ++r) p[r] = 0.f;
            chunk_compute<R>(hs, xs, lane, G, j * gs, (j + 1) * gs, p);
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += (TailT)p[r];
          }
        }
        if (gn.reaches) {
          gn.nz = nonzero_blocks<R>(gn, lane, pf, d.B);
          chunk_store<R>(gn, lane, pf, hs, xs);
        }
        gc = gn;
        gn = unit_geo<R>(d, gc.ck + gc.nsub, c_end, kmax, n0);
        if (gn.reaches) chunk_load<R>(gn, xc, n0, lane, pf);
      }
    } else {
    // Wave w handles chunks w, w + W, w + 2W, ... and the partial sums of
    // each round are added in chunk order.  The descriptor of the wave's
    // chunk two rounds ahead is loaded a round before its IR window, so the
    // window loads need not wait for it.
    ChunkGeo gc, gn;
    gc.reaches = gn.reaches = false;
    if (w < nch) gc = chunk_geo<R>(chunk_desc(d, c_first + w), c_first + w, n0);
    if (gc.reaches) {
      chunk_load<R>(gc, xc, n0, lane, pf);
      gc.nz = nonzero_blocks<R>(gc, lane, pf, d.B);
      chunk_store<R>(gc, lane, pf, hs, xs);
    }
    if (w + W < nch) gn = chunk_geo<R>(chunk_desc(d, c_first + w + W), c_first + w + W, n0);
    ChunkDesc dn{};
    if (w + 2 * W < nch) dn = chunk_desc(d, c_first + w + 2 * W);
    if (gn.reaches) chunk_load<R>(gn, xc, n0, lane, pf);
    for (int base = 0; base < nch; base += W) {
      float p[R];
#pragma unroll
      for (int r = 0; r < R; ++r) p[r] = 0.f;
      if (gc.reaches && gc.nz) chunk_compute<R>(hs, xs, lane, gc.len_pad / R, 0, gc.len_pad / R, p);
      if (gn.reaches) {
        gn.nz = nonzero_blocks<R>(gn, lane, pf, d.B);
        chunk_store<R>(gn, lane, pf, hs, xs);
      }
      gc = gn;
      gn.reaches = false;
      if (base + 2 * W + w < nch) gn = chunk_geo<R>(dn, c_first + base + 2 * W + w, n0);
      if (base + 3 * W + w < nch) dn = chunk_desc(d, c_first + base + 3 * W + w);
      if (gn.reaches) chunk_load<R>(gn, xc, n0, lane, pf);
      {
        lds_write_row<R>(pbuf + (w * 64 + lane) * Geo<R>::R4, p);
        __syncthreads();
        const int nv = min(W, nch - base);
        for (int v = 0; v < nv; ++v) {
          const int src = pbuf + (v * 64 + lane) * Geo<R>::R4 + q0;
          if constexpr (EVEN && QM % 4 == 0) {
#pragma unroll
            for (int q = 0; q < QM; q += 4) {
              const vf4 t = lds_read4(src + q);
              acc[q] += (TailT)t.x;
              acc[q + 1] += (TailT)t.y;
              acc[q + 2] += (TailT)t.z;
              acc[q + 3] += (TailT)t.w;
            }
          } else {
#pragma unroll
            for (int q = 0; q < QM; ++q)
              if (q < qn) acc[q] += (TailT)g_lds[src + q];
          }
        }
        __syncthreads();
      }
    }
    }
  }

  {
    GLB float* yc = gw(d.y) + (int64_t)c * d.y_cstride;
    const bool whole = W == 1 && qn == QM && nq + QM <= d.n_out && s0 + QM <= d.Rcap;
    if (whole && nq + QM <= d.S) {          // all emitted: outputs out, slots cleared
      float yv[QM];
      TailT z[QM];
#pragma unroll
      for (int q = 0; q < QM; ++q) {
        yv[q] = (float)acc[q];
        z[q] = (TailT)0;
      }
      store_run<float, QM>(yc + nq, yv);
      store_run<TailT, QM>(ring + s0, z);
    } else if (whole && nq >= d.S) {        // all kept in the tail
      store_run<TailT, QM>(ring + s0, acc);
    } else {
#pragma unroll
      for (int q = 0; q < QM; ++q) {
        const int n = nq + q;
        if (q < qn && n < d.n_out) {
          int slot = d.head + n;
          if (slot >= d.Rcap) slot -= d.Rcap;
          if (n < d.S) {
            yc[n] = (float)acc[q];
            ring[slot] = (TailT)0;
          } else {
            ring[slot] = acc[q];
          }
        }
      }
    }
  }
}

template <int R, int W>
constexpr int lds_bytes() {
  return 4 * (W * Geo<R>::WF + (W > 1 ? W * 64 * Geo<R>::R4 : 0));
}

template <int R, int W, typename TailT>
__global__ __launch_bounds__(64 * W) void k_gather(GatherCall d, int n_tiles) {
  const int tile = d.tile_order == 0 ? xcd_remap(blockIdx.x, n_tiles)
                   : d.tile_order == 1 ? center_out(blockIdx.x, n_tiles) : (int)blockIdx.x;
  gather_tile<R, W, TailT>(d, blockIdx.y, tile);
}

// Batched: one packed table (header, call descriptors, per-call tail type,
// work items, a counter).  The persistent workgroups take items one at a
// time from the shared counter (a work queue; the host lists the items in
// the order they should be taken: largest first when sizes differ much),
// so a workgroup that finishes early takes more, whatever the items really
// cost.  Each item is a run of consecutive output tiles of one channel of
// one call; each call's tail type is chosen per stream.  Which workgroup
// computes a tile does not change its result (one wave computes a tile,
// summing in the fixed chunk order).
// MIXED: some calls keep an FP64 tail (both tail types compiled in);
// otherwise the FP32-tail code alone, which needs fewer registers.
template <int R, bool MIXED>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_gather_batched(
    unsigned char* __restrict__ table) {
  const BatchHeader hd = *reinterpret_cast<const BatchHeader*>(table);
  const GatherCall* __restrict__ calls = reinterpret_cast<const GatherCall*>(table + hd.off_calls);
  const int32_t* __restrict__ call_fp64 = reinterpret_cast<const int32_t*>(table + hd.off_fp64);
  const WorkItem* __restrict__ items = reinterpret_cast<const WorkItem*>(table + hd.off_items);
  int* next = reinterpret_cast<int*>(table + hd.off_next);
  const int lane = threadIdx.x & 63;
  auto take = [&]() {
    int v = 0;
    if (lane == 0) v = atomicAdd(next, 1);
    return __builtin_amdgcn_readfirstlane(v);
  };
  int it = take();
  while (it < hd.n_items) {
    const int it_next = take();   // in flight while this item runs
    const WorkItem wi = items[it];
    const GatherCall& d = calls[wi.call];   // read in place (a local copy would spill)
    const bool f64 = MIXED && call_fp64[wi.call] != 0;
    for (int t = wi.tile; t < wi.tile + wi.count; ++t) {
      if constexpr (MIXED) {
        if (f64)
          gather_tile<R, 1, double>(d, wi.channel, t);
        else
          gather_tile<R, 1, float>(d, wi.channel, t);
      } else {
        gather_tile<R, 1, float>(d, wi.channel, t);
      }
      __syncthreads();
    }
    it = it_next;
  }
}

template <int R, int W>
hipError_t launch_rw(const GatherCall& call, bool fp64, hipStream_t st) {
  const int n_tiles = (call.n_out + Geo<R>::T - 1) / Geo<R>::T;
  dim3 grid(n_tiles, call.channels);
  constexpr int shmem = lds_bytes<R, W>();
  if (fp64)
    hipLaunchKernelGGL((k_gather<R, W, double>), grid, dim3(64 * W), shmem, st, call, n_tiles);
  else
    hipLaunchKernelGGL((k_gather<R, W, float>), grid, dim3(64 * W), shmem, st, call, n_tiles);
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
hipError_t launch_batched_r(unsigned char* table_dev, int n_wg, bool mixed, hipStream_t st) {
  constexpr int shmem = lds_bytes<R, 1>();
  if (mixed)
    hipLaunchKernelGGL((k_gather_batched<R, true>), dim3(n_wg), dim3(64), shmem, st, table_dev);
  else
    hipLaunchKernelGGL((k_gather_batched<R, false>), dim3(n_wg), dim3(64), shmem, st, table_dev);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gather(const GatherCall& call, bool tail_fp64, int r, int w, hipStream_t st) {
  if (call.n_out <= 0 || call.channels <= 0) return hipSuccess;
  switch (r) {
    case 4: return launch_r<4>(call, tail_fp64, w, st);
    case 8: return launch_r<8>(call, tail_fp64, w, st);
    case 12: return launch_r<12>(call, tail_fp64, w, st);
    case 14: return launch_r<14>(call, tail_fp64, w, st);
    case 16: return launch_r<16>(call, tail_fp64, w, st);
    default: return hipErrorInvalidValue;
  }
}

// Resident one-wave workgroups per CU, from the register count and LDS use
// the runtime reports for the kernel: each SIMD holds 512 registers per
// lane (in granules of 8) and at most 8 waves; a CU has 4 SIMDs and 160 KB
// of LDS.  Computed once per kernel (the planner asks on every step).
template <int R, bool MIXED>
int batched_occupancy() {
  static int cached = 0;
  if (cached) return cached;
  hipFuncAttributes a{};
  int per_cu = 8;
  if (hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_gather_batched<R, MIXED>)) == hipSuccess &&
      a.numRegs > 0) {
    const int regs = (a.numRegs + 7) / 8 * 8;
    const int waves_simd = std::min(8, 512 / regs);
    const int lds = lds_bytes<R, 1>() + (int)a.sharedSizeBytes;
    per_cu = std::max(1, std::min(4 * waves_simd, lds > 0 ? 163840 / lds : 32));
  }
  cached = per_cu;
  return per_cu;
}

int gather_batched_waves_per_cu(int r, bool mixed) {
  switch (r) {
    case 4: return mixed ? batched_occupancy<4, true>() : batched_occupancy<4, false>();
    case 8: return mixed ? batched_occupancy<8, true>() : batched_occupancy<8, false>();
    case 12: return mixed ? batched_occupancy<12, true>() : batched_occupancy<12, false>();
    case 16: return mixed ? batched_occupancy<16, true>() : batched_occupancy<16, false>();
    default: return 8;
  }
}

hipError_t launch_gather_batched(unsigned char* table_dev, int n_wg, int r, bool mixed, hipStream_t st) {
  if (n_wg <= 0) return hipSuccess;
  switch (r) {
    case 4: return launch_batched_r<4>(table_dev, n_wg, mixed, st);
    case 8: return launch_batched_r<8>(table_dev, n_wg, mixed, st);
    case 12: return launch_batched_r<12>(table_dev, n_wg, mixed, st);
    case 16: return launch_batched_r<16>(table_dev, n_wg, mixed, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace taches
