/*
 * CPU oracle for the streaming taches convolution.  TEST INFRASTRUCTURE ONLY:
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load or call this library.  The GPU product path never links it and
 * shares no code with it.
 *
 * What it computes (Section 3.2, Eq. 4): every input sample e[n0] adds its
 * "tache" e[n0] * h[n - n0] to the output, and the output is the sum of all
 * taches.  With an impulse response that can change between blocks, the
 * tache of each sample uses the IR that is active when that sample is
 * consumed; taches already in the residue keep ringing with the IR that
 * produced them (Abstract; Section 6).  A queued IR may also take over at a
 * given sample of the next block (the "even sample-by-sample" update of
 * Section 6): the taches of that block's earlier samples use the old IR.
 *
 * How (Section 4.2, buffer form): the not-yet-emitted part of the sum is
 * kept in a circular residue r of Lmax slots; slot (p + k) mod Lmax holds the
 * pending sum of the output k samples after the current one.  For each input
 * sample, in input order:
 *   1. its tache is added: r[(p + k) mod Lmax] += e0 * h[k] for k = 0 .. L-1
 *      (Eq. 4: input sample n0 contributes e0 * h[n - n0] to output n, and
 *      output n = n0 + k sits k slots after the current one);
 *   2. the current output is r[p] (it now holds every tache that reaches it,
 *      its own sample's h[0] term included: zero latency);
 *   3. r[p] is set to 0, ready for the output Lmax samples later;
 *   4. p advances by one slot, modulo Lmax.
 * The residue and index are stream state kept across calls (the residue
 * carries the remaining parts of past taches from one block to the next).
 *
 * Precision.  OR_FP64: residue in double; a product of two floats is exact
 * in double, so only the additions round.  OR_FP32_FMA: residue in float,
 * one rounding per multiply-accumulate (fmaf), the per-MAC requantization
 * model of Section 5.5.  OR_FP32_MULADD: residue in float, product and sum
 * rounded separately.  Build with -ffp-contract=off so that the compiler
 * does not fuse the OR_FP64 and OR_FP32_MULADD loops.
 *
 * Channels: C independent channels share the IR; x and y are planar [C][B].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { OR_FP64 = 0, OR_FP32_FMA = 1, OR_FP32_MULADD = 2 };
enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOIR = -2, OR_ENOMEM = -3 };

typedef struct or_stream {
  int B, Lmax, C, prec;
  int p;                 /* residue index, shared by all channels */
  double *r64;           /* [C][Lmax] */
  float *r32;            /* [C][Lmax] */
  float *active;         /* [Lmax] active IR (float, as given) */
  int La;                /* active IR length, 0 = none yet */
  float *pending;        /* [Lmax] */
  int Lp;                /* pending IR length, 0 = none */
  int off_p;             /* sample of the next block from which the pending IR applies */
} or_stream;

or_stream *or_open(int B, int Lmax, int C, int prec) {
  if (B < 1 || Lmax < 1 || C < 1 || prec < OR_FP64 || prec > OR_FP32_MULADD) return NULL;
  or_stream *s = (or_stream *)calloc(1, sizeof(or_stream));
  if (!s) return NULL;
  s->B = B; s->Lmax = Lmax; s->C = C; s->prec = prec;
  size_t n = (size_t)C * (size_t)Lmax;
  if (prec == OR_FP64) s->r64 = (double *)calloc(n, sizeof(double));
  else s->r32 = (float *)calloc(n, sizeof(float));
  s->active = (float *)calloc((size_t)Lmax, sizeof(float));
  s->pending = (float *)calloc((size_t)Lmax, sizeof(float));
  if ((!s->r64 && !s->r32) || !s->active || !s->pending) {
    free(s->r64); free(s->r32); free(s->active); free(s->pending); free(s);
    return NULL;
  }
  return s;
}

void or_close(or_stream *s) {
  if (!s) return;
  free(s->r64); free(s->r32); free(s->active); free(s->pending); free(s);
}

/* Queue an IR; it becomes active at sample `offset` (0 <= offset < B) of the
 * next or_process call: samples before it keep the current IR.  The last IR
 * set before a call wins. */
int or_set_ir_at(or_stream *s, const float *h, int L, int offset) {
  if (!s || !h || L < 1 || L > s->Lmax || offset < 0 || offset >= s->B) return OR_EINVAL;
  memcpy(s->pending, h, (size_t)L * sizeof(float));
  s->Lp = L;
  s->off_p = offset;
  return OR_OK;
}

/* Queue an IR for the whole next block. */
int or_set_ir(or_stream *s, const float *h, int L) { return or_set_ir_at(s, h, L, 0); }

/* Add the tache of one input sample (value e0, IR h of L taps) to one
 * channel's residue, then emit and clear the current slot p (the caller
 * advances p).  Each slot receives its products in input-sample order. */
static double tache_step64(double *r, int Lmax, int p, double e0, const float *h, int L) {
  for (int k = 0; k < L; ++k) {
    int j = p + k;                       /* (p + k) mod Lmax: p < Lmax and k < L <= Lmax */
    if (j >= Lmax) j -= Lmax;
    r[j] += e0 * (double)h[k];
  }
  double out = r[p];
  r[p] = 0.0;
  return out;
}

/* Same in float: fused = one rounding per multiply-accumulate (fmaf);
 * otherwise the product is rounded to float, then the sum. */
static float tache_step32(float *r, int Lmax, int p, float e0, const float *h, int L, int fused) {
  for (int k = 0; k < L; ++k) {
    int j = p + k;
    if (j >= Lmax) j -= Lmax;
    if (fused) {
      r[j] = fmaf(e0, h[k], r[j]);
    } else {
      const float t = e0 * h[k];
      r[j] = r[j] + t;
    }
  }
  float out = r[p];
  r[p] = 0.0f;
  return out;
}

/* Process one block of B samples per channel.  x: [C][B] floats; y: [C][B]
 * doubles (FP32 modes store their float results widened exactly).
 * Returns OR_ENOIR (y untouched) if no IR was ever set. */
int or_process(or_stream *s, const float *x, double *y) {
  if (!s || !x || !y) return OR_EINVAL;
  const int B = s->B, Lmax = s->Lmax;
  int sw = B;                            /* first sample that uses the queued IR */
  if (s->Lp > 0) sw = s->off_p;
  if (sw == 0) {                         /* the queued IR takes effect here */
    float *t = s->active; s->active = s->pending; s->pending = t;
    s->La = s->Lp; s->Lp = 0;
    sw = B;
  }
  if (s->La == 0) return OR_ENOIR;       /* no IR for the block's first sample */
  int p0 = s->p;
  for (int c = 0; c < s->C; ++c) {       /* channels are independent */
    int p = p0;
    const float *xc = x + (size_t)c * B;
    double *yc = y + (size_t)c * B;
    for (int n = 0; n < B; ++n) {
      const float *h = n < sw ? s->active : s->pending;
      const int L = n < sw ? s->La : s->Lp;
      if (s->prec == OR_FP64)
        yc[n] = tache_step64(s->r64 + (size_t)c * Lmax, Lmax, p, (double)xc[n], h, L);
      else
        yc[n] = (double)tache_step32(s->r32 + (size_t)c * Lmax, Lmax, p, xc[n], h, L, s->prec == OR_FP32_FMA);
      p = (p + 1 == Lmax) ? 0 : p + 1;
    }
  }
  if (sw < B) {                          /* the queued IR took over inside the block */
    float *t = s->active; s->active = s->pending; s->pending = t;
    s->La = s->Lp; s->Lp = 0;
  }
  s->p = (int)(((long)p0 + B) % Lmax);
  return OR_OK;
}

/* Copy out the residue of channel c in output order: out[k] is the pending
 * sum for the k-th next output sample (k = 0 .. Lmax-1). */
int or_get_residue(const or_stream *s, int c, double *out) {
  if (!s || !out || c < 0 || c >= s->C) return OR_EINVAL;
  for (int k = 0; k < s->Lmax; ++k) {
    int slot = (s->p + k) % s->Lmax;
    out[k] = s->prec == OR_FP64 ? s->r64[(size_t)c * s->Lmax + slot]
                                : (double)s->r32[(size_t)c * s->Lmax + slot];
  }
  return OR_OK;
}

/* Whole-signal driver for one channel of one stream: n_blocks blocks of B
 * samples from x (zero beyond n_x), IR schedule given as ir_of_block[b] =
 * index into (irs, lens) of the IR set before block b (-1 = no change),
 * taking over at sample off_of_block[b] of block b (NULL = at its start).
 * Writes n_blocks*B outputs into y.  Used to run many channels/streams from
 * parallel host threads; it calls only the functions above. */
int or_run_channel(int B, int Lmax, int prec, const float *x, long n_x, int n_blocks,
                   const float *const *irs, const int *lens, const int *ir_of_block,
                   const int *off_of_block, double *y) {
  or_stream *s = or_open(B, Lmax, 1, prec);
  if (!s) return OR_ENOMEM;
  float *xb = (float *)malloc((size_t)B * sizeof(float));
  if (!xb) { or_close(s); return OR_ENOMEM; }
  int rc = OR_OK;
  for (int b = 0; b < n_blocks && rc == OR_OK; ++b) {
    int k = ir_of_block[b];
    if (k >= 0) rc = or_set_ir_at(s, irs[k], lens[k], off_of_block ? off_of_block[b] : 0);
    if (rc != OR_OK) break;
    for (int i = 0; i < B; ++i) {
      long m = (long)b * B + i;
      xb[i] = m < n_x ? x[m] : 0.0f;
    }
    rc = or_process(s, xb, y + (size_t)b * B);
  }
  free(xb);
  or_close(s);
  return rc;
}
