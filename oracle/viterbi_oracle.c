/*
 * CPU oracle for soft-decision Viterbi decoding of convolutional codes.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU decoder; it builds its own trellis
 * from the generator polynomials.
 *
 * It is deliberately plain and slow: one scalar loop over stages, one over
 * states, no blocking, no vector intrinsics, no reordering beyond what the
 * paper's equations state.  Paper references are to arXiv 2011.13579
 * ("High-Throughput Parallel Viterbi Decoder on GPU Tensor Cores").
 *
 *   encoder          §II-A, encoder equation: output bit b of stage t is the
 *                    XOR of g_b[k] * in_{t-(K-1-k)} over k; the state is the
 *                    previous K-1 inputs with in_{t-1} in the MSB.
 *   branch metric    §II-B, Eq. (BM): delta = sum_b (-1)^{alpha_out[b]} l[b],
 *                    summed in order b = 0 .. beta-1.
 *   path metric      §II-B, Eq. (PM) and Eq. (SP0), the forward procedure
 *                    of Algorithm 1, evaluated branch by branch (every
 *                    state pushes its two candidates to the states it
 *                    leads to; a candidate displaces the kept one only
 *                    when strictly larger, sources in increasing order, so
 *                    a tie keeps the lower-index previous state); the
 *                    survivor is stored as the one bit that tells the two
 *                    previous states of a state apart.
 *   traceback        the decoding of Algorithm 2: from the chosen final
 *                    state, shift the register back stage by stage; the
 *                    state after a stage holds that stage's input bit on
 *                    top.
 *   radix-4          §VIII-A, Eqs. (radix4:BM), (radix4:PM), (radix4:SP0):
 *                    super-branch metric over 2*beta soft values, maximum
 *                    over prv(prv(j)), two stages per iteration.
 *
 * Precision modes: "f64" evaluates the equations in double precision on the
 * float32 inputs; "f32" evaluates them in single precision (the precision the
 * paper requires for the path-metric accumulator, §IX-B); "i64" evaluates
 * them exactly in 64-bit integers on int8 inputs.  Unreachable states (known
 * start) hold minus infinity; in the integer mode this is an explicit flag.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXK 9
#define ORC_MAXNS (1 << (ORC_MAXK - 1))

typedef struct {
  int32_t K;        /* constraint length, 3..9 */
  int32_t beta;     /* outputs per input bit, 2..4 */
  uint32_t gen[4];  /* generator tap masks, bit K-1 = current input */
} orc_code;

typedef struct {
  int64_t llr_offset;  /* element index of stage 0, soft value 0 */
  int64_t bit_offset;  /* where output bit 0 goes (one byte per bit) */
  int32_t n_stages;    /* S */
  int32_t out_begin;   /* first stage whose decoded bit is emitted */
  int32_t n_out;       /* number of decoded bits emitted */
  int32_t start_known; /* 1: encoder starts in state 0; 0: unknown start */
  int32_t end_state;   /* >= 0: trace back from it; -1: from the best state */
  int32_t code;        /* index into the code array */
} orc_frame;

/* ------------------------------------------------------------------ */
/* Trellis, written out from the encoder equation (§II-A).            */
/* ------------------------------------------------------------------ */

typedef struct {
  int K, beta, ns;
  int next[ORC_MAXNS][2];    /* next[i][u]: state after input u from i   */
  int out[ORC_MAXNS][2];     /* out[i][u]: beta-bit branch output word   */
  int prv[ORC_MAXNS][2];     /* the two previous states, ascending order */
  int prv_in[ORC_MAXNS];     /* input bit on any branch into j           */
} orc_trellis;

static int parity32(uint32_t x) {
  int p = 0;
  while (x) { p ^= (int)(x & 1u); x >>= 1; }
  return p;
}

static void build_trellis(const orc_code* c, orc_trellis* tr) {
  tr->K = c->K;
  tr->beta = c->beta;
  tr->ns = 1 << (c->K - 1);
  int cnt[ORC_MAXNS];
  memset(cnt, 0, sizeof cnt);
  for (int i = 0; i < tr->ns; ++i) {
    for (int u = 0; u < 2; ++u) {
      /* shift register: current input at bit K-1, state bits below it */
      uint32_t reg = ((uint32_t)u << (c->K - 1)) | (uint32_t)i;
      int j = (int)(reg >> 1);
      int word = 0;
      for (int b = 0; b < c->beta; ++b)
        word |= parity32(c->gen[b] & reg) << b;
      tr->next[i][u] = j;
      tr->out[i][u] = word;
    }
  }
  /* invert the next-state map to list the two predecessors of each state */
  for (int i = 0; i < tr->ns; ++i)
    for (int u = 0; u < 2; ++u) {
      int j = tr->next[i][u];
      tr->prv[j][cnt[j]++] = i;
      tr->prv_in[j] = u;
    }
  for (int j = 0; j < tr->ns; ++j)
    if (tr->prv[j][0] > tr->prv[j][1]) {
      int t = tr->prv[j][0];
      tr->prv[j][0] = tr->prv[j][1];
      tr->prv[j][1] = t;
    }
}

/* Exported for the table tests: next, out, prv as flat int arrays. */
int orc_trellis_tables(const orc_code* c, int32_t* next, int32_t* out, int32_t* prv) {
  if (c->K < 2 || c->K > ORC_MAXK || c->beta < 1 || c->beta > 4) return -1;
  orc_trellis tr;
  build_trellis(c, &tr);
  for (int i = 0; i < tr.ns; ++i)
    for (int u = 0; u < 2; ++u) {
      next[2 * i + u] = tr.next[i][u];
      out[2 * i + u] = tr.out[i][u];
      prv[2 * i + u] = tr.prv[i][u];
    }
  return 0;
}

/* Encoder (§II-A).  msg: n bytes of 0/1; coded: S*beta bytes, time-major. */
int orc_encode(const orc_code* c, const uint8_t* msg, int32_t n, int32_t terminate,
               uint8_t* coded) {
  if (c->K < 2 || c->K > ORC_MAXK) return -1;
  orc_trellis tr;
  build_trellis(c, &tr);
  int S = n + (terminate ? c->K - 1 : 0);
  int s = 0;
  for (int t = 0; t < S; ++t) {
    int u = t < n ? (msg[t] & 1) : 0;
    int w = tr.out[s][u];
    for (int b = 0; b < c->beta; ++b) coded[(int64_t)t * c->beta + b] = (uint8_t)((w >> b) & 1);
    s = tr.next[s][u];
  }
  return S;
}

/* ------------------------------------------------------------------ */
/* Radix-2 forward procedure and traceback (§II-B).                    */
/*                                                                    */
/* Forward: Eq. (PM) evaluated branch by branch.  At stage t every     */
/* state i sends, for each input u, the candidate PM_i + delta(i, u)   */
/* (delta from Eq. (BM)) to the state next[i][u] the branch enters.    */
/* Sources are visited in increasing index and a later candidate       */
/* displaces the kept one only when it is strictly larger, so a tie    */
/* keeps the lower-index previous state.  The two previous states of a */
/* state differ only in their least significant bit (the oldest input, */
/* shifted out of the register), so the survivor of Eq. (SP0) is kept  */
/* as that single bit per state and stage.                             */
/*                                                                    */
/* Traceback: from the chosen final state, the register is shifted     */
/* back one stage at a time: the state after stage t holds the input   */
/* of stage t in its top bit, and the state before it is that state    */
/* shifted up by one with the stored bit entering at the bottom.       */
/* ------------------------------------------------------------------ */

/* Per-thread scratch: decision bits (stage t, state j: bit j % 64 of
 * word t * wps + j / 64) and, when requested, the margin |c' - c''|
 * between the two candidates of every node (stage-major). */
typedef struct {
  uint64_t* dec;
  double* margin;
  size_t cap_words;  /* words dec holds */
  size_t cap_nodes;  /* entries margin holds */
} orc_scratch;

static int words_per_stage(int ns) { return (ns + 63) / 64; }

static int scratch_reserve(orc_scratch* s, int S, int ns, int want_margin) {
  const size_t words = (size_t)(S > 0 ? S : 1) * (size_t)words_per_stage(ns);
  const size_t nodes = (size_t)(S > 0 ? S : 1) * (size_t)ns;
  if (words > s->cap_words) {
    free(s->dec);
    s->dec = (uint64_t*)malloc(words * sizeof(uint64_t));
    s->cap_words = s->dec ? words : 0;
    if (!s->dec) return -1;
  }
  if (want_margin && nodes > s->cap_nodes) {
    free(s->margin);
    s->margin = (double*)malloc(nodes * sizeof(double));
    s->cap_nodes = s->margin ? nodes : 0;
    if (!s->margin) return -1;
  }
  return 0;
}

/* Record the survivor bit of state j at stage t: the low bit of the kept
 * previous state. */
static void set_decision(uint64_t* dec_t, int j, int i) {
  const uint64_t m = (uint64_t)1 << (j & 63);
  if (i & 1) dec_t[j >> 6] |= m;
  else dec_t[j >> 6] &= ~m;
}

/* Walk back from state js after the last stage, writing the emitted bits;
 * returns the smallest margin met along the path (infinity without
 * margins). */
static double traceback_bits(const orc_trellis* tr, const orc_scratch* sc, const orc_frame* fr,
                             int js, int want_margin, uint8_t* bits) {
  const int ns = tr->ns, wps = words_per_stage(ns), top = tr->K - 2;
  double gmin = INFINITY;
  int j = js;
  for (int t = fr->n_stages - 1; t >= 0; --t) {
    if (want_margin) {
      double m = sc->margin[(size_t)t * ns + j];
      if (m < gmin) gmin = m;
    }
    int rel = t - fr->out_begin;
    if (rel >= 0 && rel < fr->n_out) bits[fr->bit_offset + rel] = (uint8_t)(j >> top);
    int d = (int)((sc->dec[(size_t)t * wps + (j >> 6)] >> (j & 63)) & 1u);
    j = ((j << 1) | d) & (ns - 1);
  }
  return gmin;
}

/* The three precision modes share one shape; each is written out in its
 * own arithmetic type. */

static int decode_f64(const orc_trellis* tr, const orc_frame* fr, const float* llr,
                      uint8_t* bits, double* metric, int32_t* end_state, double* gap,
                      orc_scratch* sc) {
  const int ns = tr->ns, beta = tr->beta, S = fr->n_stages, wps = words_per_stage(ns);
  const int want_margin = gap != NULL;
  if (scratch_reserve(sc, S, ns, want_margin)) return -2;
  double pm[ORC_MAXNS], nw[ORC_MAXNS];
  int got[ORC_MAXNS];
  for (int j = 0; j < ns; ++j) pm[j] = (fr->start_known && j != 0) ? -INFINITY : 0.0;
  for (int t = 0; t < S; ++t) {
    const float* l = llr + fr->llr_offset + (int64_t)t * beta;
    uint64_t* dec_t = sc->dec + (size_t)t * wps;
    for (int j = 0; j < ns; ++j) got[j] = 0;
    for (int i = 0; i < ns; ++i)
      for (int u = 0; u < 2; ++u) {
        const int j = tr->next[i][u];
        double delta = 0.0; /* Eq. (BM) */
        for (int b = 0; b < beta; ++b) delta += ((tr->out[i][u] >> b) & 1) ? -(double)l[b] : (double)l[b];
        const double c = pm[i] + delta;
        if (got[j] && want_margin)
          sc->margin[(size_t)t * ns + j] = (isinf(c) || isinf(nw[j])) ? INFINITY : fabs(c - nw[j]);
        if (!got[j] || c > nw[j]) {
          nw[j] = c;
          set_decision(dec_t, j, i);
        }
        got[j] = 1;
      }
    for (int j = 0; j < ns; ++j) pm[j] = nw[j];
  }
  int js = fr->end_state;
  if (js < 0) { js = 0; for (int j = 1; j < ns; ++j) if (pm[j] > pm[js]) js = j; }
  double g = traceback_bits(tr, sc, fr, js, want_margin, bits);
  if (gap) {
    if (fr->end_state < 0)
      for (int j = 0; j < ns; ++j)
        if (j != js && pm[js] - pm[j] < g) g = pm[js] - pm[j];
    gap[0] = g;
  }
  metric[0] = pm[js];
  end_state[0] = js;
  return 0;
}

static int decode_f32(const orc_trellis* tr, const orc_frame* fr, const float* llr,
                      uint8_t* bits, float* metric, int32_t* end_state, orc_scratch* sc) {
  const int ns = tr->ns, beta = tr->beta, S = fr->n_stages, wps = words_per_stage(ns);
  if (scratch_reserve(sc, S, ns, 0)) return -2;
  float pm[ORC_MAXNS], nw[ORC_MAXNS];
  int got[ORC_MAXNS];
  for (int j = 0; j < ns; ++j) pm[j] = (fr->start_known && j != 0) ? -INFINITY : 0.0f;
  for (int t = 0; t < S; ++t) {
    const float* l = llr + fr->llr_offset + (int64_t)t * beta;
    uint64_t* dec_t = sc->dec + (size_t)t * wps;
    for (int j = 0; j < ns; ++j) got[j] = 0;
    for (int i = 0; i < ns; ++i)
      for (int u = 0; u < 2; ++u) {
        const int j = tr->next[i][u];
        float delta = 0.0f; /* Eq. (BM), summed in single precision */
        for (int b = 0; b < beta; ++b) delta += ((tr->out[i][u] >> b) & 1) ? -l[b] : l[b];
        const float c = pm[i] + delta;
        if (!got[j] || c > nw[j]) {
          nw[j] = c;
          set_decision(dec_t, j, i);
        }
        got[j] = 1;
      }
    for (int j = 0; j < ns; ++j) pm[j] = nw[j];
  }
  int js = fr->end_state;
  if (js < 0) { js = 0; for (int j = 1; j < ns; ++j) if (pm[j] > pm[js]) js = j; }
  traceback_bits(tr, sc, fr, js, 0, bits);
  metric[0] = pm[js];
  end_state[0] = js;
  return 0;
}

static int decode_i64(const orc_trellis* tr, const orc_frame* fr, const int8_t* llr,
                      uint8_t* bits, int64_t* metric, int32_t* end_state, orc_scratch* sc) {
  const int ns = tr->ns, beta = tr->beta, S = fr->n_stages, wps = words_per_stage(ns);
  if (scratch_reserve(sc, S, ns, 0)) return -2;
  int64_t pm[ORC_MAXNS], nw[ORC_MAXNS];
  int ok[ORC_MAXNS], got[ORC_MAXNS]; /* ok = reachable; unreachable is minus infinity */
  for (int j = 0; j < ns; ++j) { pm[j] = 0; ok[j] = !(fr->start_known && j != 0); }
  for (int t = 0; t < S; ++t) {
    const int8_t* l = llr + fr->llr_offset + (int64_t)t * beta;
    uint64_t* dec_t = sc->dec + (size_t)t * wps;
    for (int j = 0; j < ns; ++j) { got[j] = 0; nw[j] = 0; }
    for (int w = 0; w < wps; ++w) dec_t[w] = 0;
    for (int i = 0; i < ns; ++i) {
      if (!ok[i]) continue; /* minus infinity never wins */
      for (int u = 0; u < 2; ++u) {
        const int j = tr->next[i][u];
        int64_t delta = 0; /* Eq. (BM), exact */
        for (int b = 0; b < beta; ++b) delta += ((tr->out[i][u] >> b) & 1) ? -(int64_t)l[b] : (int64_t)l[b];
        const int64_t c = pm[i] + delta;
        if (!got[j] || c > nw[j]) {
          nw[j] = c;
          set_decision(dec_t, j, i);
        }
        got[j] = 1;
      }
    }
    for (int j = 0; j < ns; ++j) { pm[j] = nw[j]; ok[j] = got[j]; }
  }
  int js = fr->end_state;
  if (js < 0) {
    js = -1;
    for (int j = 0; j < ns; ++j)
      if (ok[j] && (js < 0 || pm[j] > pm[js])) js = j;
    if (js < 0) js = 0;
  }
  traceback_bits(tr, sc, fr, js, 0, bits);
  metric[0] = ok[js] ? pm[js] : INT64_MIN;
  end_state[0] = js;
  return 0;
}

/* ------------------------------------------------------------------ */
/* Radix-4 (§VIII-A), exact integers.                                  */
/* ------------------------------------------------------------------ */

/* The unique two-stage path i -> m -> j inside a dragonfly (§VII); returns
 * the middle state or -1 if j is not two stages from i. */
static int middle_state(const orc_trellis* tr, int i, int j, int* u1, int* u2) {
  for (int a = 0; a < 2; ++a) {
    int m = tr->next[i][a];
    for (int b = 0; b < 2; ++b)
      if (tr->next[m][b] == j) { *u1 = a; *u2 = b; return m; }
  }
  return -1;
}

static int decode_r4_i64(const orc_trellis* tr, const orc_frame* fr, const int8_t* llr,
                         uint8_t* bits, int64_t* metric, int32_t* end_state) {
  const int ns = tr->ns, beta = tr->beta, S = fr->n_stages;
  const int8_t* l = llr + fr->llr_offset;
  int64_t pm[ORC_MAXNS], nw[ORC_MAXNS];
  int ok[ORC_MAXNS], nok[ORC_MAXNS];
  /* decisions: for each iteration, the chosen left state of every right state */
  int n_iter = (S + 1) / 2 + 1;
  int16_t* phi = (int16_t*)malloc((size_t)n_iter * ns * sizeof(int16_t));
  int* it_t0 = (int*)malloc((size_t)n_iter * sizeof(int)); /* first stage of the iteration */
  int* it_w = (int*)malloc((size_t)n_iter * sizeof(int));  /* 1 or 2 stages */
  if (!phi || !it_t0 || !it_w) { free(phi); free(it_t0); free(it_w); return -2; }
  for (int j = 0; j < ns; ++j) { pm[j] = 0; ok[j] = !(fr->start_known && j != 0); }
  int t = 0, it = 0;
  if (S & 1) {
    /* an odd stage count starts with one radix-2 stage */
    for (int j = 0; j < ns; ++j) {
      int best = -1; int64_t bv = 0;
      for (int q = 0; q < 2; ++q) {
        int i = tr->prv[j][q];
        if (!ok[i]) continue;
        int64_t d = 0;
        for (int b = 0; b < beta; ++b) {
          int64_t v = l[b];
          d += ((tr->out[i][tr->prv_in[j]] >> b) & 1) ? -v : v;
        }
        int64_t c = pm[i] + d;
        if (best < 0 || c > bv) { best = i; bv = c; } /* smallest index on ties */
      }
      nok[j] = best >= 0; nw[j] = bv; phi[(size_t)it * ns + j] = (int16_t)(best < 0 ? tr->prv[j][0] : best);
    }
    memcpy(pm, nw, sizeof pm); memcpy(ok, nok, sizeof ok);
    it_t0[it] = 0; it_w[it] = 1; ++it; t = 1;
  }
  for (; t < S; t += 2, ++it) { /* S - t is even here */
    for (int j = 0; j < ns; ++j) {
      int best = -1; int64_t bv = 0;
      /* candidates i in prv(prv(j)), visited in ascending index order */
      int cand[4], nc = 0;
      for (int q = 0; q < 2; ++q)
        for (int r = 0; r < 2; ++r) cand[nc++] = tr->prv[tr->prv[j][q]][r];
      for (int a = 0; a < 4; ++a)
        for (int b2 = a + 1; b2 < 4; ++b2)
          if (cand[b2] < cand[a]) { int x = cand[a]; cand[a] = cand[b2]; cand[b2] = x; }
      for (int q = 0; q < 4; ++q) {
        int i = cand[q];
        if (!ok[i]) continue;
        int u1 = 0, u2 = 0;
        int m = middle_state(tr, i, j, &u1, &u2);
        /* super-branch output: the 2*beta bits of i->m then m->j, Eq. (radix4:BM) */
        int64_t d = 0;
        for (int b = 0; b < 2 * beta; ++b) {
          int w = b < beta ? tr->out[i][u1] : tr->out[m][u2];
          int bit = (w >> (b % beta)) & 1;
          int64_t v = l[(int64_t)t * beta + b];
          d += bit ? -v : v;
        }
        int64_t c = pm[i] + d;
        if (best < 0 || c > bv) { best = i; bv = c; }
      }
      nok[j] = best >= 0; nw[j] = bv;
      phi[(size_t)it * ns + j] = (int16_t)(best < 0 ? cand[0] : best);
    }
    memcpy(pm, nw, sizeof pm); memcpy(ok, nok, sizeof ok);
    it_t0[it] = t; it_w[it] = 2;
  }
  int js = fr->end_state;
  if (js < 0) {
    js = -1;
    for (int j = 0; j < ns; ++j) if (ok[j] && (js < 0 || pm[j] > pm[js])) js = j;
    if (js < 0) js = 0;
  }
  metric[0] = ok[js] ? pm[js] : INT64_MIN;
  end_state[0] = js;
  /* traceback, two stages per iteration */
  int j = js;
  for (int k = it - 1; k >= 0; --k) {
    int i = phi[(size_t)k * ns + j];
    int t0 = it_t0[k];
    int ub[2];
    if (it_w[k] == 2) {
      int u1 = 0, u2 = 0;
      middle_state(tr, i, j, &u1, &u2);
      ub[0] = u1; ub[1] = u2;
    } else {
      ub[0] = tr->prv_in[j];
    }
    for (int q = 0; q < it_w[k]; ++q) {
      int rel = t0 + q - fr->out_begin;
      if (rel >= 0 && rel < fr->n_out) bits[fr->bit_offset + rel] = (uint8_t)ub[q];
    }
    j = i;
  }
  free(phi); free(it_t0); free(it_w);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Batched entry points: frames are independent; threads over frames. */
/* ------------------------------------------------------------------ */

enum { ORC_F64 = 0, ORC_F32 = 1, ORC_I64 = 2, ORC_R4_I64 = 3 };

typedef struct {
  int mode;
  const orc_code* codes;
  int n_codes;
  const orc_frame* frames;
  int n_frames;
  const void* llr;
  uint8_t* bits;
  void* metric;
  int32_t* end_state;
  double* gap;
  int next;          /* next frame to take */
  int err;
  pthread_mutex_t mu;
} orc_job;

static void* worker(void* arg) {
  orc_job* job = (orc_job*)arg;
  orc_scratch sc = {0, 0, 0, 0};  /* grows to the largest frame seen */
  orc_trellis* trs = (orc_trellis*)malloc(sizeof(orc_trellis) * (size_t)job->n_codes);
  if (!trs) { pthread_mutex_lock(&job->mu); job->err = -2; pthread_mutex_unlock(&job->mu); return NULL; }
  for (int c = 0; c < job->n_codes; ++c) build_trellis(&job->codes[c], &trs[c]);
  for (;;) {
    pthread_mutex_lock(&job->mu);
    int f = job->next++;
    pthread_mutex_unlock(&job->mu);
    if (f >= job->n_frames) break;
    const orc_frame* fr = &job->frames[f];
    const orc_trellis* tr = &trs[fr->code];
    int rc = 0;
    switch (job->mode) {
      case ORC_F64:
        rc = decode_f64(tr, fr, (const float*)job->llr, job->bits, (double*)job->metric + f,
                        job->end_state + f, job->gap ? job->gap + f : NULL, &sc);
        break;
      case ORC_F32:
        rc = decode_f32(tr, fr, (const float*)job->llr, job->bits, (float*)job->metric + f,
                        job->end_state + f, &sc);
        break;
      case ORC_I64:
        rc = decode_i64(tr, fr, (const int8_t*)job->llr, job->bits, (int64_t*)job->metric + f,
                        job->end_state + f, &sc);
        break;
      case ORC_R4_I64:
        rc = decode_r4_i64(tr, fr, (const int8_t*)job->llr, job->bits,
                           (int64_t*)job->metric + f, job->end_state + f);
        break;
      default: rc = -1;
    }
    if (rc) { pthread_mutex_lock(&job->mu); job->err = rc; pthread_mutex_unlock(&job->mu); }
  }
  free(sc.dec);
  free(sc.margin);
  free(trs);
  return NULL;
}

static int validate(const orc_code* codes, int n_codes, const orc_frame* frames, int n_frames) {
  for (int c = 0; c < n_codes; ++c) {
    if (codes[c].K < 2 || codes[c].K > ORC_MAXK) return -1;
    if (codes[c].beta < 1 || codes[c].beta > 4) return -1;
  }
  for (int f = 0; f < n_frames; ++f) {
    if (frames[f].code < 0 || frames[f].code >= n_codes) return -1;
    if (frames[f].n_stages < 0 || frames[f].n_out < 0) return -1;
    if (frames[f].out_begin < 0 || frames[f].out_begin + frames[f].n_out > frames[f].n_stages) return -1;
    if (frames[f].end_state >= (1 << (codes[frames[f].code].K - 1))) return -1;
  }
  return 0;
}

int orc_decode(int mode, const orc_code* codes, int32_t n_codes, const orc_frame* frames,
               int32_t n_frames, const void* llr, uint8_t* bits, void* metric,
               int32_t* end_state, double* gap, int32_t n_threads) {
  int rc = validate(codes, n_codes, frames, n_frames);
  if (rc) return rc;
  if (gap && mode != ORC_F64) return -1;
  orc_job job;
  memset(&job, 0, sizeof job);
  job.mode = mode; job.codes = codes; job.n_codes = n_codes;
  job.frames = frames; job.n_frames = n_frames; job.llr = llr;
  job.bits = bits; job.metric = metric; job.end_state = end_state; job.gap = gap;
  pthread_mutex_init(&job.mu, NULL);
  if (n_threads < 1) n_threads = 1;
  if (n_threads > n_frames) n_threads = n_frames > 0 ? n_frames : 1;
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)n_threads);
  if (!th) return -2;
  int started = 0;
  for (int k = 1; k < n_threads; ++k)
    if (pthread_create(&th[k], NULL, worker, &job) == 0) ++started;
    else break;
  worker(&job);
  for (int k = 1; k <= started; ++k) pthread_join(th[k], NULL);
  free(th);
  pthread_mutex_destroy(&job.mu);
  return job.err;
}

/* ------------------------------------------------------------------ */
/* int8 quantiser: q = saturate_127(round_half_even(l * scale)), the  */
/* product rounded once in single precision.                          */
/* ------------------------------------------------------------------ */
void orc_quantize_i8(const float* llr, int8_t* q, int64_t n, float scale) {
  for (int64_t k = 0; k < n; ++k) {
    volatile float p = llr[k] * scale;
    float r = rintf(p);
    if (r > 127.0f) r = 127.0f;
    if (r < -127.0f) r = -127.0f;
    if (r != r) r = 0.0f;
    q[k] = (int8_t)r;
  }
}

/* ------------------------------------------------------------------ */
/* Forward procedure only, exact integers: records, after every stage, */
/* max_j PM_j - min_j PM_j over the reachable states (for the bounded- */
/* spread invariant used to size integer path metrics).                */
/* ------------------------------------------------------------------ */
int orc_forward_spread_i64(const orc_code* c, const int8_t* llr, int32_t S, int32_t start_known,
                           int64_t* spread) {
  if (c->K < 2 || c->K > ORC_MAXK || c->beta < 1 || c->beta > 4) return -1;
  orc_trellis tr;
  build_trellis(c, &tr);
  const int ns = tr.ns, beta = tr.beta;
  int64_t pm[ORC_MAXNS], nw[ORC_MAXNS];
  int ok[ORC_MAXNS], nok[ORC_MAXNS];
  for (int j = 0; j < ns; ++j) { pm[j] = 0; ok[j] = !(start_known && j != 0); }
  for (int t = 0; t < S; ++t) {
    for (int j = 0; j < ns; ++j) {
      int ia = tr.prv[j][1], ib = tr.prv[j][0];
      int u = tr.prv_in[j];
      int64_t da = 0, db = 0;
      for (int b = 0; b < beta; ++b) {
        int64_t v = llr[(int64_t)t * beta + b];
        da += ((tr.out[ia][u] >> b) & 1) ? -v : v;
        db += ((tr.out[ib][u] >> b) & 1) ? -v : v;
      }
      int64_t pa = pm[ia] + da, pb = pm[ib] + db;
      int a_wins = ok[ia] && (!ok[ib] || pa > pb);
      nw[j] = a_wins ? pa : pb;
      nok[j] = a_wins ? 1 : ok[ib];
    }
    memcpy(pm, nw, sizeof(int64_t) * ns);
    memcpy(ok, nok, sizeof(int) * ns);
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    for (int j = 0; j < ns; ++j)
      if (ok[j]) { if (pm[j] < lo) lo = pm[j]; if (pm[j] > hi) hi = pm[j]; }
    spread[t] = hi - lo;
  }
  return 0;
}
