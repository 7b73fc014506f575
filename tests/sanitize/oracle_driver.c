/* Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * CPU oracle (test infrastructure).  It calls every exported oracle routine
 * on frames of many shapes -- empty, one stage, odd and even lengths, known
 * and unknown starts, fixed and free ends, output windows inside frames,
 * mixed codes K = 3..9 and beta = 2..4, several threads -- and checks that
 * noiseless soft values decode to the message with the metric sum|l| in
 * every precision mode and in the radix-4 recursion.  Any sanitizer report
 * or failed check ends it with a nonzero status. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct { int32_t K, beta; uint32_t gen[4]; } orc_code;
typedef struct {
  int64_t llr_offset, bit_offset;
  int32_t n_stages, out_begin, n_out, start_known, end_state, code;
} orc_frame;

int orc_trellis_tables(const orc_code* c, int32_t* next, int32_t* out, int32_t* prv);
int orc_encode(const orc_code* c, const uint8_t* msg, int32_t n, int32_t terminate, uint8_t* coded);
int orc_decode(int mode, const orc_code* codes, int32_t n_codes, const orc_frame* frames,
               int32_t n_frames, const void* llr, uint8_t* bits, void* metric, int32_t* end_state,
               double* gap, int32_t n_threads);
void orc_quantize_i8(const float* llr, int8_t* q, int64_t n, float scale);
int orc_forward_spread_i64(const orc_code* c, const int8_t* llr, int32_t S, int32_t start_known,
                           int64_t* spread);

static uint64_t rs = 88172645463325252ull;
static uint32_t rnd(void) { rs ^= rs << 13; rs ^= rs >> 7; rs ^= rs << 17; return (uint32_t)rs; }

#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); exit(3); } } while (0)

int main(void) {
  const orc_code codes[] = {
      {3, 2, {07, 05, 0, 0}},           {5, 2, {023, 035, 0, 0}},
      {7, 2, {0133, 0171, 0, 0}},       {9, 3, {0557, 0663, 0711, 0}},
      {4, 4, {017, 013, 015, 011}},     {8, 2, {0247, 0371, 0, 0}},
  };
  const int nc = (int)(sizeof codes / sizeof codes[0]);
  for (int c = 0; c < nc; ++c) {
    int32_t nx[512], out[512], prv[512];
    CHECK(orc_trellis_tables(&codes[c], nx, out, prv) == 0);
  }
  /* a batch of frames of every code and many shapes, laid out back to back */
  enum { NF = 120 };
  orc_frame fr[NF];
  uint8_t* msgs[NF];
  int64_t llr_total = 0, bit_total = 0;
  for (int f = 0; f < NF; ++f) {
    const int c = f % nc;
    const int K = codes[c].K;
    int S;
    switch (f % 7) {
      case 0: S = 0; break;
      case 1: S = 1; break;
      case 2: S = K - 1; break;
      default: S = 1 + (int)(rnd() % 700);
    }
    const int term = (f % 3 == 0) && S >= K - 1;
    const int n = term ? S - (K - 1) : S;
    fr[f].llr_offset = llr_total;
    fr[f].bit_offset = bit_total;
    fr[f].n_stages = S;
    fr[f].out_begin = 0;
    fr[f].n_out = n;
    fr[f].start_known = 1;
    fr[f].end_state = term ? 0 : -1;
    fr[f].code = c;
    msgs[f] = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
    for (int t = 0; t < n; ++t) msgs[f][t] = (uint8_t)(rnd() & 1);
    llr_total += (int64_t)S * codes[c].beta;
    bit_total += n;
  }
  float* lf = (float*)malloc((size_t)(llr_total + 1) * sizeof(float));
  int8_t* li = (int8_t*)malloc((size_t)(llr_total + 1));
  double sum_abs[NF];
  for (int f = 0; f < NF; ++f) {
    const orc_code* cd = &codes[fr[f].code];
    const int S = fr[f].n_stages;
    uint8_t* coded = (uint8_t*)malloc((size_t)(S > 0 ? S : 1) * cd->beta);
    CHECK(orc_encode(cd, msgs[f], fr[f].n_out, fr[f].end_state == 0, coded) == S);
    sum_abs[f] = 0;
    for (int64_t k = 0; k < (int64_t)S * cd->beta; ++k) {
      const float a = 1.0f + (float)(rnd() % 50);
      lf[fr[f].llr_offset + k] = coded[k] ? -a : a;
      li[fr[f].llr_offset + k] = (int8_t)(coded[k] ? -(int)a : (int)a);
      sum_abs[f] += a;
    }
    free(coded);
  }
  uint8_t* bits = (uint8_t*)malloc((size_t)(bit_total + 1));
  double m64[NF], gap[NF];
  float m32[NF];
  int64_t mi[NF];
  int32_t end[NF];
  for (int threads = 1; threads <= 5; threads += 4) {
    for (int mode = 0; mode < 4; ++mode) {
      memset(bits, 0xAA, (size_t)(bit_total + 1));
      void* metric = mode == 0 ? (void*)m64 : mode == 1 ? (void*)m32 : (void*)mi;
      const void* llr = mode >= 2 ? (const void*)li : (const void*)lf;
      CHECK(orc_decode(mode, codes, nc, fr, NF, llr, bits, metric, end, mode == 0 ? gap : NULL,
                       threads) == 0);
      for (int f = 0; f < NF; ++f) {
        for (int t = 0; t < fr[f].n_out; ++t) CHECK(bits[fr[f].bit_offset + t] == msgs[f][t]);
        const double m = mode == 0 ? m64[f] : mode == 1 ? (double)m32[f] : (double)mi[f];
        CHECK(fabs(m - sum_abs[f]) <= 1e-6 * (1.0 + sum_abs[f]));
      }
    }
  }
  /* output windows inside frames, unknown starts, fixed nonzero end states */
  for (int f = 0; f < NF; ++f) {
    const int S = fr[f].n_stages;
    if (S < 3) continue;
    fr[f].out_begin = 1 + (int)(rnd() % (S / 2));
    fr[f].n_out = (int)(rnd() % (S - fr[f].out_begin + 1));
    fr[f].start_known = (int)(rnd() & 1);
    fr[f].end_state = (rnd() & 1) ? -1 : (int)(rnd() % (1u << (codes[fr[f].code].K - 1)));
  }
  for (int mode = 0; mode < 4; ++mode) {
    void* metric = mode == 0 ? (void*)m64 : mode == 1 ? (void*)m32 : (void*)mi;
    const void* llr = mode >= 2 ? (const void*)li : (const void*)lf;
    CHECK(orc_decode(mode, codes, nc, fr, NF, llr, bits, metric, end, mode == 0 ? gap : NULL, 3) == 0);
  }
  /* rejected descriptors */
  orc_frame bad = fr[5];
  bad.code = nc;
  CHECK(orc_decode(2, codes, nc, &bad, 1, li, bits, mi, end, NULL, 1) != 0);
  bad = fr[5];
  bad.end_state = 1 << 9;
  CHECK(orc_decode(2, codes, nc, &bad, 1, li, bits, mi, end, NULL, 1) != 0);
  /* quantiser and spread */
  orc_quantize_i8(lf, li, llr_total, 0.75f);
  int64_t* spread = (int64_t*)malloc(800 * sizeof(int64_t));
  for (int c = 0; c < nc; ++c) {
    const int64_t n = llr_total / codes[c].beta < 800 ? llr_total / codes[c].beta : 800;
    CHECK(orc_forward_spread_i64(&codes[c], li, (int32_t)n, c & 1, spread) == 0);
  }
  free(spread);
  for (int f = 0; f < NF; ++f) free(msgs[f]);
  free(lf); free(li); free(bits);
  puts("oracle sanitizer driver: ok");
  return 0;
}
