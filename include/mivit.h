/*
 * mivit.h - soft-decision Viterbi decoding of convolutional codes on AMD
 * Instinct MI355X (gfx950).  Plain C ABI: no C++ or framework types cross it.
 *
 * The operation is the decoder of arXiv 2011.13579 ("High-Throughput
 * Parallel Viterbi Decoder on GPU Tensor Cores"):
 *   - §II-A  encoder equation and trellis (K, beta, generator polynomials);
 *   - §II-B  branch metric Eq. (BM), path metric Eq. (PM), survivor Eq. (SP0),
 *            forward procedure (Algorithm 1) and traceback (Algorithm 2);
 *   - §III   long streams split into frames that overlap their neighbours;
 *   - §VI-§VIII radix-4 form: Eqs. (radix4:BM), (radix4:PM), (radix4:SP0),
 *            two trellis stages per iteration.
 *
 * Conventions shared by every entry point
 *   Trellis      state = previous K-1 input bits, most recent in the MSB;
 *                generator bit K-1 taps the current input, bit 0 the oldest.
 *                Output bit b of a branch uses gen[b].
 *   Soft values  one per coded bit, time-major: stage t of a frame occupies
 *                elements [t*beta, (t+1)*beta) after the frame's offset.
 *                Positive favours coded bit 0 (§II-C).  float32 or int8.
 *   Decisions    Eq. (PM) with a strict comparison: on a tie the lower-index
 *                previous state is kept.  Radix-4 keeps the smallest local
 *                left index y, which yields the same path.  With an unknown
 *                final state the best final state is used, ties to the
 *                lowest index.
 *   Arithmetic   float32 frames run Eqs. (BM)/(PM) in IEEE single precision
 *                (Eq. (BM) summed over b in increasing order, then one add to
 *                the path metric).  int8 frames run them exactly in integers.
 *   Output bits  packed 32 per uint32, least significant bit first.
 *   Pointers     soft values, bits, metrics and gradients are DEVICE
 *                pointers owned by the caller.  Descriptor arrays (codes,
 *                frames, options) are HOST pointers, copied at plan time.
 *   Streams      'stream' is a hipStream_t (NULL = the default stream).
 *                Decoding calls are asynchronous on that stream.
 *   Errors       every call returns a status; invalid arguments are rejected
 *                before any device work is queued; no call aborts the process.
 */
#ifndef MIVIT_H
#define MIVIT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MIVIT_OK = 0,
  MIVIT_EINVAL = -1,       /* invalid argument or descriptor */
  MIVIT_ENOMEM = -2,       /* device or host allocation failed */
  MIVIT_EHIP = -3,         /* a HIP runtime call failed */
  MIVIT_EUNSUPPORTED = -4  /* valid request the library does not implement */
} mivit_status;

/* Soft-value types.  float16 values are decoded in float32 arithmetic (each
 * converts exactly), halving the soft-value bytes of a float32 batch (the
 * paper's half-precision channel input with single-precision metrics,
 * §IX-B); radix 2 and variant 0 only (other variants: MIVIT_EUNSUPPORTED). */
typedef enum { MIVIT_F32 = 0, MIVIT_I8 = 1, MIVIT_F16 = 2 } mivit_dtype;

/* A convolutional code (§II-A): 3 <= K <= 9, 2 <= beta <= 4, 0 < gen[b] < 2^K,
 * and every generator has bit K-1 and bit 0 set (the premise of the
 * branch-output corollary of §IV, met by the standard codes); other codes are
 * rejected with MIVIT_EUNSUPPORTED. */
typedef struct {
  int32_t K;
  int32_t beta;
  uint32_t gen[4];
} mivit_code;

/* frame flags */
#define MIVIT_START_KNOWN 1u /* encoder started in state 0 (else: unknown start,
                                all-zero initial path metrics as in Algorithm 1) */
#define MIVIT_END_ZERO 2u    /* trace back from state 0 (terminated frame); else
                                from the best final state */

/* One frame: an independent run of the trellis over n_stages stages. */
typedef struct {
  int64_t llr_offset; /* element index (in soft values) of stage 0, value 0 */
  int64_t bit_offset; /* bit index in the output of emitted bit 0; multiple of 32 */
  int32_t n_stages;   /* S >= 0 trellis stages (terminated: N + K - 1) */
  int32_t out_begin;  /* first stage whose decoded bit is emitted */
  int32_t n_out;      /* decoded bits emitted: stages [out_begin, out_begin+n_out) */
  int16_t code;       /* index into the plan's code array */
  uint16_t flags;     /* MIVIT_START_KNOWN | MIVIT_END_ZERO */
} mivit_frame;

/* Plan options.  Zero-initialised means: choose automatically. */
typedef struct {
  int32_t dtype;    /* mivit_dtype of every frame's soft values */
  int32_t radix;    /* 0: choose; 2: radix-2; 4: radix-4 (int8 only);
                       8: radix-8, three stages per iteration (the
                       radix-2^rho form of §VIII with rho = 3; int8 only,
                       every code K >= 4, variant 0) */
  int32_t chunk;    /* >0: split every frame longer than chunk stages into
                       windows of chunk core stages plus 'overlap' stages on
                       each side (§III); 0: decode whole frames */
  int32_t overlap;  /* stages of overlap on each side of a chunk, >= 0 */
  int32_t variant;  /* kernel variant for tuning and comparison; 0: default
                       (butterfly exchanges through DPP and permlane swaps;
                       radix 2 with K = 8 or 9: one frame per wavefront with
                       2^(K-1)/64 states per lane in registers; radix 4
                       with K = 5 or 7, beta = 2: two frames per register
                       in packed 16-bit metrics; K = 7 batches that fill
                       the device with groups of eight equal-length frames
                       run four states per lane, eight frames per
                       wavefront); 1 and 2: radix-2 forward
                       exchanging through LDS swizzles (1: both
                       previous-state metrics fetched, 2: one partner metric
                       per lane; K = 8, 9: metrics exchanged through LDS
                       every stage), radix 4 through LDS, one frame per lane
                       group and 32-bit metrics; 3: radix 4 with the
                       candidate additions on the int8 matrix cores, one
                       16 x 16 x 32 MFMA per iteration holding all sixteen
                       dragonflies through the dragonfly groups of
                       §VIII-D-2 (int8, K = 7, beta = 2 codes with at most
                       four groups, radix 4 only; else MIVIT_EUNSUPPORTED);
                       4: radix 4 packed with one state per lane and two
                       frames per wavefront (int8, K = 5 or 7, beta = 2,
                       radix 4 only; else MIVIT_EUNSUPPORTED); 5: radix 4
                       packed with four states per lane for any batch (int8,
                       K = 7, beta = 2, radix 4 only; else
                       MIVIT_EUNSUPPORTED); 6 and 7: radix 2 with each
                       frame's states in the registers of two (6: K = 8
                       or 9) or four (7: K = 9) wavefronts, the stages on
                       a wavefront bit exchanging through LDS (float32
                       only; else MIVIT_EUNSUPPORTED): a long frame's
                       serial chain runs with fewer instructions per
                       wavefront; 8: radix 2 with K = 8 or 9, int8, beta
                       <= 3, two states per register in packed 16-bit
                       metrics (else MIVIT_EUNSUPPORTED) */
  uint32_t flags;   /* MIVIT_PLAN_* scheduling options, below */
  int32_t reserved[2]; /* must be zero */
} mivit_opts;

/* Plan scheduling flags (batch scheduling; the paper runs one kernel per
 * frame set, §III).  Frames of different codes always form separate parts
 * that run concurrently on plan-owned streams, forked from and joined back
 * into the caller's stream.
 *   MIVIT_PLAN_GRAPH       mivit_decode records its whole launch sequence in
 *                          a hipGraph on the first call with a given (llr,
 *                          bits, metric, end_state, stream) and replays the
 *                          graph on later calls with the same arguments (up
 *                          to 8 recorded argument sets per plan).
 *   MIVIT_PLAN_PERSISTENT  the rotating forward kernels run as persistent
 *                          grids: each wavefront takes frame groups in table
 *                          order (longest frames first) from a device work
 *                          counter until the table is exhausted.
 *   MIVIT_PLAN_AUTOTUNE    plan creation times every valid kernel choice of
 *                          each code's part (radix, exchange variant,
 *                          persistent launch; radix 4 only when 'radix' is 0
 *                          or 4, radix 8 only when it is 0 or 8, radix 2
 *                          only when it is 0 or 2) on
 *                          synthetic soft values with the plan's frame
 *                          shapes and keeps the fastest.  All choices give
 *                          identical results (for int8, radices 2, 4 and 8
 *                          the same path, ties included).  Uses extra device memory
 *                          for the plan's soft-value extent while creating.
 *   MIVIT_PLAN_NO_SPLIT    keep every frame of the packed radix-4 kernel in one
 *                          wavefront.  By default, when the batch has fewer
 *                          wavefront entries than about four per SIMD, each
 *                          long entry is cut into parts of whole 48-iteration
 *                          periods decoded concurrently; a part after the
 *                          first starts 192 stages early from all-zero path
 *                          metrics (the unknown start of §III's frames) and
 *                          keeps no decisions from them.  Its decisions are
 *                          exact when its metrics where its own stages begin
 *                          differ from the true ones by a constant in every
 *                          state; a check after the forward pass compares the
 *                          range-controlled metrics there bit for bit and
 *                          re-decodes, from the true metrics, every pair
 *                          whose check fails.  Results never depend on it. */
#define MIVIT_PLAN_GRAPH 1u
#define MIVIT_PLAN_AUTOTUNE 2u
#define MIVIT_PLAN_PERSISTENT 4u
#define MIVIT_PLAN_NO_SPLIT 8u

typedef struct mivit_plan mivit_plan;

/* Build a plan for a fixed batch description: validates the descriptors,
 * expands chunked frames into windows, orders the work longest first and
 * reserves the survivor memory (bit-packed decisions, 2^(K-1) bits per stage
 * per frame or window, §III) on the current device.  codes/frames/opts are
 * host pointers and are copied.  On success *plan owns device memory until
 * mivit_plan_destroy.  Errors: MIVIT_EINVAL (bad code or frame, overlapping
 * or unaligned outputs, radix 4 or 8 with float soft values),
 * MIVIT_EUNSUPPORTED (among others: a code without both end taps, radix 8
 * with K = 3 or a nonzero variant, float16 with a nonzero variant),
 * MIVIT_ENOMEM, MIVIT_EHIP. */
mivit_status mivit_plan_create(mivit_plan** plan, const mivit_code* codes, int32_t n_codes,
                               const mivit_frame* frames, int32_t n_frames,
                               const mivit_opts* opts);

/* mivit_plan_create on a given device (the plan's device argument of the
 * boundary): device >= 0 builds the plan there, with that device made
 * current for the call and the caller's current device restored after it;
 * device < 0 means the current device.  Every later call on the plan runs on
 * its device whatever device is current then.  Errors: MIVIT_EINVAL
 * (plan NULL, device not below the device count), those of
 * mivit_plan_create, MIVIT_EHIP (the device count cannot be read). */
mivit_status mivit_plan_create_on(mivit_plan** plan, int32_t device, const mivit_code* codes,
                                  int32_t n_codes, const mivit_frame* frames, int32_t n_frames,
                                  const mivit_opts* opts);

/* Decode every frame of the plan (forward procedure, then traceback).
 *   llr        device, float32, float16 or int8 per the plan's dtype, read-only
 *   bits       device uint32 words; frame f writes the words covering
 *              [bit_offset, bit_offset + n_out), zero-padding the last one
 *   metric     device, one per frame: float32 (float32 and float16 plans) or int64 (int8
 *              plans): the path metric of the decoded path, Eq. (PM) at the
 *              last stage.  For a chunked frame, that of its last window.
 *              May be NULL.
 *   end_state  device int32 per frame: the state traceback started from
 *              (last window for chunked frames).  May be NULL.
 * Asynchronous on 'stream'.  One plan must not be used by two overlapping
 * calls (it owns the survivor memory). */
mivit_status mivit_decode(mivit_plan* plan, const void* llr, uint32_t* bits, void* metric,
                          int32_t* end_state, void* stream);

/* The two phases of mivit_decode, for callers that time or overlap them.
 * mivit_forward runs the forward procedure (Algorithm 1 / Eq. (radix4:PM)),
 * storing the decisions in the plan and writing metric and end_state as
 * mivit_decode does; mivit_traceback then runs Algorithm 2 and writes bits.
 * A traceback must follow the forward call of the same plan on the same
 * stream; between them the plan must not be used by another call. */
mivit_status mivit_forward(mivit_plan* plan, const void* llr, void* metric, int32_t* end_state,
                           void* stream);
mivit_status mivit_traceback(mivit_plan* plan, uint32_t* bits, void* stream);

/* Backward of the best path metric (not in the paper; follows from
 * Eq. (BM) being linear in the soft values): for every frame f and every
 * stage t and output bit b,
 *   grad_llr[llr_offset_f + t*beta + b] = grad_metric[f] * (-1)^{c_{t,b}}
 * where c is the codeword of the decoded bits (re-encoded, §II-A; tail bits
 * of terminated frames are zero).  bits is the output of mivit_decode for the
 * same plan; grad_metric and grad_llr are device float32.  Plans with chunked
 * frames, frames without MIVIT_START_KNOWN (the re-encoding starts from state
 * 0) or frames whose emitted bits do not cover every stage but a zero tail
 * are rejected with MIVIT_EUNSUPPORTED. */
mivit_status mivit_decode_grad(mivit_plan* plan, const uint32_t* bits, const float* grad_metric,
                               float* grad_llr, void* stream);

/* One-call decode of equal-length frames: the input of Algorithm 1 (beta
 * soft values per stage) for n_frames frames laid out back to back, and the
 * output of Algorithm 2 (the decoded bits) plus the best path metric of
 * Eq. (PM), without building a plan.
 *   llr        device, dtype values; frame f, stage t, value b at element
 *              f*S*beta + t*beta + b, S = n_info + K - 1 when terminated,
 *              else n_info.  Read-only.
 *   dtype      mivit_dtype of the soft values.
 *   code       host pointer, copied; validated as for mivit_plan_create.
 *   terminated 1: every frame starts and ends in state 0 (K-1 zero tail
 *              inputs, not emitted); 0: known start, best final state.
 *   bits       device uint32 words; frame f writes words [f*W, (f+1)*W),
 *              W = ceil(n_info/32), bit k of the frame at bit k % 32 of word
 *              f*W + k/32, the last word zero-padded.  Never NULL.
 *   metric     device, n_frames values: float32 (float32 and float16 soft
 *              values) or int64 (int8).  May be NULL.
 * Kernels: packed radix 4 for int8 soft values of K = 5 or 7 rate-1/2 codes,
 * radix 2 otherwise; results are those of a plan over the same frames.
 * Asynchronous on 'stream'.  The library keeps a plan (and its survivor
 * memory, 2^(K-1) bits per stage and frame) per (device, stream, code,
 * dtype, n_frames, n_info, terminated), at most 16, releasing the least
 * recently used one after its stream has drained; calls that overlap on one
 * stream are ordered by it, calls on different streams never share memory.
 * n_frames == 0 or zero stages: nothing to do, MIVIT_OK.
 * Errors: MIVIT_EINVAL (null pointer, negative count, bad dtype or
 * terminated flag), the code errors of mivit_plan_create, MIVIT_ENOMEM,
 * MIVIT_EHIP. */
mivit_status mivit_decode_uniform(const void* llr, int32_t dtype, const mivit_code* code,
                                  int32_t n_frames, int32_t n_info, int32_t terminated,
                                  uint32_t* bits, void* metric, void* stream);

/* mivit_decode_uniform for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, layout, kernels and results, but the call's
 * tables and survivor memory live in one fixed 64 MiB device array of the
 * library (each GPU the library runs on holds it until the process ends),
 * and the call allocates nothing and copies nothing from the host: it
 * launches a table kernel, the forward and the traceback kernel.
 *   Limit: about 256 B of tables per frame plus the survivor memory, which
 *   for K <= 7 radix 2 is 2^(K-1)/8 B per stage (whole 32-stage blocks),
 *   for the packed radix-4 kernel 2^(K-1)/8 B per stage and frame (whole
 *   16-stage groups per frame pair), for K = 8, 9 2^(K-1)/8 B per stage
 *   (whole 32-stage blocks); e.g. 1024 K=7 frames of 8192 stages fit.
 *   A larger batch returns MIVIT_ENOMEM before any launch.
 * Every call on a GPU shares that GPU's array: calls that overlap on one
 * GPU (two streams, two threads) race and must be ordered by the caller;
 * each call writes every table and survivor word it reads. */
mivit_status mivit_decode_uniform_noalloc(const void* llr, int32_t dtype, const mivit_code* code,
                                          int32_t n_frames, int32_t n_info, int32_t terminated,
                                          uint32_t* bits, void* metric, void* stream);

/* Release a plan's device and host memory (waits for the device first). */
mivit_status mivit_plan_destroy(mivit_plan* plan);

/* Plan facts for callers and tools. */
typedef struct {
  int64_t n_items;         /* frames after chunking */
  int64_t survivor_bytes;  /* device memory reserved for decisions */
  int64_t total_stages;    /* sum of stages over work items */
  int32_t radix;           /* radix in use */
  int32_t dtype;
  int64_t llr_elems;       /* soft values the frames address: max(llr_offset + S*beta) */
  int64_t bit_words;       /* output words the frames address: max(ceil((bit_offset + n_out)/32)) */
  int32_t n_frames;        /* frames as passed to mivit_plan_create */
  int32_t device;          /* HIP device the plan lives on */
} mivit_plan_info;
mivit_status mivit_plan_get_info(const mivit_plan* plan, mivit_plan_info* info);

/* Human-readable summary of the plan's parts (one per code): kernel, variant,
 * launch form, items, wavefronts.  Writes at most len bytes including the
 * terminating zero into the host buffer buf (truncating). */
mivit_status mivit_plan_describe(const mivit_plan* plan, char* buf, int32_t len);

/* Host pipeline (not in the paper, which leaves the host transfers aside;
 * its §III notes that frames and streams give the GPU independent work):
 * decode a sequence of batches held in host memory, each laid out exactly as
 * the plan's frames describe, with the copy of one batch to the device, the
 * decode of another and the copy of a third one's results back in flight at
 * once (three HIP streams, `depth` device buffer sets of the plan's extents).
 *
 * mivit_pipe_create: depth 2..8 buffer sets on the plan's device; the plan
 *   must outlive the pipe and must not be used by other calls while
 *   mivit_pipe_run runs.
 * mivit_pipe_run: batch b reads llr_elems soft values (the plan's dtype) at
 *   host_llr + b * llr_elems, writes bit_words words at host_bits +
 *   b * bit_words and, if host_metric is not NULL, n_frames metrics (float32,
 *   or int64 for int8 plans) at host_metric + b * n_frames; the sizes are
 *   those of mivit_plan_get_info.  Blocks until every batch's results are in
 *   host memory.  The copies overlap the decodes only for page-locked host
 *   memory (hipHostMalloc, or torch's pin_memory); other host memory still
 *   gives the same results.  Errors: MIVIT_EINVAL for null arguments or
 *   n_batches < 0; a decode's own status; MIVIT_EHIP if a copy fails.
 * mivit_pipe_destroy: waits for the pipe's streams and frees its memory. */
typedef struct mivit_pipe mivit_pipe;
mivit_status mivit_pipe_create(mivit_pipe** pipe, mivit_plan* plan, int32_t depth);
mivit_status mivit_pipe_run(mivit_pipe* pipe, const void* host_llr, uint32_t* host_bits,
                            void* host_metric, int64_t n_batches);
mivit_status mivit_pipe_destroy(mivit_pipe* pipe);

/* Continuous stream across calls (the frames with overlap of §III for one
 * stream whose soft values arrive in pieces): the stream is cut into windows
 * exactly as a plan with the same chunk and overlap cuts it as one frame
 * (cores of opts->chunk stages, opts->overlap stages on each side, a window
 * at the stream's start with a known start state when flags has
 * MIVIT_START_KNOWN, the last window ending in state 0 when flags has
 * MIVIT_END_ZERO).  Each window is decoded once its right overlap has
 * arrived and its core bits are emitted in stream order, one bit per stage,
 * so the bits of all calls, concatenated, equal that plan's output.  The
 * soft values not yet consumed (fewer than chunk + 2*overlap stages) stay in
 * a device buffer between calls.
 *
 * mivit_stream_create: code and opts as for mivit_plan_create (host
 *   pointers, copied), with opts->chunk > 0 a multiple of 32 and
 *   opts->overlap >= 0; flags: MIVIT_START_KNOWN | MIVIT_END_ZERO;
 *   max_push_stages > 0 bounds one push.  Reserves two device buffers of
 *   chunk + 2*overlap + max_push_stages stages on the current device.
 *   Errors: MIVIT_EINVAL, those of mivit_plan_create, MIVIT_ENOMEM.
 * mivit_stream_push: appends n_stages stages (0 <= n_stages <=
 *   max_push_stages) of soft values, device memory of the stream's dtype,
 *   beta values per stage; writes the bits of every window now complete to
 *   the device words at bits (from bit 0; at most max_push_stages + chunk
 *   + 2*overlap bits, always a multiple of chunk) and their number to the
 *   host int64 *n_bits.  Asynchronous on 'stream'; llr may be reused once
 *   the stream has passed this call.  Window plans (one per distinct run of
 *   windows, up to 8 kept) are created on first use.
 * mivit_stream_finish: the stream has ended; writes the bits of the
 *   remaining windows (at most chunk + 2*overlap) to bits and their number
 *   to *n_bits, and waits for the device.  No push may follow.
 * mivit_stream_destroy: waits for the device and frees the stream.
 * Calls on one stream object must be made one at a time, on one HIP stream
 * (or with the caller ordering them).  After an error, destroy the stream. */
typedef struct mivit_stream mivit_stream;
mivit_status mivit_stream_create(mivit_stream** stream_obj, const mivit_code* code,
                                 const mivit_opts* opts, uint32_t flags,
                                 int64_t max_push_stages);
mivit_status mivit_stream_push(mivit_stream* stream_obj, const void* llr, int64_t n_stages,
                               uint32_t* bits, int64_t* n_bits, void* stream);
mivit_status mivit_stream_finish(mivit_stream* stream_obj, uint32_t* bits, int64_t* n_bits,
                                 void* stream);
mivit_status mivit_stream_destroy(mivit_stream* stream_obj);

/* int8 quantiser for soft values (the paper uses float inputs; this is the
 * library's choice): q[k] = saturate_127(round_half_even(fl32(llr[k] *
 * scale))); the product is rounded to float32 first.  llr: device float32
 * [n]; q: device int8 [n]; scale > 0.  NaN maps to 0. */
mivit_status mivit_quantize_i8(const float* llr, int8_t* q, int64_t n, float scale,
                               void* stream);

/* Static text for a status code. */
const char* mivit_strerror(mivit_status status);

/* Library version string. */
const char* mivit_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MIVIT_H */
