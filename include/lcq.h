/*
 * lcq.h -- C ABI of the MI355X (gfx950) guaranteed-error-bound quantizers.
 *
 * Implements the quantizer stage of Fallin & Burtscher, "Lessons Learned on
 * the Path to Guaranteeing the Error Bound in Lossy Quantizers" (CoDaC'24):
 * point-wise ABS (section 2.1.1), REL (section 2.1.2) and NOA (section 2.1.3)
 * bounds for float32 / float64 arrays.  Every value is binned, reconstructed
 * exactly as the decoder will reconstruct it, checked against the bound and
 * stored losslessly when the check fails, when its bin leaves the valid range
 * (section 3.3) or when it is NaN, INF or denormal (sections 2.2, 3.1).  REL
 * bins an approximate log2 and reconstructs with the matching approximate
 * 2^y (section 3.2); no floating-point contraction is used anywhere
 * (section 3.2), so the output is a pure function of the input bits.
 *
 * Conventions for every entry point:
 *  - Pointers named d_* are device pointers (HIP device memory) owned by the
 *    caller; the library keeps no reference to them after the call returns.
 *    They must be 16-byte aligned, else LCQ_ERR_ARG.
 *  - Calls are asynchronous on the given HIP stream (0 = null stream) and
 *    allocate no memory.  Calls on different streams must use different
 *    workspaces; calls that share a workspace must be ordered (same stream).
 *  - Argument errors are detected on the host before anything is launched
 *    and leave every buffer untouched.  LCQ_ERR_HIP reports a failed launch.
 *  - The library never reads or writes outside the ranges the sizes below
 *    describe, whatever the data or stream contents.
 *
 * Stream format (byte-exact, identical for any launch configuration):
 *   [0,64)   header, little-endian: u32 magic "LCQ1", u8 version (1),
 *            u8 dtype, u8 quantizer, u8 log2(chunk) (10), u64 n,
 *            u64 n_outliers, f64 eb as passed, then four u64 words holding
 *            the raw bits (zero-extended) of the field type's step, bound,
 *            aux0 (NOA: range minimum; REL: lower-side bound) and aux1
 *            (NOA: range maximum; otherwise 0)
 *   [64, 64+4n)              int32 code per value; INT32_MIN marks a value
 *                            stored losslessly ("outlier")
 *   ct = align16(64+4n)      u64 per 1024-value chunk: outliers before it
 *   out = align16(ct + 8*ceil(n/1024))
 *                            raw bits of the outliers, in input order
 *   size = out + n_outliers * sizeof(T); all padding bytes are zero.
 */
#ifndef LCQ_H
#define LCQ_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { LCQ_F32 = 0, LCQ_F64 = 1 } lcq_dtype;
typedef enum { LCQ_ABS = 0, LCQ_REL = 1, LCQ_NOA = 2 } lcq_quantizer;
typedef enum {
  LCQ_OK = 0,
  LCQ_ERR_ARG = 1,      /* bad enum, null / misaligned pointer, bad bound   */
  LCQ_ERR_CAPACITY = 2, /* output or workspace smaller than required        */
  LCQ_ERR_STREAM = 3,   /* stream header or structure does not match        */
  LCQ_ERR_HIP = 4       /* a HIP runtime call failed                        */
} lcq_status;

/* Largest n any entry point accepts (2^38 values). */
#define LCQ_MAX_N (1ull << 38)

/* Worst-case size in bytes of a stream of n values: every value stored
 * losslessly (section 3.1: a value whose double-check fails keeps its
 * original bits, and nothing bounds how many fail), plus the header and
 * chunk table of the format above.  The capacity lcq_quantize requires.
 * Returns 0 for a bad dtype or n. */
uint64_t lcq_max_stream_bytes(lcq_dtype t, uint64_t n);

/* Bytes of device workspace lcq_quantize / lcq_dequantize need for n values
 * of type t under quantizer q.  No passage of the paper defines it: it is
 * this library's GPU scratch (outlier counts, staged outliers and group sums
 * of the outlier compaction, NOA's per-workgroup range pairs).  The
 * workspace needs no initialisation; its first 8 bytes hold the status word
 * of the last lcq_dequantize (each decode call tags the word with its own
 * epoch and replaces whatever it held). */
uint64_t lcq_workspace_bytes(lcq_quantizer q, lcq_dtype t, uint64_t n);

/* Quantize d_in[0..n) of type t under bound eb (sections 2.1, 3.1-3.3).
 *  eb:        the user's bound; must be finite and > 0, and < 1 for REL.
 *             ABS guarantees |x - x'| <= eb, NOA |x - x'| <= eb * R with R the
 *             range of the finite values, REL same sign and
 *             |x| / (1+eb) <= |x'| <= |x| (1+eb).
 *  d_stream:  receives the stream; stream_cap >= lcq_max_stream_bytes(t, n).
 *  d_stream_bytes: device u64 that receives the stream's size (written by
 *             the last kernel; read it after the stream is synchronised).
 *  d_ws:      workspace of ws_bytes >= lcq_workspace_bytes(q, t, n).
 * Never fails because of the data: every value has an encoding. */
lcq_status lcq_quantize(lcq_quantizer q, lcq_dtype t, double eb,
                        const void *d_in, uint64_t n,
                        void *d_stream, uint64_t stream_cap,
                        uint64_t *d_stream_bytes,
                        void *d_ws, uint64_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * lcq_quantize, but the workspace is a fixed array of
 * LCQ_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, reserved when
 * the library's code is loaded on that GPU and held until the process ends.
 * The caller passes the input, the stream buffer and the size word as for
 * lcq_quantize.  The call allocates nothing; its first call on a device
 * looks the array's address up once.
 *  - LCQ_ERR_CAPACITY when lcq_workspace_bytes(q, t, n) exceeds
 *    LCQ_NOALLOC_SCRATCH_BYTES (float32: up to about 2.6e8 values, float64:
 *    about 6.5e7), checked on the host before anything is launched;
 *    LCQ_ERR_HIP if the array's address cannot be found.  Other errors as
 *    for lcq_quantize.
 *  - Every call on one GPU shares that GPU's array: calls that overlap on
 *    one GPU (different streams, or host threads without ordering) race and
 *    give undefined streams.  Calls ordered on one stream are safe; each
 *    clears the state it needs, so the previous call's leftovers are
 *    harmless. */
#define LCQ_NOALLOC_SCRATCH_BYTES (128ull << 20)
lcq_status lcq_quantize_noalloc(lcq_quantizer q, lcq_dtype t, double eb,
                                const void *d_in, uint64_t n,
                                void *d_stream, uint64_t stream_cap,
                                uint64_t *d_stream_bytes, hipStream_t stream);

/* Decode a stream into d_out[0..n) of type t (the decoder has no
 * double-check, section 6).  stream_bytes is the number of valid bytes at
 * d_stream; the host checks that the codes and chunk table of n values fit.
 * The header, the outlier count and the chunk table are validated on the
 * device; a mismatch is recorded in the workspace status word (read it with
 * lcq_stream_status) and leaves d_out unspecified but nothing outside it is
 * written.  d_ws needs at least 8 bytes. */
lcq_status lcq_dequantize(lcq_dtype t, const void *d_stream, uint64_t stream_bytes,
                          void *d_out, uint64_t n,
                          void *d_ws, uint64_t ws_bytes, hipStream_t stream);

/* Synchronises `stream` and stores in *h_err the status (LCQ_OK or
 * LCQ_ERR_STREAM) of the last lcq_dequantize that used d_ws.  The paper
 * defines no stream validation (its decompressor trusts its input, section
 * 6); this call reports the checks this library's decoder makes on the
 * format above, so a corrupted stream is refused instead of decoded. */
lcq_status lcq_stream_status(const void *d_ws, hipStream_t stream, int32_t *h_err);

/* Static description of a status code. */
const char *lcq_status_string(lcq_status s);

/* Measurement hook: when set (non-null), every following lcq_quantize /
 * lcq_dequantize call made from the calling host thread records `before`
 * immediately before and `after` immediately after the launch of its main
 * kernel (the per-value pass), on the call's stream.  Pass nulls to clear. */
void lcq_profile_events(hipEvent_t before, hipEvent_t after);

/* Measurement hook: when set (non-null), every following two-pass
 * lcq_quantize call from the calling host thread also records `mid` between
 * its two kernels (the streaming pass and the scan pass), so each pass can
 * be timed on its own.  Pass null to clear. */
void lcq_profile_mid_event(hipEvent_t mid);

/* ------------------------------------------------- section 6 ablations --
 * The two variants the paper measures its guarantee against (section 6,
 * Table 7 and Tables 5-6).  They do NOT guarantee the bound / CPU-GPU
 * parity; they exist to measure what the guarantee costs.
 *   LCQ_ABL_ABS_UNCHECKED  ABS without the double-check of section 3.1:
 *                          every finite normal value whose bin is in range
 *                          gets its bin, even where the reconstruction
 *                          misses the bound.
 *   LCQ_ABL_REL_LIBM       REL with the math library's log2 / exp2 (on the
 *                          device: the GPU's; for the bin width on the host:
 *                          the host's) in place of the approximations of
 *                          section 3.2.  The double-check still bounds every
 *                          value, but codes may differ between CPU and GPU.
 * Streams use the LCQ1 layout with the kind as the header's quantizer byte;
 * lcq_dequantize rejects them, lcq_dequantize_ablation decodes exactly the
 * given kind.  Arguments, buffers and errors as for lcq_quantize /
 * lcq_dequantize; the workspace is lcq_workspace_bytes(LCQ_ABS or LCQ_REL,
 * t, n).  Both always use the default (chunk-per-wavefront) kernels. */
typedef enum { LCQ_ABL_ABS_UNCHECKED = 3, LCQ_ABL_REL_LIBM = 4 } lcq_ablation;

lcq_status lcq_quantize_ablation(lcq_ablation kind, lcq_dtype t, double eb,
                                 const void *d_in, uint64_t n,
                                 void *d_stream, uint64_t stream_cap, uint64_t *d_stream_bytes,
                                 void *d_ws, uint64_t ws_bytes, hipStream_t stream);
lcq_status lcq_dequantize_ablation(lcq_ablation kind, lcq_dtype t,
                                   const void *d_stream, uint64_t stream_bytes,
                                   void *d_out, uint64_t n,
                                   void *d_ws, uint64_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------ lossless packing stage --
 * A lossless back-end for LCQ1 streams (the paper passes the quantizer's
 * output on to further lossless stages without naming them; this stage is
 * this library's own).  Per chunk of 1024 codes, c'_j = code_j or 0 for an
 * outlier sentinel, and z_j = zigzag(c'_j) (plain) or zigzag(c'_j - c'_{j-1})
 * (delta, c'_{-1} = 0, mod 2^32), zigzag(v) = (v << 1) ^ (v >> 31); the mode
 * with the smaller bit width w of the chunk's largest z is kept (plain on a
 * tie) and z_j is stored in bits [j w, j w + w), least significant first.
 *   [0,64)                   LCQ1 header with magic "LCQP"
 *   [64, 64+8C)              the LCQ1 chunk table
 *   ot = align16(64+8C)      u64 record offset per chunk, C+1 entries (the
 *                            last is the payload size)
 *   pl = align16(ot+8(C+1))  records, 16-byte aligned: u8 w, u8 mode (0
 *                            plain, 1 delta), u8 has_bitmap, 13 zero bytes;
 *                            if has_bitmap a 128-byte outlier bitmap (bit
 *                            i%8 of byte i/8); ceil(len*w/8) bytes of bits;
 *                            zeros to the next 16-byte boundary
 *   oo = align16(pl+payload) the k raw outliers; size = oo + k*s
 * lcq_pack reads an LCQ1 stream of n values (checked on the device, status
 * in the first 8 bytes of d_ws, read with lcq_stream_status) and writes the
 * packed stream and its size (device u64); packed_cap >=
 * lcq_pack_max_bytes(t, n), ws_bytes >= lcq_pack_workspace_bytes(t, n).
 * lcq_unpack restores the LCQ1 stream byte for byte (stream_cap >=
 * lcq_max_stream_bytes(t, n) suffices; ws >= 8 bytes); every offset, width
 * and record extent is checked on the device and a mismatch is recorded in
 * the status word (output then unspecified, nothing written outside it). */
uint64_t lcq_pack_max_bytes(lcq_dtype t, uint64_t n);        /* 0: bad dtype / n */
uint64_t lcq_pack_workspace_bytes(lcq_dtype t, uint64_t n);  /* 0: bad dtype / n */
lcq_status lcq_pack(lcq_dtype t, const void *d_stream, uint64_t stream_bytes, uint64_t n,
                    void *d_packed, uint64_t packed_cap, uint64_t *d_packed_bytes,
                    void *d_ws, uint64_t ws_bytes, hipStream_t stream);
lcq_status lcq_unpack(lcq_dtype t, const void *d_packed, uint64_t packed_bytes, uint64_t n,
                      void *d_stream, uint64_t stream_cap, uint64_t *d_stream_bytes,
                      void *d_ws, uint64_t ws_bytes, hipStream_t stream);

/* ----------------------------------------- fused compress / decompress --
 * The quantizer (sections 2.2, 3.1-3.3) and the packing stage above in one
 * call each, for HBM-bound use: the int32 codes never reach memory.
 * lcq_compress writes exactly the bytes lcq_pack(lcq_quantize(...)) writes
 * for the same q, t, eb and input (packed_cap >= lcq_pack_max_bytes(t, n),
 * ws_bytes >= lcq_compress_workspace_bytes(q, t, n), arguments and errors
 * as for lcq_quantize; never fails because of the data).  Its input is read
 * twice: the first pass classifies, bins and checks every value (sections
 * 2.2, 3.1-3.3) and sizes the records; the second takes the outliers from
 * the first pass's flags and recomputes the other values' bins with the
 * encoder's own operations, so both see the same codes.
 * lcq_decompress decodes a packed stream into d_out[0..n) with exactly the
 * values lcq_dequantize(lcq_unpack(...)) gives; the header, every record's
 * offset, width and extent, and every chunk-table entry are checked on the
 * device, a mismatch recorded in the status word (first 8 bytes of d_ws,
 * >= 8 bytes; read with lcq_stream_status) and the output then unspecified
 * (nothing outside it is written).  The workspace needs no initialisation. */
uint64_t lcq_compress_workspace_bytes(lcq_quantizer q, lcq_dtype t, uint64_t n); /* 0: bad args */
lcq_status lcq_compress(lcq_quantizer q, lcq_dtype t, double eb,
                        const void *d_in, uint64_t n,
                        void *d_packed, uint64_t packed_cap, uint64_t *d_packed_bytes,
                        void *d_ws, uint64_t ws_bytes, hipStream_t stream);
lcq_status lcq_decompress(lcq_dtype t, const void *d_packed, uint64_t packed_bytes,
                          void *d_out, uint64_t n,
                          void *d_ws, uint64_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------- in-line outlier layout --
 * The paper's own layout (section 3.1): outliers stored in-line with the
 * bins.  One word of the field type's width per value -- its code (the same
 * int32 code as above, sign-extended) or, for a value stored losslessly, its
 * raw bits -- and one flag bit per value saying which.  Same decisions and
 * decoded values as the separate-list layout; fixed size, no scan.
 *   [0,64)   header as above but magic "LCQI" and byte 7 = 0, word 2 = 0
 *   [64, 64 + n*s)            one word per value
 *   fl = align16(64 + n*s)    ceil(n/8) bytes; bit i%8 of byte i/8 set when
 *                             value i is stored raw; unused bits zero
 *   size = fl + ceil(n/8)
 */
uint64_t lcq_inline_stream_bytes(lcq_dtype t, uint64_t n);  /* 0: bad dtype / n */
uint64_t lcq_inline_workspace_bytes(lcq_quantizer q);      /* 0: bad quantizer */

/* As lcq_quantize, into the in-line layout; stream_cap >=
 * lcq_inline_stream_bytes(t, n), ws_bytes >= lcq_inline_workspace_bytes(q). */
lcq_status lcq_quantize_inline(lcq_quantizer q, lcq_dtype t, double eb,
                               const void *d_in, uint64_t n,
                               void *d_stream, uint64_t stream_cap,
                               void *d_ws, uint64_t ws_bytes, hipStream_t stream);

/* As lcq_dequantize, from the in-line layout (header validated on the
 * device, status in the first 8 bytes of d_ws, read with lcq_stream_status). */
lcq_status lcq_dequantize_inline(lcq_dtype t, const void *d_stream, uint64_t stream_bytes,
                                 void *d_out, uint64_t n,
                                 void *d_ws, uint64_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------- batch --
 * Many fields of uneven size, mixed dtype, quantizer and bound, quantized or
 * dequantized by one graph launch.  Each field's stream and decode are
 * byte-identical to what lcq_quantize / lcq_dequantize give for it alone.
 */
typedef struct {
  lcq_quantizer q;
  lcq_dtype t;
  double eb;                 /* as for lcq_quantize                          */
  const void *d_in;          /* quantize input, n values (16-byte aligned)    */
  uint64_t n;
  void *d_stream;            /* quantize output / dequantize input            */
  uint64_t stream_cap;       /* >= lcq_max_stream_bytes(t, n)                 */
  uint64_t *d_stream_bytes;  /* receives the stream size (device u64)         */
  void *d_out;               /* dequantize output, n values; may be null if   */
                             /* the plan is only used to quantize (then       */
                             /* lcq_batch_dequantize returns LCQ_ERR_ARG and  */
                             /* launches nothing)                             */
} lcq_field;

typedef struct lcq_batch_plan lcq_batch_plan;

/* Number of batch kernel variants the tuner may choose with "batch=<k>". */
int32_t lcq_batch_variants(void);

/* Device workspace a plan over these fields needs (0 for bad arguments).
 * `tune` is null (all defaults) or a tuning string, as the autotuner writes
 * it, with up to three integer keys, each key followed by its value after
 * any of '=', ':', '"' or blanks (so "batch=0 f32=4 f64=2" and
 * {"batch": 0, "f32": 4, "f64": 2} read alike):
 *   batch  kernel variant, < lcq_batch_variants() (default 0: the two-pass
 *          chunk form; 1.. look-back tile shapes);
 *   f32    chunk form: 1024-value chunks per wavefront in each quantize work
 *   f64    item, for float32 / float64 fields: 1, 2, 4, 8 or 16 (default 1).
 * Any other value of a present key makes the string invalid. */
uint64_t lcq_batch_workspace_bytes(const lcq_field *f, uint32_t nf, const char *tune);

/* Validates every field like lcq_quantize does, derives the per-field
 * parameters, uploads field descriptors and work-item tables into d_ws (the
 * plan's workspace; it must stay alive and unused by others until the plan
 * is destroyed), and captures the quantize and dequantize launches into HIP
 * graphs.  Synchronises `stream`.  The caller keeps every field buffer alive
 * while the plan is used.  On success *out receives the plan. */
lcq_status lcq_batch_plan_create(const lcq_field *f, uint32_t nf, const char *tune,
                                 void *d_ws, uint64_t ws_bytes, hipStream_t stream,
                                 lcq_batch_plan **out);

/* Quantize / dequantize every field of the plan: one hipGraphLaunch on s.
 * lcq_batch_dequantize returns LCQ_ERR_ARG, before any launch, for a plan
 * with a field of n > 0 values whose d_out is null. */
lcq_status lcq_batch_quantize(lcq_batch_plan *p, hipStream_t s);
lcq_status lcq_batch_dequantize(lcq_batch_plan *p, hipStream_t s);

/* Synchronises s; *h_first_bad receives the index of the first field whose
 * last batch dequantize found its stream inconsistent, or -1. */
lcq_status lcq_batch_status(lcq_batch_plan *p, hipStream_t s, int64_t *h_first_bad);

void lcq_batch_plan_destroy(lcq_batch_plan *p);

/* -------------------------------------------------------------- serving --
 * Continuous batching: lcq_serve runs an open-loop schedule of requests.  A
 * request is admitted (first come, first served) as soon as one of
 * n_streams HIP streams is free and its output and workspace fit in the
 * device arena; admitted requests run concurrently; completions free their
 * slot and memory at once.  Every output is compared on the device with the
 * caller's expected bytes.  Blocking; host-side single loop.  Ordering: the
 * call first waits for all work already queued on the device (any stream),
 * so inputs, expected bytes and the arena may come from pending work; it
 * returns after every request's work has finished.
 */
typedef struct {
  int32_t op;             /* 0 = quantize, 1 = dequantize                      */
  lcq_quantizer q;        /* quantize only                                     */
  lcq_dtype t;
  double eb;              /* quantize only                                     */
  const void *d_in;       /* quantize: n values; dequantize: the stream        */
  uint64_t n;             /* values                                            */
  uint64_t in_bytes;      /* dequantize: valid stream bytes at d_in            */
  const void *d_expect;   /* expected output (stream / n values) or null       */
  uint64_t expect_bytes;  /* quantize: expected stream size (<= the capacity)  */
  int64_t arrival_ns;     /* arrival, ns after the start; non-decreasing       */
} lcq_request;

typedef struct {
  int64_t admit_ns;       /* launch time, ns after the start                  */
  int64_t done_ns;        /* completion seen by the loop, ns after the start  */
  uint64_t mismatched;    /* differing 16-byte words vs expected; +2^40 if    */
                          /* the stream size differs                          */
  int32_t status;         /* lcq_status of the request                        */
  int32_t stream;         /* slot it ran on                                   */
} lcq_request_result;

typedef struct {
  uint32_t n_streams;     /* concurrent slots (1..64)                          */
  void *d_arena;          /* device memory outputs / workspaces come from      */
  uint64_t arena_bytes;   /* the admission budget                              */
  void *d_scratch;        /* >= 8 bytes per request (mismatch counters)        */
  uint64_t scratch_bytes;
} lcq_server_config;

lcq_status lcq_serve(const lcq_server_config *cfg, const lcq_request *req, uint32_t nreq,
                     lcq_request_result *res);

/* Launch-shape tuning.  Each operation comes in lcq_tune_variants()
 * kernel variants; all produce the same bytes.  Variants 0-5: one
 * workgroup-wide tile per workgroup (loads in flight per thread x rounds;
 * quantize finds its outlier offset by a decoupled look-back over earlier
 * tiles).  Variant 6 (the default): one wavefront per 1024-value chunk;
 * quantize runs two kernels, a streaming pass that writes codes,
 * per-chunk outlier counts and staged outliers, then a scan pass that
 * writes the chunk table, the outliers and the header.  op 0 = quantize,
 * 1 = dequantize.  Process-wide; the tuner
 * (paper_2407_15037_amd/autotune.py) measures them and sets the fastest.
 * lcq_tune_set returns LCQ_ERR_ARG for a bad op, dtype or variant;
 * lcq_tune_get returns -1 for a bad op or dtype. */
int32_t lcq_tune_variants(void);
lcq_status lcq_tune_set(int32_t op, lcq_dtype t, int32_t variant);
int32_t lcq_tune_get(int32_t op, lcq_dtype t);

/* Testing hook for the bounded waits (the look-back tile kernels' outlier
 * offsets, the batched form's NOA parameter waits).  A workgroup waits for
 * what the tiles before it publish; after `polls` polls without an answer
 * it computes the missing tile's value from that tile's input itself (same
 * result, more work).  Default 4096; 0 makes every wait fall back
 * immediately.  Process-wide; affects launches and plans made after the
 * call. */
void lcq_debug_set_lookback_spin(uint32_t polls);

#ifdef __cplusplus
}
#endif
#endif
