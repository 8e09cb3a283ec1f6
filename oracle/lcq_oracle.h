/*
 * lcq_oracle.h -- the CPU oracle of the guaranteed-error-bound quantizers
 * (Fallin & Burtscher, "Lessons Learned on the Path to Guaranteeing the
 * Error Bound in Lossy Quantizers", CoDaC'24).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is a plain, slow, single-threaded
 * C implementation (plus a chunk-parallel wrapper of the same steps) that
 * the tests, the smoke check and the benchmark's CPU baseline compare the
 * HIP library against.  The product path never links,
 * loads or calls it.  It shares no code, header or constant with the HIP
 * library: both are written independently from the same definitions.
 *
 * Status codes, enums and the stream layout are restated here on purpose
 * (they are a file format, so they must agree byte for byte).
 *
 * Every function is synchronous, uses host pointers only and allocates
 * nothing (the chunk-parallel wrapper starts threads).  It refuses to run (ORC_ERR_FPENV) unless the x87/SSE control
 * state is round-to-nearest with flush-to-zero and denormals-are-zero off,
 * so that every float operation is the IEEE-754 one the paper relies on
 * (section 3.2).
 */
#ifndef LCQ_ORACLE_H
#define LCQ_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_F32 = 0, ORC_F64 = 1 };
enum { ORC_ABS = 0, ORC_REL = 1, ORC_NOA = 2 };
/* The two ablations of section 6 (not error-bound guaranteeing by design):
 * ABS without the double-check of section 3.1, and REL with the C library's
 * log2 / exp2 in place of the approximations of section 3.2.  Their streams
 * carry these codes in the header's quantizer byte.  Parity unpinned: the
 * REL_LIBM codes (host and device math libraries round apart; pinned only
 * at exact powers of two and through the bound). */
enum { ORC_ABS_UNCHECKED = 3, ORC_REL_LIBM = 4 };
enum { ORC_OK = 0, ORC_ERR_ARG = 1, ORC_ERR_CAPACITY = 2, ORC_ERR_STREAM = 3,
       ORC_ERR_FPENV = 5 };

/* Per-field parameters after derivation (all floating values as raw bits of
 * the field type, zero-extended to 64 bits). */
typedef struct {
  uint64_t step;      /* bin width in the quantized domain                     */
  uint64_t inv;       /* 1 / step                                              */
  uint64_t bound;     /* ABS: e; NOA: ebR; REL: eh                             */
  uint64_t aux0;      /* NOA: lo; REL: el; ABS: 0                              */
  uint64_t aux1;      /* NOA: hi; otherwise 0                                  */
  uint64_t lambda;    /* REL: half bin width in log2 space; otherwise 0        */
  int32_t degenerate; /* NOA with no usable range: every value stored lossless */
  int32_t pad;
} orc_params;

/* Worst-case stream size (every value an outlier). */
uint64_t orc_max_stream_bytes(int dtype, uint64_t n);

/* Parameter derivation only (NOA reads the input for its range). */
int orc_params_derive(int q, int dtype, double eb, const void *in, uint64_t n,
                      orc_params *out);

/* Quantize n values of dtype at in[] into stream[0..cap); writes the stream
 * size to *stream_bytes. */
int orc_quantize(int q, int dtype, double eb, const void *in, uint64_t n,
                 void *stream, uint64_t cap, uint64_t *stream_bytes);

/* Decode a stream produced by orc_quantize (or by anything that follows the
 * same format) into out[0..n). */
int orc_dequantize(int dtype, const void *stream, uint64_t bytes, void *out,
                   uint64_t n);

/* Chunk-parallel wrapper: the same computation as orc_quantize /
 * orc_dequantize, with the values split at CHUNK boundaries over nthreads
 * threads (<= 0: one per online CPU, at most 256); output bytes and status
 * codes equal the single-threaded calls'.  orc_threads_used reports the
 * thread count a given nthreads resolves to (ranges never outnumber the
 * chunks, so a small field may use fewer). */
int orc_quantize_mt(int q, int dtype, double eb, const void *in, uint64_t n,
                    void *stream, uint64_t cap, uint64_t *stream_bytes, int nthreads);
int orc_dequantize_mt(int dtype, const void *stream, uint64_t bytes, void *out,
                      uint64_t n, int nthreads);
int orc_threads_used(int nthreads);

/* The two approximations of section 3.2, element-wise over arrays, exposed
 * so the tests can pin them. */
void orc_log2approx_f32(const float *in, float *out, uint64_t n);
void orc_pow2approx_f32(const float *in, float *out, uint64_t n);
void orc_log2approx_f64(const double *in, double *out, uint64_t n);
void orc_pow2approx_f64(const double *in, double *out, uint64_t n);

/* In-line outlier layout (the paper's own, section 3.1): one word of the
 * field type's width per value -- the value's code, or its raw bits when it
 * is stored losslessly -- plus one flag bit per value.  Fixed size
 * orc_inline_stream_bytes(dtype, n). */
uint64_t orc_inline_stream_bytes(int dtype, uint64_t n);
int orc_quantize_inline(int q, int dtype, double eb, const void *in, uint64_t n,
                        void *stream, uint64_t cap, uint64_t *stream_bytes);
int orc_dequantize_inline(int dtype, const void *stream, uint64_t bytes, void *out,
                          uint64_t n);

/* Lossless packing stage for LCQ1 streams (per 1024-code chunk: plain or
 * delta zigzag codes at the chunk's smallest bit width, an outlier bitmap
 * for chunks with outliers; layout in lcq_oracle.c).  orc_pack rewrites an
 * LCQ1 stream, orc_unpack restores it byte for byte. */
uint64_t orc_pack_max_bytes(int dtype, uint64_t n);
int orc_pack(int dtype, const void *stream, uint64_t bytes, uint64_t n, void *out,
             uint64_t cap, uint64_t *out_bytes);
int orc_unpack(int dtype, const void *packed, uint64_t bytes, uint64_t n, void *out,
               uint64_t cap, uint64_t *out_bytes);

#ifdef __cplusplus
}
#endif
#endif
