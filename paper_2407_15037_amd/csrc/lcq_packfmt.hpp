// lcq_packfmt.hpp -- device helpers of the packed (LCQP) stream format,
// shared by the packing stage (lcq_pack.hip) and the fused compress /
// decompress path (lcq_compress.hip).
//
// Per chunk of 1024 codes, with c'_j = code_j or 0 for an outlier sentinel:
//   plain mode  z_j = zigzag(c'_j)
//   delta mode  z_j = zigzag(c'_j - c'_{j-1}), c'_{-1} = 0 (mod 2^32)
// w = bit length of the chunk's largest z (0..32), the narrower mode kept
// (plain on a tie); z_j occupies bits [j w, j w + w) of the chunk's record,
// least significant bit first.  A chunk with outliers also carries a
// 1024-bit outlier bitmap.
//
//   [0,64)                  LCQ1 header with magic "LCQP"
//   [64, 64+8C)             LCQ1 chunk table
//   ot = align16(64+8C)     u64 record offset per chunk (+1: payload size)
//   pl = align16(ot+8(C+1)) records: 16-byte header (u8 w, u8 mode, u8
//                           has_bitmap, 13 zero bytes), [128-byte bitmap],
//                           packed bits, zeros to a 16-byte boundary
//   oo = align16(pl+payload) the k raw outliers
//
// Lane layout: the chunk kernels' W x NSUB (lcq_chunk.hpp): lane l holds
// positions 64 W j + W l + e of the chunk, e < W, j < NSUB.
#pragma once
#include <hip/hip_runtime.h>

#include "lcq_math.hpp"
#include "lcq_tile.hpp"

namespace lcq {

constexpr uint32_t kMagicPacked = 0x5051434Cu;  // "LCQP"
constexpr unsigned kRowPad = 4;  // words past a record's bits in an LDS row (keeps 16-byte rows)
// Largest record: header, bitmap and 1024 values of 32 bits.
constexpr unsigned kMaxRecord = 16 + 128 + 4 * (unsigned)kChunk;

__host__ __device__ inline uint64_t packed_table_offset(uint64_t C) { return align16(64 + 8 * C); }
__host__ __device__ inline uint64_t packed_payload_offset(uint64_t C) {
  return align16(packed_table_offset(C) + 8 * (C + 1));
}
__host__ __device__ inline uint64_t record_bytes(uint64_t len, unsigned w, unsigned hb) {
  return 16 + (hb ? 128 : 0) + align16((len * w + 7) / 8);
}
// Header word 0 of a packed stream of dtype t (quantizer byte masked off).
__host__ __device__ inline uint64_t packed_word0(int dtype) {
  return (uint64_t)kMagicPacked | (1ull << 32) | ((uint64_t)dtype << 40) |
         ((uint64_t)kLog2Chunk << 56);
}

// Values of chunk c below n, and a lane's position inside its chunk (32-bit
// bounds tests).
__device__ __forceinline__ unsigned chunk_len(uint64_t n, uint64_t c) {
  const uint64_t left = n - c * kChunk;
  return left >= kChunk ? kChunk : (unsigned)left;
}
template <int W> __device__ __forceinline__ unsigned chunk_pos(int j, int lane) {
  return (unsigned)(64 * W * j + W * lane);
}

__device__ __forceinline__ uint32_t zigzag(uint32_t v) {
  return (v << 1) ^ (uint32_t)((int32_t)v >> 31);
}
__device__ __forceinline__ uint32_t unzigzag(uint32_t z) { return (z >> 1) ^ (0u - (z & 1u)); }
__device__ __forceinline__ unsigned bitlen(uint32_t v) { return v ? 32u - (unsigned)__clz((int)v) : 0u; }

// z values of a chunk from its c' values (sentinels already 0) in plain
// (DELTA false) or delta mode; 0 at positions len and beyond (FULL: len is
// 1024).
template <bool DELTA, int W, int NSUB, bool FULL = false>
__device__ __forceinline__ void chunk_z(const uint32_t (&cv)[NSUB][W], unsigned len, int lane,
                                        uint32_t (&z)[NSUB][W]) {
  uint32_t carry = 0;  // last c' of the previous sub-block
#pragma unroll
  for (int j = 0; j < NSUB; j++) {
    const unsigned p = chunk_pos<W>(j, lane);
    uint32_t prev = 0;
    if constexpr (DELTA) {
      prev = lane_up1(cv[j][W - 1], carry);
      carry = lane63(cv[j][W - 1]);
    }
#pragma unroll
    for (int e = 0; e < W; e++) {
      const uint32_t d = DELTA ? cv[j][e] - prev : cv[j][e];
      z[j][e] = (FULL || p + e < len) ? zigzag(d) : 0u;
      prev = cv[j][e];
    }
  }
}

// OR of v over the wavefront (uniform): the prefix pattern of
// wave_incl_add with OR, read from lane 63.
__device__ __forceinline__ uint32_t wave_or_u(uint32_t v) {
  v |= dpp_mov<dpp::kRowShr1>(0u, v);
  v |= dpp_mov<dpp::kRowShr2>(0u, v);
  v |= dpp_mov<dpp::kRowShr4>(0u, v);
  v |= dpp_mov<dpp::kRowShr8>(0u, v);
  v |= dpp_mov<dpp::kRowBcast15, 0xa>(0u, v);
  v |= dpp_mov<dpp::kRowBcast31, 0xc>(0u, v);
  return lane63(v);
}

// Width and mode of a chunk from its c' values (sentinels already 0; same
// on every lane), from extremes instead of every z: the plain width is that
// of the largest zigzag of the c' values, the delta width that of their
// differences (mod 2^32, read as int32).  FULL: the chunk has 1024 values
// (no position to mask).
template <bool FULL, int W, int NSUB>
__device__ __forceinline__ void chunk_width(const uint32_t (&cv)[NSUB][W], unsigned len,
                                               int lane, unsigned &w, unsigned &mode) {
  int32_t plo = 0, phi = 0, dlo = 0, dhi = 0;
  uint32_t carry = 0;  // last c' of the previous sub-block
#pragma unroll
  for (int j = 0; j < NSUB; j++) {
    uint32_t prev = lane_up1(cv[j][W - 1], carry);
    carry = lane63(cv[j][W - 1]);
    const unsigned p = chunk_pos<W>(j, lane);
#pragma unroll
    for (int e = 0; e < W; e++) {
      const bool in = FULL || p + e < len;
      const int32_t v = in ? (int32_t)cv[j][e] : 0;
      const int32_t d = in ? (int32_t)(cv[j][e] - prev) : 0;
      plo = min(plo, v);
      phi = max(phi, v);
      dlo = min(dlo, d);
      dhi = max(dhi, d);
      prev = cv[j][e];
    }
  }
  // the largest zigzag code of a lane's range [lo, hi] is that of lo or
  // of hi, and no lane's exceeds that of the chunk's own extremes (lanes
  // hold them), so the chunk's width is the bit length of the largest
  // per-lane one -- the bit length of their OR
  const unsigned wp = bitlen(wave_or_u(max(zigzag((uint32_t)plo), zigzag((uint32_t)phi))));
  const unsigned wd = bitlen(wave_or_u(max(zigzag((uint32_t)dlo), zigzag((uint32_t)dhi))));
  mode = wd < wp ? 1u : 0u;
  w = mode ? wd : wp;
}

// Packed words of a chunk of len values at w bits each (zeros up to the
// record's 16-byte end): a multiple of 4.
__device__ __forceinline__ unsigned packed_words(unsigned len, unsigned w) {
  return (unsigned)(align16(((uint64_t)len * w + 7) / 8) / 4);
}

// The chunk's packed bits -- z values at w bits each, position p at bits
// [p w, p w + w), least significant first -- assembled in the wavefront's
// LDS row by atomic ORs.  A lane's values of a sub-block are consecutive
// positions, so they go two at a time: the pair as one 64-bit piece (2 w <=
// 64 bits), shifted to its bit offset inside its first word, lands in at
// most three words.  z is zero past the chunk's end, so those positions add
// nothing, and every word touched lies inside the 1024-word row.  LDS
// operations of one wavefront complete in issue order, so wavefront-scope
// fences suffice between the clearing, the ORs and later reads.
template <int W, int NSUB>
__device__ __forceinline__ void pack_bits(const uint32_t (&z)[NSUB][W], unsigned len, unsigned w,
                                          uint32_t *row, int lane) {
  static_assert(W % 2 == 0, "values go in pairs");
  const unsigned nwords = packed_words(len, w);
  const nt_u4 zero = {0u, 0u, 0u, 0u};
  for (unsigned t = lane; 4 * t < nwords; t += 64) reinterpret_cast<nt_u4 *>(row)[t] = zero;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (w) {
    const unsigned lane_bp = (unsigned)(W * lane) * w;  // the lane's first bit in a sub-block
#pragma unroll
    for (int j = 0; j < NSUB; j++)
#pragma unroll
      for (int e = 0; e < W; e += 2) {
        const unsigned bp = lane_bp + (unsigned)(64 * W * j + e) * w;
        const unsigned q = bp >> 5, sh = bp & 31u;
        const uint64_t piece = (uint64_t)z[j][e] | ((uint64_t)z[j][e + 1] << w);
        const uint64_t lo = piece << sh;  // bits [0, 64) of the shifted piece
        const uint32_t hi = sh ? (uint32_t)(piece >> (64 - sh)) : 0u;  // bits [64, 96)
        __hip_atomic_fetch_or(row + q, (uint32_t)lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        if (sh + 2 * w > 32)
          __hip_atomic_fetch_or(row + q + 1, (uint32_t)(lo >> 32), __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_WAVEFRONT);
        if (sh + 2 * w > 64)
          __hip_atomic_fetch_or(row + q + 2, hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// The row's nwords packed words to dst (16-byte aligned), 128-bit stores.
__device__ __forceinline__ void copy_words(const uint32_t *row, unsigned nwords, uint32_t *dst,
                                           int lane) {
  for (unsigned t = lane; 4 * t < nwords; t += 64)
    __builtin_nontemporal_store(reinterpret_cast<const nt_u4 *>(row)[t],
                                reinterpret_cast<nt_u4 *>(dst) + t);
}

// A record's 16-byte header and (hb) its outlier bitmap; flags: bit W j + e
// marks the lane's position 64 W j + W lane + e as an outlier.
template <int W, int NSUB>
__device__ __forceinline__ void write_record_head(uint8_t *rec, unsigned w, unsigned mode,
                                                  unsigned hb, unsigned flags, int lane) {
  if (lane < 4) {
    const uint32_t word = lane == 0 ? (w | (mode << 8) | (hb << 16)) : 0u;
    reinterpret_cast<uint32_t *>(rec)[lane] = word;
  }
  if (hb) {
    constexpr int LANES = 32 / W;  // lanes per bitmap word
    constexpr unsigned kLaneMask = (1u << W) - 1;
#pragma unroll
    for (int j = 0; j < NSUB; j++) {
      const unsigned fw = gather_flag_word<W>((flags >> (W * j)) & kLaneMask, lane);
      if ((lane & (LANES - 1)) == 0)
        reinterpret_cast<uint32_t *>(rec + 16)[2 * W * j + lane / LANES] = fw;
    }
  }
}

// Whether [off, nxt) of a payload of `payload` bytes can be a record: whole
// 16-byte units inside the payload, at least a header, at most kMaxRecord.
__device__ __forceinline__ bool record_extent_ok(uint64_t off, uint64_t nxt, uint64_t payload) {
  return (off & 15) == 0 && off <= nxt && nxt <= payload && nxt - off >= 16 &&
         nxt - off <= kMaxRecord && ((nxt - off) & 15) == 0;
}

// Stage a record's nwords packed words (16-byte aligned at pw) in the
// wavefront's LDS row with 128-bit loads, then order them before the
// wavefront's reads.
__device__ __forceinline__ void stage_words(const uint8_t *pw, unsigned nwords, uint32_t *row,
                                            int lane) {
  const nt_u4 *pw4 = reinterpret_cast<const nt_u4 *>(pw);
  for (unsigned t = lane; 4 * t < nwords; t += 64) {
    const nt_u4 v = __builtin_nontemporal_load(pw4 + t);
    row[4 * t] = v.x;
    row[4 * t + 1] = v.y;
    row[4 * t + 2] = v.z;
    row[4 * t + 3] = v.w;
  }
  // each wavefront reads only its own row: LDS operations of one wavefront
  // complete in issue order, so a wavefront-scope fence orders them
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Codes of sub-block j of a chunk from its staged record bits (row), width
// w, mode and bitmap bm (null without one): sentinels where the bitmap says
// so.  Positions past the chunk's end get whatever the row holds past the record's
// bits (their codes are never stored or counted by the callers, and in
// delta mode they only feed later positions of the same kind).  carry: the
// running delta-mode sum, updated for the next sub-block.  The row must have one readable word past
// the chunk's 1024 (kRowPad): the word after a value's first is always
// read, and only used when the value straddles into it.
template <int W>
__device__ __forceinline__ void record_codes_sub(const uint32_t *row, const uint8_t *bm,
                                                 unsigned w, unsigned mode, int lane, int j,
                                                 uint32_t &carry, int32_t (&out)[W]) {
  const uint32_t mask = w == 32 ? 0xFFFFFFFFu : ((1u << w) - 1u);
  const unsigned lane_bp = (unsigned)(W * lane) * w;  // the lane's first bit in a sub-block
  const unsigned l0 = chunk_pos<W>(j, lane);         // position in the chunk
  uint32_t v[W];
#pragma unroll
  for (int e = 0; e < W; e++) {
    // value bits [bp, bp + w): one funnel shift of the word pair (q, q+1)
    // (the upper word only matters when the value straddles into it, and
    // then it lies inside the record; otherwise its bits are masked off)
    const unsigned bp = lane_bp + (unsigned)(64 * W * j + e) * w;
    const unsigned q = bp >> 5, sh = bp & 31u;
    const uint32_t lo = row[q], hi = row[q + 1];  // (one paired LDS read)
    const uint32_t z = __builtin_amdgcn_alignbit(hi, lo, sh) & mask;  // (mask 0 when w is 0)
    v[e] = unzigzag(z);
  }
  if (mode) {
    // prefix sum over the chunk in position order (mod 2^32)
#pragma unroll
    for (int e = 1; e < W; e++) v[e] += v[e - 1];
    const uint32_t incl = wave_incl_add(v[W - 1]);
    const uint32_t excl = incl - v[W - 1] + carry;
#pragma unroll
    for (int e = 0; e < W; e++) v[e] += excl;
    carry += lane63(incl);
  }
  const unsigned fl = bm ? (bm[l0 / 8] >> (l0 % 8)) & ((1u << W) - 1u) : 0u;
#pragma unroll
  for (int e = 0; e < W; e++) out[e] = ((fl >> e) & 1u) ? kSent : (int32_t)v[e];
}

// The codes of every sub-block (record_codes_sub).
template <int W, int NSUB>
__device__ __forceinline__ void record_codes(const uint32_t *row, const uint8_t *bm, unsigned w,
                                             unsigned mode, int lane, int32_t (&out)[NSUB][W]) {
  uint32_t carry = 0;
#pragma unroll
  for (int j = 0; j < NSUB; j++) record_codes_sub<W>(row, bm, w, mode, lane, j, carry, out[j]);
}

}  // namespace lcq
