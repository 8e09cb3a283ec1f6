// lcq_chunk.hpp -- chunk-per-wavefront quantize / dequantize for gfx950.
//
// One 64-lane wavefront owns one 1024-value chunk of the stream format (the
// granularity of its chunk table).  With W = 16 / sizeof(T), lane l holds
// values 64 W j + W l + e of the chunk (e < W): each sub-block j is one
// contiguous run of 64 W values, so every load and store instruction of a
// wavefront covers one contiguous 1 KiB (values) or 1 KiB / 512 B (codes,
// float32 / float64) range.  Ranks of outliers inside a chunk follow from
// ballots alone; no LDS and no barrier is needed for them.
//
// Quantize runs as two passes instead of one pass with a decoupled
// look-back:
//   pass 1  per value classify / bin / reconstruct / verify (sections 2.2,
//           3.1-3.3), int32 code stores, the chunk's outlier count, and the
//           first stage_cap<T>() outliers' raw bits staged per chunk; one
//           atomic add per workgroup into the sum of its group of
//           workgroups.
//   pass 2  one workgroup per group: exclusive scan of the chunk counts
//           (the chunk table), copy of staged outliers to their final,
//           input-ordered place, header and size.  A chunk with more than
//           stage_cap<T>() outliers has its codes rescanned and its raw bits
//           read from the input, by a workgroup chosen so that runs of
//           such chunks spread over all of them.
// Dequantize gathers each outlier's bits before the single store of its
// values and checks every chunk-table entry against the counted sentinels.
#pragma once
#include <hip/hip_runtime.h>

#include "lcq_math.hpp"
#include "lcq_tile.hpp"

#pragma clang fp contract(off)

namespace lcq {

// Streamed data is touched once: its loads and stores are non-temporal
// (clang's nontemporal builtins need native vector types).
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef int nt_i4 __attribute__((ext_vector_type(4)));
typedef int nt_i2 __attribute__((ext_vector_type(2)));

// Outliers staged per chunk in pass 1: 512 bytes (float32) or 2 KiB
// (float64) per 1024-value chunk.  Hard stretches of data put tens to
// hundreds of outliers into a chunk (float32 REL at bounds near 1e-5: up to
// about 100; float64 values placed on bin borders: about 200); a chunk over
// the cap is rescanned from its codes and input in pass 2, at the cost of
// reading both again.
template <typename T> constexpr int stage_cap() { return sizeof(T) == 4 ? 128 : 256; }
// Pass 2 copies the staged rows of chunks with at most kDirect outliers in
// the chunk's own group; rows of chunks with more (hard stretches of data
// come in runs) are spread over every pass-2 workgroup, as are the rescans.
constexpr int kDirect = 32;
constexpr uint64_t kMaxGroups = 1024;  // pass-2 workgroups (groups) at most
constexpr uint64_t kGroupChunks = 64;  // chunks per group at least

// Pass-1 workgroups per pass-2 group for a field of `ntiles` pass-1
// workgroups of `chunks_per_tile` chunks each: at least kGroupChunks chunks
// per group (fewer, fuller pass-2 workgroups for many small fields), at
// most kMaxGroups groups.
__host__ __device__ inline uint64_t tiles_per_group(uint64_t ntiles, uint64_t chunks_per_tile) {
  const uint64_t by_size = (kGroupChunks + chunks_per_tile - 1) / chunks_per_tile;
  const uint64_t by_count = (ntiles + kMaxGroups - 1) / kMaxGroups;
  return by_size > by_count ? by_size : by_count;
}

// A lane holds W = 16 / sizeof(T) consecutive values of each sub-block (one
// 128-bit access), so a chunk is NSUB = 1024 / (64 W) sub-blocks and every
// lane holds 16 values of it: 4 x 4 (float32) or 8 x 2 (float64).
template <typename T> struct ChunkShape {
  static constexpr int W = 16 / (int)sizeof(T);
  static constexpr int NSUB = (int)kChunk / (64 * W);
  static_assert(W * NSUB == 16, "16 values per lane per chunk");
};

// W consecutive values at i0 (zeros past n).
template <typename T, int W>
__device__ __forceinline__ void load_vals(const T *in, uint64_t i0, uint64_t n, T (&x)[W]) {
  if (i0 + W <= n) {
    if constexpr (sizeof(T) == 4) {
      const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4 *>(in + i0));
      x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
    } else {
      const nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2 *>(in + i0));
      x[0] = v.x; x[1] = v.y;
    }
  } else {
#pragma unroll
    for (int e = 0; e < W; e++) x[e] = (i0 + e < n) ? in[i0 + e] : (T)0;
  }
}

template <typename T, int W>
__device__ __forceinline__ void store_vals(T *out, uint64_t i0, uint64_t n, const T (&y)[W]) {
  if (i0 + W <= n) {
    if constexpr (sizeof(T) == 4) {
      const nt_f4 o = {y[0], y[1], y[2], y[3]};
      __builtin_nontemporal_store(o, reinterpret_cast<nt_f4 *>(out + i0));
    } else {
      const nt_d2 o = {y[0], y[1]};
      __builtin_nontemporal_store(o, reinterpret_cast<nt_d2 *>(out + i0));
    }
  } else {
#pragma unroll
    for (int e = 0; e < W; e++)
      if (i0 + e < n) out[i0 + e] = y[e];
  }
}

template <int W>
__device__ __forceinline__ void load_codes(const int32_t *codes, uint64_t i0, uint64_t n,
                                           int32_t (&c)[W]) {
  if (i0 + W <= n) {
    if constexpr (W == 4) {
      const nt_i4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_i4 *>(codes + i0));
      c[0] = v.x; c[1] = v.y; c[2] = v.z; c[3] = v.w;
    } else {
      const nt_i2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_i2 *>(codes + i0));
      c[0] = v.x; c[1] = v.y;
    }
  } else {
#pragma unroll
    for (int e = 0; e < W; e++) c[e] = (i0 + e < n) ? codes[i0 + e] : 0;
  }
}

// (FULL: the caller knows all W lie below n)
template <int W, bool FULL = false>
__device__ __forceinline__ void store_codes(int32_t *codes, uint64_t i0, uint64_t n,
                                            const int32_t (&c)[W]) {
  if (FULL || i0 + W <= n) {
    if constexpr (W == 4) {
      const nt_i4 o = {c[0], c[1], c[2], c[3]};
      __builtin_nontemporal_store(o, reinterpret_cast<nt_i4 *>(codes + i0));
    } else {
      const nt_i2 o = {c[0], c[1]};
      __builtin_nontemporal_store(o, reinterpret_cast<nt_i2 *>(codes + i0));
    }
  } else {
#pragma unroll
    for (int e = 0; e < W; e++)
      if (i0 + e < n) codes[i0 + e] = c[e];
  }
}

// Sub-block j of chunk c, lane's first value.
template <int W>
__device__ __forceinline__ uint64_t chunk_value(uint64_t c, int j, int lane) {
  return c * kChunk + (uint64_t)(64 * W) * (unsigned)j + (uint64_t)W * (unsigned)lane;
}

// Ranks of flagged values of one sub-block inside the wavefront's chunk:
// returns the count of the sub-block to every lane, and in `pre` the number
// of flagged values of lower lanes.  `fl` holds the lane's W flags.
template <int W>
__device__ __forceinline__ unsigned sub_ranks(unsigned fl, uint64_t lt, unsigned &pre) {
  unsigned tot = 0;
  pre = 0;
#pragma unroll
  for (int e = 0; e < W; e++) {
    const uint64_t b = __ballot((fl >> e) & 1u);
    tot += (unsigned)__popcll(b);
    pre += (unsigned)__popcll(b & lt);
  }
  return tot;
}

// ------------------------------------------------------------- pass 1 ---
template <typename T> struct StageField {
  const T *in;
  uint64_t n;
  int32_t *codes;                 // stream + 64
  uint32_t *counts;               // one per chunk
  typename FT<T>::U *stage;       // stage_cap<T>() per chunk
  unsigned long long *group;      // one sum per group of workgroups
  uint64_t tiles_per_group;
  FieldParams<T> p;
};

// The 16 values per lane of chunk c (zeros past n).
template <typename T>
__device__ __forceinline__ void load_chunk(const T *in, uint64_t n, uint64_t c, int lane,
                                           T (&x)[ChunkShape<T>::NSUB][ChunkShape<T>::W]) {
  constexpr int W = ChunkShape<T>::W, NSUB = ChunkShape<T>::NSUB;
#pragma unroll
  for (int j = 0; j < NSUB; j++) load_vals<T, W>(in, chunk_value<W>(c, j, lane), n, x[j]);
}

// Number of set bits of the wavefront mask b in lanes below this one, plus
// acc.
__device__ __forceinline__ unsigned lanes_below(uint64_t b, unsigned acc) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(b >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)b, acc));
}

// Wavefront mask of the lanes whose value e of sub-block j lies below n,
// for a chunk with `left` values from its first one on (all lanes when the
// chunk is full).  Uniform: scalar arithmetic only.
template <int W>
__device__ __forceinline__ uint64_t valid_lanes(uint64_t left, int j, int e) {
  if (left >= kChunk) return ~0ull;
  const int64_t t = (int64_t)left - (int64_t)(64 * W * j + e);  // values from lane 0's
  if (t <= 0) return 0;
  const uint64_t lanes = ((uint64_t)t + W - 1) / W;
  return lanes >= 64 ? ~0ull : ((1ull << lanes) - 1);
}

// Pass 1 for chunk c held in x (c is uniform over the wavefront): codes,
// staged outliers and the chunk's count; returns the count.  Sub-block by
// sub-block: each value's outlier flag is one wavefront mask, and a
// sub-block with outliers puts them into the wavefront's LDS row `srow` at
// their ranks (running rank = outliers of earlier sub-blocks + set bits of
// lower lanes); the first stage_cap<T>() then leave in contiguous stores.
// k: the encoder's operands (enc_consts_pinned: held in vector registers).
template <typename T, int Q>
__device__ __forceinline__ unsigned encode_chunk(const StageField<T> &f, uint64_t c, int lane,
                                                 const T (&x)[ChunkShape<T>::NSUB][ChunkShape<T>::W],
                                                 typename FT<T>::U *srow, const EncK<T> &k) {
  constexpr int W = ChunkShape<T>::W, NSUB = ChunkShape<T>::NSUB;
  constexpr unsigned kCap = (unsigned)stage_cap<T>();
  const uint64_t n = f.n;
  const uint64_t left = n - c * kChunk;
  const bool full = left >= kChunk;
  unsigned cnt = 0;
#pragma unroll
  for (int j = 0; j < NSUB; j++) {
    const uint64_t i0 = chunk_value<W>(c, j, lane);
    int32_t code[W];
    uint64_t b[W], any = 0;
#pragma unroll
    for (int e = 0; e < W; e++) {
      code[e] = encode<T, Q>(x[j][e], f.p, k);
      b[e] = __ballot(code[e] == kSent) & valid_lanes<W>(left, j, e);
      any |= b[e];
    }
    store_codes<W>(f.codes, i0, n, code);
    if (any) {  // uniform
      unsigned r = cnt;
#pragma unroll
      for (int e = 0; e < W; e++) {
        r = lanes_below(b[e], r);
        cnt += (unsigned)__popcll(b[e]);
      }
#pragma unroll
      for (int e = 0; e < W; e++) {
        const bool mine = full ? code[e] == kSent : ((b[e] >> lane) & 1u) != 0;
        if (mine) {
          if (r < kCap) srow[r] = to_bits(x[j][e]);
          r++;
        }
      }
    }
  }
  // other lanes' LDS writes above, then this lane's read: a wavefront-scope
  // fence orders them (LDS accesses of one wavefront complete in issue
  // order, so it costs no wait)
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const unsigned staged = min(cnt, kCap);  // uniform
  for (unsigned b = 0; b < staged; b += 64)
    if (b + (unsigned)lane < staged) f.stage[c * kCap + b + lane] = srow[b + lane];
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // before the next chunk's writes
  if (lane == 0) f.counts[c] = cnt;
  return cnt;
}

// Pass 1 for the CPW * stage_waves<T>() chunks of workgroup `tile`, PF chunks per
// wavefront loaded before any is encoded.
template <typename T, int Q, int CPW, int PF>
__device__ void quant_chunks(const StageField<T> &f, uint64_t tile) {
  static_assert(PF > 0 && CPW % PF == 0, "whole prefetch groups");
  constexpr int kSW = stage_waves<T>();
  constexpr int W = ChunkShape<T>::W, NSUB = ChunkShape<T>::NSUB;
  __shared__ unsigned s_cnt[kSW];
  __shared__ typename FT<T>::U s_stage[kSW][stage_cap<T>()];  // one row per wavefront
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: chunk logic is scalar
  const uint64_t nch = n_chunks(f.n);
  const EncK<T> k = enc_consts_pinned<T, Q>(f.p);
  unsigned wsum = 0;
#pragma unroll
  for (int r0 = 0; r0 < CPW; r0 += PF) {
    T x[PF][NSUB][W];
#pragma unroll
    for (int p = 0; p < PF; p++) {
      const uint64_t c = (tile * CPW + r0 + p) * kSW + wave;
      if (c < nch) load_chunk<T>(f.in, f.n, c, lane, x[p]);
    }
#pragma unroll
    for (int p = 0; p < PF; p++) {
      const uint64_t c = (tile * CPW + r0 + p) * kSW + wave;
      if (c < nch) wsum += encode_chunk<T, Q>(f, c, lane, x[p], s_stage[wave], k);  // uniform
    }
  }
  if (lane == 0) s_cnt[wave] = wsum;
  __syncthreads();
  if (tid == 0) {
    unsigned long long t = 0;
#pragma unroll
    for (int w = 0; w < kSW; w++) t += s_cnt[w];
    if (t) atomicAdd(f.group + tile / f.tiles_per_group, t);
  }
}

// Pass 1 for the cpw * kWaves chunks of workgroup `tile`, cpw given at run
// time (the batched form, where every workgroup item first loads its
// field's descriptor): one chunk per wavefront at a time, chunk (tile cpw +
// r) kWaves + wave in round r.
template <typename T, int Q>
__device__ void quant_chunks_n(const StageField<T> &f, uint64_t tile, unsigned cpw) {
  constexpr int W = ChunkShape<T>::W, NSUB = ChunkShape<T>::NSUB;
  __shared__ unsigned s_cnt[kWaves];
  __shared__ typename FT<T>::U s_stage[kWaves][stage_cap<T>()];  // one row per wavefront
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: chunk logic is scalar
  const uint64_t nch = n_chunks(f.n);
  const EncK<T> k = enc_consts_pinned<T, Q>(f.p);
  unsigned wsum = 0;
  for (unsigned r = 0; r < cpw; r++) {
    const uint64_t c = (tile * cpw + r) * kWaves + wave;
    if (c >= nch) break;  // uniform
    T x[NSUB][W];
    load_chunk<T>(f.in, f.n, c, lane, x);
    wsum += encode_chunk<T, Q>(f, c, lane, x, s_stage[wave], k);
  }
  if (lane == 0) s_cnt[wave] = wsum;
  __syncthreads();
  if (tid == 0) {
    unsigned long long t = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) t += s_cnt[w];
    if (t) atomicAdd(f.group + tile / f.tiles_per_group, t);
  }
}

// ------------------------------------------------------------- pass 2 ---
template <typename T> struct FinishField {
  const T *in;
  uint64_t n;
  uint8_t *stream;
  uint64_t *stream_bytes;
  const uint32_t *counts;
  const typename FT<T>::U *stage;
  const unsigned long long *group;
  uint64_t chunks_per_group;
  uint64_t ngroups;
  const DevParams *noa;  // NOA: header words 4-7 come from here
  uint64_t hdr[8];
};

// Outliers of chunk c from its codes and the input (a chunk with more
// outliers than were staged), written to outl from index P on.  One wavefront; all
// code and value loads of the chunk are issued before the first rank.
template <typename T>
__device__ void rescan_chunk(const FinishField<T> &f, typename FT<T>::U *outl, uint64_t c,
                             uint64_t P, int lane) {
  constexpr int W = ChunkShape<T>::W, NSUB = ChunkShape<T>::NSUB;
  const int32_t *codes = reinterpret_cast<const int32_t *>(f.stream + 64);
  int32_t cc[NSUB][W];
  T x[NSUB][W];
#pragma unroll
  for (int j = 0; j < NSUB; j++) load_codes<W>(codes, chunk_value<W>(c, j, lane), f.n, cc[j]);
  load_chunk<T>(f.in, f.n, c, lane, x);
  const uint64_t left = f.n - c * kChunk;
  uint64_t run = P;
#pragma unroll
  for (int j = 0; j < NSUB; j++) {
    uint64_t b[W];
    uint64_t r = run;
#pragma unroll
    for (int e = 0; e < W; e++) {
      b[e] = __ballot(cc[j][e] == kSent) & valid_lanes<W>(left, j, e);
      r = lanes_below(b[e], (unsigned)0) + r;
      run += (uint64_t)__popcll(b[e]);
    }
#pragma unroll
    for (int e = 0; e < W; e++)
      if ((b[e] >> lane) & 1u) outl[r++] = to_bits(x[j][e]);
  }
}

// The staged row of chunk c (cnt <= stage cap outliers) to outl from index
// P on.  One wavefront; every load is issued before the first store.
template <typename T>
__device__ __forceinline__ void copy_staged(const FinishField<T> &f, typename FT<T>::U *outl,
                                            uint64_t c, uint64_t P, unsigned cnt, int lane) {
  using U = typename FT<T>::U;
  constexpr unsigned kCap = (unsigned)stage_cap<T>();
  constexpr int kR = (int)kCap / 64;
  U v[kR];
#pragma unroll
  for (int r = 0; r < kR; r++) {
    const unsigned i = (unsigned)lane + 64u * r;
    if (i < cnt) v[r] = f.stage[c * kCap + i];
  }
#pragma unroll
  for (int r = 0; r < kR; r++) {
    const unsigned i = (unsigned)lane + 64u * r;
    if (i < cnt) outl[P + i] = v[r];
  }
}

static_assert(LCQ_MAX_N / kChunk <= 0xFFFFFFFFull, "chunk indices fit 32 bits");

// Index of chunk c's first outlier, from the pass-1 group sums and chunk
// counts alone (so any workgroup can find it before the chunk table is
// written).  One wavefront; uniform result.
template <typename T>
__device__ uint64_t chunk_first_outlier(const FinishField<T> &f, uint64_t c, int lane) {
  // chunk and group indices fit 32 bits (n <= LCQ_MAX_N = 2^38)
  const uint64_t gc = (uint32_t)c / (uint32_t)f.chunks_per_group;
  unsigned long long s = 0;
  // eight loads per lane in flight per round (unconditional loads at a
  // clamped index, masked afterwards)
  for (uint64_t i0 = (uint64_t)lane; i0 < gc; i0 += 64 * 8) {
#pragma unroll
    for (int k = 0; k < 8; k++) {
      const uint64_t i = i0 + 64 * (uint64_t)k;
      const unsigned long long v = f.group[i < gc ? i : 0];
      s += i < gc ? v : 0ull;
    }
  }
  for (uint64_t i0 = gc * f.chunks_per_group + (uint64_t)lane; i0 < c; i0 += 64 * 8) {
#pragma unroll
    for (int k = 0; k < 8; k++) {
      const uint64_t i = i0 + 64 * (uint64_t)k;
      const unsigned v = f.counts[i < c ? i : 0];
      s += i < c ? v : 0u;
    }
  }
  return wave_sum(s);
}

// Pass 2 for group g: chunk-table entries of its chunks, their outliers,
// and (last group) header, padding and stream size.
template <typename T>
__device__ void quant_finish(const FinishField<T> &f, uint64_t g) {
  using U = typename FT<T>::U;
  __shared__ unsigned long long s_red[kWaves];
  __shared__ unsigned s_wt[kWaves];
  __shared__ uint64_t s_P[kBlock];
  __shared__ unsigned s_c[kBlock];
  constexpr unsigned kCap = (unsigned)stage_cap<T>();
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t n = f.n;
  const uint64_t nch = n_chunks(n);
  uint64_t *chunk_tab = reinterpret_cast<uint64_t *>(f.stream + chunk_table_offset(n));
  U *outl = reinterpret_cast<U *>(f.stream + outlier_offset(n));

  const uint64_t c0 = g * f.chunks_per_group;
  const uint64_t c1 = min(c0 + f.chunks_per_group, nch);
  // the first batch's count (and the first count of the rescan duty below)
  // is loaded before the earlier groups are summed
  unsigned cnt_next = c0 + tid < c1 ? f.counts[c0 + tid] : 0u;
  const uint64_t cd0 = g + (uint64_t)tid * f.ngroups;
  const unsigned duty0 = cd0 < nch ? f.counts[cd0] : 0u;

  // outliers of all earlier groups: every load issued before the first add
  // (unconditional loads at a clamped index, masked afterwards)
  static_assert(kMaxGroups % kBlock == 0, "whole rounds of group sums");
  unsigned long long b = 0;
#pragma unroll
  for (int k = 0; k < (int)(kMaxGroups / kBlock); k++) {
    const uint64_t i = (uint64_t)tid + (uint64_t)k * kBlock;
    const unsigned long long v = f.group[i < g ? i : 0];
    b += i < g ? v : 0ull;
  }
  b = wave_sum(b);
  if (lane == 0) s_red[wave] = b;
  __syncthreads();
  uint64_t run = 0;
#pragma unroll
  for (int w = 0; w < kWaves; w++) run += s_red[w];

  for (uint64_t cb = c0; cb < c1; cb += kBlock) {
    const uint64_t c = cb + tid;
    const unsigned cnt = cnt_next;
    cnt_next = cb + kBlock + tid < c1 ? f.counts[cb + kBlock + tid] : 0u;
    const unsigned incl = wave_incl_add(cnt);
    if (lane == 63) s_wt[wave] = incl;
    __syncthreads();
    uint64_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) {
      if (w < wave) before += s_wt[w];
      total += s_wt[w];
    }
    const uint64_t P = run + before + (incl - cnt);
    if (c < c1) chunk_tab[c] = P;
    s_P[tid] = before + (incl - cnt);  // batch-relative first outlier of each chunk
    s_c[tid] = cnt;                    // (read after the barrier below)
    const int m = (int)min<uint64_t>((uint64_t)kBlock, c1 - cb);
    __syncthreads();  // s_P and s_c whole
    // staged outliers of chunks with at most kDirect of them: half a
    // wavefront per chunk, word r of a row moved by lane r of the half (one
    // row read and one contiguous run written per instruction); the loads
    // of a round are all issued before its stores
    {
      constexpr int kHalves = kBlock / kDirect, kRound = 16;
      static_assert(kDirect == 32, "a directly copied row is one half wavefront");
      const int h = tid / kDirect, r = tid % kDirect;
      for (int i0 = h; i0 < m; i0 += kHalves * kRound) {
        U v[kRound];
        uint64_t dst[kRound];
        bool mv[kRound];
#pragma unroll
        for (int u = 0; u < kRound; u++) {
          const int i = i0 + u * kHalves;
          const unsigned ci = i < m ? s_c[i] : 0u;
          mv[u] = ci <= (unsigned)kDirect && (unsigned)r < ci;
          dst[u] = mv[u] ? run + s_P[i] + (unsigned)r : 0;
          if (mv[u]) v[u] = f.stage[(cb + (uint64_t)i) * kCap + r];
        }
#pragma unroll
        for (int u = 0; u < kRound; u++)
          if (mv[u]) outl[dst[u]] = v[u];
      }
    }
    run += total;
    __syncthreads();  // s_wt, s_P, s_c are rewritten by the next batch
  }

  // Chunks with more than kDirect outliers are finished not by their own
  // group: workgroup g takes chunks g, g + ngroups, g + 2 ngroups, ... so
  // that runs of such chunks (a stretch of hard data) spread over every
  // workgroup instead of queueing behind one.  One wavefront per such
  // chunk: its staged row is copied, or, past the stage cap, its outliers
  // are rescanned from its codes and input.
  for (uint64_t t0 = 0; g + t0 * f.ngroups < nch; t0 += kBlock) {
    const uint64_t c = g + (t0 + (uint64_t)tid) * f.ngroups;
    const unsigned cn = t0 == 0 ? duty0 : (c < nch ? f.counts[c] : 0u);
    const bool ov = cn > (unsigned)kDirect;
    if (!__syncthreads_or(ov)) continue;
    const uint64_t wb = __ballot(ov);
    if (lane == 0) s_wt[wave] = (unsigned)__popcll(wb);
    __syncthreads();
    unsigned base = 0, nov = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) {
      if (w < wave) base += s_wt[w];
      nov += s_wt[w];
    }
    if (ov) {  // compact list of this batch's chunks and their counts
      s_P[base + lanes_below(wb, 0u)] = c;
      s_c[base + lanes_below(wb, 0u)] = cn;
    }
    __syncthreads();
    for (unsigned i = (unsigned)wave; i < nov; i += kWaves) {
      const uint64_t cv = s_P[i];
      const unsigned cc = s_c[i];
      const uint64_t P = chunk_first_outlier<T>(f, cv, lane);
      if (cc <= kCap) copy_staged<T>(f, outl, cv, P, cc, lane);
      else rescan_chunk<T>(f, outl, cv, P, lane);
    }
    __syncthreads();  // s_wt, s_P and s_c are rewritten by the next batch
  }

  if (g == f.ngroups - 1 && tid == 0) {
    const uint64_t k = run;
    const uint64_t ct = chunk_table_offset(n);
    const uint64_t ce = ct + 8 * nch;
    const uint64_t oo = outlier_offset(n);
    for (uint64_t x = 64 + 4 * n; x < ct; x++) f.stream[x] = 0;
    for (uint64_t x = ce; x < oo; x++) f.stream[x] = 0;
    uint64_t h[8];
#pragma unroll
    for (int i = 0; i < 8; i++) h[i] = f.hdr[i];
    h[2] = k;
    if (f.noa) {
      h[4] = f.noa->step;
      h[5] = f.noa->bound;
      h[6] = f.noa->lo;
      h[7] = f.noa->hi;
    }
    uint64_t *hd = reinterpret_cast<uint64_t *>(f.stream);
#pragma unroll
    for (int i = 0; i < 8; i++) hd[i] = h[i];
    *f.stream_bytes = oo + k * sizeof(T);
  }
}

// ---------------------------------------------------------- dequantize ---
// The 16 codes per lane of chunk c (zeros past n).
template <int W, int NSUB>
__device__ __forceinline__ void load_chunk_codes(const int32_t *codes, uint64_t n, uint64_t c,
                                                 int lane, int32_t (&cc)[NSUB][W]) {
#pragma unroll
  for (int j = 0; j < NSUB; j++) load_codes<W>(codes, chunk_value<W>(c, j, lane), n, cc[j]);
}

// Decode chunk c from its codes cc: gather its outliers, check its
// chunk-table entry, store its values (LIBM: the library-exp2 REL ablation).
// cur and nxt: the chunk's chunk-table entry and the next one (the
// outlier count after the last chunk), loaded by the caller; the outliers
// are at outl (their LCQ1 place for decode_chunk).  REL: the stream's
// quantizer is REL (a template parameter, so each value's decode is
// straight-line code and a sentinel's zero one select).
template <typename T, bool LIBM, bool REL>
__device__ __forceinline__ void decode_chunk_at(const DField<T> &f, uint64_t cur, uint64_t nxt,
                                                const typename FT<T>::U *outl, uint64_t c,
                                                int lane, uint64_t lt,
                                                const int32_t (&cc)[ChunkShape<T>::NSUB][ChunkShape<T>::W]) {
  constexpr int W = ChunkShape<T>::W, NSUB = ChunkShape<T>::NSUB;
  constexpr unsigned kLaneMask = (1u << W) - 1;
  const uint64_t n = f.n;
  unsigned om = 0;
  T y[NSUB][W];
#pragma unroll
  for (int j = 0; j < NSUB; j++) {
    const uint64_t i0 = chunk_value<W>(c, j, lane);
#pragma unroll
    for (int e = 0; e < W; e++) {
      const bool sent = cc[j][e] == kSent;
      const T v = decode<T, LIBM>(cc[j][e], f.step, REL);  // (harmless for a sentinel)
      y[j][e] = sent ? (T)0 : v;
      if (sent && i0 + e < n) om |= 1u << (W * j + e);
    }
  }
  uint64_t cnt = 0;
  if (__ballot(om != 0)) {
#pragma unroll
    for (int j = 0; j < NSUB; j++) {
      unsigned pre;
      const unsigned tot = sub_ranks<W>((om >> (W * j)) & kLaneMask, lt, pre);
      uint64_t r = cur + cnt + pre;
#pragma unroll
      for (int e = 0; e < W; e++) {
        if ((om >> (W * j + e)) & 1u) {
          // ranks are checked against the outlier count: never read past it
          y[j][e] = (r < f.k) ? from_bits(outl[r]) : (T)0;
          r++;
        }
      }
      cnt += tot;
    }
  }
  // the chunk-table entry must count exactly the sentinels before it
  if (lane == 0 && (cur > f.k || nxt - cur != cnt || (c == 0 && cur != 0)))
    report_status(f.status, f.tag, LCQ_ERR_STREAM);
#pragma unroll
  for (int j = 0; j < NSUB; j++) store_vals<T, W>(f.out, chunk_value<W>(c, j, lane), n, y[j]);
}

// decode_chunk_at with the quantizer kind (uniform) made a template
// parameter.  (Making the chunk's fullness one too -- four inlined copies,
// 32-bit position tests -- measured slower: 8-16 us on the REL dequantize,
// 11-47 us on the fused decompress.)
template <typename T, bool LIBM>
__device__ __forceinline__ void decode_chunk_any(const DField<T> &f, uint64_t cur, uint64_t nxt,
                                                 const typename FT<T>::U *outl, uint64_t c,
                                                 int lane, uint64_t lt,
                                                 const int32_t (&cc)[ChunkShape<T>::NSUB][ChunkShape<T>::W]) {
  if (f.rel) decode_chunk_at<T, LIBM, true>(f, cur, nxt, outl, c, lane, lt, cc);
  else decode_chunk_at<T, LIBM, false>(f, cur, nxt, outl, c, lane, lt, cc);
}

template <typename T, bool LIBM>
__device__ __forceinline__ void decode_chunk(const DField<T> &f, uint64_t c, int lane, uint64_t lt,
                                             const int32_t (&cc)[ChunkShape<T>::NSUB][ChunkShape<T>::W]) {
  using U = typename FT<T>::U;
  const uint64_t *chunk_tab = reinterpret_cast<const uint64_t *>(f.stream + chunk_table_offset(f.n));
  const U *outl = reinterpret_cast<const U *>(f.stream + outlier_offset(f.n));
  const uint64_t cur = chunk_tab[c];
  const uint64_t nxt = (c + 1 < n_chunks(f.n)) ? chunk_tab[c + 1] : f.k;
  decode_chunk_any<T, LIBM>(f, cur, nxt, outl, c, lane, lt, cc);
}

// Decode the CPW * kWaves chunks of workgroup `tile`, PF chunks per
// wavefront loaded at a time.
template <typename T, int CPW, int PF, bool LIBM = false>
__device__ void dequant_chunks(const DField<T> &f, uint64_t tile) {
  static_assert(PF > 0 && CPW % PF == 0, "whole prefetch groups");
  constexpr int W = ChunkShape<T>::W, NSUB = ChunkShape<T>::NSUB;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t n = f.n;
  const uint64_t nch = n_chunks(n);
  const int32_t *codes = reinterpret_cast<const int32_t *>(f.stream + 64);
  const uint64_t lt = __lanemask_lt();
#pragma unroll
  for (int r0 = 0; r0 < CPW; r0 += PF) {
    int32_t cc[PF][NSUB][W];
#pragma unroll
    for (int p = 0; p < PF; p++) {
      const uint64_t c = (tile * CPW + r0 + p) * kWaves + wave;
      if (c < nch) load_chunk_codes<W, NSUB>(codes, n, c, lane, cc[p]);
    }
#pragma unroll
    for (int p = 0; p < PF; p++) {
      const uint64_t c = (tile * CPW + r0 + p) * kWaves + wave;
      if (c < nch) decode_chunk<T, LIBM>(f, c, lane, lt, cc[p]);  // uniform
    }
  }
}

}  // namespace lcq
