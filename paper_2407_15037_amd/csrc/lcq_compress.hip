// lcq_compress.hip -- the quantizer and the lossless packing stage fused,
// for gfx950.
//
// lcq_compress writes the bytes lcq_pack(lcq_quantize(x)) would, without
// the int32 codes ever reaching memory; lcq_decompress decodes a packed
// stream straight to values, as lcq_dequantize(lcq_unpack(p)) would.  Both
// directions are bound by HBM bandwidth, and the codes are the bulky
// intermediate (4 bytes per value against about 1.4 packed): not storing
// and re-reading them is what fusing buys.  The price on the compress side
// is reading the input twice, once to size the records and once to write
// them: the second pass takes the outliers from the first pass's flags and
// recomputes only the bins, with the same operations as the encoder, so
// both passes see the same codes.
//
// Kernels (one wavefront per 1024-value chunk, the chunk kernels' lane
// layout, lcq_chunk.hpp):
//   k_cmp_stage   pass 1: classify / bin / reconstruct / verify (sections
//                 2.2, 3.1-3.3) of each value; the chunk's outliers staged as
//                 in the two-pass quantize; its record's width, mode and
//                 size; per workgroup one atomic add of its outlier count and
//                 one of its record bytes into its group's sums
//   k_cmp_finish  pass 2, one workgroup per group: chunk table and record
//                 offsets (two exclusive scans), outliers copied to their
//                 place behind the payload, and (last group) header, padding
//                 and size
//   k_cmp_write   pass 3: each chunk's codes again from the input -- the
//                 outliers as pass 1 flagged them, the other values' bins
//                 recomputed -- and its record (header, outlier bitmap,
//                 packed bits assembled in LDS) written at its offset
//   k_decompress  per chunk: record checks, codes from the record's bits,
//                 then the dequantize path's decode and outlier gather
//                 (section 3) and one store of the values
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>

#include "lcq.h"
#include "lcq_chunk.hpp"
#include "lcq_host.hpp"
#include "lcq_math.hpp"
#include "lcq_packfmt.hpp"
#include "lcq_range.hpp"
#include "lcq_tile.hpp"

#pragma clang fp contract(off)

using namespace lcq;

namespace {

struct CmpArgs {
  const void *in;
  uint64_t n;
  uint8_t *out;                // packed stream
  uint64_t *out_bytes;
  uint32_t *counts;            // outliers per chunk
  uint32_t *meta;              // w | mode << 8 | hb << 16 per chunk
  uint32_t *sizes;             // record bytes per chunk
  uint16_t *flags;             // per lane of a chunk with outliers: its outlier flags
  void *stage;                 // stage_cap<T>() raw outliers per chunk
  unsigned long long *group;   // outliers per group of workgroups
  unsigned long long *rgroup;  // record bytes per group
  uint64_t tiles_per_group, chunks_per_group, ngroups;
  const DevParams *noa;        // NOA: parameters computed on the device
  uint64_t step, inv, bound, low;  // ABS / REL parameters (raw bits)
  uint64_t hdr[8];                 // header of the packed stream
};

template <typename T, int Q>
__device__ __forceinline__ FieldParams<T> cmp_params(const CmpArgs &a) {
  using U = typename FT<T>::U;
  if constexpr (Q == kNOA) return params_from<T>(*a.noa);
  FieldParams<T> p;
  p.step = from_bits((U)a.step);
  p.inv = from_bits((U)a.inv);
  p.bound = from_bits((U)a.bound);
  p.low = from_bits((U)a.low);
  p.lossless_all = 0;
  return p;
}

// Codes of chunk c (values x in the chunk lane layout) as c' values --
// the code, or 0 for an outlier -- and the outlier flags (bit W j + e: the
// lane's position j, e, below len).  STAGE: the first stage_cap<T>()
// outliers also go, at their ranks, through the wavefront's LDS row srow to
// stage_row, as encode_chunk stages them.  FULL: the chunk has 1024 values.
// Returns the chunk's outlier count.
template <typename T, int Q, bool STAGE, bool FULL>
__device__ __forceinline__ unsigned encode_keep(
    const T (&x)[ChunkShape<T>::NSUB][ChunkShape<T>::W], const FieldParams<T> &p,
    const EncK<T> &k, unsigned len, int lane, typename FT<T>::U *srow,
    typename FT<T>::U *stage_row, uint32_t (&cv)[ChunkShape<T>::NSUB][ChunkShape<T>::W],
    unsigned &flags) {
  constexpr int W = ChunkShape<T>::W, NSUB = ChunkShape<T>::NSUB;
  constexpr unsigned kCap = (unsigned)stage_cap<T>();
  unsigned cnt = 0;
  flags = 0;
#pragma unroll
  for (int j = 0; j < NSUB; j++) {
    const unsigned pos = chunk_pos<W>(j, lane);
    bool fs[W];
    uint64_t b[W], any = 0;
#pragma unroll
    for (int e = 0; e < W; e++) {
      const int32_t code = encode<T, Q>(x[j][e], p, k);
      const bool s = code == kSent;
      fs[e] = FULL ? s : (s && pos + e < len);
      b[e] = __ballot(fs[e]);
      any |= b[e];
      cv[j][e] = s ? 0u : (uint32_t)code;
      flags |= (fs[e] ? 1u : 0u) << (W * j + e);
    }
    if (any) {  // uniform
      unsigned r = cnt;
#pragma unroll
      for (int e = 0; e < W; e++) {
        r = lanes_below(b[e], r);
        cnt += (unsigned)__popcll(b[e]);
      }
      if constexpr (STAGE) {
#pragma unroll
        for (int e = 0; e < W; e++) {
          if (fs[e]) {
            if (r < kCap) srow[r] = to_bits(x[j][e]);
            r++;
          }
        }
      }
    }
  }
  if constexpr (STAGE) {
    // other lanes' LDS writes, then this lane's reads: LDS accesses of one
    // wavefront complete in issue order, so a wavefront-scope fence orders
    // them
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const unsigned staged = min(cnt, kCap);  // uniform
    for (unsigned b0 = 0; b0 < staged; b0 += 64)
      if (b0 + (unsigned)lane < staged) stage_row[b0 + lane] = srow[b0 + lane];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
  return cnt;
}

// Pass 1 for one chunk: its outliers staged, its count, width, mode and
// record size (all lanes get the count and the record size).
template <typename T, int Q, bool FULL>
__device__ __forceinline__ void stage_chunk(const CmpArgs &a, const FieldParams<T> &p,
                                            const EncK<T> &k, uint64_t c, unsigned len, int lane,
                                            const T (&x)[ChunkShape<T>::NSUB][ChunkShape<T>::W],
                                            typename FT<T>::U *srow, unsigned &cnt, unsigned &rb) {
  using U = typename FT<T>::U;
  constexpr int W = ChunkShape<T>::W, NSUB = ChunkShape<T>::NSUB;
  constexpr unsigned kCap = (unsigned)stage_cap<T>();
  uint32_t cv[NSUB][W];
  unsigned flags;
  cnt = encode_keep<T, Q, true, FULL>(x, p, k, len, lane, srow,
                                      static_cast<U *>(a.stage) + c * kCap, cv, flags);
  unsigned w, mode;
  chunk_width<FULL, W, NSUB>(cv, len, lane, w, mode);
  const unsigned hb = cnt ? 1u : 0u;
  rb = (unsigned)record_bytes(len, w, hb);
  if (hb) a.flags[c * 64 + lane] = (uint16_t)flags;
  if (lane == 0) {
    a.counts[c] = cnt;
    a.meta[c] = w | (mode << 8) | (hb << 16);
    a.sizes[c] = rb;
  }
}

// The 16 values per lane of chunk c, with ordinary (cache-allocating)
// loads when the chunk is full: the read-only first pass measured faster
// with them than with streaming loads (6 us ABS, 12-18 us REL on the 512^3
// float32 field).
template <typename T>
__device__ __forceinline__ void load_chunk_cached(const T *in, uint64_t n, uint64_t c, int lane,
                                                  T (&x)[ChunkShape<T>::NSUB][ChunkShape<T>::W]) {
  constexpr int W = ChunkShape<T>::W, NSUB = ChunkShape<T>::NSUB;
  if (n - c * kChunk >= kChunk) {
#pragma unroll
    for (int j = 0; j < NSUB; j++) {
      const uint64_t i0 = chunk_value<W>(c, j, lane);
      if constexpr (sizeof(T) == 4) {
        const nt_f4 v = *reinterpret_cast<const nt_f4 *>(in + i0);
        x[j][0] = v.x; x[j][1] = v.y; x[j][2] = v.z; x[j][3] = v.w;
      } else {
        const nt_d2 v = *reinterpret_cast<const nt_d2 *>(in + i0);
        x[j][0] = v.x; x[j][1] = v.y;
      }
    }
  } else {
    load_chunk<T>(in, n, c, lane, x);
  }
}

// Pass 1 for the kCmpCpw * kWaves chunks of workgroup blockIdx.x: chunk
// (tile kCmpCpw + r) kWaves + wave in round r, every round's input loaded
// before the first is encoded.  (2 and 4 chunks per wavefront measured
// slower than 1 on the 512^3 float32 field: compress 263-272 us against
// 253 us for ABS; their registers cost more occupancy than the extra loads
// in flight gain.)
constexpr int kCmpCpw = 1;

template <typename T, int Q>
__global__ __launch_bounds__(kBlock) void k_cmp_stage(CmpArgs a) {
  using U = typename FT<T>::U;
  constexpr int W = ChunkShape<T>::W, NSUB = ChunkShape<T>::NSUB;
  constexpr unsigned kCap = (unsigned)stage_cap<T>();
  __shared__ unsigned s_cnt[kWaves], s_rb[kWaves];
  __shared__ U s_stage[kWaves][kCap];  // one row per wavefront
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: chunk logic is scalar
  const uint64_t n = a.n, nch = n_chunks(n);
  const FieldParams<T> p = cmp_params<T, Q>(a);
  const EncK<T> k = enc_consts_pinned<T, Q>(p);
  unsigned cnt = 0, rb = 0;
  T x[kCmpCpw][NSUB][W];
#pragma unroll
  for (int r = 0; r < kCmpCpw; r++) {
    const uint64_t c = ((uint64_t)blockIdx.x * kCmpCpw + r) * kWaves + wave;
    if (c < nch) load_chunk_cached<T>(static_cast<const T *>(a.in), n, c, lane, x[r]);
  }
#pragma unroll
  for (int r = 0; r < kCmpCpw; r++) {
    const uint64_t c = ((uint64_t)blockIdx.x * kCmpCpw + r) * kWaves + wave;
    if (c < nch) {  // uniform over the wavefront
      const unsigned len = chunk_len(n, c);
      unsigned cc, rr;
      if (len == kChunk) stage_chunk<T, Q, true>(a, p, k, c, len, lane, x[r], s_stage[wave], cc, rr);
      else stage_chunk<T, Q, false>(a, p, k, c, len, lane, x[r], s_stage[wave], cc, rr);
      cnt += cc;
      rb += rr;
    }
  }
  if (lane == 0) {
    s_cnt[wave] = cnt;
    s_rb[wave] = rb;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long t = 0, r = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) {
      t += s_cnt[w];
      r += s_rb[w];
    }
    const uint64_t g = blockIdx.x / a.tiles_per_group;
    if (t) atomicAdd(a.group + g, t);
    if (r) atomicAdd(a.rgroup + g, r);
  }
}

// Outliers of chunk c found by encoding it again (a chunk with more
// outliers than were staged), written to outl from index P on.  One
// wavefront.
template <typename T, int Q>
__device__ void rescan_encode(const CmpArgs &a, const FieldParams<T> &p,
                              typename FT<T>::U *outl, uint64_t c, uint64_t P, int lane) {
  constexpr int W = ChunkShape<T>::W, NSUB = ChunkShape<T>::NSUB;
  const EncK<T> k = enc_consts<T, Q>(p);
  const uint64_t n = a.n;
  T x[NSUB][W];
  load_chunk<T>(static_cast<const T *>(a.in), n, c, lane, x);
  const uint64_t left = n - c * kChunk;
  uint64_t run = P;
#pragma unroll
  for (int j = 0; j < NSUB; j++) {
    uint64_t b[W];
    uint64_t r = run;
#pragma unroll
    for (int e = 0; e < W; e++) {
      b[e] = __ballot(encode<T, Q>(x[j][e], p, k) == kSent) & valid_lanes<W>(left, j, e);
      r = lanes_below(b[e], (unsigned)0) + r;
      run += (uint64_t)__popcll(b[e]);
    }
#pragma unroll
    for (int e = 0; e < W; e++)
      if ((b[e] >> lane) & 1u) outl[r++] = to_bits(x[j][e]);
  }
}

// Pass 2 for group g.  The outliers' place follows the payload, whose size
// (all groups' record bytes) every workgroup sums for itself.
template <typename T, int Q>
__global__ __launch_bounds__(kBlock) void k_cmp_finish(CmpArgs a) {
  using U = typename FT<T>::U;
  __shared__ unsigned long long s_red[3][kWaves];
  __shared__ unsigned s_wt[2][kWaves];
  __shared__ uint64_t s_P[kBlock];
  __shared__ unsigned s_c[kBlock];
  constexpr unsigned kCap = (unsigned)stage_cap<T>();
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t g = blockIdx.x;
  const uint64_t n = a.n, nch = n_chunks(n);
  const uint64_t ot = packed_table_offset(nch), pl = packed_payload_offset(nch);
  FinishField<T> f{};
  f.in = static_cast<const T *>(a.in);
  f.n = n;
  f.stream = a.out;
  f.counts = a.counts;
  f.stage = static_cast<const U *>(a.stage);
  f.group = a.group;
  f.chunks_per_group = a.chunks_per_group;
  f.ngroups = a.ngroups;

  const uint64_t c0 = g * a.chunks_per_group;
  const uint64_t c1 = min(c0 + a.chunks_per_group, nch);
  // the first batch's counts and sizes, and the first heavy-chunk duty
  // count, are loaded before the group sums are reduced
  unsigned cnt_next = c0 + tid < c1 ? a.counts[c0 + tid] : 0u;
  unsigned sz_next = c0 + tid < c1 ? a.sizes[c0 + tid] : 0u;
  const uint64_t cd0 = g + (uint64_t)tid * a.ngroups;
  const unsigned duty0 = cd0 < nch ? a.counts[cd0] : 0u;

  // outliers and record bytes of the earlier groups, and the record bytes
  // of all groups (unconditional loads at a clamped index, masked after)
  static_assert(kMaxGroups % kBlock == 0, "whole rounds of group sums");
  unsigned long long bo = 0, br = 0, bt = 0;
#pragma unroll
  for (int r = 0; r < (int)(kMaxGroups / kBlock); r++) {
    const uint64_t i = (uint64_t)tid + (uint64_t)r * kBlock;
    const unsigned long long vo = a.group[i < g ? i : 0];
    const unsigned long long vr = a.rgroup[i < a.ngroups ? i : 0];
    bo += i < g ? vo : 0ull;
    br += i < g ? vr : 0ull;
    bt += i < a.ngroups ? vr : 0ull;
  }
  bo = wave_sum(bo);
  br = wave_sum(br);
  bt = wave_sum(bt);
  if (lane == 0) {
    s_red[0][wave] = bo;
    s_red[1][wave] = br;
    s_red[2][wave] = bt;
  }
  __syncthreads();
  uint64_t run = 0, rrun = 0, payload = 0;
#pragma unroll
  for (int w = 0; w < kWaves; w++) {
    run += s_red[0][w];
    rrun += s_red[1][w];
    payload += s_red[2][w];
  }
  const uint64_t oo = align16(pl + payload);
  U *outl = reinterpret_cast<U *>(a.out + oo);
  uint64_t *chunk_tab = reinterpret_cast<uint64_t *>(a.out + 64);
  uint64_t *offs = reinterpret_cast<uint64_t *>(a.out + ot);

  for (uint64_t cb = c0; cb < c1; cb += kBlock) {
    const uint64_t c = cb + tid;
    const unsigned cnt = cnt_next, sz = sz_next;
    cnt_next = cb + kBlock + tid < c1 ? a.counts[cb + kBlock + tid] : 0u;
    sz_next = cb + kBlock + tid < c1 ? a.sizes[cb + kBlock + tid] : 0u;
    // (a batch's record bytes fit 32 bits)
    const unsigned incl = wave_incl_add(cnt), sincl = wave_incl_add(sz);
    if (lane == 63) {
      s_wt[0][wave] = incl;
      s_wt[1][wave] = sincl;
    }
    __syncthreads();
    uint64_t before = 0, total = 0, sbefore = 0, stotal = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) {
      if (w < wave) {
        before += s_wt[0][w];
        sbefore += s_wt[1][w];
      }
      total += s_wt[0][w];
      stotal += s_wt[1][w];
    }
    if (c < c1) {
      chunk_tab[c] = run + before + (incl - cnt);
      offs[c] = rrun + sbefore + (sincl - sz);
    }
    s_P[tid] = before + (incl - cnt);  // batch-relative first outlier of each chunk
    s_c[tid] = cnt;
    const int m = (int)min<uint64_t>((uint64_t)kBlock, c1 - cb);
    __syncthreads();  // s_P and s_c whole
    // staged rows of chunks with at most kDirect outliers: half a wavefront
    // per chunk, word r of a row moved by lane r of the half
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
    rrun += stotal;
    __syncthreads();  // s_wt, s_P, s_c are rewritten by the next batch
  }

  // chunks with more than kDirect outliers, spread over every workgroup
  // (workgroup g takes chunks g, g + ngroups, ...): one wavefront per chunk
  // copies its staged row or, past the stage cap, encodes the chunk again
  for (uint64_t t0 = 0; g + t0 * a.ngroups < nch; t0 += kBlock) {
    const uint64_t c = g + (t0 + (uint64_t)tid) * a.ngroups;
    const unsigned cn = t0 == 0 ? duty0 : (c < nch ? a.counts[c] : 0u);
    const bool ov = cn > (unsigned)kDirect;
    if (!__syncthreads_or(ov)) continue;
    const uint64_t wb = __ballot(ov);
    if (lane == 0) s_wt[0][wave] = (unsigned)__popcll(wb);
    __syncthreads();
    unsigned base = 0, nov = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) {
      if (w < wave) base += s_wt[0][w];
      nov += s_wt[0][w];
    }
    if (ov) {
      s_P[base + lanes_below(wb, 0u)] = c;
      s_c[base + lanes_below(wb, 0u)] = cn;
    }
    __syncthreads();
    for (unsigned i = (unsigned)wave; i < nov; i += kWaves) {
      const uint64_t cv = s_P[i];
      const unsigned cc = s_c[i];
      const uint64_t P = chunk_first_outlier<T>(f, cv, lane);
      if (cc <= kCap) copy_staged<T>(f, outl, cv, P, cc, lane);
      else rescan_encode<T, Q>(a, cmp_params<T, Q>(a), outl, cv, P, lane);
    }
    __syncthreads();  // s_wt, s_P and s_c are rewritten by the next batch
  }

  if (g == a.ngroups - 1 && tid == 0) {
    const uint64_t k = run;
    uint64_t h[8];
#pragma unroll
    for (int i = 0; i < 8; i++) h[i] = a.hdr[i];
    h[2] = k;
    if constexpr (Q == kNOA) {
      h[4] = a.noa->step;
      h[5] = a.noa->bound;
      h[6] = a.noa->lo;
      h[7] = a.noa->hi;
    }
    uint64_t *hd = reinterpret_cast<uint64_t *>(a.out);
#pragma unroll
    for (int i = 0; i < 8; i++) hd[i] = h[i];
    offs[nch] = payload;
    for (uint64_t x = 64 + 8 * nch; x < ot; x++) a.out[x] = 0;
    for (uint64_t x = ot + 8 * (nch + 1); x < pl; x++) a.out[x] = 0;
    for (uint64_t x = pl + payload; x < oo; x++) a.out[x] = 0;
    *a.out_bytes = oo + k * sizeof(T);
  }
}

// c' of x: 0 for an outlier, else x's code -- its bin computed by the
// same operations as in encode (section 3.3 for REL), in the same order;
// the classification, reconstruction and check that decided which values
// are outliers were made by the first pass, whose flags say so.
template <typename T, int Q>
__device__ __forceinline__ uint32_t bin_code(T x, const FieldParams<T> &p, bool outlier) {
  if constexpr (is_rel_q<Q>()) {
    const T q = rel_bin(x, p.inv);
    const int32_t b = (int32_t)(outlier ? (T)0 : q);  // in range when not an outlier
    const uint32_t hi = (uint32_t)(to_bits(x) >> (sizeof(T) * 8 - 32));
    const uint32_t code = __builtin_amdgcn_alignbit((uint32_t)b, hi, 31);
    return outlier ? 0u : code;
  } else {
    const T q = rint_t(x * p.inv);
    return (uint32_t)(int32_t)(outlier ? (T)0 : q);  // in range when not an outlier
  }
}

// Pass 3 for one chunk: its c' values again (the first pass's outlier
// flags, the bins recomputed), its record written at rec.
template <typename T, int Q, bool FULL>
__device__ __forceinline__ void write_chunk(const CmpArgs &a, const FieldParams<T> &p, uint64_t c,
                                            uint32_t m, unsigned len, int lane,
                                            const T (&x)[ChunkShape<T>::NSUB][ChunkShape<T>::W],
                                            uint32_t *row, uint8_t *rec) {
  constexpr int W = ChunkShape<T>::W, NSUB = ChunkShape<T>::NSUB;
  const unsigned w = m & 0xFF, mode = (m >> 8) & 1, hb = (m >> 16) & 1;
  const unsigned flags = hb ? (unsigned)a.flags[c * 64 + lane] : 0u;
  uint32_t cv[NSUB][W];
#pragma unroll
  for (int j = 0; j < NSUB; j++) {
    const unsigned pos = chunk_pos<W>(j, lane);
#pragma unroll
    for (int e = 0; e < W; e++) {
      // positions past the end count as outliers: c' 0, no bin computed
      const bool out = ((flags >> (W * j + e)) & 1u) != 0 || (!FULL && pos + e >= len);
      cv[j][e] = bin_code<T, Q>(x[j][e], p, out);
    }
  }
  uint32_t z[NSUB][W];
  if (mode) chunk_z<true, W, NSUB, FULL>(cv, len, lane, z);
  else chunk_z<false, W, NSUB, FULL>(cv, len, lane, z);
  pack_bits<W, NSUB>(z, len, w, row, lane);
  write_record_head<W, NSUB>(rec, w, mode, hb, flags, lane);
  copy_words(row, packed_words(len, w), reinterpret_cast<uint32_t *>(rec + 16 + (hb ? 128 : 0)),
             lane);
}

template <typename T, int Q>
__global__ __launch_bounds__(kBlock) void k_cmp_write(CmpArgs a) {
  constexpr int W = ChunkShape<T>::W, NSUB = ChunkShape<T>::NSUB;
  __shared__ uint32_t s_w[kWaves][kChunk];  // each wavefront's packed words
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t n = a.n, nch = n_chunks(n);
  const uint64_t c = (uint64_t)blockIdx.x * kWaves + wave;
  if (c >= nch) return;  // uniform over the wavefront; no barrier follows
  const uint64_t ot = packed_table_offset(nch), pl = packed_payload_offset(nch);
  const FieldParams<T> p = cmp_params<T, Q>(a);
  const uint32_t m = a.meta[c];
  const unsigned len = chunk_len(n, c);
  uint8_t *rec = a.out + pl + reinterpret_cast<const uint64_t *>(a.out + ot)[c];
  T x[NSUB][W];
  load_chunk<T>(static_cast<const T *>(a.in), n, c, lane, x);
  if (len == kChunk) write_chunk<T, Q, true>(a, p, c, m, len, lane, x, s_w[wave], rec);
  else write_chunk<T, Q, false>(a, p, c, m, len, lane, x, s_w[wave], rec);
}

struct DcmpArgs {
  const uint8_t *in;  // packed stream
  uint64_t in_bytes;
  uint64_t n;
  void *out;
  unsigned long long *status;
  uint64_t epoch;
  int dtype;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_decompress(DcmpArgs a) {
  using U = typename FT<T>::U;
  constexpr int W = ChunkShape<T>::W, NSUB = ChunkShape<T>::NSUB;
  __shared__ uint32_t s_rec[kWaves][kMaxRecord / 4 + kRowPad];  // each wavefront's whole record
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t n = a.n, nch = n_chunks(n);
  const uint64_t ot = packed_table_offset(nch), pl = packed_payload_offset(nch);
  const unsigned long long tag = (unsigned long long)(a.epoch << 16);
  // header and table bounds (the host checked in_bytes >= pl)
  const uint64_t *hd = reinterpret_cast<const uint64_t *>(a.in);
  const uint64_t h0 = hd[0], k = hd[2];
  const int q = (int)((h0 >> 48) & 0xFF);
  const uint64_t *offs = reinterpret_cast<const uint64_t *>(a.in + ot);
  const uint64_t payload = offs[nch];
  const bool bad = (h0 & ~(0xFFull << 48)) != packed_word0(a.dtype) || q > 2 || hd[1] != n ||
                   k > n || payload > a.in_bytes - pl ||
                   align16(pl + payload) + k * sizeof(T) > a.in_bytes;
  if (blockIdx.x == 0 && threadIdx.x == 0)
    report_status(a.status, tag, bad ? LCQ_ERR_STREAM : LCQ_OK);
  if (bad || n == 0) return;
  const uint64_t c = (uint64_t)blockIdx.x * kWaves + wave;
  if (c >= nch) return;  // uniform over the wavefront; no barrier follows
  // the record's extent from the offset table: whole 16-byte units inside
  // the payload, at most the largest record
  const uint64_t off = offs[c], nxt = offs[c + 1];
  // the chunk-table entries the decode checks, loaded with the offsets
  const uint64_t *chunk_tab = reinterpret_cast<const uint64_t *>(a.in + 64);
  const uint64_t ct_cur = chunk_tab[c], ct_nxt = c + 1 < nch ? chunk_tab[c + 1] : k;
  const unsigned len = chunk_len(n, c);
  bool ok = record_extent_ok(off, nxt, payload);
  if (!ok) {
    if (lane == 0) report_status(a.status, tag, LCQ_ERR_STREAM);
    return;
  }
  // the whole record (header, bitmap, bits) staged in LDS with 128-bit
  // loads, one round trip; then its header decides the rest
  uint32_t *row = s_rec[wave];
  stage_words(a.in + pl + off, (unsigned)((nxt - off) / 4), row, lane);
  const uint32_t h = row[0];
  const unsigned w = h & 0xFF, mode = (h >> 8) & 0xFF, hb = (h >> 16) & 0xFF;
  ok = w <= 32 && mode <= 1 && hb <= 1 && nxt - off == record_bytes(len, w, hb);
  if (!ok) {
    if (lane == 0) report_status(a.status, tag, LCQ_ERR_STREAM);
    return;
  }
  int32_t cc[NSUB][W];
  record_codes<W, NSUB>(row + (hb ? 36 : 4), hb ? reinterpret_cast<const uint8_t *>(row + 4) : nullptr,
                        w, mode, lane, cc);
  DField<T> f;
  f.stream = a.in;
  f.n = n;
  f.k = k;
  f.step = from_bits((U)hd[4]);
  f.rel = q == kREL;
  f.out = static_cast<T *>(a.out);
  f.status = a.status;
  f.tag = tag;
  const U *outl = reinterpret_cast<const U *>(a.in + align16(pl + payload));
  decode_chunk_any<T, false>(f, ct_cur, ct_nxt, outl, c, lane, __lanemask_lt(), cc);
}

__global__ void k_clear_cmp(uint64_t *p, uint64_t count) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// ------------------------------------------------------------ workspace ---
// [0,8)       status word of the last decompress that used it
// [64,128)    NOA parameters (DevParams)
// [256, ...)  outliers per group, then record bytes per group (kMaxGroups
//             each), cleared by every compress
// then        counts, meta and record sizes (4 bytes per chunk each), the
//             outlier flags (2 bytes per lane of a chunk), the staged
//             outliers (stage_cap<T>() per chunk), NOA's range pairs
constexpr uint64_t kCwParams = 64, kCwGroups = 256;
uint64_t al256(uint64_t v) { return (v + 255) & ~255ull; }
uint64_t cw_counts_off() { return al256(kCwGroups + 16 * kMaxGroups); }
uint64_t cw_meta_off(uint64_t C) { return al256(cw_counts_off() + 4 * C); }
uint64_t cw_sizes_off(uint64_t C) { return al256(cw_meta_off(C) + 4 * C); }
uint64_t cw_flags_off(uint64_t C) { return al256(cw_sizes_off(C) + 4 * C); }
uint64_t cw_stage_off(uint64_t C) { return al256(cw_flags_off(C) + 128 * C); }
uint64_t cw_partials_off(lcq_dtype t, uint64_t C) {
  const uint64_t cap = t == LCQ_F64 ? 8ull * stage_cap<double>() : 4ull * stage_cap<float>();
  return al256(cw_stage_off(C) + cap * C);
}
uint64_t cw_need(lcq_quantizer q, lcq_dtype t, uint64_t n) {
  return cw_partials_off(t, n_chunks(n)) + (q == LCQ_NOA ? 16ull * kMinmaxBlocks : 0);
}

lcq_status check_launch_cmp() { return hipGetLastError() == hipSuccess ? LCQ_OK : LCQ_ERR_HIP; }

// Decode-call epochs tag the status word (as for the other decoders);
// seeded from the clock so a workspace left over from another process
// cannot match.
std::atomic<uint64_t> g_cmp_epoch{
    ((uint64_t)std::chrono::steady_clock::now().time_since_epoch().count() ^ 0x3C3C3C3C3ull) &
    0xFFFFFFFFFFFull};

template <typename T, int Q>
lcq_status run_compress(double eb, const void *d_in, uint64_t n, void *d_out, uint64_t *d_bytes,
                        void *d_ws, hipStream_t s) {
  const int dt = sizeof(T) == 8 ? LCQ_F64 : LCQ_F32;
  const HostParams hp = host_params<T>(Q, eb);
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  const uint64_t C = n_chunks(n);
  const uint64_t ntiles = (C + kWaves - 1) / kWaves;  // pass 3: one chunk per wavefront
  const uint64_t stiles = (C + kWaves * kCmpCpw - 1) / (kWaves * kCmpCpw);  // pass 1
  CmpArgs a{};
  a.in = d_in;
  a.n = n;
  a.out = static_cast<uint8_t *>(d_out);
  a.out_bytes = d_bytes;
  a.counts = reinterpret_cast<uint32_t *>(ws + cw_counts_off());
  a.meta = reinterpret_cast<uint32_t *>(ws + cw_meta_off(C));
  a.sizes = reinterpret_cast<uint32_t *>(ws + cw_sizes_off(C));
  a.flags = reinterpret_cast<uint16_t *>(ws + cw_flags_off(C));
  a.stage = ws + cw_stage_off(C);
  a.group = reinterpret_cast<unsigned long long *>(ws + kCwGroups);
  a.rgroup = a.group + kMaxGroups;
  a.tiles_per_group = tiles_per_group(stiles, kWaves * kCmpCpw);
  a.chunks_per_group = a.tiles_per_group * kWaves * kCmpCpw;
  a.ngroups = std::max<uint64_t>(1, (stiles + a.tiles_per_group - 1) / a.tiles_per_group);
  a.noa = reinterpret_cast<const DevParams *>(ws + kCwParams);
  a.step = hp.step;
  a.inv = hp.inv;
  a.bound = hp.bound;
  a.low = hp.low;
  a.hdr[0] = (header_word0(dt, Q) & ~0xFFFFFFFFull) | kMagicPacked;
  a.hdr[1] = n;
  a.hdr[2] = 0;
  a.hdr[3] = __builtin_bit_cast(uint64_t, eb);
  a.hdr[4] = hp.step;
  a.hdr[5] = hp.bound;
  a.hdr[6] = hp.aux0;
  a.hdr[7] = hp.aux1;
  uint64_t *clear_ptr = reinterpret_cast<uint64_t *>(a.group);
  const uint64_t clear_count = 2 * kMaxGroups;
  if (Q == kNOA) {
    T *partials = reinterpret_cast<T *>(ws + cw_partials_off((lcq_dtype)dt, C));
    launch_noa_range<T>(static_cast<const T *>(d_in), n, partials, clear_ptr, clear_count,
                        from_bits((typename FT<T>::U)hp.eb_down),
                        reinterpret_cast<DevParams *>(ws + kCwParams), s);
  } else {
    hipLaunchKernelGGL(k_clear_cmp, dim3((unsigned)(clear_count / kBlock)), dim3(kBlock), 0, s,
                       clear_ptr, clear_count);
  }
  if (ntiles)
    hipLaunchKernelGGL((k_cmp_stage<T, Q>), dim3((unsigned)stiles), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL((k_cmp_finish<T, Q>), dim3((unsigned)a.ngroups), dim3(kBlock), 0, s, a);
  if (ntiles)
    hipLaunchKernelGGL((k_cmp_write<T, Q>), dim3((unsigned)ntiles), dim3(kBlock), 0, s, a);
  return check_launch_cmp();
}

}  // namespace

extern "C" {

uint64_t lcq_compress_workspace_bytes(lcq_quantizer q, lcq_dtype t, uint64_t n) {
  if ((t != LCQ_F32 && t != LCQ_F64) || (q != LCQ_ABS && q != LCQ_REL && q != LCQ_NOA) ||
      n > LCQ_MAX_N)
    return 0;
  return cw_need(q, t, n);
}

lcq_status lcq_compress(lcq_quantizer q, lcq_dtype t, double eb, const void *d_in, uint64_t n,
                        void *d_packed, uint64_t packed_cap, uint64_t *d_packed_bytes, void *d_ws,
                        uint64_t ws_bytes, hipStream_t stream) {
  if (q != LCQ_ABS && q != LCQ_REL && q != LCQ_NOA) return LCQ_ERR_ARG;
  if (t != LCQ_F32 && t != LCQ_F64) return LCQ_ERR_ARG;
  if (!(eb > 0.0) || !std::isfinite(eb) || (q == LCQ_REL && !(eb < 1.0))) return LCQ_ERR_ARG;
  if (n > LCQ_MAX_N) return LCQ_ERR_ARG;
  if ((n && !d_in) || !d_packed || !d_packed_bytes || !d_ws) return LCQ_ERR_ARG;
  if ((n && !aligned16(d_in)) || !aligned16(d_packed) || !aligned16(d_ws) ||
      ((uintptr_t)d_packed_bytes & 7u))
    return LCQ_ERR_ARG;
  if (packed_cap < lcq_pack_max_bytes(t, n)) return LCQ_ERR_CAPACITY;
  if (ws_bytes < cw_need(q, t, n)) return LCQ_ERR_CAPACITY;
  if (t == LCQ_F32) {
    switch (q) {
      case LCQ_ABS: return run_compress<float, kABS>(eb, d_in, n, d_packed, d_packed_bytes, d_ws, stream);
      case LCQ_REL: return run_compress<float, kREL>(eb, d_in, n, d_packed, d_packed_bytes, d_ws, stream);
      default: return run_compress<float, kNOA>(eb, d_in, n, d_packed, d_packed_bytes, d_ws, stream);
    }
  }
  switch (q) {
    case LCQ_ABS: return run_compress<double, kABS>(eb, d_in, n, d_packed, d_packed_bytes, d_ws, stream);
    case LCQ_REL: return run_compress<double, kREL>(eb, d_in, n, d_packed, d_packed_bytes, d_ws, stream);
    default: return run_compress<double, kNOA>(eb, d_in, n, d_packed, d_packed_bytes, d_ws, stream);
  }
}

lcq_status lcq_decompress(lcq_dtype t, const void *d_packed, uint64_t packed_bytes, void *d_out,
                          uint64_t n, void *d_ws, uint64_t ws_bytes, hipStream_t stream) {
  if (t != LCQ_F32 && t != LCQ_F64) return LCQ_ERR_ARG;
  if (n > LCQ_MAX_N) return LCQ_ERR_ARG;
  if (!d_packed || (n && !d_out) || !d_ws) return LCQ_ERR_ARG;
  if (!aligned16(d_packed) || (n && !aligned16(d_out)) || !aligned16(d_ws)) return LCQ_ERR_ARG;
  if (ws_bytes < 8) return LCQ_ERR_CAPACITY;
  const uint64_t C = n_chunks(n);
  if (packed_bytes < packed_payload_offset(C)) return LCQ_ERR_STREAM;
  DcmpArgs a{};
  a.in = static_cast<const uint8_t *>(d_packed);
  a.in_bytes = packed_bytes;
  a.n = n;
  a.out = d_out;
  a.status = static_cast<unsigned long long *>(d_ws);
  a.epoch = g_cmp_epoch.fetch_add(1) + 1;
  a.dtype = (int)t;
  const uint64_t ntiles = std::max<uint64_t>(1, (C + kWaves - 1) / kWaves);
  if (t == LCQ_F32)
    hipLaunchKernelGGL(k_decompress<float>, dim3((unsigned)ntiles), dim3(kBlock), 0, stream, a);
  else
    hipLaunchKernelGGL(k_decompress<double>, dim3((unsigned)ntiles), dim3(kBlock), 0, stream, a);
  return check_launch_cmp();
}

}  // extern "C"
