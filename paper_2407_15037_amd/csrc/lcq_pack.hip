// lcq_pack.hip -- lossless packing stage for LCQ1 streams on gfx950.
//
// The paper hands the quantizer's output to further lossless stages of its
// framework without naming them; this stage is defined here (format and
// shared device helpers in lcq_packfmt.hpp).  The LCQ1 chunk table and
// outliers are carried over verbatim, so unpacking restores the LCQ1 stream
// byte for byte.
//
// Kernels (one wavefront per chunk, the chunk-per-wavefront mapping; full
// chunks take code paths without per-position masks):
//   k_pack_plan   widths, modes and record sizes; one atomic add per
//                 workgroup into its group's byte count
//   k_pack_scan   one workgroup per group: record offsets, header, padding,
//                 packed size
//   k_pack_write  records (each chunk's packed bits assembled in LDS by
//                 atomic ORs and stored 128 bits at a time), chunk table,
//                 outliers
//   k_unpack      per chunk: the whole record staged in LDS, record checks,
//                 bit extraction, inverse zigzag, wavefront prefix sum
//                 (delta mode), sentinels from the bitmap; header, chunk
//                 table, outliers
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>

#include "lcq.h"
#include "lcq_chunk.hpp"
#include "lcq_host.hpp"
#include "lcq_math.hpp"
#include "lcq_packfmt.hpp"
#include "lcq_tile.hpp"

using namespace lcq;

namespace {

constexpr int kCW = 4;                           // codes per lane per sub-block
constexpr int kCSub = (int)kChunk / (64 * kCW);  // 4 sub-blocks per chunk

// The LCQ1 header of an input stream describes exactly this call.
__device__ __forceinline__ bool lcq1_header_ok(const uint8_t *s, uint64_t bytes, int dtype,
                                               uint64_t n, uint64_t &k) {
  const uint64_t *hd = reinterpret_cast<const uint64_t *>(s);
  const uint64_t h0 = hd[0];
  k = hd[2];
  const uint64_t sz = dtype == LCQ_F64 ? 8 : 4;
  return (h0 & ~(0xFFull << 48)) == header_word0(dtype, 0) && ((h0 >> 48) & 0xFF) <= 2 &&
         hd[1] == n && k <= n && outlier_offset(n) + k * sz <= bytes;
}

// One chunk's codes as c' (sentinels -> 0) and flags, lane's 16 positions.
struct ChunkCodes {
  uint32_t cv[kCSub][kCW];
  unsigned flags;  // bit 4 j + e: outlier sentinel
};

// CACHED: ordinary loads (the plan pass: measured faster there than
// streaming loads); otherwise streaming loads.  FULL: the chunk has 1024
// codes (no position to mask).
template <bool CACHED, bool FULL>
__device__ __forceinline__ void load_chunk(const int32_t *codes, uint64_t n, uint64_t c, int lane,
                                           ChunkCodes &cc) {
  cc.flags = 0;
  const unsigned len = chunk_len(n, c);
#pragma unroll
  for (int j = 0; j < kCSub; j++) {
    const uint64_t i0 = chunk_value<kCW>(c, j, lane);
    const unsigned p = chunk_pos<kCW>(j, lane);
    int32_t v[kCW];
    if (CACHED && (FULL || p + kCW <= len)) {
      const nt_i4 q = *reinterpret_cast<const nt_i4 *>(codes + i0);
      v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else if (FULL) {
      const nt_i4 q = __builtin_nontemporal_load(reinterpret_cast<const nt_i4 *>(codes + i0));
      v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
      load_codes<kCW>(codes, i0, n, v);
    }
#pragma unroll
    for (int e = 0; e < kCW; e++) {
      const bool sent = v[e] == kSent && (FULL || p + e < len);
      cc.cv[j][e] = sent ? 0u : (uint32_t)v[e];
      if (sent) cc.flags |= 1u << (kCW * j + e);
    }
  }
}

// Width, mode, bitmap flag and record size of chunk c (same on every lane).
template <bool FULL>
__device__ __forceinline__ unsigned plan_chunk(const int32_t *codes, uint64_t n, uint64_t c,
                                               int lane, unsigned &meta) {
  ChunkCodes cc;
  load_chunk<true, FULL>(codes, n, c, lane, cc);
  const unsigned len = chunk_len(n, c);
  unsigned w, mode;
  chunk_width<FULL, kCW, kCSub>(cc.cv, len, lane, w, mode);
  const unsigned hb = __ballot(cc.flags != 0) ? 1u : 0u;
  meta = w | (mode << 8) | (hb << 16);
  return (unsigned)record_bytes(len, w, hb);
}

// Record of chunk c (width, mode and bitmap flag in meta) at rec, its packed
// bits assembled in the wavefront's LDS row.
template <bool FULL>
__device__ __forceinline__ void write_chunk_record(const int32_t *codes, uint64_t n, uint64_t c,
                                                   int lane, uint32_t meta, uint32_t *row,
                                                   uint8_t *rec) {
  const unsigned w = meta & 0xFF, mode = (meta >> 8) & 1, hb = (meta >> 16) & 1;
  const unsigned len = chunk_len(n, c);
  ChunkCodes cc;
  load_chunk<false, FULL>(codes, n, c, lane, cc);
  uint32_t z[kCSub][kCW];
  if (mode) lcq::chunk_z<true, kCW, kCSub, FULL>(cc.cv, len, lane, z);
  else lcq::chunk_z<false, kCW, kCSub, FULL>(cc.cv, len, lane, z);
  pack_bits<kCW, kCSub>(z, len, w, row, lane);
  write_record_head<kCW, kCSub>(rec, w, mode, hb, cc.flags, lane);
  copy_words(row, packed_words(len, w), reinterpret_cast<uint32_t *>(rec + 16 + (hb ? 128 : 0)),
             lane);
}

struct PackArgs {
  const uint8_t *in;      // LCQ1 stream
  uint64_t in_bytes;
  uint64_t n;
  uint8_t *out;           // packed stream
  uint64_t *out_bytes;
  uint32_t *sizes;        // record bytes per chunk
  uint32_t *meta;         // w | mode << 8 | hb << 16 per chunk
  unsigned long long *group;
  uint64_t tiles_per_group, chunks_per_group, ngroups;
  unsigned long long *status;
  uint64_t epoch;
  int dtype;
};

__global__ __launch_bounds__(64 * kStageWaves) void k_pack_plan(PackArgs a) {
  __shared__ unsigned s_tot[kStageWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t n = a.n, nch = n_chunks(n);
  uint64_t k;
  if (!lcq1_header_ok(a.in, a.in_bytes, a.dtype, n, k)) return;  // uniform over the grid
  const uint64_t c = (uint64_t)blockIdx.x * kStageWaves + wave;
  unsigned size = 0;
  if (c < nch) {
    const int32_t *codes = reinterpret_cast<const int32_t *>(a.in + 64);
    unsigned meta;
    if (chunk_len(n, c) == kChunk) size = plan_chunk<true>(codes, n, c, lane, meta);
    else size = plan_chunk<false>(codes, n, c, lane, meta);
    if (lane == 0) {
      a.sizes[c] = size;
      a.meta[c] = meta;
    }
  }
  if (lane == 0) s_tot[wave] = size;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
#pragma unroll
    for (int i = 0; i < kStageWaves; i++) t += s_tot[i];
    if (t) atomicAdd(a.group + blockIdx.x / a.tiles_per_group, t);
  }
}

__global__ __launch_bounds__(kBlock) void k_pack_scan(PackArgs a) {
  __shared__ unsigned long long s_red[kWaves];
  __shared__ unsigned long long s_wt[kWaves];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t n = a.n, nch = n_chunks(n);
  const uint64_t g = blockIdx.x;
  uint64_t k;
  const bool ok = lcq1_header_ok(a.in, a.in_bytes, a.dtype, n, k);
  if (g == 0 && tid == 0) report_status(a.status, a.epoch << 16, ok ? LCQ_OK : LCQ_ERR_STREAM);
  if (!ok) return;
  const uint64_t ot = packed_table_offset(nch), pl = packed_payload_offset(nch);
  uint64_t *offs = reinterpret_cast<uint64_t *>(a.out + ot);

  unsigned long long b = 0;
  for (uint64_t i = tid; i < g; i += kBlock) b += a.group[i];
  b = wave_sum(b);
  if (lane == 0) s_red[wave] = b;
  __syncthreads();
  uint64_t run = 0;
#pragma unroll
  for (int w = 0; w < kWaves; w++) run += s_red[w];

  const uint64_t c0 = g * a.chunks_per_group, c1 = min(c0 + a.chunks_per_group, nch);
  for (uint64_t cb = c0; cb < c1; cb += kBlock) {
    const uint64_t c = cb + tid;
    const unsigned long long sz = c < c1 ? a.sizes[c] : 0ull;
    unsigned long long incl = sz;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned long long t = __shfl_up(incl, o, 64);
      if (lane >= o) incl += t;
    }
    if (lane == 63) s_wt[wave] = incl;
    __syncthreads();
    uint64_t before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) {
      if (w < wave) before += s_wt[w];
      total += s_wt[w];
    }
    if (c < c1) offs[c] = run + before + (incl - sz);
    run += total;
    __syncthreads();  // s_wt is rewritten by the next batch
  }

  if (g == a.ngroups - 1 && tid == 0) {
    const uint64_t s = a.dtype == LCQ_F64 ? 8 : 4;
    const uint64_t oo = align16(pl + run);
    offs[nch] = run;
    const uint64_t *hin = reinterpret_cast<const uint64_t *>(a.in);
    uint64_t *hout = reinterpret_cast<uint64_t *>(a.out);
    hout[0] = (hin[0] & ~0xFFFFFFFFull) | kMagicPacked;
#pragma unroll
    for (int i = 1; i < 8; i++) hout[i] = hin[i];
    for (uint64_t x = 64 + 8 * nch; x < ot; x++) a.out[x] = 0;
    for (uint64_t x = ot + 8 * (nch + 1); x < pl; x++) a.out[x] = 0;
    for (uint64_t x = pl + run; x < oo; x++) a.out[x] = 0;
    *a.out_bytes = oo + k * s;
  }
}

// Records, chunk table and outliers.  Each chunk's packed bits are
// assembled in LDS (pack_bits) and leave in 128-bit stores.
__global__ __launch_bounds__(kBlock) void k_pack_write(PackArgs a) {
  __shared__ uint32_t s_w[kWaves][kChunk];  // each wavefront's packed words
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t n = a.n, nch = n_chunks(n);
  uint64_t k;
  if (!lcq1_header_ok(a.in, a.in_bytes, a.dtype, n, k)) return;  // uniform over the grid
  const uint64_t ot = packed_table_offset(nch), pl = packed_payload_offset(nch);
  const uint64_t c = (uint64_t)blockIdx.x * kWaves + wave;
  if (c < nch) {  // uniform over the wavefront
    const int32_t *codes = reinterpret_cast<const int32_t *>(a.in + 64);
    const uint32_t m = a.meta[c];
    uint8_t *rec = a.out + pl + reinterpret_cast<const uint64_t *>(a.out + ot)[c];
    if (chunk_len(n, c) == kChunk) write_chunk_record<true>(codes, n, c, lane, m, s_w[wave], rec);
    else write_chunk_record<false>(codes, n, c, lane, m, s_w[wave], rec);
    if (lane == 0) {
      const uint64_t *ct_in = reinterpret_cast<const uint64_t *>(a.in + chunk_table_offset(n));
      reinterpret_cast<uint64_t *>(a.out + 64)[c] = ct_in[c];
    }
  }
  // outliers, grid-stride over the raw words
  const uint64_t s = a.dtype == LCQ_F64 ? 8 : 4;
  const uint64_t payload = reinterpret_cast<const uint64_t *>(a.out + ot)[nch];
  const uint64_t oo = align16(pl + payload);
  const uint64_t words = k * s / 4;
  const uint32_t *src = reinterpret_cast<const uint32_t *>(a.in + outlier_offset(n));
  uint32_t *dst = reinterpret_cast<uint32_t *>(a.out + oo);
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < words;
       i += (uint64_t)gridDim.x * kBlock)
    dst[i] = src[i];
}

struct UnpackArgs {
  const uint8_t *in;      // packed stream
  uint64_t in_bytes;
  uint64_t n;
  uint8_t *out;           // LCQ1 stream
  uint64_t out_cap;
  uint64_t *out_bytes;
  unsigned long long *status;
  uint64_t epoch;
  int dtype;
};

__global__ __launch_bounds__(kBlock) void k_unpack(UnpackArgs a) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t n = a.n, nch = n_chunks(n);
  const uint64_t s = a.dtype == LCQ_F64 ? 8 : 4;
  const uint64_t ot = packed_table_offset(nch), pl = packed_payload_offset(nch);
  const unsigned long long tag = (unsigned long long)(a.epoch << 16);
  // header and table bounds (the host checked in_bytes >= pl)
  const uint64_t *hd = reinterpret_cast<const uint64_t *>(a.in);
  const uint64_t h0 = hd[0], k = hd[2];
  const uint64_t *offs = reinterpret_cast<const uint64_t *>(a.in + ot);
  const uint64_t payload = offs[nch];
  const bool bad = (h0 & ~(0xFFull << 48)) != packed_word0(a.dtype) || ((h0 >> 48) & 0xFF) > 2 || hd[1] != n ||
                   k > n || payload > a.in_bytes - pl ||
                   align16(pl + payload) + k * s > a.in_bytes ||
                   outlier_offset(n) + k * s > a.out_cap;
  if (blockIdx.x == 0 && threadIdx.x == 0)
    report_status(a.status, tag, bad ? LCQ_ERR_STREAM : LCQ_OK);
  if (bad) return;
  __shared__ uint32_t s_rec[kWaves][kMaxRecord / 4 + kRowPad];  // each wavefront's whole record
  const uint64_t c = (uint64_t)blockIdx.x * kWaves + wave;
  const bool act = c < nch;  // uniform over the wavefront
  bool ok = false;
  unsigned w = 0, mode = 0, hb = 0;
  unsigned len = 0;
  uint32_t *row = s_rec[wave];
  if (act) {
    // the record's extent from the offset table, then the whole record
    // (header, bitmap, bits) staged in LDS in one round trip
    const uint64_t off = offs[c], nxt = offs[c + 1];
    len = chunk_len(n, c);
    ok = record_extent_ok(off, nxt, payload);
    if (ok) {
      stage_words(a.in + pl + off, (unsigned)((nxt - off) / 4), row, lane);
      const uint32_t h = row[0];
      w = h & 0xFF;
      mode = (h >> 8) & 0xFF;
      hb = (h >> 16) & 0xFF;
      ok = w <= 32 && mode <= 1 && hb <= 1 && nxt - off == record_bytes(len, w, hb);
    }
    if (!ok && lane == 0) report_status(a.status, tag, LCQ_ERR_STREAM);
  }
  if (ok) {
    const unsigned ulen = len;
    const uint32_t *bits = row + (hb ? 36 : 4);
    const uint8_t *bm = hb ? reinterpret_cast<const uint8_t *>(row + 4) : nullptr;
    int32_t *codes = reinterpret_cast<int32_t *>(a.out + 64);
    uint32_t carry = 0;
#pragma unroll
    for (int j = 0; j < kCSub; j++) {  // each sub-block stored as soon as it is decoded
      int32_t out[kCW];
      record_codes_sub<kCW>(bits, bm, w, mode, lane, j, carry, out);
      const uint64_t i0 = chunk_value<kCW>(c, j, lane);
      const unsigned l0 = chunk_pos<kCW>(j, lane);  // position in the chunk
      if (l0 + kCW <= ulen) {
        store_codes<kCW, true>(codes, i0, n, out);
      } else {
#pragma unroll
        for (int e = 0; e < kCW; e++)
          if (l0 + e < ulen) codes[i0 + e] = out[e];
      }
    }
    if (lane == 0) {
      reinterpret_cast<uint64_t *>(a.out + chunk_table_offset(n))[c] =
          reinterpret_cast<const uint64_t *>(a.in + 64)[c];
    }
  }
  // header, padding, outliers
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    uint64_t *hout = reinterpret_cast<uint64_t *>(a.out);
    hout[0] = (h0 & ~0xFFFFFFFFull) | kMagic;
#pragma unroll
    for (int i = 1; i < 8; i++) hout[i] = hd[i];
    const uint64_t ct = chunk_table_offset(n), ce = ct + 8 * nch, oo = outlier_offset(n);
    for (uint64_t x = 64 + 4 * n; x < ct; x++) a.out[x] = 0;
    for (uint64_t x = ce; x < oo; x++) a.out[x] = 0;
    *a.out_bytes = oo + k * s;
  }
  const uint64_t words = k * s / 4;
  const uint32_t *src = reinterpret_cast<const uint32_t *>(a.in + align16(pl + payload));
  uint32_t *dst = reinterpret_cast<uint32_t *>(a.out + outlier_offset(n));
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < words;
       i += (uint64_t)gridDim.x * kBlock)
    dst[i] = src[i];
}

__global__ void k_clear_pk(uint64_t *p, uint64_t count) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// Workspace of lcq_pack: status word, group sums, record sizes, metadata.
uint64_t pk_sizes_off() { return align16(256 + 8 * kMaxGroups); }
uint64_t pk_meta_off(uint64_t C) { return align16(pk_sizes_off() + 4 * C); }

lcq_status check_launch_pk() { return hipGetLastError() == hipSuccess ? LCQ_OK : LCQ_ERR_HIP; }

// Call epochs tag the status word (as for the decoders); seeded from the
// clock so a workspace left over from another process cannot match.
std::atomic<uint64_t> g_pk_epoch{
    ((uint64_t)std::chrono::steady_clock::now().time_since_epoch().count() ^ 0x5A5A5A5A5ull) &
    0xFFFFFFFFFFFull};

}  // namespace

extern "C" {

uint64_t lcq_pack_max_bytes(lcq_dtype t, uint64_t n) {
  if ((t != LCQ_F32 && t != LCQ_F64) || n > LCQ_MAX_N) return 0;
  const uint64_t s = t == LCQ_F64 ? 8 : 4, C = n_chunks(n);
  return align16(packed_payload_offset(C) + C * record_bytes(kChunk, 32, 1)) + s * n;
}

uint64_t lcq_pack_workspace_bytes(lcq_dtype t, uint64_t n) {
  if ((t != LCQ_F32 && t != LCQ_F64) || n > LCQ_MAX_N) return 0;
  return pk_meta_off(n_chunks(n)) + 4 * n_chunks(n);
}

lcq_status lcq_pack(lcq_dtype t, const void *d_stream, uint64_t stream_bytes, uint64_t n,
                    void *d_packed, uint64_t packed_cap, uint64_t *d_packed_bytes, void *d_ws,
                    uint64_t ws_bytes, hipStream_t stream) {
  if (t != LCQ_F32 && t != LCQ_F64) return LCQ_ERR_ARG;
  if (n > LCQ_MAX_N) return LCQ_ERR_ARG;
  if (!d_stream || !d_packed || !d_packed_bytes || !d_ws) return LCQ_ERR_ARG;
  if (!aligned16(d_stream) || !aligned16(d_packed) || !aligned16(d_ws) ||
      ((uintptr_t)d_packed_bytes & 7u))
    return LCQ_ERR_ARG;
  if (stream_bytes < outlier_offset(n)) return LCQ_ERR_STREAM;
  if (packed_cap < lcq_pack_max_bytes(t, n)) return LCQ_ERR_CAPACITY;
  if (ws_bytes < lcq_pack_workspace_bytes(t, n)) return LCQ_ERR_CAPACITY;
  const uint64_t C = n_chunks(n);
  const uint64_t ntiles = (C + kWaves - 1) / kWaves;
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  PackArgs a{};
  a.in = static_cast<const uint8_t *>(d_stream);
  a.in_bytes = stream_bytes;
  a.n = n;
  a.out = static_cast<uint8_t *>(d_packed);
  a.out_bytes = d_packed_bytes;
  a.sizes = reinterpret_cast<uint32_t *>(ws + pk_sizes_off());
  a.meta = reinterpret_cast<uint32_t *>(ws + pk_meta_off(C));
  a.group = reinterpret_cast<unsigned long long *>(ws + 256);
  // the plan pass in workgroups of kStageWaves chunks (one group add each)
  const uint64_t ptiles = (C + kStageWaves - 1) / kStageWaves;
  a.tiles_per_group = tiles_per_group(ptiles, kStageWaves);
  a.chunks_per_group = a.tiles_per_group * kStageWaves;
  a.ngroups = std::max<uint64_t>(1, (ptiles + a.tiles_per_group - 1) / a.tiles_per_group);
  a.status = reinterpret_cast<unsigned long long *>(ws);
  a.epoch = g_pk_epoch.fetch_add(1) + 1;
  a.dtype = (int)t;
  const unsigned cg = (unsigned)std::min<uint64_t>((a.ngroups + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_clear_pk, dim3(cg), dim3(kBlock), 0, stream,
                     reinterpret_cast<uint64_t *>(a.group), a.ngroups);
  if (ntiles)
    hipLaunchKernelGGL(k_pack_plan, dim3((unsigned)ptiles), dim3(64 * kStageWaves), 0, stream, a);
  hipLaunchKernelGGL(k_pack_scan, dim3((unsigned)a.ngroups), dim3(kBlock), 0, stream, a);
  if (ntiles) hipLaunchKernelGGL(k_pack_write, dim3((unsigned)ntiles), dim3(kBlock), 0, stream, a);
  return check_launch_pk();
}

lcq_status lcq_unpack(lcq_dtype t, const void *d_packed, uint64_t packed_bytes, uint64_t n,
                      void *d_stream, uint64_t stream_cap, uint64_t *d_stream_bytes, void *d_ws,
                      uint64_t ws_bytes, hipStream_t stream) {
  if (t != LCQ_F32 && t != LCQ_F64) return LCQ_ERR_ARG;
  if (n > LCQ_MAX_N) return LCQ_ERR_ARG;
  if (!d_packed || !d_stream || !d_stream_bytes || !d_ws) return LCQ_ERR_ARG;
  if (!aligned16(d_packed) || !aligned16(d_stream) || !aligned16(d_ws) ||
      ((uintptr_t)d_stream_bytes & 7u))
    return LCQ_ERR_ARG;
  if (ws_bytes < 8) return LCQ_ERR_CAPACITY;
  const uint64_t C = n_chunks(n);
  if (packed_bytes < packed_payload_offset(C)) return LCQ_ERR_STREAM;
  if (stream_cap < outlier_offset(n)) return LCQ_ERR_CAPACITY;
  UnpackArgs a{};
  a.in = static_cast<const uint8_t *>(d_packed);
  a.in_bytes = packed_bytes;
  a.n = n;
  a.out = static_cast<uint8_t *>(d_stream);
  a.out_cap = stream_cap;
  a.out_bytes = d_stream_bytes;
  a.status = static_cast<unsigned long long *>(d_ws);
  a.epoch = g_pk_epoch.fetch_add(1) + 1;
  a.dtype = (int)t;
  const uint64_t ntiles = std::max<uint64_t>(1, (C + kWaves - 1) / kWaves);
  hipLaunchKernelGGL(k_unpack, dim3((unsigned)ntiles), dim3(kBlock), 0, stream, a);
  return check_launch_pk();
}

}  // extern "C"
