// lcq_batch.hip -- batched quantize / dequantize of many fields of uneven
// size, mixed dtype, quantizer and bound in one graph launch.
//
// Quantize: one kernel over a device-side table of work items, one
// workgroup per item in table order.  The table holds, in order: the NOA
// range slices of every NOA field (phase A), then every quantize tile of
// every field (phase B), each field's tiles in increasing order (largest
// fields first).  A phase-A item reduces its slice's finite min / max; the
// field's last slice to finish derives the field's parameters on the device
// and raises the field's ready flag.  A phase-B item of a NOA field waits for
// that flag (bounded, with a fallback that derives the parameters from the
// input), then runs the plain path's per-tile code:
//   chunk variant  the streaming pass of the two-pass quantize (codes, chunk
//                  counts, staged outliers); a second kernel then runs one
//                  workgroup per (field, chunk group) to write chunk tables,
//                  outliers and headers;
//   tile variants  quant_tile with its decoupled look-back inside each field
//                  (bounded wait, fallback counting from the input).
//
// Dequantize: one kernel with a workgroup per dequantize tile of every field
// (independent tiles, one wavefront per chunk), mapped through an item table.
//
// Both are captured once into HIP graphs at plan creation; running the batch
// is one hipGraphLaunch.  Every field's stream and decode are byte-identical
// to what the plain entry points produce for that field alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lcq.h"
#include "lcq_host.hpp"
#include "lcq_math.hpp"
#include "lcq_tile.hpp"
#include "lcq_chunk.hpp"

#pragma clang fp contract(off)

using namespace lcq;

namespace {

// Batch quantize variants: variant 0 is the two-pass chunk form (one chunk
// per wavefront at a time, cpw chunks per wavefront and workgroup item, cpw
// chosen per dtype); 1-3 are look-back tile shapes (slots, rounds) per
// dtype.  The tuner picks the variant and the chunk form's cpw per dtype.
struct BatchShape {
  Shape f32, f64;
  bool chunk;
};
constexpr int kNumBatchVariants = 4;
constexpr BatchShape kBatchVariants[kNumBatchVariants] = {
    {{0, 0}, {0, 0}, true},     // chunk-per-wavefront, two passes
    {{4, 4}, {4, 8}, false},    // 16384-value tiles
    {{4, 2}, {4, 4}, false},    // 8192
    {{4, 1}, {4, 2}, false},    // 4096
};
constexpr uint64_t kChunkTile = kChunk * kWaves;  // values per chunk-form workgroup and cpw
constexpr unsigned kMaxCpw = 16;                   // chunks per wavefront per item, at most

// A plan's tuning: variant, and the chunk form's chunks per wavefront per
// dtype.
struct Tune {
  int bv;
  unsigned cpw32, cpw64;
  unsigned cpw(int dtype) const { return dtype == LCQ_F64 ? cpw64 : cpw32; }
};
constexpr uint64_t kSlice = 1ull << 18;  // values per NOA range item
constexpr uint64_t kDeqTile = kChunk * kWaves;  // codes per dequantize workgroup

// Device descriptor of one field.
struct BField {
  const void *in;
  uint64_t n;
  uint8_t *stream;
  uint64_t stream_cap;
  uint64_t *stream_bytes;
  void *out;
  uint64_t state_off;    // first look-back word of this field (tile variants)
  uint64_t ntiles;       // quantize tiles
  uint64_t counts_off, stage_off, group_off;  // chunk variant: workspace offsets
  uint64_t tiles_per_group, chunks_per_group, ngroups;
  uint64_t cpw;          // chunk variant: chunks per wavefront per item
  uint64_t step, inv, bound, low;  // host-derived parameters (ABS / REL)
  uint64_t hdr[8];
  uint64_t eb_down;      // NOA: RD_T(eb)
  uint64_t partial_off;  // NOA: first (min, max) pair of this field
  uint32_t nslices;      // NOA: range items of this field
  uint32_t noa_idx;      // NOA: index of the field's DevParams / counters
  int32_t dtype, q;
};

// Workspace layout of a plan (byte offsets).
struct Layout {
  uint64_t head, fields, items_q, items_d, items_f, params, done, state, groups, counts, stage,
      partials, dstatus, args, total;
  uint64_t clear_begin, clear_words;  // u64 words zeroed before each quantize
};

struct BatchQArgs {
  const BField *fields;
  const uint64_t *items;  // (field << 32) | (local index); phase A first
  uint64_t n_a, n_items;
  const uint64_t *items_f;  // chunk variant: (field << 32) | group
  uint8_t *ws;              // workspace base (chunk variant areas)
  unsigned *head;
  DevParams *params;
  unsigned *done;
  uint64_t *state;
  uint8_t *partials;
  unsigned spin_limit;   // look-back polls before a predecessor is counted directly
  unsigned ready_polls;  // NOA parameter-flag polls before deriving them directly
};

// Values the caller knows are the same on every lane, moved to scalar
// registers (so the loads they address become scalar loads).
template <typename P> __device__ __forceinline__ P *uni_ptr(P *p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint64_t lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const uint64_t hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return reinterpret_cast<P *>(lo | (hi << 32));
}
// Copy of a descriptor every lane reads at the same address, word by word
// into scalar registers.  (The kernel writes global memory, so the compiler
// cannot prove these loads unclobbered and would otherwise keep every field
// of the descriptor, and everything computed from it, in vector registers.)
template <typename S> __device__ __forceinline__ S uload(const S *p) {
  static_assert(sizeof(S) % 4 == 0, "descriptor of whole words");
  S out;
  unsigned w[sizeof(S) / 4];
  __builtin_memcpy(w, p, sizeof(S));
#pragma unroll
  for (unsigned k = 0; k < sizeof(S) / 4; k++) w[k] = __builtin_amdgcn_readfirstlane(w[k]);
  __builtin_memcpy(&out, w, sizeof(S));
  return out;
}

template <typename T>
__device__ __forceinline__ void range_item(const BatchQArgs &a, const BField &f, uint64_t slice) {
  const uint64_t b = slice * kSlice;
  const uint64_t e = min(b + kSlice, f.n);
  T lo, hi;
  block_minmax<T>(static_cast<const T *>(f.in), b, e, lo, hi);
  __shared__ int s_last;
  T *parts = reinterpret_cast<T *>(a.partials + f.partial_off);
  if (threadIdx.x == 0) {
    parts[2 * slice] = lo;
    parts[2 * slice + 1] = hi;
    // release our pair; the field's last slice (acquire) sees every pair
    const unsigned prev = __hip_atomic_fetch_add(a.done + f.noa_idx, 1u, __ATOMIC_ACQ_REL,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    s_last = prev == f.nslices - 1;
  }
  __syncthreads();
  if (!__builtin_amdgcn_readfirstlane(s_last)) return;
  // the field's range from every slice, then its parameters
  T l2 = (T)INFINITY, h2 = (T)-INFINITY;
  for (uint32_t i = threadIdx.x; i < f.nslices; i += kBlock) {
    l2 = fmin(l2, __hip_atomic_load(parts + 2 * i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    h2 = fmax(h2, __hip_atomic_load(parts + 2 * i + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    l2 = fmin(l2, __shfl_xor(l2, o, 64));
    h2 = fmax(h2, __shfl_xor(h2, o, 64));
  }
  __shared__ T s_lo[kWaves], s_hi[kWaves];
  if ((threadIdx.x & 63) == 0) {
    s_lo[threadIdx.x >> 6] = l2;
    s_hi[threadIdx.x >> 6] = h2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kWaves; w++) {
      l2 = fmin(l2, s_lo[w]);
      h2 = fmax(h2, s_hi[w]);
    }
    DevParams d = noa_params<T>(l2, h2, from_bits((typename FT<T>::U)f.eb_down));
    DevParams *dst = a.params + f.noa_idx;
    dst->step = d.step;
    dst->inv = d.inv;
    dst->bound = d.bound;
    dst->lo = d.lo;
    dst->hi = d.hi;
    dst->lossless_all = d.lossless_all;
    __hip_atomic_store(&dst->ready, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Parameters of a NOA field for one of its phase-B workgroups.  Every range
// item of the field left the queue before this one and never waits, so the
// ready flag comes; the wait is bounded all the same: past the bound this
// workgroup derives the same parameters from the whole field itself (min /
// max do not depend on order).
template <typename T>
__device__ DevParams noa_field_params(const BatchQArgs &a, const BField &bf) {
  DevParams *dp = a.params + bf.noa_idx;
  __shared__ int s_ready;
  __shared__ DevParams s_dp;
  if (threadIdx.x == 0) {
    int r = __hip_atomic_load(&dp->ready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    for (unsigned polls = 0; r == 0 && polls < a.ready_polls; polls++) {
      __builtin_amdgcn_s_sleep(2);
      r = __hip_atomic_load(&dp->ready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    }
    s_ready = r;
  }
  __syncthreads();
  DevParams d;
  if (__builtin_amdgcn_readfirstlane(s_ready)) {
    d.step = __hip_atomic_load(&dp->step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    d.inv = __hip_atomic_load(&dp->inv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    d.bound = __hip_atomic_load(&dp->bound, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    d.lo = __hip_atomic_load(&dp->lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    d.hi = __hip_atomic_load(&dp->hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    d.lossless_all =
        __hip_atomic_load(&dp->lossless_all, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    T lo, hi;
    block_minmax<T>(static_cast<const T *>(bf.in), 0, bf.n, lo, hi);
    if (threadIdx.x == 0) s_dp = noa_params<T>(lo, hi, from_bits((typename FT<T>::U)bf.eb_down));
    __syncthreads();
    d = s_dp;
  }
  return d;
}

template <typename T, int Q>
__device__ __forceinline__ FieldParams<T> field_params(const BatchQArgs &a, const BField &bf,
                                                       DevParams *noa_out) {
  using U = typename FT<T>::U;
  if constexpr (Q == kNOA) {
    const DevParams d = noa_field_params<T>(a, bf);
    if (noa_out) *noa_out = d;
    return params_from<T>(d);
  }
  FieldParams<T> p;
  p.step = from_bits((U)bf.step);
  p.inv = from_bits((U)bf.inv);
  p.bound = from_bits((U)bf.bound);
  p.low = from_bits((U)bf.low);
  p.lossless_all = 0;
  return p;
}

template <typename T, int Q, int SL, int RD>
__device__ __forceinline__ void tile_item(const BatchQArgs &a, const BField &bf, uint64_t tile) {
  QField<T> f;
  f.in = static_cast<const T *>(bf.in);
  f.n = bf.n;
  f.stream = bf.stream;
  f.stream_bytes = bf.stream_bytes;
  f.state = a.state + bf.state_off;
  f.ntiles = bf.ntiles;
#pragma unroll
  for (int i = 0; i < 8; i++) f.hdr[i] = bf.hdr[i];
  DevParams d;
  f.p = field_params<T, Q>(a, bf, &d);
  if constexpr (Q == kNOA) {
    f.hdr[4] = d.step;
    f.hdr[5] = d.bound;
    f.hdr[6] = d.lo;
    f.hdr[7] = d.hi;
  }
  quant_tile<T, Q, SL, RD>(f, tile, a.spin_limit);
}

// Chunk variant, pass 1: the workgroup's 4 chunks of one field.
template <typename T, int Q>
__device__ __forceinline__ void chunk_item(const BatchQArgs &a, const BField &bf, uint64_t tile) {
  using U = typename FT<T>::U;
  StageField<T> f;
  f.in = static_cast<const T *>(bf.in);
  f.n = bf.n;
  f.codes = reinterpret_cast<int32_t *>(bf.stream + 64);
  f.counts = reinterpret_cast<uint32_t *>(a.ws + bf.counts_off);
  f.stage = reinterpret_cast<U *>(a.ws + bf.stage_off);
  f.group = reinterpret_cast<unsigned long long *>(a.ws + bf.group_off);
  f.tiles_per_group = bf.tiles_per_group;
  f.p = field_params<T, Q>(a, bf, nullptr);
  quant_chunks_n<T, Q>(f, tile, (unsigned)bf.cpw);
}

// One workgroup per work item, in queue order: the hardware dispatcher hands
// the item table to the workgroups front to back (range items first, then
// each field's tiles in increasing order).  No atomic head is needed; every
// wait inside an item (a NOA field's parameters, a predecessor tile's
// outlier count) is bounded with a fallback that computes the awaited value
// from the input, so no dispatch order can stall the grid.
template <int SL32, int RD32, int SL64, int RD64, bool CHUNK>
__global__ __launch_bounds__(kBlock) void k_batch_quantize(const BatchQArgs *ap) {
  const BatchQArgs a = uload(ap);
  const unsigned cur = blockIdx.x;
  const uint64_t it = uload(a.items + cur);
  const BField f = uload(a.fields + (it >> 32));
  const uint64_t local = it & 0xFFFFFFFFull;
  if (cur < a.n_a) {
    if (f.dtype == LCQ_F32) range_item<float>(a, f, local);
    else range_item<double>(a, f, local);
    return;
  }
  if constexpr (CHUNK) {
    if (f.dtype == LCQ_F32) {
      if (f.q == kABS) chunk_item<float, kABS>(a, f, local);
      else if (f.q == kREL) chunk_item<float, kREL>(a, f, local);
      else chunk_item<float, kNOA>(a, f, local);
    } else {
      if (f.q == kABS) chunk_item<double, kABS>(a, f, local);
      else if (f.q == kREL) chunk_item<double, kREL>(a, f, local);
      else chunk_item<double, kNOA>(a, f, local);
    }
  } else {
    if (f.dtype == LCQ_F32) {
      if (f.q == kABS) tile_item<float, kABS, SL32, RD32>(a, f, local);
      else if (f.q == kREL) tile_item<float, kREL, SL32, RD32>(a, f, local);
      else tile_item<float, kNOA, SL32, RD32>(a, f, local);
    } else {
      if (f.q == kABS) tile_item<double, kABS, SL64, RD64>(a, f, local);
      else if (f.q == kREL) tile_item<double, kREL, SL64, RD64>(a, f, local);
      else tile_item<double, kNOA, SL64, RD64>(a, f, local);
    }
  }
}

// Chunk variant, pass 2: one workgroup per (field, chunk group).  Every NOA
// field's range items finished in the previous kernel, so its parameters
// are published.
template <typename T>
__device__ __forceinline__ void finish_item(const BatchQArgs &a, const BField &bf, uint64_t g) {
  using U = typename FT<T>::U;
  FinishField<T> f;
  f.in = static_cast<const T *>(bf.in);
  f.n = bf.n;
  f.stream = bf.stream;
  f.stream_bytes = bf.stream_bytes;
  f.counts = reinterpret_cast<const uint32_t *>(a.ws + bf.counts_off);
  f.stage = reinterpret_cast<const U *>(a.ws + bf.stage_off);
  f.group = reinterpret_cast<const unsigned long long *>(a.ws + bf.group_off);
  f.chunks_per_group = bf.chunks_per_group;
  f.ngroups = bf.ngroups;
  f.noa = bf.q == kNOA ? a.params + bf.noa_idx : nullptr;
#pragma unroll
  for (int i = 0; i < 8; i++) f.hdr[i] = bf.hdr[i];
  quant_finish<T>(f, g);
}

__global__ __launch_bounds__(kBlock) void k_batch_finish(const BatchQArgs *ap) {
  const BatchQArgs a = uload(ap);
  const uint64_t it = uload(a.items_f + blockIdx.x);
  const BField f = uload(a.fields + (it >> 32));
  const uint64_t g = it & 0xFFFFFFFFull;
  if (f.dtype == LCQ_F32) finish_item<float>(a, f, g);
  else finish_item<double>(a, f, g);
}

struct BatchDArgs {
  const BField *fields;
  const uint64_t *items;
  uint64_t n_items;
  unsigned long long *status;  // one word per field
};

template <typename T>
__device__ void deq_item(const BatchDArgs &a, const BField &bf, uint32_t fi, uint64_t tile) {
  using U = typename FT<T>::U;
  const uint64_t n = bf.n;
  const uint64_t *hd = reinterpret_cast<const uint64_t *>(bf.stream);
  const uint64_t h0 = hd[0];
  const uint64_t k = hd[2];
  const int q = (int)((h0 >> 48) & 0xFF);
  const bool bad = (h0 & ~(0xFFull << 48)) != header_word0(bf.dtype, 0) || q > 2 ||
                   hd[1] != n || k > n || outlier_offset(n) + k * sizeof(T) > bf.stream_cap;
  if (bad) {
    if (threadIdx.x == 0) atomicMax(a.status + fi, (unsigned long long)LCQ_ERR_STREAM);
    return;
  }
  DField<T> f;
  f.stream = bf.stream;
  f.n = n;
  f.k = k;
  f.step = from_bits((U)hd[4]);
  f.rel = (q == kREL);
  f.out = static_cast<T *>(bf.out);
  f.status = a.status + fi;
  f.tag = 0;
  dequant_chunks<T, 1, 1>(f, tile);
}

__global__ __launch_bounds__(kBlock) void k_batch_dequantize(BatchDArgs a) {
  const uint64_t it = a.items[blockIdx.x];
  const uint32_t fi = (uint32_t)(it >> 32);
  const BField &f = a.fields[fi];
  const uint64_t tile = it & 0xFFFFFFFFull;
  if (f.dtype == LCQ_F32) deq_item<float>(a, f, fi, tile);
  else deq_item<double>(a, f, fi, tile);
}

__global__ void k_batch_clear(uint64_t *p, uint64_t count) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

uint64_t up256(uint64_t v) { return (v + 255) & ~255ull; }

// Staged raw bits of one chunk (pass 1 of the chunk form).
uint64_t stage_bytes_per_chunk(int dtype) {
  return dtype == LCQ_F64 ? 8ull * stage_cap<double>() : 4ull * stage_cap<float>();
}

struct Counts {
  uint64_t n_a = 0, n_b = 0, n_d = 0, n_f = 0, states = 0, partial_bytes = 0;
  uint64_t group_words = 0, count_bytes = 0, stage_bytes = 0;
  uint32_t n_noa = 0;
};

uint64_t qtile_len(int dtype, const Tune &tn) {
  const int bv = tn.bv;
  if (kBatchVariants[bv].chunk) return kChunkTile * tn.cpw(dtype);
  const Shape s = dtype == LCQ_F64 ? kBatchVariants[bv].f64 : kBatchVariants[bv].f32;
  return (uint64_t)kBlock * (dtype == LCQ_F64 ? 2 : 4) * s.slots * s.rounds;
}

// Quantize workgroups of a field: chunk variant n = 0 has none (its header
// comes from pass 2); tile variants give n = 0 one header-only tile.
uint64_t field_tiles(const lcq_field &x, const Tune &tn) {
  const int bv = tn.bv;
  const uint64_t tl = qtile_len(x.t, tn);
  if (kBatchVariants[bv].chunk) return (x.n + tl - 1) / tl;
  return x.n ? (x.n + tl - 1) / tl : 1;
}

// Chunk variant: pass-2 groups of a field (at most kMaxGroups, at least 1).
void field_groups(uint64_t ntiles, unsigned cpw, uint64_t &tiles_per_group, uint64_t &ngroups) {
  tiles_per_group = lcq::tiles_per_group(ntiles, (kChunkTile / kChunk) * cpw);
  ngroups = std::max<uint64_t>(1, (ntiles + tiles_per_group - 1) / tiles_per_group);
}

Counts count(const lcq_field *f, uint32_t nf, const Tune &tn) {
  const int bv = tn.bv;
  Counts c;
  const bool chunk = kBatchVariants[bv].chunk;
  for (uint32_t i = 0; i < nf; i++) {
    const uint64_t nt = field_tiles(f[i], tn);
    c.n_b += nt;
    if (chunk) {
      uint64_t tpg, ng;
      field_groups(nt, tn.cpw(f[i].t), tpg, ng);
      c.n_f += ng;
      c.group_words += ng;
      c.count_bytes += up256(4 * n_chunks(f[i].n));
      c.stage_bytes += up256(stage_bytes_per_chunk(f[i].t) * n_chunks(f[i].n));
    } else {
      c.states += nt;
    }
    c.n_d += (f[i].n + kDeqTile - 1) / kDeqTile;
    if (f[i].q == LCQ_NOA) {
      const uint64_t ns = std::max<uint64_t>(1, (f[i].n + kSlice - 1) / kSlice);
      c.n_a += ns;
      c.partial_bytes += up256(ns * 2 * (f[i].t == LCQ_F64 ? 8 : 4));
      c.n_noa++;
    }
  }
  return c;
}

Layout layout_for(const Counts &c, uint32_t nf) {
  Layout L{};
  uint64_t o = 0;
  L.head = o;          o += 256;
  L.params = o;        o += up256(sizeof(DevParams) * std::max<uint32_t>(c.n_noa, 1));
  L.done = o;          o += up256(4ull * std::max<uint32_t>(c.n_noa, 1));
  L.dstatus = o;       o += up256(8ull * std::max<uint32_t>(nf, 1));
  L.state = o;         o += up256(8 * std::max<uint64_t>(c.states, 1));
  L.groups = o;        o += up256(8 * std::max<uint64_t>(c.group_words, 1));
  L.clear_begin = 0;
  L.clear_words = o / 8;  // head, params (ready flags), done, status, state, group sums
  L.args = o;          o += up256(sizeof(BatchQArgs));
  L.fields = o;        o += up256(sizeof(BField) * std::max<uint32_t>(nf, 1));
  L.items_q = o;       o += up256(8 * std::max<uint64_t>(c.n_a + c.n_b, 1));
  L.items_d = o;       o += up256(8 * std::max<uint64_t>(c.n_d, 1));
  L.items_f = o;       o += up256(8 * std::max<uint64_t>(c.n_f, 1));
  L.counts = o;        o += std::max<uint64_t>(c.count_bytes, 256);
  L.stage = o;         o += std::max<uint64_t>(c.stage_bytes, 256);
  L.partials = o;      o += std::max<uint64_t>(c.partial_bytes, 256);
  L.total = o;
  return L;
}

// Value of integer key `key` in a tuning string: the first run of digits
// after the key (so "batch=2", "f32=4" and {"batch": 2, "f32": 4} read
// alike); `dflt` when the key is absent, -1 when no digits follow it.
long tune_value(const char *tune, const char *key, long dflt) {
  const char *p = tune ? std::strstr(tune, key) : nullptr;
  if (!p) return dflt;
  p += std::strlen(key);
  while (*p && (*p == '"' || *p == ':' || *p == '=' || *p == ' ')) p++;
  if (*p < '0' || *p > '9') return -1;
  long v = 0;
  while (*p >= '0' && *p <= '9' && v < 1000000) v = v * 10 + (*p++ - '0');
  return v;
}

// Tuning from the string ("batch", and "f32" / "f64" chunks per wavefront
// per item for the chunk form, each 1, 2, 4, 8 or 16; defaults 0, 1, 1).
// bv < 0 marks an invalid string.
Tune parse_tune(const char *tune) {
  Tune t{0, 1, 1};
  const long v = tune_value(tune, "batch", 0);
  const long c32 = tune_value(tune, "f32", 1), c64 = tune_value(tune, "f64", 1);
  const auto ok_cpw = [](long c) { return c >= 1 && c <= (long)kMaxCpw && (c & (c - 1)) == 0; };
  if (v < 0 || v >= kNumBatchVariants || !ok_cpw(c32) || !ok_cpw(c64)) {
    t.bv = -1;
    return t;
  }
  t.bv = (int)v;
  t.cpw32 = (unsigned)c32;
  t.cpw64 = (unsigned)c64;
  return t;
}

lcq_status launch_batch_quantize(int bv, const BatchQArgs *a, unsigned grid, hipStream_t s) {
  const dim3 g(grid), b(kBlock);
  switch (bv) {
    case 1: hipLaunchKernelGGL((k_batch_quantize<4, 4, 4, 8, false>), g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_batch_quantize<4, 2, 4, 4, false>), g, b, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_batch_quantize<4, 1, 4, 2, false>), g, b, 0, s, a); break;
    default: hipLaunchKernelGGL((k_batch_quantize<0, 0, 0, 0, true>), g, b, 0, s, a); break;
  }
  return hipGetLastError() == hipSuccess ? LCQ_OK : LCQ_ERR_HIP;
}

}  // namespace

struct lcq_batch_plan {
  int variant;
  Tune tune;
  uint32_t nf;
  bool can_decode;  // every field with values has a decode buffer
  uint8_t *ws;
  Layout L;
  Counts c;
  unsigned grid;
  hipGraph_t gq = nullptr, gd = nullptr;
  hipGraphExec_t eq = nullptr, ed = nullptr;
};

extern "C" {

int32_t lcq_batch_variants(void) { return kNumBatchVariants; }

uint64_t lcq_batch_workspace_bytes(const lcq_field *f, uint32_t nf, const char *tune) {
  const Tune tn = parse_tune(tune);
  if (tn.bv < 0 || (nf && !f)) return 0;
  return layout_for(count(f, nf, tn), nf).total;
}

lcq_status lcq_batch_plan_create(const lcq_field *f, uint32_t nf, const char *tune, void *d_ws,
                                 uint64_t ws_bytes, hipStream_t stream, lcq_batch_plan **out) {
  if (!out || (nf && !f) || !d_ws || !aligned16(d_ws)) return LCQ_ERR_ARG;
  *out = nullptr;
  const Tune tn = parse_tune(tune);
  const int bv = tn.bv;
  if (bv < 0) return LCQ_ERR_ARG;
  for (uint32_t i = 0; i < nf; i++) {
    const lcq_field &x = f[i];
    if (x.q != LCQ_ABS && x.q != LCQ_REL && x.q != LCQ_NOA) return LCQ_ERR_ARG;
    if (x.t != LCQ_F32 && x.t != LCQ_F64) return LCQ_ERR_ARG;
    if (!(x.eb > 0.0) || !std::isfinite(x.eb) || (x.q == LCQ_REL && !(x.eb < 1.0))) return LCQ_ERR_ARG;
    if (x.n > LCQ_MAX_N || x.n >= (1ull << 32) * 1024) return LCQ_ERR_ARG;
    if (x.n && (!x.d_in || !aligned16(x.d_in))) return LCQ_ERR_ARG;
    if (!x.d_stream || !aligned16(x.d_stream) || !x.d_stream_bytes ||
        ((uintptr_t)x.d_stream_bytes & 7u))
      return LCQ_ERR_ARG;
    if (x.d_out && !aligned16(x.d_out)) return LCQ_ERR_ARG;
    if (x.stream_cap < lcq_max_stream_bytes(x.t, x.n)) return LCQ_ERR_CAPACITY;
  }
  const Counts c = count(f, nf, tn);
  const Layout L = layout_for(c, nf);
  if (ws_bytes < L.total) return LCQ_ERR_CAPACITY;
  if (c.n_a + c.n_b >= (1ull << 32) || c.n_f >= (1ull << 32) || c.n_d >= (1ull << 32))
    return LCQ_ERR_ARG;

  // descriptors and item tables
  std::vector<BField> bf(nf);
  std::vector<uint64_t> items_a, items_b, items_d, items_f;
  items_a.reserve(c.n_a);
  items_b.reserve(c.n_b);
  items_d.reserve(c.n_d);
  items_f.reserve(c.n_f);
  uint64_t state_off = 0, part_off = 0, group_off = 0, count_off = 0, stage_off = 0;
  uint32_t noa_idx = 0;
  for (uint32_t i = 0; i < nf; i++) {
    const lcq_field &x = f[i];
    BField &d = bf[i];
    std::memset(&d, 0, sizeof d);
    d.in = x.d_in;
    d.n = x.n;
    d.stream = static_cast<uint8_t *>(x.d_stream);
    d.stream_cap = x.stream_cap;
    d.stream_bytes = x.d_stream_bytes;
    d.out = x.d_out;
    d.dtype = x.t;
    d.q = x.q;
    const HostParams hp = x.t == LCQ_F64 ? host_params<double>(x.q, x.eb) : host_params<float>(x.q, x.eb);
    d.step = hp.step;
    d.inv = hp.inv;
    d.bound = hp.bound;
    d.low = hp.low;
    d.eb_down = hp.eb_down;
    d.hdr[0] = header_word0(x.t, x.q);
    d.hdr[1] = x.n;
    d.hdr[2] = 0;
    d.hdr[3] = __builtin_bit_cast(uint64_t, x.eb);
    d.hdr[4] = hp.step;
    d.hdr[5] = hp.bound;
    d.hdr[6] = hp.aux0;
    d.hdr[7] = hp.aux1;
    d.ntiles = field_tiles(x, tn);
    d.cpw = tn.cpw(x.t);
    if (kBatchVariants[bv].chunk) {
      field_groups(d.ntiles, tn.cpw(x.t), d.tiles_per_group, d.ngroups);
      d.chunks_per_group = d.tiles_per_group * (kChunkTile / kChunk) * d.cpw;
      d.group_off = L.groups + 8 * group_off;
      d.counts_off = L.counts + count_off;
      d.stage_off = L.stage + stage_off;
      group_off += d.ngroups;
      count_off += up256(4 * n_chunks(x.n));
      stage_off += up256(stage_bytes_per_chunk(x.t) * n_chunks(x.n));
      for (uint64_t g = 0; g < d.ngroups; g++) items_f.push_back(((uint64_t)i << 32) | g);
    } else {
      d.state_off = state_off;
      state_off += d.ntiles;
    }
    if (x.q == LCQ_NOA) {
      d.noa_idx = noa_idx++;
      d.nslices = (uint32_t)std::max<uint64_t>(1, (x.n + kSlice - 1) / kSlice);
      d.partial_off = part_off;
      part_off += up256((uint64_t)d.nslices * 2 * (x.t == LCQ_F64 ? 8 : 4));
      for (uint32_t s = 0; s < d.nslices; s++) items_a.push_back(((uint64_t)i << 32) | s);
    }
    const uint64_t ndt = (x.n + kDeqTile - 1) / kDeqTile;
    for (uint64_t t = 0; t < ndt; t++) items_d.push_back(((uint64_t)i << 32) | t);
  }
  // phase B: larger fields first (their tiles are the long tail), each
  // field's tiles in increasing order
  std::vector<uint32_t> order(nf);
  for (uint32_t i = 0; i < nf; i++) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](uint32_t a, uint32_t b) { return f[a].n * (f[a].t == LCQ_F64 ? 8 : 4) >
                                                        f[b].n * (f[b].t == LCQ_F64 ? 8 : 4); });
  for (uint32_t i : order) {
    for (uint64_t t = 0; t < bf[i].ntiles; t++) items_b.push_back(((uint64_t)i << 32) | t);
  }
  std::vector<uint64_t> items_q(items_a);
  items_q.insert(items_q.end(), items_b.begin(), items_b.end());

  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  if (nf && hipMemcpyAsync(ws + L.fields, bf.data(), sizeof(BField) * nf, hipMemcpyHostToDevice, stream) != hipSuccess) return LCQ_ERR_HIP;
  if (!items_q.empty() && hipMemcpyAsync(ws + L.items_q, items_q.data(), 8 * items_q.size(), hipMemcpyHostToDevice, stream) != hipSuccess) return LCQ_ERR_HIP;
  if (!items_d.empty() && hipMemcpyAsync(ws + L.items_d, items_d.data(), 8 * items_d.size(), hipMemcpyHostToDevice, stream) != hipSuccess) return LCQ_ERR_HIP;
  if (!items_f.empty() && hipMemcpyAsync(ws + L.items_f, items_f.data(), 8 * items_f.size(), hipMemcpyHostToDevice, stream) != hipSuccess) return LCQ_ERR_HIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return LCQ_ERR_HIP;

  lcq_batch_plan *p = new (std::nothrow) lcq_batch_plan();
  if (!p) return LCQ_ERR_ARG;
  p->variant = bv;
  p->tune = tn;
  p->nf = nf;
  p->can_decode = true;
  for (uint32_t i = 0; i < nf; i++)
    if (f[i].n && !f[i].d_out) p->can_decode = false;
  p->ws = ws;
  p->L = L;
  p->c = c;
  // one workgroup per work item
  p->grid = (unsigned)(c.n_a + c.n_b);

  BatchQArgs qa{};
  qa.fields = reinterpret_cast<const BField *>(ws + L.fields);
  qa.items = reinterpret_cast<const uint64_t *>(ws + L.items_q);
  qa.n_a = c.n_a;
  qa.n_items = c.n_a + c.n_b;
  qa.head = reinterpret_cast<unsigned *>(ws + L.head);
  qa.params = reinterpret_cast<DevParams *>(ws + L.params);
  qa.done = reinterpret_cast<unsigned *>(ws + L.done);
  qa.state = reinterpret_cast<uint64_t *>(ws + L.state);
  qa.partials = ws + L.partials;
  qa.items_f = reinterpret_cast<const uint64_t *>(ws + L.items_f);
  qa.ws = ws;
  qa.spin_limit = g_spin_limit.load();
  qa.ready_polls = g_spin_limit.load() ? (1u << 15) : 0u;
  BatchDArgs da{};
  da.fields = qa.fields;
  da.items = reinterpret_cast<const uint64_t *>(ws + L.items_d);
  da.n_items = c.n_d;
  da.status = reinterpret_cast<unsigned long long *>(ws + L.dstatus);

  if (hipMemcpyAsync(ws + L.args, &qa, sizeof qa, hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    delete p;
    return LCQ_ERR_HIP;
  }
  const BatchQArgs *qa_dev = reinterpret_cast<const BatchQArgs *>(ws + L.args);

  // capture: clear + quantize; clear + dequantize
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) { delete p; return LCQ_ERR_HIP; }
  lcq_status st = LCQ_OK;
  const unsigned cgrid = (unsigned)std::min<uint64_t>((L.clear_words + kBlock - 1) / kBlock, 1024);
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) st = LCQ_ERR_HIP;
  if (st == LCQ_OK) {
    hipLaunchKernelGGL(k_batch_clear, dim3(cgrid), dim3(kBlock), 0, cs,
                       reinterpret_cast<uint64_t *>(ws), L.clear_words);
    if (qa.n_items) st = launch_batch_quantize(bv, qa_dev, p->grid, cs);
    if (st == LCQ_OK && kBatchVariants[bv].chunk && c.n_f) {
      hipLaunchKernelGGL(k_batch_finish, dim3((unsigned)c.n_f), dim3(kBlock), 0, cs, qa_dev);
      if (hipGetLastError() != hipSuccess) st = LCQ_ERR_HIP;
    }
    if (hipStreamEndCapture(cs, &p->gq) != hipSuccess) st = LCQ_ERR_HIP;
  }
  if (st == LCQ_OK && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) st = LCQ_ERR_HIP;
  if (st == LCQ_OK) {
    const uint64_t sw = up256(8ull * std::max<uint32_t>(nf, 1)) / 8;
    hipLaunchKernelGGL(k_batch_clear, dim3(1), dim3(kBlock), 0, cs,
                       reinterpret_cast<uint64_t *>(ws + L.dstatus), sw);
    if (c.n_d) hipLaunchKernelGGL(k_batch_dequantize, dim3((unsigned)c.n_d), dim3(kBlock), 0, cs, da);
    if (hipGetLastError() != hipSuccess) st = LCQ_ERR_HIP;
    if (hipStreamEndCapture(cs, &p->gd) != hipSuccess) st = LCQ_ERR_HIP;
  }
  if (st == LCQ_OK && hipGraphInstantiate(&p->eq, p->gq, nullptr, nullptr, 0) != hipSuccess) st = LCQ_ERR_HIP;
  if (st == LCQ_OK && hipGraphInstantiate(&p->ed, p->gd, nullptr, nullptr, 0) != hipSuccess) st = LCQ_ERR_HIP;
  (void)hipStreamDestroy(cs);
  if (st != LCQ_OK) {
    lcq_batch_plan_destroy(p);
    return st;
  }
  *out = p;
  return LCQ_OK;
}

lcq_status lcq_batch_quantize(lcq_batch_plan *p, hipStream_t s) {
  if (!p) return LCQ_ERR_ARG;
  return hipGraphLaunch(p->eq, s) == hipSuccess ? LCQ_OK : LCQ_ERR_HIP;
}

lcq_status lcq_batch_dequantize(lcq_batch_plan *p, hipStream_t s) {
  if (!p || !p->can_decode) return LCQ_ERR_ARG;
  return hipGraphLaunch(p->ed, s) == hipSuccess ? LCQ_OK : LCQ_ERR_HIP;
}

lcq_status lcq_batch_status(lcq_batch_plan *p, hipStream_t s, int64_t *h_first_bad) {
  if (!p || !h_first_bad) return LCQ_ERR_ARG;
  std::vector<uint64_t> st(std::max<uint32_t>(p->nf, 1));
  if (p->nf && hipMemcpyAsync(st.data(), p->ws + p->L.dstatus, 8ull * p->nf,
                              hipMemcpyDeviceToHost, s) != hipSuccess)
    return LCQ_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return LCQ_ERR_HIP;
  *h_first_bad = -1;
  for (uint32_t i = 0; i < p->nf; i++)
    if (st[i] & 0xFFFF) {
      *h_first_bad = i;
      break;
    }
  return LCQ_OK;
}

void lcq_batch_plan_destroy(lcq_batch_plan *p) {
  if (!p) return;
  if (p->eq) (void)hipGraphExecDestroy(p->eq);
  if (p->ed) (void)hipGraphExecDestroy(p->ed);
  if (p->gq) (void)hipGraphDestroy(p->gq);
  if (p->gd) (void)hipGraphDestroy(p->gd);
  delete p;
}

}  // extern "C"
