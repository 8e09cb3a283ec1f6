// lcq_tile.hpp -- workgroup-level building blocks shared by the plain and the
// batched kernels: one quantize tile (with its outlier-offset look-back), one
// dequantize tile, one NOA range slice, and the NOA parameter derivation.
//
// A tile is ROUNDS x SLOTS "slots"; a slot is one 128-bit load per thread of
// a 256-thread workgroup (1024 float32 / 512 float64 values, 1024 codes),
// laid out so a wavefront reads 1 KiB contiguous bytes per load.  Input
// order inside a tile is slot-major, then thread, then element, which is
// the order the outlier ranks follow.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lcq_math.hpp"

#pragma clang fp contract(off)

namespace lcq {

constexpr int kBlock = 256;  // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;
// Wavefronts per workgroup of the quantize first pass (one chunk each),
// per dtype: for float32, 8 halves its group-counter atomic adds against 4
// (REL, with outliers in almost every chunk, adds on every workgroup):
// measured quantize ABS 195 -> 188 us, REL 203 -> 199 us on the 512^3 field
// (16: REL 249 us); for float64 (half the chunks per byte) 8 measured slower
// than 4 on the 384^3 grid (ABS pass 1 109 -> 112 us), so it keeps 4.  The
// pack plan takes 8 (kStageWaves).
constexpr int kStageWaves = 8;
template <typename T> constexpr int stage_waves() { return sizeof(T) == 4 ? 8 : 4; }

// look-back state word: 2-bit flag | 62-bit count
constexpr uint64_t kFlagAgg = 1ull << 62;   // the tile's own outlier count
constexpr uint64_t kFlagIncl = 2ull << 62;  // outliers up to and including the tile
constexpr uint64_t kValMask = (1ull << 62) - 1;

template <typename T> struct Vec;
template <> struct Vec<float> { using type = float4; };
template <> struct Vec<double> { using type = double2; };
template <typename T> constexpr int vec_elems() { return 16 / (int)sizeof(T); }

// Field parameters produced on the device (NOA), as raw bits of the type.
struct DevParams {
  uint64_t step, inv, bound, lo, hi;
  int32_t lossless_all, ready;
};

__device__ __forceinline__ uint64_t load_state(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_state(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Cross-lane steps on DPP (the data-parallel-primitive operand forms of
// the gfx9 family): a value from another lane in the same instruction,
// with no LDS round trip as in a permute shuffle.  A lane whose source is
// outside its row (row shifts), outside the wavefront (wave shift) or in a
// row left out by the row mask keeps `old`.  Callers run them with all 64
// lanes active: a lane reads the others' registers whatever their state.
namespace dpp {
constexpr int kQuadXor1 = 0xB1, kQuadXor2 = 0x4E;  // quad_perm [1,0,3,2], [2,3,0,1]
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowMirror = 0x140, kRowHalfMirror = 0x141;  // lane i of 16 / of 8 reads 15-i / 7-i
constexpr int kWaveShr1 = 0x138;    // lane l reads lane l - 1
constexpr int kRowBcast15 = 0x142;  // row r reads lane 16 r - 1
constexpr int kRowBcast31 = 0x143;  // rows 2, 3 read lane 31
}  // namespace dpp
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t old, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWS, 0xf, false);
}
// v of lane l - 1; lane 0 gets fill.  fill goes through an empty asm so
// that the compiler cannot see a constant 0 in it: with one, it folds the
// shift into the consuming subtraction (v_subrev_u32 with the shifted
// operand), and that form measured wrong on gfx950 (the difference came
// out negated on most lanes), while the plain shifted move with `old`, and
// the folded add and or forms the other helpers compile to, measured right.
__device__ __forceinline__ uint32_t lane_up1(uint32_t v, uint32_t fill) {
  asm volatile("" : "+v"(fill));
  return dpp_mov<dpp::kWaveShr1>(fill, v);
}
// Inclusive prefix sum over the wavefront's lanes (mod 2^32): within each
// row of 16 lanes by shifts of 1, 2, 4 and 8, then rows 1 and 3 add the
// last lane of the row below them and rows 2 and 3 the last lane of rows
// 0-1.
__device__ __forceinline__ uint32_t wave_incl_add(uint32_t v) {
  v += dpp_mov<dpp::kRowShr1>(0u, v);
  v += dpp_mov<dpp::kRowShr2>(0u, v);
  v += dpp_mov<dpp::kRowShr4>(0u, v);
  v += dpp_mov<dpp::kRowShr8>(0u, v);
  v += dpp_mov<dpp::kRowBcast15, 0xa>(0u, v);
  v += dpp_mov<dpp::kRowBcast31, 0xc>(0u, v);
  return v;
}
// v of lane 63 (a uniform value).
__device__ __forceinline__ uint32_t lane63(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T> __device__ __forceinline__ FieldParams<T> params_from(const DevParams &d) {
  using U = typename FT<T>::U;
  FieldParams<T> p;
  p.step = from_bits((U)d.step);
  p.inv = from_bits((U)d.inv);
  p.bound = from_bits((U)d.bound);
  p.low = (T)0;
  p.lossless_all = d.lossless_all;
  return p;
}

// Everything a workgroup needs to quantize one tile of one field.
template <typename T> struct QField {
  const T *in;
  uint64_t n;
  uint8_t *stream;
  uint64_t *stream_bytes;  // written by the field's last tile
  uint64_t *state;         // one look-back word per tile of this field
  uint64_t ntiles;
  FieldParams<T> p;
  uint64_t hdr[8];         // header words; word 2 (outlier count) is filled in
};

template <typename T, int SLOTS, int ROUNDS> struct QuantShape {
  static constexpr int W = vec_elems<T>();
  static constexpr int NSLOT = SLOTS * ROUNDS;
  static constexpr uint64_t SLOT = (uint64_t)kBlock * W;  // values per slot
  static constexpr uint64_t TILE = SLOT * NSLOT;
  static constexpr int SLOTS_PER_CHUNK = (int)(kChunk / SLOT);
  static constexpr int CHUNKS = (int)(TILE / kChunk);
  static_assert(kChunk % SLOT == 0, "a chunk is a whole number of slots");
  static_assert(TILE % kChunk == 0, "a tile is a whole number of chunks");
  static_assert(NSLOT * W <= 64, "outlier flags of a thread fit 64 bits");
  static_assert(NSLOT <= 64, "slot totals are scanned by one wavefront");
};

// Outliers among the values of tile u, counted by one wavefront straight
// from the input (encode is a pure function of the value bits, so this is
// what the tile's own workgroup counts).
template <typename T, int Q>
__device__ uint64_t wave_count_tile(const T *in, uint64_t n, uint64_t u, uint64_t tile_len,
                                    const FieldParams<T> &p, int lane) {
  uint64_t cnt = 0;
  const uint64_t base = u * tile_len;
  for (uint64_t i = lane; i < tile_len; i += 64) {
    const uint64_t g = base + i;
    if (g < n) cnt += (encode<T, Q>(in[g], p) == kSent);
  }
  return wave_sum(cnt);
}

// Exclusive outlier prefix of `tile` (> 0) by one wavefront: decoupled
// look-back.  Each round issues DEPTH loads per lane, so one memory
// round trip inspects the DEPTH * 64 nearest unvisited predecessors
// (batch j, lane l: tile pos - 64 j - l); the batches are then taken nearest
// first, and the look-back ends at the nearest tile that has published its
// inclusive prefix.  A tile that has published nothing after `spin_limit`
// polls has its count computed here from its input instead, so the wait
// ends whatever the dispatch order.
template <typename T, int Q, int DEPTH>
__device__ uint64_t look_back(uint64_t *state, uint64_t tile, uint64_t tile_len, int lane,
                              unsigned spin_limit, const T *in, uint64_t n,
                              const FieldParams<T> &p) {
  uint64_t excl = 0;
  int64_t pos = (int64_t)tile - 1;
  while (true) {
    uint64_t s[DEPTH];
#pragma unroll
    for (int j = 0; j < DEPTH; j++) {
      const int64_t idx = pos - 64 * j - lane;
      s[j] = idx >= 0 ? load_state(state + idx) : kFlagIncl;  // before tile 0: prefix 0
    }
#pragma unroll
    for (int j = 0; j < DEPTH; j++) {
      const int64_t idx = pos - 64 * j - lane;
      uint64_t sj = s[j];
      for (unsigned polls = 0; (sj >> 62) == 0 && polls < spin_limit; polls++) {
        __builtin_amdgcn_s_sleep(1);
        sj = load_state(state + idx);
      }
      uint64_t pending = __ballot((sj >> 62) == 0);
      while (pending) {
        const int l = __ffsll((unsigned long long)pending) - 1;
        const uint64_t c =
            wave_count_tile<T, Q>(in, n, (uint64_t)(pos - 64 * j - l), tile_len, p, lane);
        if (lane == l) sj = kFlagAgg | c;
        pending &= pending - 1;
      }
      const uint64_t incl = __ballot((sj >> 62) == 2);
      uint64_t v = sj & kValMask;
      if (incl) {
        const int first = __ffsll((unsigned long long)incl) - 1;
        if (lane > first) v = 0;
        return excl + wave_sum(v);
      }
      excl += wave_sum(v);
    }
    pos -= 64 * DEPTH;
  }
}

// Exclusive scan over `count` (<= 64) per-slot totals by wavefront 0;
// writes spre[0..count] (spre[count] = total) and returns the total to
// every lane.
__device__ __forceinline__ unsigned wave_scan_slots(const unsigned (*wtot)[kWaves], int count,
                                                    unsigned *spre, int lane) {
  unsigned v = 0;
  if (lane < count)
    for (int w = 0; w < kWaves; w++) v += wtot[lane][w];
  unsigned incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane < count) spre[lane] = incl - v;
  if (lane == count - 1) spre[count] = incl;
  return __shfl(incl, count - 1, 64);
}

// Quantize one tile of a field: per value classify / bin / reconstruct /
// verify (sections 2.2, 3.1-3.3), code stores, in-tile outlier ranks, the
// tile's outlier offset by look-back, chunk-table entries and the outliers'
// raw bits.  The field's last tile also writes the header and the size.
// DEPTH: look-back loads per lane per round trip; UNROLL: unroll the rounds
// (more loads in flight, more registers).
template <typename T, int Q, int SLOTS, int ROUNDS, int DEPTH = 1, bool UNROLL = true>
__device__ void quant_tile(const QField<T> &f, uint64_t tile, unsigned spin_limit) {
  using F = FT<T>;
  using U = typename F::U;
  using V = typename Vec<T>::type;
  using S = QuantShape<T, SLOTS, ROUNDS>;
  constexpr int W = S::W;
  constexpr int NSLOT = S::NSLOT;

  __shared__ unsigned s_wtot[NSLOT][kWaves];
  __shared__ unsigned s_spre[NSLOT + 1];
  __shared__ uint64_t s_prefix;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t n = f.n;
  const uint64_t base = tile * S::TILE;
  int32_t *codes = reinterpret_cast<int32_t *>(f.stream + 64);

  uint64_t omask = 0;
  auto one_round = [&](int r) {
    V v[SLOTS];
#pragma unroll
    for (int j = 0; j < SLOTS; j++) {
      const uint64_t i0 = base + ((uint64_t)(r * SLOTS + j) * kBlock + tid) * W;
      if (i0 + W <= n) {
        v[j] = *reinterpret_cast<const V *>(f.in + i0);
      } else {
        T tmp[W];
#pragma unroll
        for (int e = 0; e < W; e++) tmp[e] = (i0 + e < n) ? f.in[i0 + e] : (T)0;
        __builtin_memcpy(&v[j], tmp, sizeof(V));
      }
    }
#pragma unroll
    for (int j = 0; j < SLOTS; j++) {
      const int s = r * SLOTS + j;
      const uint64_t i0 = base + ((uint64_t)s * kBlock + tid) * W;
      T x[W];
      __builtin_memcpy(x, &v[j], sizeof(V));
      int32_t c[W];
#pragma unroll
      for (int e = 0; e < W; e++) {
        c[e] = encode<T, Q>(x[e], f.p);
        if (c[e] == kSent && i0 + e < n) omask |= 1ull << (s * W + e);
      }
      if (i0 + W <= n) {
        if constexpr (W == 4) {
          *reinterpret_cast<int4 *>(codes + i0) = make_int4(c[0], c[1], c[2], c[3]);
        } else {
          *reinterpret_cast<int2 *>(codes + i0) = make_int2(c[0], c[1]);
        }
      } else {
#pragma unroll
        for (int e = 0; e < W; e++)
          if (i0 + e < n) codes[i0 + e] = c[e];
      }
    }
  };
  if constexpr (UNROLL) {
#pragma unroll
    for (int r = 0; r < ROUNDS; r++) one_round(r);
  } else {
#pragma unroll 1
    for (int r = 0; r < ROUNDS; r++) one_round(r);
  }

  // ---- in-tile ranks: wave totals per slot, then a scan over slots
  const bool any = __syncthreads_or(omask != 0);
  if (any) {
#pragma unroll
    for (int s = 0; s < NSLOT; s++) {
      unsigned tot = 0;
#pragma unroll
      for (int e = 0; e < W; e++) tot += __popcll(__ballot((omask >> (s * W + e)) & 1u));
      if (lane == 0) s_wtot[s][wave] = tot;
    }
    __syncthreads();
  }

  // ---- tile offset: wave 0 scans the slot totals, publishes, looks back
  if (wave == 0) {
    uint64_t tile_total = 0;
    if (any) tile_total = wave_scan_slots(s_wtot, NSLOT, s_spre, lane);
    if (tile == 0) {
      if (lane == 0) {
        store_state(f.state, kFlagIncl | tile_total);
        s_prefix = 0;
      }
    } else {
      if (lane == 0) store_state(f.state + tile, kFlagAgg | tile_total);
      const uint64_t excl =
          look_back<T, Q, DEPTH>(f.state, tile, S::TILE, lane, spin_limit, f.in, n, f.p);
      if (lane == 0) {
        store_state(f.state + tile, kFlagIncl | (excl + tile_total));
        s_prefix = excl;
      }
    }
    if (tile == f.ntiles - 1 && lane == 0) {
      // header, padding and size (the last tile owns the end of the stream)
      const uint64_t k = s_prefix + tile_total;
      const uint64_t ct = chunk_table_offset(n);
      const uint64_t ce = ct + 8 * n_chunks(n);
      const uint64_t oo = outlier_offset(n);
      for (uint64_t b = 64 + 4 * n; b < ct; b++) f.stream[b] = 0;
      for (uint64_t b = ce; b < oo; b++) f.stream[b] = 0;
      uint64_t *hd = reinterpret_cast<uint64_t *>(f.stream);
#pragma unroll
      for (int i = 0; i < 8; i++) hd[i] = (i == 2) ? k : f.hdr[i];
      *f.stream_bytes = oo + k * sizeof(T);
    }
  }
  __syncthreads();
  const uint64_t prefix = s_prefix;

  // ---- chunk table: outliers before each chunk of the tile
  uint64_t *chunk_tab = reinterpret_cast<uint64_t *>(f.stream + chunk_table_offset(n));
  if (tid < S::CHUNKS) {
    const uint64_t cidx = tile * S::CHUNKS + tid;
    if (cidx * kChunk < n) chunk_tab[cidx] = prefix + (any ? s_spre[tid * S::SLOTS_PER_CHUNK] : 0u);
  }

  // ---- outliers: raw bits (re-read from the input), input order
  if (any) {
    U *outl = reinterpret_cast<U *>(f.stream + outlier_offset(n));
    const U *inb = reinterpret_cast<const U *>(f.in);
    const uint64_t lt = __lanemask_lt();
#pragma unroll
    for (int s = 0; s < NSLOT; s++) {
      if (s_spre[s + 1] == s_spre[s]) continue;  // no outlier in this slot (uniform)
      unsigned pre = 0;
#pragma unroll
      for (int e = 0; e < W; e++) pre += __popcll(__ballot((omask >> (s * W + e)) & 1u) & lt);
      const unsigned m = (unsigned)(omask >> (s * W)) & ((1u << W) - 1);
      if (m) {
        uint64_t off = prefix + s_spre[s] + pre;
        for (int w = 0; w < wave; w++) off += s_wtot[s][w];
        const uint64_t i0 = base + ((uint64_t)s * kBlock + tid) * W;
#pragma unroll
        for (int e = 0; e < W; e++)
          if ((m >> e) & 1u) outl[off++] = inb[i0 + e];
      }
    }
  }
}

// Record `code` in a decode status word (epoch << 16 | code) for the call
// tagged `tag`.  A word carrying another epoch -- an earlier call, or whatever
// the workspace held before -- is replaced; within one epoch the larger code
// wins.  Every successful exchange ends one reporting thread, so the loop
// ends once the other reporters of the moment have finished.
__device__ inline void report_status(unsigned long long *w, unsigned long long tag,
                                     unsigned long long code) {
  unsigned long long old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    if ((old >> 16) == (tag >> 16) && (old & 0xFFFFull) >= code) return;
    const unsigned long long prev = atomicCAS(w, old, tag | code);
    if (prev == old) return;
    old = prev;
  }
}

// Everything a workgroup needs to decode one tile of one stream.
template <typename T> struct DField {
  const uint8_t *stream;
  uint64_t n;
  uint64_t k;       // outlier count from the header
  T step;
  bool rel;
  T *out;
  unsigned long long *status;
  unsigned long long tag;  // (epoch << 16)
};

template <int SLOTS, int ROUNDS> struct DeqShape {
  static constexpr int NSLOT = SLOTS * ROUNDS;
  static constexpr uint64_t TILE = (uint64_t)kBlock * 4 * NSLOT;  // codes
  static constexpr int CHUNKS = NSLOT;  // one slot of 1024 codes = one chunk
  static_assert((uint64_t)kBlock * 4 == kChunk, "a dequantize slot is one chunk");
  static_assert(NSLOT * 4 <= 64, "outlier flags of a thread fit 64 bits");
};

// Decode one tile: 128-bit code loads, reconstruction, 128-bit stores; the
// outliers' ranks come from the chunk table plus in-tile ballots and their
// bits are gathered from the stream.  Every chunk-table entry the tile
// covers (and the next one) is checked against the counted sentinels.
template <typename T, int SLOTS, int ROUNDS>
__device__ void dequant_tile(const DField<T> &f, uint64_t tile) {
  using U = typename FT<T>::U;
  using S = DeqShape<SLOTS, ROUNDS>;
  constexpr int NSLOT = S::NSLOT;
  __shared__ unsigned s_wtot[NSLOT][kWaves];
  __shared__ unsigned s_spre[NSLOT + 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t n = f.n;
  const uint64_t base = tile * S::TILE;
  const int32_t *codes = reinterpret_cast<const int32_t *>(f.stream + 64);
  const uint64_t *chunk_tab = reinterpret_cast<const uint64_t *>(f.stream + chunk_table_offset(n));
  const U *outl = reinterpret_cast<const U *>(f.stream + outlier_offset(n));

  uint64_t omask = 0;
#pragma unroll
  for (int r = 0; r < ROUNDS; r++) {
    int4 c[SLOTS];
#pragma unroll
    for (int j = 0; j < SLOTS; j++) {
      const uint64_t i0 = base + ((uint64_t)(r * SLOTS + j) * kBlock + tid) * 4;
      if (i0 + 4 <= n) {
        c[j] = *reinterpret_cast<const int4 *>(codes + i0);
      } else {
        int t[4];
#pragma unroll
        for (int e = 0; e < 4; e++) t[e] = (i0 + e < n) ? codes[i0 + e] : 0;
        c[j] = make_int4(t[0], t[1], t[2], t[3]);
      }
    }
#pragma unroll
    for (int j = 0; j < SLOTS; j++) {
      const int s = r * SLOTS + j;
      const uint64_t i0 = base + ((uint64_t)s * kBlock + tid) * 4;
      const int32_t cc[4] = {c[j].x, c[j].y, c[j].z, c[j].w};
      T y[4];
#pragma unroll
      for (int e = 0; e < 4; e++) {
        // outliers get their bits after the ranks are known; 0 until then
        const bool sent = cc[e] == kSent;
        y[e] = sent ? (T)0 : decode<T>(cc[e], f.step, f.rel);
        if (sent && i0 + e < n) omask |= 1ull << (s * 4 + e);
      }
      if (i0 + 4 <= n) {
        if constexpr (sizeof(T) == 4) {
          float4 o;
          __builtin_memcpy(&o, y, 16);
          *reinterpret_cast<float4 *>(f.out + i0) = o;
        } else {
          double2 o0, o1;
          __builtin_memcpy(&o0, y, 16);
          __builtin_memcpy(&o1, y + 2, 16);
          *reinterpret_cast<double2 *>(f.out + i0) = o0;
          *reinterpret_cast<double2 *>(f.out + i0 + 2) = o1;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; e++)
          if (i0 + e < n) f.out[i0 + e] = y[e];
      }
    }
  }

  const bool any = __syncthreads_or(omask != 0);
  if (any) {
#pragma unroll
    for (int s = 0; s < NSLOT; s++) {
      unsigned tot = 0;
#pragma unroll
      for (int e = 0; e < 4; e++) tot += __popcll(__ballot((omask >> (s * 4 + e)) & 1u));
      if (lane == 0) s_wtot[s][wave] = tot;
    }
    __syncthreads();
    if (wave == 0) wave_scan_slots(s_wtot, NSLOT, s_spre, lane);
    __syncthreads();
  }

  // chunk-table consistency: entries of this tile and the one after it
  const uint64_t first = chunk_tab[tile * S::CHUNKS];
  if (tid <= S::CHUNKS) {
    const uint64_t cidx = tile * S::CHUNKS + tid;
    const uint64_t before = first + (any ? s_spre[tid] : 0u);
    bool bad = false;
    if (cidx * kChunk < n) bad = chunk_tab[cidx] != before;
    else if ((cidx - 1) * kChunk < n) bad = before != f.k;  // the count closes at the end
    if (bad) report_status(f.status, f.tag, LCQ_ERR_STREAM);
  }
  if (tid == 0 && first > f.k) report_status(f.status, f.tag, LCQ_ERR_STREAM);

  if (any) {
    const uint64_t lt = __lanemask_lt();
#pragma unroll
    for (int s = 0; s < NSLOT; s++) {
      if (s_spre[s + 1] == s_spre[s]) continue;
      unsigned pre = 0;
#pragma unroll
      for (int e = 0; e < 4; e++) pre += __popcll(__ballot((omask >> (s * 4 + e)) & 1u) & lt);
      const unsigned m = (unsigned)(omask >> (s * 4)) & 0xFu;
      if (m) {
        uint64_t off = first + s_spre[s] + pre;
        for (int w = 0; w < wave; w++) off += s_wtot[s][w];
        const uint64_t i0 = base + ((uint64_t)s * kBlock + tid) * 4;
#pragma unroll
        for (int e = 0; e < 4; e++) {
          if ((m >> e) & 1u) {
            // rank checked against the outlier count: never read past it
            f.out[i0 + e] = (off < f.k) ? from_bits(outl[off]) : (T)0;
            off++;
          }
        }
      }
    }
  }
}

// Finite min / max of in[begin, end) by one workgroup (-0 counts as +0);
// the result is valid in thread 0.
template <typename T>
__device__ void block_minmax(const T *in, uint64_t begin, uint64_t end, T &lo, T &hi) {
  using F = FT<T>;
  using V = typename Vec<T>::type;
  constexpr int W = vec_elems<T>();
  __shared__ T s_lo[kWaves], s_hi[kWaves];
  lo = (T)INFINITY;
  hi = (T)-INFINITY;
  auto take = [&](T x) {
    const bool fin = ((to_bits(x) >> F::kMant) & F::kExpMask) != F::kExpMask;
    const T y = (x == (T)0) ? (T)0 : x;
    lo = fin ? fmin(lo, y) : lo;
    hi = fin ? fmax(hi, y) : hi;
  };
  // begin is a multiple of W (slices are whole vectors); the tail is scalar
  const uint64_t vb = begin / W, ve = end / W;
  const V *vin = reinterpret_cast<const V *>(in);
  // eight 128-bit loads in flight per thread, then the remainder one by one
  constexpr int U = 8;
  uint64_t i = vb + threadIdx.x;
  for (; i + (U - 1) * kBlock < ve; i += U * kBlock) {
    V v[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      // streamed once here: non-temporal loads
      typedef T nv __attribute__((ext_vector_type(16 / sizeof(T))));
      const nv t = __builtin_nontemporal_load(reinterpret_cast<const nv *>(vin + i + u * kBlock));
      __builtin_memcpy(&v[u], &t, sizeof(V));
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      T x[W];
      __builtin_memcpy(x, &v[u], sizeof(V));
#pragma unroll
      for (int e = 0; e < W; e++) take(x[e]);
    }
  }
  for (; i < ve; i += kBlock) {
    V v = vin[i];
    T x[W];
    __builtin_memcpy(x, &v, sizeof(V));
#pragma unroll
    for (int e = 0; e < W; e++) take(x[e]);
  }
  for (uint64_t i = ve * W + threadIdx.x; i < end; i += kBlock) take(in[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_lo[wave] = lo;
    s_hi[wave] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int w = 1; w < kWaves; w++) {
      lo = fmin(lo, s_lo[w]);
      hi = fmax(hi, s_hi[w]);
    }
  __syncthreads();
}

// NOA parameters from the finite range (section 2.1.3): R = hi - lo
// (overflow clamped to the largest finite value), then ebR = RD(eb) * R with
// each rounded step followed by one step toward zero, so ebR <= eb * R
// exactly; no usable range -> every value lossless.
template <typename T> __device__ DevParams noa_params(T lo, T hi, T eb_down) {
  using U = typename FT<T>::U;
  const T tmax = from_bits((U)(((U)FT<T>::kExpMask << FT<T>::kMant) - 1));
  T r = hi - lo;
  if (r == (T)INFINITY) r = tmax;
  if (r > (T)0) r = step_down(r);
  const T b = eb_down * r;
  T ebr = b;
  if (b > (T)0) ebr = step_down(b);
  DevParams d;
  d.lo = to_bits(lo);
  d.hi = to_bits(hi);
  d.ready = 0;
  if (ebr > (T)0) {
    const T step = ebr + ebr;
    d.bound = to_bits(ebr);
    d.step = to_bits(step);
    d.inv = to_bits((T)1 / step);
    d.lossless_all = 0;
  } else {
    d.bound = 0;
    d.step = 0;
    d.inv = 0;
    d.lossless_all = 1;
  }
  return d;
}

// Header word 0: magic, version 1, dtype, quantizer, log2(chunk).
__host__ __device__ inline uint64_t header_word0(int dtype, int q) {
  return (uint64_t)kMagic | (1ull << 32) | ((uint64_t)dtype << 40) | ((uint64_t)q << 48) |
         ((uint64_t)kLog2Chunk << 56);
}

}  // namespace lcq

namespace lcq {

// ------------------------------------------------- in-line outlier layout --
// One word of the field type's width per value (its code sign-extended, or
// its raw bits when stored losslessly) plus one flag bit per value.
constexpr uint32_t kMagicInline = 0x4951434Cu;  // "LCQI"

__host__ __device__ inline uint64_t inline_flags_offset(uint64_t n, uint64_t s) {
  return align16(64 + s * n);
}
__host__ __device__ inline uint64_t inline_stream_bytes(uint64_t n, uint64_t s) {
  return inline_flags_offset(n, s) + (n + 7) / 8;
}

// OR together the W-bit masks of `lanes` consecutive lanes into one 32-bit
// word held by the first lane of each group (lane-major bit order, as the
// values are laid out).
template <int W> __device__ __forceinline__ unsigned gather_flag_word(unsigned m, int lane) {
  constexpr int LANES = 32 / W;
  static_assert(LANES == 8 || LANES == 16, "groups of 8 or 16 lanes");
  unsigned v = m << (W * (lane & (LANES - 1)));
  // the OR of each quad (exchanges with lane xor 1, then xor 2), of each 8
  // lanes (lane i with 7 - i: the other quad), of each 16 (i with 15 - i)
  v |= dpp_mov<dpp::kQuadXor1>(0u, v);
  v |= dpp_mov<dpp::kQuadXor2>(0u, v);
  v |= dpp_mov<dpp::kRowHalfMirror>(0u, v);
  if constexpr (LANES == 16) v |= dpp_mov<dpp::kRowMirror>(0u, v);
  return v;
}

// Store a flag word at byte offset `b` of the flag array of `nbytes` bytes;
// the tail of the array is written byte by byte.
__device__ __forceinline__ void store_flag_word(uint8_t *flags, uint64_t b, uint64_t nbytes,
                                                unsigned v) {
  if (b + 4 <= nbytes) {
    *reinterpret_cast<unsigned *>(flags + b) = v;
  } else {
    for (uint64_t i = 0; i < 4 && b + i < nbytes; i++) flags[b + i] = (uint8_t)(v >> (8 * i));
  }
}

// Vector types for non-temporal 128-bit accesses (every stream here is
// touched once).
template <typename T> struct NtVec;
template <> struct NtVec<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct NtVec<double> { typedef double type __attribute__((ext_vector_type(2))); };
typedef uint32_t nt_u4 __attribute__((ext_vector_type(4)));
typedef uint64_t nt_u2 __attribute__((ext_vector_type(2)));

// Quantize one tile in the in-line layout: a pure map, no scan.
template <typename T, int Q, int SLOTS>
__device__ void quant_tile_inline(const QField<T> &f, uint64_t tile) {
  using U = typename FT<T>::U;
  using V = typename Vec<T>::type;
  constexpr int W = vec_elems<T>();
  constexpr uint64_t TILE = (uint64_t)kBlock * W * SLOTS;
  const int tid = threadIdx.x, lane = tid & 63;
  const uint64_t n = f.n;
  const uint64_t base = tile * TILE;
  U *words = reinterpret_cast<U *>(f.stream + 64);
  const uint64_t fl = inline_flags_offset(n, sizeof(T));
  const uint64_t nflag = (n + 7) / 8;
  uint8_t *flags = f.stream + fl;

  V v[SLOTS];
#pragma unroll
  for (int j = 0; j < SLOTS; j++) {
    const uint64_t i0 = base + ((uint64_t)j * kBlock + tid) * W;
    if (i0 + W <= n) {
      const typename NtVec<T>::type t =
          __builtin_nontemporal_load(reinterpret_cast<const typename NtVec<T>::type *>(f.in + i0));
      __builtin_memcpy(&v[j], &t, sizeof(V));
    } else {
      T tmp[W];
#pragma unroll
      for (int e = 0; e < W; e++) tmp[e] = (i0 + e < n) ? f.in[i0 + e] : (T)0;
      __builtin_memcpy(&v[j], tmp, sizeof(V));
    }
  }
#pragma unroll
  for (int j = 0; j < SLOTS; j++) {
    const uint64_t i0 = base + ((uint64_t)j * kBlock + tid) * W;
    T x[W];
    __builtin_memcpy(x, &v[j], sizeof(V));
    U w[W];
    unsigned m = 0;
#pragma unroll
    for (int e = 0; e < W; e++) {
      const int32_t c = encode<T, Q>(x[e], f.p);
      const bool raw = c == kSent;
      // a code is stored sign-extended to the word; a raw value as its bits
      w[e] = raw ? to_bits(x[e]) : (U)(typename std::make_signed<U>::type)c;
      if (raw && i0 + e < n) m |= 1u << e;
    }
    if (i0 + W <= n) {
      if constexpr (sizeof(T) == 4) {
        const nt_u4 o = {(uint32_t)w[0], (uint32_t)w[1], (uint32_t)w[2], (uint32_t)w[3]};
        __builtin_nontemporal_store(o, reinterpret_cast<nt_u4 *>(words + i0));
      } else {
        const nt_u2 o = {(uint64_t)w[0], (uint64_t)w[1]};
        __builtin_nontemporal_store(o, reinterpret_cast<nt_u2 *>(words + i0));
      }
    } else {
#pragma unroll
      for (int e = 0; e < W; e++)
        if (i0 + e < n) words[i0 + e] = w[e];
    }
    const unsigned fw = gather_flag_word<W>(m, lane);
    constexpr int LANES = 32 / W;
    if ((lane & (LANES - 1)) == 0 && i0 < n) store_flag_word(flags, i0 / 8, nflag, fw);
  }
  if (tile == 0 && tid == 0) {
    uint64_t *hd = reinterpret_cast<uint64_t *>(f.stream);
#pragma unroll
    for (int i = 0; i < 8; i++) hd[i] = f.hdr[i];
  }
  if (tile == (n ? (n - 1) / TILE : 0) && tid == 0)
    for (uint64_t b = 64 + sizeof(T) * n; b < fl; b++) f.stream[b] = 0;
}

// Decode one tile of the in-line layout.
template <typename T, int SLOTS>
__device__ void dequant_tile_inline(const uint8_t *stream, uint64_t n, T step, bool rel, T *out,
                                    uint64_t tile) {
  using U = typename FT<T>::U;
  using V = typename Vec<T>::type;
  constexpr int W = vec_elems<T>();
  constexpr uint64_t TILE = (uint64_t)kBlock * W * SLOTS;
  const int tid = threadIdx.x;
  const uint64_t base = tile * TILE;
  const U *words = reinterpret_cast<const U *>(stream + 64);
  const uint8_t *flags = stream + inline_flags_offset(n, sizeof(T));
#pragma unroll
  for (int j = 0; j < SLOTS; j++) {
    const uint64_t i0 = base + ((uint64_t)j * kBlock + tid) * W;
    if (i0 >= n) continue;
    U w[W];
    if (i0 + W <= n) {
      if constexpr (sizeof(T) == 4) {
        const nt_u4 q4 = __builtin_nontemporal_load(reinterpret_cast<const nt_u4 *>(words + i0));
        w[0] = q4.x; w[1] = q4.y; w[2] = q4.z; w[3] = q4.w;
      } else {
        const nt_u2 q2 = __builtin_nontemporal_load(reinterpret_cast<const nt_u2 *>(words + i0));
        w[0] = q2.x; w[1] = q2.y;
      }
    } else {
#pragma unroll
      for (int e = 0; e < W; e++) w[e] = (i0 + e < n) ? words[i0 + e] : (U)0;
    }
    // the thread's W flag bits: W divides 8, so they sit in one byte
    const unsigned m = (flags[i0 / 8] >> (i0 % 8)) & ((1u << W) - 1);
    T y[W];
#pragma unroll
    for (int e = 0; e < W; e++)
      y[e] = ((m >> e) & 1u) ? from_bits(w[e]) : decode<T>((int32_t)(uint32_t)w[e], step, rel);
    if (i0 + W <= n) {
      typename NtVec<T>::type o;
      __builtin_memcpy(&o, y, sizeof(V));
      __builtin_nontemporal_store(o, reinterpret_cast<typename NtVec<T>::type *>(out + i0));
    } else {
#pragma unroll
      for (int e = 0; e < W; e++)
        if (i0 + e < n) out[i0 + e] = y[e];
    }
  }
}

}  // namespace lcq
