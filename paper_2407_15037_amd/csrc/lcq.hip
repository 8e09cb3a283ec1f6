// lcq.hip -- gfx950 kernels and the C ABI (include/lcq.h) of the ABS / REL /
// NOA guaranteed-error-bound quantizers (Fallin & Burtscher, CoDaC'24).
//
// Kernels (all memory-bound; no MFMA, nothing here is a contraction):
//   k_clear        zero the look-back state before a quantize
//   k_minmax       NOA pass 1: finite min / max per block (section 2.1.3);
//                  also clears the look-back state
//   k_noa_params   NOA pass 2 (one block): reduce the block results, derive
//                  ebR, step and 1/step on the device (no host round trip)
//   k_quantize     one tile per workgroup (tile = workgroup index, no
//                  atomic counter): 128-bit loads, classify / bin /
//                  reconstruct / verify per value (sections 2.2, 3.1-3.3),
//                  int32 code stores, ballot + LDS block scan of the outlier
//                  flags, single-pass decoupled look-back (bounded wait) for
//                  the tile's outlier offset, chunk-table entries, outlier
//                  scatter; the last tile writes the header and stream size
//   k_dequantize   one tile per workgroup, independent tiles: 128-bit code
//                  loads, chunk-table base + ballot rank for the outliers,
//                  reconstruction (section 3.2 for REL), 128-bit stores
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstring>

#include "lcq.h"
#include "lcq_math.hpp"

#pragma clang fp contract(off)

using namespace lcq;

namespace {

// ------------------------------------------------------------ workspace ---
// [0,8)      status word of the last dequantize: (epoch << 16) | status
// [64,128)   NOA parameters written by k_noa_params (DevParams)
// [256, ...) look-back state, one u64 per tile (cleared before each quantize)
// then       NOA per-block (min, max) pairs
constexpr uint64_t kWsParams = 64;
constexpr uint64_t kWsState = 256;
constexpr int kMinmaxBlocks = 2048;
constexpr int kBlock = 256;   // threads per workgroup (4 wave64)
constexpr int kSlots = 4;     // 128-bit loads in flight per thread

template <typename T> constexpr int vec_elems() { return 16 / (int)sizeof(T); }
template <typename T> constexpr uint64_t quant_tile() { return (uint64_t)kBlock * kSlots * vec_elems<T>(); }
constexpr uint64_t kDeqTile = (uint64_t)kBlock * kSlots * 4;  // codes per dequantize tile

struct DevParams {
  uint64_t step, inv, bound, lo, hi;  // raw bits of the field type
  int32_t lossless_all, pad;
};

// look-back state word: 2-bit flag | 62-bit count
constexpr uint64_t kFlagAgg = 1ull << 62;   // tile's own outlier count
constexpr uint64_t kFlagIncl = 2ull << 62;  // outliers up to and including the tile
constexpr uint64_t kValMask = (1ull << 62) - 1;

thread_local hipEvent_t g_ev_before = nullptr, g_ev_after = nullptr;
std::atomic<uint64_t> g_epoch{0};
std::atomic<unsigned> g_spin_limit{4096};

template <typename T> struct Vec;
template <> struct Vec<float> { using type = float4; };
template <> struct Vec<double> { using type = double2; };

__device__ __forceinline__ uint64_t load_state(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_state(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Outliers among the values of tile `u`, counted by one wave from the input
// (encode is a pure function of the value bits, so this equals what the
// tile's own workgroup counts).
template <typename T, int Q, uint64_t TILE>
__device__ uint64_t wave_count_tile(const T *in, uint64_t n, uint64_t u, const FieldParams<T> &p,
                                    int lane) {
  uint64_t cnt = 0;
  const uint64_t base = u * TILE;
  for (uint64_t i = lane; i < TILE; i += 64) {
    const uint64_t g = base + i;
    if (g < n) cnt += (encode<T, Q>(in[g], p) == kSent);
  }
  return wave_sum(cnt);
}

// Exclusive outlier prefix of `tile` (> 0), computed by wave 0 of the
// workgroup (decoupled look-back).  Lane l inspects tile (pos - l); a window
// ends at the nearest tile that has published its inclusive prefix.  Tiles
// are workgroup indices; the hardware dispatches workgroups in index order,
// so a predecessor is normally resident or finished and publishes its own
// count before it looks back.  The wait is nevertheless bounded: a
// predecessor that has published nothing after `spin_limit` polls has its
// count computed here from its input instead, so no order of dispatch can
// make a workgroup wait forever.
template <typename T, int Q, uint64_t TILE>
__device__ uint64_t look_back(uint64_t *state, uint64_t tile, int lane, unsigned spin_limit,
                              const T *in, uint64_t n, const FieldParams<T> &p) {
  uint64_t excl = 0;
  int64_t pos = (int64_t)tile - 1;
  while (true) {
    const int64_t idx = pos - lane;
    uint64_t s = kFlagIncl;  // before tile 0: inclusive prefix 0
    if (idx >= 0) {
      s = load_state(state + idx);
      for (unsigned polls = 0; (s >> 62) == 0 && polls < spin_limit; polls++) {
        __builtin_amdgcn_s_sleep(1);
        s = load_state(state + idx);
      }
    }
    uint64_t pending = __ballot((s >> 62) == 0);
    while (pending) {
      const int l = __ffsll((unsigned long long)pending) - 1;
      const uint64_t c = wave_count_tile<T, Q, TILE>(in, n, (uint64_t)(pos - l), p, lane);
      if (lane == l) s = kFlagAgg | c;
      pending &= pending - 1;
    }
    const uint64_t incl = __ballot((s >> 62) == 2);
    uint64_t v = s & kValMask;
    if (incl) {
      const int first = __ffsll((unsigned long long)incl) - 1;
      if (lane > first) v = 0;
      excl += wave_sum(v);
      return excl;
    }
    excl += wave_sum(v);
    pos -= 64;
  }
}

template <typename T> __device__ __forceinline__ FieldParams<T> dev_params(const DevParams &d) {
  using U = typename FT<T>::U;
  FieldParams<T> p;
  p.step = from_bits((U)d.step);
  p.inv = from_bits((U)d.inv);
  p.bound = from_bits((U)d.bound);
  p.low = (T)0;
  p.lossless_all = d.lossless_all;
  return p;
}

struct QuantArgs {
  const void *in;
  uint64_t n;
  uint8_t *stream;
  uint64_t *stream_bytes;
  uint64_t *state;
  unsigned spin_limit;    // look-back polls before counting a predecessor directly
  const DevParams *noa;   // NOA only: parameters computed on the device
  uint64_t ntiles;
  double eb;
  // ABS / REL parameters (raw bits of T), and the header's aux words
  uint64_t step, inv, bound, low, aux0, aux1;
};

template <typename T, int Q>
__global__ __launch_bounds__(kBlock) void k_quantize(QuantArgs a) {
  using F = FT<T>;
  using U = typename F::U;
  using V = typename Vec<T>::type;
  constexpr int W = vec_elems<T>();
  constexpr int NWAVE = kBlock / 64;
  constexpr uint64_t TILE = quant_tile<T>();
  constexpr uint64_t SLOT = (uint64_t)kBlock * W;          // values per slot
  constexpr int SLOTS_PER_CHUNK = (int)(kChunk / SLOT);    // 1 (f32) or 2 (f64)
  constexpr int CHUNKS_PER_TILE = (int)(TILE / kChunk);
  static_assert(kChunk % SLOT == 0 && TILE % kChunk == 0, "tile must cover whole chunks");

  __shared__ unsigned int s_wtot[kSlots][NWAVE];
  __shared__ uint64_t s_prefix;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const uint64_t tile = blockIdx.x;
  const uint64_t base = tile * TILE;
  const uint64_t n = a.n;

  FieldParams<T> p;
  if (Q == kNOA) {
    p = dev_params<T>(*a.noa);
  } else {
    p.step = from_bits((U)a.step);
    p.inv = from_bits((U)a.inv);
    p.bound = from_bits((U)a.bound);
    p.low = from_bits((U)a.low);
    p.lossless_all = 0;
  }

  const T *in = static_cast<const T *>(a.in);
  int32_t *codes = reinterpret_cast<int32_t *>(a.stream + 64);

  // ---- load: slot j of thread t holds values base + (j*kBlock + t)*W ...
  V v[kSlots];
#pragma unroll
  for (int j = 0; j < kSlots; j++) {
    const uint64_t i0 = base + ((uint64_t)j * kBlock + tid) * W;
    if (i0 + W <= n) {
      v[j] = *reinterpret_cast<const V *>(in + i0);
    } else {
      T tmp[W];
#pragma unroll
      for (int e = 0; e < W; e++) tmp[e] = (i0 + e < n) ? in[i0 + e] : (T)0;
      __builtin_memcpy(&v[j], tmp, sizeof(V));
    }
  }

  // ---- per value: classify, bin, reconstruct, verify; store codes
  unsigned int omask[kSlots];
  bool any = false;
#pragma unroll
  for (int j = 0; j < kSlots; j++) {
    const uint64_t i0 = base + ((uint64_t)j * kBlock + tid) * W;
    T x[W];
    __builtin_memcpy(x, &v[j], sizeof(V));
    int32_t c[W];
    unsigned int m = 0;
#pragma unroll
    for (int e = 0; e < W; e++) {
      c[e] = encode<T, Q>(x[e], p);
      if (c[e] == kSent && i0 + e < n) m |= 1u << e;
    }
    omask[j] = m;
    any |= (m != 0);
    if (i0 + W <= n) {
      if (W == 4) {
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

  // ---- rank the outliers inside the tile (input order = slot-major)
  const bool tile_any = __syncthreads_or(any);
  unsigned int lane_pre[kSlots];
  if (tile_any) {
    const uint64_t lt = __lanemask_lt();
#pragma unroll
    for (int j = 0; j < kSlots; j++) {
      unsigned int pre = 0, tot = 0;
#pragma unroll
      for (int e = 0; e < W; e++) {
        const uint64_t b = __ballot((omask[j] >> e) & 1u);
        pre += __popcll(b & lt);
        tot += __popcll(b);
      }
      lane_pre[j] = pre;
      if (lane == 0) s_wtot[j][wave] = tot;
    }
  } else if (tid < kSlots * NWAVE) {
    s_wtot[tid / NWAVE][tid % NWAVE] = 0;
  }
  __syncthreads();

  unsigned int tile_total = 0;
#pragma unroll
  for (int j = 0; j < kSlots; j++)
#pragma unroll
    for (int w = 0; w < NWAVE; w++) tile_total += s_wtot[j][w];

  // ---- tile offset: publish, look back, publish inclusive
  if (tile == 0) {
    if (tid == 0) {
      store_state(a.state, kFlagIncl | tile_total);
      s_prefix = 0;
    }
  } else {
    if (tid == 0) store_state(a.state + tile, kFlagAgg | tile_total);
    if (wave == 0) {
      const uint64_t excl = look_back<T, Q, TILE>(a.state, tile, lane, a.spin_limit, in, n, p);
      if (lane == 0) {
        store_state(a.state + tile, kFlagIncl | (excl + tile_total));
        s_prefix = excl;
      }
    }
  }
  __syncthreads();
  const uint64_t prefix = s_prefix;

  // ---- chunk table: outliers before each chunk of this tile
  uint64_t *chunk_tab = reinterpret_cast<uint64_t *>(a.stream + chunk_table_offset(n));
  if (tid < CHUNKS_PER_TILE) {
    const uint64_t cidx = tile * CHUNKS_PER_TILE + tid;
    if (cidx * kChunk < n) {
      uint64_t before = prefix;
      for (int j = 0; j < tid * SLOTS_PER_CHUNK; j++)
        for (int w = 0; w < NWAVE; w++) before += s_wtot[j][w];
      chunk_tab[cidx] = before;
    }
  }

  // ---- scatter outliers (raw bits, input order)
  if (tile_any) {
    U *outl = reinterpret_cast<U *>(a.stream + outlier_offset(n));
    uint64_t slot_base = prefix;
#pragma unroll
    for (int j = 0; j < kSlots; j++) {
      uint64_t off = slot_base;
      for (int w = 0; w < wave; w++) off += s_wtot[j][w];
      off += lane_pre[j];
      if (omask[j]) {
        U xb[W];
        __builtin_memcpy(xb, &v[j], sizeof(V));
        unsigned int m = omask[j];
#pragma unroll
        for (int e = 0; e < W; e++) {
          if ((m >> e) & 1u) outl[off++] = xb[e];
        }
      }
      for (int w = 0; w < NWAVE; w++) slot_base += s_wtot[j][w];
    }
  }

  // ---- last tile: header, padding, stream size
  if (tile == a.ntiles - 1 && tid == 0) {
    const uint64_t k = prefix + tile_total;
    const uint64_t ct = chunk_table_offset(n);
    const uint64_t ce = ct + 8 * n_chunks(n);
    const uint64_t oo = outlier_offset(n);
    for (uint64_t b = 64 + 4 * n; b < ct; b++) a.stream[b] = 0;
    for (uint64_t b = ce; b < oo; b++) a.stream[b] = 0;
    uint64_t h[8];
    h[0] = (uint64_t)kMagic | (1ull << 32) | ((uint64_t)(sizeof(T) == 8 ? 1 : 0) << 40) |
           ((uint64_t)Q << 48) | ((uint64_t)kLog2Chunk << 56);
    h[1] = n;
    h[2] = k;
    h[3] = __builtin_bit_cast(uint64_t, a.eb);
    if (Q == kNOA) {
      h[4] = a.noa->step;
      h[5] = a.noa->bound;
      h[6] = a.noa->lo;
      h[7] = a.noa->hi;
    } else {
      h[4] = a.step;
      h[5] = a.bound;
      h[6] = a.aux0;
      h[7] = a.aux1;
    }
    uint64_t *hd = reinterpret_cast<uint64_t *>(a.stream);
    for (int i = 0; i < 8; i++) hd[i] = h[i];
    *a.stream_bytes = oo + k * sizeof(T);
  }
}

// Header-only stream (n = 0).
template <typename T, int Q>
__global__ void k_header_only(QuantArgs a) {
  uint64_t *hd = reinterpret_cast<uint64_t *>(a.stream);
  hd[0] = (uint64_t)kMagic | (1ull << 32) | ((uint64_t)(sizeof(T) == 8 ? 1 : 0) << 40) |
          ((uint64_t)Q << 48) | ((uint64_t)kLog2Chunk << 56);
  hd[1] = 0;
  hd[2] = 0;
  hd[3] = __builtin_bit_cast(uint64_t, a.eb);
  if (Q == kNOA) {
    hd[4] = a.noa->step;
    hd[5] = a.noa->bound;
    hd[6] = a.noa->lo;
    hd[7] = a.noa->hi;
  } else {
    hd[4] = a.step;
    hd[5] = a.bound;
    hd[6] = a.aux0;
    hd[7] = a.aux1;
  }
  *a.stream_bytes = 64;
}

__global__ void k_clear(uint64_t *p, uint64_t count) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// NOA pass 1: finite min / max of this block's share; -0 counts as +0.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_minmax(const T *in, uint64_t n, T *partials,
                                                   uint64_t *clear, uint64_t clear_count) {
  using F = FT<T>;
  using V = typename Vec<T>::type;
  constexpr int W = vec_elems<T>();
  const uint64_t gtid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint64_t gsize = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = gtid; i < clear_count; i += gsize) clear[i] = 0;

  T lo = (T)INFINITY, hi = (T)-INFINITY;
  auto take = [&](T x) {
    const bool fin = ((to_bits(x) >> F::kMant) & F::kExpMask) != F::kExpMask;
    const T y = (x == (T)0) ? (T)0 : x;
    lo = fin ? fmin(lo, y) : lo;
    hi = fin ? fmax(hi, y) : hi;
  };
  const uint64_t nv = n / W;
  const V *vin = reinterpret_cast<const V *>(in);
  for (uint64_t i = gtid; i < nv; i += gsize) {
    V v = vin[i];
    T x[W];
    __builtin_memcpy(x, &v, sizeof(V));
#pragma unroll
    for (int e = 0; e < W; e++) take(x[e]);
  }
  for (uint64_t i = nv * W + gtid; i < n; i += gsize) take(in[i]);

#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
  }
  __shared__ T s_lo[kBlock / 64], s_hi[kBlock / 64];
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_lo[wave] = lo;
    s_hi[wave] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; w++) {
      lo = fmin(lo, s_lo[w]);
      hi = fmax(hi, s_hi[w]);
    }
    partials[2 * blockIdx.x] = lo;
    partials[2 * blockIdx.x + 1] = hi;
  }
}

// NOA pass 2: R = hi - lo over finite values, ebR <= eb * R (each rounded
// step followed by one step down), step = 2 ebR, inv = 1 / step.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_noa_params(const T *partials, int nparts, T eb_down,
                                                       DevParams *out) {
  T lo = (T)INFINITY, hi = (T)-INFINITY;
  for (int i = threadIdx.x; i < nparts; i += kBlock) {
    lo = fmin(lo, partials[2 * i]);
    hi = fmax(hi, partials[2 * i + 1]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
  }
  __shared__ T s_lo[kBlock / 64], s_hi[kBlock / 64];
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_lo[wave] = lo;
    s_hi[wave] = hi;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int w = 1; w < kBlock / 64; w++) {
    lo = fmin(lo, s_lo[w]);
    hi = fmax(hi, s_hi[w]);
  }
  const T tmax = from_bits((typename FT<T>::U)(((typename FT<T>::U)FT<T>::kExpMask << FT<T>::kMant) - 1));
  T r = hi - lo;
  if (r == (T)INFINITY) r = tmax;
  if (r > (T)0) r = step_down(r);
  const T b = eb_down * r;
  T ebr = b;
  if (b > (T)0) ebr = step_down(b);
  DevParams d;
  d.lo = to_bits(lo);
  d.hi = to_bits(hi);
  d.pad = 0;
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
  *out = d;
}

// ------------------------------------------------------------ dequantize ---
struct DeqArgs {
  const uint8_t *stream;
  uint64_t stream_bytes;
  uint64_t n;
  void *out;
  unsigned long long *status;
  uint64_t epoch;
  int dtype;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dequantize(DeqArgs a) {
  using U = typename FT<T>::U;
  constexpr int NWAVE = kBlock / 64;
  constexpr int CHUNKS_PER_TILE = (int)(kDeqTile / kChunk);
  __shared__ unsigned int s_wtot[kSlots][NWAVE];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t n = a.n;
  const uint64_t *hd = reinterpret_cast<const uint64_t *>(a.stream);
  const uint64_t h0 = hd[0];
  const uint64_t k = hd[2];
  const int q = (int)((h0 >> 48) & 0xFF);
  const uint64_t oo = outlier_offset(n);
  int err = 0;
  if ((uint32_t)h0 != kMagic || ((h0 >> 32) & 0xFF) != 1 ||
      (int)((h0 >> 40) & 0xFF) != a.dtype || q > 2 || ((h0 >> 56) & 0xFF) != kLog2Chunk ||
      hd[1] != n || k > n || oo + k * sizeof(T) > a.stream_bytes)
    err = LCQ_ERR_STREAM;
  const unsigned long long tag = (unsigned long long)(a.epoch << 16);
  if (blockIdx.x == 0 && tid == 0) atomicMax(a.status, tag | (unsigned long long)err);
  if (err || n == 0) return;

  const T step = from_bits((U)hd[4]);
  const bool rel = (q == kREL);
  const int32_t *codes = reinterpret_cast<const int32_t *>(a.stream + 64);
  const uint64_t *chunk_tab = reinterpret_cast<const uint64_t *>(a.stream + chunk_table_offset(n));
  const U *outl = reinterpret_cast<const U *>(a.stream + oo);
  T *out = static_cast<T *>(a.out);

  const uint64_t tile = blockIdx.x;
  const uint64_t base = tile * kDeqTile;

  int4 c[kSlots];
#pragma unroll
  for (int j = 0; j < kSlots; j++) {
    const uint64_t i0 = base + ((uint64_t)j * kBlock + tid) * 4;
    if (i0 + 4 <= n) {
      c[j] = *reinterpret_cast<const int4 *>(codes + i0);
    } else {
      int t[4];
#pragma unroll
      for (int e = 0; e < 4; e++) t[e] = (i0 + e < n) ? codes[i0 + e] : 0;
      c[j] = make_int4(t[0], t[1], t[2], t[3]);
    }
  }

  unsigned int omask[kSlots];
  bool any = false;
#pragma unroll
  for (int j = 0; j < kSlots; j++) {
    const int cc[4] = {c[j].x, c[j].y, c[j].z, c[j].w};
    const uint64_t i0 = base + ((uint64_t)j * kBlock + tid) * 4;
    unsigned int m = 0;
#pragma unroll
    for (int e = 0; e < 4; e++)
      if (cc[e] == kSent && i0 + e < n) m |= 1u << e;
    omask[j] = m;
    any |= (m != 0);
  }
  const bool tile_any = __syncthreads_or(any);
  unsigned int lane_pre[kSlots];
  uint64_t first = 0;
  if (tile_any) {
    const uint64_t lt = __lanemask_lt();
#pragma unroll
    for (int j = 0; j < kSlots; j++) {
      unsigned int pre = 0, tot = 0;
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const uint64_t b = __ballot((omask[j] >> e) & 1u);
        pre += __popcll(b & lt);
        tot += __popcll(b);
      }
      lane_pre[j] = pre;
      if (lane == 0) s_wtot[j][wave] = tot;
    }
    __syncthreads();
  }
  // chunk-table consistency: every entry of this tile, and the next tile's
  // first entry (or the outlier count after the last tile), must equal the
  // outliers counted before it (a dequantize slot is exactly one chunk)
  static_assert((uint64_t)kBlock * 4 == kChunk, "one dequantize slot per chunk");
  first = chunk_tab[tile * CHUNKS_PER_TILE];
  if (tid <= CHUNKS_PER_TILE) {
    const uint64_t cidx = tile * CHUNKS_PER_TILE + tid;
    uint64_t before = first;
    if (tile_any)
      for (int j = 0; j < tid; j++)
        for (int w = 0; w < NWAVE; w++) before += s_wtot[j][w];
    if (cidx * kChunk < n) {
      if (chunk_tab[cidx] != before) atomicMax(a.status, tag | (unsigned long long)LCQ_ERR_STREAM);
    } else if ((cidx - 1) * kChunk < n && before != k) {
      // first chunk past the end: the tile's total must close the count
      atomicMax(a.status, tag | (unsigned long long)LCQ_ERR_STREAM);
    }
  }
  if (first > k && tid == 0) atomicMax(a.status, tag | (unsigned long long)LCQ_ERR_STREAM);

  uint64_t slot_base = first;
#pragma unroll
  for (int j = 0; j < kSlots; j++) {
    const uint64_t i0 = base + ((uint64_t)j * kBlock + tid) * 4;
    const int cc[4] = {c[j].x, c[j].y, c[j].z, c[j].w};
    uint64_t off = slot_base;
    if (tile_any) {
      for (int w = 0; w < wave; w++) off += s_wtot[j][w];
      off += lane_pre[j];
    }
    T y[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
      if ((omask[j] >> e) & 1u) {
        // rank checked against the outlier count: never read past the stream
        y[e] = (off < k) ? from_bits(outl[off]) : (T)0;
        off++;
      } else {
        y[e] = decode<T>(cc[e], step, rel);
      }
    }
    if (i0 + 4 <= n) {
      if (sizeof(T) == 4) {
        float4 o;
        __builtin_memcpy(&o, y, 16);
        *reinterpret_cast<float4 *>(out + i0) = o;
      } else {
        double2 o0, o1;
        __builtin_memcpy(&o0, y, 16);
        __builtin_memcpy(&o1, y + 2, 16);
        *reinterpret_cast<double2 *>(out + i0) = o0;
        *reinterpret_cast<double2 *>(out + i0 + 2) = o1;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; e++)
        if (i0 + e < n) out[i0 + e] = y[e];
    }
    if (tile_any)
      for (int w = 0; w < NWAVE; w++) slot_base += s_wtot[j][w];
  }
}

// ----------------------------------------------------------- host side ---
bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Largest float not above the positive double v.
float round_down_f32(double v) {
  float t = (float)v;
  if ((double)t > v) t = std::nextafter(t, -INFINITY);
  return t;
}

// Exact test of c * (1 + eb) <= eb for 0 < c, 0 < eb < 1, with integers:
// for c in [eb/2, eb] the difference d = eb - c is an exact double
// (Sterbenz), so the test is  mc*me * 2^(ec+ee) <= md * 2^ed  on the
// 53-bit integer significands.
bool rel_low_ok(double c, double eb) {
  if (c > eb) return false;
  if (c < 0.5 * eb) return true;
  const double d = eb - c;
  if (d == 0.0) return false;
  int ec, ee, ed;
  const uint64_t mc = (uint64_t)std::ldexp(std::frexp(c, &ec), 53);
  const uint64_t me = (uint64_t)std::ldexp(std::frexp(eb, &ee), 53);
  const uint64_t md = (uint64_t)std::ldexp(std::frexp(d, &ed), 53);
  const unsigned __int128 lhs = (unsigned __int128)mc * me;  // < 2^106
  const int s = ed - ec - ee + 53;  // lhs * 2^(ec+ee-106) vs md * 2^(ed-53)
  if (s < 0) return false;          // rhs < 2^53 * 2^-1 ... below lhs >= 2^104
  if (s > 60) return true;          // rhs >= 2^113 > lhs
  return lhs <= ((unsigned __int128)md << s);
}

// Largest double not above eb / (1 + eb).
double rel_low_double(double eb) {
  double c = eb / (1.0 + eb);
  while (!rel_low_ok(c, eb)) c = std::nextafter(c, 0.0);
  while (rel_low_ok(std::nextafter(c, INFINITY), eb)) c = std::nextafter(c, INFINITY);
  return c;
}

struct HostParams {
  uint64_t step, inv, bound, low, aux0, aux1;
  uint64_t eb_down;  // NOA: round-down of eb in the field type
};

template <typename T> T rd_t(double eb);
template <> float rd_t<float>(double eb) { return round_down_f32(eb); }
template <> double rd_t<double>(double eb) { return eb; }

template <typename T> HostParams host_params(int q, double eb) {
  HostParams h{};
  const T e = rd_t<T>(eb);
  if (q == kABS) {
    const T step = e + e;
    h.step = to_bits(step);
    h.inv = to_bits((T)1 / step);
    h.bound = to_bits(e);
  } else if (q == kREL) {
    const T el = rd_t<T>(rel_low_double(eb));
    const T lam = log2approx<T>((T)1 + e);
    const T step = lam + lam;
    h.step = to_bits(step);
    h.inv = to_bits((T)1 / step);
    h.bound = to_bits(e);
    h.low = to_bits(el);
    h.aux0 = to_bits(el);
  } else {
    h.eb_down = to_bits(e);
  }
  return h;
}

uint64_t ws_need(lcq_quantizer q, lcq_dtype t, uint64_t n) {
  const uint64_t tile = t == LCQ_F64 ? quant_tile<double>() : quant_tile<float>();
  const uint64_t ntiles = (n + tile - 1) / tile;
  uint64_t b = kWsState + 8 * ntiles;
  if (q == LCQ_NOA) b = ((b + 255) & ~255ull) + 16ull * kMinmaxBlocks;
  return b;
}

lcq_status check_launch() {
  return hipGetLastError() == hipSuccess ? LCQ_OK : LCQ_ERR_HIP;
}

template <typename T, int Q>
lcq_status run_quantize(double eb, const void *d_in, uint64_t n, void *d_stream,
                        uint64_t *d_bytes, void *d_ws, hipStream_t s) {
  const HostParams hp = host_params<T>(Q, eb);
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  QuantArgs a{};
  a.in = d_in;
  a.n = n;
  a.stream = static_cast<uint8_t *>(d_stream);
  a.stream_bytes = d_bytes;
  a.state = reinterpret_cast<uint64_t *>(ws + kWsState);
  a.spin_limit = g_spin_limit.load(std::memory_order_relaxed);
  a.noa = reinterpret_cast<const DevParams *>(ws + kWsParams);
  a.eb = eb;
  a.step = hp.step;
  a.inv = hp.inv;
  a.bound = hp.bound;
  a.low = hp.low;
  a.aux0 = hp.aux0;
  a.aux1 = hp.aux1;
  const uint64_t tile = quant_tile<T>();
  a.ntiles = (n + tile - 1) / tile;
  const uint64_t clear_words = a.ntiles;
  uint64_t *clear_ptr = reinterpret_cast<uint64_t *>(ws + kWsState);

  if (Q == kNOA) {
    uint64_t poff = ((kWsState + 8 * a.ntiles + 255) & ~255ull);
    T *partials = reinterpret_cast<T *>(ws + poff);
    uint64_t want = (n + (uint64_t)kBlock * vec_elems<T>() * 4 - 1) /
                    ((uint64_t)kBlock * vec_elems<T>() * 4);
    int nb = (int)(want < 1 ? 1 : (want > (uint64_t)kMinmaxBlocks ? kMinmaxBlocks : want));
    hipLaunchKernelGGL(k_minmax<T>, dim3(nb), dim3(kBlock), 0, s, static_cast<const T *>(d_in),
                       n, partials, clear_ptr, clear_words);
    hipLaunchKernelGGL(k_noa_params<T>, dim3(1), dim3(kBlock), 0, s, partials, nb,
                       from_bits((typename FT<T>::U)hp.eb_down),
                       reinterpret_cast<DevParams *>(ws + kWsParams));
  } else if (clear_words) {
    const int nb = (int)std::min<uint64_t>((clear_words + kBlock - 1) / kBlock, 1024);
    hipLaunchKernelGGL(k_clear, dim3(nb), dim3(kBlock), 0, s, clear_ptr, clear_words);
  }
  if (n == 0) {
    hipLaunchKernelGGL((k_header_only<T, Q>), dim3(1), dim3(1), 0, s, a);
    return check_launch();
  }
  if (g_ev_before) (void)hipEventRecord(g_ev_before, s);
  hipLaunchKernelGGL((k_quantize<T, Q>), dim3((unsigned)a.ntiles), dim3(kBlock), 0, s, a);
  if (g_ev_after) (void)hipEventRecord(g_ev_after, s);
  return check_launch();
}

}  // namespace

// ------------------------------------------------------------------- ABI ---
extern "C" {

uint64_t lcq_max_stream_bytes(lcq_dtype t, uint64_t n) {
  if ((t != LCQ_F32 && t != LCQ_F64) || n > LCQ_MAX_N) return 0;
  return outlier_offset(n) + n * (t == LCQ_F64 ? 8 : 4);
}

uint64_t lcq_workspace_bytes(lcq_quantizer q, lcq_dtype t, uint64_t n) {
  if ((t != LCQ_F32 && t != LCQ_F64) || (q != LCQ_ABS && q != LCQ_REL && q != LCQ_NOA) ||
      n > LCQ_MAX_N)
    return 0;
  return ws_need(q, t, n);
}

lcq_status lcq_quantize(lcq_quantizer q, lcq_dtype t, double eb, const void *d_in, uint64_t n,
                        void *d_stream, uint64_t stream_cap, uint64_t *d_stream_bytes,
                        void *d_ws, uint64_t ws_bytes, hipStream_t stream) {
  if (q != LCQ_ABS && q != LCQ_REL && q != LCQ_NOA) return LCQ_ERR_ARG;
  if (t != LCQ_F32 && t != LCQ_F64) return LCQ_ERR_ARG;
  if (!(eb > 0.0) || !std::isfinite(eb) || (q == LCQ_REL && !(eb < 1.0))) return LCQ_ERR_ARG;
  if (n > LCQ_MAX_N) return LCQ_ERR_ARG;
  if ((n && !d_in) || !d_stream || !d_stream_bytes || !d_ws) return LCQ_ERR_ARG;
  if ((n && !aligned16(d_in)) || !aligned16(d_stream) || !aligned16(d_ws) ||
      ((uintptr_t)d_stream_bytes & 7u))
    return LCQ_ERR_ARG;
  if (stream_cap < lcq_max_stream_bytes(t, n)) return LCQ_ERR_CAPACITY;
  if (ws_bytes < ws_need(q, t, n)) return LCQ_ERR_CAPACITY;
  if (t == LCQ_F32) {
    switch (q) {
      case LCQ_ABS: return run_quantize<float, kABS>(eb, d_in, n, d_stream, d_stream_bytes, d_ws, stream);
      case LCQ_REL: return run_quantize<float, kREL>(eb, d_in, n, d_stream, d_stream_bytes, d_ws, stream);
      default: return run_quantize<float, kNOA>(eb, d_in, n, d_stream, d_stream_bytes, d_ws, stream);
    }
  }
  switch (q) {
    case LCQ_ABS: return run_quantize<double, kABS>(eb, d_in, n, d_stream, d_stream_bytes, d_ws, stream);
    case LCQ_REL: return run_quantize<double, kREL>(eb, d_in, n, d_stream, d_stream_bytes, d_ws, stream);
    default: return run_quantize<double, kNOA>(eb, d_in, n, d_stream, d_stream_bytes, d_ws, stream);
  }
}

lcq_status lcq_dequantize(lcq_dtype t, const void *d_stream, uint64_t stream_bytes, void *d_out,
                          uint64_t n, void *d_ws, uint64_t ws_bytes, hipStream_t stream) {
  if (t != LCQ_F32 && t != LCQ_F64) return LCQ_ERR_ARG;
  if (n > LCQ_MAX_N) return LCQ_ERR_ARG;
  if (!d_stream || (n && !d_out) || !d_ws) return LCQ_ERR_ARG;
  if (!aligned16(d_stream) || (n && !aligned16(d_out)) || !aligned16(d_ws)) return LCQ_ERR_ARG;
  if (ws_bytes < 8) return LCQ_ERR_CAPACITY;
  if (stream_bytes < outlier_offset(n)) return LCQ_ERR_STREAM;
  DeqArgs a{};
  a.stream = static_cast<const uint8_t *>(d_stream);
  a.stream_bytes = stream_bytes;
  a.n = n;
  a.out = d_out;
  a.status = static_cast<unsigned long long *>(d_ws);
  a.epoch = g_epoch.fetch_add(1) + 1;
  a.dtype = (int)t;
  const uint64_t ntiles = n ? (n + kDeqTile - 1) / kDeqTile : 1;
  if (g_ev_before) (void)hipEventRecord(g_ev_before, stream);
  if (t == LCQ_F32)
    hipLaunchKernelGGL(k_dequantize<float>, dim3((unsigned)ntiles), dim3(kBlock), 0, stream, a);
  else
    hipLaunchKernelGGL(k_dequantize<double>, dim3((unsigned)ntiles), dim3(kBlock), 0, stream, a);
  if (g_ev_after) (void)hipEventRecord(g_ev_after, stream);
  return check_launch();
}

lcq_status lcq_stream_status(const void *d_ws, hipStream_t stream, int32_t *h_err) {
  if (!d_ws || !h_err) return LCQ_ERR_ARG;
  uint64_t v = 0;
  if (hipMemcpyAsync(&v, d_ws, 8, hipMemcpyDeviceToHost, stream) != hipSuccess) return LCQ_ERR_HIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return LCQ_ERR_HIP;
  *h_err = (int32_t)(v & 0xFFFF);
  return LCQ_OK;
}

const char *lcq_status_string(lcq_status s) {
  switch (s) {
    case LCQ_OK: return "ok";
    case LCQ_ERR_ARG: return "invalid argument";
    case LCQ_ERR_CAPACITY: return "buffer smaller than required";
    case LCQ_ERR_STREAM: return "stream does not match its header or structure";
    case LCQ_ERR_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

void lcq_debug_set_lookback_spin(uint32_t polls) { g_spin_limit.store(polls); }

void lcq_profile_events(hipEvent_t before, hipEvent_t after) {
  g_ev_before = before;
  g_ev_after = after;
}

}  // extern "C"
