// lcq.hip -- gfx950 kernels and C ABI (include/lcq.h) of the plain, single-
// field ABS / REL / NOA guaranteed-error-bound quantizers (Fallin & Burtscher,
// CoDaC'24).  The per-tile work lives in lcq_tile.hpp and is shared with the
// batched path (lcq_batch.hip).
//
// Kernels (all memory-bound; no MFMA, nothing here is a contraction):
//   k_clear        zero the look-back state before a quantize (ABS / REL)
//   k_minmax       NOA pass 1 (lcq_range.hpp): finite min / max per
//                  workgroup (section 2.1.3); also zeroes the look-back state
//   k_noa_params   NOA pass 2 (lcq_range.hpp, one workgroup): reduce the
//                  per-workgroup results and derive ebR, step, 1/step on the
//                  device
//   k_quantize     one tile per workgroup, tile = workgroup index (no atomic
//                  counter): quant_tile (classify / bin / reconstruct / verify,
//                  code stores, in-tile ranks, bounded decoupled look-back,
//                  chunk table, outliers; last tile writes header and size)
//   k_dequantize   one tile per workgroup, independent tiles: dequant_tile
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>

#include "lcq.h"
#include "lcq_host.hpp"
#include "lcq_math.hpp"
#include "lcq_tile.hpp"
#include "lcq_chunk.hpp"
#include "lcq_range.hpp"

#pragma clang fp contract(off)

namespace lcq {
std::atomic<int> g_variant[2][2] = {{{6}, {6}}, {{6}, {6}}};  // [op][dtype]
std::atomic<unsigned> g_spin_limit{4096};
}  // namespace lcq

using namespace lcq;

namespace {

// ------------------------------------------------------------ workspace ---
// [0,8)      status word of the last dequantize: (epoch << 16) | status
// [64,128)   NOA parameters written by k_noa_params (DevParams)
// [256, ...) look-back state, one u64 per tile (cleared before each quantize)
// then       NOA per-workgroup (min, max) pairs
constexpr uint64_t kWsParams = 64;
constexpr uint64_t kWsState = 256;
constexpr uint64_t kMinTileF32 = 4096, kMinTileF64 = 2048;  // smallest quantize tile of any variant

thread_local hipEvent_t g_ev_before = nullptr, g_ev_after = nullptr, g_ev_mid = nullptr;
// Decode-call epochs tag the status word; starting from the clock keeps a
// workspace left over from another process from matching a new call.
uint64_t epoch_seed() {
  return (uint64_t)std::chrono::steady_clock::now().time_since_epoch().count() & 0xFFFFFFFFFFFull;
}
std::atomic<uint64_t> g_epoch{epoch_seed()};

struct PlainQ {
  const void *in;
  uint64_t n;
  uint8_t *stream;
  uint64_t *stream_bytes;
  uint64_t *state;
  uint64_t ntiles;
  unsigned spin_limit;
  const DevParams *noa;  // NOA: parameters computed on the device
  uint64_t step, inv, bound, low;
  uint64_t hdr[8];
};

template <typename T, int Q>
__device__ __forceinline__ QField<T> plain_field(const PlainQ &a) {
  using U = typename FT<T>::U;
  QField<T> f;
  f.in = static_cast<const T *>(a.in);
  f.n = a.n;
  f.stream = a.stream;
  f.stream_bytes = a.stream_bytes;
  f.state = a.state;
  f.ntiles = a.ntiles;
#pragma unroll
  for (int i = 0; i < 8; i++) f.hdr[i] = a.hdr[i];
  if constexpr (Q == kNOA) {
    const DevParams d = *a.noa;
    f.p = params_from<T>(d);
    f.hdr[4] = d.step;
    f.hdr[5] = d.bound;
    f.hdr[6] = d.lo;
    f.hdr[7] = d.hi;
  } else {
    f.p.step = from_bits((U)a.step);
    f.p.inv = from_bits((U)a.inv);
    f.p.bound = from_bits((U)a.bound);
    f.p.low = from_bits((U)a.low);
    f.p.lossless_all = 0;
  }
  return f;
}

template <typename T, int Q, int SL, int RD, int DP, bool UR>
__global__ __launch_bounds__(kBlock) void k_quantize(PlainQ a) {
  const QField<T> f = plain_field<T, Q>(a);
  quant_tile<T, Q, SL, RD, DP, UR>(f, blockIdx.x, a.spin_limit);
}

// Header-only stream (n = 0).
template <typename T, int Q>
__global__ void k_header_only(PlainQ a) {
  const QField<T> f = plain_field<T, Q>(a);
  uint64_t *hd = reinterpret_cast<uint64_t *>(a.stream);
  for (int i = 0; i < 8; i++) hd[i] = f.hdr[i];
  hd[1] = 0;
  hd[2] = 0;
  *a.stream_bytes = 64;
}

__global__ void k_clear(uint64_t *p, uint64_t count) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// Two-pass chunk-per-wavefront quantize (lcq_chunk.hpp).
struct StageQ {
  const void *in;
  uint64_t n;
  uint8_t *stream;
  uint64_t *stream_bytes;
  uint32_t *counts;
  void *stage;
  unsigned long long *group;
  uint64_t tiles_per_group, chunks_per_group, ngroups;
  const DevParams *noa;
  uint64_t step, inv, bound, low;  // ABS / REL parameters (raw bits)
  uint64_t hdr[8];
};

template <typename T, int Q>
__device__ __forceinline__ FieldParams<T> stage_params(const StageQ &a) {
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

template <typename T, int Q, int CPW, int PF>
__global__ __launch_bounds__(64 * stage_waves<T>()) void k_quant_stage(StageQ a) {
  using U = typename FT<T>::U;
  StageField<T> f;
  f.in = static_cast<const T *>(a.in);
  f.n = a.n;
  f.codes = reinterpret_cast<int32_t *>(a.stream + 64);
  f.counts = a.counts;
  f.stage = static_cast<U *>(a.stage);
  f.group = a.group;
  f.tiles_per_group = a.tiles_per_group;
  f.p = stage_params<T, Q>(a);
  quant_chunks<T, Q, CPW, PF>(f, blockIdx.x);
}

template <typename T, int Q>
__global__ __launch_bounds__(kBlock) void k_quant_finish(StageQ a) {
  using U = typename FT<T>::U;
  FinishField<T> f;
  f.in = static_cast<const T *>(a.in);
  f.n = a.n;
  f.stream = a.stream;
  f.stream_bytes = a.stream_bytes;
  f.counts = a.counts;
  f.stage = static_cast<const U *>(a.stage);
  f.group = a.group;
  f.chunks_per_group = a.chunks_per_group;
  f.ngroups = a.ngroups;
  f.noa = Q == kNOA ? a.noa : nullptr;
#pragma unroll
  for (int i = 0; i < 8; i++) f.hdr[i] = a.hdr[i];
  quant_finish<T>(f, blockIdx.x);
}

// In-line layout (the paper's own, section 3.1): a pure map per tile.
constexpr int kInlineSlots = 4;

template <typename T, int Q>
__global__ __launch_bounds__(kBlock) void k_quantize_inline(PlainQ a) {
  const QField<T> f = plain_field<T, Q>(a);
  quant_tile_inline<T, Q, kInlineSlots>(f, blockIdx.x);
}

// ------------------------------------------------------------ dequantize ---
struct PlainD {
  const uint8_t *stream;
  uint64_t stream_bytes;
  uint64_t n;
  void *out;
  unsigned long long *status;
  uint64_t epoch;
  int dtype;
};

// Header check shared by the dequantize kernels; fills f and returns false
// (after recording the status) when the stream does not describe this call.
// `want_q` < 0 accepts the three quantizers, else exactly that (ablation)
// quantizer code.
template <typename T>
__device__ __forceinline__ bool deq_setup(const PlainD &a, DField<T> &f, int want_q = -1) {
  using U = typename FT<T>::U;
  const uint64_t n = a.n;
  const uint64_t *hd = reinterpret_cast<const uint64_t *>(a.stream);
  const uint64_t h0 = hd[0];
  const uint64_t k = hd[2];
  const int q = (int)((h0 >> 48) & 0xFF);
  const uint64_t oo = outlier_offset(n);
  // the header must describe exactly this call's stream (dtype, n, layout)
  const bool bad_q = want_q < 0 ? q > 2 : q != want_q;
  const bool bad = (h0 & ~(0xFFull << 48)) != header_word0(a.dtype, 0) || bad_q ||
                   hd[1] != n || k > n || oo + k * sizeof(T) > a.stream_bytes;
  const unsigned long long tag = (unsigned long long)(a.epoch << 16);
  if (blockIdx.x == 0 && threadIdx.x == 0)
    report_status(a.status, tag, bad ? LCQ_ERR_STREAM : LCQ_OK);
  if (bad || n == 0) return false;
  f.stream = a.stream;
  f.n = n;
  f.k = k;
  f.step = from_bits((U)hd[4]);
  f.rel = (q == kREL || q == kREL_LIBM);
  f.out = static_cast<T *>(a.out);
  f.status = a.status;
  f.tag = tag;
  return true;
}

template <typename T, int CPW, int PF>
__global__ __launch_bounds__(kBlock) void k_dequantize_chunks(PlainD a) {
  DField<T> f;
  if (deq_setup<T>(a, f)) dequant_chunks<T, CPW, PF>(f, blockIdx.x);
}

// Decoder of the section 6 ablation streams (quantizer code Q in the header).
template <typename T, int Q>
__global__ __launch_bounds__(kBlock) void k_dequantize_ablation(PlainD a) {
  DField<T> f;
  if (deq_setup<T>(a, f, Q)) dequant_chunks<T, 1, 1, Q == kREL_LIBM>(f, blockIdx.x);
}

template <typename T, int SL, int RD>
__global__ __launch_bounds__(kBlock) void k_dequantize(PlainD a) {
  DField<T> f;
  if (deq_setup<T>(a, f)) dequant_tile<T, SL, RD>(f, blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dequantize_inline(PlainD a) {
  using U = typename FT<T>::U;
  const uint64_t n = a.n;
  const uint64_t *hd = reinterpret_cast<const uint64_t *>(a.stream);
  const uint64_t h0 = hd[0];
  const int q = (int)((h0 >> 48) & 0xFF);
  const uint64_t want0 = (uint64_t)kMagicInline | (1ull << 32) | ((uint64_t)a.dtype << 40);
  const bool bad = (h0 & ~(0xFFull << 48)) != want0 || q > 2 || hd[1] != n ||
                   inline_stream_bytes(n, sizeof(T)) > a.stream_bytes;
  const unsigned long long tag = (unsigned long long)(a.epoch << 16);
  if (blockIdx.x == 0 && threadIdx.x == 0)
    report_status(a.status, tag, bad ? LCQ_ERR_STREAM : LCQ_OK);
  if (bad || n == 0) return;
  dequant_tile_inline<T, kInlineSlots>(a.stream, n, from_bits((U)hd[4]), q == kREL,
                                      static_cast<T *>(a.out), blockIdx.x);
}

// ----------------------------------------------------------- host side ---
// Workspace layout beyond the status word and the NOA parameters:
//   single-pass variants  one look-back word per tile at kWsState
//   two-pass variants     group sums at kWsState, chunk counts, staged raw
//                         bits (stage_cap<T>() per chunk)
//   NOA                   per-workgroup (min, max) pairs after both
uint64_t align256(uint64_t v) { return (v + 255) & ~255ull; }
uint64_t ws_counts_off() { return align256(kWsState + 8 * kMaxGroups); }
uint64_t ws_stage_off(uint64_t n) { return align256(ws_counts_off() + 4 * n_chunks(n)); }
uint64_t ws_partials_off(lcq_dtype t, uint64_t n) {
  const uint64_t s = t == LCQ_F64 ? 8 : 4;
  const uint64_t tile = t == LCQ_F64 ? kMinTileF64 : kMinTileF32;
  const uint64_t lookback_end = kWsState + 8 * ((n + tile - 1) / tile);
  const uint64_t cap = t == LCQ_F64 ? stage_cap<double>() : stage_cap<float>();
  const uint64_t staged_end = ws_stage_off(n) + cap * s * n_chunks(n);
  return align256(std::max(lookback_end, staged_end));
}
uint64_t ws_need(lcq_quantizer q, lcq_dtype t, uint64_t n) {
  return ws_partials_off(t, n) + (q == LCQ_NOA ? 16ull * kMinmaxBlocks : 0);
}

lcq_status check_launch() { return hipGetLastError() == hipSuccess ? LCQ_OK : LCQ_ERR_HIP; }

constexpr int kAblationVariant = 6;  // the default chunk-per-wavefront kernels
static_assert(kQVariants[kAblationVariant].cpw > 0 && kDVariants[kAblationVariant].cpw == 1,
              "ablation variant is the two-pass chunk form");

template <typename T, int Q, int V>
void launch_quantize(const PlainQ &a, const StageQ &sq, hipStream_t s) {
  constexpr QShape sh = kQVariants[V];
  if constexpr (sh.cpw > 0) {
    hipLaunchKernelGGL((k_quant_stage<T, Q, sh.cpw, sh.pf>), dim3((unsigned)a.ntiles),
                       dim3(64 * stage_waves<T>()), 0, s, sq);
    if (g_ev_mid) (void)hipEventRecord(g_ev_mid, s);
    hipLaunchKernelGGL((k_quant_finish<T, Q>), dim3((unsigned)sq.ngroups), dim3(kBlock), 0, s,
                       sq);
  } else {
    hipLaunchKernelGGL((k_quantize<T, Q, sh.slots, sh.rounds, sh.depth, sh.unroll>),
                       dim3((unsigned)a.ntiles), dim3(kBlock), 0, s, a);
  }
}

template <typename T, int Q>
void launch_quantize_variant(int v, const PlainQ &a, const StageQ &sq, hipStream_t s) {
  switch (v) {
    case 1: return launch_quantize<T, Q, 1>(a, sq, s);
    case 2: return launch_quantize<T, Q, 2>(a, sq, s);
    case 3: return launch_quantize<T, Q, 3>(a, sq, s);
    case 4: return launch_quantize<T, Q, 4>(a, sq, s);
    case 5: return launch_quantize<T, Q, 5>(a, sq, s);
    case 6: return launch_quantize<T, Q, 6>(a, sq, s);
    default: return launch_quantize<T, Q, 0>(a, sq, s);
  }
}

template <typename T, int V>
void launch_dequantize(uint64_t ntiles, const PlainD &a, hipStream_t s) {
  constexpr Shape sh = kDVariants[V];
  if constexpr (sh.cpw > 0) {
    hipLaunchKernelGGL((k_dequantize_chunks<T, sh.cpw, sh.pf>), dim3((unsigned)ntiles),
                       dim3(kBlock), 0, s, a);
  } else {
    hipLaunchKernelGGL((k_dequantize<T, sh.slots, sh.rounds>), dim3((unsigned)ntiles),
                       dim3(kBlock), 0, s, a);
  }
}

template <typename T>
void launch_dequantize_variant(int v, uint64_t ntiles, const PlainD &a, hipStream_t s) {
  switch (v) {
    case 1: return launch_dequantize<T, 1>(ntiles, a, s);
    case 2: return launch_dequantize<T, 2>(ntiles, a, s);
    case 3: return launch_dequantize<T, 3>(ntiles, a, s);
    case 4: return launch_dequantize<T, 4>(ntiles, a, s);
    case 5: return launch_dequantize<T, 5>(ntiles, a, s);
    case 6: return launch_dequantize<T, 6>(ntiles, a, s);
    default: return launch_dequantize<T, 0>(ntiles, a, s);
  }
}

template <typename T, int Q>
lcq_status run_quantize(double eb, const void *d_in, uint64_t n, void *d_stream,
                        uint64_t *d_bytes, void *d_ws, hipStream_t s) {
  const int dt = sizeof(T) == 8 ? LCQ_F64 : LCQ_F32;
  // the ablations always run the default chunk kernels, so their timing
  // compares like with like
  const int v = Q >= kABS_UNCHECKED ? kAblationVariant
                                    : g_variant[0][dt].load(std::memory_order_relaxed);
  const HostParams hp = host_params<T>(Q, eb);
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  PlainQ a{};
  a.in = d_in;
  a.n = n;
  a.stream = static_cast<uint8_t *>(d_stream);
  a.stream_bytes = d_bytes;
  a.state = reinterpret_cast<uint64_t *>(ws + kWsState);
  a.spin_limit = g_spin_limit.load(std::memory_order_relaxed);
  a.noa = reinterpret_cast<const DevParams *>(ws + kWsParams);
  a.step = hp.step;
  a.inv = hp.inv;
  a.bound = hp.bound;
  a.low = hp.low;
  a.hdr[0] = header_word0(dt, Q);
  a.hdr[1] = n;
  a.hdr[2] = 0;
  a.hdr[3] = __builtin_bit_cast(uint64_t, eb);
  a.hdr[4] = hp.step;
  a.hdr[5] = hp.bound;
  a.hdr[6] = hp.aux0;
  a.hdr[7] = hp.aux1;
  const uint64_t tile = quant_tile_len((lcq_dtype)dt, v);
  a.ntiles = (n + tile - 1) / tile;

  // two-pass variants: groups of whole workgroups, one pass-2 workgroup each
  const bool staged = kQVariants[v].cpw > 0;
  StageQ sq{};
  uint64_t *clear_ptr = a.state;
  uint64_t clear_count = a.ntiles;
  if (staged) {
    sq.in = d_in;
    sq.n = n;
    sq.stream = a.stream;
    sq.stream_bytes = d_bytes;
    sq.counts = reinterpret_cast<uint32_t *>(ws + ws_counts_off());
    sq.stage = ws + ws_stage_off(n);
    sq.group = reinterpret_cast<unsigned long long *>(ws + kWsState);
    sq.tiles_per_group = tiles_per_group(a.ntiles, tile / kChunk);
    sq.chunks_per_group = sq.tiles_per_group * (tile / kChunk);
    sq.ngroups = (a.ntiles + sq.tiles_per_group - 1) / sq.tiles_per_group;
    sq.noa = a.noa;
    sq.step = a.step;
    sq.inv = a.inv;
    sq.bound = a.bound;
    sq.low = a.low;
    for (int i = 0; i < 8; i++) sq.hdr[i] = a.hdr[i];
    clear_ptr = reinterpret_cast<uint64_t *>(sq.group);
    clear_count = sq.ngroups;
  }

  if (Q == kNOA) {
    T *partials = reinterpret_cast<T *>(ws + ws_partials_off((lcq_dtype)dt, n));
    launch_noa_range<T>(static_cast<const T *>(d_in), n, partials, clear_ptr, clear_count,
                        from_bits((typename FT<T>::U)hp.eb_down),
                        reinterpret_cast<DevParams *>(ws + kWsParams), s);
  } else if (clear_count) {
    const unsigned nb = (unsigned)std::min<uint64_t>((clear_count + kBlock - 1) / kBlock, 1024);
    hipLaunchKernelGGL(k_clear, dim3(nb), dim3(kBlock), 0, s, clear_ptr, clear_count);
  }
  if (n == 0) {
    hipLaunchKernelGGL((k_header_only<T, Q>), dim3(1), dim3(1), 0, s, a);
    return check_launch();
  }
  if (g_ev_before) (void)hipEventRecord(g_ev_before, s);
  if constexpr (Q >= kABS_UNCHECKED) launch_quantize<T, Q, kAblationVariant>(a, sq, s);
  else launch_quantize_variant<T, Q>(v, a, sq, s);
  if (g_ev_after) (void)hipEventRecord(g_ev_after, s);
  return check_launch();
}

template <typename T, int Q>
lcq_status run_quantize_inline(double eb, const void *d_in, uint64_t n, void *d_stream,
                               void *d_ws, hipStream_t s) {
  const int dt = sizeof(T) == 8 ? LCQ_F64 : LCQ_F32;
  const HostParams hp = host_params<T>(Q, eb);
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  PlainQ a{};
  a.in = d_in;
  a.n = n;
  a.stream = static_cast<uint8_t *>(d_stream);
  a.noa = reinterpret_cast<const DevParams *>(ws + kWsParams);
  a.step = hp.step;
  a.inv = hp.inv;
  a.bound = hp.bound;
  a.low = hp.low;
  a.hdr[0] = (uint64_t)kMagicInline | (1ull << 32) | ((uint64_t)dt << 40) | ((uint64_t)Q << 48);
  a.hdr[1] = n;
  a.hdr[2] = 0;
  a.hdr[3] = __builtin_bit_cast(uint64_t, eb);
  a.hdr[4] = hp.step;
  a.hdr[5] = hp.bound;
  a.hdr[6] = hp.aux0;
  a.hdr[7] = hp.aux1;
  if (Q == kNOA) {
    T *partials = reinterpret_cast<T *>(ws + kWsState);
    launch_noa_range<T>(static_cast<const T *>(d_in), n, partials, nullptr, 0,
                        from_bits((typename FT<T>::U)hp.eb_down),
                        reinterpret_cast<DevParams *>(ws + kWsParams), s);
  }
  const uint64_t tile = (uint64_t)kBlock * (16 / sizeof(T)) * kInlineSlots;
  const uint64_t ntiles = n ? (n + tile - 1) / tile : 1;
  if (g_ev_before) (void)hipEventRecord(g_ev_before, s);
  hipLaunchKernelGGL((k_quantize_inline<T, Q>), dim3((unsigned)ntiles), dim3(kBlock), 0, s, a);
  if (g_ev_after) (void)hipEventRecord(g_ev_after, s);
  return check_launch();
}

uint64_t ws_need_inline(lcq_quantizer q) {
  return q == LCQ_NOA ? kWsState + 16ull * kMinmaxBlocks : 8;
}

}  // namespace

// ------------------------------------------------- allocation-free form ---
// The quantize workspace of lcq_quantize_noalloc: one fixed array per GPU,
// reserved when the code object is loaded and held until the process ends.
// On the host, `scratch` is only a stand-in for the symbol, not a device
// address; host code uses the address hipGetSymbolAddress returns for the
// current device (each GPU holds its own copy at its own address).
static __device__ __align__(256) uint8_t scratch[LCQ_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
lcq_status scratch_address(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LCQ_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LCQ_ERR_HIP;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return LCQ_OK;
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

lcq_status lcq_quantize_noalloc(lcq_quantizer q, lcq_dtype t, double eb, const void *d_in,
                                uint64_t n, void *d_stream, uint64_t stream_cap,
                                uint64_t *d_stream_bytes, hipStream_t stream) {
  if (q != LCQ_ABS && q != LCQ_REL && q != LCQ_NOA) return LCQ_ERR_ARG;
  if (t != LCQ_F32 && t != LCQ_F64) return LCQ_ERR_ARG;
  if (n > LCQ_MAX_N) return LCQ_ERR_ARG;
  if (ws_need(q, t, n) > LCQ_NOALLOC_SCRATCH_BYTES) return LCQ_ERR_CAPACITY;
  void *ws = nullptr;
  const lcq_status st = scratch_address(&ws);
  if (st != LCQ_OK) return st;
  // every word of the workspace a quantize reads is written earlier in the
  // same call (group sums and look-back words are cleared by its first
  // kernel), so what the previous call left in the array does not matter
  return lcq_quantize(q, t, eb, d_in, n, d_stream, stream_cap, d_stream_bytes, ws,
                      LCQ_NOALLOC_SCRATCH_BYTES, stream);
}

lcq_status lcq_dequantize(lcq_dtype t, const void *d_stream, uint64_t stream_bytes, void *d_out,
                          uint64_t n, void *d_ws, uint64_t ws_bytes, hipStream_t stream) {
  if (t != LCQ_F32 && t != LCQ_F64) return LCQ_ERR_ARG;
  if (n > LCQ_MAX_N) return LCQ_ERR_ARG;
  if (!d_stream || (n && !d_out) || !d_ws) return LCQ_ERR_ARG;
  if (!aligned16(d_stream) || (n && !aligned16(d_out)) || !aligned16(d_ws)) return LCQ_ERR_ARG;
  if (ws_bytes < 8) return LCQ_ERR_CAPACITY;
  if (stream_bytes < outlier_offset(n)) return LCQ_ERR_STREAM;
  const int v = g_variant[1][t].load(std::memory_order_relaxed);
  PlainD a{};
  a.stream = static_cast<const uint8_t *>(d_stream);
  a.stream_bytes = stream_bytes;
  a.n = n;
  a.out = d_out;
  a.status = static_cast<unsigned long long *>(d_ws);
  a.epoch = g_epoch.fetch_add(1) + 1;
  a.dtype = (int)t;
  const uint64_t tile = deq_tile_len(v);
  const uint64_t ntiles = n ? (n + tile - 1) / tile : 1;
  if (g_ev_before) (void)hipEventRecord(g_ev_before, stream);
  if (t == LCQ_F32) launch_dequantize_variant<float>(v, ntiles, a, stream);
  else launch_dequantize_variant<double>(v, ntiles, a, stream);
  if (g_ev_after) (void)hipEventRecord(g_ev_after, stream);
  return check_launch();
}

lcq_status lcq_quantize_ablation(lcq_ablation kind, lcq_dtype t, double eb, const void *d_in,
                                 uint64_t n, void *d_stream, uint64_t stream_cap,
                                 uint64_t *d_stream_bytes, void *d_ws, uint64_t ws_bytes,
                                 hipStream_t stream) {
  if (kind != LCQ_ABL_ABS_UNCHECKED && kind != LCQ_ABL_REL_LIBM) return LCQ_ERR_ARG;
  if (t != LCQ_F32 && t != LCQ_F64) return LCQ_ERR_ARG;
  if (!(eb > 0.0) || !std::isfinite(eb) || (kind == LCQ_ABL_REL_LIBM && !(eb < 1.0)))
    return LCQ_ERR_ARG;
  if (n > LCQ_MAX_N) return LCQ_ERR_ARG;
  if ((n && !d_in) || !d_stream || !d_stream_bytes || !d_ws) return LCQ_ERR_ARG;
  if ((n && !aligned16(d_in)) || !aligned16(d_stream) || !aligned16(d_ws) ||
      ((uintptr_t)d_stream_bytes & 7u))
    return LCQ_ERR_ARG;
  if (stream_cap < lcq_max_stream_bytes(t, n)) return LCQ_ERR_CAPACITY;
  const lcq_quantizer base = kind == LCQ_ABL_ABS_UNCHECKED ? LCQ_ABS : LCQ_REL;
  if (ws_bytes < ws_need(base, t, n)) return LCQ_ERR_CAPACITY;
  if (t == LCQ_F32) {
    if (kind == LCQ_ABL_ABS_UNCHECKED)
      return run_quantize<float, kABS_UNCHECKED>(eb, d_in, n, d_stream, d_stream_bytes, d_ws, stream);
    return run_quantize<float, kREL_LIBM>(eb, d_in, n, d_stream, d_stream_bytes, d_ws, stream);
  }
  if (kind == LCQ_ABL_ABS_UNCHECKED)
    return run_quantize<double, kABS_UNCHECKED>(eb, d_in, n, d_stream, d_stream_bytes, d_ws, stream);
  return run_quantize<double, kREL_LIBM>(eb, d_in, n, d_stream, d_stream_bytes, d_ws, stream);
}

lcq_status lcq_dequantize_ablation(lcq_ablation kind, lcq_dtype t, const void *d_stream,
                                   uint64_t stream_bytes, void *d_out, uint64_t n, void *d_ws,
                                   uint64_t ws_bytes, hipStream_t stream) {
  if (kind != LCQ_ABL_ABS_UNCHECKED && kind != LCQ_ABL_REL_LIBM) return LCQ_ERR_ARG;
  if (t != LCQ_F32 && t != LCQ_F64) return LCQ_ERR_ARG;
  if (n > LCQ_MAX_N) return LCQ_ERR_ARG;
  if (!d_stream || (n && !d_out) || !d_ws) return LCQ_ERR_ARG;
  if (!aligned16(d_stream) || (n && !aligned16(d_out)) || !aligned16(d_ws)) return LCQ_ERR_ARG;
  if (ws_bytes < 8) return LCQ_ERR_CAPACITY;
  if (stream_bytes < outlier_offset(n)) return LCQ_ERR_STREAM;
  PlainD a{};
  a.stream = static_cast<const uint8_t *>(d_stream);
  a.stream_bytes = stream_bytes;
  a.n = n;
  a.out = d_out;
  a.status = static_cast<unsigned long long *>(d_ws);
  a.epoch = g_epoch.fetch_add(1) + 1;
  a.dtype = (int)t;
  const uint64_t tile = deq_tile_len(kAblationVariant);
  const dim3 grid((unsigned)(n ? (n + tile - 1) / tile : 1));
  if (g_ev_before) (void)hipEventRecord(g_ev_before, stream);
  if (t == LCQ_F32) {
    if (kind == LCQ_ABL_ABS_UNCHECKED)
      hipLaunchKernelGGL((k_dequantize_ablation<float, kABS_UNCHECKED>), grid, dim3(kBlock), 0, stream, a);
    else
      hipLaunchKernelGGL((k_dequantize_ablation<float, kREL_LIBM>), grid, dim3(kBlock), 0, stream, a);
  } else {
    if (kind == LCQ_ABL_ABS_UNCHECKED)
      hipLaunchKernelGGL((k_dequantize_ablation<double, kABS_UNCHECKED>), grid, dim3(kBlock), 0, stream, a);
    else
      hipLaunchKernelGGL((k_dequantize_ablation<double, kREL_LIBM>), grid, dim3(kBlock), 0, stream, a);
  }
  if (g_ev_after) (void)hipEventRecord(g_ev_after, stream);
  return check_launch();
}

uint64_t lcq_inline_stream_bytes(lcq_dtype t, uint64_t n) {
  if ((t != LCQ_F32 && t != LCQ_F64) || n > LCQ_MAX_N) return 0;
  return inline_stream_bytes(n, t == LCQ_F64 ? 8 : 4);
}

uint64_t lcq_inline_workspace_bytes(lcq_quantizer q) {
  if (q != LCQ_ABS && q != LCQ_REL && q != LCQ_NOA) return 0;
  return ws_need_inline(q);
}

lcq_status lcq_quantize_inline(lcq_quantizer q, lcq_dtype t, double eb, const void *d_in,
                               uint64_t n, void *d_stream, uint64_t stream_cap, void *d_ws,
                               uint64_t ws_bytes, hipStream_t stream) {
  if (q != LCQ_ABS && q != LCQ_REL && q != LCQ_NOA) return LCQ_ERR_ARG;
  if (t != LCQ_F32 && t != LCQ_F64) return LCQ_ERR_ARG;
  if (!(eb > 0.0) || !std::isfinite(eb) || (q == LCQ_REL && !(eb < 1.0))) return LCQ_ERR_ARG;
  if (n > LCQ_MAX_N) return LCQ_ERR_ARG;
  if ((n && !d_in) || !d_stream || !d_ws) return LCQ_ERR_ARG;
  if ((n && !aligned16(d_in)) || !aligned16(d_stream) || !aligned16(d_ws)) return LCQ_ERR_ARG;
  if (stream_cap < lcq_inline_stream_bytes(t, n)) return LCQ_ERR_CAPACITY;
  if (ws_bytes < ws_need_inline(q)) return LCQ_ERR_CAPACITY;
  if (t == LCQ_F32) {
    switch (q) {
      case LCQ_ABS: return run_quantize_inline<float, kABS>(eb, d_in, n, d_stream, d_ws, stream);
      case LCQ_REL: return run_quantize_inline<float, kREL>(eb, d_in, n, d_stream, d_ws, stream);
      default: return run_quantize_inline<float, kNOA>(eb, d_in, n, d_stream, d_ws, stream);
    }
  }
  switch (q) {
    case LCQ_ABS: return run_quantize_inline<double, kABS>(eb, d_in, n, d_stream, d_ws, stream);
    case LCQ_REL: return run_quantize_inline<double, kREL>(eb, d_in, n, d_stream, d_ws, stream);
    default: return run_quantize_inline<double, kNOA>(eb, d_in, n, d_stream, d_ws, stream);
  }
}

lcq_status lcq_dequantize_inline(lcq_dtype t, const void *d_stream, uint64_t stream_bytes,
                                 void *d_out, uint64_t n, void *d_ws, uint64_t ws_bytes,
                                 hipStream_t stream) {
  if (t != LCQ_F32 && t != LCQ_F64) return LCQ_ERR_ARG;
  if (n > LCQ_MAX_N) return LCQ_ERR_ARG;
  if (!d_stream || (n && !d_out) || !d_ws) return LCQ_ERR_ARG;
  if (!aligned16(d_stream) || (n && !aligned16(d_out)) || !aligned16(d_ws)) return LCQ_ERR_ARG;
  if (ws_bytes < 8) return LCQ_ERR_CAPACITY;
  const uint64_t s = t == LCQ_F64 ? 8 : 4;
  if (stream_bytes < inline_stream_bytes(n, s)) return LCQ_ERR_STREAM;
  PlainD a{};
  a.stream = static_cast<const uint8_t *>(d_stream);
  a.stream_bytes = stream_bytes;
  a.n = n;
  a.out = d_out;
  a.status = static_cast<unsigned long long *>(d_ws);
  a.epoch = g_epoch.fetch_add(1) + 1;
  a.dtype = (int)t;
  const uint64_t tile = (uint64_t)kBlock * (16 / s) * kInlineSlots;
  const uint64_t ntiles = n ? (n + tile - 1) / tile : 1;
  if (g_ev_before) (void)hipEventRecord(g_ev_before, stream);
  if (t == LCQ_F32)
    hipLaunchKernelGGL(k_dequantize_inline<float>, dim3((unsigned)ntiles), dim3(kBlock), 0, stream, a);
  else
    hipLaunchKernelGGL(k_dequantize_inline<double>, dim3((unsigned)ntiles), dim3(kBlock), 0, stream, a);
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

int32_t lcq_tune_variants(void) { return kNumVariants; }

lcq_status lcq_tune_set(int32_t op, lcq_dtype t, int32_t variant) {
  if ((op != 0 && op != 1) || (t != LCQ_F32 && t != LCQ_F64) || variant < 0 ||
      variant >= kNumVariants)
    return LCQ_ERR_ARG;
  g_variant[op][t].store(variant);
  return LCQ_OK;
}

int32_t lcq_tune_get(int32_t op, lcq_dtype t) {
  if ((op != 0 && op != 1) || (t != LCQ_F32 && t != LCQ_F64)) return -1;
  return g_variant[op][t].load();
}

void lcq_profile_events(hipEvent_t before, hipEvent_t after) {
  g_ev_before = before;
  g_ev_after = after;
}

void lcq_profile_mid_event(hipEvent_t mid) { g_ev_mid = mid; }

}  // extern "C"
