// lcq_host.hpp -- host-side parameter derivation shared by the plain and the
// batched entry points (sections 2.1, 2.2 and 3.2 of the paper), and the
// launch-shape variants the tuner chooses among.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdint>

#include "lcq.h"
#include "lcq_math.hpp"
#include "lcq_tile.hpp"

#pragma clang fp contract(off)

namespace lcq {

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Largest float not above the positive double v (the user's bound rounded
// down, so the guarantee holds for the decimal value the user asked for).
inline float round_down_f32(double v) {
  float t = (float)v;
  if ((double)t > v) t = std::nextafter(t, -INFINITY);
  return t;
}

// Exact test of c * (1 + eb) <= eb for c > 0, 0 < eb < 1, in integers: for
// c in [eb/2, eb] the difference d = eb - c is an exact double (Sterbenz),
// so the test is mc*me * 2^(ec+ee) <= md * 2^ed on the 53-bit integer
// significands.
inline bool rel_low_ok(double c, double eb) {
  if (c > eb) return false;
  if (c < 0.5 * eb) return true;
  const double d = eb - c;
  if (d == 0.0) return false;
  int ec, ee, ed;
  const uint64_t mc = (uint64_t)std::ldexp(std::frexp(c, &ec), 53);
  const uint64_t me = (uint64_t)std::ldexp(std::frexp(eb, &ee), 53);
  const uint64_t md = (uint64_t)std::ldexp(std::frexp(d, &ed), 53);
  const unsigned __int128 lhs = (unsigned __int128)mc * me;  // < 2^106
  const int s = ed - ec - ee + 53;  // compare lhs with md * 2^s
  if (s < 0) return false;          // md * 2^s < 2^52 <= lhs / 2^52
  if (s > 60) return true;          // md * 2^s >= 2^113 > lhs
  return lhs <= ((unsigned __int128)md << s);
}

// Largest double not above eb / (1 + eb) (the lower side of the REL range,
// section 2.1.2: |x'| >= |x| / (1 + eb)  <=>  |x| - |x'| <= |x| eb/(1+eb)).
inline double rel_low_double(double eb) {
  double c = eb / (1.0 + eb);
  while (!rel_low_ok(c, eb)) c = std::nextafter(c, 0.0);
  while (rel_low_ok(std::nextafter(c, INFINITY), eb)) c = std::nextafter(c, INFINITY);
  return c;
}

template <typename T> inline T rd_t(double eb);
template <> inline float rd_t<float>(double eb) { return round_down_f32(eb); }
template <> inline double rd_t<double>(double eb) { return eb; }

// Host-derived parameters (ABS, REL); NOA only gets its rounded bound here
// and the rest on the device from the data's range.
struct HostParams {
  uint64_t step, inv, bound, low;  // raw bits of T
  uint64_t aux0, aux1;             // header aux words
  uint64_t eb_down;                // RD_T(eb)
};

template <typename T> inline HostParams host_params(int q, double eb) {
  HostParams h{};
  const T e = rd_t<T>(eb);
  h.eb_down = to_bits(e);
  if (q == kABS || q == kABS_UNCHECKED) {
    const T step = e + e;  // bins of width 2e (section 2.2)
    h.step = to_bits(step);
    h.inv = to_bits((T)1 / step);
    h.bound = to_bits(e);
  } else if (q == kREL || q == kREL_LIBM) {
    // upper side checked against eh = RD(eb), lower side against
    // el = RD(eb/(1+eb)); bins of width 2*lambda in approximate-log2 space
    // with lambda = log2approx(1 + eh)  (section 3.2; the library-log2
    // ablation takes lambda = log2(1 + eh))
    const T el = rd_t<T>(rel_low_double(eb));
    const T lam = q == kREL_LIBM ? lib_log2((T)1 + e) : log2approx<T>((T)1 + e);
    const T step = lam + lam;
    h.step = to_bits(step);
    h.inv = to_bits((T)1 / step);
    h.bound = to_bits(e);
    h.low = to_bits(el);
    h.aux0 = to_bits(el);
  }
  return h;
}

template <typename T> inline FieldParams<T> field_params(const HostParams &h) {
  using U = typename FT<T>::U;
  FieldParams<T> p;
  p.step = from_bits((U)h.step);
  p.inv = from_bits((U)h.inv);
  p.bound = from_bits((U)h.bound);
  p.low = from_bits((U)h.low);
  p.lossless_all = 0;
  return p;
}

// Launch-shape variants.  Variants 0-5 are the single-pass kernels: a slot
// is one 128-bit load per thread of a 256-thread workgroup and a tile is
// slots x rounds of them; quantize variants also choose the look-back depth
// (loads per lane per round trip) and whether the rounds are unrolled.
// Variant 6 is the chunk-per-wavefront kernel (two-pass quantize): cpw
// chunks per wavefront per workgroup, pf of them loaded at a time.  (More
// chunks per wavefront, and software-pipelined forms, measured slower at
// every size tried and were removed.)
struct Shape {
  int slots, rounds;
  int cpw = 0, pf = 0;  // cpw > 0: chunk-per-wavefront kernel
};
struct QShape {
  int slots, rounds, depth;
  bool unroll;
  int cpw = 0, pf = 0;  // cpw > 0: two-pass chunk-per-wavefront kernel
};
constexpr int kNumVariants = 7;
constexpr QShape kQVariants[kNumVariants] = {
    {4, 1, 1, true}, {4, 4, 1, true}, {4, 4, 4, true},
    {4, 4, 1, false}, {4, 2, 2, true}, {4, 1, 4, true},
    {0, 0, 0, true, 1, 1}};
constexpr Shape kDVariants[kNumVariants] = {{4, 1}, {2, 2}, {4, 2}, {4, 4}, {2, 1}, {8, 1},
                                            {0, 0, 1, 1}};

// Values per quantize tile / codes per dequantize tile of a variant.
inline uint64_t quant_tile_len(lcq_dtype t, int v) {
  if (kQVariants[v].cpw)
    return (uint64_t)kChunk * (t == LCQ_F64 ? stage_waves<double>() : stage_waves<float>()) *
           kQVariants[v].cpw;
  const uint64_t w = t == LCQ_F64 ? 2 : 4;
  return (uint64_t)kBlock * w * kQVariants[v].slots * kQVariants[v].rounds;
}
inline uint64_t deq_tile_len(int v) {
  if (kDVariants[v].cpw) return (uint64_t)kChunk * kWaves * kDVariants[v].cpw;
  return (uint64_t)kBlock * 4 * kDVariants[v].slots * kDVariants[v].rounds;
}

// Process-wide tuning: variant per (operation, dtype); 0 = quantize.
extern std::atomic<int> g_variant[2][2];
extern std::atomic<unsigned> g_spin_limit;

}  // namespace lcq
