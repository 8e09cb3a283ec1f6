// lcq_math.hpp -- per-value arithmetic of the quantizers, shared by the host
// parameter derivation and the gfx950 kernels of this library.
//
// Everything here is IEEE-754 binary32/binary64 with round-to-nearest-even and
// subnormals kept; the translation unit is compiled with -ffp-contract=off and
// '#pragma clang fp contract(off)' so that no multiply-add is fused
// (section 3.2 of the paper: FMA contraction makes CPU and GPU disagree).
#pragma once
#include <stdint.h>

#pragma clang fp contract(off)

#define LCQ_HD __host__ __device__ __forceinline__

namespace lcq {

constexpr uint32_t kChunk = 1024;  // values per chunk-table entry
constexpr uint32_t kLog2Chunk = 10;
constexpr int32_t kSent = INT32_MIN;  // code of a value stored losslessly
constexpr uint32_t kMagic = 0x3151434Cu;  // "LCQ1"
constexpr double kMaxBin = 1073741824.0;  // 2^30; bins lie in (-2^30, 2^30)

template <typename T> struct FT;
template <> struct FT<float> {
  using U = uint32_t;
  static constexpr int kMant = 23;
  static constexpr U kExpMask = 0xFFu;
  static constexpr U kFracMask = 0x007FFFFFu;
  static constexpr U kSign = 0x80000000u;
  static constexpr int kBias = 127;
};
template <> struct FT<double> {
  using U = uint64_t;
  static constexpr int kMant = 52;
  static constexpr U kExpMask = 0x7FFu;
  static constexpr U kFracMask = 0x000FFFFFFFFFFFFFull;
  static constexpr U kSign = 0x8000000000000000ull;
  static constexpr int kBias = 1023;
};

LCQ_HD uint32_t to_bits(float x) { return __builtin_bit_cast(uint32_t, x); }
LCQ_HD uint64_t to_bits(double x) { return __builtin_bit_cast(uint64_t, x); }
LCQ_HD float from_bits(uint32_t u) { return __builtin_bit_cast(float, u); }
LCQ_HD double from_bits(uint64_t u) { return __builtin_bit_cast(double, u); }

LCQ_HD float rint_t(float x) { return __builtin_rintf(x); }
LCQ_HD double rint_t(double x) { return __builtin_rint(x); }
LCQ_HD float abs_t(float x) { return __builtin_fabsf(x); }
LCQ_HD double abs_t(double x) { return __builtin_fabs(x); }

// Next value toward zero of a positive value (positive infinity steps to the
// largest finite value).
template <typename T> LCQ_HD T step_down(T v) { return from_bits(to_bits(v) - 1); }

// Approximate log2 of section 3.2 (Mitchell): for |a| = 2^e (1 + m) it is
// e + m, computed as the float 1.m plus the float (E - bias - 1), where E is
// the biased exponent field.  The sign bit is ignored.
template <typename T> LCQ_HD T log2approx(T a) {
  using F = FT<T>;
  using U = typename F::U;
  const U u = to_bits(a);
  const int E = (int)((u >> F::kMant) & F::kExpMask);
  const T mant = from_bits((U)((U)F::kBias << F::kMant) | (u & F::kFracMask));
  return mant + (T)(E - (F::kBias + 1));
}

// Approximate 2^y of section 3.2, the inverse of log2approx: t = y + bias,
// k = trunc(t) is the exponent field, t - (k - 1) in [1,2) gives the fraction
// field.  t is clamped to [0, max exponent field] (NaN -> 0) first so the
// conversion is always defined; every code the encoder emits is inside.
template <typename T> LCQ_HD T pow2approx(T y) {
  using F = FT<T>;
  using U = typename F::U;
  // clamp to [0, max exponent field]; a (quiet) NaN t becomes 0 because
  // fmax returns the non-NaN operand -- t is an arithmetic result, never a
  // signalling NaN
  T t = y + (T)F::kBias;
  t = fmin(fmax(t, (T)0), (T)F::kExpMask);
  const int k = (int)t;
  const T g = t - (T)(k - 1);
  return from_bits((U)(((U)k << F::kMant) | (to_bits(g) & F::kFracMask)));
}

// Device forms, value for value the same as the plain ones above, in fewer
// instructions.
// - REL's bin rint(log2approx(x) * inv), float32 (rel_bin): with d the
//   integer (|x| bits) - 127 * 2^23 = (E - 127) 2^23 + fraction field,
//   log2approx(x) = e + m is d * 2^-23 rounded once to float, i.e. the
//   int-to-float conversion of d (one rounding to 24 bits, round to nearest
//   even) scaled by 2^-23.  2d is one shift-and-add of x's bits (the shift
//   drops the sign; for normal x, 1 <= E <= 254, it fits in an int32), its
//   conversion is log2approx(x) * 2^24 exactly, and inv * 2^-24 is exact
//   (inv >= 1/2 here, so no underflow), so the product and its rounding are
//   those of log2approx(x) * inv.  Non-normal x (stored losslessly whatever
//   the bin) give some finite bin.
// - pow2: t is finite here (a finite bin times a finite step), so the clamp
//   is one median-of-three; for t >= 0, t - (k - 1) = fract(t) + 1 exactly
//   when t >= 1 (both sides exact) and with the same single rounding of
//   t + 1 when t < 1 (k = 0).
// (lgoff: -127 * 2^24 mod 2^32, passed in so that a kernel can hold it in a
// scalar register)
template <typename T> __device__ __forceinline__ T rel_bin(T x, T inv, uint32_t lgoff = 0x81000000u) {
  if constexpr (sizeof(T) == 4) {
    const int32_t d2 = (int32_t)((to_bits(x) << 1) + lgoff);  // 2d
    return rint_t((float)d2 * (inv * 0x1p-24f));
  } else {
    return rint_t(log2approx(x) * inv);
  }
}
// (emax: the largest exponent field as a value of T, passed in so that a
// kernel can hold it in a register)
template <typename T> __device__ __forceinline__ T pow2approx_dev(T y, T emax) {
  if constexpr (sizeof(T) == 4) {
    const float t = __builtin_amdgcn_fmed3f(y + 127.0f, 0.0f, emax);
    const int k = (int)t;
    const float g = __builtin_amdgcn_fractf(t) + 1.0f;
    return from_bits((uint32_t)(((uint32_t)k << 23) | (to_bits(g) & 0x007FFFFFu)));
  } else {
    using F = FT<T>;
    using U = typename F::U;
    T t = y + (T)F::kBias;
    t = fmin(fmax(t, (T)0), emax);
    const int k = (int)t;
    const T g = t - (T)(k - 1);
    return from_bits((U)(((U)k << F::kMant) | (to_bits(g) & F::kFracMask)));
  }
}
template <typename T> __device__ __forceinline__ T pow2approx_dev(T y) {
  return pow2approx_dev(y, (T)FT<T>::kExpMask);
}

// Parameters of one field in the field's type.
template <typename T> struct FieldParams {
  T step;   // bin width
  T inv;    // 1 / step
  T bound;  // ABS: e, NOA: ebR, REL: upper-side relative bound eh
  T low;    // REL: lower-side relative bound el; otherwise unused
  int lossless_all;  // NOA field with no usable range: every value lossless
};

enum : int { kABS = 0, kREL = 1, kNOA = 2 };
// The two ablations of section 6 (no guarantee by design): ABS without the
// double-check, and REL with the math library's log2 / exp2 in place of the
// section 3.2 approximations.
enum : int { kABS_UNCHECKED = 3, kREL_LIBM = 4 };
template <int Q> constexpr bool is_rel_q() { return Q == kREL || Q == kREL_LIBM; }

LCQ_HD float lib_log2(float x) { return log2f(x); }
LCQ_HD double lib_log2(double x) { return log2(x); }
LCQ_HD float lib_exp2(float x) { return exp2f(x); }
LCQ_HD double lib_exp2(double x) { return exp2(x); }

// Whether x may be quantized at all (sections 2.2 and 3.1): INF, NaN and
// denormals are stored losslessly, and for REL zeros too.  One class test:
// bits 3 and 8 of its mask are the negative and positive normals, bits 5
// and 6 the negative and positive zeros.
template <int Q> constexpr int class_mask() {
  constexpr int kNormal = (1 << 3) | (1 << 8), kZero = (1 << 5) | (1 << 6);
  return is_rel_q<Q>() ? kNormal : (kNormal | kZero);
}
template <typename T> __device__ __forceinline__ bool class_test(T x, int m) {
  if constexpr (sizeof(T) == 4) return __builtin_amdgcn_classf(x, m);
  else return __builtin_amdgcn_class(x, m);
}
template <typename T, int Q> __device__ __forceinline__ bool quantizable(T x) {
  return class_test(x, class_mask<Q>());
}

// Operands of the per-value encoder that its instructions cannot take as
// immediates or as a second scalar operand (the class-test mask, the upper
// end of pow2approx's clamp, the sentinel code, REL's two side bounds read
// by one select).  A kernel may hold them in vector registers for its whole
// run (pin_v); otherwise the compiler rebuilds each one at every use.
template <typename T> struct EncK {
  T emax, bound, low;
  int32_t sent;
  int cls;
  uint32_t lgoff;  // rel_bin's offset
};
template <typename T, int Q>
__device__ __forceinline__ EncK<T> enc_consts(const FieldParams<T> &p) {
  return EncK<T>{(T)FT<T>::kExpMask, p.bound, p.low, kSent, class_mask<Q>(), 0x81000000u};
}
// v, held in a vector register from here on (an empty asm the compiler
// cannot see through, so it keeps the register instead of re-creating v).
template <typename V> __device__ __forceinline__ V pin_v(V v) {
  asm volatile("" : "+v"(v));
  return v;
}
template <typename T, int Q>
__device__ __forceinline__ EncK<T> enc_consts_pinned(const FieldParams<T> &p) {
  EncK<T> k = enc_consts<T, Q>(p);
  k.emax = pin_v(k.emax);
  k.bound = pin_v(k.bound);
  k.low = pin_v(k.low);
  k.sent = pin_v(k.sent);
  k.cls = pin_v(k.cls);
  asm volatile("" : "+s"(k.lgoff));  // a scalar operand of the shift-and-add
  return k;
}

// One value -> its int32 code, or kSent if it must be stored losslessly.
// Evaluates every step for every lane (no data-dependent branches) and only
// converts the bin to int where it is in range.  k: enc_consts (or their
// pinned copies).
template <typename T, int Q>
__device__ __forceinline__ int32_t encode(T x, const FieldParams<T> &p, const EncK<T> &k) {
  using F = FT<T>;
  using U = typename F::U;
  const U u = to_bits(x);
  bool ok = class_test(x, k.cls);
  if (Q == kNOA) ok = ok && !p.lossless_all;

  if constexpr (is_rel_q<Q>()) {
    // |x| (an absolute-value source modifier where it is used, not an
    // instruction of its own)
    const T a = abs_t(x);
    // (the approximate log2 reads only the exponent and fraction fields)
    const T q = Q == kREL_LIBM ? rint_t(lib_log2(a) * p.inv) : rel_bin(x, p.inv, k.lgoff);
    // section 3.3: both range tests, on the float, before any conversion
    ok = ok && (q > (T)-kMaxBin) && (q < (T)kMaxBin);
    // qb is integral and inside (-2^30, 2^30), so (T)(int)qb == qb exactly
    const T qb = ok ? q : (T)0;
    const int32_t b = (int32_t)qb;
    const T rec = Q == kREL_LIBM ? lib_exp2(qb * p.step) : pow2approx_dev(qb * p.step, k.emax);
    // section 3.1 double-check against the side of the section 2.1.2 range
    // that rec lies on: (rec - a) < eh a above a, (a - rec) < el a below;
    // |rec - a| equals (a - rec) when rec < a (round-to-nearest is
    // symmetric under negation), so one subtraction serves both sides
    const bool up = rec >= a;
    const T diff = abs_t(rec - a);
    ok = ok & (diff < (up ? k.bound : k.low) * a);  // bitwise: no branch per value
    // (b << 1) | sign bit of x: one funnel shift of the pair (b, high word
    // of x)
    const uint32_t hi = (uint32_t)(u >> (sizeof(T) * 8 - 32));
    const uint32_t code = __builtin_amdgcn_alignbit((uint32_t)b, hi, 31);
    return ok ? (int32_t)code : k.sent;
  } else {
    const T q = rint_t(x * p.inv);
    ok = ok && (q > (T)-kMaxBin) && (q < (T)kMaxBin);
    const T qb = ok ? q : (T)0;  // integral, in range: (T)(int)qb == qb
    const int32_t b = (int32_t)qb;
    const T rec = qb * p.step;
    if constexpr (Q != kABS_UNCHECKED) ok = ok && (abs_t(x - rec) <= p.bound);
    return ok ? b : k.sent;
  }
}
template <typename T, int Q> __device__ __forceinline__ int32_t encode(T x, const FieldParams<T> &p) {
  return encode<T, Q>(x, p, enc_consts<T, Q>(p));
}

// One non-sentinel code -> its value (the decoder side of encode; LIBM: the
// library-exp2 ablation).
template <typename T, bool LIBM = false>
__device__ __forceinline__ T decode(int32_t c, T step, bool rel) {
  using F = FT<T>;
  using U = typename F::U;
  if (rel) {
    const U sgn = (U)(c & 1);
    const int32_t b = c >> 1;  // arithmetic shift: c = 2b + sign
    const T a = LIBM ? lib_exp2((T)b * step) : pow2approx_dev((T)b * step);
    return from_bits((U)(to_bits(a) | (sgn << (sizeof(T) * 8 - 1))));
  }
  return (T)c * step;
}

// Stream layout.
LCQ_HD uint64_t align16(uint64_t v) { return (v + 15u) & ~(uint64_t)15u; }
LCQ_HD uint64_t n_chunks(uint64_t n) { return (n + kChunk - 1) / kChunk; }
LCQ_HD uint64_t chunk_table_offset(uint64_t n) { return align16(64 + 4 * n); }
LCQ_HD uint64_t outlier_offset(uint64_t n) {
  return align16(chunk_table_offset(n) + 8 * n_chunks(n));
}

}  // namespace lcq
