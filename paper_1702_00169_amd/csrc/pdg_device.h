// Device helpers shared by the kernel translation units: state access and
// the precision policies.
#pragma once

#include <float.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "pdg_internal.h"

#ifndef PDG_NONTEMPORAL
#define PDG_NONTEMPORAL 0
#endif

namespace pdg {
namespace {

// State traffic: every value is read once and written once per kernel, so
// the loads and stores may carry the streaming (non-temporal) hint.
template <class T>
__device__ __forceinline__ T ld_state(const T *p) {
#if PDG_NONTEMPORAL
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}
template <class T>
__device__ __forceinline__ void st_state(T *p, T v) {
#if PDG_NONTEMPORAL
  __builtin_nontemporal_store(v, p);
#else
  *p = v;
#endif
}

template <int PREC>
struct Pol;
template <>
struct Pol<kF64> {
  using St = double;  // state
  using Rt = double;  // recurrence / arithmetic
};
template <>
struct Pol<kF32> {
  using St = float;
  using Rt = float;
};
template <>
struct Pol<kRefine> {
  using St = double;
  using Rt = double;
};
template <>
struct Pol<kP48> {
  using St = double;  // values as the kernels see them (stored packed, State<kP48>)
  using Rt = double;
};

// Element access to the state: a plain array of Pol<PREC>::St.
template <int PREC>
struct State {
  using St = typename Pol<PREC>::St;
  using Rt = typename Pol<PREC>::Rt;
  using Raw = St;  // a value as loaded, before conversion (see State<kP48>)
  St *p;
  static State make(StateBuf b) { return State{static_cast<St *>(b.p)}; }
  __device__ __forceinline__ Raw ldr(int64_t i) const { return ld_state(p + i); }
  __device__ __forceinline__ Rt dec(Raw r) const { return (Rt)r; }
  __device__ __forceinline__ Rt ld(int64_t i) const { return (Rt)ld_state(p + i); }
  __device__ __forceinline__ void st(int64_t i, Rt v) const { st_state(p + i, (St)v); }
  // The state from element off on (off uniform across the workgroup), indexed
  // by a 32-bit offset: the base stays in scalar registers.
  __device__ __forceinline__ State at(int64_t off) const { return State{p + off}; }
  __device__ __forceinline__ Raw ldr32(uint32_t i) const { return ld_state(p + i); }
  __device__ __forceinline__ void st32(uint32_t i, Rt v) const { st_state(p + i, (St)v); }
};

// 48-bit state: value x is kept as h = x rounded to binary32 (nearest) and
// l = round((x - h) / u) in int16, with u = 2^(e - 39) for h in the binade
// [2^e, 2^(e+1)) (e = -126 for zero and subnormal h).  |x - h| <= 2^(e - 24),
// so |l| <= 2^15; l is clamped to +-32767, which only a residual within u / 2
// of half a binary32 ulp reaches.  The stored value h + l u (exact in
// binary64) is within u / 2 of x, or u after a clamp: a relative rounding of
// at most 2^-39 (a 40-bit significand, against 53 bits for binary64).
// Non-finite h decodes to itself.
__device__ __forceinline__ double p48_unit(float h, int sign_of_exp) {
  const uint32_t eb = (__float_as_uint(h) >> 23) & 0xffu;
  const int e = eb ? (int)eb - 127 : -126;
  // 2^(+-(e - 39)) built from its binary64 exponent field
  const int ex = sign_of_exp > 0 ? e - 39 : 39 - e;
  return __hiloint2double((ex + 1023) << 20, 0);
}
__device__ __forceinline__ double p48_decode(float h, int16_t l) {
  return (double)h + (double)l * p48_unit(h, 1);
}
__device__ __forceinline__ void p48_encode(double x, float &h, int16_t &l) {
  h = (float)x;
  const double r = x - (double)h;  // exact (h is within a factor 2 of x)
  double q = rint(r * p48_unit(h, -1));
  q = fmin(fmax(q, -32767.0), 32767.0);
  l = (int16_t)(int)q;
}

template <>
struct State<kP48> {
  using Rt = double;
  // Loading the two planes and decoding are separate steps, so that a kernel
  // can issue all of its loads before it decodes any of them.
  struct Raw {
    float h;
    int16_t l;
  };
  float *hi;
  int16_t *lo;
  static State make(StateBuf b) {
    return State{static_cast<float *>(b.p), reinterpret_cast<int16_t *>(static_cast<char *>(b.p) + 4 * b.n)};
  }
  __device__ __forceinline__ Raw ldr(int64_t i) const { return Raw{ld_state(hi + i), ld_state(lo + i)}; }
  __device__ __forceinline__ double dec(Raw r) const { return p48_decode(r.h, r.l); }
  __device__ __forceinline__ double ld(int64_t i) const { return p48_decode(ld_state(hi + i), ld_state(lo + i)); }
  __device__ __forceinline__ void st(int64_t i, double v) const {
    float h;
    int16_t l;
    p48_encode(v, h, l);
    st_state(hi + i, h);
    st_state(lo + i, l);
  }
  __device__ __forceinline__ State at(int64_t off) const { return State{hi + off, lo + off}; }
  __device__ __forceinline__ Raw ldr32(uint32_t i) const { return Raw{ld_state(hi + i), ld_state(lo + i)}; }
  __device__ __forceinline__ void st32(uint32_t i, double v) const {
    float h;
    int16_t l;
    p48_encode(v, h, l);
    st_state(hi + i, h);
    st_state(lo + i, l);
  }
};


}  // namespace
}  // namespace pdg
