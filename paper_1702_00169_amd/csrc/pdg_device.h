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


}  // namespace
}  // namespace pdg
