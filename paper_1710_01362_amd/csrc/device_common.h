// Complex double helpers shared by the device translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "ttns_internal.h"

namespace ttns {

__device__ __forceinline__ cd cz() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ cd cadd(cd a, cd b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cd csub(cd a, cd b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cd cscale(cd a, double s) { return make_double2(a.x * s, a.y * s); }
// c + a * b
__device__ __forceinline__ cd cfma(cd a, cd b, cd c) {
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
// c + conj(a) * b
__device__ __forceinline__ cd cjfma(cd a, cd b, cd c) {
  return make_double2(fma(a.x, b.x, fma(a.y, b.y, c.x)), fma(a.x, b.y, fma(-a.y, b.x, c.y)));
}
__device__ __forceinline__ double cabs2(cd a) { return a.x * a.x + a.y * a.y; }

}  // namespace ttns
