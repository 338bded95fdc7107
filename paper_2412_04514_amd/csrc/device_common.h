// Device helpers shared by the HIP kernels: grid-cell arithmetic and the
// sorted-record layout (x, y, z, original index as bits) of votess_grid_sort.
#pragma once
#include <hip/hip_runtime.h>
#include "internal.h"

namespace votess {
namespace {

__device__ __forceinline__ int axis_cell(double x, double lo, double ih, int g) {
  double c = floor((x - lo) * ih);
  c = fmin(fmax(c, 0.0), (double)(g - 1));  // NaN -> 0
  return (int)c;
}

__device__ __forceinline__ int cell_of(double x, double y, double z, const GridDev& G) {
  return axis_cell(x, G.lo0, G.ih0, G.g0) + G.g0 * (axis_cell(y, G.lo1, G.ih1, G.g1) + G.g1 * axis_cell(z, G.lo2, G.ih2, G.g2));
}

// Squared distance with no fused multiply-add, so every kernel that ranks
// points by it (k-NN lists, the clip's list and stream phases) computes the
// same value.
__device__ __forceinline__ float dist2_nc(float x, float y, float z) {
  return __fadd_rn(__fadd_rn(__fmul_rn(x, x), __fmul_rn(y, y)), __fmul_rn(z, z));
}
__device__ __forceinline__ double dist2_nc(double x, double y, double z) {
  return __dadd_rn(__dadd_rn(__dmul_rn(x, x), __dmul_rn(y, y)), __dmul_rn(z, z));
}

template <typename T> struct Rec;
template <> struct Rec<float> {
  using type = float4;
  __device__ static float4 make(float x, float y, float z, int id) { return make_float4(x, y, z, __int_as_float(id)); }
  __device__ static int id(const float4& r) { return __float_as_int(r.w); }
};
template <> struct Rec<double> {
  using type = double4;
  __device__ static double4 make(double x, double y, double z, int id) {
    return make_double4(x, y, z, __longlong_as_double((long long)id));
  }
  __device__ static int id(const double4& r) { return (int)__double_as_longlong(r.w); }
};

}  // namespace
}  // namespace votess
