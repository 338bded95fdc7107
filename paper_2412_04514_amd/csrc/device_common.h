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

// Squared distance with every product and sum rounded on its own, so every
// kernel that ranks points by it (k-NN lists, the clip's list and stream
// phases) computes the same bits: the clip tells a list member from a later
// candidate of equal distance by comparing these values exactly.  Contraction
// is switched off here rather than relying on __fmul_rn / __fadd_rn, which
// HIP defines as the plain operators: those fuse into FMAs, differently in
// each kernel.
__device__ __forceinline__ float dist2_nc(float x, float y, float z) {
#pragma clang fp contract(off)
  const float xx = x * x, yy = y * y, zz = z * z;
  return (xx + yy) + zz;
}
__device__ __forceinline__ double dist2_nc(double x, double y, double z) {
#pragma clang fp contract(off)
  const double xx = x * x, yy = y * y, zz = z * z;
  return (xx + yy) + zz;
}

// Dense grid cells (more than kSubMin points) carry a sub-grid over a box
// [lo, lo + e] that holds the central 90% of their points along each axis:
// m0 x m1 x m2 sub-cells with m0 m1 m2 <= count / 2, near-cubic; points
// inside such a cell are ordered by sub-cell id s0 + m0 (s1 + m1 s2),
// s_a = clamp(floor((x_a - lo_a) ih_a), 0, m_a - 1), ih_a = m_a / e_a.
// Its record in sub_start (16-byte aligned): m0, m1, m2, 0, lo[3] and ih[3]
// as doubles, then the m0 m1 m2 + 1 sub-cell starts relative to the cell's
// first point.
constexpr int kSubMin = 16;
#ifndef VOTESS_SUB_PTS
#define VOTESS_SUB_PTS 2
#endif
constexpr int kSubPts = VOTESS_SUB_PTS;  // points per sub-cell the sub-grid aims at (>= 2)
constexpr int kSubHead = 16;  // int32 words before the starts
constexpr int kSubBins = 1024;  // histogram bins per axis for the sub-grid box
__device__ __forceinline__ int sub_axis(double x, double lo, double ih, int m) {
  double s = floor((x - lo) * ih);
  s = fmin(fmax(s, 0.0), (double)(m - 1));  // NaN -> 0
  return (int)s;
}
struct SubCell {
  int m0, m1, m2;
  double lo0, lo1, lo2, ih0, ih1, ih2;
  const int* start;  // m0 m1 m2 + 1 starts
};
__device__ __forceinline__ SubCell sub_cell(const int* rec) {
  SubCell c;
  const int4 m = *(const int4*)rec;
  c.m0 = m.x;
  c.m1 = m.y;
  c.m2 = m.z;
  const double2 a = *(const double2*)(rec + 4), b = *(const double2*)(rec + 8), d = *(const double2*)(rec + 12);
  c.lo0 = a.x;
  c.lo1 = a.y;
  c.lo2 = b.x;
  c.ih0 = b.y;
  c.ih1 = d.x;
  c.ih2 = d.y;
  c.start = rec + kSubHead;
  return c;
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
