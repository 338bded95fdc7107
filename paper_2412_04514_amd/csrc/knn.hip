// k-nearest-neighbour search over the grid (paper, Summary: after the grid
// sort "a k-nearest neighbors search is performed").
//
// One query per lane, queries in grid-sorted order so that neighbouring lanes
// scan overlapping grid cells (L1/L2 reuse).  Each lane walks Chebyshev rings
// r = 0, 1, 2, ... of grid cells around its own cell; a full x-row of a ring is
// one contiguous range of sorted points.  The k best candidates live in VGPRs
// as an ascending list updated by an unrolled compare-swap pass (no dynamic
// register indexing), entered only when a candidate beats the current k-th.
// The search stops after ring r once the list is full and its k-th distance
// is below rho_r, the distance from the query to the nearest face of the
// scanned block (faces on the grid boundary are at infinity).
#include "internal.h"
#include "device_common.h"

#include <cfloat>

namespace votess {
namespace {

// Ascending (d^2, sorted index) list.  FP32 distances pack into one u64 key:
// the bits of a non-negative float order like the float.
template <int K>
struct ListF32 {
  unsigned long long key[K];
  __device__ void init() {
#pragma unroll
    for (int i = 0; i < K; ++i) key[i] = ~0ull;
  }
  __device__ bool better(float d2, int idx) const {
    const unsigned long long x = ((unsigned long long)__float_as_uint(d2) << 32) | (unsigned)idx;
    return x < key[K - 1];
  }
  __device__ void insert(float d2, int idx) {
    unsigned long long x = ((unsigned long long)__float_as_uint(d2) << 32) | (unsigned)idx;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const unsigned long long a = key[i];
      const bool lt = x < a;
      key[i] = lt ? x : a;
      x = lt ? a : x;
    }
  }
  __device__ double worst() const { return (double)__uint_as_float((unsigned)(key[K - 1] >> 32)); }
  __device__ bool full() const { return key[K - 1] != ~0ull; }
  __device__ int idx(int i) const { return key[i] == ~0ull ? -1 : (int)(unsigned)(key[i] & 0xffffffffu); }
  __device__ double d2(int i) const { return (double)__uint_as_float((unsigned)(key[i] >> 32)); }
};

template <int K>
struct ListF64 {
  double d[K];
  int id[K];
  __device__ void init() {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      d[i] = DBL_MAX;
      id[i] = 0x7fffffff;
    }
  }
  __device__ bool better(double x, int idx) const {
    return x < d[K - 1] || (x == d[K - 1] && idx < id[K - 1]);
  }
  __device__ void insert(double x, int idx) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const double a = d[i];
      const int b = id[i];
      const bool lt = x < a || (x == a && idx < b);
      d[i] = lt ? x : a;
      id[i] = lt ? idx : b;
      x = lt ? a : x;
      idx = lt ? b : idx;
    }
  }
  __device__ double worst() const { return d[K - 1]; }
  __device__ bool full() const { return id[K - 1] != 0x7fffffff; }
  __device__ int idx(int i) const { return id[i] == 0x7fffffff ? -1 : id[i]; }
  __device__ double d2(int i) const { return d[i]; }
};

template <typename T, typename D, int K>
__global__ __launch_bounds__(64) void k_knn(const typename Rec<T>::type* __restrict__ rec, int n, GridDev G,
                                            const int* __restrict__ cell_start, const int* __restrict__ queries,
                                            int nq, int* __restrict__ knn, unsigned* __restrict__ err) {
  using List = typename std::conditional<std::is_same<D, float>::value, ListF32<K>, ListF64<K>>::type;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const int s = queries ? queries[q] : q;
  const auto pr = rec[s];
  const D px = (D)pr.x, py = (D)pr.y, pz = (D)pr.z;
  const int cx = axis_cell((double)pr.x, G.lo0, G.ih0, G.g0);
  const int cy = axis_cell((double)pr.y, G.lo1, G.ih1, G.g1);
  const int cz = axis_cell((double)pr.z, G.lo2, G.ih2, G.g2);
  const double ext = fmax(G.hi0 - G.lo0, fmax(G.hi1 - G.lo1, G.hi2 - G.lo2));
  const double margin = 1e-9 * ext;  // covers floor() rounding at grid-cell borders
  // a float d^2 may be low by a few ulp: stop only below rho^2 (1 - 1e-6)
  const double stop_scale = std::is_same<D, float>::value ? (1.0 - 1e-6) : 1.0;

  List L;
  L.init();
  auto scan = [&](int b, int e) {
    for (int j = b; j < e; ++j) {
      if (j == s) continue;
      const auto qr = rec[j];
      const D dx = (D)qr.x - px, dy = (D)qr.y - py, dz = (D)qr.z - pz;
      const D d2 = dist2_nc(dx, dy, dz);
      if (L.better(d2, j)) L.insert(d2, j);
    }
  };
  for (int r = 0;; ++r) {
    const int z0 = max(cz - r, 0), z1 = min(cz + r, G.g2 - 1);
    const int y0 = max(cy - r, 0), y1 = min(cy + r, G.g1 - 1);
    const int x0 = max(cx - r, 0), x1 = min(cx + r, G.g0 - 1);
    for (int z = z0; z <= z1; ++z) {
      const bool zface = (z == cz - r) || (z == cz + r);
      for (int y = y0; y <= y1; ++y) {
        const int row = G.g0 * (y + G.g1 * z);
        if (zface || y == cy - r || y == cy + r) {
          scan(cell_start[row + x0], cell_start[row + x1 + 1]);
        } else {
          if (cx - r >= 0) scan(cell_start[row + cx - r], cell_start[row + cx - r + 1]);
          if (r > 0 && cx + r < G.g0) scan(cell_start[row + cx + r], cell_start[row + cx + r + 1]);
        }
      }
    }
    const bool covers = cx - r <= 0 && cy - r <= 0 && cz - r <= 0 && cx + r >= G.g0 - 1 && cy + r >= G.g1 - 1 &&
                        cz + r >= G.g2 - 1;
    if (covers) break;
    if (L.full()) {
      double rho = 1e300;
      const double p0 = (double)pr.x, p1 = (double)pr.y, p2 = (double)pr.z;
      if (cx - r > 0) rho = fmin(rho, p0 - (G.lo0 + (cx - r) * G.h0));
      if (cx + r + 1 < G.g0) rho = fmin(rho, (G.lo0 + (cx + r + 1) * G.h0) - p0);
      if (cy - r > 0) rho = fmin(rho, p1 - (G.lo1 + (cy - r) * G.h1));
      if (cy + r + 1 < G.g1) rho = fmin(rho, (G.lo1 + (cy + r + 1) * G.h1) - p1);
      if (cz - r > 0) rho = fmin(rho, p2 - (G.lo2 + (cz - r) * G.h2));
      if (cz + r + 1 < G.g2) rho = fmin(rho, (G.lo2 + (cz + r + 1) * G.h2) - p2);
      rho -= margin;
      if (rho > 0.0 && L.worst() < rho * rho * stop_scale) break;
    }
  }
  int* out = knn + (size_t)q * K;
#pragma unroll
  for (int i = 0; i < K; ++i) out[i] = L.idx(i);
  if (L.idx(0) >= 0 && L.d2(0) == 0.0) atomicOr(err, ERR_DUPLICATE);
}

template <typename T, typename D>
votess_status dispatch_k(int k, const void* sorted, int n, const GridDev& G, const int32_t* cs, const int32_t* qs,
                         int nq, int32_t* knn, unsigned* err, hipStream_t st) {
  using R4 = typename Rec<T>::type;
  const R4* rec = (const R4*)sorted;
  const unsigned blocks = (unsigned)((nq + 63) / 64);
#define VT_KNN_CASE(KK)                                                           \
  case KK:                                                                        \
    k_knn<T, D, KK><<<blocks, 64, 0, st>>>(rec, n, G, cs, qs, nq, knn, err);     \
    break;
  switch (k) {
    VT_KNN_CASE(8)
    VT_KNN_CASE(12)
    VT_KNN_CASE(16)
    VT_KNN_CASE(24)
    VT_KNN_CASE(32)
    VT_KNN_CASE(48)
    VT_KNN_CASE(64)
    default:
      return fail(VOTESS_EINVAL, "knn: k=%d has no kernel (k must be one of 8,12,16,24,32,48,64)", k);
  }
#undef VT_KNN_CASE
  VT_HIP(hipGetLastError());
  return VOTESS_OK;
}

}  // namespace

votess_status launch_knn(votess_ctx* ctx, const void* sorted, votess_dtype dt, int n, const GridDev& G,
                         const int32_t* cell_start, const int32_t* queries, int nq, int k, votess_dtype dist,
                         int32_t* knn, hipStream_t st) {
  if (nq == 0) return VOTESS_OK;
  if (dt == VOTESS_F64 && dist == VOTESS_F32)
    return fail(VOTESS_EINVAL, "knn: F32 distances need F32 positions");
  if (dt == VOTESS_F32) {
    if (dist == VOTESS_F32) return dispatch_k<float, float>(k, sorted, n, G, cell_start, queries, nq, knn, ctx->d_err, st);
    return dispatch_k<float, double>(k, sorted, n, G, cell_start, queries, nq, knn, ctx->d_err, st);
  }
  return dispatch_k<double, double>(k, sorted, n, G, cell_start, queries, nq, knn, ctx->d_err, st);
}

}  // namespace votess
