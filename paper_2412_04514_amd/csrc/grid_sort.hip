// Grid sort of the generators (paper, Summary section: the points are first
// binned into a uniform grid) as a counting sort:
//   a1  cell id of every point + atomic histogram (the atomic's return value is
//       the point's provisional rank inside its cell);
//   a2  exclusive scan of the histogram -> cell_start;
//   a3  scatter of (x, y, z, id) records to cell_start + rank, then a per-cell
//       reorder to ascending original index so the result is deterministic.
// Also hosts the generic device exclusive scan used by CSR assembly.
#include "internal.h"
#include "device_common.h"

namespace votess {

GridDev to_dev(const votess_grid& g) {
  GridDev d;
  d.g0 = g.g[0]; d.g1 = g.g[1]; d.g2 = g.g[2];
  d.lo0 = g.lo[0]; d.lo1 = g.lo[1]; d.lo2 = g.lo[2];
  d.hi0 = g.hi[0]; d.hi1 = g.hi[1]; d.hi2 = g.hi[2];
  d.ih0 = g.inv_h[0]; d.ih1 = g.inv_h[1]; d.ih2 = g.inv_h[2];
  d.h0 = (g.hi[0] - g.lo[0]) / g.g[0];
  d.h1 = (g.hi[1] - g.lo[1]) / g.g[1];
  d.h2 = (g.hi[2] - g.lo[2]) / g.g[2];
  return d;
}

namespace {

constexpr int kLdsSortMax = 4096; // larger cells sort their keys in global memory
constexpr int kDenseBlocks = 2048; // blocks of the dense-cell pass (grid-stride over the dense cells)

template <typename T>
__global__ void k_cell_rank(const T* __restrict__ pts, int n, GridDev G, int* __restrict__ count,
                            int2* __restrict__ cr, unsigned* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = pts[3 * (size_t)i], y = pts[3 * (size_t)i + 1], z = pts[3 * (size_t)i + 2];
  const bool inside = x >= G.lo0 && x <= G.hi0 && y >= G.lo1 && y <= G.hi1 && z >= G.lo2 && z <= G.hi2;
  if (!inside) atomicOr(err, ERR_OUT_OF_BOX);
  const int c = cell_of(x, y, z, G);
  const int r = atomicAdd(&count[c], 1);
  cr[i] = make_int2(c, r);
}

template <typename T>
__global__ void k_scatter(const T* __restrict__ pts, int n, const int2* __restrict__ cr,
                          const int* __restrict__ cell_start, typename Rec<T>::type* __restrict__ tmp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int2 c = cr[i];
  tmp[cell_start[c.x] + c.y] = Rec<T>::make(pts[3 * (size_t)i], pts[3 * (size_t)i + 1], pts[3 * (size_t)i + 2], i);
}

// One thread per grid cell: rank-by-count reorder of small cells; large cells
// are queued for k_order_big.
template <typename T>
__global__ void k_order_small(const typename Rec<T>::type* __restrict__ tmp, const int* __restrict__ cell_start,
                              int ncells, typename Rec<T>::type* __restrict__ out, int* __restrict__ perm,
                              int* __restrict__ big, int* __restrict__ nbig, int2* __restrict__ subinfo) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  const int b = cell_start[c], e = cell_start[c + 1];
  const int len = e - b;
  if (subinfo) subinfo[c] = make_int2(-1, 0);
  if (len == 0) return;
  if (len > kSubMin) {  // dense cell: sub-grid order, one block per cell
    big[atomicAdd(nbig, 1)] = c;
    return;
  }
  for (int t = b; t < e; ++t) {
    const auto r = tmp[t];
    const int id = Rec<T>::id(r);
    int rank = 0;
    for (int u = b; u < e; ++u) rank += Rec<T>::id(tmp[u]) < id;
    out[b + rank] = r;
    perm[b + rank] = id;
  }
}

// Bitonic sort (all comparators ascending: the first stage of each merge
// compares mirrored pairs), over len keys; virtual padding to a power of two
// is +inf, so comparisons with an index >= len are skipped.
// Keys are unique, so the payload (source position) follows its key.
__device__ __forceinline__ void cswap(unsigned long long* key, unsigned* val, int t, int p) {
  const unsigned long long a = key[t], b = key[p];
  if (b < a) {
    key[t] = b;
    key[p] = a;
    const unsigned va = val[t];
    val[t] = val[p];
    val[p] = va;
  }
}
__device__ void block_bitonic(unsigned long long* key, unsigned* val, int len) {
  int P = 1;
  while (P < len) P <<= 1;
  for (int k = 2; k <= P; k <<= 1) {
    for (int t = threadIdx.x; t < len; t += blockDim.x) {
      const int p = t ^ (k - 1);
      if (p > t && p < len) cswap(key, val, t, p);
    }
    __syncthreads();
    for (int j = k >> 2; j >= 1; j >>= 1) {
      for (int t = threadIdx.x; t < len; t += blockDim.x) {
        const int p = t ^ j;
        if (p > t && p < len) cswap(key, val, t, p);
      }
      __syncthreads();
    }
  }
}

// Sub-grid of a dense cell from the extents of its box: near-cubic
// sub-cells, m0 m1 m2 <= count / kSubPts (each m_a >= 1).
__device__ void plan_sub(int count, double e0, double e1, double e2, int& m0, int& m1, int& m2) {
  const double target = (double)(count / kSubPts);
  const double s = cbrt(target / (e0 * e1 * e2));
  m0 = (int)fmin(fmax(floor(e0 * s), 1.0), 4096.0);
  m1 = (int)fmin(fmax(floor(e1 * s), 1.0), 4096.0);
  m2 = (int)fmin(fmax(floor(e2 * s), 1.0), 4096.0);
  while ((long long)m0 * m1 * m2 > count / kSubPts) {
    if (m0 >= m1 && m0 >= m2) --m0;
    else if (m1 >= m2) --m1;
    else --m2;
  }
}

// One block per dense cell: order its points by (sub-cell, original index)
// and write its sub-grid record (see device_common.h).  The sub-grid spans,
// per axis, the central 90% of the cell's points (from a histogram of
// kSubBins bins over their bounding box); points beyond fall in the edge
// sub-cells.
template <typename T>
__global__ __launch_bounds__(256) void k_order_big(const typename Rec<T>::type* __restrict__ tmp,
                                                   const int* __restrict__ cell_start, const int* __restrict__ big,
                                                   const int* __restrict__ nbig, GridDev G,
                                                   typename Rec<T>::type* __restrict__ out, int* __restrict__ perm,
                                                   unsigned long long* __restrict__ gkey, unsigned* __restrict__ gval,
                                                   int2* __restrict__ subinfo, int* __restrict__ sub_start,
                                                   int* __restrict__ sub_total) {
  __shared__ unsigned long long skey[kLdsSortMax];
  __shared__ unsigned sval[kLdsSortMax];
  __shared__ double sbox[4][6];
  __shared__ int shist[3][kSubBins];
  __shared__ int soff, sm[3];
  __shared__ double slo[3], sih[3];
  const int nb = *nbig;
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int q = blockIdx.x; q < nb; q += gridDim.x) {
    const int c = big[q];
    const int b = cell_start[c], len = cell_start[c + 1] - b;
    const bool lds = len <= kLdsSortMax;
    unsigned long long* key = lds ? skey : gkey + b;
    unsigned* val = lds ? sval : gval + b;
    if (subinfo) {
      // bounding box of the cell's points
      double mn0 = 1e300, mn1 = 1e300, mn2 = 1e300, mx0 = -1e300, mx1 = -1e300, mx2 = -1e300;
      for (int t = threadIdx.x; t < len; t += blockDim.x) {
        const auto r = tmp[b + t];
        mn0 = fmin(mn0, (double)r.x); mx0 = fmax(mx0, (double)r.x);
        mn1 = fmin(mn1, (double)r.y); mx1 = fmax(mx1, (double)r.y);
        mn2 = fmin(mn2, (double)r.z); mx2 = fmax(mx2, (double)r.z);
      }
      for (int o = 32; o >= 1; o >>= 1) {
        mn0 = fmin(mn0, __shfl_xor(mn0, o, 64)); mx0 = fmax(mx0, __shfl_xor(mx0, o, 64));
        mn1 = fmin(mn1, __shfl_xor(mn1, o, 64)); mx1 = fmax(mx1, __shfl_xor(mx1, o, 64));
        mn2 = fmin(mn2, __shfl_xor(mn2, o, 64)); mx2 = fmax(mx2, __shfl_xor(mx2, o, 64));
      }
      if (lane == 0) {
        sbox[wid][0] = mn0; sbox[wid][1] = mn1; sbox[wid][2] = mn2;
        sbox[wid][3] = mx0; sbox[wid][4] = mx1; sbox[wid][5] = mx2;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        const int nw = (int)(blockDim.x + 63) >> 6;
        for (int w = 1; w < nw; ++w) {
          mn0 = fmin(mn0, sbox[w][0]); mn1 = fmin(mn1, sbox[w][1]); mn2 = fmin(mn2, sbox[w][2]);
          mx0 = fmax(mx0, sbox[w][3]); mx1 = fmax(mx1, sbox[w][4]); mx2 = fmax(mx2, sbox[w][5]);
        }
        sbox[0][0] = mn0; sbox[0][1] = mn1; sbox[0][2] = mn2;
        sbox[0][3] = mx0; sbox[0][4] = mx1; sbox[0][5] = mx2;
      }
      for (int t = threadIdx.x; t < 3 * kSubBins; t += blockDim.x) (&shist[0][0])[t] = 0;
      __syncthreads();
      // per-axis histograms over the bounding box
      for (int t = threadIdx.x; t < len; t += blockDim.x) {
        const auto r = tmp[b + t];
        const double x[3] = {(double)r.x, (double)r.y, (double)r.z};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const double lo = sbox[0][a], w = sbox[0][3 + a] - lo;
          const int bin = w > 0.0 ? (int)fmin((x[a] - lo) / w * kSubBins, (double)(kSubBins - 1)) : 0;
          atomicAdd(&shist[a][bin], 1);
        }
      }
      __syncthreads();
      if (threadIdx.x < 3) {
        // the box of the central 90% of the points along this axis
        const int a = threadIdx.x;
        const double lo = sbox[0][a], w = sbox[0][3 + a] - lo;
        const int cut_lo = len / 20, cut_hi = len - len / 20;
        int acc = 0, blo = 0, bhi = kSubBins - 1;
        bool got_lo = false;
        for (int i = 0; i < kSubBins; ++i) {
          const int next = acc + shist[a][i];
          if (!got_lo && next > cut_lo) { blo = i; got_lo = true; }
          if (next >= cut_hi) { bhi = i; break; }
          acc = next;
        }
        slo[a] = lo + w * ((double)blo / kSubBins);
        sih[a] = fmax(w * ((double)(bhi + 1 - blo) / kSubBins), (a == 0 ? G.h0 : a == 1 ? G.h1 : G.h2) * 0x1p-30);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        // sih holds the extents here
        const double e0 = sih[0], e1 = sih[1], e2 = sih[2];
        int m0, m1, m2;
        plan_sub(len, e0, e1, e2, m0, m1, m2);
        sm[0] = m0; sm[1] = m1; sm[2] = m2;
        sih[0] = m0 / e0; sih[1] = m1 / e1; sih[2] = m2 / e2;
        const int words = (kSubHead + m0 * m1 * m2 + 1 + 3) & ~3;
        soff = atomicAdd(sub_total, words);
      }
      __syncthreads();
    }
    const int m0 = subinfo ? sm[0] : 1, m1 = subinfo ? sm[1] : 1, m2 = subinfo ? sm[2] : 1;
    const double lo0 = subinfo ? slo[0] : 0.0, lo1 = subinfo ? slo[1] : 0.0, lo2 = subinfo ? slo[2] : 0.0;
    const double ih0 = subinfo ? sih[0] : 0.0, ih1 = subinfo ? sih[1] : 0.0, ih2 = subinfo ? sih[2] : 0.0;
    for (int t = threadIdx.x; t < len; t += blockDim.x) {
      const auto r = tmp[b + t];
      unsigned sid = 0;
      if (subinfo)
        sid = (unsigned)(sub_axis(r.x, lo0, ih0, m0) + m0 * (sub_axis(r.y, lo1, ih1, m1) + m1 * sub_axis(r.z, lo2, ih2, m2)));
      key[t] = ((unsigned long long)sid << 32) | (unsigned)Rec<T>::id(r);
      val[t] = (unsigned)t;
    }
    __syncthreads();
    block_bitonic(key, val, len);
    for (int t = threadIdx.x; t < len; t += blockDim.x) {
      out[b + t] = tmp[b + (int)val[t]];
      perm[b + t] = (int)(unsigned)(key[t] & 0xffffffffu);
    }
    if (subinfo) {
      const int off = soff;
      const int ns = m0 * m1 * m2;
      int* rec = sub_start + off;
      if (threadIdx.x == 0) {
        *(int4*)rec = make_int4(m0, m1, m2, 0);
        *(double2*)(rec + 4) = make_double2(lo0, lo1);
        *(double2*)(rec + 8) = make_double2(lo2, ih0);
        *(double2*)(rec + 12) = make_double2(ih1, ih2);
        subinfo[c] = make_int2(off, ns);
      }
      for (int sc = threadIdx.x; sc <= ns; sc += blockDim.x) {
        // first position whose sub-cell id is >= sc
        int lo = 0, hi = len;
        const unsigned long long want = (unsigned long long)sc << 32;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (key[mid] < want) lo = mid + 1;
          else hi = mid;
        }
        rec[kSubHead + sc] = lo;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- scan
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

template <typename T>
__device__ T block_excl_scan(T v, T* total) {
  __shared__ T wsum[kScanBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kScanBlock / 64; ++i) {
    if (i < w) off += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

// Exclusive scan of in[0..n_in) (virtually extended with zeros) into
// out[0..n_out); per-block totals to sums.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(kScanBlock) void k_scan_local(const Tin* __restrict__ in, int64_t n_in,
                                                           Tout* __restrict__ out, int64_t n_out,
                                                           Tout* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  Tout v[kScanItems];
  Tout s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + i;
    v[i] = idx < n_in ? (Tout)in[idx] : (Tout)0;
    s += v[i];
  }
  Tout tot;
  Tout run = block_excl_scan<Tout>(s, &tot);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + i;
    if (idx < n_out) out[idx] = run;
    run += v[i];
  }
  if (threadIdx.x == 0 && sums) sums[blockIdx.x] = tot;
}

template <typename Tout>
__global__ __launch_bounds__(kScanBlock) void k_scan_add(Tout* __restrict__ out, int64_t n_out,
                                                         const Tout* __restrict__ offs) {
  const Tout o = offs[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  for (int i = threadIdx.x; i < kScanTile; i += kScanBlock) {
    const int64_t idx = base + i;
    if (idx < n_out) out[idx] += o;
  }
}

// Exclusive scan of a[0..cnt) in place by one 256-thread block (chunks of
// 2048 with a running carry).
__device__ void block_scan_inplace(int* a, int cnt) {
  int carry = 0;
  for (int base = 0; base < cnt; base += kScanTile) {
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      const int idx = base + (int)threadIdx.x * kScanItems + i;
      v[i] = idx < cnt ? a[idx] : 0;
      s += v[i];
    }
    int tot;
    int run = block_excl_scan<int>(s, &tot) + carry;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      const int idx = base + (int)threadIdx.x * kScanItems + i;
      if (idx < cnt) a[idx] = run;
      run += v[i];
    }
    carry += tot;
  }
  __syncthreads();
}

// Counts of a dense cell's sub-cells live in LDS when there are at most this
// many (the common case), else in the global scratch at the cell's range.
constexpr int kCntLds = 4096;
// A sub-cell holding more points than this (crowded: the points sit far
// tighter than the central 90% box the sub-grid spans) has its cell ordered
// by the bitonic network instead of the per-sub-cell rank count below.
constexpr int kCrowd = 256;

// One block per dense cell (grid-stride over the dense-cell list): plan the
// cell's sub-grid (as k_order_big), then a counting sort by sub-cell -- LDS
// atomic counts give each point its sub-cell and a provisional slot, a block
// scan turns counts into the sub-cell starts (written to the record as they
// are) -- and within a sub-cell each point's final rank is the number of its
// points with a smaller original index.  Per-point scratch lives in global
// memory at the cell's own range [b, b + len).
template <typename T>
__global__ __launch_bounds__(256) void k_order_dense(const typename Rec<T>::type* __restrict__ tmp,
                                                     const int* __restrict__ cell_start, const int* __restrict__ big,
                                                     const int* __restrict__ nbig, GridDev G,
                                                     typename Rec<T>::type* __restrict__ out, int* __restrict__ perm,
                                                     unsigned* __restrict__ g_sid, unsigned* __restrict__ g_rank,
                                                     unsigned* __restrict__ g_slot, int* __restrict__ g_cnt,
                                                     unsigned long long* __restrict__ gkey, unsigned* __restrict__ gval,
                                                     int2* __restrict__ subinfo, int* __restrict__ sub_start,
                                                     int* __restrict__ sub_total) {
  __shared__ int s_cnt[kCntLds];
  __shared__ double sbox[4][6];
  __shared__ int shist[3][kSubBins];
  __shared__ int soff, sm[3], s_crowd, s_bin[3][2];
  __shared__ double slo[3], sih[3];
  const int nb = *nbig;
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int q = blockIdx.x; q < nb; q += gridDim.x) {
    const int c = big[q];
    const int b = cell_start[c], len = cell_start[c + 1] - b;
    // ---- sub-grid plan: bounding box, per-axis histograms, central 90%
    double mn0 = 1e300, mn1 = 1e300, mn2 = 1e300, mx0 = -1e300, mx1 = -1e300, mx2 = -1e300;
    for (int t = threadIdx.x; t < len; t += blockDim.x) {
      const auto r = tmp[b + t];
      mn0 = fmin(mn0, (double)r.x); mx0 = fmax(mx0, (double)r.x);
      mn1 = fmin(mn1, (double)r.y); mx1 = fmax(mx1, (double)r.y);
      mn2 = fmin(mn2, (double)r.z); mx2 = fmax(mx2, (double)r.z);
    }
    for (int o = 32; o >= 1; o >>= 1) {
      mn0 = fmin(mn0, __shfl_xor(mn0, o, 64)); mx0 = fmax(mx0, __shfl_xor(mx0, o, 64));
      mn1 = fmin(mn1, __shfl_xor(mn1, o, 64)); mx1 = fmax(mx1, __shfl_xor(mx1, o, 64));
      mn2 = fmin(mn2, __shfl_xor(mn2, o, 64)); mx2 = fmax(mx2, __shfl_xor(mx2, o, 64));
    }
    if (lane == 0) {
      sbox[wid][0] = mn0; sbox[wid][1] = mn1; sbox[wid][2] = mn2;
      sbox[wid][3] = mx0; sbox[wid][4] = mx1; sbox[wid][5] = mx2;
    }
    for (int t = threadIdx.x; t < 3 * kSubBins; t += blockDim.x) (&shist[0][0])[t] = 0;
    if (threadIdx.x == 0) s_crowd = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
      const int nw = (int)(blockDim.x + 63) >> 6;
      for (int w = 1; w < nw; ++w) {
        mn0 = fmin(mn0, sbox[w][0]); mn1 = fmin(mn1, sbox[w][1]); mn2 = fmin(mn2, sbox[w][2]);
        mx0 = fmax(mx0, sbox[w][3]); mx1 = fmax(mx1, sbox[w][4]); mx2 = fmax(mx2, sbox[w][5]);
      }
      sbox[0][0] = mn0; sbox[0][1] = mn1; sbox[0][2] = mn2;
      sbox[0][3] = mx0; sbox[0][4] = mx1; sbox[0][5] = mx2;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < len; t += blockDim.x) {
      const auto r = tmp[b + t];
      const double x[3] = {(double)r.x, (double)r.y, (double)r.z};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double lo = sbox[0][a], w = sbox[0][3 + a] - lo;
        const int bin = w > 0.0 ? (int)fmin((x[a] - lo) / w * kSubBins, (double)(kSubBins - 1)) : 0;
        atomicAdd(&shist[a][bin], 1);
      }
    }
    __syncthreads();
    {
      // the box of the central 90% per axis: the first bin whose inclusive
      // prefix count exceeds len/20, and the first that reaches len - len/20,
      // found from a block-wide prefix scan (four bins per thread)
      static_assert(kSubBins == 4 * 256, "four histogram bins per thread");
      const int cut_lo = len / 20, cut_hi = len - len / 20;
      for (int a = 0; a < 3; ++a) {
        int v[4], sum = 0;
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) {
          v[k2] = shist[a][threadIdx.x * 4 + k2];
          sum += v[k2];
        }
        int tot;
        int run = block_excl_scan<int>(sum, &tot);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) {
          const int prev = run;
          run += v[k2];
          if (prev <= cut_lo && run > cut_lo) s_bin[a][0] = (int)threadIdx.x * 4 + k2;
          if (prev < cut_hi && run >= cut_hi) s_bin[a][1] = (int)threadIdx.x * 4 + k2;
        }
      }
      __syncthreads();
      if (threadIdx.x < 3) {
        const int a = threadIdx.x;
        const double lo = sbox[0][a], w = sbox[0][3 + a] - lo;
        const int blo = s_bin[a][0], bhi = s_bin[a][1];
        slo[a] = lo + w * ((double)blo / kSubBins);
        sih[a] = fmax(w * ((double)(bhi + 1 - blo) / kSubBins), (a == 0 ? G.h0 : a == 1 ? G.h1 : G.h2) * 0x1p-30);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const double e0 = sih[0], e1 = sih[1], e2 = sih[2];  // extents here
      int m0, m1, m2;
      plan_sub(len, e0, e1, e2, m0, m1, m2);
      sm[0] = m0; sm[1] = m1; sm[2] = m2;
      sih[0] = m0 / e0; sih[1] = m1 / e1; sih[2] = m2 / e2;
      const int words = (kSubHead + m0 * m1 * m2 + 1 + 3) & ~3;
      soff = atomicAdd(sub_total, words);
    }
    __syncthreads();
    const int m0 = sm[0], m1 = sm[1], m2 = sm[2];
    const int ns = m0 * m1 * m2;
    const double lo0 = slo[0], lo1 = slo[1], lo2 = slo[2], ih0 = sih[0], ih1 = sih[1], ih2 = sih[2];
    // ---- counting sort by sub-cell
    int* cnt = ns + 1 <= kCntLds ? s_cnt : g_cnt + b;  // ns + 1 <= len / 2 + 1 <= len entries
    for (int sc = threadIdx.x; sc <= ns; sc += blockDim.x) cnt[sc] = 0;
    __syncthreads();
    for (int t = threadIdx.x; t < len; t += blockDim.x) {
      const auto r = tmp[b + t];
      const unsigned sid =
          (unsigned)(sub_axis(r.x, lo0, ih0, m0) + m0 * (sub_axis(r.y, lo1, ih1, m1) + m1 * sub_axis(r.z, lo2, ih2, m2)));
      g_sid[b + t] = sid;
      g_rank[b + t] = (unsigned)atomicAdd(&cnt[sid], 1);
    }
    __syncthreads();
    int crowd = 0;
    for (int sc = threadIdx.x; sc < ns; sc += blockDim.x) crowd |= cnt[sc] > kCrowd;
    if (crowd) s_crowd = 1;
    block_scan_inplace(cnt, ns + 1);  // cnt[sc] = first point of sub-cell sc, cnt[ns] = len
    int* rec = sub_start + soff;
    if (threadIdx.x == 0) {
      *(int4*)rec = make_int4(m0, m1, m2, 0);
      *(double2*)(rec + 4) = make_double2(lo0, lo1);
      *(double2*)(rec + 8) = make_double2(lo2, ih0);
      *(double2*)(rec + 12) = make_double2(ih1, ih2);
      subinfo[c] = make_int2(soff, ns);
    }
    for (int sc = threadIdx.x; sc <= ns; sc += blockDim.x) rec[kSubHead + sc] = cnt[sc];
    if (!s_crowd) {
      // provisional slots, then each point's rank among its sub-cell's ids
      for (int t = threadIdx.x; t < len; t += blockDim.x)
        g_slot[b + cnt[g_sid[b + t]] + (int)g_rank[b + t]] = (unsigned)Rec<T>::id(tmp[b + t]);
      __syncthreads();
      for (int t = threadIdx.x; t < len; t += blockDim.x) {
        const auto r = tmp[b + t];
        const unsigned id = (unsigned)Rec<T>::id(r);
        const unsigned sid = g_sid[b + t];
        const int s0 = cnt[sid], s1 = cnt[sid + 1];
        int rank = 0;
        for (int u = s0; u < s1; ++u) rank += g_slot[b + u] < id;
        out[b + s0 + rank] = r;
        perm[b + s0 + rank] = (int)id;
      }
    } else {
      // crowded sub-cells: sort (sub-cell, original index) keys instead
      unsigned long long* key = gkey + b;
      unsigned* val = gval + b;
      for (int t = threadIdx.x; t < len; t += blockDim.x) {
        key[t] = ((unsigned long long)g_sid[b + t] << 32) | (unsigned)Rec<T>::id(tmp[b + t]);
        val[t] = (unsigned)t;
      }
      __syncthreads();
      block_bitonic(key, val, len);
      for (int t = threadIdx.x; t < len; t += blockDim.x) {
        out[b + t] = tmp[b + (int)val[t]];
        perm[b + t] = (int)(unsigned)(key[t] & 0xffffffffu);
      }
    }
    __syncthreads();
  }
}

template <typename Tin, typename Tout>
votess_status scan_impl(const Tin* in, int64_t n, Tout* out, Workspace& ws, hipStream_t st) {
  const int64_t n_out = n + 1;
  const int64_t nb = (n_out + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    k_scan_local<Tin, Tout><<<1, kScanBlock, 0, st>>>(in, n, out, n_out, (Tout*)nullptr);
    VT_HIP(hipGetLastError());
    return VOTESS_OK;
  }
  Tout* sums = ws.take<Tout>(nb);
  Tout* offs = ws.take<Tout>(nb + 1);
  k_scan_local<Tin, Tout><<<(unsigned)nb, kScanBlock, 0, st>>>(in, n, out, n_out, sums);
  VT_HIP(hipGetLastError());
  VT_TRY((scan_impl<Tout, Tout>(sums, nb, offs, ws, st)));
  k_scan_add<Tout><<<(unsigned)nb, kScanBlock, 0, st>>>(out, n_out, offs);
  VT_HIP(hipGetLastError());
  return VOTESS_OK;
}

}  // namespace

size_t scan_workspace(int64_t n) {
  size_t bytes = 0;
  int64_t m = n + 1;
  while (true) {
    const int64_t nb = (m + kScanTile - 1) / kScanTile;
    if (nb <= 1) break;
    bytes += Workspace::align(nb * 8) + Workspace::align((nb + 1) * 8);
    m = nb + 1;
  }
  return bytes + 1024;
}

votess_status scan_i32(const int32_t* in, int64_t n, int32_t* out, Workspace& ws, hipStream_t st) {
  return scan_impl<int32_t, int32_t>(in, n, out, ws, st);
}
votess_status scan_i32_to_i64(const int32_t* in, int64_t n, int64_t* out, Workspace& ws, hipStream_t st) {
  return scan_impl<int32_t, int64_t>(in, n, out, ws, st);
}

size_t grid_sort_workspace(int64_t n, int64_t ncells) {
  // cell/rank pairs, counts, unordered records (<= 32 B), dense-cell list,
  // global sort keys and payloads, the dense-cell scratch (sub-cell id,
  // provisional slot, slot ids, counts: four ints per point), scan scratch
  return Workspace::align(n * 8) + Workspace::align(ncells * 4 + 4) + Workspace::align(n * 32) +
         Workspace::align(ncells * 4 + 64) + Workspace::align(n * 8) + Workspace::align(n * 4) +
         4 * Workspace::align(n * 4 + 4) + scan_workspace(ncells) + 4096;
}

// dense cells hold > 16 points each: sum of (16 + count / 2 + 1 + 3) <= n / 2 + 20 n / 17
int64_t sub_capacity(int64_t n) { return n / 2 + (20 * n) / 17 + 1024; }

votess_status launch_grid_sort(votess_ctx* ctx, const void* pts, votess_dtype dt, int n, const GridDev& G,
                               int64_t ncells, int32_t* cell_start, int32_t* perm, void* sorted, int32_t* subinfo,
                               int32_t* sub_start, Workspace& ws, hipStream_t st) {
  const size_t mark = ws.used;
  int2* cr = ws.take<int2>(n > 0 ? n : 1);
  int* count = ws.take<int>(ncells + 1);
  void* tmp = ws.take<char>((size_t)(n > 0 ? n : 1) * (dt == VOTESS_F32 ? 16 : 32));
  int* big = ws.take<int>(ncells + 16);
  int* nbig = ctx->d_counter;
  unsigned long long* gkey = ws.take<unsigned long long>(n > 0 ? n : 1);
  unsigned* gval = ws.take<unsigned>(n > 0 ? n : 1);
  unsigned* g_sid = ws.take<unsigned>(n + 1);
  unsigned* g_rank = ws.take<unsigned>(n + 1);
  unsigned* g_slot = ws.take<unsigned>(n + 1);
  int* g_cnt = ws.take<int>(n + 1);
  int* sub_total = ctx->d_counter + 1;
  VT_HIP(hipMemsetAsync(count, 0, (ncells + 1) * sizeof(int), st));
  VT_HIP(hipMemsetAsync(nbig, 0, 2 * sizeof(int), st));
  const int TB = 256;
  const unsigned nblk = (unsigned)((n + TB - 1) / TB);
  if (n > 0) {
    if (dt == VOTESS_F32)
      k_cell_rank<float><<<nblk, TB, 0, st>>>((const float*)pts, n, G, count, cr, ctx->d_err);
    else
      k_cell_rank<double><<<nblk, TB, 0, st>>>((const double*)pts, n, G, count, cr, ctx->d_err);
    VT_HIP(hipGetLastError());
  }
  VT_TRY(scan_i32(count, ncells, cell_start, ws, st));
  if (n > 0) {
    const unsigned cblk = (unsigned)((ncells + TB - 1) / TB);
    if (dt == VOTESS_F32) {
      k_scatter<float><<<nblk, TB, 0, st>>>((const float*)pts, n, cr, cell_start, (float4*)tmp);
      k_order_small<float><<<cblk, TB, 0, st>>>((const float4*)tmp, cell_start, (int)ncells, (float4*)sorted, perm,
                                                big, nbig, (int2*)subinfo);
      if (subinfo)
        k_order_dense<float><<<kDenseBlocks, 256, 0, st>>>((const float4*)tmp, cell_start, big, nbig, G,
                                                           (float4*)sorted, perm, g_sid, g_rank, g_slot, g_cnt, gkey,
                                                           gval, (int2*)subinfo, sub_start, sub_total);
      else
        k_order_big<float><<<512, 256, 0, st>>>((const float4*)tmp, cell_start, big, nbig, G, (float4*)sorted, perm,
                                                gkey, gval, (int2*)subinfo, sub_start, sub_total);
    } else {
      k_scatter<double><<<nblk, TB, 0, st>>>((const double*)pts, n, cr, cell_start, (double4*)tmp);
      k_order_small<double><<<cblk, TB, 0, st>>>((const double4*)tmp, cell_start, (int)ncells, (double4*)sorted,
                                                 perm, big, nbig, (int2*)subinfo);
      if (subinfo)
        k_order_dense<double><<<kDenseBlocks, 256, 0, st>>>((const double4*)tmp, cell_start, big, nbig, G,
                                                            (double4*)sorted, perm, g_sid, g_rank, g_slot, g_cnt,
                                                            gkey, gval, (int2*)subinfo, sub_start, sub_total);
      else
        k_order_big<double><<<512, 256, 0, st>>>((const double4*)tmp, cell_start, big, nbig, G, (double4*)sorted,
                                                 perm, gkey, gval, (int2*)subinfo, sub_start, sub_total);
    }
    VT_HIP(hipGetLastError());
  }
  ws.used = mark;
  return VOTESS_OK;
}

}  // namespace votess
