// Grid sort of the generators (paper, Summary: "the input set of points is
// sorted into a grid") as a counting sort:
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

constexpr int kSmallCell = 16;    // cells up to this size are reordered by one thread
constexpr int kLdsSortMax = 4096; // larger cells sort their keys in global memory

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
                              int* __restrict__ big, int* __restrict__ nbig) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  const int b = cell_start[c], e = cell_start[c + 1];
  const int len = e - b;
  if (len == 0) return;
  if (len > kSmallCell) {
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
template <typename KeyPtr>
__device__ void block_bitonic(KeyPtr key, int len) {
  int P = 1;
  while (P < len) P <<= 1;
  for (int k = 2; k <= P; k <<= 1) {
    for (int t = threadIdx.x; t < len; t += blockDim.x) {
      const int p = t ^ (k - 1);
      if (p > t && p < len) {
        const unsigned long long a = key[t], b = key[p];
        if (b < a) { key[t] = b; key[p] = a; }
      }
    }
    __syncthreads();
    for (int j = k >> 2; j >= 1; j >>= 1) {
      for (int t = threadIdx.x; t < len; t += blockDim.x) {
        const int p = t ^ j;
        if (p > t && p < len) {
          const unsigned long long a = key[t], b = key[p];
          if (b < a) { key[t] = b; key[p] = a; }
        }
      }
      __syncthreads();
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_order_big(const typename Rec<T>::type* __restrict__ tmp,
                                                   const int* __restrict__ cell_start, const int* __restrict__ big,
                                                   const int* __restrict__ nbig, typename Rec<T>::type* __restrict__ out,
                                                   int* __restrict__ perm, unsigned long long* __restrict__ gkey) {
  __shared__ unsigned long long skey[kLdsSortMax];
  const int nb = *nbig;
  for (int q = blockIdx.x; q < nb; q += gridDim.x) {
    const int c = big[q];
    const int b = cell_start[c], len = cell_start[c + 1] - b;
    const bool lds = len <= kLdsSortMax;
    unsigned long long* key = lds ? skey : gkey + b;
    for (int t = threadIdx.x; t < len; t += blockDim.x)
      key[t] = ((unsigned long long)(unsigned)Rec<T>::id(tmp[b + t]) << 32) | (unsigned)t;
    __syncthreads();
    block_bitonic(key, len);
    for (int t = threadIdx.x; t < len; t += blockDim.x) {
      const unsigned long long kv = key[t];
      out[b + t] = tmp[b + (int)(kv & 0xffffffffu)];
      perm[b + t] = (int)(kv >> 32);
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
  // cell/rank pairs, counts, unordered records (<= 32 B), big-cell list,
  // global sort keys, scan scratch
  return Workspace::align(n * 8) + Workspace::align(ncells * 4 + 4) + Workspace::align(n * 32) +
         Workspace::align(ncells * 4 + 64) + Workspace::align(n * 8) + scan_workspace(ncells) + 4096;
}

votess_status launch_grid_sort(votess_ctx* ctx, const void* pts, votess_dtype dt, int n, const GridDev& G,
                               int64_t ncells, int32_t* cell_start, int32_t* perm, void* sorted, Workspace& ws,
                               hipStream_t st) {
  const size_t mark = ws.used;
  int2* cr = ws.take<int2>(n > 0 ? n : 1);
  int* count = ws.take<int>(ncells + 1);
  void* tmp = ws.take<char>((size_t)(n > 0 ? n : 1) * (dt == VOTESS_F32 ? 16 : 32));
  int* big = ws.take<int>(ncells + 16);
  int* nbig = ctx->d_counter;
  unsigned long long* gkey = ws.take<unsigned long long>(n > 0 ? n : 1);
  VT_HIP(hipMemsetAsync(count, 0, (ncells + 1) * sizeof(int), st));
  VT_HIP(hipMemsetAsync(nbig, 0, sizeof(int), st));
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
                                                big, nbig);
      k_order_big<float><<<512, 256, 0, st>>>((const float4*)tmp, cell_start, big, nbig, (float4*)sorted, perm, gkey);
    } else {
      k_scatter<double><<<nblk, TB, 0, st>>>((const double*)pts, n, cr, cell_start, (double4*)tmp);
      k_order_small<double><<<cblk, TB, 0, st>>>((const double4*)tmp, cell_start, (int)ncells, (double4*)sorted,
                                                 perm, big, nbig);
      k_order_big<double><<<512, 256, 0, st>>>((const double4*)tmp, cell_start, big, nbig, (double4*)sorted, perm,
                                               gkey);
    }
    VT_HIP(hipGetLastError());
  }
  ws.used = mark;
  return VOTESS_OK;
}

}  // namespace votess
