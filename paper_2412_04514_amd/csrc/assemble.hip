// Retry compaction (cells whose certificate failed, in order) and output assembly: the
// per-cell neighbour lists become one CSR array of rows of neighbour indices
// (paper, Features section: a jagged array of natural neighbours), rows in original input order by default or in
// grid-sorted order, each row ascending; volumes, face areas, centroids and
// vertices follow.
#include "internal.h"

namespace votess {
namespace {

// Cells of `cells` (or 0..nc-1) whose status bit is in `mask`, written to out
// in their input order, so that a compacted list of grid-sorted cells stays
// grid-sorted (neighbouring queries share cache lines in the k-NN and clip).
// Three steps: per-block counts, one scan of the counts, per-block writes.
constexpr int kCompactBlock = 256;

__device__ __forceinline__ bool compact_take(const uint8_t* __restrict__ status, const int* __restrict__ cells,
                                             int nc, unsigned mask, int t, int& id) {
  id = 0;
  if (t >= nc) return false;
  id = cells ? cells[t] : t;
  return (mask >> status[id]) & 1u;
}

__global__ __launch_bounds__(kCompactBlock) void k_compact_count(const uint8_t* __restrict__ status,
                                                                 const int* __restrict__ cells, int nc,
                                                                 unsigned mask, int* __restrict__ bcount) {
  __shared__ int wsum[kCompactBlock / 64];
  int id;
  const bool take = compact_take(status, cells, nc, mask, blockIdx.x * kCompactBlock + threadIdx.x, id);
  const unsigned long long b = __ballot(take);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = __popcll(b);
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < kCompactBlock / 64; ++w) s += wsum[w];
    bcount[blockIdx.x] = s;
  }
}

// Exclusive scan of nb block counts in place (one block), total to *count.
__global__ __launch_bounds__(1024) void k_compact_scan(int* __restrict__ bcount, int nb, int* __restrict__ count) {
  __shared__ int part[1024];
  const int per = (nb + 1023) / 1024;
  const int b0 = threadIdx.x * per, b1 = min(b0 + per, nb);
  int s = 0;
  for (int i = b0; i < b1; ++i) s += bcount[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {  // Hillis-Steele inclusive scan of the per-thread sums
    const int v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int run = part[threadIdx.x] - s;
  for (int i = b0; i < b1; ++i) {
    const int c = bcount[i];
    bcount[i] = run;
    run += c;
  }
  if (threadIdx.x == 1023) *count = part[1023];
}

__global__ __launch_bounds__(kCompactBlock) void k_compact_write(const uint8_t* __restrict__ status,
                                                                 const int* __restrict__ cells, int nc,
                                                                 unsigned mask, const int* __restrict__ boff,
                                                                 int* __restrict__ out) {
  __shared__ int wsum[kCompactBlock / 64];
  int id;
  const bool take = compact_take(status, cells, nc, mask, blockIdx.x * kCompactBlock + threadIdx.x, id);
  const unsigned long long b = __ballot(take);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) wsum[w] = __popcll(b);
  __syncthreads();
  int base = boff[blockIdx.x];
  for (int v = 0; v < w; ++v) base += wsum[v];
  if (take) out[base + __popcll(b & ((1ull << lane) - 1ull))] = id;
}

__global__ void k_rows_count(const int* __restrict__ nbr_count, const int* __restrict__ perm, int n, int sorted_space,
                             int* __restrict__ counts) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  counts[sorted_space ? s : perm[s]] = nbr_count[s];
}

// A group of 16 lanes per row (rows of at most 64 entries, four per lane):
// the lanes read the row's neighbour ids in one coalesced load, map them to
// the output index space, stage them in LDS, and rank each of their entries
// against the whole row (equal ids, which a periodic row may hold, are
// ranked by position); the group then writes its row with one store to
// contiguous addresses, so that each output row reaches L2 whole rather than
// one id at a time from rows scattered over the array.  Areas move with
// their ids; volumes and centroids with their rows.
constexpr int kFillBlock = 256;
constexpr int kFillLanes = 16;
constexpr int kFillMax = 64;
__global__ __launch_bounds__(kFillBlock) void k_rows_fill(
    const int* __restrict__ nbr_count, const int* __restrict__ nbr, int max_nbr, const int* __restrict__ perm,
    const double* __restrict__ vol_sorted, const double* __restrict__ area_sorted,
    const double* __restrict__ cen_sorted, int n, int sorted_space, const long long* __restrict__ row_ptr,
    int* __restrict__ col, double* __restrict__ volume, double* __restrict__ area, double* __restrict__ centroid) {
  constexpr int R = kFillBlock / kFillLanes, J = kFillMax / kFillLanes;
  __shared__ int ids[R * (kFillMax + 1)];  // rows padded by a word: the groups' rows start in distinct banks
  const int l = threadIdx.x & (kFillLanes - 1), g = threadIdx.x / kFillLanes;
  const int s = blockIdx.x * R + g;
  if (s >= n) return;  // whole groups leave together
  const int r = sorted_space ? s : perm[s];
  if (l == 0) volume[r] = vol_sorted[s];
  if (centroid && l < 3) centroid[(size_t)r * 3 + l] = cen_sorted[(size_t)s * 3 + l];
  // a row longer than the staging stride (a host-fallback cell) is written
  // by the host
  const int cnt = nbr_count[s];
  if (cnt > max_nbr) return;
  const int* src = nbr + (size_t)s * max_nbr;
  int* row = ids + g * (kFillMax + 1);
  int v[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int e = l + j * kFillLanes;
    v[j] = 0;
    if (e < cnt) {
      v[j] = sorted_space ? src[e] : perm[src[e]];
      row[e] = v[j];
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  int rank[J] = {};
  const int nj = (cnt + kFillLanes - 1) / kFillLanes;
  for (int x = 0; x < cnt; ++x) {
    const int w = row[x];
#pragma unroll
    for (int j = 0; j < J; ++j)
      if (j < nj) rank[j] += w < v[j] || (w == v[j] && x < l + j * kFillLanes);
  }
  const long long o = row_ptr[r];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int e = l + j * kFillLanes;
    if (e < cnt) {
      col[o + rank[j]] = v[j];
      if (area) area[o + rank[j]] = area_sorted[(size_t)s * max_nbr + e];
    }
  }
}

__global__ void k_vrows_count(const int* __restrict__ vcount, const int* __restrict__ perm, int n, int sorted_space,
                              int* __restrict__ counts) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  counts[sorted_space ? s : perm[s]] = vcount[s];
}

__global__ void k_vrows_fill(const int* __restrict__ vcount, const double* __restrict__ verts,
                             const int* __restrict__ vplanes, int max_vert, const int* __restrict__ perm, int n,
                             int sorted_space, const long long* __restrict__ vrow_ptr, double* __restrict__ vxyz,
                             int* __restrict__ vout) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int r = sorted_space ? s : perm[s];
  const long long o = vrow_ptr[r];
  const int cnt = vcount[s];
  if (cnt > max_vert) return;  // written by the host (a host-fallback cell)
  for (int e = 0; e < cnt; ++e) {
    const size_t si = ((size_t)s * max_vert + e) * 3;
    for (int a = 0; a < 3; ++a) {
      vxyz[(o + e) * 3 + a] = verts[si + a];
      const int p = vplanes[si + a];
      vout[(o + e) * 3 + a] = (p < 0 || sorted_space) ? p : perm[p];
    }
  }
}

}  // namespace

votess_status launch_compact_failed(const uint8_t* status, const int32_t* cells, int nc, int32_t* out_cells,
                                    int32_t* d_count, uint8_t want_status_mask, Workspace& ws, hipStream_t st) {
  if (nc <= 0) {
    VT_HIP(hipMemsetAsync(d_count, 0, sizeof(int), st));
    return VOTESS_OK;
  }
  const int nb = (nc + kCompactBlock - 1) / kCompactBlock;
  const size_t mark = ws.used;
  const size_t need = Workspace::align(ws.used) + (size_t)nb * sizeof(int);
  if (need > ws.cap) return fail(VOTESS_ENOMEM, "compaction: workspace of %zu bytes < %zu", ws.cap, need);
  int* bcount = ws.take<int>(nb);
  k_compact_count<<<(unsigned)nb, kCompactBlock, 0, st>>>(status, cells, nc, want_status_mask, bcount);
  VT_HIP(hipGetLastError());
  k_compact_scan<<<1, 1024, 0, st>>>(bcount, nb, d_count);
  VT_HIP(hipGetLastError());
  k_compact_write<<<(unsigned)nb, kCompactBlock, 0, st>>>(status, cells, nc, want_status_mask, bcount, out_cells);
  VT_HIP(hipGetLastError());
  ws.used = mark;  // the stream orders the kernels before any later use of the space
  return VOTESS_OK;
}

votess_status launch_assemble(const int32_t* nbr_count, const int32_t* nbr, int max_nbr, const double* vol_sorted,
                              const double* area_sorted, const double* cen_sorted, const int32_t* perm, int n,
                              int index_space, int64_t* row_ptr, int32_t* col, double* volume, double* area,
                              double* centroid, Workspace& ws, hipStream_t st, int64_t* nnz_h) {
  const unsigned b = (unsigned)((n + 255) / 256);
  if (col == nullptr) {  // phase 1: counts -> row_ptr, nnz to the host
    const size_t mark = ws.used;
    int* counts = ws.take<int>(n > 0 ? n : 1);
    if (n > 0) {
      k_rows_count<<<b, 256, 0, st>>>(nbr_count, perm, n, index_space, counts);
      VT_HIP(hipGetLastError());
    }
    VT_TRY(scan_i32_to_i64(counts, n, row_ptr, ws, st));
    VT_HIP(hipMemcpyAsync(nnz_h, row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    VT_HIP(hipStreamSynchronize(st));
    ws.used = mark;
    return VOTESS_OK;
  }
  if (max_nbr > kFillMax) return fail(VOTESS_EINVAL, "assemble: rows longer than %d", kFillMax);
  if ((area && !area_sorted) || (centroid && !cen_sorted)) return fail(VOTESS_EINVAL, "assemble: null face input");
  if (n > 0) {  // phase 2: fill
    constexpr int rows_per_block = kFillBlock / kFillLanes;
    k_rows_fill<<<(unsigned)((n + rows_per_block - 1) / rows_per_block), kFillBlock, 0, st>>>(
        nbr_count, nbr, max_nbr, perm, vol_sorted, area_sorted, cen_sorted, n, index_space,
        (const long long*)row_ptr, col, volume, area, centroid);
    VT_HIP(hipGetLastError());
  }
  return VOTESS_OK;
}

votess_status launch_assemble_vertices(const int32_t* vcount, const double* verts, const int32_t* vplanes,
                                       int max_vert, const int32_t* perm, int n, int index_space,
                                       int64_t* vrow_ptr, double* vxyz, int32_t* vout, Workspace& ws,
                                       hipStream_t st, int64_t* nv_h) {
  const unsigned b = (unsigned)((n + 255) / 256);
  if (vxyz == nullptr) {
    const size_t mark = ws.used;
    int* counts = ws.take<int>(n > 0 ? n : 1);
    if (n > 0) {
      k_vrows_count<<<b, 256, 0, st>>>(vcount, perm, n, index_space, counts);
      VT_HIP(hipGetLastError());
    }
    VT_TRY(scan_i32_to_i64(counts, n, vrow_ptr, ws, st));
    VT_HIP(hipMemcpyAsync(nv_h, vrow_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    VT_HIP(hipStreamSynchronize(st));
    ws.used = mark;
    return VOTESS_OK;
  }
  if (n > 0) {
    k_vrows_fill<<<b, 256, 0, st>>>(vcount, verts, vplanes, max_vert, perm, n, index_space,
                                    (const long long*)vrow_ptr, vxyz, vout);
    VT_HIP(hipGetLastError());
  }
  return VOTESS_OK;
}

}  // namespace votess
