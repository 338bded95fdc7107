// Periodic boxes: the box [lo, hi) is a 3-torus of periods L = hi - lo, and
// the cell of p_i is the region nearer p_i than any image p_j + m L.  The
// method is unchanged -- nearest neighbours, bisector clipping, the
// security radius (paper, Summary section) -- and so are the kernels: the
// points are padded with their images within a margin w around the box
// (ghosts, materialised in HBM), the padded set is sorted into a grid of the
// enlarged box [lo - w, hi + w], and only the original points are clipped.
// A cell certified with radius R is the periodic cell as soon as 2R < w:
// every image within 2R of its generator is then among the ghosts, and the
// enlarged box's walls lie farther than R.  Cells with 2R >= w are computed
// again with the margin doubled.  Neighbours are reported by the index of
// the point whose image shares the face (once per image).  The padded set is
// held in double whatever the input type: the image x + L of a float x is in
// general not a float (it needs one more bit), and images must be exact.
// So periodic cells are clipped in FP64.
#include "internal.h"
#include "device_common.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace votess {
namespace {

constexpr int kPerNbr = 64;  // per-cell staging of neighbours (longer host rows go straight to the CSR)

// Images of coordinate x kept along one axis: shifts m with
// lo - w <= x + m L < lo + L + w, among [m_lo, m_hi] (a range wide enough
// for any w <= kMaxPeriods L).
constexpr int kMaxPeriods = 4;
__device__ __forceinline__ bool keep_image(double x, int m, double lo, double L, double w) {
  const double y = x + m * L;
  return y >= lo - w && y < lo + L + w;
}

template <typename T>
__global__ void k_ghost_count(const T* __restrict__ pts, int n, double lo0, double lo1, double lo2, double L0,
                              double L1, double L2, double w, int* __restrict__ counts, unsigned* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x[3] = {(double)pts[3 * (size_t)i], (double)pts[3 * (size_t)i + 1], (double)pts[3 * (size_t)i + 2]};
  const double lo[3] = {lo0, lo1, lo2}, L[3] = {L0, L1, L2};
  int c[3];
  bool inside = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    inside = inside && x[a] >= lo[a] && x[a] < lo[a] + L[a];
    c[a] = 0;
    for (int m = -kMaxPeriods; m <= kMaxPeriods; ++m) c[a] += keep_image(x[a], m, lo[a], L[a], w);
  }
  if (!inside) atomicOr(err, ERR_OUT_OF_BOX);
  counts[i] = inside ? c[0] * c[1] * c[2] - 1 : 0;
}

// originals first (rows 0..n-1), then each point's images at n + offs[i],
// all in double (x + m L is exact for float x and for double x whose
// exponent is near L's)
template <typename T>
__global__ void k_ghost_write(const T* __restrict__ pts, int n, double lo0, double lo1, double lo2, double L0,
                              double L1, double L2, double w, const int* __restrict__ offs, double* __restrict__ ext,
                              int* __restrict__ src) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x[3] = {(double)pts[3 * (size_t)i], (double)pts[3 * (size_t)i + 1], (double)pts[3 * (size_t)i + 2]};
  const double lo[3] = {lo0, lo1, lo2}, L[3] = {L0, L1, L2};
  for (int a = 0; a < 3; ++a) ext[3 * (size_t)i + a] = x[a];
  src[i] = i;
  const bool inside = x[0] >= lo0 && x[0] < lo0 + L0 && x[1] >= lo1 && x[1] < lo1 + L1 && x[2] >= lo2 && x[2] < lo2 + L2;
  if (!inside) return;
  size_t o = (size_t)n + offs[i];
  for (int mz = -kMaxPeriods; mz <= kMaxPeriods; ++mz) {
    if (!keep_image(x[2], mz, lo[2], L[2], w)) continue;
    for (int my = -kMaxPeriods; my <= kMaxPeriods; ++my) {
      if (!keep_image(x[1], my, lo[1], L[1], w)) continue;
      for (int mx = -kMaxPeriods; mx <= kMaxPeriods; ++mx) {
        if (!keep_image(x[0], mx, lo[0], L[0], w) || (mx == 0 && my == 0 && mz == 0)) continue;
        ext[3 * o] = x[0] + mx * L[0];
        ext[3 * o + 1] = x[1] + my * L[1];
        ext[3 * o + 2] = x[2] + mz * L[2];
        src[o] = i;
        ++o;
      }
    }
  }
}

// 1 for sorted positions s holding a pending original point
__global__ void k_pending_flags(const int* __restrict__ perm, int n_ext, int n, const uint8_t* __restrict__ done,
                                uint8_t* __restrict__ flag) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_ext) return;
  const int e = perm[s];
  flag[s] = (e < n && !done[e]) ? 1 : 0;
}

// Results of the clipped cells (row t = cells[t]) whose security ball lies
// inside the margin, moved to their original rows with neighbours mapped
// sorted -> padded -> source index.
__global__ void k_periodic_gather(const int* __restrict__ cells, int nc, const int* __restrict__ perm,
                                  const int* __restrict__ src, const uint8_t* __restrict__ status,
                                  const int* __restrict__ cnt, const int* __restrict__ nbr,
                                  const double* __restrict__ vol, const double* __restrict__ area,
                                  const double* __restrict__ cen, const double* __restrict__ r2, double guard2,
                                  int* __restrict__ o_cnt, int* __restrict__ o_nbr, double* __restrict__ o_vol,
                                  double* __restrict__ o_area, double* __restrict__ o_cen, uint8_t* __restrict__ done) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc) return;
  if (status[t] != VOTESS_CELL_CERTIFIED || !(4.0 * r2[t] < guard2)) return;
  const int i = perm[cells[t]];
  const int c = cnt[t];
  o_cnt[i] = c;
  o_vol[i] = vol[t];
  for (int e = 0; e < c && e < kPerNbr; ++e) {
    o_nbr[(size_t)i * kPerNbr + e] = src[perm[nbr[(size_t)t * kPerNbr + e]]];
    if (o_area) o_area[(size_t)i * kPerNbr + e] = area[(size_t)t * kPerNbr + e];
  }
  if (o_cen)
    for (int a = 0; a < 3; ++a) o_cen[(size_t)i * 3 + a] = cen[(size_t)t * 3 + a];
  done[i] = 1;
}

struct DBuf {
  votess_ctx* ctx = nullptr;
  void* p = nullptr;
  ~DBuf() { dev_free(ctx, p); }
  votess_status alloc(votess_ctx* c, size_t bytes) {
    dev_free(c, p);
    ctx = c;
    p = dev_alloc(c, bytes);
    if (!p) return fail(VOTESS_ENOMEM, "periodic: device allocation of %zu bytes", bytes);
    return VOTESS_OK;
  }
  template <typename T>
  T* get() const { return (T*)p; }
};

}  // namespace

votess_status tessellate_periodic(votess_ctx* ctx, const void* pts, votess_dtype dtype, int n, const votess_box* box,
                                  const votess_params& P, votess_result* out, hipStream_t st) {
  votess_stats& S = out->stats;
  const bool wantf = P.want_faces != 0;
  // the padded set is double (exact images), so is the clipping
  const size_t esz = 8;
  const votess_dtype xdt = VOTESS_F64, dist = VOTESS_F64;
  double L[3], vol = 1.0, lmin = 1e300;
  for (int a = 0; a < 3; ++a) {
    L[a] = box->hi[a] - box->lo[a];
    vol *= L[a];
    lmin = std::min(lmin, L[a]);
  }
  const size_t nn = (size_t)std::max(n, 1);
  DBuf o_cnt, o_nbr, o_vol, o_area, o_cen, done, counts, offs, flags, cells;
  VT_TRY(o_cnt.alloc(ctx, nn * 4));
  VT_TRY(o_nbr.alloc(ctx, nn * kPerNbr * 4));
  VT_TRY(o_vol.alloc(ctx, nn * 8));
  VT_TRY(done.alloc(ctx, nn));
  VT_TRY(counts.alloc(ctx, nn * 4));
  VT_TRY(offs.alloc(ctx, (nn + 1) * 4));
  if (wantf) {
    VT_TRY(o_area.alloc(ctx, nn * kPerNbr * 8));
    VT_TRY(o_cen.alloc(ctx, nn * 3 * 8));
  }
  VT_HIP(hipMemsetAsync(done.p, 0, nn, st));
  VT_HIP(hipMemsetAsync(o_cnt.p, 0, nn * 4, st));
  VT_HIP(hipMemsetAsync(ctx->d_err, 0, 4, st));
  // host-fallback rows longer than the staging: original row, mapped ids, areas
  struct LongRow {
    int row;
    std::vector<int32_t> ids;
    std::vector<double> area;
  };
  std::vector<LongRow> long_rows;

  // margin: four mean spacings, doubled while some cell's ball pokes out
  double w = 4.0 * std::cbrt(vol / std::max(n, 1));
  const unsigned nb = (unsigned)((nn + 255) / 256);
  int pending = n;
  for (int attempt = 0; pending > 0; ++attempt) {
    if (w > kMaxPeriods * lmin) w = kMaxPeriods * lmin;
    const double guard = w * (1.0 - 1e-9);  // 2R below it: every image within 2R is padded in
    // ---- padded point set
    if (dtype == VOTESS_F32)
      k_ghost_count<float><<<nb, 256, 0, st>>>((const float*)pts, n, box->lo[0], box->lo[1], box->lo[2], L[0], L[1],
                                               L[2], w, counts.get<int>(), ctx->d_err);
    else
      k_ghost_count<double><<<nb, 256, 0, st>>>((const double*)pts, n, box->lo[0], box->lo[1], box->lo[2], L[0],
                                                L[1], L[2], w, counts.get<int>(), ctx->d_err);
    VT_HIP(hipGetLastError());
    VT_TRY(ctx->ws.reserve(scan_workspace(n) + 4096));
    VT_TRY(scan_i32(counts.get<int>(), n, offs.get<int>(), ctx->ws, st));
    int nghost = 0;
    uint32_t errs = 0;
    VT_HIP(hipMemcpyAsync(&nghost, offs.get<int>() + n, 4, hipMemcpyDeviceToHost, st));
    VT_HIP(hipMemcpyAsync(&errs, ctx->d_err, 4, hipMemcpyDeviceToHost, st));
    VT_HIP(hipStreamSynchronize(st));
    if (errs & ERR_OUT_OF_BOX) return fail(VOTESS_EOUTOFBOX, "periodic: a point lies outside [lo, hi) (or is NaN)");
    const int64_t n_ext64 = (int64_t)n + nghost;
    if (n_ext64 >= (1LL << 31) - 1) return fail(VOTESS_EINVAL, "periodic: %lld padded points", (long long)n_ext64);
    const int n_ext = (int)n_ext64;
    DBuf ext, src;
    VT_TRY(ext.alloc(ctx, (size_t)n_ext * 3 * esz));
    VT_TRY(src.alloc(ctx, (size_t)n_ext * 4));
    if (dtype == VOTESS_F32)
      k_ghost_write<float><<<nb, 256, 0, st>>>((const float*)pts, n, box->lo[0], box->lo[1], box->lo[2], L[0], L[1],
                                               L[2], w, offs.get<int>(), ext.get<double>(), src.get<int>());
    else
      k_ghost_write<double><<<nb, 256, 0, st>>>((const double*)pts, n, box->lo[0], box->lo[1], box->lo[2], L[0],
                                                L[1], L[2], w, offs.get<int>(), ext.get<double>(), src.get<int>());
    VT_HIP(hipGetLastError());
    // ---- grid sort of the padded set over the enlarged box
    votess_box xb;
    for (int a = 0; a < 3; ++a) {
      xb.lo[a] = box->lo[a] - w;
      xb.hi[a] = box->hi[a] + w;
    }
    votess_grid grid;
    VT_TRY(votess_grid_plan(n_ext, &xb, P.pts_per_cell, &grid));
    DBuf cs, perm, sorted, subinfo, sub_start;
    VT_TRY(cs.alloc(ctx, (grid.ncells + 1) * 4));
    VT_TRY(perm.alloc(ctx, (size_t)n_ext * 4));
    VT_TRY(sorted.alloc(ctx, (size_t)n_ext * 4 * esz));
    VT_TRY(subinfo.alloc(ctx, grid.ncells * 8));
    VT_TRY(sub_start.alloc(ctx, (size_t)sub_capacity(n_ext) * 4));
    VT_TRY(ctx->ws.reserve(std::max(grid_sort_workspace(n_ext, grid.ncells), scan_workspace(n_ext) + 4096)));
    {
      const size_t mark = ctx->ws.used;
      VT_TRY(launch_grid_sort(ctx, ext.p, xdt, n_ext, to_dev(grid), grid.ncells, cs.get<int>(), perm.get<int>(),
                              sorted.p, subinfo.get<int>(), sub_start.get<int>(), ctx->ws, st));
      ctx->ws.used = mark;
    }
    // ---- the pending originals, in sorted (grid) order
    VT_TRY(flags.alloc(ctx, (size_t)n_ext));
    VT_TRY(cells.alloc(ctx, (size_t)n_ext * 4));
    k_pending_flags<<<(unsigned)((n_ext + 255) / 256), 256, 0, st>>>(perm.get<int>(), n_ext, n, done.get<uint8_t>(),
                                                                     flags.get<uint8_t>());
    VT_HIP(hipGetLastError());
    VT_TRY(launch_compact_failed(flags.get<uint8_t>(), nullptr, n_ext, cells.get<int>(), ctx->d_counter, 1u << 1,
                                 ctx->ws, st));
    int nc = 0;
    VT_HIP(hipMemcpyAsync(&nc, ctx->d_counter, 4, hipMemcpyDeviceToHost, st));
    VT_HIP(hipStreamSynchronize(st));
    if (nc == 0) break;
    // ---- k-NN + clip with the stream phase, large kernel, host fallback
    const int k = 64;
    DBuf knn, status, cnt, nbr, cvol, r2, carea, ccen, counters;
    VT_TRY(knn.alloc(ctx, (size_t)nc * k * 4));
    VT_TRY(status.alloc(ctx, (size_t)nc));
    VT_TRY(cnt.alloc(ctx, (size_t)nc * 4));
    VT_TRY(nbr.alloc(ctx, (size_t)nc * kPerNbr * 4));
    VT_TRY(cvol.alloc(ctx, (size_t)nc * 8));
    VT_TRY(r2.alloc(ctx, (size_t)nc * 8));
    VT_TRY(counters.alloc(ctx, 64));
    VT_HIP(hipMemsetAsync(counters.p, 0, 64, st));
    if (wantf) {
      VT_TRY(carea.alloc(ctx, (size_t)nc * kPerNbr * 8));
      VT_TRY(ccen.alloc(ctx, (size_t)nc * 3 * 8));
    }
    SubGrid SG;
    SG.info = subinfo.get<int2>();
    SG.start = sub_start.get<int>();
    const GridDev GD = to_dev(grid);
    VT_TRY(launch_knn(ctx, sorted.p, xdt, n_ext, GD, cs.get<int>(), SG, cells.get<int>(), nc, k, dist,
                      knn.get<int>(), st));
    ClipLaunch c;
    c.sorted = sorted.p;
    c.dtype = xdt;
    c.n = n_ext;
    for (int a = 0; a < 3; ++a) {
      c.lo[a] = xb.lo[a];
      c.hi[a] = xb.hi[a];
    }
    c.cells = cells.get<int>();
    c.nc = nc;
    c.knn = knn.get<int>();
    c.k = k;
    c.precision = VOTESS_CLIP_F64;
    c.eps = P.eps > 0 ? P.eps : 1e-6;
    c.knn_dist = dist;
    c.max_nbr = kPerNbr;
    c.max_vert = 0;
    c.capacity = 0;
    c.out_by_id = 0;
    c.status = status.get<uint8_t>();
    c.nbr_count = cnt.get<int>();
    c.nbr = nbr.get<int>();
    c.volume = cvol.get<double>();
    c.kneeded = nullptr;
    c.vcount = nullptr;
    c.verts = nullptr;
    c.vplanes = nullptr;
    c.area = wantf ? carea.get<double>() : nullptr;
    c.centroid = wantf ? ccen.get<double>() : nullptr;
    c.r2out = r2.get<double>();
    c.counters = counters.get<unsigned long long>();
    c.stream = P.gpu_stream != 0;
    c.cell_start = cs.get<int>();
    c.grid = GD;
    c.sub = SG;
    VT_TRY(launch_clip(c, st));
    // the cells' statuses are by row t: compact rows, not ids
    DBuf rows, ids2, knn2;
    VT_TRY(rows.alloc(ctx, (size_t)nc * 4));
    VT_TRY(launch_compact_failed(status.get<uint8_t>(), nullptr, nc, rows.get<int>(), ctx->d_counter,
                                 1u << VOTESS_CELL_CAPACITY, ctx->ws, st));
    int ncap = 0;
    VT_HIP(hipMemcpyAsync(&ncap, ctx->d_counter, 4, hipMemcpyDeviceToHost, st));
    VT_HIP(hipStreamSynchronize(st));
    S.capacity_cells += ncap;
    std::vector<int> rows_h;
    if (ncap > 0) {
      // overflow of the fast kernel: the large-capacity kernel on the same
      // lists, rows gathered and scattered back on the host
      rows_h.resize(ncap);
      std::vector<int> cells_h(nc);
      VT_HIP(hipMemcpyAsync(rows_h.data(), rows.p, (size_t)ncap * 4, hipMemcpyDeviceToHost, st));
      VT_HIP(hipMemcpyAsync(cells_h.data(), cells.p, (size_t)nc * 4, hipMemcpyDeviceToHost, st));
      VT_HIP(hipStreamSynchronize(st));
      std::vector<int> sub_ids(ncap);
      for (int t = 0; t < ncap; ++t) sub_ids[t] = cells_h[rows_h[t]];
      VT_TRY(ids2.alloc(ctx, (size_t)ncap * 4));
      VT_HIP(hipMemcpyAsync(ids2.p, sub_ids.data(), (size_t)ncap * 4, hipMemcpyHostToDevice, st));
      VT_TRY(knn2.alloc(ctx, (size_t)ncap * k * 4));
      VT_TRY(launch_knn(ctx, sorted.p, xdt, n_ext, GD, cs.get<int>(), SG, ids2.get<int>(), ncap, k, dist,
                        knn2.get<int>(), st));
      DBuf st2, cnt2, nbr2, vol2, r22, area2, cen2;
      VT_TRY(st2.alloc(ctx, ncap));
      VT_TRY(cnt2.alloc(ctx, (size_t)ncap * 4));
      VT_TRY(nbr2.alloc(ctx, (size_t)ncap * kPerNbr * 4));
      VT_TRY(vol2.alloc(ctx, (size_t)ncap * 8));
      VT_TRY(r22.alloc(ctx, (size_t)ncap * 8));
      if (wantf) {
        VT_TRY(area2.alloc(ctx, (size_t)ncap * kPerNbr * 8));
        VT_TRY(cen2.alloc(ctx, (size_t)ncap * 3 * 8));
      }
      ClipLaunch c2 = c;
      c2.cells = ids2.get<int>();
      c2.nc = ncap;
      c2.knn = knn2.get<int>();
      c2.capacity = 1;
      c2.status = st2.get<uint8_t>();
      c2.nbr_count = cnt2.get<int>();
      c2.nbr = nbr2.get<int>();
      c2.volume = vol2.get<double>();
      c2.r2out = r22.get<double>();
      c2.area = wantf ? area2.get<double>() : nullptr;
      c2.centroid = wantf ? cen2.get<double>() : nullptr;
      VT_TRY(launch_clip(c2, st));
      // scatter the large kernel's rows back to their rows of the first clip
      std::vector<uint8_t> s2(ncap);
      std::vector<int> n2(ncap), b2((size_t)ncap * kPerNbr);
      std::vector<double> v2(ncap), r2h(ncap), a2(wantf ? (size_t)ncap * kPerNbr : 0), c2h(wantf ? (size_t)ncap * 3 : 0);
      VT_HIP(hipMemcpyAsync(s2.data(), st2.p, ncap, hipMemcpyDeviceToHost, st));
      VT_HIP(hipMemcpyAsync(n2.data(), cnt2.p, (size_t)ncap * 4, hipMemcpyDeviceToHost, st));
      VT_HIP(hipMemcpyAsync(b2.data(), nbr2.p, b2.size() * 4, hipMemcpyDeviceToHost, st));
      VT_HIP(hipMemcpyAsync(v2.data(), vol2.p, (size_t)ncap * 8, hipMemcpyDeviceToHost, st));
      VT_HIP(hipMemcpyAsync(r2h.data(), r22.p, (size_t)ncap * 8, hipMemcpyDeviceToHost, st));
      if (wantf) {
        VT_HIP(hipMemcpyAsync(a2.data(), area2.p, a2.size() * 8, hipMemcpyDeviceToHost, st));
        VT_HIP(hipMemcpyAsync(c2h.data(), cen2.p, c2h.size() * 8, hipMemcpyDeviceToHost, st));
      }
      VT_HIP(hipStreamSynchronize(st));
      for (int t = 0; t < ncap; ++t) {
        const int r = rows_h[t];
        VT_HIP(hipMemcpyAsync(status.get<uint8_t>() + r, &s2[t], 1, hipMemcpyHostToDevice, st));
        VT_HIP(hipMemcpyAsync(cnt.get<int>() + r, &n2[t], 4, hipMemcpyHostToDevice, st));
        VT_HIP(hipMemcpyAsync(nbr.get<int>() + (size_t)r * kPerNbr, &b2[(size_t)t * kPerNbr], kPerNbr * 4,
                              hipMemcpyHostToDevice, st));
        VT_HIP(hipMemcpyAsync(cvol.get<double>() + r, &v2[t], 8, hipMemcpyHostToDevice, st));
        VT_HIP(hipMemcpyAsync(r2.get<double>() + r, &r2h[t], 8, hipMemcpyHostToDevice, st));
        if (wantf) {
          VT_HIP(hipMemcpyAsync(carea.get<double>() + (size_t)r * kPerNbr, &a2[(size_t)t * kPerNbr], kPerNbr * 8,
                                hipMemcpyHostToDevice, st));
          VT_HIP(hipMemcpyAsync(ccen.get<double>() + (size_t)r * 3, &c2h[(size_t)t * 3], 24, hipMemcpyHostToDevice,
                                st));
        }
      }
      VT_HIP(hipStreamSynchronize(st));
    }
    // ---- the rest (still uncertified) on the host
    VT_TRY(launch_compact_failed(status.get<uint8_t>(), nullptr, nc, rows.get<int>(), ctx->d_counter,
                                 (1u << VOTESS_CELL_RADIUS) | (1u << VOTESS_CELL_CAPACITY) |
                                     (1u << VOTESS_CELL_UNRESOLVED),
                                 ctx->ws, st));
    int nhost = 0;
    unsigned long long cntr[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    VT_HIP(hipMemcpyAsync(&nhost, ctx->d_counter, 4, hipMemcpyDeviceToHost, st));
    VT_HIP(hipMemcpyAsync(cntr, counters.p, sizeof(cntr), hipMemcpyDeviceToHost, st));
    VT_HIP(hipStreamSynchronize(st));
    S.rechecks += (int64_t)cntr[0];
    S.refined_cells += (int64_t)cntr[3];
    S.streamed_cells += (int64_t)cntr[4];
    if (S.npasses < VOTESS_MAX_PASSES) {
      S.pass_k[S.npasses] = k;
      S.pass_cells[S.npasses] = nc;
      S.pass_failed[S.npasses] = nhost;
      S.pass_streamed[S.npasses] = (int64_t)cntr[5];
      S.npasses++;
    }
    if (nhost > 0) {
      if (!P.host_fallback)
        return fail(VOTESS_EUNRESOLVED, "%d cells were not certified on the GPU and the host fallback is off", nhost);
      std::vector<int> hrows(nhost), cells_h(nc), perm_h(n_ext), src_h(n_ext), cs_h(grid.ncells + 1);
      std::vector<char> rec((size_t)n_ext * 4 * esz);
      VT_HIP(hipMemcpyAsync(hrows.data(), rows.p, (size_t)nhost * 4, hipMemcpyDeviceToHost, st));
      VT_HIP(hipMemcpyAsync(cells_h.data(), cells.p, (size_t)nc * 4, hipMemcpyDeviceToHost, st));
      VT_HIP(hipMemcpyAsync(perm_h.data(), perm.p, (size_t)n_ext * 4, hipMemcpyDeviceToHost, st));
      VT_HIP(hipMemcpyAsync(src_h.data(), src.p, (size_t)n_ext * 4, hipMemcpyDeviceToHost, st));
      VT_HIP(hipMemcpyAsync(cs_h.data(), cs.p, cs_h.size() * 4, hipMemcpyDeviceToHost, st));
      VT_HIP(hipMemcpyAsync(rec.data(), sorted.p, rec.size(), hipMemcpyDeviceToHost, st));
      VT_HIP(hipStreamSynchronize(st));
      std::vector<int32_t> hid(nhost);
      for (int t = 0; t < nhost; ++t) hid[t] = cells_h[hrows[t]];
      std::vector<HostCellOut> res;
      host_fallback_cells(rec.data(), xdt, n_ext, grid, cs_h.data(), hid.data(), nhost, false, wantf,
                          P.host_threads, res);
      S.fallback_cells += nhost;
      std::vector<uint8_t> hst(nhost);
      std::vector<int> hcnt(nhost), hnbr((size_t)nhost * kPerNbr, -1);
      std::vector<double> hvol(nhost), hr2(nhost), harea(wantf ? (size_t)nhost * kPerNbr : 0),
          hcen(wantf ? (size_t)nhost * 3 : 0);
      for (int t = 0; t < nhost; ++t) {
        const HostCellOut& o = res[t];
        if (!o.ok) return fail(VOTESS_EUNRESOLVED, "host fallback could not build cell %d", hid[t]);
        const int row = perm_h[hid[t]];
        hst[t] = VOTESS_CELL_CERTIFIED;
        hvol[t] = o.volume;
        hr2[t] = o.r2;
        const int m = (int)o.nbr.size();
        // neighbours go straight to source indices here
        hcnt[t] = std::min(m, kPerNbr);
        if (m > kPerNbr && 4.0 * o.r2 < guard * guard) {
          LongRow lr;
          lr.row = row;
          for (int e = 0; e < m; ++e) {
            lr.ids.push_back(src_h[perm_h[o.nbr[e]]]);
            lr.area.push_back(wantf ? o.area[e] : 0.0);
          }
          long_rows.push_back(std::move(lr));
          hcnt[t] = m;
        }
        for (int e = 0; e < std::min(m, kPerNbr); ++e) {
          hnbr[(size_t)t * kPerNbr + e] = o.nbr[e];
          if (wantf) harea[(size_t)t * kPerNbr + e] = o.area[e];
        }
        if (wantf)
          for (int a = 0; a < 3; ++a) hcen[(size_t)t * 3 + a] = o.centroid[a];
      }
      for (int t = 0; t < nhost; ++t) {
        const int r = hrows[t];
        VT_HIP(hipMemcpyAsync(status.get<uint8_t>() + r, &hst[t], 1, hipMemcpyHostToDevice, st));
        VT_HIP(hipMemcpyAsync(cnt.get<int>() + r, &hcnt[t], 4, hipMemcpyHostToDevice, st));
        VT_HIP(hipMemcpyAsync(nbr.get<int>() + (size_t)r * kPerNbr, &hnbr[(size_t)t * kPerNbr], kPerNbr * 4,
                              hipMemcpyHostToDevice, st));
        VT_HIP(hipMemcpyAsync(cvol.get<double>() + r, &hvol[t], 8, hipMemcpyHostToDevice, st));
        VT_HIP(hipMemcpyAsync(r2.get<double>() + r, &hr2[t], 8, hipMemcpyHostToDevice, st));
        if (wantf) {
          VT_HIP(hipMemcpyAsync(carea.get<double>() + (size_t)r * kPerNbr, &harea[(size_t)t * kPerNbr], kPerNbr * 8,
                                hipMemcpyHostToDevice, st));
          VT_HIP(hipMemcpyAsync(ccen.get<double>() + (size_t)r * 3, &hcen[(size_t)t * 3], 24, hipMemcpyHostToDevice,
                                st));
        }
      }
      VT_HIP(hipStreamSynchronize(st));
    }
    // ---- cells whose ball lies inside the margin are final
    k_periodic_gather<<<(unsigned)((nc + 255) / 256), 256, 0, st>>>(
        cells.get<int>(), nc, perm.get<int>(), src.get<int>(), status.get<uint8_t>(), cnt.get<int>(), nbr.get<int>(),
        cvol.get<double>(), wantf ? carea.get<double>() : nullptr, wantf ? ccen.get<double>() : nullptr,
        r2.get<double>(), guard * guard, o_cnt.get<int>(), o_nbr.get<int>(), o_vol.get<double>(),
        wantf ? o_area.get<double>() : nullptr, wantf ? o_cen.get<double>() : nullptr, done.get<uint8_t>());
    VT_HIP(hipGetLastError());
    VT_TRY(launch_compact_failed(done.get<uint8_t>(), nullptr, n, cells.get<int>(), ctx->d_counter, 1u << 0, ctx->ws,
                                 st));
    VT_HIP(hipMemcpyAsync(&pending, ctx->d_counter, 4, hipMemcpyDeviceToHost, st));
    VT_HIP(hipStreamSynchronize(st));
    if (pending > 0 && w >= kMaxPeriods * lmin)
      return fail(VOTESS_EUNRESOLVED, "periodic: %d cells reach farther than %d periods", pending, kMaxPeriods);
    w *= 2.0;
    if (attempt > 16) return fail(VOTESS_EUNRESOLVED, "periodic: margin did not converge");
  }

  // ---- CSR over the original rows (neighbours already source indices)
  DBuf row_ptr, col, volume, area, centroid;
  VT_TRY(row_ptr.alloc(ctx, (nn + 1) * 8));
  VT_TRY(volume.alloc(ctx, nn * 8));
  int64_t nnz = 0;
  VT_TRY(ctx->ws.reserve(scan_workspace(n) + nn * 4 + 4096));
  VT_TRY(launch_assemble(o_cnt.get<int>(), o_nbr.get<int>(), kPerNbr, o_vol.get<double>(), nullptr, nullptr, nullptr,
                         n, 1, row_ptr.get<int64_t>(), nullptr, nullptr, nullptr, nullptr, ctx->ws, st, &nnz));
  VT_TRY(col.alloc(ctx, (size_t)std::max<int64_t>(nnz, 1) * 4));
  if (wantf) {
    VT_TRY(area.alloc(ctx, (size_t)std::max<int64_t>(nnz, 1) * 8));
    VT_TRY(centroid.alloc(ctx, nn * 3 * 8));
  }
  VT_TRY(launch_assemble(o_cnt.get<int>(), o_nbr.get<int>(), kPerNbr, o_vol.get<double>(),
                         wantf ? o_area.get<double>() : nullptr, wantf ? o_cen.get<double>() : nullptr, nullptr, n, 1,
                         row_ptr.get<int64_t>(), col.get<int>(), volume.get<double>(),
                         wantf ? area.get<double>() : nullptr, wantf ? centroid.get<double>() : nullptr, ctx->ws, st,
                         &nnz));
  // long host rows, sorted ascending (areas alongside), at their row offsets
  std::vector<std::vector<int32_t>> ci(long_rows.size());
  std::vector<std::vector<double>> cd(long_rows.size());
  std::vector<int64_t> off(long_rows.size(), 0);
  for (size_t t = 0; t < long_rows.size(); ++t)
    VT_HIP(hipMemcpyAsync(&off[t], row_ptr.get<int64_t>() + long_rows[t].row, 8, hipMemcpyDeviceToHost, st));
  VT_HIP(hipStreamSynchronize(st));
  for (size_t t = 0; t < long_rows.size(); ++t) {
    std::vector<std::pair<int32_t, double>> e(long_rows[t].ids.size());
    for (size_t q = 0; q < e.size(); ++q) e[q] = {long_rows[t].ids[q], long_rows[t].area[q]};
    std::sort(e.begin(), e.end());
    for (const auto& x : e) {
      ci[t].push_back(x.first);
      cd[t].push_back(x.second);
    }
    VT_HIP(hipMemcpyAsync(col.get<int>() + off[t], ci[t].data(), ci[t].size() * 4, hipMemcpyHostToDevice, st));
    if (wantf)
      VT_HIP(hipMemcpyAsync(area.get<double>() + off[t], cd[t].data(), cd[t].size() * 8, hipMemcpyHostToDevice, st));
  }
  VT_HIP(hipStreamSynchronize(st));
  out->n = n;
  out->nnz = nnz;
  out->row_ptr = (int64_t*)row_ptr.p;
  out->col = (int32_t*)col.p;
  out->volume = (double*)volume.p;
  row_ptr.p = col.p = volume.p = nullptr;
  if (wantf) {
    out->area = (double*)area.p;
    out->centroid = (double*)centroid.p;
    area.p = centroid.p = nullptr;
  }
  return VOTESS_OK;
}

}  // namespace votess
