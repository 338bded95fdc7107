// C ABI of the library and the host orchestrator of votess_tessellate:
// grid sort -> k-NN -> clip, a GPU retry ladder at doubled k for cells whose
// certificate failed, a large-capacity kernel for cells that overflowed the
// fast kernel, the host fallback last, then CSR assembly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "internal.h"

namespace votess {

static thread_local char g_err[1024] = "no error";

votess_status fail(votess_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

void* dev_alloc(votess_ctx* ctx, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (ctx->alloc) return ctx->alloc(bytes, ctx->user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void dev_free(votess_ctx* ctx, void* p) {
  if (!p) return;
  if (ctx->release) ctx->release(p, ctx->user);
  else (void)hipFree(p);
}

votess_status Workspace::reserve(size_t bytes) {
  used = 0;
  if (bytes <= cap) return VOTESS_OK;
  if (base) dev_free(ctx, base);
  base = nullptr;
  cap = 0;
  const size_t want = std::max(bytes, (size_t)1 << 20);
  base = (char*)dev_alloc(ctx, want);
  if (!base) return fail(VOTESS_ENOMEM, "workspace of %zu bytes", want);
  cap = want;
  return VOTESS_OK;
}

// sub-grid buffers: both or neither, records read as 16-byte vectors
votess_status check_sub(const int32_t* subinfo, const int32_t* sub_start, int64_t n, const char* where) {
  if ((subinfo == nullptr) != (sub_start == nullptr))
    return fail(VOTESS_EINVAL, "%s: subinfo and sub_start go together", where);
  if (sub_start && ((uintptr_t)sub_start & 15u))
    return fail(VOTESS_EINVAL, "%s: sub_start must be 16-byte aligned", where);
  if (subinfo && sub_capacity(n) > INT32_MAX) return fail(VOTESS_EINVAL, "%s: n too large for sub-grids", where);
  return VOTESS_OK;
}

namespace {

struct Buf {  // owned device buffer from the context allocator
  votess_ctx* ctx = nullptr;
  void* p = nullptr;
  Buf() = default;
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  ~Buf() { reset(); }
  void reset() {
    if (p) dev_free(ctx, p);
    p = nullptr;
  }
  template <typename T>
  T* get() const { return (T*)p; }
  void* release() {
    void* q = p;
    p = nullptr;
    return q;
  }
};

votess_status alloc_buf(votess_ctx* ctx, Buf& b, size_t bytes) {
  b.reset();
  b.ctx = ctx;
  b.p = dev_alloc(ctx, bytes);
  if (!b.p) return fail(VOTESS_ENOMEM, "device allocation of %zu bytes", bytes);
  return VOTESS_OK;
}

votess_status check_box(const votess_box* box) {
  if (!box) return fail(VOTESS_EINVAL, "box is null");
  for (int a = 0; a < 3; ++a)
    if (!(box->lo[a] < box->hi[a]) || !std::isfinite(box->lo[a]) || !std::isfinite(box->hi[a]))
      return fail(VOTESS_EINVAL, "box axis %d: need finite lo < hi", a);
  return VOTESS_OK;
}

bool valid_k(int k) {
  return k == 8 || k == 12 || k == 16 || k == 24 || k == 32 || k == 48 || k == 64 || k == 128 || k == kMaxK;
}

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t st;
  double* acc;
  bool ok = false;
  Timer(hipStream_t s, double* out) : st(s), acc(out) {
    ok = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess;
    if (ok) (void)hipEventRecord(a, st);
  }
  void stop() {
    if (!ok) return;
    (void)hipEventRecord(b, st);
    (void)hipEventSynchronize(b);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    *acc += ms;
    ok = false;
  }
  ~Timer() {
    stop();
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

}  // namespace
}  // namespace votess

using namespace votess;

extern "C" {

const int32_t votess_buckets[VOTESS_NBUCKET] = {8, 12, 16, 24, 32, 48, 64};

const char* votess_last_error(void) { return g_err; }
const char* votess_version(void) { return VOTESS_VERSION; }

votess_ctx* votess_create(int device) {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    fail(VOTESS_EHIP, "no HIP device %d", device);
    return nullptr;
  }
  if (hipSetDevice(device) != hipSuccess) {
    fail(VOTESS_EHIP, "hipSetDevice(%d) failed", device);
    return nullptr;
  }
  votess_ctx* ctx = new votess_ctx;
  ctx->device = device;
  ctx->ws.ctx = ctx;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cu = prop.multiProcessorCount;
  if (hipMalloc(&ctx->d_err, 256) != hipSuccess || hipMalloc(&ctx->d_counter, 256) != hipSuccess ||
      hipMemset(ctx->d_err, 0, 256) != hipSuccess || hipMemset(ctx->d_counter, 0, 256) != hipSuccess) {
    fail(VOTESS_ENOMEM, "context scratch");
    votess_destroy(ctx);
    return nullptr;
  }
  if (init_noalloc_scratch(ctx) != VOTESS_OK) {
    votess_destroy(ctx);
    return nullptr;
  }
  return ctx;
}

void votess_destroy(votess_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->ws.base) dev_free(ctx, ctx->ws.base);
  if (ctx->d_err) (void)hipFree(ctx->d_err);
  if (ctx->d_counter) (void)hipFree(ctx->d_counter);
  delete ctx;
}

void votess_set_allocator(votess_ctx* ctx, votess_alloc_fn alloc, votess_release_fn release, void* user) {
  if (!ctx) return;
  if (ctx->ws.base) dev_free(ctx, ctx->ws.base);
  ctx->ws.base = nullptr;
  ctx->ws.cap = 0;
  ctx->alloc = (alloc && release) ? alloc : nullptr;
  ctx->release = (alloc && release) ? release : nullptr;
  ctx->user = user;
}

votess_status votess_ctx_errors(votess_ctx* ctx, void* stream, uint32_t* errors_h) {
  if (!ctx || !errors_h) return fail(VOTESS_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  VT_HIP(hipMemcpyAsync(errors_h, ctx->d_err, 4, hipMemcpyDeviceToHost, st));
  VT_HIP(hipMemsetAsync(ctx->d_err, 0, 4, st));
  VT_HIP(hipStreamSynchronize(st));
  return VOTESS_OK;
}

votess_status votess_grid_plan(int64_t n, const votess_box* box, double pts_per_cell, votess_grid* out) {
  VT_TRY(check_box(box));
  if (!out || n < 0 || !(pts_per_cell > 0)) return fail(VOTESS_EINVAL, "grid_plan: bad n / pts_per_cell / out");
  double vol = 1.0;
  for (int a = 0; a < 3; ++a) vol *= box->hi[a] - box->lo[a];
  const double scale = std::cbrt((double)std::max<int64_t>(n, 1) / (pts_per_cell * vol));
  int64_t G = 1;
  for (int a = 0; a < 3; ++a) {
    const double ext = box->hi[a] - box->lo[a];
    long long g = std::llround(ext * scale);
    g = std::max(1LL, std::min(g, 1LL << 20));
    out->g[a] = (int32_t)g;
    out->lo[a] = box->lo[a];
    out->hi[a] = box->hi[a];
    out->inv_h[a] = (double)g / ext;
    G *= g;
  }
  if (G >= (1LL << 31) - 1) return fail(VOTESS_EINVAL, "grid_plan: %lld grid cells is too many", (long long)G);
  out->ncells = G;
  return VOTESS_OK;
}

static votess_status check_grid(const votess_grid* g) {
  if (!g) return fail(VOTESS_EINVAL, "grid is null");
  if (g->g[0] < 1 || g->g[1] < 1 || g->g[2] < 1 || g->ncells != (int64_t)g->g[0] * g->g[1] * g->g[2])
    return fail(VOTESS_EINVAL, "grid: inconsistent sizes");
  return VOTESS_OK;
}

int64_t votess_sub_capacity(int64_t n) { return sub_capacity(n < 0 ? 0 : n); }


votess_status votess_grid_sort(votess_ctx* ctx, const void* pts, votess_dtype dtype, int64_t n,
                               const votess_box* box, const votess_grid* grid, int32_t* cell_start, int32_t* perm,
                               void* sorted, int32_t* subinfo, int32_t* sub_start, void* stream) {
  if (!ctx) return fail(VOTESS_EINVAL, "ctx is null");
  VT_TRY(check_box(box));
  VT_TRY(check_grid(grid));
  if (n < 0 || n >= (1LL << 31) - 1) return fail(VOTESS_EINVAL, "grid_sort: n out of range");
  if (n > 0 && (!pts || !perm || !sorted)) return fail(VOTESS_EINVAL, "grid_sort: null buffer");
  if (!cell_start) return fail(VOTESS_EINVAL, "grid_sort: null cell_start");
  VT_TRY(check_sub(subinfo, sub_start, n, "grid_sort"));
  if (dtype != VOTESS_F32 && dtype != VOTESS_F64) return fail(VOTESS_EINVAL, "bad dtype");
  VT_HIP(hipSetDevice(ctx->device));
  VT_TRY(ctx->ws.reserve(grid_sort_workspace(n, grid->ncells)));
  votess_grid g2 = *grid;
  for (int a = 0; a < 3; ++a) {
    g2.lo[a] = box->lo[a];
    g2.hi[a] = box->hi[a];
  }
  return launch_grid_sort(ctx, pts, dtype, (int)n, to_dev(g2), grid->ncells, cell_start, perm, sorted, subinfo,
                          sub_start, ctx->ws, (hipStream_t)stream);
}

votess_status votess_knn(votess_ctx* ctx, const void* sorted, votess_dtype dtype, int64_t n,
                         const votess_grid* grid, const int32_t* cell_start, const int32_t* subinfo,
                         const int32_t* sub_start, const int32_t* queries, int64_t nq, int32_t k, votess_dtype dist,
                         int32_t* knn, void* stream) {
  if (!ctx) return fail(VOTESS_EINVAL, "ctx is null");
  VT_TRY(check_grid(grid));
  if (!valid_k(k)) return fail(VOTESS_EINVAL, "knn: k=%d not in {8,12,16,24,32,48,64,128,256}", k);
  if (!queries) nq = n;
  if (n < 0 || nq < 0 || n >= (1LL << 31) - 1) return fail(VOTESS_EINVAL, "knn: bad sizes");
  if (nq > 0 && (!sorted || !cell_start || !knn)) return fail(VOTESS_EINVAL, "knn: null buffer");
  VT_HIP(hipSetDevice(ctx->device));
  VT_TRY(check_sub(subinfo, sub_start, n, "knn"));
  SubGrid sg;
  sg.info = (const int2*)subinfo;
  sg.start = sub_start;
  return launch_knn(ctx, sorted, dtype, (int)n, to_dev(*grid), cell_start, sg, queries, (int)nq, k, dist, knn,
                    (hipStream_t)stream);
}

votess_status votess_clip_cells(votess_ctx* ctx, const void* sorted, votess_dtype dtype, int64_t n,
                                const votess_box* box, const int32_t* cells, int64_t nc, const int32_t* knn,
                                int32_t k, const votess_clip_opts* opts, uint8_t* status, int32_t* nbr_count,
                                int32_t* nbr, double* volume, int32_t* kneeded, int32_t* vcount, double* verts,
                                int32_t* vplanes, double* area, double* centroid, void* stream) {
  if (!ctx || !opts) return fail(VOTESS_EINVAL, "clip: null ctx/opts");
  VT_TRY(check_box(box));
  if (!cells) nc = n;
  if (n < 0 || nc < 0 || n >= (1LL << 31) - 1) return fail(VOTESS_EINVAL, "clip: bad sizes");
  if (k < 0 || k > 64 || (k == 0 && !opts->stream))
    return fail(VOTESS_EINVAL, "clip: k must be in [1, 64], or 0 with the stream phase");
  if (opts->max_nbr < 1) return fail(VOTESS_EINVAL, "clip: max_nbr must be >= 1");
  if (opts->max_vert > 0 && (!vcount || !verts || !vplanes)) return fail(VOTESS_EINVAL, "clip: null vertex buffers");
  if (nc > 0 && (!sorted || (k > 0 && !knn) || !status || !nbr_count || !nbr || !volume))
    return fail(VOTESS_EINVAL, "clip: null buffer");
  if (opts->precision == VOTESS_CLIP_F32_RECHECK && dtype != VOTESS_F32)
    return fail(VOTESS_EINVAL, "clip: F32_RECHECK needs F32 positions");
  VT_HIP(hipSetDevice(ctx->device));
  ClipLaunch a;
  a.sorted = sorted;
  a.dtype = dtype;
  a.n = (int)n;
  for (int i = 0; i < 3; ++i) {
    a.lo[i] = box->lo[i];
    a.hi[i] = box->hi[i];
  }
  a.cells = cells;
  a.nc = (int)nc;
  a.knn = knn;
  a.k = k;
  a.precision = opts->precision;
  a.eps = opts->eps > 0 ? opts->eps : 1e-6;
  a.knn_dist = opts->knn_dist;
  a.max_nbr = opts->max_nbr;
  a.max_vert = opts->max_vert;
  a.capacity = opts->capacity;
  a.out_by_id = opts->out_by_id;
  a.status = status;
  a.nbr_count = nbr_count;
  a.nbr = nbr;
  a.volume = volume;
  a.kneeded = kneeded;
  a.vcount = vcount;
  a.verts = verts;
  a.vplanes = vplanes;
  a.area = area;
  a.centroid = centroid;
  a.counters = nullptr;
  a.stream = opts->stream;
  if (opts->stream) {
    if (!opts->grid || !opts->cell_start) return fail(VOTESS_EINVAL, "clip: stream needs grid and cell_start");
    VT_TRY(check_grid(opts->grid));
    a.grid = to_dev(*opts->grid);
    a.cell_start = opts->cell_start;
    VT_TRY(check_sub(opts->subinfo, opts->sub_start, n, "clip"));
    a.sub.info = (const int2*)opts->subinfo;
    a.sub.start = opts->sub_start;
  }
  return launch_clip(a, (hipStream_t)stream);
}

void votess_params_default(votess_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->k0 = 32;
  p->max_gpu_retries = 1;
  p->pts_per_cell = 2.0;
  p->precision = VOTESS_CLIP_F64;
  p->eps = 1e-6;
  p->kmodel = nullptr;
  p->tau = 0.9;
  p->want_vertices = 0;
  p->index_space = 0;
  p->host_fallback = 1;
  p->host_threads = 0;
  p->force_fail_every = 0;
  p->gpu_stream = 1;
}

void votess_result_free(votess_ctx* ctx, votess_result* r) {
  if (!ctx || !r) return;
  dev_free(ctx, r->row_ptr);
  dev_free(ctx, r->col);
  dev_free(ctx, r->volume);
  dev_free(ctx, r->vrow_ptr);
  dev_free(ctx, r->vxyz);
  dev_free(ctx, r->vplanes);
  dev_free(ctx, r->area);
  dev_free(ctx, r->centroid);
  r->area = nullptr;
  r->centroid = nullptr;
  r->row_ptr = nullptr;
  r->col = nullptr;
  r->volume = nullptr;
  r->vrow_ptr = nullptr;
  r->vxyz = nullptr;
  r->vplanes = nullptr;
}

}  // extern "C"

// --------------------------------------------------------------- tessellate
namespace votess {
votess_status learned_first_pass(votess_ctx* ctx, votess_kmodel* km, double tau, const void* sorted, int n,
                                 const votess_grid& grid, const int32_t* cell_start, const ClipLaunch& base,
                                 int stream, int32_t* cells_buf, votess_stats& S, hipStream_t st);
}

namespace {

constexpr int kMaxNbr = 64;
constexpr int kMaxVert = 256;

// Marks every m-th sorted cell as uncertified (testing aid for the fallback).
__global__ void k_force_fail(uint8_t* status, int n, int every) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n && s % every == 0) status[s] = VOTESS_CELL_RADIUS;
}

// Rows of host-fallback cells longer than the per-cell staging, written
// straight into the result: neighbours (with their face areas) mapped to the
// output index space and sorted ascending at row_ptr[r], or vertices (plane
// ids mapped likewise) at vrow_ptr[r].  Copies on `st` from host staging that
// lives until the final synchronisation.
votess_status write_long_rows(const std::vector<int>& rows, const std::vector<HostCellOut>& cells,
                              const std::vector<int32_t>& ids, const int32_t* perm_d, int n, int index_space,
                              bool faces, const int64_t* row_ptr, int32_t* col, double* area, const int64_t* vrow_ptr,
                              double* vxyz, int32_t* vplanes, hipStream_t st) {
  if (rows.empty()) return VOTESS_OK;
  std::vector<int32_t> perm_h;
  if (index_space == 0) {
    perm_h.resize(n);
    VT_HIP(hipMemcpyAsync(perm_h.data(), perm_d, (size_t)n * 4, hipMemcpyDeviceToHost, st));
  }
  std::vector<int64_t> off(rows.size(), 0);
  const int64_t* rp = col ? row_ptr : vrow_ptr;
  VT_HIP(hipStreamSynchronize(st));
  auto map = [&](int32_t x) { return (x < 0 || index_space != 0) ? x : perm_h[x]; };
  for (size_t t = 0; t < rows.size(); ++t) {
    const int s = ids[rows[t]];
    const int r = index_space != 0 ? s : perm_h[s];
    VT_HIP(hipMemcpyAsync(&off[t], rp + r, 8, hipMemcpyDeviceToHost, st));
  }
  VT_HIP(hipStreamSynchronize(st));
  std::vector<std::vector<int32_t>> ci(rows.size());
  std::vector<std::vector<double>> cd(rows.size());
  for (size_t t = 0; t < rows.size(); ++t) {
    const HostCellOut& o = cells[rows[t]];
    if (col) {
      if ((int)o.nbr.size() <= kMaxNbr) continue;
      std::vector<std::pair<int32_t, double>> e(o.nbr.size());
      for (size_t k = 0; k < o.nbr.size(); ++k) e[k] = {map(o.nbr[k]), faces ? o.area[k] : 0.0};
      std::sort(e.begin(), e.end());
      for (const auto& x : e) {
        ci[t].push_back(x.first);
        cd[t].push_back(x.second);
      }
      VT_HIP(hipMemcpyAsync(col + off[t], ci[t].data(), ci[t].size() * 4, hipMemcpyHostToDevice, st));
      if (faces && area) VT_HIP(hipMemcpyAsync(area + off[t], cd[t].data(), cd[t].size() * 8, hipMemcpyHostToDevice, st));
    } else if (vxyz) {
      if ((int)o.vplanes.size() / 3 <= kMaxVert) continue;
      for (int32_t x : o.vplanes) ci[t].push_back(map(x));
      VT_HIP(hipMemcpyAsync(vxyz + off[t] * 3, o.verts.data(), o.verts.size() * 8, hipMemcpyHostToDevice, st));
      VT_HIP(hipMemcpyAsync(vplanes + off[t] * 3, ci[t].data(), ci[t].size() * 4, hipMemcpyHostToDevice, st));
    }
  }
  VT_HIP(hipStreamSynchronize(st));
  return VOTESS_OK;
}

}  // namespace

extern "C" votess_status votess_tessellate(votess_ctx* ctx, const void* pts, votess_dtype dtype, int64_t n64,
                                           const votess_box* box, const votess_params* params_in,
                                           votess_result* out, void* stream) {
  if (!ctx || !out) return fail(VOTESS_EINVAL, "tessellate: null ctx/out");
  VT_TRY(check_box(box));
  if (n64 < 0 || n64 >= (1LL << 31) - 1) return fail(VOTESS_EINVAL, "tessellate: n out of range");
  if (n64 > 0 && !pts) return fail(VOTESS_EINVAL, "tessellate: null points");
  if (dtype != VOTESS_F32 && dtype != VOTESS_F64) return fail(VOTESS_EINVAL, "bad dtype");
  votess_params P;
  votess_params_default(&P);
  if (params_in) P = *params_in;
  const bool fused = P.k0 == 0 && !P.kmodel;
  if (P.k0 == 0 && (P.kmodel || !P.gpu_stream || P.force_fail_every))
    return fail(VOTESS_EINVAL, "tessellate: k0=0 (no list) needs the stream phase and no k-model");
  if (!fused && !valid_k(P.k0)) return fail(VOTESS_EINVAL, "tessellate: k0=%d not in {8,12,16,24,32,48,64}", P.k0);
  if (P.precision == VOTESS_CLIP_F32_RECHECK && dtype != VOTESS_F32)
    return fail(VOTESS_EINVAL, "tessellate: F32_RECHECK needs F32 positions");
  if (P.max_gpu_retries < 0 || P.max_gpu_retries > VOTESS_MAX_PASSES - 2)
    return fail(VOTESS_EINVAL, "tessellate: max_gpu_retries out of range");
  std::memset(out, 0, sizeof(*out));
  const int n = (int)n64;
  hipStream_t st = (hipStream_t)stream;
  VT_HIP(hipSetDevice(ctx->device));
  votess_stats& S = out->stats;
  auto t_start = std::chrono::steady_clock::now();
  if (P.periodic) {
    if (P.kmodel || P.want_vertices || P.index_space != 0 || P.force_fail_every)
      return fail(VOTESS_EINVAL, "tessellate: periodic boxes take no kmodel, vertices, sorted index space or forced "
                                 "failures");
    VT_TRY(tessellate_periodic(ctx, pts, dtype, n, box, P, out, st));
    S.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    return VOTESS_OK;
  }

  votess_grid grid;
  VT_TRY(votess_grid_plan(n, box, P.pts_per_cell, &grid));
  const size_t esz = dtype == VOTESS_F32 ? 4 : 8;
  const bool wantv = P.want_vertices != 0;
  const bool wantf = P.want_faces != 0;
  const votess_dtype dist = P.precision == VOTESS_CLIP_F32_RECHECK ? VOTESS_F32 : VOTESS_F64;

  Buf cell_start, perm, sorted, status, nbr_count, nbr, vol, vcount, verts, vplanes, knn, cells, cells2, counters;
  Buf subinfo, sub_start, farea, fcen;
  const size_t nn = (size_t)std::max(n, 1);
  VT_TRY(alloc_buf(ctx, cell_start, (grid.ncells + 1) * 4));
  VT_TRY(alloc_buf(ctx, subinfo, grid.ncells * 8));
  VT_TRY(alloc_buf(ctx, sub_start, (size_t)sub_capacity(n) * 4));
  VT_TRY(alloc_buf(ctx, perm, nn * 4));
  VT_TRY(alloc_buf(ctx, sorted, nn * 4 * esz));
  VT_TRY(alloc_buf(ctx, status, nn));
  VT_TRY(alloc_buf(ctx, nbr_count, nn * 4));
  VT_TRY(alloc_buf(ctx, nbr, nn * kMaxNbr * 4));
  VT_TRY(alloc_buf(ctx, vol, nn * 8));
  VT_TRY(alloc_buf(ctx, cells, nn * 4));
  VT_TRY(alloc_buf(ctx, cells2, nn * 4));
  VT_TRY(alloc_buf(ctx, counters, 64));
  if (wantv) {
    VT_TRY(alloc_buf(ctx, vcount, nn * 4));
    VT_TRY(alloc_buf(ctx, verts, nn * kMaxVert * 3 * 8));
    VT_TRY(alloc_buf(ctx, vplanes, nn * kMaxVert * 3 * 4));
  }
  if (wantf) {
    VT_TRY(alloc_buf(ctx, farea, nn * kMaxNbr * 8));
    VT_TRY(alloc_buf(ctx, fcen, nn * 3 * 8));
  }
  VT_TRY(ctx->ws.reserve(std::max(grid_sort_workspace(n, grid.ncells), scan_workspace(n) + nn * 4 + 4096)));
  VT_HIP(hipMemsetAsync(ctx->d_err, 0, 4, st));
  VT_HIP(hipMemsetAsync(counters.p, 0, 64, st));

  // ---- a1-a3 grid sort
  {
    Timer T(st, &S.ms_sort);
    VT_TRY(votess_grid_sort(ctx, pts, dtype, n, box, &grid, cell_start.get<int32_t>(), perm.get<int32_t>(),
                            sorted.p, subinfo.get<int32_t>(), sub_start.get<int32_t>(), stream));
  }
  uint32_t errs = 0;
  VT_TRY(votess_ctx_errors(ctx, stream, &errs));
  if (errs & ERR_OUT_OF_BOX) return fail(VOTESS_EOUTOFBOX, "a point lies outside the box (or is NaN)");

  ClipLaunch base;
  base.sorted = sorted.p;
  base.dtype = dtype;
  base.n = n;
  for (int a = 0; a < 3; ++a) {
    base.lo[a] = box->lo[a];
    base.hi[a] = box->hi[a];
  }
  base.precision = P.precision;
  base.eps = P.eps > 0 ? P.eps : 1e-6;
  base.knn_dist = dist;
  base.max_nbr = kMaxNbr;
  base.max_vert = wantv ? kMaxVert : 0;
  base.capacity = 0;
  base.out_by_id = 1;
  base.status = status.get<uint8_t>();
  base.nbr_count = nbr_count.get<int32_t>();
  base.nbr = nbr.get<int32_t>();
  base.volume = vol.get<double>();
  base.kneeded = nullptr;
  base.vcount = wantv ? vcount.get<int32_t>() : nullptr;
  base.verts = wantv ? verts.get<double>() : nullptr;
  base.vplanes = wantv ? vplanes.get<int32_t>() : nullptr;
  base.area = wantf ? farea.get<double>() : nullptr;
  base.centroid = wantf ? fcen.get<double>() : nullptr;
  base.counters = counters.get<unsigned long long>();
  const GridDev GD = to_dev(grid);
  base.grid = GD;
  base.cell_start = cell_start.get<int32_t>();
  base.sub.info = subinfo.get<int2>();
  base.sub.start = sub_start.get<int32_t>();
  const SubGrid SG = base.sub;
  // the last list pass on the GPU streams uncertified cells on by grid rings
  const bool stream_last = P.gpu_stream != 0 && P.force_fail_every == 0;
  // doublings of k after the first pass (the learned pass ends at the
  // largest bucket), up to the largest k-NN kernel
  const int k_first = P.kmodel ? 64 : P.k0;
  int nretry = 0;
  for (int kk = k_first; !fused && nretry < P.max_gpu_retries && kk < kMaxK; ++nretry) kk = std::min(2 * kk, kMaxK);

  // cells that entered the stream phase so far (device counter 5)
  auto stream_entries = [&](int64_t& out_v) -> votess_status {
    unsigned long long v = 0;
    VT_HIP(hipMemcpyAsync(&v, counters.get<unsigned long long>() + 5, 8, hipMemcpyDeviceToHost, st));
    VT_HIP(hipStreamSynchronize(st));
    out_v = (int64_t)v;
    return VOTESS_OK;
  };
  int64_t entered = 0, entered_before = 0;
  // ---- first pass over all cells
  int k = P.k0;
  int nfail = 0;
  int32_t* cur = cells.get<int32_t>();
  int32_t* nxt = cells2.get<int32_t>();
  if (n > 0) {
    if (P.kmodel) {
      VT_TRY(learned_first_pass(ctx, P.kmodel, P.tau, sorted.p, n, grid, cell_start.get<int32_t>(), base,
                                stream_last && nretry == 0, cur, S, st));
      k = 64;  // retries of the learned pass continue from the largest bucket
    } else {
      if (!fused) {
        VT_TRY(alloc_buf(ctx, knn, nn * (size_t)k * 4));
        Timer T(st, &S.ms_knn);
        VT_TRY(launch_knn(ctx, sorted.p, dtype, n, GD, cell_start.get<int32_t>(), SG, nullptr, n, k, dist,
                          knn.get<int32_t>(), st));
      }
      {
        Timer T(st, &S.ms_clip);
        ClipLaunch c = base;
        c.cells = nullptr;
        c.nc = n;
        c.knn = fused ? nullptr : knn.get<int32_t>();
        c.k = k;
        c.stream = stream_last && nretry == 0;
        VT_TRY(launch_clip(c, st));
      }
      S.pass_k[S.npasses] = k;
      S.pass_cells[S.npasses] = n;
    }
    VT_TRY(votess_ctx_errors(ctx, stream, &errs));
    if (errs & ERR_DUPLICATE) return fail(VOTESS_EDUPLICATE, "two points coincide exactly");
    if (P.force_fail_every > 0) {
      k_force_fail<<<(n + 255) / 256, 256, 0, st>>>(status.get<uint8_t>(), n, P.force_fail_every);
      VT_HIP(hipGetLastError());
    }
    // radius failures retry at 2k; capacity overflows go to the large kernel
    VT_TRY(launch_compact_failed(status.get<uint8_t>(), nullptr, n, cur, ctx->d_counter,
                                 (1u << VOTESS_CELL_RADIUS) | (1u << VOTESS_CELL_CAPACITY), ctx->ws, st));
    VT_HIP(hipMemcpyAsync(&nfail, ctx->d_counter, 4, hipMemcpyDeviceToHost, st));
    VT_HIP(hipStreamSynchronize(st));
    if (!P.kmodel && S.npasses < VOTESS_MAX_PASSES) {
      VT_TRY(stream_entries(entered));
      S.pass_streamed[S.npasses] = entered - entered_before;
      entered_before = entered;
      S.pass_failed[S.npasses++] = nfail;
    }
    if (P.kmodel) VT_TRY(stream_entries(entered_before));
  }
  // ---- GPU retry ladder: cells whose radius test failed retry at doubled k;
  // cells that overflowed the fast kernel rerun in the large-capacity kernel
  auto capacity_pass = [&](const int32_t* ids, int cnt, int kk, bool strm) -> votess_status {
    int ncap = 0;
    VT_TRY(launch_compact_failed(status.get<uint8_t>(), ids, cnt, nxt, ctx->d_counter, 1u << VOTESS_CELL_CAPACITY,
                                 ctx->ws, st));
    VT_HIP(hipMemcpyAsync(&ncap, ctx->d_counter, 4, hipMemcpyDeviceToHost, st));
    VT_HIP(hipStreamSynchronize(st));
    if (ncap == 0) return VOTESS_OK;
    S.capacity_cells += ncap;
    Buf knn2;
    if (kk > 0) {  // (no list in the fused form: the large kernel streams from ring 0 too)
      VT_TRY(alloc_buf(ctx, knn2, (size_t)ncap * kk * 4));
      Timer T(st, &S.ms_knn);
      VT_TRY(launch_knn(ctx, sorted.p, dtype, n, GD, cell_start.get<int32_t>(), SG, nxt, ncap, kk, dist,
                        knn2.get<int32_t>(), st));
    }
    Timer T(st, &S.ms_clip);
    ClipLaunch c2 = base;
    c2.cells = nxt;
    c2.nc = ncap;
    c2.knn = knn2.get<int32_t>();
    c2.k = kk;
    c2.capacity = 1;
    c2.stream = strm ? 1 : 0;
    return launch_clip(c2, st);
  };
  for (int r = 0; r < nretry && nfail > 0 && P.force_fail_every == 0 && k < kMaxK; ++r) {
    k = std::min(2 * k, kMaxK);
    VT_TRY(alloc_buf(ctx, knn, (size_t)nfail * k * 4));
    {
      Timer T(st, &S.ms_knn);
      VT_TRY(launch_knn(ctx, sorted.p, dtype, n, GD, cell_start.get<int32_t>(), SG, cur, nfail, k, dist,
                        knn.get<int32_t>(), st));
    }
    {
      Timer T(st, &S.ms_clip);
      ClipLaunch c = base;
      c.cells = cur;
      c.nc = nfail;
      c.knn = knn.get<int32_t>();
      c.k = k;
      c.stream = stream_last && r == nretry - 1;
      VT_TRY(launch_clip(c, st));
    }
    VT_TRY(capacity_pass(cur, nfail, k, stream_last && r == nretry - 1));
    const int cells_in = nfail;
    VT_TRY(launch_compact_failed(status.get<uint8_t>(), cur, nfail, nxt, ctx->d_counter,
                                 (1u << VOTESS_CELL_RADIUS) | (1u << VOTESS_CELL_CAPACITY), ctx->ws, st));
    VT_HIP(hipMemcpyAsync(&nfail, ctx->d_counter, 4, hipMemcpyDeviceToHost, st));
    VT_HIP(hipStreamSynchronize(st));
    if (S.npasses < VOTESS_MAX_PASSES) {
      VT_TRY(stream_entries(entered));
      S.pass_k[S.npasses] = k;
      S.pass_cells[S.npasses] = cells_in;
      S.pass_streamed[S.npasses] = entered - entered_before;
      entered_before = entered;
      S.pass_failed[S.npasses++] = nfail;
    }
    std::swap(cur, nxt);
  }
  // capacity overflows that no retry revisited (no retries left, or k at its maximum)
  if (nfail > 0 && P.force_fail_every == 0) VT_TRY(capacity_pass(cur, nfail, k, stream_last));
  // ---- everything not certified goes to the host
  int nhost = 0;
  if (n > 0) {
    VT_TRY(launch_compact_failed(status.get<uint8_t>(), nullptr, n, nxt, ctx->d_counter,
                                 (1u << VOTESS_CELL_RADIUS) | (1u << VOTESS_CELL_CAPACITY) |
                                     (1u << VOTESS_CELL_UNRESOLVED), ctx->ws,
                                 st));
    VT_HIP(hipMemcpyAsync(&nhost, ctx->d_counter, 4, hipMemcpyDeviceToHost, st));
    unsigned long long cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    VT_HIP(hipMemcpyAsync(cnt, counters.p, sizeof(cnt), hipMemcpyDeviceToHost, st));
    VT_HIP(hipStreamSynchronize(st));
    S.unresolved_cells = (int64_t)cnt[1];
    S.rechecks = (int64_t)cnt[0];
    S.refined_cells = (int64_t)cnt[3];
    S.streamed_cells = (int64_t)cnt[4];
  }
  // host-fallback cells whose rows exceed the per-cell staging (indices into
  // long_cells / long_ids)
  std::vector<int> long_rows;
  std::vector<HostCellOut> long_cells;
  std::vector<int32_t> long_ids;
  if (nhost > 0) {
    if (!P.host_fallback)
      return fail(VOTESS_EUNRESOLVED, "%d cells were not certified on the GPU and the host fallback is off", nhost);
    auto t0 = std::chrono::steady_clock::now();
    std::vector<int32_t> ids(nhost), cs(grid.ncells + 1);
    std::vector<char> rec((size_t)n * 4 * esz);
    VT_HIP(hipMemcpyAsync(ids.data(), nxt, (size_t)nhost * 4, hipMemcpyDeviceToHost, st));
    VT_HIP(hipMemcpyAsync(cs.data(), cell_start.p, cs.size() * 4, hipMemcpyDeviceToHost, st));
    VT_HIP(hipMemcpyAsync(rec.data(), sorted.p, rec.size(), hipMemcpyDeviceToHost, st));
    VT_HIP(hipStreamSynchronize(st));
    std::sort(ids.begin(), ids.end());
    std::vector<HostCellOut> res;
    host_fallback_cells(rec.data(), dtype, n, grid, cs.data(), ids.data(), nhost, wantv, wantf, P.host_threads,
                        res);
    // write back per cell (small transfers, batched through host staging)
    std::vector<int32_t> h_cnt(nhost), h_nbr((size_t)nhost * kMaxNbr, -1), h_vc;
    std::vector<double> h_vol(nhost), h_v, h_area, h_cen;
    if (wantf) {
      h_area.assign((size_t)nhost * kMaxNbr, 0.0);
      h_cen.assign((size_t)nhost * 3, 0.0);
    }
    std::vector<int32_t> h_vp;
    std::vector<uint8_t> h_st(nhost);
    if (wantv) {
      h_vc.resize(nhost);
      h_v.assign((size_t)nhost * kMaxVert * 3, 0.0);
      h_vp.assign((size_t)nhost * kMaxVert * 3, 0);
    }
    for (int i = 0; i < nhost; ++i) {
      const HostCellOut& o = res[i];
      if (!o.ok) return fail(VOTESS_EUNRESOLVED, "host fallback could not build cell %d", ids[i]);
      // rows longer than the per-cell staging (more than kMaxNbr neighbours
      // or kMaxVert vertices) keep their true counts here and are written
      // into the CSR by the host after the fill kernels (long_rows)
      const int nnb = (int)o.nbr.size();
      h_cnt[i] = (int32_t)nnb;
      std::copy(o.nbr.begin(), o.nbr.begin() + std::min(nnb, kMaxNbr), h_nbr.begin() + (size_t)i * kMaxNbr);
      h_vol[i] = o.volume;
      h_st[i] = VOTESS_CELL_CERTIFIED;
      if (wantf) {
        std::copy(o.area.begin(), o.area.begin() + std::min(nnb, kMaxNbr), h_area.begin() + (size_t)i * kMaxNbr);
        std::copy(o.centroid, o.centroid + 3, h_cen.begin() + (size_t)i * 3);
      }
      const int nv = (int)o.vplanes.size() / 3;
      if (wantv) {
        h_vc[i] = nv;
        std::copy(o.verts.begin(), o.verts.begin() + 3 * std::min(nv, kMaxVert), h_v.begin() + (size_t)i * kMaxVert * 3);
        std::copy(o.vplanes.begin(), o.vplanes.begin() + 3 * std::min(nv, kMaxVert),
                  h_vp.begin() + (size_t)i * kMaxVert * 3);
      }
      if (nnb > kMaxNbr || (wantv && nv > kMaxVert)) long_rows.push_back(i);
    }
    long_cells.swap(res);
    long_ids = ids;
    for (int i = 0; i < nhost; ++i) {  // contiguous id runs go in one copy each
      int e = i;
      while (e + 1 < nhost && ids[e + 1] == ids[e] + 1) ++e;
      const int s0 = ids[i], len = e - i + 1;
      VT_HIP(hipMemcpyAsync(nbr_count.get<int32_t>() + s0, &h_cnt[i], len * 4, hipMemcpyHostToDevice, st));
      VT_HIP(hipMemcpyAsync(nbr.get<int32_t>() + (size_t)s0 * kMaxNbr, &h_nbr[(size_t)i * kMaxNbr],
                            (size_t)len * kMaxNbr * 4, hipMemcpyHostToDevice, st));
      VT_HIP(hipMemcpyAsync(vol.get<double>() + s0, &h_vol[i], len * 8, hipMemcpyHostToDevice, st));
      VT_HIP(hipMemcpyAsync(status.get<uint8_t>() + s0, &h_st[i], len, hipMemcpyHostToDevice, st));
      if (wantf) {
        VT_HIP(hipMemcpyAsync(farea.get<double>() + (size_t)s0 * kMaxNbr, &h_area[(size_t)i * kMaxNbr],
                              (size_t)len * kMaxNbr * 8, hipMemcpyHostToDevice, st));
        VT_HIP(hipMemcpyAsync(fcen.get<double>() + (size_t)s0 * 3, &h_cen[(size_t)i * 3], (size_t)len * 3 * 8,
                              hipMemcpyHostToDevice, st));
      }
      if (wantv) {
        VT_HIP(hipMemcpyAsync(vcount.get<int32_t>() + s0, &h_vc[i], len * 4, hipMemcpyHostToDevice, st));
        VT_HIP(hipMemcpyAsync(verts.get<double>() + (size_t)s0 * kMaxVert * 3, &h_v[(size_t)i * kMaxVert * 3],
                              (size_t)len * kMaxVert * 3 * 8, hipMemcpyHostToDevice, st));
        VT_HIP(hipMemcpyAsync(vplanes.get<int32_t>() + (size_t)s0 * kMaxVert * 3, &h_vp[(size_t)i * kMaxVert * 3],
                              (size_t)len * kMaxVert * 3 * 4, hipMemcpyHostToDevice, st));
      }
      i = e;
    }
    VT_HIP(hipStreamSynchronize(st));
    S.fallback_cells = nhost;
    S.ms_fallback = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }

  // ---- a9 assembly
  {
    Timer T(st, &S.ms_assemble);
    Buf row_ptr, col, volume, area, centroid;
    VT_TRY(alloc_buf(ctx, row_ptr, (nn + 1) * 8));
    VT_TRY(alloc_buf(ctx, volume, nn * 8));
    int64_t nnz = 0;
    VT_TRY(launch_assemble(nbr_count.get<int32_t>(), nbr.get<int32_t>(), kMaxNbr, vol.get<double>(), nullptr, nullptr,
                           perm.get<int32_t>(), n, P.index_space, row_ptr.get<int64_t>(), nullptr, nullptr, nullptr,
                           nullptr, ctx->ws, st, &nnz));
    VT_TRY(alloc_buf(ctx, col, (size_t)std::max<int64_t>(nnz, 1) * 4));
    if (wantf) {
      VT_TRY(alloc_buf(ctx, area, (size_t)std::max<int64_t>(nnz, 1) * 8));
      VT_TRY(alloc_buf(ctx, centroid, nn * 3 * 8));
    }
    VT_TRY(launch_assemble(nbr_count.get<int32_t>(), nbr.get<int32_t>(), kMaxNbr, vol.get<double>(),
                           wantf ? farea.get<double>() : nullptr, wantf ? fcen.get<double>() : nullptr,
                           perm.get<int32_t>(), n, P.index_space, row_ptr.get<int64_t>(), col.get<int32_t>(),
                           volume.get<double>(), wantf ? area.get<double>() : nullptr,
                           wantf ? centroid.get<double>() : nullptr, ctx->ws, st, &nnz));
    VT_TRY(write_long_rows(long_rows, long_cells, long_ids, perm.get<int32_t>(), n, P.index_space, wantf,
                           row_ptr.get<int64_t>(), col.get<int32_t>(), wantf ? area.get<double>() : nullptr, nullptr,
                           nullptr, nullptr, st));
    out->n = n;
    out->nnz = nnz;
    if (wantv) {
      Buf vrow, vxyz, vpl;
      VT_TRY(alloc_buf(ctx, vrow, (nn + 1) * 8));
      int64_t nv = 0;
      VT_TRY(launch_assemble_vertices(vcount.get<int32_t>(), verts.get<double>(), vplanes.get<int32_t>(), kMaxVert,
                                      perm.get<int32_t>(), n, P.index_space, vrow.get<int64_t>(), nullptr, nullptr,
                                      ctx->ws, st, &nv));
      VT_TRY(alloc_buf(ctx, vxyz, (size_t)std::max<int64_t>(nv, 1) * 24));
      VT_TRY(alloc_buf(ctx, vpl, (size_t)std::max<int64_t>(nv, 1) * 12));
      VT_TRY(launch_assemble_vertices(vcount.get<int32_t>(), verts.get<double>(), vplanes.get<int32_t>(), kMaxVert,
                                      perm.get<int32_t>(), n, P.index_space, vrow.get<int64_t>(),
                                      vxyz.get<double>(), vpl.get<int32_t>(), ctx->ws, st, &nv));
      VT_TRY(write_long_rows(long_rows, long_cells, long_ids, perm.get<int32_t>(), n, P.index_space, false, nullptr,
                             nullptr, nullptr, vrow.get<int64_t>(), vxyz.get<double>(), vpl.get<int32_t>(), st));
      out->nvert = nv;
      out->vrow_ptr = (int64_t*)vrow.release();
      out->vxyz = (double*)vxyz.release();
      out->vplanes = (int32_t*)vpl.release();
    }
    VT_HIP(hipStreamSynchronize(st));
    out->row_ptr = (int64_t*)row_ptr.release();
    out->col = (int32_t*)col.release();
    out->volume = (double*)volume.release();
    if (wantf) {
      out->area = (double*)area.release();
      out->centroid = (double*)centroid.release();
    }
  }
  S.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  return VOTESS_OK;
}
