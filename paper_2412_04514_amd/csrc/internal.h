// Internal declarations shared by the HIP kernels and the host orchestrator.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstddef>
#include <string>
#include <vector>

#include "../../include/votess.h"

#define VOTESS_VERSION "0.1.0"

namespace votess {

// ------------------------------------------------------------------ errors
votess_status fail(votess_status s, const char* fmt, ...);
// Largest list length of the k-NN kernels (the GPU retry ladder stops there).
constexpr int kMaxK = 256;
// Sub-grid buffers of votess_grid_sort: both or neither, 16-byte aligned.
votess_status check_sub(const int32_t* subinfo, const int32_t* sub_start, int64_t n, const char* where);
#define VT_HIP(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::votess::fail(VOTESS_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)
#define VT_TRY(expr)                     \
  do {                                   \
    votess_status s_ = (expr);           \
    if (s_ != VOTESS_OK) return s_;      \
  } while (0)

// Device error bits (votess_ctx_errors).
enum : uint32_t { ERR_OUT_OF_BOX = 1u, ERR_DUPLICATE = 2u };

// ------------------------------------------------------------- device grid
struct GridDev {
  int g0, g1, g2;
  double lo0, lo1, lo2;
  double hi0, hi1, hi2;
  double ih0, ih1, ih2;  // g / extent
  double h0, h1, h2;     // extent / g
};
GridDev to_dev(const votess_grid& g);

// -------------------------------------------------------------- workspace
// Bump allocator over one growable device buffer owned by the context.
struct Workspace {
  votess_ctx* ctx = nullptr;
  char* base = nullptr;
  size_t cap = 0, used = 0;
  votess_status reserve(size_t bytes);
  template <typename T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + count * sizeof(T);
    return reinterpret_cast<T*>(base + off);
  }
  static size_t align(size_t b) { return (b + 255) & ~size_t(255); }
};

}  // namespace votess

struct votess_ctx {
  int device = 0;
  votess_alloc_fn alloc = nullptr;
  votess_release_fn release = nullptr;
  void* user = nullptr;
  uint32_t* d_err = nullptr;   // device error word
  int* d_counter = nullptr;    // small device scratch counters [16]
  votess::Workspace ws;
  int num_cu = 0;
  void* noalloc_scratch = nullptr;  // device address of the static scratch (votess_features_noalloc)
};

namespace votess {

void* dev_alloc(votess_ctx* ctx, size_t bytes);
void dev_free(votess_ctx* ctx, void* p);
// looks up the device address of the allocation-free pass's static scratch
// on the context's (current) device (learned.hip)
votess_status init_noalloc_scratch(votess_ctx* ctx);

// --------------------------------------------------------------- launchers
// grid sort (grid_sort.hip)
size_t grid_sort_workspace(int64_t n, int64_t ncells);
votess_status launch_grid_sort(votess_ctx* ctx, const void* pts, votess_dtype dt, int n, const GridDev& G,
                               int64_t ncells, int32_t* cell_start, int32_t* perm, void* sorted, int32_t* subinfo,
                               int32_t* sub_start, Workspace& ws, hipStream_t st);
int64_t sub_capacity(int64_t n);

// Sub-grids of dense cells: subinfo[2 c] = offset into sub_start (or -1),
// subinfo[2 c + 1] = m; sub_start[offset + s] = first point of sub-cell s
// relative to cell_start[c], for s = 0..m^3.
struct SubGrid {
  const int2* info = nullptr;
  const int* start = nullptr;
};

// exclusive scan: out[0..n] with out[n] = total (grid_sort.hip)
size_t scan_workspace(int64_t n);
votess_status scan_i32(const int32_t* in, int64_t n, int32_t* out, Workspace& ws, hipStream_t st);
votess_status scan_i32_to_i64(const int32_t* in, int64_t n, int64_t* out, Workspace& ws, hipStream_t st);

// k-NN (knn.hip)
votess_status launch_knn(votess_ctx* ctx, const void* sorted, votess_dtype dt, int n, const GridDev& G,
                         const int32_t* cell_start, const SubGrid& sub, const int32_t* queries, int nq, int k,
                         votess_dtype dist, int32_t* knn, hipStream_t st);

// clipping (clip.hip)
struct ClipLaunch {
  const void* sorted;
  votess_dtype dtype;
  int n;
  double lo[3], hi[3];
  const int32_t* cells;
  int nc;
  const int32_t* knn;
  int k;
  int knn_stride = 0;  // entries per list row (0: k); a row may be longer than the k entries used
  int knn_by_id = 0;   // 1: list row of a cell = its sorted id (else its position in `cells`)
  votess_precision precision;
  double eps;
  votess_dtype knn_dist;
  int max_nbr, max_vert, capacity, out_by_id;
  uint8_t* status;
  int32_t* nbr_count;
  int32_t* nbr;
  double* volume;
  int32_t* kneeded;
  int32_t* vcount;
  double* verts;
  int32_t* vplanes;
  double* area = nullptr;        // [rows, max_nbr] face areas next to nbr (nullable)
  double* centroid = nullptr;    // [rows, 3] cell centroids (nullable)
  double* r2out = nullptr;       // [rows] R^2 of each certified cell (nullable; an upper bound on the float path)
  unsigned long long* counters;  // [8]: rechecks, unresolved, capacity, refined, streamed (certified by the
                                 // stream phase), stream entries -- nullable
  int stream = 0;                // 1: uncertified cells continue by grid rings
  const int32_t* cell_start = nullptr;
  GridDev grid{};
  SubGrid sub{};
};
votess_status launch_clip(const ClipLaunch& a, hipStream_t st);

// compaction of cells by status (assemble.hip)
// order-preserving; takes nc/256 ints of `ws` for the duration of its kernels
votess_status launch_compact_failed(const uint8_t* status, const int32_t* cells, int nc, int32_t* out_cells,
                                    int32_t* d_count, uint8_t want_status_mask, Workspace& ws, hipStream_t st);

// CSR assembly (assemble.hip)
// area_sorted / cen_sorted (nullable) travel with their rows into area / centroid.
votess_status launch_assemble(const int32_t* nbr_count, const int32_t* nbr, int max_nbr, const double* vol_sorted,
                              const double* area_sorted, const double* cen_sorted, const int32_t* perm, int n,
                              int index_space, int64_t* row_ptr, int32_t* col, double* volume, double* area,
                              double* centroid, Workspace& ws, hipStream_t st, int64_t* nnz_h);
votess_status launch_assemble_vertices(const int32_t* vcount, const double* verts, const int32_t* vplanes,
                                       int max_vert, const int32_t* perm, int n, int index_space,
                                       int64_t* vrow_ptr, double* vxyz, int32_t* vout, Workspace& ws,
                                       hipStream_t st, int64_t* nv_h);

// periodic boxes (periodic.hip): ghost-padded tessellation of the torus
votess_status tessellate_periodic(votess_ctx* ctx, const void* pts, votess_dtype dtype, int n, const votess_box* box,
                                  const votess_params& P, votess_result* out, hipStream_t st);

// host fallback (fallback.cpp): exact cells with unbounded k on the CPU.
struct HostCellOut {
  std::vector<int32_t> nbr;     // sorted indices of neighbours (unordered)
  std::vector<double> area;     // face area per entry of nbr (want_faces)
  double volume = 0.0;
  double centroid[3] = {0.0, 0.0, 0.0};  // (want_faces)
  std::vector<double> verts;    // absolute xyz
  std::vector<int32_t> vplanes; // sorted indices or -1..-6
  double r2 = 0.0;              // largest squared distance from the generator to a vertex
  bool ok = false;
};
void host_fallback_cells(const void* sorted_h, votess_dtype dt, int n, const votess_grid& grid,
                         const int32_t* cell_start_h, const int32_t* cells, int ncells, bool want_vertices,
                         bool want_faces, int threads, std::vector<HostCellOut>& out);

}  // namespace votess
