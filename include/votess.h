/*
 * votess.h -- C ABI of the MI355X (gfx950) cell-by-cell 3D Voronoi library.
 *
 * The method (paper, Summary section): sort the generators into a uniform
 * grid, find each generator's k nearest neighbours over the grid, and build
 * each Voronoi cell by clipping a bounding box with the perpendicular
 * bisectors between the generator and its neighbours, nearest first.  A
 * security-radius test certifies a cell (once every vertex lies within R of
 * the generator, no point farther than 2R can cut it; Ray et al. 2018, cited
 * by the paper), and cells that cannot be certified go to a fallback.  The
 * outputs are cell geometry and the natural-neighbour lists (Features
 * section); no combinatorial mesh is built.
 *
 * Conventions
 *  - Plain C.  Every call returns a votess_status; on error a thread-local
 *    message is available from votess_last_error().  No exception crosses
 *    the ABI.
 *  - Pointers are DEVICE pointers (HIP device memory) unless the name ends in
 *    _h (host memory).  `stream` is a hipStream_t passed as void* (NULL =
 *    the default stream); every device call is enqueued on it.
 *  - Lower-level calls (grid_sort, knn, clip_cells, features, kmodel_*)
 *    write into caller-owned buffers, validate sizes and pointers
 *    synchronously and return without synchronising the stream.  Data errors
 *    found by kernels (a point outside the box, a duplicate point) are OR-ed
 *    into a device error word that votess_ctx_errors() reads (it synchronises).
 *  - votess_tessellate allocates its outputs through the context allocator
 *    (default: hipMalloc) and synchronises the stream before returning; the
 *    caller owns the result and releases it with votess_result_free.
 *  - Index spaces: a "sorted index" is a position in the grid-sorted order
 *    produced by votess_grid_sort; an "original index" is a row of the input.
 *    Box walls appear only in vertex plane triples, as ids -1..-6 for
 *    x-, x+, y-, y+, z-, z+.
 */
#ifndef VOTESS_H
#define VOTESS_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define VOTESS_API __attribute__((visibility("default")))
#else
#define VOTESS_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VOTESS_OK = 0,
  VOTESS_EINVAL = 1,      /* bad argument (null pointer, bad size, bad box) */
  VOTESS_EOUTOFBOX = 2,   /* a point lies outside the closed box, or is NaN */
  VOTESS_EDUPLICATE = 3,  /* two points coincide exactly */
  VOTESS_ENOMEM = 4,      /* allocation failed */
  VOTESS_EHIP = 5,        /* a HIP runtime call failed */
  VOTESS_EUNRESOLVED = 6, /* a cell could be neither certified nor computed by the fallback */
  VOTESS_ECAPACITY = 7    /* an output buffer was too small */
} votess_status;

typedef enum { VOTESS_F32 = 0, VOTESS_F64 = 1 } votess_dtype;

/* Clip arithmetic.  F64: all clipping in double.  F32_RECHECK: clipping in
 * float; a plane-side test whose |margin| <= eps * scale and a security-radius
 * comparison whose |d^2 - 4R^2| <= eps * d^2 are recomputed in double on the
 * GPU from the exact inputs (needs F32 input positions). */
typedef enum { VOTESS_CLIP_F64 = 0, VOTESS_CLIP_F32_RECHECK = 1 } votess_precision;

/* Per-cell status written by votess_clip_cells. */
enum {
  VOTESS_CELL_CERTIFIED = 0, /* the cell is the exact Voronoi cell */
  VOTESS_CELL_RADIUS = 1,    /* the k-list ended before the security radius closed */
  VOTESS_CELL_CAPACITY = 2,  /* vertex / plane capacity of the kernel exceeded */
  VOTESS_CELL_UNRESOLVED = 3 /* an FP64 recheck was itself inside its error bound */
};

typedef struct votess_ctx votess_ctx;

typedef struct {
  double lo[3], hi[3]; /* closed axis-aligned box; lo < hi on every axis */
} votess_box;

/* Uniform grid over the box: cell (ix,iy,iz) has id ix + g0*(iy + g1*iz);
 * ix = clamp(floor((x - lo0) * inv_h0), 0, g0 - 1) computed in double. */
typedef struct {
  int32_t g[3];
  int64_t ncells;
  double lo[3];
  double hi[3];
  double inv_h[3];
} votess_grid;

/* ---------------------------------------------------------------- context */

/* Creates a context on HIP device `device`.  Returns NULL on failure. */
VOTESS_API votess_ctx* votess_create(int device);
VOTESS_API void votess_destroy(votess_ctx* ctx);

/* Thread-local message describing the last non-OK status (never NULL). */
VOTESS_API const char* votess_last_error(void);

/* Library version string. */
VOTESS_API const char* votess_version(void);

/* Device allocator used for votess_tessellate outputs and its internal
 * workspace.  alloc(bytes, user) returns device memory or NULL; release(ptr,
 * user) frees it.  Passing NULL restores hipMalloc/hipFree. */
typedef void* (*votess_alloc_fn)(size_t bytes, void* user);
typedef void (*votess_release_fn)(void* ptr, void* user);
VOTESS_API void votess_set_allocator(votess_ctx* ctx, votess_alloc_fn alloc, votess_release_fn release, void* user);

/* Reads (and clears) the device error word: 0 or a bit-or of
 * 1 = point outside the box / NaN, 2 = duplicate point.  Synchronises `stream`. */
VOTESS_API votess_status votess_ctx_errors(votess_ctx* ctx, void* stream, uint32_t* errors_h);

/* ---------------------------------------------------------- grid sort (a1-a3) */

/* Grid with about `pts_per_cell` points per grid cell (paper, Summary section:
 * the points are first binned into a uniform grid): per axis
 * g_a = max(1, round(ext_a * (n / (pts_per_cell * vol))^(1/3))).  Host only. */
VOTESS_API votess_status votess_grid_plan(int64_t n, const votess_box* box, double pts_per_cell, votess_grid* out_h);

/* Counting sort of the points into the grid.
 *   pts        [n,3] of dtype, row-major (input order)
 *   cell_start [ncells+1] int32 out: first sorted index of each grid cell
 *   perm       [n] int32 out: perm[s] = original index of sorted point s
 *   sorted     [n,4] of dtype out: (x, y, z, id) where id is the original
 *              index stored as the bit pattern of an int32 (F32) / int64 (F64)
 *   subinfo    [2*ncells] int32 out (nullable): sub-grids of dense cells.  A
 *              cell with more than 16 points gets a sub-grid over the
 *              bounding box [lo, lo + e] of its points: m0 x m1 x m2 sub-cells,
 *              m_a = max(1, floor(e_a s)), s = cbrt((count/2) / (e0 e1 e2)),
 *              then the largest m_a lowered until m0 m1 m2 <= count/2; a
 *              point's sub-cell is s_a = clamp(floor((x_a - lo_a) ih_a), 0,
 *              m_a - 1), ih_a = m_a / e_a, id s0 + m0 (s1 + m1 s2).
 *              subinfo[2c] = offset of the cell's record in sub_start (-1
 *              for other cells), subinfo[2c+1] = m0 m1 m2
 *   sub_start  [votess_sub_capacity(n)] int32 out (nullable with subinfo),
 *              16-byte aligned: per dense cell a record at its offset (a
 *              multiple of 4): m0, m1, m2, 0, then lo[3] and ih[3] as doubles,
 *              then the m0 m1 m2 + 1 sub-cell starts relative to cell_start[c]
 * Within a cell points are ordered by ascending original index; with
 * subinfo, a dense cell's points are ordered by (sub-cell, original index).
 * Deterministic.  Requires n < 2^31.  Points outside the box raise device
 * error bit 1. */
VOTESS_API votess_status votess_grid_sort(votess_ctx* ctx, const void* pts, votess_dtype dtype, int64_t n,
                               const votess_box* box, const votess_grid* grid, int32_t* cell_start,
                               int32_t* perm, void* sorted, int32_t* subinfo, int32_t* sub_start, void* stream);

/* Entries (int32) sub_start needs for n points: n/2 + 20n/17 + 1024. */
VOTESS_API int64_t votess_sub_capacity(int64_t n);

/* ------------------------------------------------------------- k-NN (a4) */

/* The k nearest other points of each query (paper, Summary section: the
 * neighbour search after the grid sort), by a shell-expanding search over the
 * grid.
 *   sorted, cell_start, subinfo, sub_start  from votess_grid_sort (the last
 *              two nullable: dense cells are then scanned whole)
 *   queries    [nq] sorted indices, or NULL for all n points (nq = n)
 *   dist       arithmetic of the squared distances: F64, or F32 (F32 input only)
 *   knn        [nq,k] int32 out: sorted indices ascending by (d^2, sorted index),
 *              padded with -1 when fewer than k other points exist
 * k is one of 8, 12, 16, 24, 32, 48, 64, 128, 256.  A zero distance raises device error
 * bit 2 (duplicate). */
VOTESS_API votess_status votess_knn(votess_ctx* ctx, const void* sorted, votess_dtype dtype, int64_t n,
                         const votess_grid* grid, const int32_t* cell_start, const int32_t* subinfo,
                         const int32_t* sub_start, const int32_t* queries, int64_t nq, int32_t k, votess_dtype dist,
                         int32_t* knn, void* stream);

/* ------------------------------------------------------- clipping (a6) */

typedef struct {
  votess_precision precision; /* F64 or F32_RECHECK */
  double eps;                 /* recheck threshold (F32_RECHECK), default 1e-6 */
  votess_dtype knn_dist;      /* arithmetic the k-lists were built with */
  int32_t max_nbr;            /* row stride of nbr (>= 1) */
  int32_t max_vert;           /* row stride of verts / vplanes (0: no vertices) */
  int32_t capacity;           /* 0: fast kernel, 1: large-capacity kernel */
  int32_t out_by_id;          /* 1: write row cells[t] instead of row t */
  int32_t stream;             /* 1: a cell its list does not certify keeps clipping by grid
                                 rings (unbounded k); needs k-lists in the clip precision */
  const votess_grid* grid;    /* stream only: the grid of votess_grid_sort */
  const int32_t* cell_start;  /* stream only: [ncells+1] from votess_grid_sort */
  const int32_t* subinfo;     /* stream only, nullable: sub-grids from votess_grid_sort */
  const int32_t* sub_start;
} votess_clip_opts;

/* Clips the box by the bisectors of each cell's k-list, nearest first, and
 * stops at the security radius (paper, Summary section; the radius lemma of
 * Ray et al. 2018 that it cites): before bisector m the cell is certified when
 * d_m^2 > 4 R^2 (R = farthest vertex from the generator); after the whole
 * list it is certified when d_k^2 > 4 R^2, or when the list holds all n-1
 * other points.  With opts->stream, k = 0 is allowed (knn may be NULL): the
 * fused form, where every cell is clipped straight from the grid rings
 * around its generator (the stream phase from ring 0) and no k-NN list is
 * computed or stored.
 *   cells      [nc] sorted indices (NULL = all n points, nc = n)
 *   knn        [nc,k] from votess_knn for the same cells
 *   status     [rows] u8 out: VOTESS_CELL_*
 *   nbr_count  [rows] int32 out; nbr [rows,max_nbr] int32 out: sorted indices
 *              of the natural neighbours (faces of positive area), unordered
 *   volume     [rows] double out
 *   kneeded    [rows] int32 out (nullable): least list size that certifies
 *              (valid where status == CERTIFIED)
 *   vcount     [rows] int32, verts [rows,max_vert,3] double (absolute),
 *   vplanes    [rows,max_vert,3] int32 (sorted indices or -1..-6)   (nullable)
 *   area       [rows,max_nbr] double out (nullable): area of the face shared
 *              with nbr[row, e], at the same position
 *   centroid   [rows,3] double out (nullable): cell centroid (absolute)
 * Face areas and centroids are computed in double from double vertices
 * (solved from the exact inputs on the F32_RECHECK path).  Every output of a
 * row that is not CERTIFIED is 0 (counts) or left unwritten (lists).
 * rows = n when out_by_id, else nc. */
VOTESS_API votess_status votess_clip_cells(votess_ctx* ctx, const void* sorted, votess_dtype dtype, int64_t n,
                                const votess_box* box, const int32_t* cells, int64_t nc, const int32_t* knn,
                                int32_t k, const votess_clip_opts* opts, uint8_t* status, int32_t* nbr_count,
                                int32_t* nbr, double* volume, int32_t* kneeded, int32_t* vcount, double* verts,
                                int32_t* vplanes, double* area, double* centroid, void* stream);

/* ------------------------------------------------------ whole tessellation */

typedef struct votess_kmodel votess_kmodel;

typedef struct {
  int32_t k0;               /* first list size (default 32); 0: the fused form (no k-NN pass, every
                               cell clipped from the grid rings; needs gpu_stream, no kmodel) */
  int32_t max_gpu_retries;  /* doublings of k on the GPU after the first pass, up to k = 256
                               (default 1; the learned first pass ends at k = 64) */
  double pts_per_cell;      /* grid density (default 2) */
  votess_precision precision;
  double eps;               /* default 1e-6 */
  votess_kmodel* kmodel;    /* learned-k: per-cell list size from the network (nullable).  The
                               first pass lists the 64 nearest of every cell once; the features
                               read each list's first 16 entries and a cell in bucket k is
                               clipped by its list's first k entries */
  double tau;               /* learned-k decision threshold (default 0.9) */
  int32_t want_vertices;    /* 1: also return vertices */
  int32_t index_space;      /* 0: original indices (default), 1: sorted indices */
  int32_t host_fallback;    /* 1 (default): uncertified cells go to the CPU fallback */
  int32_t host_threads;     /* 0: all hardware threads */
  int32_t force_fail_every; /* >0: testing aid, every m-th cell skips the GPU passes */
  int32_t gpu_stream;       /* 1 (default): the last GPU pass keeps clipping uncertified
                               cells by grid rings (no bound on k) instead of leaving
                               them to the host */
  int32_t want_faces;       /* 1: also return face areas and cell centroids */
  int32_t periodic;         /* 1: the box is a 3-torus (points in [lo, hi)): every cell is the region
                               nearer its generator than any periodic image of any point; a row lists
                               the index of each point whose image shares a face, once per image.
                               Clipping is FP64 (a float point's periodic image is not a float in
                               general).  Not with kmodel, want_vertices, index_space 1 or
                               force_fail_every. */
} votess_params;

#define VOTESS_MAX_PASSES 8
typedef struct {
  int32_t npasses;
  int32_t pass_k[VOTESS_MAX_PASSES];
  int64_t pass_cells[VOTESS_MAX_PASSES];
  int64_t pass_failed[VOTESS_MAX_PASSES];
  int64_t capacity_cells;   /* cells sent to the large-capacity kernel */
  int64_t fallback_cells;   /* cells computed on the host */
  int64_t unresolved_cells; /* cells whose FP64 recheck stayed inside its bound */
  int64_t rechecks;         /* F32_RECHECK: predicates redone in FP64 (all passes) */
  int64_t refined_cells;    /* F32_RECHECK: thin cells whose outputs were solved in FP64 */
  int64_t streamed_cells;   /* cells certified by the GPU stream phase */
  int64_t bucket_cells[8];  /* learned-k: cells per bucket */
  double ms_sort, ms_knn, ms_clip, ms_features, ms_mlp, ms_assemble, ms_fallback, ms_total;
  /* per pass: cells its list left uncertified that went on into the stream
   * phase (pass_failed counts the cells still uncertified after it) */
  int64_t pass_streamed[VOTESS_MAX_PASSES];
} votess_stats;

typedef struct {
  int64_t n, nnz;
  int64_t* row_ptr; /* [n+1] device */
  int32_t* col;     /* [nnz] device: neighbours of each row, ascending */
  double* volume;   /* [n] device */
  int64_t nvert;
  int64_t* vrow_ptr; /* [n+1] device (want_vertices) */
  double* vxyz;      /* [nvert,3] device */
  int32_t* vplanes;  /* [nvert,3] device: sorted plane ids per vertex */
  double* area;      /* [nnz] device (want_faces): area of the face shared with col[e] */
  double* centroid;  /* [n,3] device (want_faces): cell centroids */
  votess_stats stats;
} votess_result;

VOTESS_API void votess_params_default(votess_params* p_h);

/* One call (paper, Features section: the library function that computes the
 * tessellation and returns the natural neighbours as a jagged array): grid
 * sort, k-NN, clip with the GPU retry ladder (k, 2k, ...), then the host
 * fallback (exact CPU cell, unbounded k) for cells still uncertified, then
 * CSR assembly.  `pts` [n,3] dtype device, input order.
 * Rows of the result are in original order (or sorted order with
 * index_space = 1), neighbours ascending; with want_faces, area[e] is the
 * area of the face the row's cell shares with col[e], and centroid the
 * cells' centres of mass, both computed in double.  The result's device
 * buffers belong to the caller: free them with votess_result_free. */
VOTESS_API votess_status votess_tessellate(votess_ctx* ctx, const void* pts, votess_dtype dtype, int64_t n,
                                const votess_box* box, const votess_params* params, votess_result* out_h,
                                void* stream);
VOTESS_API void votess_result_free(votess_ctx* ctx, votess_result* res_h);

/* -------------------------------------------- learned list size (k-model) */

#define VOTESS_NFEAT 12
#define VOTESS_NHID 64
#define VOTESS_NBUCKET 7
/* Buckets of list sizes the network chooses from. */
extern VOTESS_API const int32_t votess_buckets[VOTESS_NBUCKET]; /* {8,12,16,24,32,48,64} */

/* Network 12 -> 64 -> 64 -> 7, ReLU, BF16 weights and activations with FP32
 * accumulation (MFMA), FP32 master weights and Adam state on the device.
 * Parameter layout (flat FP32, 5447 values): W1[64][12] b1[64] W2[64][64]
 * b2[64] W3[7][64] b3[7].  Feature standardisation mean[12], std[12]. */
#define VOTESS_NPARAM 5447
VOTESS_API votess_kmodel* votess_kmodel_create(votess_ctx* ctx, uint64_t seed);
VOTESS_API void votess_kmodel_destroy(votess_kmodel* m);
VOTESS_API votess_status votess_kmodel_set_params(votess_kmodel* m, const float* params_h, const float* mean_h,
                                       const float* std_h);
VOTESS_API votess_status votess_kmodel_get_params(votess_kmodel* m, float* params_h, float* mean_h, float* std_h);

/* Features of each query from a 16-NN pass: 12 floats per query (see the
 * design notes for the definitions).  F32 sorted input only. */
VOTESS_API votess_status votess_features(votess_ctx* ctx, const void* sorted, int64_t n, const votess_grid* grid,
                              const int32_t* cell_start, const int32_t* subinfo, const int32_t* sub_start,
                              const int32_t* queries, int64_t nq, float* feats, void* stream);

/* The same features as votess_features, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the 16-NN lists live in a static device
 * array of the library (votess_features_noalloc_max() queries, 4 MiB per
 * device, held until the process ends), so the call allocates nothing.
 * nq above that maximum is EINVAL.  Every call on a device shares that
 * device's array: calls that overlap on one GPU (different streams or
 * threads) race.  Enqueued on `stream`; does not synchronise. */
VOTESS_API int64_t votess_features_noalloc_max(void);
VOTESS_API votess_status votess_features_noalloc(votess_ctx* ctx, const void* sorted, int64_t n,
                                                 const votess_grid* grid, const int32_t* cell_start,
                                                 const int32_t* subinfo, const int32_t* sub_start,
                                                 const int32_t* queries, int64_t nq, float* feats, void* stream);

/* logits [nq,7] float = network(standardised feats). */
VOTESS_API votess_status votess_kmodel_forward(votess_kmodel* m, const float* feats, int64_t nq, float* logits, void* stream);

/* Softmax cross-entropy gradient of the mean loss over the batch w.r.t. the
 * parameters (flat layout as above), computed at the BF16-rounded weights and
 * activations.  grads [5447] float out, loss [1] float out (device). */
VOTESS_API votess_status votess_kmodel_grad(votess_kmodel* m, const float* feats, const uint8_t* labels, int64_t nb,
                                 float* grads, float* loss, void* stream);

/* One Adam step (beta 0.9/0.999, eps 1e-8) on a batch; loss [1] out (nullable). */
VOTESS_API votess_status votess_kmodel_train_step(votess_kmodel* m, const float* feats, const uint8_t* labels, int64_t nb,
                                       float lr, float* loss, void* stream);

/* Bucket per query: least b with P(label <= b) >= tau; bucket [nq] u8 out. */
VOTESS_API votess_status votess_kmodel_choose(votess_kmodel* m, const float* feats, int64_t nq, float tau, uint8_t* bucket,
                                   void* stream);

/* Training labels from the method's own run (the label-recording clip of
 * votess_clip_cells with a 64-long list: its status and kneeded outputs):
 * labels[i] = least b with votess_buckets[b] >= kneeded[i], or the largest
 * bucket (6) when status[i] is not CERTIFIED or the cell needed more than 64.
 * [n] device buffers; enqueued on `stream`. */
VOTESS_API votess_status votess_kmodel_labels(votess_ctx* ctx, const uint8_t* status, const int32_t* kneeded,
                                              int64_t n, uint8_t* labels, void* stream);

/* Feature standardisation fitted on the device: mean and population
 * standard deviation (plus 1e-6) of each of the 12 features over feats
 * [n,12], summed in double in a fixed order (deterministic).  Sets the
 * model's mean/std; synchronises `stream`. */
VOTESS_API votess_status votess_kmodel_fit_norm(votess_kmodel* m, const float* feats, int64_t n, void* stream);

/* Versioned k-model blob (host memory): a header (magic "VTKM", version,
 * network shape, bucket sizes, tau), the 5447 FP32 parameters, mean[12],
 * std[12] and an FNV-1a checksum.  votess_kmodel_save writes it to blob_h
 * (cap bytes; *len_h = votess_kmodel_blob_size(); blob_h NULL only reports
 * the size, too small a cap is ECAPACITY) and synchronises the device.
 * votess_kmodel_load checks magic, version, shape, buckets and checksum
 * (EINVAL otherwise), creates a model on ctx holding those parameters (Adam
 * state zero) into *out_h, and returns the saved tau in *tau_h (nullable). */
VOTESS_API size_t votess_kmodel_blob_size(void);
VOTESS_API votess_status votess_kmodel_save(votess_kmodel* m, double tau, void* blob_h, size_t cap, size_t* len_h);
VOTESS_API votess_status votess_kmodel_load(votess_ctx* ctx, const void* blob_h, size_t len, votess_kmodel** out_h,
                                            double* tau_h);

#ifdef __cplusplus
}
#endif
#endif /* VOTESS_H */
