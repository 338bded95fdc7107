// Cell clipping with the security-radius certificate (paper, Summary section:
// each cell starts as a bounding box that is cut, one neighbour at a time, by
// the bisector plane between the generator and that neighbour, and a
// security-radius condition proves the result complete; the radius lemma is
// the one of Ray et al. 2018, cited by the paper).
//
// MI355X design
//  * A group of L lanes owns one cell; a 64-lane wave (= one workgroup) holds
//    64/L cells.  Lane j of a group handles vertex slots t = j, j+L, ...
//  * The polyhedron is kept in dual form in LDS: a list of clipping planes
//    (box walls + bisectors, at most PMAX alive at once, slots recycled) and a
//    list of triangles, one per vertex, each naming its three planes in
//    counter-clockwise order seen from outside.  Vertex positions are cached
//    next to the triangles, in seed-relative coordinates.
//  * Clipping by plane m: every lane tests its vertices (n.v > c means
//    outside), a ballot tells the group whether anything is cut.  For a cut,
//    the directed dual edges of the removed triangles are marked in a per-cell
//    bit matrix; an edge whose twin is unmarked lies on the boundary of the
//    removed region and becomes a new triangle (a, b, m).  New vertices are
//    solved from their three planes (Cramer), so no error accumulates from
//    earlier vertices.  Then the alive-plane mask and the radius R^2 are
//    rebuilt with group reductions.
//  * Certificate: before plane m, the cell is final when d_m^2 > 4 R^2; after
//    the list, when d_k^2 > 4 R^2 or the list holds every other point.
//  * Volume: sum over vertices of corner terms det(F_f, v, e_fh - e_fg) / 6,
//    with F_f the foot of the seed on face f and e_fg the point of line f^g
//    nearest to the seed (a fan of each face from its foot, split at the edge
//    anchors), accumulated in double.
//  * Optional per-face outputs, in double from double vertices: the area of
//    each neighbour's face (the same corner terms, per face) and the cell
//    centroid (each corner term split into two signed tetrahedra from the
//    seed, weighted by their corner means).
//  * F32_RECHECK: tests and radii in float; a plane-side test whose margin is
//    below eps of its scale, and a certificate comparison with
//    |d^2 - 4 R^2| <= eps d^2, are redone in double from the exact inputs.
#include "internal.h"
#include "device_common.h"

#include <cfloat>

namespace votess {
namespace {

constexpr unsigned kEmpty = 0xFFFFFFFFu;
constexpr int ST_RUN = -1;

struct ClipArgs {
  const void* rec;
  int n;
  double lo0, lo1, lo2, hi0, hi1, hi2;
  const int* cells;
  int nc;
  const int* knn;
  int k;
  int kstride;    // entries per list row
  int knn_by_id;  // list row of a cell: its sorted id (else its position in cells)
  double eps;
  double dmargin;  // applied to d^2 in certificate tests (k-lists built in float)
  int max_nbr, max_vert, out_by_id;
  uint8_t* status;
  int* nbr_count;
  int* nbr;
  double* volume;
  int* kneeded;
  int* vcount;
  double* verts;
  int* vplanes;
  double* area;      // [rows, max_nbr] next to nbr (nullable)
  double* centroid;  // [rows, 3] (nullable)
  double* r2out;     // [rows] (nullable): R^2 of the certified cell (an upper bound on the float path)
  unsigned long long* counters;
  // stream phase (cells the list did not certify keep clipping by grid rings)
  int stream;
  const int* cell_start;
  GridDev grid;
  SubGrid sub;  // sub-grids of dense cells (info null: none)
};

template <typename R>
struct V3 {
  R x, y, z;
};

template <typename R>
__device__ __forceinline__ V3<R> cross(const V3<R>& a, const V3<R>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename R>
__device__ __forceinline__ R dot(const V3<R>& a, const V3<R>& b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}

// Vertex of planes a, b, c: solve [na; nb; nc] x = [ca, cb, cc].
template <typename R>
__device__ __forceinline__ V3<R> solve3(const V3<R>& na, R ca, const V3<R>& nb, R cb, const V3<R>& nc, R cc) {
  const V3<R> bc = cross(nb, nc), ca_ = cross(nc, na), ab = cross(na, nb);
  const R det = dot(na, bc);
  const R inv = R(1) / det;
  return {(ca * bc.x + cb * ca_.x + cc * ab.x) * inv, (ca * bc.y + cb * ca_.y + cc * ab.y) * inv,
          (ca * bc.z + cb * ca_.z + cc * ab.z) * inv};
}

// c - n.v as if in twice the working precision: each product split exactly
// by an FMA, each sum by an error-free two-sum, the error terms added last.
// The residual of a vertex of nearly singular planes survives cancellation.
__device__ __forceinline__ double residual2(const V3<double>& n, double c, const V3<double>& v) {
#pragma clang fp contract(off)
  double s = c, err = 0.0;
  const double a[3] = {n.x, n.y, n.z}, b[3] = {v.x, v.y, v.z};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double p = a[i] * b[i];
    const double ep = fma(a[i], b[i], -p);  // a b = p + ep exactly
    const double t = s - p;                 // s - p = t + es exactly
    const double z = t - s;
    const double es = (s - (t - z)) + (-p - z);
    s = t;
    err += es - ep;
  }
  return s + err;
}

// The same residual for a bisector plane (n, |n|^2 / 2) without rounding its
// offset: c - n.v = sum_i n_i (n_i / 2 - v_i), each difference split by a
// two-sum, each product by an FMA.  The double offset |n|^2 / 2 is rounded by
// u c, which a vertex of nearly parallel planes amplifies by its
// conditioning; this residual has no such term (n itself is exact for float
// inputs).
__device__ __forceinline__ double residual_bis(const V3<double>& n, const V3<double>& v) {
#pragma clang fp contract(off)
  double s = 0.0, err = 0.0;
  const double a[3] = {n.x, n.y, n.z}, b[3] = {v.x, v.y, v.z};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double h = 0.5 * a[i];  // exact
    const double d = h - b[i];    // h - b = d + ed exactly
    const double z0 = d - h;
    const double ed = (h - (d - z0)) + (-b[i] - z0);
    const double p = a[i] * d;
    const double ep = fma(a[i], d, -p);  // a d = p + ep exactly
    const double t = s + p;              // s + p = t + es exactly
    const double z = t - s;
    const double es = (s - (t - z)) + (p - z);
    s = t;
    err += es + ep + a[i] * ed;
  }
  return s + err;
}

// Vertex of three planes, refined once against its accurate residual (for
// the planes flagged as bisectors, with their offsets taken exactly): a few
// ulps of |v| unless the normals are singular to within ~u.
__device__ __forceinline__ V3<double> solve3_refined(const V3<double>& na, double ca, bool ba, const V3<double>& nb,
                                                     double cb, bool bb, const V3<double>& nc, double cc, bool bc_) {
  const V3<double> bc = cross(nb, nc), ca_ = cross(nc, na), ab = cross(na, nb);
  const double inv = 1.0 / dot(na, bc);
  auto apply = [&](double x, double y, double z) -> V3<double> {
    return {(x * bc.x + y * ca_.x + z * ab.x) * inv, (x * bc.y + y * ca_.y + z * ab.y) * inv,
            (x * bc.z + y * ca_.z + z * ab.z) * inv};
  };
  const V3<double> v = apply(ca, cb, cc);
  const V3<double> d = apply(ba ? residual_bis(na, v) : residual2(na, ca, v), bb ? residual_bis(nb, v) : residual2(nb, cb, v),
                             bc_ ? residual_bis(nc, v) : residual2(nc, cc, v));
  return {v.x + d.x, v.y + d.y, v.z + d.z};
}

// Float vertex of three planes with a first-order forward error bound (max
// norm): rounding of the cross products, the sums, the division and of the
// plane data (normals may be off by an ulp, offsets by two).
__device__ __forceinline__ V3<float> solve3_err(const V3<float>& na, float ca, const V3<float>& nb, float cb,
                                                const V3<float>& nc, float cc, float& err) {
  const V3<float> bc = cross(nb, nc), ca_ = cross(nc, na), ab = cross(na, nb);
  auto perm = [](const V3<float>& a, const V3<float>& b) {
    return V3<float>{fabsf(a.y * b.z) + fabsf(a.z * b.y), fabsf(a.z * b.x) + fabsf(a.x * b.z),
                     fabsf(a.x * b.y) + fabsf(a.y * b.x)};
  };
  const V3<float> pbc = perm(nb, nc), pca = perm(nc, na), pab = perm(na, nb);
  const float det = dot(na, bc);
  const float inv = 1.0f / det;
  const V3<float> v = {(ca * bc.x + cb * ca_.x + cc * ab.x) * inv, (ca * bc.y + cb * ca_.y + cc * ab.y) * inv,
                       (ca * bc.z + cb * ca_.z + cc * ab.z) * inv};
  const float u8 = 8.0f * (0.5f * FLT_EPSILON);
  const float dD = u8 * (fabsf(na.x) * pbc.x + fabsf(na.y) * pbc.y + fabsf(na.z) * pbc.z);
  const float aa = fabsf(ca), ab_ = fabsf(cb), ac = fabsf(cc);
  const float ai = fabsf(inv);
  const float ex = (u8 * (aa * pbc.x + ab_ * pca.x + ac * pab.x) + fabsf(v.x) * dD) * ai + FLT_EPSILON * fabsf(v.x);
  const float ey = (u8 * (aa * pbc.y + ab_ * pca.y + ac * pab.y) + fabsf(v.y) * dD) * ai + FLT_EPSILON * fabsf(v.y);
  const float ez = (u8 * (aa * pbc.z + ab_ * pca.z + ac * pab.z) + fabsf(v.z) * dD) * ai + FLT_EPSILON * fabsf(v.z);
  err = fmaxf(ex, fmaxf(ey, ez));
  return v;
}

template <typename M>
__device__ __forceinline__ M bitm(int i) {
  return M(1) << i;
}

// Lane moves inside a row of 16 lanes by DPP, which stays in the vector ALU
// (controls: quad_perm [1,0,3,2] = 0xB1 takes lane ^ 1, [2,3,0,1] = 0x4E
// lane ^ 2, [3,2,1,0] = 0x1B reverses a quad; row_shr:n = 0x110 + n takes
// lane - n; row_mirror = 0x140 takes lane 15 - i, row_half_mirror = 0x141
// lane 7 - i within each eight).  Moves across rows use the LDS permute.
template <int CTRL>
__device__ __forceinline__ unsigned dpp_mov(unsigned v) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, true);
}
// the word of lane ^ m (m is a constant once the callers' loops unroll)
__device__ __forceinline__ unsigned xor_word(unsigned v, int m) {
  switch (m) {
    case 1: return dpp_mov<0xB1>(v);
    case 2: return dpp_mov<0x4E>(v);
    case 4: return dpp_mov<0x141>(dpp_mov<0x1B>(v));  // i -> 3 - i in the quad, then 7 - i
    case 8: return dpp_mov<0x140>(dpp_mov<0x141>(v));  // 7 - i in the eight, then 15 - i
    default: return (unsigned)__shfl_xor((int)v, m, 64);
  }
}
// the word of lane - n (n = 1, 2, 4, 8; lanes below n of the row receive 0)
__device__ __forceinline__ unsigned up_word(unsigned v, int n) {
  switch (n) {
    case 1: return dpp_mov<0x111>(v);
    case 2: return dpp_mov<0x112>(v);
    case 4: return dpp_mov<0x114>(v);
    default: return dpp_mov<0x118>(v);
  }
}
// value of lane ^ m inside groups of w lanes; every lane of the group is
// active
template <typename T>
__device__ __forceinline__ T shfl_xor_w(T v, int m, int w) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "one or two words");
  if (m >= 16) return __shfl_xor(v, m, w);
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, xor_word(__builtin_bit_cast(unsigned, v), m));
  } else {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned long long r =
        ((unsigned long long)xor_word((unsigned)(u >> 32), m) << 32) | xor_word((unsigned)u, m);
    return __builtin_bit_cast(T, r);
  }
}

// FP64 plane of a cell (generator p): the bisector with point `id` (>= 0) or
// box wall -id-1 (x-, x+, y-, y+, z-, z+); n . x <= c relative to p.  All
// arguments are values, so that no selection below goes through memory.
template <typename Rec4>
__device__ __forceinline__ void plane64_of(int id, const Rec4* rec, double px, double py, double pz, double lo0,
                                           double lo1, double lo2, double hi0, double hi1, double hi2, V3<double>& n,
                                           double& c) {
  if (id >= 0) {
    const Rec4 q = rec[id];
    n = {(double)q.x - px, (double)q.y - py, (double)q.z - pz};
    c = 0.5 * dot(n, n);
  } else {
    const int w = -id - 1, ax = w >> 1;
    const bool hi = w & 1;
    const double lo_a = ax == 0 ? lo0 : (ax == 1 ? lo1 : lo2);
    const double hi_a = ax == 0 ? hi0 : (ax == 1 ? hi1 : hi2);
    const double p_a = ax == 0 ? px : (ax == 1 ? py : pz);
    const double sgn = hi ? 1.0 : -1.0;
    n = {ax == 0 ? sgn : 0.0, ax == 1 ? sgn : 0.0, ax == 2 ? sgn : 0.0};
    c = hi ? hi_a - p_a : p_a - lo_a;
  }
}

// The fast kernels (TMAX = 64) are held to 3 waves per SIMD: the compiler
// would otherwise give the stream variants ~225 VGPRs (2 waves), and with
// the third wave hiding load latency they run ~20% faster despite ~90 bytes
// per lane of spills.
template <typename P, typename R, int L, int TMAX, int PMAX, bool RECHECK, bool STREAM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(TMAX <= 64 ? 3 : 1))) void k_clip(ClipArgs a) {
  using Rec4 = typename Rec<P>::type;
  using M = typename std::conditional<(PMAX <= 32), unsigned, unsigned long long>::type;
  constexpr int G = 64 / L;
  constexpr int S = TMAX / L;
  constexpr int TP = TMAX + 1;
  constexpr unsigned long long LOWL = (L == 64) ? ~0ull : ((1ull << L) - 1);
  constexpr M PFULL = (PMAX == 8 * (int)sizeof(M)) ? ~M(0) : ((M(1) << PMAX) - 1);
  static_assert(S <= 32, "slot mask is 32 bits");
  static_assert(TMAX <= 256, "vertex slots are numbered in one byte");

  __shared__ R vx[G * TP], vy[G * TP], vz[G * TP];
  __shared__ unsigned tri[G * TP];
  __shared__ R pnx[G * PMAX], pny[G * PMAX], pnz[G * PMAX], pnc[G * PMAX];
  __shared__ int pid[G * PMAX];
  __shared__ M omask[G * PMAX];
  __shared__ unsigned snew[G * PMAX];
  __shared__ unsigned char sslot[G * PMAX];  // free slot taken by new triangle r
  constexpr int TE = RECHECK ? G * TP : 1;
  __shared__ float verr[TE];  // forward error bound of each float vertex
  // stream phase of the float clip: radius of each vertex's ball through the
  // seed, widened past the vertex's error bound and the rounding of the tests
  // that use it (the double clip recomputes it where needed: measured faster)
  constexpr bool kVrad = STREAM && RECHECK;
  constexpr int VRD = kVrad ? G * TP : 1;
  __shared__ float vrad[VRD];
  // stream phase: vertex slots whose ball can reach the current grid row /
  // dense cell (see below)
  constexpr int RL = STREAM ? G * TMAX : 1;
  __shared__ unsigned char relR[RL], relD[RL];
  // stream phase: geometry of the dense cell being scanned (cell corner,
  // sub-grid origin and sub-cell widths), per group
  constexpr int DG = STREAM ? G * 9 : 1;
  __shared__ double dgeo[DG];
  // stream phase: the flower box in coordinates, per group (read only when a
  // dense cell is entered, so it need not occupy registers)
  constexpr int FWG = STREAM ? G * 6 : 1;
  __shared__ double fwbox[FWG];
  // stream phase: point ranges of up to L sub-rows of the dense cell being
  // scanned (offsets into the cell), per group
  constexpr int SRL = STREAM ? G * L : 1;
  __shared__ int2 srl[SRL];
  // stream phase: the group's enumeration state (grid ring, x-run, dense
  // sub-block, flower box in cells).  Every value is the same for all lanes
  // of a group; held here rather than in registers, which the rest of the
  // kernel needs.
  struct Enum {
    int fb0, fb1, fb2, fb3, fb4, fb5;
    int rr, zz, yy, part, zhi, ylo, yhi;
    int rx, rx1, rrow;
    int dm, dm0, dm1, dbase, dsx0, dsx1, dsy0, dsy1, dsz0, dsz1, dsto;
    int dq1, dq2, kyn, kzn, dq, dqn, srn, srp;
  };
  __shared__ Enum senum[STREAM ? G : 1];

  const Rec4* rec = (const Rec4*)a.rec;
  const int lane = threadIdx.x;
  const int g = lane / L, j = lane % L;
  const int gb = g * L;
  const int vb = g * TP, pb = g * PMAX;
  // XCD-aware block order (blocks are dealt round-robin over the eight XCDs):
  // launched block b clips logical block (b mod 8) per + b / 8, so each XCD
  // takes a contiguous stretch of grid-sorted cells, whose neighbours its L2
  // then holds
  const int nblk = (a.nc + G - 1) / G, per = (nblk + 7) / 8;
  const int lblk = (int)(blockIdx.x % 8u) * per + (int)(blockIdx.x / 8u);
  if (lblk >= nblk) return;  // the whole (one-wave) block
  const long long t_idx = (long long)lblk * G + g;
  const bool have = t_idx < a.nc;
  const int sid = have ? (a.cells ? a.cells[t_idx] : (int)t_idx) : 0;
  const int row = a.out_by_id ? sid : (int)t_idx;
  const Rec4 pr = rec[sid];
  const double p64x = pr.x, p64y = pr.y, p64z = pr.z;
  const R px = (R)pr.x, py = (R)pr.y, pz = (R)pr.z;

  auto group_any = [&](bool v) -> bool { return ((__ballot(v) >> gb) & LOWL) != 0ull; };
  auto gor = [&](M v) -> M {
#pragma unroll
    for (int o = 1; o < L; o <<= 1) v |= shfl_xor_w(v, o, L);
    return v;
  };
  auto gmax = [&](R v) -> R {
#pragma unroll
    for (int o = 1; o < L; o <<= 1) v = fmax(v, shfl_xor_w(v, o, L));
    return v;
  };
  auto gmaxi = [&](int v) -> int {
#pragma unroll
    for (int o = 1; o < L; o <<= 1) v = max(v, shfl_xor_w(v, o, L));
    return v;
  };
  auto gsumd = [&](double v) -> double {
#pragma unroll
    for (int o = 1; o < L; o <<= 1) v += shfl_xor_w(v, o, L);
    return v;
  };
  auto gexcl = [&](int v, int& tot) -> int {
    int x = v;
#pragma unroll
    for (int o = 1; o < L; o <<= 1) {
      const int y = L <= 16 ? (int)up_word((unsigned)x, o) : __shfl_up(x, o, L);
      if (j >= o) x += y;
    }
    tot = __shfl(x, L - 1, L);
    return x - v;
  };

  // FP64 plane of slot f, from the exact inputs (used by the recheck).
  const double blo0 = a.lo0, blo1 = a.lo1, blo2 = a.lo2, bhi0 = a.hi0, bhi1 = a.hi1, bhi2 = a.hi2;
  auto plane64 = [&](int f, V3<double>& n, double& c) {
    plane64_of(pid[pb + f], rec, p64x, p64y, p64z, blo0, blo1, blo2, bhi0, bhi1, bhi2, n, c);
  };
  auto vertex64 = [&](unsigned u) -> V3<double> {
    V3<double> na, nb, nc;
    double ca, cb, cc;
    plane64(u & 0xFF, na, ca);
    plane64((u >> 8) & 0xFF, nb, cb);
    plane64((u >> 16) & 0xFF, nc, cc);
    return solve3<double>(na, ca, nb, cb, nc, cc);
  };

  // ---- initial cell: the box, in seed-relative coordinates
  for (int t = j; t < TMAX; t += L) tri[vb + t] = kEmpty;
  for (int f = j; f < PMAX; f += L) omask[pb + f] = 0;
  const R lx = (R)(a.lo0 - p64x), hx = (R)(a.hi0 - p64x);
  const R ly = (R)(a.lo1 - p64y), hy = (R)(a.hi1 - p64y);
  const R lz = (R)(a.lo2 - p64z), hz = (R)(a.hi2 - p64z);
  for (int v = j; v < 8; v += L) {
    const int bx = v & 1, by = (v >> 1) & 1, bz = (v >> 2) & 1;
    vx[vb + v] = bx ? hx : lx;
    vy[vb + v] = by ? hy : ly;
    vz[vb + v] = bz ? hz : lz;
    const unsigned X = bx, Y = 2 + by, Z = 4 + bz;
    // (X, Y, Z) is counter-clockwise seen from outside iff an odd number of
    // the three coordinates are on the high side
    tri[vb + v] = ((bx + by + bz) & 1) ? (X | (Y << 8) | (Z << 16)) : (X | (Z << 8) | (Y << 16));
    if (RECHECK) verr[vb + v] = FLT_EPSILON * fmax(fabs((double)vx[vb + v]), fmax(fabs((double)vy[vb + v]), fabs((double)vz[vb + v])));
  }
  for (int f = j; f < 6; f += L) {
    const int ax = f >> 1;
    const bool hi = f & 1;
    const R sgn = hi ? R(1) : R(-1);
    pnx[pb + f] = ax == 0 ? sgn : R(0);
    pny[pb + f] = ax == 1 ? sgn : R(0);
    pnz[pb + f] = ax == 2 ? sgn : R(0);
    pnc[pb + f] = ax == 0 ? (hi ? hx : -lx) : (ax == 1 ? (hi ? hy : -ly) : (hi ? hz : -lz));
    pid[pb + f] = -(f + 1);
  }
  int st = have ? ST_RUN : VOTESS_CELL_CERTIFIED;
  int H = 8;
  M alive = M(0x3F);
  R R2 = fmax(lx * lx, hx * hx) + fmax(ly * ly, hy * hy) + fmax(lz * lz, hz * hz);
  // float path: bounds on the true R^2 from each vertex's forward error bound,
  // R2lo <= R^2 <= R2hi; a radius test is rechecked only between them
  float R2hi, R2lo;
  {
    const double r = sqrt((double)R2), e = FLT_EPSILON * r;
    R2hi = (float)((r + e) * (r + e) * (1.0 + 1e-6));
    R2lo = (float)((r - e) * (r - e) * (1.0 - 1e-6));
  }
  // radius predicates of the float path: certain / uncertain (else certainly not)
  auto rad_certain = [&](R dd2) -> bool {
    return (double)dd2 * a.dmargin * (1.0 - a.eps) > 4.0 * (double)R2hi;
  };
  auto rad_uncertain = [&](R dd2) -> bool {
    return !rad_certain(dd2) && (double)dd2 * a.dmargin * (1.0 + a.eps) > 4.0 * (double)R2lo;
  };
  bool fmarg = false;  // the last F test was inside its recheck window
  bool in_stream = false;  // the group's cell is in the stream phase (vrad kept)
  // |v| (1 + 1e-5) + 4 verr.  verr bounds each coordinate of the float
  // vertex, so the true ball's centre lies within verr per axis and its radius
  // within sqrt(3) verr: 4 verr > (1 + sqrt(3)) verr covers both; the relative
  // 1e-5 covers the rounding of this radius and of the box-ball tests, made in
  // the clip's precision.
  auto ball_rad = [&](R X, R Y, R Z, float e) -> R {
    if constexpr (sizeof(R) == 4) {
      return sqrtf(X * X + Y * Y + Z * Z) * (1.0f + 1e-5f) + 4.0f * e;
    } else {
      return sqrt(X * X + Y * Y + Z * Z) * (1.0 + 1e-5);
    }
  };
  // the ball radius of vertex slot t (at X, Y, Z)
  auto vball = [&](int t, R X, R Y, R Z) -> R {
    if constexpr (kVrad) {
      return vrad[vb + t];
    } else {
      return ball_rad(X, Y, Z, RECHECK ? verr[vb + t] : 0.0f);
    }
  };
  bool fprev = false;
  int kneed = 0;
  int nrecheck = 0;
  __syncthreads();

  // Recheck of the security radius in double: R^2 from vertices solved in FP64.
  auto radius64 = [&](bool need) -> double {
    double r2 = 0.0;
    if (need) {
      for (int t = j; t < H; t += L) {
        const unsigned u = tri[vb + t];
        if (u == kEmpty) continue;
        const V3<double> v = vertex64(u);
        r2 = fmax(r2, dot(v, v));
      }
    }
#pragma unroll
    for (int o = 1; o < L; o <<= 1) r2 = fmax(r2, shfl_xor_w(r2, o, L));
    return r2;
  };
  const double kDmargin = a.dmargin;

  // Tests plane (n, c) of candidate nb against every vertex and, if it cuts,
  // replaces the removed triangles.  Called by every lane (wave-uniform).
  // Always inlined: as a call, its captures live in scratch memory.
  auto apply_plane = [&](bool run, R nx, R ny, R nz, R c, R d2, int nb) __attribute__((always_inline)) {
    // ---- test the plane against every vertex
    unsigned out = 0;
    bool unresolved = false;
    if (run) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int t = j + L * s;
        if (t < H) {
          const unsigned u = tri[vb + t];
          if (u != kEmpty) {
            const R X = vx[vb + t], Y = vy[vb + t], Z = vz[vb + t];
            const R sv = nx * X + ny * Y + nz * Z - c;
            bool o = sv > R(0);
            if (RECHECK) {
              const R scale = fabs(nx * X) + fabs(ny * Y) + fabs(nz * Z) + c;
              const R nrm1 = fabs(nx) + fabs(ny) + fabs(nz);
              if (fabs(sv) <= (R)a.eps * scale + nrm1 * (R)verr[vb + t]) {
                const Rec4 q = rec[nb];
                const V3<double> n64 = {(double)q.x - p64x, (double)q.y - p64y, (double)q.z - p64z};
                const double c64 = 0.5 * dot(n64, n64);
                const V3<double> v64 = vertex64(u);
                const double s64 = dot(n64, v64) - c64;
                const double sc64 = fabs(n64.x * v64.x) + fabs(n64.y * v64.y) + fabs(n64.z * v64.z) + c64;
                if (fabs(s64) <= 1e-12 * sc64) unresolved = true;
                o = s64 > 0.0;
                ++nrecheck;
              }
            }
            if (o) out |= 1u << s;
          }
        }
      }
    }
    if (RECHECK) {
      if (group_any(unresolved) && run) {
        st = VOTESS_CELL_UNRESOLVED;
        run = false;
        out = 0;
      }
    }
    const bool any_out = group_any(out != 0u);  // ballot by every lane
    const bool cut = run && any_out;
    if (!__any(cut)) {
      if (run) {  // no cut: R unchanged and d_m^2 <= 4 R^2 (E_m was false)
        fprev = false;
        fmarg = false;
      }
      return;
    }

    // ---- cut: new plane slot
    int ps = -1;
    bool doit = cut;
    if (doit) {
      const M fr = ~alive & PFULL;
      if (fr == M(0)) {
        st = VOTESS_CELL_CAPACITY;
        doit = false;
      } else {
        ps = (sizeof(M) == 4) ? (__ffs((unsigned)fr) - 1) : (__ffsll((unsigned long long)fr) - 1);
      }
    }
    if (doit && j == 0) {
      pnx[pb + ps] = nx;
      pny[pb + ps] = ny;
      pnz[pb + ps] = nz;
      pnc[pb + ps] = c;
      pid[pb + ps] = nb;
    }
    if (!doit) out = 0;
    // mark the directed dual edges of removed triangles
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if ((out >> s) & 1u) {
        const unsigned u = tri[vb + j + L * s];
        const int A = u & 0xFF, B = (u >> 8) & 0xFF, C = (u >> 16) & 0xFF;
        atomicOr(&omask[pb + A], bitm<M>(B));
        atomicOr(&omask[pb + B], bitm<M>(C));
        atomicOr(&omask[pb + C], bitm<M>(A));
      }
    }
    __syncthreads();
    // boundary edges: twin not removed
    int nbnd = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if ((out >> s) & 1u) {
        const unsigned u = tri[vb + j + L * s];
        const int A = u & 0xFF, B = (u >> 8) & 0xFF, C = (u >> 16) & 0xFF;
        nbnd += !((omask[pb + B] >> A) & 1) + !((omask[pb + C] >> B) & 1) + !((omask[pb + A] >> C) & 1);
      }
    }
    int btot;
    int off = gexcl(nbnd, btot);
    if (doit && (btot < 3 || btot > PMAX)) {  // inconsistent topology (rounding): give up on the cell
      st = VOTESS_CELL_UNRESOLVED;
      doit = false;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (doit && ((out >> s) & 1u)) {
        const unsigned u = tri[vb + j + L * s];
        const int A = u & 0xFF, B = (u >> 8) & 0xFF, C = (u >> 16) & 0xFF;
        if (!((omask[pb + B] >> A) & 1)) snew[pb + off++] = A | (B << 8);
        if (!((omask[pb + C] >> B) & 1)) snew[pb + off++] = B | (C << 8);
        if (!((omask[pb + A] >> C) & 1)) snew[pb + off++] = C | (A << 8);
      }
    }
    __syncthreads();
    // clear the bit matrix rows and free the removed slots
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if ((out >> s) & 1u) {
        const int t = j + L * s;
        const unsigned u = tri[vb + t];
        omask[pb + (u & 0xFF)] = 0;
        omask[pb + ((u >> 8) & 0xFF)] = 0;
        omask[pb + ((u >> 16) & 0xFF)] = 0;
        if (doit) tri[vb + t] = kEmpty;
      }
    }
    __syncthreads();
    // new triangles (a, b, ps) into free slots, in slot order: the slot loop
    // only assigns the r-th free slot to new triangle r; lane r then solves
    // its vertex, so that a cut runs the solve once rather than once per slot
    // index any lane of the wave fills
    int base = 0, hnew = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int t = j + L * s;
      const bool fr = doit && tri[vb + t] == kEmpty;
      const unsigned gbits = (unsigned)((__ballot(fr) >> gb) & LOWL);
      const int r = base + __popc(gbits & ((1u << j) - 1u));
      base += __popc(gbits);
      if (fr && r < btot) {
        sslot[pb + r] = (unsigned char)t;
        hnew = t + 1;
      }
    }
    if (doit && base < btot) {
      st = VOTESS_CELL_CAPACITY;
      doit = false;
    }
    hnew = gmaxi(hnew);
    __syncthreads();
    const R mx = nx, my = ny, mz = nz, mc = c;
    for (int r = j; doit && r < btot; r += L) {
      const int t = sslot[pb + r];
      const unsigned e = snew[pb + r];
      const int A = e & 0xFF, B = (e >> 8) & 0xFF;
      V3<R> v;
      float ev = 0.0f;
      if constexpr (RECHECK) {
        float e;
        v = solve3_err({pnx[pb + A], pny[pb + A], pnz[pb + A]}, pnc[pb + A], {pnx[pb + B], pny[pb + B], pnz[pb + B]},
                       pnc[pb + B], {mx, my, mz}, mc, e);
        const float vm = fmaxf(fabsf(v.x), fmaxf(fabsf(v.y), fabsf(v.z)));
        if (!(e <= 16.0 * a.eps * vm)) {
          // ill-conditioned float vertex: solve it in double from the exact
          // planes and keep the rounded value (bound: one ulp)
          const V3<double> w = vertex64((unsigned)A | ((unsigned)B << 8) | ((unsigned)ps << 16));
          v = {(float)w.x, (float)w.y, (float)w.z};
          e = FLT_EPSILON * (float)fmax(fabs(w.x), fmax(fabs(w.y), fabs(w.z)));
          ++nrecheck;
        }
        verr[vb + t] = e;
        ev = e;
      } else {
        v = solve3<R>({pnx[pb + A], pny[pb + A], pnz[pb + A]}, pnc[pb + A], {pnx[pb + B], pny[pb + B], pnz[pb + B]},
                      pnc[pb + B], {mx, my, mz}, mc);
      }
      vx[vb + t] = v.x;
      vy[vb + t] = v.y;
      vz[vb + t] = v.z;
      if constexpr (kVrad) {
        if (in_stream) vrad[vb + t] = ball_rad(v.x, v.y, v.z, ev);
      }
      tri[vb + t] = (unsigned)A | ((unsigned)B << 8) | ((unsigned)ps << 16);
    }
    __syncthreads();
    // rebuild the alive-plane mask and R^2
    if (doit) H = max(H, hnew);
    M al = 0;
    R r2 = 0;
    float em = 0.0f, eml = 0.0f;
    if (doit) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int t = j + L * s;
        if (t < H) {
          const unsigned u = tri[vb + t];
          if (u != kEmpty) {
            al |= bitm<M>(u & 0xFF) | bitm<M>((u >> 8) & 0xFF) | bitm<M>((u >> 16) & 0xFF);
            const R X = vx[vb + t], Y = vy[vb + t], Z = vz[vb + t];
            r2 = fmax(r2, X * X + Y * Y + Z * Z);
            if (RECHECK) {
              const float n2 = (float)(X * X + Y * Y + Z * Z), n1 = (float)(fabs(X) + fabs(Y) + fabs(Z));
              const float e = verr[vb + t];
              em = fmaxf(em, n2 + e * (2.0f * n1 + e));
              eml = fmaxf(eml, n2 - 2.0f * e * n1);
            }
          }
        }
      }
    }
    al = gor(al);
    r2 = gmax(r2);
    if (RECHECK) {
#pragma unroll
      for (int o = 1; o < L; o <<= 1) {
        em = fmaxf(em, shfl_xor_w(em, o, L));
        eml = fmaxf(eml, shfl_xor_w(eml, o, L));
      }
    }
    if (doit) {
      alive = al;
      R2 = r2;
      if (RECHECK) {
        R2hi = em * (1.0f + 4.0f * FLT_EPSILON);
        R2lo = eml * (1.0f - 4.0f * FLT_EPSILON);
        fprev = rad_certain(d2);
        fmarg = rad_uncertain(d2);
      } else {
        fprev = (R)(d2 * (R)kDmargin) > R(4) * R2;
      }
    }
  };

  // The list is read two planes ahead (the index of plane m+2, the record of
  // plane m+1), so that the two dependent loads of a plane overlap the work
  // of the one before it.
  const int* klist = a.knn + (size_t)(have ? (a.knn_by_id ? (long long)sid : t_idx) : 0) * a.kstride;
  int nb_next = have && a.k > 0 ? klist[0] : -1;
  Rec4 q_next = rec[nb_next >= 0 ? nb_next : sid];
  int nb_next2 = have && a.k > 1 ? klist[1] : -1;
  int m = 0;
  for (; m < a.k; ++m) {
    bool run = st == ST_RUN;
    if (!__any(run)) break;
    int nb = -1;
    R nx = 0, ny = 0, nz = 0, d2 = 0, c = 0;
    const int nb_cur = nb_next;
    const Rec4 q_cur = q_next;
    if (run) {
      nb_next = nb_next2;
      q_next = rec[nb_next >= 0 ? nb_next : sid];
      nb_next2 = m + 2 < a.k ? klist[m + 2] : -1;
    }
    if (run) {
      nb = nb_cur;
      if (nb < 0) {  // padded list: it holds every other point
        st = VOTESS_CELL_CERTIFIED;
        kneed = m;
        run = false;
      }
    }
    bool cert_check = false, cert_recheck = false;
    if (run) {
      const Rec4 q = q_cur;
      nx = (R)q.x - px;
      ny = (R)q.y - py;
      nz = (R)q.z - pz;
      d2 = dist2_nc(nx, ny, nz);
      c = R(0.5) * d2;
      if (RECHECK) {
        cert_check = rad_certain(d2);
        cert_recheck = rad_uncertain(d2);
      } else {
        cert_check = (R)(d2 * (R)kDmargin) > R(4) * R2;
      }
    }
    if (RECHECK) {
      if (__any(cert_recheck)) {
        const double r64 = radius64(cert_recheck);
        if (cert_recheck) {
          const Rec4 q = rec[nb];
          const V3<double> n64 = {(double)q.x - p64x, (double)q.y - p64y, (double)q.z - p64z};
          const double d64 = dot(n64, n64);
          cert_check = d64 * kDmargin > 4.0 * r64;
          if (fabs(d64 - 4.0 * r64) <= 1e-12 * d64) st = VOTESS_CELL_UNRESOLVED;
          ++nrecheck;
        }
      }
      if (st != ST_RUN) run = false;
    }
    if (run && cert_check) {
      st = VOTESS_CELL_CERTIFIED;
      kneed = fprev ? m : m + 1;
      run = false;
    }

    apply_plane(run, nx, ny, nz, c, d2, nb);
  }
  // ---- end of the list: certified if d_k^2 > 4 R_k^2 or the list holds all others
  if (RECHECK) {  // a marginal final radius test is redone in double
    const bool need = st == ST_RUN && fmarg;
    if (__any(need)) {
      const double r64 = radius64(need);
      if (need) {
        const Rec4 q = rec[klist[a.k - 1]];
        const V3<double> n64 = {(double)q.x - p64x, (double)q.y - p64y, (double)q.z - p64z};
        const double d64 = dot(n64, n64);
        fprev = d64 * kDmargin > 4.0 * r64;
        if (fabs(d64 - 4.0 * r64) <= 1e-12 * d64) st = VOTESS_CELL_UNRESOLVED;
        ++nrecheck;
      }
    }
  }
  if (st == ST_RUN) {
    if (fprev || a.k >= a.n - 1) {
      st = VOTESS_CELL_CERTIFIED;
      kneed = a.k;
    } else {
      st = VOTESS_CELL_RADIUS;
    }
  }


  // ---- stream phase: a cell its list did not certify keeps clipping by grid
  // rings around its seed, restricted to the bounding box of its "flower" (the
  // union of the balls centred at its vertices that pass through the seed: a
  // point outside every such ball is on the inner side of its bisector at
  // every vertex, so it cannot cut; flowers only shrink as the cell does).
  // Points already in the list are skipped by their (d^2, sorted index) key,
  // points beyond the security radius by d^2 > 4 R^2.  The cell is final once
  // the scanned block of rings contains the flower box.
  // With no list at all (k = 0) every cell starts here, at ring 0: the
  // fused form, with no k-NN pass and no list in memory.
  if constexpr (STREAM) {
    const bool nolist = a.k == 0;
    const int ik0 = (have && st == VOTESS_CELL_RADIUS && !nolist) ? klist[a.k - 1] : -1;
    const bool strm = have && st == VOTESS_CELL_RADIUS && (nolist || ik0 >= 0);  // a full list that did not certify
    if (strm) st = ST_RUN;
    if constexpr (kVrad) {
      // ball radii of the current vertices (kept up to date from here on)
      in_stream = strm;
      for (int t = j; t < H; t += L)
        if (strm && tri[vb + t] != kEmpty) vrad[vb + t] = ball_rad(vx[vb + t], vy[vb + t], vz[vb + t], verr[vb + t]);
      __syncthreads();
    }
    if (strm && j == 0 && a.counters) atomicAdd(&a.counters[5], 1ull);
    const GridDev& Gd = a.grid;
    const int cx = axis_cell(p64x, Gd.lo0, Gd.ih0, Gd.g0);
    const int cy = axis_cell(p64y, Gd.lo1, Gd.ih1, Gd.g1);
    const int cz = axis_cell(p64z, Gd.lo2, Gd.ih2, Gd.g2);
    const double gmarg = 1e-9 * fmax(Gd.hi0 - Gd.lo0, fmax(Gd.hi1 - Gd.lo1, Gd.hi2 - Gd.lo2));
    R dk2 = R(-1);  // no list: every candidate lies beyond it
    int ik = -1;
    if (strm && !nolist) {
      ik = ik0;
      const Rec4 q = rec[ik];
      dk2 = dist2_nc((R)q.x - px, (R)q.y - py, (R)q.z - pz);
    }
    // A box (seed-relative bounds, already widened by gmarg) that lies inside
    // the list's ball holds list members only: every point in it is closer
    // than the list's last one even after the rounding of d^2.
    const double dk2in = (double)dk2 * (1.0 - 1e-6);
    auto in_list_ball = [&](double ax, double bx, double ay, double by, double az, double bz) -> bool {
      const double f = fmax(ax * ax, bx * bx) + fmax(ay * ay, by * by) + fmax(az * az, bz * bz);
      return f < dk2in;
    };
    // A vertex whose widened ball reaches less than the list's ball from the
    // seed (twice its radius below that ball's) can only hold list members:
    // the flower box and the per-box vertex lists leave it out.
    const R rlim = dk2in > 0.0 ? (R)(0.5 * sqrt(dk2in) * (1.0 - 1e-6)) : R(-1);
    // flower box in grid cells, from the current vertices whose ball leaves
    // the list's ball (group reduction)
    Enum& E_ = senum[STREAM ? g : 0];
    int &fb0 = E_.fb0, &fb1 = E_.fb1, &fb2 = E_.fb2, &fb3 = E_.fb3, &fb4 = E_.fb4, &fb5 = E_.fb5;
    fb0 = 0; fb1 = -1; fb2 = 0; fb3 = -1; fb4 = 0; fb5 = -1;
    double* fwb = fwbox + (STREAM ? g * 6 : 0);  // the same box in coordinates
    auto flower_box = [&]() {
      double mn0 = 1e300, mn1 = 1e300, mn2 = 1e300, mx0 = -1e300, mx1 = -1e300, mx2 = -1e300;
      for (int t = j; t < H; t += L) {
        if (tri[vb + t] == kEmpty) continue;
        const R rv = vball(t, vx[vb + t], vy[vb + t], vz[vb + t]);
        if (rv < rlim) continue;
        const double X = vx[vb + t], Y = vy[vb + t], Z = vz[vb + t];
        const double rad = rv;
        mn0 = fmin(mn0, X - rad); mx0 = fmax(mx0, X + rad);
        mn1 = fmin(mn1, Y - rad); mx1 = fmax(mx1, Y + rad);
        mn2 = fmin(mn2, Z - rad); mx2 = fmax(mx2, Z + rad);
      }
#pragma unroll
      for (int o = 1; o < L; o <<= 1) {
        mn0 = fmin(mn0, shfl_xor_w(mn0, o, L)); mx0 = fmax(mx0, shfl_xor_w(mx0, o, L));
        mn1 = fmin(mn1, shfl_xor_w(mn1, o, L)); mx1 = fmax(mx1, shfl_xor_w(mx1, o, L));
        mn2 = fmin(mn2, shfl_xor_w(mn2, o, L)); mx2 = fmax(mx2, shfl_xor_w(mx2, o, L));
      }
      if (mn0 > mx0) {  // every ball inside the list's: the seed's own cell closes the scan
        mn0 = mx0 = mn1 = mx1 = mn2 = mx2 = 0.0;
      }
      const double fw0 = p64x + mn0 - gmarg, fw1 = p64x + mx0 + gmarg;
      const double fw2 = p64y + mn1 - gmarg, fw3 = p64y + mx1 + gmarg;
      const double fw4 = p64z + mn2 - gmarg, fw5 = p64z + mx2 + gmarg;
      if (j == 0) {
        fwb[0] = fw0; fwb[1] = fw1; fwb[2] = fw2; fwb[3] = fw3; fwb[4] = fw4; fwb[5] = fw5;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      fb0 = axis_cell(fw0, Gd.lo0, Gd.ih0, Gd.g0);
      fb1 = axis_cell(fw1, Gd.lo0, Gd.ih0, Gd.g0);
      fb2 = axis_cell(fw2, Gd.lo1, Gd.ih1, Gd.g1);
      fb3 = axis_cell(fw3, Gd.lo1, Gd.ih1, Gd.g1);
      fb4 = axis_cell(fw4, Gd.lo2, Gd.ih2, Gd.g2);
      fb5 = axis_cell(fw5, Gd.lo2, Gd.ih2, Gd.g2);
    };
    int &rr = E_.rr, &zz = E_.zz, &yy = E_.yy, &part = E_.part, &zhi = E_.zhi, &ylo = E_.ylo, &yhi = E_.yhi;
    rr = -1; zz = 0; yy = 0; part = 0; zhi = -1; ylo = 0; yhi = -1;
    int jcur = 0, jend = 0;
    // the x-run being split at dense cells, and the sub-block of the dense
    // cell being scanned (sub-cells that meet the flower box)
    int &rx = E_.rx, &rx1 = E_.rx1, &rrow = E_.rrow;
    rx = 1; rx1 = 0; rrow = 0;
    // dense cell rows: z and y outward from the seed's row (0, +1, -1, +2, ...)
    int &dm = E_.dm, &dm0 = E_.dm0, &dm1 = E_.dm1, &dbase = E_.dbase, &dsx0 = E_.dsx0, &dsx1 = E_.dsx1,
        &dsy0 = E_.dsy0, &dsy1 = E_.dsy1, &dsz0 = E_.dsz0, &dsz1 = E_.dsz1;
    dm = 0; dm0 = 0; dm1 = 0; dbase = 0; dsx0 = 0; dsx1 = -1; dsy0 = 0; dsy1 = -1; dsz0 = 0; dsz1 = -1;
    int &dq1 = E_.dq1, &dq2 = E_.dq2, &kyn = E_.kyn, &kzn = E_.kzn;
    dq1 = 0; dq2 = 0; kyn = 0; kzn = 0;
    // next sub-row ordinal, their count; listed ranges, next one
    int &dq = E_.dq, &dqn = E_.dqn, &srn = E_.srn, &srp = E_.srp;
    dq = 0; dqn = 0; srn = 0; srp = 0;
    int& dsto = E_.dsto;  // the dense cell's sub-grid record: a.sub.start + dsto
    dsto = 0;
    unsigned pend = 0;
    int myj = -1;
    R myd2 = R(0);
    const R skip_scale = RECHECK ? R(1) - R(2e-6) : R(1) - R(1e-12);
    // box of the current vertices whose ball leaves the list's ball
    // (relative to the seed, widened by their error bounds): a candidate d
    // beyond the list can cut only if such a vertex v has d.v > |d|^2 / 2,
    // and max_v d.v <= sum_a max(d_a lo_a, d_a hi_a).  The cell only
    // shrinks: a d that cuts the smaller cell cuts the larger one at some
    // vertex, whose ball then holds d, a point beyond the list, so that
    // vertex was in the older box, which is still a valid bound.
    R bl0 = 0, bl1 = 0, bl2 = 0, bh0 = 0, bh1 = 0, bh2 = 0;
    bool box_ok = false;
    auto vertex_box = [&]() {
      R a0 = R(3.0e38), a1 = R(3.0e38), a2 = R(3.0e38), b0 = R(-3.0e38), b1 = R(-3.0e38), b2 = R(-3.0e38);
      for (int t = j; t < H; t += L) {
        if (tri[vb + t] == kEmpty) continue;
        if (vball(t, vx[vb + t], vy[vb + t], vz[vb + t]) < rlim) continue;
        const R e = RECHECK ? (R)verr[vb + t] : R(0);
        const R X = vx[vb + t], Y = vy[vb + t], Z = vz[vb + t];
        a0 = fmin(a0, X - e); b0 = fmax(b0, X + e);
        a1 = fmin(a1, Y - e); b1 = fmax(b1, Y + e);
        a2 = fmin(a2, Z - e); b2 = fmax(b2, Z + e);
      }
#pragma unroll
      for (int o = 1; o < L; o <<= 1) {
        a0 = fmin(a0, shfl_xor_w(a0, o, L)); b0 = fmax(b0, shfl_xor_w(b0, o, L));
        a1 = fmin(a1, shfl_xor_w(a1, o, L)); b1 = fmax(b1, shfl_xor_w(b1, o, L));
        a2 = fmin(a2, shfl_xor_w(a2, o, L)); b2 = fmax(b2, shfl_xor_w(b2, o, L));
      }
      bl0 = a0; bl1 = a1; bl2 = a2; bh0 = b0; bh1 = b1; bh2 = b2;
    };
    // relative slack of that test: above the rounding of the plane tests
    // (and of the float path's rechecks)
    const R sup_slack = RECHECK ? R(4e-6) : R(1e-12);
    // A point cuts the cell iff it lies in the ball of some vertex v through
    // the seed (centre v, radius |v|).  For a box of candidates (a grid row or
    // a dense cell's sub-block), the vertices whose ball meets the box are
    // listed in `out`; none: the box cannot hold a cutting point.  The balls
    // are widened past rounding and the float path's vertex error bounds.
    // Lists name vertex slots, so a cut (which reuses slots) invalidates them.
    // Box bounds enter the tests in the clip's precision rounded outward, so
    // that the box only grows.
    auto out_lo = [](double v) -> R {
      if constexpr (sizeof(R) == 4) {
        const float f = (float)v;
        return (double)f > v ? nextafterf(f, -INFINITY) : f;
      } else {
        return v;
      }
    };
    auto out_hi = [](double v) -> R {
      if constexpr (sizeof(R) == 4) {
        const float f = (float)v;
        return (double)f < v ? nextafterf(f, INFINITY) : f;
      } else {
        return v;
      }
    };
    auto relevant = [&](unsigned char* out, double x0, double x1, double y0, double y1, double z0,
                        double z1) -> int {
      if (in_list_ball(x0 - p64x - gmarg, x1 - p64x + gmarg, y0 - p64y - gmarg, y1 - p64y + gmarg, z0 - p64z - gmarg,
                       z1 - p64z + gmarg))
        return 0;  // (group-uniform)
      const R ax = out_lo(x0 - p64x - gmarg), bx = out_hi(x1 - p64x + gmarg);
      const R ay = out_lo(y0 - p64y - gmarg), by = out_hi(y1 - p64y + gmarg);
      const R az = out_lo(z0 - p64z - gmarg), bz = out_hi(z1 - p64z + gmarg);
      unsigned bits = 0;
#pragma unroll
      for (int s2 = 0; s2 < S; ++s2) {
        const int t = j + L * s2;
        if (t < H && tri[vb + t] != kEmpty) {
          const R X = vx[vb + t], Y = vy[vb + t], Z = vz[vb + t];
          const R rv = vball(t, X, Y, Z);
          const R gx = fmax(R(0), fmax(ax - X, X - bx)), gy = fmax(R(0), fmax(ay - Y, Y - by)),
                  gz = fmax(R(0), fmax(az - Z, Z - bz));
          if (rv >= rlim && gx * gx + gy * gy + gz * gz <= rv * rv) bits |= 1u << s2;
        }
      }
      int tot;
      int w = gexcl(__popc(bits), tot);
#pragma unroll
      for (int s2 = 0; s2 < S; ++s2)
        if ((bits >> s2) & 1u) out[g * TMAX + w++] = (unsigned char)(j + L * s2);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      return tot;
    };
    int nR = 0, nD = 0;
    bool okR = false, okD = false;  // lists valid for the current vertices
    // can sub-row (sy, sz) of the dense cell's sub-block hold a cutting point:
    // not inside the list's ball, and (while the dense cell's vertex list is
    // valid) meeting the ball of a listed vertex?  (one sub-row per lane)
    auto sub_row_relevant = [&](int sy, int sz) -> bool {
      const double* dgp = dgeo + g * 9;
      const int m2 = a.sub.start[dsto + 2];
      const double X0 = dsx0 == 0 ? dgp[0] : dgp[3] + dsx0 * dgp[6];
      const double X1 = dsx1 == dm0 - 1 ? dgp[0] + Gd.h0 : dgp[3] + (dsx1 + 1) * dgp[6];
      const double Y0 = sy == 0 ? dgp[1] : dgp[4] + sy * dgp[7];
      const double Y1 = sy == dm1 - 1 ? dgp[1] + Gd.h1 : dgp[4] + (sy + 1) * dgp[7];
      const double Z0 = sz == 0 ? dgp[2] : dgp[5] + sz * dgp[8];
      const double Z1 = sz == m2 - 1 ? dgp[2] + Gd.h2 : dgp[5] + (sz + 1) * dgp[8];
      if (in_list_ball(X0 - p64x - gmarg, X1 - p64x + gmarg, Y0 - p64y - gmarg, Y1 - p64y + gmarg, Z0 - p64z - gmarg,
                       Z1 - p64z + gmarg))
        return false;
      if (!okD) return true;
      const R ax = out_lo(X0 - p64x - gmarg), bx = out_hi(X1 - p64x + gmarg);
      const R ay = out_lo(Y0 - p64y - gmarg), by = out_hi(Y1 - p64y + gmarg);
      const R az = out_lo(Z0 - p64z - gmarg), bz = out_hi(Z1 - p64z + gmarg);
      for (int i = 0; i < nD; ++i) {
        const int t = relD[g * TMAX + i];
        const R X = vx[vb + t], Y = vy[vb + t], Z = vz[vb + t];
        const R rv = vball(t, X, Y, Z);
        const R gx = fmax(R(0), fmax(ax - X, X - bx)), gy = fmax(R(0), fmax(ay - Y, Y - by)),
                gz = fmax(R(0), fmax(az - Z, Z - bz));
        if (gx * gx + gy * gy + gz * gz <= rv * rv) return true;
      }
      return false;
    };
    bool rdense = false;  // the current range lies in a dense cell
    while (__any(strm && st == ST_RUN)) {
      const bool act = strm && st == ST_RUN;
      // refill this group's batch of candidates (group-uniform loop)
      if (act && pend == 0u) {
        if (!box_ok) {
          vertex_box();
          box_ok = true;
        }
        bool done = false;
        while (!done) {
          if (jcur >= jend) {
            // next contiguous range of points: a sub-cell x-run of a dense
            // cell, a stretch of sparse cells of the current x-run, or the
            // ring's next x-run of grid cells
            bool have_run = false;
            while (!have_run) {
              if (dm > 0) {
                // the dense cell's sub-rows inside the flower box, one x-run
                // each, rows nearer the seed first: the next L of them are
                // tested and their ranges read at once, one per lane, and the
                // non-empty ranges listed
                if (srp >= srn) {
                  if (dq >= dqn) {
                    dm = 0;
                    continue;
                  }
                  const int q = dq + j;
                  dq += L;
                  bool keep = false;
                  int lo = 0, hi = 0;
                  if (q < dqn) {
                    const int qz = q / kyn, qy = q - qz * kyn;
                    const int sz = dq2 + ((qz & 1) ? (qz + 1) >> 1 : -(qz >> 1));
                    const int sy = dq1 + ((qy & 1) ? (qy + 1) >> 1 : -(qy >> 1));
                    if (sz >= dsz0 && sz <= dsz1 && sy >= dsy0 && sy <= dsy1 && sub_row_relevant(sy, sz)) {
                      const int rowb = kSubHead + dm0 * (sy + dm1 * sz);
                      lo = a.sub.start[dsto + rowb + dsx0];
                      hi = a.sub.start[dsto + rowb + dsx1 + 1];
                      keep = lo < hi;
                    }
                  }
                  int tot;
                  const int w = gexcl(keep ? 1 : 0, tot);
                  if (keep) srl[g * L + w] = make_int2(lo, hi);
                  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                  srn = tot;
                  srp = 0;
                  continue;
                }
                const int2 rg = srl[g * L + srp];
                ++srp;
                jcur = dbase + rg.x;
                jend = dbase + rg.y;
                have_run = true;
                rdense = true;
                continue;
              }
              if (rx <= rx1) {
                int xe = rx1 + 1;
                if (a.sub.info) {
                  // the stretch of cells without sub-grids: the group reads L
                  // consecutive cells' records at once and ends it at the
                  // first dense one
                  xe = rx;
                  for (;;) {
                    const int xc = xe + j;
                    const bool dn = xc <= rx1 && a.sub.info[rrow + xc].x >= 0;
                    const unsigned long long dmask = (__ballot(dn) >> gb) & LOWL;
                    if (dmask) {
                      xe += __ffsll((long long)dmask) - 1;
                      break;
                    }
                    xe += L;
                    if (xe > rx1) {
                      xe = rx1 + 1;
                      break;
                    }
                  }
                }
                if (xe > rx) {
                  jcur = a.cell_start[rrow + rx];
                  jend = a.cell_start[rrow + xe];
                  rx = xe;
                  have_run = jcur < jend;
                  rdense = false;
                  continue;
                }
                // dense cell rx: its sub-cells inside the flower box
                const int2 info = a.sub.info[rrow + rx];
                const SubCell sc = sub_cell(a.sub.start + info.x);
                dsx0 = sub_axis(fwb[0], sc.lo0, sc.ih0, sc.m0);
                dsx1 = sub_axis(fwb[1], sc.lo0, sc.ih0, sc.m0);
                dsy0 = sub_axis(fwb[2], sc.lo1, sc.ih1, sc.m1);
                dsy1 = sub_axis(fwb[3], sc.lo1, sc.ih1, sc.m1);
                dsz0 = sub_axis(fwb[4], sc.lo2, sc.ih2, sc.m2);
                dsz1 = sub_axis(fwb[5], sc.lo2, sc.ih2, sc.m2);
                {
                  // the sub-block's box (edge sub-cells reach the cell's faces)
                  const double cxl = Gd.lo0 + rx * Gd.h0, cyl = Gd.lo1 + yy * Gd.h1, czl = Gd.lo2 + zz * Gd.h2;
                  const double w0 = 1.0 / sc.ih0, w1 = 1.0 / sc.ih1, w2 = 1.0 / sc.ih2;
                  const double X0 = dsx0 == 0 ? cxl : sc.lo0 + dsx0 * w0;
                  const double X1 = dsx1 == sc.m0 - 1 ? cxl + Gd.h0 : sc.lo0 + (dsx1 + 1) * w0;
                  const double Y0 = dsy0 == 0 ? cyl : sc.lo1 + dsy0 * w1;
                  const double Y1 = dsy1 == sc.m1 - 1 ? cyl + Gd.h1 : sc.lo1 + (dsy1 + 1) * w1;
                  const double Z0 = dsz0 == 0 ? czl : sc.lo2 + dsz0 * w2;
                  const double Z1 = dsz1 == sc.m2 - 1 ? czl + Gd.h2 : sc.lo2 + (dsz1 + 1) * w2;
                  nD = relevant(relD, X0, X1, Y0, Y1, Z0, Z1);
                  okD = true;
                  if (j == 0) {
                    double* dgp = dgeo + g * 9;
                    dgp[0] = cxl; dgp[1] = cyl; dgp[2] = czl;
                    dgp[3] = sc.lo0; dgp[4] = sc.lo1; dgp[5] = sc.lo2;
                    dgp[6] = w0; dgp[7] = w1; dgp[8] = w2;
                  }
                  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                  if (nD == 0) {
                    ++rx;
                    continue;
                  }
                }
                dsto = info.x;
                dbase = a.cell_start[rrow + rx];
                dm = 1;
                dm0 = sc.m0;
                dm1 = sc.m1;
                dq1 = min(max(sub_axis(p64y, sc.lo1, sc.ih1, sc.m1), dsy0), dsy1);
                dq2 = min(max(sub_axis(p64z, sc.lo2, sc.ih2, sc.m2), dsz0), dsz1);
                // offsets 0, +1, -1, ... up to the farther end of each range
                kyn = 2 * max(dq1 - dsy0, dsy1 - dq1) + 1;
                kzn = 2 * max(dq2 - dsz0, dsz1 - dq2) + 1;
                dq = 0;
                dqn = kyn * kzn;
                srn = srp = 0;
                ++rx;
                continue;
              }
              if (rr < 0 || zz > zhi) {
                // ring rr finished (or none yet): final when the block contains the flower box
                flower_box();
                if (rr >= 0 && cx - rr <= fb0 && cx + rr >= fb1 && cy - rr <= fb2 && cy + rr >= fb3 &&
                    cz - rr <= fb4 && cz + rr >= fb5) {
                  done = true;
                  break;
                }
                ++rr;
                zz = max(cz - rr, fb4);
                zhi = min(cz + rr, fb5);
                ylo = max(cy - rr, fb2);
                yhi = min(cy + rr, fb3);
                yy = ylo;
                part = 0;
                if (ylo > yhi) zz = zhi + 1;  // empty ring
                continue;
              }
              const bool face = zz == cz - rr || zz == cz + rr || yy == cy - rr || yy == cy + rr;
              int x0 = 1, x1 = 0;
              if (part == 0) {
                if (face) { x0 = max(cx - rr, fb0); x1 = min(cx + rr, fb1); }
                else if (cx - rr >= fb0) { x0 = x1 = cx - rr; }
                part = 1;
              } else if (part == 1) {
                if (!face && rr > 0 && cx + rr <= fb1) { x0 = x1 = cx + rr; }
                part = 2;
              } else {
                part = 0;
                if (++yy > yhi) { yy = ylo; ++zz; }
                continue;
              }
              if (x0 <= x1) {
                const double Y0 = Gd.lo1 + yy * Gd.h1, Z0 = Gd.lo2 + zz * Gd.h2;
                nR = relevant(relR, Gd.lo0 + x0 * Gd.h0, Gd.lo0 + (x1 + 1) * Gd.h0, Y0, Y0 + Gd.h1, Z0, Z0 + Gd.h2);
                okR = true;
                if (nR > 0) {
                  rrow = Gd.g0 * (yy + Gd.g1 * zz);
                  rx = x0;
                  rx1 = x1;
                }
              }
            }
            if (done) break;
          }
          // batch of up to L candidates, one per lane: the rest of the current
          // range, then (in a dense cell) the following listed sub-rows;
          // filtered by list key and radius
          int jj = -1;
          {
            int nb = 0;
            for (;;) {
              const int take = min(L - nb, jend - jcur);
              if (j >= nb && j < nb + take) jj = jcur + (j - nb);
              nb += take;
              jcur += take;
              if (nb == L || !rdense || srp >= srn) break;
              const int2 rg = srl[g * L + srp];
              ++srp;
              jcur = dbase + rg.x;
              jend = dbase + rg.y;
            }
          }
          bool pass = false;
          myj = -1;
          if (jj >= 0 && jj != sid) {
            const Rec4 q = rec[jj];
            const R d2c = dist2_nc((R)q.x - px, (R)q.y - py, (R)q.z - pz);
            const bool beyond_list = d2c > dk2 || (d2c == dk2 && jj > ik);
            pass = beyond_list && d2c * skip_scale <= R(4) * (RECHECK ? (R)R2hi : R2);
            if (pass) {
              const R ex = (R)q.x - px, ey = (R)q.y - py, ez = (R)q.z - pz;
              const R sup = fmax(ex * bl0, ex * bh0) + fmax(ey * bl1, ey * bh1) + fmax(ez * bl2, ez * bh2);
              const R mag = fabs(ex) * fmax(fabs(bl0), fabs(bh0)) + fabs(ey) * fmax(fabs(bl1), fabs(bh1)) +
                            fabs(ez) * fmax(fabs(bl2), fabs(bh2));
              pass = sup >= R(0.5) * d2c - sup_slack * (mag + d2c);
              if (pass) {
                // exact: some vertex on the far side of the bisector (up to
                // the plane test's own uncertainty window), against the
                // vertices listed for this range, or all of them
                const R cc = R(0.5) * d2c;
                const R nrm1 = fabs(ex) + fabs(ey) + fabs(ez);
                auto side = [&](int t) -> bool {
                  const R X = vx[vb + t], Y = vy[vb + t], Z = vz[vb + t];
                  const R sv = ex * X + ey * Y + ez * Z - cc;
                  const R scale = fabs(ex * X) + fabs(ey * Y) + fabs(ez * Z) + cc;
                  const R win = RECHECK ? (R)a.eps * scale + nrm1 * (R)verr[vb + t] : R(1e-12) * scale;
                  return sv > -win;
                };
                bool cuts = false;
                if (rdense ? okD : okR) {
                  const unsigned char* rl = rdense ? relD : relR;
                  const int nr = rdense ? nD : nR;
                  for (int i = 0; i < nr && !cuts; ++i) cuts = side(rl[g * TMAX + i]);
                } else {
                  for (int t = 0; t < H && !cuts; ++t)
                    if (tri[vb + t] != kEmpty) cuts = side(t);
                }
                pass = cuts;
              }
            }
            myj = jj;
            myd2 = d2c;
          }
          pend = (unsigned)((__ballot(pass) >> gb) & LOWL);
          if (!pass) myj = -1;
          if (pend) break;
        }
        if (done) {
          st = VOTESS_CELL_CERTIFIED;
          kneed = a.k + 1;
        }
      }
      // nearest pending candidate of the group
      bool run2 = act && st == ST_RUN && pend != 0u;
      R best = (run2 && myj >= 0 && ((pend >> j) & 1u)) ? myd2 : R(3.0e38);
      int bl = j;
#pragma unroll
      for (int o = 1; o < L; o <<= 1) {
        const R ob = shfl_xor_w(best, o, L);
        const int ol = shfl_xor_w(bl, o, L);
        if (ob < best || (ob == best && ol < bl)) { best = ob; bl = ol; }
      }
      const int nb2 = __shfl(myj, gb + bl, 64);
      R nx = 0, ny = 0, nz = 0, c = 0, d2 = 0;
      if (run2) {
        pend &= ~(1u << bl);
        const Rec4 q = rec[nb2];
        nx = (R)q.x - px;
        ny = (R)q.y - py;
        nz = (R)q.z - pz;
        d2 = dist2_nc(nx, ny, nz);
        c = R(0.5) * d2;
        // the radius may have shrunk since the batch was filtered
        if (d2 * skip_scale > R(4) * (RECHECK ? (R)R2hi : R2)) run2 = false;
      }
      const M alive_prev = alive;
      apply_plane(run2, nx, ny, nz, c, d2, nb2);
      if (alive != alive_prev) {
        box_ok = false;
        okR = okD = false;
      }
    }
    if (strm && st == VOTESS_CELL_CERTIFIED && j == 0 && a.counters) atomicAdd(&a.counters[4], 1ull);
  }

  // ---- outputs
  const bool cert = have && st == VOTESS_CELL_CERTIFIED;
  // volume: corner terms in double.  `exact` takes vertices and planes in
  // double from the inputs (float path, ill-conditioned cells only).
  // Anchor of edge f^g: the point of the line nearest the seed,
  // (c_f (n_g x d) - c_g (n_f x d)) / |d|^2 with d = n_f x n_g.  Its error
  // grows like 1/sin of the angle between the planes; a solve of the 2x2 Gram
  // system would square that, which shows on the faces of nearly parallel
  // neighbours.
  auto anchor = [&](const V3<double>& nf, double cf, const V3<double>& ng, double cg) -> V3<double> {
    const V3<double> d = cross(nf, ng);
    const V3<double> gd = cross(ng, d), fd = cross(nf, d);
    const double inv = 1.0 / dot(d, d);
    return {(cf * gd.x - cg * fd.x) * inv, (cf * gd.y - cg * fd.y) * inv, (cf * gd.z - cg * fd.z) * inv};
  };
  // the three planes and the position of vertex slot t, in double: cached,
  // or (exact) planes from the exact inputs, or (refined) cached or exact
  // planes with the vertex solved and refined in double
  auto corner_geom = [&](unsigned u, int t, bool exact, V3<double>& na, double& ca, V3<double>& nb_, double& cb,
                         V3<double>& nc, double& cc, V3<double>& v, bool refined = false) {
    const int A = u & 0xFF, B = (u >> 8) & 0xFF, C = (u >> 16) & 0xFF;
    if (exact) {
      plane64(A, na, ca);
      plane64(B, nb_, cb);
      plane64(C, nc, cc);
      v = refined ? solve3_refined(na, ca, pid[pb + A] >= 0, nb_, cb, pid[pb + B] >= 0, nc, cc, pid[pb + C] >= 0)
                  : solve3<double>(na, ca, nb_, cb, nc, cc);
    } else if (refined) {
      na = {(double)pnx[pb + A], (double)pny[pb + A], (double)pnz[pb + A]};
      ca = (double)pnc[pb + A];
      nb_ = {(double)pnx[pb + B], (double)pny[pb + B], (double)pnz[pb + B]};
      cb = (double)pnc[pb + B];
      nc = {(double)pnx[pb + C], (double)pny[pb + C], (double)pnz[pb + C]};
      cc = (double)pnc[pb + C];
      // bisector offsets are taken exactly only where the cached plane holds
      // the exact normal (double planes)
      constexpr bool kExactN = sizeof(R) == 8;
      v = solve3_refined(na, ca, kExactN && pid[pb + A] >= 0, nb_, cb, kExactN && pid[pb + B] >= 0, nc, cc,
                         kExactN && pid[pb + C] >= 0);
    } else {
      const int A = u & 0xFF, B = (u >> 8) & 0xFF, C = (u >> 16) & 0xFF;
      na = {(double)pnx[pb + A], (double)pny[pb + A], (double)pnz[pb + A]};
      ca = (double)pnc[pb + A];
      nb_ = {(double)pnx[pb + B], (double)pny[pb + B], (double)pnz[pb + B]};
      cb = (double)pnc[pb + B];
      nc = {(double)pnx[pb + C], (double)pny[pb + C], (double)pnz[pb + C]};
      cc = (double)pnc[pb + C];
      v = {(double)vx[vb + t], (double)vy[vb + t], (double)vz[vb + t]};
    }
  };
  auto cell_volume = [&](bool on, bool exact) -> double {
    double acc = 0.0;
    if (on) {
      for (int t = j; t < H; t += L) {
        const unsigned u = tri[vb + t];
        if (u == kEmpty) continue;
        V3<double> na, nb_, nc, v;
        double ca, cb, cc;
        // double planes: every vertex refined once (a vertex of nearly
        // parallel planes is otherwise off by its conditioning times u R)
        corner_geom(u, t, exact, na, ca, nb_, cb, nc, cc, v, exact || sizeof(R) == 8);
        const V3<double> eab = anchor(na, ca, nb_, cb), ebc = anchor(nb_, cb, nc, cc), eca = anchor(nc, cc, na, ca);
        const double fa = ca / dot(na, na), fb = cb / dot(nb_, nb_), fc = cc / dot(nc, nc);
        const V3<double> Fa = {fa * na.x, fa * na.y, fa * na.z};
        const V3<double> Fb = {fb * nb_.x, fb * nb_.y, fb * nb_.z};
        const V3<double> Fc = {fc * nc.x, fc * nc.y, fc * nc.z};
        acc += dot(Fa, cross(v, V3<double>{eca.x - eab.x, eca.y - eab.y, eca.z - eab.z}));
        acc += dot(Fb, cross(v, V3<double>{eab.x - ebc.x, eab.y - ebc.y, eab.z - ebc.z}));
        acc += dot(Fc, cross(v, V3<double>{ebc.x - eca.x, ebc.y - eca.y, ebc.z - eca.z}));
      }
    }
    return gsumd(acc) / 6.0;
  };
  double vol = cell_volume(cert, false);
  // Float vertices carry an absolute error ~u R; a cell much thinner than its
  // radius (R^3 > 16 V, i.e. u R^3 / V > 1e-6) cannot get its volume to 1e-5
  // from them, so its outputs are recomputed from vertices solved in double.
  bool refine = false;
  if (RECHECK) {
    refine = cert && (double)R2 * sqrt((double)R2) > 16.0 * vol;
    if (__any(refine)) {
      const double v2 = cell_volume(refine, true);
      if (refine) vol = v2;
    }
  }
  // Per-face outputs are computed in double from vertices solved in double
  // and refined once (a vertex of nearly parallel planes is otherwise off by
  // its conditioning times u, and so are the areas of its faces): planes
  // cached on the FP64 path, from the exact inputs on the float path.
  constexpr bool kExactFaces = RECHECK;
  // Cell centroid: the corner terms of the volume split into signed
  // tetrahedra from the seed, (0, F_f, v, e_fh) and (0, F_f, e_fg, v); the
  // first moment of each is its volume times the mean of its corners.
  double cmx = 0.0, cmy = 0.0, cmz = 0.0;
  if (a.centroid) {
    double w6 = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
    auto tet = [&](const V3<double>& x, const V3<double>& y, const V3<double>& z) {
      const double w = dot(x, cross(y, z));
      w6 += w;
      mx += w * (x.x + y.x + z.x);
      my += w * (x.y + y.y + z.y);
      mz += w * (x.z + y.z + z.z);
    };
    if (cert) {
      for (int t = j; t < H; t += L) {
        const unsigned u = tri[vb + t];
        if (u == kEmpty) continue;
        V3<double> na, nb_, nc, v;
        double ca, cb, cc;
        corner_geom(u, t, kExactFaces, na, ca, nb_, cb, nc, cc, v, true);
        const V3<double> eab = anchor(na, ca, nb_, cb), ebc = anchor(nb_, cb, nc, cc), eca = anchor(nc, cc, na, ca);
        const double fa = ca / dot(na, na), fb = cb / dot(nb_, nb_), fc = cc / dot(nc, nc);
        const V3<double> Fa = {fa * na.x, fa * na.y, fa * na.z};
        const V3<double> Fb = {fb * nb_.x, fb * nb_.y, fb * nb_.z};
        const V3<double> Fc = {fc * nc.x, fc * nc.y, fc * nc.z};
        tet(Fa, v, eca);
        tet(Fa, eab, v);
        tet(Fb, v, eab);
        tet(Fb, ebc, v);
        tet(Fc, v, ebc);
        tet(Fc, eca, v);
      }
    }
    const double V6 = gsumd(w6);
    mx = gsumd(mx);
    my = gsumd(my);
    mz = gsumd(mz);
    // moment / volume = (sum w m / 24) / (sum w / 6)
    if (V6 > 0.0) {
      cmx = p64x + mx / (4.0 * V6);
      cmy = p64y + my / (4.0 * V6);
      cmz = p64z + mz / (4.0 * V6);
    }
  }
  // Face areas: lane j owns plane slots j, j+L, ..., the slots it writes to
  // the neighbour list below.  A face is the fan of the volume's corner
  // terms: the corner of vertex v on face f, between edges f^g and f^h,
  // spans the area n_f . (v x (e_fh - e_fg)) / (2 |n_f|).  Every lane walks
  // all vertex slots in order, so each face sums its corners in slot order.
  constexpr int FO = PMAX / L;
  static_assert(FO * L == PMAX, "plane slots split evenly over the lanes");
  double farea[FO];
#pragma unroll
  for (int q = 0; q < FO; ++q) farea[q] = 0.0;
  if (a.area && cert) {
    for (int t = 0; t < H; ++t) {
      const unsigned u = tri[vb + t];
      if (u == kEmpty) continue;
      const int A = u & 0xFF, B = (u >> 8) & 0xFF, C = (u >> 16) & 0xFF;
      const bool oa = A % L == j, ob = B % L == j, oc = C % L == j;
      if (!(oa || ob || oc)) continue;
      V3<double> na, nb_, nc, v;
      double ca, cb, cc;
      corner_geom(u, t, kExactFaces, na, ca, nb_, cb, nc, cc, v, true);
      const V3<double> eab = anchor(na, ca, nb_, cb), ebc = anchor(nb_, cb, nc, cc), eca = anchor(nc, cc, na, ca);
      auto corner = [&](const V3<double>& n, const V3<double>& e1, const V3<double>& e0) -> double {
        return dot(n, cross(v, V3<double>{e1.x - e0.x, e1.y - e0.y, e1.z - e0.z})) / (2.0 * sqrt(dot(n, n)));
      };
      const double xa = oa ? corner(na, eca, eab) : 0.0;
      const double xb = ob ? corner(nb_, eab, ebc) : 0.0;
      const double xc = oc ? corner(nc, ebc, eca) : 0.0;
#pragma unroll
      for (int q = 0; q < FO; ++q) {
        const int f = j + q * L;
        farea[q] += (A == f ? xa : 0.0) + (B == f ? xb : 0.0) + (C == f ? xc : 0.0);
      }
    }
  }
  // neighbours: alive bisector planes
  int nnb = 0;
  for (int f = j; f < PMAX; f += L) nnb += cert && ((alive >> f) & 1) && pid[pb + f] >= 0;
  int ntot;
  int noff = gexcl(nnb, ntot);
  if (cert) {
#pragma unroll
    for (int q = 0; q < FO; ++q) {
      const int f = j + q * L;
      if (((alive >> f) & 1) && pid[pb + f] >= 0) {
        if (noff < a.max_nbr) {
          a.nbr[(size_t)row * a.max_nbr + noff] = pid[pb + f];
          if (a.area) a.area[(size_t)row * a.max_nbr + noff] = farea[q];
        }
        ++noff;
      }
    }
  }
  // vertices
  int vtot = 0;
  if (a.max_vert > 0) {
    int nv = 0;
    for (int t = j; t < H; t += L) nv += cert && tri[vb + t] != kEmpty;
    int voff = gexcl(nv, vtot);
    if (cert) {
      for (int t = j; t < H; t += L) {
        const unsigned u = tri[vb + t];
        if (u == kEmpty) continue;
        if (voff < a.max_vert) {
          const size_t o = ((size_t)row * a.max_vert + voff) * 3;
          V3<double> v = {(double)vx[vb + t], (double)vy[vb + t], (double)vz[vb + t]};
          if (refine) v = vertex64(u);
          a.verts[o + 0] = p64x + v.x;
          a.verts[o + 1] = p64y + v.y;
          a.verts[o + 2] = p64z + v.z;
          a.vplanes[o + 0] = pid[pb + (u & 0xFF)];
          a.vplanes[o + 1] = pid[pb + ((u >> 8) & 0xFF)];
          a.vplanes[o + 2] = pid[pb + ((u >> 16) & 0xFF)];
        }
        ++voff;
      }
    }
  }
  if (RECHECK) {
    int rc = nrecheck;
#pragma unroll
    for (int o = 1; o < L; o <<= 1) rc += shfl_xor_w(rc, o, L);
    nrecheck = rc;
  }
  if (have && j == 0) {
    int fin = st;
    if (fin == VOTESS_CELL_CERTIFIED && (ntot > a.max_nbr || (a.max_vert > 0 && vtot > a.max_vert)))
      fin = VOTESS_CELL_CAPACITY;
    a.status[row] = (uint8_t)fin;
    a.nbr_count[row] = fin == VOTESS_CELL_CERTIFIED ? ntot : 0;
    a.volume[row] = fin == VOTESS_CELL_CERTIFIED ? vol : 0.0;
    if (a.centroid) {
      const bool ok = fin == VOTESS_CELL_CERTIFIED;
      a.centroid[(size_t)row * 3 + 0] = ok ? cmx : 0.0;
      a.centroid[(size_t)row * 3 + 1] = ok ? cmy : 0.0;
      a.centroid[(size_t)row * 3 + 2] = ok ? cmz : 0.0;
    }
    if (a.kneeded) a.kneeded[row] = kneed;
    if (a.r2out) a.r2out[row] = fin == VOTESS_CELL_CERTIFIED ? (RECHECK ? (double)R2hi : (double)R2) : 0.0;
    if (a.vcount) a.vcount[row] = fin == VOTESS_CELL_CERTIFIED ? vtot : 0;
    if (a.counters) {
      if (nrecheck) atomicAdd(&a.counters[0], (unsigned long long)nrecheck);
      if (fin == VOTESS_CELL_UNRESOLVED) atomicAdd(&a.counters[1], 1ull);
      if (fin == VOTESS_CELL_CAPACITY) atomicAdd(&a.counters[2], 1ull);
      if (refine && fin == VOTESS_CELL_CERTIFIED) atomicAdd(&a.counters[3], 1ull);
    }
  }
}

template <typename P, typename R, int L, int TMAX, int PMAX, bool RECHECK>
votess_status run(const ClipArgs& ca, hipStream_t st) {
  constexpr int G = 64 / L;
  const unsigned blocks = (unsigned)(8 * (((ca.nc + G - 1) / G + 7) / 8));
  if (ca.stream)
    k_clip<P, R, L, TMAX, PMAX, RECHECK, true><<<blocks, 64, 0, st>>>(ca);
  else
    k_clip<P, R, L, TMAX, PMAX, RECHECK, false><<<blocks, 64, 0, st>>>(ca);
  VT_HIP(hipGetLastError());
  return VOTESS_OK;
}

}  // namespace

votess_status launch_clip(const ClipLaunch& a, hipStream_t st) {
  if (a.nc == 0) return VOTESS_OK;
  ClipArgs c;
  c.rec = a.sorted;
  c.n = a.n;
  c.lo0 = a.lo[0]; c.lo1 = a.lo[1]; c.lo2 = a.lo[2];
  c.hi0 = a.hi[0]; c.hi1 = a.hi[1]; c.hi2 = a.hi[2];
  c.cells = a.cells;
  c.nc = a.nc;
  c.knn = a.knn;
  c.k = a.k;
  c.kstride = a.knn_stride > 0 ? a.knn_stride : a.k;
  c.knn_by_id = a.knn_by_id;
  c.eps = a.eps;
  // k-lists ordered by float distances may misplace near-ties by a few ulp:
  // certify only with that much slack
  c.dmargin = a.knn_dist == VOTESS_F32 ? (1.0 - 8.0 * (double)FLT_EPSILON) : 1.0;
  c.max_nbr = a.max_nbr;
  c.max_vert = a.max_vert;
  c.out_by_id = a.out_by_id;
  c.status = a.status;
  c.nbr_count = a.nbr_count;
  c.nbr = a.nbr;
  c.volume = a.volume;
  c.kneeded = a.kneeded;
  c.vcount = a.vcount;
  c.verts = a.verts;
  c.vplanes = a.vplanes;
  c.area = a.area;
  c.centroid = a.centroid;
  c.r2out = a.r2out;
  c.counters = a.counters;
  c.stream = a.stream;
  c.cell_start = a.cell_start;
  c.grid = a.grid;
  c.sub = a.sub;
  const bool f32 = a.precision == VOTESS_CLIP_F32_RECHECK;
  if (f32 && a.dtype != VOTESS_F32) return fail(VOTESS_EINVAL, "clip: F32_RECHECK needs F32 positions");
  if (a.stream && (a.knn_dist == VOTESS_F32) != f32)
    return fail(VOTESS_EINVAL, "clip: the stream phase needs k-lists built in the clip precision");
  if (a.stream && !a.cell_start) return fail(VOTESS_EINVAL, "clip: the stream phase needs cell_start");
  // the fast kernel: 16 lanes per cell, measured faster than 8 (fewer cells
  // per wave diverge in the stream phase) and than 4 or 32
  if (a.capacity == 0) {
    if (f32) return run<float, float, 16, 64, 32, true>(c, st);
    if (a.dtype == VOTESS_F32) return run<float, double, 16, 64, 32, false>(c, st);
    return run<double, double, 16, 64, 32, false>(c, st);
  }
  // the large-capacity kernel: 32 lanes per cell (two cells per wave keep its
  // LDS per workgroup low enough for more than one wave per SIMD)
  if (f32) return run<float, float, 32, 256, 64, true>(c, st);
  if (a.dtype == VOTESS_F32) return run<float, double, 32, 256, 64, false>(c, st);
  return run<double, double, 32, 256, 64, false>(c, st);
}

}  // namespace votess
