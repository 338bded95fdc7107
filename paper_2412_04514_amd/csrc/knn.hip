// k-nearest-neighbour search over the grid (paper, Summary section: the
// neighbour search that follows the grid sort).
//
// A group of G lanes serves one query (queries in grid-sorted order, so that
// neighbouring groups scan overlapping grid cells), in two phases:
//   A. a seed block around the query -- sub-cells of its own dense cell, or
//      grid cells -- grown ring by ring until the cell / sub-cell starts show
//      at least K other points in it, then scanned whole: the list is full;
//   B. every other grid-cell row, and sub-cell row of a dense cell, that
//      meets the ball of the list's current k-th distance, each row cut to
//      the ball (which shrinks as the list improves): one contiguous range of
//      sorted points per row, split at dense cells.
// The control flow is the same in every lane of the group; the candidates of
// a range are taken G at a time (one coalesced load), and each that beats the
// current k-th is inserted by rank into the ascending list, which the group
// holds as E = K / G consecutive entries per lane.
#include "internal.h"
#include "device_common.h"

#include <cfloat>
#include <climits>

namespace votess {
namespace {

// List keys ordered by (d^2, sorted index).  FP32 distances pack into one
// u64: the bits of a non-negative float order like the float.
template <typename D>
struct KeyOps;
template <>
struct KeyOps<float> {
  using Key = unsigned long long;
  __device__ static Key make(float d2, int j) { return ((unsigned long long)__float_as_uint(d2) << 32) | (unsigned)j; }
  __device__ static Key inf() { return ~0ull; }
  __device__ static bool less(Key a, Key b) { return a < b; }
  __device__ static bool finite(Key a) { return a != ~0ull; }
  __device__ static double d2(Key a) { return (double)__uint_as_float((unsigned)(a >> 32)); }
  __device__ static int idx(Key a) { return a == ~0ull ? -1 : (int)(unsigned)(a & 0xffffffffu); }
  __device__ static Key shfl(Key a, int src) { return __shfl(a, src, 64); }
  __device__ static Key pick(bool c, Key a, Key b) { return c ? a : b; }
  // f applied to each 32-bit word of the key
  template <class F>
  __device__ static Key each_word(Key a, F f) {
    return ((unsigned long long)f((unsigned)(a >> 32)) << 32) | f((unsigned)a);
  }
};
template <>
struct KeyOps<double> {
  struct Key {
    double d;
    int i;
  };
  __device__ static Key make(double d2, int j) { return {d2, j}; }
  __device__ static Key inf() { return {DBL_MAX, INT_MAX}; }
  __device__ static bool less(const Key& a, const Key& b) { return a.d < b.d || (a.d == b.d && a.i < b.i); }
  __device__ static bool finite(const Key& a) { return a.i != INT_MAX; }
  __device__ static double d2(const Key& a) { return a.d; }
  __device__ static int idx(const Key& a) { return a.i == INT_MAX ? -1 : a.i; }
  __device__ static Key shfl(const Key& a, int src) { return {__shfl(a.d, src, 64), __shfl(a.i, src, 64)}; }
  // field by field: a choice between two structs as lvalues would select
  // their addresses and keep the list in scratch memory
  __device__ static Key pick(bool c, const Key& a, const Key& b) { return {c ? a.d : b.d, c ? a.i : b.i}; }
  template <class F>
  __device__ static Key each_word(const Key& a, F f) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(a.d);
    const unsigned long long w = ((unsigned long long)f((unsigned)(u >> 32)) << 32) | f((unsigned)u);
    return {__longlong_as_double((long long)w), (int)f((unsigned)a.i)};
  }
};

// Moves of 32-bit words between the lanes of a group of G consecutive lanes.
// For G = 4, 8 or 16 they are DPP row operations, which stay in the vector
// ALU (controls: quad_perm [1,0,3,2] = 0xB1 takes lane ^ 1, [2,3,0,1] = 0x4E
// lane ^ 2, [3,2,1,0] = 0x1B reverses a quad, [3,3,3,3] = 0xFF broadcasts
// its last lane; row_shr:1 = 0x111 takes lane - 1 within a row of 16;
// row_mirror = 0x140 takes lane 15 - i within the row, row_half_mirror =
// 0x141 lane 7 - i within each eight); a group of 32 or 64 uses the LDS
// permute.  Every lane of the group is active.
template <int CTRL>
__device__ __forceinline__ unsigned dpp_mov(unsigned v) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, true);
}
template <int G>
struct LaneMove {
  static constexpr bool kDpp = G == 4 || G == 8 || G == 16;
  // the word of lane l ^ m (m a power of two below G)
  __device__ static unsigned xor_(unsigned v, int m) {
    if constexpr (kDpp) {
      if (m == 1) return dpp_mov<0xB1>(v);
      if (m == 2) return dpp_mov<0x4E>(v);
      if (m == 4) return dpp_mov<0x141>(dpp_mov<0x1B>(v));  // i -> 3 - i in the quad, then 7 - i
      if (m == 8) return dpp_mov<0x140>(dpp_mov<0x141>(v));  // 7 - i in the eight, then 15 - i
    }
    return (unsigned)__shfl_xor((int)v, m, 64);
  }
  // the word of lane l - 1 (what group lane 0 receives is not used)
  __device__ static unsigned prev(unsigned v, int lane) {
    if constexpr (kDpp) return dpp_mov<0x111>(v);
    return (unsigned)__shfl((int)v, lane > 0 ? lane - 1 : 0, 64);
  }
  // the word of the group's last lane
  __device__ static unsigned last(unsigned v, int gb, int l) {
    if constexpr (G == 4) {
      return dpp_mov<0xFF>(v);
    } else if constexpr (G == 8) {
      const unsigned a = dpp_mov<0xFF>(v);  // each quad: its last lane
      const unsigned b = dpp_mov<0x141>(a);  // the other quad's
      return l < 4 ? b : a;
    } else if constexpr (G == 16) {
      const unsigned a = dpp_mov<0xFF>(v), b = dpp_mov<0x140>(a), c = dpp_mov<0x141>(a), d = dpp_mov<0x140>(c);
      return l < 4 ? b : (l < 8 ? d : (l < 12 ? c : a));
    } else {
      return (unsigned)__shfl((int)v, gb + G - 1, 64);
    }
  }
};

// Ascending list of K keys over a group of G lanes: lane l holds ranks
// l E .. l E + E - 1.  Every call is made by all G lanes of the group.
template <typename D, int G, int E>
struct GroupList {
  using O = KeyOps<D>;
  using Key = typename O::Key;
  Key key[E];
  __device__ void init() {
#pragma unroll
    for (int e = 0; e < E; ++e) key[e] = O::inf();
  }
  using LM = LaneMove<G>;
  __device__ Key worst(int gb, int l) const {
    return O::each_word(key[E - 1], [&](unsigned w) { return LM::last(w, gb, l); });
  }
  // insert x (the same in every lane): its rank is the number of smaller
  // keys; ranks above it move up by one, the old k-th falls off
  __device__ void insert(const Key& x, int lane, int l) {
    int c = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) c += O::less(key[e], x) ? 1 : 0;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) c += (int)LM::xor_((unsigned)c, o);
    const Key prev = O::each_word(key[E - 1], [&](unsigned w) { return LM::prev(w, lane); });
#pragma unroll
    for (int e = E - 1; e >= 0; --e) {
      const int p = l * E + e;
      const Key below = O::pick(e > 0, key[e > 0 ? e - 1 : 0], prev);
      key[e] = O::pick(p < c, key[e], O::pick(p == c, x, below));
    }
  }
  // Sorts the K keys ascending in place (K and E powers of two): a bitonic
  // network over positions i = l E + e, exchanges inside a lane in
  // registers, across lanes by shuffles.  Keys are distinct (the index is
  // part of the key), so the result is the same as inserting them one by one.
  __device__ void sort(int l) {
#pragma unroll
    for (int ks = 2; ks <= G * E; ks <<= 1) {
#pragma unroll
      for (int js = ks >> 1; js > 0; js >>= 1) {
        if (js < E) {
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const int pe = e ^ js;
            if (pe > e) {
              const bool up = ((l * E + e) & ks) == 0;
              const Key a = key[e], b = key[pe];
              const bool sw = up ? O::less(b, a) : O::less(a, b);
              key[e] = O::pick(sw, b, a);
              key[pe] = O::pick(sw, a, b);
            }
          }
        } else {
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const int i = l * E + e;
            const Key o = O::each_word(key[e], [&](unsigned w) { return LM::xor_(w, js / E); });
            const bool keep_min = (((i & ks) == 0) == ((i & js) == 0));
            const bool o_less = O::less(o, key[e]);
            key[e] = O::pick(keep_min == o_less, o, key[e]);
          }
        }
      }
    }
  }
};

// Held to 6 waves per SIMD (80 VGPRs; the k = 64 float kernel keeps 132
// bytes per lane in scratch): the search is latency-bound; at k = 64 on
// clustered input six waves measured faster than five (3%), four (10%,
// without spills), seven (5%) and eight (16%).
// Blocks are taken in an XCD-aware order: the hardware deals launched
// blocks round-robin over the eight XCDs, so launched block b runs logical
// block (b mod 8) per + b / 8 (per = blocks / 8, rounded up; the launch is
// padded to 8 per) and each XCD works on one contiguous stretch of the
// grid-sorted queries, whose candidates its own L2 then holds.
template <typename T, typename D, int K, int GS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_knn(const typename Rec<T>::type* __restrict__ rec, int n, GridDev G,
                                             const int* __restrict__ cell_start, SubGrid sub,
                                             const int* __restrict__ queries, int nq, int* __restrict__ knn,
                                             unsigned* __restrict__ err, int nblocks) {
  constexpr int E = K / GS;
  static_assert(E * GS == K, "K must be a multiple of GS");
  using O = KeyOps<D>;
  using Key = typename O::Key;
  const int per = (nblocks + 7) / 8;
  const int lb = (int)(blockIdx.x % 8u) * per + (int)(blockIdx.x / 8u);
  if (lb >= nblocks) return;
  const int lane = threadIdx.x & 63;
  const int l = lane & (GS - 1), gb = lane - l;
  const int q = (int)(((long long)lb * blockDim.x + threadIdx.x) / GS);
  if (q >= nq) return;  // whole groups leave together
  const int s = queries ? queries[q] : q;
  const auto pr = rec[s];
  const D px = (D)pr.x, py = (D)pr.y, pz = (D)pr.z;
  const int cx = axis_cell((double)pr.x, G.lo0, G.ih0, G.g0);
  const int cy = axis_cell((double)pr.y, G.lo1, G.ih1, G.g1);
  const int cz = axis_cell((double)pr.z, G.lo2, G.ih2, G.g2);
  const double ext = fmax(G.hi0 - G.lo0, fmax(G.hi1 - G.lo1, G.hi2 - G.lo2));
  const double margin = 1e-9 * ext;  // covers floor() rounding at cell borders

  GroupList<D, GS, E> L;
  L.init();
  Key wk = O::inf();  // the list's k-th key (group-uniform)
  // The first K candidates are not inserted one by one: they are gathered in
  // LDS (per group, in scan order) and sorted once: K and E powers of two,
  // K <= 64 for float keys and <= 32 for (double, index) keys (larger
  // networks no longer stay in registers).
  constexpr bool kSortFill = K <= (sizeof(Key) == 8 ? 64 : 32) && ((K & (K - 1)) == 0) && ((E & (E - 1)) == 0);
  constexpr int FB = kSortFill ? (256 / GS) * K : 1;
  __shared__ Key sfill[FB];
  Key* gfill = sfill + (kSortFill ? ((threadIdx.x & 255) / GS) * K : 0);
  // phase B: point ranges of up to GS sub-rows of a dense cell (two per
  // sub-row at most), per group
  __shared__ int2 srng[(256 / GS) * 2 * GS];
  int2* grng = srng + ((threadIdx.x & 255) / GS) * 2 * GS;
  bool filling = kSortFill;
  int nfill = 0;
  const double p0 = (double)pr.x, p1 = (double)pr.y, p2 = (double)pr.z;
  const unsigned long long gmask = (GS == 64) ? ~0ull : ((1ull << GS) - 1ull);

  // one candidate per lane (ck: its key, infinite when !valid): gathered
  // into the initial fill while that lasts, else inserted when it beats the
  // k-th
  auto consider = [&](bool valid, Key ck) {
    bool pass;
    if (kSortFill && filling) {
      const unsigned long long vm = (__ballot(valid) >> gb) & gmask;
      const int pos = nfill + __popcll(vm & ((1ull << l) - 1ull));
      if (valid && pos < K) gfill[pos] = ck;
      nfill += __popcll(vm);
      if (nfill < K) return;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
      for (int e = 0; e < E; ++e) L.key[e] = gfill[l * E + e];
      L.sort(l);
      wk = L.worst(gb, l);
      filling = false;
      pass = valid && pos >= K && O::less(ck, wk);  // the batch's candidates past the first K
    } else {
      pass = O::less(ck, wk);
    }
    unsigned long long m = (__ballot(pass) >> gb) & gmask;
    while (m) {
      const int b = __ffsll((long long)m) - 1;
      const Key x = O::shfl(ck, gb + b);
      L.insert(x, lane, l);
      wk = L.worst(gb, l);
      pass = pass && l != b && O::less(ck, wk);
      m = (__ballot(pass) >> gb) & gmask;
    }
  };
  // candidates [jb, je), GS at a time; each that beats the k-th is inserted
  // with float keys the records of a batch are loaded one batch ahead, so
  // that their latency overlaps the previous batch's ranking and insertions
  // (with (double, index) keys the extra registers cost more than it saves)
  constexpr bool kPrefetch = sizeof(Key) == 8;
  auto scan = [&](int jb, int je) {
    auto nxt = rec[jb + l < je ? jb + l : s];
    for (int base = jb; base < je; base += GS) {
      const int j = base + l;
      const auto qr = kPrefetch ? nxt : rec[j < je ? j : s];
      if (kPrefetch && base + GS < je) nxt = rec[base + GS + l < je ? base + GS + l : s];
      Key ck = O::inf();
      const bool valid = j < je && j != s;
      if (valid) ck = O::make(dist2_nc((D)qr.x - px, (D)qr.y - py, (D)qr.z - pz), j);
      consider(valid, ck);
    }
  };
  // candidates of the n ranges listed in grng, GS at a time, a batch taking
  // the rest of one range and the start of the next ones
  auto scan_list = [&](int n) {
    int r = 0;
    int cur = 0, end = 0;
    if (n > 0) {
      cur = grng[0].x;
      end = grng[0].y;
    }
    while (r < n) {
      int jj = -1, nb = 0;
      while (nb < GS && r < n) {
        const int take = min(GS - nb, end - cur);
        if (l >= nb && l < nb + take) jj = cur + (l - nb);
        nb += take;
        cur += take;
        if (cur >= end && ++r < n) {
          cur = grng[r].x;
          end = grng[r].y;
        }
      }
      Key ck = O::inf();
      const bool valid = jj >= 0 && jj != s;
      if (valid) {
        const auto qr = rec[jj];
        ck = O::make(dist2_nc((D)qr.x - px, (D)qr.y - py, (D)qr.z - pz), jj);
      }
      consider(valid, ck);
    }
  };
  // scans the rows (y, z) of a block [y0, y1] x [z0, z1]: row_range(y, z)
  // gives a row's point range; GS rows at a time, one per lane, listed and
  // scanned together.  Rows go outward from row (yc, zc) (offsets 0, +1, -1,
  // +2, ... in z, and in y within each z), so that the list's first K
  // candidates lie near the query and fewer later ones displace them.
  auto scan_rows = [&](int y0, int y1, int z0, int z1, int yc, int zc, auto row_range) {
    const int ny = 2 * max(yc - y0, y1 - yc) + 1, npairs = ny * (2 * max(zc - z0, z1 - zc) + 1);
    for (int pb = 0; pb < npairs; pb += GS) {
      const int pi = pb + l;
      int2 rg = make_int2(0, 0);
      if (pi < npairs) {
        const int kz = pi / ny, ky = pi - kz * ny;
        const int z = zc + ((kz & 1) ? (kz + 1) >> 1 : -(kz >> 1));
        const int y = yc + ((ky & 1) ? (ky + 1) >> 1 : -(ky >> 1));
        if (z >= z0 && z <= z1 && y >= y0 && y <= y1) rg = row_range(y, z);
      }
      const bool k0 = rg.x < rg.y;
      const unsigned long long b0 = (__ballot(k0) >> gb) & gmask;
      if (k0) grng[__popcll(b0 & ((1ull << l) - 1ull))] = rg;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      scan_list(__popcll(b0));
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
  };
  // number of points in the rows of a block, summed over the group's lanes
  auto count_rows = [&](int y0, int y1, int z0, int z1, auto row_range) -> int {
    const int ny = y1 - y0 + 1, npairs = ny * (z1 - z0 + 1);
    int cnt = 0;
    for (int pi = l; pi < npairs; pi += GS) {
      const int2 rg = row_range(y0 + pi % ny, z0 + pi / ny);
      cnt += rg.y - rg.x;
    }
#pragma unroll
    for (int o = 1; o < GS; o <<= 1) cnt += __shfl_xor(cnt, o, 64);
    return cnt;
  };
  // squared search radius: the k-th distance with slack for float rounding
  // of d^2 (the list is full whenever it is used)
  auto rad2 = [&]() { return O::d2(wk) * (1.0 + 1e-6); };
  // distance from p to [a, b], less the rounding margin
  auto gap = [&](double p, double a_, double b_) { return fmax(0.0, fmax(a_ - p, p - b_) - margin); };

  // ---- phase A: a seed block around the query that holds at least K other
  // points (counted from the cell and sub-cell starts), scanned whole; it
  // fills the list, and its k-th distance bounds the search
  const int c0 = cx + G.g0 * (cy + G.g1 * cz);
  const int2 info0 = sub.info ? sub.info[c0] : make_int2(-1, 0);
  const bool seed_sub = info0.x >= 0 && cell_start[c0 + 1] - cell_start[c0] >= K + 1;
  int bx0, bx1, by0, by1, bz0, bz1;  // the seed block: sub-cells of the own cell, or grid cells
  if (seed_sub) {
    const int* srec = sub.start + info0.x;
    const SubCell sc = sub_cell(srec);
    const int base0 = cell_start[c0];
    const int qx = sub_axis(p0, sc.lo0, sc.ih0, sc.m0), qy = sub_axis(p1, sc.lo1, sc.ih1, sc.m1),
              qz = sub_axis(p2, sc.lo2, sc.ih2, sc.m2);
    auto srow = [&](int y, int z) {
      const int row = kSubHead + sc.m0 * (y + sc.m1 * z);
      return make_int2(base0 + srec[row + bx0], base0 + srec[row + bx1 + 1]);
    };
    for (int rs = 0;; ++rs) {
      bx0 = max(qx - rs, 0); bx1 = min(qx + rs, sc.m0 - 1);
      by0 = max(qy - rs, 0); by1 = min(qy + rs, sc.m1 - 1);
      bz0 = max(qz - rs, 0); bz1 = min(qz + rs, sc.m2 - 1);
      const int cnt = count_rows(by0, by1, bz0, bz1, srow);
      if (cnt >= K + 1 || (bx0 == 0 && by0 == 0 && bz0 == 0 && bx1 == sc.m0 - 1 && by1 == sc.m1 - 1 &&
                           bz1 == sc.m2 - 1))
        break;
    }
    scan_rows(by0, by1, bz0, bz1, qy, qz, srow);
  } else {
    auto grow = [&](int y, int z) {
      const int row = G.g0 * (y + G.g1 * z);
      return make_int2(cell_start[row + bx0], cell_start[row + bx1 + 1]);
    };
    for (int r = 0;; ++r) {
      bx0 = max(cx - r, 0); bx1 = min(cx + r, G.g0 - 1);
      by0 = max(cy - r, 0); by1 = min(cy + r, G.g1 - 1);
      bz0 = max(cz - r, 0); bz1 = min(cz + r, G.g2 - 1);
      const int cnt = count_rows(by0, by1, bz0, bz1, grow);
      if (cnt >= K + 1 || (bx0 == 0 && by0 == 0 && bz0 == 0 && bx1 == G.g0 - 1 && by1 == G.g1 - 1 &&
                           bz1 == G.g2 - 1))
        break;
    }
    scan_rows(by0, by1, bz0, bz1, cy, cz, grow);
  }

  if (kSortFill && filling) {  // fewer than K other points: sort what there is
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
    for (int e = 0; e < E; ++e) L.key[e] = O::pick(l * E + e < nfill, gfill[l * E + e], O::inf());
    L.sort(l);
    wk = L.worst(gb, l);
    filling = false;
  }

  // ---- phase B: every other grid cell / sub-cell row that meets the ball of
  // the list's k-th distance (re-cut to the shrinking ball row by row)
  // a dense cell c (grid coordinates ccx, ccy, ccz), without the seed block
  // when it is the query's own cell
  auto scan_dense = [&](int c, int ccx, int ccy, int ccz, bool own) {
    const int* drec = sub.start + sub.info[c].x;
    const SubCell sc = sub_cell(drec);
    const int base = cell_start[c];
    const double w1 = 1.0 / sc.ih1, w2 = 1.0 / sc.ih2;
    const double ylo = G.lo1 + ccy * G.h1, yhi = ylo + G.h1, zlo = G.lo2 + ccz * G.h2, zhi = zlo + G.h2;
    // sub-rows (sy, sz) of the square that meets the ball, GS at a time, one
    // per lane: each lane cuts its sub-row to the ball and reads its point
    // range(s); the non-empty ranges are listed and scanned together
    const double r0 = sqrt(rad2()) + margin;
    const int sz0 = sub_axis(p2 - r0, sc.lo2, sc.ih2, sc.m2), sz1 = sub_axis(p2 + r0, sc.lo2, sc.ih2, sc.m2);
    const int sy0 = sub_axis(p1 - r0, sc.lo1, sc.ih1, sc.m1), sy1 = sub_axis(p1 + r0, sc.lo1, sc.ih1, sc.m1);
    const int ny = sy1 - sy0 + 1, npairs = ny * (sz1 - sz0 + 1);
    for (int pb = 0; pb < npairs; pb += GS) {
      const int pi = pb + l;
      int lo0 = 0, hi0 = 0, lo1 = 0, hi1 = 0;
      if (pi < npairs) {
        const int sz = sz0 + pi / ny, sy = sy0 + pi % ny;
        const double za = sz == 0 ? zlo : sc.lo2 + sz * w2, zb = sz == sc.m2 - 1 ? zhi : sc.lo2 + (sz + 1) * w2;
        const double ya = sy == 0 ? ylo : sc.lo1 + sy * w1, yb = sy == sc.m1 - 1 ? yhi : sc.lo1 + (sy + 1) * w1;
        const double gz = gap(p2, za, zb), gy = gap(p1, ya, yb);
        const double rem = rad2() - gz * gz - gy * gy;
        if (rem >= 0.0) {
          const double rx = sqrt(rem) + margin;
          int sx0 = sub_axis(p0 - rx, sc.lo0, sc.ih0, sc.m0), sx1 = sub_axis(p0 + rx, sc.lo0, sc.ih0, sc.m0);
          const int row = kSubHead + sc.m0 * (sy + sc.m1 * sz);
          if (own && sy >= by0 && sy <= by1 && sz >= bz0 && sz <= bz1) {
            // the seed block's sub-cells were scanned whole
            if (sx0 < bx0) {
              lo0 = base + drec[row + sx0];
              hi0 = base + drec[row + min(sx1, bx0 - 1) + 1];
            }
            sx0 = max(sx0, bx1 + 1);
          }
          if (sx0 <= sx1) {
            lo1 = base + drec[row + sx0];
            hi1 = base + drec[row + sx1 + 1];
          }
        }
      }
      const bool k0 = lo0 < hi0, k1 = lo1 < hi1;
      const unsigned long long b0 = (__ballot(k0) >> gb) & gmask, b1 = (__ballot(k1) >> gb) & gmask;
      const unsigned long long below = (1ull << l) - 1ull;
      const int w = __popcll(b0 & below) + __popcll(b1 & below);
      if (k0) grng[w] = make_int2(lo0, hi0);
      if (k1) grng[w + (k0 ? 1 : 0)] = make_int2(lo1, hi1);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      scan_list(__popcll(b0) + __popcll(b1));
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
  };
  if (O::finite(wk)) {
    const double rz = sqrt(rad2()) + margin;
    const int gz0 = axis_cell(p2 - rz, G.lo2, G.ih2, G.g2), gz1 = axis_cell(p2 + rz, G.lo2, G.ih2, G.g2);
    for (int z = gz0; z <= gz1; ++z) {
      const double gz = gap(p2, G.lo2 + z * G.h2, G.lo2 + (z + 1) * G.h2);
      const double remz = rad2() - gz * gz;
      if (remz < 0.0) continue;
      const double ry = sqrt(remz) + margin;
      const int gy0 = axis_cell(p1 - ry, G.lo1, G.ih1, G.g1), gy1 = axis_cell(p1 + ry, G.lo1, G.ih1, G.g1);
      for (int y = gy0; y <= gy1; ++y) {
        const double gy = gap(p1, G.lo1 + y * G.h1, G.lo1 + (y + 1) * G.h1);
        const double rem = rad2() - gz * gz - gy * gy;
        if (rem < 0.0) continue;
        const double rx = sqrt(rem) + margin;
        const int x0 = axis_cell(p0 - rx, G.lo0, G.ih0, G.g0), x1 = axis_cell(p0 + rx, G.lo0, G.ih0, G.g0);
        const int row = G.g0 * (y + G.g1 * z);
        // grid cells of the seed block were scanned whole
        const bool in_seed = !seed_sub && y >= by0 && y <= by1 && z >= bz0 && z <= bz1;
        int x = x0;
        while (x <= x1) {
          if (in_seed && x >= bx0 && x <= bx1) {
            x = bx1 + 1;
            continue;
          }
          const int lim = (in_seed && x < bx0) ? min(x1, bx0 - 1) : x1;
          int xe = x;
          if (sub.info) {
            // the stretch of cells without sub-grids: the group reads GS
            // consecutive cells' records at once and ends it at the first
            // dense one
            for (;;) {
              const int xc = xe + l;
              const bool dense = xc <= lim && sub.info[row + xc].x >= 0;
              const unsigned long long dm = (__ballot(dense) >> gb) & gmask;
              if (dm) {
                xe += __ffsll((long long)dm) - 1;
                break;
              }
              xe += GS;
              if (xe > lim) {
                xe = lim + 1;
                break;
              }
            }
          } else {
            xe = lim + 1;
          }
          if (xe > x) {  // a stretch of cells without sub-grids
            scan(cell_start[row + x], cell_start[row + xe]);
            x = xe;
            continue;
          }
          scan_dense(row + x, x, y, z, seed_sub && row + x == c0);
          ++x;
        }
      }
    }
  }
  int* out = knn + (size_t)q * K + l * E;
#pragma unroll
  for (int e = 0; e < E; ++e) out[e] = O::idx(L.key[e]);
  if (l == 0 && O::finite(L.key[0]) && O::d2(L.key[0]) == 0.0) atomicOr(err, ERR_DUPLICATE);
}

template <typename T, typename D>
votess_status dispatch_k(int k, const void* sorted, int n, const GridDev& G, const int32_t* cs, const SubGrid& sub,
                         const int32_t* qs, int nq, int32_t* knn, unsigned* err, hipStream_t st) {
  using R4 = typename Rec<T>::type;
  const R4* rec = (const R4*)sorted;
#define VT_KNN_CASE(KK, GG)                                                                 \
  case KK: {                                                                                \
    const int blocks = (int)(((long long)nq * GG + 255) / 256);                             \
    const unsigned launched = (unsigned)(8 * ((blocks + 7) / 8));                           \
    k_knn<T, D, KK, GG><<<launched, 256, 0, st>>>(rec, n, G, cs, sub, qs, nq, knn, err, blocks); \
    break;                                                                                  \
  }
  switch (k) {
    VT_KNN_CASE(8, 4)
    VT_KNN_CASE(12, 4)
    VT_KNN_CASE(16, 4)
    VT_KNN_CASE(24, 8)
    VT_KNN_CASE(32, 8)
    VT_KNN_CASE(48, 16)
    VT_KNN_CASE(64, 16)
    VT_KNN_CASE(128, 16)
    VT_KNN_CASE(256, 32)
    default:
      return fail(VOTESS_EINVAL, "knn: k=%d has no kernel (k must be one of 8,12,16,24,32,48,64,128,256)", k);
  }
#undef VT_KNN_CASE
  VT_HIP(hipGetLastError());
  return VOTESS_OK;
}

}  // namespace

votess_status launch_knn(votess_ctx* ctx, const void* sorted, votess_dtype dt, int n, const GridDev& G,
                         const int32_t* cell_start, const SubGrid& sub, const int32_t* queries, int nq, int k,
                         votess_dtype dist, int32_t* knn, hipStream_t st) {
  if (nq == 0) return VOTESS_OK;
  if (dt == VOTESS_F64 && dist == VOTESS_F32)
    return fail(VOTESS_EINVAL, "knn: F32 distances need F32 positions");
  if (dt == VOTESS_F32) {
    if (dist == VOTESS_F32) return dispatch_k<float, float>(k, sorted, n, G, cell_start, sub, queries, nq, knn, ctx->d_err, st);
    return dispatch_k<float, double>(k, sorted, n, G, cell_start, sub, queries, nq, knn, ctx->d_err, st);
  }
  return dispatch_k<double, double>(k, sorted, n, G, cell_start, sub, queries, nq, knn, ctx->d_err, st);
}

}  // namespace votess
