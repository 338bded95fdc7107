// FP64 CPU oracle for the cell-by-cell 3D Voronoi method.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
// calls this file; only the test suite, the smoke check and the benchmark's
// CPU-baseline leg do.  It shares no code, header or table with the HIP path.
//
// What it computes (paper, Summary section): the Voronoi cell of every
// generator, built by clipping a bounding box with the perpendicular bisectors
// between the generator and its neighbours, with a security-radius test that
// proves the cell complete; outputs are cell geometry and natural-neighbour
// lists (Features section).  The security-radius lemma is the one of the cited
// method (Ray et al. 2018, "Meshless Voronoi on the GPU"): if every vertex of
// the current polyhedron lies within R of the seed, no point farther than 2R
// can cut it, because its bisector is at distance > R from the seed.
//
// Representation: primal polyhedron, coordinates relative to the seed; each
// face is a cyclic vertex list, counter-clockwise seen from outside, tagged
// with its plane id (>= 0: neighbour index; -1..-6: box walls x-,x+,y-,y+,z-,z+).
// Clipping is Sutherland-Hodgman per face plus a cap face on the new plane.
// All arithmetic is IEEE double; the build uses -ffp-contract=off.
//
// Readings where the paper is silent (each listed in the design notes):
//  * the box is user-given and closed; points outside it are an error;
//  * a vertex exactly on a clipping plane (s == 0) counts as inside;
//  * a neighbour is a face of positive area; box walls are not neighbours;
//  * the certificate is strict: certified iff d^2 > 4 R^2.
//
// The oracle enumerates candidates with its own uniform grid (about four
// points per grid cell) ring by ring (Chebyshev shells), in (d^2, index) order
// inside a ring, and stops when the scanned block provably contains every
// point closer than 2R.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <map>
#include <tuple>
#include <vector>
#include <omp.h>

namespace {

using V3 = std::array<double, 3>;

inline double dot3(const V3& a, const V3& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline V3 sub3(const V3& a, const V3& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
inline V3 cross3(const V3& a, const V3& b) {
  return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}

struct Work {            // counts of the method's elementary operations
  int64_t tested = 0;    // bisector planes tested against the polyhedron
  int64_t cuts = 0;      // planes that removed at least one vertex
  int64_t evals = 0;     // vertex-versus-plane evaluations
  int64_t created = 0;   // vertices created by cuts
  int64_t r2 = 0;        // vertex norms evaluated to update R^2 after cuts
};

struct Poly {
  std::vector<V3> v;
  std::vector<std::vector<int>> f;
  std::vector<int64_t> fid;

  void box(const double lo[3], const double hi[3], const V3& p) {
    v.resize(8);
    for (int i = 0; i < 8; ++i)
      v[i] = {((i & 1) ? hi[0] : lo[0]) - p[0], ((i & 2) ? hi[1] : lo[1]) - p[1],
              ((i & 4) ? hi[2] : lo[2]) - p[2]};
    // vertex i has x from bit 0, y from bit 1, z from bit 2
    f = {{0, 4, 6, 2}, {1, 3, 7, 5}, {0, 1, 5, 4}, {2, 6, 7, 3}, {0, 2, 3, 1}, {4, 5, 7, 6}};
    fid = {-1, -2, -3, -4, -5, -6};
  }

  double radius2() const {
    double r = 0.0;
    for (const V3& x : v) r = std::max(r, dot3(x, x));
    return r;
  }

  // Clip by {x : n.x <= c}; returns true if some vertex was removed.
  bool clip(const V3& n, double c, int64_t id, Work& w) {
    const int nv = (int)v.size();
    std::vector<double> s(nv);
    bool any = false;
    for (int i = 0; i < nv; ++i) {
      s[i] = dot3(n, v[i]) - c;
      any = any || (s[i] > 0.0);
    }
    w.tested += 1;
    w.evals += nv;
    if (!any) return false;
    w.cuts += 1;

    std::vector<V3> nvtx;
    std::vector<int> remap(nv, -1);
    for (int i = 0; i < nv; ++i)
      if (!(s[i] > 0.0)) {
        remap[i] = (int)nvtx.size();
        nvtx.push_back(v[i]);
      }
    std::map<std::pair<int, int>, int> epts;  // crossing edge -> new vertex
    auto edge_point = [&](int a, int b) {
      // a inside (s <= 0), b outside (s > 0), or the reverse
      const int i = std::min(a, b), o = std::max(a, b);
      auto it = epts.find({i, o});
      if (it != epts.end()) return it->second;
      const int in = (s[a] > 0.0) ? b : a, out = (s[a] > 0.0) ? a : b;
      const double t = s[in] / (s[in] - s[out]);
      const V3 x = {v[in][0] + t * (v[out][0] - v[in][0]), v[in][1] + t * (v[out][1] - v[in][1]),
                    v[in][2] + t * (v[out][2] - v[in][2])};
      const int k = (int)nvtx.size();
      nvtx.push_back(x);
      epts[{i, o}] = k;
      w.created += 1;
      return k;
    };

    std::vector<std::vector<int>> nf;
    std::vector<int64_t> nfid;
    std::map<int, int> cap_next;  // entry point -> exit point, walking the cap
    for (size_t k = 0; k < f.size(); ++k) {
      const std::vector<int>& cyc = f[k];
      const int m = (int)cyc.size();
      std::vector<int> poly;
      int exit_pt = -1, entry_pt = -1;
      for (int i = 0; i < m; ++i) {
        const int a = cyc[i], b = cyc[(i + 1) % m];
        const bool ao = s[a] > 0.0, bo = s[b] > 0.0;
        if (!ao) poly.push_back(remap[a]);
        if (ao != bo) {
          const int x = edge_point(a, b);
          poly.push_back(x);
          if (!ao) exit_pt = x; else entry_pt = x;
        }
      }
      if (exit_pt >= 0 && entry_pt >= 0) cap_next[entry_pt] = exit_pt;
      if (poly.size() >= 3) {
        nf.push_back(std::move(poly));
        nfid.push_back(fid[k]);
      }
    }
    if (!cap_next.empty()) {
      std::vector<int> cap;
      const int start = cap_next.begin()->first;
      int x = start;
      do {
        cap.push_back(x);
        x = cap_next.at(x);
      } while (x != start && cap.size() <= cap_next.size());
      if (cap.size() >= 3) {
        nf.push_back(std::move(cap));
        nfid.push_back(id);
      }
    }
    v.swap(nvtx);
    f.swap(nf);
    fid.swap(nfid);
    return true;
  }

  double volume() const {  // origin (the seed) is inside: every term >= 0
    double vol = 0.0;
    for (const auto& cyc : f)
      for (size_t i = 1; i + 1 < cyc.size(); ++i)
        vol += dot3(v[cyc[0]], cross3(v[cyc[i]], v[cyc[i + 1]]));
    return vol / 6.0;
  }

  // First moment about the seed.  The same fan tetrahedra as volume(): the
  // centroid of a tetrahedron is the mean of its four corners, and one
  // corner is the seed (the origin here).
  V3 moment() const {
    V3 m = {0, 0, 0};
    for (const auto& cyc : f)
      for (size_t i = 1; i + 1 < cyc.size(); ++i) {
        const V3& a = v[cyc[0]];
        const V3& b = v[cyc[i]];
        const V3& c = v[cyc[i + 1]];
        const double w = dot3(a, cross3(b, c)) / 24.0;  // volume / 4
        for (int k = 0; k < 3; ++k) m[k] += w * (a[k] + b[k] + c[k]);
      }
    return m;
  }

  double face_area(size_t k) const {
    const auto& cyc = f[k];
    V3 a = {0, 0, 0};
    for (size_t i = 1; i + 1 < cyc.size(); ++i) {
      const V3 t = cross3(sub3(v[cyc[i]], v[cyc[0]]), sub3(v[cyc[i + 1]], v[cyc[0]]));
      a = {a[0] + t[0], a[1] + t[1], a[2] + t[2]};
    }
    return 0.5 * std::sqrt(dot3(a, a));
  }
};

// ---------------------------------------------------------------------------
// Volume of a finished cell in long double (64-bit mantissa on x86) from its
// combinatorics alone: every vertex is re-solved from three of the planes it
// lies on (Cramer's rule, seed-relative, exact plane data: n = q - p is exact
// for double inputs), and the faces' vertex cycles are fanned from their
// first vertex.  The primal clip interpolates new vertices between vertices
// at the box's scale, so on cells far smaller than the box its double
// vertices carry errors of order u times the box size; this volume has no
// such error and is the reference the FP64 volume bar uses.
using LD = long double;
struct V3L {
  LD x, y, z;
};
inline V3L crossL(const V3L& a, const V3L& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline LD dotL(const V3L& a, const V3L& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// plane id >= 0: bisector with point id; -1..-6: walls x-, x+, y-, y+, z-, z+
inline void planeL(int64_t id, const double* P, int64_t i, const double* lo, const double* hi, V3L& n, LD& c) {
  if (id >= 0) {
    n = {(LD)P[3 * id] - (LD)P[3 * i], (LD)P[3 * id + 1] - (LD)P[3 * i + 1], (LD)P[3 * id + 2] - (LD)P[3 * i + 2]};
    c = dotL(n, n) / 2;
  } else {
    const int w = (int)(-id - 1), ax = w >> 1;
    const bool up = w & 1;
    n = {0, 0, 0};
    (ax == 0 ? n.x : ax == 1 ? n.y : n.z) = up ? 1 : -1;
    c = up ? (LD)hi[ax] - (LD)P[3 * i + ax] : (LD)P[3 * i + ax] - (LD)lo[ax];
  }
}

template <typename PlaneFn>
double volume_ld_with(const Poly& C, PlaneFn plane) {
  const size_t nv = C.v.size();
  std::vector<std::vector<int64_t>> inc(nv);
  for (size_t k = 0; k < C.f.size(); ++k)
    for (int x : C.f[k]) inc[x].push_back(C.fid[k]);
  std::vector<V3L> w(nv);
  for (size_t x = 0; x < nv; ++x) {
    auto& s = inc[x];
    std::sort(s.begin(), s.end());
    s.erase(std::unique(s.begin(), s.end()), s.end());
    w[x] = {(LD)C.v[x][0], (LD)C.v[x][1], (LD)C.v[x][2]};
    if (s.size() < 3) continue;
    V3L na, nb, nc;
    LD ca, cb, cc;
    plane(s[0], na, ca);
    plane(s[1], nb, cb);
    plane(s[2], nc, cc);
    const V3L bc = crossL(nb, nc), ca_ = crossL(nc, na), ab = crossL(na, nb);
    const LD det = dotL(na, bc);
    if (det == 0) continue;
    w[x] = {(ca * bc.x + cb * ca_.x + cc * ab.x) / det, (ca * bc.y + cb * ca_.y + cc * ab.y) / det,
            (ca * bc.z + cb * ca_.z + cc * ab.z) / det};
  }
  LD vol = 0;
  for (const auto& cyc : C.f)
    for (size_t k = 1; k + 1 < cyc.size(); ++k) vol += dotL(w[cyc[0]], crossL(w[cyc[k]], w[cyc[k + 1]]));
  return (double)(vol / 6);
}

double volume_ld(const Poly& C, const double* P, int64_t i, const double* lo, const double* hi) {
  return volume_ld_with(C, [&](int64_t id, V3L& n, LD& c) { planeL(id, P, i, lo, hi, n, c); });
}

// ---------------------------------------------------------------------------
// The oracle's own uniform grid (about four points per grid cell).
struct Grid {
  int g[3];
  double lo[3], hi[3], h[3];
  std::vector<int64_t> start;  // [G+1]
  std::vector<int64_t> idx;    // point indices bucketed by grid cell

  void build(const double* P, int64_t n, const double* blo, const double* bhi) {
    double vol = 1.0;
    for (int a = 0; a < 3; ++a) vol *= (bhi[a] - blo[a]);
    const double scale = std::cbrt((double)std::max<int64_t>(n, 1) / (4.0 * vol));
    for (int a = 0; a < 3; ++a) {
      lo[a] = blo[a];
      hi[a] = bhi[a];
      g[a] = std::max(1, (int)std::lround((bhi[a] - blo[a]) * scale));
      h[a] = (bhi[a] - blo[a]) / g[a];
    }
    const int64_t G = (int64_t)g[0] * g[1] * g[2];
    std::vector<std::pair<int64_t, int64_t>> key(n);
    for (int64_t i = 0; i < n; ++i) key[i] = {cell_of(&P[3 * i]), i};
    std::sort(key.begin(), key.end());
    start.assign(G + 1, 0);
    idx.resize(n);
    for (int64_t i = 0; i < n; ++i) {
      idx[i] = key[i].second;
      start[key[i].first + 1] += 1;
    }
    for (int64_t c = 0; c < G; ++c) start[c + 1] += start[c];
  }
  int coord(double x, int a) const {
    int c = (int)std::floor((x - lo[a]) / h[a]);
    return std::min(std::max(c, 0), g[a] - 1);
  }
  int64_t cell_of(const double* p) const {
    return coord(p[0], 0) + (int64_t)g[0] * (coord(p[1], 1) + (int64_t)g[1] * coord(p[2], 2));
  }
};

// Streams the other points of seed i ring by ring.  `ring(r, out)` appends the
// indices in Chebyshev ring r; `rho(r)` bounds from below the distance from the
// seed to any point outside the block of rings 0..r (infinite if the block
// covers the grid); `covers(r)` tells whether the block is the whole grid.
struct Rings {
  const Grid& G;
  const double* P;
  int c[3];
  V3 p;
  double margin;
  Rings(const Grid& G_, const double* P_, int64_t i) : G(G_), P(P_) {
    p = {P[3 * i], P[3 * i + 1], P[3 * i + 2]};
    for (int a = 0; a < 3; ++a) c[a] = G.coord(p[a], a);
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) ext = std::max(ext, G.hi[a] - G.lo[a]);
    margin = 1e-9 * ext;  // covers floor() rounding at grid-cell borders
  }
  void ring(int r, std::vector<int64_t>& out) const {
    for (int z = c[2] - r; z <= c[2] + r; ++z) {
      if (z < 0 || z >= G.g[2]) continue;
      for (int y = c[1] - r; y <= c[1] + r; ++y) {
        if (y < 0 || y >= G.g[1]) continue;
        for (int x = c[0] - r; x <= c[0] + r; ++x) {
          if (x < 0 || x >= G.g[0]) continue;
          const int d = std::max({std::abs(x - c[0]), std::abs(y - c[1]), std::abs(z - c[2])});
          if (d != r) continue;
          const int64_t cell = x + (int64_t)G.g[0] * (y + (int64_t)G.g[1] * z);
          for (int64_t t = G.start[cell]; t < G.start[cell + 1]; ++t) out.push_back(G.idx[t]);
        }
      }
    }
  }
  bool covers(int r) const {
    for (int a = 0; a < 3; ++a)
      if (c[a] - r > 0 || c[a] + r + 1 < G.g[a]) return false;
    return true;
  }
  double rho(int r) const {
    double best = std::numeric_limits<double>::infinity();
    for (int a = 0; a < 3; ++a) {
      if (c[a] - r > 0) best = std::min(best, p[a] - (G.lo[a] + (c[a] - r) * G.h[a]));
      if (c[a] + r + 1 < G.g[a]) best = std::min(best, (G.lo[a] + (c[a] + r + 1) * G.h[a]) - p[a]);
    }
    return best - margin;
  }
  double d2(int64_t j) const {
    const V3 q = {P[3 * j], P[3 * j + 1], P[3 * j + 2]};
    const V3 n = sub3(q, p);
    return dot3(n, n);
  }
  V3 normal(int64_t j) const { return sub3({P[3 * j], P[3 * j + 1], P[3 * j + 2]}, p); }
};

int validate(const double* P, int64_t n, const double* lo, const double* hi) {
  for (int a = 0; a < 3; ++a)
    if (!(lo[a] < hi[a])) return 1;
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      const double x = P[3 * i + a];
      if (!(x >= lo[a] && x <= hi[a])) return 2;
    }
  std::vector<int64_t> o(n);
  for (int64_t i = 0; i < n; ++i) o[i] = i;
  std::sort(o.begin(), o.end(), [&](int64_t a, int64_t b) {
    return std::lexicographical_compare(P + 3 * a, P + 3 * a + 3, P + 3 * b, P + 3 * b + 3);
  });
  for (int64_t i = 1; i < n; ++i)
    if (std::equal(P + 3 * o[i], P + 3 * o[i] + 3, P + 3 * o[i - 1])) return 3;
  return 0;
}

// One exact cell: clip by rings until the certificate closes (or, with
// `all`, by every other point in index order -- no early stop at all).
void exact_cell(const Grid& G, const double* P, int64_t n, const double* lo, const double* hi, int64_t i,
                bool all, Poly& C, Work& w) {
  Rings R(G, P, i);
  C.box(lo, hi, R.p);
  if (all) {
    for (int64_t j = 0; j < n; ++j)
      if (j != i) C.clip(R.normal(j), 0.5 * R.d2(j), j, w);
    return;
  }
  std::vector<int64_t> cand;
  std::vector<std::pair<double, int64_t>> ord;
  for (int r = 0;; ++r) {
    cand.clear();
    R.ring(r, cand);
    ord.clear();
    for (int64_t j : cand)
      if (j != i) ord.push_back({R.d2(j), j});
    std::sort(ord.begin(), ord.end());
    double r2 = C.radius2();
    for (const auto& e : ord) {
      if (e.first > 4.0 * r2) break;  // cannot cut; later ones are farther
      if (C.clip(R.normal(e.second), 0.5 * e.first, e.second, w)) r2 = C.radius2();
    }
    if (R.covers(r)) break;
    const double rho = R.rho(r);
    if (rho > 0.0 && rho * rho > 4.0 * r2) break;
  }
}

// The method's view of one cell: the other points in exact (d^2, index) order,
// produced lazily from the rings (a point is released once no unscanned point
// can precede it).
struct SortedStream {
  Rings R;
  int64_t self;
  int r = -1;
  bool done = false;
  std::vector<std::pair<double, int64_t>> buf;
  size_t next = 0, safe = 0;
  SortedStream(const Grid& G, const double* P, int64_t i) : R(G, P, i), self(i) {}
  bool pop(std::pair<double, int64_t>& out) {
    while (next >= safe) {
      if (done) {
        if (next >= buf.size()) return false;
        safe = buf.size();
        break;
      }
      ++r;
      std::vector<int64_t> cand;
      R.ring(r, cand);
      for (int64_t j : cand)
        if (j != self) buf.push_back({R.d2(j), j});
      std::sort(buf.begin() + next, buf.end());
      if (R.covers(r)) {
        done = true;
        safe = buf.size();
      } else {
        const double rho = R.rho(r);
        safe = next;
        if (rho > 0.0)
          while (safe < buf.size() && buf[safe].first < rho * rho) ++safe;
      }
    }
    out = buf[next++];
    return true;
  }
};

// ---------------------------------------------------------------------------
// Periodic boxes (the box is a 3-torus of periods L = hi - lo): the cell of
// p_i is the set of points of R^3 nearer to p_i than to every image
// p_j + m L (m in Z^3, (j, m) != (i, 0)).  It lies in the cube p_i +- L/2,
// whose faces are exactly the bisectors with p_i's own six nearest images,
// so that cube is the starting polytope; the other images are enumerated by
// Chebyshev rings of the grid unrolled over R^3 (cell u maps to grid cell
// u mod g with image shift floor(u / g)).  A plane is named by its point
// and image shift: id = j * 32^3 + (mx + 15) + 32 (my + 15) + 32^2 (mz + 15),
// shifts -15..16 per axis (the cell lies within |L| / 2 of p_i; a ring
// enumeration over an elongated box with few grid cells may still need
// several periods along its short axes).
constexpr int64_t kShiftCodes = 32768;
inline int64_t image_id(int64_t j, int mx, int my, int mz) {
  return j * kShiftCodes + (mx + 15) + 32 * (my + 15) + 1024 * (mz + 15);
}
inline void image_of(int64_t id, int64_t& j, int m[3]) {
  j = id / kShiftCodes;
  int64_t c = id % kShiftCodes;
  m[0] = (int)(c % 32) - 15;
  m[1] = (int)((c / 32) % 32) - 15;
  m[2] = (int)(c / 1024) - 15;
}
inline int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// returns false if an image shift falls outside -15..16
bool exact_cell_periodic(const Grid& G, const double* P, const double* lo, const double* hi, int64_t i, Poly& C,
                         Work& w) {
  const V3 p = {P[3 * i], P[3 * i + 1], P[3 * i + 2]};
  double L[3], clo[3], chi[3];
  int c[3];
  double ext = 0.0;
  for (int a = 0; a < 3; ++a) {
    L[a] = hi[a] - lo[a];
    clo[a] = p[a] - 0.5 * L[a];
    chi[a] = p[a] + 0.5 * L[a];
    c[a] = G.coord(p[a], a);
    ext = std::max(ext, L[a]);
  }
  // the cube p +- L/2 built directly in seed-relative coordinates, so that
  // its corners are exactly +-L/2 (the bisectors of farther images of p_i
  // pass exactly through its edges and corners and must not cut them)
  C.box(clo, chi, p);
  for (int k = 0; k < 8; ++k)
    C.v[k] = {(k & 1) ? 0.5 * L[0] : -0.5 * L[0], (k & 2) ? 0.5 * L[1] : -0.5 * L[1], (k & 4) ? 0.5 * L[2] : -0.5 * L[2]};
  C.fid = {image_id(i, -1, 0, 0), image_id(i, 1, 0, 0), image_id(i, 0, -1, 0),
           image_id(i, 0, 1, 0), image_id(i, 0, 0, -1), image_id(i, 0, 0, 1)};
  const double margin = 1e-9 * ext;
  std::vector<std::tuple<double, int64_t, V3>> ord;
  for (int r = 0;; ++r) {
    ord.clear();
    for (int dz = -r; dz <= r; ++dz)
      for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
          if (std::max({std::abs(dx), std::abs(dy), std::abs(dz)}) != r) continue;
          const int64_t u[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
          int m[3];
          int64_t wc[3];
          for (int a = 0; a < 3; ++a) {
            m[a] = (int)floor_div(u[a], G.g[a]);
            wc[a] = u[a] - (int64_t)m[a] * G.g[a];
            if (m[a] < -15 || m[a] > 16) return false;
          }
          const int64_t cell = wc[0] + (int64_t)G.g[0] * (wc[1] + (int64_t)G.g[1] * wc[2]);
          for (int64_t t = G.start[cell]; t < G.start[cell + 1]; ++t) {
            const int64_t j = G.idx[t];
            if (j == i && m[0] == 0 && m[1] == 0 && m[2] == 0) continue;
            // (p_j - p_i) + m L: exact m L for p_i's own images
            const V3 nrm = {(P[3 * j] - p[0]) + m[0] * L[0], (P[3 * j + 1] - p[1]) + m[1] * L[1],
                            (P[3 * j + 2] - p[2]) + m[2] * L[2]};
            ord.push_back({dot3(nrm, nrm), image_id(j, m[0], m[1], m[2]), nrm});
          }
        }
    std::sort(ord.begin(), ord.end(), [](const auto& a, const auto& b) {
      return std::get<0>(a) < std::get<0>(b) || (std::get<0>(a) == std::get<0>(b) && std::get<1>(a) < std::get<1>(b));
    });
    double r2 = C.radius2();
    for (const auto& e : ord) {
      if (std::get<0>(e) > 4.0 * r2) break;  // cannot cut; later ones are farther
      if (C.clip(std::get<2>(e), 0.5 * std::get<0>(e), std::get<1>(e), w)) r2 = C.radius2();
    }
    // distance from p to the nearest face of the unrolled block of rings 0..r
    double rho = std::numeric_limits<double>::infinity();
    for (int a = 0; a < 3; ++a) {
      const double h = L[a] / G.g[a];
      rho = std::min(rho, p[a] - (lo[a] + (c[a] - r) * h));
      rho = std::min(rho, (lo[a] + (c[a] + r + 1) * h) - p[a]);
    }
    rho -= margin;
    if (rho > 0.0 && rho * rho > 4.0 * r2) break;
  }
  return true;
}

double volume_ld_periodic(const Poly& C, const double* P, int64_t i, const double* lo, const double* hi) {
  return volume_ld_with(C, [&](int64_t id, V3L& n, LD& c) {
    int64_t j;
    int m[3];
    image_of(id, j, m);
    n = {(LD)P[3 * j] + (LD)m[0] * ((LD)hi[0] - (LD)lo[0]) - (LD)P[3 * i],
         (LD)P[3 * j + 1] + (LD)m[1] * ((LD)hi[1] - (LD)lo[1]) - (LD)P[3 * i + 1],
         (LD)P[3 * j + 2] + (LD)m[2] * ((LD)hi[2] - (LD)lo[2]) - (LD)P[3 * i + 2]};
    c = dotL(n, n) / 2;
  });
}

struct Result {
  int64_t n = 0;
  std::vector<int64_t> row_ptr;
  std::vector<int32_t> col;
  std::vector<double> area;  // face area per (row, col) entry
  std::vector<double> vol;
  std::vector<double> vol_ld;  // [n] volume_ld() (flag 4), else empty
  std::vector<double> cen;   // [n,3] cell centroids (absolute)
  std::vector<int64_t> vrow_ptr;
  std::vector<double> vxyz;
  std::vector<int32_t> vplanes;  // three smallest incident plane ids
  std::vector<int32_t> vdeg;     // number of incident faces (3 on generic input)
  std::vector<int64_t> work;     // per cell: tested, cuts, evals, created
  std::vector<int32_t> euler;    // per cell: V - E + F
};

}  // namespace

extern "C" {

typedef struct Result orc_result;

// Computes every cell, or only the cells listed in `cells` (others are left
// empty).  flags: 1 = clip by all other points (no certificate), 2 = keep
// vertices, 4 = also the long-double volume of each cell, 8 = periodic box
// (neighbours are the indices of the points whose images share a face, a
// point appearing once per image; vertices are not kept; points must lie in
// [lo, hi)).  Returns 0, or 1 bad box, 2 point outside box, 3 duplicate,
// 4 unsupported flag combination, 5 image shift out of range.
int orc_tessellate(const double* P, int64_t n, const double* lo, const double* hi, const int64_t* cells, int64_t nc,
                   int flags, int nthreads, orc_result** out) {
  *out = nullptr;
  const bool periodic = flags & 8;
  if (periodic && (flags & 3)) return 4;
  const int bad = validate(P, n, lo, hi);
  if (bad) return bad;
  if (periodic)
    for (int64_t i = 0; i < n; ++i)
      for (int a = 0; a < 3; ++a)
        if (!(P[3 * i + a] < hi[a])) return 2;
  int shift_error = 0;
  Grid G;
  G.build(P, n, lo, hi);
  const bool all = flags & 1, keepv = flags & 2, want_ld = flags & 4;
  std::vector<std::vector<int32_t>> nb(n);
  std::vector<std::vector<double>> ar(n);
  std::vector<std::vector<double>> vx(keepv ? n : 0);
  std::vector<std::vector<int32_t>> vp(keepv ? n : 0), vd(keepv ? n : 0);
  Result* res = new Result;
  res->n = n;
  res->vol.assign(n, 0.0);
  if (want_ld) res->vol_ld.assign(n, 0.0);
  res->cen.assign(3 * n, 0.0);
  res->work.assign(4 * n, 0);
  res->euler.assign(n, 0);
  if (nthreads > 0) omp_set_num_threads(nthreads);
  if (!cells) nc = n;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < nc; ++t) {
    const int64_t i = cells ? cells[t] : t;
    if (i < 0 || i >= n) continue;
    Poly C;
    Work w;
    if (periodic) {
      if (!exact_cell_periodic(G, P, lo, hi, i, C, w)) {
#pragma omp atomic write
        shift_error = 1;
        continue;
      }
    } else {
      exact_cell(G, P, n, lo, hi, i, all, C, w);
    }
    res->vol[i] = C.volume();
    if (want_ld) res->vol_ld[i] = periodic ? volume_ld_periodic(C, P, i, lo, hi) : volume_ld(C, P, i, lo, hi);
    const V3 mom = C.moment();
    for (int a = 0; a < 3; ++a) res->cen[3 * i + a] = P[3 * i + a] + (res->vol[i] > 0.0 ? mom[a] / res->vol[i] : 0.0);
    res->work[4 * i + 0] = w.tested;
    res->work[4 * i + 1] = w.cuts;
    res->work[4 * i + 2] = w.evals;
    res->work[4 * i + 3] = w.created;
    int64_t edges2 = 0;
    std::vector<std::pair<int32_t, double>> row;
    for (size_t k = 0; k < C.f.size(); ++k) {
      edges2 += (int64_t)C.f[k].size();
      if (C.fid[k] < 0) continue;
      const double a = C.face_area(k);
      if (a > 0.0) row.push_back({(int32_t)(periodic ? C.fid[k] / kShiftCodes : C.fid[k]), a});
    }
    res->euler[i] = (int32_t)((int64_t)C.v.size() - edges2 / 2 + (int64_t)C.f.size());
    std::sort(row.begin(), row.end());
    for (auto& e : row) {
      nb[i].push_back(e.first);
      ar[i].push_back(e.second);
    }
    if (keepv) {
      std::vector<std::vector<int32_t>> inc(C.v.size());
      for (size_t k = 0; k < C.f.size(); ++k)
        for (int x : C.f[k]) inc[x].push_back((int32_t)C.fid[k]);
      for (size_t x = 0; x < C.v.size(); ++x) {
        auto& s = inc[x];
        std::sort(s.begin(), s.end());
        s.erase(std::unique(s.begin(), s.end()), s.end());
        for (int a = 0; a < 3; ++a) vx[i].push_back(C.v[x][a] + P[3 * i + a]);
        for (int a = 0; a < 3; ++a) vp[i].push_back(a < (int)s.size() ? s[a] : INT32_MIN);
        vd[i].push_back((int32_t)s.size());
      }
    }
  }
  if (shift_error) {
    delete res;
    return 5;
  }
  res->row_ptr.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) res->row_ptr[i + 1] = res->row_ptr[i] + (int64_t)nb[i].size();
  for (int64_t i = 0; i < n; ++i) {
    res->col.insert(res->col.end(), nb[i].begin(), nb[i].end());
    res->area.insert(res->area.end(), ar[i].begin(), ar[i].end());
  }
  if (keepv) {
    res->vrow_ptr.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) res->vrow_ptr[i + 1] = res->vrow_ptr[i] + (int64_t)vd[i].size();
    for (int64_t i = 0; i < n; ++i) {
      res->vxyz.insert(res->vxyz.end(), vx[i].begin(), vx[i].end());
      res->vplanes.insert(res->vplanes.end(), vp[i].begin(), vp[i].end());
      res->vdeg.insert(res->vdeg.end(), vd[i].begin(), vd[i].end());
    }
  }
  *out = res;
  return 0;
}

int64_t orc_nnz(const orc_result* r) { return (int64_t)r->col.size(); }
int64_t orc_nvert(const orc_result* r) { return (int64_t)r->vdeg.size(); }

// Any output pointer may be null.
void orc_fetch(const orc_result* r, int64_t* row_ptr, int32_t* col, double* area, double* vol, int64_t* work,
               int32_t* euler, int64_t* vrow_ptr, double* vxyz, int32_t* vplanes, int32_t* vdeg) {
  auto cp = [](void* dst, const void* src, size_t bytes) {
    if (dst && bytes) std::memcpy(dst, src, bytes);
  };
  cp(row_ptr, r->row_ptr.data(), r->row_ptr.size() * sizeof(int64_t));
  cp(col, r->col.data(), r->col.size() * sizeof(int32_t));
  cp(area, r->area.data(), r->area.size() * sizeof(double));
  cp(vol, r->vol.data(), r->vol.size() * sizeof(double));
  cp(work, r->work.data(), r->work.size() * sizeof(int64_t));
  cp(euler, r->euler.data(), r->euler.size() * sizeof(int32_t));
  cp(vrow_ptr, r->vrow_ptr.data(), r->vrow_ptr.size() * sizeof(int64_t));
  cp(vxyz, r->vxyz.data(), r->vxyz.size() * sizeof(double));
  cp(vplanes, r->vplanes.data(), r->vplanes.size() * sizeof(int32_t));
  cp(vdeg, r->vdeg.data(), r->vdeg.size() * sizeof(int32_t));
}

// Long-double volumes [n] (flag 4 only; zero for rows not computed).
void orc_fetch_vol_ld(const orc_result* r, double* v) {
  if (v && !r->vol_ld.empty()) std::memcpy(v, r->vol_ld.data(), r->vol_ld.size() * sizeof(double));
}

// Cell centroids [n,3] (zero for rows not computed).
void orc_fetch_centroid(const orc_result* r, double* cen) {
  if (cen && !r->cen.empty()) std::memcpy(cen, r->cen.data(), r->cen.size() * sizeof(double));
}

void orc_free(orc_result* r) { delete r; }

// The method with a list of the k nearest neighbours, for every seed in
// `cells` (or all seeds when cells == null).  The k nearest are taken in exact
// (d^2, index) order; the box is clipped by q_1, q_2, ... and the cell is
// certified at list size k iff d_m^2 > 4 R_m^2 for some m <= k, where R_m is the
// vertex radius after clipping by q_1..q_m, or iff the list holds all n-1 other
// points.  Outputs per cell:
//   kneeded[c]  least list size that certifies (capped: kcap+1 means "more"),
//   tested/evals/created/r2upd[c]  work of the method at list size `kwork`
//                (planes tested before the early stop, vertex evaluations,
//                vertices created, vertex norms evaluated to update R^2 after
//                each cut); pass kwork <= 0 to skip.
// Returns 0 or a validation code as orc_tessellate.
int orc_kneeded(const double* P, int64_t n, const double* lo, const double* hi, const int64_t* cells, int64_t nc,
                int64_t kcap, int64_t kwork, int nthreads, int32_t* kneeded, int64_t* tested, int64_t* evals,
                int64_t* created, int64_t* r2upd) {
  const int bad = validate(P, n, lo, hi);
  if (bad) return bad;
  Grid G;
  G.build(P, n, lo, hi);
  if (!cells) nc = n;
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < nc; ++t) {
    const int64_t i = cells ? cells[t] : t;
    SortedStream S(G, P, i);
    Poly C;
    C.box(lo, hi, S.R.p);
    Work w, wk;
    double r2 = C.radius2();
    int64_t kn = -1;
    int64_t m = 0;
    bool fprev = false;   // F_{m-1}: d_{m-1}^2 > 4 R_{m-1}^2
    bool early = false;   // the early check E_m has fired
    const int64_t limit = std::max<int64_t>(kcap, kwork);
    std::pair<double, int64_t> e;
    while (m < limit && S.pop(e)) {
      ++m;
      if (e.first > 4.0 * r2) {  // E_m: q_m (and all later points) cannot cut
        if (kn < 0) kn = fprev ? m - 1 : m;
        early = true;
        break;
      }
      const bool in_k = (kwork > 0 && m <= kwork);
      Work& ww = in_k ? wk : w;
      if (C.clip(S.R.normal(e.second), 0.5 * e.first, e.second, ww)) {
        r2 = C.radius2();
        ww.r2 += (int64_t)C.v.size();
      }
      fprev = e.first > 4.0 * r2;  // F_m
      if (fprev && kn < 0) kn = m;
    }
    if (kn < 0 && !early && m == n - 1) kn = n - 1;  // the list holds every other point
    if (kn < 0 || kn > kcap) kn = kcap + 1;
    kneeded[t] = (int32_t)kn;
    if (tested) tested[t] = wk.tested;
    if (evals) evals[t] = wk.evals;
    if (created) created[t] = wk.created;
    if (r2upd) r2upd[t] = wk.r2;
  }
  return 0;
}

}  // extern "C"
