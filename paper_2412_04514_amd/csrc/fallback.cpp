// Host fallback for cells the GPU passes could not certify (paper, Summary
// section: cells that fail validation are recomputed on the CPU).  Each cell is clipped with no bound on the neighbour count:
// grid rings around the seed are consumed in order, each ring's points nearest
// first, until the scanned block provably contains every point within 2R of
// the seed (R = farthest vertex).  The polyhedron uses the same dual form as
// the GPU kernel (planes + counter-clockwise plane triangles), in double.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <thread>
#include <unordered_set>

#include "internal.h"

namespace votess {
namespace {

struct Pl {
  double x, y, z, c;
  int id;
};

struct DualCell {
  std::vector<Pl> pl;
  std::vector<std::array<int, 3>> tri;
  std::vector<std::array<double, 3>> pos;

  static std::array<double, 3> solve(const Pl& a, const Pl& b, const Pl& m) {
    auto cr = [](double ax, double ay, double az, double bx, double by, double bz) {
      return std::array<double, 3>{ay * bz - az * by, az * bx - ax * bz, ax * by - ay * bx};
    };
    const auto bc = cr(b.x, b.y, b.z, m.x, m.y, m.z);
    const auto ca = cr(m.x, m.y, m.z, a.x, a.y, a.z);
    const auto ab = cr(a.x, a.y, a.z, b.x, b.y, b.z);
    const double det = a.x * bc[0] + a.y * bc[1] + a.z * bc[2];
    std::array<double, 3> v;
    for (int i = 0; i < 3; ++i) v[i] = (a.c * bc[i] + b.c * ca[i] + m.c * ab[i]) / det;
    return v;
  }

  // solve() refined once against the residual c - n.v accumulated as if in
  // twice the working precision (FMA-split products, error-free sums): a
  // vertex of nearly parallel planes is then good to a few ulps.
  static std::array<double, 3> solve_refined(const Pl& a, const Pl& b, const Pl& m) {
#pragma clang fp contract(off)
    const std::array<double, 3> v = solve(a, b, m);
    auto resid = [&](const Pl& q) {
      const double n[3] = {q.x, q.y, q.z};
      double s = q.c, err = 0.0;
      for (int i = 0; i < 3; ++i) {
        const double p = n[i] * v[i];
        const double ep = std::fma(n[i], v[i], -p);
        const double t = s - p;
        const double z = t - s;
        const double es = (s - (t - z)) + (-p - z);
        s = t;
        err += es - ep;
      }
      return s + err;
    };
    const std::array<double, 3> d = solve(Pl{a.x, a.y, a.z, resid(a), a.id}, Pl{b.x, b.y, b.z, resid(b), b.id},
                                          Pl{m.x, m.y, m.z, resid(m), m.id});
    return {v[0] + d[0], v[1] + d[1], v[2] + d[2]};
  }

  void box(const double lo[3], const double hi[3], const double p[3]) {
    pl.clear();
    tri.clear();
    pos.clear();
    for (int f = 0; f < 6; ++f) {
      const int ax = f >> 1;
      const bool hs = f & 1;
      Pl q{0, 0, 0, 0, -(f + 1)};
      (&q.x)[ax] = hs ? 1.0 : -1.0;
      q.c = hs ? hi[ax] - p[ax] : p[ax] - lo[ax];
      pl.push_back(q);
    }
    for (int v = 0; v < 8; ++v) {
      const int bx = v & 1, by = (v >> 1) & 1, bz = (v >> 2) & 1;
      pos.push_back({(bx ? hi[0] : lo[0]) - p[0], (by ? hi[1] : lo[1]) - p[1], (bz ? hi[2] : lo[2]) - p[2]});
      const int X = bx, Y = 2 + by, Z = 4 + bz;
      if ((bx + by + bz) & 1) tri.push_back({X, Y, Z});
      else tri.push_back({X, Z, Y});
    }
  }

  double radius2() const {
    double r = 0.0;
    for (const auto& v : pos) r = std::max(r, v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    return r;
  }

  // Returns false if the topology came out inconsistent.
  bool clip(const Pl& m, bool& cut) {
    cut = false;
    std::vector<char> out(tri.size());
    bool any = false;
    for (size_t t = 0; t < tri.size(); ++t) {
      const auto& v = pos[t];
      out[t] = (m.x * v[0] + m.y * v[1] + m.z * v[2] - m.c) > 0.0;
      any = any || out[t];
    }
    if (!any) return true;
    cut = true;
    const int mi = (int)pl.size();
    pl.push_back(m);
    auto key = [](int a, int b) { return ((long long)a << 32) | (unsigned)b; };
    std::unordered_set<long long> rem;
    for (size_t t = 0; t < tri.size(); ++t)
      if (out[t])
        for (int e = 0; e < 3; ++e) rem.insert(key(tri[t][e], tri[t][(e + 1) % 3]));
    std::vector<std::array<int, 3>> ntri;
    std::vector<std::array<double, 3>> npos;
    std::vector<std::array<int, 3>> added;
    for (size_t t = 0; t < tri.size(); ++t) {
      if (!out[t]) {
        ntri.push_back(tri[t]);
        npos.push_back(pos[t]);
        continue;
      }
      for (int e = 0; e < 3; ++e) {
        const int a = tri[t][e], b = tri[t][(e + 1) % 3];
        if (!rem.count(key(b, a))) added.push_back({a, b, mi});
      }
    }
    if (added.size() < 3) return false;
    for (const auto& t : added) {
      ntri.push_back(t);
      npos.push_back(solve(pl[t[0]], pl[t[1]], pl[t[2]]));
    }
    tri.swap(ntri);
    pos.swap(npos);
    return true;
  }

  double volume() const {
    auto dot = [](const std::array<double, 3>& a, const std::array<double, 3>& b) {
      return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    };
    auto crs = [](const std::array<double, 3>& a, const std::array<double, 3>& b) {
      return std::array<double, 3>{a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    };
    auto nrm = [&](int f) { return std::array<double, 3>{pl[f].x, pl[f].y, pl[f].z}; };
    auto anchor = [&](int f, int g) {  // nearest point of line f^g: see faces()
      const auto nf = nrm(f), ng = nrm(g);
      const auto d = crs(nf, ng), gd = crs(ng, d), fd = crs(nf, d);
      const double inv = 1.0 / dot(d, d);
      std::array<double, 3> e;
      for (int k = 0; k < 3; ++k) e[k] = (pl[f].c * gd[k] - pl[g].c * fd[k]) * inv;
      return e;
    };
    auto foot = [&](int f) {
      const auto n = nrm(f);
      const double s = pl[f].c / dot(n, n);
      return std::array<double, 3>{s * n[0], s * n[1], s * n[2]};
    };
    double vol = 0.0;
    for (size_t t = 0; t < tri.size(); ++t) {
      const int a = tri[t][0], b = tri[t][1], c = tri[t][2];
      const auto& v = pos[t];
      const auto eab = anchor(a, b), ebc = anchor(b, c), eca = anchor(c, a);
      auto diff = [](const std::array<double, 3>& x, const std::array<double, 3>& y) {
        return std::array<double, 3>{x[0] - y[0], x[1] - y[1], x[2] - y[2]};
      };
      vol += dot(foot(a), crs(v, diff(eca, eab)));
      vol += dot(foot(b), crs(v, diff(eab, ebc)));
      vol += dot(foot(c), crs(v, diff(ebc, eca)));
    }
    return vol / 6.0;
  }

  // Per-plane face areas and the first moment about the seed, from the same
  // corner terms as volume() with refined vertices: the corner of vertex v on
  // face f between edges
  // f^g and f^h spans n_f . (v x (e_fh - e_fg)) / (2 |n_f|), and splits into
  // the signed tetrahedra (0, F_f, v, e_fh) and (0, F_f, e_fg, v).
  void faces(std::vector<double>& area, double mom[3], double& vol6) const {
    using A3 = std::array<double, 3>;
    auto dot = [](const A3& a, const A3& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
    auto crs = [](const A3& a, const A3& b) {
      return A3{a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    };
    auto diff = [](const A3& x, const A3& y) { return A3{x[0] - y[0], x[1] - y[1], x[2] - y[2]}; };
    auto nrm = [&](int f) { return A3{pl[f].x, pl[f].y, pl[f].z}; };
    // nearest point of line f^g to the seed, (c_f (n_g x d) - c_g (n_f x d)) /
    // |d|^2 with d = n_f x n_g: error ~ 1/sin(angle), not its square as
    // through the 2x2 Gram system
    auto anchor = [&](int f, int g) {
      const A3 nf = nrm(f), ng = nrm(g);
      const A3 d = crs(nf, ng), gd = crs(ng, d), fd = crs(nf, d);
      const double inv = 1.0 / dot(d, d);
      return A3{(pl[f].c * gd[0] - pl[g].c * fd[0]) * inv, (pl[f].c * gd[1] - pl[g].c * fd[1]) * inv,
                (pl[f].c * gd[2] - pl[g].c * fd[2]) * inv};
    };
    auto foot = [&](int f) {
      const A3 n = nrm(f);
      const double s = pl[f].c / dot(n, n);
      return A3{s * n[0], s * n[1], s * n[2]};
    };
    area.assign(pl.size(), 0.0);
    mom[0] = mom[1] = mom[2] = 0.0;
    vol6 = 0.0;
    auto tet = [&](const A3& x, const A3& y, const A3& z) {
      const double w = dot(x, crs(y, z));
      vol6 += w;
      for (int k = 0; k < 3; ++k) mom[k] += w * (x[k] + y[k] + z[k]);
    };
    for (size_t t = 0; t < tri.size(); ++t) {
      const int a = tri[t][0], b = tri[t][1], c = tri[t][2];
      const A3 v = solve_refined(pl[a], pl[b], pl[c]);
      const A3 eab = anchor(a, b), ebc = anchor(b, c), eca = anchor(c, a);
      const A3 na = nrm(a), nb = nrm(b), nc = nrm(c);
      area[a] += dot(na, crs(v, diff(eca, eab))) / (2.0 * std::sqrt(dot(na, na)));
      area[b] += dot(nb, crs(v, diff(eab, ebc))) / (2.0 * std::sqrt(dot(nb, nb)));
      area[c] += dot(nc, crs(v, diff(ebc, eca))) / (2.0 * std::sqrt(dot(nc, nc)));
      const A3 Fa = foot(a), Fb = foot(b), Fc = foot(c);
      tet(Fa, v, eca);
      tet(Fa, eab, v);
      tet(Fb, v, eab);
      tet(Fb, ebc, v);
      tet(Fc, v, ebc);
      tet(Fc, eca, v);
    }
    for (int k = 0; k < 3; ++k) mom[k] /= 24.0;
  }
};

struct HostGrid {
  const votess_grid& g;
  const int32_t* start;
  int coord(double x, int a) const {
    double c = std::floor((x - g.lo[a]) * g.inv_h[a]);
    c = std::fmin(std::fmax(c, 0.0), (double)(g.g[a] - 1));
    return (int)c;
  }
};

template <typename T>
void one_cell(const T* rec, int n, const HostGrid& G, int s, bool want_vertices, bool want_faces, HostCellOut& out) {
  const double p[3] = {(double)rec[4 * (size_t)s], (double)rec[4 * (size_t)s + 1], (double)rec[4 * (size_t)s + 2]};
  const votess_grid& g = G.g;
  int c[3];
  for (int a = 0; a < 3; ++a) c[a] = G.coord(p[a], a);
  double h[3], ext = 0.0;
  for (int a = 0; a < 3; ++a) {
    h[a] = (g.hi[a] - g.lo[a]) / g.g[a];
    ext = std::max(ext, g.hi[a] - g.lo[a]);
  }
  const double margin = 1e-9 * ext;
  DualCell C;
  C.box(g.lo, g.hi, p);
  double r2 = C.radius2();
  std::vector<std::pair<double, int>> ring;
  out.ok = true;
  for (int r = 0;; ++r) {
    ring.clear();
    for (int z = std::max(c[2] - r, 0); z <= std::min(c[2] + r, g.g[2] - 1); ++z)
      for (int y = std::max(c[1] - r, 0); y <= std::min(c[1] + r, g.g[1] - 1); ++y)
        for (int x = std::max(c[0] - r, 0); x <= std::min(c[0] + r, g.g[0] - 1); ++x) {
          if (std::max({std::abs(x - c[0]), std::abs(y - c[1]), std::abs(z - c[2])}) != r) continue;
          const int64_t cell = x + (int64_t)g.g[0] * (y + (int64_t)g.g[1] * z);
          for (int j = G.start[cell]; j < G.start[cell + 1]; ++j) {
            if (j == s) continue;
            const double dx = rec[4 * (size_t)j] - p[0], dy = rec[4 * (size_t)j + 1] - p[1],
                         dz = rec[4 * (size_t)j + 2] - p[2];
            ring.push_back({dx * dx + dy * dy + dz * dz, j});
          }
        }
    std::sort(ring.begin(), ring.end());
    for (const auto& e : ring) {
      if (e.first > 4.0 * r2) break;
      const int j = e.second;
      const double nx = rec[4 * (size_t)j] - p[0], ny = rec[4 * (size_t)j + 1] - p[1], nz = rec[4 * (size_t)j + 2] - p[2];
      bool cut;
      if (!C.clip(Pl{nx, ny, nz, 0.5 * e.first, j}, cut)) {
        out.ok = false;
        return;
      }
      if (cut) r2 = C.radius2();
    }
    bool covers = true;
    double rho = 1e300;
    for (int a = 0; a < 3; ++a) {
      if (c[a] - r > 0) {
        covers = false;
        rho = std::min(rho, p[a] - (g.lo[a] + (c[a] - r) * h[a]));
      }
      if (c[a] + r + 1 < g.g[a]) {
        covers = false;
        rho = std::min(rho, (g.lo[a] + (c[a] + r + 1) * h[a]) - p[a]);
      }
    }
    if (covers) break;
    rho -= margin;
    if (rho > 0.0 && rho * rho > 4.0 * r2) break;
  }
  out.volume = C.volume();
  out.r2 = r2;
  std::vector<char> used(C.pl.size(), 0);
  for (const auto& t : C.tri)
    for (int e = 0; e < 3; ++e) used[t[e]] = 1;
  out.nbr.clear();
  out.area.clear();
  std::vector<double> farea;
  if (want_faces) {
    double mom[3], vol6;
    C.faces(farea, mom, vol6);
    for (int a = 0; a < 3; ++a) out.centroid[a] = p[a] + (vol6 > 0.0 ? 6.0 * mom[a] / vol6 : 0.0);
  }
  for (size_t f = 0; f < C.pl.size(); ++f)
    if (used[f] && C.pl[f].id >= 0) {
      out.nbr.push_back(C.pl[f].id);
      if (want_faces) out.area.push_back(farea[f]);
    }
  if (want_vertices) {
    for (size_t t = 0; t < C.tri.size(); ++t) {
      for (int a = 0; a < 3; ++a) out.verts.push_back(C.pos[t][a] + p[a]);
      for (int a = 0; a < 3; ++a) out.vplanes.push_back(C.pl[C.tri[t][a]].id);
    }
  }
}

}  // namespace

void host_fallback_cells(const void* sorted_h, votess_dtype dt, int n, const votess_grid& grid,
                         const int32_t* cell_start_h, const int32_t* cells, int ncells, bool want_vertices,
                         bool want_faces, int threads, std::vector<HostCellOut>& out) {
  out.assign(ncells, HostCellOut());
  if (ncells == 0) return;
  HostGrid G{grid, cell_start_h};
  int nt = threads > 0 ? threads : (int)std::max(1u, std::thread::hardware_concurrency());
  nt = std::min(nt, ncells);
  std::atomic<int> next(0);
  auto work = [&]() {
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= ncells) break;
      if (dt == VOTESS_F32)
        one_cell<float>((const float*)sorted_h, n, G, cells[i], want_vertices, want_faces, out[i]);
      else
        one_cell<double>((const double*)sorted_h, n, G, cells[i], want_vertices, want_faces, out[i]);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(work);
  work();
  for (auto& t : pool) t.join();
}

}  // namespace votess
