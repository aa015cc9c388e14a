// Unstructured triangle meshes (host side, built once per mesh): edge
// numbering, the seed-point agglomeration of Sec. 3.1.2, the interface grid
// of every coarser partition (macro-edges as chains of finer faces) with the
// P^1 space on each macro-edge parameterized by arc length (the remark of
// Sec. 3 on irregular macro-edges), the index maps the GPU kernels of the
// h-transitions need, and the reference-triangle matrices of the HDG local
// problem (Sec. 2) on P^k.
#include <algorithm>
#include <cmath>
#include <map>
#include <set>
#include <stdexcept>

#include "hdg_internal.hpp"

namespace hdg {

namespace {

// row-major n x n inverse by Gauss-Jordan with partial pivoting (host)
std::vector<double> invert(std::vector<double> A, int n) {
  std::vector<double> B(n * n, 0.0);
  for (int i = 0; i < n; ++i) B[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[p * n + c])) p = r;
    if (A[p * n + c] == 0.0) throw std::runtime_error("singular reference matrix");
    if (p != c)
      for (int j = 0; j < n; ++j) {
        std::swap(A[p * n + j], A[c * n + j]);
        std::swap(B[p * n + j], B[c * n + j]);
      }
    const double d = 1.0 / A[c * n + c];
    for (int j = 0; j < n; ++j) {
      A[c * n + j] *= d;
      B[c * n + j] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        A[r * n + j] -= f * A[c * n + j];
        B[r * n + j] -= f * B[c * n + j];
      }
    }
  }
  return B;
}

double lagrange_at(const std::vector<double>& nodes, int i, double x) {
  double v = 1.0;
  for (size_t j = 0; j < nodes.size(); ++j)
    if ((int)j != i) v *= (x - nodes[j]) / (nodes[i] - nodes[j]);
  return v;
}

// nodal P^k basis of the reference triangle (0,0), (1,0), (0,1): equispaced
// lattice (i/k, j/k), j slowest; coefficients in the monomials x^a y^b
struct TriBasis {
  int k = 1, nv = 0;
  std::vector<int> ea, eb;
  std::vector<double> C;  // [nmono][nv]
  explicit TriBasis(int k_) : k(k_) {
    for (int t = 0; t <= k; ++t)
      for (int a = t; a >= 0; --a) {
        ea.push_back(a);
        eb.push_back(t - a);
      }
    nv = (int)ea.size();
    std::vector<double> V(nv * nv);
    int i = 0;
    for (int j = 0; j <= k; ++j)
      for (int ii = 0; ii <= k - j; ++ii, ++i) {
        const double x = (double)ii / k, y = (double)j / k;
        for (int m = 0; m < nv; ++m) V[i * nv + m] = std::pow(x, ea[m]) * std::pow(y, eb[m]);
      }
    C = invert(V, nv);
  }
  void eval(double x, double y, double* phi, double* dx, double* dy) const {
    for (int i = 0; i < nv; ++i) {
      phi[i] = 0.0;
      if (dx) dx[i] = dy[i] = 0.0;
    }
    for (int m = 0; m < nv; ++m) {
      const int a = ea[m], b = eb[m];
      const double v = std::pow(x, a) * std::pow(y, b);
      const double vx = a > 0 ? a * std::pow(x, a - 1) * std::pow(y, b) : 0.0;
      const double vy = b > 0 ? b * std::pow(x, a) * std::pow(y, b - 1) : 0.0;
      for (int i = 0; i < nv; ++i) {
        phi[i] += v * C[m * nv + i];
        if (dx) {
          dx[i] += vx * C[m * nv + i];
          dy[i] += vy * C[m * nv + i];
        }
      }
    }
  }
};

}  // namespace

void UHost::build_reference(int k_) {
  k = k_;
  ne = k + 1;
  TriBasis tb(k);
  nv = tb.nv;
  std::vector<double> g, gw, gll;
  gauss_points(k + 2, g, gw);
  gll_points(k, gll);
  const int q = k + 2;
  Mh.assign(nv * nv, 0.0);
  Dh.assign(2 * nv * nv, 0.0);
  std::vector<double> phi(nv), dx(nv), dy(nv);
  for (int j = 0; j < q; ++j)
    for (int i = 0; i < q; ++i) {
      // collapsed (Duffy) Gauss point: x = s (1 - r), y = r, weight w_s w_r (1 - r)
      const double x = g[i] * (1 - g[j]), y = g[j], w = gw[i] * gw[j] * (1 - g[j]);
      tb.eval(x, y, phi.data(), dx.data(), dy.data());
      for (int a = 0; a < nv; ++a)
        for (int b = 0; b < nv; ++b) {
          Mh[a * nv + b] += w * phi[a] * phi[b];
          Dh[a * nv + b] += w * dx[a] * phi[b];
          Dh[nv * nv + a * nv + b] += w * dy[a] * phi[b];
        }
    }
  Minvh = invert(Mh, nv);
  Kh.assign(4 * nv * nv, 0.0);
  for (int j = 0; j < q; ++j)
    for (int i = 0; i < q; ++i) {
      const double x = g[i] * (1 - g[j]), y = g[j], w = gw[i] * gw[j] * (1 - g[j]);
      tb.eval(x, y, phi.data(), dx.data(), dy.data());
      const double* d[2] = {dx.data(), dy.data()};
      for (int r = 0; r < 2; ++r)
        for (int rp = 0; rp < 2; ++rp)
          for (int a = 0; a < nv; ++a)
            for (int b = 0; b < nv; ++b) Kh[((r * 2 + rp) * nv + a) * nv + b] += w * d[r][a] * d[rp][b];
    }
  Gnode.assign(2 * nv * nv, 0.0);
  {
    int a = 0;
    for (int jj = 0; jj <= k; ++jj)
      for (int ii = 0; ii <= k - jj; ++ii, ++a) {
        tb.eval((double)ii / k, (double)jj / k, phi.data(), dx.data(), dy.data());
        for (int b = 0; b < nv; ++b) {
          Gnode[(0 * nv + a) * nv + b] = dx[b];
          Gnode[(1 * nv + a) * nv + b] = dy[b];
        }
      }
  }
  const double vx[3] = {0.0, 1.0, 0.0}, vy[3] = {0.0, 0.0, 1.0};
  Eh.assign(3 * nv * nv, 0.0);
  Fh.assign(3 * nv * ne, 0.0);
  Hh.assign(ne * ne, 0.0);
  Nh.assign(6 * nv * nv, 0.0);
  De.assign(6 * nv * ne, 0.0);
  for (int s = 0; s < 3; ++s) {
    const int s1 = (s + 1) % 3;
    for (int t = 0; t < q; ++t) {
      const double x = vx[s] + g[t] * (vx[s1] - vx[s]), y = vy[s] + g[t] * (vy[s1] - vy[s]);
      tb.eval(x, y, phi.data(), dx.data(), dy.data());
      const double* d[2] = {dx.data(), dy.data()};
      for (int a = 0; a < nv; ++a) {
        for (int b = 0; b < nv; ++b) Eh[(s * nv + a) * nv + b] += gw[t] * phi[a] * phi[b];
        for (int b = 0; b < ne; ++b) Fh[(s * nv + a) * ne + b] += gw[t] * phi[a] * lagrange_at(gll, b, g[t]);
        for (int r = 0; r < 2; ++r) {
          for (int b = 0; b < nv; ++b) Nh[((s * 2 + r) * nv + a) * nv + b] += gw[t] * d[r][a] * phi[b];
          for (int b = 0; b < ne; ++b)
            De[((s * 2 + r) * nv + a) * ne + b] += gw[t] * d[r][a] * lagrange_at(gll, b, g[t]);
        }
      }
      if (s == 0)
        for (int a = 0; a < ne; ++a)
          for (int b = 0; b < ne; ++b)
            Hh[a * ne + b] += gw[t] * lagrange_at(gll, a, g[t]) * lagrange_at(gll, b, g[t]);
    }
  }
  Jp.assign(ne * 2, 0.0);
  for (int a = 0; a < ne; ++a) {
    Jp[a * 2 + 0] = 1.0 - gll[a];
    Jp[a * 2 + 1] = gll[a];
  }
}

namespace {

// halve a set of triangles at the median of their centroids along the axis
// of larger centroid extent (x on ties): the floor(n/2) lowest (coordinate,
// id) first; both halves returned in increasing id
void split2(const std::vector<int>& ids, const std::vector<double>& cx, const std::vector<double>& cy,
            std::vector<int>& lo, std::vector<int>& hi) {
  lo.clear();
  hi.clear();
  if (ids.empty()) return;
  double mnx = cx[ids[0]], mxx = mnx, mny = cy[ids[0]], mxy = mny;
  for (int t : ids) {
    mnx = std::min(mnx, cx[t]);
    mxx = std::max(mxx, cx[t]);
    mny = std::min(mny, cy[t]);
    mxy = std::max(mxy, cy[t]);
  }
  const std::vector<double>& c = (mxx - mnx) >= (mxy - mny) ? cx : cy;
  std::vector<int> s(ids);
  std::sort(s.begin(), s.end(), [&](int a, int b) { return c[a] < c[b] || (c[a] == c[b] && a < b); });
  const size_t h = s.size() / 2;
  lo.assign(s.begin(), s.begin() + h);
  hi.assign(s.begin() + h, s.end());
  std::sort(lo.begin(), lo.end());
  std::sort(hi.begin(), hi.end());
}

}  // namespace

void UHost::build_mesh(long nvert_, const double* xy_, long ntri_, const int* tri_, const double* seeds, int nseeds,
                       int hlevels) {
  nvert = nvert_;
  ntri = ntri_;
  xy.assign(xy_, xy_ + 2 * nvert);
  tri.assign(tri_, tri_ + 3 * ntri);
  for (long t = 0; t < ntri; ++t) {
    for (int s = 0; s < 3; ++s)
      if (tri[3 * t + s] < 0 || tri[3 * t + s] >= nvert) throw std::invalid_argument("vertex index");
    const double* a = &xy[2 * tri[3 * t]];
    const double* b = &xy[2 * tri[3 * t + 1]];
    const double* c = &xy[2 * tri[3 * t + 2]];
    if ((b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]) <= 0.0)
      throw std::invalid_argument("triangles must be counter-clockwise and non-degenerate");
  }
  // ---- edges: interior ones by sorted vertex pair; the finest faces
  std::map<std::pair<int, int>, std::vector<std::pair<long, int>>> keys;
  for (long t = 0; t < ntri; ++t)
    for (int s = 0; s < 3; ++s) {
      const int u = tri[3 * t + s], v = tri[3 * t + (s + 1) % 3];
      keys[{std::min(u, v), std::max(u, v)}].push_back({t, s});
    }
  UHostLevel F;
  F.tri = true;
  F.ncell = ntri;
  F.sptr.resize(ntri + 1);
  for (long t = 0; t <= ntri; ++t) F.sptr[t] = 3 * t;
  F.sface.assign(3 * ntri, -1);
  nbedge = 0;
  tbnd.assign(3 * ntri, -1);
  for (auto& kv : keys) {
    if (kv.second.size() > 2) throw std::invalid_argument("an edge is shared by more than two triangles");
    if (kv.second.size() == 1) {
      tbnd[3 * kv.second[0].first + kv.second[0].second] = (int)nbedge++;
      continue;
    }
    std::sort(kv.second.begin(), kv.second.end());
    const int f = (int)F.nface++;
    for (int side = 0; side < 2; ++side) {
      const long t = kv.second[side].first;
      const int s = kv.second[side].second;
      F.sface[3 * t + s] = f;
      F.fcell.push_back((int)t);
      F.fslot.push_back(s);
    }
    F.fstart.push_back(kv.first.first);
    F.fend.push_back(kv.first.second);
    const double dx = xy[2 * kv.first.second] - xy[2 * kv.first.first];
    const double dy = xy[2 * kv.first.second + 1] - xy[2 * kv.first.first + 1];
    F.flen.push_back(std::hypot(dx, dy));
  }
  // ---- agglomeration: level 1 by nearest seed, then four-way splits
  std::vector<double> cx(ntri), cy(ntri);
  for (long t = 0; t < ntri; ++t) {
    const double* a = &xy[2 * tri[3 * t]];
    const double* b = &xy[2 * tri[3 * t + 1]];
    const double* c = &xy[2 * tri[3 * t + 2]];
    cx[t] = ((a[0] + b[0]) + c[0]) / 3.0;
    cy[t] = ((a[1] + b[1]) + c[1]) / 3.0;
  }
  std::vector<std::vector<int>> groups(nseeds);
  for (long t = 0; t < ntri; ++t) {
    int best = 0;
    double bd = 0.0;
    for (int s = 0; s < nseeds; ++s) {
      const double dx = cx[t] - seeds[2 * s], dy = cy[t] - seeds[2 * s + 1];
      const double d2 = dx * dx + dy * dy;
      if (s == 0 || d2 < bd) {
        bd = d2;
        best = s;
      }
    }
    groups[best].push_back((int)t);
  }
  groups.erase(std::remove_if(groups.begin(), groups.end(), [](const std::vector<int>& g) { return g.empty(); }),
               groups.end());
  std::vector<std::vector<int>> parts;  // parts[l][t]: macro of triangle t on agglomeration level l + 1
  for (int lev = 0; lev < hlevels; ++lev) {
    if (lev > 0) {
      std::vector<std::vector<int>> nxt;
      std::vector<int> h0, h1, q0, q1;
      for (auto& g : groups) {
        split2(g, cx, cy, h0, h1);
        for (auto* half : {&h0, &h1}) {
          if (half->empty()) continue;
          split2(*half, cx, cy, q0, q1);
          if (!q0.empty()) nxt.push_back(q0);
          if (!q1.empty()) nxt.push_back(q1);
        }
      }
      groups.swap(nxt);
    }
    std::vector<int> p(ntri, -1);
    for (size_t i = 0; i < groups.size(); ++i)
      for (int t : groups[i]) p[t] = (int)i;
    parts.push_back(p);
  }
  nmacro.clear();
  for (auto& g : parts) nmacro.push_back(*std::max_element(g.begin(), g.end()) + 1);
  // ---- levels: P^k triangles, P^1 triangles (k > 1), then T_hlevels .. T_1
  lev.clear();
  lev.push_back(F);
  lev.back().m = k + 1;
  if (k > 1) {
    lev.push_back(F);
    lev.back().m = 2;
  }
  std::vector<int> cell_of(ntri);
  for (long t = 0; t < ntri; ++t) cell_of[t] = (int)t;
  for (int l = hlevels - 1; l >= 0; --l) {
    UHostLevel& fine = lev.back();
    std::vector<int> coarse_of(fine.ncell, -1);
    for (long t = 0; t < ntri; ++t) coarse_of[cell_of[t]] = parts[l][t];
    UHostLevel C = coarsen(fine, coarse_of, (long)nmacro[l]);
    lev.push_back(C);
    cell_of = parts[l];
  }
}

// The interface grid of the coarser partition (fine cell c lies in coarse
// cell coarse_of[c]).  Faces whose two cells share a coarse cell are
// interior (E_I, eq. trace_partition); the others (E_B) are grouped by their
// pair of coarse cells, and each group into chains joined at vertices that
// exactly two of its faces share.  A chain with two distinct end vertices
// starts at the lower one; a closed chain (or one that comes back to its
// branch vertex) starts at that vertex (the lowest of a cycle) and leaves
// through its lower-numbered face there.  A macro-edge's coarse P^1 space is
// linear in the arc length s along its chain (s = 0 at the start, L at the
// end); J maps it onto the finer faces' P^1 traces.  Macro-edges are ordered
// by (lower coarse cell, higher coarse cell, lowest finer face).
UHostLevel UHost::coarsen(UHostLevel& fine, const std::vector<int>& coarse_of, long ncoarse) {
  const long nf = fine.nface;
  std::map<std::pair<int, int>, std::vector<int>> groups;
  std::vector<int> is_int(nf, 0);
  for (long f = 0; f < nf; ++f) {
    const int a = coarse_of[fine.fcell[2 * f]], b = coarse_of[fine.fcell[2 * f + 1]];
    if (a == b)
      is_int[f] = 1;
    else
      groups[{std::min(a, b), std::max(a, b)}].push_back((int)f);
  }
  struct Edge {
    int clo, chi, fmin, start, end;
    std::vector<std::pair<int, bool>> order;
  };
  std::vector<Edge> edges;
  for (auto& kv : groups) {
    std::vector<int>& fl = kv.second;  // ascending already
    std::map<int, std::vector<int>> inc;
    for (int f : fl) {
      inc[fine.fstart[f]].push_back(f);
      inc[fine.fend[f]].push_back(f);
    }
    auto deg = [&](int v) { return (int)inc[v].size(); };
    std::set<int> seen;
    for (int f0 : fl) {
      if (seen.count(f0)) continue;
      std::set<int> comp{f0};
      std::vector<int> stack{f0};
      while (!stack.empty()) {
        const int f = stack.back();
        stack.pop_back();
        for (int v : {fine.fstart[f], fine.fend[f]})
          if (deg(v) == 2)
            for (int g : inc[v])
              if (!comp.count(g)) {
                comp.insert(g);
                stack.push_back(g);
              }
      }
      seen.insert(comp.begin(), comp.end());
      std::vector<int> ends;
      for (int f : comp)
        for (int v : {fine.fstart[f], fine.fend[f]})
          if (deg(v) != 2) ends.push_back(v);
      int start;
      if (ends.size() == 2 && ends[0] != ends[1])
        start = std::min(ends[0], ends[1]);
      else if (ends.size() == 2)
        start = ends[0];
      else if (ends.empty()) {
        start = -1;
        for (int f : comp)
          for (int v : {fine.fstart[f], fine.fend[f]})
            if (start < 0 || v < start) start = v;
      } else
        throw std::runtime_error("macro-edge chain with a branch inside");
      int first = -1;
      for (int g : inc[start])
        if (comp.count(g) && (first < 0 || g < first)) first = g;
      Edge e;
      e.clo = kv.first.first;
      e.chi = kv.first.second;
      e.fmin = *comp.begin();
      e.start = start;
      std::set<int> used;
      int v = start, f = first;
      for (;;) {
        const bool fwd = fine.fstart[f] == v;
        e.order.push_back({f, fwd});
        used.insert(f);
        v = fwd ? fine.fend[f] : fine.fstart[f];
        if (deg(v) != 2) break;
        int nx = -1;
        for (int g : inc[v])
          if (!used.count(g)) {
            nx = g;
            break;
          }
        if (nx < 0) break;
        f = nx;
      }
      if (used.size() != comp.size()) throw std::runtime_error("macro-edge chain is not a simple path");
      e.end = v;
      edges.push_back(std::move(e));
    }
  }
  std::sort(edges.begin(), edges.end(), [](const Edge& a, const Edge& b) {
    if (a.clo != b.clo) return a.clo < b.clo;
    if (a.chi != b.chi) return a.chi < b.chi;
    return a.fmin < b.fmin;
  });
  UHostLevel C;
  C.m = 2;
  C.ncell = ncoarse;
  C.nface = (long)edges.size();
  fine.fE.assign(nf, -1);
  fine.fJ.assign(4 * nf, 0.0);
  std::vector<std::vector<int>> cell_edges(ncoarse);
  for (long E = 0; E < C.nface; ++E) {
    const Edge& e = edges[E];
    double L = 0.0;
    std::vector<std::pair<double, double>> pos;
    for (auto& fo : e.order) {
      const double s0 = L;
      L = L + fine.flen[fo.first];
      pos.push_back(fo.second ? std::make_pair(s0, L) : std::make_pair(L, s0));
    }
    for (size_t i = 0; i < e.order.size(); ++i) {
      const int f = e.order[i].first;
      fine.fE[f] = (int)E;
      const double p[2] = {pos[i].first, pos[i].second};
      for (int a = 0; a < 2; ++a) {
        const double t = p[a] / L;
        fine.fJ[4 * f + 2 * a + 0] = 1.0 - t;
        fine.fJ[4 * f + 2 * a + 1] = t;
      }
    }
    C.fstart.push_back(e.start);
    C.fend.push_back(e.end);
    C.flen.push_back(L);
    cell_edges[e.clo].push_back((int)E);
    cell_edges[e.chi].push_back((int)E);
  }
  // coarse cells' slots: their macro-edges in increasing order
  C.sptr.assign(ncoarse + 1, 0);
  for (long c = 0; c < ncoarse; ++c) {
    std::sort(cell_edges[c].begin(), cell_edges[c].end());
    C.sptr[c + 1] = C.sptr[c] + (long)cell_edges[c].size();
  }
  C.sface.resize(C.sptr[ncoarse]);
  C.fcell.assign(2 * C.nface, -1);
  C.fslot.assign(2 * C.nface, -1);
  for (long c = 0; c < ncoarse; ++c)
    for (size_t s = 0; s < cell_edges[c].size(); ++s) {
      const int E = cell_edges[c][s];
      C.sface[C.sptr[c] + s] = E;
      const int side = edges[E].clo == (int)c ? 0 : 1;
      C.fcell[2 * E + side] = (int)c;
      C.fslot[2 * E + side] = (int)s;
    }
  for (long E = 0; E < C.nface; ++E) {
    C.eptr.push_back((long)C.efine.size());
    for (auto& fo : edges[E].order) C.efine.push_back(fo.first);
  }
  C.eptr.push_back((long)C.efine.size());
  // per coarse cell: its fine cells, interior faces and boundary faces
  // (ascending), the local face index of every fine slot (interior faces
  // first, then boundary faces), and each boundary face's coarse slot
  fine.ncoarse = ncoarse;
  fine.ccptr.assign(ncoarse + 1, 0);
  std::vector<std::vector<int>> cells(ncoarse), ifs(ncoarse), bfs(ncoarse);
  for (long c = 0; c < fine.ncell; ++c) cells[coarse_of[c]].push_back((int)c);
  for (long f = 0; f < nf; ++f) {
    const int a = coarse_of[fine.fcell[2 * f]], b = coarse_of[fine.fcell[2 * f + 1]];
    if (is_int[f])
      ifs[a].push_back((int)f);
    else {
      bfs[a].push_back((int)f);
      bfs[b].push_back((int)f);
    }
  }
  fine.iptr.assign(ncoarse + 1, 0);
  fine.bptr.assign(ncoarse + 1, 0);
  fine.ccell.clear();
  fine.iface.clear();
  fine.bface.clear();
  fine.bslot.clear();
  fine.sloc.assign(fine.sptr[fine.ncell], -1);
  std::vector<int> loc(nf, -1);
  for (long c = 0; c < ncoarse; ++c) {
    std::sort(bfs[c].begin(), bfs[c].end());
    fine.ccptr[c + 1] = fine.ccptr[c] + (long)cells[c].size();
    fine.iptr[c + 1] = fine.iptr[c] + (long)ifs[c].size();
    fine.bptr[c + 1] = fine.bptr[c] + (long)bfs[c].size();
    for (int x : cells[c]) fine.ccell.push_back(x);
    for (size_t i = 0; i < ifs[c].size(); ++i) {
      fine.iface.push_back(ifs[c][i]);
      loc[ifs[c][i]] = (int)i;
    }
    const int nI = (int)ifs[c].size();
    for (size_t i = 0; i < bfs[c].size(); ++i) {
      const int f = bfs[c][i];
      fine.bface.push_back(f);
      const int E = fine.fE[f];
      const int slot = C.fcell[2 * E] == (int)c ? C.fslot[2 * E] : C.fslot[2 * E + 1];
      fine.bslot.push_back(slot);
      loc[f] = nI + (int)i;  // valid for c's own fine cells (set before they are read)
    }
    for (int x : cells[c])
      for (long s = fine.sptr[x]; s < fine.sptr[x + 1]; ++s)
        if (fine.sface[s] >= 0) fine.sloc[s] = loc[fine.sface[s]];
  }
  return C;
}

}  // namespace hdg
