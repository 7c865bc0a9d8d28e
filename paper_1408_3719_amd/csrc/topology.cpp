// Host topology: edges, node rings, WENO stencils and scheduling stencils.
//
// Stencil definitions (the paper fixes the stencil counts and sizes in Sec. 2.2,
// eqs. stencil and eqn.WENOstencil, and defers the construction to its
// references; these are the readings this library implements):
//   * n_e = 2 nb elements per stencil, element i first.
//   * barycentre c_j = ((x0+x1+x2)/3, (y0+y1+y2)/3), distance key
//     d2 = dx*dx + dy*dy (evaluated without fused multiply-add, so the
//     ranking is reproducible bit for bit).
//   * central stencil: breadth-first layers over face neighbours, ranked by
//     (layer, d2, index) until n_e elements are taken;
//   * sector stencils at local vertex k with apex P = X_k, e1 = X_{k+1} - P,
//     e2 = X_{k+2} - P and d = c_j - P: the primary sector admits
//     cross(d,e2) > 0 and cross(e1,d) > 0, the reverse sector admits both < 0.
//     Candidates are the elements within M+4 vertex-adjacency steps of i; the
//     admitted ones are ranked by (d2, index) and the first n_e - 1 follow i;
//     with fewer candidates the stencil is dropped (row of -1);
//   * stencil order: 0 central, 1..3 primary at vertices 0..2, 4..6 reverse.
//   * scheduling stencil S_i: symmetric closure of (union of the stencils of i)
//     and (all elements sharing a node with i) -- symmetric so the LTS update
//     criterion cannot deadlock (discussion after eq. eqn.WENOupdate), and
//     containing the vertex ring so every predictor read by the node solver
//     and the swept patches lies inside its time slab.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "host.h"

namespace aw {

// Runs fn(begin, end) over [0, n) split into contiguous chunks on up to 16
// host threads (the work items are independent).
template <class F>
void parallel_for(int n, F fn) {
  int nt = int(std::thread::hardware_concurrency());
  nt = nt < 1 ? 1 : (nt > 16 ? 16 : nt);
  if (n < 4096) nt = 1;
  if (nt == 1) {
    fn(0, n);
    return;
  }
  std::vector<std::thread> th;
  const int chunk = (n + nt - 1) / nt;
  for (int w = 0; w < nt; ++w) {
    const int b = w * chunk, e = std::min(n, b + chunk);
    if (b < e) th.emplace_back([=, &fn] { fn(b, e); });
  }
  for (auto& x : th) x.join();
}

void build_topology(int M, int NV, const double* xy, int NE, const int* tri_in, int NB,
                    const int* bedge, Topology& t) {
  const int nb = (M + 1) * (M + 2) / 2;
  const int ne = 2 * nb;
  t = Topology();
  t.NE = NE;
  t.NV = NV;
  t.ne = ne;
  t.xy.assign(xy, xy + 2 * NV);
  t.tri.assign(tri_in, tri_in + 3 * NE);
  const int* tri = t.tri.data();
  for (int i = 0; i < NE; ++i) {
    for (int k = 0; k < 3; ++k)
      if (tri[3 * i + k] < 0 || tri[3 * i + k] >= NV)
        throw std::runtime_error("triangle " + std::to_string(i) + " has a node index out of range");
    const double* p0 = xy + 2 * tri[3 * i];
    const double* p1 = xy + 2 * tri[3 * i + 1];
    const double* p2 = xy + 2 * tri[3 * i + 2];
    double a2 = (p1[0] - p0[0]) * (p2[1] - p0[1]) - (p2[0] - p0[0]) * (p1[1] - p0[1]);
    if (!(a2 > 0.0))
      throw std::runtime_error("triangle " + std::to_string(i) + " is clockwise or degenerate");
  }
  // ---- edges -------------------------------------------------------------------
  std::map<std::pair<int, int>, int> key;
  t.elem_edges.assign(3 * NE, -1);
  for (int i = 0; i < NE; ++i)
    for (int k = 0; k < 3; ++k) {
      int a = tri[3 * i + k], b = tri[3 * i + (k + 1) % 3];
      auto kk = std::make_pair(std::min(a, b), std::max(a, b));
      auto it = key.find(kk);
      int e;
      if (it == key.end()) {
        e = int(t.e_a.size());
        key[kk] = e;
        t.e_a.push_back(a);
        t.e_b.push_back(b);
        t.e_L.push_back(i);
        t.e_R.push_back(-1);
        t.e_el.push_back(k);
        t.e_er.push_back(-1);
        t.e_bc.push_back(0);
      } else {
        e = it->second;
        if (t.e_R[e] != -1 || t.e_a[e] != b || t.e_b[e] != a)
          throw std::runtime_error("mesh is not a consistently oriented manifold (edge " +
                                   std::to_string(a) + "-" + std::to_string(b) + ")");
        t.e_R[e] = i;
        t.e_er[e] = k;
      }
      t.elem_edges[3 * i + k] = e;
    }
  t.NF = int(t.e_a.size());
  t.neigh.assign(3 * NE, -1);
  for (int e = 0; e < t.NF; ++e)
    if (t.e_R[e] >= 0) {
      t.neigh[3 * t.e_L[e] + t.e_el[e]] = t.e_R[e];
      t.neigh[3 * t.e_R[e] + t.e_er[e]] = t.e_L[e];
    }
  // ---- boundary tags -------------------------------------------------------------
  int nbnd = 0;
  for (int e = 0; e < t.NF; ++e) nbnd += (t.e_R[e] < 0);
  if (nbnd != NB) throw std::runtime_error("boundary edge list does not match the mesh boundary");
  for (int j = 0; j < NB; ++j) {
    int a = bedge[3 * j], b = bedge[3 * j + 1], tag = bedge[3 * j + 2];
    auto it = key.find(std::make_pair(std::min(a, b), std::max(a, b)));
    if (it == key.end() || t.e_R[it->second] >= 0 || t.e_a[it->second] != a || t.e_b[it->second] != b)
      throw std::runtime_error("boundary edge " + std::to_string(j) + " is not a boundary edge of the mesh");
    if (tag != 1 && tag != 2) throw std::runtime_error("unknown boundary tag");
    t.e_bc[it->second] = tag;
  }
  // ---- node rings -----------------------------------------------------------------
  t.ring_ptr.assign(NV + 1, 0);
  for (int i = 0; i < 3 * NE; ++i) t.ring_ptr[tri[i] + 1]++;
  for (int k = 0; k < NV; ++k) t.ring_ptr[k + 1] += t.ring_ptr[k];
  t.ring_ent.assign(3 * NE, 0);
  {
    std::vector<int> fill(t.ring_ptr.begin(), t.ring_ptr.end() - 1);
    for (int i = 0; i < NE; ++i)
      for (int k = 0; k < 3; ++k) t.ring_ent[fill[tri[3 * i + k]]++] = i * 4 + k;
  }
  for (int k = 0; k < NV; ++k)
    if (t.ring_ptr[k + 1] == t.ring_ptr[k]) throw std::runtime_error("node " + std::to_string(k) + " is unused");
  // ---- slip walls --------------------------------------------------------------------
  t.wall_n.assign(2 * NV, 0.0);
  t.wall_pin.assign(NV, 0);
  for (int e = 0; e < t.NF; ++e) {
    if (t.e_bc[e] != 2) continue;
    int a = t.e_a[e], b = t.e_b[e];
    double dx = xy[2 * b] - xy[2 * a], dy = xy[2 * b + 1] - xy[2 * a + 1];
    double h = std::hypot(dx, dy);
    double nx = dy / h, ny = -dx / h;
    for (int k : {a, b}) {
      double ox = t.wall_n[2 * k], oy = t.wall_n[2 * k + 1];
      if ((ox != 0.0 || oy != 0.0) && std::fabs(ox * ny - oy * nx) > 1e-9) t.wall_pin[k] = 1;
      t.wall_n[2 * k] = nx;
      t.wall_n[2 * k + 1] = ny;
    }
  }
  // ---- barycentres and vertex adjacency ---------------------------------------------
  std::vector<double> bx(NE), by(NE);
  for (int i = 0; i < NE; ++i) {
    const double* p0 = xy + 2 * tri[3 * i];
    const double* p1 = xy + 2 * tri[3 * i + 1];
    const double* p2 = xy + 2 * tri[3 * i + 2];
    bx[i] = (p0[0] + p1[0] + p2[0]) / 3.0;
    by[i] = (p0[1] + p1[1] + p2[1]) / 3.0;
  }
  auto d2of = [&](int i, int j) {
    double dx = bx[j] - bx[i], dy = by[j] - by[i];
    return dx * dx + dy * dy;
  };
  std::vector<std::vector<int>> vadj(NE);
  parallel_for(NE, [&](int i0, int i1) {
    for (int i = i0; i < i1; ++i) {
      std::vector<int>& v = vadj[i];
      for (int k = 0; k < 3; ++k) {
        int nd = tri[3 * i + k];
        for (int r = t.ring_ptr[nd]; r < t.ring_ptr[nd + 1]; ++r) v.push_back(t.ring_ent[r] >> 2);
      }
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
    }
  });
  // ---- stencils (independent per element; each worker has its own marks) ------------------
  t.sten.assign(size_t(NE) * NSTEN * ne, -1);
  std::vector<std::string> errors;
  std::mutex err_mu;
  parallel_for(NE, [&](int i0, int i1) {
    std::vector<int> mark(NE, -1);
    std::vector<int> layer, next, cand, adm, ord;
    for (int i = i0; i < i1; ++i) {
      int* st = &t.sten[size_t(i) * NSTEN * ne];
      // central
      {
        int cnt = 0;
        st[cnt++] = i;
        mark[i] = 2 * i;
        layer.assign(1, i);
        while (cnt < ne && !layer.empty()) {
          next.clear();
          for (int j : layer)
            for (int k = 0; k < 3; ++k) {
              int m = t.neigh[3 * j + k];
              if (m >= 0 && mark[m] != 2 * i) {
                mark[m] = 2 * i;
                next.push_back(m);
              }
            }
          ord = next;
          std::sort(ord.begin(), ord.end(), [&](int x, int y) {
            double dx = d2of(i, x), dy = d2of(i, y);
            return dx < dy || (dx == dy && x < y);
          });
          for (int m : ord)
            if (cnt < ne) st[cnt++] = m;
          layer = next;
        }
        if (cnt < ne) {
          std::lock_guard<std::mutex> g(err_mu);
          errors.push_back("mesh too small: central stencil of element " + std::to_string(i) +
                           " cannot be filled");
          return;
        }
      }
      // candidate pool: vertex-adjacency distance 1..M+4
      cand.clear();
      mark[i] = 2 * i + 1;
      layer.assign(1, i);
      for (int depth = 1; depth <= M + 4; ++depth) {
        next.clear();
        for (int j : layer)
          for (int m : vadj[j])
            if (mark[m] != 2 * i + 1) {
              mark[m] = 2 * i + 1;
              next.push_back(m);
              cand.push_back(m);
            }
        layer.swap(next);
      }
      for (int k = 0; k < 3; ++k) {
        const double* P = xy + 2 * tri[3 * i + k];
        const double* Q1 = xy + 2 * tri[3 * i + (k + 1) % 3];
        const double* Q2 = xy + 2 * tri[3 * i + (k + 2) % 3];
        double e1x = Q1[0] - P[0], e1y = Q1[1] - P[1];
        double e2x = Q2[0] - P[0], e2y = Q2[1] - P[1];
        for (int sgn = 0; sgn < 2; ++sgn) {
          adm.clear();
          for (int j : cand) {
            double dx = bx[j] - P[0], dy = by[j] - P[1];
            double c1 = dx * e2y - dy * e2x;
            double c2 = e1x * dy - e1y * dx;
            bool in = sgn == 0 ? (c1 > 0.0 && c2 > 0.0) : (c1 < 0.0 && c2 < 0.0);
            if (in) adm.push_back(j);
          }
          if (int(adm.size()) < ne - 1) continue;
          std::sort(adm.begin(), adm.end(), [&](int x, int y) {
            double dx = d2of(i, x), dy = d2of(i, y);
            return dx < dy || (dx == dy && x < y);
          });
          int s = sgn == 0 ? 1 + k : 4 + k;
          st[s * ne] = i;
          for (int c = 0; c < ne - 1; ++c) st[s * ne + 1 + c] = adm[c];
        }
      }
    }
  });
  if (!errors.empty()) {
    std::sort(errors.begin(), errors.end());
    throw std::runtime_error(errors.front());
  }
  // ---- scheduling stencils: symmetric closure of (stencils + vertex ring) ------------------
  std::vector<std::vector<int>> U(NE);
  parallel_for(NE, [&](int i0, int i1) {
    for (int i = i0; i < i1; ++i) {
      std::vector<int>& u = U[i];
      u = vadj[i];
      const int* st = &t.sten[size_t(i) * NSTEN * ne];
      for (int s = 0; s < NSTEN; ++s)
        if (st[s * ne] >= 0)
          for (int c = 0; c < ne; ++c) u.push_back(st[s * ne + c]);
      u.push_back(i);
      std::sort(u.begin(), u.end());
      u.erase(std::unique(u.begin(), u.end()), u.end());
    }
  });
  std::vector<std::vector<int>> S(NE);
  for (int i = 0; i < NE; ++i)
    for (int j : U[i]) {
      S[i].push_back(j);
      S[j].push_back(i);
    }
  t.sched_ptr.assign(NE + 1, 0);
  t.sched_idx.clear();
  parallel_for(NE, [&](int i0, int i1) {
    for (int i = i0; i < i1; ++i) {
      std::vector<int>& v = S[i];
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
    }
  });
  for (int i = 0; i < NE; ++i) {
    t.sched_idx.insert(t.sched_idx.end(), S[i].begin(), S[i].end());
    t.sched_ptr[i + 1] = int(t.sched_idx.size());
  }
  // transposed stencil rows (counting sort by the element named)
  t.tsten_ptr.assign(NE + 1, 0);
  for (int i = 0; i < NE; ++i)
    for (int s = 0; s < NSTEN; ++s) {
      const int* st = &t.sten[(size_t(i) * NSTEN + s) * ne];
      if (st[0] < 0) continue;
      for (int c = 1; c < ne; ++c) t.tsten_ptr[st[c] + 1]++;
    }
  for (int j = 0; j < NE; ++j) t.tsten_ptr[j + 1] += t.tsten_ptr[j];
  t.tsten_idx.assign(t.tsten_ptr[NE], 0);
  std::vector<int> fill(t.tsten_ptr.begin(), t.tsten_ptr.end() - 1);
  for (int i = 0; i < NE; ++i)
    for (int c = 1; c < ne; ++c)
      for (int s = 0; s < NSTEN; ++s) {
        const int* st = &t.sten[(size_t(i) * NSTEN + s) * ne];
        if (st[0] < 0) continue;
        t.tsten_idx[fill[st[c]]++] = (i * ne + c) * 8 + s;
      }
}

}  // namespace aw
