// Host-side topology construction (see topo.hpp).
#include "topo.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>
#include <utility>

namespace gfem {

namespace {

double det3(const double* a, const double* b, const double* c) {
  return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
         a[2] * (b[0] * c[1] - b[1] * c[0]);
}

}  // namespace

// Reverse Cuthill-McKee order of the nodes of the tet graph (caller ids):
// per connected component a pseudo-peripheral start node (repeated
// breadth-first sweeps from a node of least degree, each restarting from a
// least-degree node of the last level, while the depth grows), then a
// breadth-first sweep visiting neighbours by increasing degree (ties by id);
// the whole order reversed.  Nodes in no tet come last.  Returns order[k] =
// the caller id of internal node k (before reversal order is CM).
std::vector<int32_t> rcm_order(int n, const int32_t* tets, int m) {
  std::vector<int64_t> pairs;
  pairs.reserve(12 * (size_t)m);
  for (int t = 0; t < m; ++t)
    for (int k = 0; k < 6; ++k) {
      const int64_t a = tets[4 * (size_t)t + kEdgeA[k]], b = tets[4 * (size_t)t + kEdgeB[k]];
      pairs.push_back(a * n + b);
      pairs.push_back(b * n + a);
    }
  std::sort(pairs.begin(), pairs.end());
  pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
  std::vector<int32_t> ptr(n + 1, 0), adj(pairs.size());
  for (size_t q = 0; q < pairs.size(); ++q) {
    ++ptr[pairs[q] / n + 1];
    adj[q] = (int32_t)(pairs[q] % n);
  }
  for (int i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
  auto deg = [&](int i) { return ptr[i + 1] - ptr[i]; };
  std::vector<int32_t> level(n, -1), order;
  order.reserve(n);
  std::vector<int32_t> queue;
  // breadth-first levels from s over unplaced nodes; returns the last level's nodes
  auto sweep = [&](int s, std::vector<int32_t>& seen) {
    queue.assign(1, s);
    seen.push_back(s);
    level[s] = 0;
    int depth = 0;
    for (size_t h = 0; h < queue.size(); ++h) {
      const int v = queue[h];
      depth = level[v];
      for (int q = ptr[v]; q < ptr[v + 1]; ++q)
        if (level[adj[q]] < 0) {
          level[adj[q]] = level[v] + 1;
          queue.push_back(adj[q]);
          seen.push_back(adj[q]);
        }
    }
    return depth;
  };
  std::vector<char> placed(n, 0);
  std::vector<int32_t> by_degree(n);
  std::iota(by_degree.begin(), by_degree.end(), 0);
  std::stable_sort(by_degree.begin(), by_degree.end(), [&](int a, int b) { return deg(a) < deg(b); });
  std::vector<int32_t> seen, nb;
  for (int root : by_degree) {
    if (placed[root] || deg(root) == 0) continue;
    int start = root, depth = -1;
    for (int rep = 0; rep < 8; ++rep) {
      seen.clear();
      const int d = sweep(start, seen);
      int best = -1;
      for (int v : seen)
        if (level[v] == d && (best < 0 || deg(v) < deg(best) || (deg(v) == deg(best) && v < best))) best = v;
      for (int v : seen) level[v] = -1;
      if (d <= depth) break;
      depth = d;
      start = best;
    }
    // Cuthill-McKee sweep from start
    const size_t first = order.size();
    order.push_back(start);
    placed[start] = 1;
    for (size_t h = first; h < order.size(); ++h) {
      const int v = order[h];
      nb.clear();
      for (int q = ptr[v]; q < ptr[v + 1]; ++q)
        if (!placed[adj[q]]) nb.push_back(adj[q]);
      std::sort(nb.begin(), nb.end(), [&](int a, int b) { return deg(a) != deg(b) ? deg(a) < deg(b) : a < b; });
      for (int w : nb) {
        placed[w] = 1;
        order.push_back(w);
      }
    }
  }
  std::reverse(order.begin(), order.end());
  for (int i = 0; i < n; ++i)
    if (!placed[i]) order.push_back(i);
  return order;
}

std::string build_topology(const double* xyz, int n, const int32_t* tets_in, int m, double density,
                           Topology* out, bool* degenerate, int reorder) {
  *degenerate = false;
  Topology& T = *out;
  if (n <= 0 || m <= 0) return "n_nodes and n_tets must be positive";
  for (int i = 0; i < 3 * n; ++i)
    if (!std::isfinite(xyz[i])) return "non-finite rest coordinate";
  T.n = n;
  T.m = m;
  for (size_t q = 0; q < 4 * (size_t)m; ++q)
    if (tets_in[q] < 0 || tets_in[q] >= n) {
      char buf[128];
      snprintf(buf, sizeof buf, "tet %d references node %d outside [0,%d)", (int)(q / 4), tets_in[q], n);
      return buf;
    }

  // Node numbering: the caller's order, or reverse Cuthill-McKee.
  T.perm_new.resize(n);
  T.perm_old.resize(n);
  if (reorder == 1) {
    T.perm_old = rcm_order(n, tets_in, m);
    for (int k = 0; k < n; ++k) T.perm_new[T.perm_old[k]] = k;
  } else {
    std::iota(T.perm_new.begin(), T.perm_new.end(), 0);
    std::iota(T.perm_old.begin(), T.perm_old.end(), 0);
  }
  T.X.resize(3 * (size_t)n);
  for (int i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) T.X[3 * (size_t)T.perm_new[i] + d] = xyz[3 * (size_t)i + d];

  // Validate ids, reorient negative tets (swap local nodes 2 and 3), reject flat ones.
  T.tets.resize(4 * (size_t)m);
  T.tet_swapped.assign(m, 0);
  T.vol.resize(m);
  T.reoriented = 0;
  for (int t = 0; t < m; ++t) {
    int v[4];
    for (int a = 0; a < 4; ++a) {
      int id = tets_in[4 * (size_t)t + a];
      if (id < 0 || id >= n) {
        char buf[128];
        snprintf(buf, sizeof buf, "tet %d references node %d outside [0,%d)", t, id, n);
        return buf;
      }
      v[a] = T.perm_new[id];
    }
    if (v[0] == v[1] || v[0] == v[2] || v[0] == v[3] || v[1] == v[2] || v[1] == v[3] || v[2] == v[3]) {
      *degenerate = true;
      char buf[96];
      snprintf(buf, sizeof buf, "tet %d repeats a node", t);
      return buf;
    }
    double e[3][3];
    double lmax = 0.0;
    for (int i = 1; i < 4; ++i)
      for (int d = 0; d < 3; ++d) e[i - 1][d] = T.X[3 * (size_t)v[i] + d] - T.X[3 * (size_t)v[0] + d];
    for (int k = 0; k < 6; ++k) {
      double s = 0;
      for (int d = 0; d < 3; ++d) {
        double q = T.X[3 * (size_t)v[kEdgeB[k]] + d] - T.X[3 * (size_t)v[kEdgeA[k]] + d];
        s += q * q;
      }
      lmax = std::max(lmax, std::sqrt(s));
    }
    double vol6 = det3(e[0], e[1], e[2]);
    if (std::fabs(vol6 / 6.0) <= 1e-14 * lmax * lmax * lmax) {
      *degenerate = true;
      char buf[96];
      snprintf(buf, sizeof buf, "tet %d has (near) zero volume", t);
      return buf;
    }
    if (vol6 < 0) {
      std::swap(v[2], v[3]);
      vol6 = -vol6;
      ++T.reoriented;
      T.tet_swapped[t] = 1;
    }
    T.vol[t] = vol6 / 6.0;
    for (int a = 0; a < 4; ++a) T.tets[4 * (size_t)t + a] = v[a];
  }

  // Unique edges: sort the 6m (min, max, slot) records.
  struct Rec {
    int32_t i, j, t, k;
  };
  std::vector<Rec> rec(6 * (size_t)m);
  for (int t = 0; t < m; ++t)
    for (int k = 0; k < 6; ++k) {
      int a = T.tets[4 * (size_t)t + kEdgeA[k]], b = T.tets[4 * (size_t)t + kEdgeB[k]];
      rec[6 * (size_t)t + k] = {std::min(a, b), std::max(a, b), t, k};
    }
  std::sort(rec.begin(), rec.end(), [](const Rec& x, const Rec& y) {
    if (x.i != y.i) return x.i < y.i;
    if (x.j != y.j) return x.j < y.j;
    if (x.t != y.t) return x.t < y.t;
    return x.k < y.k;
  });
  T.tet_edge.assign(6 * (size_t)m, -1);
  T.tet_flip.assign(m, 0);
  T.edge_slot.resize(6 * (size_t)m);
  T.edges.clear();
  T.edge_ptr.clear();
  for (size_t r = 0; r < rec.size(); ++r) {
    if (r == 0 || rec[r].i != rec[r - 1].i || rec[r].j != rec[r - 1].j) {
      T.edge_ptr.push_back((int32_t)r);
      T.edges.push_back(rec[r].i);
      T.edges.push_back(rec[r].j);
    }
    int e = (int)T.edge_ptr.size() - 1;
    const Rec& q = rec[r];
    T.tet_edge[(size_t)q.k * m + q.t] = e;
    T.edge_slot[r] = q.k * m + q.t;
    if (T.tets[4 * (size_t)q.t + kEdgeA[q.k]] > T.tets[4 * (size_t)q.t + kEdgeB[q.k]])
      T.tet_flip[q.t] |= (uint8_t)(1u << q.k);
  }
  T.ne = (int)T.edge_ptr.size();
  T.edge_ptr.push_back((int32_t)rec.size());
  T.nb = T.n + 2 * T.ne;

  // Block pattern: row i holds i itself and every edge neighbour, sorted.
  std::vector<int32_t> deg(n, 1);
  for (int e = 0; e < T.ne; ++e) {
    ++deg[T.edges[2 * e]];
    ++deg[T.edges[2 * e + 1]];
  }
  T.row_ptr.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) T.row_ptr[i + 1] = T.row_ptr[i] + deg[i];
  T.col.assign(T.nb, -1);
  T.blk_edge.assign(T.nb, -1);
  std::vector<int32_t> fill(T.row_ptr.begin(), T.row_ptr.end() - 1);
  // Edges are sorted by (i, j): for row i, neighbours j > i arrive in order;
  // neighbours j < i arrive in order of their own row.  Insert then sort.
  for (int i = 0; i < n; ++i) T.col[fill[i]++] = i;
  for (int e = 0; e < T.ne; ++e) {
    int i = T.edges[2 * e], j = T.edges[2 * e + 1];
    T.blk_edge[fill[i]] = e;
    T.col[fill[i]++] = j;
    T.blk_edge[fill[j]] = e;
    T.col[fill[j]++] = i;
  }
  T.diag_blk.resize(n);
  T.blk_ij.resize(T.ne);
  T.blk_ji.resize(T.ne);
  std::vector<std::pair<int32_t, int32_t>> tmp;
  for (int i = 0; i < n; ++i) {
    int s = T.row_ptr[i], e = T.row_ptr[i + 1];
    tmp.clear();
    for (int b = s; b < e; ++b) tmp.push_back({T.col[b], T.blk_edge[b]});
    std::sort(tmp.begin(), tmp.end());
    for (int b = s; b < e; ++b) {
      T.col[b] = tmp[b - s].first;
      T.blk_edge[b] = tmp[b - s].second;
      if (T.col[b] == i) {
        T.diag_blk[i] = b;
      } else {
        int ed = T.blk_edge[b];
        if (i < T.col[b])
          T.blk_ij[ed] = b;
        else
          T.blk_ji[ed] = b;
      }
    }
  }

  // Compact strictly lower / upper halves of the pattern.
  T.lptr.assign(n + 1, 0);
  T.uptr.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    T.lptr[i + 1] = T.lptr[i] + (T.diag_blk[i] - T.row_ptr[i]);
    T.uptr[i + 1] = T.uptr[i] + (T.row_ptr[i + 1] - T.diag_blk[i] - 1);
  }
  T.lcol.resize(T.ne);
  T.ucol.resize(T.ne);
  T.lpos.resize(T.ne);
  T.upos.resize(T.ne);
  for (int i = 0; i < n; ++i) {
    for (int b = T.row_ptr[i]; b < T.diag_blk[i]; ++b) {
      const int li = T.lptr[i] + (b - T.row_ptr[i]);
      T.lcol[li] = T.col[b];
      T.lpos[T.blk_edge[b]] = li;
    }
    for (int b = T.diag_blk[i] + 1; b < T.row_ptr[i + 1]; ++b) {
      const int ui = T.uptr[i] + (b - T.diag_blk[i] - 1);
      T.ucol[ui] = T.col[b];
      T.upos[T.blk_edge[b]] = ui;
    }
  }

  // Rest squared edge lengths and the consistent mass (Eq. 5):
  // m_ab = rho V (1 + delta_ab) / 20 per tet; off-diagonal per edge, row sums per node.
  T.edge_S.resize(T.ne);
  for (int e = 0; e < T.ne; ++e) {
    double s = 0;
    for (int d = 0; d < 3; ++d) {
      double q = T.X[3 * (size_t)T.edges[2 * e + 1] + d] - T.X[3 * (size_t)T.edges[2 * e] + d];
      s += q * q;
    }
    T.edge_S[e] = s;
  }
  T.edge_mass.assign(T.ne, 0.0);
  T.lumped.assign(n, 0.0);
  for (int e = 0; e < T.ne; ++e)
    for (int r = T.edge_ptr[e]; r < T.edge_ptr[e + 1]; ++r) {
      int t = T.edge_slot[r] % m;
      T.edge_mass[e] += density * T.vol[t] / 20.0;
    }
  for (int t = 0; t < m; ++t)
    for (int a = 0; a < 4; ++a) T.lumped[T.tets[4 * (size_t)t + a]] += density * T.vol[t] / 4.0;

  // Workgroup-staged assembly tables (see topo.hpp): per workgroup of
  // kElemTets tets, its (edge, tet, local edge) contributions sorted by edge,
  // then tet, then local edge; one partial record per distinct edge.
  {
    const int nwg = (m + kElemTets - 1) / kElemTets;
    T.part_base.assign(nwg + 1, 0);
    T.part_cptr.assign(1, 0);
    T.part_slot.clear();
    T.part_slot.reserve(6 * (size_t)m);
    std::vector<int32_t> part_edge;
    std::vector<std::pair<int32_t, int32_t>> loc;  // (edge, local slot)
    for (int w = 0; w < nwg; ++w) {
      const int t0 = w * kElemTets, t1 = std::min(m, t0 + kElemTets);
      loc.clear();
      for (int t = t0; t < t1; ++t)
        for (int k = 0; k < 6; ++k) loc.push_back({T.tet_edge[(size_t)k * m + t], 6 * (t - t0) + k});
      std::sort(loc.begin(), loc.end());
      for (size_t q = 0; q < loc.size(); ++q) {
        if (q > 0 && loc[q].first != loc[q - 1].first) T.part_cptr.push_back((int32_t)T.part_slot.size());
        if (q == 0 || loc[q].first != loc[q - 1].first) part_edge.push_back(loc[q].first);
        T.part_slot.push_back((uint16_t)loc[q].second);
      }
      if (!loc.empty()) T.part_cptr.push_back((int32_t)T.part_slot.size());
      T.part_base[w + 1] = (int32_t)part_edge.size();
    }
    const int np = (int)part_edge.size();
    T.edge_pptr.assign(T.ne + 1, 0);
    for (int p = 0; p < np; ++p) ++T.edge_pptr[part_edge[p] + 1];
    for (int e = 0; e < T.ne; ++e) T.edge_pptr[e + 1] += T.edge_pptr[e];
    T.edge_part.assign(np, 0);
    std::vector<int32_t> fillp(T.edge_pptr.begin(), T.edge_pptr.end() - 1);
    for (int p = 0; p < np; ++p) T.edge_part[fillp[part_edge[p]]++] = p;
  }

  // Canonical edge order (caller ids, i < j, lexicographic).
  std::vector<std::pair<std::pair<int32_t, int32_t>, int32_t>> ce(T.ne);
  for (int e = 0; e < T.ne; ++e) {
    int a = T.perm_old[T.edges[2 * e]], b = T.perm_old[T.edges[2 * e + 1]];
    ce[e] = {{std::min(a, b), std::max(a, b)}, e};
  }
  std::sort(ce.begin(), ce.end());
  T.edge_canon.resize(T.ne);
  T.edge_internal.resize(T.ne);
  for (int c = 0; c < T.ne; ++c) {
    T.edge_internal[c] = ce[c].second;
    T.edge_canon[ce[c].second] = c;
  }
  return "";
}

std::string build_nonlocal_support(const Topology& T, double radius, size_t max_entries,
                                   std::vector<int64_t>* ptr, std::vector<int32_t>* idx,
                                   std::vector<double>* w) {
  if (!(radius > 0.0) || !std::isfinite(radius)) return "non-local support radius must be positive and finite";
  const int m = T.m;
  std::vector<double> c(3 * (size_t)m);
  double lo[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL}, hi[3] = {-HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
  for (int t = 0; t < m; ++t)
    for (int d = 0; d < 3; ++d) {
      double acc = 0.0;
      for (int a = 0; a < 4; ++a) acc += T.X[3 * (size_t)T.tets[4 * (size_t)t + a] + d];
      c[3 * (size_t)t + d] = acc / 4.0;
      lo[d] = std::min(lo[d], c[3 * (size_t)t + d]);
      hi[d] = std::max(hi[d], c[3 * (size_t)t + d]);
    }
  // cells of edge >= radius, at most 512 per axis: a neighbour within radius
  // is always in one of the 27 cells around a tet's own
  double cell = radius;
  for (int d = 0; d < 3; ++d) cell = std::max(cell, (hi[d] - lo[d]) / 512.0);
  int dim[3];
  for (int d = 0; d < 3; ++d) dim[d] = std::max(1, (int)std::floor((hi[d] - lo[d]) / cell) + 1);
  auto cell_of = [&](int t, int* q) {
    for (int d = 0; d < 3; ++d)
      q[d] = std::min(dim[d] - 1, std::max(0, (int)std::floor((c[3 * (size_t)t + d] - lo[d]) / cell)));
  };
  const size_t ncell = (size_t)dim[0] * dim[1] * dim[2];
  std::vector<int32_t> cstart(ncell + 1, 0), order(m);
  for (int t = 0; t < m; ++t) {
    int q[3];
    cell_of(t, q);
    ++cstart[((size_t)q[2] * dim[1] + q[1]) * dim[0] + q[0] + 1];
  }
  for (size_t i = 0; i < ncell; ++i) cstart[i + 1] += cstart[i];
  {
    std::vector<int32_t> fill(cstart.begin(), cstart.end() - 1);
    for (int t = 0; t < m; ++t) {  // ascending within each cell
      int q[3];
      cell_of(t, q);
      order[fill[((size_t)q[2] * dim[1] + q[1]) * dim[0] + q[0]]++] = t;
    }
  }
  const double r2 = radius * radius;
  ptr->assign((size_t)m + 1, 0);
  idx->clear();
  w->clear();
  std::vector<std::pair<int32_t, double>> nb;
  for (int t = 0; t < m; ++t) {
    int q[3];
    cell_of(t, q);
    nb.clear();
    for (int z = std::max(0, q[2] - 1); z <= std::min(dim[2] - 1, q[2] + 1); ++z)
      for (int y = std::max(0, q[1] - 1); y <= std::min(dim[1] - 1, q[1] + 1); ++y)
        for (int x = std::max(0, q[0] - 1); x <= std::min(dim[0] - 1, q[0] + 1); ++x) {
          const size_t ci = ((size_t)z * dim[1] + y) * dim[0] + x;
          for (int i = cstart[ci]; i < cstart[ci + 1]; ++i) {
            const int j = order[i];
            double d2 = 0.0;
            for (int d = 0; d < 3; ++d) {
              const double dd = c[3 * (size_t)j + d] - c[3 * (size_t)t + d];
              d2 += dd * dd;
            }
            if (d2 <= r2) {
              const double u = 1.0 - d2 / r2;
              nb.push_back({j, u * u});
            }
          }
        }
    std::sort(nb.begin(), nb.end());
    double sum = 0.0;
    for (const auto& e : nb) sum += e.second;
    if (idx->size() + nb.size() > max_entries) return "non-local support too large for the device buffers";
    for (const auto& e : nb) {
      idx->push_back(e.first);
      w->push_back(e.second / sum);
    }
    (*ptr)[t + 1] = (int64_t)idx->size();
  }
  return "";
}

}  // namespace gfem
