// Host check of the topology builder (built with g++ and sanitizers by
// tests/test_topology_host.py): reads a mesh (int32 n, m; n*3 f64; m*4 i32),
// builds the topology and checks the compact lower/upper halves, their slot
// maps and the contribution slots.  Prints "err <message>" and exits 1 when
// the builder rejects the mesh, else "bad <count>" and exits with count != 0.
// With two more arguments (radius, output path) it also builds the support of
// the non-local damage criterion and writes it as int64 m, int64 entries,
// (m+1) int64 ptr, entries int32 idx, entries f64 weights (tets in input order).
// "--rcm" as the second argument renumbers the nodes in reverse Cuthill-McKee
// order, checks the permutation and prints the largest |i - j| over the edges
// (internal ids) after the count: "bad <count> band <b>".
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <string>
#include <fstream>
#include <vector>

#include "topo.hpp"

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  std::ifstream f(argv[1], std::ios::binary);
  int n = 0, m = 0;
  f.read(reinterpret_cast<char*>(&n), 4);
  f.read(reinterpret_cast<char*>(&m), 4);
  std::vector<double> X(3 * (size_t)n);
  std::vector<int32_t> T(4 * (size_t)m);
  f.read(reinterpret_cast<char*>(X.data()), 8 * X.size());
  f.read(reinterpret_cast<char*>(T.data()), 4 * T.size());
  const bool rcm = argc >= 3 && std::string(argv[2]) == "--rcm";
  gfem::Topology t;
  bool deg = false;
  const std::string err = gfem::build_topology(X.data(), n, T.data(), m, 1000.0, &t, &deg, rcm ? 1 : 0);
  if (!err.empty()) {
    printf("err %s\n", err.c_str());
    return 1;
  }
  int bad = 0;
  if (t.lptr[n] != t.ne || t.uptr[n] != t.ne || t.nb != n + 2 * t.ne) bad++;
  for (int i = 0; i < n; ++i) {
    for (int k = t.lptr[i]; k < t.lptr[i + 1]; ++k)
      if (t.lcol[k] >= i || (k > t.lptr[i] && t.lcol[k] <= t.lcol[k - 1])) bad++;
    for (int k = t.uptr[i]; k < t.uptr[i + 1]; ++k)
      if (t.ucol[k] <= i || (k > t.uptr[i] && t.ucol[k] <= t.ucol[k - 1])) bad++;
    if (t.col[t.diag_blk[i]] != i) bad++;
  }
  for (int e = 0; e < t.ne; ++e) {
    const int i = t.edges[2 * e], j = t.edges[2 * e + 1];
    const int lp = t.lpos[e], up = t.upos[e];
    if (i >= j) bad++;
    if (lp < t.lptr[j] || lp >= t.lptr[j + 1] || t.lcol[lp] != i) bad++;
    if (up < t.uptr[i] || up >= t.uptr[i + 1] || t.ucol[up] != j) bad++;
    if (t.col[t.blk_ji[e]] != i || t.blk_ji[e] - t.row_ptr[j] != lp - t.lptr[j]) bad++;
    if (t.col[t.blk_ij[e]] != j || t.blk_ij[e] - t.diag_blk[i] - 1 != up - t.uptr[i]) bad++;
    if (t.blk_edge[t.blk_ij[e]] != e || t.blk_edge[t.blk_ji[e]] != e) bad++;
  }
  // every (tet, local edge) contribution slot appears once, under its own edge
  std::vector<int> seen(6 * (size_t)m, 0);
  for (int e = 0; e < t.ne; ++e)
    for (int s = t.edge_ptr[e]; s < t.edge_ptr[e + 1]; ++s) {
      const int r = t.edge_slot[s];
      if (r < 0 || r >= 6 * m) {
        bad++;
        continue;
      }
      seen[r]++;
      if (t.tet_edge[r] != e) bad++;
    }
  for (int c : seen)
    if (c != 1) bad++;
  // workgroup-staged assembly tables: every (tet, local edge) slot of a
  // workgroup is summed into exactly one partial record; all of a record's
  // slots belong to one edge; each edge lists exactly its records, ascending
  {
    const int nwg = (m + gfem::kElemTets - 1) / gfem::kElemTets;
    const int np = (int)t.edge_part.size();
    if ((int)t.part_base.size() != nwg + 1 || t.part_base[nwg] != np || (int)t.part_cptr.size() != np + 1 ||
        t.part_cptr[np] != 6 * m || (int)t.part_slot.size() != 6 * m)
      bad++;
    std::vector<int> pedge(np, -1);
    std::vector<int> used(6 * (size_t)m, 0);
    for (int w = 0; w < nwg; ++w)
      for (int p = t.part_base[w]; p < t.part_base[w + 1]; ++p)
        for (int q = t.part_cptr[p]; q < t.part_cptr[p + 1]; ++q) {
          const int tt = w * gfem::kElemTets + t.part_slot[q] / 6, k = t.part_slot[q] % 6;
          if (tt >= m) {
            bad++;
            continue;
          }
          used[(size_t)tt * 6 + k]++;
          const int e = t.tet_edge[(size_t)k * m + tt];
          if (pedge[p] < 0) pedge[p] = e;
          else if (pedge[p] != e) bad++;
        }
    for (int c : used)
      if (c != 1) bad++;
    for (int e = 0; e < t.ne; ++e)
      for (int q = t.edge_pptr[e]; q < t.edge_pptr[e + 1]; ++q) {
        if (pedge[t.edge_part[q]] != e) bad++;
        if (q > t.edge_pptr[e] && t.edge_part[q] <= t.edge_part[q - 1]) bad++;
      }
  }
  // the numbering is a permutation and maps the caller's tets
  {
    std::vector<int> hit(n, 0);
    for (int i = 0; i < n; ++i) {
      if (t.perm_old[i] < 0 || t.perm_old[i] >= n || t.perm_new[t.perm_old[i]] != i) bad++;
      else hit[t.perm_old[i]]++;
    }
    for (int c : hit)
      if (c != 1) bad++;
    for (int q = 0; q < m; ++q) {
      int sa = 0, sb = 0;
      for (int a = 0; a < 4; ++a) {
        sa += t.tets[4 * (size_t)q + a];
        sb += t.perm_new[T[4 * (size_t)q + a]];
      }
      if (sa != sb) bad++;
    }
  }
  if (rcm) {
    int band = 0;
    for (int e = 0; e < t.ne; ++e) band = std::max(band, t.edges[2 * e + 1] - t.edges[2 * e]);
    printf("bad %d band %d\n", bad, band);
    return bad != 0;
  }
  if (argc >= 4) {
    std::vector<int64_t> ptr;
    std::vector<int32_t> idx;
    std::vector<double> w;
    const std::string e2 = gfem::build_nonlocal_support(t, std::atof(argv[2]), (size_t)1 << 31, &ptr, &idx, &w);
    if (!e2.empty()) {
      printf("err %s\n", e2.c_str());
      return 1;
    }
    std::ofstream o(argv[3], std::ios::binary);
    const int64_t hdr[2] = {m, (int64_t)idx.size()};
    o.write(reinterpret_cast<const char*>(hdr), sizeof hdr);
    o.write(reinterpret_cast<const char*>(ptr.data()), 8 * ptr.size());
    o.write(reinterpret_cast<const char*>(idx.data()), 4 * idx.size());
    o.write(reinterpret_cast<const char*>(w.data()), 8 * w.size());
  }
  printf("bad %d\n", bad);
  return bad != 0;
}
