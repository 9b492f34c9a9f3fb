// Host-side mesh topology for the graph-based FEM library: validation,
// reorientation, the induced graph (nodes + unique tet edges, Sec. 1 and
// Sec. 3.1), the fixed 3x3 block-sparse pattern (one block per node and two
// per edge), the edge -> contribution-slot map used by the deterministic
// assembly, and the consistent mass of Eq. 5.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace gfem {

// Local edge k of a tet joins local nodes kEdgeA[k] -> kEdgeB[k]; this is the
// 12,13,14,23,24,34 order of Eq. 15.
constexpr int kEdgeA[6] = {0, 0, 0, 1, 1, 2};
constexpr int kEdgeB[6] = {1, 2, 3, 2, 3, 3};

// Tets per workgroup of the element pass (its contributions are summed per
// edge in LDS before they go to memory).
constexpr int kElemTets = 128;

struct Topology {
  int n = 0;   // nodes
  int m = 0;   // tets
  int ne = 0;  // edges
  int nb = 0;  // stored 3x3 blocks = n + 2 ne

  std::vector<double> X;          // n*3 rest positions (internal order)
  std::vector<int32_t> tets;      // m*4, positively oriented (internal ids)
  std::vector<int32_t> edges;     // ne*2, i < j, sorted (internal ids)
  std::vector<int32_t> tet_edge;  // 6*m, SoA: tet_edge[k*m + t]
  std::vector<uint8_t> tet_flip;  // m: bit k set when the global edge runs b -> a
  std::vector<uint8_t> tet_swapped;  // m: 1 when local nodes 2 and 3 were swapped (negative input orientation)
  std::vector<int32_t> edge_ptr;  // ne+1: contributions of edge e are
  std::vector<int32_t> edge_slot; //   edge_slot[edge_ptr[e] .. edge_ptr[e+1]) = k*m + t
  std::vector<int32_t> row_ptr;   // n+1 block rows
  std::vector<int32_t> col;       // nb block columns, sorted per row
  std::vector<int32_t> diag_blk;  // n
  std::vector<int32_t> blk_ij;    // ne: block (i,j) of edge e, i < j
  std::vector<int32_t> blk_ji;    // ne: block (j,i)
  std::vector<int32_t> blk_edge;  // nb: edge of an off-diagonal block, -1 on the diagonal
  // Strictly lower / strictly upper halves of the pattern as compact CSR (same
  // column order as the full pattern): row i's lower blocks are entries
  // lptr[i] .. lptr[i+1] of lcol, its upper blocks uptr[i] .. uptr[i+1] of ucol.
  std::vector<int32_t> lptr, lcol, uptr, ucol;  // n+1, ne, n+1, ne
  std::vector<int32_t> lpos, upos;  // ne: compact lower / upper index of edge e's blocks (j,i) / (i,j)
  // Workgroup-staged assembly: the element pass runs kElemTets tets per
  // workgroup and sums, in LDS, its tets' contributions to each edge the
  // workgroup touches into one partial record.  Partial records are numbered
  // workgroup by workgroup, by edge within a workgroup:
  //   part_base[w] .. part_base[w+1]   partial records of workgroup w (n_wg + 1)
  //   part_cptr[p] .. part_cptr[p+1]   entries of part_slot summed into record p (P + 1)
  //   part_slot[q]                     LDS slot 6 * (t - w * kElemTets) + k, in summation order (6m)
  //   edge_pptr[e] .. edge_pptr[e+1]   entries of edge_part: edge e's partial records, ascending (ne + 1)
  std::vector<int32_t> part_base, part_cptr, edge_pptr, edge_part;
  std::vector<uint16_t> part_slot;
  std::vector<double> edge_S;     // ne: rest squared length
  std::vector<double> edge_mass;  // ne: consistent off-diagonal mass, sum rho V / 20
  std::vector<double> lumped;     // n: row sum of the consistent mass, sum rho V / 4
  std::vector<double> vol;        // m: rest volume
  int reoriented = 0;

  // Node numbering: internal id = perm_new[caller id]; caller = perm_old[internal].
  std::vector<int32_t> perm_new, perm_old;
  // Canonical (caller-order) edge index of each internal edge, and inverse.
  std::vector<int32_t> edge_canon, edge_internal;
};

// Builds the topology.  Returns "" on success, otherwise an error message;
// *degenerate is set when the failure is a flat tet.  reorder: 0 keeps the
// caller's node order internally, 1 renumbers the nodes in reverse
// Cuthill-McKee order (narrow band: the gathers of neighbouring rows stay
// close in memory whatever order the caller's ids come in).
std::string build_topology(const double* xyz, int n, const int32_t* tets, int m, double density,
                           Topology* out, bool* degenerate, int reorder = 0);

// Reverse Cuthill-McKee order of the nodes of the tet graph: entry k is the
// caller id of internal node k.
std::vector<int32_t> rcm_order(int n, const int32_t* tets, int m);

// Support of the non-local fracture criterion (Sec. 3.3, Eq. 20): for each tet
// t the tets whose rest centroids lie within `radius` of t's (t included),
// ascending, with the kernel weights (1 - (r/radius)^2)^2 normalised to sum 1
// over the support.  CSR: entries ptr[t] .. ptr[t+1] of idx / w.  Built on a
// uniform grid of cell size >= radius (each tet scans the 27 cells around its
// own).  Returns "" on success, otherwise an error message (radius not
// positive and finite, or more than max_entries entries in total).
std::string build_nonlocal_support(const Topology& T, double radius, size_t max_entries,
                                   std::vector<int64_t>* ptr, std::vector<int32_t>* idx,
                                   std::vector<double>* w);

}  // namespace gfem
