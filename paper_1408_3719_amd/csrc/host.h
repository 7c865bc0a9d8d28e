// Host-side pieces of the aderweno library: tables and topology.
#pragma once
#include <string>
#include <vector>

#include "common.h"

namespace aw {

void gauss_legendre01(int n, double* x, double* w);
void build_tables(int M, Tables& T);

// Mesh topology built once on the host (paper Sec. 2.2: fixed stencils).
struct Topology {
  int NE = 0, NV = 0, NF = 0, ne = 0;
  std::vector<double> xy;                 // [NV][2] initial node positions
  std::vector<int> tri;                   // [NE][3]
  // edges in order of first appearance (elements by index, local edges 0,1,2)
  std::vector<int> e_a, e_b, e_L, e_R, e_el, e_er, e_bc;
  std::vector<int> elem_edges;            // [NE][3]
  std::vector<int> neigh;                 // [NE][3], -1 on the boundary
  std::vector<int> ring_ptr, ring_ent;    // node -> (element*4 + local vertex), by element
  std::vector<int> sten;                  // [NE][7][ne], -1 rows: dropped
  std::vector<int> sched_ptr, sched_idx;  // symmetric scheduling stencils (sorted)
  // for each element j, the stencil rows (c >= 1) that name it, as slots
  // ((i * ne + c) * 8 + s) of row c of stencil s of element i, ascending
  std::vector<int> tsten_ptr, tsten_idx;
  std::vector<double> wall_n;             // [NV][2] slip-wall unit normal or 0
  std::vector<int> wall_pin;              // [NV]
};

// Throws std::runtime_error with a message on an invalid mesh.
void build_topology(int M, int n_nodes, const double* xy, int n_elems, const int* tri,
                    int n_bedges, const int* bedge, Topology& t);

}  // namespace aw
