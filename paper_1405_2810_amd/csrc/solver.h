// Reduced SPD solver: multifrontal block Cholesky over the coarse boxes.
//
// The block pattern of A_N (eq. reducedSystem) is fixed by the coarse grid:
// a box couples to itself and to its face neighbours.  The symbolic phase
// (host, once per model) orders the boxes by nested dissection (recursive
// bisection of the box grid along its longest axis with one separator slab),
// builds the assembly tree of fronts (a front = one separator or one small
// leaf region; its update set U = the boxes adjacent to its region, all of
// them in ancestor separators) and all index maps.  The numeric phase runs
// every step on the device, one tree level at a time:
//   assemble  zero the fronts, add the blocks of A_N, extend-add the
//             children's update matrices (children in a fixed order);
//   panel     Cholesky of a NB x NB diagonal tile in LDS, its triangular
//             inverse, and L = F Linv^T for the tile rows below it;
//   update    F(ti, tj) -= L(ti) L(tj)^T on the trailing tiles;
//   forward / backward substitution with the stored tile inverses.
#pragma once

#include "common.h"

namespace lrbms {

constexpr int kNB = 64;  // panel / tile width of the dense front kernels

struct FrontD {
  long long off;    // front storage (column-major, ld = m + u)
  long long voff;   // front vector workspace
  long long inv_off;// tile inverses, one kNB x kNB per panel
  int m, u;
  int node_off, n_nodes;   // nodes of S then U: (pos in front, p_N offset, size)
  int child_off, nchild;   // children (front ids) in extend-add order
  int n_s_nodes;
};

struct NodeRef { int pos, pn_off, size, pad; };

// Strided block add into a front: F[(dr+i) + (dc+j)*ld] += src[so + i*rs + j*cs].
struct AddTask {
  long long so;
  int rs, cs, nr, nc, dr, dc, from_front, pad;
};

struct AsmItem { int front, col0, ncol, task_off, ntask, pad; };
struct PanelItem { int front, panel, row0, nrow; };
struct UpdItem { int front, panel, ti, tj; };

struct SolverPlan {
  std::vector<FrontD> fronts;
  std::vector<NodeRef> nodes;
  std::vector<int> children;
  std::vector<int> elim;                       // elimination position of every box
  int nlevels = 0;
  // per level
  std::vector<std::vector<int>> level_fronts;  // front ids
  std::vector<std::vector<AsmItem>> asm_items;
  std::vector<AddTask> tasks;
  std::vector<std::vector<std::vector<PanelItem>>> panel_items;  // [level][panel]
  std::vector<std::vector<std::vector<UpdItem>>> upd_items;      // [level][panel]
  long long front_doubles = 0, vec_doubles = 0, inv_doubles = 0;
  double flops = 0.0;                          // factorization flops per solve
  long long front_bytes_touched = 0;
};

// Build the plan for a box grid nc[3] with box sizes ne[n_sub] and interfaces.
bool build_solver_plan(int dim, const int nc[3], const std::vector<Sub>& subs,
                       const std::vector<Iface>& ifaces, int leaf_max, SolverPlan& plan);

// Device copy of a plan plus workspaces.
struct SolverDev {
  FrontD* fronts = nullptr;
  NodeRef* nodes = nullptr;
  int* children = nullptr;
  AddTask* tasks = nullptr;
  std::vector<AsmItem*> asm_items;
  std::vector<std::vector<PanelItem*>> panel_items;
  std::vector<std::vector<UpdItem*>> upd_items;
  std::vector<int*> level_fronts;
  double* F = nullptr;
  double* V = nullptr;
  double* Inv = nullptr;
  long long bytes = 0;
};

bool solver_upload(const SolverPlan& plan, SolverDev& dev);
void solver_free(SolverDev& dev);
hipError_t solver_factor_solve(const SolverPlan& plan, const SolverDev& dev,
                               const double* blocks, const double* fN, double* pN,
                               int* status, hipStream_t st);

}  // namespace lrbms
