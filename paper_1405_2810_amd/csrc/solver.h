// Reduced SPD solver: multifrontal block Cholesky over the coarse boxes.
//
// The block pattern of A_N (eq. reducedSystem) is fixed by the coarse grid:
// a box couples to itself and to its face neighbours.  The symbolic phase
// (host, once per model) orders the boxes by nested dissection (recursive
// bisection of the box grid along its longest axis with one separator slab),
// builds the assembly tree of fronts (a front = one separator or one small
// leaf region; its update set U = the boxes adjacent to its region, all of
// them in ancestor separators) and all index maps.
//
// Every front is stored dense, column-major, with one extra row at the
// bottom that carries the right-hand side, so that the forward substitution
// happens inside the factorization.  The numeric phase runs every step on
// the device, one tree level at a time:
//   assemble  one workgroup per destination block of a front (box pair, or the
//             right-hand-side row against one box): the block of A_N or f_N
//             plus the children's update blocks, summed in a fixed order and
//             written once; then one workgroup per front factors its first
//             diagonal tile;
//   step      one launch per panel: every tile workgroup forms its rows of L
//             (F Linv^T, kept in a separate buffer), and applies the trailing
//             update F(ti,tj) -= L(ti) L(tj)^T to the columns of S; the
//             workgroup of the next diagonal tile factors it (look-ahead);
//   schur     after the last panel, the U x U block and the right-hand-side
//             row's U part in one product with all m columns of L_US
//             (one 128 x 128 output tile per workgroup, FP64 MFMA), instead
//             of one rank-64 update per panel;
//   backward  one workgroup per front, from the root down, with the stored
//             tile inverses.
// Diagonal tiles are factored by a 16-wide blocked Cholesky: the 16 x 16
// diagonal blocks are factored and inverted in registers by one wave, the
// panel solves and trailing updates are parallel over the workgroup; the
// inverse is completed block diagonal by block diagonal.
#pragma once

#include "common.h"

namespace lrbms {

constexpr int kNB = 64;       // panel / tile width of the dense front kernels
constexpr int kSB = 128;      // output tile of the deferred Schur complement
constexpr int kMaxLd = 8192;  // largest front (rows) handled by the backward sweep

struct FrontD {
  long long off;      // front storage (column-major, lda = m + u + 1, m + u columns)
  long long loff;     // rows of L below each diagonal tile, panel-major (see lpanel_base)
  long long voff;     // backward-substitution vector workspace
  long long inv_off;  // tile inverses, one kNB x kNB per panel
  int m, u;
  int node_off, n_nodes;   // nodes of S then U: (pos in front, p_N offset, size, pos in parent)
  int child_off, nchild;   // children (front ids) in extend-add order
  int n_s_nodes, npanels;
  // large fronts: the backward product L_US^T x_U split over nzc workgroups
  // of 64 U rows each, partial vectors (m each) at zoff; U row r takes x_U
  // from p_N[urow_pn[urow_off + r]]
  int nzc = 0, urow_off = 0;
  long long zoff = 0;
  int member = 0;     // member of a combined plan (0 in a single plan)
  // left-looking U-row tiles: the products of the panels before the last
  // one, summed ahead by the previous step's prefetch items into two
  // alternating buffers of pf_nt tiles x pf_ns chunks of 64 x 64 at pf_off
  int pf_nt = 0;
  int pf_ns = 0, pad = 0;
  long long pf_off = 0;
};
// Panels per prefetch chunk (one workgroup each).
constexpr int kPfPanels = 4;

// One workgroup of the split backward product: 64 U rows of one front.
struct BwItem { int front, chunk; };
// Smallest m u (front entries of L_US) whose backward product is split
// (environment variable LRBMS_BW_SPLIT_MIN, default 2^14).
long long bw_split_min();

struct NodeRef { int pos, pn_off, size, ppos; };

// Row block of one box in A_N, for the residual of the iterative refinement:
// the diagonal block (lower triangle used, as the factorization does) and
// neighbour blocks nb0 .. nb1-1 of the residual plan.
struct ResBox { long long blk_off; int pn_off, ne, nb0, nb1, member; };
// One coupling block of a box's rows: A(i, j) = blocks[blk_off + i rs + j cs]
// for the neighbour's ne unknowns at p_N[pn_off ..].
struct ResNb { long long blk_off; int pn_off, ne, rs, cs; };

// The L rows below the diagonal tile of panel b of a front (rows cs_b .. ld,
// cs_b = min(kNB (b + 1), m), the last one the forward-substituted right-hand
// side) are stored row by row, kNB doubles per row: row r of panel b starts
// at lpanel_base(f, b) + (r - cs_b) kNB.  All panels before the last are full.
__host__ __device__ inline long long lpanel_base(const FrontD& f, int b) {
  const long long ld1 = (long long)f.m + f.u + 1;
  return f.loff + (long long)kNB * (b * ld1 - 32LL * b * (b + 1));
}

// One destination block of a front (box pair, or the right-hand-side row against
// one box) with up to three sources summed in a fixed order: the block of A_N
// or f_N, then the children's update blocks.  Source element (i, j) is
// src[so + i*rs + j*cs] in the blocks of A_N (kind 0), the front storage (1) or
// f_N (2).  diag: a diagonal block, of which only the lower part is formed.
struct AsmSrc { long long so; int rs, cs, kind, pad; };
struct AsmItem { int front, dr, dc, nr, nc, diag, nsrc, pad; AsmSrc src[3]; };
// One tile of the fused panel step; tj = -1: rows only (no trailing columns).
// The trailing columns of a step are the front's S columns only: the U x U
// block and the right-hand-side row's U part are updated once, after the
// last panel, by the deferred Schur complement (SchurItem).
struct StepItem { int front, panel, ti, tj; };
// One output tile of a front's deferred Schur complement, T x T with T = kSB
// when wide, else kNB: rows m + T ti .. (U rows and the right-hand-side row),
// columns m + T tj .. (U columns), tj <= ti; on a wide diagonal tile (ti = tj)
// the kNB x kNB block above the diagonal (rows < kNB, columns >= kNB of the
// tile) is left out.  Fronts with at least kSchurWideMin U columns take wide
// tiles (fewer re-reads of L_US); smaller ones the narrow tiles, whose
// padding and launch share cost less there.
struct SchurItem { int front, ti, tj, wide; };
constexpr int kSchurWideMin = 512;

struct SolverPlan {
  std::vector<FrontD> fronts;
  std::vector<NodeRef> nodes;
  std::vector<int> children;
  std::vector<int> elim;                       // elimination position of every box
  int nlevels = 0;
  std::vector<std::vector<int>> level_fronts;  // front ids per level (height)
  std::vector<std::vector<AsmItem>> asm_items;
  std::vector<std::vector<std::vector<StepItem>>> step_items;  // [level][panel]
  // Steps with many tiles are split in two launches: step_items then holds
  // one rows-only item (tj = -1) per tile row, and upd_items the trailing
  // updates, which read both L tiles from the L store instead of forming them
  std::vector<std::vector<std::vector<StepItem>>> upd_items;   // [level][panel]
  std::vector<std::vector<BwItem>> bw_items;                    // [level]
  std::vector<std::vector<SchurItem>> schur_items;              // [level]
  std::vector<int> urow_pn;
  // residual plan (boxes in p_N order) and the number of reduced unknowns
  std::vector<ResBox> rboxes;
  std::vector<ResNb> rnbs;
  long long nN = 0;
  long long bw_part_doubles = 0;   // partial vectors of the split products (one level at a time)
  long long pf_doubles = 0;        // prefetch buffers of the panel steps (one level at a time)
  long long front_doubles = 0, vec_doubles = 0, inv_doubles = 0, lpan_doubles = 0;
  double flops = 0.0;                          // factorization flops per solve
  // algorithmic flops and bytes of every launch (for the kernel timer)
  std::vector<double> asm_flops, asm_bytes, f0_flops, f0_bytes, bw_flops, bw_bytes;  // [level]
  std::vector<double> bwg_flops, bwg_bytes;   // split backward products [level]
  std::vector<double> fw_flops, fw_bytes;     // forward substitution with a new right-hand side [level]
  std::vector<double> schur_flops, schur_bytes;   // deferred Schur complements [level]
  double res_flops = 0.0, res_bytes = 0.0;    // residual of the refinement
  std::vector<std::vector<double>> step_flops, step_bytes;                           // [level][panel]
  std::vector<std::vector<double>> upd_flops, upd_bytes;                             // [level][panel]
};

// Smallest number of tiles of one panel step that is split in two launches
// (environment variable LRBMS_STEP_SPLIT_MIN, default 1024).
int step_split_min();
void split_steps(SolverPlan& plan, int split_min);
// Work items and partial storage of the split backward products, from the
// fronts' nzc (level by level, fronts in level order).
void assign_backward_split(SolverPlan& plan);
// Offsets of the panel steps' prefetch buffers (per level, fronts side by side).
void assign_prefetch(SolverPlan& plan);

// Build the plan for the box grid with box sizes subs[].NE and interfaces;
// panel steps of at least split_min tiles are split (split_min < 0: the
// default of step_split_min()), and the backward product of every front with
// m u >= bw_min (bw_min < 0: the default of bw_split_min()).
bool build_solver_plan(int dim, const int nc[3], const std::vector<Sub>& subs,
                       const std::vector<Iface>& ifaces, int leaf_max, SolverPlan& plan,
                       int split_min = -1, long long bw_min = -1);

// One plan for several independent systems solved together: the fronts, node
// references and work lists of member k are appended level by level (levels
// counted by height, so every member keeps its own order: assembly, first
// tile, panel steps of a level before the next level; the backward sweep
// from each member's root down), with all offsets shifted into shared
// storage: front storage, L panels, inverses and vectors by the sizes of
// the members before it, blocks of A_N by blk_base[k], f_N and p_N by
// pn_base[k].  Every front is computed by the same items as in its own
// plan, so each member's result is unchanged bit for bit.
bool combine_plans(const std::vector<const SolverPlan*>& plans,
                   const std::vector<long long>& blk_base, const std::vector<long long>& pn_base,
                   SolverPlan& out);

// Host check that every access the numeric kernels derive from the plan
// stays inside its storage: fronts, L panels, inverses, vectors, node and
// child lists, and sources in A_N (nblk doubles), f_N and p_N (nN doubles).
bool plan_in_bounds(const SolverPlan& plan, long long nblk, long long nN);

// Device copy of a plan plus workspaces.
struct SolverDev {
  FrontD* fronts = nullptr;
  NodeRef* nodes = nullptr;
  int* children = nullptr;
  std::vector<AsmItem*> asm_items;
  std::vector<std::vector<StepItem*>> step_items;
  std::vector<std::vector<StepItem*>> upd_items;
  std::vector<BwItem*> bw_items;
  std::vector<SchurItem*> schur_items;
  int* urow_pn = nullptr;
  ResBox* rboxes = nullptr;
  ResNb* rnbs = nullptr;
  double* part = nullptr;
  double* pf = nullptr;     // prefetch buffers (pf_doubles)
  double* res = nullptr;   // residual of the refinement (nN)
  double* cor = nullptr;   // its correction (nN)
  std::vector<int*> level_fronts;
  double* F = nullptr;
  double* L = nullptr;
  double* V = nullptr;
  double* Inv = nullptr;
  long long bytes = 0;
};

bool solver_upload(const SolverPlan& plan, SolverDev& dev);
void solver_free(SolverDev& dev);
// Factor A_N (blocks, f_N) and solve for p_N, then `refine` steps of
// iterative refinement: the residual f_N - A_N p_N accumulated in
// double-double arithmetic (compensated products and sums), a forward and a
// backward substitution of it with the stored factor, and p_N += correction.
// A non-finite residual sets the status word to LRBMS_E_NONFINITE.
// active (device, nullable): per member of a combined plan 1 to solve, 0 to
// skip (every workgroup of a skipped member's fronts returns at once).
// ref_masks (device, nullable): the members taking refinement step k, as
// refine masks of mstride flags each (step k reads ref_masks + k mstride);
// without it every step takes the members of `active`.
hipError_t solver_factor_solve(const SolverPlan& plan, const SolverDev& dev,
                               const double* blocks, const double* fN, double* pN,
                               int* status, hipStream_t st, int refine = 0,
                               const int* active = nullptr, const int* ref_masks = nullptr,
                               int mstride = 0);
constexpr int kMaxRefine = 4;

}  // namespace lrbms
