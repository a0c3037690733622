// Host-side model object behind the opaque lrbms_model handle.
#pragma once

#include "common.h"
#include "ktimer.h"
#include "solver.h"

namespace lrbms {

struct Model {
  Geom g{};
  int nc[3] = {1, 1, 1};
  int n_sub = 0, n_iface = 0, N = 0, max_ne = 0;
  std::vector<Sub> subs;
  std::vector<Iface> ifaces;
  long long phi_len = 0, nblk = 0;
  Sub* d_subs = nullptr;
  Iface* d_ifaces = nullptr;
  double *d_perm = nullptr, *d_poro = nullptr, *d_q1 = nullptr, *d_q2 = nullptr;
  double *d_bc_val = nullptr, *d_bc_sval = nullptr;
  int8_t *d_bc_type = nullptr, *d_bc_sat = nullptr;
  double* d_phi = nullptr;      // local bases, per box (N_E, r, n_E)
  double* d_tr = nullptr;       // face traces of the bases, per interface (Iface::tr_off)
  long long tr_len = 0;
  double* d_mom = nullptr;      // mobility moments, n_moments(dim) x ncell
  double* d_blocks = nullptr;   // A_N in block storage
  double* d_fN = nullptr;
  // affine decomposition (Sec. 4.4)
  int nprof = 0, lsq_blocks = 0;
  bool lsq_ok = false;          // the profile Gram matrix is factored (least-squares fit)
  double *d_prof = nullptr, *d_gchol = nullptr, *d_theta = nullptr, *d_partial = nullptr;
  double *d_c = nullptr, *d_bq = nullptr, *d_e = nullptr, *d_dq = nullptr;
  // fine-grid scratch
  int* d_tiles = nullptr;
  int n_tiles = 0;
  double* d_scratch_sat = nullptr;
  double* d_scratch_ph = nullptr;
  int* d_status = nullptr;
  AsmLayout asm_layout;
  // reduced solver
  int leaf_max = 2;             // leaf size of the nested dissection (chosen per model)
  int split_min = -1;           // smallest panel step that is split (-1: the default)
  long long bw_min = -1;        // smallest m u whose backward product is split (-1: the default)
  int refine = 1;
  int asm_variant = 0;   // box assembly variant (AsmLayout)               // iterative refinement steps of every reduced solve
  bool checks = false;          // online calls wait for their work and return the status
  SolverPlan plan;
  SolverDev sdev;
  bool assembled = false;
  // fused batch (whose storage holds d_blocks / d_fN) or server the model is
  // attached to; the model cannot be destroyed while it is set
  void* owner = nullptr;
  hipStream_t last_stream = nullptr;
  long long dev_bytes = 0;
  // kernel timing and the fixed per-launch algorithmic figures per kernel kind
  KernelTimer timer;
  double unit_flops[KK_COUNT] = {}, unit_bytes[KK_COUNT] = {};
  ~Model();
};

// lsq: the profiles are independent and the model fits theta from s (AFFINE,
// DIRECT_FIT); without it the affine terms serve a caller-given theta only.
// basis: host bases in the model layout, or d_basis: device bases the model
// takes over (freed with the model, also when this fails).
int model_finish(Model& M, const double* basis, int nprof, const double* profiles, bool lsq,
                 double* d_basis = nullptr);
int model_create_impl(const lrbms_problem* p, const int32_t* sizes, const double* basis, int nprof,
                      const double* profiles, lrbms_model** out);

}  // namespace lrbms
