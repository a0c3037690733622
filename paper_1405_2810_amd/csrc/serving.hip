// Many simulations on one device: the batched ensemble step (all simulations
// advanced by one graph launch) and the serving loop (online steps of many
// simulations admitted by memory footprint, dispatched onto slot streams as
// slots free up, their work overlapping on the device).
//
// Both run, per simulation, exactly the calls of one online step (Alg. 3
// step 5): mobility + reduced assembly, the reduced solve, p_h and the face
// fluxes, the saturation step with the limiter; a simulation's result is the
// one the plain per-simulation path gives, bit for bit, because the same
// kernels run on the same data in the same order.
#include <algorithm>
#include <chrono>
#include <deque>
#include <memory>
#include <string>
#include <vector>

#include "common.h"
#include "model.h"
#include "solver.h"

namespace lrbms {

namespace {

// Buffers of one simulation's step that the batch or the server owns: p_N,
// the face fluxes and the next state (copied back over the caller's state).
struct StepBufs {
  double* pN = nullptr;
  double* flux = nullptr;
  double* next = nullptr;
  bool own_pN = true;
  long long bytes = 0;
  // pN_ext: p_N lives in storage the caller owns (the fused batch's p_N)
  bool alloc(const Model& M, double* pN_ext = nullptr) {
    release();
    const size_t n[3] = {(size_t)std::max(M.N, 1), (size_t)std::max(M.g.nface, 1),
                         (size_t)M.g.r * M.g.ncell};
    double** p[3] = {&pN, &flux, &next};
    own_pN = pN_ext == nullptr;
    if (!own_pN) pN = pN_ext;
    for (int k = own_pN ? 0 : 1; k < 3; ++k) {
      if (!hip_ok(hipMalloc(p[k], n[k] * sizeof(double)), "hipMalloc")) {
        release();
        return false;
      }
      bytes += (long long)(n[k] * sizeof(double));
    }
    return true;
  }
  void release() {
    if (pN && own_pN) (void)hipFree(pN);
    for (double* q : {flux, next})
      if (q) (void)hipFree(q);
    pN = flux = next = nullptr;
    own_pN = true;
    bytes = 0;
  }
};

Model* model_of(lrbms_model* m) { return reinterpret_cast<Model*>(m); }

bool mode_ok(const Model& M, int mode) {
  if (mode == LRBMS_DIRECT) return true;
  if (mode != LRBMS_DIRECT_FIT && mode != LRBMS_AFFINE) return false;
  return M.nprof > 0 && M.lsq_ok;
}

// Members of a wave: mask[i] = 1 for the listed members of a combined plan, 0
// for the others; then kMaxRefine refinement masks of `total` flags each:
// mask[(1 + k) total + i] = 1 for the listed members that take refinement
// step k (refs[j] > k).
struct MaskArgs {
  int count, total;
  int ids[64];
  int refs[64];
};
__global__ void k_set_mask(int* __restrict__ mask, MaskArgs a) {
  for (int i = threadIdx.x; i < (1 + kMaxRefine) * a.total; i += blockDim.x) mask[i] = 0;
  __syncthreads();
  if ((int)threadIdx.x < a.count) {
    const int id = a.ids[threadIdx.x], ref = a.refs[threadIdx.x];
    mask[id] = 1;
    for (int k = 0; k < kMaxRefine; ++k) mask[(1 + k) * a.total + id] = ref > k ? 1 : 0;
  }
}

// The part of one online step after the reduced solve: p_h, the fluxes, the
// saturation step with the limiter, and the new state copied over d_sat.
int sim_after_solve(lrbms_model* m, double* d_sat, uint8_t* d_flags, const StepBufs& b,
                    hipStream_t st) {
  int rc;
  if ((rc = lrbms_reconstruct_flux(m, b.pN, d_sat, b.flux, nullptr, st)) != LRBMS_OK) return rc;
  if ((rc = lrbms_transport_step(m, d_sat, b.flux, b.next, d_flags, st)) != LRBMS_OK) return rc;
  const Model& M = *model_of(m);
  const size_t bytes = (size_t)M.g.r * M.g.ncell * sizeof(double);
  if (!hip_ok(hipMemcpyAsync(d_sat, b.next, bytes, hipMemcpyDeviceToDevice, st), "state copy"))
    return LRBMS_E_HIP;
  return LRBMS_OK;
}

// One online step of one simulation on stream st; the state d_sat is
// advanced in place (through b.next).
int sim_step(lrbms_model* m, int mode, double* d_sat, uint8_t* d_flags, const StepBufs& b,
             hipStream_t st) {
  int rc;
  if ((rc = lrbms_online_assemble(m, d_sat, mode, st)) != LRBMS_OK) return rc;
  if ((rc = lrbms_online_solve(m, b.pN, st)) != LRBMS_OK) return rc;
  return sim_after_solve(m, d_sat, d_flags, b, st);
}

}  // namespace

// ---- batched ensemble ------------------------------------------------------------

struct Batch {
  std::vector<lrbms_model*> models;
  std::vector<StepBufs> bufs;
  int mode = LRBMS_DIRECT;
  bool use_graph = true;
  std::vector<hipStream_t> branch;       // one per simulation, up to kBranches
  hipStream_t origin = nullptr;          // capture origin
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<double*> cap_sat;          // state pointers the graph was captured with
  std::vector<uint8_t*> cap_flags;
  static constexpr int kBranches = 64;
  // fused reduced solve: one plan for all members, shared storage for A_N,
  // f_N and p_N (the members' block pointers point into it while the batch
  // lives), one status word
  bool fused = false;
  SolverPlan cplan;
  SolverDev cdev;
  double *cblocks = nullptr, *cfN = nullptr, *cpN = nullptr;
  int* cstatus = nullptr;
  int refine = 0;          // refinement steps of the fused solve: the members' largest
  int* cref = nullptr;     // device, kMaxRefine x n: members taking step k (nullptr: all)
  std::vector<double*> own_blocks, own_fN;
  hipEvent_t fork2 = nullptr;
  std::vector<hipEvent_t> join2;

  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    cap_sat.clear();
    cap_flags.clear();
  }
  ~Batch() {
    (void)hipDeviceSynchronize();
    drop_graph();
    // members of a fused batch get their own block storage back
    for (size_t i = 0; i < models.size(); ++i) {
      Model* M = model_of(models[i]);
      if (M->owner != this) continue;
      if (i < own_blocks.size()) {
        M->d_blocks = own_blocks[i];
        M->d_fN = own_fN[i];
      }
      M->owner = nullptr;
    }
    for (auto& b : bufs) b.release();
    solver_free(cdev);
    for (void* q : {(void*)cblocks, (void*)cfN, (void*)cpN, (void*)cstatus, (void*)cref})
      if (q) (void)hipFree(q);
    for (hipEvent_t e : join) (void)hipEventDestroy(e);
    for (hipEvent_t e : join2) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    if (fork2) (void)hipEventDestroy(fork2);
    for (hipStream_t s : branch) (void)hipStreamDestroy(s);
    if (origin) (void)hipStreamDestroy(origin);
  }

  int fork_from(hipStream_t from, hipEvent_t ev) {
    if (!hip_ok(hipEventRecord(ev, from), "fork")) return LRBMS_E_HIP;
    for (hipStream_t b : branch)
      if (!hip_ok(hipStreamWaitEvent(b, ev, 0), "fork")) return LRBMS_E_HIP;
    return LRBMS_OK;
  }
  int join_into(hipStream_t from, std::vector<hipEvent_t>& evs) {
    for (size_t b = 0; b < branch.size(); ++b)
      if (!hip_ok(hipEventRecord(evs[b], branch[b]), "join") ||
          !hip_ok(hipStreamWaitEvent(from, evs[b], 0), "join"))
        return LRBMS_E_HIP;
    return LRBMS_OK;
  }

  // Fork from `from`, one step of every simulation on its branch, join back.
  // Fused: the members' assemblies on their branches, the combined reduced
  // solve on `from`, then the members' flux and transport on their branches.
  int enqueue(hipStream_t from, double* const* d_sat, uint8_t* const* d_flags) {
    const int nb = (int)branch.size();
    int rc;
    if ((rc = fork_from(from, fork)) != LRBMS_OK) return rc;
    for (size_t i = 0; i < models.size(); ++i) {
      uint8_t* fl = d_flags ? d_flags[i] : nullptr;
      rc = fused ? lrbms_online_assemble(models[i], d_sat[i], mode, branch[i % nb])
                 : sim_step(models[i], mode, d_sat[i], fl, bufs[i], branch[i % nb]);
      if (rc != LRBMS_OK) return rc;
    }
    if ((rc = join_into(from, join)) != LRBMS_OK || !fused) return rc;
    if (!hip_ok(solver_factor_solve(cplan, cdev, cblocks, cfN, cpN, cstatus, from, refine,
                                    nullptr, cref, (int)models.size()),
                "fused reduced solve"))
      return LRBMS_E_HIP;
    if ((rc = fork_from(from, fork2)) != LRBMS_OK) return rc;
    for (size_t i = 0; i < models.size(); ++i) {
      rc = sim_after_solve(models[i], d_sat[i], d_flags ? d_flags[i] : nullptr, bufs[i],
                           branch[i % nb]);
      if (rc != LRBMS_OK) return rc;
    }
    return join_into(from, join2);
  }

  // Shared storage and the combined plan of the fused solve.
  int setup_fused() {
    const size_t n = models.size();
    std::vector<const SolverPlan*> plans;
    std::vector<long long> blk_base, pn_base;
    long long nblk = 0, nN = 0;
    for (lrbms_model* m : models) {
      const Model& M = *model_of(m);
      plans.push_back(&M.plan);
      blk_base.push_back(nblk);
      pn_base.push_back(nN);
      nblk += M.nblk;
      nN += M.N;
    }
    if (!combine_plans(plans, blk_base, pn_base, cplan) || !plan_in_bounds(cplan, nblk, nN))
      return (set_error("fused solve: plans cannot be combined"), LRBMS_E_ARG);
    if (!solver_upload(cplan, cdev)) return (set_error("fused solve: upload failed"), LRBMS_E_OOM);
    auto zalloc = [](void** p, size_t bytes) {
      return hip_ok(hipMalloc(p, std::max<size_t>(bytes, 8)), "hipMalloc") &&
             hip_ok(hipMemset(*p, 0, std::max<size_t>(bytes, 8)), "hipMemset");
    };
    if (!zalloc((void**)&cblocks, sizeof(double) * nblk) ||
        !zalloc((void**)&cfN, sizeof(double) * nN) || !zalloc((void**)&cpN, sizeof(double) * nN) ||
        !zalloc((void**)&cstatus, sizeof(int)))
      return LRBMS_E_OOM;
    // members with fewer refinement steps than the largest are masked off
    // the later steps
    refine = 0;
    bool same = true;
    for (size_t i = 0; i < n; ++i) {
      refine = std::max(refine, model_of(models[i])->refine);
      same = same && model_of(models[i])->refine == model_of(models[0])->refine;
    }
    if (!same) {
      std::vector<int> h((size_t)kMaxRefine * n);
      for (int k = 0; k < kMaxRefine; ++k)
        for (size_t i = 0; i < n; ++i) h[k * n + i] = model_of(models[i])->refine > k ? 1 : 0;
      if (!zalloc((void**)&cref, sizeof(int) * h.size()) ||
          !hip_ok(hipMemcpy(cref, h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice),
                  "refine masks"))
        return LRBMS_E_OOM;
    }
    for (size_t i = 0; i < n; ++i) {
      Model* M = model_of(models[i]);
      own_blocks.push_back(M->d_blocks);
      own_fN.push_back(M->d_fN);
      M->d_blocks = cblocks + blk_base[i];
      M->d_fN = cfN + pn_base[i];
      if (!bufs[i].alloc(*M, cpN + pn_base[i])) return LRBMS_E_OOM;
    }
    return LRBMS_OK;
  }

  int capture(double* const* d_sat, uint8_t* const* d_flags) {
    drop_graph();
    if (!hip_ok(hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal), "begin capture"))
      return LRBMS_E_HIP;
    const int rc = enqueue(origin, d_sat, d_flags);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(origin, &g);
    if (rc != LRBMS_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (!hip_ok(e, "end capture")) return LRBMS_E_HIP;
    graph = g;
    if (!hip_ok(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "graph instantiate")) {
      drop_graph();
      return LRBMS_E_HIP;
    }
    const size_t n = models.size();
    cap_sat.assign(d_sat, d_sat + n);
    if (d_flags) cap_flags.assign(d_flags, d_flags + n);
    return LRBMS_OK;
  }

  bool same_pointers(double* const* d_sat, uint8_t* const* d_flags) const {
    const size_t n = models.size();
    if (!exec || cap_sat.size() != n) return false;
    if (!std::equal(cap_sat.begin(), cap_sat.end(), d_sat)) return false;
    if (!d_flags) return cap_flags.empty();
    return cap_flags.size() == n && std::equal(cap_flags.begin(), cap_flags.end(), d_flags);
  }
};

// ---- serving loop ---------------------------------------------------------------

struct Server {
  using Clock = std::chrono::steady_clock;
  struct Sim {
    lrbms_model* m = nullptr;
    double* sat = nullptr;
    long long footprint = 0;   // model bytes + step buffers
    bool attached = false, admitted = false, busy = false;
    StepBufs bufs;
  };
  struct Req {
    int sim;
    uint64_t id;
    Clock::time_point t0;
  };
  struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    int sim = -1;
    Req req{};
    int rc = LRBMS_OK;
  };
  struct Done {
    uint64_t id;
    double ms;
    int rc;
  };
  long long budget = 0, resident = 0;
  int mode = LRBMS_DIRECT;
  std::vector<Slot> slots;
  std::vector<Sim> sims;
  std::deque<int> waiting;     // attached, not yet admitted, in attach order
  std::deque<Req> pending;     // submitted, not yet dispatched, in submit order
  std::deque<Done> done;       // completed, not yet polled

  // Fused dispatch: the pending requests of distinct admitted simulations
  // (up to one per slot) form a wave: their assemblies on the slot streams,
  // then one reduced solve by the combined plan of all admitted simulations
  // with the wave's members active and the others masked off, then their
  // fluxes and transport on the slot streams.  One wave is on the device at
  // a time (the split backward products share partial storage per level);
  // requests that arrive meanwhile join the next wave.  The combined plan
  // and its storage are rebuilt whenever the admitted set changes.
  bool fused = false;
  bool cdirty = true;
  SolverPlan cplan;
  SolverDev cdev;
  double *cblocks = nullptr, *cfN = nullptr, *cpN = nullptr;
  int* cstatus = nullptr;
  int* cmask = nullptr;                 // device, one flag per member of the combined plan
  std::vector<int> cmembers;            // member index -> simulation
  std::vector<int> cmember_of;          // simulation -> member index (-1: not a member)
  std::vector<double*> own_blocks, own_fN;
  hipStream_t wst = nullptr;
  hipEvent_t wfork = nullptr, wfork2 = nullptr, wdone = nullptr;
  std::vector<hipEvent_t> wjoin, wjoin2;
  std::vector<Req> wave;                // the wave on the device

  // Give the members back their own block storage and drop the combined plan.
  void drop_combined() {
    for (size_t k = 0; k < cmembers.size(); ++k) {
      Sim& S = sims[cmembers[k]];
      if (!S.m) continue;
      Model* M = model_of(S.m);
      M->d_blocks = own_blocks[k];
      M->d_fN = own_fN[k];
      S.bufs.release();
    }
    own_blocks.clear();
    own_fN.clear();
    cmembers.clear();
    cmember_of.assign(sims.size(), -1);
    solver_free(cdev);
    cplan = SolverPlan{};
    for (void* q : {(void*)cblocks, (void*)cfN, (void*)cpN, (void*)cstatus, (void*)cmask})
      if (q) (void)hipFree(q);
    cblocks = cfN = cpN = nullptr;
    cstatus = cmask = nullptr;
    cdirty = true;
  }

  // Combined plan and storage of every admitted simulation (no wave on the
  // device); each member's A_N, f_N and p_N live in the combined storage.
  int build_combined() {
    drop_combined();
    std::vector<const SolverPlan*> plans;
    std::vector<long long> blk_base, pn_base;
    long long nblk = 0, nN = 0;
    for (size_t i = 0; i < sims.size(); ++i) {
      if (!sims[i].attached || !sims[i].admitted) continue;
      const Model& M = *model_of(sims[i].m);
      cmember_of[i] = (int)cmembers.size();
      cmembers.push_back((int)i);
      plans.push_back(&M.plan);
      blk_base.push_back(nblk);
      pn_base.push_back(nN);
      nblk += M.nblk;
      nN += M.N;
    }
    cdirty = false;
    if (cmembers.empty()) return LRBMS_OK;
    if (!combine_plans(plans, blk_base, pn_base, cplan) || !plan_in_bounds(cplan, nblk, nN))
      return (set_error("fused serving: plans cannot be combined"), LRBMS_E_ARG);
    if (!solver_upload(cplan, cdev)) return (set_error("fused serving: upload failed"), LRBMS_E_OOM);
    auto zalloc = [](void** q, size_t bytes) {
      return hip_ok(hipMalloc(q, std::max<size_t>(bytes, 8)), "hipMalloc") &&
             hip_ok(hipMemset(*q, 0, std::max<size_t>(bytes, 8)), "hipMemset");
    };
    if (!zalloc((void**)&cblocks, sizeof(double) * nblk) ||
        !zalloc((void**)&cfN, sizeof(double) * nN) || !zalloc((void**)&cpN, sizeof(double) * nN) ||
        !zalloc((void**)&cstatus, sizeof(int)) ||
        !zalloc((void**)&cmask, sizeof(int) * (1 + kMaxRefine) * cmembers.size()))
      return LRBMS_E_OOM;
    for (size_t k = 0; k < cmembers.size(); ++k) {
      Sim& S = sims[cmembers[k]];
      Model* M = model_of(S.m);
      own_blocks.push_back(M->d_blocks);
      own_fN.push_back(M->d_fN);
      M->d_blocks = cblocks + blk_base[k];
      M->d_fN = cfN + pn_base[k];
      if (!S.bufs.alloc(*M, cpN + pn_base[k])) return LRBMS_E_OOM;
    }
    return LRBMS_OK;
  }

  int launch_wave(const std::vector<Req>& reqs) {
    const int n = (int)reqs.size();
    MaskArgs ma{};
    ma.count = n;
    ma.total = (int)cmembers.size();
    int refine = 0;   // the wave's members' largest refinement steps
    for (int i = 0; i < n; ++i) {
      ma.ids[i] = cmember_of[reqs[i].sim];
      ma.refs[i] = model_of(sims[reqs[i].sim].m)->refine;
      refine = std::max(refine, ma.refs[i]);
    }
    hipLaunchKernelGGL(k_set_mask, dim3(1), dim3(256), 0, wst, cmask, ma);
    if (!hip_ok(hipGetLastError(), "mask") || !hip_ok(hipEventRecord(wfork, wst), "event"))
      return LRBMS_E_HIP;
    const int ns = (int)slots.size();
    int rc;
    for (int i = 0; i < n; ++i) {
      hipStream_t b = slots[i % ns].st;
      Sim& S = sims[reqs[i].sim];
      if (!hip_ok(hipStreamWaitEvent(b, wfork, 0), "wait")) return LRBMS_E_HIP;
      if ((rc = lrbms_online_assemble(S.m, S.sat, mode, b)) != LRBMS_OK) return rc;
      if (!hip_ok(hipEventRecord(wjoin[i], b), "event")) return LRBMS_E_HIP;
    }
    for (int i = 0; i < n; ++i)
      if (!hip_ok(hipStreamWaitEvent(wst, wjoin[i], 0), "wait")) return LRBMS_E_HIP;
    if (!hip_ok(solver_factor_solve(cplan, cdev, cblocks, cfN, cpN, cstatus, wst, refine, cmask,
                                    cmask + cmembers.size(), (int)cmembers.size()),
                "fused reduced solve") ||
        !hip_ok(hipEventRecord(wfork2, wst), "event"))
      return LRBMS_E_HIP;
    for (int i = 0; i < n; ++i) {
      hipStream_t b = slots[i % ns].st;
      Sim& S = sims[reqs[i].sim];
      if (!hip_ok(hipStreamWaitEvent(b, wfork2, 0), "wait")) return LRBMS_E_HIP;
      if ((rc = sim_after_solve(S.m, S.sat, nullptr, S.bufs, b)) != LRBMS_OK) return rc;
      if (!hip_ok(hipEventRecord(wjoin2[i], b), "event")) return LRBMS_E_HIP;
      model_of(S.m)->last_stream = wst;
      S.busy = true;
    }
    for (int i = 0; i < n; ++i)
      if (!hip_ok(hipStreamWaitEvent(wst, wjoin2[i], 0), "wait")) return LRBMS_E_HIP;
    if (!hip_ok(hipEventRecord(wdone, wst), "event")) return LRBMS_E_HIP;
    wave = reqs;
    return LRBMS_OK;
  }

  // Fused dispatch: retire the wave on the device, admit, rebuild the
  // combined plan if the admitted set changed, and launch the next wave.
  // Retire the wave on the device if it has finished; true when none is left.
  bool retire_wave() {
    if (!wave.empty()) {
      const hipError_t e = hipEventQuery(wdone);
      if (e == hipErrorNotReady) return false;
      int st = 0;
      if (e == hipSuccess &&
          !hip_ok(hipMemcpy(&st, cstatus, sizeof(int), hipMemcpyDeviceToHost), "status"))
        st = LRBMS_E_HIP;
      const auto now = Clock::now();
      for (const Req& r : wave) {
        const double ms = std::chrono::duration<double, std::milli>(now - r.t0).count();
        done.push_back(Done{r.id, ms, e == hipSuccess ? st : LRBMS_E_HIP});
        sims[r.sim].busy = false;
      }
      wave.clear();
    }
    return true;
  }

  int progress_fused() {
    if (!retire_wave()) return LRBMS_OK;
    const size_t before = waiting.size();
    int rc = admit();
    if (rc != LRBMS_OK) return rc;
    if (waiting.size() != before) cdirty = true;
    if (cdirty && (rc = build_combined()) != LRBMS_OK) return rc;
    std::vector<Req> reqs;
    std::vector<char> taken(sims.size(), 0);
    for (auto it = pending.begin(); it != pending.end() && reqs.size() < slots.size();) {
      Sim& S = sims[it->sim];
      if (!S.admitted || S.busy || taken[it->sim]) {
        ++it;
        continue;
      }
      taken[it->sim] = 1;
      reqs.push_back(*it);
      it = pending.erase(it);
    }
    if (reqs.empty()) return LRBMS_OK;
    return launch_wave(reqs);
  }

  ~Server() {
    for (auto& s : slots) {
      if (s.st) (void)hipStreamSynchronize(s.st);
    }
    if (wst) (void)hipStreamSynchronize(wst);
    if (fused) drop_combined();
    for (auto& s : sims) {
      if (s.m) {
        model_of(s.m)->last_stream = nullptr;
        model_of(s.m)->owner = nullptr;
      }
      s.bufs.release();
    }
    for (auto& s : slots) {
      if (s.done) (void)hipEventDestroy(s.done);
      if (s.st) (void)hipStreamDestroy(s.st);
    }
    for (hipEvent_t e : wjoin) (void)hipEventDestroy(e);
    for (hipEvent_t e : wjoin2) (void)hipEventDestroy(e);
    for (hipEvent_t e : {wfork, wfork2, wdone})
      if (e) (void)hipEventDestroy(e);
    if (wst) (void)hipStreamDestroy(wst);
  }

  // Admit waiting simulations, in attach order, while they fit the budget.
  int admit() {
    while (!waiting.empty()) {
      Sim& S = sims[waiting.front()];
      if (resident + S.footprint > budget) break;
      if (!fused && !S.bufs.alloc(*model_of(S.m))) return LRBMS_E_OOM;
      S.admitted = true;
      resident += S.footprint;
      waiting.pop_front();
    }
    return LRBMS_OK;
  }

  // Retire finished requests; then admit; then dispatch pending requests in
  // submit order onto free slots (one request per simulation in flight).
  int progress() {
    if (fused) return progress_fused();
    for (auto& s : slots) {
      if (s.sim < 0) continue;
      const hipError_t e = hipEventQuery(s.done);
      if (e == hipErrorNotReady) continue;
      const double ms =
          std::chrono::duration<double, std::milli>(Clock::now() - s.req.t0).count();
      done.push_back(Done{s.req.id, ms, e == hipSuccess ? s.rc : LRBMS_E_HIP});
      sims[s.sim].busy = false;
      s.sim = -1;
    }
    int rc = admit();
    if (rc != LRBMS_OK) return rc;
    size_t free_slots = 0;
    for (auto& s : slots) free_slots += s.sim < 0;
    for (auto it = pending.begin(); it != pending.end() && free_slots > 0;) {
      Sim& S = sims[it->sim];
      if (!S.admitted || S.busy) {
        ++it;
        continue;
      }
      Slot* slot = nullptr;
      for (auto& s : slots)
        if (s.sim < 0) {
          slot = &s;
          break;
        }
      slot->sim = it->sim;
      slot->req = *it;
      slot->rc = sim_step(S.m, mode, S.sat, nullptr, S.bufs, slot->st);
      if (!hip_ok(hipEventRecord(slot->done, slot->st), "request event")) slot->rc = LRBMS_E_HIP;
      model_of(S.m)->last_stream = slot->st;
      S.busy = true;
      --free_slots;
      it = pending.erase(it);
    }
    return LRBMS_OK;
  }

  bool idle() const {
    if (!wave.empty()) return false;
    for (auto& s : slots)
      if (s.sim >= 0) return false;
    return true;
  }
};

}  // namespace lrbms

using namespace lrbms;

extern "C" {

int lrbms_batch_create(lrbms_model* const* models, int32_t n, int32_t mode, int32_t flags,
                       lrbms_batch** out) {
  try {
    if (!out || !models || n < 1) return (set_error("invalid argument"), LRBMS_E_ARG);
    *out = nullptr;
    if (flags & ~(LRBMS_BATCH_GRAPH | LRBMS_BATCH_FUSED_SOLVE))
      return (set_error("unknown batch flags"), LRBMS_E_ARG);
    for (int i = 0; i < n; ++i) {
      if (!models[i]) return (set_error("NULL model"), LRBMS_E_ARG);
      if (model_of(models[i])->owner)
        return (set_error("a model belongs to a fused batch or a server already"), LRBMS_E_ARG);
      for (int j = 0; j < i; ++j)
        if (models[j] == models[i])
          return (set_error("a model appears twice in the batch"), LRBMS_E_ARG);
      if (!mode_ok(*model_of(models[i]), mode))
        return (set_error("assembly mode not available for every model"), LRBMS_E_ARG);
    }
    auto B = std::make_unique<Batch>();
    B->models.assign(models, models + n);
    for (int i = 0; i < n; ++i) model_of(models[i])->owner = B.get();
    B->mode = mode;
    B->use_graph = (flags & LRBMS_BATCH_GRAPH) != 0;
    B->fused = (flags & LRBMS_BATCH_FUSED_SOLVE) != 0;
    B->bufs.resize(n);
    int rc;
    if (B->fused) {
      if ((rc = B->setup_fused()) != LRBMS_OK) return rc;
    } else {
      for (int i = 0; i < n; ++i)
        if (!B->bufs[i].alloc(*model_of(models[i]))) return LRBMS_E_OOM;
    }
    const int nb = std::min(n, Batch::kBranches);
    B->branch.assign(nb, nullptr);
    B->join.assign(nb, nullptr);
    B->join2.assign(nb, nullptr);
    for (int b = 0; b < nb; ++b)
      if (!hip_ok(hipStreamCreateWithFlags(&B->branch[b], hipStreamNonBlocking), "stream") ||
          !hip_ok(hipEventCreateWithFlags(&B->join[b], hipEventDisableTiming), "event") ||
          !hip_ok(hipEventCreateWithFlags(&B->join2[b], hipEventDisableTiming), "event"))
        return LRBMS_E_HIP;
    if (!hip_ok(hipStreamCreateWithFlags(&B->origin, hipStreamNonBlocking), "stream") ||
        !hip_ok(hipEventCreateWithFlags(&B->fork, hipEventDisableTiming), "event") ||
        !hip_ok(hipEventCreateWithFlags(&B->fork2, hipEventDisableTiming), "event"))
      return LRBMS_E_HIP;
    *out = reinterpret_cast<lrbms_batch*>(B.release());
    return LRBMS_OK;
  } catch (const std::bad_alloc&) {
    return (set_error("host allocation failed"), LRBMS_E_OOM);
  }
}

int lrbms_batch_step(lrbms_batch* b, double* const* d_sat, uint8_t* const* d_flags, void* stream) {
  try {
    if (!b || !d_sat) return (set_error("NULL argument"), LRBMS_E_ARG);
    Batch* B = reinterpret_cast<Batch*>(b);
    const size_t n = B->models.size();
    for (size_t i = 0; i < n; ++i) {
      if (!d_sat[i]) return (set_error("NULL state"), LRBMS_E_ARG);
      if (model_of(B->models[i])->timer.on)
        return (set_error("kernel timing is on for a model of the batch"), LRBMS_E_STATE);
    }
    hipStream_t st = (hipStream_t)stream;
    int rc;
    if (B->use_graph) {
      if (!B->same_pointers(d_sat, d_flags) && (rc = B->capture(d_sat, d_flags)) != LRBMS_OK)
        return rc;
      if (!hip_ok(hipGraphLaunch(B->exec, st), "graph launch")) return LRBMS_E_HIP;
    } else if ((rc = B->enqueue(st, d_sat, d_flags)) != LRBMS_OK) {
      return rc;
    }
    for (lrbms_model* m : B->models) model_of(m)->last_stream = st;
    return LRBMS_OK;
  } catch (const std::bad_alloc&) {
    return (set_error("host allocation failed"), LRBMS_E_OOM);
  }
}

int lrbms_batch_buffers(lrbms_batch* b, int32_t i, double** d_pN, double** d_flux) {
  if (!b) return (set_error("NULL batch"), LRBMS_E_ARG);
  Batch* B = reinterpret_cast<Batch*>(b);
  if (i < 0 || i >= (int)B->models.size()) return (set_error("index out of range"), LRBMS_E_ARG);
  if (d_pN) *d_pN = B->bufs[i].pN;
  if (d_flux) *d_flux = B->bufs[i].flux;
  return LRBMS_OK;
}

int lrbms_batch_status(lrbms_batch* b) {
  if (!b) return (set_error("NULL batch"), LRBMS_E_ARG);
  Batch* B = reinterpret_cast<Batch*>(b);
  if (!hip_ok(hipDeviceSynchronize(), "synchronize")) return LRBMS_E_HIP;
  int st = 0;
  if (B->cstatus) {
    if (!hip_ok(hipMemcpy(&st, B->cstatus, sizeof(int), hipMemcpyDeviceToHost), "status"))
      return LRBMS_E_HIP;
    if (st && !hip_ok(hipMemset(B->cstatus, 0, sizeof(int)), "status")) return LRBMS_E_HIP;
  }
  for (lrbms_model* m : B->models) {
    const int ms = lrbms_model_status(m);
    if (!st) st = ms;
  }
  return st;
}

void lrbms_batch_destroy(lrbms_batch* b) { delete reinterpret_cast<Batch*>(b); }

int lrbms_server_create(int64_t hbm_budget, int32_t max_slots, int32_t mode, lrbms_server** out) {
  try {
    if (!out || hbm_budget <= 0 || max_slots < 1 || max_slots > 64)
      return (set_error("invalid argument"), LRBMS_E_ARG);
    *out = nullptr;
    if (mode != LRBMS_DIRECT && mode != LRBMS_DIRECT_FIT && mode != LRBMS_AFFINE)
      return (set_error("unknown assembly mode"), LRBMS_E_ARG);
    auto S = std::make_unique<Server>();
    S->budget = hbm_budget;
    S->mode = mode;
    S->slots.resize(max_slots);
    for (auto& s : S->slots)
      if (!hip_ok(hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking), "stream") ||
          !hip_ok(hipEventCreateWithFlags(&s.done, hipEventDisableTiming), "event"))
        return LRBMS_E_HIP;
    *out = reinterpret_cast<lrbms_server*>(S.release());
    return LRBMS_OK;
  } catch (const std::bad_alloc&) {
    return (set_error("host allocation failed"), LRBMS_E_OOM);
  }
}

int lrbms_server_attach(lrbms_server* s, lrbms_model* m, double* d_sat, int32_t* sim_id) {
  try {
    if (!s || !m || !d_sat || !sim_id) return (set_error("NULL argument"), LRBMS_E_ARG);
    Server* S = reinterpret_cast<Server*>(s);
    const Model& M = *model_of(m);
    if (M.owner) return (set_error("model belongs to a fused batch or a server already"), LRBMS_E_ARG);
    if (!mode_ok(M, S->mode)) return (set_error("assembly mode not available"), LRBMS_E_ARG);
    if (M.timer.on) return (set_error("kernel timing is on for this model"), LRBMS_E_STATE);
    Server::Sim x;
    x.m = m;
    x.sat = d_sat;
    x.footprint = M.dev_bytes + (long long)sizeof(double) *
                                    ((long long)std::max(M.N, 1) + std::max(M.g.nface, 1) +
                                     (long long)M.g.r * M.g.ncell);
    if (x.footprint > S->budget)
      return (set_error("simulation footprint exceeds the memory budget"), LRBMS_E_ADMIT);
    // the slot streams do not wait for the caller's streams: whatever wrote
    // the state must be finished
    if (!hip_ok(hipDeviceSynchronize(), "synchronize")) return LRBMS_E_HIP;
    x.attached = true;
    S->sims.push_back(x);
    model_of(m)->owner = S;
    *sim_id = (int32_t)S->sims.size() - 1;
    S->waiting.push_back(*sim_id);
    return S->progress();
  } catch (const std::bad_alloc&) {
    return (set_error("host allocation failed"), LRBMS_E_OOM);
  }
}

int lrbms_server_submit(lrbms_server* s, int32_t sim_id, uint64_t req_id) {
  try {
    if (!s) return (set_error("NULL server"), LRBMS_E_ARG);
    Server* S = reinterpret_cast<Server*>(s);
    if (sim_id < 0 || sim_id >= (int)S->sims.size() || !S->sims[sim_id].attached)
      return (set_error("unknown simulation"), LRBMS_E_ARG);
    S->pending.push_back(Server::Req{sim_id, req_id, Server::Clock::now()});
    return S->progress();
  } catch (const std::bad_alloc&) {
    return (set_error("host allocation failed"), LRBMS_E_OOM);
  }
}

int lrbms_server_poll(lrbms_server* s, uint64_t* req_ids, double* latency_ms, int32_t* status,
                      int32_t cap, int32_t* n_done) {
  try {
    if (!s || !n_done || cap < 0 || (cap > 0 && !req_ids))
      return (set_error("invalid argument"), LRBMS_E_ARG);
    *n_done = 0;
    Server* S = reinterpret_cast<Server*>(s);
    const int rc = S->progress();
    int k = 0;
    while (k < cap && !S->done.empty()) {
      const auto& d = S->done.front();
      req_ids[k] = d.id;
      if (latency_ms) latency_ms[k] = d.ms;
      if (status) status[k] = d.rc;
      S->done.pop_front();
      ++k;
    }
    *n_done = k;
    return rc;
  } catch (const std::bad_alloc&) {
    return (set_error("host allocation failed"), LRBMS_E_OOM);
  }
}

int lrbms_server_drain(lrbms_server* s) {
  try {
    if (!s) return (set_error("NULL server"), LRBMS_E_ARG);
    Server* S = reinterpret_cast<Server*>(s);
    for (;;) {
      int rc = S->progress();
      if (rc != LRBMS_OK) return rc;
      if (S->idle()) {
        if (S->pending.empty()) return LRBMS_OK;
        // nothing in flight and nothing dispatchable: the rest waits for memory
        return (set_error("pending requests wait for memory no detach will free"), LRBMS_E_ADMIT);
      }
      if (!S->wave.empty()) (void)hipEventSynchronize(S->wdone);
      for (auto& x : S->slots)
        if (x.sim >= 0) {
          (void)hipEventSynchronize(x.done);
          break;
        }
    }
  } catch (const std::bad_alloc&) {
    return (set_error("host allocation failed"), LRBMS_E_OOM);
  }
}

int lrbms_server_detach(lrbms_server* s, int32_t sim_id) {
  try {
    if (!s) return (set_error("NULL server"), LRBMS_E_ARG);
    Server* S = reinterpret_cast<Server*>(s);
    if (sim_id < 0 || sim_id >= (int)S->sims.size() || !S->sims[sim_id].attached)
      return (set_error("unknown simulation"), LRBMS_E_ARG);
    Server::Sim& x = S->sims[sim_id];
    for (const auto& r : S->pending)
      if (r.sim == sim_id) return (set_error("simulation has pending requests"), LRBMS_E_STATE);
    for (auto& sl : S->slots)
      if (sl.sim == sim_id) (void)hipEventSynchronize(sl.done);
    int rc = LRBMS_OK;
    if (S->fused) {
      // the wave on the device ends; the members get their own storage back
      // and the combined plan is rebuilt without this simulation
      if (!S->wave.empty()) (void)hipEventSynchronize(S->wdone);
      S->retire_wave();
      S->drop_combined();
    } else {
      rc = S->progress();
    }
    if (x.admitted) S->resident -= x.footprint;
    x.bufs.release();
    S->waiting.erase(std::remove(S->waiting.begin(), S->waiting.end(), sim_id), S->waiting.end());
    model_of(x.m)->last_stream = nullptr;
    model_of(x.m)->owner = nullptr;
    x = Server::Sim{};
    if (rc == LRBMS_OK) rc = S->progress();
    return rc;
  } catch (const std::bad_alloc&) {
    return (set_error("host allocation failed"), LRBMS_E_OOM);
  }
}

int lrbms_server_info(const lrbms_server* s, lrbms_server_info_t* info) {
  if (!s || !info) return (set_error("NULL argument"), LRBMS_E_ARG);
  const Server* S = reinterpret_cast<const Server*>(s);
  info->resident_bytes = S->resident;
  info->budget_bytes = S->budget;
  info->n_pending = (int32_t)S->pending.size();
  int busy = 0, adm = 0, wait = (int)S->waiting.size();
  for (auto& sl : S->slots) busy += sl.sim >= 0;
  busy += (int)S->wave.size();
  for (auto& x : S->sims) adm += x.attached && x.admitted;
  info->n_in_flight = busy;
  info->n_admitted = adm;
  info->n_waiting = wait;
  return LRBMS_OK;
}

int lrbms_server_set_fused(lrbms_server* s, int32_t on) {
  try {
    if (!s) return (set_error("NULL server"), LRBMS_E_ARG);
    Server* S = reinterpret_cast<Server*>(s);
    if (!S->sims.empty()) return (set_error("set_fused before the first attach"), LRBMS_E_STATE);
    S->fused = on != 0;
    if (S->fused && !S->wst) {
      if (!hip_ok(hipStreamCreateWithFlags(&S->wst, hipStreamNonBlocking), "stream") ||
          !hip_ok(hipEventCreateWithFlags(&S->wfork, hipEventDisableTiming), "event") ||
          !hip_ok(hipEventCreateWithFlags(&S->wfork2, hipEventDisableTiming), "event") ||
          !hip_ok(hipEventCreateWithFlags(&S->wdone, hipEventDisableTiming), "event"))
        return LRBMS_E_HIP;
      S->wjoin.assign(S->slots.size(), nullptr);
      S->wjoin2.assign(S->slots.size(), nullptr);
      for (size_t i = 0; i < S->slots.size(); ++i)
        if (!hip_ok(hipEventCreateWithFlags(&S->wjoin[i], hipEventDisableTiming), "event") ||
            !hip_ok(hipEventCreateWithFlags(&S->wjoin2[i], hipEventDisableTiming), "event"))
          return LRBMS_E_HIP;
    }
    return LRBMS_OK;
  } catch (const std::bad_alloc&) {
    return (set_error("host allocation failed"), LRBMS_E_OOM);
  }
}

void lrbms_server_destroy(lrbms_server* s) { delete reinterpret_cast<Server*>(s); }

}  // extern "C"
