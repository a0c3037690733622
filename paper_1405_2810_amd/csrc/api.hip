// C ABI of the LRBMS online step (include/lrbms.h): model creation, the four
// online calls, inspection helpers and error reporting.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <memory>
#include <string>
#include <vector>

#include "common.h"
#include "ktimer.h"
#include "model.h"

namespace lrbms {

static thread_local std::string g_last_error;

// ---- kernel timer ---------------------------------------------------------------
thread_local KernelTimer* t_timer = nullptr;

const char* kernel_kind_name(int kind) {
  static const char* const names[KK_COUNT] = {
      "k_moments",        "k_lsq",          "k_affine_sum",     "k_asm_box",
      "k_reduce_box",     "k_asm_iface",    "k_front_asm",      "k_front_factor0",
      "k_front_step",     "k_front_backward", "k_front_update", "k_front_bw_gemv",
      "k_reconstruct",    "k_flux",           "k_transport",    "k_limiter",
      "k_residual",       "k_front_forward",  "k_front_fw_gemv",  "k_front_schur"};
  return (kind >= 0 && kind < KK_COUNT) ? names[kind] : "?";
}

hipEvent_t KernelTimer::take() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    failed = true;
    return nullptr;
  }
  return e;
}

void KernelTimer::reset() {
  for (auto& r : recs) {
    if (r.a) pool.push_back(r.a);
    if (r.b) pool.push_back(r.b);
  }
  recs.clear();
  for (int k = 0; k < KK_COUNT; ++k) n[k] = unit_n[k] = 0, ms[k] = flops[k] = bytes[k] = 0.0;
  failed = false;
}

bool KernelTimer::drain() {
  bool ok = !failed;
  for (auto& r : recs) {
    float t = 0.0f;
    if (r.a && r.b && hipEventSynchronize(r.b) == hipSuccess &&
        hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
      n[r.kind] += 1;
      ms[r.kind] += t;
      if (r.flops < 0.0) {
        unit_n[r.kind] += 1;
      } else {
        flops[r.kind] += r.flops;
        bytes[r.kind] += r.bytes;
      }
    } else {
      ok = false;
    }
    if (r.a) pool.push_back(r.a);
    if (r.b) pool.push_back(r.b);
  }
  recs.clear();
  return ok;
}

KernelTimer::~KernelTimer() {
  for (auto& r : recs) {
    if (r.a) (void)hipEventDestroy(r.a);
    if (r.b) (void)hipEventDestroy(r.b);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

void ktimer_begin(int kind, hipStream_t st) {
  KernelTimer* t = t_timer;
  if (!t) return;
  t->open = t->take();
  t->open_kind = kind;
  if (t->open && hipEventRecord(t->open, st) != hipSuccess) t->failed = true;
}

void ktimer_end(double flops, double bytes, hipStream_t st) {
  KernelTimer* t = t_timer;
  if (!t || t->open_kind < 0) return;
  hipEvent_t b = t->take();
  if (b && hipEventRecord(b, st) != hipSuccess) t->failed = true;
  t->recs.push_back(KernelTimer::Rec{t->open_kind, t->open, b, flops, bytes});
  t->open = nullptr;
  t->open_kind = -1;
}

void set_error(const std::string& msg) { g_last_error = msg; }

bool hip_ok(hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return false;
}

__global__ void k_fill_u8(uint8_t* p, int n, uint8_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
static int check_problem(const lrbms_problem* p) {
  if (!p) return (set_error("problem is NULL"), LRBMS_E_ARG);
  if (p->dim != 2 && p->dim != 3) return (set_error("dim must be 2 or 3"), LRBMS_E_ARG);
  for (int a = 0; a < 3; ++a) {
    const int na = (a < p->dim) ? p->n[a] : 1;
    const int ca = (a < p->dim) ? p->nc[a] : 1;
    if (a < p->dim && (p->n[a] < 1 || p->len[a] <= 0.0))
      return (set_error("grid sizes and lengths must be positive"), LRBMS_E_ARG);
    if (a >= p->dim && (p->n[a] != 1 || p->nc[a] != 1))
      return (set_error("n[2] and nc[2] must be 1 in 2D"), LRBMS_E_ARG);
    if (ca < 1 || ca > na) return (set_error("invalid number of coarse boxes"), LRBMS_E_ARG);
    if (a < p->dim) {
      if (!p->cuts[a]) return (set_error("cuts missing"), LRBMS_E_ARG);
      if (p->cuts[a][0] != 0 || p->cuts[a][ca] != na)
        return (set_error("cuts must start at 0 and end at n"), LRBMS_E_ARG);
      for (int i = 0; i < ca; ++i)
        if (p->cuts[a][i + 1] <= p->cuts[a][i])
          return (set_error("cuts must be strictly increasing"), LRBMS_E_ARG);
    }
  }
  if (!p->perm || !p->poro || !p->bc_type || !p->bc_val || !p->bc_sat || !p->bc_sval || !p->q1 ||
      !p->q2)
    return (set_error("problem array missing"), LRBMS_E_ARG);
  if (!(p->visc_w > 0.0) || !(p->visc_o > 0.0)) return (set_error("viscosities must be > 0"), LRBMS_E_ARG);
  if (p->relperm != 0 && p->relperm != 1) return (set_error("relperm must be 0 or 1"), LRBMS_E_ARG);
  if (p->weights != 0 && p->weights != 1) return (set_error("weights must be 0 or 1"), LRBMS_E_ARG);
  if (!(p->dt > 0.0)) return (set_error("dt must be > 0"), LRBMS_E_ARG);
  if (!(p->penalty_c > 0.0)) return (set_error("penalty_c must be > 0"), LRBMS_E_ARG);
  if (!std::isfinite(p->dens_w) || !std::isfinite(p->dens_o))
    return (set_error("densities must be finite"), LRBMS_E_ARG);
  for (int a = 0; a < 3; ++a)
    if (p->grav[a] != 0.0)
      return (set_error("gravity is not supported: grav must be zero"), LRBMS_E_ARG);
  return LRBMS_OK;
}

template <typename T>
static bool dev_copy(T** d, const T* h, size_t n, long long& bytes) {
  if (!hip_ok(hipMalloc(d, std::max<size_t>(n, 1) * sizeof(T)), "hipMalloc")) return false;
  bytes += (long long)(n * sizeof(T));
  if (n && h) return hip_ok(hipMemcpy(*d, h, n * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
  return true;
}

template <typename T>
static bool dev_zero(T** d, size_t n, long long& bytes) {
  if (!hip_ok(hipMalloc(d, std::max<size_t>(n, 1) * sizeof(T)), "hipMalloc")) return false;
  bytes += (long long)(n * sizeof(T));
  return hip_ok(hipMemset(*d, 0, std::max<size_t>(n, 1) * sizeof(T)), "hipMemset");
}

Model::~Model() {
  auto f = [](void* p) {
    if (p) (void)hipFree(p);
  };
  f(d_subs);
  f(d_ifaces);
  f(d_perm);
  f(d_poro);
  f(d_q1);
  f(d_q2);
  f(d_bc_val);
  f(d_bc_sval);
  f(d_bc_type);
  f(d_bc_sat);
  f(d_phi);
  f(d_tr);
  f(d_mom);
  f(d_blocks);
  f(d_fN);
  f(d_prof);
  f(d_gchol);
  f(d_theta);
  f(d_partial);
  f(d_c);
  f(d_bq);
  f(d_e);
  f(d_dq);
  f(d_tiles);
  f(d_scratch_sat);
  f(d_scratch_ph);
  f(d_status);
  solver_free(sdev);
  assemble_free(asm_layout);
}

// Geometry and physics constants of a checked problem (host side only, no
// allocation); nc receives the coarse box counts.
static void fill_geom(Geom& g, int nc[3], const lrbms_problem* p) {
  std::memset(&g, 0, sizeof(g));
  g.dim = p->dim;
  g.r = p->dim + 1;
  for (int a = 0; a < 3; ++a) {
    g.n[a] = a < p->dim ? p->n[a] : 1;
    g.h[a] = a < p->dim ? p->len[a] / p->n[a] : 1.0;
    nc[a] = a < p->dim ? p->nc[a] : 1;
  }
  g.ncell = g.n[0] * g.n[1] * g.n[2];
  g.vol = 1.0;
  for (int a = 0; a < p->dim; ++a) g.vol *= g.h[a];
  g.isv = 1.0 / std::sqrt(g.vol);
  double he2 = 0.0;
  for (int a = 0; a < p->dim; ++a) he2 += g.h[a] * g.h[a];
  g.he = std::sqrt(he2);
  int off = 0;
  for (int a = 0; a < 3; ++a) {
    int cnt = 0;
    if (a < p->dim) {
      int e[3] = {g.n[0], g.n[1], g.n[2]};
      e[a] += 1;
      cnt = e[0] * e[1] * e[2];
    }
    g.nfa[a] = cnt;
    g.foff[a] = off;
    off += cnt;
    double area = 1.0, hf2 = 0.0;
    for (int b = 0; b < p->dim; ++b)
      if (b != a) {
        area *= g.h[b];
        hf2 += g.h[b] * g.h[b];
      }
    g.area[a] = area;
    g.hf[a] = p->dim > 1 ? std::sqrt(hf2) : 1.0;
  }
  g.nface = off;
  g.visc_w = p->visc_w;
  g.visc_o = p->visc_o;
  g.ivw = 1.0 / p->visc_w;
  g.ivo = 1.0 / p->visc_o;
  g.relperm = p->relperm;
  g.cw = p->corey_w;
  g.co = p->corey_o;
  g.pen = p->penalty_c / std::max(p->visc_w, p->visc_o);
  g.weights = p->weights;
  g.sat_pen = p->sat_penalty_scale;
  g.limiter = p->limiter;
  g.dt = p->dt;
  {
    // largest slope of the fractional flow, sampled on [0, 1] (central
    // differences of the mobilities of the problem's law)
    auto fw = [&](double s) {
      s = std::min(1.0, std::max(0.0, s));
      double krw, kro;
      if (p->relperm == 0) {
        krw = s;
        kro = 1.0 - s;
      } else {
        krw = std::pow(s, p->corey_w);
        kro = std::pow(1.0 - s, p->corey_o);
      }
      const double lw = krw / p->visc_w, lo = kro / p->visc_o;
      return lw / (lw + lo);
    };
    const int n = 4096;
    double mx = 0.0;
    for (int i = 0; i < n; ++i) {
      const double a = (double)i / n, b = (double)(i + 1) / n;
      mx = std::max(mx, std::fabs(fw(b) - fw(a)) * n);
    }
    g.cfl_coef = g.dt * mx;
  }
}

// Fill geometry, boxes and interfaces (host side only).
static int setup_layout(Model& M, const lrbms_problem* p, const int32_t* sizes) {
  Geom& g = M.g;
  fill_geom(g, M.nc, p);
  // boxes
  M.subs.clear();
  long long phi_off = 0, blk = 0;
  int pn = 0;
  for (int ez = 0; ez < M.nc[2]; ++ez)
    for (int ey = 0; ey < M.nc[1]; ++ey)
      for (int ex = 0; ex < M.nc[0]; ++ex) {
        Sub s;
        const int e[3] = {ex, ey, ez};
        s.nE = 1;
        for (int a = 0; a < 3; ++a) {
          s.lo[a] = a < p->dim ? p->cuts[a][e[a]] : 0;
          s.hi[a] = a < p->dim ? p->cuts[a][e[a] + 1] : 1;
          s.nE *= s.hi[a] - s.lo[a];
        }
        const int id = (int)M.subs.size();
        s.NE = sizes ? sizes[id] : 0;
        s.phi_off = phi_off;
        s.pn_off = pn;
        s.blk_off = blk;
        phi_off += (long long)s.NE * g.r * s.nE;
        pn += s.NE;
        blk += (long long)s.NE * s.NE;
        M.subs.push_back(s);
      }
  M.n_sub = (int)M.subs.size();
  M.N = pn;
  M.phi_len = phi_off;
  M.ifaces.clear();
  long long tr = 0;
  for (int a = 0; a < p->dim; ++a)
    for (int ez = 0; ez < M.nc[2]; ++ez)
      for (int ey = 0; ey < M.nc[1]; ++ey)
        for (int ex = 0; ex < M.nc[0]; ++ex) {
          int e[3] = {ex, ey, ez};
          if (e[a] + 1 >= M.nc[a]) continue;
          const int lo = ex + M.nc[0] * (ey + M.nc[1] * ez);
          e[a] += 1;
          const int hi = e[0] + M.nc[0] * (e[1] + M.nc[1] * e[2]);
          Iface I;
          I.axis = a;
          I.lo = lo;
          I.hi = hi;
          I.nf = 1;
          for (int b = 0; b < 3; ++b)
            if (b != a) I.nf *= M.subs[lo].hi[b] - M.subs[lo].lo[b];
          I.blk_off = blk;
          blk += (long long)M.subs[lo].NE * M.subs[hi].NE;
          I.tr_off = tr;
          tr += (long long)(M.subs[lo].NE + M.subs[hi].NE) * (p->dim + 1) * I.nf;
          M.ifaces.push_back(I);
        }
  M.n_iface = (int)M.ifaces.size();
  M.tr_len = tr;
  M.nblk = blk;
  M.max_ne = 0;
  for (auto& s : M.subs) M.max_ne = std::max(M.max_ne, s.NE);
  return LRBMS_OK;
}

static int upload_problem(Model& M, const lrbms_problem* p) {
  Geom& g = M.g;
  long long& b = M.dev_bytes;
  const size_t nc = g.ncell, nf = g.nface;
  if (!dev_copy(&M.d_perm, p->perm, nc, b) || !dev_copy(&M.d_poro, p->poro, nc, b) ||
      !dev_copy(&M.d_q1, p->q1, nc, b) || !dev_copy(&M.d_q2, p->q2, nc, b) ||
      !dev_copy(&M.d_bc_val, p->bc_val, nf, b) || !dev_copy(&M.d_bc_sval, p->bc_sval, nf, b) ||
      !dev_copy(&M.d_bc_type, p->bc_type, nf, b) || !dev_copy(&M.d_bc_sat, p->bc_sat, nf, b))
    return LRBMS_E_OOM;
  g.perm = M.d_perm;
  g.poro = M.d_poro;
  g.q1 = M.d_q1;
  g.q2 = M.d_q2;
  g.bc_val = M.d_bc_val;
  g.bc_sval = M.d_bc_sval;
  g.bc_type = M.d_bc_type;
  g.bc_sat = M.d_bc_sat;
  if (!dev_zero(&M.d_mom, (size_t)n_moments(g.dim) * nc, b)) return LRBMS_E_OOM;
  if (!dev_zero(&M.d_scratch_sat, (size_t)g.r * nc, b)) return LRBMS_E_OOM;
  if (!dev_zero(&M.d_scratch_ph, (size_t)g.r * nc, b)) return LRBMS_E_OOM;
  if (!dev_zero(&M.d_status, 2, b)) return LRBMS_E_OOM;
  g.status = M.d_status;
  return LRBMS_OK;
}

// Cholesky of a small SPD matrix (row-major, lower factor in place). false if not SPD.
static bool small_cholesky(std::vector<double>& A, int n) {
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    A[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = s / d;
    }
    for (int k = j + 1; k < n; ++k) A[j * n + k] = 0.0;
  }
  return true;
}

// Algorithmic flops and bytes (8 B per double) of one launch of each kernel
// kind whose work does not depend on the launch: the inputs it must read and
// the outputs it must write once, and the arithmetic of what it computes.
static void set_unit_figures(Model& M) {
  const Geom& g = M.g;
  const double n = g.ncell, r = g.r, d = g.dim, nm = n_moments(g.dim), nf = g.nface;
  double phi = 0.0, blk = 0.0, asm_fl = 0.0;
  for (const Sub& S : M.subs) {
    const double rows = r * S.nE, NE = S.NE;
    phi += rows * NE;
    blk += NE * NE;
    asm_fl += 2.0 * rows * NE * (NE + 1) + 2.0 * (2 * d + 1) * r * rows * NE;
  }
  double if_bytes = 0.0, if_fl = 0.0;
  for (const Iface& I : M.ifaces) {
    const double NL = M.subs[I.lo].NE, NH = M.subs[I.hi].NE;
    if_bytes += r * I.nf * (NL + NH) + 2.0 * I.nf * nm + NL * NH;
    if_fl += 2.0 * r * I.nf * NL * NH + 4.0 * r * r * I.nf * NH;
  }
  double red = 0.0;
  for (const Sub& S : M.subs) red += (double)S.NE * (S.NE + 1);
  const int cols = assemble_cols(M.max_ne);
  for (int k = 0; k < KK_COUNT; ++k) M.unit_flops[k] = M.unit_bytes[k] = 0.0;
  M.unit_bytes[KK_MOMENTS] = 8.0 * n * (r + nm + 1);
  M.unit_bytes[KK_ASM_DIAG] = 8.0 * (phi + nm * n + n + blk + M.N);
  M.unit_flops[KK_ASM_DIAG] = asm_fl;
  M.unit_bytes[KK_ASM_REDUCE] = 8.0 * ((double)M.asm_layout.n_chunks * cols * cols + red);
  M.unit_flops[KK_ASM_REDUCE] = (double)M.asm_layout.n_chunks * cols * cols;
  M.unit_bytes[KK_ASM_IFACE] = 8.0 * if_bytes;
  M.unit_flops[KK_ASM_IFACE] = if_fl;
  M.unit_bytes[KK_LSQ] = 8.0 * (r * n + (double)M.nprof * r * n);
  M.unit_flops[KK_LSQ] = 2.0 * M.nprof * r * n;
  M.unit_bytes[KK_RECONSTRUCT] = 8.0 * (phi + M.N + r * n);
  M.unit_flops[KK_RECONSTRUCT] = 2.0 * phi;
  M.unit_bytes[KK_FLUX] = 8.0 * (2.0 * r * n + n + nf);
  M.unit_bytes[KK_TRANSPORT] = 8.0 * (2.0 * r * n + nf + 2.0 * n);
  M.unit_bytes[KK_LIMITER] = 8.0 * (2.0 * r * n + nf) + n;
}

int model_finish(Model& M, const double* basis, int nprof, const double* profiles, bool lsq,
                 double* d_basis) {
  Geom& g = M.g;
  long long& b = M.dev_bytes;
  if (d_basis) {
    M.d_phi = d_basis;
    b += M.phi_len * (long long)sizeof(double);
  }
  if (!dev_copy(&M.d_subs, M.subs.data(), M.subs.size(), b)) return LRBMS_E_OOM;
  if (!dev_copy(&M.d_ifaces, M.ifaces.data(), M.ifaces.size(), b)) return LRBMS_E_OOM;
  if (!d_basis && !dev_copy(&M.d_phi, basis, (size_t)M.phi_len, b)) return LRBMS_E_OOM;
  if (!dev_zero(&M.d_tr, (size_t)M.tr_len, b)) return LRBMS_E_OOM;
  if (!hip_ok(launch_face_traces(g, M.d_subs, M.d_ifaces, M.n_iface, M.d_phi, M.d_tr, 0), "face traces") ||
      !hip_ok(hipStreamSynchronize(0), "face traces"))
    return LRBMS_E_HIP;
  if (!dev_zero(&M.d_blocks, (size_t)M.nblk, b) || !dev_zero(&M.d_fN, (size_t)M.N, b))
    return LRBMS_E_OOM;
  // reconstruction tiles (box, first cell)
  std::vector<int> tiles;
  for (int s = 0; s < M.n_sub; ++s)
    for (int c0 = 0; c0 < M.subs[s].nE; c0 += 256) {
      tiles.push_back(s);
      tiles.push_back(c0);
    }
  M.n_tiles = (int)tiles.size() / 2;
  if (!dev_copy(&M.d_tiles, tiles.data(), tiles.size(), b)) return LRBMS_E_OOM;
  if (!hip_ok(assemble_prepare(g, M.subs, M.max_ne, M.asm_variant, M.asm_layout, b),
              "assembly layout"))
    return LRBMS_E_OOM;
  // solver
  // leaf size of the nested dissection: the one whose launch sequence is
  // shortest.  Every level costs an assembly, a first-tile factorization and
  // a backward launch, every further panel a step launch, each of roughly the
  // same latency (about 64 us per level and 28.5 us per step on gfx950 at
  // these sizes); leaves above 8 boxes lengthen the leaf fronts' steps.
  double best = 1e300;
  for (int leaf : {2, 4, 8}) {
    SolverPlan P;
    if (!build_solver_plan(g.dim, M.nc, M.subs, M.ifaces, leaf, P) ||
        !plan_in_bounds(P, M.nblk, M.N))
      continue;
    double cost = 0.0;
    for (int h = 0; h < P.nlevels; ++h) cost += 64.0 + 28.5 * (double)P.step_items[h].size();
    if (cost < best) {
      best = cost;
      M.leaf_max = leaf;
      M.plan = std::move(P);
    }
  }
  if (best == 1e300) {
    set_error("solver symbolic analysis failed");
    return LRBMS_E_ARG;
  }
  if (!solver_upload(M.plan, M.sdev)) {
    set_error("solver allocation failed");
    return LRBMS_E_OOM;
  }
  b += M.sdev.bytes;
  // profiles and the affine terms of Sec. 4.4
  M.nprof = nprof;
  if (nprof > 0) {
    const size_t L = (size_t)g.r * g.ncell;
    std::vector<double> G((size_t)nprof * nprof);
    for (int i = 0; i < nprof; ++i)
      for (int j = 0; j < nprof; ++j) {
        double s = 0.0;
        for (size_t k = 0; k < L; ++k) s += profiles[i * L + k] * profiles[j * L + k];
        G[i * nprof + j] = s;
      }
    if (lsq && !small_cholesky(G, nprof)) {
      set_error("profile Gram matrix is not positive definite (profiles must be independent)");
      return LRBMS_E_ARG;
    }
    M.lsq_ok = lsq;
    if (!dev_copy(&M.d_prof, profiles, (size_t)nprof * L, b) ||
        !dev_copy(&M.d_gchol, G.data(), G.size(), b) || !dev_zero(&M.d_theta, (size_t)nprof, b))
      return LRBMS_E_OOM;
    M.lsq_blocks = lsq_blocks(g.ncell);
    if (!dev_zero(&M.d_partial, (size_t)M.lsq_blocks * nprof, b)) return LRBMS_E_OOM;
    if (!dev_zero(&M.d_c, (size_t)M.nblk, b) || !dev_zero(&M.d_bq, (size_t)M.nblk * nprof, b) ||
        !dev_zero(&M.d_e, (size_t)M.N, b) || !dev_zero(&M.d_dq, (size_t)M.N * nprof, b))
      return LRBMS_E_OOM;
    hipStream_t st = 0;
    // c: penalty part (gamma-free), e: gamma-free right-hand side
    if (!hip_ok(launch_assemble(M.asm_layout, g, M.d_subs, M.n_sub, M.max_ne, M.d_ifaces, M.n_iface, M.d_phi, M.d_tr,
                                M.d_mom, PART_PEN | PART_RHS_CONST, M.d_c, M.d_e, st),
                "assemble c, e"))
      return LRBMS_E_HIP;
    for (int q = 0; q < nprof; ++q) {
      if (!hip_ok(launch_moments(g, M.d_prof + (size_t)q * L, GAMMA_FIELD, nullptr, 0, 0, M.d_mom,
                                 st),
                  "profile moments"))
        return LRBMS_E_HIP;
      if (!hip_ok(launch_assemble(M.asm_layout, g, M.d_subs, M.n_sub, M.max_ne, M.d_ifaces, M.n_iface, M.d_phi, M.d_tr,
                                  M.d_mom, PART_GAMMA | PART_RHS_GAMMA, M.d_bq + (size_t)q * M.nblk,
                                  M.d_dq + (size_t)q * M.N, st),
                  "assemble b_q, d_q"))
        return LRBMS_E_HIP;
    }
    if (!hip_ok(hipStreamSynchronize(st), "affine terms")) return LRBMS_E_HIP;
  }
  set_unit_figures(M);
  return LRBMS_OK;
}

int model_create_impl(const lrbms_problem* p, const int32_t* sizes, const double* basis,
                      int nprof, const double* profiles, lrbms_model** out) {
  if (!out) return (set_error("out is NULL"), LRBMS_E_ARG);
  *out = nullptr;
  int rc = check_problem(p);
  if (rc) return rc;
  if (!sizes || !basis) return (set_error("basis missing"), LRBMS_E_ARG);
  if (nprof < 0 || nprof > kMaxProfiles || (nprof > 0 && !profiles))
    return (set_error("invalid profiles"), LRBMS_E_ARG);
  std::unique_ptr<Model> M(new Model());
  const int nsub = p->nc[0] * p->nc[1] * (p->dim == 3 ? p->nc[2] : 1);
  for (int s = 0; s < nsub; ++s)
    if (sizes[s] < 1 || sizes[s] > 63)
      return (set_error("local basis sizes must be in 1..63"), LRBMS_E_ARG);
  setup_layout(*M, p, sizes);
  if ((rc = upload_problem(*M, p))) return rc;
  if ((rc = model_finish(*M, basis, nprof, profiles, true))) return rc;
  *out = reinterpret_cast<lrbms_model*>(M.release());
  return LRBMS_OK;
}

// A model whose bases are the device array d_basis (model layout, sizes per
// box), which the model takes over; freed here when the creation fails.
static int model_create_dev(const lrbms_problem* p, const std::vector<int>& sizes,
                            double* d_basis, int nprof, const double* profiles,
                            lrbms_model** out) {
  std::unique_ptr<Model> M(new Model());
  setup_layout(*M, p, sizes.data());
  int rc = upload_problem(*M, p);
  if (rc) {
    (void)hipFree(d_basis);
    return rc;
  }
  if ((rc = model_finish(*M, nullptr, nprof, profiles, true, d_basis))) return rc;
  *out = reinterpret_cast<lrbms_model*>(M.release());
  return LRBMS_OK;
}

// Device array owned by a host scope.
struct DevArray {
  double* p = nullptr;
  bool alloc(size_t n) {
    if (p) (void)hipFree(p);
    p = nullptr;
    return hip_ok(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(double)), "hipMalloc");
  }
  ~DevArray() {
    if (p) (void)hipFree(p);
  }
};

// The model's device status words (the caller has synchronized): the first
// error, else the warning, else 0; with a message for either.
static int read_status(Model& M) {
  int s[2] = {0, 0};
  if (!hip_ok(hipMemcpy(s, M.d_status, sizeof(s), hipMemcpyDeviceToHost), "status"))
    return LRBMS_E_HIP;
  if (s[0] == LRBMS_E_NOT_SPD)
    set_error("device reported a non-positive pivot in the reduced Cholesky");
  else if (s[0] == LRBMS_E_NONFINITE)
    set_error("device reported a non-finite value (reduced residual, flux or saturation)");
  else if (s[0])
    set_error("device reported an error");
  else if (s[1] == LRBMS_W_CFL)
    set_error("warning: a transport step exceeded the CFL bound of its fluxes");
  return s[0] ? s[0] : s[1];
}

// With checks on, an online call waits for its own work and returns what
// the device reported.
static int checked(Model& M, hipStream_t st) {
  if (!M.checks) return LRBMS_OK;
  if (!hip_ok(hipStreamSynchronize(st), "synchronize")) return LRBMS_E_HIP;
  return read_status(M);
}

// Read and clear the device status word of a scratch model.
static int take_status(Model& M) {
  int st = 0;
  if (!hip_ok(hipMemcpy(&st, M.d_status, sizeof(int), hipMemcpyDeviceToHost), "status")) return LRBMS_E_HIP;
  if (st && !hip_ok(hipMemset(M.d_status, 0, sizeof(int)), "status")) return LRBMS_E_HIP;
  return st;
}

struct FineSolverHandle {
  FineSolver* s = nullptr;
  ~FineSolverHandle() {
    if (s) fine_solver_destroy(s);
  }
};

static int fine_solve_checked(Model& M, FineSolver* S, const double* d_field, int kind,
                              double rtol, int maxit, double* d_p, int* iters, double* relres,
                              bool warm = false) {
  int rc = fine_solver_solve(S, M.d_mom, d_field, kind, rtol, maxit, warm, d_p, M.d_status, iters,
                             relres);
  const int st = take_status(M);
  if (st < 0 && (rc == LRBMS_OK || rc == LRBMS_E_STATE)) rc = st;
  switch (rc) {
    case LRBMS_OK: break;
    case LRBMS_E_STATE: set_error("fine pressure: CG did not reach rtol within maxit"); break;
    case LRBMS_E_NOT_SPD: set_error("fine pressure: singular cell block, non-positive curvature or indefinite preconditioner"); break;
    case LRBMS_E_NONFINITE: set_error("fine pressure: non-finite residual"); break;
    case LRBMS_E_OOM: set_error("fine pressure: device allocation failed"); break;
    default: set_error("fine pressure: HIP error"); break;
  }
  return rc;
}

static int tof_checked(Model& M, const double* d_flux, double tol, int maxit, double* d_tau,
                       int* sweeps) {
  int rc = tof_solve(M.g, d_flux, tol, maxit, d_tau, M.d_status, sweeps);
  const int st = take_status(M);
  if (st < 0 && (rc == LRBMS_OK || rc == LRBMS_E_STATE)) rc = st;
  switch (rc) {
    case LRBMS_OK: break;
    case LRBMS_E_STATE: set_error("time of flight: sweeps did not converge within maxit"); break;
    case LRBMS_E_NOT_SPD: set_error("time of flight: singular cell block (a cell without flux)"); break;
    case LRBMS_E_NONFINITE: set_error("time of flight: non-finite values"); break;
    case LRBMS_E_OOM: set_error("time of flight: device allocation failed"); break;
    default: set_error("time of flight: HIP error"); break;
  }
  return rc;
}

static double host_total_mobility(const lrbms_problem* p, double s) {
  const double sc = std::min(std::max(s, 0.0), 1.0);
  const double krw = p->relperm == 0 ? sc : std::pow(sc, p->corey_w);
  const double kro = p->relperm == 0 ? 1.0 - sc : std::pow(1.0 - sc, p->corey_o);
  return krw / p->visc_w + kro / p->visc_o;
}

// Mobility profiles of Alg. 2 step 1c as P1 fields (mean coefficient only):
// lambda(0) for q = 1, lambda(1) for q = M, and in between lambda(0) on the
// cells whose mean time of flight exceeds (q-1) T/(M-2), lambda(1) elsewhere.
static void mobility_profiles(const Geom& g, const lrbms_problem* p, const std::vector<double>& tau,
                              int nq, double T, std::vector<double>& prof) {
  const size_t L = (size_t)g.r * g.ncell;
  const double sv = std::sqrt(g.vol);
  const double l0 = host_total_mobility(p, 0.0), l1 = host_total_mobility(p, 1.0);
  prof.assign((size_t)nq * L, 0.0);
  for (int q = 1; q <= nq; ++q) {
    double* f = prof.data() + (size_t)(q - 1) * L;
    const double thr = (double)(q - 1) * T / (double)(nq - 2);
    for (int c = 0; c < g.ncell; ++c) {
      double v;
      if (q == 1) v = l0;
      else if (q == nq) v = l1;
      else v = (tau[c] / sv > thr) ? l0 : l1;
      f[c] = v * sv;
    }
  }
}

// Indices of the profiles that are linearly independent of the ones before
// them: two-pass Gram-Schmidt in q order, dropped when the remaining norm is
// <= 1e-12 of the profile's own norm.
static std::vector<int> independent_profiles(const std::vector<double>& prof, int nq, size_t L) {
  std::vector<int> keep;
  std::vector<std::vector<double>> Q;
  for (int q = 0; q < nq; ++q) {
    std::vector<double> w(prof.begin() + (size_t)q * L, prof.begin() + (size_t)(q + 1) * L);
    double nv = 0.0;
    for (double x : w) nv += x * x;
    nv = std::sqrt(nv);
    if (nv == 0.0) continue;
    for (int pass = 0; pass < 2; ++pass)
      for (auto& b : Q) {
        double d = 0.0;
        for (size_t i = 0; i < L; ++i) d += b[i] * w[i];
        for (size_t i = 0; i < L; ++i) w[i] -= d * b[i];
      }
    double nw = 0.0;
    for (double x : w) nw += x * x;
    nw = std::sqrt(nw);
    if (nw <= 1e-12 * nv) continue;
    for (auto& x : w) x /= nw;
    Q.push_back(std::move(w));
    keep.push_back(q);
  }
  return keep;
}

// State of the offline stage: the problem on the device, the fine solver, the
// profiles and the solver figures.
struct OfflineCtx {
  Model tmp;
  FineSolverHandle fs;
  DevArray field;
  std::vector<double> prof;   // [M][r*ncell]
  lrbms_offline_report R{};
  size_t L = 0;
  void note(int it, double rr) {
    R.n_solves += 1;
    R.pcg_iters_max = std::max(R.pcg_iters_max, it);
    R.pcg_iters_total += it;
    R.pcg_relres_max = std::max(R.pcg_relres_max, rr);
  }
};

static int check_offline_opts(const lrbms_offline_opts* o, const double* mu, bool need_cap) {
  if (!o || !mu) return (set_error("options or training parameters missing"), LRBMS_E_ARG);
  if (o->M < 3 || o->M > kMaxProfiles) return (set_error("M must be in 3..64"), LRBMS_E_ARG);
  if (o->n_train < 1) return (set_error("n_train must be >= 1"), LRBMS_E_ARG);
  if (need_cap && (o->ne_cap < 1 || o->ne_cap > 63))
    return (set_error("ne_cap must be in 1..63"), LRBMS_E_ARG);
  if (!(o->horizon > 0.0)) return (set_error("horizon must be > 0"), LRBMS_E_ARG);
  if (!(o->pcg_rtol > 0.0) || o->pcg_maxit < 1 || !(o->tof_tol >= 0.0) || o->tof_maxit < 1)
    return (set_error("invalid solver tolerances or iteration limits"), LRBMS_E_ARG);
  for (long long i = 0; i < (long long)o->n_train * o->M; ++i)
    if (!std::isfinite(mu[i])) return (set_error("training parameters must be finite"), LRBMS_E_ARG);
  return LRBMS_OK;
}

// Alg. 2 step 1: pressure and velocity at s0, time of flight, profiles.
static int offline_profiles(const lrbms_problem* p, const lrbms_offline_opts* o, OfflineCtx& C) {
  int rc;
  setup_layout(C.tmp, p, nullptr);
  if ((rc = upload_problem(C.tmp, p))) return rc;
  const Geom& g = C.tmp.g;
  C.L = (size_t)g.r * g.ncell;
  DevArray flux, tau;
  if (!flux.alloc(g.nface) || !tau.alloc(C.L) || !C.field.alloc(C.L)) return LRBMS_E_OOM;
  if (!(C.fs.s = fine_solver_create(g)))
    return (set_error("fine solver allocation failed"), LRBMS_E_OOM);
  int it = 0;
  double rr = 0.0;
  const double* s0 = o->d_s0 ? o->d_s0 : C.tmp.d_scratch_sat;   // zeros unless given
  rc = fine_solve_checked(C.tmp, C.fs.s, s0, GAMMA_SAT, o->pcg_rtol, o->pcg_maxit,
                          C.tmp.d_scratch_ph, &it, &rr);
  C.note(it, rr);
  if (rc) return rc;
  if (!hip_ok(launch_flux(g, C.tmp.d_scratch_ph, s0, flux.p, 0), "initial flux")) return LRBMS_E_HIP;
  if ((rc = tof_checked(C.tmp, flux.p, o->tof_tol, o->tof_maxit, tau.p, &C.R.tof_sweeps))) return rc;
  std::vector<double> h_tau(C.L);
  if (!hip_ok(hipMemcpy(h_tau.data(), tau.p, C.L * sizeof(double), hipMemcpyDeviceToHost), "tau"))
    return LRBMS_E_HIP;
  mobility_profiles(g, p, h_tau, o->M, o->horizon, C.prof);
  return LRBMS_OK;
}

// The field sum_q w_q Lambda^q, uploaded into C.field.
static int combine_profiles(OfflineCtx& C, int nq, const double* w) {
  std::vector<double> gam(C.L, 0.0);
  for (int q = 0; q < nq; ++q) {
    const double* f = C.prof.data() + (size_t)q * C.L;
    for (size_t k = 0; k < C.L; ++k) gam[k] += w[q] * f[k];
  }
  return hip_ok(hipMemcpy(C.field.p, gam.data(), C.L * sizeof(double), hipMemcpyHostToDevice),
                "gamma")
             ? LRBMS_OK
             : LRBMS_E_HIP;
}

static std::vector<double> kept_profiles(const OfflineCtx& C, int nq, bool keep) {
  std::vector<double> kept;
  if (keep)
    for (int q : independent_profiles(C.prof, nq, C.L))
      kept.insert(kept.end(), C.prof.begin() + (size_t)q * C.L,
                  C.prof.begin() + (size_t)(q + 1) * C.L);
  return kept;
}

static int build_offline_impl(const lrbms_problem* p, const lrbms_offline_opts* o,
                              const double* mu, lrbms_model** out, lrbms_offline_report* rep) {
  if (!out) return (set_error("out is NULL"), LRBMS_E_ARG);
  *out = nullptr;
  int rc = check_problem(p);
  if (rc) return rc;
  if ((rc = check_offline_opts(o, mu, true))) return rc;
  OfflineCtx C;
  if ((rc = offline_profiles(p, o, C))) return rc;
  const size_t L = C.L;
  // snapshots at gamma = sum_q mu_q Lambda^q, kept on the device
  DevArray snaps;
  if (!snaps.alloc((size_t)o->n_train * L)) return LRBMS_E_OOM;
  for (int i = 0; i < o->n_train; ++i) {
    if ((rc = combine_profiles(C, o->M, mu + (size_t)i * o->M))) return rc;
    int it = 0;
    double rr = 0.0;
    rc = fine_solve_checked(C.tmp, C.fs.s, C.field.p, GAMMA_FIELD, o->pcg_rtol, o->pcg_maxit,
                            snaps.p + (size_t)i * L, &it, &rr);
    C.note(it, rr);
    if (rc) return rc;
  }
  // Alg. 2 step 2e: local bases on the device
  std::vector<int> sizes;
  double* d_basis = nullptr;
  long long len = 0;
  if ((rc = local_bases_device(C.tmp.g, C.tmp.subs, snaps.p, o->n_train, o->ne_cap,
                               o->unit_functions != 0, o->basis_method, o->pca_eps, sizes,
                               &d_basis, len)))
    return rc;
  const std::vector<double> kept = kept_profiles(C, o->M, o->keep_profiles != 0);
  C.R.n_profiles_kept = (int)(kept.size() / L);
  if (rep) *rep = C.R;
  return model_create_dev(p, sizes, d_basis, C.R.n_profiles_kept,
                          kept.empty() ? nullptr : kept.data(), out);
}

// Alg. 2 step 2 (the greedy basis extension) with the true energy-norm error
// of Sec. 6.  The fine snapshots of the whole training set are computed
// first and stay on the device, and so do the local bases, which grow there
// (Gram-Schmidt of the worst parameter's snapshot in every box).  Every
// iteration builds the reduced model of the current bases (affine terms),
// solves the reduced systems of all training parameters (theta = mu) as one
// fused solve per chunk of up to 64 parameters (the model's plan repeated,
// members side by side), reconstructs their pressures and measures every
// |p_H - p_h| in the energy norm of b_h(., .; sum_q mubar_q Lambda^q) with
// one read-back per chunk.
static int build_greedy_impl(const lrbms_problem* p, const lrbms_offline_opts* o,
                             const double* mu, int n_max, double tol, const double* mu_bar,
                             lrbms_model** out, int32_t* chosen, double* errors, int max_iter,
                             int32_t* n_iter, lrbms_offline_report* rep) {
  if (!out) return (set_error("out is NULL"), LRBMS_E_ARG);
  *out = nullptr;
  int rc = check_problem(p);
  if (rc) return rc;
  if ((rc = check_offline_opts(o, mu, false))) return rc;
  if (n_max < 1 || !(tol >= 0.0)) return (set_error("n_max must be >= 1 and tol >= 0"), LRBMS_E_ARG);
  if ((chosen || errors) && max_iter < 1) return (set_error("max_iter must be >= 1"), LRBMS_E_ARG);
  OfflineCtx C;
  if ((rc = offline_profiles(p, o, C))) return rc;
  const size_t L = C.L;
  const int nt = o->n_train, nq = o->M;
  // every training snapshot, resident on the device
  DevArray snaps, theta;
  if (!snaps.alloc((size_t)nt * L) || !theta.alloc((size_t)nt * nq)) return LRBMS_E_OOM;
  if (!hip_ok(hipMemcpy(theta.p, mu, (size_t)nt * nq * sizeof(double), hipMemcpyHostToDevice),
              "training parameters"))
    return LRBMS_E_HIP;
  for (int i = 0; i < nt; ++i) {
    if ((rc = combine_profiles(C, nq, mu + (size_t)i * nq))) return rc;
    int it = 0;
    double rr = 0.0;
    rc = fine_solve_checked(C.tmp, C.fs.s, C.field.p, GAMMA_FIELD, o->pcg_rtol, o->pcg_maxit,
                            snaps.p + (size_t)i * L, &it, &rr);
    C.note(it, rr);
    if (rc) return rc;
  }
  // the energy norm of the error measure
  std::vector<double> wbar(nq, 1.0 / nq);
  if (mu_bar)
    for (int q = 0; q < nq; ++q) wbar[q] = mu_bar[q];
  if ((rc = combine_profiles(C, nq, wbar.data()))) return rc;
  if ((rc = fine_energy_setup(C.fs.s, C.tmp.d_mom, C.field.p))) return rc;
  // local bases, empty at the start, grown on the device
  const Model& T = C.tmp;
  DeviceBases GB;
  if ((rc = device_bases_init(T.g, T.subs, 63, GB))) return rc;
  std::vector<double> err(nt);
  int iters = 0;
  constexpr int kChunk = 64;
  while (true) {
    int total = 0;
    for (int sz : GB.sizes) total += sz;
    if (total == 0) {
      if ((rc = fine_energy_diff_batch(C.fs.s, snaps.p, (long long)L, nullptr, 0, nt, err.data())))
        return rc;
    } else {
      for (int sz : GB.sizes)
        if (sz < 1 || sz > 63)
          return (set_error("greedy: a local basis is empty or above 63 functions"), LRBMS_E_ARG);
      // the reduced model of the current bases with every profile (theta = mu)
      double* d_basis = nullptr;
      long long len = 0;
      if ((rc = device_bases_compact(T.g, T.subs, GB, &d_basis, len))) return rc;
      std::unique_ptr<Model> RM(new Model());
      setup_layout(*RM, p, GB.sizes.data());
      if ((rc = upload_problem(*RM, p))) {
        (void)hipFree(d_basis);
        return rc;
      }
      if ((rc = model_finish(*RM, nullptr, nq, C.prof.data(), false, d_basis))) return rc;
      // the training parameters' reduced solves, up to kChunk side by side
      const int cn = std::min(nt, kChunk);
      std::vector<const SolverPlan*> plans(cn, &RM->plan);
      std::vector<long long> blk_base(cn), pn_base(cn);
      for (int i = 0; i < cn; ++i) {
        blk_base[i] = (long long)i * RM->nblk;
        pn_base[i] = (long long)i * RM->N;
      }
      SolverPlan CP;
      if (!combine_plans(plans, blk_base, pn_base, CP) ||
          !plan_in_bounds(CP, (long long)cn * RM->nblk, (long long)cn * RM->N))
        return (set_error("greedy: reduced solves cannot be combined"), LRBMS_E_ARG);
      SolverDev CD;
      struct Free {
        SolverDev& d;
        ~Free() { solver_free(d); }
      } free_cd{CD};
      if (!solver_upload(CP, CD)) return (set_error("greedy: solver allocation failed"), LRBMS_E_OOM);
      DevArray blocks, fN, pN, ph, mask;
      if (!blocks.alloc((size_t)cn * RM->nblk) || !fN.alloc((size_t)cn * RM->N) ||
          !pN.alloc((size_t)cn * RM->N) || !ph.alloc((size_t)cn * L) || !mask.alloc(cn))
        return LRBMS_E_OOM;
      for (int c0 = 0; c0 < nt; c0 += cn) {
        const int cc = std::min(cn, nt - c0);
        for (int i = 0; i < cc; ++i) {
          const double* th = theta.p + (size_t)(c0 + i) * nq;
          if (!hip_ok(launch_affine_sum(RM->d_c, RM->d_bq, RM->nblk, th, nq,
                                        blocks.p + (size_t)i * RM->nblk, 0),
                      "affine sum") ||
              !hip_ok(launch_affine_sum(RM->d_e, RM->d_dq, RM->N, th, nq,
                                        fN.p + (size_t)i * RM->N, 0),
                      "affine sum"))
            return LRBMS_E_HIP;
        }
        // a short last chunk masks the members it does not use
        const int* active = nullptr;
        if (cc < cn) {
          std::vector<int> m(cn, 0);
          for (int i = 0; i < cc; ++i) m[i] = 1;
          if (!hip_ok(hipMemcpy(mask.p, m.data(), cn * sizeof(int), hipMemcpyHostToDevice), "mask"))
            return LRBMS_E_HIP;
          active = reinterpret_cast<const int*>(mask.p);
        }
        if (!hip_ok(solver_factor_solve(CP, CD, blocks.p, fN.p, pN.p, RM->d_status, 0,
                                        RM->refine, active),
                    "reduced solves"))
          return LRBMS_E_HIP;
        for (int i = 0; i < cc; ++i)
          if (!hip_ok(launch_reconstruct(RM->g, RM->d_subs, RM->n_sub, RM->d_tiles, RM->n_tiles,
                                         RM->d_phi, pN.p + (size_t)i * RM->N,
                                         ph.p + (size_t)i * L, 0),
                      "reconstruct"))
            return LRBMS_E_HIP;
        if ((rc = fine_energy_diff_batch(C.fs.s, ph.p, (long long)L, snaps.p + (size_t)c0 * L,
                                         (long long)L, cc, err.data() + c0)))
          return rc;
      }
      int st = 0;
      if (!hip_ok(hipMemcpy(&st, RM->d_status, sizeof(int), hipMemcpyDeviceToHost), "status"))
        return LRBMS_E_HIP;
      if (st) return (set_error("greedy: reduced matrix not positive definite"), st);
    }
    int k = 0;
    for (int i = 0; i < nt; ++i) {
      err[i] = std::sqrt(std::max(err[i], 0.0));
      if (err[i] > err[k]) k = i;
    }
    if (errors && iters < max_iter) errors[iters] = err[k];
    ++iters;
    if (err[k] <= tol || total >= n_max || iters > 63) break;
    if (chosen && iters - 1 < max_iter) chosen[iters - 1] = k;
    bool grew = false;
    if ((rc = device_bases_extend(T.g, GB, snaps.p + (size_t)k * L, grew))) return rc;
    if (!grew) break;
  }
  if (n_iter) *n_iter = iters;
  for (int sz : GB.sizes)
    if (sz < 1) return (set_error("greedy: a box received an empty local basis"), LRBMS_E_ARG);
  double* d_basis = nullptr;
  long long len = 0;
  if ((rc = device_bases_compact(T.g, T.subs, GB, &d_basis, len))) return rc;
  const std::vector<double> kept = kept_profiles(C, nq, o->keep_profiles != 0);
  C.R.n_profiles_kept = (int)(kept.size() / L);
  if (rep) *rep = C.R;
  return model_create_dev(p, GB.sizes, d_basis, C.R.n_profiles_kept,
                          kept.empty() ? nullptr : kept.data(), out);
}

// Transport step (Def. saturationDG) and the limiter (eq. limiterMain) on a
// model's geometry; the limiter reads the unlimited state from scratch.
static int transport_impl(Model& M, const double* d_sat, const double* d_flux, double* d_sat_out,
                          uint8_t* d_flags, hipStream_t st) {
  const Geom& g = M.g;
  if (g.limiter) {
    if (!hip_ok(launch_transport(g, d_sat, d_flux, M.d_scratch_sat, st), "transport") ||
        !hip_ok(launch_limiter(g, M.d_scratch_sat, d_flux, d_sat_out, d_flags, st), "limiter"))
      return LRBMS_E_HIP;
  } else {
    if (!hip_ok(launch_transport(g, d_sat, d_flux, d_sat_out, st), "transport")) return LRBMS_E_HIP;
    if (d_flags) {
      hipLaunchKernelGGL(k_fill_u8, dim3((g.ncell + 255) / 256), dim3(256), 0, st, d_flags,
                         g.ncell, (uint8_t)0);
      if (!hip_ok(hipGetLastError(), "fill flags")) return LRBMS_E_HIP;
    }
  }
  return LRBMS_OK;
}

// Fine reference (Alg. 1): the problem on the device and a fine solver.
struct FineModel {
  Model M;
  FineSolverHandle S;
};

}  // namespace lrbms

namespace lrbms {

// Fixed work memory of the entry points that allocate nothing (128 MiB per
// device, held until the process ends).  Host code never uses the array's
// name as an address: scratch_ptr() looks its device address up once per
// device (hipGetSymbolAddress, with that device current) and keeps it.
constexpr size_t kScratchDoubles = (128ull << 20) / sizeof(double);
static __device__ __align__(256) double scratch[kScratchDoubles];
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[64] = {};

static double* scratch_ptr() {
  int dev = 0;
  if (!hip_ok(hipGetDevice(&dev), "hipGetDevice")) return nullptr;
  if (dev < 0 || dev >= 64) return (set_error("device index out of range"), nullptr);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (!hip_ok(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress")) return nullptr;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}

}  // namespace lrbms

using namespace lrbms;

static Model* M_(lrbms_model* m) { return reinterpret_cast<Model*>(m); }
static const Model* M_(const lrbms_model* m) { return reinterpret_cast<const Model*>(m); }

extern "C" {

const char* lrbms_last_error(void) { return g_last_error.c_str(); }

int lrbms_model_create(const lrbms_problem* prob, const int32_t* basis_sizes, const double* basis,
                       int32_t n_profiles, const double* profiles, lrbms_model** out) {
  try {
    return model_create_impl(prob, basis_sizes, basis, n_profiles, profiles, out);
  } catch (const std::exception& e) {
    set_error(e.what());
    return LRBMS_E_OOM;
  }
}

int lrbms_model_create_from_snapshots(const lrbms_problem* prob, int32_t n_snap,
                                      const double* snapshots, int32_t ne_cap,
                                      int32_t unit_functions, int32_t basis_method,
                                      double pca_eps, int32_t n_profiles,
                                      const double* profiles, lrbms_model** out) {
  try {
    if (!out) return (set_error("out is NULL"), LRBMS_E_ARG);
    *out = nullptr;
    int rc = check_problem(prob);
    if (rc) return rc;
    if (n_snap < 0 || (n_snap > 0 && !snapshots) || ne_cap < 1 || ne_cap > 63)
      return (set_error("invalid snapshots or cap"), LRBMS_E_ARG);
    if (n_profiles < 0 || n_profiles > kMaxProfiles || (n_profiles > 0 && !profiles))
      return (set_error("invalid profiles"), LRBMS_E_ARG);
    Model tmp;
    setup_layout(tmp, prob, nullptr);
    // the snapshots go to the device once; Alg. 2 step 2e runs there
    const size_t L = (size_t)tmp.g.r * tmp.g.ncell;
    DevArray snaps;
    if (!snaps.alloc((size_t)n_snap * L)) return LRBMS_E_OOM;
    if (n_snap > 0 && !hip_ok(hipMemcpy(snaps.p, snapshots, (size_t)n_snap * L * sizeof(double),
                                        hipMemcpyHostToDevice),
                              "snapshots"))
      return LRBMS_E_HIP;
    std::vector<int> sizes;
    double* d_basis = nullptr;
    long long len = 0;
    if ((rc = local_bases_device(tmp.g, tmp.subs, snaps.p, n_snap, ne_cap, unit_functions != 0,
                                 basis_method, pca_eps, sizes, &d_basis, len)))
      return rc;
    return model_create_dev(prob, sizes, d_basis, n_profiles, profiles, out);
  } catch (const std::exception& e) {
    set_error(e.what());
    return LRBMS_E_OOM;
  }
}

int lrbms_model_get_info(const lrbms_model* m, lrbms_model_info* info) {
  if (!m || !info) return (set_error("NULL argument"), LRBMS_E_ARG);
  const Model* M = M_(m);
  info->dim = M->g.dim;
  info->r = M->g.r;
  info->ncell = M->g.ncell;
  info->nface = M->g.nface;
  info->n_sub = M->n_sub;
  info->n_iface = M->n_iface;
  info->N = M->N;
  info->n_profiles = M->nprof;
  info->n_block_entries = M->nblk;
  info->device_bytes = M->dev_bytes;
  return LRBMS_OK;
}

int lrbms_model_export_basis(const lrbms_model* m, int32_t* sizes, double* basis) {
  if (!m || !sizes || !basis) return (set_error("NULL argument"), LRBMS_E_ARG);
  const Model* M = M_(m);
  for (int s = 0; s < M->n_sub; ++s) sizes[s] = M->subs[s].NE;
  return hip_ok(hipMemcpy(basis, M->d_phi, M->phi_len * sizeof(double), hipMemcpyDeviceToHost),
                "export basis")
             ? LRBMS_OK
             : LRBMS_E_HIP;
}

int lrbms_model_interfaces(const lrbms_model* m, int32_t* axis, int32_t* lo, int32_t* hi) {
  if (!m || !axis || !lo || !hi) return (set_error("NULL argument"), LRBMS_E_ARG);
  const Model* M = M_(m);
  for (int t = 0; t < M->n_iface; ++t) {
    axis[t] = M->ifaces[t].axis;
    lo[t] = M->ifaces[t].lo;
    hi[t] = M->ifaces[t].hi;
  }
  return LRBMS_OK;
}

int lrbms_online_assemble(lrbms_model* m, const double* d_sat, int32_t mode, void* stream) {
  if (!m || !d_sat) return (set_error("NULL argument"), LRBMS_E_ARG);
  Model* M = M_(m);
  TimerScope timing(&M->timer);
  hipStream_t st = (hipStream_t)stream;
  const Geom& g = M->g;
  if (mode != LRBMS_DIRECT && mode != LRBMS_DIRECT_FIT && mode != LRBMS_AFFINE)
    return (set_error("unknown assembly mode"), LRBMS_E_ARG);
  if (mode != LRBMS_DIRECT && M->nprof == 0)
    return (set_error("this mode needs mobility profiles"), LRBMS_E_STATE);
  if (mode != LRBMS_DIRECT && !M->lsq_ok)
    return (set_error("this model's profiles admit no least-squares fit"), LRBMS_E_STATE);
  const int all = PART_GAMMA | PART_PEN | PART_RHS_CONST | PART_RHS_GAMMA;
  if (mode == LRBMS_DIRECT) {
    if (!hip_ok(launch_moments(g, d_sat, GAMMA_SAT, nullptr, 0, 0, M->d_mom, st), "moments"))
      return LRBMS_E_HIP;
  } else {
    if (!hip_ok(launch_lsq(g, d_sat, M->d_prof, M->nprof, M->d_gchol, M->d_partial, M->lsq_blocks,
                           M->d_theta, st),
                "least squares"))
      return LRBMS_E_HIP;
    if (mode == LRBMS_DIRECT_FIT) {
      if (!hip_ok(launch_moments(g, M->d_prof, GAMMA_COMBO, M->d_theta, M->nprof,
                                 (long long)g.r * g.ncell, M->d_mom, st),
                  "moments"))
        return LRBMS_E_HIP;
    }
  }
  if (mode == LRBMS_AFFINE) {
    if (!hip_ok(launch_affine_sum(M->d_c, M->d_bq, M->nblk, M->d_theta, M->nprof, M->d_blocks, st),
                "affine sum") ||
        !hip_ok(launch_affine_sum(M->d_e, M->d_dq, M->N, M->d_theta, M->nprof, M->d_fN, st),
                "affine sum"))
      return LRBMS_E_HIP;
  } else {
    if (!hip_ok(launch_assemble(M->asm_layout, g, M->d_subs, M->n_sub, M->max_ne, M->d_ifaces, M->n_iface,
                                M->d_phi, M->d_tr, M->d_mom, all, M->d_blocks, M->d_fN, st),
                "assemble"))
      return LRBMS_E_HIP;
  }
  M->assembled = true;
  M->last_stream = st;
  return checked(*M, st);
}

int lrbms_online_solve(lrbms_model* m, double* d_pN, void* stream) {
  if (!m || !d_pN) return (set_error("NULL argument"), LRBMS_E_ARG);
  Model* M = M_(m);
  TimerScope timing(&M->timer);
  if (!M->assembled) return (set_error("online_solve called before online_assemble"), LRBMS_E_STATE);
  hipStream_t st = (hipStream_t)stream;
  if (!hip_ok(solver_factor_solve(M->plan, M->sdev, M->d_blocks, M->d_fN, d_pN, M->d_status, st,
                                  M->refine),
              "reduced solve"))
    return LRBMS_E_HIP;
  M->last_stream = st;
  return checked(*M, st);
}

int lrbms_model_set_refinement(lrbms_model* m, int32_t steps) {
  if (!m) return (set_error("NULL argument"), LRBMS_E_ARG);
  if (steps < 0 || steps > kMaxRefine)
    return (set_error("refinement steps must be in 0..4"), LRBMS_E_ARG);
  Model* M = M_(m);
  if (M->owner) return (set_error("model belongs to a batch or server"), LRBMS_E_STATE);
  M->refine = steps;
  return LRBMS_OK;
}

// Rebuild the box assembly's work layout for variant v (0 or 1).
static int set_asm_variant(Model& M, int v) {
  if (v == M.asm_variant && M.asm_layout.chunks) return LRBMS_OK;
  const long long cols = assemble_cols(M.max_ne);
  M.dev_bytes -= (long long)M.asm_layout.n_chunks * cols * cols * (long long)sizeof(double) +
                 (2LL * M.asm_layout.n_chunks + M.n_sub + 1) * (long long)sizeof(int);
  assemble_free(M.asm_layout);
  M.asm_variant = v;
  if (!hip_ok(assemble_prepare(M.g, M.subs, M.max_ne, v, M.asm_layout, M.dev_bytes),
              "assembly layout"))
    return LRBMS_E_OOM;
  set_unit_figures(M);
  return LRBMS_OK;
}

int lrbms_model_set_assembly_variant(lrbms_model* m, int32_t variant) {
  try {
    if (!m) return (set_error("NULL argument"), LRBMS_E_ARG);
    if (variant < 0 || variant > 1) return (set_error("assembly variant must be 0 or 1"), LRBMS_E_ARG);
    Model* M = M_(m);
    if (M->owner) return (set_error("model belongs to a batch or server"), LRBMS_E_STATE);
    if (!hip_ok(hipStreamSynchronize(M->last_stream), "synchronize")) return LRBMS_E_HIP;
    return set_asm_variant(*M, variant);
  } catch (const std::bad_alloc&) {
    return (set_error("host allocation failed"), LRBMS_E_OOM);
  }
}

int lrbms_model_set_solver_shapes(lrbms_model* m, int32_t leaf_max, int32_t split_min,
                                  int32_t bw_split_min) {
  try {
    if (!m) return (set_error("NULL argument"), LRBMS_E_ARG);
    if (leaf_max < 1 || leaf_max > 64 || split_min < 0 || bw_split_min < 0)
      return (set_error("solver shapes out of range"), LRBMS_E_ARG);
    Model* M = M_(m);
    if (M->owner) return (set_error("model belongs to a batch or server"), LRBMS_E_STATE);
    const int split = split_min == 0 ? (1 << 30) : split_min;
    const long long bw = bw_split_min == 0 ? (1LL << 62) : (long long)bw_split_min;
    SolverPlan P;
    if (!build_solver_plan(M->g.dim, M->nc, M->subs, M->ifaces, leaf_max, P, split, bw) ||
        !plan_in_bounds(P, M->nblk, M->N))
      return (set_error("solver plan of these shapes does not fit"), LRBMS_E_ARG);
    if (!hip_ok(hipStreamSynchronize(M->last_stream), "synchronize")) return LRBMS_E_HIP;
    SolverDev D;
    if (!solver_upload(P, D)) {
      solver_free(D);
      return (set_error("solver allocation failed"), LRBMS_E_OOM);
    }
    M->dev_bytes += D.bytes - M->sdev.bytes;
    solver_free(M->sdev);
    M->sdev = D;
    M->plan = std::move(P);
    M->leaf_max = leaf_max;
    M->split_min = split;
    M->bw_min = bw;
    return LRBMS_OK;
  } catch (const std::bad_alloc&) {
    return (set_error("host allocation failed"), LRBMS_E_OOM);
  }
}

int lrbms_reconstruct_flux(lrbms_model* m, const double* d_pN, const double* d_sat,
                           double* d_flux, double* d_ph, void* stream) {
  if (!m || !d_pN || !d_sat || !d_flux) return (set_error("NULL argument"), LRBMS_E_ARG);
  Model* M = M_(m);
  TimerScope timing(&M->timer);
  hipStream_t st = (hipStream_t)stream;
  double* ph = d_ph ? d_ph : M->d_scratch_ph;
  if (!hip_ok(launch_reconstruct(M->g, M->d_subs, M->n_sub, M->d_tiles, M->n_tiles, M->d_phi, d_pN,
                                 ph, st),
              "reconstruct") ||
      !hip_ok(launch_flux(M->g, ph, d_sat, d_flux, st), "flux"))
    return LRBMS_E_HIP;
  M->last_stream = st;
  return checked(*M, st);
}

int lrbms_transport_step(lrbms_model* m, const double* d_sat, const double* d_flux,
                         double* d_sat_out, uint8_t* d_flags, void* stream) {
  if (!m || !d_sat || !d_flux || !d_sat_out) return (set_error("NULL argument"), LRBMS_E_ARG);
  if (d_sat_out == d_sat) return (set_error("d_sat_out must not alias d_sat"), LRBMS_E_ARG);
  Model* M = M_(m);
  TimerScope timing(&M->timer);
  const int rc = transport_impl(*M, d_sat, d_flux, d_sat_out, d_flags, (hipStream_t)stream);
  if (rc != LRBMS_OK) return rc;
  M->last_stream = (hipStream_t)stream;
  return checked(*M, (hipStream_t)stream);
}

int lrbms_fine_create(const lrbms_problem* prob, lrbms_fine** out) {
  try {
    if (!out) return (set_error("out is NULL"), LRBMS_E_ARG);
    *out = nullptr;
    int rc = check_problem(prob);
    if (rc) return rc;
    std::unique_ptr<FineModel> F(new FineModel());
    setup_layout(F->M, prob, nullptr);
    if ((rc = upload_problem(F->M, prob))) return rc;
    if (!(F->S.s = fine_solver_create(F->M.g)))
      return (set_error("fine solver allocation failed"), LRBMS_E_OOM);
    *out = reinterpret_cast<lrbms_fine*>(F.release());
    return LRBMS_OK;
  } catch (const std::exception& e) {
    set_error(e.what());
    return LRBMS_E_OOM;
  }
}

int lrbms_fine_step(lrbms_fine* f, const double* d_sat, double rtol, int32_t maxit, int32_t warm,
                    double* d_ph, double* d_flux, double* d_sat_out, uint8_t* d_flags,
                    int32_t* iterations, double* relres) {
  try {
    if (!f || !d_sat || !d_ph || !d_flux || !d_sat_out)
      return (set_error("NULL argument"), LRBMS_E_ARG);
    if (d_sat_out == d_sat) return (set_error("d_sat_out must not alias d_sat"), LRBMS_E_ARG);
    if (!(rtol > 0.0) || maxit < 1) return (set_error("rtol must be > 0 and maxit >= 1"), LRBMS_E_ARG);
    FineModel* F = reinterpret_cast<FineModel*>(f);
    int it = 0;
    double rr = 0.0;
    int rc = fine_solve_checked(F->M, F->S.s, d_sat, GAMMA_SAT, rtol, maxit, d_ph, &it, &rr,
                                warm != 0);
    if (iterations) *iterations = it;
    if (relres) *relres = rr;
    if (rc) return rc;
    if (!hip_ok(launch_flux(F->M.g, d_ph, d_sat, d_flux, 0), "flux")) return LRBMS_E_HIP;
    if ((rc = transport_impl(F->M, d_sat, d_flux, d_sat_out, d_flags, 0))) return rc;
    if (!hip_ok(hipStreamSynchronize(0), "fine step")) return LRBMS_E_HIP;
    return LRBMS_OK;
  } catch (const std::exception& e) {
    set_error(e.what());
    return LRBMS_E_OOM;
  }
}

void lrbms_fine_destroy(lrbms_fine* f) { delete reinterpret_cast<FineModel*>(f); }


int lrbms_copy_reduced_system(lrbms_model* m, double* blocks, double* fN) {
  if (!m) return (set_error("NULL argument"), LRBMS_E_ARG);
  Model* M = M_(m);
  if (!hip_ok(hipStreamSynchronize(M->last_stream), "synchronize")) return LRBMS_E_HIP;
  if (blocks && !hip_ok(hipMemcpy(blocks, M->d_blocks, M->nblk * sizeof(double),
                                  hipMemcpyDeviceToHost),
                        "copy blocks"))
    return LRBMS_E_HIP;
  if (fN && !hip_ok(hipMemcpy(fN, M->d_fN, M->N * sizeof(double), hipMemcpyDeviceToHost), "copy f"))
    return LRBMS_E_HIP;
  return LRBMS_OK;
}

int lrbms_copy_theta(lrbms_model* m, double* theta) {
  if (!m || !theta) return (set_error("NULL argument"), LRBMS_E_ARG);
  Model* M = M_(m);
  if (M->nprof == 0) return (set_error("model has no profiles"), LRBMS_E_STATE);
  if (!hip_ok(hipStreamSynchronize(M->last_stream), "synchronize")) return LRBMS_E_HIP;
  return hip_ok(hipMemcpy(theta, M->d_theta, M->nprof * sizeof(double), hipMemcpyDeviceToHost),
                "copy theta")
             ? LRBMS_OK
             : LRBMS_E_HIP;
}

int lrbms_model_status(lrbms_model* m) {
  if (!m) return (set_error("NULL argument"), LRBMS_E_ARG);
  Model* M = M_(m);
  if (!hip_ok(hipStreamSynchronize(M->last_stream), "synchronize")) return LRBMS_E_HIP;
  return read_status(*M);
}

int lrbms_model_set_checks(lrbms_model* m, int32_t on) {
  if (!m) return (set_error("NULL argument"), LRBMS_E_ARG);
  M_(m)->checks = on != 0;
  return LRBMS_OK;
}

int lrbms_profile_enable(lrbms_model* m, int32_t enable) {
  if (!m) return (set_error("NULL argument"), LRBMS_E_ARG);
  Model* M = M_(m);
  if (!hip_ok(hipStreamSynchronize(M->last_stream), "synchronize")) return LRBMS_E_HIP;
  M->timer.drain();
  M->timer.reset();
  M->timer.on = enable != 0;
  return LRBMS_OK;
}

int lrbms_profile_read(lrbms_model* m, lrbms_kernel_stat* out, int32_t cap, int32_t* n_out) {
  if (!m || !n_out || (cap > 0 && !out)) return (set_error("NULL argument"), LRBMS_E_ARG);
  Model* M = M_(m);
  KernelTimer& T = M->timer;
  const bool ok = T.drain();
  int cnt = 0;
  for (int k = 0; k < KK_COUNT; ++k) {
    if (T.n[k] == 0) continue;
    if (cnt < cap) {
      lrbms_kernel_stat& o = out[cnt];
      std::memset(&o, 0, sizeof(o));
      std::snprintf(o.name, sizeof(o.name), "%s", kernel_kind_name(k));
      o.launches = T.n[k];
      o.total_ms = T.ms[k];
      o.flops = T.flops[k] + (double)T.unit_n[k] * M->unit_flops[k];
      o.bytes = T.bytes[k] + (double)T.unit_n[k] * M->unit_bytes[k];
    }
    ++cnt;
  }
  *n_out = cnt;
  if (!ok) return (set_error("kernel timer: an event failed"), LRBMS_E_HIP);
  return LRBMS_OK;
}

int lrbms_model_autotune(lrbms_model* m, const double* d_sat, int32_t reps,
                         lrbms_tune_report* report) {
  try {
    if (!m || !d_sat || reps < 1) return (set_error("invalid argument"), LRBMS_E_ARG);
    Model* M = M_(m);
    if (M->owner) return (set_error("model belongs to a batch or server"), LRBMS_E_STATE);
    if (M->timer.on) return (set_error("kernel timing is on"), LRBMS_E_STATE);
    int rc = lrbms_online_assemble(m, d_sat, LRBMS_DIRECT, nullptr);
    if (rc != LRBMS_OK) return rc;
    DevArray pN;
    if (!pN.alloc((size_t)std::max(M->N, 1))) return LRBMS_E_OOM;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    struct Events {
      hipEvent_t& a;
      hipEvent_t& b;
      ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
      }
    } events{e0, e1};
    if (!hip_ok(hipEventCreate(&e0), "event") || !hip_ok(hipEventCreate(&e1), "event"))
      return LRBMS_E_HIP;
    auto time_plan = [&](const SolverPlan& P, const SolverDev& D, double& us) {
      for (int i = 0; i < 2; ++i)
        if (!hip_ok(solver_factor_solve(P, D, M->d_blocks, M->d_fN, pN.p, M->d_status, 0, M->refine),
                    "solve"))
          return false;
      if (!hip_ok(hipEventRecord(e0, 0), "event")) return false;
      for (int i = 0; i < reps; ++i)
        if (!hip_ok(solver_factor_solve(P, D, M->d_blocks, M->d_fN, pN.p, M->d_status, 0, M->refine),
                    "solve"))
          return false;
      float ms = 0.0f;
      if (!hip_ok(hipEventRecord(e1, 0), "event") || !hip_ok(hipEventSynchronize(e1), "event") ||
          !hip_ok(hipEventElapsedTime(&ms, e0, e1), "event"))
        return false;
      us = 1e3 * ms / reps;
      return true;
    };
    lrbms_tune_report rep{};
    // the box assembly: both variants timed on this state, the faster kept
    {
      for (int v = 0; v < 2; ++v) {
        if ((rc = set_asm_variant(*M, v)) != LRBMS_OK) return rc;
        for (int i = 0; i < 2; ++i)
          if ((rc = lrbms_online_assemble(m, d_sat, LRBMS_DIRECT, nullptr)) != LRBMS_OK) return rc;
        float ms = 0.0f;
        if (!hip_ok(hipEventRecord(e0, 0), "event")) return LRBMS_E_HIP;
        for (int i = 0; i < reps; ++i)
          if ((rc = lrbms_online_assemble(m, d_sat, LRBMS_DIRECT, nullptr)) != LRBMS_OK) return rc;
        if (!hip_ok(hipEventRecord(e1, 0), "event") || !hip_ok(hipEventSynchronize(e1), "event") ||
            !hip_ok(hipEventElapsedTime(&ms, e0, e1), "event"))
          return LRBMS_E_HIP;
        rep.asm_us[v] = 1e3 * ms / reps;
      }
      const int best = rep.asm_us[1] < rep.asm_us[0] ? 1 : 0;
      if ((rc = set_asm_variant(*M, best)) != LRBMS_OK) return rc;
      rep.asm_variant = best;
      if ((rc = lrbms_online_assemble(m, d_sat, LRBMS_DIRECT, nullptr)) != LRBMS_OK) return rc;
    }
    bool ok = time_plan(M->plan, M->sdev, rep.us_before);
    double best = 1e300;
    int best_leaf = M->leaf_max, best_split = M->split_min;
    long long best_bw = M->bw_min;
    SolverPlan best_plan;
    auto candidate = [&](int leaf, int split, long long bw) {
      SolverPlan P;
      if (!build_solver_plan(M->g.dim, M->nc, M->subs, M->ifaces, leaf, P, split, bw) ||
          !plan_in_bounds(P, M->nblk, M->N))
        return;
      SolverDev D;
      if (!solver_upload(P, D)) {
        solver_free(D);
        return;   // this shape does not fit: skip it
      }
      double us = 0.0;
      ok = time_plan(P, D, us);
      solver_free(D);
      ++rep.n_candidates;
      if (ok && us < best) {
        best = us;
        best_leaf = leaf;
        best_split = split;
        best_bw = bw;
        best_plan = std::move(P);
      }
    };
    // leaf size and step split first, then the backward split on that shape
    for (int leaf : {1, 2, 4, 8, 16})
      for (int split : {256, 1024, 1 << 30})
        if (ok) candidate(leaf, split, M->bw_min);
    const int leaf1 = best_leaf, split1 = best_split;
    const long long bw0 = M->bw_min < 0 ? bw_split_min() : M->bw_min;
    for (long long bw : {1LL << 12, 1LL << 14, 1LL << 16, 1LL << 18, 1LL << 62})
      if (ok && bw != bw0) candidate(leaf1, split1, bw);
    if (!ok) return LRBMS_E_HIP;
    if (rep.n_candidates > 0 && best < rep.us_before) {
      SolverDev D;
      if (!solver_upload(best_plan, D)) {
        solver_free(D);
        return (set_error("solver allocation failed"), LRBMS_E_OOM);
      }
      M->dev_bytes += D.bytes - M->sdev.bytes;
      solver_free(M->sdev);
      M->sdev = D;
      M->plan = std::move(best_plan);
      M->leaf_max = best_leaf;
      M->split_min = best_split;
      M->bw_min = best_bw;
    }
    rep.leaf_max = M->leaf_max;
    rep.split_min = M->split_min >= (1 << 30) ? 0 : (M->split_min < 0 ? step_split_min() : M->split_min);
    {
      const long long bw = M->bw_min < 0 ? bw_split_min() : M->bw_min;
      rep.bw_split_min = bw > INT32_MAX ? 0 : (int32_t)bw;
    }
    rep.us_per_solve = std::min(best, rep.us_before);
    // the unrefined solve's own error: one refinement step's correction
    {
      DevArray p0;
      if (!p0.alloc((size_t)std::max(M->N, 1))) return LRBMS_E_OOM;
      const int keep = std::max(M->refine, 1);
      if (!hip_ok(solver_factor_solve(M->plan, M->sdev, M->d_blocks, M->d_fN, p0.p, M->d_status, 0, 0),
                  "solve") ||
          !hip_ok(solver_factor_solve(M->plan, M->sdev, M->d_blocks, M->d_fN, pN.p, M->d_status, 0, 1),
                  "solve"))
        return LRBMS_E_HIP;
      std::vector<double> a(M->N), c(M->N);
      if (!hip_ok(hipMemcpy(a.data(), p0.p, a.size() * sizeof(double), hipMemcpyDeviceToHost),
                  "copy") ||
          !hip_ok(hipMemcpy(c.data(), pN.p, c.size() * sizeof(double), hipMemcpyDeviceToHost),
                  "copy"))
        return LRBMS_E_HIP;
      double dn = 0.0, cn = 0.0;
      for (int i = 0; i < M->N; ++i) {
        dn += (c[i] - a[i]) * (c[i] - a[i]);
        cn += c[i] * c[i];
      }
      rep.unrefined_error = cn > 0.0 ? std::sqrt(dn / cn) : 0.0;
      M->refine = (std::isfinite(rep.unrefined_error) && rep.unrefined_error < 1e-13) ? 0 : keep;
      rep.refine = M->refine;
    }
    if (report) *report = rep;
    M->last_stream = nullptr;
    return LRBMS_OK;
  } catch (const std::bad_alloc&) {
    return (set_error("host allocation failed"), LRBMS_E_OOM);
  }
}

void lrbms_model_destroy(lrbms_model* m) {
  if (!m) return;
  Model* M = M_(m);
  if (M->owner) {
    set_error("model_destroy: the model belongs to a fused batch or a server; destroy that first");
    return;
  }
  (void)hipStreamSynchronize(M->last_stream);
  delete M;
}

}  // extern "C"

namespace lrbms {
// The plan flattened into int64 records (layout parsed by the Python binding).
static std::vector<int64_t> flatten_plan(const SolverPlan& plan) {
  std::vector<int64_t> o;
  const int H = plan.nlevels;
  o.push_back((int64_t)plan.fronts.size());
  o.push_back(H);
  o.push_back((int64_t)plan.nodes.size());
  o.push_back((int64_t)plan.children.size());
  o.push_back(plan.lpan_doubles);
  o.push_back(plan.front_doubles);
  o.push_back(plan.vec_doubles);
  o.push_back(plan.inv_doubles);
  o.push_back((int64_t)(plan.flops));
  for (auto& f : plan.fronts) {
    int64_t v[12] = {f.off, f.voff, f.inv_off, f.m, f.u, f.node_off, f.n_nodes, f.child_off,
                     f.nchild, f.n_s_nodes, f.npanels, f.loff};
    o.insert(o.end(), v, v + 12);
  }
  for (auto& n : plan.nodes) {
    int64_t v[4] = {n.pos, n.pn_off, n.size, n.ppos};
    o.insert(o.end(), v, v + 4);
  }
  for (int c : plan.children) o.push_back(c);
  for (int h = 0; h < H; ++h) {
    o.push_back((int64_t)plan.level_fronts[h].size());
    for (int f : plan.level_fronts[h]) o.push_back(f);
    o.push_back((int64_t)plan.asm_items[h].size());
    for (auto& it : plan.asm_items[h]) {
      int64_t v[7] = {it.front, it.dr, it.dc, it.nr, it.nc, it.diag, it.nsrc};
      o.insert(o.end(), v, v + 7);
      for (int q = 0; q < 3; ++q) {
        int64_t w[4] = {it.src[q].so, it.src[q].rs, it.src[q].cs, it.src[q].kind};
        o.insert(o.end(), w, w + 4);
      }
    }
    // a split step lists its rows-only items, then its update items
    o.push_back((int64_t)plan.step_items[h].size());
    for (size_t p = 0; p < plan.step_items[h].size(); ++p) {
      o.push_back((int64_t)(plan.step_items[h][p].size() + plan.upd_items[h][p].size()));
      for (const auto* list : {&plan.step_items[h][p], &plan.upd_items[h][p]})
        for (auto& it : *list) {
          int64_t v[4] = {it.front, it.panel, it.ti, it.tj};
          o.insert(o.end(), v, v + 4);
        }
    }
  }
  // split backward products: partial storage, the p_N place of every split
  // front's U rows, each front's split data, the work items of every level
  o.push_back(plan.bw_part_doubles);
  o.push_back((int64_t)plan.urow_pn.size());
  for (int v : plan.urow_pn) o.push_back(v);
  for (auto& f : plan.fronts) {
    int64_t v[3] = {f.nzc, f.urow_off, f.zoff};
    o.insert(o.end(), v, v + 3);
  }
  for (int h = 0; h < H; ++h) {
    o.push_back((int64_t)plan.bw_items[h].size());
    for (auto& it : plan.bw_items[h]) {
      int64_t v[2] = {it.front, it.chunk};
      o.insert(o.end(), v, v + 2);
    }
  }
  // deferred Schur complements: per level its (front, ti, tj, wide) tiles
  for (int h = 0; h < H; ++h) {
    o.push_back((int64_t)plan.schur_items[h].size());
    for (auto& it : plan.schur_items[h]) {
      int64_t v[4] = {it.front, it.ti, it.tj, it.wide};
      o.insert(o.end(), v, v + 4);
    }
  }
  return o;
}
}  // namespace lrbms

extern "C" {

int lrbms_solver_plan_export(const lrbms_problem* prob, const int32_t* basis_sizes,
                             int32_t leaf_max, int64_t* buf, int64_t cap, int64_t* needed) {
  return lrbms_solver_plan_export_batch(&prob, &basis_sizes, &leaf_max, 1, buf, cap, needed);
}

int lrbms_solver_plan_export_batch(const lrbms_problem* const* probs,
                                   const int32_t* const* basis_sizes, const int32_t* leaf_max,
                                   int32_t n, int64_t* buf, int64_t cap, int64_t* needed) {
  try {
    if (!probs || !basis_sizes || !leaf_max || !needed || n < 1)
      return (set_error("invalid argument"), LRBMS_E_ARG);
    std::vector<SolverPlan> plans(n);
    std::vector<const SolverPlan*> ptrs;
    std::vector<long long> blk_base, pn_base;
    long long nblk = 0, nN = 0;
    for (int k = 0; k < n; ++k) {
      int rc = check_problem(probs[k]);
      if (rc) return rc;
      if (!basis_sizes[k] || leaf_max[k] < 1) return (set_error("invalid argument"), LRBMS_E_ARG);
      Model tmp;
      setup_layout(tmp, probs[k], basis_sizes[k]);
      if (!build_solver_plan(tmp.g.dim, tmp.nc, tmp.subs, tmp.ifaces, leaf_max[k], plans[k]))
        return (set_error("solver symbolic analysis failed"), LRBMS_E_ARG);
      ptrs.push_back(&plans[k]);
      blk_base.push_back(nblk);
      pn_base.push_back(nN);
      nblk += tmp.nblk;
      nN += tmp.N;
    }
    SolverPlan combined;
    const SolverPlan* plan = &plans[0];
    if (n > 1) {
      if (!combine_plans(ptrs, blk_base, pn_base, combined))
        return (set_error("plans cannot be combined"), LRBMS_E_ARG);
      plan = &combined;
    }
    if (!plan_in_bounds(*plan, nblk, nN))
      return (set_error("solver plan out of bounds"), LRBMS_E_ARG);
    const std::vector<int64_t> o = flatten_plan(*plan);
    *needed = (int64_t)o.size();
    if (buf && cap >= (int64_t)o.size()) std::copy(o.begin(), o.end(), buf);
    return LRBMS_OK;
  } catch (const std::exception& e) {
    set_error(e.what());
    return LRBMS_E_OOM;
  }
}

int lrbms_build_offline_bases(const lrbms_problem* prob, const lrbms_offline_opts* opts,
                              const double* mu, lrbms_model** out, lrbms_offline_report* report) {
  try {
    return build_offline_impl(prob, opts, mu, out, report);
  } catch (const std::exception& e) {
    set_error(e.what());
    return LRBMS_E_OOM;
  }
}

int lrbms_build_greedy_bases(const lrbms_problem* prob, const lrbms_offline_opts* opts,
                             const double* mu, int32_t n_max, double tol, const double* mu_bar,
                             lrbms_model** out, int32_t* chosen, double* errors,
                             int32_t max_iter, int32_t* n_iter, lrbms_offline_report* report) {
  try {
    return build_greedy_impl(prob, opts, mu, n_max, tol, mu_bar, out, chosen, errors, max_iter,
                             n_iter, report);
  } catch (const std::exception& e) {
    set_error(e.what());
    return LRBMS_E_OOM;
  }
}

int lrbms_fine_pressure(const lrbms_problem* prob, const double* d_field, int32_t kind,
                        double rtol, int32_t maxit, double* d_p, int32_t* iterations,
                        double* relres) {
  try {
    int rc = check_problem(prob);
    if (rc) return rc;
    if (!d_field || !d_p) return (set_error("NULL device pointer"), LRBMS_E_ARG);
    if (kind != LRBMS_FIELD_SATURATION && kind != LRBMS_FIELD_MOBILITY)
      return (set_error("kind must be LRBMS_FIELD_SATURATION or LRBMS_FIELD_MOBILITY"), LRBMS_E_ARG);
    if (!(rtol > 0.0) || maxit < 1) return (set_error("rtol must be > 0 and maxit >= 1"), LRBMS_E_ARG);
    Model tmp;
    setup_layout(tmp, prob, nullptr);
    if ((rc = upload_problem(tmp, prob))) return rc;
    FineSolverHandle fs;
    if (!(fs.s = fine_solver_create(tmp.g)))
      return (set_error("fine solver allocation failed"), LRBMS_E_OOM);
    int it = 0;
    double rr = 0.0;
    rc = fine_solve_checked(tmp, fs.s, d_field,
                            kind == LRBMS_FIELD_SATURATION ? GAMMA_SAT : GAMMA_FIELD, rtol, maxit,
                            d_p, &it, &rr);
    if (iterations) *iterations = it;
    if (relres) *relres = rr;
    return rc;
  } catch (const std::exception& e) {
    set_error(e.what());
    return LRBMS_E_OOM;
  }
}

int lrbms_time_of_flight(const lrbms_problem* prob, const double* d_flux, double tol,
                         int32_t maxit, double* d_tau, int32_t* sweeps) {
  try {
    int rc = check_problem(prob);
    if (rc) return rc;
    if (!d_flux || !d_tau) return (set_error("NULL device pointer"), LRBMS_E_ARG);
    if (!(tol >= 0.0) || maxit < 1) return (set_error("tol must be >= 0 and maxit >= 1"), LRBMS_E_ARG);
    Model tmp;
    setup_layout(tmp, prob, nullptr);
    if ((rc = upload_problem(tmp, prob))) return rc;
    int sw = 0;
    rc = tof_checked(tmp, d_flux, tol, maxit, d_tau, &sw);
    if (sweeps) *sweeps = sw;
    return rc;
  } catch (const std::exception& e) {
    set_error(e.what());
    return LRBMS_E_OOM;
  }
}

int lrbms_time_of_flight_noalloc(const lrbms_problem* prob, const double* d_flux, double tol,
                                 int32_t maxit, double* d_tau, int32_t* sweeps) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (!d_flux || !d_tau) return (set_error("NULL device pointer"), LRBMS_E_ARG);
  if (!(tol >= 0.0) || maxit < 1) return (set_error("tol must be >= 0 and maxit >= 1"), LRBMS_E_ARG);
  Geom g;
  int nc[3];
  fill_geom(g, nc, prob);
  // scratch layout: status (2 ints in one double slot), porosity, TOF work
  const size_t need = 1 + (size_t)g.ncell + tof_scratch_doubles(g);
  if (need > kScratchDoubles)
    return (set_error("time_of_flight_noalloc: the problem needs more than the fixed scratch "
                      "(128 MiB)"),
            LRBMS_E_ARG);
  double* base = scratch_ptr();
  if (!base) return LRBMS_E_HIP;
  int* status = reinterpret_cast<int*>(base);
  double* poro = base + 1;
  if (!hip_ok(hipMemsetAsync(status, 0, 2 * sizeof(int), 0), "clear status") ||
      !hip_ok(hipMemcpy(poro, prob->poro, (size_t)g.ncell * sizeof(double), hipMemcpyHostToDevice),
              "copy porosity"))
    return LRBMS_E_HIP;
  g.poro = poro;
  g.status = status;
  TofBufs B;
  tof_carve(g, poro + g.ncell, B);
  int sw = 0;
  rc = tof_solve_bufs(g, d_flux, tol, maxit, d_tau, status, &sw, B);
  if (sweeps) *sweeps = sw;
  int st[2] = {0, 0};
  if (!hip_ok(hipMemcpy(st, status, sizeof(st), hipMemcpyDeviceToHost), "status")) return LRBMS_E_HIP;
  if (st[0] < 0 && (rc == LRBMS_OK || rc == LRBMS_E_STATE)) rc = st[0];
  switch (rc) {
    case LRBMS_OK: break;
    case LRBMS_E_STATE: set_error("time of flight: sweeps did not converge within maxit"); break;
    case LRBMS_E_NOT_SPD: set_error("time of flight: singular cell block (a cell without flux)"); break;
    case LRBMS_E_NONFINITE: set_error("time of flight: non-finite values"); break;
    default: set_error("time of flight: HIP error"); break;
  }
  return rc;
}

int lrbms_model_export_profiles(const lrbms_model* m, double* profiles) {
  if (!m || !profiles) return (set_error("NULL argument"), LRBMS_E_ARG);
  const Model* M = M_(m);
  if (M->nprof == 0) return LRBMS_OK;
  const size_t n = (size_t)M->nprof * M->g.r * M->g.ncell;
  return hip_ok(hipMemcpy(profiles, M->d_prof, n * sizeof(double), hipMemcpyDeviceToHost),
                "export profiles")
             ? LRBMS_OK
             : LRBMS_E_HIP;
}

}  // extern "C"
