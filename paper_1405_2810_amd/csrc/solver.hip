// Multifrontal block Cholesky of the reduced SPD system (eq. reducedSystem)
// with nested-dissection ordering of the coarse boxes.  See solver.h.
#include "solver.h"

#include <algorithm>
#include <map>

namespace lrbms {

// ============================ symbolic (host) ================================
namespace {

struct Region {
  int lo[3], hi[3];
  int count() const { return (hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]); }
  bool contains(const int x[3]) const {
    for (int a = 0; a < 3; ++a)
      if (x[a] < lo[a] || x[a] >= hi[a]) return false;
    return true;
  }
};

struct FrontH {
  Region R;
  std::vector<int> S, U, kids;
  int parent = -1, height = 0;
};

int box_id(const int nc[3], const int x[3]) { return x[0] + nc[0] * (x[1] + nc[1] * x[2]); }

std::vector<int> region_nodes(const int nc[3], const Region& R) {
  std::vector<int> out;
  for (int z = R.lo[2]; z < R.hi[2]; ++z)
    for (int y = R.lo[1]; y < R.hi[1]; ++y)
      for (int x = R.lo[0]; x < R.hi[0]; ++x) {
        const int c[3] = {x, y, z};
        out.push_back(box_id(nc, c));
      }
  return out;
}

int nd_build(const int nc[3], const Region& R, int leaf_max, std::vector<FrontH>& out) {
  if (R.count() <= 0) return -1;
  FrontH f;
  f.R = R;
  if (R.count() <= leaf_max) {
    f.S = region_nodes(nc, R);
  } else {
    int a = 0;
    for (int b = 1; b < 3; ++b)
      if (R.hi[b] - R.lo[b] > R.hi[a] - R.lo[a]) a = b;
    const int mid = R.lo[a] + (R.hi[a] - R.lo[a]) / 2;
    Region L = R, Rr = R, Sp = R;
    L.hi[a] = mid;
    Rr.lo[a] = mid + 1;
    Sp.lo[a] = mid;
    Sp.hi[a] = mid + 1;
    const int cl = nd_build(nc, L, leaf_max, out);
    const int cr = nd_build(nc, Rr, leaf_max, out);
    if (cl >= 0) f.kids.push_back(cl);
    if (cr >= 0) f.kids.push_back(cr);
    f.S = region_nodes(nc, Sp);
  }
  out.push_back(f);
  return (int)out.size() - 1;
}

}  // namespace

bool build_solver_plan(int dim, const int nc_in[3], const std::vector<Sub>& subs,
                       const std::vector<Iface>& ifaces, int leaf_max, SolverPlan& plan) {
  int nc[3] = {nc_in[0], nc_in[1], dim == 3 ? nc_in[2] : 1};
  const int nsub = nc[0] * nc[1] * nc[2];
  if ((int)subs.size() != nsub) return false;
  std::vector<FrontH> F;
  Region all{{0, 0, 0}, {nc[0], nc[1], nc[2]}};
  nd_build(nc, all, std::max(1, leaf_max), F);
  const int nf = (int)F.size();
  // elimination order: fronts in post order, separator boxes in order
  plan.elim.assign(nsub, -1);
  int cnt = 0;
  for (auto& f : F)
    for (int v : f.S) plan.elim[v] = cnt++;
  if (cnt != nsub) return false;
  // update sets and heights
  for (int p = 0; p < nf; ++p) {
    FrontH& f = F[p];
    std::vector<int> U;
    for (int v : region_nodes(nc, f.R)) {
      int x[3] = {v % nc[0], (v / nc[0]) % nc[1], v / (nc[0] * nc[1])};
      for (int a = 0; a < 3; ++a)
        for (int s = -1; s <= 1; s += 2) {
          int y[3] = {x[0], x[1], x[2]};
          y[a] += s;
          if (y[a] < 0 || y[a] >= nc[a]) continue;
          if (!f.R.contains(y)) U.push_back(box_id(nc, y));
        }
    }
    std::sort(U.begin(), U.end(), [&](int a, int b) { return plan.elim[a] < plan.elim[b]; });
    U.erase(std::unique(U.begin(), U.end()), U.end());
    f.U = U;
    f.height = 0;
    for (int k : f.kids) {
      F[k].parent = p;
      f.height = std::max(f.height, F[k].height + 1);
    }
  }
  // coupling lookup
  std::map<std::pair<int, int>, int> iface_of;
  for (int t = 0; t < (int)ifaces.size(); ++t) iface_of[{ifaces[t].lo, ifaces[t].hi}] = t;
  // fronts, node refs, storage offsets
  plan.fronts.assign(nf, FrontD{});
  plan.nodes.clear();
  plan.children.clear();
  std::vector<std::map<int, int>> pos(nf);  // node -> position in front
  long long foff = 0, voff = 0, ioff = 0;
  int noff = 0;
  plan.flops = 0.0;
  for (int p = 0; p < nf; ++p) {
    FrontH& f = F[p];
    FrontD& d = plan.fronts[p];
    int ps = 0;
    for (int v : f.S) {
      pos[p][v] = ps;
      ps += subs[v].NE;
    }
    d.m = ps;
    for (int v : f.U) {
      pos[p][v] = ps;
      ps += subs[v].NE;
    }
    d.u = ps - d.m;
    const long long ld = d.m + d.u;
    d.off = foff;
    foff += ld * ld;
    d.voff = voff;
    voff += ld;
    d.inv_off = ioff;
    ioff += (long long)((d.m + kNB - 1) / kNB) * kNB * kNB;
    d.n_s_nodes = (int)f.S.size();
    d.node_off = noff;
    d.n_nodes = (int)(f.S.size() + f.U.size());
    noff += d.n_nodes;
    d.child_off = (int)plan.children.size();
    d.nchild = (int)f.kids.size();
    for (int k : f.kids) plan.children.push_back(k);
    const double m = d.m, u = d.u;
    plan.flops += m * m * m / 3.0 + u * m * m + u * u * m;
  }
  for (int p = 0; p < nf; ++p) {
    FrontH& f = F[p];
    auto add_ref = [&](int v, bool is_u) {
      NodeRef r;
      r.pos = pos[p].at(v);
      r.pn_off = subs[v].pn_off;
      r.size = subs[v].NE;
      r.pad = -1;
      if (is_u) {
        if (f.parent < 0 || !pos[f.parent].count(v)) return false;
        r.pad = pos[f.parent].at(v);
      }
      plan.nodes.push_back(r);
      return true;
    };
    for (int v : f.S)
      if (!add_ref(v, false)) return false;
    for (int v : f.U)
      if (!add_ref(v, true)) return false;
  }
  plan.front_doubles = foff;
  plan.vec_doubles = voff;
  plan.inv_doubles = ioff;
  // levels by height
  int H = 0;
  for (auto& f : F) H = std::max(H, f.height + 1);
  plan.nlevels = H;
  plan.level_fronts.assign(H, {});
  for (int p = 0; p < nf; ++p) plan.level_fronts[F[p].height].push_back(p);
  // assembly items and tasks: one item per (front, column box)
  plan.asm_items.assign(H, {});
  plan.tasks.clear();
  for (int h = 0; h < H; ++h) {
    for (int p : plan.level_fronts[h]) {
      FrontH& f = F[p];
      const FrontD& d = plan.fronts[p];
      std::vector<int> order = f.S;
      order.insert(order.end(), f.U.begin(), f.U.end());
      for (size_t wi = 0; wi < order.size(); ++wi) {
        const int w = order[wi];
        AsmItem it;
        it.front = p;
        it.col0 = pos[p][w];
        it.ncol = subs[w].NE;
        it.task_off = (int)plan.tasks.size();
        it.pad = 0;
        if (wi < f.S.size()) {
          for (size_t vi = wi; vi < order.size(); ++vi) {
            const int v = order[vi];
            AddTask t{};
            t.nr = subs[v].NE;
            t.nc = subs[w].NE;
            t.dr = pos[p][v];
            t.dc = pos[p][w];
            t.from_front = 0;
            if (v == w) {
              t.so = subs[v].blk_off;
              t.rs = subs[v].NE;
              t.cs = 1;
            } else if (iface_of.count({v, w})) {
              const Iface& I = ifaces[iface_of[{v, w}]];   // v = lo, w = hi: A[v][w]
              t.so = I.blk_off;
              t.rs = subs[w].NE;
              t.cs = 1;
            } else if (iface_of.count({w, v})) {
              const Iface& I = ifaces[iface_of[{w, v}]];   // A[v][w] = A[w][v]^T
              t.so = I.blk_off;
              t.rs = 1;
              t.cs = subs[v].NE;
            } else {
              continue;
            }
            plan.tasks.push_back(t);
          }
        }
        for (int k : f.kids) {
          const FrontH& fc = F[k];
          const FrontD& dc = plan.fronts[k];
          if (!pos[k].count(w) || pos[k][w] < dc.m) continue;   // w not in U of child
          const long long ldc = dc.m + dc.u;
          for (int v : fc.U) {
            if (plan.elim[v] < plan.elim[w]) continue;
            AddTask t{};
            t.nr = subs[v].NE;
            t.nc = subs[w].NE;
            t.dr = pos[p][v];
            t.dc = pos[p][w];
            t.from_front = 1;
            t.so = dc.off + pos[k][v] + (long long)pos[k][w] * ldc;
            t.rs = 1;
            t.cs = (int)ldc;
            plan.tasks.push_back(t);
          }
        }
        it.ntask = (int)plan.tasks.size() - it.task_off;
        plan.asm_items[h].push_back(it);
      }
      (void)d;
    }
  }
  // panel and update items
  plan.panel_items.assign(H, {});
  plan.upd_items.assign(H, {});
  for (int h = 0; h < H; ++h) {
    int maxp = 0;
    for (int p : plan.level_fronts[h])
      maxp = std::max(maxp, (plan.fronts[p].m + kNB - 1) / kNB);
    plan.panel_items[h].assign(maxp, {});
    plan.upd_items[h].assign(maxp, {});
    for (int p : plan.level_fronts[h]) {
      const FrontD& d = plan.fronts[p];
      const int ld = d.m + d.u;
      const int np = (d.m + kNB - 1) / kNB;
      for (int b = 0; b < np; ++b) {
        const int c0 = b * kNB, nb = std::min(kNB, d.m - c0);
        plan.panel_items[h][b].push_back(PanelItem{p, b, c0, nb});
        for (int r0 = c0 + nb; r0 < ld; r0 += kNB)
          plan.panel_items[h][b].push_back(PanelItem{p, b, r0, std::min(kNB, ld - r0)});
        const int cs = c0 + nb;
        const int nt = (ld - cs + kNB - 1) / kNB;
        for (int ti = 0; ti < nt; ++ti)
          for (int tj = 0; tj <= ti; ++tj) plan.upd_items[h][b].push_back(UpdItem{p, b, ti, tj});
      }
    }
  }
  return true;
}

// ============================ numeric (device) ===============================

__global__ __launch_bounds__(256) void k_front_assemble(const AsmItem* __restrict__ items,
                                                        const FrontD* __restrict__ fronts,
                                                        const AddTask* __restrict__ tasks,
                                                        const double* __restrict__ blocks,
                                                        double* __restrict__ F) {
  const AsmItem it = items[blockIdx.x];
  const FrontD f = fronts[it.front];
  const long long ld = f.m + f.u;
  double* Fp = F + f.off;
  for (long long idx = threadIdx.x; idx < ld * it.ncol; idx += blockDim.x)
    Fp[(idx % ld) + (it.col0 + idx / ld) * ld] = 0.0;
  __syncthreads();
  for (int t = 0; t < it.ntask; ++t) {
    const AddTask T = tasks[it.task_off + t];
    const double* src = T.from_front ? F : blocks;
    for (int idx = threadIdx.x; idx < T.nr * T.nc; idx += blockDim.x) {
      const int i = idx % T.nr, j = idx / T.nr;
      Fp[(T.dr + i) + (long long)(T.dc + j) * ld] += src[T.so + (long long)i * T.rs + (long long)j * T.cs];
    }
    __syncthreads();
  }
}

// Cholesky of the diagonal tile and its inverse (in LDS), shared by the panel kernel.
__device__ void tile_chol_inv(double (*D)[kNB + 1], double (*Li)[kNB + 1], int nb, int* status) {
  for (int k = 0; k < nb; ++k) {
    if (threadIdx.x == 0) {
      double dk = D[k][k];
      if (!(dk > 0.0) || !isfinite(dk)) {
        atomicMin(status, (int)LRBMS_E_NOT_SPD);
        dk = 1.0;
      }
      D[k][k] = sqrt(dk);
    }
    __syncthreads();
    for (int i = k + 1 + threadIdx.x; i < nb; i += blockDim.x) D[i][k] /= D[k][k];
    __syncthreads();
    const int m = nb - k - 1;
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
      const int i = k + 1 + idx % m, j = k + 1 + idx / m;
      if (j <= i) D[i][j] -= D[i][k] * D[j][k];
    }
    __syncthreads();
  }
  // column j of the inverse of the lower factor (one thread per column)
  for (int j = threadIdx.x; j < kNB; j += blockDim.x) {
    for (int i = 0; i < kNB; ++i) Li[i][j] = 0.0;
    if (j < nb) {
      Li[j][j] = 1.0 / D[j][j];
      for (int i = j + 1; i < nb; ++i) {
        double s = 0.0;
        for (int k = j; k < i; ++k) s += D[i][k] * Li[k][j];
        Li[i][j] = -s / D[i][i];
      }
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_front_panel(const PanelItem* __restrict__ items,
                                                     const FrontD* __restrict__ fronts,
                                                     double* __restrict__ F,
                                                     double* __restrict__ Inv, int* status) {
  __shared__ double D[kNB][kNB + 1];
  __shared__ double Li[kNB][kNB + 1];
  __shared__ double X[kNB][kNB + 1];
  const PanelItem it = items[blockIdx.x];
  const FrontD f = fronts[it.front];
  const long long ld = f.m + f.u;
  double* Fp = F + f.off;
  const int c0 = it.panel * kNB;
  const int nb = min(kNB, f.m - c0);
  for (int idx = threadIdx.x; idx < kNB * kNB; idx += blockDim.x) {
    const int i = idx % kNB, j = idx / kNB;
    D[i][j] = (i < nb && j < nb && j <= i) ? Fp[(c0 + i) + (c0 + j) * ld] : 0.0;
  }
  __syncthreads();
  tile_chol_inv(D, Li, nb, status);
  if (it.row0 == c0) {
    // Only the inverse of the diagonal tile is kept: the substitutions use it and
    // the other workgroups of this launch still read the unfactored tile from F.
    double* Ip = Inv + f.inv_off + (long long)it.panel * kNB * kNB;
    for (int idx = threadIdx.x; idx < kNB * kNB; idx += blockDim.x)
      Ip[idx] = Li[idx / kNB][idx % kNB];
    return;
  }
  // rows below: L = F Linv^T
  for (int idx = threadIdx.x; idx < it.nrow * nb; idx += blockDim.x) {
    const int i = idx % it.nrow, j = idx / it.nrow;
    X[i][j] = Fp[(it.row0 + i) + (c0 + j) * ld];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < it.nrow * nb; idx += blockDim.x) {
    const int i = idx % it.nrow, j = idx / it.nrow;
    double s = 0.0;
    for (int k = 0; k <= j; ++k) s += X[i][k] * Li[j][k];
    Fp[(it.row0 + i) + (c0 + j) * ld] = s;
  }
}

__global__ __launch_bounds__(256) void k_front_update(const UpdItem* __restrict__ items,
                                                      const FrontD* __restrict__ fronts,
                                                      double* __restrict__ F) {
  __shared__ double A[kNB][kNB + 1];
  __shared__ double B[kNB][kNB + 1];
  const UpdItem it = items[blockIdx.x];
  const FrontD f = fronts[it.front];
  const int ld = f.m + f.u;
  double* Fp = F + f.off;
  const int c0 = it.panel * kNB;
  const int nb = min(kNB, f.m - c0);
  const int cs = c0 + nb;
  const int R0 = cs + it.ti * kNB, C0 = cs + it.tj * kNB;
  const int nr = min(kNB, ld - R0), ncl = min(kNB, ld - C0);
  for (int idx = threadIdx.x; idx < kNB * kNB; idx += blockDim.x) {
    const int i = idx % kNB, k = idx / kNB;
    A[i][k] = (i < nr && k < nb) ? Fp[(R0 + i) + (long long)(c0 + k) * ld] : 0.0;
    B[i][k] = (i < ncl && k < nb) ? Fp[(C0 + i) + (long long)(c0 + k) * ld] : 0.0;
  }
  __syncthreads();
  // each thread: a 4x4 sub-block of the 64x64 tile
  const int ti = (threadIdx.x % 16) * 4, tj = (threadIdx.x / 16) * 4;
  double acc[4][4] = {};
  for (int k = 0; k < nb; ++k) {
    double a[4], b[4];
    for (int q = 0; q < 4; ++q) {
      a[q] = A[ti + q][k];
      b[q] = B[tj + q][k];
    }
    for (int p = 0; p < 4; ++p)
      for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * b[q];
  }
  for (int p = 0; p < 4; ++p)
    for (int q = 0; q < 4; ++q) {
      const int i = ti + p, j = tj + q;
      if (i < nr && j < ncl) Fp[(R0 + i) + (long long)(C0 + j) * ld] -= acc[p][q];
    }
}

__global__ __launch_bounds__(256) void k_front_forward(const int* __restrict__ list,
                                                       const FrontD* __restrict__ fronts,
                                                       const NodeRef* __restrict__ nodes,
                                                       const int* __restrict__ children,
                                                       const double* __restrict__ F,
                                                       const double* __restrict__ Inv,
                                                       double* __restrict__ V,
                                                       const double* __restrict__ fN) {
  __shared__ double y[kNB];
  const FrontD f = fronts[list[blockIdx.x]];
  const int ld = f.m + f.u;
  const double* Fp = F + f.off;
  double* w = V + f.voff;
  for (int i = threadIdx.x; i < ld; i += blockDim.x) w[i] = 0.0;
  __syncthreads();
  for (int n = 0; n < f.n_s_nodes; ++n) {
    const NodeRef r = nodes[f.node_off + n];
    for (int i = threadIdx.x; i < r.size; i += blockDim.x) w[r.pos + i] = fN[r.pn_off + i];
  }
  __syncthreads();
  for (int c = 0; c < f.nchild; ++c) {
    const FrontD fc = fronts[children[f.child_off + c]];
    const double* wc = V + fc.voff;
    for (int n = fc.n_s_nodes; n < fc.n_nodes; ++n) {
      const NodeRef r = nodes[fc.node_off + n];
      for (int i = threadIdx.x; i < r.size; i += blockDim.x) w[r.pad + i] += wc[r.pos + i];
    }
    __syncthreads();
  }
  const int np = (f.m + kNB - 1) / kNB;
  for (int b = 0; b < np; ++b) {
    const int c0 = b * kNB, nb = min(kNB, f.m - c0);
    const double* Li = Inv + f.inv_off + (long long)b * kNB * kNB;
    if (threadIdx.x < nb) {
      double s = 0.0;
      for (int k = 0; k <= (int)threadIdx.x; ++k) s += Li[threadIdx.x * kNB + k] * w[c0 + k];
      y[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x < nb) w[c0 + threadIdx.x] = y[threadIdx.x];
    for (int rr = c0 + nb + threadIdx.x; rr < ld; rr += blockDim.x) {
      double s = 0.0;
      for (int k = 0; k < nb; ++k) s += Fp[rr + (long long)(c0 + k) * ld] * y[k];
      w[rr] -= s;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_front_backward(const int* __restrict__ list,
                                                        const FrontD* __restrict__ fronts,
                                                        const NodeRef* __restrict__ nodes,
                                                        const double* __restrict__ F,
                                                        const double* __restrict__ Inv,
                                                        double* __restrict__ V,
                                                        double* __restrict__ pN) {
  __shared__ double xb[kNB];
  const FrontD f = fronts[list[blockIdx.x]];
  const int ld = f.m + f.u;
  const double* Fp = F + f.off;
  double* w = V + f.voff;
  for (int n = f.n_s_nodes; n < f.n_nodes; ++n) {
    const NodeRef r = nodes[f.node_off + n];
    for (int i = threadIdx.x; i < r.size; i += blockDim.x) w[r.pos + i] = pN[r.pn_off + i];
  }
  __syncthreads();
  // z = y_S - L_US^T x_U
  for (int i = threadIdx.x; i < f.m; i += blockDim.x) {
    double s = 0.0;
    for (int rr = f.m; rr < ld; ++rr) s += Fp[rr + (long long)i * ld] * w[rr];
    w[i] -= s;
  }
  __syncthreads();
  const int np = (f.m + kNB - 1) / kNB;
  for (int b = np - 1; b >= 0; --b) {
    const int c0 = b * kNB, nb = min(kNB, f.m - c0);
    const double* Li = Inv + f.inv_off + (long long)b * kNB * kNB;
    if (threadIdx.x < nb) {
      double s = 0.0;
      for (int k = threadIdx.x; k < nb; ++k) s += Li[k * kNB + threadIdx.x] * w[c0 + k];
      xb[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x < nb) w[c0 + threadIdx.x] = xb[threadIdx.x];
    for (int i = threadIdx.x; i < c0; i += blockDim.x) {
      double s = 0.0;
      for (int k = 0; k < nb; ++k) s += Fp[(c0 + k) + (long long)i * ld] * xb[k];
      w[i] -= s;
    }
    __syncthreads();
  }
  for (int n = 0; n < f.n_s_nodes; ++n) {
    const NodeRef r = nodes[f.node_off + n];
    for (int i = threadIdx.x; i < r.size; i += blockDim.x) pN[r.pn_off + i] = w[r.pos + i];
  }
}

// ============================ upload / launch ================================
template <typename T>
static bool upload(const std::vector<T>& v, T** out, long long& bytes) {
  *out = nullptr;
  if (v.empty()) return true;
  if (hipMalloc(out, v.size() * sizeof(T)) != hipSuccess) return false;
  bytes += (long long)(v.size() * sizeof(T));
  return hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) == hipSuccess;
}

bool solver_upload(const SolverPlan& plan, SolverDev& dev) {
  long long& b = dev.bytes;
  if (!upload(plan.fronts, &dev.fronts, b) || !upload(plan.nodes, &dev.nodes, b) ||
      !upload(plan.children, &dev.children, b) || !upload(plan.tasks, &dev.tasks, b))
    return false;
  const int H = plan.nlevels;
  dev.asm_items.assign(H, nullptr);
  dev.level_fronts.assign(H, nullptr);
  dev.panel_items.assign(H, {});
  dev.upd_items.assign(H, {});
  for (int h = 0; h < H; ++h) {
    if (!upload(plan.asm_items[h], &dev.asm_items[h], b) ||
        !upload(plan.level_fronts[h], &dev.level_fronts[h], b))
      return false;
    dev.panel_items[h].assign(plan.panel_items[h].size(), nullptr);
    dev.upd_items[h].assign(plan.upd_items[h].size(), nullptr);
    for (size_t p = 0; p < plan.panel_items[h].size(); ++p) {
      if (!upload(plan.panel_items[h][p], &dev.panel_items[h][p], b) ||
          !upload(plan.upd_items[h][p], &dev.upd_items[h][p], b))
        return false;
    }
  }
  auto alloc = [&](double** p, long long n) {
    if (hipMalloc(p, std::max<long long>(n, 1) * sizeof(double)) != hipSuccess) return false;
    b += n * (long long)sizeof(double);
    return hipMemset(*p, 0, std::max<long long>(n, 1) * sizeof(double)) == hipSuccess;
  };
  return alloc(&dev.F, plan.front_doubles) && alloc(&dev.V, plan.vec_doubles) &&
         alloc(&dev.Inv, plan.inv_doubles);
}

void solver_free(SolverDev& dev) {
  auto f = [](void* p) {
    if (p) (void)hipFree(p);
  };
  f(dev.fronts);
  f(dev.nodes);
  f(dev.children);
  f(dev.tasks);
  for (auto p : dev.asm_items) f(p);
  for (auto p : dev.level_fronts) f(p);
  for (auto& v : dev.panel_items)
    for (auto p : v) f(p);
  for (auto& v : dev.upd_items)
    for (auto p : v) f(p);
  f(dev.F);
  f(dev.V);
  f(dev.Inv);
  dev = SolverDev{};
}

hipError_t solver_factor_solve(const SolverPlan& plan, const SolverDev& dev,
                               const double* blocks, const double* fN, double* pN, int* status,
                               hipStream_t st) {
  const int H = plan.nlevels;
  for (int h = 0; h < H; ++h) {
    const int na = (int)plan.asm_items[h].size();
    if (na)
      hipLaunchKernelGGL(k_front_assemble, dim3(na), dim3(256), 0, st, dev.asm_items[h],
                         dev.fronts, dev.tasks, blocks, dev.F);
    for (size_t p = 0; p < plan.panel_items[h].size(); ++p) {
      const int npi = (int)plan.panel_items[h][p].size();
      if (npi)
        hipLaunchKernelGGL(k_front_panel, dim3(npi), dim3(256), 0, st, dev.panel_items[h][p],
                           dev.fronts, dev.F, dev.Inv, status);
      const int nu = (int)plan.upd_items[h][p].size();
      if (nu)
        hipLaunchKernelGGL(k_front_update, dim3(nu), dim3(256), 0, st, dev.upd_items[h][p],
                           dev.fronts, dev.F);
    }
  }
  for (int h = 0; h < H; ++h) {
    const int n = (int)plan.level_fronts[h].size();
    hipLaunchKernelGGL(k_front_forward, dim3(n), dim3(256), 0, st, dev.level_fronts[h],
                       dev.fronts, dev.nodes, dev.children, dev.F, dev.Inv, dev.V, fN);
  }
  for (int h = H - 1; h >= 0; --h) {
    const int n = (int)plan.level_fronts[h].size();
    hipLaunchKernelGGL(k_front_backward, dim3(n), dim3(256), 0, st, dev.level_fronts[h],
                       dev.fronts, dev.nodes, dev.F, dev.Inv, dev.V, pN);
  }
  return hipGetLastError();
}

}  // namespace lrbms
