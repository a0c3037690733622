// Multifrontal block Cholesky of the reduced SPD system (eq. reducedSystem)
// with nested-dissection ordering of the coarse boxes.  See solver.h.
#include "solver.h"

#include "ktimer.h"

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
  std::vector<std::map<int, int>> pos(nf);  // box -> position in front
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
    foff += (ld + 1) * ld;
    d.voff = voff;
    voff += ld;
    d.npanels = (d.m + kNB - 1) / kNB;
    d.inv_off = ioff;
    ioff += (long long)d.npanels * kNB * kNB;
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
    if (f.kids.size() > 2) return false;
    auto add_ref = [&](int v, bool is_u) {
      NodeRef r;
      r.pos = pos[p].at(v);
      r.pn_off = subs[v].pn_off;
      r.size = subs[v].NE;
      r.ppos = -1;
      if (is_u) {
        if (f.parent < 0 || !pos[f.parent].count(v)) return false;
        r.ppos = pos[f.parent].at(v);
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
  // assembly: one item per destination block of every front
  plan.asm_items.assign(H, {});
  for (int h = 0; h < H; ++h) {
    for (int p : plan.level_fronts[h]) {
      FrontH& f = F[p];
      const FrontD& d = plan.fronts[p];
      const int ld = d.m + d.u;
      if (ld + 1 > kMaxLd) return false;
      std::vector<int> order = f.S;
      order.insert(order.end(), f.U.begin(), f.U.end());
      auto child_src = [&](int k, int v, int w, AsmSrc& s) {
        // update block (v, w) of child k (w = -1: its update row at box v)
        const FrontD& dc = plan.fronts[k];
        const long long ldc = dc.m + dc.u, ldac = ldc + 1;
        if (!pos[k].count(v) || pos[k][v] < dc.m) return false;
        if (w >= 0 && (!pos[k].count(w) || pos[k][w] < dc.m)) return false;
        if (w < 0) {
          s.so = dc.off + ldc + (long long)pos[k][v] * ldac;
          s.rs = 0;
          s.cs = (int)ldac;
        } else {
          s.so = dc.off + pos[k][v] + (long long)pos[k][w] * ldac;
          s.rs = 1;
          s.cs = (int)ldac;
        }
        s.kind = 1;
        s.pad = 0;
        return true;
      };
      for (size_t wi = 0; wi < order.size(); ++wi) {
        const int w = order[wi];
        const bool w_in_s = wi < f.S.size();
        for (size_t vi = wi; vi < order.size(); ++vi) {
          const int v = order[vi];
          AsmItem it{};
          it.front = p;
          it.dr = pos[p][v];
          it.dc = pos[p][w];
          it.nr = subs[v].NE;
          it.nc = subs[w].NE;
          it.diag = v == w;
          it.nsrc = 0;
          if (w_in_s) {
            AsmSrc s{};
            s.kind = 0;
            bool have = true;
            if (v == w) {
              s.so = subs[v].blk_off;
              s.rs = subs[v].NE;
              s.cs = 1;
            } else if (iface_of.count({v, w})) {
              s.so = ifaces[iface_of[{v, w}]].blk_off;   // v = lo, w = hi: A[v][w]
              s.rs = subs[w].NE;
              s.cs = 1;
            } else if (iface_of.count({w, v})) {
              s.so = ifaces[iface_of[{w, v}]].blk_off;   // A[v][w] = A[w][v]^T
              s.rs = 1;
              s.cs = subs[v].NE;
            } else {
              have = false;
            }
            if (have) it.src[it.nsrc++] = s;
          }
          for (int k : f.kids) {
            AsmSrc s{};
            if (child_src(k, v, w, s)) it.src[it.nsrc++] = s;
          }
          plan.asm_items[h].push_back(it);
        }
        AsmItem r{};   // right-hand-side row at box w
        r.front = p;
        r.dr = ld;
        r.dc = pos[p][w];
        r.nr = 1;
        r.nc = subs[w].NE;
        r.diag = 0;
        r.nsrc = 0;
        if (w_in_s) {
          AsmSrc s{};
          s.so = subs[w].pn_off;
          s.rs = 0;
          s.cs = 1;
          s.kind = 2;
          r.src[r.nsrc++] = s;
        }
        for (int k : f.kids) {
          AsmSrc s{};
          if (child_src(k, w, -1, s)) r.src[r.nsrc++] = s;
        }
        plan.asm_items[h].push_back(r);
      }
    }
  }
  // fused panel steps
  plan.step_items.assign(H, {});
  for (int h = 0; h < H; ++h) {
    int maxp = 0;
    for (int p : plan.level_fronts[h]) maxp = std::max(maxp, plan.fronts[p].npanels);
    plan.step_items[h].assign(maxp, {});
    for (int p : plan.level_fronts[h]) {
      const FrontD& d = plan.fronts[p];
      const int ld = d.m + d.u;
      for (int b = 0; b < d.npanels; ++b) {
        const int cs = b * kNB + std::min(kNB, d.m - b * kNB);
        const int nrt = (ld + 1 - cs + kNB - 1) / kNB;
        const int nct = (ld - cs + kNB - 1) / kNB;
        for (int ti = 0; ti < nrt; ++ti) {
          if (nct == 0) {
            plan.step_items[h][b].push_back(StepItem{p, b, ti, -1});
            continue;
          }
          for (int tj = 0; tj <= std::min(ti, nct - 1); ++tj)
            plan.step_items[h][b].push_back(StepItem{p, b, ti, tj});
        }
      }
    }
  }
  // algorithmic figures per launch: Cholesky arithmetic of the work each
  // launch does, and the front entries it must read and write (8 B each)
  plan.asm_flops.assign(H, 0.0);
  plan.asm_bytes.assign(H, 0.0);
  plan.f0_flops.assign(H, 0.0);
  plan.f0_bytes.assign(H, 0.0);
  plan.bw_flops.assign(H, 0.0);
  plan.bw_bytes.assign(H, 0.0);
  plan.step_flops.assign(H, {});
  plan.step_bytes.assign(H, {});
  for (int h = 0; h < H; ++h) {
    for (const AsmItem& it : plan.asm_items[h]) {
      const double e = (double)it.nr * it.nc;
      plan.asm_flops[h] += e * std::max(it.nsrc - 1, 0);
      plan.asm_bytes[h] += 8.0 * e * (it.nsrc + 1);
    }
    plan.step_flops[h].assign(plan.step_items[h].size(), 0.0);
    plan.step_bytes[h].assign(plan.step_items[h].size(), 0.0);
    for (int p : plan.level_fronts[h]) {
      const FrontD& d = plan.fronts[p];
      const double ld = d.m + d.u;
      const double nb0 = std::min(kNB, d.m);
      plan.f0_flops[h] += 2.0 * nb0 * nb0 * nb0 / 3.0;
      plan.f0_bytes[h] += 8.0 * (nb0 * (nb0 + 1) / 2 + nb0 * nb0);
      for (int b = 0; b < d.npanels; ++b) {
        const double nb = std::min(kNB, d.m - b * kNB);
        const double cs = b * kNB + nb, t = ld - cs;
        const double nb1 = (b + 1 < d.npanels) ? std::min(kNB, d.m - (int)cs) : 0.0;
        plan.step_flops[h][b] += (t + 1) * nb * nb + t * (t + 1) * nb + 2.0 * t * nb +
                                 2.0 * nb1 * nb1 * nb1 / 3.0;
        plan.step_bytes[h][b] += 8.0 * (2.0 * (t + 1) * nb + t * (t + 1) + 2.0 * t + nb * nb +
                                        nb1 * nb1);
      }
      const double m = d.m, u = d.u;
      plan.bw_flops[h] += 2.0 * m * u + m * m;
      plan.bw_bytes[h] += 8.0 * (m * u + m * (m + 1) / 2 + 2.0 * m + u);
    }
  }
  return true;
}

// ============================ numeric (device) ===============================

typedef double Tile[kNB + 1];

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// Cholesky of the nb x nb lower tile D (LDS) and the inverse Li of its factor.
// D is overwritten by L; Li is lower triangular, zero elsewhere.  The upper
// part of D is used as scratch.  Non-positive pivots set the status word and
// are replaced by 1 so that the results stay finite.
__device__ void tile_factor(Tile* D, Tile* Li, int nb, int* status) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int idx = tid; idx < kNB * kNB; idx += blockDim.x) Li[idx / kNB][idx % kNB] = 0.0;
  __syncthreads();
  for (int s0 = 0; s0 < nb; s0 += 16) {
    const int sb = min(16, nb - s0);
    if (wave == 0) {
      // lane i < 16 holds row i of the 16 x 16 diagonal block (identity padding)
      double r[16];
#pragma unroll
      for (int j = 0; j < 16; ++j)
        r[j] = (lane < sb && j <= lane) ? D[s0 + lane][s0 + j] : (lane == j ? 1.0 : 0.0);
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        double dk = readlane_f64(r[k], k);
        if (!(dk > 0.0) || !isfinite(dk)) {
          if (lane == 0) atomicMin(status, (int)LRBMS_E_NOT_SPD);
          dk = 1.0;
        }
        const double sk = sqrt(dk);
        if (lane == k) r[k] = sk;
        else if (lane > k) r[k] = r[k] / sk;
#pragma unroll
        for (int j = k + 1; j < 16; ++j) {
          const double ljk = readlane_f64(r[k], j);
          if (lane >= j) r[j] -= r[k] * ljk;
        }
      }
      // lane j < 16 forms column j of the inverse of the block
      double c[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const double lii = readlane_f64(r[i], i);
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < i; ++k) {
          const double lik = readlane_f64(r[k], i);
          if (k >= lane) acc += lik * c[k];
        }
        c[i] = (i < lane) ? 0.0 : (i == lane ? 1.0 / lii : -acc / lii);
      }
      if (lane < sb) {
#pragma unroll
        for (int j = 0; j < 16; ++j)
          if (j <= lane) D[s0 + lane][s0 + j] = r[j];
#pragma unroll
        for (int i = 0; i < 16; ++i)
          if (i >= lane && i < sb) Li[s0 + i][s0 + lane] = c[i];
      }
    }
    __syncthreads();
    // rows below the block inside the tile: X = D(rows, block) Linv_block^T
    const int r0 = s0 + sb, nrow = nb - r0;
    double v[4];
    int cnt = 0;
    for (int idx = tid; idx < nrow * sb; idx += blockDim.x, ++cnt) {
      const int i = r0 + idx % nrow, k = idx / nrow;
      double a = 0.0;
      for (int j = 0; j <= k; ++j) a += D[i][s0 + j] * Li[s0 + k][s0 + j];
      v[cnt] = a;
    }
    __syncthreads();
    cnt = 0;
    for (int idx = tid; idx < nrow * sb; idx += blockDim.x, ++cnt)
      D[r0 + idx % nrow][s0 + idx / nrow] = v[cnt];
    __syncthreads();
    // trailing update inside the tile
    for (int idx = tid; idx < nrow * nrow; idx += blockDim.x) {
      const int i = r0 + idx % nrow, j = r0 + idx / nrow;
      if (j <= i) {
        double a = 0.0;
        for (int k = 0; k < sb; ++k) a += D[i][s0 + k] * D[j][s0 + k];
        D[i][j] -= a;
      }
    }
    __syncthreads();
  }
  // off-diagonal blocks of the inverse, block diagonal by block diagonal:
  // Linv(I,J) = -Linv(I,I) sum_{K=J}^{I-1} L(I,K) Linv(K,J)
  const int nblk = (nb + 15) / 16;
  for (int dd = 1; dd < nblk; ++dd) {
    const int nbd = nblk - dd;
    for (int idx = tid; idx < nbd * 256; idx += blockDim.x) {
      const int J = idx / 256, I = J + dd, i = (idx % 256) / 16, j = idx % 16;
      const int gi = I * 16 + i, gj = J * 16 + j;
      double a = 0.0;
      if (gi < nb && gj < nb)
        for (int k = J * 16; k < I * 16; ++k) a += D[gi][k] * Li[k][gj];
      D[J * 16 + j][I * 16 + i] = a;   // transposed, in the unused upper part
    }
    __syncthreads();
    for (int idx = tid; idx < nbd * 256; idx += blockDim.x) {
      const int J = idx / 256, I = J + dd, i = (idx % 256) / 16, j = idx % 16;
      const int gi = I * 16 + i, gj = J * 16 + j;
      if (gi < nb && gj < nb) {
        double a = 0.0;
        for (int k = I * 16; k <= gi; ++k) a += Li[gi][k] * D[J * 16 + j][k];
        Li[gi][gj] = -a;
      }
    }
    __syncthreads();
  }
}

// Load the nb x nb diagonal tile of `panel` of a front, factor it and store the
// inverse of its factor.
__device__ void factor_diag_tile(const FrontD& f, const double* Fp, long long lda, int panel,
                                 double* Inv, Tile* D, Tile* Li, int* status) {
  const int c0 = panel * kNB, nb = min(kNB, f.m - c0);
  __syncthreads();
  for (int idx = threadIdx.x; idx < kNB * kNB; idx += blockDim.x) {
    const int i = idx % kNB, j = idx / kNB;
    D[i][j] = (i < nb && j < nb && j <= i) ? Fp[(c0 + i) + (c0 + j) * lda] : 0.0;
  }
  __syncthreads();
  tile_factor(D, Li, nb, status);
  double* Ip = Inv + f.inv_off + (long long)panel * kNB * kNB;
  for (int idx = threadIdx.x; idx < kNB * kNB; idx += blockDim.x) Ip[idx] = Li[idx / kNB][idx % kNB];
}

__global__ __launch_bounds__(256) void k_front_asm(const AsmItem* __restrict__ items,
                                                   const FrontD* __restrict__ fronts,
                                                   const double* __restrict__ blocks,
                                                   const double* __restrict__ fN,
                                                   double* __restrict__ F) {
  const AsmItem it = items[blockIdx.x];
  const FrontD f = fronts[it.front];
  const long long lda = f.m + f.u + 1;
  double* Fp = F + f.off;
  for (int idx = threadIdx.x; idx < it.nr * it.nc; idx += blockDim.x) {
    const int i = idx % it.nr, j = idx / it.nr;
    double v = 0.0;
    if (!it.diag || j <= i) {
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        if (s >= it.nsrc) break;
        const AsmSrc S = it.src[s];
        const double* src = S.kind == 0 ? blocks : (S.kind == 1 ? F : fN);
        v += src[S.so + (long long)i * S.rs + (long long)j * S.cs];
      }
    }
    Fp[(it.dr + i) + (long long)(it.dc + j) * lda] = v;
  }
}

__global__ __launch_bounds__(256) void k_front_factor0(const int* __restrict__ list,
                                                       const FrontD* __restrict__ fronts,
                                                       const double* __restrict__ F,
                                                       double* __restrict__ Inv, int* status) {
  __shared__ Tile D[kNB];
  __shared__ Tile Li[kNB];
  const FrontD f = fronts[list[blockIdx.x]];
  factor_diag_tile(f, F + f.off, f.m + f.u + 1, 0, Inv, D, Li, status);
}

// out = X Li^T for X, Li in LDS (rows < nr, k < nb); thread = 4 x 4 outputs.
__device__ __forceinline__ void tile_times_inv_t(Tile* X, Tile* Li, int nb, double acc[4][4]) {
  const int ti = (threadIdx.x % 16) * 4, tj = (threadIdx.x / 16) * 4;
  for (int p = 0; p < 4; ++p)
    for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
  for (int k = 0; k < nb; ++k) {
    double a[4], b[4];
    for (int p = 0; p < 4; ++p) {
      a[p] = X[ti + p][k];
      b[p] = Li[tj + p][k];
    }
    for (int p = 0; p < 4; ++p)
      for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * b[q];
  }
}

__global__ __launch_bounds__(256) void k_front_step(const StepItem* __restrict__ items,
                                                    const FrontD* __restrict__ fronts,
                                                    double* __restrict__ F,
                                                    double* __restrict__ Lb,
                                                    double* __restrict__ Inv, int* status) {
  __shared__ Tile Li[kNB];
  __shared__ Tile A[kNB];
  __shared__ Tile B[kNB];
  const StepItem it = items[blockIdx.x];
  const FrontD f = fronts[it.front];
  const long long ld = f.m + f.u, lda = ld + 1;
  double* Fp = F + f.off;
  double* Lp = Lb + f.off;
  const int c0 = it.panel * kNB, nb = min(kNB, f.m - c0), cs = c0 + nb;
  const int R0 = cs + it.ti * kNB, nr = min((long long)kNB, lda - R0);
  const double* Ip = Inv + f.inv_off + (long long)it.panel * kNB * kNB;
  const int ti4 = (threadIdx.x % 16) * 4, tj4 = (threadIdx.x / 16) * 4;
  for (int idx = threadIdx.x; idx < kNB * kNB; idx += blockDim.x) {
    const int i = idx % kNB, k = idx / kNB;
    Li[i][k] = Ip[i * kNB + k];
    B[i][k] = (i < nr && k < nb) ? Fp[(R0 + i) + (long long)(c0 + k) * lda] : 0.0;
  }
  __syncthreads();
  double acc[4][4];
  tile_times_inv_t(B, Li, nb, acc);
  for (int p = 0; p < 4; ++p)
    for (int q = 0; q < 4; ++q) A[ti4 + p][tj4 + q] = acc[p][q];
  __syncthreads();
  if (it.tj <= 0) {
    for (int idx = threadIdx.x; idx < nr * nb; idx += blockDim.x) {
      const int i = idx % nr, k = idx / nr;
      Lp[(R0 + i) + (long long)(c0 + k) * lda] = A[i][k];
    }
  }
  if (it.tj < 0) return;
  const int C0 = cs + it.tj * kNB, ncl = min((long long)kNB, ld - C0);
  Tile* Bt = A;
  if (it.tj != it.ti) {
    for (int idx = threadIdx.x; idx < kNB * kNB; idx += blockDim.x) {
      const int i = idx % kNB, k = idx / kNB;
      B[i][k] = (i < ncl && k < nb) ? Fp[(C0 + i) + (long long)(c0 + k) * lda] : 0.0;
    }
    __syncthreads();
    tile_times_inv_t(B, Li, nb, acc);
    __syncthreads();
    for (int p = 0; p < 4; ++p)
      for (int q = 0; q < 4; ++q) B[ti4 + p][tj4 + q] = acc[p][q];
    __syncthreads();
    Bt = B;
  }
  for (int p = 0; p < 4; ++p)
    for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
  for (int k = 0; k < nb; ++k) {
    double a[4], b[4];
    for (int p = 0; p < 4; ++p) {
      a[p] = A[ti4 + p][k];
      b[p] = Bt[tj4 + p][k];
    }
    for (int p = 0; p < 4; ++p)
      for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * b[q];
  }
  for (int p = 0; p < 4; ++p)
    for (int q = 0; q < 4; ++q) {
      const int i = ti4 + p, j = tj4 + q;
      if (i < nr && j < ncl) Fp[(R0 + i) + (long long)(C0 + j) * lda] -= acc[p][q];
    }
  // look-ahead: this workgroup owns the next diagonal tile
  if (it.ti == 0 && it.tj == 0 && it.panel + 1 < f.npanels)
    factor_diag_tile(f, Fp, lda, it.panel + 1, Inv, A, B, status);
}

__global__ __launch_bounds__(256) void k_front_backward(const int* __restrict__ list,
                                                        const FrontD* __restrict__ fronts,
                                                        const NodeRef* __restrict__ nodes,
                                                        const double* __restrict__ Lb,
                                                        const double* __restrict__ Inv,
                                                        double* __restrict__ pN) {
  extern __shared__ double w[];   // m + u values
  __shared__ double xb[kNB];
  const FrontD f = fronts[list[blockIdx.x]];
  const int ld = f.m + f.u;
  const long long lda = ld + 1;
  const double* Lp = Lb + f.off;
  for (int i = threadIdx.x; i < f.m; i += blockDim.x) w[i] = Lp[ld + (long long)i * lda];
  for (int n = f.n_s_nodes; n < f.n_nodes; ++n) {
    const NodeRef r = nodes[f.node_off + n];
    for (int i = threadIdx.x; i < r.size; i += blockDim.x) w[r.pos + i] = pN[r.pn_off + i];
  }
  __syncthreads();
  // z = y_S - L_US^T x_U (row i of L_US^T is contiguous in memory)
  for (int i = threadIdx.x; i < f.m; i += blockDim.x) {
    const double* col = Lp + (long long)i * lda;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int rr = f.m;
    for (; rr + 4 <= ld; rr += 4) {
      a0 += col[rr] * w[rr];
      a1 += col[rr + 1] * w[rr + 1];
      a2 += col[rr + 2] * w[rr + 2];
      a3 += col[rr + 3] * w[rr + 3];
    }
    for (; rr < ld; ++rr) a0 += col[rr] * w[rr];
    w[i] -= (a0 + a1) + (a2 + a3);
  }
  __syncthreads();
  for (int b = f.npanels - 1; b >= 0; --b) {
    const int c0 = b * kNB, nb = min(kNB, f.m - c0);
    const double* Li = Inv + f.inv_off + (long long)b * kNB * kNB;
    // xb is read over all kNB entries below (with zero weights past nb), so
    // the tail must hold zeros, not stale values that might be non-finite.
    if ((int)threadIdx.x < kNB) {
      double s = 0.0;
      for (int k = threadIdx.x; k < nb; ++k) s += Li[k * kNB + threadIdx.x] * w[c0 + k];
      xb[threadIdx.x] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < nb) w[c0 + threadIdx.x] = xb[threadIdx.x];
    for (int i = threadIdx.x; i < c0; i += blockDim.x) {
      const double* col = Lp + c0 + (long long)i * lda;
      double a[kNB];
#pragma unroll
      for (int k = 0; k < kNB; ++k) a[k] = (k < nb) ? col[k] : 0.0;
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int k = 0; k < kNB; k += 2) {
        s0 += a[k] * xb[k];
        s1 += a[k + 1] * xb[k + 1];
      }
      w[i] -= s0 + s1;
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
      !upload(plan.children, &dev.children, b))
    return false;
  const int H = plan.nlevels;
  dev.asm_items.assign(H, nullptr);
  dev.level_fronts.assign(H, nullptr);
  dev.step_items.assign(H, {});
  for (int h = 0; h < H; ++h) {
    if (!upload(plan.asm_items[h], &dev.asm_items[h], b) ||
        !upload(plan.level_fronts[h], &dev.level_fronts[h], b))
      return false;
    dev.step_items[h].assign(plan.step_items[h].size(), nullptr);
    for (size_t p = 0; p < plan.step_items[h].size(); ++p)
      if (!upload(plan.step_items[h][p], &dev.step_items[h][p], b)) return false;
  }
  int maxld = 1;
  for (auto& f : plan.fronts) maxld = std::max(maxld, f.m + f.u);
  if (hipFuncSetAttribute((const void*)k_front_backward, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(sizeof(double) * maxld)) != hipSuccess)
    return false;
  auto alloc = [&](double** p, long long n) {
    if (hipMalloc(p, std::max<long long>(n, 1) * sizeof(double)) != hipSuccess) return false;
    b += n * (long long)sizeof(double);
    return hipMemset(*p, 0, std::max<long long>(n, 1) * sizeof(double)) == hipSuccess;
  };
  return alloc(&dev.F, plan.front_doubles) && alloc(&dev.L, plan.front_doubles) &&
         alloc(&dev.V, plan.vec_doubles) && alloc(&dev.Inv, plan.inv_doubles);
}

void solver_free(SolverDev& dev) {
  auto f = [](void* p) {
    if (p) (void)hipFree(p);
  };
  f(dev.fronts);
  f(dev.nodes);
  f(dev.children);
  for (auto p : dev.asm_items) f(p);
  for (auto p : dev.level_fronts) f(p);
  for (auto& v : dev.step_items)
    for (auto p : v) f(p);
  f(dev.F);
  f(dev.L);
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
    const int nf = (int)plan.level_fronts[h].size();
    ktimer_begin(KK_FRONT_ASM, st);
    hipLaunchKernelGGL(k_front_asm, dim3(na), dim3(256), 0, st, dev.asm_items[h], dev.fronts,
                       blocks, fN, dev.F);
    ktimer_end(plan.asm_flops[h], plan.asm_bytes[h], st);
    ktimer_begin(KK_FRONT_FACTOR0, st);
    hipLaunchKernelGGL(k_front_factor0, dim3(nf), dim3(256), 0, st, dev.level_fronts[h],
                       dev.fronts, dev.F, dev.Inv, status);
    ktimer_end(plan.f0_flops[h], plan.f0_bytes[h], st);
    for (size_t p = 0; p < plan.step_items[h].size(); ++p) {
      const int ni = (int)plan.step_items[h][p].size();
      if (ni) {
        ktimer_begin(KK_FRONT_STEP, st);
        hipLaunchKernelGGL(k_front_step, dim3(ni), dim3(256), 0, st, dev.step_items[h][p],
                           dev.fronts, dev.F, dev.L, dev.Inv, status);
        ktimer_end(plan.step_flops[h][p], plan.step_bytes[h][p], st);
      }
    }
  }
  for (int h = H - 1; h >= 0; --h) {
    const int n = (int)plan.level_fronts[h].size();
    int maxld = 0;
    for (int f : plan.level_fronts[h])
      maxld = std::max(maxld, plan.fronts[f].m + plan.fronts[f].u);
    ktimer_begin(KK_FRONT_BACKWARD, st);
    hipLaunchKernelGGL(k_front_backward, dim3(n), dim3(256), sizeof(double) * maxld, st,
                       dev.level_fronts[h], dev.fronts, dev.nodes, dev.L, dev.Inv, pN);
    ktimer_end(plan.bw_flops[h], plan.bw_bytes[h], st);
  }
  return hipGetLastError();
}

}  // namespace lrbms
