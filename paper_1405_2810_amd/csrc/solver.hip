// Multifrontal block Cholesky of the reduced SPD system (eq. reducedSystem)
// with nested-dissection ordering of the coarse boxes.  See solver.h.
#include <cstdlib>

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
                       const std::vector<Iface>& ifaces, int leaf_max, SolverPlan& plan,
                       int split_min, long long bw_min_in) {
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
  long long foff = 0, voff = 0, ioff = 0, loff = 0;
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
    d.loff = loff;
    for (int b = 0; b < d.npanels; ++b) loff += (long long)kNB * (ld + 1 - std::min(kNB * (b + 1), d.m));
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
  // large fronts: the backward product over their U rows is split, and every
  // U row's place in p_N recorded
  plan.urow_pn.clear();
  const long long bw_min = bw_min_in < 0 ? bw_split_min() : bw_min_in;
  for (FrontD& d : plan.fronts) {
    d.nzc = 0;
    d.urow_off = (int)plan.urow_pn.size();
    if (d.u == 0 || (long long)d.m * d.u < bw_min) continue;
    d.nzc = (d.u + 63) / 64;
    std::vector<int> urow(d.u, -1);
    for (int n = d.n_s_nodes; n < d.n_nodes; ++n) {
      const NodeRef& r = plan.nodes[d.node_off + n];
      for (int i = 0; i < r.size; ++i) urow[r.pos + i - d.m] = r.pn_off + i;
    }
    for (int v : urow)
      if (v < 0) return false;
    plan.urow_pn.insert(plan.urow_pn.end(), urow.begin(), urow.end());
  }
  plan.front_doubles = foff;
  plan.vec_doubles = voff;
  plan.inv_doubles = ioff;
  plan.lpan_doubles = loff;
  // residual plan: every box's row of blocks, its interfaces in index order
  plan.rboxes.clear();
  plan.rnbs.clear();
  plan.nN = 0;
  plan.res_flops = plan.res_bytes = 0.0;
  for (int v = 0; v < (int)subs.size(); ++v) {
    ResBox rb{};
    rb.blk_off = subs[v].blk_off;
    rb.pn_off = subs[v].pn_off;
    rb.ne = subs[v].NE;
    rb.nb0 = (int)plan.rnbs.size();
    double cols = rb.ne;
    for (const Iface& I : ifaces) {
      ResNb nb{};
      nb.blk_off = I.blk_off;
      if (I.lo == v) {          // A[v][hi], stored N_v x N_hi row-major
        nb.pn_off = subs[I.hi].pn_off;
        nb.ne = subs[I.hi].NE;
        nb.rs = subs[I.hi].NE;
        nb.cs = 1;
      } else if (I.hi == v) {   // A[v][lo] = A[lo][v]^T
        nb.pn_off = subs[I.lo].pn_off;
        nb.ne = subs[I.lo].NE;
        nb.rs = 1;
        nb.cs = subs[v].NE;
      } else {
        continue;
      }
      cols += nb.ne;
      plan.rnbs.push_back(nb);
    }
    rb.nb1 = (int)plan.rnbs.size();
    plan.rboxes.push_back(rb);
    plan.nN = std::max(plan.nN, (long long)rb.pn_off + rb.ne);
    plan.res_flops += 2.0 * rb.ne * cols;
    plan.res_bytes += 8.0 * (rb.ne * cols + 2.0 * rb.ne + cols);
  }
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
        const int nct = (d.m - cs + kNB - 1) / kNB;   // trailing S columns only
        for (int ti = 0; ti < nrt; ++ti) {
          // a tile of U rows only: its panel columns take the earlier
          // panels' products left-looking, in its rows-only item
          if (nct == 0 || cs + kNB * ti >= d.m) {
            plan.step_items[h][b].push_back(StepItem{p, b, ti, -1});
            continue;
          }
          for (int tj = 0; tj <= std::min(ti, nct - 1); ++tj)
            plan.step_items[h][b].push_back(StepItem{p, b, ti, tj});
        }
      }
    }
  }
  // prefetch items: in step p-1, for every U-row tile of step p (rows from
  // m on), the products of panels 0 .. p-2 in chunks of kPfPanels, one
  // workgroup per (tile, chunk); step p adds panel p-1's product itself
  for (int h = 0; h < H; ++h)
    for (int fi : plan.level_fronts[h]) {
      FrontD& d = plan.fronts[fi];
      const int ld = d.m + d.u;
      d.pf_nt = 0;
      d.pf_ns = d.npanels >= 3 ? (d.npanels - 2 + kPfPanels - 1) / kPfPanels : 0;
      for (int p = 2; p < d.npanels; ++p) {
        const int cs = p * kNB + std::min(kNB, d.m - p * kNB);
        const int nrt = (ld + 1 - cs + kNB - 1) / kNB;
        const int nsp = (p - 1 + kPfPanels - 1) / kPfPanels;
        for (int ti = 0; ti < nrt; ++ti) {
          if (cs + kNB * ti < d.m) continue;
          d.pf_nt = std::max(d.pf_nt, ti + 1);
          for (int sc = 0; sc < nsp; ++sc)
            plan.step_items[h][p - 1].push_back(StepItem{fi, p - 1, ti, -2 - sc});
        }
      }
    }
  assign_prefetch(plan);
  plan.upd_items.assign(H, {});
  for (int h = 0; h < H; ++h) plan.upd_items[h].assign(plan.step_items[h].size(), {});
  // deferred Schur complements: the lower tiles of (U + rhs row) x U
  plan.schur_items.assign(H, {});
  for (int h = 0; h < H; ++h)
    for (int p : plan.level_fronts[h]) {
      const FrontD& d = plan.fronts[p];
      if (d.u == 0) continue;
      const int wide = d.u >= kSchurWideMin ? 1 : 0, T = wide ? kSB : kNB;
      const int nrt = (d.u + 1 + T - 1) / T, nct = (d.u + T - 1) / T;
      for (int ti = 0; ti < nrt; ++ti)
        for (int tj = 0; tj <= std::min(ti, nct - 1); ++tj)
          plan.schur_items[h].push_back(SchurItem{p, ti, tj, wide});
    }
  split_steps(plan, split_min < 0 ? step_split_min() : split_min);
  assign_backward_split(plan);
  // algorithmic figures per launch: Cholesky arithmetic of the work each
  // launch does, and the front entries it must read and write (8 B each)
  plan.asm_flops.assign(H, 0.0);
  plan.asm_bytes.assign(H, 0.0);
  plan.f0_flops.assign(H, 0.0);
  plan.f0_bytes.assign(H, 0.0);
  plan.bw_flops.assign(H, 0.0);
  plan.bw_bytes.assign(H, 0.0);
  plan.bwg_flops.assign(H, 0.0);
  plan.bwg_bytes.assign(H, 0.0);
  plan.fw_flops.assign(H, 0.0);
  plan.fw_bytes.assign(H, 0.0);
  plan.schur_flops.assign(H, 0.0);
  plan.schur_bytes.assign(H, 0.0);
  plan.step_flops.assign(H, {});
  plan.step_bytes.assign(H, {});
  plan.upd_flops.assign(H, {});
  plan.upd_bytes.assign(H, {});
  for (int h = 0; h < H; ++h) {
    for (const AsmItem& it : plan.asm_items[h]) {
      const double e = (double)it.nr * it.nc;
      plan.asm_flops[h] += e * std::max(it.nsrc - 1, 0);
      plan.asm_bytes[h] += 8.0 * e * (it.nsrc + 1);
    }
    plan.step_flops[h].assign(plan.step_items[h].size(), 0.0);
    plan.step_bytes[h].assign(plan.step_items[h].size(), 0.0);
    plan.upd_flops[h].assign(plan.step_items[h].size(), 0.0);
    plan.upd_bytes[h].assign(plan.step_items[h].size(), 0.0);
    for (int p : plan.level_fronts[h]) {
      const FrontD& d = plan.fronts[p];
      const double ld = d.m + d.u;
      const double nb0 = std::min(kNB, d.m);
      plan.f0_flops[h] += 2.0 * nb0 * nb0 * nb0 / 3.0;
      plan.f0_bytes[h] += 8.0 * (nb0 * (nb0 + 1) / 2 + nb0 * nb0);
      for (int b = 0; b < d.npanels; ++b) {
        const double nb = std::min(kNB, d.m - b * kNB);
        const double cs = b * kNB + nb, t = ld - cs, sc = d.m - cs;
        const double nb1 = (b + 1 < d.npanels) ? std::min(kNB, d.m - (int)cs) : 0.0;
        // first row of the tiles of U rows only (left-looking), and the rows
        // of the tiles updated right-looking (from cs)
        const double ru0 = cs + kNB * std::ceil(sc / kNB), ts = ru0 - cs;
        const double nu = std::max(0.0, ld + 1 - std::max(ru0, (double)kNB * d.npanels));
        const double c0 = (double)b * kNB;
        // L rows (with the left-looking products of the U-row tiles), then
        // the trailing update of the S columns of the other tiles (the lower
        // trapezoid of ts rows by sc columns) and the next diagonal tile; a
        // split step counts them in its two launches
        const double fl = (t + 1) * nb * nb + 2.0 * nu * nb * c0;
        const double by = 8.0 * (2.0 * (t + 1) * nb + nb * nb + (nu + nb) * c0);
        const double ent = std::max(0.0, sc * ts - sc * (sc - 1) / 2.0);
        const double fu = 2.0 * nb * ent + 2.0 * nb1 * nb1 * nb1 / 3.0;
        const double bu = 8.0 * (2.0 * ent + nb1 * nb1);
        const bool split = !plan.upd_items[h][b].empty();
        plan.step_flops[h][b] += split ? fl : fl + fu;
        plan.step_bytes[h][b] += split ? by : by + bu;
        if (split) {
          plan.upd_flops[h][b] += fu;
          plan.upd_bytes[h][b] += bu;
        }
      }
      // deferred Schur complement: the lower part of (U + rhs row) x U read
      // and written once, L_US and the rhs row's S part read once
      if (d.u > 0) {
        const double m = d.m, u = d.u, ent = u * (u + 3) / 2.0;
        plan.schur_flops[h] += 2.0 * m * ent;
        plan.schur_bytes[h] += 8.0 * (2.0 * ent + (u + 1) * m);
      }
      // forward substitution of a new right-hand side (refinement): the
      // same entries of L as the backward, read once
      {
        const double m = d.m, u = d.u;
        plan.fw_flops[h] += 2.0 * m * u + m * m;
        plan.fw_bytes[h] += 8.0 * (m * u + m * (m + 1) / 2 + 2.0 * (m + u));
      }
      // backward: the product L_US^T x_U (in its own launch for a split
      // front, which writes nzc partial vectors that the backward sums), then
      // the triangular solve with L_SS
      const double m = d.m, u = d.u, pz = (double)d.nzc * d.m;
      if (d.nzc > 0) {
        plan.bwg_flops[h] += 2.0 * m * u;
        plan.bwg_bytes[h] += 8.0 * (m * u + u + pz);
        plan.bw_flops[h] += pz + m * m;
        plan.bw_bytes[h] += 8.0 * (pz + m * (m + 1) / 2 + 2.0 * m + u);
      } else {
        plan.bw_flops[h] += 2.0 * m * u + m * m;
        plan.bw_bytes[h] += 8.0 * (m * u + m * (m + 1) / 2 + 2.0 * m + u);
      }
    }
  }
  return true;
}

// ============================ numeric (device) ===============================

typedef double Tile[kNB + 1];
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// 1/sqrt(d): the hardware estimate refined by two Newton steps, which brings
// it to full double precision.
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
  const double h = 0.5 * d;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

// Orders the LDS accesses of one wave around this point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// c += a b for 16 x 16 blocks and an inner dimension of 4 (FP64 MFMA): lane l
// supplies a(l % 16, l / 16) and b(l / 16, l % 16); element (l / 16 + 4 v, l % 16)
// of the result is c[v].
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Work buffers of the tile factorization besides the tile itself.
struct TileAux {
  double T[4][16][17];   // one 16 x 16 product of the inverse per wave
  double cb[2][64];   // pivot column broadcast (wave 0)
  double dinv[kNB];   // 1 / L(k, k)
};

// Columns c0 .. c0+15 of the tile, rows c0 .. 63, by wave 0: lane = row,
// right-looking on unnormalized columns: pivot k subtracts a(i,k) a(j,k) / d_k
// from every later column j.  The wave issues one FP64 instruction every few
// cycles and a dependent one waits tens of cycles, so the loop keeps both the
// instruction count per pivot and the chain from d_k to d_{k+1} short:
//  * the pivot test runs on the scalar unit (integer compare of the high word:
//    a normal positive double below 1e300); a failed pivot sets the status
//    word and is replaced by 1 so that the results stay finite;
//  * 1/d_k = y0 (1 + e + e^2), e = 1 - d_k y0, from the hardware estimate y0
//    (good to ~5e-8, so e^3 is below double rounding): three operations where
//    two Newton steps take four;
//  * column k+1 is updated at once with its multiplier a(k+1,k) taken by
//    readlane; for the later columns the raw column k is broadcast through LDS
//    and their update is applied one pivot later, when the loads have landed
//    and the instructions fill the waits of the next pivot's chain (the
//    scheduling barrier keeps the compiler from sinking the loads to their
//    use); the LDS requests of one wave complete in issue order, so the
//    broadcast needs no other wait;
//  * 1/sqrt(d_k), for the scaling of the stored factor, is formed once per
//    lane after the loop.
// With inv, the inverse of the diagonal block is also formed from the
// registers.
__device__ __noinline__ void panel16(Tile* D, Tile* X, TileAux& A, int c0, bool inv, int* status) {
  const int lane = threadIdx.x & 63;
  const int row = c0 + lane;
  const bool act = row < kNB;
  const int rr = act ? row : kNB - 1;
  double a[16], ys[16], ds[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) a[t] = D[rr][c0 + t];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const long long keep = (act && c0 + t <= row) ? -1ll : 0ll;
    a[t] = __longlong_as_double(__double_as_longlong(a[t]) & keep);
  }
  bool bad = false;
  double mp = 0.0, cp[16];   // multipliers and broadcast column of the previous pivot
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    double dk = readlane_f64(a[k], k);
    const double ak1 = (k + 1 < 16) ? readlane_f64(a[k], k + 1) : 0.0;
    double cn[16];
    if (k + 2 < 16) {
      double* cb = A.cb[k & 1];
      cb[lane] = a[k];
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int t = k + 2; t < 16; ++t) cn[t] = cb[t];
    }
    __builtin_amdgcn_sched_barrier(0);
    if (k >= 1) {
#pragma unroll
      for (int t = k + 1; t < 16; ++t) a[t] = fma(-mp, cp[t], a[t]);
    }
#pragma unroll
    for (int t = k + 2; t < 16; ++t) cp[t] = cn[t];
    const int hi = __double2hiint(dk);
    const bool ok = (hi >= 0x00100000) && (hi < 0x7E37E43C);
    bad = bad || !ok;
    dk = ok ? dk : 1.0;
    ds[k] = dk;
    const double y0 = __builtin_amdgcn_rcp(dk);
    const double e = fma(-dk, y0, 1.0);
    const double g = fma(e, e, e);
    mp = a[k] * fma(y0, g, y0);
    if (k + 1 < 16) a[k + 1] = fma(-mp, ak1, a[k + 1]);
    __builtin_amdgcn_wave_barrier();
  }
  if (bad && lane == 0) atomicMin(status, (int)LRBMS_E_NOT_SPD);
  double dl = 1.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) dl = (lane == k) ? ds[k] : dl;
  const double yl = rsqrt_nr(dl);
#pragma unroll
  for (int k = 0; k < 16; ++k) ys[k] = readlane_f64(yl, k);
  // scale: L(i,k) = a(i,k) / sqrt(d_k) below the diagonal, sqrt(d_k) on it
#pragma unroll
  for (int k = 0; k < 16; ++k)
    a[k] = (lane > k) ? a[k] * ys[k] : ((lane == k) ? ds[k] * ys[k] : 0.0);
  if (lane < 16) A.dinv[c0 + lane] = yl;
  if (act) {
#pragma unroll
    for (int t = 0; t < 16; ++t) D[row][c0 + t] = (c0 + t <= row) ? a[t] : 0.0;
  }
  if (inv) {
    // inverse of the diagonal block from the registers: lane % 16 = column j,
    // x(i) = (delta_ij - sum_{k<i} L(i,k) x(k)) / L(i,i), L(i,k) read from lane i
    const int j = lane & 15;
    double x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int k = 0; k + 1 < i; k += 2) {
        s0 = fma(readlane_f64(a[k], i), x[k], s0);
        s1 = fma(readlane_f64(a[k + 1], i), x[k + 1], s1);
      }
      if (i & 1) s0 = fma(readlane_f64(a[i - 1], i), x[i - 1], s0);
      x[i] = ((i == j ? 1.0 : 0.0) - (s0 + s1)) * ys[i];
    }
    if (lane < 16) {
#pragma unroll
      for (int i = 0; i < 16; ++i) X[c0 + i][c0 + lane] = x[i];
    }
  }
}

// D(I, K) -= P(I) P(K)^T for the 16 x 16 blocks of panel J (one wave).
__device__ __forceinline__ void block_update(Tile* D, int I, int K, int J) {
  const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
  d4 c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int cc = 0; cc < 4; ++cc)
    c = mfma16(D[16 * I + r][16 * J + 4 * cc + q], D[16 * K + r][16 * J + 4 * cc + q], c);
#pragma unroll
  for (int v = 0; v < 4; ++v) D[16 * I + q + 4 * v][16 * K + r] -= c[v];
}

// Diagonal block J of X = L^{-1} by one wave from the factor in LDS:
// forward substitution with lane % 16 = column.
__device__ __noinline__ void inverse_diag_block(Tile* D, Tile* X, TileAux& A, int J) {
  const int lane = threadIdx.x & 63, r = lane & 15;
  const int c0 = 16 * J;
  double x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int k = 0; k + 1 < i; k += 2) {
      s0 = fma(D[c0 + i][c0 + k], x[k], s0);
      s1 = fma(D[c0 + i][c0 + k + 1], x[k + 1], s1);
    }
    if (i & 1) s0 = fma(D[c0 + i][c0 + i - 1], x[i - 1], s0);
    x[i] = ((i == r ? 1.0 : 0.0) - (s0 + s1)) * A.dinv[c0 + i];
  }
  if (lane < 16) {
#pragma unroll
    for (int i = 0; i < 16; ++i) X[c0 + i][c0 + lane] = x[i];
  }
}

// Off-diagonal block X(I, J) = -X(I, I) sum_{K=J}^{I-1} L(I, K) X(K, J), I > J,
// by one wave with its own 16 x 16 scratch T.
__device__ __forceinline__ void inverse_offdiag_block(Tile* D, Tile* X, double (*T)[17], int I,
                                                      int J) {
  const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
  d4 c = {0.0, 0.0, 0.0, 0.0};
  for (int K = J; K < I; ++K) {
#pragma unroll
    for (int cc = 0; cc < 4; ++cc)
      c = mfma16(D[16 * I + r][16 * K + 4 * cc + q], X[16 * K + 4 * cc + q][16 * J + r], c);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) T[q + 4 * v][r] = c[v];
  wave_lds_sync();
  d4 e = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int cc = 0; cc < 4; ++cc) e = mfma16(X[16 * I + r][16 * I + 4 * cc + q], T[4 * cc + q][r], e);
#pragma unroll
  for (int v = 0; v < 4; ++v) X[16 * I + q + 4 * v][16 * J + r] = -e[v];
}

// Cholesky factor L of the nb x nb SPD matrix held in the lower part of D
// (rows and columns nb .. 63 must hold the identity) and Ip = L^{-1} (kNB x kNB
// row-major, zero outside the lower nb x nb part).  Blocked by 16: wave 0
// factors panel J+1 right after updating its block column with panel J,
// while wave 1 inverts diagonal block J and waves 2-3 apply panel J to the
// remaining trailing blocks; the last diagonal block is inverted by wave 0
// from its registers.  The off-diagonal blocks of the inverse follow,
// diagonal by diagonal, over all waves.  D is overwritten by L (its strict
// upper part is scratch); X receives the inverse.
__device__ void tile_factor_inv(Tile* D, Tile* X, TileAux& A, double* Ip, int nb, int* status) {
  const int wave = threadIdx.x >> 6;
  const int nJ = (nb + 15) >> 4;
  // step J: panel J (factored in step J-1, or here for J = -1) is applied
  for (int J = -1; J < nJ; ++J) {
    if (wave == 0) {
      if (J + 1 < nJ) {
        for (int I = J + 1; I < nJ && J >= 0; ++I) block_update(D, I, J + 1, J);
        wave_lds_sync();
        panel16(D, X, A, 16 * (J + 1), J + 2 == nJ, status);
      }
    } else if (J >= 0 && J + 1 < nJ) {
      if (wave == 1) {
        inverse_diag_block(D, X, A, J);
      } else {
        int q = 0;
        for (int I = J + 2; I < nJ; ++I)
          for (int K = J + 2; K <= I; ++K, ++q)
            if ((q & 1) == wave - 2) block_update(D, I, K, J);
      }
    }
    __syncthreads();
  }
  for (int dd = 1; dd < nJ; ++dd) {
    for (int J = wave; J + dd < nJ; J += 4) inverse_offdiag_block(D, X, A.T[wave], J + dd, J);
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < kNB * kNB; idx += blockDim.x) {
    const int i = idx >> 6, j = idx & 63;
    Ip[idx] = (i < nb && j < nb && (j >> 4) <= (i >> 4)) ? X[i][j] : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_front_asm(const AsmItem* __restrict__ items,
                                                   const FrontD* __restrict__ fronts,
                                                   const double* __restrict__ blocks,
                                                   const double* __restrict__ fN,
                                                   double* __restrict__ F,
                                                   const int* __restrict__ active) {
  const AsmItem it = items[blockIdx.x];
  const FrontD f = fronts[it.front];
  if (active && !active[f.member]) return;
  const long long lda = f.m + f.u + 1;
  double* Fp = F + f.off;
  const int n = it.nr * it.nc;
  // four elements per thread and pass, every load of a pass issued before its stores
  for (int base = threadIdx.x; base < n; base += 4 * blockDim.x) {
    double v[4][3];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = base + u * (int)blockDim.x;
      const int i = idx % it.nr, j = idx / it.nr;
      const bool live = idx < n && (!it.diag || j <= i);
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const AsmSrc S = it.src[s];
        const double* src = S.kind == 0 ? blocks : (S.kind == 1 ? F : fN);
        v[u][s] = (live && s < it.nsrc) ? src[S.so + (long long)i * S.rs + (long long)j * S.cs] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = base + u * (int)blockDim.x;
      if (idx < n) {
        const int i = idx % it.nr, j = idx / it.nr;
        Fp[(it.dr + i) + (long long)(it.dc + j) * lda] = (v[u][0] + v[u][1]) + v[u][2];
      }
    }
  }
}

// First diagonal tile of every front of a level.
__global__ __launch_bounds__(256) void k_front_factor0(const int* __restrict__ list,
                                                       const FrontD* __restrict__ fronts,
                                                       const double* __restrict__ F,
                                                       double* __restrict__ Inv, int* status,
                                                       const int* __restrict__ active) {
  __shared__ Tile D[kNB];
  __shared__ Tile X[kNB];
  __shared__ TileAux aux;
  const FrontD f = fronts[list[blockIdx.x]];
  if (active && !active[f.member]) return;
  const long long lda = f.m + f.u + 1;
  const double* Fp = F + f.off;
  const int nb = min(kNB, f.m);
  double v[16];
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int idx = threadIdx.x + 256 * p;
    const int i = idx & 63, j = idx >> 6;
    v[p] = (i < nb && j < nb) ? ((j <= i) ? Fp[i + j * lda] : 0.0) : (i == j ? 1.0 : 0.0);
  }
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int idx = threadIdx.x + 256 * p;
    D[idx & 63][idx >> 6] = v[p];
  }
  __syncthreads();
  tile_factor_inv(D, X, aux, Inv + f.inv_off, nb, status);
}

// out = X Li^T for the 64 x 64 tiles X, Li in LDS (Li lower triangular, zero
// outside nb x nb): wave w forms row block w; out[cb] holds column block cb.
__device__ __forceinline__ void times_inv_t(Tile* Xm, Tile* Li, int nb, d4 out[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r = lane & 15, q = lane >> 4;
  const int nc = (nb + 3) >> 2;
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) out[cb] = d4{0.0, 0.0, 0.0, 0.0};
  for (int c = 0; c < nc; ++c) {
    const double a = Xm[16 * w + r][4 * c + q];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
      if (4 * c < 16 * cb + 16) out[cb] = mfma16(a, Li[16 * cb + r][4 * c + q], out[cb]);
  }
}

// One tile of panel `panel` of a front: the L rows of tile row ti
// (F rows times L_panel^{-T}, written to the L buffer) and, for tj >= 0, the
// trailing update F(ti, tj) -= L(ti) L(tj)^T.  The workgroup of tile (0, 0)
// then factors the next diagonal tile from the values it just formed.
__global__ __launch_bounds__(256) void k_front_step(const StepItem* __restrict__ items,
                                                    const FrontD* __restrict__ fronts,
                                                    double* __restrict__ F,
                                                    double* __restrict__ Lb,
                                                    double* __restrict__ Inv, int* status,
                                                    double* __restrict__ pf,
                                                    const int* __restrict__ active) {
  // Two tiles and the factorization's work area (77 KB): two workgroups fit
  // a CU.  Values that outlive a tile's reuse are held in registers.
  __shared__ Tile S0[kNB];
  __shared__ Tile S2[kNB];
  __shared__ TileAux aux;
  const StepItem it = items[xcd_item(blockIdx.x, gridDim.x)];
  const FrontD f = fronts[it.front];
  if (active && !active[f.member]) return;
  const long long ld = f.m + f.u, lda = ld + 1;
  const int tid0 = threadIdx.x;
  if (it.tj <= -2) {
    // prefetch for U-row tile ti of the next step (panel p): the products
    // sum_cp L(R, cp) L(P, cp)^T over the panels cp of chunk sc (all before
    // p - 1, so final), on FP64 MFMA, into the buffer of step p
    const int p = it.panel + 1, sc = -2 - it.tj;
    const int c0p = p * kNB, nbp = min(kNB, f.m - c0p), csp = c0p + nbp;
    const int R0p = csp + it.ti * kNB, nrp = (int)min((long long)kNB, lda - R0p);
    const int cp0 = sc * kPfPanels, cp1 = min(cp0 + kPfPanels, p - 1);
    const int lane = tid0 & 63, w = tid0 >> 6, r = lane & 15, q = lane >> 4;
    d4 c2[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) c2[cb] = d4{0.0, 0.0, 0.0, 0.0};
    double la[16], lp[16];
    auto load = [&](int cp) {
      const double* Lc = Lb + lpanel_base(f, cp);
      const int csc = kNB * (cp + 1);   // panels before the last are full
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int idx = tid0 + 256 * e, i = idx >> 6, k = idx & 63;
        la[e] = (i < nrp) ? Lc[(long long)(R0p - csc + i) * kNB + k] : 0.0;
        lp[e] = (i < nbp) ? Lc[(long long)(c0p - csc + i) * kNB + k] : 0.0;
      }
    };
    load(cp0);
    for (int cp = cp0; cp < cp1; ++cp) {
      if (cp > cp0) __syncthreads();   // the previous panel's products are done
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int idx = tid0 + 256 * e;
        S0[idx >> 6][idx & 63] = la[e];
        S2[idx >> 6][idx & 63] = lp[e];
      }
      __syncthreads();
      if (cp + 1 < cp1) load(cp + 1);   // in flight during the products
      for (int c = 0; c < kNB / 4; ++c) {
        const double a = S0[16 * w + r][4 * c + q];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) c2[cb] = mfma16(a, S2[16 * cb + r][4 * c + q], c2[cb]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) S0[16 * w + q + 4 * v][16 * cb + r] = c2[cb][v];
    __syncthreads();
    double* dst = pf + f.pf_off +
                  (((long long)(p & 1) * f.pf_nt + it.ti) * f.pf_ns + sc) * (kNB * kNB);
    for (int idx = tid0; idx < kNB * kNB; idx += 256) dst[idx] = S0[idx >> 6][idx & 63];
    return;
  }
  double* Fp = F + f.off;
  const int c0 = it.panel * kNB, nb = min(kNB, f.m - c0), cs = c0 + nb;
  const int R0 = cs + it.ti * kNB, nr = (int)min((long long)kNB, lda - R0);
  const double* Ip = Inv + f.inv_off + (long long)it.panel * kNB * kNB;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, r = lane & 15, q = lane >> 4;
  const bool upd = it.tj >= 0;
  const int C0 = cs + (upd ? it.tj : 0) * kNB;
  const int ncl = upd ? min(kNB, f.m - C0) : 0;   // S columns only
  // a tile of U rows only: the panel columns of its rows from 64 npanels on
  // have had no update yet (the rows between m and there were updated
  // right-looking, in the tile that straddles m before the last panel); the
  // earlier panels' products sum_c L(R, c) L(P, c)^T are subtracted from
  // those rows: the last panel's formed here on FP64 MFMA (L from the store),
  // the ones before it summed by the previous step's prefetch items (chunks
  // of kPfPanels panels), added in chunk order, all staged in S2
  const bool left = !upd && R0 >= f.m && it.panel > 0;
  const int mU = f.npanels * kNB;
  const int cp_first = it.panel >= 2 ? it.panel - 1 : 0;
  if (left) {
    d4 c2[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) c2[cb] = d4{0.0, 0.0, 0.0, 0.0};
    double la[16], lp[16];
    auto load = [&](int cp) {
      const double* Lc = Lb + lpanel_base(f, cp);
      const int csc = kNB * (cp + 1);   // panels before the last are full
#pragma unroll
      for (int p = 0; p < 16; ++p) {
        const int idx = tid + 256 * p, i = idx >> 6, k = idx & 63;
        la[p] = (i < nr) ? Lc[(long long)(R0 - csc + i) * kNB + k] : 0.0;
        lp[p] = (i < nb) ? Lc[(long long)(c0 - csc + i) * kNB + k] : 0.0;
      }
    };
    load(cp_first);
    for (int cp = cp_first; cp < it.panel; ++cp) {
      if (cp > cp_first) __syncthreads();   // the previous panel's products are done
#pragma unroll
      for (int p = 0; p < 16; ++p) {
        const int idx = tid + 256 * p;
        S0[idx >> 6][idx & 63] = la[p];
        S2[idx >> 6][idx & 63] = lp[p];
      }
      __syncthreads();
      if (cp + 1 < it.panel) load(cp + 1);   // in flight during the products
      for (int c = 0; c < kNB / 4; ++c) {
        const double a = S0[16 * w + r][4 * c + q];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) c2[cb] = mfma16(a, S2[16 * cb + r][4 * c + q], c2[cb]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) S2[16 * w + q + 4 * v][16 * cb + r] = c2[cb][v];
    __syncthreads();
    if (it.panel >= 2) {
      const int nsp = (it.panel - 1 + kPfPanels - 1) / kPfPanels;
      const double* src =
          pf + f.pf_off + ((long long)(it.panel & 1) * f.pf_nt + it.ti) * f.pf_ns * (kNB * kNB);
      for (int idx = tid; idx < kNB * kNB; idx += 256) {
        double a = S2[idx >> 6][idx & 63];
        for (int sc = 0; sc < nsp; ++sc) a += src[(long long)sc * (kNB * kNB) + idx];
        S2[idx >> 6][idx & 63] = a;
      }
      __syncthreads();
    }
  }
  // loads: L_panel^{-1} (row-major), the panel columns of tile row ti, and the
  // F tile (ti, tj) this workgroup updates (kept in registers)
  // (all loads are issued before the first LDS store, so their latencies overlap)
  double fold[16], li[16], bv[16];
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int idx = tid + 256 * p;
    const int i = idx & 63, k = idx >> 6;
    li[p] = Ip[idx];
    bv[p] = (i < nr && k < nb) ? Fp[(R0 + i) + (long long)(c0 + k) * lda] : 0.0;
    fold[p] = (upd && i < nr && k < ncl) ? Fp[(R0 + i) + (long long)(C0 + k) * lda] : 0.0;
  }
  // (a U-row tile's left-looking sums are in S2: each entry is read and
  // replaced by the thread that owns it)
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int idx = tid + 256 * p;
    S0[idx >> 6][idx & 63] = li[p];
    S2[idx & 63][idx >> 6] = (left && R0 + (idx & 63) >= mU) ? bv[p] - S2[idx & 63][idx >> 6] : bv[p];
  }
  __syncthreads();
  d4 acc[4];
  times_inv_t(S2, S0, nb, acc);
  __syncthreads();   // the F rows in S2 are consumed: L(ti) goes there
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int v = 0; v < 4; ++v) S2[16 * w + q + 4 * v][16 * cb + r] = acc[cb][v];
  __syncthreads();
  // a tile of the first trailing column (tj = 0) stores its L rows at its
  // end, from registers (acc), the look-ahead workgroup after the next
  // tile's factorization: a barrier waits for the workgroup's outstanding
  // stores, and these would hold up the barriers that follow
  const bool ahead = it.ti == 0 && it.tj == 0 && it.panel + 1 < f.npanels;
  double* Lrow = Lb + lpanel_base(f, it.panel) + (long long)(R0 - cs) * kNB;
  auto store_lrow = [&]() {
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * w + q + 4 * v, k = 16 * cb + r;
        if (i < nr && k < nb) Lrow[(long long)i * kNB + k] = acc[cb][v];
      }
  };
  if (it.tj < 0) {
    for (int idx = tid; idx < kNB * kNB; idx += 256) {
      const int i = idx >> 6, k = idx & 63;
      if (i < nr && k < nb) Lrow[(long long)i * kNB + k] = S2[i][k];
    }
  }
  if (!upd) return;
  // U = L(ti) L(tj)^T from At (rows) and Bt (columns)
  Tile* At = S2;
  Tile* Bt = S2;
  if (it.tj != it.ti) {
    // L(ti) stays in registers (acc) while S2 takes the F rows of tile row tj
    double yv[16];
#pragma unroll
    for (int p = 0; p < 16; ++p) {
      const int idx = tid + 256 * p;
      const int i = idx & 63, k = idx >> 6;
      yv[p] = (i < ncl && k < nb) ? Fp[(C0 + i) + (long long)(c0 + k) * lda] : 0.0;
    }
    __syncthreads();   // the L row store has read S2
#pragma unroll
    for (int p = 0; p < 16; ++p) {
      const int idx = tid + 256 * p;
      S2[idx & 63][idx >> 6] = yv[p];
    }
    __syncthreads();
    d4 acc2[4];
    times_inv_t(S2, S0, nb, acc2);
    __syncthreads();   // the panel inverse in S0 and the F rows in S2 are consumed
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        S2[16 * w + q + 4 * v][16 * cb + r] = acc[cb][v];
        S0[16 * w + q + 4 * v][16 * cb + r] = acc2[cb][v];
      }
    __syncthreads();
    Bt = S0;
  }
  // wave w forms row block w
  d4 u[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) u[cb] = d4{0.0, 0.0, 0.0, 0.0};
  const int nc = (nb + 3) >> 2;
  for (int c = 0; c < nc; ++c) {
    const double a = At[16 * w + r][4 * c + q];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) u[cb] = mfma16(a, Bt[16 * cb + r][4 * c + q], u[cb]);
  }
  __syncthreads();   // S2 is free: stage U there for coalesced read-modify-write
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int v = 0; v < 4; ++v) S2[16 * w + q + 4 * v][16 * cb + r] = u[cb][v];
  __syncthreads();
  const int nb1 = ahead ? min(kNB, f.m - cs) : 0;
  for (int p = 0; p < 16; ++p) {
    const int idx = tid + 256 * p;
    const int i = idx & 63, k = idx >> 6;
    const double nv = fold[p] - S2[i][k];
    // the next diagonal tile's own rows (i < nb1) are factored here from S0
    // and never read from the front again; rows below it (U rows of a tile
    // that straddles m) are
    if (i < nr && k < ncl && !(ahead && i < nb1)) Fp[(R0 + i) + (long long)(C0 + k) * lda] = nv;
    if (ahead) S0[i][k] = (i < nb1 && k < nb1) ? nv : (i == k ? 1.0 : 0.0);
  }
  if (!ahead) {
    if (it.tj == 0) store_lrow();
    return;
  }
  __syncthreads();
  tile_factor_inv(S0, S2, aux, Inv + f.inv_off + (long long)(it.panel + 1) * kNB * kNB, nb1,
                  status);
  store_lrow();
}

// Backward substitution L^T x = y of one front per workgroup, from the root
// down: w = (y_S, x_U); z_S = y_S - L_US^T x_U; then panel by panel from the
// last, x_b = L_bb^{-T} z_b with the stored tile inverse and
// z_{<b} -= L_{b,<b}^T x_b.  L is read row-wise from the panel-major store,
// lane = column within a panel, so every load is one coalesced row; the loads
// of a panel's update are issued before x_b is formed.
// Split backward product of a large front: for 64 U rows (one work item),
// the partial vector part[c][j] = sum over those rows r, in order, of
// L_US(r, j) x_U(r), for every column j of S.
__global__ __launch_bounds__(256) void k_front_bw_gemv(const BwItem* __restrict__ items,
                                                       const FrontD* __restrict__ fronts,
                                                       const double* __restrict__ Lpan,
                                                       const int* __restrict__ urow_pn,
                                                       const double* __restrict__ pN,
                                                       double* __restrict__ part,
                                                       const int* __restrict__ active) {
  __shared__ double xr[kNB];
  const BwItem it = items[blockIdx.x];
  const FrontD f = fronts[it.front];
  if (active && !active[f.member]) return;
  const int m = f.m, r0 = kNB * it.chunk, nr = min(kNB, f.u - r0), tid = threadIdx.x;
  if (tid < kNB) xr[tid] = tid < nr ? pN[urow_pn[f.urow_off + r0 + tid]] : 0.0;
  __syncthreads();
  double* out = part + f.zoff + (long long)it.chunk * m;
  for (int j = tid; j < m; j += blockDim.x) {
    const int b = j >> 6, k = j & 63, cs = min(kNB * (b + 1), m);
    const double* Lr = Lpan + lpanel_base(f, b) + (long long)(m - cs + r0) * kNB + k;
    double s = 0.0;
    for (int g = 0; g < nr; g += 16) {
      double a[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) a[t] = (g + t < nr) ? Lr[(long long)(g + t) * kNB] : 0.0;
#pragma unroll
      for (int t = 0; t < 16; ++t) s = fma(a[t], xr[g + t], s);
    }
    out[j] = s;
  }
}

// ysrc = nullptr: y_S is the forward-substituted right-hand side row of the
// factorization; otherwise y_S = ysrc[voff ..] (k_front_forward of a new
// right-hand side).  padd != nullptr: x_S is also added to padd (the
// refinement's correction of p_N).
// Threads of the backward sweep: kBwG waves, each a group of rows; a pass
// updates kBwP panels at once (kNB / kBwG rows of each per thread), so that
// every thread keeps kBwP x kNB / kBwG loads in flight per pass.
constexpr int kBwG = 8, kBwT = 64 * kBwG, kBwR = kNB / kBwG, kBwP = kBwG;

__global__ __launch_bounds__(kBwT) void k_front_backward(const int* __restrict__ list,
                                                        const FrontD* __restrict__ fronts,
                                                        const NodeRef* __restrict__ nodes,
                                                        const double* __restrict__ Lpan,
                                                        const double* __restrict__ Inv,
                                                        const double* __restrict__ part,
                                                        const double* __restrict__ ysrc,
                                                        double* __restrict__ pN,
                                                        double* __restrict__ padd,
                                                        const int* __restrict__ active) {
  extern __shared__ double w[];   // m + u values
  __shared__ double red[kBwG][kBwP][kNB];
  __shared__ double xb[kNB];
  const FrontD f = fronts[list[blockIdx.x]];
  if (active && !active[f.member]) return;
  const int m = f.m, u = f.u, ld = m + u, np = f.npanels, tid = threadIdx.x;
  const int k = tid & 63, g = tid >> 6;
  auto csof = [&](int b) { return min(kNB * (b + 1), m); };
  // sum over the row groups in a fixed order
  auto group_sum = [&](int q, int col) {
    double s = 0.0;
#pragma unroll
    for (int h = 0; h < kBwG; h += 2) s += red[h][q][col] + red[h + 1][q][col];
    return s;
  };
  // y_S from the right-hand-side rows, x_U from the parent
  for (int i = tid; i < m; i += kBwT) {
    const int b = i >> 6;
    w[i] = ysrc ? ysrc[f.voff + i]
                : Lpan[lpanel_base(f, b) + (long long)(ld - csof(b)) * kNB + (i - kNB * b)];
  }
  for (int n = f.n_s_nodes; n < f.n_nodes; ++n) {
    const NodeRef nr = nodes[f.node_off + n];
    for (int i = tid; i < nr.size; i += kBwT) w[nr.pos + i] = pN[nr.pn_off + i];
  }
  __syncthreads();
  // z_S = y_S - L_US^T x_U; a large front's products come in partial
  // vectors (k_front_bw_gemv), summed here in chunk order
  if (f.nzc > 0) {
    for (int j = tid; j < m; j += kBwT) {
      double acc = 0.0;
      for (int c = 0; c < f.nzc; ++c) acc += part[f.zoff + (long long)c * m + j];
      w[j] -= acc;
    }
    __syncthreads();
  }
  // otherwise: kBwP panels at a time, rows of U split over the groups
  for (int p0 = 0; p0 < np && u > 0 && f.nzc == 0; p0 += kBwP) {
    double s[kBwP];
#pragma unroll
    for (int q = 0; q < kBwP; ++q) s[q] = 0.0;
    for (int r0 = g; r0 < u; r0 += kNB) {
      double a[kBwP][kBwR];
#pragma unroll
      for (int q = 0; q < kBwP; ++q) {
        const int b = p0 + q;
        const double* Lr = Lpan + lpanel_base(f, b < np ? b : 0) +
                           (long long)(m - csof(b < np ? b : 0)) * kNB + k;
#pragma unroll
        for (int t = 0; t < kBwR; ++t) {
          const int r = r0 + kBwG * t;
          a[q][t] = (b < np && r < u) ? Lr[(long long)r * kNB] : 0.0;
        }
      }
#pragma unroll
      for (int t = 0; t < kBwR; ++t) {
        const int r = r0 + kBwG * t;
        const double xr = (r < u) ? w[m + r] : 0.0;
#pragma unroll
        for (int q = 0; q < kBwP; ++q) s[q] = fma(a[q][t], xr, s[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < kBwP; ++q) red[g][q][k] = s[q];
    __syncthreads();
    {
      const int b = p0 + g;
      if (b < np && k < min(kNB, m - kNB * b)) w[kNB * b + k] -= group_sum(g, k);
    }
    __syncthreads();
  }
  for (int b = np - 1; b >= 0; --b) {
    const int c0 = b * kNB, nb = min(kNB, m - c0);
    const double* Li = Inv + f.inv_off + (long long)b * kNB * kNB;
    // loads first: this thread's part of L_bb^{-1}, and rows c0 + kBwR g + t
    // of the kBwP panels before b (lane = column of that panel)
    double li[kBwR], a[kBwP][kBwR];
#pragma unroll
    for (int mm = 0; mm < kBwR; ++mm) {
      const int mr = kBwR * g + mm;
      li[mm] = (mr < nb && mr >= k) ? Li[mr * kNB + k] : 0.0;
    }
    auto load_rows = [&](int p1) {
#pragma unroll
      for (int q = 0; q < kBwP; ++q) {
        const int b2 = p1 - q, bb = b2 < 0 ? 0 : b2;
        const double* Lr = Lpan + lpanel_base(f, bb) + (long long)(c0 - csof(bb)) * kNB + k;
#pragma unroll
        for (int t = 0; t < kBwR; ++t) {
          const int kk = kBwR * g + t;
          a[q][t] = (b2 >= 0 && kk < nb) ? Lr[(long long)kk * kNB] : 0.0;
        }
      }
    };
    load_rows(b - 1);
    // x_b(k) = sum_{m >= k} Li(m, k) z_b(m): partial sums over the groups
    double s = 0.0;
#pragma unroll
    for (int mm = 0; mm < kBwR; ++mm) {
      const int mr = kBwR * g + mm;
      s = fma(li[mm], (mr < nb) ? w[c0 + mr] : 0.0, s);
    }
    red[g][0][k] = s;
    __syncthreads();
    if (tid < kNB) {
      const double x = (tid < nb) ? group_sum(0, tid) : 0.0;
      xb[tid] = x;
      if (tid < nb) w[c0 + tid] = x;
    }
    __syncthreads();
    // z of panels b-1 .. b-kBwP, then the older ones kBwP at a time
    for (int p1 = b - 1; p1 >= 0; p1 -= kBwP) {
      if (p1 != b - 1) load_rows(p1);
      double z[kBwP];
#pragma unroll
      for (int q = 0; q < kBwP; ++q) z[q] = 0.0;
#pragma unroll
      for (int t = 0; t < kBwR; ++t) {
        const double x = xb[kBwR * g + t];
#pragma unroll
        for (int q = 0; q < kBwP; ++q) z[q] = fma(a[q][t], x, z[q]);
      }
#pragma unroll
      for (int q = 0; q < kBwP; ++q) red[g][q][k] = z[q];
      __syncthreads();
      {
        const int b2 = p1 - g;
        if (b2 >= 0) w[kNB * b2 + k] -= group_sum(g, k);
      }
      __syncthreads();
    }
  }
  for (int n = 0; n < f.n_s_nodes; ++n) {
    const NodeRef nr = nodes[f.node_off + n];
    for (int i = tid; i < nr.size; i += kBwT) {
      const double x = w[nr.pos + i];
      pN[nr.pn_off + i] = x;
      if (padd) padd[nr.pn_off + i] += x;
    }
  }
}

// ---- iterative refinement -------------------------------------------------------
// Error-free transformations (Ogita, Rump and Oishi, "Accurate sum and dot
// product", 2005): a + b = s + e and a b = p + e exactly in floating point.
// hipcc contracts a * b + c into fma by default, which would break these
// transformations (the rounding of a b is what they capture): contraction is
// switched off inside them.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
  s = a + b;
  const double z = s - a;
  e = (a - (s - z)) + (b - z);
}

// acc (s, c): s + c ~ s_exact; adds -a x with the product and sum errors kept.
__device__ __forceinline__ void dot2_sub(double a, double x, double& s, double& c) {
#pragma clang fp contract(off)
  const double p = a * x;
  const double pe = fma(a, x, -p);   // a x = p + pe
  double t, e;
  two_sum(s, -p, t, e);
  s = t;
  c += e - pe;
}

// r = f_N - A_N p_N for one box per workgroup, lane = row of the box (64
// rows at a time), the columns of its row of blocks dealt to the four waves;
// every product and sum is compensated (Dot2), the waves' pairs are joined
// the same way, so r is accurate to about one rounding of its own size.  The
// diagonal block is read through its lower triangle, the part the
// factorization uses.
__global__ __launch_bounds__(256) void k_residual(const ResBox* __restrict__ boxes,
                                                  const ResNb* __restrict__ nbs,
                                                  const double* __restrict__ blocks,
                                                  const double* __restrict__ fN,
                                                  const double* __restrict__ pN,
                                                  double* __restrict__ res, int* status,
                                                  const int* __restrict__ active) {
  __shared__ double xs[2][4][kNB];
  const ResBox B = boxes[blockIdx.x];
  if (active && !active[B.member]) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, ne = B.ne;
  const double* D = blocks + B.blk_off;
  for (int i0 = 0; i0 < ne; i0 += kNB) {
    const int i = i0 + lane;
    const bool row = i < ne;
    double s = (wv == 0 && row) ? fN[B.pn_off + i] : 0.0, c = 0.0;
    for (int j = wv; j < ne; j += 4) {
      const double a = row ? (j <= i ? D[(long long)i * ne + j] : D[(long long)j * ne + i]) : 0.0;
      dot2_sub(a, pN[B.pn_off + j], s, c);
    }
    for (int q = B.nb0; q < B.nb1; ++q) {
      const ResNb nb = nbs[q];
      const double* A = blocks + nb.blk_off + (long long)i * nb.rs;
      for (int j = wv; j < nb.ne; j += 4) {
        const double a = row ? A[(long long)j * nb.cs] : 0.0;
        dot2_sub(a, pN[nb.pn_off + j], s, c);
      }
    }
    xs[0][wv][lane] = s;
    xs[1][wv][lane] = c;
    __syncthreads();
    if (wv == 0 && row) {
      double t = xs[0][0][lane], cc = xs[1][0][lane];
      for (int k = 1; k < 4; ++k) {
        double u, e;
        two_sum(t, xs[0][k][lane], u, e);
        t = u;
        cc += e + xs[1][k][lane];
      }
      const double r = t + cc;
      res[B.pn_off + i] = r;
      if (!isfinite(r)) atomicMin(status, (int)LRBMS_E_NONFINITE);
    }
    __syncthreads();
  }
}

// Row-block products of the substitutions, four lanes per row: lane l of wave
// g takes row 16 g + l / 4 of a 64-row block and the 16 columns 16 (l % 4) ..
// of a 64-column panel (contiguous in the panel-major L store, so the four
// lanes of a row read 128 contiguous bytes each); the four partial sums of a
// row are joined by two lane exchanges.
__device__ __forceinline__ double quad_sum(double s) {
  s += __shfl_xor(s, 1);
  s += __shfl_xor(s, 2);
  return s;
}

// Forward substitution L y = r of a new right-hand side, one workgroup per
// front, from the leaves up (one launch per level): w = (r_S, 0_U) plus the
// children's update vectors at their places in the front; then panel by
// panel y_b = L_bb^{-1} w_b with the stored tile inverse and
// w_{>b} -= L_{>b,b} y_b (a split front leaves its U rows to
// k_front_fw_gemv).  The front's vector store receives (y_S, w_U): y_S for
// the backward substitution, w_U for the parent.
__global__ __launch_bounds__(256) void k_front_forward(const int* __restrict__ list,
                                                       const FrontD* __restrict__ fronts,
                                                       const NodeRef* __restrict__ nodes,
                                                       const int* __restrict__ children,
                                                       const double* __restrict__ Lpan,
                                                       const double* __restrict__ Inv,
                                                       const double* __restrict__ r,
                                                       double* __restrict__ V,
                                                       const int* __restrict__ active) {
  extern __shared__ double w[];   // m + u values
  const FrontD f = fronts[list[blockIdx.x]];
  if (active && !active[f.member]) return;
  const int m = f.m, ld = m + f.u, np = f.npanels, tid = threadIdx.x;
  const int lane = tid & 63, g = tid >> 6, rr = 16 * g + (lane >> 2), seg = 16 * (lane & 3);
  for (int i = tid; i < ld; i += blockDim.x) w[i] = 0.0;
  __syncthreads();
  for (int n = 0; n < f.n_s_nodes; ++n) {
    const NodeRef nr = nodes[f.node_off + n];
    for (int i = tid; i < nr.size; i += blockDim.x) w[nr.pos + i] = r[nr.pn_off + i];
  }
  __syncthreads();
  // children in their fixed order; the places of one child's U nodes are distinct
  for (int c = 0; c < f.nchild; ++c) {
    const FrontD fc = fronts[children[f.child_off + c]];
    for (int n = fc.n_s_nodes; n < fc.n_nodes; ++n) {
      const NodeRef nr = nodes[fc.node_off + n];
      for (int i = tid; i < nr.size; i += blockDim.x) w[nr.ppos + i] += V[fc.voff + nr.pos + i];
    }
    __syncthreads();
  }
  const int rows_end = f.nzc > 0 ? m : ld;
  for (int b = 0; b < np; ++b) {
    const int c0 = b * kNB, nb = min(kNB, m - c0), cs = c0 + nb;
    // y_b = Linv w_b (row rr of the tile inverse, masked to its lower part)
    {
      const double* Ir = Inv + f.inv_off + (long long)b * kNB * kNB + (long long)rr * kNB + seg;
      double sacc = 0.0;
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const int k = seg + t;
        const bool on = rr < nb && k <= rr;
        sacc = fma(on ? Ir[t] : 0.0, on ? w[c0 + k] : 0.0, sacc);
      }
      sacc = quad_sum(sacc);
      __syncthreads();   // every lane has read w_b
      if ((lane & 3) == 0 && rr < nb) w[c0 + rr] = sacc;
      __syncthreads();
    }
    // w_R -= L(R, panel b) y_b for the rows after the panel
    const double* Lb = Lpan + lpanel_base(f, b) + seg;
    double y[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) y[t] = (seg + t < nb) ? w[c0 + seg + t] : 0.0;
#pragma unroll 2
    for (int R0 = cs; R0 < rows_end; R0 += kNB) {   // uniform over the workgroup
      const int R = R0 + rr;
      const bool on = R < rows_end;
      const double* Lr = Lb + (long long)(on ? R - cs : 0) * kNB;
      double sacc = 0.0;
#pragma unroll
      for (int t = 0; t < 16; ++t) sacc = fma(on ? Lr[t] : 0.0, y[t], sacc);
      sacc = quad_sum(sacc);
      if ((lane & 3) == 0 && on) w[R] -= sacc;
    }
    __syncthreads();
  }
  for (int i = tid; i < ld; i += blockDim.x) V[f.voff + i] = w[i];
}

// U rows of a split front's forward substitution: for 64 U rows (one work
// item) V[voff + m + r] -= sum_j L_US(r, j) y_S(j), y_S = V[voff ..], the
// panels one after another, four lanes per row.
__global__ __launch_bounds__(256) void k_front_fw_gemv(const BwItem* __restrict__ items,
                                                       const FrontD* __restrict__ fronts,
                                                       const double* __restrict__ Lpan,
                                                       double* __restrict__ V,
                                                       const int* __restrict__ active) {
  const BwItem it = items[blockIdx.x];
  const FrontD f = fronts[it.front];
  if (active && !active[f.member]) return;
  const int m = f.m, r0 = kNB * it.chunk, nr = min(kNB, f.u - r0), tid = threadIdx.x;
  const int lane = tid & 63, g = tid >> 6, rr = 16 * g + (lane >> 2), seg = 16 * (lane & 3);
  const bool on = rr < nr;
  const double* y = V + f.voff;
  double sacc = 0.0;
  for (int b = 0; b < f.npanels; ++b) {
    const int c0 = b * kNB, nb = min(kNB, m - c0), cs = c0 + nb;
    const double* Lr = Lpan + lpanel_base(f, b) + (long long)(m - cs + r0 + (on ? rr : 0)) * kNB + seg;
    double a[16], yv[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const bool k_on = seg + t < nb;
      a[t] = (on && k_on) ? Lr[t] : 0.0;
      yv[t] = k_on ? y[c0 + seg + t] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) sacc = fma(a[t], yv[t], sacc);
  }
  sacc = quad_sum(sacc);
  if ((lane & 3) == 0 && on) V[f.voff + m + r0 + rr] -= sacc;
}

// Split every step of at least split_min items that still holds trailing
// updates: each tile row keeps one rows-only item (its item with tj <= 0
// becomes tj = -1), the items with tj >= 0 move to the update launch.
void split_steps(SolverPlan& plan, int split_min) {
  for (int h = 0; h < plan.nlevels; ++h)
    for (size_t b = 0; b < plan.step_items[h].size(); ++b) {
      std::vector<StepItem>& items = plan.step_items[h][b];
      size_t n_upd = 0;
      for (const StepItem& it : items) n_upd += it.tj >= 0;
      if (n_upd == 0 || (long long)items.size() < split_min) continue;
      std::vector<StepItem> rows;
      std::vector<StepItem>& upd = plan.upd_items[h][b];
      for (const StepItem& it : items) {
        if (it.tj <= -2) {
          rows.push_back(it);   // a prefetch item stays as it is
          continue;
        }
        if (it.tj <= 0) rows.push_back(StepItem{it.front, it.panel, it.ti, -1});
        if (it.tj >= 0) upd.push_back(it);
      }
      items.swap(rows);
    }
}

void assign_prefetch(SolverPlan& plan) {
  plan.pf_doubles = 0;
  for (int h = 0; h < plan.nlevels; ++h) {
    long long off = 0;
    for (int fi : plan.level_fronts[h]) {
      FrontD& d = plan.fronts[fi];
      d.pf_off = off;
      off += 2LL * d.pf_nt * d.pf_ns * kNB * kNB;
    }
    plan.pf_doubles = std::max(plan.pf_doubles, off);
  }
}

void assign_backward_split(SolverPlan& plan) {
  plan.bw_items.assign(plan.nlevels, {});
  plan.bw_part_doubles = 0;
  for (int h = 0; h < plan.nlevels; ++h) {
    long long off = 0;
    for (int fi : plan.level_fronts[h]) {
      FrontD& d = plan.fronts[fi];
      if (d.nzc == 0) continue;
      d.zoff = off;
      off += (long long)d.nzc * d.m;
      for (int c = 0; c < d.nzc; ++c) plan.bw_items[h].push_back(BwItem{fi, c});
    }
    plan.bw_part_doubles = std::max(plan.bw_part_doubles, off);
  }
}

long long bw_split_min() {
  const char* e = std::getenv("LRBMS_BW_SPLIT_MIN");
  return e && *e ? std::atoll(e) : (1LL << 14);
}

int step_split_min() {
  const char* e = std::getenv("LRBMS_STEP_SPLIT_MIN");
  return e && *e ? std::atoi(e) : 1024;
}

bool combine_plans(const std::vector<const SolverPlan*>& plans,
                   const std::vector<long long>& blk_base, const std::vector<long long>& pn_base,
                   SolverPlan& out) {
  if (plans.empty() || blk_base.size() != plans.size() || pn_base.size() != plans.size())
    return false;
  for (long long b : pn_base)
    if (b < 0 || b >= (1LL << 30)) return false;   // p_N offsets are int
  out = SolverPlan{};
  int H = 0;
  for (const SolverPlan* P : plans) H = std::max(H, P->nlevels);
  out.nlevels = H;
  out.level_fronts.assign(H, {});
  out.asm_items.assign(H, {});
  out.step_items.assign(H, {});
  out.asm_flops.assign(H, 0.0);
  out.asm_bytes.assign(H, 0.0);
  out.f0_flops.assign(H, 0.0);
  out.f0_bytes.assign(H, 0.0);
  out.bw_flops.assign(H, 0.0);
  out.bw_bytes.assign(H, 0.0);
  out.bwg_flops.assign(H, 0.0);
  out.bwg_bytes.assign(H, 0.0);
  out.fw_flops.assign(H, 0.0);
  out.fw_bytes.assign(H, 0.0);
  out.schur_flops.assign(H, 0.0);
  out.schur_bytes.assign(H, 0.0);
  out.schur_items.assign(H, {});
  out.step_flops.assign(H, {});
  out.step_bytes.assign(H, {});
  out.upd_items.assign(H, {});
  out.upd_flops.assign(H, {});
  out.upd_bytes.assign(H, {});
  for (int h = 0; h < H; ++h) {
    size_t np = 0;
    for (const SolverPlan* P : plans)
      if (h < P->nlevels) np = std::max(np, P->step_items[h].size());
    out.step_items[h].assign(np, {});
    out.step_flops[h].assign(np, 0.0);
    out.step_bytes[h].assign(np, 0.0);
    out.upd_items[h].assign(np, {});
    out.upd_flops[h].assign(np, 0.0);
    out.upd_bytes[h].assign(np, 0.0);
  }
  for (size_t k = 0; k < plans.size(); ++k) {
    const SolverPlan& P = *plans[k];
    const int fbase = (int)out.fronts.size();
    const int nbase = (int)out.nodes.size();
    const int cbase = (int)out.children.size();
    const long long front0 = out.front_doubles;
    const int ubase = (int)out.urow_pn.size();
    for (int v : P.urow_pn) out.urow_pn.push_back(v + (int)pn_base[k]);
    for (FrontD f : P.fronts) {
      f.member = (int)k;
      f.urow_off += ubase;
      f.off += out.front_doubles;
      f.loff += out.lpan_doubles;
      f.voff += out.vec_doubles;
      f.inv_off += out.inv_doubles;
      f.node_off += nbase;
      f.child_off += cbase;
      out.fronts.push_back(f);
    }
    for (NodeRef r : P.nodes) {
      r.pn_off += (int)pn_base[k];
      out.nodes.push_back(r);
    }
    for (int c : P.children) out.children.push_back(c + fbase);
    const int rbase = (int)out.rnbs.size();
    for (ResBox rb : P.rboxes) {
      rb.member = (int)k;
      rb.blk_off += blk_base[k];
      rb.pn_off += (int)pn_base[k];
      rb.nb0 += rbase;
      rb.nb1 += rbase;
      out.rboxes.push_back(rb);
    }
    for (ResNb nb : P.rnbs) {
      nb.blk_off += blk_base[k];
      nb.pn_off += (int)pn_base[k];
      out.rnbs.push_back(nb);
    }
    out.nN = std::max(out.nN, P.nN + pn_base[k]);
    out.res_flops += P.res_flops;
    out.res_bytes += P.res_bytes;
    out.front_doubles += P.front_doubles;
    out.lpan_doubles += P.lpan_doubles;
    out.vec_doubles += P.vec_doubles;
    out.inv_doubles += P.inv_doubles;
    out.flops += P.flops;
    for (int h = 0; h < P.nlevels; ++h) {
      for (int f : P.level_fronts[h]) out.level_fronts[h].push_back(f + fbase);
      for (AsmItem it : P.asm_items[h]) {
        it.front += fbase;
        for (int q = 0; q < it.nsrc; ++q) {
          AsmSrc& S = it.src[q];
          S.so += S.kind == 0 ? blk_base[k] : (S.kind == 1 ? front0 : pn_base[k]);
        }
        out.asm_items[h].push_back(it);
      }
      for (size_t b = 0; b < P.step_items[h].size(); ++b) {
        for (StepItem it : P.step_items[h][b]) {
          it.front += fbase;
          out.step_items[h][b].push_back(it);
        }
        for (StepItem it : P.upd_items[h][b]) {
          it.front += fbase;
          out.upd_items[h][b].push_back(it);
        }
        out.step_flops[h][b] += P.step_flops[h][b];
        out.step_bytes[h][b] += P.step_bytes[h][b];
        out.upd_flops[h][b] += P.upd_flops[h][b];
        out.upd_bytes[h][b] += P.upd_bytes[h][b];
      }
      out.asm_flops[h] += P.asm_flops[h];
      out.asm_bytes[h] += P.asm_bytes[h];
      out.f0_flops[h] += P.f0_flops[h];
      out.f0_bytes[h] += P.f0_bytes[h];
      out.bw_flops[h] += P.bw_flops[h];
      out.bw_bytes[h] += P.bw_bytes[h];
      out.bwg_flops[h] += P.bwg_flops[h];
      out.bwg_bytes[h] += P.bwg_bytes[h];
      out.fw_flops[h] += P.fw_flops[h];
      out.fw_bytes[h] += P.fw_bytes[h];
      out.schur_flops[h] += P.schur_flops[h];
      out.schur_bytes[h] += P.schur_bytes[h];
      for (SchurItem it : P.schur_items[h]) {
        it.front += fbase;
        out.schur_items[h].push_back(it);
      }
    }
  }
  // the members' steps side by side can be large enough to split (the
  // per-launch figures then stay those of the members' own launches)
  split_steps(out, step_split_min());
  assign_backward_split(out);
  assign_prefetch(out);
  return true;
}

bool plan_in_bounds(const SolverPlan& plan, long long nblk, long long nN) {
  const long long nf = (long long)plan.fronts.size();
  for (const FrontD& f : plan.fronts) {
    const long long ld = (long long)f.m + f.u;
    if (f.m < 1 || f.u < 0 || ld + 1 > kMaxLd) return false;
    if (f.npanels != (f.m + kNB - 1) / kNB) return false;
    if (f.off < 0 || f.off + (ld + 1) * ld > plan.front_doubles) return false;
    if (f.voff < 0 || f.voff + ld > plan.vec_doubles) return false;
    if (f.inv_off < 0 || f.inv_off + (long long)f.npanels * kNB * kNB > plan.inv_doubles)
      return false;
    const int last = f.npanels - 1;
    const long long cs = std::min(kNB * (last + 1), f.m);
    if (f.loff < 0 || lpanel_base(f, last) + (ld + 1 - cs) * kNB > plan.lpan_doubles) return false;
    if (f.pf_nt < 0 || f.pf_ns < 0 || f.pf_off < 0 ||
        f.pf_off + 2LL * f.pf_nt * f.pf_ns * kNB * kNB > plan.pf_doubles)
      return false;
    if (f.node_off < 0 || f.n_s_nodes > f.n_nodes ||
        (long long)f.node_off + f.n_nodes > (long long)plan.nodes.size())
      return false;
    if (f.child_off < 0 || (long long)f.child_off + f.nchild > (long long)plan.children.size())
      return false;
    for (int n = 0; n < f.n_nodes; ++n) {
      const NodeRef& r = plan.nodes[f.node_off + n];
      if (r.pos < 0 || r.size < 0 || r.pos + r.size > ld) return false;
      if (r.pn_off < 0 || (long long)r.pn_off + r.size > nN) return false;
    }
    if (f.nzc != 0) {
      if (f.nzc != (f.u + 63) / 64 || f.urow_off < 0 ||
          (long long)f.urow_off + f.u > (long long)plan.urow_pn.size() || f.zoff < 0 ||
          f.zoff + (long long)f.nzc * f.m > plan.bw_part_doubles)
        return false;
      for (int rr = 0; rr < f.u; ++rr) {
        const int v = plan.urow_pn[f.urow_off + rr];
        if (v < 0 || v >= nN) return false;
      }
    }
  }
  for (int c : plan.children)
    if (c < 0 || c >= nf) return false;
  if (plan.nN > nN) return false;
  for (const ResBox& rb : plan.rboxes) {
    if (rb.ne < 1 || rb.pn_off < 0 || (long long)rb.pn_off + rb.ne > plan.nN ||
        rb.blk_off < 0 || rb.blk_off + (long long)rb.ne * rb.ne > nblk || rb.nb0 < 0 ||
        rb.nb1 < rb.nb0 || rb.nb1 > (int)plan.rnbs.size())
      return false;
    for (int q = rb.nb0; q < rb.nb1; ++q) {
      const ResNb& nb = plan.rnbs[q];
      if (nb.ne < 1 || nb.pn_off < 0 || (long long)nb.pn_off + nb.ne > plan.nN ||
          nb.blk_off < 0 || nb.rs < 1 || nb.cs < 1 ||
          nb.blk_off + (long long)(rb.ne - 1) * nb.rs + (long long)(nb.ne - 1) * nb.cs >= nblk)
        return false;
    }
  }
  auto span_ok = [](long long so, int nr, int nc, int rs, int cs, long long size) {
    const long long lo = so + std::min(0LL, (long long)(nr - 1) * rs) +
                         std::min(0LL, (long long)(nc - 1) * cs);
    const long long hi = so + std::max(0LL, (long long)(nr - 1) * rs) +
                         std::max(0LL, (long long)(nc - 1) * cs);
    return lo >= 0 && hi < size;
  };
  if ((int)plan.level_fronts.size() != plan.nlevels || (int)plan.asm_items.size() != plan.nlevels ||
      (int)plan.step_items.size() != plan.nlevels || (int)plan.upd_items.size() != plan.nlevels)
    return false;
  for (int h = 0; h < plan.nlevels; ++h) {
    for (int f : plan.level_fronts[h])
      if (f < 0 || f >= nf) return false;
    for (const AsmItem& it : plan.asm_items[h]) {
      if (it.front < 0 || it.front >= nf || it.nsrc < 0 || it.nsrc > 3) return false;
      const FrontD& f = plan.fronts[it.front];
      const int ld = f.m + f.u;
      if (it.nr < 1 || it.nc < 1 || it.dr < 0 || it.dc < 0 || it.dr + it.nr > ld + 1 ||
          it.dc + it.nc > ld)
        return false;
      for (int q = 0; q < it.nsrc; ++q) {
        const AsmSrc& S = it.src[q];
        const long long size = S.kind == 0 ? nblk : (S.kind == 1 ? plan.front_doubles : nN);
        if (S.kind < 0 || S.kind > 2 || !span_ok(S.so, it.nr, it.nc, S.rs, S.cs, size))
          return false;
      }
    }
    if (plan.upd_items[h].size() != plan.step_items[h].size()) return false;
    if ((int)plan.bw_items.size() != plan.nlevels) return false;
    if ((int)plan.schur_items.size() != plan.nlevels) return false;
    for (const SchurItem& it : plan.schur_items[h]) {
      if (it.front < 0 || it.front >= nf) return false;
      const FrontD& f = plan.fronts[it.front];
      const int T = it.wide ? kSB : kNB;
      if (f.u < 1 || (it.wide != 0 && it.wide != 1) || it.ti < 0 || it.tj < 0 || it.tj > it.ti ||
          T * it.ti > f.u || T * it.tj >= f.u)
        return false;
    }
    for (const BwItem& it : plan.bw_items[h])
      if (it.front < 0 || it.front >= nf || it.chunk < 0 || it.chunk >= plan.fronts[it.front].nzc)
        return false;
    for (const auto& items : plan.upd_items[h])
      for (const StepItem& it : items)
        if (it.tj < 0) return false;
    std::vector<const std::vector<StepItem>*> lists;
    for (const auto& items : plan.step_items[h]) lists.push_back(&items);
    for (const auto& items : plan.upd_items[h]) lists.push_back(&items);
    for (const auto* lp : lists)
      for (const StepItem& it : *lp) {
        if (it.front < 0 || it.front >= nf) return false;
        const FrontD& f = plan.fronts[it.front];
        if (it.tj <= -2) {
          // prefetch for tile ti of step panel + 1, chunk -2 - tj
          const int p = it.panel + 1, sc = -2 - it.tj;
          if (p < 2 || p >= f.npanels || sc >= f.pf_ns || it.ti < 0 || it.ti >= f.pf_nt ||
              sc * kPfPanels >= p - 1)
            return false;
          const int csp = p * kNB + std::min(kNB, f.m - p * kNB);
          if (csp + it.ti * kNB < f.m || csp + it.ti * kNB > f.m + f.u) return false;
          continue;
        }
        if (it.panel < 0 || it.panel >= f.npanels || it.ti < 0 || it.tj < -1 ||
            (it.tj >= 0 && it.tj > it.ti))
          return false;
        const int ld = f.m + f.u;
        const int cs = it.panel * kNB + std::min(kNB, f.m - it.panel * kNB);
        if (cs + it.ti * kNB > ld) return false;
        if (it.tj >= 0 && cs + it.tj * kNB >= ld) return false;
      }
  }
  return true;
}

// Trailing update of one tile (ti, tj >= 0) of a split panel step: both L
// tiles come from the L store written by the rows-only launch of the same
// step (the values the fused step forms itself), then F(ti,tj) -= L(ti)
// L(tj)^T; the workgroup of tile (0, 0) factors the next diagonal tile.
__global__ __launch_bounds__(256) void k_front_update(const StepItem* __restrict__ items,
                                                      const FrontD* __restrict__ fronts,
                                                      double* __restrict__ F,
                                                      const double* __restrict__ Lb,
                                                      double* __restrict__ Inv, int* status,
                                                      const int* __restrict__ active) {
  // two tiles: L(ti) and L(tj); the product is staged in the first once
  // both are consumed, and the look-ahead factorization works in both
  __shared__ Tile S0[kNB];
  __shared__ Tile S1[kNB];
  __shared__ TileAux aux;
  Tile* S2 = S1;
  const StepItem it = items[xcd_item(blockIdx.x, gridDim.x)];
  const FrontD f = fronts[it.front];
  if (active && !active[f.member]) return;
  const long long ld = f.m + f.u, lda = ld + 1;
  double* Fp = F + f.off;
  const int c0 = it.panel * kNB, nb = min(kNB, f.m - c0), cs = c0 + nb;
  const int R0 = cs + it.ti * kNB, nr = (int)min((long long)kNB, lda - R0);
  const int C0 = cs + it.tj * kNB, ncl = min(kNB, f.m - C0);   // S columns only
  const bool diag = it.tj == it.ti;
  const double* Lp = Lb + lpanel_base(f, it.panel);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, r = lane & 15, q = lane >> 4;
  // loads: the F tile (kept in registers) and both L tiles (row-major rows of
  // the L store, kNB doubles each), all issued before the first LDS store
  double fold[16], la[16], lb[16];
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int idx = tid + 256 * p;
    const int i = idx & 63, k = idx >> 6;
    fold[p] = (i < nr && k < ncl) ? Fp[(R0 + i) + (long long)(C0 + k) * lda] : 0.0;
    const int li = idx >> 6, lk = idx & 63;
    la[p] = (li < nr && lk < nb) ? Lp[(long long)(R0 - cs + li) * kNB + lk] : 0.0;
    lb[p] = (!diag && li < ncl && lk < nb) ? Lp[(long long)(C0 - cs + li) * kNB + lk] : 0.0;
  }
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int idx = tid + 256 * p;
    S1[idx >> 6][idx & 63] = la[p];
    S0[idx >> 6][idx & 63] = lb[p];
  }
  __syncthreads();
  const Tile* Bt = diag ? S1 : S0;
  // U = L(ti) L(tj)^T: wave w forms row block w
  d4 u[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) u[cb] = d4{0.0, 0.0, 0.0, 0.0};
  const int nc = (nb + 3) >> 2;
  for (int c = 0; c < nc; ++c) {
    const double a = S1[16 * w + r][4 * c + q];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) u[cb] = mfma16(a, Bt[16 * cb + r][4 * c + q], u[cb]);
  }
  __syncthreads();   // every wave is done with both L tiles
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int v = 0; v < 4; ++v) S2[16 * w + q + 4 * v][16 * cb + r] = u[cb][v];
  __syncthreads();
  const bool ahead = it.ti == 0 && it.tj == 0 && it.panel + 1 < f.npanels;
  const int nb1 = ahead ? min(kNB, f.m - cs) : 0;
  for (int p = 0; p < 16; ++p) {
    const int idx = tid + 256 * p;
    const int i = idx & 63, k = idx >> 6;
    const double nv = fold[p] - S2[i][k];
    if (i < nr && k < ncl) Fp[(R0 + i) + (long long)(C0 + k) * lda] = nv;
    if (ahead) S0[i][k] = (i < nb1 && k < nb1) ? nv : (i == k ? 1.0 : 0.0);
  }
  if (!ahead) return;
  __syncthreads();
  tile_factor_inv(S0, S1, aux, Inv + f.inv_off + (long long)(it.panel + 1) * kNB * kNB, nb1,
                  status);
}

// Deferred Schur complement of one front, one 64 x 64 output tile per
// workgroup: F(R, C) -= sum_k L(R, k) L(C, k) over the m columns of S, rows R
// of U and the right-hand-side row, columns C of U, the product accumulated
// on FP64 MFMA over the front's panels (L tiles from the panel-major store,
// the next panel's loads in flight during the current panel's products),
// then one read-modify-write of the tile.
// Wide tile (kSB x kSB): wave (wr, wc) forms rows 64 wr.., columns 64 wc..
// of the tile from L rows staged 16 columns at a time; after the products the
// same memory stages U, 32 columns at a time, for a coalesced
// read-modify-write of the front.  Two workgroups per CU (the accumulators of
// a wave's 64 x 64 block take 128 registers, the next stage's loads 32).
__device__ __forceinline__ void schur_wide(const SchurItem& it, const FrontD& f, double* F,
                                           const double* __restrict__ Lb, double* Sbuf) {
  constexpr int KC = 16, SPP = kNB / KC;   // stages per full panel
  constexpr int UC = 32;   // columns of U per pass of the read-modify-write
  static_assert(kSB * (UC + 1) <= 2 * kSB * (KC + 1), "U staging fits");
  double(*SA)[KC + 1] = reinterpret_cast<double(*)[KC + 1]>(Sbuf);
  double(*SB)[KC + 1] = reinterpret_cast<double(*)[KC + 1]>(Sbuf + kSB * (KC + 1));
  double(*SU)[UC + 1] = reinterpret_cast<double(*)[UC + 1]>(Sbuf);
  const long long ld = f.m + f.u, lda = ld + 1;
  double* Fp = F + f.off;
  const int m = f.m;
  const int R0 = m + it.ti * kSB, nr = (int)min((long long)kSB, lda - R0);
  const int C0 = m + it.tj * kSB, ncl = (int)min((long long)kSB, ld - C0);
  const bool diag = it.ti == it.tj;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, r = lane & 15, q = lane >> 4;
  // wave (wr, wc) forms rows 64 wr.., columns 64 wc.. of the tile; on a
  // diagonal tile the block above the diagonal is not formed
  const int wr = w >> 1, wc = w & 1;
  const bool idle = diag && wr < wc;
  // stage c: panel c / SPP, columns KC (c % SPP) .. of it (the last panel
  // has as many stages as it has columns to cover)
  const int nb_last = m - (f.npanels - 1) * kNB;
  const int nst = SPP * (f.npanels - 1) + (nb_last + KC - 1) / KC;
  constexpr int NL = kSB * KC / 256;   // loads per thread and block per stage
  double la[NL], lb[NL];
  auto load = [&](int c) {
    const int b = c / SPP, k0 = KC * (c % SPP);
    const int c0 = b * kNB, nb = min(kNB, m - c0), cs = c0 + nb;
    const double* Lp = Lb + lpanel_base(f, b);
#pragma unroll
    for (int e = 0; e < NL; ++e) {
      const int idx = tid + 256 * e, li = idx / KC, k = k0 + idx % KC;
      la[e] = (li < nr && k < nb) ? Lp[(long long)(R0 - cs + li) * kNB + k] : 0.0;
      lb[e] = (!diag && li < ncl && k < nb) ? Lp[(long long)(C0 - cs + li) * kNB + k] : 0.0;
    }
  };
  d4 acc[4][4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = d4{0.0, 0.0, 0.0, 0.0};
  load(0);
  for (int c = 0; c < nst; ++c) {
    if (c > 0) __syncthreads();   // every wave is done with the previous stage
#pragma unroll
    for (int e = 0; e < NL; ++e) {
      const int idx = tid + 256 * e;
      SA[idx / KC][idx % KC] = la[e];
      SB[idx / KC][idx % KC] = lb[e];
    }
    __syncthreads();
    if (c + 1 < nst) load(c + 1);
    if (!idle) {
      const int nb = min(kNB, m - (c / SPP) * kNB), kk = min(KC, nb - KC * (c % SPP));
      const int nk = (kk + 3) >> 2;
      double(*Bt)[KC + 1] = diag ? SA : SB;
      for (int s4 = 0; s4 < nk; ++s4) {
        double a[4], bv[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) a[rb] = SA[64 * wr + 16 * rb + r][4 * s4 + q];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) bv[cb] = Bt[64 * wc + 16 * cb + r][4 * s4 + q];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = mfma16(a[rb], bv[cb], acc[rb][cb]);
      }
    }
  }
  // F(R0 + i, C0 + col) -= U(i, col), 32 columns per pass through SU: pass
  // pc takes column blocks 2 (pc % 2) and 2 (pc % 2) + 1 of the waves wc = pc / 2
#pragma unroll
  for (int pc = 0; pc < kSB / UC; ++pc) {
    if (UC * pc >= ncl) break;
    __syncthreads();   // the stage buffers (or the previous pass's SU) are free
    if (wc == (pc >> 1) && !idle) {
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const d4 a4 = (pc & 1) ? acc[rb][2 + h] : acc[rb][h];
            SU[64 * wr + 16 * rb + q + 4 * v][16 * h + r] = a4[v];
          }
    }
    __syncthreads();
    double fold[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int idx = tid + 256 * e, i = idx & (kSB - 1), col = UC * pc + (idx >> 7);
      const bool ok = i < nr && col < ncl && !(diag && i < kNB && col >= kNB);
      fold[e] = ok ? Fp[(R0 + i) + (long long)(C0 + col) * lda] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int idx = tid + 256 * e, i = idx & (kSB - 1), kc = idx >> 7, col = UC * pc + kc;
      const bool ok = i < nr && col < ncl && !(diag && i < kNB && col >= kNB);
      if (ok) Fp[(R0 + i) + (long long)(C0 + col) * lda] = fold[e] - SU[i][kc];
    }
  }
}

// Narrow tile (kNB x kNB): wave w forms row block w; the L rows of the tile's
// row and column blocks staged a panel at a time, the next panel's loads in
// flight during the products.
__device__ __forceinline__ void schur_narrow(const SchurItem& it, const FrontD& f, double* F,
                                             const double* __restrict__ Lb, double* Sbuf) {
  Tile* SA = reinterpret_cast<Tile*>(Sbuf);
  Tile* SB = reinterpret_cast<Tile*>(Sbuf + kNB * (kNB + 1));
  const long long ld = f.m + f.u, lda = ld + 1;
  double* Fp = F + f.off;
  const int m = f.m;
  const int R0 = m + it.ti * kNB, nr = (int)min((long long)kNB, lda - R0);
  const int C0 = m + it.tj * kNB, ncl = (int)min((long long)kNB, ld - C0);
  const bool diag = it.ti == it.tj;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, r = lane & 15, q = lane >> 4;
  double la[16], lb[16];
  auto load = [&](int b) {
    const int c0 = b * kNB, nb = min(kNB, m - c0), cs = c0 + nb;
    const double* Lp = Lb + lpanel_base(f, b);
#pragma unroll
    for (int p = 0; p < 16; ++p) {
      const int idx = tid + 256 * p, li = idx >> 6, lk = idx & 63;
      la[p] = (li < nr && lk < nb) ? Lp[(long long)(R0 - cs + li) * kNB + lk] : 0.0;
      lb[p] = (!diag && li < ncl && lk < nb) ? Lp[(long long)(C0 - cs + li) * kNB + lk] : 0.0;
    }
  };
  d4 acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = d4{0.0, 0.0, 0.0, 0.0};
  load(0);
  for (int b = 0; b < f.npanels; ++b) {
    if (b > 0) __syncthreads();   // every wave is done with the previous tiles
#pragma unroll
    for (int p = 0; p < 16; ++p) {
      const int idx = tid + 256 * p;
      SA[idx >> 6][idx & 63] = la[p];
      SB[idx >> 6][idx & 63] = lb[p];
    }
    __syncthreads();
    if (b + 1 < f.npanels) load(b + 1);
    const Tile* Bt = diag ? SA : SB;
    const int nc = (min(kNB, m - b * kNB) + 3) >> 2;
    for (int c = 0; c < nc; ++c) {
      const double a = SA[16 * w + r][4 * c + q];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[cb] = mfma16(a, Bt[16 * cb + r][4 * c + q], acc[cb]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int v = 0; v < 4; ++v) SA[16 * w + q + 4 * v][16 * cb + r] = acc[cb][v];
  __syncthreads();
  double fold[16];
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int idx = tid + 256 * p, i = idx & 63, k = idx >> 6;
    fold[p] = (i < nr && k < ncl) ? Fp[(R0 + i) + (long long)(C0 + k) * lda] : 0.0;
  }
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int idx = tid + 256 * p, i = idx & 63, k = idx >> 6;
    if (i < nr && k < ncl) Fp[(R0 + i) + (long long)(C0 + k) * lda] = fold[p] - SA[i][k];
  }
}

__global__ __launch_bounds__(256, 2) void k_front_schur(const SchurItem* __restrict__ items,
                                                     const FrontD* __restrict__ fronts,
                                                     double* __restrict__ F,
                                                     const double* __restrict__ Lb,
                                                     const int* __restrict__ active) {
  constexpr int NW = 2 * kSB * (16 + 1), NN = 2 * kNB * (kNB + 1);
  __shared__ double Sbuf[NW > NN ? NW : NN];
  const SchurItem it = items[xcd_item(blockIdx.x, gridDim.x)];
  const FrontD f = fronts[it.front];
  if (active && !active[f.member]) return;
  if (it.wide)
    schur_wide(it, f, F, Lb, Sbuf);
  else
    schur_narrow(it, f, F, Lb, Sbuf);
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
  dev.upd_items.assign(H, {});
  for (int h = 0; h < H; ++h) {
    if (!upload(plan.asm_items[h], &dev.asm_items[h], b) ||
        !upload(plan.level_fronts[h], &dev.level_fronts[h], b))
      return false;
    dev.step_items[h].assign(plan.step_items[h].size(), nullptr);
    dev.upd_items[h].assign(plan.step_items[h].size(), nullptr);
    for (size_t p = 0; p < plan.step_items[h].size(); ++p)
      if (!upload(plan.step_items[h][p], &dev.step_items[h][p], b) ||
          !upload(plan.upd_items[h][p], &dev.upd_items[h][p], b))
        return false;
  }
  dev.bw_items.assign(H, nullptr);
  dev.schur_items.assign(H, nullptr);
  for (int h = 0; h < H; ++h)
    if (!upload(plan.bw_items[h], &dev.bw_items[h], b) ||
        !upload(plan.schur_items[h], &dev.schur_items[h], b))
      return false;
  if (!upload(plan.urow_pn, &dev.urow_pn, b) || !upload(plan.rboxes, &dev.rboxes, b) ||
      !upload(plan.rnbs, &dev.rnbs, b))
    return false;
  int maxld = 1;
  for (auto& f : plan.fronts) maxld = std::max(maxld, f.m + f.u);
  if (hipFuncSetAttribute((const void*)k_front_backward, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(sizeof(double) * maxld)) != hipSuccess ||
      hipFuncSetAttribute((const void*)k_front_forward, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(sizeof(double) * maxld)) != hipSuccess)
    return false;
  auto alloc = [&](double** p, long long n) {
    if (hipMalloc(p, std::max<long long>(n, 1) * sizeof(double)) != hipSuccess) return false;
    b += n * (long long)sizeof(double);
    return hipMemset(*p, 0, std::max<long long>(n, 1) * sizeof(double)) == hipSuccess;
  };
  return alloc(&dev.F, plan.front_doubles) && alloc(&dev.L, plan.lpan_doubles) &&
         alloc(&dev.V, plan.vec_doubles) && alloc(&dev.Inv, plan.inv_doubles) &&
         alloc(&dev.part, plan.bw_part_doubles) && alloc(&dev.pf, plan.pf_doubles) &&
         alloc(&dev.res, plan.nN) &&
         alloc(&dev.cor, plan.nN);
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
  for (auto& v : dev.upd_items)
    for (auto p : v) f(p);
  for (auto p : dev.bw_items) f(p);
  for (auto p : dev.schur_items) f(p);
  f(dev.urow_pn);
  f(dev.rboxes);
  f(dev.rnbs);
  f(dev.res);
  f(dev.cor);
  f(dev.part);
  f(dev.pf);
  f(dev.F);
  f(dev.L);
  f(dev.V);
  f(dev.Inv);
  dev = SolverDev{};
}

// Backward substitution from the root down: x = L^{-T} y with y the
// factorization's right-hand-side rows (ysrc = nullptr) or a forward
// substitution's vectors; x into pN, and added to padd when given.
static void backward_sweep(const SolverPlan& plan, const SolverDev& dev, const double* ysrc,
                           double* pN, double* padd, hipStream_t st, const int* active) {
  const int H = plan.nlevels;
  for (int h = H - 1; h >= 0; --h) {
    const int n = (int)plan.level_fronts[h].size();
    int maxld = 0;
    for (int f : plan.level_fronts[h])
      maxld = std::max(maxld, plan.fronts[f].m + plan.fronts[f].u);
    const int nbw = (int)plan.bw_items[h].size();
    if (nbw) {
      ktimer_begin(KK_FRONT_BW_GEMV, st);
      hipLaunchKernelGGL(k_front_bw_gemv, dim3(nbw), dim3(256), 0, st, dev.bw_items[h],
                         dev.fronts, dev.L, dev.urow_pn, pN, dev.part, active);
      ktimer_end(plan.bwg_flops[h], plan.bwg_bytes[h], st);
    }
    ktimer_begin(KK_FRONT_BACKWARD, st);
    hipLaunchKernelGGL(k_front_backward, dim3(n), dim3(kBwT), sizeof(double) * maxld, st,
                       dev.level_fronts[h], dev.fronts, dev.nodes, dev.L, dev.Inv, dev.part, ysrc,
                       pN, padd, active);
    ktimer_end(plan.bw_flops[h], plan.bw_bytes[h], st);
  }
}

hipError_t solver_factor_solve(const SolverPlan& plan, const SolverDev& dev,
                               const double* blocks, const double* fN, double* pN, int* status,
                               hipStream_t st, int refine, const int* active,
                               const int* ref_masks, int mstride) {
  const int H = plan.nlevels;
  for (int h = 0; h < H; ++h) {
    const int na = (int)plan.asm_items[h].size();
    const int nf = (int)plan.level_fronts[h].size();
    ktimer_begin(KK_FRONT_ASM, st);
    hipLaunchKernelGGL(k_front_asm, dim3(na), dim3(256), 0, st, dev.asm_items[h], dev.fronts,
                       blocks, fN, dev.F, active);
    ktimer_end(plan.asm_flops[h], plan.asm_bytes[h], st);
    ktimer_begin(KK_FRONT_FACTOR0, st);
    hipLaunchKernelGGL(k_front_factor0, dim3(nf), dim3(256), 0, st, dev.level_fronts[h],
                       dev.fronts, dev.F, dev.Inv, status, active);
    ktimer_end(plan.f0_flops[h], plan.f0_bytes[h], st);
    for (size_t p = 0; p < plan.step_items[h].size(); ++p) {
      const int ni = (int)plan.step_items[h][p].size();
      if (ni) {
        ktimer_begin(KK_FRONT_STEP, st);
        hipLaunchKernelGGL(k_front_step, dim3(ni), dim3(256), 0, st, dev.step_items[h][p],
                           dev.fronts, dev.F, dev.L, dev.Inv, status, dev.pf, active);
        ktimer_end(plan.step_flops[h][p], plan.step_bytes[h][p], st);
      }
      const int nu = (int)plan.upd_items[h][p].size();
      if (nu) {
        ktimer_begin(KK_FRONT_UPDATE, st);
        hipLaunchKernelGGL(k_front_update, dim3(nu), dim3(256), 0, st, dev.upd_items[h][p],
                           dev.fronts, dev.F, dev.L, dev.Inv, status, active);
        ktimer_end(plan.upd_flops[h][p], plan.upd_bytes[h][p], st);
      }
    }
    const int ns = (int)plan.schur_items[h].size();
    if (ns) {
      ktimer_begin(KK_FRONT_SCHUR, st);
      hipLaunchKernelGGL(k_front_schur, dim3(ns), dim3(256), 0, st, dev.schur_items[h], dev.fronts,
                         dev.F, dev.L, active);
      ktimer_end(plan.schur_flops[h], plan.schur_bytes[h], st);
    }
  }
  backward_sweep(plan, dev, nullptr, pN, nullptr, st, active);
  const int nbox = (int)plan.rboxes.size();
  for (int it = 0; it < std::min(refine, kMaxRefine) && nbox > 0; ++it) {
    const int* am = ref_masks ? ref_masks + (long long)it * mstride : active;
    ktimer_begin(KK_RESIDUAL, st);
    hipLaunchKernelGGL(k_residual, dim3(nbox), dim3(256), 0, st, dev.rboxes, dev.rnbs, blocks, fN,
                       pN, dev.res, status, am);
    ktimer_end(plan.res_flops, plan.res_bytes, st);
    for (int h = 0; h < H; ++h) {
      const int n = (int)plan.level_fronts[h].size();
      int maxld = 0;
      for (int f : plan.level_fronts[h])
        maxld = std::max(maxld, plan.fronts[f].m + plan.fronts[f].u);
      ktimer_begin(KK_FRONT_FORWARD, st);
      hipLaunchKernelGGL(k_front_forward, dim3(n), dim3(256), sizeof(double) * maxld, st,
                         dev.level_fronts[h], dev.fronts, dev.nodes, dev.children, dev.L, dev.Inv,
                         dev.res, dev.V, am);
      ktimer_end(plan.fw_flops[h], plan.fw_bytes[h], st);
      const int nbw = (int)plan.bw_items[h].size();
      if (nbw) {
        ktimer_begin(KK_FRONT_FW_GEMV, st);
        hipLaunchKernelGGL(k_front_fw_gemv, dim3(nbw), dim3(256), 0, st, dev.bw_items[h],
                           dev.fronts, dev.L, dev.V, am);
        ktimer_end(plan.bwg_flops[h], plan.bwg_bytes[h], st);
      }
    }
    backward_sweep(plan, dev, dev.V, dev.cor, pN, st, am);
  }
  return hipGetLastError();
}

}  // namespace lrbms
