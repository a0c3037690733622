// Discrete SWIP operator of Def. pressureDG on one cell, templated on the
// dimension so that every per-dof array stays in registers: face terms,
// face moments of the mobility, the right-hand side l_h, and the r x r
// stencil blocks of a cell (self block and one block per face neighbour).
// Shared by the online reduced assembly and the offline fine solves.
#pragma once

#include "common.h"

namespace lrbms {

// ---------------------------------------------------------------------------
// Face terms of b_h (Def. pressureDG) on the face of axis A of a test cell,
// for one trial function given by its coefficients on the test cell (ps) and
// on the cell across the face (po):
//   -int {gamma kappa d_n v}[w] - int {gamma kappa d_n w}[v] + sigma_f/h_f int [v][w].
// alpha = +1: the face is on the +A side of the test cell (the test cell is
// the low-side cell); on a boundary face alpha is the sign of the outward
// normal, weight 1 and sigma_f = penalty * kappa.  ms / mo: int_f gamma and
// int_f gamma xi_t (tangential axes t in increasing order) from the test side
// / the other side.  Adds the r test rows to Y.
template <int D, int A>
__device__ __forceinline__ void face_terms(const Geom& g, double alpha, bool interior, double ks,
                                           double ko, const double (&ms)[D], const double (&mo)[D],
                                           const double (&ps)[D + 1], const double (&po)[D + 1],
                                           bool gam, bool pen, double (&Y)[D + 1]) {
  constexpr int NT = D - 1;
  constexpr int TX[2] = {(A == 0) ? 1 : 0, (A == 2) ? 1 : 2};   // tangential axes
  const double isv = g.isv;
  const double gf = kSqrt3 * 2.0 / g.h[A] * isv;
  const double as = alpha, ao = -alpha;
  double js, jo, ws, wo, sig, nd;
  if (interior) {
    js = alpha;
    jo = -alpha;
    const double klo = alpha > 0 ? ks : ko, khi = alpha > 0 ? ko : ks;
    double wlo, whi;
    if (g.weights == 0) {
      wlo = khi / (klo + khi);
      whi = klo / (klo + khi);
    } else {
      wlo = klo / (klo + khi);
      whi = khi / (klo + khi);
    }
    ws = alpha > 0 ? wlo : whi;
    wo = alpha > 0 ? whi : wlo;
    sig = g.pen * 2.0 * klo * khi / (klo + khi);
    nd = gf;
  } else {
    js = 1.0;
    jo = 0.0;
    ws = 1.0;
    wo = 0.0;
    sig = g.pen * ks;
    nd = alpha * gf;
  }
  if (gam) {
    // trial normal derivative against the test trace
    const double cs = ws * ks * nd * ps[A + 1];
    const double cq = interior ? wo * ko * nd * po[A + 1] : 0.0;
    const double A0 = cs * ms[0] + (interior ? cq * mo[0] : 0.0);
    Y[0] -= js * isv * A0;
    Y[A + 1] -= js * isv * kSqrt3 * as * A0;
#pragma unroll
    for (int ti = 0; ti < NT; ++ti) {
      const double At = cs * ms[1 + ti] + (interior ? cq * mo[1 + ti] : 0.0);
      Y[TX[ti] + 1] -= js * isv * kSqrt3 * At;
    }
    // test normal derivative against the trial jump
    double jm = js * (ps[0] * ms[0] + kSqrt3 * as * ps[A + 1] * ms[0]);
#pragma unroll
    for (int ti = 0; ti < NT; ++ti) jm += js * kSqrt3 * ps[TX[ti] + 1] * ms[1 + ti];
    if (interior) {
      jm += jo * (po[0] * ms[0] + kSqrt3 * ao * po[A + 1] * ms[0]);
#pragma unroll
      for (int ti = 0; ti < NT; ++ti) jm += jo * kSqrt3 * po[TX[ti] + 1] * ms[1 + ti];
    }
    Y[A + 1] -= ws * ks * nd * isv * jm;
  }
  if (pen) {
    const double P = sig / g.hf[A] * (isv * isv) * g.area[A] * js;
    double J0 = js * (ps[0] + kSqrt3 * as * ps[A + 1]);
    if (interior) J0 += jo * (po[0] + kSqrt3 * ao * po[A + 1]);
    Y[0] += P * J0;
    Y[A + 1] += P * kSqrt3 * as * J0;
#pragma unroll
    for (int ti = 0; ti < NT; ++ti) {
      const int t = TX[ti] + 1;
      Y[t] += P * (js * ps[t] + (interior ? jo * po[t] : 0.0));
    }
  }
}

template <int D>
__device__ __forceinline__ void face_moments(const Geom& g, const double* __restrict__ mom, int c,
                                             int a, int dir, double (&m)[D]) {
  const int s = mom_slot(D, a, dir);
#pragma unroll
  for (int q = 0; q < D; ++q) m[q] = mom[(long long)(s + q) * g.ncell + c];
}

// l_h(phi_k) of test cell e (eq. rhsP: sources, Neumann data with the minus
// sign, Dirichlet penalty and consistency terms).
template <int D>
__device__ __forceinline__ void cell_rhs(const Geom& g, int e, const int (&x)[3],
                                         const double* __restrict__ mom, int parts,
                                         double (&Y)[D + 1]) {
  if (parts & PART_RHS_CONST) Y[0] += g.q1[e] * g.vol * g.isv;
#pragma unroll
  for (int a = 0; a < D; ++a) {
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
      const int xa = x[a] + (dir ? 1 : -1);
      if (xa >= 0 && xa < g.n[a]) continue;
      int xf[3] = {x[0], x[1], x[2]};
      xf[a] += dir;
      const int fid = face_index(g, a, xf);
      const int bt = g.bc_type[fid];
      const double val = g.bc_val[fid];
      const double al = dir ? 1.0 : -1.0;
      const double tw0 = g.area[a] * g.isv, twa = tw0 * kSqrt3 * al;   // int_f phi_0, phi_{a+1}
      if (bt == LRBMS_BC_NEUMANN && (parts & PART_RHS_CONST)) {
        Y[0] -= val * tw0;
        Y[a + 1] -= val * twa;
      } else if (bt == LRBMS_BC_DIRICHLET) {
        if (parts & PART_RHS_CONST) {
          const double sg = g.pen * g.perm[e] / g.hf[a];
          Y[0] += sg * val * tw0;
          Y[a + 1] += sg * val * twa;
        }
        if (parts & PART_RHS_GAMMA) {
          const double gf = kSqrt3 * 2.0 / g.h[a] * g.isv;
          const double m0 = mom[(long long)mom_slot(D, a, dir) * g.ncell + e];
          Y[a + 1] -= val * g.perm[e] * m0 * (al * gf);
        }
      }
    }
  }
}

// Column kp of the r x r blocks of the fine operator at test cell e: the self
// block (volume term and the own-side terms of every face) and, per face
// (index 2a + dir), the block against the trial dofs of the neighbour across
// it (zero when the neighbour is outside the box or the face is on the
// boundary).  Faces are visited in the order (a, dir) = (0,-), (0,+), (1,-) ...
template <int D, int A>
__device__ __forceinline__ void stencil_axis(const Geom& g, const Sub& S, int e,
                                             const int (&x)[3], double ke,
                                             const double* __restrict__ mom, bool gam, bool pen,
                                             const double (&unit)[D + 1], double (&self)[D + 1],
                                             double (&nbr)[2 * D][D + 1]) {
  const double zero[D + 1] = {};
#pragma unroll
  for (int dir = 0; dir < 2; ++dir) {
    double (&nb)[D + 1] = nbr[2 * A + dir];
#pragma unroll
    for (int k = 0; k <= D; ++k) nb[k] = 0.0;
    double ms[D];
    face_moments<D>(g, mom, e, A, dir, ms);
    int xn[3] = {x[0], x[1], x[2]};
    xn[A] += dir ? 1 : -1;
    const double alpha = dir ? 1.0 : -1.0;
    if (xn[A] >= 0 && xn[A] < g.n[A]) {
      const int en = cell_index(g, xn);
      double mo[D];
      face_moments<D>(g, mom, en, A, 1 - dir, mo);
      const double ko = g.perm[en];
      face_terms<D, A>(g, alpha, true, ke, ko, ms, mo, unit, zero, gam, pen, self);
      if (xn[A] >= S.lo[A] && xn[A] < S.hi[A])
        face_terms<D, A>(g, alpha, true, ke, ko, ms, mo, zero, unit, gam, pen, nb);
    } else {
      int xf[3] = {x[0], x[1], x[2]};
      xf[A] += dir;
      if (g.bc_type[face_index(g, A, xf)] == LRBMS_BC_DIRICHLET)
        face_terms<D, A>(g, alpha, false, ke, 0.0, ms, ms, unit, zero, gam, pen, self);
    }
  }
}

template <int D>
__device__ __forceinline__ void cell_stencil(const Geom& g, const Sub& S, int e, const int (&x)[3],
                                             const double* __restrict__ mom, int parts, int kp,
                                             double (&self)[D + 1], double (&nbr)[2 * D][D + 1]) {
  const bool gam = parts & PART_GAMMA, pen = parts & PART_PEN;
  double unit[D + 1];
#pragma unroll
  for (int k = 0; k <= D; ++k) {
    unit[k] = (k == kp) ? 1.0 : 0.0;
    self[k] = 0.0;
  }
  const double ke = g.perm[e];
  if (gam) {
    const double mv = mom[e];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double gf = kSqrt3 * 2.0 / g.h[a] * g.isv;
      self[a + 1] += ke * mv * (gf * gf) * unit[a + 1];
    }
  }
  stencil_axis<D, 0>(g, S, e, x, ke, mom, gam, pen, unit, self, nbr);
  stencil_axis<D, 1>(g, S, e, x, ke, mom, gam, pen, unit, self, nbr);
  if constexpr (D == 3) stencil_axis<D, 2>(g, S, e, x, ke, mom, gam, pen, unit, self, nbr);
}

}  // namespace lrbms
