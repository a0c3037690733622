// Fine-grid kernels of the online step on gfx950:
//   pressure reconstruction p_h = sum_i (p_N)_i phi_i      (Alg. 3 step 5b)
//   face fluxes of the conservative velocity              (Def. velocityDG)
//   DG upwind explicit Euler saturation step              (Def. saturationDG)
//   slope limiter                                         (eq. limiterMain)
// and the matrix-free fine SWIP operator used by the offline snapshot solves.
//
// Readings (same as the CPU reference): RT0 on rectangles (one normal flux per
// face, u_a linear in x_a only); v_N |f| as the flux on Neumann faces; upwind
// trace taken from the low-side cell when the flux along +axis is >= 0; s_D on
// saturation Dirichlet faces, the interior trace on other boundary faces;
// shock detector with |int_f [s]| over inflow faces; the limited state keeps
// the cell mean and scales the slope by min_i m_i; 2-point Gauss rules.
//
// All kernels are one thread per cell or per face with x-fastest indexing, so
// neighbouring threads touch neighbouring addresses of the SoA arrays.
#include "common.h"
#include "ktimer.h"

namespace lrbms {

__device__ __forceinline__ double p1_value(const double* co, int d, const double sq[3], double isv) {
  double v = co[0];
  for (int a = 0; a < d; ++a) v += sq[a] * co[a + 1];
  return v * isv;
}

// ---------------------------------------------------------------------------
// p_h on the cells of one tile (box, first cell): coalesced over cells.
// Eight basis functions per pass: their 8 r coefficients and p_N entries are
// loaded before the multiply-adds (indices past N_E are clamped and their
// weight set to zero).
template <int D>
__global__ __launch_bounds__(256) void k_reconstruct(Geom g, const Sub* __restrict__ subs,
                                                     const int* __restrict__ tiles,
                                                     const double* __restrict__ phi,
                                                     const double* __restrict__ pN,
                                                     double* __restrict__ ph) {
  constexpr int R = D + 1, U = 8;
  const int sub = tiles[2 * blockIdx.x], c0 = tiles[2 * blockIdx.x + 1];
  const Sub S = subs[sub];
  const int l = c0 + threadIdx.x;
  if (l >= S.nE) return;
  const int bx = S.hi[0] - S.lo[0], by = S.hi[1] - S.lo[1];
  const int x[3] = {S.lo[0] + l % bx, S.lo[1] + (l / bx) % by, S.lo[2] + l / (bx * by)};
  const int e = cell_index(g, x);
  double acc[R];
#pragma unroll
  for (int k = 0; k < R; ++k) acc[k] = 0.0;
  const double* base = phi + S.phi_off + l;
  const long long cs = (long long)R * S.nE;
  for (int i0 = 0; i0 < S.NE; i0 += U) {
    double v[U][R], pv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = min(i0 + u, S.NE - 1);
      pv[u] = pN[S.pn_off + i];
#pragma unroll
      for (int k = 0; k < R; ++k) v[u][k] = base[i * cs + (long long)k * S.nE];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double p = (i0 + u < S.NE) ? pv[u] : 0.0;
#pragma unroll
      for (int k = 0; k < R; ++k) acc[k] += v[u][k] * p;
    }
  }
#pragma unroll
  for (int k = 0; k < R; ++k) ph[(long long)k * g.ncell + e] = acc[k];
}

hipError_t launch_reconstruct(const Geom& g, const Sub* d_subs, int n_sub, const int* d_tiles,
                              int n_tiles, const double* phi, const double* pN, double* ph,
                              hipStream_t st) {
  (void)n_sub;
  ktimer_begin(KK_RECONSTRUCT, st);
  if (g.dim == 2)
    hipLaunchKernelGGL(k_reconstruct<2>, dim3(n_tiles), dim3(256), 0, st, g, d_subs, d_tiles, phi,
                       pN, ph);
  else
    hipLaunchKernelGGL(k_reconstruct<3>, dim3(n_tiles), dim3(256), 0, st, g, d_subs, d_tiles, phi,
                       pN, ph);
  ktimer_end(-1.0, -1.0, st);
  return hipGetLastError();
}

// Decode a global face number: axis, face coordinates.
__device__ __forceinline__ void face_coords(const Geom& g, int fid, int& a, int x[3]) {
  a = (fid >= g.foff[2] && g.dim == 3) ? 2 : (fid >= g.foff[1] ? 1 : 0);
  int l = fid - g.foff[a];
  int e0 = g.n[0], e1 = g.n[1];
  if (a == 0) e0 += 1;
  if (a == 1) e1 += 1;
  x[0] = l % e0;
  x[1] = (l / e0) % e1;
  x[2] = l / (e0 * e1);
}

// Integral of the total mobility lambda(s) over the face of axis a at local
// coordinate xi_a of a cell with coefficients co (2-point Gauss in the
// tangential directions).
template <int D>
__device__ __forceinline__ double face_mobility_co(const Geom& g, const double (&co)[4], int a,
                                                   double xia) {
  int tax[2] = {0, 0}, nt = 0;
#pragma unroll
  for (int b = 0; b < D; ++b)
    if (b != a) tax[nt++] = b;
  const double gp = 1.0 / kSqrt3;
  double sum = 0.0;
#pragma unroll
  for (int p = 0; p < (1 << (D - 1)); ++p) {
    double sq[3] = {0, 0, 0};
    sq[a] = kSqrt3 * xia;
#pragma unroll
    for (int ti = 0; ti < D - 1; ++ti) sq[tax[ti]] = kSqrt3 * (((p >> ti) & 1) ? gp : -gp);
    sum += total_mobility(g, p1_value(co, D, sq, g.isv));
  }
  return sum * g.area[a] / (1 << (D - 1));
}

// One thread per face, templated on the dimension; the loads of both cells
// and of the face data are issued before the arithmetic.
template <int D>
__global__ __launch_bounds__(256) void k_flux(Geom g, const double* __restrict__ ph,
                                              const double* __restrict__ sat,
                                              double* __restrict__ flux) {
  constexpr int R = D + 1;
  const int fid = blockIdx.x * blockDim.x + threadIdx.x;
  if (fid >= g.nface) return;
  int a, x[3];
  face_coords(g, fid, a, x);
  const int nc = g.ncell;
  int xl[3] = {x[0], x[1], x[2]};
  xl[a] -= 1;
  const bool has_lo = x[a] >= 1, has_hi = x[a] < g.n[a];
  // cells on both sides (a boundary face uses its one cell twice)
  const int c0 = has_lo ? cell_index(g, xl) : cell_index(g, x);
  const int c1 = has_hi ? cell_index(g, x) : c0;
  double s0[4] = {0, 0, 0, 0}, s1[4] = {0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < R; ++k) {
    s0[k] = sat[(long long)k * nc + c0];
    s1[k] = sat[(long long)k * nc + c1];
  }
  const double k0 = g.perm[c0], k1 = g.perm[c1];
  const double p00 = ph[c0], p0a = ph[(long long)(a + 1) * nc + c0];
  const double p10 = ph[c1], p1a = ph[(long long)(a + 1) * nc + c1];
  const int bt = g.bc_type[fid];
  const double val = g.bc_val[fid];
  const double gf = kSqrt3 * 2.0 / g.h[a] * g.isv;
  if (has_lo && has_hi) {
    double w0, w1;
    if (g.weights == 0) {
      w0 = k1 / (k0 + k1);
      w1 = k0 / (k0 + k1);
    } else {
      w0 = k0 / (k0 + k1);
      w1 = k1 / (k0 + k1);
    }
    const double g0 = face_mobility_co<D>(g, s0, a, 1.0);
    const double g1 = face_mobility_co<D>(g, s1, a, -1.0);
    const double jump = g.area[a] * g.isv * ((p00 + kSqrt3 * p0a) - (p10 - kSqrt3 * p1a));
    const double sig = g.pen * 2.0 * k0 * k1 / (k0 + k1) / g.hf[a];
    flux[fid] = -(w0 * k0 * g0 * (gf * p0a) + w1 * k1 * g1 * (gf * p1a)) + sig * jump;
    return;
  }
  const double al = has_lo ? 1.0 : -1.0;           // outward normal sign
  double out = 0.0;
  if (bt == LRBMS_BC_NEUMANN) {
    out = val * g.area[a];
  } else if (bt == LRBMS_BC_DIRICHLET) {
    const double kc = k0;
    const double gm = face_mobility_co<D>(g, s0, a, al);
    const double p0 = p00, pa = p0a;
    const double sig = g.pen * kc / g.hf[a];
    const double trace = g.area[a] * g.isv * (p0 + kSqrt3 * al * pa);
    out = -kc * gm * (al * gf * pa) + sig * (trace - val * g.area[a]);
  }
  flux[fid] = al * out;
}

hipError_t launch_flux(const Geom& g, const double* ph, const double* sat, double* flux,
                       hipStream_t st) {
  ktimer_begin(KK_FLUX, st);
  if (g.dim == 2)
    hipLaunchKernelGGL(k_flux<2>, dim3((g.nface + 255) / 256), dim3(256), 0, st, g, ph, sat, flux);
  else
    hipLaunchKernelGGL(k_flux<3>, dim3((g.nface + 255) / 256), dim3(256), 0, st, g, ph, sat, flux);
  ktimer_end(-1.0, -1.0, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------

// One thread per cell, templated on the dimension; every load of the cell and
// its face neighbours (states, permeabilities, fluxes, boundary data) is
// issued before the arithmetic, so their latencies overlap.
template <int D>
__global__ __launch_bounds__(256) void k_transport(Geom g, const double* __restrict__ sat,
                                                   const double* __restrict__ flux,
                                                   double* __restrict__ out) {
  constexpr int R = D + 1, NF = 2 * D;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.ncell) return;
  const int nc = g.ncell;
  int x[3];
  cell_coords(g, e, x);
  // ---- loads
  double se[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < R; ++k) se[k] = sat[(long long)k * nc + e];
  const double q2 = g.q2[e], ke = g.perm[e], phi = g.poro[e];
  double F[NF], kn[NF], bsv[NF], sn[NF][4];
  int8_t bsd[NF];
  bool inter[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const int a = f >> 1, dir = f & 1;
    int xf[3] = {x[0], x[1], x[2]};
    xf[a] += dir;
    const int fid = face_index(g, a, xf);
    int xn[3] = {x[0], x[1], x[2]};
    xn[a] += dir ? 1 : -1;
    inter[f] = xn[a] >= 0 && xn[a] < g.n[a];
    const int en = inter[f] ? cell_index(g, xn) : e;   // boundary: a valid cell, unused
    F[f] = flux[fid];
    kn[f] = g.perm[en];
    bsd[f] = g.bc_sat[fid];
    bsv[f] = g.bc_sval[fid];
#pragma unroll
    for (int k = 0; k < 4; ++k) sn[f][k] = k < R ? sat[(long long)k * nc + en] : 0.0;
  }
  // ---- arithmetic
  double Rr[4] = {0.0, 0.0, 0.0, 0.0};
  Rr[0] += q2 * g.vol * g.isv;
  const double gp = 1.0 / kSqrt3;
  // volume term int_e u f_w(s) . grad v
  {
    constexpr int nq = 1 << D;
    double acc[3] = {0, 0, 0};
#pragma unroll
    for (int p = 0; p < nq; ++p) {
      double xi[3], sq[3];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        xi[a] = ((p >> a) & 1) ? gp : -gp;
        sq[a] = kSqrt3 * xi[a];
      }
      const double fw = frac_flow(g, p1_value(se, D, sq, g.isv));
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const double t = 0.5 * (1.0 + xi[a]);
        const double ua = ((1.0 - t) * F[2 * a] + t * F[2 * a + 1]) / g.area[a];
        acc[a] += ua * fw * (g.vol / nq);
      }
    }
#pragma unroll
    for (int a = 0; a < D; ++a) Rr[a + 1] += (kSqrt3 * 2.0 / g.h[a] * g.isv) * acc[a];
  }
  // face terms
#pragma unroll
  for (int a = 0; a < D; ++a) {
    int tax[2] = {0, 0}, nt = 0;
#pragma unroll
    for (int b = 0; b < D; ++b)
      if (b != a) tax[nt++] = b;
    constexpr int nq = 1 << (D - 1);
    const double wq = g.area[a] / nq;
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
      const int f = 2 * a + dir;
      const double Ff = F[f];
      const double al = dir ? 1.0 : -1.0;   // position of the face in this cell
      const bool interior = inter[f];
      const bool sd = !interior && bsd[f] == 1;
      const double sval = interior ? 0.0 : bsv[f];
      double sig;
      if (interior) {
        const double klo = dir ? ke : kn[f], khi = dir ? kn[f] : ke;
        sig = g.sat_pen * (g.pen * 2.0 * klo * khi / (klo + khi)) / g.hf[a];
      } else {
        sig = g.sat_pen * (g.pen * ke) / g.hf[a];
      }
      double acc[4] = {0, 0, 0, 0};
#pragma unroll
      for (int p = 0; p < nq; ++p) {
        double sqe[3] = {0, 0, 0}, sqn[3] = {0, 0, 0};
        double xt[2] = {0, 0};
        sqe[a] = kSqrt3 * al;
        sqn[a] = -kSqrt3 * al;
#pragma unroll
        for (int ti = 0; ti < D - 1; ++ti) {
          xt[ti] = ((p >> ti) & 1) ? gp : -gp;
          sqe[tax[ti]] = kSqrt3 * xt[ti];
          sqn[tax[ti]] = kSqrt3 * xt[ti];
        }
        const double ve = p1_value(se, D, sqe, g.isv);
        double tot;
        if (interior) {
          const double vn = p1_value(sn[f], D, sqn, g.isv);
          const double vlo = dir ? ve : vn, vhi = dir ? vn : ve;
          const double up = (Ff >= 0.0) ? vlo : vhi;
          tot = (Ff / g.area[a]) * frac_flow(g, up) + sig * (vlo - vhi);
        } else {
          const double fout = al * Ff;
          const double chi = sd ? sval : ve;
          tot = (fout / g.area[a]) * frac_flow(g, chi) + (sd ? sig * (ve - sval) : 0.0);
        }
        // test trace of this cell: isv * {1, sqrt3*al, sqrt3*xi_t}
        const double tw = tot * wq * g.isv;
        acc[0] += tw;
        acc[a + 1] += tw * kSqrt3 * al;
#pragma unroll
        for (int ti = 0; ti < D - 1; ++ti) acc[tax[ti] + 1] += tw * kSqrt3 * xt[ti];
      }
      // [v] = +v on the low-side cell (face on its +a side), -v on the high-side cell;
      // a boundary face has [v] = v
      const double jv = interior ? al : 1.0;
#pragma unroll
      for (int k = 0; k < R; ++k) Rr[k] -= jv * acc[k];
    }
  }
#pragma unroll
  for (int k = 0; k < R; ++k) out[(long long)k * nc + e] = se[k] + g.dt * Rr[k] / phi;
}

hipError_t launch_transport(const Geom& g, const double* sat, const double* flux, double* sat_bar,
                            hipStream_t st) {
  ktimer_begin(KK_TRANSPORT, st);
  if (g.dim == 2)
    hipLaunchKernelGGL(k_transport<2>, dim3((g.ncell + 255) / 256), dim3(256), 0, st, g, sat, flux,
                       sat_bar);
  else
    hipLaunchKernelGGL(k_transport<3>, dim3((g.ncell + 255) / 256), dim3(256), 0, st, g, sat, flux,
                       sat_bar);
  ktimer_end(-1.0, -1.0, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ double gradient_scale(double gi, double di) {
  const bool big = fabs(gi) > 1e-8 && fabs(di) > 1e-8;
  if (big && gi * di < 0.0) return 0.0;
  if (big && gi * di > 0.0 && fabs(gi) > fabs(di)) return di / gi;
  return 1.0;
}

// One thread per cell, templated on the dimension; the loads of the cell and
// its face neighbours are issued before the arithmetic.
template <int D>
__global__ __launch_bounds__(256) void k_limiter(Geom g, const double* __restrict__ sb,
                                                 const double* __restrict__ flux,
                                                 double* __restrict__ out,
                                                 uint8_t* __restrict__ flags) {
  constexpr int R = D + 1, NF = 2 * D;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.ncell) return;
  const int nc = g.ncell;
  int x[3];
  cell_coords(g, e, x);
  // ---- loads
  double se[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < R; ++k) se[k] = sb[(long long)k * nc + e];
  double F[NF], bsv[NF], sn[NF][4];
  int8_t bsd[NF];
  bool inter[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const int a = f >> 1, dir = f & 1;
    int xf[3] = {x[0], x[1], x[2]};
    xf[a] += dir;
    const int fid = face_index(g, a, xf);
    int xn[3] = {x[0], x[1], x[2]};
    xn[a] += dir ? 1 : -1;
    inter[f] = xn[a] >= 0 && xn[a] < g.n[a];
    const int en = inter[f] ? cell_index(g, xn) : e;   // boundary: a valid cell, unused
    F[f] = flux[fid];
    bsd[f] = g.bc_sat[fid];
    bsv[f] = g.bc_sval[fid];
#pragma unroll
    for (int k = 0; k < 4; ++k) sn[f][k] = (k < R && inter[f]) ? sb[(long long)k * nc + en] : 0.0;
  }
  // ---- arithmetic
  const double mean = se[0] * g.isv;
  bool outside = false;
#pragma unroll
  for (int p = 0; p < (1 << D); ++p) {
    double sq[3];
#pragma unroll
    for (int a = 0; a < D; ++a) sq[a] = ((p >> a) & 1) ? kSqrt3 : -kSqrt3;
    const double v = p1_value(se, D, sq, g.isv);
    if (v < 0.0 || v > 1.0) outside = true;
  }
  const double gp = 1.0 / kSqrt3;
  double S = 0.0, mmin = 1.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    int tax[2] = {0, 0}, nt = 0;
#pragma unroll
    for (int b = 0; b < D; ++b)
      if (b != a) tax[nt++] = b;
    constexpr int nq = 1 << (D - 1);
    const double wq = g.area[a] / nq;
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
      const int f = 2 * a + dir;
      const double al = dir ? 1.0 : -1.0;
      const bool interior = inter[f];
      const bool inflow = (al * F[f]) < 0.0;
      const bool sd = !interior && bsd[f] == 1;
      if (inflow && (interior || sd)) {
        double J = 0.0;
#pragma unroll
        for (int p = 0; p < nq; ++p) {
          double sqe[3] = {0, 0, 0}, sqn[3] = {0, 0, 0};
          sqe[a] = kSqrt3 * al;
          sqn[a] = -kSqrt3 * al;
#pragma unroll
          for (int ti = 0; ti < D - 1; ++ti) {
            const double xt = ((p >> ti) & 1) ? gp : -gp;
            sqe[tax[ti]] = kSqrt3 * xt;
            sqn[tax[ti]] = kSqrt3 * xt;
          }
          const double ve = p1_value(se, D, sqe, g.isv);
          double jmp;
          if (interior) {
            const double vn = p1_value(sn[f], D, sqn, g.isv);
            jmp = dir ? (ve - vn) : (vn - ve);   // low side minus high side
          } else {
            jmp = ve - bsv[f];
          }
          J += jmp * wq;
        }
        S += fabs(J);
      }
      if (interior) {
        const double ga = kSqrt3 * 2.0 / g.h[a] * g.isv * se[a + 1];
        const double gi = ga * (al * g.h[a]);
        const double di = sn[f][0] * g.isv - mean;
        mmin = fmin(mmin, gradient_scale(gi, di));
      }
    }
  }
  S = S / (0.08 * D * sqrt(g.he) * g.vol);
  const bool flag = (S > 1.0) || outside;
  out[e] = se[0];
#pragma unroll
  for (int k = 1; k < R; ++k) out[(long long)k * nc + e] = flag ? se[k] * mmin : se[k];
  if (flags) flags[e] = flag ? 1 : 0;
}

hipError_t launch_limiter(const Geom& g, const double* sat_bar, const double* flux,
                          double* sat_out, uint8_t* flags, hipStream_t st) {
  ktimer_begin(KK_LIMITER, st);
  if (g.dim == 2)
    hipLaunchKernelGGL(k_limiter<2>, dim3((g.ncell + 255) / 256), dim3(256), 0, st, g, sat_bar,
                       flux, sat_out, flags);
  else
    hipLaunchKernelGGL(k_limiter<3>, dim3((g.ncell + 255) / 256), dim3(256), 0, st, g, sat_bar,
                       flux, sat_out, flags);
  ktimer_end(-1.0, -1.0, st);
  return hipGetLastError();
}

}  // namespace lrbms
