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
// The reconstruction is one thread per cell of a box tile; the face-based
// kernels work on tiles of cells staged in LDS with a one-cell halo.
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

// ---- tiles of the face-based kernels -------------------------------------------
// A workgroup of 256 threads takes a tile of cells (16 x 16 in 2D, 8 x 8 x 4 in
// 3D): the tile's cell data with a one-cell halo are staged in LDS (coalesced
// rows), every face of the tile is evaluated once by one thread, and for the
// cell-based results every thread then gathers its cell from the face values.
// Each face's quadrature thus runs once instead of once per adjacent cell.
template <int D>
struct TileShape;
template <>
struct TileShape<2> {
  static constexpr int X = 16, Y = 16, Z = 1;
};
template <>
struct TileShape<3> {
  static constexpr int X = 8, Y = 8, Z = 4;
};

template <int D>
struct Tiling {
  using T = TileShape<D>;
  static constexpr int R = D + 1;
  static constexpr int HX = T::X + 2, HY = T::Y + 2, HZ = (D == 3) ? T::Z + 2 : 1;
  static constexpr int ZO = (D == 3) ? 1 : 0;            // halo offset along z
  static constexpr int NH = HX * HY * HZ;                 // cells of the halo box
  static constexpr int FX = (T::X + 1) * T::Y * T::Z;     // faces of the tile per axis
  static constexpr int FY = T::X * (T::Y + 1) * T::Z;
  static constexpr int FZ = (D == 3) ? T::X * T::Y * (T::Z + 1) : 0;
  static constexpr int NF = FX + FY + FZ;
  // halo-box index of the tile-local cell l (l in [-1, extent])
  __device__ static int hidx(const int l[3]) { return (l[0] + 1) + HX * ((l[1] + 1) + HY * (l[2] + ZO)); }
  // tile-local face number of the face along axis a at local face coordinates l
  __device__ static int fidx(int a, const int l[3]) {
    if (a == 0) return l[0] + (T::X + 1) * (l[1] + T::Y * l[2]);
    if (a == 1) return FX + l[0] + T::X * (l[1] + (T::Y + 1) * l[2]);
    return FX + FY + l[0] + T::X * (l[1] + T::Y * l[2]);
  }
  __device__ static void fdecode(int lf, int& a, int l[3]) {
    int e0 = T::X, e1 = T::Y;
    if (lf < FX) {
      a = 0;
      e0 += 1;
    } else if (lf < FX + FY) {
      a = 1;
      lf -= FX;
      e1 += 1;
    } else {
      a = 2;
      lf -= FX + FY;
    }
    l[0] = lf % e0;
    l[1] = (lf / e0) % e1;
    l[2] = lf / (e0 * e1);
  }
};

// Stage coefficients (and optionally permeabilities) of the tile's halo box.
template <int D>
__device__ __forceinline__ void stage_halo(const Geom& g, const double* __restrict__ src,
                                           const int o[3], double (*sh)[Tiling<D>::NH],
                                           double* shk) {
  using TL = Tiling<D>;
  const int nc = g.ncell;
  for (int h = threadIdx.x; h < TL::NH; h += blockDim.x) {
    const int x[3] = {o[0] + h % TL::HX - 1, o[1] + (h / TL::HX) % TL::HY - 1,
                      o[2] + h / (TL::HX * TL::HY) - TL::ZO};
    bool in = true;
#pragma unroll
    for (int a = 0; a < D; ++a) in = in && x[a] >= 0 && x[a] < g.n[a];
    const int c = in ? cell_index(g, x) : 0;
    double v[TL::R];
#pragma unroll
    for (int k = 0; k < TL::R; ++k) v[k] = in ? src[(long long)k * nc + c] : 0.0;
    const double kv = (shk && in) ? g.perm[c] : 1.0;
#pragma unroll
    for (int k = 0; k < TL::R; ++k) sh[k][h] = v[k];
    if (shk) shk[h] = kv;
  }
}

// Value of the P1 state of halo cell h at reference point sq (sqrt(3) xi).
template <int D>
__device__ __forceinline__ double halo_value(double (*sh)[Tiling<D>::NH], int h, const double sq[3],
                                             double isv) {
  double v = sh[0][h];
#pragma unroll
  for (int a = 0; a < D; ++a) v += sq[a] * sh[a + 1][h];
  return v * isv;
}

template <int D>
static dim3 tile_grid(const Geom& g) {
  using T = TileShape<D>;
  return dim3((g.n[0] + T::X - 1) / T::X, (g.n[1] + T::Y - 1) / T::Y,
              D == 3 ? (g.n[2] + T::Z - 1) / T::Z : 1);
}

// Def. velocityDG, one thread per face of a tile with the states, pressures
// and permeabilities of the tile and its halo in LDS: interior faces
// -sum_l w_l kappa_l int_f lambda(s_l) grad p_l . n + sigma_f/h_f int_f [p];
// Dirichlet faces the one-sided form against p_D; Neumann faces v_N |f|.  A
// tile writes the faces on its low sides, and the domain's last faces.
template <int D>
__global__ __launch_bounds__(256) void k_flux(Geom g, const double* __restrict__ ph,
                                              const double* __restrict__ sat,
                                              double* __restrict__ flux) {
  using TL = Tiling<D>;
  using T = TileShape<D>;
  constexpr int R = D + 1;
  __shared__ double shs[R][TL::NH];
  __shared__ double shp[R][TL::NH];
  __shared__ double shk[TL::NH];
  const int o[3] = {(int)blockIdx.x * T::X, (int)blockIdx.y * T::Y, (int)blockIdx.z * T::Z};
  stage_halo<D>(g, sat, o, shs, shk);
  stage_halo<D>(g, ph, o, shp, nullptr);
  __syncthreads();
  const int ext[3] = {T::X, T::Y, T::Z};
  for (int lf = threadIdx.x; lf < TL::NF; lf += blockDim.x) {
    int a, l[3];
    TL::fdecode(lf, a, l);
    int x[3] = {o[0] + l[0], o[1] + l[1], o[2] + l[2]};
    bool valid = x[a] <= g.n[a] && (l[a] < ext[a] || x[a] == g.n[a]);
#pragma unroll
    for (int b = 0; b < D; ++b)
      if (b != a) valid = valid && x[b] < g.n[b];
    if (!valid) continue;
    const int fid = face_index(g, a, x);
    const bool has_lo = x[a] >= 1, has_hi = x[a] < g.n[a];
    int lo[3] = {l[0], l[1], l[2]};
    lo[a] -= 1;
    const int h0 = has_lo ? TL::hidx(lo) : TL::hidx(l);
    const int h1 = has_hi ? TL::hidx(l) : h0;
    double s0[4] = {0, 0, 0, 0}, s1[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < R; ++k) {
      s0[k] = shs[k][h0];
      s1[k] = shs[k][h1];
    }
    const double k0 = shk[h0], k1 = shk[h1];
    const double p00 = shp[0][h0], p0a = shp[a + 1][h0];
    const double p10 = shp[0][h1], p1a = shp[a + 1][h1];
    const double gf = kSqrt3 * 2.0 / g.h[a] * g.isv;
    double F;
    if (has_lo && has_hi) {
      const double ik = 1.0 / (k0 + k1);
      double w0, w1;
      if (g.weights == 0) {
        w0 = k1 * ik;
        w1 = k0 * ik;
      } else {
        w0 = k0 * ik;
        w1 = k1 * ik;
      }
      const double g0 = face_mobility_co<D>(g, s0, a, 1.0);
      const double g1 = face_mobility_co<D>(g, s1, a, -1.0);
      const double jump = g.area[a] * g.isv * ((p00 + kSqrt3 * p0a) - (p10 - kSqrt3 * p1a));
      const double sig = g.pen * 2.0 * k0 * k1 * ik / g.hf[a];
      F = -(w0 * k0 * g0 * (gf * p0a) + w1 * k1 * g1 * (gf * p1a)) + sig * jump;
    } else {
      const double al = has_lo ? 1.0 : -1.0;   // outward normal sign
      const int bt = g.bc_type[fid];
      const double val = g.bc_val[fid];
      double out = 0.0;
      if (bt == LRBMS_BC_NEUMANN) {
        out = val * g.area[a];
      } else if (bt == LRBMS_BC_DIRICHLET) {
        const double gm = face_mobility_co<D>(g, s0, a, al);
        const double sig = g.pen * k0 / g.hf[a];
        const double trace = g.area[a] * g.isv * (p00 + kSqrt3 * al * p0a);
        out = -k0 * gm * (al * gf * p0a) + sig * (trace - val * g.area[a]);
      }
      F = al * out;
    }
    flux[fid] = F;
    if (!isfinite(F)) atomicMin(g.status, (int)LRBMS_E_NONFINITE);
  }
}

hipError_t launch_flux(const Geom& g, const double* ph, const double* sat, double* flux,
                       hipStream_t st) {
  ktimer_begin(KK_FLUX, st);
  if (g.dim == 2)
    hipLaunchKernelGGL(k_flux<2>, tile_grid<2>(g), dim3(256), 0, st, g, ph, sat, flux);
  else
    hipLaunchKernelGGL(k_flux<3>, tile_grid<3>(g), dim3(256), 0, st, g, ph, sat, flux);
  ktimer_end(-1.0, -1.0, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------

// Def. saturationDG with explicit Euler: out = s + dt/phi (q2 term + volume
// term int_e u f_w(s) . grad v - upwind face terms - jump penalty); RT0
// velocity of the face fluxes; 2-point Gauss rules.
template <int D>
__global__ __launch_bounds__(256) void k_transport(Geom g, const double* __restrict__ sat,
                                                   const double* __restrict__ flux,
                                                   double* __restrict__ out) {
  using TL = Tiling<D>;
  using T = TileShape<D>;
  constexpr int R = D + 1, NQF = 1 << (D - 1), NQC = 1 << D;
  __shared__ double shs[R][TL::NH];
  __shared__ double shk[TL::NH];
  __shared__ double shF[TL::NF];
  __shared__ double shA[D][TL::NF];
  const int o[3] = {(int)blockIdx.x * T::X, (int)blockIdx.y * T::Y, (int)blockIdx.z * T::Z};
  stage_halo<D>(g, sat, o, shs, shk);
  __syncthreads();
  const double gp = 1.0 / kSqrt3;
  // ---- faces: A0 = sum_q tot_q w_q / sqrt|e|, At = the same times xi_t
  for (int lf = threadIdx.x; lf < TL::NF; lf += blockDim.x) {
    int a, l[3];
    TL::fdecode(lf, a, l);
    int x[3] = {o[0] + l[0], o[1] + l[1], o[2] + l[2]};
    bool valid = x[a] <= g.n[a];
#pragma unroll
    for (int b = 0; b < D; ++b)
      if (b != a) valid = valid && x[b] < g.n[b];
    double F = 0.0, A[D];
#pragma unroll
    for (int k = 0; k < D; ++k) A[k] = 0.0;
    if (valid) {
      const int fid = face_index(g, a, x);
      F = flux[fid];
      const bool has_lo = x[a] >= 1, has_hi = x[a] < g.n[a];
      int lo[3] = {l[0], l[1], l[2]};
      lo[a] -= 1;
      const int hlo = TL::hidx(lo), hhi = TL::hidx(l);
      int tax[2] = {0, 0}, nt = 0;
#pragma unroll
      for (int b = 0; b < D; ++b)
        if (b != a) tax[nt++] = b;
      const double wq = g.area[a] / NQF, Fa = F / g.area[a];
      if (has_lo && has_hi) {
        const double klo = shk[hlo], khi = shk[hhi];
        const double sig = g.sat_pen * (g.pen * 2.0 * klo * khi / (klo + khi)) / g.hf[a];
#pragma unroll
        for (int q = 0; q < NQF; ++q) {
          double sl[3] = {0, 0, 0}, sh[3] = {0, 0, 0}, xt[2] = {0, 0};
          sl[a] = kSqrt3;
          sh[a] = -kSqrt3;
#pragma unroll
          for (int ti = 0; ti < D - 1; ++ti) {
            xt[ti] = ((q >> ti) & 1) ? gp : -gp;
            sl[tax[ti]] = kSqrt3 * xt[ti];
            sh[tax[ti]] = kSqrt3 * xt[ti];
          }
          const double vlo = halo_value<D>(shs, hlo, sl, g.isv);
          const double vhi = halo_value<D>(shs, hhi, sh, g.isv);
          const double up = (F >= 0.0) ? vlo : vhi;
          const double tw = (Fa * frac_flow(g, up) + sig * (vlo - vhi)) * wq * g.isv;
          A[0] += tw;
#pragma unroll
          for (int ti = 0; ti < D - 1; ++ti) A[ti + 1] += tw * xt[ti];
        }
      } else {
        // boundary face: one cell, outward sign al (+1: the face is its high face)
        const double al = has_lo ? 1.0 : -1.0;
        const int hc = has_lo ? hlo : hhi;
        const bool sd = g.bc_sat[fid] == 1;
        const double sval = g.bc_sval[fid];
        const double sig = g.sat_pen * (g.pen * shk[hc]) / g.hf[a];
        const double fout = al * Fa;
#pragma unroll
        for (int q = 0; q < NQF; ++q) {
          double sq[3] = {0, 0, 0}, xt[2] = {0, 0};
          sq[a] = kSqrt3 * al;
#pragma unroll
          for (int ti = 0; ti < D - 1; ++ti) {
            xt[ti] = ((q >> ti) & 1) ? gp : -gp;
            sq[tax[ti]] = kSqrt3 * xt[ti];
          }
          const double ve = halo_value<D>(shs, hc, sq, g.isv);
          const double chi = sd ? sval : ve;
          const double tw = (fout * frac_flow(g, chi) + (sd ? sig * (ve - sval) : 0.0)) * wq * g.isv;
          A[0] += tw;
#pragma unroll
          for (int ti = 0; ti < D - 1; ++ti) A[ti + 1] += tw * xt[ti];
        }
      }
    }
    shF[lf] = F;
#pragma unroll
    for (int k = 0; k < D; ++k) shA[k][lf] = A[k];
  }
  __syncthreads();
  // ---- cells
  const int tid = threadIdx.x;
  const int l[3] = {tid % T::X, (tid / T::X) % T::Y, tid / (T::X * T::Y)};
  const int x[3] = {o[0] + l[0], o[1] + l[1], o[2] + l[2]};
#pragma unroll
  for (int a = 0; a < D; ++a)
    if (x[a] >= g.n[a]) return;
  const int nc = g.ncell, e = cell_index(g, x), h = TL::hidx(l);
  double se[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < R; ++k) se[k] = shs[k][h];
  const double q2 = g.q2[e], phi = g.poro[e];
  double Flo[3], Fhi[3];
  int flo[3], fhi[3];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    int lh[3] = {l[0], l[1], l[2]};
    flo[a] = TL::fidx(a, l);
    lh[a] += 1;
    fhi[a] = TL::fidx(a, lh);
    Flo[a] = shF[flo[a]];
    Fhi[a] = shF[fhi[a]];
  }
  double Rr[4] = {0.0, 0.0, 0.0, 0.0};
  Rr[0] += q2 * g.vol * g.isv;
  {
    double acc[3] = {0, 0, 0};
#pragma unroll
    for (int p = 0; p < NQC; ++p) {
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
        acc[a] += ((1.0 - t) * Flo[a] + t * Fhi[a]) * fw;
      }
    }
    // u_a = F / |f_a| at the point; the cell rule weighs |e| / 2^d
#pragma unroll
    for (int a = 0; a < D; ++a)
      Rr[a + 1] += (kSqrt3 * 2.0 / g.h[a] * g.isv) * (acc[a] * (g.vol / NQC / g.area[a]));
  }
  // face terms: [v] = +v on the low-side cell, -v on the high-side cell, v on a
  // boundary face
#pragma unroll
  for (int a = 0; a < D; ++a) {
    int tax[2] = {0, 0}, nt = 0;
#pragma unroll
    for (int b = 0; b < D; ++b)
      if (b != a) tax[nt++] = b;
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
      const int lf = dir ? fhi[a] : flo[a];
      const double al = dir ? 1.0 : -1.0;
      const bool interior = dir ? (x[a] + 1 < g.n[a]) : (x[a] >= 1);
      const double jv = interior ? al : 1.0;
      const double A0 = shA[0][lf];
      Rr[0] -= jv * A0;
      Rr[a + 1] -= jv * (kSqrt3 * al * A0);
#pragma unroll
      for (int ti = 0; ti < D - 1; ++ti) Rr[tax[ti] + 1] -= jv * (kSqrt3 * shA[ti + 1][lf]);
    }
  }
  bool bad = false;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const double v = se[k] + g.dt * Rr[k] / phi;
    out[(long long)k * nc + e] = v;
    bad |= !isfinite(v);
  }
  if (bad) atomicMin(g.status, (int)LRBMS_E_NONFINITE);
  // CFL number of the cell: outflow over phi |e| times dt max |f_w'|
  double outflow = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) outflow += fmax(0.0, -Flo[a]) + fmax(0.0, Fhi[a]);
  if (g.cfl_coef * outflow > kCflWarn * phi * g.vol) atomicMax(g.status + 1, (int)LRBMS_W_CFL);
}

hipError_t launch_transport(const Geom& g, const double* sat, const double* flux, double* sat_bar,
                            hipStream_t st) {
  ktimer_begin(KK_TRANSPORT, st);
  if (g.dim == 2)
    hipLaunchKernelGGL(k_transport<2>, tile_grid<2>(g), dim3(256), 0, st, g, sat, flux, sat_bar);
  else
    hipLaunchKernelGGL(k_transport<3>, tile_grid<3>(g), dim3(256), 0, st, g, sat, flux, sat_bar);
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

// eq. limiterMain on tiles: every face's |int_f [s]| (interior faces and
// saturation-Dirichlet faces) once, then per cell the shock detector over its
// inflow faces, the vertex test, and the gradient scales against the face
// neighbours' means.
template <int D>
__global__ __launch_bounds__(256) void k_limiter(Geom g, const double* __restrict__ sb,
                                                 const double* __restrict__ flux,
                                                 double* __restrict__ out,
                                                 uint8_t* __restrict__ flags) {
  using TL = Tiling<D>;
  using T = TileShape<D>;
  constexpr int R = D + 1, NQF = 1 << (D - 1);
  __shared__ double shs[R][TL::NH];
  __shared__ double shF[TL::NF];
  __shared__ double shJ[TL::NF];
  const int o[3] = {(int)blockIdx.x * T::X, (int)blockIdx.y * T::Y, (int)blockIdx.z * T::Z};
  stage_halo<D>(g, sb, o, shs, nullptr);
  __syncthreads();
  const double gp = 1.0 / kSqrt3;
  for (int lf = threadIdx.x; lf < TL::NF; lf += blockDim.x) {
    int a, l[3];
    TL::fdecode(lf, a, l);
    int x[3] = {o[0] + l[0], o[1] + l[1], o[2] + l[2]};
    bool valid = x[a] <= g.n[a];
#pragma unroll
    for (int b = 0; b < D; ++b)
      if (b != a) valid = valid && x[b] < g.n[b];
    double F = 0.0, J = 0.0;
    if (valid) {
      const int fid = face_index(g, a, x);
      F = flux[fid];
      const bool has_lo = x[a] >= 1, has_hi = x[a] < g.n[a];
      int lo[3] = {l[0], l[1], l[2]};
      lo[a] -= 1;
      const int hlo = TL::hidx(lo), hhi = TL::hidx(l);
      int tax[2] = {0, 0}, nt = 0;
#pragma unroll
      for (int b = 0; b < D; ++b)
        if (b != a) tax[nt++] = b;
      const double wq = g.area[a] / NQF;
      const bool interior = has_lo && has_hi;
      const bool sd = !interior && g.bc_sat[fid] == 1;
      const double sval = sd ? g.bc_sval[fid] : 0.0;
      if (interior || sd) {
        const double al = has_lo ? 1.0 : -1.0;
        const int hc = has_lo ? hlo : hhi;
#pragma unroll
        for (int q = 0; q < NQF; ++q) {
          double sl[3] = {0, 0, 0}, sh[3] = {0, 0, 0};
          sl[a] = interior ? kSqrt3 : kSqrt3 * al;
          sh[a] = -kSqrt3;
#pragma unroll
          for (int ti = 0; ti < D - 1; ++ti) {
            const double xt = ((q >> ti) & 1) ? gp : -gp;
            sl[tax[ti]] = kSqrt3 * xt;
            sh[tax[ti]] = kSqrt3 * xt;
          }
          // low side minus high side; a Dirichlet face: the cell's trace minus s_D
          const double jmp = interior ? halo_value<D>(shs, hlo, sl, g.isv) - halo_value<D>(shs, hhi, sh, g.isv)
                                      : halo_value<D>(shs, hc, sl, g.isv) - sval;
          J += jmp * wq;
        }
      }
    }
    shF[lf] = F;
    shJ[lf] = fabs(J);
  }
  __syncthreads();
  const int tid = threadIdx.x;
  const int l[3] = {tid % T::X, (tid / T::X) % T::Y, tid / (T::X * T::Y)};
  const int x[3] = {o[0] + l[0], o[1] + l[1], o[2] + l[2]};
#pragma unroll
  for (int a = 0; a < D; ++a)
    if (x[a] >= g.n[a]) return;
  const int nc = g.ncell, e = cell_index(g, x), h = TL::hidx(l);
  double se[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < R; ++k) se[k] = shs[k][h];
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
  double S = 0.0, mmin = 1.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
      int lf3[3] = {l[0], l[1], l[2]};
      lf3[a] += dir;
      const int lf = TL::fidx(a, lf3);
      const double al = dir ? 1.0 : -1.0;
      const bool interior = dir ? (x[a] + 1 < g.n[a]) : (x[a] >= 1);
      // inflow: outward-normal flux below zero; shJ is zero on faces without a jump
      if (al * shF[lf] < 0.0) S += shJ[lf];
      if (interior) {
        int ln[3] = {l[0], l[1], l[2]};
        ln[a] += dir ? 1 : -1;
        const double ga = kSqrt3 * 2.0 / g.h[a] * g.isv * se[a + 1];
        const double gi = ga * (al * g.h[a]);
        const double di = shs[0][TL::hidx(ln)] * g.isv - mean;
        mmin = fmin(mmin, gradient_scale(gi, di));
      }
    }
  }
  S = S / (0.08 * D * sqrt(g.he) * g.vol);
  const bool flag = (S > 1.0) || outside;
  out[e] = se[0];
  bool bad = !isfinite(se[0]);
#pragma unroll
  for (int k = 1; k < R; ++k) {
    const double v = flag ? se[k] * mmin : se[k];
    out[(long long)k * nc + e] = v;
    bad |= !isfinite(v);
  }
  if (flags) flags[e] = flag ? 1 : 0;
  if (bad) atomicMin(g.status, (int)LRBMS_E_NONFINITE);
}

hipError_t launch_limiter(const Geom& g, const double* sat_bar, const double* flux,
                          double* sat_out, uint8_t* flags, hipStream_t st) {
  ktimer_begin(KK_LIMITER, st);
  if (g.dim == 2)
    hipLaunchKernelGGL(k_limiter<2>, tile_grid<2>(g), dim3(256), 0, st, g, sat_bar, flux, sat_out,
                       flags);
  else
    hipLaunchKernelGGL(k_limiter<3>, tile_grid<3>(g), dim3(256), 0, st, g, sat_bar, flux, sat_out,
                       flags);
  ktimer_end(-1.0, -1.0, st);
  return hipGetLastError();
}

}  // namespace lrbms
