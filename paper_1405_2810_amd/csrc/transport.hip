// Fine-grid kernels of the online step on gfx950:
//   pressure reconstruction p_h = sum_i (p_N)_i phi_i      (Alg. 3 step 5b)
//   face fluxes of the conservative velocity              (Def. velocityDG)
//   DG upwind explicit Euler saturation step              (Def. saturationDG)
//   slope limiter                                         (eq. limiterMain)
//
// Readings (same as the CPU reference): RT0 on rectangles (one normal flux per
// face, u_a linear in x_a only); v_N |f| as the flux on Neumann faces; upwind
// trace taken from the low-side cell when the flux along +axis is >= 0; s_D on
// saturation Dirichlet faces, the interior trace on other boundary faces;
// shock detector with |int_f [s]| over inflow faces; the limited state keeps
// the cell mean and scales the slope by min_i m_i; 2-point Gauss rules.
//
// The reconstruction is one thread per cell of a box tile; the face-based
// kernels work on tiles of cells staged in LDS with a one-cell halo.  They
// are instantiated per dimension and per relative permeability law; their
// time goes to vector instructions (the quadratures, the face and cell index
// arithmetic), so the tiles are laid out to keep that count low: per-axis face
// bodies with compile-time extents, results held in registers across the
// barrier that lets them overwrite the halo, which raises the workgroups per
// CU.
#include <type_traits>

#include "common.h"
#include "ktimer.h"

namespace lrbms {

// The relative permeability law as a template argument of the fine-grid
// kernels, so that the common laws carry no call to the general power:
// 0 linear, 1 Corey with both exponents 2, 2 any other Corey exponents.
// Each form gives the same values as mobilities().
inline int law_of(const Geom& g) {
  if (g.relperm == 0) return 0;
  return (g.cw == 2.0 && g.co == 2.0) ? 1 : 2;
}

template <int LAW>
__device__ __forceinline__ void mobilities_law(const Geom& g, double s, double& lw, double& lo) {
  if (LAW == 2) {
    mobilities(g, s, lw, lo);
    return;
  }
  const double sc = clip01(s);
  double krw, kro;
  if (LAW == 0) {
    krw = sc;
    kro = 1.0 - sc;
  } else {
    const double so = 1.0 - sc;
    krw = sc * sc;
    kro = so * so;
  }
  lw = krw * g.ivw;
  lo = kro * g.ivo;
}

template <int LAW>
__device__ __forceinline__ double total_mobility_law(const Geom& g, double s) {
  double lw, lo;
  mobilities_law<LAW>(g, s, lw, lo);
  return lw + lo;
}

template <int LAW>
__device__ __forceinline__ double frac_flow_law(const Geom& g, double s) {
  double lw, lo;
  mobilities_law<LAW>(g, s, lw, lo);
  return lw * rcp_refined(lw + lo);
}

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

// Tangential axes of the faces normal to axis A, in increasing order.
template <int A>
struct Tang {
  static constexpr int t0 = A == 0 ? 1 : 0, t1 = A == 2 ? 1 : 2;
};

// Integral of the total mobility lambda(s) over the face of axis A at local
// coordinate xi_A of a cell with coefficients co (2-point Gauss in the
// tangential directions).
template <int D, int LAW, int A>
__device__ __forceinline__ double face_mobility_co(const Geom& g, const double (&co)[4], double xia) {
  const double gp = 1.0 / kSqrt3;
  double sum = 0.0;
#pragma unroll
  for (int p = 0; p < (1 << (D - 1)); ++p) {
    double sq[3] = {0, 0, 0};
    sq[A] = kSqrt3 * xia;
    sq[Tang<A>::t0] = kSqrt3 * ((p & 1) ? gp : -gp);
    if (D == 3) sq[Tang<A>::t1] = kSqrt3 * (((p >> 1) & 1) ? gp : -gp);
    sum += total_mobility_law<LAW>(g, p1_value(co, D, sq, g.isv));
  }
  return sum * g.area[A] / (1 << (D - 1));
}

// ---- tiles of the face-based kernels -------------------------------------------
// A workgroup of 256 threads takes a tile of cells (16 x 16 in 2D, 8 x 8 x 4 in
// 3D): the tile's cell data with a one-cell halo are staged in LDS, every face
// of the tile is evaluated once by one thread, and for the cell-based results
// every thread then gathers its cell from the face values.  Each face's
// quadrature thus runs once instead of once per adjacent cell.  The faces of
// a tile are numbered axis by axis; a thread's face loop branches once per
// face to a body specialised for the face's axis, so that every per-axis
// quantity (extents, spacings, tangential axes) is a compile-time index.
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

constexpr int kTileThreads = 256;

template <int D>
struct Tiling {
  using T = TileShape<D>;
  static_assert(T::X * T::Y * T::Z == kTileThreads, "one thread per tile cell");
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
  // local face coordinates of the j-th face along axis A
  template <int A>
  __device__ static void fdecode(int j, int l[3]) {
    constexpr int e0 = T::X + (A == 0 ? 1 : 0), e1 = T::Y + (A == 1 ? 1 : 0);
    l[0] = j % e0;
    l[1] = (j / e0) % e1;
    l[2] = j / (e0 * e1);
  }
};

// Calls f(axis, lf, j) for the tile faces lf = threadIdx.x + k 256, where j is
// the face's number among the tile faces of its axis.
template <int D, class Fn>
__device__ __forceinline__ void for_tile_faces(Fn&& f) {
  using TL = Tiling<D>;
  for (int lf = threadIdx.x; lf < TL::NF; lf += kTileThreads) {
    if (lf < TL::FX)
      f(std::integral_constant<int, 0>(), lf, lf);
    else if (D == 2 || lf < TL::FX + TL::FY)
      f(std::integral_constant<int, 1>(), lf, lf - TL::FX);
    else
      f(std::integral_constant<int, D - 1>(), lf, lf - TL::FX - TL::FY);
  }
}

// Global number of the j-th tile face along axis A (x = its face
// coordinates), or -1 when the face lies outside the domain.
template <int D, int A>
__device__ __forceinline__ int tile_face(const Geom& g, const int o[3], int j, int l[3], int x[3]) {
  Tiling<D>::template fdecode<A>(j, l);
#pragma unroll
  for (int b = 0; b < 3; ++b) x[b] = o[b] + l[b];
  bool valid = x[A] <= g.n[A];
#pragma unroll
  for (int b = 0; b < D; ++b)
    if (b != A) valid = valid && x[b] < g.n[b];
  return valid ? face_index(g, A, x) : -1;
}

// One thread's share of the tile's halo box (coefficients, optionally the
// permeabilities): every global load is issued before the first LDS store, so
// a thread has all of them in flight at once; halo cells outside the domain
// read cell 0 and are replaced by zero state (permeability 1).
template <int D, bool PERM>
struct HaloRegs {
  using TL = Tiling<D>;
  static constexpr int NIT = (TL::NH + kTileThreads - 1) / kTileThreads;
  double v[NIT][TL::R];
  double kv[PERM ? NIT : 1];
  __device__ __forceinline__ void load(const Geom& g, const double* __restrict__ src,
                                       const int o[3]) {
    const int nc = g.ncell;
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int h = (int)threadIdx.x + kTileThreads * it;
      const int x[3] = {o[0] + h % TL::HX - 1, o[1] + (h / TL::HX) % TL::HY - 1,
                        o[2] + h / (TL::HX * TL::HY) - TL::ZO};
      bool in = h < TL::NH;
#pragma unroll
      for (int a = 0; a < D; ++a) in = in && x[a] >= 0 && x[a] < g.n[a];
      const int c = in ? cell_index(g, x) : 0;
#pragma unroll
      for (int k = 0; k < TL::R; ++k) {
        const double t = src[(long long)k * nc + c];
        v[it][k] = in ? t : 0.0;
      }
      if (PERM) {
        const double t = g.perm[c];
        kv[it] = in ? t : 1.0;
      }
    }
  }
  __device__ __forceinline__ void store(double (*sh)[TL::NH], double* shk) const {
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int h = (int)threadIdx.x + kTileThreads * it;
      if (h < TL::NH) {
#pragma unroll
        for (int k = 0; k < TL::R; ++k) sh[k][h] = v[it][k];
        if (PERM) shk[h] = kv[it];
      }
    }
  }
};

// The fluxes of a tile's faces (zero outside the domain) into LDS; each
// thread issues the loads of all its faces before its first store.
template <int D>
__device__ __forceinline__ void stage_face_fluxes(const Geom& g, const double* __restrict__ flux,
                                                  const int o[3], double* shF) {
  using TL = Tiling<D>;
  constexpr int NIT = (TL::NF + kTileThreads - 1) / kTileThreads;
  double F[NIT];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int lf = (int)threadIdx.x + kTileThreads * it;
    int l[3], x[3], fid = -1;
    if (lf < TL::FX)
      fid = tile_face<D, 0>(g, o, lf, l, x);
    else if (D == 2 || lf < TL::FX + TL::FY)
      fid = lf < TL::NF ? tile_face<D, 1>(g, o, lf - TL::FX, l, x) : -1;
    else if (lf < TL::NF)
      fid = tile_face<D, D - 1>(g, o, lf - TL::FX - TL::FY, l, x);
    const double t = flux[fid >= 0 ? fid : 0];
    F[it] = fid >= 0 ? t : 0.0;
  }
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int lf = (int)threadIdx.x + kTileThreads * it;
    if (lf < TL::NF) shF[lf] = F[it];
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

// One-dimensional grid over the tiles (x fastest, then y, then z).  The
// hardware deals workgroups to the eight XCDs in turn; xcd_item gives each XCD
// a contiguous run of tiles (a slab across z), so the halo cells a tile shares
// with its neighbours are mostly read from the XCD's own L2.
template <int D>
__host__ __device__ __forceinline__ void tile_counts(const Geom& g, int t[3]) {
  using T = TileShape<D>;
  t[0] = (g.n[0] + T::X - 1) / T::X;
  t[1] = (g.n[1] + T::Y - 1) / T::Y;
  t[2] = D == 3 ? (g.n[2] + T::Z - 1) / T::Z : 1;
}

template <int D>
static dim3 tile_grid(const Geom& g) {
  int t[3];
  tile_counts<D>(g, t);
  return dim3(t[0] * t[1] * t[2]);
}

template <int D>
__device__ __forceinline__ void tile_origin(const Geom& g, int o[3]) {
  using T = TileShape<D>;
  int t[3];
  tile_counts<D>(g, t);
  const int i = xcd_item((int)blockIdx.x, t[0] * t[1] * t[2]);
  o[0] = (i % t[0]) * T::X;
  o[1] = ((i / t[0]) % t[1]) * T::Y;
  o[2] = (i / (t[0] * t[1])) * T::Z;
}

// Launch of a face kernel instantiated for the dimension and the law.
#define LRBMS_FACE_LAUNCH(KERNEL, g, st, ...)                                              \
  do {                                                                                     \
    const int law_ = law_of(g);                                                            \
    if ((g).dim == 2) {                                                                    \
      const dim3 grid_ = tile_grid<2>(g);                                                  \
      if (law_ == 0) hipLaunchKernelGGL((KERNEL<2, 0>), grid_, dim3(256), 0, st, __VA_ARGS__); \
      else if (law_ == 1) hipLaunchKernelGGL((KERNEL<2, 1>), grid_, dim3(256), 0, st, __VA_ARGS__); \
      else hipLaunchKernelGGL((KERNEL<2, 2>), grid_, dim3(256), 0, st, __VA_ARGS__);       \
    } else {                                                                               \
      const dim3 grid_ = tile_grid<3>(g);                                                  \
      if (law_ == 0) hipLaunchKernelGGL((KERNEL<3, 0>), grid_, dim3(256), 0, st, __VA_ARGS__); \
      else if (law_ == 1) hipLaunchKernelGGL((KERNEL<3, 1>), grid_, dim3(256), 0, st, __VA_ARGS__); \
      else hipLaunchKernelGGL((KERNEL<3, 2>), grid_, dim3(256), 0, st, __VA_ARGS__);       \
    }                                                                                      \
  } while (0)

// Def. velocityDG, one thread per face of a tile with the states, pressures
// and permeabilities of the tile and its halo in LDS: interior faces
// -sum_l w_l kappa_l int_f lambda(s_l) grad p_l . n + sigma_f/h_f int_f [p];
// Dirichlet faces the one-sided form against p_D; Neumann faces v_N |f|.  A
// tile writes the faces on its low sides, and the domain's last faces.
template <int D, int LAW>
__global__ __launch_bounds__(256) void k_flux(Geom g, const double* __restrict__ ph,
                                              const double* __restrict__ sat,
                                              double* __restrict__ flux) {
  using TL = Tiling<D>;
  using T = TileShape<D>;
  constexpr int R = D + 1;
  __shared__ double shs[R][TL::NH];
  __shared__ double shp[R][TL::NH];
  __shared__ double shk[TL::NH];
  int o[3];
  tile_origin<D>(g, o);
  {
    HaloRegs<D, true> rs;
    HaloRegs<D, false> rp;
    rs.load(g, sat, o);
    rp.load(g, ph, o);
    rs.store(shs, shk);
    rp.store(shp, nullptr);
  }
  __syncthreads();
  for_tile_faces<D>([&](auto AX, int lf, int j) {
    (void)lf;
    constexpr int a = decltype(AX)::value;
    constexpr int ext = a == 0 ? T::X : (a == 1 ? T::Y : T::Z);
    int l[3];
    TL::template fdecode<a>(j, l);
    const int x[3] = {o[0] + l[0], o[1] + l[1], o[2] + l[2]};
    bool valid = x[a] <= g.n[a] && (l[a] < ext || x[a] == g.n[a]);
#pragma unroll
    for (int b = 0; b < D; ++b)
      if (b != a) valid = valid && x[b] < g.n[b];
    if (!valid) return;
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
      const double g0 = face_mobility_co<D, LAW, a>(g, s0, 1.0);
      const double g1 = face_mobility_co<D, LAW, a>(g, s1, -1.0);
      const double jump = g.area[a] * g.isv * ((p00 + kSqrt3 * p0a) - (p10 - kSqrt3 * p1a));
      const double sig = g.pen * 2.0 * k0 * k1 * ik * (1.0 / g.hf[a]);
      F = -(w0 * k0 * g0 * (gf * p0a) + w1 * k1 * g1 * (gf * p1a)) + sig * jump;
    } else {
      const double al = has_lo ? 1.0 : -1.0;   // outward normal sign
      const int bt = g.bc_type[fid];
      const double val = g.bc_val[fid];
      double out = 0.0;
      if (bt == LRBMS_BC_NEUMANN) {
        out = val * g.area[a];
      } else if (bt == LRBMS_BC_DIRICHLET) {
        const double gm = face_mobility_co<D, LAW, a>(g, s0, al);
        const double sig = g.pen * k0 / g.hf[a];
        const double trace = g.area[a] * g.isv * (p00 + kSqrt3 * al * p0a);
        out = -k0 * gm * (al * gf * p0a) + sig * (trace - val * g.area[a]);
      }
      F = al * out;
    }
    flux[fid] = F;
    if (!isfinite(F)) atomicMin(g.status, (int)LRBMS_E_NONFINITE);
  });
}

hipError_t launch_flux(const Geom& g, const double* ph, const double* sat, double* flux,
                       hipStream_t st) {
  ktimer_begin(KK_FLUX, st);
  LRBMS_FACE_LAUNCH(k_flux, g, st, g, ph, sat, flux);
  ktimer_end(-1.0, -1.0, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------

// Def. saturationDG with explicit Euler: out = s + dt/phi (q2 term + volume
// term int_e u f_w(s) . grad v - upwind face terms - jump penalty); RT0
// velocity of the face fluxes; 2-point Gauss rules.
template <int D, int LAW>
__global__ __launch_bounds__(256) void k_transport(Geom g, const double* __restrict__ sat,
                                                   const double* __restrict__ flux,
                                                   double* __restrict__ out) {
  using TL = Tiling<D>;
  using T = TileShape<D>;
  constexpr int R = D + 1, NQF = 1 << (D - 1), NQC = 1 << D;
  // The halo (states, permeabilities) is needed by the face pass only: the
  // face results are kept in registers until every thread has passed it and
  // then stored over the halo, which keeps the workgroup's LDS small enough
  // for five workgroups per CU in 3D.
  constexpr int NHALO = (R + 1) * TL::NH, NA = D * TL::NF;
  __shared__ double shHA[NHALO > NA ? NHALO : NA];
  __shared__ double shF[TL::NF];
  double(*shs)[TL::NH] = reinterpret_cast<double(*)[TL::NH]>(shHA);
  double* shk = shHA + R * TL::NH;
  double(*shA)[TL::NF] = reinterpret_cast<double(*)[TL::NF]>(shHA);
  int o[3];
  tile_origin<D>(g, o);
  // this thread's cell (the cell pass below), its source and porosity loaded
  // with the halo and the face fluxes
  const int tid = threadIdx.x;
  const int l[3] = {tid % T::X, (tid / T::X) % T::Y, tid / (T::X * T::Y)};
  const int x[3] = {o[0] + l[0], o[1] + l[1], o[2] + l[2]};
  bool cell_in = true;
#pragma unroll
  for (int a = 0; a < D; ++a) cell_in = cell_in && x[a] < g.n[a];
  const int e = cell_in ? cell_index(g, x) : 0;
  const double q2 = g.q2[e], phi = g.poro[e];
  {
    HaloRegs<D, true> rs;
    rs.load(g, sat, o);
    stage_face_fluxes<D>(g, flux, o, shF);
    rs.store(shs, shk);
  }
  __syncthreads();
  const double gp = 1.0 / kSqrt3;
  // ---- faces: A0 = sum_q tot_q w_q / sqrt|e|, At = the same times xi_t
  auto face = [&](auto AX, int lf, int j, double (&A)[D]) {
    constexpr int a = decltype(AX)::value;
    constexpr int t0 = Tang<a>::t0, t1 = Tang<a>::t1;
    int lfc[3], xf[3];
    const int fid = tile_face<D, a>(g, o, j, lfc, xf);
    const double F = shF[lf];
    const double iarea = 1.0 / g.area[a], ihf = 1.0 / g.hf[a];
    if (fid >= 0) {
      const bool has_lo = xf[a] >= 1, has_hi = xf[a] < g.n[a];
      int lo[3] = {lfc[0], lfc[1], lfc[2]};
      lo[a] -= 1;
      const int hlo = TL::hidx(lo), hhi = TL::hidx(lfc);
      const double wq = g.area[a] / NQF, Fa = F * iarea;
      if (has_lo && has_hi) {
        const double klo = shk[hlo], khi = shk[hhi];
        const double sig = g.sat_pen * (g.pen * 2.0 * klo * khi / (klo + khi)) * ihf;
#pragma unroll
        for (int q = 0; q < NQF; ++q) {
          double sl[3] = {0, 0, 0}, sh[3] = {0, 0, 0}, xt[2] = {0, 0};
          sl[a] = kSqrt3;
          sh[a] = -kSqrt3;
          xt[0] = (q & 1) ? gp : -gp;
          sl[t0] = sh[t0] = kSqrt3 * xt[0];
          if (D == 3) {
            xt[1] = ((q >> 1) & 1) ? gp : -gp;
            sl[t1] = sh[t1] = kSqrt3 * xt[1];
          }
          const double vlo = halo_value<D>(shs, hlo, sl, g.isv);
          const double vhi = halo_value<D>(shs, hhi, sh, g.isv);
          const double up = (F >= 0.0) ? vlo : vhi;
          const double tw = (Fa * frac_flow_law<LAW>(g, up) + sig * (vlo - vhi)) * wq * g.isv;
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
        const double sig = g.sat_pen * (g.pen * shk[hc]) * ihf;
        const double fout = al * Fa;
#pragma unroll
        for (int q = 0; q < NQF; ++q) {
          double sq[3] = {0, 0, 0}, xt[2] = {0, 0};
          sq[a] = kSqrt3 * al;
          xt[0] = (q & 1) ? gp : -gp;
          sq[t0] = kSqrt3 * xt[0];
          if (D == 3) {
            xt[1] = ((q >> 1) & 1) ? gp : -gp;
            sq[t1] = kSqrt3 * xt[1];
          }
          const double ve = halo_value<D>(shs, hc, sq, g.isv);
          const double chi = sd ? sval : ve;
          const double tw =
              (fout * frac_flow_law<LAW>(g, chi) + (sd ? sig * (ve - sval) : 0.0)) * wq * g.isv;
          A[0] += tw;
#pragma unroll
          for (int ti = 0; ti < D - 1; ++ti) A[ti + 1] += tw * xt[ti];
        }
      }
    }
  };
  constexpr int NFI = (TL::NF + kTileThreads - 1) / kTileThreads;
  double Ar[NFI][D];
#pragma unroll
  for (int it = 0; it < NFI; ++it) {
    const int lf = tid + kTileThreads * it;
#pragma unroll
    for (int k = 0; k < D; ++k) Ar[it][k] = 0.0;
    if (lf < TL::FX)
      face(std::integral_constant<int, 0>(), lf, lf, Ar[it]);
    else if (D == 2 || lf < TL::FX + TL::FY) {
      if (lf < TL::NF) face(std::integral_constant<int, 1>(), lf, lf - TL::FX, Ar[it]);
    } else if (lf < TL::NF) {
      face(std::integral_constant<int, D - 1>(), lf, lf - TL::FX - TL::FY, Ar[it]);
    }
  }
  const int h = TL::hidx(l);
  double se[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < R; ++k) se[k] = shs[k][h];
  __syncthreads();
#pragma unroll
  for (int it = 0; it < NFI; ++it) {
    const int lf = tid + kTileThreads * it;
    if (lf < TL::NF) {
#pragma unroll
      for (int k = 0; k < D; ++k) shA[k][lf] = Ar[it][k];
    }
  }
  __syncthreads();
  // ---- cells
  if (!cell_in) return;
  const int nc = g.ncell;
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
      const double fw = frac_flow_law<LAW>(g, p1_value(se, D, sq, g.isv));
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
  const double dtp = g.dt / phi;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const double v = se[k] + dtp * Rr[k];
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
  LRBMS_FACE_LAUNCH(k_transport, g, st, g, sat, flux, sat_bar);
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
  // The face jumps are kept in registers until every thread has passed the
  // face pass and then stored over the halo's slope coefficients, which the
  // cell pass no longer reads (it takes the neighbours' means only).
  static_assert((R - 1) * TL::NH >= TL::NF, "jumps fit over the slopes");
  __shared__ double shs[R][TL::NH];
  __shared__ double shF[TL::NF];
  double* shJ = &shs[1][0];
  int o[3];
  tile_origin<D>(g, o);
  {
    HaloRegs<D, false> rs;
    rs.load(g, sb, o);
    stage_face_fluxes<D>(g, flux, o, shF);
    rs.store(shs, nullptr);
  }
  __syncthreads();
  const double gp = 1.0 / kSqrt3;
  auto face = [&](auto AX, int lf, int j) -> double {
    (void)lf;
    constexpr int a = decltype(AX)::value;
    constexpr int t0 = Tang<a>::t0, t1 = Tang<a>::t1;
    int l[3], x[3];
    const int fid = tile_face<D, a>(g, o, j, l, x);
    double J = 0.0;
    if (fid >= 0) {
      const bool has_lo = x[a] >= 1, has_hi = x[a] < g.n[a];
      int lo[3] = {l[0], l[1], l[2]};
      lo[a] -= 1;
      const int hlo = TL::hidx(lo), hhi = TL::hidx(l);
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
          {
            const double xt = (q & 1) ? gp : -gp;
            sl[t0] = sh[t0] = kSqrt3 * xt;
          }
          if (D == 3) {
            const double xt = ((q >> 1) & 1) ? gp : -gp;
            sl[t1] = sh[t1] = kSqrt3 * xt;
          }
          // low side minus high side; a Dirichlet face: the cell's trace minus s_D
          const double jmp = interior ? halo_value<D>(shs, hlo, sl, g.isv) - halo_value<D>(shs, hhi, sh, g.isv)
                                      : halo_value<D>(shs, hc, sl, g.isv) - sval;
          J += jmp * wq;
        }
      }
    }
    return fabs(J);
  };
  const int tid = threadIdx.x;
  constexpr int NFI = (TL::NF + kTileThreads - 1) / kTileThreads;
  double Jr[NFI];
#pragma unroll
  for (int it = 0; it < NFI; ++it) {
    const int lf = tid + kTileThreads * it;
    Jr[it] = 0.0;
    if (lf < TL::FX)
      Jr[it] = face(std::integral_constant<int, 0>(), lf, lf);
    else if (D == 2 || lf < TL::FX + TL::FY) {
      if (lf < TL::NF) Jr[it] = face(std::integral_constant<int, 1>(), lf, lf - TL::FX);
    } else if (lf < TL::NF) {
      Jr[it] = face(std::integral_constant<int, D - 1>(), lf, lf - TL::FX - TL::FY);
    }
  }
  const int l[3] = {tid % T::X, (tid / T::X) % T::Y, tid / (T::X * T::Y)};
  const int x[3] = {o[0] + l[0], o[1] + l[1], o[2] + l[2]};
  const int h = TL::hidx(l);
  double se[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < R; ++k) se[k] = shs[k][h];
  __syncthreads();
#pragma unroll
  for (int it = 0; it < NFI; ++it) {
    const int lf = tid + kTileThreads * it;
    if (lf < TL::NF) shJ[lf] = Jr[it];
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < D; ++a)
    if (x[a] >= g.n[a]) return;
  const int nc = g.ncell, e = cell_index(g, x);
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
