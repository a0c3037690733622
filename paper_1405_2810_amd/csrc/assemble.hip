// Reduced assembly on gfx950.
//
// Mobility moments (a1), the Galerkin projection A_N = Phi^T A(gamma) Phi and
// f_N = Phi^T l(gamma) of the SWIP forms of Sec. 3.2 onto the broken reduced
// space W_N (Def. coarseScalePressure), the affine sum of eq. reducedSystem
// and the least-squares fit of eq. leastSquaresFit.
//
// Readings of the printed forms used throughout (same as the CPU reference):
// consistency terms with a minus sign, Neumann term -int v_N w, SWIP mean
// weights (or the literal ones on request), two-valued mobility on faces
// (each side of the weighted mean uses its own trace), outward normal and
// weight 1 on Dirichlet faces, h_f = face diameter, zero gravity.
//
// The box kernel evaluates the r x r stencil blocks of the fine operator once
// per cell into LDS, applies them to the columns of Phi_E sixteen cells at a
// time, and contracts Phi_E^T (K Phi_E) on FP64 MFMA; the right-hand side
// rides along as one more column.  The interface kernel does the same for the
// fine faces of one coarse interface.  Everything is templated on the
// dimension so that per-dof arrays stay in registers.
#include <algorithm>

#include "common.h"
#include "ktimer.h"
#include "swip.h"

namespace lrbms {

// ---------------------------------------------------------------------------
// a1: mobility moments per cell.  gamma is lambda(s_h) (kind GAMMA_SAT), a P1
// field (GAMMA_FIELD) or sum_q theta_q Lambda^q (GAMMA_COMBO); integrals by the
// 2-point Gauss rules, which are exact for the quadratic mobility of a P1 state.
template <int D, int KIND>
__global__ __launch_bounds__(256) void k_moments(Geom g, const double* __restrict__ src,
                                                 const double* __restrict__ theta, int nprof,
                                                 long long pstride, double* __restrict__ mom) {
  constexpr int R = D + 1;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  const int nc = g.ncell;
  double co[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (KIND == GAMMA_COMBO) {
      double v = 0.0;
      for (int q = 0; q < nprof; ++q) v += theta[q] * src[q * pstride + (long long)k * nc + c];
      co[k] = v;
    } else {
      co[k] = src[(long long)k * nc + c];
    }
  }
  // value of gamma at local point xi (sq holds sqrt(3) xi_a)
  auto gam = [&](const double (&sq)[3]) {
    double v = co[0];
#pragma unroll
    for (int a = 0; a < D; ++a) v += sq[a] * co[a + 1];
    v *= g.isv;
    return KIND == GAMMA_SAT ? total_mobility(g, v) : v;
  };
  const double gp = 1.0 / kSqrt3;
  double sq[3] = {0.0, 0.0, 0.0};
  double sum = 0.0;
  constexpr int nq = 1 << D;
#pragma unroll
  for (int p = 0; p < nq; ++p) {
#pragma unroll
    for (int a = 0; a < D; ++a) sq[a] = kSqrt3 * (((p >> a) & 1) ? gp : -gp);
    sum += gam(sq);
  }
  double out[1 + 2 * D * D];
  out[0] = sum * g.vol / nq;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    int tax[2] = {0, 0}, nt = 0;
#pragma unroll
    for (int b = 0; b < D; ++b)
      if (b != a) tax[nt++] = b;
    const double w = g.area[a] / (1 << (D - 1));
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
      double m0 = 0.0, mt[2] = {0.0, 0.0};
#pragma unroll
      for (int p = 0; p < (1 << (D - 1)); ++p) {
        double xi[3] = {0.0, 0.0, 0.0};
        xi[a] = dir ? 1.0 : -1.0;
#pragma unroll
        for (int ti = 0; ti < D - 1; ++ti) xi[tax[ti]] = ((p >> ti) & 1) ? gp : -gp;
#pragma unroll
        for (int b = 0; b < D; ++b) sq[b] = kSqrt3 * xi[b];
        const double v = gam(sq);
        m0 += v;
#pragma unroll
        for (int ti = 0; ti < D - 1; ++ti) mt[ti] += v * xi[tax[ti]];
      }
      const int s0 = mom_slot(D, a, dir);
      out[s0] = m0 * w;
#pragma unroll
      for (int ti = 0; ti < D - 1; ++ti) out[s0 + 1 + ti] = mt[ti] * w;
    }
  }
#pragma unroll
  for (int k = 0; k < 1 + 2 * D * D; ++k) mom[(long long)k * nc + c] = out[k];
}

hipError_t launch_moments(const Geom& g, const double* src, int kind, const double* theta,
                          int nprof, long long prof_stride, double* mom, hipStream_t st) {
  const int nb = (g.ncell + 255) / 256;
  ktimer_begin(KK_MOMENTS, st);
#define LRBMS_MOMENTS(D, K)                                                                  \
  hipLaunchKernelGGL((k_moments<D, K>), dim3(nb), dim3(256), 0, st, g, src, theta, nprof,      \
                     prof_stride, mom)
  if (g.dim == 2) {
    if (kind == GAMMA_SAT) LRBMS_MOMENTS(2, GAMMA_SAT);
    else if (kind == GAMMA_FIELD) LRBMS_MOMENTS(2, GAMMA_FIELD);
    else LRBMS_MOMENTS(2, GAMMA_COMBO);
  } else {
    if (kind == GAMMA_SAT) LRBMS_MOMENTS(3, GAMMA_SAT);
    else if (kind == GAMMA_FIELD) LRBMS_MOMENTS(3, GAMMA_FIELD);
    else LRBMS_MOMENTS(3, GAMMA_COMBO);
  }
#undef LRBMS_MOMENTS
  ktimer_end(-1.0, -1.0, st);
  return hipGetLastError();
}

// c += a b for 16 x 16 blocks and an inner dimension of 4 (FP64 MFMA): lane l
// supplies a(l % 16, l / 16) and b(l / 16, l % 16); element (l / 16 + 4 v, l % 16)
// of the result is c[v].
typedef double d4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Cells per workgroup chunk and per staged piece of the box assembly.
template <int D> struct AsmShape {
  static constexpr int R = D + 1;
  static constexpr int NF = 1 + 2 * D;          // self block + one per face
  static constexpr int CH = 64;                 // cells per chunk
  // LDS doubles per cell of stencil blocks: odd, so that the 16 cells one
  // wave reads at a time fall in different banks
  static constexpr int KS = (NF * R * R) | 1;
  static constexpr int PC = 16;                 // cells per staged piece
  static constexpr int PR = PC * R;             // rows per staged piece
};

// Staged Phi and Y rows of one piece: row (cell p, dof k) at p G + k LDP.
// G is odd, so the sixteen lanes of a store (sixteen cells, one column) use
// sixteen different banks; with G = R LDP, even in 3D, four of them shared
// one.  The contraction reads row 4 c + q at sixteen consecutive columns per
// sixteen lanes, free of conflicts at any stride.
template <int D, int NEP> struct Staged {
  static constexpr int R = AsmShape<D>::R, PC = AsmShape<D>::PC, LDP = NEP + 1;
  static constexpr int G = (R * LDP) | 1;
  static constexpr int size = PC * G;          // doubles per array
  static_assert(R == 4 || G == R * LDP, "rows of one cell adjacent unless R = 4");
  __device__ static constexpr int at(int p, int k) { return p * G + k * LDP; }
  __device__ static constexpr int row(int rw) {
    if constexpr (R == 4) return at(rw >> 2, rw & 3);
    else return rw * LDP;
  }
};

// 3D boxes with up to 47 basis functions: the apply phase loads one axis of
// neighbours at a time and chunks hold 32 cells, so that a workgroup needs
// at most 244 registers per lane and 79 KB of LDS (two workgroups per CU);
// elsewhere all loads of a thread are issued first and chunks hold 64 cells.
template <int D, int NEP> struct BoxPlan {
  static constexpr bool kPhased = D == 3 && NEP <= 48;
  static constexpr int CH = kPhased ? 32 : AsmShape<D>::CH;
};


template <int D, int NEP>
__host__ __device__ constexpr size_t box_lds_doubles() {
  using S = AsmShape<D>;
  return (size_t)BoxPlan<D, NEP>::CH * S::KS + 2 * (size_t)Staged<D, NEP>::size;
}

// The one-item variant of the box assembly: six waves per workgroup and one
// (cell, column) item per thread and piece, so that a thread holds the Phi
// values of one cell and of its 2d neighbours (one load round trip per
// piece); chunks of 30 (3D) or 64 (2D) cells keep a workgroup at or below
// 53 KB of LDS and 128 registers per lane.  Rows per piece rounded up to a
// multiple of 4 (zero rows) for the contraction.
template <int D, int NEP> struct Box1 {
  static constexpr int NT = 384;
  static constexpr int R = D + 1;
  static constexpr int PC = NT / NEP;          // cells per piece
  static constexpr int PR = PC * R;            // rows per piece
  static constexpr int PRP = (PR + 3) / 4 * 4;
  static constexpr int CH = D == 3 ? 30 : 64;  // cells per chunk
  static constexpr int LDP = NEP + 1;
  static constexpr int NTI = NEP / 16, NT2 = NTI * NTI, TPW = (NT2 + 5) / 6;
  static_assert(NT % NEP == 0, "one item per thread");
  static constexpr size_t lds_doubles = (size_t)CH * AsmShape<D>::KS + 2 * (size_t)PRP * LDP;
};

int box_chunk_cells(int dim, int nep, int variant) {
  if (variant == 1) return dim == 3 ? Box1<3, 64>::CH : Box1<2, 64>::CH;
  return (dim == 3 && nep <= 48) ? 32 : 64;
}

template <int D, int NEP>
__host__ __device__ constexpr size_t iface_lds_doubles() {
  return 2 * (size_t)Staged<D, NEP>::size;
}

// Diagonal blocks A[E][E] and f_E, one workgroup per (box, chunk of cells):
//   stencil   the self and neighbour blocks of every cell of the chunk, once
//             per (cell, trial dof), into LDS;
//   apply     for 16 cells at a time, Y = K Phi for every (cell, column) pair
//             (coalesced reads of the column-major Phi^E; neighbours outside
//             the box contribute nothing), staged in LDS with the Phi rows;
//             the right-hand side l_h rides along as column N_E;
//   contract  partial(i, j) += sum_rows Phi(row, i) Y(row, j) on FP64 MFMA,
//             16 x 16 output tiles spread over the four waves.
// The chunk partials of a box are summed in chunk order by k_reduce_box.
template <int D, int NEP>
__global__ __launch_bounds__(256) void k_asm_box(Geom g, const Sub* __restrict__ subs,
                                                 const int* __restrict__ chunks,
                                                 const double* __restrict__ phi,
                                                 const double* __restrict__ mom, int parts,
                                                 double* __restrict__ partial) {
  using SH = AsmShape<D>;
  using ST = Staged<D, NEP>;
  constexpr int R = SH::R, NF = SH::NF, PC = SH::PC, PR = SH::PR;
  constexpr int NTI = NEP / 16, NT2 = NTI * NTI, TPW = (NT2 + 3) / 4;
  extern __shared__ double lds[];
  constexpr int CH = BoxPlan<D, NEP>::CH;
  double* Kst = lds;                                   // [CH][KS >= NF R R]
  double* PhiS = Kst + (size_t)CH * SH::KS;            // Staged rows
  double* YS = PhiS + ST::size;                        // Staged rows
  // consecutive chunks of a box share the Phi rows of their neighbour cells
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const int sub = chunks[2 * item], c0 = chunks[2 * item + 1];
  const Sub S = subs[sub];
  const int NE = S.NE, nE = S.nE;
  const int cc = min(CH, nE - c0);
  const int ext[3] = {S.hi[0] - S.lo[0], S.hi[1] - S.lo[1], S.hi[2] - S.lo[2]};
  const int tid = threadIdx.x;
  const bool want_mat = parts & (PART_GAMMA | PART_PEN);
  const bool want_rhs = parts & (PART_RHS_CONST | PART_RHS_GAMMA);
  auto box_xyz = [&](int l, int (&x)[3]) {
    x[0] = S.lo[0] + l % ext[0];
    x[1] = S.lo[1] + (l / ext[0]) % ext[1];
    x[2] = S.lo[2] + l / (ext[0] * ext[1]);
  };
  // stencil
  if (want_mat) {
    for (int it = tid; it < cc * R; it += 256) {
      const int lc = it % cc, kp = it / cc;
      int x[3];
      box_xyz(c0 + lc, x);
      const int e = cell_index(g, x);
      double self[R], nbr[2 * D][R];
      cell_stencil<D>(g, S, e, x, mom, parts, kp, self, nbr);
      double* K = Kst + (size_t)lc * SH::KS;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        K[k * R + kp] = self[k];
#pragma unroll
        for (int f = 0; f < 2 * D; ++f) K[((1 + f) * R + k) * R + kp] = nbr[f][k];
      }
    }
  }
  __syncthreads();
  const int lane = tid & 63, w = tid >> 6, r = lane & 15, q = lane >> 4;
  const int nJ = NE / 16 + 1, nlive = ((NE + 15) / 16) * nJ;   // live output tiles
  d4 acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  constexpr int IT = PC * NEP / 256;             // (cell, column) items per thread and piece
  constexpr int NB = 2 * D;
  for (int p0 = 0; p0 < cc; p0 += PC) {
    const int lp = tid % PC, lc = p0 + lp;
    double ps[IT][R], Y[IT][R];
    if constexpr (BoxPlan<D, NEP>::kPhased) {
      // apply, one axis at a time: self values, then the two neighbours along
      // each axis (the loads of a phase issued together; the phases kept
      // apart so that one phase's registers serve the next)
      const int l = c0 + lc;
      const int bl[3] = {l % ext[0], (l / ext[0]) % ext[1], l / (ext[0] * ext[1])};
      const int bst[3] = {1, ext[0], ext[0] * ext[1]};
#pragma unroll
      for (int u = 0; u < IT; ++u) {
        const int col = (tid + 256 * u) / PC;
        const bool live = lc < cc && col < NE;
        const double* cp = phi + S.phi_off + (long long)col * R * nE;
#pragma unroll
        for (int k = 0; k < R; ++k) {
          ps[u][k] = live ? cp[(long long)k * nE + l] : 0.0;
          Y[u][k] = 0.0;
        }
      }
      const double* K = Kst + (size_t)(lc < cc ? lc : 0) * SH::KS;
      if (lc < cc && want_mat) {
#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
          for (int kp = 0; kp < R; ++kp) {
            const double kv = K[k * R + kp];
#pragma unroll
            for (int u = 0; u < IT; ++u) Y[u][k] = fma(kv, ps[u][kp], Y[u][k]);
          }
      }
#pragma unroll
      for (int a = 0; a < D; ++a) {
        asm volatile("" ::: "memory");   // keep the next phase's loads here
        double po[IT][2][R];
#pragma unroll
        for (int u = 0; u < IT; ++u) {
          const int col = (tid + 256 * u) / PC;
          const bool live = lc < cc && col < NE;
          const double* cp = phi + S.phi_off + (long long)col * R * nE;
#pragma unroll
          for (int dir = 0; dir < 2; ++dir) {
            const int ba = bl[a] + (dir ? 1 : -1);
            const bool in = live && want_mat && ba >= 0 && ba < ext[a];
            const int ln = l + (dir ? bst[a] : -bst[a]);
#pragma unroll
            for (int k = 0; k < R; ++k) po[u][dir][k] = in ? cp[(long long)k * nE + ln] : 0.0;
          }
        }
        if (lc < cc && want_mat) {
#pragma unroll
          for (int dir = 0; dir < 2; ++dir)
#pragma unroll
            for (int k = 0; k < R; ++k)
#pragma unroll
              for (int kp = 0; kp < R; ++kp) {
                const double kv = K[((1 + 2 * a + dir) * R + k) * R + kp];
#pragma unroll
                for (int u = 0; u < IT; ++u) Y[u][k] = fma(kv, po[u][dir][kp], Y[u][k]);
              }
        }
      }
    } else {
      // apply: the Phi values of all items of this thread are loaded first
      double po[IT][NB][R];
#pragma unroll
      for (int u = 0; u < IT; ++u) {
        const int it = tid + 256 * u;
        const int col = it / PC;
        const int l = c0 + lc;
        const bool live = lc < cc && col < NE;
        const double* cp = phi + S.phi_off + (long long)col * R * nE;
        const int bl[3] = {l % ext[0], (l / ext[0]) % ext[1], l / (ext[0] * ext[1])};
        const int bst[3] = {1, ext[0], ext[0] * ext[1]};
#pragma unroll
        for (int k = 0; k < R; ++k) ps[u][k] = live ? cp[(long long)k * nE + l] : 0.0;
#pragma unroll
        for (int f = 0; f < NB; ++f) {
          const int a = f >> 1, dir = f & 1;
          const int ba = bl[a] + (dir ? 1 : -1);
          const bool in = live && want_mat && ba >= 0 && ba < ext[a];
          const int ln = l + (dir ? bst[a] : -bst[a]);
#pragma unroll
          for (int k = 0; k < R; ++k) po[u][f][k] = in ? cp[(long long)k * nE + ln] : 0.0;
        }
      }
      // Y = K Phi for all items of this thread (one cell, IT columns: 256 is a
      // multiple of PC), each stencil value read from LDS once; columns beyond
      // N_E have zero Phi and so zero Y
#pragma unroll
      for (int u = 0; u < IT; ++u)
#pragma unroll
        for (int k = 0; k < R; ++k) Y[u][k] = 0.0;
      if (lc < cc && want_mat) {
        const double* K = Kst + (size_t)lc * SH::KS;
#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
          for (int kp = 0; kp < R; ++kp) {
            const double kv = K[k * R + kp];
#pragma unroll
            for (int u = 0; u < IT; ++u) Y[u][k] = fma(kv, ps[u][kp], Y[u][k]);
          }
#pragma unroll
        for (int f = 0; f < NB; ++f)
#pragma unroll
          for (int k = 0; k < R; ++k)
#pragma unroll
            for (int kp = 0; kp < R; ++kp) {
              const double kv = K[((1 + f) * R + k) * R + kp];
#pragma unroll
              for (int u = 0; u < IT; ++u) Y[u][k] = fma(kv, po[u][f][kp], Y[u][k]);
            }
      }
    }
#pragma unroll
    for (int u = 0; u < IT; ++u) {
      const int col = (tid + 256 * u) / PC;
      if (lc < cc && col == NE && want_rhs) {
        int x[3];
        box_xyz(c0 + lc, x);
#pragma unroll
        for (int k = 0; k < R; ++k) Y[u][k] = 0.0;
        cell_rhs<D>(g, cell_index(g, x), x, mom, parts, Y[u]);
      }
#pragma unroll
      for (int k = 0; k < R; ++k) {
        PhiS[ST::at(lp, k) + col] = ps[u][k];
        YS[ST::at(lp, k) + col] = Y[u][k];
      }
    }
    __syncthreads();
    // contract: only the 16 x 16 tiles that hold rows < N_E and columns
    // <= N_E (the rest of the padded width is zero), spread over the waves
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tile = w + 4 * t;
      if (tile < nlive) {
        const int I = tile / nJ, J = tile % nJ;
#pragma unroll
        for (int c = 0; c < PR / 4; ++c)
          acc[t] = mfma16(PhiS[ST::row(4 * c + q) + 16 * I + r],
                          YS[ST::row(4 * c + q) + 16 * J + r], acc[t]);
      }
    }
    __syncthreads();
  }
  double* out = partial + (size_t)item * NEP * NEP;
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int tile = w + 4 * t;
    if (tile < nlive) {
      const int I = tile / nJ, J = tile % nJ;
#pragma unroll
      for (int v = 0; v < 4; ++v) out[(size_t)(16 * I + q + 4 * v) * NEP + 16 * J + r] = acc[t][v];
    }
  }
}

// Diagonal blocks A[E][E] and f_E, the one-item variant (Box1): one
// workgroup of six waves per (box, chunk), the steps of k_asm_box:
//   stencil   the self and neighbour blocks of every cell of the chunk into LDS;
//   apply     for PC = 384 / NEP cells at a time, thread (cell, column) loads
//             the Phi values of its cell and of the cell's 2d neighbours at
//             once and forms Y = K Phi (the right-hand side l_h as column
//             N_E); Phi and Y rows staged in LDS;
//   contract  partial(i, j) += sum_rows Phi(row, i) Y(row, j) on FP64 MFMA,
//             16 x 16 output tiles spread over the six waves.
template <int D, int NEP>
__global__ __launch_bounds__(384, 4) void k_asm_box1(Geom g, const Sub* __restrict__ subs,
                                                     const int* __restrict__ chunks,
                                                     const double* __restrict__ phi,
                                                     const double* __restrict__ mom, int parts,
                                                     double* __restrict__ partial) {
  using B = Box1<D, NEP>;
  using SH = AsmShape<D>;
  constexpr int R = B::R, PC = B::PC, PR = B::PR, PRP = B::PRP, LDP = B::LDP, CH = B::CH;
  constexpr int NT = B::NT, NTI = B::NTI, NT2 = B::NT2, TPW = B::TPW, NB = 2 * D;
  extern __shared__ double lds[];
  double* Kst = lds;                                   // [CH][KS]
  double* PhiS = Kst + (size_t)CH * SH::KS;            // [PRP][LDP]
  double* YS = PhiS + (size_t)PRP * LDP;               // [PRP][LDP]
  // consecutive chunks of a box share the Phi rows of their neighbour cells
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const int sub = chunks[2 * item], c0 = chunks[2 * item + 1];
  const Sub S = subs[sub];
  const int NE = S.NE, nE = S.nE;
  const int cc = min(CH, nE - c0);
  const int ext[3] = {S.hi[0] - S.lo[0], S.hi[1] - S.lo[1], S.hi[2] - S.lo[2]};
  const int tid = threadIdx.x;
  const bool want_mat = parts & (PART_GAMMA | PART_PEN);
  const bool want_rhs = parts & (PART_RHS_CONST | PART_RHS_GAMMA);
  auto box_xyz = [&](int l, int (&x)[3]) {
    x[0] = S.lo[0] + l % ext[0];
    x[1] = S.lo[1] + (l / ext[0]) % ext[1];
    x[2] = S.lo[2] + l / (ext[0] * ext[1]);
  };
  // the padding rows of the contraction stay zero
  for (int i = tid; i < (PRP - PR) * LDP; i += NT) {
    PhiS[(size_t)PR * LDP + i] = 0.0;
    YS[(size_t)PR * LDP + i] = 0.0;
  }
  if (want_mat) {
    for (int it = tid; it < cc * R; it += NT) {
      const int lc = it % cc, kp = it / cc;
      int x[3];
      box_xyz(c0 + lc, x);
      const int e = cell_index(g, x);
      double self[R], nbr[NB][R];
      cell_stencil<D>(g, S, e, x, mom, parts, kp, self, nbr);
      double* K = Kst + (size_t)lc * SH::KS;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        K[k * R + kp] = self[k];
#pragma unroll
        for (int f = 0; f < NB; ++f) K[((1 + f) * R + k) * R + kp] = nbr[f][k];
      }
    }
  }
  __syncthreads();
  const int lane = tid & 63, w = tid >> 6, r = lane & 15, q = lane >> 4;
  // only the output tiles that hold rows < N_E and columns <= N_E
  const int nJ = NE / 16 + 1, nlive = ((NE + 15) / 16) * nJ;
  d4 acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  const int lp = tid % PC, col = tid / PC;
  const double* cp = phi + S.phi_off + (long long)min(col, NE - 1) * R * nE;
  const int bst[3] = {1, ext[0], ext[0] * ext[1]};
  for (int p0 = 0; p0 < cc; p0 += PC) {
    const int lc = p0 + lp, l = c0 + lc;
    const bool cell = lc < cc, live = cell && col < NE;
    const int bl[3] = {l % ext[0], (l / ext[0]) % ext[1], l / (ext[0] * ext[1])};
    double ps[R], po[NB][R], Y[R];
#pragma unroll
    for (int k = 0; k < R; ++k) ps[k] = live ? cp[(long long)k * nE + l] : 0.0;
#pragma unroll
    for (int f = 0; f < NB; ++f) {
      const int a = f >> 1, dir = f & 1;
      const int ba = bl[a] + (dir ? 1 : -1);
      const bool in = live && want_mat && ba >= 0 && ba < ext[a];
      const int ln = l + (dir ? bst[a] : -bst[a]);
#pragma unroll
      for (int k = 0; k < R; ++k) po[f][k] = in ? cp[(long long)k * nE + ln] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) Y[k] = 0.0;
    if (cell && want_mat) {
      const double* K = Kst + (size_t)lc * SH::KS;
#pragma unroll
      for (int k = 0; k < R; ++k)
#pragma unroll
        for (int kp = 0; kp < R; ++kp) Y[k] = fma(K[k * R + kp], ps[kp], Y[k]);
#pragma unroll
      for (int f = 0; f < NB; ++f) {
        // one block's stencil values in flight at a time (register budget)
        asm volatile("" ::: "memory");
#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
          for (int kp = 0; kp < R; ++kp) Y[k] = fma(K[((1 + f) * R + k) * R + kp], po[f][kp], Y[k]);
      }
    }
    if (cell && col == NE && want_rhs) {
      int x[3];
      box_xyz(l, x);
#pragma unroll
      for (int k = 0; k < R; ++k) Y[k] = 0.0;
      cell_rhs<D>(g, cell_index(g, x), x, mom, parts, Y);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
      PhiS[(size_t)(lp * R + k) * LDP + col] = ps[k];
      YS[(size_t)(lp * R + k) * LDP + col] = Y[k];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tile = w + 6 * t;
      if (tile < nlive) {
        const int I = tile / nJ, J = tile % nJ;
#pragma unroll
        for (int c = 0; c < PRP / 4; ++c)
          acc[t] = mfma16(PhiS[(size_t)(4 * c + q) * LDP + 16 * I + r],
                          YS[(size_t)(4 * c + q) * LDP + 16 * J + r], acc[t]);
      }
    }
    __syncthreads();
  }
  double* out = partial + (size_t)item * NEP * NEP;
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int tile = w + 6 * t;
    if (tile < nlive) {
      const int I = tile / nJ, J = tile % nJ;
#pragma unroll
      for (int v = 0; v < 4; ++v) out[(size_t)(16 * I + q + 4 * v) * NEP + 16 * J + r] = acc[t][v];
    }
  }
}

// Sum the chunk partials of every box in chunk order; write A[E][E] and f_E.
// Workgroup (box, y) takes entries 256 y .. 256 y + 255 of the box's
// NE x (NE + 1) values; eight chunks' loads are issued before their sums.
template <int NEP>
__global__ __launch_bounds__(256) void k_reduce_box(const Sub* __restrict__ subs,
                                                    const int* __restrict__ first_chunk,
                                                    const double* __restrict__ partial,
                                                    int has_mat, int has_rhs,
                                                    double* __restrict__ blocks,
                                                    double* __restrict__ fN) {
  constexpr int U = 8;
  const Sub S = subs[blockIdx.x];
  const int q0 = first_chunk[blockIdx.x], q1 = first_chunk[blockIdx.x + 1];
  const int NE = S.NE, ncol = NE + 1;
  const int idx = blockIdx.y * 256 + threadIdx.x;
  if (idx >= NE * ncol) return;
  const int i = idx / ncol, j = idx % ncol;
  const double* src = partial + (size_t)i * NEP + j;
  double v = 0.0;
  int c = q0;
  for (; c + U <= q1; c += U) {
    double t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) t[u] = src[(size_t)(c + u) * NEP * NEP];
#pragma unroll
    for (int u = 0; u < U; ++u) v += t[u];
  }
  for (; c < q1; ++c) v += src[(size_t)c * NEP * NEP];
  if (j < NE) {
    if (has_mat) blocks[S.blk_off + (long long)i * NE + j] = v;
  } else if (has_rhs) {
    fN[S.pn_off + i] = v;
  }
}

// Coupling block A[lo][hi] of one coarse interface, one workgroup per
// interface: for 16 fine faces at a time, Y(row, j) = the face terms of the
// lo-side test dofs against basis function j of the hi box, staged in LDS with
// the lo-side Phi rows, then contracted on FP64 MFMA.  The Phi values on both
// sides come from the interface's face traces (k_face_traces).
template <int D, int A, int NEP>
__device__ __forceinline__ void iface_body(const Geom& g, const Sub& SL, const Sub& SH2,
                                           const Iface& I, const double* __restrict__ tr,
                                           const double* __restrict__ mom, int parts,
                                           double* __restrict__ blocks, double* PhiS, double* YS) {
  using SHP = AsmShape<D>;
  using ST = Staged<D, NEP>;
  constexpr int R = SHP::R, PC = SHP::PC, PR = SHP::PR;
  constexpr int NTI = NEP / 16, NT2 = NTI * NTI, TPW = (NT2 + 3) / 4;
  constexpr int T0 = (A == 0) ? 1 : 0, T1 = (A == 2) ? 1 : 2;
  const int NL = SL.NE, NH = SH2.NE;
  // only the output tiles that hold rows < N_lo and columns < N_hi
  const int nJ = (NH + 15) / 16, nlive = ((NL + 15) / 16) * nJ;
  const bool gam = parts & PART_GAMMA, pen = parts & PART_PEN;
  const int ext0 = SL.hi[T0] - SL.lo[T0];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, r = lane & 15, q = lane >> 4;
  const double zero[R] = {};
  d4 acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  constexpr int IT = PC * NEP / 256;   // columns per thread and piece, all on one fine face
  const int lq = tid % PC;
  for (int q0 = 0; q0 < I.nf; q0 += PC) {
    // the fine face of this thread: cells on both sides, moments, permeabilities
    const int fq = q0 + lq;
    const bool live = fq < I.nf;
    int x0[3] = {0, 0, 0}, x1[3];
    x0[A] = SL.hi[A] - 1;
    x0[T0] = SL.lo[T0] + (live ? fq : 0) % ext0;
    if (D == 3) x0[T1] = SL.lo[T1] + (live ? fq : 0) / ext0;
    for (int b = 0; b < 3; ++b) x1[b] = x0[b];
    x1[A] = SH2.lo[A];
    const int e0 = cell_index(g, x0), e1 = cell_index(g, x1);
    double ms[D], mo[D];
    face_moments<D>(g, mom, e0, A, 1, ms);
    face_moments<D>(g, mom, e1, A, 0, mo);
    const double k0 = g.perm[e0], k1 = g.perm[e1];
    // face traces of every column of this thread (contiguous over the fine
    // faces), loaded before any arithmetic
    double po[IT][R], pl[IT][R];
    const double* tl = tr + I.tr_off;
    const double* th = tl + (long long)NL * R * I.nf;
#pragma unroll
    for (int u = 0; u < IT; ++u) {
      const int col = (tid + 256 * u) / PC;
      const bool hi_ok = live && col < NH, lo_ok = live && col < NL;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        po[u][k] = hi_ok ? th[((long long)col * R + k) * I.nf + fq] : 0.0;
        pl[u][k] = lo_ok ? tl[((long long)col * R + k) * I.nf + fq] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < IT; ++u) {
      const int col = (tid + 256 * u) / PC;
      double Y[R];
#pragma unroll
      for (int k = 0; k < R; ++k) Y[k] = 0.0;
      if (live && col < NH)
        face_terms<D, A>(g, 1.0, true, k0, k1, ms, mo, zero, po[u], gam, pen, Y);
#pragma unroll
      for (int k = 0; k < R; ++k) {
        PhiS[ST::at(lq, k) + col] = pl[u][k];
        YS[ST::at(lq, k) + col] = Y[k];
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tile = w + 4 * t;
      if (tile < nlive) {
        const int Ti = tile / nJ, Tj = tile % nJ;
#pragma unroll
        for (int c = 0; c < PR / 4; ++c)
          acc[t] = mfma16(PhiS[ST::row(4 * c + q) + 16 * Ti + r],
                          YS[ST::row(4 * c + q) + 16 * Tj + r], acc[t]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int tile = w + 4 * t;
    if (tile < nlive) {
      const int Ti = tile / nJ, Tj = tile % nJ;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * Ti + q + 4 * v, j = 16 * Tj + r;
        if (i < NL && j < NH) blocks[I.blk_off + (long long)i * NH + j] = acc[t][v];
      }
    }
  }
}

template <int D, int NEP>
__global__ __launch_bounds__(256) void k_asm_iface(Geom g, const Sub* __restrict__ subs,
                                                   const Iface* __restrict__ ifs,
                                                   const double* __restrict__ tr,
                                                   const double* __restrict__ mom, int parts,
                                                   double* __restrict__ blocks) {
  extern __shared__ double lds[];
  double* PhiS = lds;
  double* YS = lds + Staged<D, NEP>::size;
  const Iface I = ifs[blockIdx.x];
  const Sub SL = subs[I.lo], SH2 = subs[I.hi];
  if (I.axis == 0)
    iface_body<D, 0, NEP>(g, SL, SH2, I, tr, mom, parts, blocks, PhiS, YS);
  else if (I.axis == 1)
    iface_body<D, 1, NEP>(g, SL, SH2, I, tr, mom, parts, blocks, PhiS, YS);
  else if constexpr (D == 3)
    iface_body<D, 2, NEP>(g, SL, SH2, I, tr, mom, parts, blocks, PhiS, YS);
}

// Face traces of the local bases, one workgroup per coarse interface: for
// fine face q of the interface (q = t0 + ext0 t1 over the tangential axes of
// the low box), the r coefficients of every basis function of the low box at
// its cell on the face and of the high box at its cell across it, stored
// (function, coefficient, q) with q fastest, so that the interface assembly
// reads them contiguously.  Set-up work, once per model.
__global__ __launch_bounds__(256) void k_face_traces(Geom g, const Sub* __restrict__ subs,
                                                     const Iface* __restrict__ ifs,
                                                     const double* __restrict__ phi,
                                                     double* __restrict__ tr) {
  const Iface I = ifs[blockIdx.x];
  const Sub SL = subs[I.lo], SH = subs[I.hi];
  const int A = I.axis, T0 = (A == 0) ? 1 : 0, T1 = (A == 2) ? 1 : 2, r = g.r;
  const int ext0 = SL.hi[T0] - SL.lo[T0];
  const long long nlo = (long long)SL.NE * r * I.nf, n = nlo + (long long)SH.NE * r * I.nf;
  for (long long idx = threadIdx.x; idx < n; idx += blockDim.x) {
    const bool lo = idx < nlo;
    const long long j = lo ? idx : idx - nlo;
    const int q = (int)(j % I.nf), k = (int)((j / I.nf) % r), col = (int)(j / ((long long)I.nf * r));
    const Sub& S = lo ? SL : SH;
    int x[3] = {0, 0, 0};
    x[A] = lo ? SL.hi[A] - 1 : SH.lo[A];
    x[T0] = SL.lo[T0] + q % ext0;
    if (g.dim == 3) x[T1] = SL.lo[T1] + q / ext0;
    const int ex0 = S.hi[0] - S.lo[0], ex1 = S.hi[1] - S.lo[1];
    const int l = (x[0] - S.lo[0]) + ex0 * ((x[1] - S.lo[1]) + ex1 * (x[2] - S.lo[2]));
    tr[I.tr_off + idx] = phi[S.phi_off + ((long long)col * r + k) * S.nE + l];
  }
}

hipError_t launch_face_traces(const Geom& g, const Sub* d_subs, const Iface* d_ifaces, int n_iface,
                              const double* phi, double* tr, hipStream_t st) {
  if (n_iface == 0) return hipSuccess;
  hipLaunchKernelGGL(k_face_traces, dim3(n_iface), dim3(256), 0, st, g, d_subs, d_ifaces, phi, tr);
  return hipGetLastError();
}

int assemble_cols(int max_ne) { return ((max_ne + 1 + 15) / 16) * 16; }

template <int D, int NEP>
static hipError_t launch_assemble_t(const AsmLayout& L, const Geom& g, const Sub* d_subs,
                                    int n_sub, const Iface* d_ifaces, int n_iface,
                                    const double* phi, const double* tr, const double* mom,
                                    int parts, double* blocks, double* fN, hipStream_t st) {
  const bool has_mat = (parts & (PART_GAMMA | PART_PEN)) && blocks;
  const bool has_rhs = (parts & (PART_RHS_CONST | PART_RHS_GAMMA)) && fN;
  const int pdiag = (has_mat ? (PART_GAMMA | PART_PEN) & parts : 0) |
                    (has_rhs ? (PART_RHS_CONST | PART_RHS_GAMMA) & parts : 0);
  if (n_sub > 0 && pdiag) {
    ktimer_begin(KK_ASM_DIAG, st);
    using B1 = Box1<D, NEP>;
    constexpr size_t lds0 = sizeof(double) * box_lds_doubles<D, NEP>();
    constexpr size_t lds1 = sizeof(double) * B1::lds_doubles;
    if (L.variant == 1) {
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_asm_box1<D, NEP>), dim3(L.n_chunks), dim3(B1::NT), lds1,
                         st, g, d_subs, L.chunks, phi, mom, pdiag, L.partial);
    } else {
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_asm_box<D, NEP>), dim3(L.n_chunks), dim3(256), lds0, st,
                         g, d_subs, L.chunks, phi, mom, pdiag, L.partial);
    }
    ktimer_end(-1.0, -1.0, st);
    ktimer_begin(KK_ASM_REDUCE, st);
    // NE (NE + 1) < NEP^2 values per box (NE < NEP), NEP a multiple of 16
    constexpr int kSplit = NEP * NEP / 256;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_reduce_box<NEP>), dim3(n_sub, kSplit), dim3(256), 0, st, d_subs,
                       L.first_chunk, L.partial, has_mat ? 1 : 0, has_rhs ? 1 : 0, blocks, fN);
    ktimer_end(-1.0, -1.0, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (n_iface > 0 && has_mat) {
    const size_t lds = sizeof(double) * iface_lds_doubles<D, NEP>();
    ktimer_begin(KK_ASM_IFACE, st);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_asm_iface<D, NEP>), dim3(n_iface), dim3(256), lds, st, g,
                       d_subs, d_ifaces, tr, mom, parts, blocks);
    ktimer_end(-1.0, -1.0, st);
    return hipGetLastError();
  }
  return hipSuccess;
}

template <int D, int NEP>
static hipError_t set_lds_limits() {
  hipError_t e = hipFuncSetAttribute((const void*)k_asm_box<D, NEP>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(sizeof(double) * box_lds_doubles<D, NEP>()));
  if (e != hipSuccess) return e;
  using B1 = Box1<D, NEP>;
  e = hipFuncSetAttribute((const void*)k_asm_box1<D, NEP>,
                          hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(sizeof(double) * B1::lds_doubles));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_asm_iface<D, NEP>,
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(sizeof(double) * iface_lds_doubles<D, NEP>()));
}

template <int D>
static hipError_t set_lds_limits_d(int nep) {
  switch (nep) {
    case 16: return set_lds_limits<D, 16>();
    case 32: return set_lds_limits<D, 32>();
    case 48: return set_lds_limits<D, 48>();
    default: return set_lds_limits<D, 64>();
  }
}

hipError_t assemble_prepare(const Geom& g, const std::vector<Sub>& subs, int max_ne,
                            int variant, AsmLayout& L, long long& bytes) {
  if (max_ne + 1 > 64 || variant < 0 || variant > 1) return hipErrorInvalidValue;
  L.variant = variant;
  std::vector<int> chunks, first(1, 0);
  const int ch = box_chunk_cells(g.dim, assemble_cols(max_ne), variant);
  for (size_t s = 0; s < subs.size(); ++s) {
    for (int c0 = 0; c0 < subs[s].nE; c0 += ch) {
      chunks.push_back((int)s);
      chunks.push_back(c0);
    }
    first.push_back((int)chunks.size() / 2);
  }
  L.n_chunks = (int)chunks.size() / 2;
  const int nep = assemble_cols(max_ne);
  hipError_t e;
  if ((e = hipMalloc(&L.chunks, chunks.size() * sizeof(int))) != hipSuccess) return e;
  if ((e = hipMemcpy(L.chunks, chunks.data(), chunks.size() * sizeof(int),
                     hipMemcpyHostToDevice)) != hipSuccess)
    return e;
  if ((e = hipMalloc(&L.first_chunk, first.size() * sizeof(int))) != hipSuccess) return e;
  if ((e = hipMemcpy(L.first_chunk, first.data(), first.size() * sizeof(int),
                     hipMemcpyHostToDevice)) != hipSuccess)
    return e;
  const size_t np = (size_t)L.n_chunks * nep * nep;
  if ((e = hipMalloc(&L.partial, np * sizeof(double))) != hipSuccess) return e;
  bytes += (long long)(np * sizeof(double) + (chunks.size() + first.size()) * sizeof(int));
  return g.dim == 2 ? set_lds_limits_d<2>(nep) : set_lds_limits_d<3>(nep);
}

void assemble_free(AsmLayout& L) {
  if (L.chunks) (void)hipFree(L.chunks);
  if (L.first_chunk) (void)hipFree(L.first_chunk);
  if (L.partial) (void)hipFree(L.partial);
  L = AsmLayout{};
}

template <int D>
static hipError_t launch_assemble_d(const AsmLayout& L, const Geom& g, const Sub* d_subs,
                                    int n_sub, int max_ne, const Iface* d_ifaces, int n_iface,
                                    const double* phi, const double* tr, const double* mom,
                                    int parts, double* blocks, double* fN, hipStream_t st) {
  switch (assemble_cols(max_ne)) {
    case 16:
      return launch_assemble_t<D, 16>(L, g, d_subs, n_sub, d_ifaces, n_iface, phi, tr, mom, parts,
                                      blocks, fN, st);
    case 32:
      return launch_assemble_t<D, 32>(L, g, d_subs, n_sub, d_ifaces, n_iface, phi, tr, mom, parts,
                                      blocks, fN, st);
    case 48:
      return launch_assemble_t<D, 48>(L, g, d_subs, n_sub, d_ifaces, n_iface, phi, tr, mom, parts,
                                      blocks, fN, st);
    default:
      return launch_assemble_t<D, 64>(L, g, d_subs, n_sub, d_ifaces, n_iface, phi, tr, mom, parts,
                                      blocks, fN, st);
  }
}

hipError_t launch_assemble(const AsmLayout& L, const Geom& g, const Sub* d_subs, int n_sub,
                           int max_ne, const Iface* d_ifaces, int n_iface, const double* phi,
                           const double* tr, const double* mom, int parts, double* blocks,
                           double* fN, hipStream_t st) {
  if (g.dim == 2)
    return launch_assemble_d<2>(L, g, d_subs, n_sub, max_ne, d_ifaces, n_iface, phi, tr, mom,
                                parts, blocks, fN, st);
  return launch_assemble_d<3>(L, g, d_subs, n_sub, max_ne, d_ifaces, n_iface, phi, tr, mom,
                              parts, blocks, fN, st);
}

// ---------------------------------------------------------------------------
// eq. reducedSystem: out = base + sum_q theta_q terms[q] (q in increasing order).
__global__ __launch_bounds__(256) void k_affine_sum(const double* __restrict__ base,
                                                    const double* __restrict__ terms, long long n,
                                                    const double* __restrict__ theta, int nq,
                                                    double* __restrict__ out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    double v = base[i];
    for (int q = 0; q < nq; ++q) v = v + theta[q] * terms[(long long)q * n + i];
    out[i] = v;
  }
}

hipError_t launch_affine_sum(const double* base, const double* terms, long long n,
                             const double* theta, int nq, double* out, hipStream_t st) {
  long long nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  if (nb < 1) nb = 1;
  ktimer_begin(KK_AFFINE_SUM, st);
  hipLaunchKernelGGL(k_affine_sum, dim3((unsigned)nb), dim3(256), 0, st, base, terms, n, theta,
                     nq, out);
  ktimer_end(2.0 * (double)n * nq, 8.0 * (double)n * (nq + 2), st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// eq. leastSquaresFit: r_q = (Lambda^q, Pi lambda(s))_{L2} with the P1
// projection Pi lambda(s) evaluated by the 2-point Gauss rule; theta solves
// G theta = r with the Cholesky factor of the profile Gram matrix G.  Each
// thread projects kLsqCells cells (strided by the workgroup size, so that the
// reads stay coalesced), then one block reduction per profile.
constexpr int kLsqCells = 4;

int lsq_blocks(int ncell) { return (ncell + 256 * kLsqCells - 1) / (256 * kLsqCells); }

template <int D>
__global__ __launch_bounds__(256) void k_lsq_partial(Geom g, const double* __restrict__ sat,
                                                     const double* __restrict__ prof, int nprof,
                                                     double* __restrict__ partial) {
  constexpr int R = D + 1, NQ = 1 << D;
  __shared__ double red[4];
  const int nc = g.ncell, tid = threadIdx.x;
  const double gp = 1.0 / kSqrt3, w = g.vol / NQ;
  double lp[kLsqCells][R];
#pragma unroll
  for (int t = 0; t < kLsqCells; ++t) {
    const int c = (blockIdx.x * kLsqCells + t) * 256 + tid;
#pragma unroll
    for (int k = 0; k < R; ++k) lp[t][k] = 0.0;
    if (c >= nc) continue;
    double co[R];
#pragma unroll
    for (int k = 0; k < R; ++k) co[k] = sat[(long long)k * nc + c];
#pragma unroll
    for (int p = 0; p < NQ; ++p) {
      double sq[D];
      double v = co[0];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        sq[a] = kSqrt3 * (((p >> a) & 1) ? gp : -gp);
        v += sq[a] * co[a + 1];
      }
      const double lam = total_mobility(g, v * g.isv) * w;
      lp[t][0] += lam * g.isv;
#pragma unroll
      for (int a = 0; a < D; ++a) lp[t][a + 1] += lam * sq[a] * g.isv;
    }
  }
  for (int q = 0; q < nprof; ++q) {
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < kLsqCells; ++t) {
      const int c = (blockIdx.x * kLsqCells + t) * 256 + tid;
      if (c < nc) {
#pragma unroll
        for (int k = 0; k < R; ++k)
          s = fma(prof[(long long)q * R * nc + (long long)k * nc + c], lp[t][k], s);
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((tid & 63) == 0) red[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) partial[(long long)blockIdx.x * nprof + q] = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
  }
}

__global__ void k_lsq_final(const double* __restrict__ partial, int nblocks, int nprof,
                            const double* __restrict__ L, double* __restrict__ theta) {
  __shared__ double y[kMaxProfiles];
  const int q = threadIdx.x;
  if (q < nprof) {
    double v = 0.0;
    for (int b = 0; b < nblocks; ++b) v += partial[(long long)b * nprof + q];
    y[q] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // forward then backward substitution with the lower Cholesky factor L
    for (int i = 0; i < nprof; ++i) {
      double v = y[i];
      for (int k = 0; k < i; ++k) v -= L[i * nprof + k] * y[k];
      y[i] = v / L[i * nprof + i];
    }
    for (int i = nprof - 1; i >= 0; --i) {
      double v = y[i];
      for (int k = i + 1; k < nprof; ++k) v -= L[k * nprof + i] * y[k];
      y[i] = v / L[i * nprof + i];
    }
    for (int i = 0; i < nprof; ++i) theta[i] = y[i];
  }
}

hipError_t launch_lsq(const Geom& g, const double* sat, const double* prof, int nprof,
                      const double* gchol, double* partial, int nblocks, double* theta,
                      hipStream_t st) {
  ktimer_begin(KK_LSQ, st);
  if (g.dim == 2)
    hipLaunchKernelGGL(k_lsq_partial<2>, dim3(nblocks), dim3(256), 0, st, g, sat, prof, nprof,
                       partial);
  else
    hipLaunchKernelGGL(k_lsq_partial<3>, dim3(nblocks), dim3(256), 0, st, g, sat, prof, nprof,
                       partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lsq_final, dim3(1), dim3(64), 0, st, partial, nblocks, nprof, gchol, theta);
  ktimer_end(-1.0, -1.0, st);
  return hipGetLastError();
}

}  // namespace lrbms
