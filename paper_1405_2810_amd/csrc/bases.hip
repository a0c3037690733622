// Local reduced bases on the device: Gram-Schmidt (Alg. 2 step 2e) or the
// method of snapshots (PCA, Alg. 2 step 3) of global snapshots restricted to
// every coarse box, one workgroup per box, the snapshots resident in device
// memory.
#include "common.h"

namespace lrbms {

namespace {

constexpr int kGsThreads = 256;

// Sum over the workgroup (fixed order: lanes by butterfly, then the four
// waves in order); every thread gets the result.
__device__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();   // the previous sum's readers are done with red
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// Box s: candidate vectors written into its slot region (cap vectors of
// r n_E coefficients, coefficient-major like the model's bases): the unit
// function first (when asked), then the restrictions of the snapshots in
// order; two passes of modified Gram-Schmidt against the vectors kept so
// far, rejection when the remaining L2(E) norm is <= 1e-8 of the original;
// at most cap vectors.  sizes[s] receives the number kept.  Every thread
// works on the coefficients i = tid + 256 k of a vector, so that between the
// sums (which synchronize) no thread reads another's values.
__device__ bool gs_extend_slot(double* base, long long len, int nb, double* red);

__global__ __launch_bounds__(kGsThreads) void k_local_gs(Geom g, const Sub* __restrict__ subs,
                                                        const long long* __restrict__ slot_off,
                                                        const double* __restrict__ snaps,
                                                        int nsnap, int cap, int unit,
                                                        double* __restrict__ slots,
                                                        int* __restrict__ sizes) {
  __shared__ double red[4];
  const Sub S = subs[blockIdx.x];
  const int nE = S.nE, r = g.r;
  const long long len = (long long)r * nE, L = (long long)r * g.ncell;
  const int bx = S.hi[0] - S.lo[0], by = S.hi[1] - S.lo[1];
  double* base = slots + slot_off[blockIdx.x];
  const int tid = threadIdx.x;
  int nb = 0;
  if (unit) {
    // 1_E: the constant coefficient sqrt(|e|) in every cell, normalized
    double part = 0.0;
    for (long long i = tid; i < len; i += kGsThreads) {
      const double v = i < nE ? sqrt(g.vol) : 0.0;
      base[i] = v;
      part += v * v;
    }
    const double nrm = sqrt(block_sum(part, red));
    for (long long i = tid; i < len; i += kGsThreads) base[i] = base[i] / nrm;
    nb = 1;
  }
  for (int q = 0; q < nsnap && nb < cap; ++q) {
    double* v = base + (long long)nb * len;
    const double* sq = snaps + (long long)q * L;
    double part = 0.0;
    for (long long i = tid; i < len; i += kGsThreads) {
      const int k = (int)(i / nE), l = (int)(i % nE);
      const int x[3] = {S.lo[0] + l % bx, S.lo[1] + (l / bx) % by, S.lo[2] + l / (bx * by)};
      const double a = sq[(long long)k * g.ncell + cell_index(g, x)];
      v[i] = a;
      part += a * a;
    }
    (void)part;
    if (gs_extend_slot(base, len, nb, red)) ++nb;
  }
  if (tid == 0) sizes[blockIdx.x] = nb;
}


// Coefficients per thread of a candidate that the staged form of the
// Gram-Schmidt step below holds in LDS (vectors of up to 32 x 256
// coefficients).
constexpr int kGsRegs = 32;

// The step below with the candidate staged in LDS (each thread its own
// coefficients, so no barrier beyond the sums') and this thread's
// coefficients of each kept vector loaded once per projection, for its dot
// product and its update; the candidate is written back once, when kept.
// The same operations in the same order as the form in memory.
__device__ bool gs_extend_staged(double* base, long long len, int nb, double* red) {
  __shared__ double vs[kGsRegs * kGsThreads];
  const int tid = threadIdx.x;
  double* v = base + (long long)nb * len;
  double part = 0.0;
#pragma unroll
  for (int t = 0; t < kGsRegs; ++t) {
    const long long i = tid + (long long)kGsThreads * t;
    const double x = i < len ? v[i] : 0.0;
    vs[tid + kGsThreads * t] = x;
    part += x * x;
  }
  const double nv = sqrt(block_sum(part, red));
  if (nv == 0.0) return false;
  for (int pass = 0; pass < 2; ++pass)
    for (int j = 0; j < nb; ++j) {
      const double* b = base + (long long)j * len;
      double br[kGsRegs];
#pragma unroll
      for (int t = 0; t < kGsRegs; ++t) {
        const long long i = tid + (long long)kGsThreads * t;
        br[t] = i < len ? b[i] : 0.0;
      }
      double d = 0.0;
#pragma unroll
      for (int t = 0; t < kGsRegs; ++t) d += br[t] * vs[tid + kGsThreads * t];
      const double dot = block_sum(d, red);
#pragma unroll
      for (int t = 0; t < kGsRegs; ++t) vs[tid + kGsThreads * t] -= dot * br[t];
    }
  part = 0.0;
#pragma unroll
  for (int t = 0; t < kGsRegs; ++t) {
    const double x = vs[tid + kGsThreads * t];
    part += x * x;
  }
  const double nw = sqrt(block_sum(part, red));
  if (nw <= 1e-8 * nv) return false;
#pragma unroll
  for (int t = 0; t < kGsRegs; ++t) {
    const long long i = tid + (long long)kGsThreads * t;
    if (i < len) v[i] = vs[tid + kGsThreads * t] / nw;
  }
  return true;
}

// Two-pass modified Gram-Schmidt of the candidate in slot nb against slots
// 0 .. nb-1; the candidate is normalized and kept (returns true) unless its
// remaining norm is <= 1e-8 of its norm.  Threads own the coefficients
// i = tid + 256 k.
__device__ bool gs_extend_slot(double* base, long long len, int nb, double* red) {
  if (len <= (long long)kGsRegs * kGsThreads) return gs_extend_staged(base, len, nb, red);
  const int tid = threadIdx.x;
  double* v = base + (long long)nb * len;
  double part = 0.0;
  for (long long i = tid; i < len; i += kGsThreads) part += v[i] * v[i];
  const double nv = sqrt(block_sum(part, red));
  if (nv == 0.0) return false;
  for (int pass = 0; pass < 2; ++pass)
    for (int j = 0; j < nb; ++j) {
      const double* b = base + (long long)j * len;
      double d = 0.0;
      for (long long i = tid; i < len; i += kGsThreads) d += b[i] * v[i];
      const double dot = block_sum(d, red);
      for (long long i = tid; i < len; i += kGsThreads) v[i] -= dot * b[i];
    }
  part = 0.0;
  for (long long i = tid; i < len; i += kGsThreads) part += v[i] * v[i];
  const double nw = sqrt(block_sum(part, red));
  if (nw <= 1e-8 * nv) return false;
  for (long long i = tid; i < len; i += kGsThreads) v[i] = v[i] / nw;
  return true;
}

constexpr int kMaxPcaSnaps = 64;

// Box s, the method of snapshots: the restrictions x_q of the snapshots,
// each with its components along the basis so far removed (the unit
// function when asked, one pass), into the box's region of X; their Gram
// matrix G(i, j) = x_i . x_j; its eigenpairs by cyclic Jacobi rotations
// (one wave; the 63-lane tournament order of the rotation pairs); the fewest
// leading modes whose discarded eigenvalues sum to at most eps^2 of the
// total (eigenvalues clipped at 0, modes below 1e-30 of the total dropped);
// mode i = X v_i / sqrt(lambda_i) in decreasing order, each added to the
// basis by Gram-Schmidt (as k_local_gs) while it holds fewer than cap.
__global__ __launch_bounds__(kGsThreads) void k_local_pca(Geom g, const Sub* __restrict__ subs,
                                                         const long long* __restrict__ slot_off,
                                                         const long long* __restrict__ x_off,
                                                         const double* __restrict__ snaps,
                                                         int nsnap, int cap, int unit,
                                                         double eps, double* __restrict__ slots,
                                                         double* __restrict__ X,
                                                         int* __restrict__ sizes) {
  __shared__ double red[4];
  __shared__ double G[kMaxPcaSnaps][kMaxPcaSnaps + 1];
  __shared__ double V[kMaxPcaSnaps][kMaxPcaSnaps + 1];
  __shared__ double lam[kMaxPcaSnaps];
  __shared__ int order[kMaxPcaSnaps];
  __shared__ double rot[kMaxPcaSnaps / 2][2];
  __shared__ int keep_s;
  const Sub S = subs[blockIdx.x];
  const int nE = S.nE, r = g.r, n = nsnap;
  const long long len = (long long)r * nE, L = (long long)r * g.ncell;
  const int bx = S.hi[0] - S.lo[0], by = S.hi[1] - S.lo[1];
  double* base = slots + slot_off[blockIdx.x];
  double* Xb = X + x_off[blockIdx.x];
  const int tid = threadIdx.x;
  int nb = 0;
  if (unit) {
    double part = 0.0;
    for (long long i = tid; i < len; i += kGsThreads) {
      const double v = i < nE ? sqrt(g.vol) : 0.0;
      base[i] = v;
      part += v * v;
    }
    const double nrm = sqrt(block_sum(part, red));
    for (long long i = tid; i < len; i += kGsThreads) base[i] = base[i] / nrm;
    nb = 1;
  }
  // restrictions, minus their components along the basis so far (one pass)
  for (int q = 0; q < n; ++q) {
    double* x = Xb + (long long)q * len;
    const double* sq = snaps + (long long)q * L;
    for (long long i = tid; i < len; i += kGsThreads) {
      const int k = (int)(i / nE), l = (int)(i % nE);
      const int c[3] = {S.lo[0] + l % bx, S.lo[1] + (l / bx) % by, S.lo[2] + l / (bx * by)};
      x[i] = sq[(long long)k * g.ncell + cell_index(g, c)];
    }
    for (int j = 0; j < nb; ++j) {
      const double* b = base + (long long)j * len;
      double d = 0.0;
      for (long long i = tid; i < len; i += kGsThreads) d += b[i] * x[i];
      const double dot = block_sum(d, red);
      for (long long i = tid; i < len; i += kGsThreads) x[i] -= dot * b[i];
    }
  }
  // Gram matrix (each entry a fixed-order sum)
  __syncthreads();   // X written by other threads' coefficient sets is read below
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      const double* xi = Xb + (long long)i * len;
      const double* xj = Xb + (long long)j * len;
      double d = 0.0;
      for (long long k = tid; k < len; k += kGsThreads) d += xi[k] * xj[k];
      const double v = block_sum(d, red);
      if (tid == 0) G[i][j] = G[j][i] = v;
    }
  // Jacobi eigenvalue iteration by wave 0; lane = row/column index
  const int m = n + (n & 1);   // even size for the tournament (padding row/column of zeros)
  if (tid < 64) {
    const int a = tid;
    for (int b = 0; b < m; ++b) {
      if (a < m) {
        if (a >= n || b >= n) G[a][b] = 0.0;
        V[a][b] = a == b ? 1.0 : 0.0;
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    double scale = 0.0;
    for (int i = 0; i < n; ++i) scale = fmax(scale, fabs(G[i][i]));
    for (int sweep = 0; sweep < 40; ++sweep) {
      double off = 0.0;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) off = fmax(off, fabs(G[i][j]));
      if (!(off > 1e-17 * scale)) break;
      for (int round = 0; round < m - 1; ++round) {
        // pairs of the round: positions k and m-1-k of the rotating list
        // (index m-1 fixed, the others shifted by the round)
        if (a < m / 2) {
          auto idx = [&](int pos) { return pos == m - 1 ? m - 1 : (pos + round) % (m - 1); };
          int p = idx(a), q = idx(m - 1 - a);
          if (p > q) { const int t = p; p = q; q = t; }
          const double gpq = G[p][q], gpp = G[p][p], gqq = G[q][q];
          double c = 1.0, s = 0.0;
          if (gpq != 0.0) {
            const double th = (gqq - gpp) / (2.0 * gpq);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
          rot[a][0] = c;
          rot[a][1] = s;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // rows: G <- J^T G, then columns: G <- G J, V <- V J (lane = the
        // other index)
        if (a < m) {
          for (int k = 0; k < m / 2; ++k) {
            auto idx = [&](int pos) { return pos == m - 1 ? m - 1 : (pos + round) % (m - 1); };
            int p = idx(k), q = idx(m - 1 - k);
            if (p > q) { const int t = p; p = q; q = t; }
            const double c = rot[k][0], s = rot[k][1];
            const double gp = G[p][a], gq = G[q][a];
            G[p][a] = c * gp - s * gq;
            G[q][a] = s * gp + c * gq;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (a < m) {
          for (int k = 0; k < m / 2; ++k) {
            auto idx = [&](int pos) { return pos == m - 1 ? m - 1 : (pos + round) % (m - 1); };
            int p = idx(k), q = idx(m - 1 - k);
            if (p > q) { const int t = p; p = q; q = t; }
            const double c = rot[k][0], s = rot[k][1];
            const double gp = G[a][p], gq = G[a][q];
            G[a][p] = c * gp - s * gq;
            G[a][q] = s * gp + c * gq;
            const double vp = V[a][p], vq = V[a][q];
            V[a][p] = c * vp - s * vq;
            V[a][q] = s * vp + c * vq;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
    }
    if (a == 0) {
      // eigenvalues in decreasing order (ties by index), clipped at zero
      double tot = 0.0;
      for (int i = 0; i < n; ++i) {
        lam[i] = fmax(G[i][i], 0.0);
        order[i] = i;
      }
      for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
          if (lam[order[j]] > lam[order[i]]) {
            const int t = order[i];
            order[i] = order[j];
            order[j] = t;
          }
      for (int i = 0; i < n; ++i) tot += lam[order[i]];
      int keep = n;
      for (int k = 1; k <= n; ++k) {
        double rest = 0.0;
        for (int i = k; i < n; ++i) rest += lam[order[i]];
        if (rest <= eps * eps * tot) {
          keep = k;
          break;
        }
      }
      if (!(tot > 0.0)) keep = 0;
      for (int i = 0; i < keep; ++i)
        if (lam[order[i]] <= 1e-30 * tot) {
          keep = i;
          break;
        }
      keep_s = keep;
    }
  }
  __syncthreads();
  const int keep = keep_s;
  for (int i = 0; i < keep && nb < cap; ++i) {
    const int e = order[i];
    const double w = 1.0 / sqrt(lam[e]);
    double* v = base + (long long)nb * len;
    for (long long k = tid; k < len; k += kGsThreads) {
      double acc = 0.0;
      for (int q = 0; q < n; ++q) acc += Xb[(long long)q * len + k] * V[q][e];
      v[k] = acc * w;
    }
    if (gs_extend_slot(base, len, nb, red)) ++nb;
  }
  if (tid == 0) sizes[blockIdx.x] = nb;
}

// Box s: its first sizes[s] vectors from the slot region to the model layout.
__global__ __launch_bounds__(256) void k_basis_compact(const Sub* __restrict__ subs, int r,
                                                       const long long* __restrict__ slot_off,
                                                       const long long* __restrict__ out_off,
                                                       const int* __restrict__ sizes,
                                                       const double* __restrict__ slots,
                                                       double* __restrict__ out) {
  const long long n = (long long)sizes[blockIdx.x] * r * subs[blockIdx.x].nE;
  const double* src = slots + slot_off[blockIdx.x];
  double* dst = out + out_off[blockIdx.x];
  for (long long i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// Box s: the restriction of one snapshot into the next free slot, kept by
// the Gram-Schmidt step of k_local_gs (sizes[s] grows by one) unless it is
// rejected or the box holds cap functions already.
__global__ __launch_bounds__(kGsThreads) void k_extend_gs(Geom g, const Sub* __restrict__ subs,
                                                         const long long* __restrict__ slot_off,
                                                         const double* __restrict__ snap, int cap,
                                                         double* __restrict__ slots,
                                                         int* __restrict__ sizes) {
  __shared__ double red[4];
  const Sub S = subs[blockIdx.x];
  const int nE = S.nE, nb = sizes[blockIdx.x];
  if (nb >= cap) return;
  const long long len = (long long)g.r * nE;
  const int bx = S.hi[0] - S.lo[0], by = S.hi[1] - S.lo[1];
  double* base = slots + slot_off[blockIdx.x];
  double* v = base + (long long)nb * len;
  for (long long i = threadIdx.x; i < len; i += kGsThreads) {
    const int k = (int)(i / nE), l = (int)(i % nE);
    const int x[3] = {S.lo[0] + l % bx, S.lo[1] + (l / bx) % by, S.lo[2] + l / (bx * by)};
    v[i] = snap[(long long)k * g.ncell + cell_index(g, x)];
  }
  if (gs_extend_slot(base, len, nb, red) && threadIdx.x == 0) sizes[blockIdx.x] = nb + 1;
}

template <typename T>
struct DevBuf {
  T* p = nullptr;
  bool alloc(size_t n) {
    return hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) == hipSuccess;
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

int local_bases_device(const Geom& g, const std::vector<Sub>& subs, const double* d_snaps,
                       int nsnap, int cap, bool unit, int method, double pca_eps,
                       std::vector<int>& sizes, double** d_basis, long long& len) {
  *d_basis = nullptr;
  if (method != LRBMS_BASIS_GS && method != LRBMS_BASIS_PCA)
    return (set_error("unknown basis method"), LRBMS_E_ARG);
  if (method == LRBMS_BASIS_PCA && (nsnap > kMaxPcaSnaps || !(pca_eps >= 0.0)))
    return (set_error("PCA takes at most 64 snapshots and eps >= 0"), LRBMS_E_ARG);
  const int n = (int)subs.size();
  std::vector<long long> slot_off(n), out_off(n), x_off(n);
  long long slots_len = 0, x_len = 0;
  for (int s = 0; s < n; ++s) {
    slot_off[s] = slots_len;
    slots_len += (long long)cap * g.r * subs[s].nE;
    x_off[s] = x_len;
    x_len += (long long)nsnap * g.r * subs[s].nE;
  }
  DevBuf<Sub> d_subs;
  DevBuf<long long> d_slot_off, d_out_off, d_x_off;
  DevBuf<int> d_sizes;
  DevBuf<double> d_slots, d_x;
  const bool pca = method == LRBMS_BASIS_PCA;
  if (!d_subs.alloc(n) || !d_slot_off.alloc(n) || !d_out_off.alloc(n) || !d_sizes.alloc(n) ||
      !d_slots.alloc((size_t)slots_len) || !d_x_off.alloc(n) ||
      !d_x.alloc(pca ? (size_t)x_len : 1))
    return (set_error("local bases: device allocation failed"), LRBMS_E_OOM);
  if (!hip_ok(hipMemcpy(d_subs.p, subs.data(), n * sizeof(Sub), hipMemcpyHostToDevice), "subs") ||
      !hip_ok(hipMemcpy(d_slot_off.p, slot_off.data(), n * sizeof(long long),
                        hipMemcpyHostToDevice),
              "offsets") ||
      !hip_ok(hipMemcpy(d_x_off.p, x_off.data(), n * sizeof(long long), hipMemcpyHostToDevice),
              "offsets"))
    return LRBMS_E_HIP;
  if (pca)
    hipLaunchKernelGGL(k_local_pca, dim3(n), dim3(kGsThreads), 0, 0, g, d_subs.p, d_slot_off.p,
                       d_x_off.p, d_snaps, nsnap, cap, unit ? 1 : 0, pca_eps, d_slots.p, d_x.p,
                       d_sizes.p);
  else
    hipLaunchKernelGGL(k_local_gs, dim3(n), dim3(kGsThreads), 0, 0, g, d_subs.p, d_slot_off.p,
                       d_snaps, nsnap, cap, unit ? 1 : 0, d_slots.p, d_sizes.p);
  sizes.assign(n, 0);
  if (!hip_ok(hipGetLastError(), "local Gram-Schmidt") ||
      !hip_ok(hipMemcpy(sizes.data(), d_sizes.p, n * sizeof(int), hipMemcpyDeviceToHost), "sizes"))
    return LRBMS_E_HIP;
  len = 0;
  for (int s = 0; s < n; ++s) {
    if (sizes[s] < 1) return (set_error("a box received an empty local basis"), LRBMS_E_ARG);
    out_off[s] = len;
    len += (long long)sizes[s] * g.r * subs[s].nE;
  }
  if (!hip_ok(hipMemcpy(d_out_off.p, out_off.data(), n * sizeof(long long), hipMemcpyHostToDevice),
              "offsets"))
    return LRBMS_E_HIP;
  double* out = nullptr;
  if (hipMalloc(&out, std::max<long long>(len, 1) * sizeof(double)) != hipSuccess)
    return (set_error("local bases: device allocation failed"), LRBMS_E_OOM);
  hipLaunchKernelGGL(k_basis_compact, dim3(n), dim3(256), 0, 0, d_subs.p, g.r, d_slot_off.p,
                     d_out_off.p, d_sizes.p, d_slots.p, out);
  if (!hip_ok(hipGetLastError(), "basis layout") ||
      !hip_ok(hipStreamSynchronize(0), "basis layout")) {
    (void)hipFree(out);
    return LRBMS_E_HIP;
  }
  *d_basis = out;
  return LRBMS_OK;
}

int device_bases_init(const Geom& g, const std::vector<Sub>& subs, int cap, DeviceBases& B) {
  device_bases_free(B);
  B.cap = cap;
  B.n = (int)subs.size();
  B.sizes.assign(B.n, 0);
  B.slot_off.assign(B.n, 0);
  long long total = 0;
  for (int s = 0; s < B.n; ++s) {
    B.slot_off[s] = total;
    total += (long long)cap * g.r * subs[s].nE;
  }
  if (hipMalloc(&B.d_subs, std::max(B.n, 1) * sizeof(Sub)) != hipSuccess ||
      hipMalloc(&B.d_slot_off, std::max(B.n, 1) * sizeof(long long)) != hipSuccess ||
      hipMalloc(&B.d_sizes, std::max(B.n, 1) * sizeof(int)) != hipSuccess ||
      hipMalloc(&B.d_slots, std::max<long long>(total, 1) * sizeof(double)) != hipSuccess)
    return (set_error("local bases: device allocation failed"), LRBMS_E_OOM);
  if (!hip_ok(hipMemcpy(B.d_subs, subs.data(), B.n * sizeof(Sub), hipMemcpyHostToDevice), "subs") ||
      !hip_ok(hipMemcpy(B.d_slot_off, B.slot_off.data(), B.n * sizeof(long long),
                        hipMemcpyHostToDevice),
              "offsets") ||
      !hip_ok(hipMemset(B.d_sizes, 0, std::max(B.n, 1) * sizeof(int)), "sizes"))
    return LRBMS_E_HIP;
  return LRBMS_OK;
}

int device_bases_extend(const Geom& g, DeviceBases& B, const double* d_snap, bool& grew) {
  hipLaunchKernelGGL(k_extend_gs, dim3(B.n), dim3(kGsThreads), 0, 0, g, B.d_subs, B.d_slot_off,
                     d_snap, B.cap, B.d_slots, B.d_sizes);
  std::vector<int> now(B.n);
  if (!hip_ok(hipGetLastError(), "basis extension") ||
      !hip_ok(hipMemcpy(now.data(), B.d_sizes, B.n * sizeof(int), hipMemcpyDeviceToHost), "sizes"))
    return LRBMS_E_HIP;
  grew = false;
  for (int s = 0; s < B.n; ++s) grew = grew || now[s] != B.sizes[s];
  B.sizes = now;
  return LRBMS_OK;
}

int device_bases_compact(const Geom& g, const std::vector<Sub>& subs, const DeviceBases& B,
                         double** d_basis, long long& len) {
  *d_basis = nullptr;
  std::vector<long long> out_off(B.n);
  len = 0;
  for (int s = 0; s < B.n; ++s) {
    out_off[s] = len;
    len += (long long)B.sizes[s] * g.r * subs[s].nE;
  }
  DevBuf<long long> d_out_off;
  double* out = nullptr;
  if (!d_out_off.alloc(B.n) ||
      hipMalloc(&out, std::max<long long>(len, 1) * sizeof(double)) != hipSuccess)
    return (set_error("local bases: device allocation failed"), LRBMS_E_OOM);
  if (!hip_ok(hipMemcpy(d_out_off.p, out_off.data(), B.n * sizeof(long long),
                        hipMemcpyHostToDevice),
              "offsets")) {
    (void)hipFree(out);
    return LRBMS_E_HIP;
  }
  hipLaunchKernelGGL(k_basis_compact, dim3(B.n), dim3(256), 0, 0, B.d_subs, g.r, B.d_slot_off,
                     d_out_off.p, B.d_sizes, B.d_slots, out);
  if (!hip_ok(hipGetLastError(), "basis layout") ||
      !hip_ok(hipStreamSynchronize(0), "basis layout")) {
    (void)hipFree(out);
    return LRBMS_E_HIP;
  }
  *d_basis = out;
  return LRBMS_OK;
}

void device_bases_free(DeviceBases& B) {
  for (void* q : {(void*)B.d_subs, (void*)B.d_slot_off, (void*)B.d_sizes, (void*)B.d_slots})
    if (q) (void)hipFree(q);
  B.d_subs = nullptr;
  B.d_slot_off = nullptr;
  B.d_sizes = nullptr;
  B.d_slots = nullptr;
}

}  // namespace lrbms
