"""Problem descriptions and seeded generators.

Index conventions shared by every consumer (they are data layout, not
arithmetic):

* cells are numbered ``c = i + nx*(j + ny*k)`` (x fastest); per-cell arrays
  have length ``nx*ny*nz`` (``nz = 1`` in 2D);
* faces are numbered axis by axis: all x-faces, then y-faces, then z-faces.
  The x-face at ``(i, j, k)`` with ``i in [0, nx]`` has number
  ``i + (nx+1)*(j + ny*k)``; y-faces ``i + nx*(j + (ny+1)*k)`` with
  ``j in [0, ny]``; z-faces ``i + nx*(j + ny*k)`` with ``k in [0, nz]``.
  Per-face arrays have one entry per face (interior entries are ignored);
* boundary tags: ``bc_type`` 0 = interior, 1 = Neumann (outward flux density
  ``bc_val``), 2 = Dirichlet pressure (``bc_val``); ``bc_sat`` 1 marks a
  saturation Dirichlet (inflow) face with value ``bc_sval``.

Units are SI.  Physical constants for the configurations are listed in
``CONFIGS``; the seeded fields follow the recipes in the module functions.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

BC_INTERIOR, BC_NEUMANN, BC_DIRICHLET = 0, 1, 2
RELPERM_LINEAR, RELPERM_COREY = 0, 1
WEIGHTS_SWIP, WEIGHTS_LITERAL = 0, 1


@dataclasses.dataclass
class Problem:
    dim: int
    n: tuple                      # (nx, ny, nz); nz = 1 in 2D
    L: tuple                      # domain lengths (Lx, Ly, Lz); Lz = 1 in 2D
    cuts: List[np.ndarray]        # coarse box cut indices per axis (nc[a]+1 each)
    perm: np.ndarray              # [ncell] scalar permeability (m^2)
    poro: np.ndarray              # [ncell] porosity
    visc_w: float
    visc_o: float
    relperm: int                  # RELPERM_LINEAR or RELPERM_COREY
    corey_w: float
    corey_o: float
    bc_type: np.ndarray           # [nface] int8
    bc_val: np.ndarray            # [nface] float64
    bc_sat: np.ndarray            # [nface] int8
    bc_sval: np.ndarray           # [nface] float64
    q1: np.ndarray                # [ncell] pressure source density (1/s)
    q2: np.ndarray                # [ncell] saturation source density (1/s)
    penalty_c: float              # c_f of the penalty parameter
    weights: int                  # WEIGHTS_SWIP or WEIGHTS_LITERAL
    sat_penalty_scale: float      # multiplies sigma_f in the saturation equation
    limiter: int                  # 1 = apply the slope limiter after each Euler step
    dt: float
    n_steps: int = 1
    # offline options
    M: int = 8                    # number of mobility profiles
    n_train: int = 8              # number of training snapshots
    ne_cap: int = 10              # maximum local basis size N_E
    basis_method: str = "gs"      # "gs" or "pca"
    pca_eps: float = 1e-4
    unit_functions: bool = True   # put 1_E first in every local basis
    t_end: float = 0.0            # horizon T of the mobility profiles (0: n_steps * dt)
    seed: int = 0
    name: str = ""
    # densities and gravity of the problem statement; no configuration here
    # has gravity, so the densities never enter the equations
    dens_w: float = 1000.0
    dens_o: float = 1000.0
    grav: tuple = (0.0, 0.0, 0.0)

    @property
    def ncell(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def nc(self) -> tuple:
        return tuple(len(c) - 1 for c in self.cuts)

    @property
    def nface(self) -> int:
        return int(sum(face_counts(self.dim, self.n)))

    @property
    def h(self) -> tuple:
        return tuple(self.L[a] / self.n[a] for a in range(3))

    def copy(self, **kw) -> "Problem":
        d = {f.name: getattr(self, f.name) for f in dataclasses.fields(self)}
        for k, v in d.items():
            if isinstance(v, np.ndarray):
                d[k] = v.copy()
            elif isinstance(v, list):
                d[k] = [np.array(x) for x in v]
        d.update(kw)
        return Problem(**d)


def face_counts(dim: int, n: Sequence[int]) -> tuple:
    nx, ny, nz = n
    fx = (nx + 1) * ny * nz
    fy = nx * (ny + 1) * nz
    fz = nx * ny * (nz + 1) if dim == 3 else 0
    return fx, fy, fz


def _face_ids(dim, n, axis, sel):
    """Face numbers of the faces along ``axis`` whose (i, j, k) satisfy sel."""
    nx, ny, nz = n
    fx, fy, fz = face_counts(dim, n)
    ext = [nx, ny, nz]
    ext[axis] += 1
    k, j, i = np.meshgrid(np.arange(ext[2]), np.arange(ext[1]), np.arange(ext[0]),
                          indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    m = sel(i, j, k)
    off = [0, fx, fx + fy][axis]
    return off + (i + ext[0] * (j + ext[1] * k))[m]


def gaussian_field(shape, h, corr_len, rng) -> np.ndarray:
    """Zero-mean, unit-variance Gaussian field with squared-exponential
    covariance exp(-r^2 / (2 l^2)), by FFT filtering of white noise on a grid
    padded to twice the size in every direction.

    ``shape`` is (nz, ny, nx) (C order, x fastest); ``h`` the cell sizes in the
    same order.  The result is rescaled to unit sample variance.
    """
    pshape = [2 * s for s in shape]
    noise = rng.standard_normal(pshape)
    k2 = np.zeros(pshape)
    for ax, (ps, hh) in enumerate(zip(pshape, h)):
        kk = 2.0 * np.pi * np.fft.fftfreq(ps, d=hh)
        sh = [1] * len(pshape)
        sh[ax] = ps
        k2 = k2 + (kk ** 2).reshape(sh)
    filt = np.exp(-0.25 * k2 * corr_len ** 2)
    g = np.real(np.fft.ifftn(np.fft.fftn(noise) * filt))
    g = g[tuple(slice(0, s) for s in shape)]
    g = g - g.mean()
    sd = g.std()
    return g / sd if sd > 0 else g


def even_cuts(n: int, nc: int) -> np.ndarray:
    return np.array([(i * n) // nc for i in range(nc + 1)], dtype=np.int32)


def seeded_cuts(n: int, nc: int, rng, min_width: int) -> np.ndarray:
    """Uneven cut positions: nc boxes with widths >= min_width."""
    free = n - nc * min_width
    assert free >= 0
    w = rng.dirichlet(np.ones(nc)) * free
    wi = np.floor(w).astype(int)
    rem = free - wi.sum()
    wi[np.argsort(-(w - wi))[:rem]] += 1
    widths = wi + min_width
    return np.concatenate([[0], np.cumsum(widths)]).astype(np.int32)


def random_saturation(prob: Problem, rng, lo=0.0, hi=1.0, slope=0.2) -> np.ndarray:
    """A random P1 saturation state in the L2-orthonormal cell basis
    (coefficient k of cell c at index k*ncell + c).  Cell means are uniform in
    [lo+slope, hi-slope] and every slope coefficient keeps all vertex values
    inside [lo, hi]."""
    nce = prob.ncell
    d = prob.dim
    vol = float(np.prod(prob.h[:d]))
    r = d + 1
    s = np.zeros(r * nce)
    mean = rng.uniform(lo + slope, hi - slope, nce)
    s[:nce] = mean * math.sqrt(vol)
    for a in range(d):
        # value = |e|^-1/2 (c0 + sqrt(3) sum_a c_a xi_a); bound each slope term
        s[(a + 1) * nce:(a + 2) * nce] = (rng.uniform(-1, 1, nce) * slope / d
                                         * math.sqrt(vol) / math.sqrt(3.0))
    return s


def smooth_fields(prob: Problem, count: int, rng, corr: float = 0.3) -> list:
    """Seeded smooth random P1 fields (SoA, orthonormal cell basis): cell
    means from a Gaussian field of correlation length ``corr`` times the
    domain size, small random slopes.  Timing inputs only."""
    nx, ny, nz = prob.n
    d = prob.dim
    vol = float(np.prod(prob.h[:d]))
    out = []
    for _ in range(count):
        shape = (ny, nx) if d == 2 else (nz, ny, nx)
        hh = (prob.h[1], prob.h[0]) if d == 2 else (prob.h[2], prob.h[1], prob.h[0])
        g = gaussian_field(shape, hh, corr * max(prob.L[:d]), rng).ravel()
        f = np.zeros((d + 1) * prob.ncell)
        f[:prob.ncell] = g * math.sqrt(vol)
        f[prob.ncell:] = 0.05 * rng.standard_normal(d * prob.ncell) * math.sqrt(vol)
        out.append(f)
    return out


def wave_fields(prob: Problem, count: int, rng) -> list:
    """Seeded plane-wave P1 fields (SoA, orthonormal cell basis): cell means
    sin(k . x + phase) at the cell centres with seeded wave vectors of up to
    four periods across the domain, small random slopes.  Cheap stand-ins
    for snapshots when only timing matters."""
    d = prob.dim
    vol = float(np.prod(prob.h[:d]))
    axes = [(np.arange(prob.n[a]) + 0.5) / prob.n[a] for a in range(d)]
    X = np.meshgrid(*axes[::-1], indexing="ij")[::-1]   # x fastest in ravel order
    out = []
    for _ in range(count):
        k = rng.uniform(-4.0, 4.0, d) * 2.0 * math.pi
        ph = rng.uniform(0.0, 2.0 * math.pi)
        g = np.sin(sum(k[a] * X[a] for a in range(d)) + ph).ravel()
        f = np.zeros((d + 1) * prob.ncell)
        f[:prob.ncell] = g * math.sqrt(vol)
        f[prob.ncell:] = 0.05 * rng.standard_normal(d * prob.ncell) * math.sqrt(vol)
        out.append(f)
    return out


def ensemble_caps(prob: Problem, rng, lo: int = 5, hi: int = 60) -> np.ndarray:
    """Seeded local basis size per coarse box (lexicographic box order),
    uniform in [lo, hi]."""
    n_sub = int(np.prod([len(c) - 1 for c in prob.cuts[:prob.dim]]))
    return rng.integers(lo, hi + 1, n_sub).astype(np.int32)


def training_params(M: int, n_train: int, rng) -> np.ndarray:
    """Training parameters mu in the simplex (sum 1, entries >= 1e-4): first
    the M unit vectors (the profiles themselves), then seeded Dirichlet
    draws."""
    rows = [np.eye(M)[q] for q in range(min(M, n_train))]
    for _ in range(max(0, n_train - M)):
        mu = rng.dirichlet(np.ones(M))
        mu = np.maximum(mu, 1e-4)
        rows.append(mu / mu.sum())
    return np.array(rows)


# ----------------------------------------------------------------------------
# Configurations.  ``Q`` (injection rate) and ``dt`` are fixed constants per
# configuration (set so that the initial injector-producer pressure drop is of
# order 1e6 Pa and the explicit transport step stays within a CFL number of
# about 0.2); see make_problem for the rest of the recipe.
CONFIGS: Dict[str, dict] = {
    # 2D unit square, 64x64, 4x4 coarse boxes, quarter five-spot
    "cfg1": dict(dim=2, n=(64, 64, 1), L=(1.0, 1.0, 1.0), nc=(4, 4, 1), corr=0.1,
                 sigma=1.0, ratio=10.0, steps=20, M=8, n_train=10, ne_cap=10,
                 wells="quarter5", Q=2.0e-6, dt=1.6, seed=11, t_end=4.0e4),
    # 2D 256x256, 16x16 coarse boxes
    "cfg2": dict(dim=2, n=(256, 256, 1), L=(1.0, 1.0, 1.0), nc=(16, 16, 1), corr=0.05,
                 sigma=2.0, ratio=5.0, steps=200, M=16, n_train=26, ne_cap=25,
                 wells="quarter5", Q=1.2e-6, dt=0.2, seed=22, t_end=8.0e4),
    # 3D layered + channelized 60x220x85 on 600x2200x170 m, 6x22x5 coarse boxes
    "cfg3": dict(dim=3, n=(60, 220, 85), L=(600.0, 2200.0, 170.0), nc=(6, 22, 5),
                 corr=0.1, sigma=3.0, ratio=10.0, steps=100, M=16, n_train=41,
                 ne_cap=40, wells="five3d", Q=1.0e-2, dt=1.0e4, seed=33, t_end=2.0e9,
                 channels=True),
    # the 3D workload's coarse grid (6x22x5 boxes, N_E = 40, sigma_logk = 3 with
    # channels) on a fine grid half as fine per axis (30x110x40 cells), small
    # enough for the oracle's element-by-element parity
    "cfg3s": dict(dim=3, n=(30, 110, 40), L=(600.0, 2200.0, 170.0), nc=(6, 22, 5),
                  corr=0.1, sigma=3.0, ratio=10.0, steps=100, M=16, n_train=41,
                  ne_cap=40, wells="five3d", Q=1.0e-2, dt=1.0e4, seed=33, t_end=2.0e9,
                  channels=True),
    # shaped like the paper's 2D benchmark (Sec. 6): [0,300] x [0,60] m, 400 x 160
    # cells, linear relative permeabilities, the printed viscosities, water
    # entering on the left (p = 10, s = 1), outward flux 3e-4 on the right,
    # no flow on top and bottom, no sources, T = 3e5 s; its permeability and
    # porosity fields are not given, so a seeded log-normal field
    # (kappa_g = 1e-10 m^2) and porosity 0.2 stand in; 8 x 2 boxes.  The
    # printed step (50 s, 6000 steps) gives this stand-in a CFL number of
    # 1.3 (its flow concentrates in the high-permeability streaks), so the
    # step is 15 s (CFL about 0.4, 20000 steps)
    "paper": dict(dim=2, n=(400, 160, 1), L=(300.0, 60.0, 1.0), nc=(8, 2, 1), corr=0.1 * 300.0,
                  sigma=1.0, steps=6000, M=8, n_train=8, ne_cap=25, wells="paper", Q=0.0,
                  dt=15.0, seed=44, t_end=3.0e5, kg=1.0e-10, visc_w=0.00130581, visc_o=0.008,
                  relperm=0, p_left=10.0, v_right=3.0e-4),
    # ensemble members: 2D 256x256 and 3D 64x64x32 on seeded uneven coarse
    # partitions (boxes of 16..48 cells per side in 2D, 8..24 x 8..24 x 4..12
    # in 3D), local basis sizes drawn per box by ensemble_caps
    "ens2d": dict(dim=2, n=(256, 256, 1), L=(1.0, 1.0, 1.0), nc=(8, 8, 1), corr=0.05,
                  sigma=2.0, ratio=5.0, steps=200, M=16, n_train=26, ne_cap=60,
                  wells="quarter5", Q=1.2e-6, dt=0.2, seed=101, uneven=True, t_end=8.0e4),
    "ens3d": dict(dim=3, n=(64, 64, 32), L=(640.0, 640.0, 64.0), nc=(4, 4, 4), corr=0.1,
                  sigma=3.0, ratio=10.0, steps=100, M=16, n_train=26, ne_cap=60,
                  wells="five3d", Q=4.0e-3, dt=1.0e4, seed=201, uneven=True, t_end=2.0e9),
    # small cases for tests
    "tiny2d": dict(dim=2, n=(8, 8, 1), L=(1.0, 1.0, 1.0), nc=(2, 2, 1), corr=0.2,
                   sigma=1.0, ratio=10.0, steps=5, M=4, n_train=6, ne_cap=6,
                   wells="quarter5", Q=5.0e-6, dt=40.0, seed=5, t_end=1.0e4),
    "small2d": dict(dim=2, n=(32, 24, 1), L=(1.0, 0.75, 1.0), nc=(3, 2, 1), corr=0.1,
                    sigma=1.0, ratio=10.0, steps=10, M=6, n_train=9, ne_cap=8,
                    wells="quarter5", Q=5.0e-6, dt=2.5, seed=7, uneven=True, t_end=1.5e4),
    "small3d": dict(dim=3, n=(12, 10, 6), L=(120.0, 100.0, 12.0), nc=(2, 2, 2),
                    corr=0.2, sigma=1.0, ratio=10.0, steps=5, M=5, n_train=8,
                    ne_cap=8, wells="five3d", Q=1.0e-3, dt=5.0e3, seed=9, t_end=1.5e7),
}


def make_problem(name: str, seed: Optional[int] = None, **overrides) -> Problem:
    """Instantiate a named configuration.

    Recipe: kappa = 1e-13 * exp(sigma * g), g from ``gaussian_field`` (2D: one
    field; 3D: one 2D field per layer with a seeded per-layer offset, plus
    seeded sinuous channels of kappa = 1e-13 * e^6 when ``channels``);
    porosity 0.2; water viscosity 1e-3 Pa s, oil viscosity ``ratio`` times
    that; quadratic Corey relative permeabilities; no gravity; s0 = 0.
    Wells: ``quarter5`` puts the injector source in cell (0, 0) and the
    producer as Dirichlet p = 0 on the outer faces of cell (nx-1, ny-1);
    ``five3d`` puts a uniform-rate injector column at the centre and Dirichlet
    p = 0 producers on the lateral outer faces of the four corner columns.
    All other boundary faces are no-flow Neumann faces.  The injected fluid is
    water (q2 = q1).
    """
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    if seed is None:
        seed = cfg["seed"]
    rng = np.random.default_rng(seed)
    dim = cfg["dim"]
    n = tuple(cfg["n"])
    L = tuple(cfg["L"])
    nx, ny, nz = n
    h = [L[a] / n[a] for a in range(3)]
    vol = h[0] * h[1] * (h[2] if dim == 3 else 1.0)
    kg = cfg.get("kg", 1e-13)
    if dim == 2:
        g = gaussian_field((ny, nx), (h[1], h[0]), cfg["corr"], rng)
        g = g.reshape(1, ny, nx)
    else:
        lat = cfg["corr"] * max(L[0], L[1])
        base = gaussian_field((ny, nx), (h[1], h[0]), lat, rng)
        g = np.empty((nz, ny, nx))
        for k in range(nz):
            layer = gaussian_field((ny, nx), (h[1], h[0]), lat, rng)
            g[k] = 0.5 * base + 0.5 * layer + 0.5 * rng.standard_normal()
        g = (g - g.mean()) / g.std()
    logk = cfg["sigma"] * g
    perm = kg * np.exp(logk)
    if cfg.get("channels"):
        xs = (np.arange(nx) + 0.5) * h[0]
        ys = (np.arange(ny) + 0.5) * h[1]
        n_ch = max(1, nz // 8)
        for _ in range(n_ch):
            k0 = int(rng.integers(0, nz - 3))
            thick = int(rng.integers(2, 5))
            y0 = rng.uniform(0.2, 0.8) * L[1]
            amp = rng.uniform(0.05, 0.15) * L[1]
            wl = rng.uniform(0.3, 0.8) * L[0]
            ph = rng.uniform(0, 2 * np.pi)
            width = rng.uniform(0.02, 0.05) * L[1]
            yc = y0 + amp * np.sin(2 * np.pi * xs / wl + ph)
            mask = np.abs(ys[:, None] - yc[None, :]) < 0.5 * width   # (ny, nx)
            for k in range(k0, min(nz, k0 + thick)):
                perm[k][mask] = kg * math.exp(6.0)
    perm = perm.ravel().astype(np.float64)
    poro = np.full(nx * ny * nz, 0.2)

    nf = face_counts(dim, n)
    nface = sum(nf)
    bc_type = np.zeros(nface, dtype=np.int8)
    bc_val = np.zeros(nface)
    bc_sat = np.zeros(nface, dtype=np.int8)
    bc_sval = np.zeros(nface)
    # every boundary face: no-flow Neumann
    for a in range(dim):
        ids = _face_ids(dim, n, a, lambda i, j, k, a=a, ext=n:
                        ((i, j, k)[a] == 0) | ((i, j, k)[a] == ext[a]))
        bc_type[ids] = BC_NEUMANN
    q1 = np.zeros(nx * ny * nz)
    Q = cfg["Q"]
    if cfg["wells"] == "quarter5":
        q1[0] = Q / vol
        prod_x = _face_ids(dim, n, 0, lambda i, j, k: (i == nx) & (j == ny - 1))
        prod_y = _face_ids(dim, n, 1, lambda i, j, k: (i == nx - 1) & (j == ny))
        bc_type[prod_x] = BC_DIRICHLET
        bc_type[prod_y] = BC_DIRICHLET
    elif cfg["wells"] == "five3d":
        ic, jc = nx // 2, ny // 2
        for k in range(nz):
            q1[ic + nx * (jc + ny * k)] = Q / (nz * vol)
        for (ci, cj) in [(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)]:
            fx = _face_ids(dim, n, 0, lambda i, j, k, ci=ci, cj=cj:
                           (j == cj) & (i == (0 if ci == 0 else nx)))
            fy = _face_ids(dim, n, 1, lambda i, j, k, ci=ci, cj=cj:
                           (i == ci) & (j == (0 if cj == 0 else ny)))
            bc_type[fx] = BC_DIRICHLET
            bc_type[fy] = BC_DIRICHLET
    elif cfg["wells"] == "paper":
        # left: p = p_left and s = 1; right: outward flux v_right; others no flow
        left = _face_ids(dim, n, 0, lambda i, j, k: i == 0)
        right = _face_ids(dim, n, 0, lambda i, j, k: i == nx)
        bc_type[left] = BC_DIRICHLET
        bc_val[left] = cfg.get("p_left", 10.0)
        bc_sat[left] = 1
        bc_sval[left] = 1.0
        bc_val[right] = cfg.get("v_right", 3e-4)
    else:
        raise ValueError(cfg["wells"])
    q2 = q1.copy()

    if cfg.get("uneven"):
        cuts = [seeded_cuts(n[a], cfg["nc"][a], rng, max(2, n[a] // (2 * cfg["nc"][a])))
                if a < dim else np.array([0, 1], dtype=np.int32) for a in range(3)]
    else:
        cuts = [even_cuts(n[a], cfg["nc"][a]) if a < dim else np.array([0, 1], dtype=np.int32)
                for a in range(3)]

    visc_w = cfg.get("visc_w", 1e-3)
    visc_o = cfg.get("visc_o", cfg.get("ratio", 1.0) * visc_w)
    c0 = 4.0 if dim == 2 else 30.0
    penalty_c = c0 * max(visc_w, visc_o) / min(visc_w, visc_o)
    return Problem(dim=dim, n=n, L=L if dim == 3 else (L[0], L[1], 1.0), cuts=cuts,
                   perm=perm, poro=poro, visc_w=visc_w, visc_o=visc_o,
                   relperm=cfg.get("relperm", RELPERM_COREY), corey_w=cfg.get("corey_w", 2.0),
                   corey_o=cfg.get("corey_o", 2.0),
                   bc_type=bc_type, bc_val=bc_val, bc_sat=bc_sat, bc_sval=bc_sval,
                   q1=q1, q2=q2, penalty_c=penalty_c, weights=cfg.get("weights", WEIGHTS_SWIP),
                   sat_penalty_scale=1.0, limiter=cfg.get("limiter", 1), dt=cfg["dt"],
                   n_steps=cfg["steps"],
                   M=cfg["M"], n_train=cfg["n_train"], ne_cap=cfg["ne_cap"],
                   basis_method=cfg.get("basis_method", "gs"),
                   pca_eps=cfg.get("pca_eps", 1e-4), unit_functions=True,
                   t_end=cfg.get("t_end", 0.0),
                   seed=seed, name=name)
