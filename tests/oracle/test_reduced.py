"""Pins of the oracle's reduced (LRBMS) method: limit cases and identities
stated in the paper or implied by the Galerkin structure."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from synth import make_problem, random_saturation, training_params
from oracle.fem import Grid
from oracle.pressure import Mobility, fine_pressure, reconstruct_flux
from oracle.offline import (local_bases, subdomain_cells, build_offline, dedupe_profiles,
                            greedy, pca_modes, restrict, training_mobility, mobility_profiles)
from oracle.online import (Model, online_step, reduced_system, solve_reduced, lsq_theta,
                           projected_mobility, DIRECT, DIRECT_FIT, AFFINE)
from oracle.schemes import fine_impes, lrbms_impes


def test_full_local_spaces_give_fine_solution():
    """T_H local spaces equal to V_h restricted to each box (every fine dof a
    basis function): the reduced space is V_h and the reduced pressure is
    the fine pressure (the limit case discussed after Alg. 2)."""
    p = make_problem("tiny2d")
    g = Grid(p)
    s = random_saturation(p, np.random.default_rng(1))
    phis = local_bases(g, p, [], method="full")
    m = Model(p, phis)
    out = online_step(m, s, DIRECT)
    ph = fine_pressure(g, p, s=s)
    assert np.abs(out["ph"] - ph).max() <= 1e-9 * np.abs(ph).max()


def test_lrbms_full_space_equals_fine_impes():
    """With full local spaces, Alg. 3 (DIRECT) reproduces Alg. 1 step for step."""
    p = make_problem("tiny2d")
    g = Grid(p)
    m = Model(p, local_bases(g, p, [], method="full"))
    s0 = np.zeros(g.r * g.ncell)
    sf, _ = fine_impes(g, p, s0, 4)
    sr, _ = lrbms_impes(m, s0, 4, DIRECT)
    assert np.abs(sf - sr).max() <= 1e-9 * np.abs(sf).max()


def _snapshot_model(name="small2d", k=4, seed=2, unit=True):
    p = make_problem(name)
    g = Grid(p)
    rng = np.random.default_rng(seed)
    states = [random_saturation(p, rng) for _ in range(k)]
    snaps = [fine_pressure(g, p, s=s) for s in states]
    phis = local_bases(g, p, snaps, method="gs", cap=100, unit=unit)
    return p, g, states, snaps, Model(p, phis)


def test_snapshot_reproduction():
    """A snapshot in the span of the basis is reproduced by the reduced
    solve at its own mobility (Galerkin projection of an element of W_N)."""
    p, g, states, snaps, m = _snapshot_model()
    for s, ph in zip(states, snaps):
        A, f = reduced_system(m, s, DIRECT)
        pH = m.B @ solve_reduced(A, f)
        assert np.abs(pH - ph).max() <= 1e-9 * np.abs(ph).max()


def test_reduced_matrix_symmetric_positive_definite():
    p, g, states, snaps, m = _snapshot_model(k=3)
    s = random_saturation(p, np.random.default_rng(9))
    A, _ = reduced_system(m, s, DIRECT)
    Ad = A.toarray()
    assert np.abs(Ad - Ad.T).max() <= 1e-13 * np.abs(Ad).max()
    assert np.linalg.eigvalsh(Ad).min() > 0


def test_local_bases_orthonormal_and_local():
    p, g, states, snaps, m = _snapshot_model(k=3)
    for phi in m.basis.phis:
        X = phi.reshape(phi.shape[0], -1)
        assert np.allclose(X @ X.T, np.eye(phi.shape[0]), atol=1e-12)
    B = m.B.tocsc()
    for E, cells in enumerate(subdomain_cells(g, p)):
        cols = range(m.basis.offsets[E], m.basis.offsets[E + 1])
        rows = np.unique(B[:, list(cols)].nonzero()[0]) % g.ncell
        assert set(rows) <= set(cells)


def _affine_model(name="small2d"):
    p = make_problem(name)
    g = Grid(p)
    params = training_params(p.M, p.n_train, np.random.default_rng(p.seed))
    off = build_offline(g, p, params)
    profiles = [off["profiles"][k] for k in off["keep"]]
    return p, g, off, Model(p, off["basis"].phis, profiles)


@pytest.fixture(scope="module")
def affine_model():
    return _affine_model()


def test_direct_fit_equals_affine(affine_model):
    """b_h is linear in gamma and the penalty is mobility-free, so the
    affine sum c + sum theta_q b_q equals Phi^T A(sum theta_q Lambda^q) Phi
    (eq. reducedSystem vs Def. coarseScalePressure)."""
    p, g, off, m = affine_model
    s = random_saturation(p, np.random.default_rng(5))
    A1, f1 = reduced_system(m, s, AFFINE)
    A2, f2 = reduced_system(m, s, DIRECT_FIT)
    assert abs(A1 - A2).max() <= 1e-12 * abs(A2).max()
    assert np.abs(f1 - f2).max() <= 1e-12 * max(np.abs(f2).max(), 1e-300)


def test_lsq_exact_in_profile_span(affine_model):
    """If Pi lambda(s) lies in the span of the profiles the fit reproduces it.
    The profiles are piecewise constant, so a saturation that is constant
    per cell with lambda(s_e) equal to a profile combination is built from
    the inverse of the Corey law on each cell.  theta is a convex combination,
    so the target stays inside the range of lambda, as each profile does."""
    p, g, off, m = affine_model
    theta = np.array([0.6, 0.4] + [0.0] * (len(m.profiles) - 2))
    target = sum(t * q for t, q in zip(theta, m.profiles))       # P1 field (means only)
    lam_cells = target[:g.ncell] / math.sqrt(g.vol)
    # invert lambda(s) = s^2/eta_w + (1-s)^2/eta_o on the branch s >= s*
    a = 1 / p.visc_w + 1 / p.visc_o
    b = -2 / p.visc_o
    c = 1 / p.visc_o - lam_cells
    sc = (-b + np.sqrt(b * b - 4 * a * c)) / (2 * a)
    s = np.zeros(g.r * g.ncell)
    s[:g.ncell] = sc * math.sqrt(g.vol)
    fit = sum(t * q for t, q in zip(lsq_theta(g, p, s, m.profiles), m.profiles))
    assert np.abs(fit - target).max() <= 1e-10 * np.abs(target).max()


def test_profile_endpoints_and_dedupe(affine_model):
    p, g, off, m = affine_model
    prof = off["profiles"]
    nc = g.ncell
    l0, l1 = 1 / p.visc_o, 1 / p.visc_w
    assert np.allclose(prof[0][:nc] / math.sqrt(g.vol), l0)
    assert np.allclose(prof[-1][:nc] / math.sqrt(g.vol), l1)
    # Lambda^1 and Lambda^M are both constant fields: one of them is dropped
    assert len(off["keep"]) <= len(prof) - 1
    # profiles are monotone in q: a cell swept at threshold q is swept at all larger q
    swept = np.stack([np.isclose(q[:nc] / math.sqrt(g.vol), l1) for q in prof[1:-1]])
    assert np.all(np.diff(swept.astype(int), axis=0) >= 0)


def test_coarse_conservation_with_unit_functions():
    """With 1_E in every local basis, testing the reduced equation with 1_E
    gives coarse mass conservation of the reconstructed flux when the flux
    uses the same mobility as the pressure (DIRECT)."""
    p, g, states, snaps, m = _snapshot_model(k=3, unit=True)
    s = random_saturation(p, np.random.default_rng(11))
    out = online_step(m, s, DIRECT)
    from oracle.pressure import cell_outflow
    net = cell_outflow(g, out["F"])
    for cells in subdomain_cells(g, p):
        assert abs(net[cells].sum() - (p.q1[cells] * g.vol).sum()) <= 1e-10 * np.abs(out["F"]).max()


def test_greedy_reproduces_selected_snapshots():
    """Alg. 2 greedy with the true error: every selected training snapshot
    lies in the final space, so its error vanishes; the max error history
    ends below the tolerance."""
    p = make_problem("tiny2d")
    g = Grid(p)
    p0 = fine_pressure(g, p, s=np.zeros(g.r * g.ncell))
    F0 = reconstruct_flux(g, p, p0, Mobility(g, p, s=np.zeros(g.r * g.ncell)))
    from oracle.tof import time_of_flight
    tau = time_of_flight(g, p, F0)
    prof = mobility_profiles(g, p, tau, p.M, p.n_steps * p.dt * 50)
    params = training_params(p.M, 10, np.random.default_rng(0))
    phis, chosen, hist = greedy(g, p, prof, params, n_max=10 ** 6, tol=1e-8)
    assert len(chosen) >= 2
    m = Model(p, phis)
    for k in chosen:
        gam = Mobility(g, p, field=training_mobility(prof, params[k]))
        from oracle.online import assemble_direct
        A, f = assemble_direct(m, gam)
        pH = m.B @ solve_reduced(A, f)
        ph = fine_pressure(g, p, field=training_mobility(prof, params[k]))
        assert np.abs(pH - ph).max() <= 1e-8 * np.abs(ph).max()


def test_pca_energy_criterion():
    rng = np.random.default_rng(0)
    base = [rng.standard_normal((3, 20)) for _ in range(3)]
    vecs = [sum(rng.standard_normal() * b for b in base) + 1e-7 * rng.standard_normal((3, 20))
            for _ in range(8)]
    modes = pca_modes(vecs, 1e-4)
    assert len(modes) == 3
    X = np.stack([v.ravel() for v in vecs], 1)
    Q = np.stack([m.ravel() for m in modes], 1)
    resid = X - Q @ (Q.T @ X)
    assert (resid ** 2).sum() <= 1e-8 * (X ** 2).sum()


def test_direct_fit_equals_affine_with_dirichlet_pressure(affine_model):
    """The same identity for the right-hand side when the Dirichlet pressure
    is not zero, so that the lambda-dependent terms d_q of f_N do not vanish
    (with p_D = 0 they are zero and their sign or scale is not seen)."""
    p, g, off, m = affine_model
    p2 = p.copy()
    p2.bc_val[p2.bc_type == 2] = 2.0e5
    m2 = Model(p2, off["basis"].phis, m.profiles)
    assert max(np.abs(d).max() for d in m2.terms["d"]) > 0.0
    s = random_saturation(p2, np.random.default_rng(6))
    A1, f1 = reduced_system(m2, s, AFFINE)
    A2, f2 = reduced_system(m2, s, DIRECT_FIT)
    assert abs(A1 - A2).max() <= 1e-12 * abs(A2).max()
    assert np.abs(f1 - f2).max() <= 1e-12 * np.abs(f2).max()


def test_projected_mobility_closed_form():
    """L2 projection of lambda(s) onto P1 for s = a + b xi on each cell of a
    strip (xi in [-1, 1] along x) with quadratic Corey laws: lambda = alpha +
    beta xi + gamma xi^2 with alpha = a^2/eta_w + (1-a)^2/eta_o,
    beta = 2ab/eta_w - 2b(1-a)/eta_o, gamma = b^2 (1/eta_w + 1/eta_o); the mean
    coefficient is sqrt|e| (alpha + gamma/3), the x coefficient
    sqrt|e| beta / sqrt(3), the y coefficient 0 (eq. leastSquaresFit's
    right-hand side; the 2-point Gauss rule is exact for these cubics)."""
    p = make_problem("tiny2d", n=(4, 1, 1), L=(1.0, 0.25, 1.0), nc=(1, 1, 1))
    p.relperm, p.corey_w, p.corey_o = 1, 2.0, 2.0
    g = Grid(p)
    a = np.array([0.2, 0.45, 0.7, 0.5])
    b = np.array([0.1, -0.15, 0.2, 0.0])
    nc, sv = g.ncell, math.sqrt(g.vol)
    s = np.zeros(g.r * nc)
    s[:nc] = a * sv
    s[nc:2 * nc] = b * sv / math.sqrt(3)          # s = a + b xi
    ew, eo = p.visc_w, p.visc_o
    alpha = a ** 2 / ew + (1 - a) ** 2 / eo
    beta = 2 * a * b / ew - 2 * b * (1 - a) / eo
    gamma = b ** 2 * (1 / ew + 1 / eo)
    got = projected_mobility(g, p, s)
    assert np.allclose(got[:nc], sv * (alpha + gamma / 3), rtol=1e-13)
    assert np.allclose(got[nc:2 * nc], sv * beta / math.sqrt(3), rtol=1e-12, atol=1e-18)
    assert np.abs(got[2 * nc:]).max() <= 1e-12 * np.abs(got).max()


def test_gram_schmidt_keeps_orthonormality_on_nearly_dependent_vectors():
    """The local bases must be orthonormal in L2(E): extending a basis one
    vector at a time with nearly dependent snapshots (monomials on close
    nodes, condition number ~1e11) keeps |Q^T Q - I| at rounding level (one
    classical Gram-Schmidt pass would not)."""
    from oracle.offline import gs_extend
    x = np.linspace(1.0, 1.1, 40)
    basis = []
    kept = 0
    for j in range(8):
        kept += gs_extend(basis, x ** j)
    Q = np.stack(basis, axis=1)
    assert kept == len(basis) >= 6
    assert np.abs(Q.T @ Q - np.eye(Q.shape[1])).max() <= 1e-13


def test_mobility_profile_thresholds_by_hand():
    """Alg. 2 step 1c: Lambda^1 = lambda(0), Lambda^M = lambda(1) and, for
    1 < q < M, lambda(0) where the cell-mean time of flight exceeds
    (q-1) T/(M-2), else lambda(1).  M = 5, T = 3: thresholds 1, 2, 3 for
    q = 2, 3, 4, against cell means 0.5, 1.5, 2.5, 3.5."""
    from oracle.fem import mobilities
    p = make_problem("tiny2d", n=(4, 1, 1), L=(1.0, 0.25, 1.0), nc=(1, 1, 1))
    g = Grid(p)
    tau = np.zeros(g.r * g.ncell)
    tau[:g.ncell] = np.array([0.5, 1.5, 2.5, 3.5]) * math.sqrt(g.vol)
    prof = mobility_profiles(g, p, tau, 5, 3.0)
    l0 = mobilities(np.array([0.0]), p)[2][0]
    l1 = mobilities(np.array([1.0]), p)[2][0]
    want = [[l0] * 4, [l1, l0, l0, l0], [l1, l1, l0, l0], [l1, l1, l1, l0], [l1] * 4]
    got = [q[:g.ncell] / math.sqrt(g.vol) for q in prof]
    assert len(got) == 5
    for w, q in zip(want, got):
        assert np.allclose(q, w, rtol=1e-14)
    assert all(np.abs(q[g.ncell:]).max() == 0.0 for q in prof)


def test_greedy_energy_norm_of_a_constant_by_hand():
    """The greedy's error measure is the energy norm of b_h(., .; lambda-bar):
    for a constant error e = c the gradient and every interior jump vanish,
    so only the Dirichlet faces' penalty is left,
    |e|^2 = c^2 sum over Dirichlet faces of sigma_f |f| / h_f with
    sigma_f = (c_f / max eta) kappa of the boundary cell (eq. penaltyParam,
    reading: h_f = face diameter)."""
    from oracle.offline import energy_error
    from oracle.pressure import assemble
    p = make_problem("small2d")
    g = Grid(p)
    rng = np.random.default_rng(3)
    prof = [np.concatenate([rng.uniform(0.5, 2.0, g.ncell) * math.sqrt(g.vol),
                            np.zeros((g.r - 1) * g.ncell)]) for _ in range(2)]
    A_bar = assemble(g, p, Mobility(g, p, field=training_mobility(prof, np.array([0.5, 0.5]))))
    c = 3.0
    e = np.zeros(g.r * g.ncell)
    e[:g.ncell] = c * math.sqrt(g.vol)
    want = 0.0
    cf = p.penalty_c / max(p.visc_w, p.visc_o)
    for a in range(g.dim):
        f = g.faces[a]
        dirichlet = p.bc_type[f["gid"]] == 2
        cell = np.where(f["lo"] >= 0, f["lo"], f["hi"])[dirichlet]
        hf = f["hf"] if np.isscalar(f["hf"]) else f["hf"][dirichlet]
        want += np.sum(cf * np.asarray(p.perm)[cell] * f["area"] / hf)
    assert want > 0.0
    got = energy_error(g, p, A_bar, e, np.zeros_like(e))
    assert abs(got - c * math.sqrt(want)) <= 1e-12 * c * math.sqrt(want)
