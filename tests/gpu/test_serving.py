"""Many simulations on one device, through the C ABI: the batched ensemble
step (one graph launch, or direct launches on per-simulation branches) and
the serving loop (admission by memory footprint, continuous dispatch onto
slot streams).  Each simulation's state after every step must equal, bit for
bit, what the plain per-simulation path gives (the same kernels on the same
data in the same order; the plain path itself is checked against the oracle
by the parity tests).  Graph replays alternate with the plain path's own
launches and synchronizations, and every replay is checked."""
import numpy as np
import pytest

from synth import make_problem, random_saturation, smooth_fields, training_params

from .helpers import log

pytestmark = pytest.mark.gpu

NAMES = ["tiny2d", "cfg1", "small2d", "small3d"]


@pytest.fixture(scope="module")
def L():
    from paper_1405_2810_amd import lrbms
    return lrbms


def _model(L, name, seed=0):
    p = make_problem(name)
    snaps = smooth_fields(p, p.ne_cap + 2, np.random.default_rng(100 + seed))
    return p, L.Model.from_snapshots(p, snaps, ne_cap=p.ne_cap, unit_functions=True)


def _offline_model(L, name):
    p = make_problem(name)
    params = training_params(p.M, p.n_train, np.random.default_rng(p.seed))
    T = p.t_end if p.t_end > 0 else p.n_steps * p.dt
    m, _ = L.Model.build_offline(p, params, ne_cap=p.ne_cap, horizon=T)
    return p, m


def _state(p, seed):
    import torch
    s = random_saturation(p, np.random.default_rng(seed))
    return torch.tensor(s, dtype=torch.float64, device="cuda")


class Plain:
    """The plain per-simulation path: the four calls on one stream."""

    def __init__(self, m, sat, mode):
        import torch
        self.m, self.mode = m, mode
        self.sat = sat.clone()
        self.pN = torch.zeros(m.info["N"], dtype=torch.float64, device="cuda")
        self.flux = torch.zeros(m.info["nface"], dtype=torch.float64, device="cuda")
        self.nxt = torch.zeros_like(sat)
        self.flags = torch.zeros(m.info["ncell"], dtype=torch.uint8, device="cuda")

    def step(self):
        self.m.assemble(self.sat, self.mode)
        self.m.solve(self.pN)
        self.m.reconstruct_flux(self.pN, self.sat, self.flux)
        self.m.transport_step(self.sat, self.flux, self.nxt, self.flags)
        self.sat.copy_(self.nxt)


def _check_batch(L, probs, models, mode, graph, steps=4, fused=False):
    import torch
    sats = [_state(p, 40 + i) for i, p in enumerate(probs)]
    flags = [torch.full((m.info["ncell"],), 7, dtype=torch.uint8, device="cuda") for m in models]
    ref = [Plain(m, s, mode) for m, s in zip(models, sats)]
    B = L.Batch(models, mode=mode, graph=graph, fused=fused)
    try:
        for k in range(steps):
            if k == 2:
                # new state tensors: the graph is captured again
                sats = [s.clone() for s in sats]
            B.step(sats, flags)
            for r in ref:
                r.step()
            torch.cuda.synchronize()
            for i, (s, r) in enumerate(zip(sats, ref)):
                assert torch.equal(s, r.sat), (i, k)
                assert torch.equal(flags[i], r.flags), (i, k)
                pN_addr, _ = B.buffers(i)
                assert pN_addr
            log(f"[batch] mode={mode} graph={graph} fused={fused} step {k}: "
                f"{len(models)} simulations equal")
        assert B.status() == 0
    finally:
        B.close()


@pytest.mark.parametrize("graph,fused", [(True, False), (False, False), (True, True),
                                         (False, True)])
def test_batch_direct_equals_plain(L, graph, fused):
    """Fused: one reduced solve for all members; the plain path runs each
    member's own solver on the same assembled systems, so p_N and every
    state must still agree bit for bit."""
    built = [_model(L, n, i) for i, n in enumerate(NAMES)]
    probs, models = [b[0] for b in built], [b[1] for b in built]
    try:
        _check_batch(L, probs, models, L.DIRECT, graph, fused=fused)
    finally:
        for m in models:
            m.close()


@pytest.mark.parametrize("fused", [False, True])
def test_batch_affine_equals_plain(L, fused):
    built = [_offline_model(L, n) for n in ["tiny2d", "small2d"]]
    probs, models = [b[0] for b in built], [b[1] for b in built]
    try:
        _check_batch(L, probs, models, L.AFFINE, True, steps=3, fused=fused)
    finally:
        for m in models:
            m.close()


def test_fused_batch_of_many_grids(L):
    """Ten members of five grids (2D and 3D, even and uneven partitions,
    basis sizes 6..40) in one fused solve, with 0, 1 or 2 refinement steps
    (a member leaves the fused refinement after its own steps)."""
    names = NAMES + ["cfg1", "small2d", "small3d", "tiny2d", "cfg1", "small3d"]
    built = [_model(L, n, 10 + i) for i, n in enumerate(names)]
    probs, models = [b[0] for b in built], [b[1] for b in built]
    for i, m in enumerate(models):
        m.set_refinement(i % 3)
    try:
        _check_batch(L, probs, models, L.DIRECT, True, steps=3, fused=True)
        # a model of a fused batch cannot join another one meanwhile
        B = L.Batch(models[:2], fused=True)
        with pytest.raises(L.LrbmsError) as ei:
            L.Batch(models[1:3], fused=True)
        assert ei.value.code == -1
        B.close()
    finally:
        for m in models:
            m.close()


def test_fused_batch_with_ensemble_basis_sizes(L):
    """Members built like the benchmark ensemble's: local bases of 61
    plane-wave fields plus 1_E truncated to seeded sizes of 5..60 per box (so
    the 64-column assembly tiles and the skipping of tiles past a box's own
    size are taken), each member autotuned (assembly variant, solver shapes,
    refinement), 2D and 3D, in a fused graph batch and a fused batch of
    direct launches: every member equal to its plain path."""
    from synth import CONFIGS, ensemble_caps, wave_fields
    probs, models = [], []
    try:
        for i, name in enumerate(["small2d", "small3d", "small2d", "small3d"]):
            p = make_problem(name, seed=CONFIGS[name]["seed"] + i)
            full = L.Model.from_snapshots(p, wave_fields(p, 61, np.random.default_rng(70 + i)),
                                          ne_cap=60, unit_functions=True)
            caps = ensemble_caps(p, np.random.default_rng(80 + i))
            m = full.truncated(caps)
            full.close()
            m.autotune(_state(p, 90 + i), reps=1)
            probs.append(p)
            models.append(m)
        widest = max(int(m.export_basis()[0].max()) for m in models)
        assert widest > 48, widest   # the 64-column assembly tiles are used
        _check_batch(L, probs, models, L.DIRECT, True, steps=3, fused=True)
        _check_batch(L, probs, models, L.DIRECT, False, steps=3, fused=True)
    finally:
        for m in models:
            m.close()


def test_batch_arguments(L):
    p, m = _model(L, "tiny2d")
    try:
        with pytest.raises(L.LrbmsError) as ei:
            L.Batch([m, m])
        assert ei.value.code == -1
        with pytest.raises(L.LrbmsError) as ei:
            L.Batch([m], mode=L.AFFINE)     # no profiles
        assert ei.value.code == -1
        B = L.Batch([m])
        m.profile_enable(True)
        with pytest.raises(L.LrbmsError) as ei:
            B.step([_state(p, 1)])
        assert ei.value.code == -2
        m.profile_enable(False)
        # a member of a batch is not destroyed before the batch
        L.lib().lrbms_model_destroy(m._h)
        assert b"destroy that first" in L.lib().lrbms_last_error()
        assert L.lib().lrbms_model_status(m._h) == 0   # still alive
        B.close()
    finally:
        m.close()


def _footprint(m):
    i = m.info
    return i["device_bytes"] + 8 * (max(i["N"], 1) + max(i["nface"], 1) + i["r"] * i["ncell"])


@pytest.mark.parametrize("fused", [False, True])
def test_server_mix_equals_alone(L, fused):
    """Requests of four simulations of different grids (0, 1, 2 and 1
    refinement steps), interleaved in a seeded order over three slots (fused:
    waves of up to three requests whose reduced solves run as one
    combined-plan solve): every simulation ends where its plain path, run
    alone, ends."""
    import torch
    built = [_model(L, n, i) for i, n in enumerate(NAMES)]
    probs, models = [b[0] for b in built], [b[1] for b in built]
    for m, k in zip(models, [0, 1, 2, 1]):
        m.set_refinement(k)
    steps = 5
    sats = [_state(p, 60 + i) for i, p in enumerate(probs)]
    alone = [Plain(m, s, L.DIRECT) for m, s in zip(models, sats)]
    for r in alone:
        for _ in range(steps):
            r.step()
    torch.cuda.synchronize()
    order = np.repeat(np.arange(len(models)), steps)
    np.random.default_rng(5).shuffle(order)
    S = L.Server(hbm_budget=sum(_footprint(m) for m in models), max_slots=3, fused=fused)
    try:
        ids = [S.attach(m, s) for m, s in zip(models, sats)]
        info = S.info()
        assert info["n_admitted"] == len(models) and info["n_waiting"] == 0
        done = []
        for k, sim in enumerate(order):
            S.submit(ids[sim], 1000 + k)
            done += S.poll()
        S.drain()
        done += S.poll()
        assert sorted(d[0] for d in done) == [1000 + k for k in range(len(order))]
        assert all(d[2] == 0 and d[1] > 0.0 for d in done)
        lat = np.array([d[1] for d in done])
        log(f"[serve] {len(done)} requests, latency p50 {np.percentile(lat, 50):.3f} ms "
            f"p99 {np.percentile(lat, 99):.3f} ms")
        for i, (s, r) in enumerate(zip(sats, alone)):
            assert torch.equal(s, r.sat), i
        for m in models:
            assert m.status() == 0
    finally:
        S.close()
        for m in models:
            m.close()


@pytest.mark.parametrize("fused", [False, True])
def test_server_admission_by_footprint(L, fused):
    """A budget that holds two of three simulations: the third waits, its
    requests wait with it, and it is admitted (and served, with the same
    result as alone) once another simulation is detached."""
    import torch
    built = [_model(L, n, i) for i, n in enumerate(["small2d", "cfg1", "tiny2d"])]
    probs, models = [b[0] for b in built], [b[1] for b in built]
    fp = [_footprint(m) for m in models]
    budget = fp[0] + fp[1] + fp[2] // 2
    assert fp[0] + fp[2] <= budget
    sats = [_state(p, 80 + i) for i, p in enumerate(probs)]
    alone = [Plain(m, s, L.DIRECT) for m, s in zip(models, sats)]
    for r in alone:
        for _ in range(2):
            r.step()
    torch.cuda.synchronize()
    S = L.Server(hbm_budget=budget, max_slots=4, fused=fused)
    try:
        ids = [S.attach(m, s) for m, s in zip(models, sats)]
        info = S.info()
        assert info["n_admitted"] == 2 and info["n_waiting"] == 1
        assert info["resident_bytes"] == fp[0] + fp[1]
        for k in range(2):
            for i in ids:
                S.submit(i, 10 * i + k)
        with pytest.raises(L.LrbmsError) as ei:
            S.drain()
        assert ei.value.code == -7
        assert S.info()["n_pending"] == 2
        for i in (0, 1):
            assert torch.equal(sats[i], alone[i].sat)
        S.detach(ids[1])
        info = S.info()
        assert info["n_admitted"] == 2 and info["n_waiting"] == 0
        S.drain()
        assert torch.equal(sats[2], alone[2].sat)
        done = S.poll()
        assert sorted(d[0] for d in done) == sorted(10 * i + k for i in ids for k in range(2))
        # a footprint above the whole budget (the model detached above)
        with pytest.raises(L.LrbmsError) as ei:
            L.Server(hbm_budget=fp[1] - 1).attach(models[1], sats[1])
        assert ei.value.code == -7
        # a model attached to this server belongs to it: no second owner
        with pytest.raises(L.LrbmsError) as ei:
            L.Batch([models[0]])
        assert ei.value.code == -1
    finally:
        S.close()
        for m in models:
            m.close()
