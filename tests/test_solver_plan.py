"""The reduced solver's symbolic analysis (exported by the library, host
only) drives a NumPy emulation of the numeric kernels step by step; the
emulation must solve block-pattern SPD systems exactly as a dense solver does.
This checks the nested-dissection tree, the index maps and the work lists
without a GPU."""
import numpy as np
import pytest

from synth import make_problem

NB = 64
SB = 128   # output tile of the deferred Schur complement


def _ifaces(p):
    nc = [len(c) - 1 for c in p.cuts] if p.dim == 3 else [len(p.cuts[0]) - 1, len(p.cuts[1]) - 1, 1]
    out = []
    for a in range(p.dim):
        for ez in range(nc[2]):
            for ey in range(nc[1]):
                for ex in range(nc[0]):
                    e = [ex, ey, ez]
                    if e[a] + 1 >= nc[a]:
                        continue
                    lo = ex + nc[0] * (ey + nc[1] * ez)
                    e[a] += 1
                    out.append((a, lo, e[0] + nc[0] * (e[1] + nc[1] * e[2])))
    return out


def _random_system(p, sizes, rng):
    offs = np.concatenate([[0], np.cumsum(sizes)])
    N = offs[-1]
    A = np.zeros((N, N))
    blocks = []
    for E, ne in enumerate(sizes):
        M = rng.standard_normal((ne, ne))
        D = M @ M.T + 8 * ne * np.eye(ne)
        A[offs[E]:offs[E + 1], offs[E]:offs[E + 1]] = D
        blocks.append(D.ravel())
    for a, lo, hi in _ifaces(p):
        B = rng.standard_normal((sizes[lo], sizes[hi]))
        A[offs[lo]:offs[lo + 1], offs[hi]:offs[hi + 1]] = B
        A[offs[hi]:offs[hi + 1], offs[lo]:offs[lo + 1]] = B.T
        blocks.append(B.ravel())
    return A, np.concatenate(blocks), rng.standard_normal(N)


def _factor_tile(Fp, m, panel, Inv, f):
    c0 = panel * NB
    nb = min(NB, m - c0)
    D = np.tril(Fp[c0:c0 + nb, c0:c0 + nb])
    Lt = np.linalg.cholesky(D + np.tril(D, -1).T)
    pad = np.zeros((NB, NB))
    pad[:nb, :nb] = np.linalg.inv(Lt)
    o = f["inv_off"] + panel * NB * NB
    Inv[o:o + NB * NB] = pad.ravel()


def emulate(plan, blocks, fN, refine=False):
    """The numeric phase as the device kernels execute it: fronts column-major
    with a right-hand-side row at the bottom, fused panel steps with the L rows
    in a separate panel-major store, look-ahead tile factorization, backward
    sweep reading L row-wise; the trailing updates of a panel step touch the
    S columns only, and each front's U x U block and the right-hand-side row's
    U part are updated once after its last panel (deferred Schur complement);
    a split front's product L_US^T x_U is formed
    first in partial vectors, one per 64 U rows read through the plan's U-row
    map, and the backward subtracts their sum in chunk order."""
    F = np.zeros(plan["front_doubles"])
    Lb = np.zeros(plan["lpan_doubles"])
    V = np.zeros(plan["vec_doubles"])
    Inv = np.zeros(plan["inv_doubles"])
    fr, nodes = plan["fronts"], plan["nodes"]

    def view(buf, f):
        ld = f["m"] + f["u"]
        return buf[f["off"]:f["off"] + (ld + 1) * ld].reshape(ld + 1, ld, order="F")

    def lpanel(f, b):
        """rows cs_b .. ld of panel b, NB doubles per row (row-major)"""
        ld1 = f["m"] + f["u"] + 1
        base = f["loff"] + NB * (b * ld1 - 32 * b * (b + 1))
        cs = min(NB * (b + 1), f["m"])
        return buf_rows(base, ld1 - cs), cs

    def buf_rows(base, nrows):
        return Lb[base:base + nrows * NB].reshape(nrows, NB)

    for lev in plan["levels"]:
        for it in lev["asm"]:
            f = fr[it["front"]]
            Fp = view(F, f)
            i = np.arange(it["nr"])[:, None]
            j = np.arange(it["nc"])[None, :]
            v = np.zeros((it["nr"], it["nc"]))
            for S in it["src"]:
                v = v + {0: blocks, 1: F, 2: fN}[S["kind"]][S["so"] + i * S["rs"] + j * S["cs"]]
            if it["diag"]:
                v = np.tril(v)
            Fp[it["dr"]:it["dr"] + it["nr"], it["dc"]:it["dc"] + it["nc"]] = v
        for fi in lev["fronts"]:
            _factor_tile(view(F, fr[fi]), fr[fi]["m"], 0, Inv, fr[fi])
        for items in lev["steps"]:
            for it in items:
                if it["tj"] <= -2:
                    # a prefetch item: part of the left-looking sum below,
                    # formed one step ahead (same products, another grouping)
                    continue
                f = fr[it["front"]]
                Fp = view(F, f)
                ld = f["m"] + f["u"]
                p = it["panel"]
                c0 = p * NB
                nb = min(NB, f["m"] - c0)
                cs = c0 + nb
                Li = Inv[f["inv_off"] + p * NB * NB:f["inv_off"] + (p + 1) * NB * NB].reshape(NB, NB)[:nb, :nb]
                R0 = cs + it["ti"] * NB
                nr = min(NB, ld + 1 - R0)
                if it["tj"] < 0 and R0 >= f["m"] and p > 0:
                    # a tile of U rows: the earlier panels' products, left-looking,
                    # for its rows from 64 npanels on (the rows before were in the
                    # tile straddling m, updated right-looking)
                    lo = max(R0, NB * f["npanels"])
                    for cp in range(p):
                        rows_c, cs_c = lpanel(f, cp)
                        Fp[lo:R0 + nr, c0:cs] -= (rows_c[lo - cs_c:R0 - cs_c + nr, :]
                                                  @ rows_c[c0 - cs_c:c0 - cs_c + (cs - c0), :].T)
                A = Fp[R0:R0 + nr, c0:cs] @ Li.T
                if it["tj"] <= 0:
                    rows, cs_b = lpanel(f, p)
                    rows[R0 - cs_b:R0 - cs_b + nr, :nb] = A
                if it["tj"] < 0:
                    continue
                C0 = cs + it["tj"] * NB
                ncl = min(NB, f["m"] - C0)      # S columns only
                Bt = A if it["tj"] == it["ti"] else Fp[C0:C0 + ncl, c0:cs] @ Li.T
                Fp[R0:R0 + nr, C0:C0 + ncl] -= A @ Bt[:ncl].T
                if it["ti"] == 0 and it["tj"] == 0 and p + 1 < f["npanels"]:
                    _factor_tile(Fp, f["m"], p + 1, Inv, f)
        # deferred Schur complement: (U + rhs row) x U minus L_US L_US^T over
        # all m columns, tile by tile, the panels in order
        for fi, ti, tj, wide in lev["schur"]:
            f = fr[fi]
            Fp = view(F, f)
            ld, m = f["m"] + f["u"], f["m"]
            T = SB if wide else NB
            R0, C0 = m + ti * T, m + tj * T
            nr, ncl = min(T, ld + 1 - R0), min(T, ld - C0)
            acc = np.zeros((nr, ncl))
            for b in range(f["npanels"]):
                rows, cs_b = lpanel(f, b)
                nbb = min(NB, m - b * NB)
                acc += rows[R0 - cs_b:R0 - cs_b + nr, :nbb] @ rows[C0 - cs_b:C0 - cs_b + ncl, :nbb].T
            if wide and ti == tj:
                acc[:NB, NB:] = 0.0   # the block above the diagonal is not formed
            Fp[R0:R0 + nr, C0:C0 + ncl] -= acc

    def rhs_rows(f):
        ld, m = f["m"] + f["u"], f["m"]
        y = np.zeros(m)
        for b in range(f["npanels"]):
            rows, cs_b = lpanel(f, b)
            nbb = min(NB, m - b * NB)
            y[b * NB:b * NB + nbb] = rows[ld - cs_b, :nbb]
        return y

    pN = _backward(plan, lpanel, Inv, rhs_rows, np.zeros_like(fN))
    if refine:
        return pN, (lpanel, Inv)
    return pN


def _forward(plan, lpanel, Inv, r):
    """Forward substitution L y = r of a new right-hand side as
    k_front_forward and k_front_fw_gemv run it: per front (leaves first)
    w = (r_S, 0) plus the children's update vectors at their parent places,
    panel by panel y_b = Linv_b w_b and w_{>b} -= L_{>b,b} y_b (a split
    front's U rows afterwards, chunk by chunk); the front's vector store
    receives (y_S, w_U)."""
    fr, nodes = plan["fronts"], plan["nodes"]
    V = np.full(plan["vec_doubles"], np.nan)
    for lev in plan["levels"]:
        for fi in lev["fronts"]:
            f = fr[fi]
            ld, m = f["m"] + f["u"], f["m"]
            w = np.zeros(ld)
            for n in nodes[f["node_off"]:f["node_off"] + f["n_s_nodes"]]:
                w[n["pos"]:n["pos"] + n["size"]] = r[n["pn_off"]:n["pn_off"] + n["size"]]
            for c in plan["children"][f["child_off"]:f["child_off"] + f["nchild"]]:
                fc = fr[c]
                for n in nodes[fc["node_off"] + fc["n_s_nodes"]:fc["node_off"] + fc["n_nodes"]]:
                    w[n["ppos"]:n["ppos"] + n["size"]] += V[fc["voff"] + n["pos"]:fc["voff"] + n["pos"] + n["size"]]
            rows_end = m if f["nzc"] > 0 else ld
            for b in range(f["npanels"]):
                c0, nb = b * NB, min(NB, m - b * NB)
                Li = Inv[f["inv_off"] + b * NB * NB:f["inv_off"] + (b + 1) * NB * NB].reshape(NB, NB)[:nb, :nb]
                w[c0:c0 + nb] = np.tril(Li) @ w[c0:c0 + nb]
                rows, cs_b = lpanel(f, b)
                w[c0 + nb:rows_end] -= rows[0:rows_end - cs_b, :nb] @ w[c0:c0 + nb]
            V[f["voff"]:f["voff"] + ld] = w
        for fi, c in lev["bw"]:
            f = fr[fi]
            m, r0 = f["m"], NB * c
            nr = min(NB, f["u"] - r0)
            y = V[f["voff"]:f["voff"] + m]
            acc = np.zeros(nr)
            for b in range(f["npanels"]):
                rows, cs_b = lpanel(f, b)
                nbb = min(NB, m - b * NB)
                acc += rows[m - cs_b + r0:m - cs_b + r0 + nr, :nbb] @ y[b * NB:b * NB + nbb]
            V[f["voff"] + m + r0:f["voff"] + m + r0 + nr] -= acc
    return V


def _backward(plan, lpanel, Inv, y_of, pN):
    """Backward sweep L^T x = y from the root down; y_S of a front from y_of."""
    fr, nodes = plan["fronts"], plan["nodes"]
    part = np.full(max(plan["bw_part_doubles"], 1), np.nan)
    urow = np.asarray(plan["urow_pn"], dtype=np.int64)
    for lev in reversed(plan["levels"]):
        for fi, c in lev["bw"]:
            f = fr[fi]
            m = f["m"]
            r0 = NB * c
            nr = min(NB, f["u"] - r0)
            xr = pN[urow[f["urow_off"] + r0:f["urow_off"] + r0 + nr]]
            assert f["zoff"] + (c + 1) * m <= plan["bw_part_doubles"]
            out = part[f["zoff"] + c * m:f["zoff"] + (c + 1) * m]
            for b in range(f["npanels"]):
                rows, cs_b = lpanel(f, b)
                nbb = min(NB, m - b * NB)
                out[b * NB:b * NB + nbb] = rows[m - cs_b + r0:m - cs_b + r0 + nr, :nbb].T @ xr
        for fi in lev["fronts"]:
            f = fr[fi]
            ld, m = f["m"] + f["u"], f["m"]
            w = np.zeros(ld)
            w[:m] = y_of(f)
            for n in nodes[f["node_off"] + f["n_s_nodes"]:f["node_off"] + f["n_nodes"]]:
                w[n["pos"]:n["pos"] + n["size"]] = pN[n["pn_off"]:n["pn_off"] + n["size"]]
            if f["nzc"] > 0:
                acc = np.zeros(m)
                for c in range(f["nzc"]):
                    acc += part[f["zoff"] + c * m:f["zoff"] + (c + 1) * m]
                w[:m] -= acc
            for b in range(f["npanels"] if f["nzc"] == 0 else 0):
                rows, cs_b = lpanel(f, b)
                nbb = min(NB, m - b * NB)
                w[b * NB:b * NB + nbb] -= rows[m - cs_b:ld - cs_b, :nbb].T @ w[m:]
            for b in reversed(range(f["npanels"])):
                c0, nb = b * NB, min(NB, m - b * NB)
                Li = Inv[f["inv_off"] + b * NB * NB:f["inv_off"] + (b + 1) * NB * NB].reshape(NB, NB)[:nb, :nb]
                xb = Li.T @ w[c0:c0 + nb]
                w[c0:c0 + nb] = xb
                for b2 in range(b):
                    rows, cs2 = lpanel(f, b2)
                    w[b2 * NB:(b2 + 1) * NB] -= rows[c0 - cs2:c0 - cs2 + nb, :].T @ xb
            for n in nodes[f["node_off"]:f["node_off"] + f["n_s_nodes"]]:
                pN[n["pn_off"]:n["pn_off"] + n["size"]] = w[n["pos"]:n["pos"] + n["size"]]
    return pN


@pytest.mark.parametrize("name,ne,leaf", [("tiny2d", 6, 2), ("small2d", 8, 2), ("small3d", 8, 2),
                                          ("cfg1", 10, 1), ("cfg1", 30, 2), ("tiny2d", 40, 1)])
def test_plan_emulation_solves(name, ne, leaf):
    from paper_1405_2810_amd.lrbms import solver_plan
    p = make_problem(name)
    nsub = int(np.prod([len(c) - 1 for c in p.cuts]))
    rng = np.random.default_rng(ne)
    sizes = rng.integers(max(1, ne // 2), ne + 1, nsub)
    plan = solver_plan(p, sizes, leaf)
    A, blocks, f = _random_system(p, sizes, rng)
    x = emulate(plan, blocks, f)
    ref = np.linalg.solve(A, f)
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


def test_plan_emulation_wide_schur_tiles():
    """Fronts with at least 512 U columns take 128 x 128 Schur tiles (the
    256 x 256 grid's 16 x 16 boxes with 36 functions each): the plan still
    solves the system, against a sparse direct solve of the same blocks."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    from paper_1405_2810_amd.lrbms import solver_plan
    p = make_problem("cfg2")
    nsub = int(np.prod([len(c) - 1 for c in p.cuts]))
    sizes = np.full(nsub, 36, dtype=np.int64)
    plan = solver_plan(p, sizes, 4)
    assert any(it[3] for lev in plan["levels"] for it in lev["schur"])
    assert any(not it[3] for lev in plan["levels"] for it in lev["schur"])
    rng = np.random.default_rng(5)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    rows, cols, vals, blocks = [], [], [], []

    def put(r0, c0, B):
        i, j = np.meshgrid(np.arange(B.shape[0]), np.arange(B.shape[1]), indexing="ij")
        rows.append((r0 + i).ravel())
        cols.append((c0 + j).ravel())
        vals.append(B.ravel())

    for E, ne in enumerate(sizes):
        M = rng.standard_normal((ne, ne))
        D = M @ M.T + 8 * ne * np.eye(ne)
        put(offs[E], offs[E], D)
        blocks.append(D.ravel())
    for a, lo, hi in _ifaces(p):
        B = rng.standard_normal((sizes[lo], sizes[hi]))
        put(offs[lo], offs[hi], B)
        put(offs[hi], offs[lo], B.T)
        blocks.append(B.ravel())
    N = int(offs[-1])
    A = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    f = rng.standard_normal(N)
    x = emulate(plan, np.concatenate(blocks), f)
    ref = spla.spsolve(A, f)
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


def test_combined_plan_solves_every_member():
    """The plan of a fused batch (members of different grids, basis sizes and
    leaf sizes, one after another in shared storage) solves every member's
    system exactly as a dense solver does, and leaves no member's unknowns
    untouched."""
    from paper_1405_2810_amd.lrbms import solver_plan, solver_plan_batch
    specs = [("tiny2d", 6, 2), ("small3d", 8, 4), ("small2d", 8, 2), ("cfg1", 12, 1),
             ("small3d", 5, 2)]
    rng = np.random.default_rng(17)
    probs, sizes, leaves, systems = [], [], [], []
    for name, ne, leaf in specs:
        p = make_problem(name)
        nsub = int(np.prod([len(c) - 1 for c in p.cuts]))
        sz = rng.integers(max(1, ne // 2), ne + 1, nsub)
        probs.append(p)
        sizes.append(sz)
        leaves.append(leaf)
        systems.append(_random_system(p, sz, rng))
    plan = solver_plan_batch(probs, sizes, leaves)
    single = [solver_plan(p, sz, lf) for p, sz, lf in zip(probs, sizes, leaves)]
    assert len(plan["fronts"]) == sum(len(q["fronts"]) for q in single)
    assert len(plan["levels"]) == max(len(q["levels"]) for q in single)
    blocks = np.concatenate([b for _, b, _ in systems])
    fN = np.concatenate([f for _, _, f in systems])
    x = emulate(plan, blocks, fN)
    off = 0
    for (A, _, f) in systems:
        ref = np.linalg.solve(A, f)
        got = x[off:off + len(f)]
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
        off += len(f)
    assert off == len(x)


def test_combined_plan_export_arguments():
    from paper_1405_2810_amd.lrbms import LrbmsError, solver_plan_batch
    p = make_problem("tiny2d")
    with pytest.raises(LrbmsError):
        solver_plan_batch([p], [np.full(4, 3)], [0])


@pytest.mark.parametrize("combined", [False, True])
def test_split_backward_maps(monkeypatch, combined):
    """Every front with U rows split (LRBMS_BW_SPLIT_MIN=1): each split
    front has one chunk per 64 U rows and one work item per chunk, its U-row
    map sends every U row to the p_N place its node reference gives, the
    partial vectors of a level fit their storage, and the emulated solve with
    the split products is exact (single plans and the combined plan of a
    fused batch, whose maps are shifted into shared storage)."""
    from paper_1405_2810_amd.lrbms import solver_plan, solver_plan_batch
    monkeypatch.setenv("LRBMS_BW_SPLIT_MIN", "1")
    specs = [("tiny2d", 6, 2), ("small3d", 8, 4), ("cfg1", 12, 1), ("small2d", 70, 2)]
    rng = np.random.default_rng(23)
    probs, sizes, leaves, systems = [], [], [], []
    for name, ne, leaf in specs:
        p = make_problem(name)
        nsub = int(np.prod([len(c) - 1 for c in p.cuts]))
        sz = rng.integers(max(1, ne // 2), ne + 1, nsub)
        probs.append(p)
        sizes.append(sz)
        leaves.append(leaf)
        systems.append(_random_system(p, sz, rng))
    plans = ([solver_plan_batch(probs, sizes, leaves)] if combined else
             [solver_plan(p, sz, lf) for p, sz, lf in zip(probs, sizes, leaves)])
    groups = [systems] if combined else [[s] for s in systems]
    for plan, group in zip(plans, groups):
        n_split = 0
        for fi, f in enumerate(plan["fronts"]):
            assert f["nzc"] == ((f["u"] + 63) // 64 if f["u"] > 0 else 0)
            n_split += f["nzc"] > 0
            u_nodes = plan["nodes"][f["node_off"] + f["n_s_nodes"]:f["node_off"] + f["n_nodes"]]
            for n in u_nodes:
                for i in range(n["size"]):
                    assert plan["urow_pn"][f["urow_off"] + n["pos"] + i - f["m"]] == n["pn_off"] + i
        assert n_split > 0
        for lev in plan["levels"]:
            want = sorted((fi, c) for fi in lev["fronts"] for c in range(plan["fronts"][fi]["nzc"]))
            assert sorted(lev["bw"]) == want
        blocks = np.concatenate([b for _, b, _ in group])
        fN = np.concatenate([f for _, _, f in group])
        x = emulate(plan, blocks, fN)
        off = 0
        for (A, _, f) in group:
            ref = np.linalg.solve(A, f)
            got = x[off:off + len(f)]
            assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
            off += len(f)
        assert off == len(x)


@pytest.mark.parametrize("split", [False, True])
def test_refinement_sweeps_solve_new_rhs(monkeypatch, split):
    """The refinement's substitutions with the stored factor (forward sweep
    with the children's update vectors, split U-row products, backward sweep
    from the front vectors) solve a new right-hand side exactly as a dense
    solver does, for single plans and the combined plan of a fused batch."""
    from paper_1405_2810_amd.lrbms import solver_plan, solver_plan_batch
    if split:
        monkeypatch.setenv("LRBMS_BW_SPLIT_MIN", "1")
    specs = [("tiny2d", 6, 2), ("small3d", 8, 4), ("cfg1", 12, 1), ("small2d", 70, 2)]
    rng = np.random.default_rng(29)
    probs, sizes, leaves, systems = [], [], [], []
    for name, ne, leaf in specs:
        p = make_problem(name)
        nsub = int(np.prod([len(c) - 1 for c in p.cuts]))
        sz = rng.integers(max(1, ne // 2), ne + 1, nsub)
        probs.append(p)
        sizes.append(sz)
        leaves.append(leaf)
        systems.append(_random_system(p, sz, rng))
    plans = [solver_plan(p, sz, lf) for p, sz, lf in zip(probs, sizes, leaves)]
    plans.append(solver_plan_batch(probs, sizes, leaves))
    groups = [[s] for s in systems] + [systems]
    for plan, group in zip(plans, groups):
        blocks = np.concatenate([b for _, b, _ in group])
        fN = np.concatenate([f for _, _, f in group])
        _, (lpanel, Inv) = emulate(plan, blocks, fN, refine=True)
        r = rng.standard_normal(len(fN))
        V = _forward(plan, lpanel, Inv, r)
        d = _backward(plan, lpanel, Inv, lambda f: V[f["voff"]:f["voff"] + f["m"]],
                      np.full(len(fN), np.nan))
        off = 0
        for (A, _, _) in group:
            n = A.shape[0]
            ref = np.linalg.solve(A, r[off:off + n])
            assert np.linalg.norm(d[off:off + n] - ref) <= 1e-10 * np.linalg.norm(ref)
            off += n


@pytest.mark.parametrize("name,ne,leaf", [("small3d", 40, 1), ("cfg1", 10, 16)])
def test_prefetch_items_cover_the_left_looking_sums(name, ne, leaf):
    """Step p-1 of every front carries, for each U-row tile of step p >= 2
    (rows from m on), one prefetch item per chunk of 4 of the panels
    0 .. p-2, and nothing else of that kind: the step-p tile then adds only
    panel p-1's product itself."""
    from paper_1405_2810_amd.lrbms import solver_plan
    p = make_problem(name)
    sizes = np.full(int(np.prod(p.nc[:p.dim])), ne, dtype=np.int32)
    plan = solver_plan(p, sizes, leaf)
    fr = plan["fronts"]
    found = {}
    for lev in plan["levels"]:
        for items in lev["steps"]:
            for it in items:
                if it["tj"] <= -2:
                    key = (it["front"], it["panel"] + 1, it["ti"], -2 - it["tj"])
                    assert key not in found
                    found[key] = True
    want = {}
    n_multi = 0
    for fi, f in enumerate(fr):
        ld = f["m"] + f["u"]
        n_multi += f["npanels"] >= 3
        for q in range(2, f["npanels"]):
            cs = q * NB + min(NB, f["m"] - q * NB)
            nrt = (ld + 1 - cs + NB - 1) // NB
            for ti in range(nrt):
                if cs + NB * ti < f["m"]:
                    continue
                for sc in range((q - 1 + 3) // 4):
                    want[(fi, q, ti, sc)] = True
    assert n_multi > 0 or name == "cfg1"
    assert set(found) == set(want)
