"""The reduced solver's symbolic analysis (exported by the library, host
only) drives a NumPy emulation of the numeric kernels step by step; the
emulation must solve block-pattern SPD systems exactly as a dense solver does.
This checks the nested-dissection tree, the index maps and the work lists
without a GPU."""
import numpy as np
import pytest

from synth import make_problem

NB = 64


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


def emulate(plan, blocks, fN):
    """The numeric phase as the device kernels execute it (column-major fronts,
    lower triangle, tile inverses)."""
    F = np.zeros(plan["front_doubles"])
    V = np.zeros(plan["vec_doubles"])
    Inv = np.zeros(plan["inv_doubles"])
    fr, nodes, tasks, ch = plan["fronts"], plan["nodes"], plan["tasks"], plan["children"]
    col = lambda f: F[f["off"]:f["off"] + (f["m"] + f["u"]) ** 2].reshape(
        f["m"] + f["u"], f["m"] + f["u"], order="F")
    for lev in plan["levels"]:
        for it in lev["asm"]:
            f = fr[it["front"]]
            Fp = col(f)
            Fp[:, it["col0"]:it["col0"] + it["ncol"]] = 0.0
            for t in tasks[it["task_off"]:it["task_off"] + it["ntask"]]:
                src = F if t["from_front"] else blocks
                i = np.arange(t["nr"])[:, None]
                j = np.arange(t["nc"])[None, :]
                Fp[t["dr"]:t["dr"] + t["nr"], t["dc"]:t["dc"] + t["nc"]] += \
                    src[t["so"] + i * t["rs"] + j * t["cs"]]
        for pitems, uitems in lev["panels"]:
            snap = {}
            for it in pitems:
                f = fr[it["front"]]
                Fp = col(f)
                c0 = it["panel"] * NB
                nb = min(NB, f["m"] - c0)
                D = np.tril(Fp[c0:c0 + nb, c0:c0 + nb]).copy()
                snap.setdefault(it["front"], D)
            for it in pitems:
                f = fr[it["front"]]
                Fp = col(f)
                c0 = it["panel"] * NB
                nb = min(NB, f["m"] - c0)
                Lt = np.linalg.cholesky(snap[it["front"]] + np.tril(snap[it["front"]], -1).T)
                Li = np.linalg.inv(Lt)
                if it["row0"] == c0:
                    pad = np.zeros((NB, NB))
                    pad[:nb, :nb] = Li
                    o = f["inv_off"] + it["panel"] * NB * NB
                    Inv[o:o + NB * NB] = pad.ravel()
                else:
                    r0, nr = it["row0"], it["nrow"]
                    Fp[r0:r0 + nr, c0:c0 + nb] = Fp[r0:r0 + nr, c0:c0 + nb] @ Li.T
            for it in uitems:
                f = fr[it["front"]]
                Fp = col(f)
                ld = f["m"] + f["u"]
                c0 = it["panel"] * NB
                nb = min(NB, f["m"] - c0)
                cs = c0 + nb
                R0, C0 = cs + it["ti"] * NB, cs + it["tj"] * NB
                nr, ncl = min(NB, ld - R0), min(NB, ld - C0)
                Fp[R0:R0 + nr, C0:C0 + ncl] -= Fp[R0:R0 + nr, c0:c0 + nb] @ Fp[C0:C0 + ncl, c0:c0 + nb].T
    pN = np.zeros_like(fN)
    for lev in plan["levels"]:
        for fi in lev["fronts"]:
            f = fr[fi]
            ld = f["m"] + f["u"]
            Fp = col(f)
            w = np.zeros(ld)
            for n in nodes[f["node_off"]:f["node_off"] + f["n_s_nodes"]]:
                w[n["pos"]:n["pos"] + n["size"]] = fN[n["pn_off"]:n["pn_off"] + n["size"]]
            for c in ch[f["child_off"]:f["child_off"] + f["nchild"]]:
                fc = fr[c]
                wc = V[fc["voff"]:fc["voff"] + fc["m"] + fc["u"]]
                for n in nodes[fc["node_off"] + fc["n_s_nodes"]:fc["node_off"] + fc["n_nodes"]]:
                    w[n["ppos"]:n["ppos"] + n["size"]] += wc[n["pos"]:n["pos"] + n["size"]]
            for b in range((f["m"] + NB - 1) // NB):
                c0, nb = b * NB, min(NB, f["m"] - b * NB)
                Li = Inv[f["inv_off"] + b * NB * NB:f["inv_off"] + (b + 1) * NB * NB].reshape(NB, NB)[:nb, :nb]
                y = Li @ w[c0:c0 + nb]
                w[c0:c0 + nb] = y
                w[c0 + nb:] -= Fp[c0 + nb:, c0:c0 + nb] @ y
            V[f["voff"]:f["voff"] + ld] = w
    for lev in reversed(plan["levels"]):
        for fi in lev["fronts"]:
            f = fr[fi]
            ld, m = f["m"] + f["u"], f["m"]
            Fp = col(f)
            w = V[f["voff"]:f["voff"] + ld].copy()
            for n in nodes[f["node_off"] + f["n_s_nodes"]:f["node_off"] + f["n_nodes"]]:
                w[n["pos"]:n["pos"] + n["size"]] = pN[n["pn_off"]:n["pn_off"] + n["size"]]
            w[:m] -= Fp[m:, :m].T @ w[m:]
            for b in reversed(range((m + NB - 1) // NB)):
                c0, nb = b * NB, min(NB, m - b * NB)
                Li = Inv[f["inv_off"] + b * NB * NB:f["inv_off"] + (b + 1) * NB * NB].reshape(NB, NB)[:nb, :nb]
                xb = Li.T @ w[c0:c0 + nb]
                w[c0:c0 + nb] = xb
                w[:c0] -= Fp[c0:c0 + nb, :c0].T @ xb
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
