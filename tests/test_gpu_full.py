"""GPU checks at the full workload sizes, in the launch configurations the
benchmark times: sampled outputs the oracle computes one slice at a time, the
oracle's whole D = 8, chi = 200 move stored by tests/golden/make_cfg4_move.py,
and properties that hold at any size."""
import os

import numpy as np
import pytest

import paper_1808_10804_amd as st
from oracle import u1
from synth import config, batched_draws
from workload import oracle_side, device_side, to_dense, rel

pytestmark = pytest.mark.gpu


def _corner1_rows(w, T, a, ys):
    """C~1[x4 in ys, d, x1, r] from the oracle's definition, sliced on x4."""
    e = lambda s, *o: np.einsum(s, *o, optimize="optimal")
    ct = e("ab,bux->aux", T["C1"], T["T1"])
    ctt = e("aux,yla->yxlu", ct, T["T4"][ys])
    return e("yxlu,lurd->ydxr", ctt, a)


def _gpu_rows(Cn, legs, ys):
    """The GPU corner [x1, x4, r, d] restricted to x4 in ys, as [x4, d, x1, r]."""
    L = [u1.Leg(s, d) for s, d in legs]
    out = np.zeros((len(ys), L[3].size, L[0].size, L[2].size))
    qx4 = L[1].state_charges()
    off = L[1].offsets()
    for lab, blk in Cn.block_dict().items():
        q1, q4, qr, qd = lab
        for i, y in enumerate(ys):
            if qx4[y] != q4:
                continue
            iy = y - off[q4]
            s1, sr, sd = (u1.block_slices(L, lab)[k] for k in (0, 2, 3))
            out[i, sd, s1, sr] = blk[:, iy, :, :].transpose(2, 0, 1)
    return out


@pytest.fixture(scope="module")
def cfg4():
    c = config(4)
    return c, oracle_side(c, c["seed"])


CFG4_REF = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg4_leftmove.npz")
# relative Frobenius tolerances of the move against the FP64 oracle; bf16x3
# and BF16 are reported (bf16x3 misses the 1e-5 target on whole moves: its
# bound here is its measured level, to catch regressions)
MOVE_TOL = {"f64": 1e-12, "f32": 1e-5, "bf16x6": 1e-5, "bf16x3": 1e-4, "bf16": 1e-1}


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x6", "bf16x3", "bf16"])
def test_cfg4_move_vs_oracle(prec):
    """One full left move at D = 8, chi = 200 in every precision against the
    dense FP64 oracle's move of the same draws: the whole spectrum of the cut,
    the kept states per charge (asserted when the gap at the cut exceeds 100
    times the tolerance), and the gauge-invariant left column through 16 x 16
    seeded random projections on (x1, x3) and 16 full r-slices."""
    ref = np.load(CFG4_REF)
    c = config(4)
    assert int(ref["seed"]) == c["seed"] and int(ref["chi"]) == c["chi_target"]
    dev = device_side(c, c["seed"], "f64" if prec == "f64" else "f32")
    env = st.CtmEnv([dev[k] for k in ("C1", "C2", "C3", "C4")], [dev[k] for k in ("T1", "T2", "T3", "T4")])
    print(f"cfg4 move {prec}", flush=True)
    stats = env.move(dev["a"], c["chi_target"], prec=prec)
    sv_ref = ref["sv"]
    assert [int(q) for q in ref["sv_q"]] == sorted(stats["sv_sectors"])
    assert [int(n) for n in ref["sv_n"]] == [stats["sv_sectors"][q] for q in sorted(stats["sv_sectors"])]
    e_sv = rel(env.singular_values(), sv_ref)
    kept_ref = {int(q): int(n) for q, n in zip(ref["kept_q"], ref["kept_n"])}
    L = u1.left_column(to_dense(env.get(0)), to_dense(env.get(7)), to_dense(env.get(3)))
    G = np.einsum("ia,arb,jb->ijr", ref["U1"], L, ref["U3"], optimize=True)
    S = np.stack([L[x, :, z] for x, z in zip(ref["slice_x1"], ref["slice_x3"])])
    e_G, e_S = rel(G, ref["G"]), rel(S, ref["slices"])
    gap = float(ref["gap"])
    print(f"cfg4 move {prec}: spectrum {e_sv:.3e}, left column projections {e_G:.3e}, slices {e_S:.3e}, "
          f"kept {stats['kept']} (oracle {kept_ref}, gap {gap:.2e}), {stats['ms_total']:.1f} ms", flush=True)
    tol = MOVE_TOL[prec]
    if gap > 100 * tol:
        assert stats["kept"] == kept_ref
    assert e_sv <= tol and e_G <= tol and e_S <= tol


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_cfg4_corner_sampled_rows(cfg4, prec):
    c, (w, T, a, _) = cfg4
    dev = device_side(c, c["seed"], "f32")
    Cn, info = st.enlarged_corner(1, dev["C1"], dev["T1"], dev["T4"], dev["a"], prec=prec)
    assert info["useful_flops"] == sum(s["flops"] for s in u1.corner_tables(w, 1))
    rng = np.random.default_rng(4)
    nX = u1.Leg(w.chi, 1).size
    ys = sorted(rng.choice(nX, size=6, replace=False).tolist())
    ref = _corner1_rows(w, T, a, ys)
    got = _gpu_rows(Cn, Cn.legs(), ys)
    err = rel(got, ref)
    print(f"cfg4 corner1 {prec} sampled rows: rel err {err:.3e}")
    assert err <= 1e-5


def test_cfg4_move_properties(cfg4):
    """Full move at D=8, chi=200 in FP32: identities that hold at any size."""
    c, (w, T, a, _) = cfg4
    dev = device_side(c, c["seed"], "f32")
    env = st.CtmEnv([dev[k] for k in ("C1", "C2", "C3", "C4")], [dev[k] for k in ("T1", "T2", "T3", "T4")])
    stats = env.move(dev["a"], c["chi_target"], prec="f32")
    kept = stats["kept"]
    assert 0 < sum(kept.values()) <= c["chi_target"]
    assert 0.0 <= stats["trunc_err"] < 1.0
    sv = env.singular_values()
    assert np.all(sv >= 0)
    # per sector: descending; the kept values are the global top ones
    pos, tops = 0, []
    for Q, n in sorted(stats["sv_sectors"].items()):
        s = sv[pos:pos + n]
        assert np.all(np.diff(s) <= 1e-12 * max(1.0, s[0]))
        tops += list(s[:kept.get(Q, 0)])
        pos += n
    assert np.isclose(min(tops), np.sort(sv)[::-1][sum(kept.values()) - 1])
    # P~ P = I per sector (FP64 projectors)
    P, Pt = env.projectors()
    pb, ptb = P.block_dict(), Pt.block_dict()
    for Q, k in kept.items():
        rows = sorted(l for l in pb if l[2] == Q)
        Pq = np.concatenate([pb[l].reshape(-1, k) for l in rows], axis=0)
        Ptq = np.concatenate([ptb[(Q, l[0], l[1])].reshape(k, -1) for l in rows], axis=1)
        assert np.allclose(Ptq @ Pq, np.eye(k), atol=1e-8)
    # unit Frobenius norms of the renormalised tensors
    for idx in (0, 3, 7):
        assert np.isclose(np.linalg.norm(env.get(idx).download()), 1.0, rtol=1e-5)


def test_cfg5_batched_full():
    """All 64 corners of the batched workload, the grouped bf16x3 graph launch:
    every corner against the library's FP64 corner (the path pinned against
    the oracle at cfgs 1 and 2, in FP64 storage of the same draws) and the
    four smallest against the oracle itself, within 1e-5; a replay with the
    same inputs equals the first call bit for bit, in a new buffer; a replay
    with every C1 negated in place (same buffers, so the same graph) gives the
    negated corners (to the split products' rounding: the bf16 MFMA's sums
    are not exactly odd in their inputs) and leaves the earlier results
    intact."""
    c5 = config(5)
    draws = batched_draws(c5["seed"], c5["batch"], c5["D_choices"], c5["chi_range"])
    cfgs = [dict(phys=c5["phys"], virt=d["virt"], chi=d["chi"], flux=c5["flux"]) for d in draws]
    devs = [device_side(cf, c5["seed"], "f32", batch=b) for b, cf in enumerate(cfgs)]
    args = [[d[k] for d in devs] for k in ("C1", "T1", "T4", "a")]
    outs, info = st.enlarged_corners_batched(*args, prec="bf16x3", use_graph=True)
    first = [o.download() for o in outs]
    worst = 0.0
    for b, cf in enumerate(cfgs):
        d64 = device_side(cf, c5["seed"], "f64", batch=b)
        ref64, _ = st.enlarged_corner(1, d64["C1"], d64["T1"], d64["T4"], d64["a"], prec="f64")
        worst = max(worst, rel(first[b], ref64.download()))
        del d64, ref64
    print(f"cfg5: worst bf16x3 corner vs the FP64 path: rel err {worst:.3e}")
    assert worst <= 1e-5
    small = sorted(range(len(draws)), key=lambda b: (draws[b]["D"], draws[b]["chi_total"]))[:4]
    for b in small:
        w, T, a, _ = oracle_side(cfgs[b], c5["seed"], batch=b)
        ref = u1.enlarged_corners(w, T, a)[0].transpose(2, 0, 3, 1)
        assert rel(to_dense(outs[b], u1.corner_tables(w, 1)[2]["out"].legs), ref) <= 1e-5
    same, _ = st.enlarged_corners_batched(*args, prec="bf16x3", use_graph=True)   # replay
    for d in devs:
        d["C1"].upload(-d["C1"].download())
    outs2, _ = st.enlarged_corners_batched(*args, prec="bf16x3", use_graph=True)   # replay, new values
    for b in range(len(devs)):
        assert np.array_equal(outs[b].download(), first[b])
        assert np.array_equal(same[b].download(), first[b])
        assert rel(outs2[b].download(), -first[b]) <= 1e-5
