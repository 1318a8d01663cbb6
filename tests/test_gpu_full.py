"""GPU checks at the full workload sizes, in the launch configurations the
benchmark times: sampled outputs the oracle computes one slice at a time, and
properties that hold at any size."""
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
    """All 64 corners of the batched workload: the grouped bf16x3 graph launch
    against per-contraction FP32 launches, and two of them against the oracle."""
    c5 = config(5)
    draws = batched_draws(c5["seed"], c5["batch"], c5["D_choices"], c5["chi_range"])
    cfgs = [dict(phys=c5["phys"], virt=d["virt"], chi=d["chi"], flux=c5["flux"]) for d in draws]
    devs = [device_side(cf, c5["seed"], "f32", batch=b) for b, cf in enumerate(cfgs)]
    args = [[d[k] for d in devs] for k in ("C1", "T1", "T4", "a")]
    outs, info = st.enlarged_corners_batched(*args, prec="bf16x3", use_graph=True)
    outs2, _ = st.enlarged_corners_batched(*args, prec="bf16x3", use_graph=True)   # replay
    worst = 0.0
    for b, dv in enumerate(devs):
        single, _ = st.enlarged_corner(1, dv["C1"], dv["T1"], dv["T4"], dv["a"], prec="f32")
        x, y = outs[b].download(), single.download()
        assert np.array_equal(x, outs2[b].download())
        worst = max(worst, rel(x, y))
    print(f"cfg5: worst bf16x3 vs f32 rel diff {worst:.3e}")
    assert worst <= 2e-5
    small = sorted(range(len(draws)), key=lambda b: (draws[b]["D"], draws[b]["chi_total"]))[:2]
    for b in small:
        w, T, a, _ = oracle_side(cfgs[b], c5["seed"], batch=b)
        ref = u1.enlarged_corners(w, T, a)[0].transpose(2, 0, 3, 1)
        assert rel(to_dense(outs[b], u1.corner_tables(w, 1)[2]["out"].legs), ref) <= 1e-5
