"""Device sector matching (symten_match_blocks) against the oracle's brute
force (Sec. 2: pairs of blocks with equal labels on the contracted legs,
results grouped by the labels of the open legs), bit-exact: the three
corner contractions of cfgs 1, 2 and 4 (every allowed block of each operand,
so cfg 1's CTT . a step has the 157 pairs of the full allowed intermediate),
the random U(1) and Z2 structures of the host planner's property test, and
lists cut at a capacity with the full counts reported."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings

import paper_1808_10804_amd as st
from oracle import u1
from synth import config
from test_planner_property_host import contractions

pytestmark = pytest.mark.gpu


def _check(legs_a, fa, legs_b, fb, ax_a, ax_b, group="u1"):
    modulus = 2 if group == "z2" else 0
    A = st.Tensor.meta(legs_a, flux=fa, dtype="f32", group=group)
    B = st.Tensor.meta(legs_b, flux=fb, dtype="f32", group=group)
    La = [u1.Leg(s, d) for s, d in legs_a]
    Lb = [u1.Leg(s, d) for s, d in legs_b]
    SA = u1.Struct(La, u1.allowed_blocks(La, fa, modulus))
    SB = u1.Struct(Lb, u1.allowed_blocks(Lb, fb, modulus))
    o = u1.pair_table(SA, SB, list(ax_a), list(ax_b))
    pairs, outl, cnt = st.match_blocks(A, B, list(ax_a), list(ax_b))
    assert cnt[4] == 0
    assert (cnt[0], cnt[1]) == (len(SA.blocks), len(SB.blocks))
    assert cnt[2] == len(o["pairs"]) and cnt[3] == len(o["outputs"])
    got_pairs = [(SA.blocks[a], SB.blocks[b]) for a, b, _, _ in pairs]
    assert got_pairs == o["pairs"]
    outs = [tuple(int(x) for x in r) for r in outl]
    assert outs == o["out"].blocks
    for (ta, tb), (_, _, ob, _) in zip(o["pairs"], pairs):
        assert outs[ob] == tuple(ta[i] for i in range(len(La)) if i not in ax_a) + \
            tuple(tb[j] for j in range(len(Lb)) if j not in ax_b)
    assert int(pairs[:, 3].sum()) == o["flops"]
    return cnt


@pytest.mark.parametrize("ci", [1, 2, 4])
def test_corner_steps_match_oracle(ci):
    c = config(ci)
    w = u1.Workload(c["phys"], c["virt"], c["chi"], c["flux"])
    sec = lambda legs: [(l.sectors(), l.dir) for l in legs]
    C, T1, T4, a = sec(w.C_legs), sec(w.T_legs["T1"]), sec(w.T_legs["T4"]), sec(w.a_legs)
    cnt1 = _check(C, 0, T1, 0, [1], [0])                      # C1 . T1 -> [xa, u, x1]
    CT = [C[0], T1[1], T1[2]]
    cnt2 = _check(CT, 0, T4, 0, [0], [2])                     # CT . T4 -> [u, x1, y, l]
    CTT = [CT[1], CT[2], T4[0], T4[1]]
    cnt3 = _check(CTT, 0, a, 0, [3, 0], [0, 1])               # CTT . a over (l, u)
    print(f"cfg {ci}: pairs {cnt1[2]}, {cnt2[2]}, {cnt3[2]}; outputs {cnt1[3]}, {cnt2[3]}, {cnt3[3]}")
    if ci == 1:
        assert (cnt1[2], cnt2[2], cnt3[2]) == (9, 27, 157)


@settings(max_examples=200, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(contractions())
def test_random_structures_match_oracle(case):
    group, legs_a, legs_b, fa, fb, ax_a, ax_b = case
    _check(legs_a, fa, legs_b, fb, ax_a, ax_b, group)


def test_capacity_cut_reports_full_counts():
    c = config(1)
    w = u1.Workload(c["phys"], c["virt"], c["chi"], c["flux"])
    sec = lambda legs: [(l.sectors(), l.dir) for l in legs]
    T4, a = sec(w.T_legs["T4"]), sec(w.a_legs)
    CTT = [(w.dd, -1), (w.chi, -1), T4[0], T4[1]]
    A = st.Tensor.meta(CTT, flux=0, dtype="f32")
    B = st.Tensor.meta(a, flux=0, dtype="f32")
    full, outs, cnt = st.match_blocks(A, B, [3, 0], [0, 1])
    cut, outs_cut, cnt2 = st.match_blocks(A, B, [3, 0], [0, 1], pair_cap=50, out_cap=10)
    assert cnt2[4] == 1 and list(cnt2[:4]) == list(cnt[:4])
    assert np.array_equal(cut, full[:50])
    assert np.array_equal(outs_cut, outs[:10])
