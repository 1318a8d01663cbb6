"""Host-side checks of the library's SU(2) bookkeeping (no GPU): its
Clebsch-Gordan coefficients and coupling-tree blocks against the oracle, and
the terms of SU(2) contraction plans against the recoupling scalars computed
here from the oracle's basis tensors."""
import itertools

import numpy as np
import pytest

import paper_1808_10804_amd as st
from oracle import su2
from synth import config

IN, OUT = 1, -1


def test_cg_matches_oracle_small_spins():
    worst = 0.0
    for tj1, tj2 in itertools.product(range(0, 5), repeat=2):
        for tJ in range(abs(tj1 - tj2), tj1 + tj2 + 1, 2):
            for tm1, tm2 in itertools.product(su2.ms(tj1), su2.ms(tj2)):
                if abs(tm1 + tm2) <= tJ:
                    worst = max(worst, abs(st.su2_cg(tj1, tm1, tj2, tm2, tJ, tm1 + tm2)
                                           - su2.cg(tj1, tm1, tj2, tm2, tJ, tm1 + tm2)))
    assert worst < 1e-15


@pytest.mark.parametrize("args", [(9, 3, 7, -1, 10, 2), (12, 0, 12, 0, 12, 0), (11, -5, 8, 4, 5, -1),
                                  (16, 6, 14, -8, 4, -2), (20, 10, 20, -10, 0, 0)])
def test_cg_matches_oracle_large_spins(args):
    assert abs(st.su2_cg(*args) - su2.cg(*args)) < 1e-13


def _cg_range_points(n, seed):
    """Coefficients across the library's advertised range (doubled spins
    0..64, J up to 128): random points plus the extremes (J at either end of
    the triangle, stretched and zero projections)."""
    rng = np.random.default_rng(seed)
    pts = [(64, 64, 64, -64, 0, 0), (64, 64, 64, 64, 128, 128), (64, 0, 64, 0, 128, 0), (64, 0, 64, 0, 64, 0),
           (64, 2, 64, 0, 2, 2), (63, -63, 1, 1, 62, -62), (64, 30, 62, -31, 96, -1), (1, 1, 64, -64, 63, -63)]
    while len(pts) < n:
        tj1, tj2 = (int(x) for x in rng.integers(0, 65, 2))
        tJ = int(rng.choice(np.arange(abs(tj1 - tj2), tj1 + tj2 + 1, 2)))
        tm1 = int(rng.choice(su2.ms(tj1)))
        cands = [m for m in su2.ms(tj2) if abs(tm1 + m) <= tJ]
        if cands:
            tm2 = int(rng.choice(cands))
            pts.append((tj1, tm1, tj2, tm2, tJ, tm1 + tm2))
    return pts


def test_cg_matches_sympy_across_advertised_range():
    """Racah's alternating sum in extended precision keeps FP64 accuracy up to
    2j = 64: absolute error at most a few ulps of 1, relative error 1e-12."""
    worst_abs = worst_rel = 0.0
    for args in _cg_range_points(300, 11):
        got, ref = st.su2_cg(*args), su2.cg(*args)
        worst_abs = max(worst_abs, abs(got - ref))
        if ref != 0.0:
            worst_rel = max(worst_rel, abs(got - ref) / abs(ref))
    assert worst_abs < 4e-15, worst_abs
    assert worst_rel < 1e-12, worst_rel


def test_cg_orthogonality_at_large_spin():
    """Sum over m1 + m2 = M of <j1 m1; j2 m2|J M><j1 m1; j2 m2|J' M> = delta_JJ'
    at j1 = 32, j2 = 31 (every J, M = 1 and M = 61)."""
    tj1, tj2 = 64, 62
    for tM in (2, 122):
        Js = [J for J in range(abs(tj1 - tj2), tj1 + tj2 + 1, 2) if J >= abs(tM)]
        rows = [(m1, tM - m1) for m1 in su2.ms(tj1) if abs(tM - m1) <= tj2]
        U = np.array([[st.su2_cg(tj1, m1, tj2, m2, J, tM) for J in Js] for m1, m2 in rows])
        assert np.abs(U.T @ U - np.eye(len(Js))).max() < 1e-13


def test_cg_selection_rules():
    assert st.su2_cg(2, 0, 2, 0, 2, 0) == 0.0      # parity zero of <1 0; 1 0 | 1 0>
    assert st.su2_cg(1, 1, 1, 1, 0, 2) == 0.0      # |M| > J
    assert st.su2_cg(2, 2, 2, 0, 2, 0) == 0.0      # m1 + m2 != M
    assert st.su2_cg(2, 0, 2, 0, 6, 0) == 0.0      # triangle rule


SU2_LEGSETS = [
    [({0: 1, 1: 2, 2: 1}, IN), ({1: 2, 2: 1}, IN), ({0: 1, 1: 1, 2: 1, 3: 1}, OUT)],
    [({1: 1}, IN), ({0: 1, 1: 3, 2: 1}, IN), ({0: 1, 1: 3, 2: 1}, IN), ({0: 1, 1: 1}, OUT), ({1: 2, 2: 1}, OUT)],
    [({0: 1, 2: 1}, IN), ({1: 1, 3: 1}, OUT), ({0: 1, 1: 1, 2: 2}, OUT), ({1: 1, 2: 1}, OUT)],
    [({0: 2, 1: 1}, OUT), ({1: 1, 2: 1}, OUT), ({0: 1, 1: 1}, OUT)],
]


def test_cfg3_fused_leg_is_the_product_of_virtual_legs():
    c = config(3)
    assert su2.fuse(su2.Leg(c["virt"], IN), su2.Leg(c["virt"], IN), IN).sectors() == c["dd"]


def _cfg3_legs():
    c = config(3)
    X, dd = c["chi"], c["dd"]
    return {"C1": [(X, IN), (X, OUT)], "T1": [(X, IN), (dd, OUT), (X, OUT)],
            "T4": [(X, IN), (dd, OUT), (X, OUT)], "a": [(dd, IN), (dd, IN), (dd, OUT), (dd, OUT)]}


@pytest.mark.parametrize("spec", SU2_LEGSETS + list(_cfg3_legs().values()))
def test_blocks_match_oracle(spec):
    T = st.Tensor.meta(spec, group="su2")
    got = [(lab, tr) for (lab, _, _, _), tr in zip(T.blocks(), T.trees())]
    legs = [su2.Leg(s, d) for s, d in spec]
    assert got == su2.blocks(legs)
    assert T.nnz == su2.nnz(legs)
    for (lab, shp, _, _), (tj, _) in zip(T.blocks(), su2.blocks(legs)):
        assert shp == tuple(l.n(t) for l, t in zip(legs, tj))


def _terms(specA, specB, conA, conB, perm):
    """Non-zero recoupling scalars X = <c_b, c_A . c_B> / <c_b, c_b> of every
    (A block, B block, output block), from the oracle's basis tensors."""
    LA = [su2.Leg(s, d) for s, d in specA]
    LB = [su2.Leg(s, d) for s, d in specB]
    fA = [l for l in range(len(LA)) if l not in conA]
    fB = [l for l in range(len(LB)) if l not in conB]
    Lo_un = [LA[l] for l in fA] + [LB[l] for l in fB]
    Lo = [Lo_un[p] for p in perm]
    out_blocks = su2.blocks(Lo)
    terms = {}
    for ia, (tja, tra) in enumerate(su2.blocks(LA)):
        ca = su2.cgc_tensor(LA, tja, tra)
        for ib, (tjb, trb) in enumerate(su2.blocks(LB)):
            if any(tja[x] != tjb[y] for x, y in zip(conA, conB)):
                continue
            cb = su2.cgc_tensor(LB, tjb, trb)
            p = np.tensordot(ca, cb, axes=(conA, conB)).transpose(perm)
            tjo = tuple(([tja[l] for l in fA] + [tjb[l] for l in fB])[q] for q in perm)
            for ob, (tj, tr) in enumerate(out_blocks):
                if tj != tjo:
                    continue
                co = su2.cgc_tensor(Lo, tj, tr)
                x = np.sum(co * p) / np.sum(co * co)
                if abs(x) > 1e-13:
                    terms[(ia, ib, ob)] = x
    return terms, LA, LB, Lo, out_blocks, fA, fB


CONTRACTIONS = [
    # (A legs, B legs, contracted A legs, contracted B legs, out perm)
    ([({0: 1, 1: 2}, IN), ({1: 2, 2: 1}, IN), ({0: 1, 1: 1, 2: 1}, OUT)],
     [({0: 1, 1: 1, 2: 1}, IN), ({1: 1, 3: 1}, OUT), ({0: 2, 2: 1}, OUT)], [2], [0], [0, 1, 2, 3]),
    ([({0: 1, 1: 2}, IN), ({1: 2, 2: 1}, IN), ({0: 1, 1: 1, 2: 1}, OUT)],
     [({0: 1, 1: 1, 2: 1}, IN), ({1: 1, 3: 1}, OUT), ({0: 2, 2: 1}, OUT)], [2], [0], [3, 1, 0, 2]),
    ([({1: 2, 3: 1}, IN), ({0: 1, 2: 2}, IN), ({1: 1, 2: 1}, OUT), ({0: 1, 1: 1}, OUT)],
     [({1: 1, 2: 1}, IN), ({0: 1, 1: 1}, IN), ({1: 2, 2: 1}, OUT)], [2, 3], [0, 1], [2, 0, 1]),
]


@pytest.mark.parametrize("case", range(len(CONTRACTIONS)))
def test_plan_terms_match_recoupling_scalars(case):
    """Pairs, output blocks and useful flops of the library's plan equal the
    counts implied by the non-zero recoupling scalars computed here."""
    specA, specB, conA, conB, perm = CONTRACTIONS[case]
    terms, LA, LB, Lo, out_blocks, fA, fB = _terms(specA, specB, conA, conB, perm)
    A = st.Tensor.meta(specA, group="su2")
    B = st.Tensor.meta(specB, group="su2")
    info, O = st.plan_info(A, B, conA, conB, out_perm=perm)
    reached = sorted({ob for (_, _, ob) in terms})
    got = [(lab, tr) for (lab, _, _, _), tr in zip(O.blocks(), O.trees())]
    assert got == [out_blocks[ob] for ob in reached]
    assert info["pairs"] == len(terms)
    # one GEMM per output block; its K runs over the distinct A blocks of its
    # terms (B blocks summed with their scalars) or over the distinct B
    # blocks, whichever is shorter
    ba, bb = su2.blocks(LA), su2.blocks(LB)
    fl = 0
    for ob in reached:
        tj = out_blocks[ob][0]
        mn = np.prod([Lo[j].n(tj[j]) for j in range(len(Lo))])
        ia_set = {ia for (ia, ib, o) in terms if o == ob}
        ib_set = {ib for (ia, ib, o) in terms if o == ob}
        ka = sum(np.prod([LA[l].n(ba[ia][0][l]) for l in conA]) for ia in ia_set)
        kb = sum(np.prod([LB[l].n(bb[ib][0][l]) for l in conB]) for ib in ib_set)
        fl += 2 * mn * min(ka, kb)
    assert info["useful_flops"] == fl
    # output legs are the free legs in the requested order
    assert [({t: n for t, n in zip(l.tjs, l.mult)}, l.dir) for l in Lo] == O.legs()


def test_cfg3_corner_plans():
    """The three steps of the SU(2) enlarged corner plan on the host."""
    L = _cfg3_legs()
    T = {k: st.Tensor.meta(v, group="su2") for k, v in L.items()}
    i1, s1 = st.plan_info(T["C1"], T["T1"], [1], [0])
    i2, s2 = st.plan_info(s1, T["T4"], [0], [2])
    i3, s3 = st.plan_info(s2, T["a"], [3, 0], [0, 1])
    assert s3.rank == 4 and [d for _, d in s3.legs()] == [OUT, IN, OUT, OUT]
    assert i3["pairs"] > 0 and i3["useful_flops"] > i2["useful_flops"] > i1["useful_flops"]
