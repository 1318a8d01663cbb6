"""Property test of the host contraction planner (no GPU): for random leg
structures, fluxes and choices of contracted legs, U(1) and Z2, the planned
contraction has exactly the oracle's matched block pairs, output blocks,
output legs, flux and useful flops (the integer bookkeeping of Sec. 2's
block-sparse contraction, bit-exact).  Examples are derandomised, so every
run checks the same cases."""
from hypothesis import HealthCheck, given, settings, strategies as S

import paper_1808_10804_amd as st
from oracle import u1

POOL = {"u1": [-4, -2, 0, 2, 4], "z2": [0, 1]}


@S.composite
def contractions(draw):
    """Two tensors with a reference block each (one sector per leg, the
    flux set to that block's total charge), B's reference charges on the
    contracted legs equal to A's, so every case has at least one matched
    pair; the other sectors make the structures around it."""
    group = draw(S.sampled_from(["u1", "z2"]))
    mod = 2 if group == "z2" else 0

    def leg(ref=None):
        qs = draw(S.sets(S.sampled_from(POOL[group]), min_size=1, max_size=4))
        ref = draw(S.sampled_from(sorted(qs))) if ref is None else ref
        qs = sorted(set(qs) | {ref})
        return {q: draw(S.integers(1, 3)) for q in qs}, draw(S.sampled_from([1, -1])), ref

    ra, rb = draw(S.integers(1, 4)), draw(S.integers(1, 4))
    nc = draw(S.integers(1, min(ra, rb)))
    if ra + rb - 2 * nc < 1:          # keep an output leg
        nc -= 1
    if nc < 1:
        ra, nc = ra + 1, 1
    A = [leg() for _ in range(ra)]
    ax_a = draw(S.permutations(list(range(ra))))[:nc]
    ax_b = draw(S.permutations(list(range(rb))))[:nc]
    B = [leg() for _ in range(rb)]
    for i, j in zip(ax_a, ax_b):      # contracted pairs: same sectors, opposite directions
        B[j] = (dict(A[i][0]), -A[i][1], A[i][2])

    def flux(legs):
        f = sum(d * r for _, d, r in legs)
        return f % mod if mod else f
    legs_a = [(sec, d) for sec, d, _ in A]
    legs_b = [(sec, d) for sec, d, _ in B]
    return group, legs_a, legs_b, flux(A), flux(B), ax_a, ax_b


@settings(max_examples=200, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(contractions())
def test_plan_matches_oracle_pair_table(case):
    group, legs_a, legs_b, fa, fb, ax_a, ax_b = case
    modulus = 2 if group == "z2" else 0
    A = st.Tensor.meta(legs_a, flux=fa, dtype="f32", group=group)
    B = st.Tensor.meta(legs_b, flux=fb, dtype="f32", group=group)
    La = [u1.Leg(s, d) for s, d in legs_a]
    Lb = [u1.Leg(s, d) for s, d in legs_b]
    SA = u1.Struct(La, u1.allowed_blocks(La, fa, modulus))
    SB = u1.Struct(Lb, u1.allowed_blocks(Lb, fb, modulus))
    assert [b[0] for b in A.blocks()] == SA.blocks and [b[0] for b in B.blocks()] == SB.blocks
    s, m = st.plan_info(A, B, ax_a, ax_b)
    o = u1.pair_table(SA, SB, ax_a, ax_b)
    assert s["pairs"] == len(o["pairs"])
    assert s["out_blocks"] == len(o["outputs"])
    assert s["useful_flops"] == o["flops"]
    assert [b[0] for b in m.blocks()] == o["out"].blocks
    assert m.legs() == [(l.sectors(), l.dir) for l in o["out"].legs]
    assert m.flux == ((fa + fb) % 2 if modulus else fa + fb)
    assert s["gemm_flops"] >= s["useful_flops"]
