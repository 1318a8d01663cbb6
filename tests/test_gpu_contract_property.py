"""Property test of device contractions: the random U(1) and Z2 leg
structures of the host planner's property test (ranks 1-5, up to four
sectors of dimension 1-3 per leg, any directions and contracted legs),
filled with seeded Gaussian values inside the addition rule, contracted on
the device in FP64, FP32, bf16x3 and bf16x6 (FP32 storage) with a random output
permutation, and compared with np.tensordot of the dense embeddings;
nothing appears outside the output's addition rule.  Each element is held
to the componentwise bound of a dot product, |error| <= g * sum |a||b|, a
bound relative to the sum of |a||b| rather than to the result, which may
cancel.  For precision unit u, g collects three parts:
  - input rounding: none in FP64, 2u when FP64 values are stored in FP32;
  - accumulation over the contracted dimension K: K u;
  - output rounding: u.
bf16x3 adds its split error: with x = hi + lo in bf16 (unit 2^-8), dropping
lo*lo and rounding lo leave at most about 3 (2^-8)^2 per product.  bf16x6
splits the FP32 value exactly into hi + mid + lo; the dropped mid*lo,
lo*mid and lo*lo add at most about 3 (2^-8)^3 per product."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings

import paper_1808_10804_amd as st
from oracle import u1
from test_planner_property_host import contractions
from workload import from_dense, to_dense

pytestmark = pytest.mark.gpu

U = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "bf16x3": 2.0 ** -24, "bf16x6": 2.0 ** -24}
SPLIT = {"bf16x3": 3 * 2.0 ** -16, "bf16x6": 3 * 2.0 ** -24}


@settings(max_examples=60, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(contractions())
def test_contract_matches_dense(case):
    group, legs_a, legs_b, fa, fb, ax_a, ax_b = case
    modulus = 2 if group == "z2" else 0
    rng = np.random.default_rng(1818)
    La = [u1.Leg(s, d) for s, d in legs_a]
    Lb = [u1.Leg(s, d) for s, d in legs_b]
    A = rng.standard_normal([l.size for l in La]) * u1.conserving_mask(La, fa, modulus)
    B = rng.standard_normal([l.size for l in Lb]) * u1.conserving_mask(Lb, fb, modulus)
    perm = [int(p) for p in rng.permutation(len(legs_a) + len(legs_b) - 2 * len(ax_a))]
    ref = np.tensordot(A, B, axes=(ax_a, ax_b)).transpose(perm)
    scale = np.tensordot(np.abs(A), np.abs(B), axes=(ax_a, ax_b)).transpose(perm)
    K = int(np.prod([La[i].size for i in ax_a]))
    for prec in ("f64", "f32", "bf16x3", "bf16x6"):
        store = "f64" if prec == "f64" else "f32"
        Ad = from_dense(A, legs_a, flux=fa, dtype=store, group=group)
        Bd = from_dense(B, legs_b, flux=fb, dtype=store, group=group)
        Cd = st.contract(Ad, Bd, ax_a, ax_b, out_perm=perm, prec=prec)
        got = to_dense(Cd)
        assert got.shape == ref.shape
        g = (K + (1 if prec == "f64" else 3)) * U[prec] + SPLIT.get(prec, 0.0)
        assert np.all(np.abs(got - ref) <= g * scale), (group, prec, legs_a, legs_b, ax_a, ax_b)
        Lc = [u1.Leg(s, d) for s, d in Cd.legs()]
        assert np.all(got[~u1.conserving_mask(Lc, Cd.flux, modulus)] == 0)
