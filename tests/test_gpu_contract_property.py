"""Property test of device contractions: the random U(1) and Z2 leg
structures of the host planner's property test (ranks 1-5, up to four
sectors of dimension 1-3 per leg, any directions and contracted legs),
filled with seeded Gaussian values inside the addition rule, contracted on
the device in FP64 and FP32 and compared with np.tensordot of the dense
embeddings; nothing appears outside the output's addition rule."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings

import paper_1808_10804_amd as st
from oracle import u1
from test_planner_property_host import contractions
from workload import from_dense, to_dense, rel

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-13, "f32": 1e-6}


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
    ref = np.tensordot(A, B, axes=(ax_a, ax_b))
    for prec in ("f64", "f32"):
        Ad = from_dense(A, legs_a, flux=fa, dtype=prec, group=group)
        Bd = from_dense(B, legs_b, flux=fb, dtype=prec, group=group)
        Cd = st.contract(Ad, Bd, ax_a, ax_b, prec=prec)
        got = to_dense(Cd)
        assert got.shape == ref.shape
        assert rel(got, ref) <= TOL[prec], (group, prec, legs_a, legs_b, ax_a, ax_b)
        Lc = [u1.Leg(s, d) for s, d in Cd.legs()]
        assert np.all(got[~u1.conserving_mask(Lc, Cd.flux, modulus)] == 0)
