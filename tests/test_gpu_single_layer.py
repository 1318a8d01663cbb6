"""GPU checks of the single-layer enlarged corner (A and A* absorbed
separately, Sec. 3.2's alternative to the double layer): every corner against
the oracle's dense corner and against the library's double-layer corner, in
FP64, FP32 and bf16x3, for U(1) and Z2."""
import numpy as np
import pytest

import paper_1808_10804_amd as st
from oracle import u1
from synth import config
from workload import oracle_side, device_side, to_dense, rel, from_dense

pytestmark = pytest.mark.gpu

NAMES = {1: ("C1", "T1", "T4"), 2: ("C2", "T1", "T2"), 3: ("C3", "T3", "T2"), 4: ("C4", "T3", "T4")}
PERM = {1: (2, 0, 3, 1), 2: (0, 2, 1, 3), 3: (2, 0, 3, 1), 4: (2, 0, 1, 3)}   # oracle -> library leg order


@pytest.mark.parametrize("which", [1, 2, 3, 4])
def test_single_layer_corner_cfg1_f64(which):
    c = config(1)
    w, T, a, _ = oracle_side(c, c["seed"])
    dev = device_side(c, c["seed"], "f64")
    n = NAMES[which]
    S, info = st.enlarged_corner_single_layer(which, dev[n[0]], dev[n[1]], dev[n[2]], dev["A"], prec="f64")
    D, _ = st.enlarged_corner(which, dev[n[0]], dev[n[1]], dev[n[2]], dev["a"], prec="f64")
    assert S.legs() == D.legs() and S.flux == D.flux
    ref = u1.enlarged_corners(w, T, a)[which - 1].transpose(PERM[which])
    legs = u1.corner_tables(w, which)[2]["out"].legs
    err = rel(to_dense(S, legs), ref)
    print(f"  corner {which}: single vs oracle {err:.2e}, vs double layer {rel(to_dense(S, legs), to_dense(D, legs)):.2e}")
    assert err <= 1e-13
    assert rel(to_dense(S, legs), to_dense(D, legs)) <= 1e-13


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("bf16x3", 1e-5)])
def test_single_layer_corner_cfg2(prec, tol):
    c = config(2)
    w, T, a, _ = oracle_side(c, c["seed"])
    dev = device_side(c, c["seed"], "f32")
    S, info = st.enlarged_corner_single_layer(1, dev["C1"], dev["T1"], dev["T4"], dev["A"], prec=prec)
    _, dinfo = st.enlarged_corner(1, dev["C1"], dev["T1"], dev["T4"], dev["a"], prec=prec)
    ref = u1.enlarged_corners(w, T, a)[0].transpose(2, 0, 3, 1)
    err = rel(to_dense(S, u1.corner_tables(w, 1)[2]["out"].legs), ref)
    print(f"  cfg2 corner 1 {prec}: rel err {err:.2e}; useful flops single {info['useful_flops']:.3e} "
          f"double {dinfo['useful_flops']:.3e}")
    assert err <= tol
    assert info["useful_flops"] < dinfo["useful_flops"]


def test_single_layer_corner_z2():
    """A Z2 site tensor of flux 1 and a random Z2 environment: the
    single-layer corner equals the double-layer one."""
    rng = np.random.default_rng(11)
    v, ph, chi = {0: 2, 1: 1}, {0: 1, 1: 1}, {0: 3, 1: 2}

    def rand(legs, flux):
        L = [u1.Leg(s, d) for s, d in legs]
        return from_dense(rng.standard_normal([l.size for l in L]) * u1.conserving_mask(L, flux, modulus=2),
                          legs, flux=flux, group="z2")
    A = rand([(ph, 1), (v, 1), (v, 1), (v, -1), (v, -1)], 1)
    a = st.double_layer(A)
    dd = a.legs()[0][0]
    C1 = rand([(chi, 1), (chi, -1)], 0)
    T1 = rand([(chi, 1), (dd, -1), (chi, -1)], 0)
    T4 = rand([(chi, 1), (dd, -1), (chi, -1)], 0)
    S, _ = st.enlarged_corner_single_layer(1, C1, T1, T4, A, prec="f64")
    D, _ = st.enlarged_corner(1, C1, T1, T4, a, prec="f64")
    assert S.legs() == D.legs()
    assert rel(to_dense(S), to_dense(D)) <= 1e-13
