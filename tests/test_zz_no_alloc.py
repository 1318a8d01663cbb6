"""The allocation-free contraction (symten_contract_noalloc) against
symten_contract on the same inputs: the enlarged-corner step CTT . a of the
D = 6, chi = 64 workload, then the smaller D = 4, chi = 16 one, in FP32, FP64
and the bf16x6 split, one call after another through the shared work area;
every block of the caller's tensor that the contraction reaches equals the
library's result within the stated tolerance (the same kernels and order of
accumulation, so in practice bit for bit), the others are zero, and an
earlier call's output is not touched by a later one.  A contraction larger
than the work area is refused on the host with SYMTEN_E_CAPACITY."""
import numpy as np
import pytest

import paper_1808_10804_amd as st
from synth import config
from workload import device_side, rel

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16x6": 1e-5}


def _ctt_and_a(ci, dtype):
    c = config(ci)
    dev = device_side(c, c["seed"], dtype)
    prec = "f64" if dtype == "f64" else "f32"
    CT = st.contract(dev["C1"], dev["T1"], [1], [0], prec=prec)
    CTT = st.contract(CT, dev["T4"], [0], [2], prec=prec)
    return CTT, dev["a"]


def _check(out, ref, prec):
    got, want = out.block_dict(), ref.block_dict()
    for lab, blk in got.items():
        if lab in want:
            assert rel(blk, want[lab]) <= TOL[prec], (lab, rel(blk, want[lab]))
        else:
            assert not np.any(blk), lab
    assert set(want) <= set(got)


def test_noalloc_matches_contract_twice_in_a_row():
    cases = [(2, "f32", "f32"), (1, "f32", "f32"), (1, "f64", "f64"), (2, "f32", "bf16x6")]
    kept = []
    for ci, dtype, prec in cases:
        print(f"noalloc: cfg {ci} CTT.a {prec}", flush=True)
        CTT, a = _ctt_and_a(ci, dtype)
        ref = st.contract(CTT, a, [3, 0], [0, 1], prec=prec)
        out = st.Tensor.create(ref.legs(), ref.flux, dtype)
        out.upload(np.full(out.nnz, 7.0))              # stale values are overwritten or zeroed
        st.contract_noalloc(out, CTT, a, [3, 0], [0, 1], prec=prec)
        _check(out, ref, prec)
        print(f"noalloc: cfg {ci} {prec}: equal to symten_contract bit for bit: "
              f"{all(np.array_equal(out.block_dict()[k], v) for k, v in ref.block_dict().items())}", flush=True)
        kept.append((out, out.download()))
    for out, values in kept:                          # later calls left earlier outputs alone
        assert np.array_equal(out.download(), values)


def test_noalloc_refuses_more_than_the_work_area():
    c = config(4)
    dev = device_side(c, c["seed"], "f32")
    CT = st.contract(dev["C1"], dev["T1"], [1], [0], prec="f32")
    CTT = st.contract(CT, dev["T4"], [0], [2], prec="f32")
    info, meta = st.plan_info(CTT, dev["a"], [3, 0], [0, 1])
    out = st.Tensor.create(meta.legs(), meta.flux, "f32")
    with pytest.raises(st.SymtenError) as e:
        st.contract_noalloc(out, CTT, dev["a"], [3, 0], [0, 1], prec="f32")
    assert e.value.code == -7 and "work area" in str(e.value)


def test_noalloc_rejects_a_wrong_output():
    CTT, a = _ctt_and_a(1, "f32")
    ref = st.contract(CTT, a, [3, 0], [0, 1], prec="f32")
    legs = ref.legs()
    wrong = st.Tensor.create(legs[:-1] + [(legs[-1][0], -legs[-1][1])], ref.flux, "f32")
    with pytest.raises(st.SymtenError) as e:
        st.contract_noalloc(wrong, CTT, a, [3, 0], [0, 1], prec="f32")
    assert e.value.code == -1
