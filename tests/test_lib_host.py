"""Host-side checks of libsymten (no GPU): exports, block enumeration and
contraction planning bit-exact against the oracle's brute force, error codes."""
import ctypes as C
import os
import re

import pytest

import paper_1808_10804_amd as st
from paper_1808_10804_amd import _lib
from oracle import u1
from oracle.u1 import Workload
from synth import config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "symten.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    names = set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\**\s+\**([a-z_0-9]+)\s*\(", hdr, flags=re.M))
    assert {"symten_create", "symten_contract", "ctm_move"} <= names
    L = C.CDLL(_lib.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing
    assert set(_lib.SIGNATURES) == names


def _legs_of(w, name):
    legs, flux = w.legs_of(name)
    return [(l.sectors(), l.dir) for l in legs], flux


def _meta(w, name, dtype="f64"):
    legs, flux = _legs_of(w, name)
    return st.Tensor.meta(legs, flux=flux, dtype=dtype)


@pytest.mark.parametrize("ci", [1, 2, 4])
def test_block_enumeration_matches_oracle(ci):
    c = config(ci)
    w = Workload(c["phys"], c["virt"], c["chi"], c["flux"])
    for name in ["A", "C1", "T1", "T2", "T3", "T4"]:
        t = _meta(w, name)
        legs, flux = w.legs_of(name)
        ob = u1.allowed_blocks(legs, flux)
        lb = [b[0] for b in t.blocks()]
        assert lb == ob
        assert t.nnz == u1.nnz(legs, flux)
        # contiguous row-major layout in canonical order
        pos = 0
        for lab, shp, off, strides in t.blocks():
            assert off == pos
            exp, acc = [], 1
            for d in reversed(shp):
                exp.insert(0, acc)
                acc *= d
            assert strides == tuple(exp)
            pos += acc


def _a_meta(w, dtype="f64"):
    return st.Tensor.meta([(l.sectors(), l.dir) for l in w.a_legs], flux=0, dtype=dtype)


CORNER_INPUTS = {1: ("C1", "T1", "T4"), 2: ("C2", "T1", "T2"), 3: ("C3", "T3", "T2"), 4: ("C4", "T3", "T4")}
CORNER_LEGS = {1: ([1], [0], [0], [2], [3, 0], [0, 1]), 2: ([0], [2], [0], [0], [1, 2], [1, 2]),
               3: ([1], [0], [0], [2], [3, 0], [2, 3]), 4: ([0], [2], [0], [0], [2, 1], [0, 3])}


def _corner_plan(w, which):
    cn, ta, tb = CORNER_INPUTS[which]
    l = CORNER_LEGS[which]
    s1, m1 = st.plan_info(_meta(w, cn), _meta(w, ta), l[0], l[1])
    s2, m2 = st.plan_info(m1, _meta(w, tb), l[2], l[3])
    s3, m3 = st.plan_info(m2, _a_meta(w), l[4], l[5])
    return [(s1, m1), (s2, m2), (s3, m3)]


@pytest.mark.parametrize("ci", [1, 2, 4])
@pytest.mark.parametrize("which", [1, 2, 3, 4])
def test_corner_plans_bit_exact(ci, which):
    c = config(ci)
    w = Workload(c["phys"], c["virt"], c["chi"], c["flux"])
    lib_steps = _corner_plan(w, which)
    orc_steps = u1.corner_tables(w, which)
    for (s, m), o in zip(lib_steps, orc_steps):
        assert s["pairs"] == len(o["pairs"])
        assert s["out_blocks"] == len(o["outputs"])
        assert s["useful_flops"] == o["flops"]
        assert [b[0] for b in m.blocks()] == o["out"].blocks
        assert [leg for leg in m.legs()] == [(l.sectors(), l.dir) for l in o["out"].legs]
        # the fused charge-sector GEMMs never do less than the useful work
        assert s["gemm_flops"] >= s["useful_flops"]


@pytest.mark.parametrize("ci", [1, 2])
def test_halves_plans_bit_exact(ci):
    c = config(ci)
    w = Workload(c["phys"], c["virt"], c["chi"], c["flux"])
    corners = {k: _corner_plan(w, k)[2][1] for k in (1, 2, 3, 4)}
    t = u1.move_tables(w, w.chi)
    su, mu = st.plan_info(corners[1], corners[2], [0, 2], [0, 2])
    sd, md = st.plan_info(corners[4], corners[3], [0, 3], [0, 2])
    for s, m, o in [(su, mu, t["hu"]), (sd, md, t["hd"])]:
        assert (s["pairs"], s["out_blocks"], s["useful_flops"]) == (len(o["pairs"]), len(o["outputs"]), o["flops"])
        assert [b[0] for b in m.blocks()] == o["out"].blocks
    # one dense GEMM per fused charge of the left cut, sized n_Q x n_Q x n_Q
    nL = u1.fused_sectors(w, "diff")
    assert su["groups"] == len(nL)
    assert su["gemm_flops"] == sum(2 * n ** 3 for n in nL.values())


def test_out_perm_and_flux():
    legsA = [({-1: 2, 1: 3}, 1), ({0: 2, 2: 1}, -1)]
    legsB = [({0: 2, 2: 1}, 1), ({-1: 1, 1: 2}, -1), ({0: 4}, 1)]
    A = st.Tensor.meta(legsA, flux=1, dtype="f32")
    B = st.Tensor.meta(legsB, flux=-1, dtype="f32")
    s, m = st.plan_info(A, B, [1], [0], out_perm=[2, 0, 1])
    assert m.flux == 0
    assert [l for l in m.legs()] == [legsB[2], legsA[0], legsB[1]]
    SA = u1.Struct.allowed([u1.Leg(*l) for l in legsA], 1)
    SB = u1.Struct.allowed([u1.Leg(*l) for l in legsB], -1)
    o = u1.pair_table(SA, SB, [1], [0])
    assert s["useful_flops"] == o["flops"] and s["pairs"] == len(o["pairs"])
    perm_blocks = sorted(tuple(b[i] for i in (2, 0, 1)) for b in o["out"].blocks)
    assert [b[0] for b in m.blocks()] == perm_blocks


def test_zero_pairs_is_an_empty_tensor():
    A = st.Tensor.meta([({0: 2}, 1), ({2: 3}, -1)], flux=-2, dtype="f32")
    B = st.Tensor.meta([({2: 3}, 1), ({4: 1}, -1)], flux=-2, dtype="f32")
    B2 = st.Tensor.meta([({2: 3}, 1), ({4: 1}, -1)], flux=0, dtype="f32")   # no allowed block
    assert B2.num_blocks == 0
    s, m = st.plan_info(A, B2, [1], [0])
    assert s["pairs"] == 0 and m.num_blocks == 0 and s["groups"] == 0


def test_error_codes():
    A = st.Tensor.meta([({0: 2}, 1), ({1: 3}, -1)], flux=-1, dtype="f32")
    Bsame = st.Tensor.meta([({1: 3}, -1), ({0: 2}, 1)], flux=-1, dtype="f32")
    Bdims = st.Tensor.meta([({1: 4}, 1), ({0: 2}, -1)], flux=1, dtype="f32")
    with pytest.raises(st.SymtenError) as e:
        st.plan_info(A, Bsame, [1], [0])      # same direction
    assert e.value.code == -2
    with pytest.raises(st.SymtenError) as e:
        st.plan_info(A, Bdims, [1], [0])      # different sector dims
    assert e.value.code == -2
    B = st.Tensor.meta([({1: 3}, 1), ({0: 2}, -1)], flux=1, dtype="f32")
    with pytest.raises(st.SymtenError) as e:
        st.plan_info(A, B, [1], [0], out_perm=[0, 0])
    assert e.value.code == -1
    with pytest.raises(st.SymtenError) as e:
        st.plan_info(A, B, [5], [0])
    assert e.value.code == -1
    # SU(2): flux must be 0 (no quantum-number shift), spins are >= 0
    with pytest.raises(st.SymtenError) as e:
        st.Tensor.meta([({0: 1}, 1), ({0: 1}, -1)], flux=2, group="su2")
    assert e.value.code == -3
    with pytest.raises(st.SymtenError) as e:
        st.Tensor.meta([({-1: 1}, 1), ({1: 1}, -1)], flux=0, group="su2")
    assert e.value.code == -1
    # mixing groups in one contraction
    S = st.Tensor.meta([({1: 3}, 1), ({0: 2}, -1)], flux=0, group="su2")
    with pytest.raises(st.SymtenError) as e:
        st.plan_info(A, S, [1], [0])
    assert e.value.code == -3
    # device operations on metadata-only tensors fail cleanly
    with pytest.raises(st.SymtenError) as e:
        A.upload([0.0] * A.nnz)
    assert e.value.code == -1
    with pytest.raises(st.SymtenError) as e:
        st.contract(A, B, [1], [0])
    assert e.value.code == -1
    # bad descriptors
    with pytest.raises(st.SymtenError):
        st.Tensor.meta([({0: 1}, 2)], flux=0)
    with pytest.raises(st.SymtenError):
        st.Tensor.meta([({0: -1}, 1)], flux=0)


def test_ctm_entry_points_reject_bad_arguments():
    """Argument checks of the CTM driver entry points run before any device
    work: null environments, a bad patch size and bad run options."""
    import ctypes as C
    from paper_1808_10804_amd import _lib
    L = _lib.lib()
    k = C.c_double()
    assert L.ctm_site_partition(None, None, 1, C.byref(k), None, None) == -1
    assert L.ctm_run(None, None, None, None, None) == -1
    o, r = _lib.RunOpts(8, 8, 0, 3, 15, 1e-8), _lib.RunResult()
    assert L.ctm_run(None, None, C.byref(o), C.byref(r), None) == -1


def test_cell_and_corner_entry_points_reject_bad_arguments():
    """Argument checks of the unit-cell, single-layer corner and operator
    double-layer entry points run before any device work."""
    import ctypes as C
    from paper_1808_10804_amd import _lib
    L = _lib.lib()
    h = C.c_void_p()
    assert L.ctm_cell_create(None, 2, 2, None, None) == -1
    assert L.ctm_cell_create(C.byref(h), 0, 2, None, None) == -1
    assert L.ctm_cell_get(None, 0, 0, 0, C.byref(h)) == -1
    assert L.ctm_cell_move(None, None, 0, 8, 0, None) == -1
    k = C.c_double()
    assert L.ctm_cell_site_partition(None, 0, 0, None, 1, C.byref(k), None, None) == -1
    assert L.symten_enlarged_corner_single_layer(None, 1, None, None, None, None, 0, None, None) == -1
    assert L.symten_double_layer_op(None, None, None, None) == -1
    assert L.ctm_expectation(None, None, 1, 1, None, C.byref(k), None) == -1
    assert L.ctm_heisenberg_bond_energy(None, None, C.byref(k), C.byref(k), None) == -1


def test_z2_descriptors():
    """Z2 labels are parities 0, 1 and the flux a parity; blocks obey the sum
    rule mod 2 (the parity generating function: 2 x 2 legs of {0: 1, 1: 1}
    give half of the 2^4 entries)."""
    t = st.Tensor.meta([({0: 1, 1: 1}, 1)] * 2 + [({0: 1, 1: 1}, -1)] * 2, flux=1, group="z2")
    assert t.nnz == 8 and all(sum(q) % 2 == 1 for q, _, _, _ in t.blocks())
    with pytest.raises(st.SymtenError):
        st.Tensor.meta([({0: 1, 2: 1}, 1)], flux=0, group="z2")
    with pytest.raises(st.SymtenError):
        st.Tensor.meta([({0: 1, 1: 1}, 1)], flux=2, group="z2")


def test_allocator_registration():
    """The allocator pair: both or neither; nulls return to the library pool."""
    L = _lib.lib()
    a = _lib.ALLOC_FN(lambda n, ctx: None)
    f = _lib.FREE_FN(lambda p, n, ctx: None)
    assert L.symten_set_allocator(C.cast(a, C.c_void_p), None, None) == _lib.OK - 1
    assert L.symten_set_allocator(C.cast(a, C.c_void_p), C.cast(f, C.c_void_p), None) == _lib.OK
    assert L.symten_set_allocator(None, None, None) == _lib.OK


def test_nbytes_of_metadata_tensor():
    t = st.Tensor.meta([({0: 3, 1: 5}, 1), ({0: 3, 1: 5}, -1)], flux=0, dtype="f64")
    assert t.nbytes == t.nnz * 8 == 34 * 8
