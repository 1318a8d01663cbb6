"""Pins of the SU(2) oracle (expansion of reduced tensors) against facts that
do not come from the oracle itself: tabulated Clebsch-Gordan values, the
rank-2 example of Sec. 2, orthogonality and completeness of the coupling-tree
basis, invariance under rotations, and S^z conservation."""
import itertools
from math import sqrt

import numpy as np
import pytest

from oracle import su2, u1

IN, OUT = su2.IN, su2.OUT


def _rand(legs, seed):
    return np.random.default_rng(seed).standard_normal(su2.nnz(legs))


def test_cg_tabulated_values():
    """Condon-Shortley values from the standard tables (j1 x 1/2 and 1 x 1)."""
    cg = su2.cg
    assert np.isclose(cg(1, 1, 1, -1, 2, 0), 1 / sqrt(2))
    assert np.isclose(cg(1, -1, 1, 1, 2, 0), 1 / sqrt(2))
    assert np.isclose(cg(1, 1, 1, -1, 0, 0), 1 / sqrt(2))
    assert np.isclose(cg(1, -1, 1, 1, 0, 0), -1 / sqrt(2))
    assert np.isclose(cg(2, 2, 1, -1, 1, 1), sqrt(2 / 3))
    assert np.isclose(cg(2, 0, 1, 1, 1, 1), -sqrt(1 / 3))
    assert np.isclose(cg(2, 0, 2, 0, 0, 0), -sqrt(1 / 3))
    assert np.isclose(cg(2, 2, 2, -2, 0, 0), sqrt(1 / 3))
    assert np.isclose(cg(2, 0, 2, 0, 2, 0), 0.0)
    assert np.isclose(cg(2, 2, 2, 0, 4, 2), sqrt(1 / 2))
    assert cg(1, 1, 1, 1, 0, 2) == 0.0          # |M| > J
    assert cg(2, 0, 2, 0, 6, 0) == 0.0          # triangle rule


@pytest.mark.parametrize("tj1,tj2", [(1, 1), (2, 1), (2, 2), (3, 2), (4, 3)])
def test_cg_orthogonality(tj1, tj2):
    """The coupled states form an orthonormal basis of V_j1 x V_j2."""
    rows = []
    for tJ in range(abs(tj1 - tj2), tj1 + tj2 + 1, 2):
        for tM in su2.ms(tJ):
            rows.append([su2.cg(tj1, m1, tj2, m2, tJ, tM) for m1 in su2.ms(tj1) for m2 in su2.ms(tj2)])
    U = np.array(rows)
    assert U.shape == ((tj1 + 1) * (tj2 + 1),) * 2
    assert np.allclose(U @ U.T, np.eye(len(U)), atol=1e-14)


def test_rank2_example_sec2():
    """Sec. 2's rank-2 example (values in tests/golden/sec2_rank2_example.json,
    as the paper prints them): an (in, out) tensor on spins 0, 1/2, 1 is block
    diagonal, each block a reduced matrix times an identity of size 2j+1, so
    it holds 1, 4 and 9 times as many elements as its reduced block, and the
    block (1/2, 0) is zero; one spin-1/2 multiplet has total dimension 2 and
    reduced dimension 1.  With S^z alone, the S^z = 0 block gathers the
    S = 0 and S = 1 states and S = 1/2 splits into the blocks S^z = +-1/2."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sec2_rank2_example.json")))
    leg = {0: 2, 1: 1, 2: 3}
    legs = [su2.Leg(leg, IN), su2.Leg(leg, OUT)]
    assert [tj for tj, _ in su2.blocks(legs)] == [(t, t) for t in g["doubled_spins"]]
    v = _rand(legs, 1)
    dense = su2.expand(legs, v)
    pos, seen = 0, 0
    for tj, size, ratio in zip(g["doubled_spins"], g["cgc_identity_size"], g["elements_per_reduced_element"]):
        n = leg[tj]
        m = v[pos:pos + n * n].reshape(n, n)
        pos += n * n
        o = legs[0].offsets()[tj]
        blk = dense[o:o + n * size, o:o + n * size]
        assert np.allclose(blk, np.kron(m, np.eye(size)), atol=0)
        assert blk.size == ratio * m.size
        seen += blk.size
    assert np.count_nonzero(dense) <= seen    # nothing off the diagonal blocks
    fb = [int(round(2 * x)) for x in g["forbidden_block"]]
    o1, o0 = legs[0].offsets()[fb[0]], legs[1].offsets()[fb[1]]
    assert not dense[o1:o1 + leg[fb[0]] * (fb[0] + 1), o0:o0 + leg[fb[1]] * (fb[1] + 1)].any()
    assert su2.Leg({1: 1}, IN).size == 2 and su2.Leg({1: 1}, IN).reduced_size == 1
    # the abelian alternative: S^z sectors of the same leg
    sz = su2.Leg(leg, IN).u1_leg().sectors()
    zero_spins = [tj for tj in leg if tj % 2 == 0]
    assert [tj / 2 for tj in zero_spins] == g["abelian_sz_blocks"]["sz_zero_block_spins"]
    assert sz[0] == sum(leg[tj] for tj in zero_spins)
    assert sorted(q / 2 for q in sz if q % 2) == g["abelian_sz_blocks"]["half_integer_blocks"]
    assert sz[1] == sz[-1] == leg[1]


LEGSETS = [
    [({0: 1, 1: 2, 2: 1}, IN), ({1: 2, 2: 1}, IN), ({0: 1, 1: 1, 2: 1, 3: 1}, OUT)],
    [({1: 1}, IN), ({0: 1, 1: 3, 2: 1}, IN), ({0: 1, 1: 3, 2: 1}, IN), ({0: 1, 1: 1}, OUT), ({1: 2, 2: 1}, OUT)],
    [({0: 1, 2: 1}, IN), ({1: 1, 3: 1}, OUT), ({0: 1, 1: 1, 2: 2}, OUT), ({1: 1, 2: 1}, OUT)],
]


@pytest.mark.parametrize("spec", LEGSETS)
def test_tree_basis_complete_and_orthogonal(spec):
    """For every spin tuple the canonical trees are as many as the invariant
    tensors (counted from S^z states), mutually orthogonal, norm^2 = 2K+1."""
    legs = [su2.Leg(s, d) for s, d in spec]
    bl = su2.blocks(legs)
    by_spins = {}
    for tj, tree in bl:
        by_spins.setdefault(tj, []).append(tree)
    for tj in itertools.product(*[l.tjs for l in legs]):
        assert len(by_spins.get(tj, [])) == su2.invariant_count(tj)
    for tj, trees in by_spins.items():
        cs = [su2.cgc_tensor(legs, tj, t).reshape(-1) for t in trees]
        G = np.array([[x @ y for y in cs] for x in cs])
        assert np.allclose(G, np.diag([t[-1] + 1.0 for t in trees]), atol=1e-13)


@pytest.mark.parametrize("spec", LEGSETS)
def test_expanded_tensor_invariant(spec):
    """Expanded tensors are unchanged by the same real rotation d(beta) on every
    leg and conserve S^z: the two facts that together fix SU(2) invariance."""
    legs = [su2.Leg(s, d) for s, d in spec]
    dense = su2.expand(legs, _rand(legs, 2))
    for beta in (0.3, 1.1, 2.9):
        assert np.allclose(su2.rotate(dense, legs, beta), dense, atol=1e-12)
    # S^z: the U(1) reordering is a valid charge-conserving block tensor
    du, ulegs = su2.to_u1(dense, legs)
    mask = u1.conserving_mask(ulegs, 0)
    assert np.all(du[~mask] == 0)
    # not trivially zero
    assert np.linalg.norm(dense) > 0.1


def test_rotation_matrices_are_representations():
    """d(a) d(b) = d(a+b) and orthogonality: the rotations used above are the
    real spin-j representation of rotations about y."""
    for tj in range(0, 5):
        da, db, dab = su2.wigner_d(tj, 0.4), su2.wigner_d(tj, 0.9), su2.wigner_d(tj, 1.3)
        assert np.allclose(da @ db, dab, atol=1e-13)
        assert np.allclose(da @ da.T, np.eye(tj + 1), atol=1e-13)


@pytest.mark.parametrize("spec", LEGSETS)
def test_reduce_inverts_expand(spec):
    legs = [su2.Leg(s, d) for s, d in spec]
    v = _rand(legs, 3)
    assert np.allclose(su2.reduce(legs, su2.expand(legs, v)), v, atol=1e-13)


def test_non_invariant_tensor_is_detected():
    """A dense tensor that is not invariant is not reproduced by its reduction
    (guards against a reduce that simply copies)."""
    legs = [su2.Leg({1: 1}, IN), su2.Leg({1: 1}, OUT)]
    t = np.array([[1.0, 0.0], [0.0, 0.0]])            # |up><up| only
    back = su2.expand(legs, su2.reduce(legs, t))
    assert np.allclose(back, 0.5 * np.eye(2))


def test_contraction_of_expanded_tensors_is_invariant():
    """The dense product of two expanded tensors over a shared leg is again
    invariant and is reproduced exactly by reduce + expand."""
    A = [su2.Leg({0: 1, 1: 2}, IN), su2.Leg({1: 2, 2: 1}, IN), su2.Leg({0: 1, 1: 1, 2: 1}, OUT)]
    B = [su2.Leg({0: 1, 1: 1, 2: 1}, IN), su2.Leg({1: 1, 3: 1}, OUT), su2.Leg({0: 2, 2: 1}, OUT)]
    ta, tb = su2.expand(A, _rand(A, 4)), su2.expand(B, _rand(B, 5))
    tc = np.tensordot(ta, tb, axes=([2], [0]))
    C = A[:2] + B[1:]
    assert np.allclose(su2.expand(C, su2.reduce(C, tc)), tc, atol=1e-12)
    assert np.allclose(su2.rotate(tc, C, 0.7), tc, atol=1e-12)


def test_fused_double_layer_leg():
    """The fused (ket, bra) leg of the SU(2) workload: virtual multiplets
    {0:1, 1/2:3, 1:1} give {0:11, 1/2:12, 1:12, 3/2:6, 2:1}, 100 states, and its
    S^z content equals the U(1) fusion of the expanded legs."""
    v = su2.Leg({0: 1, 1: 3, 2: 1}, IN)
    F = su2.fuse(v, v, IN)
    assert F.sectors() == {0: 11, 1: 12, 2: 12, 3: 6, 4: 1}
    assert F.size == v.size ** 2 == 100
    vu = v.u1_leg()
    fu, _ = u1.fuse(vu, vu, +1, +1, IN)
    assert F.u1_leg().sectors() == fu.sectors()


@pytest.mark.parametrize("dirs", [(IN, IN, OUT), (OUT, IN, IN), (IN, OUT, OUT), (OUT, OUT, IN), (OUT, IN, OUT)])
def test_fusion_isometry_is_unitary(dirs):
    la, lb = su2.Leg({0: 1, 1: 2, 2: 1}, dirs[0]), su2.Leg({1: 1, 2: 2}, dirs[1])
    legs, v = su2.fusion_isometry(la, lb, dirs[2])
    F = su2.expand(legs, v).reshape(la.size * lb.size, -1)
    assert F.shape[0] == F.shape[1]
    assert np.allclose(F.T @ F, np.eye(F.shape[1]), atol=1e-14)
    assert np.allclose(F @ F.T, np.eye(F.shape[0]), atol=1e-14)


def test_double_layer_su2_pins():
    """The fused double layer is an invariant tensor (reduce + expand gives it
    back; a bra leg run in the ket's direction breaks this), the fusion keeps
    the Frobenius norm, and unfusing gives a PSD (ket) x (bra) matrix with
    trace |A|^2."""
    v = {0: 1, 1: 2, 2: 1}
    A_legs = [su2.Leg({1: 1}, IN), su2.Leg(v, IN), su2.Leg(v, IN), su2.Leg(v, OUT), su2.Leg(v, OUT)]
    vals = _rand(A_legs, 7)
    a_legs, ared, ad = su2.double_layer(A_legs, vals)
    assert [l.dir for l in a_legs] == [IN, IN, OUT, OUT]
    assert a_legs[0].sectors() == su2.fuse(A_legs[1], A_legs[1], IN).sectors()
    assert np.allclose(su2.expand(a_legs, ared), ad, atol=1e-13)
    A = su2.expand(A_legs, vals)
    a8 = np.einsum("sabcd,sefgh->aebfcgdh", A, A)
    assert np.isclose(np.linalg.norm(ad), np.linalg.norm(a8))
    # unfuse with the transposed isometries
    u = ad
    for x, vl in enumerate(A_legs[1:]):
        Fl, Fv = su2.fusion_isometry(su2.Leg(vl.sectors(), -vl.dir), su2.Leg(vl.sectors(), vl.dir), vl.dir)
        F = su2.expand(Fl, Fv)
        u = np.tensordot(u, F, axes=([0], [2]))          # fused leg -> (ket, bra), appended
    n = A_legs[1].size
    M = u.reshape([n, n] * 4).transpose(0, 2, 4, 6, 1, 3, 5, 7).reshape(n ** 4, n ** 4)
    assert np.allclose(M, M.T, atol=1e-12)
    assert np.min(np.linalg.eigvalsh(M)) > -1e-10 * np.max(np.abs(M))
    assert np.isclose(np.trace(M), np.sum(A * A))
