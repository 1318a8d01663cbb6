"""Pins of the U(1) oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed-form
counts, an independent algorithm (generating functions, explicit loops, a
row-by-row transfer contraction of the whole network), library routines on
the full matrix, or identities the projector construction must satisfy.
"""
import itertools

import numpy as np
import pytest

from oracle import u1
from oracle.u1 import IN, OUT, Leg, Workload
from synth import config, draw, TENSOR_INDEX, SITE_AND_ENV

TINY = dict(phys={-1: 1, 1: 1}, virt={0: 1, 2: 1}, chi={-2: 1, 0: 2, 2: 1}, flux=1)


def make(cfgd, seed):
    w = Workload(cfgd["phys"], cfgd["virt"], cfgd["chi"], cfgd["flux"])
    vals = {n: draw((seed, TENSOR_INDEX[n]), w.nnz_of(n)) for n in SITE_AND_ENV}
    T = w.dense_tensors(vals)
    a, a_legs = u1.double_layer(T["A"], w.A_legs)
    return w, T, a, a_legs


@pytest.fixture(scope="module")
def tiny():
    return make(TINY, 7)


@pytest.fixture(scope="module")
def cfg1():
    return make(config(1), 1809)


# ---------------------------------------------------------------- blocks ---

def test_embed_roundtrip_and_zero_pattern():
    legs = [Leg({-1: 1, 1: 2}, IN), Leg({-2: 2, 0: 1, 2: 3}, IN), Leg({-1: 2, 1: 1, 3: 1}, OUT)]
    n = u1.nnz(legs, 0)
    vals = np.arange(1, n + 1, dtype=float)
    dense = u1.embed(legs, 0, vals)
    mask = u1.conserving_mask(legs, 0)
    # entries outside charge-conserving positions are exactly zero (Sec. 2:
    # symmetry-forbidden blocks are identically zero)
    assert np.all(dense[~mask] == 0.0)
    assert np.count_nonzero(dense) == n == mask.sum()
    # canonical order: blocks lexicographic in charges, row-major inside
    pos = 0
    for b in u1.allowed_blocks(legs, 0):
        blk = u1.extract_block(dense, legs, b)
        assert np.array_equal(blk.ravel(), vals[pos:pos + blk.size])
        pos += blk.size


def _gf_count(legs, flux, weighted):
    """Coefficient of x^flux in prod_l sum_s w_s x^(dir q_s): an independent
    count of allowed blocks (w=1) or allowed entries (w=dim)."""
    poly = {0: 1}
    for leg in legs:
        nxt = {}
        for e, c in poly.items():
            for q, d in zip(leg.charges, leg.dims):
                k = e + leg.dir * q
                nxt[k] = nxt.get(k, 0) + c * (d if weighted else 1)
        poly = nxt
    return poly.get(flux, 0)


@pytest.mark.parametrize("ci", [1, 2, 4])
def test_counts_match_generating_function(ci):
    c = config(ci)
    w = Workload(c["phys"], c["virt"], c["chi"], c["flux"])
    for name in ["A", "C1", "T1", "T2"]:
        legs, flux = w.legs_of(name)
        assert len(u1.allowed_blocks(legs, flux)) == _gf_count(legs, flux, False)
        assert u1.nnz(legs, flux) == _gf_count(legs, flux, True)
    assert u1.nnz(w.a_legs, 0) == _gf_count(w.a_legs, 0, True)


def test_cfg1_integer_table():
    c = config(1)
    w = Workload(c["phys"], c["virt"], c["chi"], c["flux"])
    dl = u1.double_layer_table(w)
    # A: 35 blocks / 126 entries; a: 85 blocks / 12870 entries; 617 outer
    # products (16^2 + 19^2 blocks with physical charge -1 / +1)
    assert (dl["A_blocks"], dl["A_nnz"]) == (35, 126)
    assert (len(dl["a"].blocks), dl["a"].nnz()) == (85, 12870)
    assert dl["n_pairs"] == 617 == 16 ** 2 + 19 ** 2
    assert w.dd == {-4: 1, -2: 4, 0: 6, 2: 4, 4: 1}
    assert len(u1.allowed_blocks(w.C_legs, 0)) == 3
    assert len(u1.allowed_blocks(w.T_legs["T1"], 0)) == 9 and u1.nnz(w.T_legs["T1"], 0) == 1120
    s1, s2, s3 = u1.corner_tables(w, 1)
    # C1.T1: chi-sector sums 2*sum_b chi_b^2 * sum_{u+x=b} dD(u) chi(x) = 14080
    assert (len(s1["pairs"]), len(s1["outputs"]), s1["flops"]) == (9, 9, 14080)
    assert (len(s2["pairs"]), len(s2["outputs"]), s2["flops"]) == (27, 27, 160000)
    # CTT.a: the intermediate CTT[u,x1,y,l] holds the 27 blocks reached from
    # C1.T1.T4 (u + x1 = y - l in {-2,0,2}); each pairs with the a blocks of
    # charge l+u = y-x1, of which there are 5-|y-x1|/2:  3*sum_{x1,y}(5-|y-x1|/2)
    closed = 3 * sum(5 - abs(y - x) // 2 for x in (-2, 0, 2) for y in (-2, 0, 2))
    assert closed == 111
    assert (len(s3["pairs"]), len(s3["outputs"])) == (111, 37)
    assert s3["out"].nnz() == 14784
    nL = u1.fused_sectors(w, "diff")
    assert nL == {-6: 4, -4: 24, -2: 60, 0: 80, 2: 60, 4: 24, 6: 4}
    assert sum(v * v for v in nL.values()) == 14784
    assert sum(v ** 3 for v in nL.values()) == 971776


def test_pair_table_reconstructs_dense_contraction(cfg1):
    """Summing the products of the matched block pairs gives the dense
    contraction of the embedded tensors (Sec. 2 contraction rule)."""
    w, T, a, _ = cfg1
    s1, s2, s3 = u1.corner_tables(w, 1)
    CT_dense = np.einsum("ab,bux->aux", T["C1"], T["T1"])
    C = u1.Struct.allowed(w.C_legs, 0)
    T1s = u1.Struct.allowed(w.T_legs["T1"], 0)
    out = np.zeros_like(CT_dense)
    out_legs = s1["out"].legs
    for ta, tb in s1["pairs"]:
        A = u1.extract_block(T["C1"], C.legs, ta)
        B = u1.extract_block(T["T1"], T1s.legs, tb)
        o = (ta[0], tb[1], tb[2])
        out[u1.block_slices(out_legs, o)] += np.tensordot(A, B, axes=([1], [0]))
    assert np.allclose(out, CT_dense, rtol=0, atol=1e-13)
    # and the step-3 output blocks cover every nonzero of the dense corner
    c1 = u1.enlarged_corners(w, T, a)[0]          # [x4, d, x1, r]
    c1p = c1.transpose(2, 0, 3, 1)                 # -> [x1, x4, r, d]
    covered = np.zeros(c1p.shape, bool)
    for o in s3["outputs"]:
        covered[u1.block_slices(s3["out"].legs, o)] = True
    assert np.all(c1p[~covered] == 0.0)
    assert np.count_nonzero(c1p[covered]) == covered.sum()


def test_single_sector_reduces_to_dense():
    """With one trivial charge sector on every leg, block-sparse work is the
    dense work 2 m n k."""
    legsA = [Leg({0: 5}, IN), Leg({0: 7}, OUT)]
    legsB = [Leg({0: 7}, IN), Leg({0: 3}, IN), Leg({0: 4}, OUT)]
    t = u1.pair_table(u1.Struct.allowed(legsA, 0), u1.Struct.allowed(legsB, 0), [1], [0])
    assert t["flops"] == 2 * 5 * 7 * 12 and len(t["pairs"]) == 1


# ----------------------------------------------------------- double layer ---

def test_double_layer_properties(cfg1):
    w, T, a, a_legs = cfg1
    A = T["A"]
    assert [leg.sectors() for leg in a_legs] == [w.dd] * 4
    # zero outside the fused charge rule (flux 0)
    assert np.all(a[~u1.conserving_mask(w.a_legs, 0)] == 0.0)
    # a = sum_s A A*: as a matrix (ket legs) x (bra legs) it is positive
    # semi-definite, and its trace over ket=bra is ||A||^2.  Undo the fusion
    # with the fuse permutation to get the (ket, bra) product index back.
    n = w.A_legs[1].size
    perms = [u1.fuse(leg, leg, +1, -1, leg.dir)[1] for leg in w.A_legs[1:]]
    a8 = np.zeros((n * n,) * 4)
    a8[np.ix_(*perms)] = a
    a8 = a8.reshape(n, n, n, n, n, n, n, n).transpose(0, 2, 4, 6, 1, 3, 5, 7).reshape(n ** 4, n ** 4)
    ev = np.linalg.eigvalsh(0.5 * (a8 + a8.T))
    assert ev.min() > -1e-12 * ev.max()
    assert np.isclose(np.trace(a8), np.sum(A * A), rtol=1e-13)


# ---------------------------------------------------------------- corners ---

def test_corners_match_explicit_loops(tiny):
    w, T, a, _ = tiny
    c1, c2, c3, c4 = u1.enlarged_corners(w, T, a)
    nX, nD = c1.shape[0], c1.shape[1]
    C1, C2, C3, C4 = T["C1"], T["C2"], T["C3"], T["C4"]
    T1, T2, T3, T4 = T["T1"], T["T2"], T["T3"], T["T4"]
    R = range
    b1 = np.zeros_like(c1)
    b2 = np.zeros_like(c2)
    b3 = np.zeros_like(c3)
    b4 = np.zeros_like(c4)
    for p, q, l, u in itertools.product(R(nX), R(nX), R(nD), R(nD)):
        for o1, o2, o3, o4 in itertools.product(R(nX), R(nD), R(nX), R(nD)):
            # C~1[x4,d,x1,r]: C1[p,q] T1[q,u,x1] T4[x4,l,p] a[l,u,r,d]
            b1[o1, o2, o3, o4] += C1[p, q] * T1[q, u, o3] * T4[o1, l, p] * a[l, u, o4, o2]
            # C~2[x1,l,x2,d]: C2[p,q] T1[x1,u,p] T2[q,r,x2] a[l,u,r,d]  (r -> l loop var)
            b2[o1, o2, o3, o4] += C2[p, q] * T1[o1, u, p] * T2[q, l, o3] * a[o2, u, l, o4]
            # C~3[x2,u,x3,l]: C3[p,q] T2[x2,r,p] T3[q,d,x3] a[l,u,r,d]  (r,d -> l,u)
            b3[o1, o2, o3, o4] += C3[p, q] * T2[o1, l, p] * T3[q, u, o3] * a[o4, o2, l, u]
            # C~4[x4,u,x3,r]: C4[p,q] T4[q,l,x4] T3[x3,d,p] a[l,u,r,d]  (d -> u)
            b4[o1, o2, o3, o4] += C4[p, q] * T4[q, l, o1] * T3[o3, u, p] * a[l, o2, o4, u]
    for x, y in [(c1, b1), (c2, b2), (c3, b3), (c4, b4)]:
        assert np.allclose(x, y, rtol=1e-13, atol=1e-13)


def _network_by_rows(T, a):
    """Value of the closed 4x4 network (two environment rows around two rows
    of double-layer sites), contracted row by row from the top."""
    def e(spec, *ops):
        return np.einsum(spec, *ops, optimize="optimal")
    top = e("ab,bux,xvc,ce->auve", T["C1"], T["T1"], T["T1"], T["C2"])
    m = e("auve,yla->uvely", top, T["T4"])
    m = e("uvely,lurd->velyrd", m, a)
    m = e("velyrd,rvsD->elydsD", m, a)
    m1 = e("elydsD,esz->ydDz", m, T["T2"])
    m = e("ydDz,Yly->dDzYl", m1, T["T4"])
    m = e("dDzYl,ldrp->DzYrp", m, a)
    m = e("DzYrp,rDsq->zYpsq", m, a)
    m2 = e("zYpsq,zsZ->YpqZ", m, T["T2"])
    bot = e("cY,xpc,Xqx,ZX->YpqZ", T["C4"], T["T3"], T["T3"], T["C3"])
    return float(np.sum(m2 * bot))


@pytest.mark.parametrize("which", ["tiny", "cfg1"])
def test_halves_reproduce_network_value(which, tiny, cfg1):
    """Tr(H_u H_d^T) equals the whole network contracted row by row: pins the
    wiring of all four corners, the fat-bond fusion and both halves."""
    w, T, a, _ = tiny if which == "tiny" else cfg1
    corners = u1.enlarged_corners(w, T, a)
    (M1, M2, M3, M4), Fd, Fs = u1.corner_matrices(w, corners)
    Hu, Hd = u1.halves(M1, M2, M3, M4)
    Z = _network_by_rows(T, a)
    assert np.isclose(np.sum(Hu * Hd), Z, rtol=1e-11)


def test_corner_matrices_block_diagonal(cfg1):
    w, T, a, _ = cfg1
    (M1, M2, M3, M4), Fd, Fs = u1.corner_matrices(w, u1.enlarged_corners(w, T, a))
    for M, Fr, Fc in [(M1, Fd, Fs), (M2, Fs, Fs), (M3, Fs, Fd), (M4, Fd, Fd)]:
        qr, qc = Fr.state_charges(), Fc.state_charges()
        off = qr[:, None] != qc[None, :]
        assert np.all(M[off] == 0.0)
        assert np.count_nonzero(M[~off]) > 0.99 * (~off).sum()
    # fused order: Q ascending, then chi charge ascending, then (i_chi, i_D)
    F, perm = u1.fuse(Leg(w.chi, IN), Leg(w.dd, IN), +1, -1, IN)
    nD = Leg(w.dd, IN).size
    qchi = Leg(w.chi, IN).state_charges()[perm // nD]
    qd = Leg(w.dd, IN).state_charges()[perm % nD]
    key = list(zip(qchi - qd, qchi, perm // nD, perm % nD))
    assert key == sorted(key)


# ------------------------------------------------------------- projectors ---

@pytest.fixture(scope="module")
def move1(cfg1):
    w, T, a, _ = cfg1
    return w, u1.ctm_left_move(w, T, a, 16)


def test_projector_identities(move1):
    w, mv = move1
    pr = mv["proj"]
    P, Pt = pr["P"], pr["Pt"]
    k = P.shape[1]
    assert k == 16 and sum(pr["kept"].values()) == 16
    assert np.allclose(Pt @ P, np.eye(k), atol=1e-9)
    Pi = P @ Pt
    assert np.allclose(Pi @ Pi, Pi, atol=1e-8 * np.abs(Pi).max())
    for Q, d in pr["per_Q"].items():
        # R_u (P P~) R_d^T = U_chi S_chi V_chi^T (kept part of the SVD)
        kq = pr["kept"].get(Q, 0)
        if kq == 0:
            continue
        Pq, Ptq = pr["blocks"][Q]
        lhs = d["Ru"] @ Pq @ Ptq @ d["Rd"].T
        rhs = d["U"][:, :kq] @ np.diag(d["s"][:kq]) @ d["V"][:, :kq].T
        assert np.allclose(lhs, rhs, atol=1e-10 * d["s"][0])
        # Eckart-Young: ||M - U S V^T||_F^2 = sum of discarded s^2
        assert np.isclose(np.linalg.norm(d["M"] - rhs) ** 2, np.sum(d["s"][kq:] ** 2),
                          rtol=1e-8, atol=1e-20 * d["s"][0] ** 2)
    # the SVD of the full block-diagonal M has the union of the block spectra
    nL = mv["F_left"]
    Mfull = np.zeros((nL.size, nL.size))
    off = nL.offsets()
    for Q, d in pr["per_Q"].items():
        Mfull[off[Q]:off[Q] + d["n"], off[Q]:off[Q] + d["n"]] = d["M"]
    s_full = np.linalg.svd(Mfull, compute_uv=False)
    s_union = np.sort(np.concatenate([d["s"] for d in pr["per_Q"].values()]))[::-1]
    assert np.allclose(s_full, s_union, rtol=1e-10, atol=1e-12 * s_full[0])
    # truncation error and global top-chi selection
    kept_s = np.sort(np.concatenate([pr["svals"][Q][:kq] for Q, kq in pr["kept"].items()]))
    assert np.allclose(kept_s, s_union[:16][::-1])
    assert np.isclose(pr["trunc_err"], np.sum(s_union[16:] ** 2) / np.sum(s_union ** 2))
    # sign gauge: largest-magnitude entry of every row of P~ is positive
    for r in Pt:
        assert r[np.argmax(np.abs(r))] > 0


def test_dense_qr_of_block_diagonal_is_block_diagonal(move1):
    w, mv = move1
    Hu = mv["Hu"]
    F = mv["F_left"]
    _, R = np.linalg.qr(Hu.T)
    q = F.state_charges()
    assert np.all(R[q[:, None] != q[None, :]] == 0.0)
    off = F.offsets()
    for Q, d in mv["proj"]["per_Q"].items():
        blk = R[off[Q]:off[Q] + d["n"], off[Q]:off[Q] + d["n"]]
        assert np.allclose(np.abs(blk), np.abs(d["Ru"]), atol=1e-10 * np.abs(blk).max())


def test_no_truncation_left_column(tiny):
    """Without truncation P P~ is the identity, and the renormalised left
    column equals the unprojected column C1 T1 . T4 a . C4 T3 up to the three
    normalisation factors."""
    w, T, a, _ = tiny
    mv = u1.ctm_left_move(w, T, a, 10 ** 6)
    n = mv["F_left"].size
    assert mv["Pi"].shape == (n, n)
    assert np.allclose(mv["Pi"], np.eye(n), atol=1e-8)
    L0 = np.einsum("ab,bux,yla,lurd,py,zdp->xrz", T["C1"], T["T1"], T["T4"], a, T["C4"], T["T3"],
                   optimize=True)
    n1, n2, n3 = mv["norms"]
    assert np.allclose(mv["L"] * n1 * n2 * n3, L0, rtol=1e-8, atol=1e-10 * np.abs(L0).max())
    for X in (mv["C1"], mv["T4"], mv["C4"]):
        assert np.isclose(np.linalg.norm(X), 1.0)


def test_new_leg_charges(move1):
    """Renormalised tensors obey the addition rule with the new leg's sectors."""
    w, mv = move1
    k = mv["proj"]["new_leg"]
    X = Leg(w.chi, IN)
    D = Leg(w.dd, IN)
    assert np.all(mv["C1"][~u1.conserving_mask([k, X.flipped()], 0)] == 0.0)
    assert np.all(mv["T4"][~u1.conserving_mask([k, D.flipped(), k.flipped()], 0)] == 0.0)
    assert np.all(mv["C4"][~u1.conserving_mask([X, k.flipped()], 0)] == 0.0)


def test_truncation_never_splits_a_degenerate_set():
    """Singular values 3, 2 (charge 0) and 2 (charge 1): chi = 2 would keep
    one of the equal pair, so only the 3 is kept; chi = 3 keeps all three; a
    pair split by 1e-6 (beyond the 1e-8 spread of a degenerate set) is cut
    as usual."""
    F = u1.Leg({0: 2, 1: 1}, u1.IN)

    def kept(s1, chi):
        return u1.projectors(np.eye(3), np.diag([3.0, 2.0, s1]), F, F, chi)["kept"]
    assert kept(2.0, 2) == {0: 1}
    assert kept(2.0, 3) == {0: 2, 1: 1}
    assert kept(2.0 * (1 - 1e-6), 2) == {0: 2}
    assert kept(2.0 * (1 - 1e-6), 1) == {0: 1}


# ------------------------------------------------------ move flop counts ---

def _sector_move_flops(chi, dd, kept):
    """Useful flops of the halves and of the renormalisation of one left
    move, summed over sector labels instead of enumerated block pairs.

    Charge rules (clockwise bonds): a left-cut state (x, u) has fused charge
    Q = q_x - q_u, so n_Q = sum_{x - u = Q} chi_x dd_u.  Each half multiplies
    two block-diagonal corner matrices whose three fat bonds all have sizes
    n_Q when the legs are symmetric under q -> -q: 2 sum_Q n_Q^3 per half.
    C1' = (C1 T1) P and C4' = (C4 T3) P~ each cost 2 sum_Q chi_Q k_Q n_Q.
    T4' = ((P~ T4) a) P in three steps:
      P~[K,c,e] T4[y,l,c]    K = c - e, y = l + c     m = k_K dd_e, k = chi_c, n = chi_y dd_l
      X1[K,e,y,l] a[l,e,r,d] l + e = r + d            m = k_K chi_y, k = dd_e dd_l, n = dd_r dd_d
      X2[K,y,r,d] P[y,d,K']  K' = y - d               m = k_K dd_r, k = chi_y dd_d, n = k_K'
    where X2 block (K, y, r, d) exists when some (l, e) with l + e = r + d,
    chi_{y-l} > 0 reaches it (then K = y - r - d).
    """
    g = lambda m, q: m.get(q, 0)
    nQ = {}
    for x, cx in chi.items():
        for u, du in dd.items():
            nQ[x - u] = nQ.get(x - u, 0) + cx * du
    assert all(nQ[q] == nQ.get(-q, 0) for q in nQ), "closed form needs symmetric legs"
    halves = 4 * sum(n ** 3 for n in nQ.values())
    c1 = c4 = 2 * sum(g(chi, Q) * k * g(nQ, Q) for Q, k in kept.items())
    x1 = 2 * sum(g(kept, c - e) * de * cc * g(chi, l + c) * dl
                 for c, cc in chi.items() for e, de in dd.items() for l, dl in dd.items())
    x2 = 0
    for y, cy in chi.items():
        for l, dl in dd.items():
            if not g(chi, y - l):
                continue
            for e, de in dd.items():
                K = y - l - e
                for r, dr in dd.items():
                    x2 += 2 * g(kept, K) * cy * de * dl * dr * g(dd, l + e - r)
    t4 = 0
    for y, cy in chi.items():
        for r, dr in dd.items():
            for d, dd_d in dd.items():
                reached = any(g(chi, y - l) and g(dd, r + d - l) for l in dd)
                if reached:
                    t4 += 2 * g(kept, y - r - d) * dr * cy * dd_d * g(kept, y - d)
    return halves, c1 + c4 + x1 + x2 + t4


@pytest.mark.parametrize("ci", [1, 2])
def test_move_flops_match_sector_sums(ci):
    """The oracle's halves and renormalisation flop counts (block-pair
    enumeration) equal sums over sector labels; cfg 1's halves are
    4 sum_Q n_Q^3 = 4 * 971776."""
    c = config(ci)
    w = Workload(c["phys"], c["virt"], c["chi"], c["flux"])
    nL = u1.fused_sectors(w, "diff")
    kept_tables = [{0: min(16, nL[0])}, {q: min(4, n) for q, n in nL.items() if abs(q) <= 2},
                   {-2: 3, 0: 7, 4: 1}]
    for kept in kept_tables:
        fl = u1.move_gemm_flops(w, kept)
        halves, renorm = _sector_move_flops(w.chi, w.dd, kept)
        assert fl["halves"] == halves
        assert fl["renorm"] == renorm
    if ci == 1:
        assert halves == 4 * 971776 == 3887104
