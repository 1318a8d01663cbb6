"""Pins of the whole-environment oracle: the dense move equals the pinned
U(1) oracle's move; the partition function per site is invariant under a
quarter turn of the network, exact on a product network, and (on a 2 x 2
patch) exact on a two-copy environment whose 1 x 1 estimate is provably
biased; the closed networks agree with independently written contractions;
the iteration with the error estimate of Sec. 3 follows its rules; and the
CTM reproduces the square-ice entropy (Lieb: W = (4/3)^(3/2) states per site;
a textbook result, not from the paper)."""
import numpy as np
import pytest

from oracle import ctm, u1
from synth import config
from workload import oracle_side

W_ICE = (4.0 / 3.0) ** 1.5


def test_dense_left_move_matches_u1_oracle():
    c = config(1)
    w, T, a, _ = oracle_side(c, c["seed"])
    mv = u1.ctm_left_move(w, T, a, c["chi_target"])
    C = [T["C1"], T["C2"], T["C3"], T["C4"]]
    Tt = [T["T1"], T["T2"], T["T3"], T["T4"]]
    C1n, T4n, C4n, s = ctm.left_move(C, Tt, a, c["chi_target"])
    L1 = u1.left_column(mv["C1"], mv["T4"], mv["C4"])
    L2 = u1.left_column(C1n, T4n, C4n)
    assert np.linalg.norm(L1 - L2) <= 1e-12 * np.linalg.norm(L1)
    ref = np.sort(np.concatenate(list(mv["proj"]["svals"].values())))[::-1]
    assert np.allclose(s, ref[:len(s)], rtol=0, atol=1e-13 * ref[0])


def test_site_partition_quarter_turn_and_product_network():
    rng = np.random.default_rng(0)
    C = [rng.standard_normal((3, 3)) for _ in range(4)]
    T = [rng.standard_normal((3, 2, 3)) for _ in range(4)]
    a = rng.standard_normal((2, 2, 2, 2))
    k0, z0 = ctm.site_partition(C, T, a)
    k1, z1 = ctm.site_partition(*ctm.rotate(C, T, a))
    assert np.isclose(k0, k1, rtol=1e-13)
    assert np.isclose(z0[0], z1[0]) and np.isclose(z0[3], z1[3])
    assert np.isclose(z0[1], z1[2]) and np.isclose(z0[2], z1[1])     # a row turns into a column
    # one-dimensional bonds: every Z is a product and kappa is the site weight
    c, t, al = 0.7, 1.9, 2.3
    k, _ = ctm.site_partition([np.full((1, 1), c)] * 4, [np.full((1, 1, 1), t)] * 4, np.full((1, 1, 1, 1), al))
    assert np.isclose(k, al, rtol=1e-14)


def _random_env(seed, chi=3, D=2):
    rng = np.random.default_rng(seed)
    C = [rng.standard_normal((chi, chi)) for _ in range(4)]
    T = [rng.standard_normal((chi, D, chi)) for _ in range(4)]
    return C, T, rng.standard_normal((D, D, D, D))


def test_closed_networks_match_hand_written_contractions():
    """z_block (the generated network contracted in list order) against the pairwise
    contractions of site_partition for n, m <= 1 and against explicitly
    spelled 2 x 1 and 2 x 2 networks."""
    C, T, a = _random_env(1)
    _, z = ctm.site_partition(C, T, a)
    for (n, m), ref in zip(((0, 0), (1, 0), (0, 1), (1, 1)), z):
        assert np.isclose(ctm.z_block(C, T, a, n, m), ref, rtol=1e-12)
    C1, C2, C3, C4 = C
    T1, T2, T3, T4 = T
    # top: C1 T1 T1 C2; right: T2 T2; C3; bottom: T3 T3 (right to left); C4; left: T4 T4 (bottom to top)
    z22 = np.einsum("ab,buc,cwd,de,erf,fsg,gh,hti,iyj,jk,kLm,mla,lupv,pwrq,Lvxy,xqst->",
                    C1, T1, T1, C2, T2, T2, C3, T3, T3, C4, T4, T4, a, a, a, a, optimize="greedy")
    z21 = np.einsum("ab,buc,cwd,de,erf,fg,gqi,ivj,jk,kla,lupv,pwrq->",
                    C1, T1, T1, C2, T2, C3, T3, T3, C4, T4, a, a, optimize="greedy")
    assert np.isclose(ctm.z_block(C, T, a, 2, 2), z22, rtol=1e-12)
    assert np.isclose(ctm.z_block(C, T, a, 2, 1), z21, rtol=1e-12)


def test_closed_networks_quarter_turn():
    """Turning the network a quarter turn exchanges columns and rows."""
    C, T, a = _random_env(2)
    Cr, Tr, ar = ctm.rotate(C, T, a)
    for n in range(3):
        for m in range(3):
            assert np.isclose(ctm.z_block(Cr, Tr, ar, n, m), ctm.z_block(C, T, a, m, n), rtol=1e-12)


def test_block_estimator_product_network():
    c, t, al = 0.7, 1.9, 2.3
    Cs, Ts, a = [np.full((1, 1), c)] * 4, [np.full((1, 1, 1), t)] * 4, np.full((1, 1, 1, 1), al)
    for b in (1, 2):
        k, z = ctm.site_partition_block(Cs, Ts, a, b)
        assert np.isclose(k, al, rtol=1e-14)
        assert np.isclose(z[3], c ** 4 * t ** (4 * b) * al ** (b * b), rtol=1e-14)


def test_block_estimator_two_parity_copies():
    """A bond of two states (charge parities 0, 1), corners diagonal with
    unequal weights c_i = (1, r_i), every edge tensor moving parity p to 1 - p
    with weight t, one-state site tensor alpha.  Then
    Z_nm = t^(2n+2m) alpha^(nm) sum_p c1_p c2_(p+n) c3_(p+n+m) c4_(p+m): the
    1 x 1 ratio is alpha times a corner factor that is not 1, the 2 x 2 ratio
    is exactly alpha^4."""
    r = [1.0, 1.7, 0.6, 2.2, 0.9]
    c = [None] + [np.array([1.0, r[i]]) for i in range(1, 5)]
    t, al = 1.3, 1.45
    Cs = [np.diag(c[i]) for i in range(1, 5)]
    Te = np.zeros((2, 1, 2))
    Te[0, 0, 1] = Te[1, 0, 0] = t
    a = np.full((1, 1, 1, 1), al)
    Ts = [Te] * 4

    def zf(n, m):
        return t ** (2 * n + 2 * m) * al ** (n * m) * sum(
            c[1][p] * c[2][(p + n) % 2] * c[3][(p + n + m) % 2] * c[4][(p + m) % 2] for p in (0, 1))
    for n in range(3):
        for m in range(3):
            assert np.isclose(ctm.z_block(Cs, Ts, a, n, m), zf(n, m), rtol=1e-13)
    k1, _ = ctm.site_partition_block(Cs, Ts, a, 1)
    bias = zf(1, 1) * zf(0, 0) / (zf(1, 0) * zf(0, 1)) / al
    assert abs(bias - 1.0) > 0.05
    assert np.isclose(k1, al * bias, rtol=1e-13)
    k2, _ = ctm.site_partition_block(Cs, Ts, a, 2)
    assert np.isclose(k2, al, rtol=1e-13)


def test_run_follows_the_error_rules():
    """On a product network every step leaves kappa unchanged, so each chi
    stops after one step, the second chi agrees with the first and the run
    ends there; with max_steps = 2 and tol = 0 on a random network, two steps
    at each of the chis 4, 8 (chi_max 15 stops the doubling) and the errors
    are the changes between the recorded values."""
    c, t, al = 0.7, 1.9, 2.3
    Cs, Ts, a = [np.full((1, 1), c)] * 4, [np.full((1, 1, 1), t)] * 4, np.full((1, 1, 1, 1), al)
    _, _, r = ctm.run(Cs, Ts, a, 2, chi_max=128, block=2, max_steps=15, tol=1e-8)
    assert (r["steps"], r["levels"], r["total_steps"], r["chi"]) == (1, 2, 2, 4)
    assert np.isclose(r["kappa"], al) and r["error"] < 1e-12
    C, T, ad = _random_env(3, chi=4)
    vals = []
    Ck, Tk = C, T
    for chi in (4, 8):
        vals.append([ctm.site_partition_block(Ck, Tk, ad, 1)[0]])
        for _ in range(2):
            for d in range(4):
                Ck, Tk, _ = ctm.move(Ck, Tk, ad, chi, d)
            vals[-1].append(ctm.site_partition_block(Ck, Tk, ad, 1)[0])
    _, _, r = ctm.run(C, T, ad, 4, chi_max=15, block=1, max_steps=2, tol=0.0)
    assert (r["steps"], r["levels"], r["total_steps"], r["chi"]) == (2, 2, 4, 8)
    h = vals[1]
    assert r["kappa"] == h[-1]
    assert r["err_steps"] == max(abs(h[1] - h[0]), abs(h[2] - h[1]))
    assert r["err_chi"] == abs(vals[1][-1] - vals[0][-1])
    assert r["error"] == max(r["err_steps"], r["err_chi"])


@pytest.mark.parametrize("block", [1, 2])
def test_square_ice_entropy(block):
    a = ctm.vertex_tensor(ctm.ice_weights())
    assert np.count_nonzero(a) == 6
    C, T = ctm.initial_environment()
    _, _, r = ctm.run(C, T, a, 8, block=block, max_steps=300, tol=1e-9)
    assert abs(r["kappa"] - W_ICE) <= 1e-3 * W_ICE


# ------------------------------------------------ expectation values (Sec. 3)
def _u1_state(seed, virt={-1: 1, 0: 1, 1: 1}):
    """A random U(1) site tensor A[phys, l, u, r, d] with spin-1/2 physical
    states, dense embedding (flux +1)."""
    legs = [u1.Leg({-1: 1, 1: 1}, u1.IN)] + [u1.Leg(virt, d) for d in (u1.IN, u1.IN, u1.OUT, u1.OUT)]
    rng = np.random.default_rng(seed)
    A = rng.standard_normal([l.size for l in legs]) * u1.conserving_mask(legs, 1)
    return A, legs


def test_operator_double_layer_pins():
    """Identity between the layers gives the double layer; the trace over
    every (ket, bra) pair is sum op[t, k] <A_k, A_t> (the Gram matrix of the
    physical slices); an operator that raises the charge by 2 gives a tensor
    whose non-zero entries all carry fused flux +2."""
    A, legs = _u1_state(5)
    a, a_legs = u1.double_layer(A, legs)
    sz, sp, sm = u1.spin_operators(legs[0])
    assert np.allclose(sz, np.diag([-0.5, 0.5])) and np.allclose(sp, [[0, 0], [1, 0]]) and np.allclose(sm, sp.T)
    assert np.allclose(u1.double_layer_op(A, legs, np.eye(2)), a, rtol=0, atol=1e-14)
    G = np.einsum("kabcd,tabcd->kt", A, A)
    rng = np.random.default_rng(6)
    op = rng.standard_normal((2, 2))
    b = u1.double_layer_op(A, legs, op)
    n = [l.size for l in legs[1:]]
    perms = [u1.fuse(l, l, +1, -1, l.dir)[1] for l in legs[1:]]
    b8 = np.zeros([x * x for x in n])
    b8[np.ix_(*perms)] = b
    b8 = b8.reshape(n[0], n[0], n[1], n[1], n[2], n[2], n[3], n[3])
    assert np.isclose(np.einsum("aabbccdd->", b8), np.sum(op * G.T), rtol=1e-13)
    bp = u1.double_layer_op(A, legs, sp)
    assert np.count_nonzero(bp) > 0
    assert np.all(bp[~u1.conserving_mask(a_legs, 2)] == 0)


def test_heisenberg_ferromagnet_product_state():
    """D = 1 with every spin up (or down): the product state is exact with the
    trivial environment and <S_i . S_j> = 1/4 on both bonds."""
    for q in (1, -1):
        legs = [u1.Leg({-1: 1, 1: 1}, u1.IN)] + [u1.Leg({0: 1}, d) for d in (u1.IN, u1.IN, u1.OUT, u1.OUT)]
        A = np.zeros((2, 1, 1, 1, 1))
        A[(q + 1) // 2] = 1.7
        C, T = [np.ones((1, 1))] * 4, [np.ones((1, 1, 1))] * 4
        eh, ev = ctm.heisenberg_bond_energy(C, T, A, legs)
        assert np.isclose(eh, 0.25, rtol=1e-14) and np.isclose(ev, 0.25, rtol=1e-14)


def test_heisenberg_su2_invariant_state():
    """An SU(2)-invariant site tensor (from the SU(2) oracle, expanded to
    S^z states) in the traced open boundary: the two-site reduced state is a
    singlet-triplet mixture, so <S+ S-> + <S- S+> = 4 <Sz Sz> on each bond,
    <Sz> = 0 on a site, and the bond energy is 3 <Sz Sz>."""
    from oracle import su2
    v = {0: 1, 1: 1}
    sl = [su2.Leg({1: 1}, su2.IN)] + [su2.Leg(v, d) for d in (su2.IN, su2.IN, su2.OUT, su2.OUT)]
    vals = np.random.default_rng(7).standard_normal(su2.nnz(sl))
    A, legs = su2.to_u1(su2.expand(sl, vals), sl)
    a, a_legs = u1.double_layer(A, legs)
    C, T = _identity_env_from(legs)
    sz, sp, sm = u1.spin_operators(legs[0])
    bz, bp, bm = (u1.double_layer_op(A, legs, o) for o in (sz, sp, sm))
    assert abs(ctm.expectation(C, T, a, [bz], 1, 1)) < 1e-13
    for n, m in ((2, 1), (1, 2)):
        zz = ctm.expectation(C, T, a, [bz, bz], n, m)
        pm = ctm.expectation(C, T, a, [bp, bm], n, m) + ctm.expectation(C, T, a, [bm, bp], n, m)
        assert abs(zz) > 1e-3
        assert np.isclose(pm, 4 * zz, rtol=1e-11)
    eh, ev = ctm.heisenberg_bond_energy(C, T, A, legs)
    assert np.isclose(eh, 3 * ctm.expectation(C, T, a, [bz, bz], 2, 1), rtol=1e-11)
    assert np.isclose(ev, 3 * ctm.expectation(C, T, a, [bz, bz], 1, 2), rtol=1e-11)


def _identity_env_from(A_legs):
    """chi = 1 environment pairing ket and bra states on every D^2 leg (the
    traced open boundary), in the fused order of the double layer."""
    Ts = []
    # T1 meets a's up leg, T2 the right, T3 the down, T4 the left leg
    for l in (A_legs[2], A_legs[3], A_legs[4], A_legs[1]):
        F, perm = u1.fuse(l, l, +1, -1, l.dir)
        n = l.size
        t = np.zeros((1, F.size, 1))
        t[0, [f for f, p in enumerate(perm) if p // n == p % n], 0] = 1.0
        Ts.append(t)
    return [np.ones((1, 1))] * 4, Ts


def test_expectation_sums_over_a_decomposition():
    """a = sum of the six square-ice vertices: the one-site expectations of
    the single vertices add up to 1 in a converged environment, and the
    two-site ones over all 36 pairs too."""
    w = ctm.ice_weights()
    a = ctm.vertex_tensor(w)
    C, T = ctm.initial_environment()
    C, T, _ = ctm.run(C, T, a, 8, block=2, max_steps=40, tol=1e-9)
    parts = [ctm.vertex_tensor({k: 1.0}) for k in w]
    assert np.isclose(sum(ctm.expectation(C, T, a, [p], 1, 1) for p in parts), 1.0, rtol=1e-12)
    assert np.isclose(sum(ctm.expectation(C, T, a, [p, q], 2, 1) for p in parts for q in parts), 1.0, rtol=1e-12)


# ------------------------------------------------ Z2 charges and the Ising model
def test_z2_mask_and_fusion_counts():
    """Parity conservation: with legs {0: d0, 1: d1} the number of allowed
    entries is ((d0 + d1)^R + s (d0 - d1)^R) / 2 (s = +1 for flux 0, -1 for
    flux 1: the parity generating function); fusing two such legs gives
    sectors {0: a0 b0 + a1 b1, 1: a0 b1 + a1 b0}."""
    d0, d1 = 2, 3
    for R in (2, 3, 4):
        legs = [u1.Leg({0: d0, 1: d1}, (+1, -1)[k % 2]) for k in range(R)]
        for flux, sgn in ((0, 1), (1, -1)):
            n = int(np.count_nonzero(u1.conserving_mask(legs, flux, modulus=2)))
            assert n == ((d0 + d1) ** R + sgn * (d0 - d1) ** R) // 2
    F, perm = u1.fuse(u1.Leg({0: 2, 1: 3}, u1.IN), u1.Leg({0: 4, 1: 1}, u1.IN), +1, -1, u1.IN, modulus=2)
    assert F.sectors() == {0: 2 * 4 + 3 * 1, 1: 2 * 1 + 3 * 4}
    assert sorted(perm) == list(range(25))


def test_onsager_formula_limits():
    """beta -> 0: ln 2; small beta: the high-temperature expansion
    ln 2 + 2 ln cosh(beta) + tanh(beta)^4 + O(tanh^6)."""
    assert np.isclose(ctm.onsager_log_z(0.0), np.log(2.0), rtol=0, atol=1e-15)
    b = 0.05
    ht = np.log(2.0) + 2 * np.log(np.cosh(b)) + np.tanh(b) ** 4
    assert abs(ctm.onsager_log_z(b) - ht) < 5 * np.tanh(b) ** 6
    # n-independence away from the critical point
    assert abs(ctm.onsager_log_z(0.3, 256) - ctm.onsager_log_z(0.3, 512)) < 1e-14


def test_ising_tensor_pins():
    """Parity conservation of the site tensor, and a 1 x 1 torus: the 2 x 2
    spin sum of exp(beta s s') over the bonds of one site with itself, i.e.
    sum_s exp(2 beta) = 2 exp(2 beta), equals the trace of a over (l, r) and
    (u, d)."""
    beta = 0.37
    a = ctm.ising_tensor(beta)
    legs = [u1.Leg({0: 1, 1: 1}, d) for d in (u1.IN, u1.IN, u1.OUT, u1.OUT)]
    assert np.all(a[~u1.conserving_mask(legs, 0, modulus=2)] == 0)
    assert np.isclose(np.einsum("abab->", a), 2 * np.exp(2 * beta), rtol=1e-14)


@pytest.mark.parametrize("beta", [0.3, 0.6])
def test_ising_free_energy(beta):
    """The dense CTM on the Ising tensor reproduces Onsager's ln Z per site
    away from the critical point (beta_c = 0.4407)."""
    a = ctm.ising_tensor(beta)
    C, T = ctm.ising_initial_environment()
    _, _, r = ctm.run(C, T, a, 16, block=1, max_steps=100, tol=1e-13)
    assert abs(np.log(r["kappa"]) - ctm.onsager_log_z(beta)) < 1e-9


# ------------------------------------------------ unit cells
def test_cell_of_one_site_is_the_1x1_move():
    c = config(1)
    w, T, a, _ = oracle_side(c, c["seed"])
    C0 = [T["C1"], T["C2"], T["C3"], T["C4"]]
    T0 = [T["T1"], T["T2"], T["T3"], T["T4"]]
    for d in range(4):
        Co, To, s = ctm.move(C0, T0, a, 16, d)
        cell, sv = ctm.cell_move([[(C0, T0)]], [[a]], 16, d)
        Cc, Tc = cell[0][0]
        i, j = d, (d + 3) % 4
        L1, L2 = u1.left_column(Co[i], To[j], Co[j]), u1.left_column(Cc[i], Tc[j], Cc[j])
        assert np.linalg.norm(L1 - L2) <= 1e-12 * np.linalg.norm(L1)
        assert np.allclose(sv[0], s, rtol=0, atol=1e-13 * s[0])


def test_uniform_2x2_cell_left_move_is_sequential():
    """Four copies of one site and its environment.  The columns are moved one
    after the other: column 1 absorbs column 0 (one 1 x 1 left move), then
    column 0 absorbs the updated column 1 (two 1 x 1 left moves); the rows of
    each column stay equal, and every cut's spectrum is the 1 x 1 one of the
    same step."""
    c = config(1)
    w, T, a, _ = oracle_side(c, c["seed"])
    C, Tt = [T["C1"], T["C2"], T["C3"], T["C4"]], [T["T1"], T["T2"], T["T3"], T["T4"]]
    cell = [[(C, Tt), (C, Tt)], [(C, Tt), (C, Tt)]]
    cell, sv = ctm.cell_move(cell, [[a, a], [a, a]], 12, 0)
    C1, T1, s1 = ctm.move(C, Tt, a, 12, 0)
    C2, T2, s2 = ctm.move(C1, T1, a, 12, 0)
    col = lambda Cs, Ts: u1.left_column(Cs[0], Ts[3], Cs[3])
    for x, (Cr, Tr) in ((1, (C1, T1)), (0, (C2, T2))):
        for y in range(2):
            L = col(*cell[x][y])
            assert np.linalg.norm(L - col(Cr, Tr)) <= 1e-11 * np.linalg.norm(L)
    for v, ref in zip(sv, [s1, s1, s2, s2]):
        assert np.allclose(v, ref, rtol=0, atol=1e-12 * ref[0])


def test_cell_rotation_four_turns_is_identity():
    rng = np.random.default_rng(4)
    cell = [[([rng.standard_normal((2, 2)) for _ in range(4)], [rng.standard_normal((2, 3, 2)) for _ in range(4)])
             for _ in range(3)] for _ in range(2)]
    A = [[rng.standard_normal((3, 3, 3, 3)) for _ in range(3)] for _ in range(2)]
    c2, a2 = cell, A
    for _ in range(4):
        c2, a2 = ctm.cell_rotate(c2, a2)
    for x in range(2):
        for y in range(3):
            assert np.array_equal(a2[x][y], A[x][y])
            for u, v in zip(c2[x][y][0] + c2[x][y][1], cell[x][y][0] + cell[x][y][1]):
                assert np.array_equal(u, v)
    c1, a1 = ctm.cell_rotate(cell, A)
    assert len(c1) == 3 and len(c1[0]) == 2                       # Lx' = Ly, Ly' = Lx
    assert np.array_equal(a1[0][1], A[0][0].transpose(1, 2, 3, 0))   # top-left goes to bottom-left


@pytest.mark.parametrize("beta", [0.3, 0.38])
def test_ising_cell_from_unequal_starts(beta):
    """The Ising model (disordered phase, beta < beta_c = 0.4407, where the
    fixed point is unique) on a 2 x 2 cell whose four sites start from
    different environments (chi = 2, positive random entries on the allowed
    parity blocks): every site's environment converges to the fixed point
    and reproduces Onsager's ln Z per site."""
    a = ctm.ising_tensor(beta)
    rng = np.random.default_rng(8)
    par = np.array([0, 1])

    def env():
        C = [np.diag(rng.uniform(0.5, 1.5, 2)) for _ in range(4)]
        T = []
        for _ in range(4):
            t = rng.uniform(0.5, 1.5, (2, 2, 2))
            t[(par[:, None, None] + par[None, :, None] + par[None, None, :]) % 2 == 1] = 0.0
            T.append(t)
        return C, T
    cell = [[env() for _ in range(2)] for _ in range(2)]
    A = [[a, a], [a, a]]
    for _ in range(40):
        for d in range(4):
            cell, _ = ctm.cell_move(cell, A, 12, d)
    for x in range(2):
        for y in range(2):
            k, _ = ctm.site_partition(*cell[x][y], a)
            assert abs(np.log(k) - ctm.onsager_log_z(beta)) < 1e-8
