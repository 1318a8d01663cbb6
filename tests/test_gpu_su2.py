"""GPU parity of the SU(2) reduced path: reduced contractions, the enlarged
corner and the S^z expansion, against the oracle's CG expansion (dense
contraction of expanded tensors, reduced again), and at the full workload
size against the U(1) path run on the expanded inputs."""
import numpy as np
import pytest

import paper_1808_10804_amd as st
from oracle import su2
from synth import config, draw
from workload import rel, to_dense
from workload_su2 import IN, OUT, corner_legs, su2_values, device, dense, reduced_full

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16x3": 1e-5}

# sizes chosen so that several output blocks span more than one GEMM tile and
# the concatenated K of the recoupling terms ends on a ragged tail
CASES = [
    ([({0: 9, 1: 12, 2: 5}, IN), ({1: 11, 2: 7}, IN), ({0: 6, 1: 10, 2: 4}, OUT)],
     [({0: 6, 1: 10, 2: 4}, IN), ({1: 7, 3: 3}, OUT), ({0: 8, 2: 5}, OUT)], [2], [0], [0, 1, 2, 3]),
    ([({0: 9, 1: 12, 2: 5}, IN), ({1: 11, 2: 7}, IN), ({0: 6, 1: 10, 2: 4}, OUT)],
     [({0: 6, 1: 10, 2: 4}, IN), ({1: 7, 3: 3}, OUT), ({0: 8, 2: 5}, OUT)], [2], [0], [3, 1, 0, 2]),
    ([({1: 7, 3: 2}, IN), ({0: 5, 2: 6}, IN), ({1: 6, 2: 3}, OUT), ({0: 4, 1: 5}, OUT)],
     [({1: 6, 2: 3}, IN), ({0: 4, 1: 5}, IN), ({1: 9, 2: 4}, OUT)], [2, 3], [0, 1], [2, 0, 1]),
]


def _case(i, seed):
    specA, specB, conA, conB, perm = CASES[i]
    LA = [su2.Leg(s, d) for s, d in specA]
    LB = [su2.Leg(s, d) for s, d in specB]
    va = draw((seed, i, 0), su2.nnz(LA))
    vb = draw((seed, i, 1), su2.nnz(LB))
    return specA, specB, conA, conB, perm, LA, LB, va, vb


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("i", range(len(CASES)))
def test_su2_contraction_parity(i, prec):
    specA, specB, conA, conB, perm, LA, LB, va, vb = _case(i, 1811)
    dt = "f64" if prec == "f64" else "f32"
    A = st.Tensor.create(specA, dtype=dt, group="su2").upload(va)
    B = st.Tensor.create(specB, dtype=dt, group="su2").upload(vb)
    print(f"su2 contraction case {i} {prec}", flush=True)
    O = st.contract(A, B, conA, conB, out_perm=perm, prec=prec)
    got, Lo = reduced_full(O)
    tc = np.tensordot(su2.expand(LA, va), su2.expand(LB, vb), axes=(conA, conB)).transpose(perm)
    ref = su2.reduce(Lo, tc)
    err = rel(got, ref)
    print(f"  rel err {err:.3e}")
    assert err <= TOL[prec]
    # the reduced result reproduces the whole dense product
    assert rel(su2.expand(Lo, got), tc) <= max(TOL[prec], 1e-12)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_su2_to_u1_parity(dt):
    specA = CASES[2][0]
    LA = [su2.Leg(s, d) for s, d in specA]
    va = draw((1811, 9, 0), su2.nnz(LA))
    A = st.Tensor.create(specA, dtype=dt, group="su2").upload(va)
    U = A.to_u1()
    ref, ulegs = su2.to_u1(su2.expand(LA, va), LA)
    assert [l.sectors() for l in ulegs] == [s for s, _ in U.legs()]
    got = to_dense(U, ulegs)
    assert rel(got, ref) <= (1e-15 if dt == "f64" else 1e-7)


SMALL = dict(chi={0: 3, 1: 4, 2: 2}, dd={0: 2, 1: 3, 2: 2})


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_su2_corner_small_vs_oracle(prec):
    """C~1 = ((C1 T1) T4) a in reduced form against the dense corner of the
    expanded tensors."""
    legs = corner_legs(SMALL["chi"], SMALL["dd"])
    vals = su2_values(legs, 1811)
    dt = "f64" if prec == "f64" else "f32"
    dev = device(legs, vals, dt)
    Cn, info = st.enlarged_corner(1, dev["C1"], dev["T1"], dev["T4"], dev["a"], prec=prec)
    got, Lo = reduced_full(Cn)
    D = dense(legs, vals)
    e = lambda s, *o: np.einsum(s, *o, optimize="optimal")
    ct = e("ab,bux->aux", D["C1"], D["T1"])
    ctt = e("aux,yla->xylu", ct, D["T4"])
    corner = e("xylu,lurd->xyrd", ctt, D["a"])     # legs [x1, x4, r, d]
    assert [l.tjs for l in Lo] == [sorted(SMALL["chi"]), sorted(SMALL["chi"]), sorted(SMALL["dd"]),
                                   sorted(SMALL["dd"])]
    ref = su2.reduce(Lo, corner)
    err = rel(got, ref)
    print(f"su2 small corner {prec}: rel err {err:.3e}")
    assert err <= TOL[prec]


def test_cfg3_corner_reduced_vs_u1_expanded():
    """Full SU(2) workload: the reduced corner, expanded to S^z components,
    equals the U(1) corner computed from the expanded inputs (both FP32)."""
    c = config(3)
    legs = corner_legs(c["chi"], c["dd"])
    vals = su2_values(legs, c["seed"])
    dev = device(legs, vals, "f32")
    print("cfg3 su2 corner", flush=True)
    Cn, info = st.enlarged_corner(1, dev["C1"], dev["T1"], dev["T4"], dev["a"], prec="f32")
    U = {n: t.to_u1() for n, t in dev.items()}
    print("cfg3 u1-expanded corner", flush=True)
    Cu, info_u = st.enlarged_corner(1, U["C1"], U["T1"], U["T4"], U["a"], prec="f32")
    Ce = Cn.to_u1()
    bu, be = Cu.block_dict(), Ce.block_dict()
    num = den = 0.0
    for lab, x in be.items():
        y = bu.get(lab)
        if y is None:
            num += float(np.sum(x.astype(np.float64) ** 2))
            continue
        num += float(np.sum((x - y) ** 2))
        den += float(np.sum(y ** 2))
    for lab, y in bu.items():
        if lab not in be:
            num += float(np.sum(y ** 2))
            den += float(np.sum(y ** 2))
    err = (num / den) ** 0.5
    print(f"cfg3: reduced {info['useful_flops']:.3e} flops, expanded {info_u['useful_flops']:.3e}; rel diff {err:.3e}")
    assert err <= 1e-5
    assert info["useful_flops"] < info_u["useful_flops"]


def test_cfg3_expansion_of_inputs_vs_oracle():
    """The library's S^z expansion of the full-size C1 and T1 against the
    oracle's (the U(1) comparison above relies on it)."""
    c = config(3)
    legs = corner_legs(c["chi"], c["dd"])
    vals = su2_values(legs, c["seed"])
    dev = device({k: legs[k] for k in ("C1", "T1")}, vals, "f64")
    for n in ("C1", "T1"):
        L = [su2.Leg(s, d) for s, d in legs[n]]
        ref, ulegs = su2.to_u1(su2.expand(L, vals[n]), L)
        assert rel(to_dense(dev[n].to_u1(), ulegs), ref) <= 1e-15


# ---------------------------------------------------------------- SU(2) move
def _env_legs(chi, dd):
    L = corner_legs(chi, dd)
    for n in ("C2", "C3", "C4"):
        L[n] = [(chi, IN), (chi, OUT)]
    L["T2"] = [(chi, IN), (dd, IN), (chi, OUT)]
    L["T3"] = [(chi, IN), (dd, IN), (chi, OUT)]
    return L


def _su2_env(legs, vals, dt):
    dev = device(legs, vals, dt)
    env = st.CtmEnv([dev[k] for k in ("C1", "C2", "C3", "C4")], [dev[k] for k in ("T1", "T2", "T3", "T4")])
    return env, dev


def _expanded_u1(legs, vals):
    """Dense S^z-ordered arrays of the SU(2) tensors and the U(1) sector lists
    of their chi and D^2 legs (oracle expansion)."""
    out = {}
    for n, spec in legs.items():
        L = [su2.Leg(s, d) for s, d in spec]
        out[n], _ = su2.to_u1(su2.expand(L, vals[n]), L)
    chi_u1 = su2.Leg(legs["C1"][0][0], IN).u1_leg().sectors()
    dd_u1 = su2.Leg(legs["a"][0][0], IN).u1_leg().sectors()
    return out, chi_u1, dd_u1


def _dense_u1(t):
    """Device SU(2) tensor -> dense array in the S^z state order (oracle expansion)."""
    v, L = reduced_full(t)
    d, _ = su2.to_u1(su2.expand(L, v), L)
    return d


def _spectrum_states(sv, stats):
    """Reduced singular values repeated 2J+1 times, descending."""
    out, pos = [], 0
    for tj, n in sorted(stats["sv_sectors"].items()):
        out += list(np.repeat(sv[pos:pos + n], tj + 1))
        pos += n
    return np.sort(np.array(out))[::-1]


SMALL_MOVE = dict(chi={0: 2, 1: 2, 2: 1}, dd={0: 2, 1: 2, 2: 1}, chi_target=7)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_su2_move_small_vs_oracle(prec):
    """SU(2) left move against the oracle's U(1) move on the CG-expanded
    tensors, truncated to the same number of states: spectrum (each reduced
    value 2J+1 times), the projector P P~ on the cut, and the gauge-invariant
    left column."""
    from types import SimpleNamespace
    from oracle import u1
    legs = _env_legs(SMALL_MOVE["chi"], SMALL_MOVE["dd"])
    vals = su2_values(legs, 1811)
    dt = "f64" if prec == "f64" else "f32"
    env, dev = _su2_env(legs, vals, dt)
    print(f"su2 small move {prec}", flush=True)
    stats = env.move(dev["a"], SMALL_MOVE["chi_target"], prec=prec)
    kept_states = sum((tj + 1) * k for tj, k in stats["kept"].items())
    assert 0 < kept_states <= SMALL_MOVE["chi_target"]
    D, chi_u1, dd_u1 = _expanded_u1(legs, vals)
    w = SimpleNamespace(chi=chi_u1, dd=dd_u1)
    mv = u1.ctm_left_move(w, D, D["a"], kept_states)
    assert sum(mv["proj"]["kept"].values()) == kept_states
    tol = 1e-12 if prec == "f64" else 1e-5
    # spectrum
    ref = np.sort(np.concatenate([s for _, s in sorted(mv["proj"]["svals"].items())]))[::-1]
    got = _spectrum_states(env.singular_values(), stats)
    n = min(len(got), len(ref))
    assert np.max(np.abs(got[:n] - ref[:n])) <= tol * ref[0]
    # projector on the cut, in the oracle's fused (chi, D^2) order
    P, Pt = env.projectors()
    Pd, Ptd = _dense_u1(P), _dense_u1(Pt)
    nX, nD = Pd.shape[0], Pd.shape[1]
    Pi = np.einsum("xdk,kye->xdye", Pd, Ptd).reshape(nX * nD, nX * nD)
    _, perm = u1._fat(w, "diff")
    err_pi = rel(Pi[np.ix_(perm, perm)], mv["Pi"])
    # left column
    Lg = u1.left_column(_dense_u1(env.get(0)), _dense_u1(env.get(7)), _dense_u1(env.get(3)))
    err_l = rel(Lg, mv["L"])
    print(f"  kept states {kept_states}, Pi rel err {err_pi:.3e}, left column rel err {err_l:.3e}")
    assert err_pi <= tol and err_l <= tol


def test_cfg3_move_reduced_vs_u1_expanded():
    """Full SU(2) workload (FP32): the reduced move against the FP64 U(1) move
    (the path pinned against the oracle at cfgs 1 and 2) on the library's S^z
    expansion of the same tensors, truncated to the same number of states:
    spectra and the gauge-invariant left column, within the FP32 tolerance."""
    from oracle import u1
    c = config(3)
    legs = _env_legs(c["chi"], c["dd"])
    vals = su2_values(legs, c["seed"])
    env, dev = _su2_env(legs, vals, "f32")
    print("cfg3 su2 move", flush=True)
    stats = env.move(dev["a"], c["chi_target"], prec="f32")
    kept_states = sum((tj + 1) * k for tj, k in stats["kept"].items())
    assert 0 < kept_states <= c["chi_target"]
    _, dev64 = _su2_env(legs, vals, "f64")
    U = {n: t.to_u1() for n, t in dev64.items()}
    envu = st.CtmEnv([U[k] for k in ("C1", "C2", "C3", "C4")], [U[k] for k in ("T1", "T2", "T3", "T4")])
    print("cfg3 u1-expanded move (FP64)", flush=True)
    stu = envu.move(U["a"], kept_states, prec="f64")
    assert sum(stu["kept"].values()) == kept_states
    got = _spectrum_states(env.singular_values(), stats)
    ref = np.sort(envu.singular_values())[::-1]
    n = min(len(got), len(ref))
    err_s = np.max(np.abs(got[:n] - ref[:n])) / ref[0]
    Lg = u1.left_column(_dense_u1(env.get(0)), _dense_u1(env.get(7)), _dense_u1(env.get(3)))
    Lu = u1.left_column(to_dense(envu.get(0)), to_dense(envu.get(7)), to_dense(envu.get(3)))
    err_l = rel(Lg, Lu)
    print(f"cfg3 move: kept states {kept_states}, spectrum err {err_s:.3e}, left column rel diff {err_l:.3e}; "
          f"reduced flops {stats['flops_corners'] + stats['flops_halves'] + stats['flops_renorm']:.3e}, "
          f"expanded {stu['flops_corners'] + stu['flops_halves'] + stu['flops_renorm']:.3e}")
    assert err_s <= 1e-5 and err_l <= 1e-5


# ------------------------------------------------------- SU(2) double layer
def _site_legs(virt):
    return [({1: 1}, IN), (virt, IN), (virt, IN), (virt, OUT), (virt, OUT)]


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_su2_double_layer_vs_oracle(dt):
    spec = _site_legs({0: 1, 1: 2, 2: 1})
    L = [su2.Leg(s, d) for s, d in spec]
    vals = draw((1811, 0), su2.nnz(L))
    A = st.Tensor.create(spec, dtype=dt, group="su2").upload(vals)
    print(f"su2 double layer {dt}", flush=True)
    a = st.double_layer(A)
    got, La = reduced_full(a)
    a_legs, ref, _ = su2.double_layer(L, vals)
    assert [(l.sectors(), l.dir) for l in La] == [(l.sectors(), l.dir) for l in a_legs]
    err = rel(got, ref)
    print(f"  rel err {err:.3e}")
    assert err <= (1e-13 if dt == "f64" else 1e-6)


def test_cfg3_double_layer_legs_and_norm():
    """Full-size SU(2) site tensor: the fused legs are the workload's D^2 leg
    and the dense norm of a (sum over blocks of (2K+1) |m|^2) equals
    |sum_s A_s (x) A_s|, computed from the physical Gram matrix of A."""
    c = config(3)
    spec = [(c["phys"], IN), (c["virt"], IN), (c["virt"], IN), (c["virt"], OUT), (c["virt"], OUT)]
    L = [su2.Leg(s, d) for s, d in spec]
    vals = draw((c["seed"], 0), su2.nnz(L))
    A = st.Tensor.create(spec, dtype="f64", group="su2").upload(vals)
    a = st.double_layer(A)
    assert [(s, d) for s, d in a.legs()] == [(c["dd"], IN), (c["dd"], IN), (c["dd"], OUT), (c["dd"], OUT)]
    v = a.download()
    pos, n2 = 0, 0.0
    for (lab, shp, _, _), tr in zip(a.blocks(), a.trees()):
        k = int(np.prod(shp))
        n2 += (tr[-1] + 1) * float(np.sum(v[pos:pos + k] ** 2))
        pos += k
    Ad = su2.expand(L, vals).reshape(L[0].size, -1)
    G = Ad @ Ad.T
    assert np.isclose(n2, np.sum(G * G), rtol=1e-12)


def test_su2_moves_in_every_direction_vs_oracle():
    """SU(2) moves toward the top, right, bottom and then left again (the
    turned network's reversed legs go through the S^z basis), each against
    the whole-environment oracle's move on the CG-expanded tensors truncated
    to the states the SU(2) move kept: spectrum, the closed networks Z_00 ..
    Z_11 of the whole environment after every move, and the updated edge
    after the first (later edges have open legs on bonds whose gauge the two
    sides choose differently), FP64.  The sequence checks that the
    environment stays consistent with the caller's site tensor (half-integer
    spins on the D^2 legs)."""
    from oracle import ctm, u1
    legs = _env_legs(SMALL_MOVE["chi"], SMALL_MOVE["dd"])
    vals = su2_values(legs, 1811)
    env, dev = _su2_env(legs, vals, "f64")
    D, _, _ = _expanded_u1(legs, vals)
    C = [D[k] for k in ("C1", "C2", "C3", "C4")]
    T = [D[k] for k in ("T1", "T2", "T3", "T4")]
    first = True
    for d in (1, 2, 3, 0):
        print(f"su2 move direction {d}", flush=True)
        stats = env.move(dev["a"], SMALL_MOVE["chi_target"], prec="f64", direction=d)
        kept_states = sum((tj + 1) * k for tj, k in stats["kept"].items())
        C, T, s = ctm.move(C, T, D["a"], kept_states, d)
        assert len(s) == kept_states
        got = _spectrum_states(env.singular_values(), stats)
        assert np.max(np.abs(got[:len(s)] - s)) <= 1e-11 * s[0]
        Cg = [_dense_u1(env.get(k)) for k in range(4)]
        Tg = [_dense_u1(env.get(4 + k)) for k in range(4)]
        # the closed networks of the whole environment (every bond summed, so
        # the gauge of the new bonds drops out)
        kg, zg = ctm.site_partition(Cg, Tg, D["a"])
        ko, zo = ctm.site_partition(C, T, D["a"])
        msg = f"  kept states {kept_states}, kappa {kg:.12f} / {ko:.12f}"
        if first:
            # after the first move the updated edge's open legs are old bonds
            i, j = d, (d + 3) % 4
            err = rel(u1.left_column(Cg[i], Tg[j], Cg[j]), u1.left_column(C[i], T[j], C[j]))
            msg += f", updated edge rel err {err:.2e}"
            assert err <= 1e-10
        print(msg)
        assert abs(kg - ko) <= 1e-10 * abs(ko)
        assert np.allclose(zg, zo, rtol=1e-10)
        first = False


@pytest.mark.parametrize("block", [1, 2])
def test_su2_site_partition_vs_oracle(block):
    """kappa of an SU(2) environment contracted on reduced blocks (the closing
    trace counts a spin-j block 2j+1 times) against the oracle's kappa of the
    CG-expanded dense tensors, before and after one left move (the oracle's
    move truncated to the states the SU(2) move kept), FP64.  The draws
    (seed 1813) give positive 2 x 2 ratios, whose fourth root kappa is."""
    from oracle import ctm
    legs = _env_legs(SMALL_MOVE["chi"], SMALL_MOVE["dd"])
    vals = su2_values(legs, 1813)
    env, dev = _su2_env(legs, vals, "f64")
    D, _, _ = _expanded_u1(legs, vals)
    C = [D[k] for k in ("C1", "C2", "C3", "C4")]
    T = [D[k] for k in ("T1", "T2", "T3", "T4")]
    for stage in ("initial", "after a move"):
        if stage != "initial":
            stats = env.move(dev["a"], SMALL_MOVE["chi_target"], prec="f64")
            kept_states = sum((tj + 1) * k for tj, k in stats["kept"].items())
            C, T, _ = ctm.move(C, T, D["a"], kept_states, 0)
        kg, zg = env.site_partition(dev["a"], block=block)
        ko, zo = ctm.site_partition_block(C, T, D["a"], block)
        print(f"{stage}: kappa {kg:.14e} / {ko:.14e}", flush=True)
        assert abs(kg - ko) <= 1e-10 * abs(ko)
        assert np.allclose(zg, zo, rtol=1e-10)


def test_su2_run_vs_oracle():
    """ctm_run on an SU(2) environment (chi in states, whole multiplets kept)
    against the oracle's run on the CG-expanded dense tensors (its truncation
    never splits a degenerate set, so it keeps the same multiplets): two
    steps of four moves, step counts, kappa and the step error, FP64."""
    from oracle import ctm
    legs = _env_legs(SMALL_MOVE["chi"], SMALL_MOVE["dd"])
    vals = su2_values(legs, 1811)
    env, dev = _su2_env(legs, vals, "f64")
    D, _, _ = _expanded_u1(legs, vals)
    C = [D[k] for k in ("C1", "C2", "C3", "C4")]
    T = [D[k] for k in ("T1", "T2", "T3", "T4")]
    chi = SMALL_MOVE["chi_target"]
    r = env.run(dev["a"], chi=chi, prec="f64", max_steps=2, tol=0.0)
    _, _, ro = ctm.run(C, T, D["a"], chi, max_steps=2, tol=0.0)
    print(r, ro, flush=True)
    assert r["steps"] == ro["steps"] == 2 and r["levels"] == ro["levels"] == 1
    assert abs(r["kappa"] - ro["kappa"]) <= 1e-9 * abs(ro["kappa"])
    assert abs(r["err_steps"] - ro["err_steps"]) <= 1e-9 * abs(ro["kappa"])


def test_u1_expansion_keeps_multiplets_over_ten_moves():
    """Ten truncating moves (directions 0..3 in turn) of an SU(2) environment
    and, side by side, of the library's S^z expansion of it on the U(1)
    path, FP64, each U(1) move truncated to the states the SU(2) move kept.
    The U(1) path treats each S^z sector on its own; its truncation keeps a
    degenerate set whole (Sec. 3's scheme, multiplets split by rounding only),
    so after every move its kept table is the SU(2) table counted by S^z
    components (sector 2m holds every kept multiplet with 2J >= |2m| of the
    same parity), bit for bit, its kept spectrum is the reduced spectrum with
    each value 2J+1 times, and the two environments close to the same kappa."""
    c = dict(chi={0: 2, 1: 2, 2: 1}, dd={0: 2, 1: 2, 2: 1}, chi_target=7)
    legs = _env_legs(c["chi"], c["dd"])
    vals = su2_values(legs, 1817)
    env, dev = _su2_env(legs, vals, "f64")
    U = {n: t.to_u1() for n, t in dev.items()}
    envu = st.CtmEnv([U[k] for k in ("C1", "C2", "C3", "C4")], [U[k] for k in ("T1", "T2", "T3", "T4")])
    for i in range(10):
        d = i % 4
        print(f"move {i} direction {d}", flush=True)
        s2 = env.move(dev["a"], c["chi_target"], prec="f64", direction=d)
        k2 = {tj: n for tj, n in s2["kept"].items() if n > 0}
        states = sum((tj + 1) * n for tj, n in k2.items())
        assert 0 < states <= c["chi_target"]
        s1 = envu.move(U["a"], states, prec="f64", direction=d)
        k1 = {q: n for q, n in s1["kept"].items() if n > 0}
        want = {}
        for tj, n in k2.items():
            for q in range(-tj, tj + 1, 2):
                want[q] = want.get(q, 0) + n
        got = _spectrum_states(env.singular_values(), s2)[:states]
        ref = np.sort(envu.singular_values())[::-1][:states]
        err = np.max(np.abs(got - ref)) / ref[0]
        kg, _ = env.site_partition(dev["a"])
        ku, _ = envu.site_partition(U["a"])
        print(f"  kept su2 {k2} u1 {k1}; spectrum {err:.2e}; kappa {kg:.14e} / {ku:.14e}", flush=True)
        assert k1 == want, (i, k1, want)
        assert err <= 1e-10, (i, err)
        assert abs(kg - ku) <= 1e-10 * abs(ku), (i, kg, ku)


def test_su2_heisenberg_energy_vs_oracle():
    """Bond energies of an SU(2) state (spin 1/2, virtual multiplets j = 0, 1/2)
    in an SU(2) environment: the library measures the S^z components (the
    environment expanded, the double layers with Sz, S+, S- built in the same
    S^z basis of the fused multiplets); the oracle contracts dense tensors in
    SU(2) state order with operator double layers from its own fusion
    isometries.  Both bonds, FP64."""
    from oracle import ctm
    virt = {0: 1, 1: 1}
    A_spec = {"A": [({1: 1}, IN), (virt, IN), (virt, IN), (virt, OUT), (virt, OUT)]}
    A_vals = su2_values(A_spec, 1815)
    A_dev = device(A_spec, A_vals, "f64")["A"]
    A_legs = [su2.Leg(s, d) for s, d in A_spec["A"]]
    Ad = su2.expand(A_legs, A_vals["A"])
    dd = su2.double_layer(A_legs, A_vals["A"])[0][0].sectors()
    assert dd == SMALL_MOVE["dd"]
    legs = _env_legs(SMALL_MOVE["chi"], dd)
    legs.pop("a")
    vals = su2_values(legs, 1815)
    dev = device(legs, vals, "f64")
    env = st.CtmEnv([dev[k] for k in ("C1", "C2", "C3", "C4")], [dev[k] for k in ("T1", "T2", "T3", "T4")])
    e_h, e_v = env.heisenberg_bond_energy(A_dev)

    def layer(op):
        out = np.einsum("tk,klurd,tmvse->lmuvrsde", op, Ad, Ad)    # (ket, bra) pairs per bond
        for v in A_legs[1:]:
            Fl, Fv = su2.fusion_isometry(su2.Leg(v.sectors(), -v.dir), su2.Leg(v.sectors(), v.dir), v.dir)
            out = np.tensordot(out, su2.expand(Fl, Fv), axes=([0, 1], [0, 1]))
        return out
    sz = np.diag([-0.5, 0.5])
    sp = np.array([[0.0, 0.0], [1.0, 0.0]])     # <+1/2| S+ |-1/2> = 1 (rows: bra)
    sm = sp.T.copy()
    a, bz, bp, bm = layer(np.eye(2)), layer(sz), layer(sp), layer(sm)
    C = [su2.expand([su2.Leg(s, d) for s, d in legs[k]], vals[k]) for k in ("C1", "C2", "C3", "C4")]
    T = [su2.expand([su2.Leg(s, d) for s, d in legs[k]], vals[k]) for k in ("T1", "T2", "T3", "T4")]

    def bond(n, m):
        x = lambda s1, s2: ctm.expectation(C, T, a, [s1, s2], n, m)
        return x(bz, bz) + 0.5 * (x(bp, bm) + x(bm, bp))
    eo_h, eo_v = bond(2, 1), bond(1, 2)
    print(f"energies: horizontal {e_h:.14e} / {eo_h:.14e}, vertical {e_v:.14e} / {eo_v:.14e}", flush=True)
    assert abs(e_h - eo_h) <= 1e-10 * max(1.0, abs(eo_h))
    assert abs(e_v - eo_v) <= 1e-10 * max(1.0, abs(eo_v))
