"""Edge cases of the truncation in one left move, against the dense FP64
oracle: a cut that falls inside a degenerate pair of singular values (the
pair is dropped whole: the U(1) counterpart of keeping SU(2) multiplets
whole, as the paper's reduced truncation does), chi above the number of
non-negligible values (everything above the route's noise floor is kept),
and chi = 1.  In FP64 and, on FP32 storage, with FP32, bf16x6 and bf16x3
sector products, whose projector stage takes the singular values from the
Gram matrix Y Y^T and drops values at or below sqrt(N eps) s_max."""
import numpy as np
import pytest

import paper_1808_10804_amd as st
from oracle import ctm, u1
from synth import config
from workload import oracle_side, to_dense, rel, from_dense

pytestmark = pytest.mark.gpu


def _mirror(sectors):
    """Index map of a leg under charge conjugation q -> -q (sectors laid
    out by ascending charge, the same offset inside the sector)."""
    qs = sorted(sectors)
    off, pos = {}, 0
    for q in qs:
        off[q] = pos
        pos += sectors[q]
    m = np.empty(pos, dtype=int)
    for q in qs:
        assert sectors[-q] == sectors[q]
        m[off[q]:off[q] + sectors[q]] = off[-q] + np.arange(sectors[q])
    return m


def _symmetrise(x, maps):
    """(x + x with every index mirrored) / 2: invariant under q -> -q."""
    return 0.5 * (x + x[np.ix_(*maps)])


PRECS = ["f64", "f32", "bf16x6", "bf16x3"]
TOL = {"f64": 1e-12, "f32": 1e-5, "bf16x6": 1e-5, "bf16x3": 1e-5}
# the left column's tolerance: FP64 1e-10 (the projectors' s^-1/2); the
# others the FP32 target, bf16x3 its measured move level (it misses 1e-5 on
# whole moves)
LTOL = {"f64": 1e-10, "f32": 1e-5, "bf16x6": 1e-5, "bf16x3": 5e-5}
# rounding unit of the values the projector stage sees
UNIT = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "bf16x6": 2.0 ** -24, "bf16x3": 2.0 ** -17}


def _workload(conjugation_symmetric, dtype="f64"):
    c = config(1)
    w, T, a, _ = oracle_side(c, c["seed"])
    if conjugation_symmetric:
        mc, md = _mirror(w.chi), _mirror(w.dd)
        for k in ("C1", "C2", "C3", "C4"):
            T[k] = _symmetrise(T[k], [mc, mc])
        for k in ("T1", "T2", "T3", "T4"):
            T[k] = _symmetrise(T[k], [mc, md, mc])
        a = _symmetrise(a, [md, md, md, md])
    chi_l, dd_l = w.chi, w.dd
    dev = {k: from_dense(T[k], [(chi_l, 1), (chi_l, -1)], dtype=dtype) for k in ("C1", "C2", "C3", "C4")}
    for k, d in (("T1", -1), ("T4", -1), ("T2", 1), ("T3", 1)):
        dev[k] = from_dense(T[k], [(chi_l, 1), (dd_l, d), (chi_l, -1)], dtype=dtype)
    dev["a"] = from_dense(a, [(dd_l, 1), (dd_l, 1), (dd_l, -1), (dd_l, -1)], dtype=dtype)
    return w, T, a, dev


def _move_both(w, T, a, dev, chi, prec="f64"):
    C0 = [T["C1"], T["C2"], T["C3"], T["C4"]]
    T0 = [T["T1"], T["T2"], T["T3"], T["T4"]]
    C1o, T4o, C4o, so = ctm.left_move(C0, T0, a, chi)
    env = st.CtmEnv([dev[k] for k in ("C1", "C2", "C3", "C4")], [dev[k] for k in ("T1", "T2", "T3", "T4")])
    stats = env.move(dev["a"], chi, prec=prec)
    # the whole spectrum of the cut, descending; the kept values lead it
    sg = np.sort(env.singular_values())[::-1][:sum(stats["kept"].values())]
    # the new legs laid out by charge on the device, by value in the oracle:
    # the left column contracts them away
    C1g, T4g, C4g = (to_dense(env.get(k)) for k in (0, 7, 3))
    return so, sg, stats, u1.left_column(C1o, T4o, C4o), u1.left_column(C1g, T4g, C4g)


@pytest.mark.parametrize("prec", PRECS)
def test_cut_inside_a_degenerate_pair(prec):
    """With the network invariant under q -> -q, the cut sectors Q and -Q have
    the same spectrum.  chi is put between the two members of such a pair:
    both sides drop the pair and keep chi - 1 states, with the same values
    and the same (gauge-invariant) left column."""
    w, T, a, dev = _workload(True, "f64" if prec == "f64" else "f32")
    C0 = [T["C1"], T["C2"], T["C3"], T["C4"]]
    T0 = [T["T1"], T["T2"], T["T3"], T["T4"]]
    s_all = ctm.left_move(C0, T0, a, 10 ** 6)[3]
    pairs = [p for p in range(4, len(s_all) - 1)
             if abs(s_all[p] - s_all[p + 1]) <= 1e-12 * s_all[0]
             and s_all[p - 1] - s_all[p] > 1e-6 * s_all[0]]
    assert pairs, "no degenerate pair in the symmetric spectrum"
    p = pairs[0]
    chi = p + 1                                  # keeps s[p], not its partner s[p + 1]
    print(f"degenerate pair at {p}, {p + 1}: {s_all[p]:.15e} {s_all[p + 1]:.15e}; chi {chi}", flush=True)
    so, sg, stats, Lo, Lg = _move_both(w, T, a, dev, chi, prec)
    err = rel(Lg, Lo)
    print(f"{prec}: kept {sum(stats['kept'].values())}, left column {err:.3e}", flush=True)
    assert len(so) == chi - 1                    # the oracle dropped the pair
    assert sum(stats["kept"].values()) == chi - 1
    assert np.allclose(sg, so, rtol=0, atol=TOL[prec] * so[0])
    assert err <= LTOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_chi_above_the_available_states(prec):
    """chi far above the cut's rank: every value above the route's cutoff is
    kept, the oracle's values above the same cutoff in number (the Gram
    route's floor sqrt(N eps) s_max, N the largest block of the cut)."""
    w, T, a, dev = _workload(False, "f64" if prec == "f64" else "f32")
    so, sg, stats, Lo, Lg = _move_both(w, T, a, dev, 100000, prec)
    if prec == "f64":
        cut = 1e-14
    else:
        F = u1.fuse(u1.Leg(w.chi, 1), u1.Leg(w.dd, 1), +1, -1, 1)[0]
        cut = np.sqrt(max(F.dims) * 2.0 ** -52)
    assert stats["cutoff"] == pytest.approx(cut, rel=1e-12)
    s_all = ctm.left_move([T[k] for k in ("C1", "C2", "C3", "C4")], [T[k] for k in ("T1", "T2", "T3", "T4")],
                          a, 10 ** 6)[3]
    above = s_all[s_all > cut * s_all[0]]
    n = sum(stats["kept"].values())
    err = rel(Lg, Lo)
    print(f"{prec}: kept {n} of chi 100000 (oracle {len(so)}, {len(above)} above the cutoff {cut:.1e}), "
          f"s_min/s_max {above[-1] / above[0]:.3e}, left column {err:.3e}", flush=True)
    assert n == len(above) == len(sg)
    assert np.allclose(sg, above, rtol=0, atol=TOL[prec] * above[0])
    if prec == "f64":
        # the projectors carry s^-1/2: FP64 errors of order 1e-16 s_max in
        # the smallest kept triplets grow by s_max / s_min in the column
        assert err <= max(1e-10, 1e-13 * so[0] / so[-1])
    else:
        # on the other routes the oracle keeps values the library drops; the
        # column is compared with the oracle's move truncated to the same
        # states, where the rounding of the inputs grows by s_max / s_min
        C1o, T4o, C4o, _ = ctm.left_move([T[k] for k in ("C1", "C2", "C3", "C4")],
                                         [T[k] for k in ("T1", "T2", "T3", "T4")], a, n)
        err = rel(Lg, u1.left_column(C1o, T4o, C4o))
        print(f"{prec}: left column against the oracle at chi {n}: {err:.3e}", flush=True)
        assert err <= max(LTOL[prec], 10 * UNIT[prec] * above[0] / above[-1])


@pytest.mark.parametrize("prec", PRECS)
def test_chi_one(prec):
    """chi = 1 keeps the largest value alone (the random workload has no
    degeneracy at the top)."""
    w, T, a, dev = _workload(False, "f64" if prec == "f64" else "f32")
    so, sg, stats, Lo, Lg = _move_both(w, T, a, dev, 1, prec)
    assert len(so) == 1 and sum(stats["kept"].values()) == 1
    assert abs(sg[0] - so[0]) <= TOL[prec] * so[0]
    assert rel(Lg, Lo) <= LTOL[prec]


def test_many_sectors_split_size_classes():
    """Seventeen chi sectors of dimension 2 at bond dimension 3: the cut has 21
    charge sectors, seventeen of them within a factor 2 of the largest (18),
    more than one batched eigensolve takes (16), so the size class is split.  Spectrum, kept count
    and left column against the dense oracle, in FP64."""
    from workload import device_side
    c = config(1)
    c.update(virt={-2: 1, 0: 1, 2: 1}, chi={q: 2 for q in range(-16, 18, 2)}, chi_target=40)
    w, T, a, _ = oracle_side(c, 4242)
    dev = device_side(c, 4242, "f64")
    n_cut = len({qc + qd for qc in w.chi for qd in w.dd})
    assert n_cut == 21
    so, sg, stats, Lo, Lg = _move_both(w, T, a, dev, c["chi_target"])
    err = rel(Lg, Lo)
    print(f"{n_cut} cut sectors, kept {len(so)}, left column {err:.3e}", flush=True)
    assert len(stats["sv_sectors"]) == n_cut
    assert sum(stats["kept"].values()) == len(so)
    assert np.allclose(sg, so, rtol=0, atol=1e-12 * so[0])
    assert err <= 1e-10


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x6"])
@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_nonfinite_input_fails_with_linalg(prec, bad):
    """A NaN or Inf in an environment tensor reaches the halves of the cut;
    the move stops with SYMTEN_E_LINALG (the non-finite entries are replaced
    by zeros before the eigensolve, which only ever sees finite matrices) and
    leaves the environment as it was."""
    w, T, a, dev = _workload(False, "f64" if prec == "f64" else "f32")
    v = dev["C1"].download()
    v[len(v) // 2] = bad
    dev["C1"].upload(v)
    env = st.CtmEnv([dev[k] for k in ("C1", "C2", "C3", "C4")], [dev[k] for k in ("T1", "T2", "T3", "T4")])
    before = [env.get(k).download() for k in range(8)]
    with pytest.raises(st.SymtenError) as e:
        env.move(dev["a"], 16, prec=prec)
    assert e.value.code == -6 and "NaN or Inf" in str(e.value), str(e.value)
    after = [env.get(k).download() for k in range(8)]
    for x, y in zip(before, after):
        assert np.array_equal(x, y, equal_nan=True)
