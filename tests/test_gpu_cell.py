"""GPU checks of the unit-cell CTM (one projector pair per cut, columns
moved one after the other): a one-site cell against the 1x1 move, a 2 x 2
cell of four different sites against the oracle's cell move toward each
side, and the Ising model on a 2 x 2 cell from unequal starts against
Onsager."""
import numpy as np
import pytest

import paper_1808_10804_amd as st
from oracle import ctm, u1
from synth import config
from workload import oracle_side, device_side, to_dense, rel, from_dense

pytestmark = pytest.mark.gpu

ENV = ("C1", "C2", "C3", "C4", "T1", "T2", "T3", "T4")


def _site(c, batch):
    """One site of the D=4, chi=16 workload drawn with its own batch index:
    device tensors and the oracle's dense ones."""
    w, T, a, _ = oracle_side(c, c["seed"], batch=batch)
    dev = device_side(c, c["seed"], "f64", batch=batch)
    return dev, ([T[k] for k in ENV[:4]], [T[k] for k in ENV[4:]]), a


def _column(Cs, Ts, j):
    """Gauge-invariant updated edge after a move toward side j."""
    i, k = j, (j + 3) % 4
    return u1.left_column(Cs[i], Ts[k], Cs[k])


@pytest.mark.parametrize("direction", [0, 1, 2, 3])
def test_one_site_cell_equals_1x1_move(direction):
    c = config(1)
    dev, (C0, T0), a = _site(c, 0)
    cell = st.CtmCell([[([dev[k] for k in ENV[:4]], [dev[k] for k in ENV[4:]])]])
    cell.move([[dev["a"]]], 16, prec="f64", direction=direction)
    dev2, _, _ = _site(c, 0)
    env = st.CtmEnv([dev2[k] for k in ENV[:4]], [dev2[k] for k in ENV[4:]])
    env.move(dev2["a"], 16, prec="f64", direction=direction)
    Cg = [to_dense(cell.get(0, 0, k)) for k in range(4)]
    Tg = [to_dense(cell.get(0, 0, 4 + k)) for k in range(4)]
    Ce = [to_dense(env.get(k)) for k in range(4)]
    Te = [to_dense(env.get(4 + k)) for k in range(4)]
    assert rel(_column(Cg, Tg, direction), _column(Ce, Te, direction)) <= 1e-12
    s1 = np.sort(env.singular_values())[::-1]
    sc = cell.singular_values()
    assert np.allclose(sc, s1[:len(sc)], rtol=0, atol=1e-13)


@pytest.mark.parametrize("direction", [0, 1, 2, 3])
def test_2x2_cell_vs_oracle(direction):
    """Four different sites (and environments) of the same leg structure:
    after one move toward `direction`, every site's updated edge (gauge
    invariant: its two chi bonds are the cuts above and below it, each
    carrying one projector pair) and the spectra of all cuts against the
    oracle's cell move, FP64.  (Kappa of one site's environment is no check
    here: in a cell its corners meet across two different cuts.)"""
    c = config(1)
    sites = [[_site(c, 2 * x + y) for y in range(2)] for x in range(2)]
    cell = st.CtmCell([[([s[0][k] for k in ENV[:4]], [s[0][k] for k in ENV[4:]]) for s in col] for col in sites])
    a_dev = [[s[0]["a"] for s in col] for col in sites]
    a_or = [[s[2] for s in col] for col in sites]
    print(f"cell move direction {direction}", flush=True)
    cell.move(a_dev, 12, prec="f64", direction=direction)
    oc, sv = ctm.cell_move([[s[1] for s in col] for col in sites], a_or, 12, direction)
    for x in range(2):
        for y in range(2):
            Cg = [to_dense(cell.get(x, y, k)) for k in range(4)]
            Tg = [to_dense(cell.get(x, y, 4 + k)) for k in range(4)]
            err = rel(_column(Cg, Tg, direction), _column(*oc[x][y], direction))
            print(f"  site ({x},{y}): column rel err {err:.2e}")
            assert err <= 1e-10
    got = cell.singular_values()
    ref = np.concatenate(sv)
    assert got.shape == ref.shape
    assert np.allclose(got, ref, rtol=0, atol=1e-12 * ref.max())


@pytest.mark.parametrize("beta", [0.3, 0.38])
def test_ising_2x2_cell(beta):
    """Z2 Ising tensors on a 2 x 2 cell whose sites start from the oracle's
    unequal random environments: every site reproduces Onsager."""
    a = ctm.ising_tensor(beta)
    rng = np.random.default_rng(8)
    par = np.array([0, 1])
    D = [({0: 1, 1: 1}, d) for d in (1, 1, -1, -1)]
    adev = from_dense(a, D, group="z2")

    def env():
        Cs = [from_dense(np.diag(rng.uniform(0.5, 1.5, 2)), [({0: 1, 1: 1}, 1), ({0: 1, 1: 1}, -1)], group="z2")
              for _ in range(4)]
        Ts = []
        for dd in (-1, 1, 1, -1):
            t = rng.uniform(0.5, 1.5, (2, 2, 2))
            t[(par[:, None, None] + par[None, :, None] + par[None, None, :]) % 2 == 1] = 0.0
            Ts.append(from_dense(t, [({0: 1, 1: 1}, 1), ({0: 1, 1: 1}, dd), ({0: 1, 1: 1}, -1)], group="z2"))
        return Cs, Ts
    cell = st.CtmCell([[env() for _ in range(2)] for _ in range(2)])
    A = [[adev, adev], [adev, adev]]
    for _ in range(40):
        for d in range(4):
            cell.move(A, 12, prec="f64", direction=d)
    exact = ctm.onsager_log_z(beta)
    for x in range(2):
        for y in range(2):
            k, _ = cell.site_partition(x, y, adev)
            print(f"  beta {beta} site ({x},{y}): ln kappa - Onsager = {np.log(k) - exact:.1e}")
            assert abs(np.log(k) - exact) < 1e-10


def test_cell_move_returns_with_its_stream_synchronised():
    """ctm_cell_move returns with the caller's stream idle (a torch stream of
    default priority, queried without waiting), toward every side."""
    import torch
    c = config(1)
    dev, _, _ = _site(c, 0)
    cell = st.CtmCell([[([dev[k] for k in ENV[:4]], [dev[k] for k in ENV[4:]])]])
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for d in range(4):
            cell.move([[dev["a"]]], 16, prec="f64", direction=d, stream=s.cuda_stream)
            assert s.query(), f"stream busy after the cell move toward {d}"
    s.synchronize()


def test_1x1_entry_points_refuse_a_cell():
    """A unit-cell environment goes through the cell entry points only: the
    1x1 partition function and run refuse it (SYMTEN_E_INVAL) instead of
    reading the tensors the cell was created with."""
    import ctypes as C
    from paper_1808_10804_amd import _lib
    c = config(1)
    dev, _, _ = _site(c, 0)
    cell = st.CtmCell([[([dev[k] for k in ENV[:4]], [dev[k] for k in ENV[4:]])]])
    k = C.c_double()
    assert _lib.lib().ctm_site_partition(cell._h, dev["a"]._h, 1, C.byref(k), None, None) == -1
    o, r = _lib.RunOpts(16, 16, 0, 1, 1, 0.0), _lib.RunResult()
    assert _lib.lib().ctm_run(cell._h, dev["a"]._h, C.byref(o), C.byref(r), None) == -1
    # the cell's own entry point still works
    kappa, _ = cell.site_partition(0, 0, dev["a"])
    assert np.isfinite(kappa)
