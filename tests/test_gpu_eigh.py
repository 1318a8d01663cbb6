"""The projector stage's own FP64 symmetric eigensolver (symten_eigh):
every eigenvalue and the eigenvectors of the largest ones of symmetric
matrices shaped like the stage's inputs (Sec. 3: the singular triplets of
each sector's matrix, taken from its Gram or Jordan-Wielandt matrix).

Checked against LAPACK's symmetric eigensolver (numpy.linalg.eigh) for the
values and well-separated vectors, and by properties that fix the result
at any size: the residual ||A z - lambda z||, orthonormality of the
vectors, and for degenerate eigenvalues the projector onto the cluster's
eigenspace.  Sizes span one workgroup per matrix, several per matrix on
one XCD, and the largest order the LDS holds; one call mixes them (several
matrices share each launch)."""
import numpy as np
import pytest
import torch

import paper_1808_10804_amd as st

pytestmark = pytest.mark.gpu

TOL = 1e-13   # relative to max |lambda|: a few hundred ulps at n ~ 1000


def _orth(rng, n):
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    return q * np.sign(np.diag(r))


def _gram(rng, m, n, decay=0.0):
    """Y Y^T of a Gaussian m x n matrix Y, optionally with decaying columns."""
    y = rng.standard_normal((m, n))
    if decay:
        y *= np.exp(-decay * np.arange(n))[None, :]
    return y @ y.T


def _jw(rng, m, n):
    y = rng.standard_normal((m, n))
    return np.block([[np.zeros((m, m)), y], [y.T, np.zeros((n, n))]])


def _check(A, k, w, Z, label):
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    wref, zref = np.linalg.eigh(A)
    scale = max(np.max(np.abs(wref)), np.finfo(float).tiny)
    ew = np.max(np.abs(w - wref)) / scale
    print(f"{label}: n={n} k={k} eigenvalues {ew:.2e}", flush=True)
    assert ew <= TOL, (label, ew)
    if k == 0:
        return
    lam = w[::-1][:k]
    res = np.linalg.norm(A @ Z - Z * lam[None, :], axis=0) / scale
    orth = np.max(np.abs(Z.T @ Z - np.eye(k)))
    print(f"   residual {res.max():.2e} orthogonality {orth:.2e}", flush=True)
    assert res.max() <= TOL, (label, res.max())
    assert orth <= TOL, (label, orth)
    # vectors of the k largest: compare eigenspaces cluster by cluster
    # (clusters: reference eigenvalues closer than 1e-8 relative)
    wr = wref[::-1]
    zr = zref[:, ::-1]
    j = 0
    while j < k:
        c = 1
        while j + c < n and wr[j + c - 1] - wr[j + c] <= 1e-8 * scale:
            c += 1
        if j + c <= k:   # the whole cluster was asked for
            Pg = Z[:, j:j + c] @ Z[:, j:j + c].T
            Pr = zr[:, j:j + c] @ zr[:, j:j + c].T
            err = np.max(np.abs(Pg - Pr))
            gap = min(wr[j - 1] - wr[j] if j > 0 else np.inf,
                      wr[j + c - 1] - wr[j + c] if j + c < n else np.inf) / scale
            # eigenvector perturbation bound: eps ||A|| / gap (times a modest n factor)
            bound = max(TOL, 64 * n * np.finfo(float).eps / max(gap, 1e-300))
            assert err <= bound, (label, j, c, err, bound)
        j += c


def _run(mats, ks, label):
    dev = [torch.from_numpy(np.ascontiguousarray(m)).to("cuda") for m in mats]
    out = st.eigh(dev, ks)
    for i, ((w, Z), A, k) in enumerate(zip(out, mats, ks)):
        _check(A, k, w.cpu().numpy(), Z.cpu().numpy(), f"{label}[{i}]")


def test_max_order_covers_the_stage_blocks():
    nmax = st.eigh_max_order()
    print(f"largest order: {nmax}", flush=True)
    # the D = 6, chi = 64 cut's largest Gram (696) and Jordan-Wielandt (1392) blocks
    assert nmax >= 1392


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 130, 257])
def test_small_orders(n):
    rng = np.random.default_rng(100 + n)
    A = rng.standard_normal((n, n))
    A = A + A.T
    _run([A], [min(n, 9)], f"gaussian n={n}")


def test_gram_shaped_like_the_cut():
    """Gram matrices of the sizes of the D = 6, chi = 64 cut (696, 528, 224,
    48, 4), flat leading spectrum, many values near zero, in one call."""
    rng = np.random.default_rng(7)
    sizes = [696, 528, 528, 224, 224, 48, 48, 4, 4]
    mats = [_gram(rng, n, n, decay=0.02) for n in sizes]
    ks = [min(n, 65) for n in sizes]
    _run(mats, ks, "gram")


def test_jordan_wielandt():
    """[[0, Y], [Y^T, 0]] with square and rectangular Y: eigenvalues +-s and
    |m - n| zeros; the largest spans two XCDs' worth of workgroups."""
    rng = np.random.default_rng(8)
    mats = [_jw(rng, 696, 696), _jw(rng, 300, 200), _jw(rng, 5, 9)]
    _run(mats, [65, 40, 5], "jw")


def test_degenerate_clusters_and_structure():
    """Exactly repeated eigenvalues (one cluster of 4, one of 2, asked for
    whole), a diagonal matrix (every reflector the identity), a zero matrix
    and a rank-one matrix."""
    rng = np.random.default_rng(9)
    n = 200
    lam = rng.standard_normal(n)
    lam[-4:] = 5.0
    lam[-6:-4] = 4.0
    Q = _orth(rng, n)
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    D = np.diag(rng.standard_normal(50))
    Zm = np.zeros((30, 30))
    u = rng.standard_normal(40)
    R1 = np.outer(u, u)
    _run([A, D, Zm, R1], [6, 10, 3, 1], "structured")


def test_largest_order():
    rng = np.random.default_rng(10)
    n = st.eigh_max_order()
    A = _gram(rng, n, n // 2)
    _run([A], [8], f"largest n={n}")


def test_refuses_bad_arguments():
    A = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(st.SymtenError):
        st.eigh([A], [5])            # more vectors than the order
    n = st.eigh_max_order() + 1
    B = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    with pytest.raises(st.SymtenError) as e:
        st.eigh([B], [1])
    assert e.value.code == -7
