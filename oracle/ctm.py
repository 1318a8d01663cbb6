"""Whole-environment CTM on dense FP64 arrays: the move in all four
directions, the partition function per site, and the iteration.

TEST INFRASTRUCTURE ONLY: used by tests/ to check the library's multi-move
driver; never by the product library.

Tensors follow the conventions of the U(1) oracle: C_i[in, out] and
T_i[chi in, D, chi out] with the chi bonds running clockwise
C1 -> T1 -> C2 -> T2 -> C3 -> T3 -> C4 -> T4 -> C1, a[l, u, r, d].  Dense
arrays carry no charge labels, so a symmetric tensor is handled through its
embedding and the move below is the projector scheme of Sec. 3 (the one the
paper cites) without sector bookkeeping: the fused cut index is (chi, D)
row-major and the truncation is the global top-chi of one dense SVD.
"""
import numpy as np

from . import u1

CUTOFF = 1e-14
DEGENERATE_REL = 1e-8


def _e(spec, *ops):
    return np.einsum(spec, *ops, optimize="optimal")


def left_move(C, T, a, chi):
    """One left move: new (C1, T4, C4), each of unit Frobenius norm, and the
    kept singular values.  C = [C1..C4], T = [T1..T4]."""
    C1, C2, C3, C4 = C
    T1, T2, T3, T4 = T
    # enlarged corners (rows, cols as in the U(1) oracle)
    c1 = _e("yxlu,lurd->ydxr", _e("aux,yla->yxlu", _e("ab,bux->aux", C1, T1), T4), a)   # [x4, d | x1, r]
    c2 = _e("xzur,lurd->xlzd", _e("cxu,crz->xzur", _e("bc,xub->cxu", C2, T1), T2), a)   # [x1, l | x2, d]
    c3 = _e("zydr,lurd->yuzl", _e("edz,yre->zydr", _e("ef,fdz->edz", C3, T3), T2), a)   # [x2, u | x3, l]
    c4 = _e("zDly,lurD->yuzr", _e("qzD,qly->zDly", _e("pq,zDp->qzD", C4, T3), T4), a)   # [x4, u | x3, r]
    m = lambda c: c.reshape(c.shape[0] * c.shape[1], -1)
    Hu = m(c1) @ m(c2)
    Hd = m(c4) @ m(c3).T
    # QR of the transposed halves, SVD of R_u R_d^T, top chi
    _, Ru = np.linalg.qr(Hu.T)
    _, Rd = np.linalg.qr(Hd.T)
    U, s, Vt = np.linalg.svd(Ru @ Rd.T)
    k = int(min(chi, np.sum(s > CUTOFF * s[0])))
    while 1 < k < len(s) and s[k] >= (1.0 - DEGENERATE_REL) * s[k - 1]:
        k -= 1                                     # a degenerate set is never split
    sq = np.sqrt(s[:k])
    P = Rd.T @ Vt[:k].T / sq                       # [(x4, d), k]
    Pt = (U[:, :k] / sq).T @ Ru                    # [k, (x4, u)]
    nX4, nD = C1.shape[0], T1.shape[1]
    CT = _e("ab,bux->aux", C1, T1)                 # [xa, u, x1]
    C1n = P.T @ CT.reshape(CT.shape[0] * CT.shape[1], -1)
    T4a = _e("ylx,lurd->ydxur", T4, a)             # [(y, d), (x, u), r]
    T4a = T4a.reshape(T4.shape[0] * a.shape[3], T4.shape[2] * a.shape[1], a.shape[2])
    T4n = _e("fk,fgr,hg->krh", P, T4a, Pt)
    C4T3 = _e("pq,zDp->zqD", C4, T3)               # [z, (q, D)]
    C4n = C4T3.reshape(C4T3.shape[0], -1) @ Pt.T
    nrm = lambda x: x / np.linalg.norm(x)
    return nrm(C1n), nrm(T4n), nrm(C4n), s[:k]


def rotate(C, T, a):
    """The network turned a quarter counterclockwise: C1' = C2, ..., C4' = C1,
    T1' = T2, ..., T4' = T1, a'[l, u, r, d] = a[u, r, d, l] (dense arrays need
    no relabelling of directions)."""
    return [C[1], C[2], C[3], C[0]], [T[1], T[2], T[3], T[0]], a.transpose(1, 2, 3, 0)


def move(C, T, a, chi, direction):
    """Move toward `direction` (0 left, 1 top, 2 right, 3 bottom): the left
    move of the network turned `direction` quarter turns, turned back."""
    C, T = list(C), list(T)
    ar = a
    for _ in range(direction):
        C, T, ar = rotate(C, T, ar)
    C[0], T[3], C[3], s = left_move(C, T, ar, chi)
    for _ in range(4 - direction):
        C, T, ar = rotate(C, T, ar)
    return C, T, s


def site_partition(C, T, a):
    """kappa = Z_11 Z_00 / (Z_10 Z_01) and the four Z (Z_00, Z_10, Z_01, Z_11)."""
    C1, C2, C3, C4 = C
    T1, T2, T3, T4 = T
    e = np.einsum               # two operands at a time
    z00 = e("ab,ba->", e("ab,bc->ac", C1, C2), e("cd,da->ca", C3, C4))
    top = e("abc,cd->abd", e("ab,buc->auc", C1, T1), C2)                  # [a, u, d]
    bot = e("def,fa->dea", e("de,euf->duf", C3, T3), C4)                  # [d, u, a]
    z10 = e("aud,dua->", top, bot)
    left = e("fra,ab->frb", T4, e("ab,bc->ac", C1, C2))                   # [f, r, c]
    right = e("crd,de->cre", T2, e("de,ef->df", C3, C4))                  # [c, r, f]
    z01 = e("frc,crf->", left, right)
    x = e("aud,dre->aure", top, T2)                                       # [a, u, r, e]
    x = e("aure,lurq->aelq", x, a)                                        # [a, e, l, q]
    x = e("aelq,ef->aflq", x, C3)
    x = e("aflq,fqg->alg", x, T3)
    x = e("alg,gh->alh", x, C4)
    z11 = e("alh,hla->", x, T4)
    return z11 * z00 / (z10 * z01), (z00, z10, z01, z11)


def network(C, T, a, n, m, sites=None):
    """The closed network Z_nm as (tensor, bond labels) pairs: the corners,
    n edge tensors on the top and bottom sides, m on the left and right, and
    the n x m site tensors.  Bond names: h (top chi bonds, left to right),
    v (right side, top to bottom), g (bottom, right to left), w (left side,
    bottom to top), ("V", i, j) the D bond below row i of column j (row 0 =
    the top edge), ("H", i, j) the D bond right of column j in row i (column
    0 = the left edge).  Listed top row first, then row by row (right edge,
    sites right to left, left edge), then the bottom row, so that every
    tensor shares a bond with those before it.  sites (optional): n*m site
    tensors replacing a, row-major (row 0 on top, column 0 on the left)."""
    C1, C2, C3, C4 = C
    T1, T2, T3, T4 = T
    net = [(C1, [("w", m), ("h", 0)])]
    net += [(T1, [("h", j - 1), ("V", 0, j), ("h", j)]) for j in range(1, n + 1)]
    net.append((C2, [("h", n), ("v", 0)]))
    for i in range(1, m + 1):
        net.append((T2, [("v", i - 1), ("H", i, n), ("v", i)]))
        net += [(a if sites is None else sites[(i - 1) * n + (j - 1)],
                 [("H", i, j - 1), ("V", i - 1, j), ("H", i, j), ("V", i, j)]) for j in range(n, 0, -1)]
        net.append((T4, [("w", m - i), ("H", i, 0), ("w", m - i + 1)]))
    net.append((C3, [("v", m), ("g", 0)]))
    net += [(T3, [("g", n - j), ("V", m, j), ("g", n - j + 1)]) for j in range(n, 0, -1)]
    net.append((C4, [("g", n), ("w", 0)]))
    return net


def z_block(C, T, a, n, m, sites=None):
    """Z_nm: the tensors of `network` contracted one after another, each over
    every bond it shares with the part already contracted."""
    net = network(C, T, a, n, m, sites)
    X, xl = net[0]
    for t, tl in net[1:]:
        shared = [b for b in xl if b in tl]
        X = np.tensordot(X, t, axes=([xl.index(b) for b in shared], [tl.index(b) for b in shared]))
        xl = [b for b in xl if b not in shared] + [b for b in tl if b not in shared]
    assert xl == []
    return float(X)


def site_partition_block(C, T, a, b):
    """kappa on a b x b patch: kappa^(b^2) = Z_bb Z_00 / (Z_b0 Z_0b); b = 2
    cancels the unequal corner weights of environments whose bonds alternate
    between two charge parities from site to site."""
    z = tuple(z_block(C, T, a, n, m) for n, m in ((0, 0), (b, 0), (0, b), (b, b)))
    r = z[3] * z[0] / (z[1] * z[2])
    return (r if b == 1 else r ** (1.0 / (b * b))), z


def expectation(C, T, a, sites, n, m):
    """Z_nm(sites) / Z_nm(a)."""
    return z_block(C, T, a, n, m, sites) / z_block(C, T, a, n, m)


def heisenberg_bond_energy(C, T, A, A_legs):
    """<S_i . S_j> = <Sz Sz> + (<S+ S-> + <S- S+>)/2 on a horizontal (2 x 1
    patch) and a vertical (1 x 2) bond, from dense double layers with the
    spin operators between the layers."""
    from oracle import u1
    sz, sp, sm = u1.spin_operators(A_legs[0])
    a = u1.double_layer(A, A_legs)[0]
    bz, bp, bm = (u1.double_layer_op(A, A_legs, o) for o in (sz, sp, sm))

    def bond(n, m):
        return (expectation(C, T, a, [bz, bz], n, m)
                + 0.5 * (expectation(C, T, a, [bp, bm], n, m) + expectation(C, T, a, [bm, bp], n, m)))
    return bond(2, 1), bond(1, 2)


def run(C, T, a, chi, chi_max=None, block=1, max_steps=15, tol=1e-8):
    """The CTM error estimate of Sec. 3.  At fixed chi: steps (one move
    toward each side) until kappa changes by less than tol, or max_steps; the
    first error is the largest change among the last three values (the value
    before the first step included).  Then chi doubles while it stays within
    chi_max, until the values at two successive chis differ by less than tol;
    the second error is that difference.  Returns the final environment and
    a dict (kappa, err_steps, err_chi, error, steps, total_steps, chi,
    levels)."""
    chi_max = chi if chi_max is None else chi_max
    values = []                  # the result at each chi
    total = 0
    while True:
        history = [site_partition_block(C, T, a, block)[0]]
        while len(history) - 1 < max_steps:
            for d in range(4):
                C, T, _ = move(C, T, a, chi, d)
            history.append(site_partition_block(C, T, a, block)[0])
            if abs(history[-1] - history[-2]) < tol:
                break
        steps = len(history) - 1
        total += steps
        last3 = history[-3:]
        err_steps = max(abs(y - x) for x, y in zip(last3, last3[1:]))
        values.append(history[-1])
        err_chi = abs(values[-1] - values[-2]) if len(values) > 1 else 0.0
        if (len(values) > 1 and err_chi < tol) or 2 * chi > chi_max:
            break
        chi *= 2
    return C, T, dict(kappa=values[-1], err_steps=err_steps, err_chi=err_chi, error=max(err_steps, err_chi),
                      steps=steps, total_steps=total, chi=chi, levels=len(values))


# --------------------------------------------------------------------------
# Classical vertex models with U(1) arrow conservation
# --------------------------------------------------------------------------
ARROW = {-1: 0, +1: 1}      # bond state index of charge -1, +1 (charge ascending)


def vertex_tensor(weights):
    """a[l, u, r, d] on bonds with charges -1, +1 (arrows), non-zero only when
    l + u = r + d (two in, two out): `weights` maps (l, u, r, d) charge tuples
    to weights."""
    a = np.zeros((2, 2, 2, 2))
    for (l, u, r, d), w in weights.items():
        assert l + u == r + d
        a[ARROW[l], ARROW[u], ARROW[r], ARROW[d]] = w
    return a


def ice_weights():
    """Square ice (the six-vertex model with unit weights)."""
    q = (-1, 1)
    return {(l, u, r, d): 1.0 for l in q for u in q for r in q for d in q if l + u == r + d}


# charges of the initial environment bond: both parities, so that the edge
# tensors can carry the odd bond charges
INIT_CHI = {-1: 1, 0: 1, 1: 1}


def initial_environment():
    """All allowed blocks of C (in, out) and T (in, D, out) set to 1, with the
    chi bond {-1, 0, +1} and the D bond {-1, +1}; T1, T4 have the D leg out,
    T2, T3 in (the conventions of a)."""
    xs = [-1, 0, 1]
    ds = [-1, 1]
    C = np.eye(3)
    Tout = np.zeros((3, 2, 3))     # q_in - q_D - q_out = 0
    Tin = np.zeros((3, 2, 3))      # q_in + q_D - q_out = 0
    for i, qi in enumerate(xs):
        for j, qd in enumerate(ds):
            for o, qo in enumerate(xs):
                if qi - qd - qo == 0:
                    Tout[i, j, o] = 1.0
                if qi + qd - qo == 0:
                    Tin[i, j, o] = 1.0
    return [C, C, C, C], [Tout, Tin, Tin, Tout]


# --------------------------------------------------------------------------
# The classical Ising model with Z2-symmetric tensors
# --------------------------------------------------------------------------
def ising_tensor(beta):
    """Site tensor of the square-lattice Ising model (J = 1) in the parity
    basis of the bonds: exp(beta s s') = cosh(beta) + s s' sinh(beta) =
    sum_p c_p s^p s'^p with c_0 = cosh, c_1 = sinh; each bond weight is split
    as sqrt(c_p) to its two sites, and the sum over the site spin leaves
    a[p_l, p_u, p_r, p_d] = 2 prod_i sqrt(c_(p_i)) when the parities add up to
    0 mod 2, else 0 (Z2 conservation)."""
    c = np.array([np.cosh(beta), np.sinh(beta)])
    a = np.zeros((2, 2, 2, 2))
    for p in np.ndindex(2, 2, 2, 2):
        if sum(p) % 2 == 0:
            a[p] = 2.0 * np.prod(np.sqrt(c[list(p)]))
    return a


def onsager_log_z(beta, n=512):
    """ln Z per site of the square-lattice Ising model (Onsager):
    ln 2 + (1 / 8 pi^2) int int ln[cosh(2b)^2 - sinh(2b)(cos t1 + cos t2)]
    over [0, 2 pi]^2, by the trapezoid rule on an n x n grid (exponentially
    accurate for a smooth periodic integrand, i.e. away from the critical
    point)."""
    t = 2.0 * np.pi * np.arange(n) / n
    c1, c2 = np.meshgrid(np.cos(t), np.cos(t), indexing="ij")
    f = np.log(np.cosh(2 * beta) ** 2 - np.sinh(2 * beta) * (c1 + c2))
    return np.log(2.0) + 0.5 * f.mean()


def ising_initial_environment():
    """chi = 1 environment of charge-0 bonds: C = 1, T[0, p, 0] = 1 for the
    even bond parity p = 0 (the only block the rule allows)."""
    t = np.zeros((1, 2, 1))
    t[0, 0, 0] = 1.0
    return [np.ones((1, 1))] * 4, [t] * 4


# --------------------------------------------------------------------------
# Unit cells of Lx x Ly sites (the paper times a 2 x 2 cell)
# --------------------------------------------------------------------------
# cell[x][y] = (C, T): the environment of site (x, y) as in the 1 x 1 case
# (C1 top-left .. C4 bottom-left, T1 top .. T4 left); a[x][y] its site tensor.
# x grows to the right, y downwards; indices are periodic.  The cut y lies
# between site rows y and y + 1.

def _corners(C, T, a, which):
    """Enlarged corner `which` (1..4) of one site's environment as a matrix,
    with the rows and columns of left_move."""
    C1, C2, C3, C4 = C
    T1, T2, T3, T4 = T
    if which == 1:
        c = _e("yxlu,lurd->ydxr", _e("aux,yla->yxlu", _e("ab,bux->aux", C1, T1), T4), a)
    elif which == 2:
        c = _e("xzur,lurd->xlzd", _e("cxu,crz->xzur", _e("bc,xub->cxu", C2, T1), T2), a)
    elif which == 3:
        c = _e("zydr,lurd->yuzl", _e("edz,yre->zydr", _e("ef,fdz->edz", C3, T3), T2), a)
    else:
        c = _e("zDly,lurD->yuzr", _e("qzD,qly->zDly", _e("pq,zDp->qzD", C4, T3), T4), a)
    return c.reshape(c.shape[0] * c.shape[1], -1)


def _cut_projectors(m1, m2, m3, m4, chi):
    """P, P~ and the kept singular values of one horizontal cut from the four
    enlarged corners around it (the scheme of left_move)."""
    Hu = m1 @ m2
    Hd = m4 @ m3.T
    _, Ru = np.linalg.qr(Hu.T)
    _, Rd = np.linalg.qr(Hd.T)
    U, s, Vt = np.linalg.svd(Ru @ Rd.T)
    k = int(min(chi, np.sum(s > CUTOFF * s[0])))
    while 1 < k < len(s) and s[k] >= (1.0 - DEGENERATE_REL) * s[k - 1]:
        k -= 1
    sq = np.sqrt(s[:k])
    return Rd.T @ Vt[:k].T / sq, (U[:, :k] / sq).T @ Ru, s[:k]


def cell_left_move(cell, a, chi):
    """Left move of a unit cell: column by column (x = 0 .. Lx - 1), the
    projectors of every cut y from the 2 x 2 block of sites (x, y) .. (x + 1,
    y + 1), then the left column of the sites (x + 1, y) renormalised:
    C1'(x+1, y) = P(y-1)^T C1 T1 (x, y), T4'(x+1, y) = P~(y-1) T4 a (x, y) P(y),
    C4'(x+1, y) = C4 T3 (x, y) P~(y)^T, each to unit norm.  Returns the new
    cell and the kept singular values of every cut."""
    Lx, Ly = len(cell), len(cell[0])
    cell = [[(list(C), list(T)) for (C, T) in col] for col in cell]
    svals = []
    for x in range(Lx):
        x1 = (x + 1) % Lx
        P, Pt = {}, {}
        for y in range(Ly):
            y1 = (y + 1) % Ly
            m1 = _corners(*cell[x][y], a[x][y], 1)
            m2 = _corners(*cell[x1][y], a[x1][y], 2)
            m3 = _corners(*cell[x1][y1], a[x1][y1], 3)
            m4 = _corners(*cell[x][y1], a[x][y1], 4)
            P[y], Pt[y], s = _cut_projectors(m1, m2, m3, m4, chi)
            svals.append(s)
        new = []
        for y in range(Ly):
            (C1, C2, C3, C4), (T1, T2, T3, T4) = cell[x][y]
            ym = (y - 1) % Ly
            CT = _e("ab,bux->aux", C1, T1)
            C1n = P[ym].T @ CT.reshape(CT.shape[0] * CT.shape[1], -1)
            T4a = _e("ylx,lurd->ydxur", T4, a[x][y])
            T4a = T4a.reshape(T4.shape[0] * a[x][y].shape[3], T4.shape[2] * a[x][y].shape[1], a[x][y].shape[2])
            T4n = _e("fk,fgr,hg->krh", P[y], T4a, Pt[ym])
            C4T3 = _e("pq,zDp->zqD", C4, T3)
            C4n = C4T3.reshape(C4T3.shape[0], -1) @ Pt[y].T
            new.append((C1n, T4n, C4n))
        nrm = lambda t: t / np.linalg.norm(t)
        for y in range(Ly):
            C, T = cell[x1][y]
            C[0], T[3], C[3] = (nrm(t) for t in new[y])
    return cell, svals


def cell_rotate(cell, a):
    """The cell turned a quarter counterclockwise: site (x, y) moves to
    (y, Lx - 1 - x), and every site's environment and tensor turn as in
    rotate."""
    Lx, Ly = len(cell), len(cell[0])
    nc = [[None] * Lx for _ in range(Ly)]
    na = [[None] * Lx for _ in range(Ly)]
    for x in range(Lx):
        for y in range(Ly):
            C, T, ar = rotate(*cell[x][y], a[x][y])
            nc[y][Lx - 1 - x] = (C, T)
            na[y][Lx - 1 - x] = ar
    return nc, na


def cell_move(cell, a, chi, direction):
    """Move toward `direction` (0 left .. 3 bottom) of a unit cell: the left
    move of the cell turned `direction` quarter turns, turned back."""
    for _ in range(direction):
        cell, a = cell_rotate(cell, a)
    cell, s = cell_left_move(cell, a, chi)
    for _ in range(4 - direction):
        cell, a = cell_rotate(cell, a)
    return cell, s
