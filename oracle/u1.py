"""U(1) symmetric tensors embedded densely, and one CTM left move, in FP64.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
baseline of the benchmark; never by the product library.

Conventions (the paper leaves leg directions free as long as they are
consistent, Sec. 3.1):

* A leg is a list of charge sectors {q: d} (q in units of 2 S^z) and a
  direction, +1 (incoming) or -1 (outgoing).  Its states are ordered by charge
  ascending, then by the index inside the sector.
* A block is allowed when sum_l dir_l * q_l == flux (the abelian addition
  rule, Sec. 2); every other entry of the dense tensor is exactly zero.
* Canonical block order is lexicographic in the sector indices (leg 0
  slowest); inside a block, values are row-major.  Random values are laid out
  in that order.
* Site tensor A[s, l, u, r, d] has directions (in, in, in, out, out) and flux
  +1; the double layer a[L, U, R, D] (in, in, out, out) has flux 0.
* Environment bonds run clockwise C1 -> T1 -> C2 -> T2 -> C3 -> T3 -> C4 ->
  T4 -> C1.  Corners are C[in, out]; edges are T[chi_in, D2, chi_out] with the
  D2 leg outgoing for T1 and T4 and incoming for T2 and T3.
"""
import itertools
import numpy as np

IN, OUT = +1, -1
TRUNC_REL_CUTOFF = 1e-14   # singular values <= cutoff * s_max are dropped
DEGENERATE_REL = 1e-8   # relative spread of a degenerate set of singular values


class Leg:
    """Charge sectors {q: d} (only d > 0 kept) plus a direction."""

    def __init__(self, sectors, direction):
        items = sorted((int(q), int(d)) for q, d in dict(sectors).items() if int(d) > 0)
        self.charges = [q for q, _ in items]
        self.dims = [d for _, d in items]
        self.dir = int(direction)

    @property
    def size(self):
        return int(sum(self.dims))

    def sectors(self):
        return dict(zip(self.charges, self.dims))

    def offsets(self):
        return dict(zip(self.charges, np.concatenate([[0], np.cumsum(self.dims)[:-1]]).astype(int)))

    def state_charges(self):
        return np.repeat(np.array(self.charges, dtype=np.int64), self.dims)

    def flipped(self):
        return Leg(self.sectors(), -self.dir)

    def dim(self, q):
        return self.sectors().get(q, 0)

    def __repr__(self):
        return f"Leg({self.sectors()}, {'in' if self.dir > 0 else 'out'})"


# --------------------------------------------------------------------------
# Blocks and dense embedding (Sec. 2, Eq. tensor-blocks and the rank-2 example)
# --------------------------------------------------------------------------

def allowed_blocks(legs, flux, modulus=0):
    """Charge tuples of all blocks obeying sum dir*q == flux (modulo
    `modulus` for Z_n charges), canonical order."""
    out = []
    for qs in itertools.product(*[leg.charges for leg in legs]):
        s = sum(leg.dir * q for leg, q in zip(legs, qs)) - flux
        if (s % modulus == 0) if modulus else s == 0:
            out.append(tuple(qs))
    return out


def block_shape(legs, qs):
    return tuple(leg.dim(q) for leg, q in zip(legs, qs))


def block_slices(legs, qs):
    return tuple(slice(leg.offsets()[q], leg.offsets()[q] + leg.dim(q)) for leg, q in zip(legs, qs))


def nnz(legs, flux, modulus=0):
    return int(sum(np.prod(block_shape(legs, b)) for b in allowed_blocks(legs, flux, modulus)))


def embed(legs, flux, values, modulus=0):
    """Dense FP64 array whose allowed blocks hold ``values`` in canonical
    block order, row-major inside each block; zero elsewhere."""
    values = np.asarray(values, dtype=np.float64)
    dense = np.zeros([leg.size for leg in legs])
    pos = 0
    for b in allowed_blocks(legs, flux, modulus):
        shp = block_shape(legs, b)
        n = int(np.prod(shp))
        dense[block_slices(legs, b)] = values[pos:pos + n].reshape(shp)
        pos += n
    if pos != values.size:
        raise ValueError(f"embed: {values.size} values for {pos} allowed entries")
    return dense


def conserving_mask(legs, flux, modulus=0):
    """Boolean array, True where the state charges obey the addition rule
    (modulo `modulus` for Z_n charges, e.g. 2 for parities)."""
    tot = np.zeros([leg.size for leg in legs], dtype=np.int64)
    for ax, leg in enumerate(legs):
        shape = [1] * len(legs)
        shape[ax] = leg.size
        tot = tot + leg.dir * leg.state_charges().reshape(shape)
    return (tot - flux) % modulus == 0 if modulus else tot == flux


def extract_block(dense, legs, qs):
    return dense[block_slices(legs, qs)]


# --------------------------------------------------------------------------
# Leg fusion
# --------------------------------------------------------------------------

def fuse(leg_a, leg_b, sa, sb, direction, modulus=0):
    """Fuse two legs into one leg with charge Q = sa*q_a + sb*q_b (taken
    modulo `modulus` for Z_n charges).

    Fused states are ordered by Q ascending, then q_a ascending, then
    (i_a, i_b) row-major.  Returns (fused leg, perm) where perm[f] is the
    product-space index i_a * size_b + i_b of fused state f.
    """
    qa, qb = leg_a.state_charges(), leg_b.state_charges()
    entries = []
    for ia in range(leg_a.size):
        for ib in range(leg_b.size):
            Q = sa * qa[ia] + sb * qb[ib]
            entries.append((int(Q % modulus) if modulus else int(Q), qa[ia], ia, ib))
    entries.sort()
    perm = np.array([ia * leg_b.size + ib for _, _, ia, ib in entries], dtype=np.int64)
    sectors = {}
    for Q, _, _, _ in entries:
        sectors[Q] = sectors.get(Q, 0) + 1
    return Leg(sectors, direction), perm


# --------------------------------------------------------------------------
# Workload tensors
# --------------------------------------------------------------------------

class Workload:
    """Legs of one symmetric CTM workload (site + environment), U(1)."""

    def __init__(self, phys, virt, chi, flux=1):
        self.flux_A = int(flux)
        self.phys = Leg(phys, IN)
        v = Leg(virt, IN)
        self.A_legs = [self.phys, Leg(virt, IN), Leg(virt, IN), Leg(virt, OUT), Leg(virt, OUT)]
        # double-layer leg: (ket, bra) fused with Q = q_ket - q_bra
        dd, _ = fuse(v, v, +1, -1, IN)
        self.dd = dd.sectors()
        self.a_legs = [Leg(self.dd, IN), Leg(self.dd, IN), Leg(self.dd, OUT), Leg(self.dd, OUT)]
        self.chi = dict(chi)
        X = self.chi
        self.C_legs = [Leg(X, IN), Leg(X, OUT)]
        self.T_legs = {
            "T1": [Leg(X, IN), Leg(self.dd, OUT), Leg(X, OUT)],
            "T2": [Leg(X, IN), Leg(self.dd, IN), Leg(X, OUT)],
            "T3": [Leg(X, IN), Leg(self.dd, IN), Leg(X, OUT)],
            "T4": [Leg(X, IN), Leg(self.dd, OUT), Leg(X, OUT)],
        }

    def legs_of(self, name):
        if name == "A":
            return self.A_legs, self.flux_A
        if name.startswith("C"):
            return self.C_legs, 0
        return self.T_legs[name], 0

    def nnz_of(self, name):
        legs, flux = self.legs_of(name)
        return nnz(legs, flux)

    def dense_tensors(self, values):
        """values: dict name -> flat FP64 values in canonical block order."""
        out = {}
        for name, vals in values.items():
            legs, flux = self.legs_of(name)
            out[name] = embed(legs, flux, vals)
        return out


def double_layer(A, A_legs, modulus=0):
    """a = sum_sigma A[sigma,...] A*[sigma,...] with every (ket, bra) pair of
    virtual legs fused into one leg of charge q_ket - q_bra (Sec. 3.2: the
    rank-4 double-layer tensor).  A is real, so A* = A."""
    a8 = np.einsum("sabcd,sefgh->aebfcgdh", A, A)
    perms, legs = [], []
    for leg in A_legs[1:]:
        F, p = fuse(leg, leg, +1, -1, leg.dir, modulus)
        perms.append(p)
        legs.append(F)
    n = [leg.size for leg in A_legs[1:]]
    a4 = a8.reshape(n[0] * n[0], n[1] * n[1], n[2] * n[2], n[3] * n[3])
    return a4[np.ix_(*perms)], legs


def double_layer_op(A, A_legs, op, modulus=0):
    """The double layer with a one-site operator between the layers:
    b = sum over (s_bra, s_ket) of op[s_bra, s_ket] A[s_ket, ...] (ket)
    A[s_bra, ...] (bra), legs fused as in double_layer; for real A the
    network with b in place of a gives <psi|O|psi> (Sec. 3's expectation
    values)."""
    b8 = np.einsum("tk,kabcd,tefgh->aebfcgdh", op, A, A)
    perms = [fuse(leg, leg, +1, -1, leg.dir, modulus)[1] for leg in A_legs[1:]]
    n = [leg.size for leg in A_legs[1:]]
    b4 = b8.reshape(n[0] * n[0], n[1] * n[1], n[2] * n[2], n[3] * n[3])
    return b4[np.ix_(*perms)]


def spin_operators(phys_leg):
    """Sz, S+, S- on a physical leg with charges 2m, m = -S..S (one state
    each, charge order), as matrices [bra, ket]."""
    ms = [q / 2.0 for q in phys_leg.charges]
    assert phys_leg.dims == [1] * len(ms) and all(b - a == 1.0 for a, b in zip(ms, ms[1:]))
    S = ms[-1]
    n = len(ms)
    sz, sp = np.diag(ms), np.zeros((n, n))
    for k in range(n - 1):
        sp[k + 1, k] = np.sqrt(S * (S + 1) - ms[k] * (ms[k] + 1))
    return sz, sp, sp.T.copy()


# --------------------------------------------------------------------------
# Enlarged corners, halves, projectors, renormalisation
# --------------------------------------------------------------------------
#
# Fat bonds pair a chi leg with a D2 leg.  The fused charge of a fat bond is
# Q = q_chi - q_D2 where the chi leg and the D2 leg flow in opposite senses
# (left and bottom bonds), and Q = q_chi + q_D2 where they flow the same way
# (top and right bonds).  Fused order: Q, then q_chi, then (i_chi, i_D2).

def _fat(w, rule):
    chi_leg = Leg(w.chi, IN)
    dd_leg = Leg(w.dd, IN)
    s = -1 if rule == "diff" else +1
    return fuse(chi_leg, dd_leg, +1, s, IN)


def enlarged_corners(w, T, a):
    """Dense enlarged corners as rank-4 arrays.

    C~1[x4, d, x1, r] = C1[xa, xb] T1[xb, u, x1] T4[x4, l, xa] a[l, u, r, d]
    C~2[x1, l, x2, d] = C2[xb, xc] T1[x1, u, xb] T2[xc, r, x2] a[l, u, r, d]
    C~3[x2, u, x3, l] = C3[xe, xf] T2[x2, r, xe] T3[xf, d, x3] a[l, u, r, d]
    C~4[x4, u, x3, r] = C4[xc, xd] T4[xd, l, x4] T3[x3, d, xc] a[l, u, r, d]
    """
    def e(spec, *ops):   # two operands at a time, BLAS-backed
        return np.einsum(spec, *ops, optimize="optimal")
    c1 = e("yxlu,lurd->ydxr", e("aux,yla->yxlu", e("ab,bux->aux", T["C1"], T["T1"]), T["T4"]), a)
    c2 = e("xzur,lurd->xlzd", e("cxu,crz->xzur", e("bc,xub->cxu", T["C2"], T["T1"]), T["T2"]), a)
    c3 = e("zydr,lurd->yuzl", e("edz,yre->zydr", e("ef,fdz->edz", T["C3"], T["T3"]), T["T2"]), a)
    c4 = e("zDly,lurD->yuzr", e("qzD,qly->zDly", e("pq,zDp->qzD", T["C4"], T["T3"]), T["T4"]), a)
    return c1, c2, c3, c4


def corner_matrices(w, corners):
    """Fuse each enlarged corner into a matrix (rows, cols) over fat bonds.

    C~1: rows left-cut (diff), cols top bond (sum)
    C~2: rows top bond (sum), cols right cut (sum)
    C~3: rows right cut (sum), cols bottom bond (diff)
    C~4: rows left-cut (diff), cols bottom bond (diff)
    """
    Fd, pd = _fat(w, "diff")
    Fs, ps = _fat(w, "sum")
    c1, c2, c3, c4 = corners
    n = c1.shape[0] * c1.shape[1]

    def mat(c, pr, pc):
        return c.reshape(n, n)[np.ix_(pr, pc)]

    return (mat(c1, pd, ps), mat(c2, ps, ps), mat(c3, ps, pd), mat(c4, pd, pd)), Fd, Fs


def halves(M1, M2, M3, M4):
    """Upper half H_u = C~1 C~2 and lower half H_d = C~4 C~3^T, both with
    rows on the left cut and columns on the right cut."""
    return M1 @ M2, M4 @ M3.T


def projectors(Hu, Hd, F_left, F_right, chi, cutoff=TRUNC_REL_CUTOFF):
    """QR/SVD projectors for the left cut, per fused charge Q.

    H_u^T = Q_u R_u, H_d^T = Q_d R_d, M = R_u R_d^T = U S V^T; keep the chi
    largest singular values over all sectors (ties: charge ascending, then
    index ascending; values <= cutoff*s_max dropped);
    P = R_d^T V S^-1/2 (attached below the upper half),
    P~ = S^-1/2 U^T R_u (attached above the lower half).
    Sign gauge: the largest-magnitude entry of each row of P~ is positive
    (lowest index on ties).
    """
    offL, offR = F_left.offsets(), F_right.offsets()
    per_Q = {}
    for Q in F_left.charges:
        n = F_left.dim(Q)
        m = F_right.dim(Q)
        if m == 0:
            continue
        rs = slice(offL[Q], offL[Q] + n)
        cs = slice(offR[Q], offR[Q] + m)
        _, Ru = np.linalg.qr(Hu[rs, cs].T)
        _, Rd = np.linalg.qr(Hd[rs, cs].T)
        Mq = Ru @ Rd.T
        U, s, Vt = np.linalg.svd(Mq)
        per_Q[Q] = dict(Ru=Ru, Rd=Rd, M=Mq, U=U, s=s, V=Vt.T, n=n)
    allsv = sorted(((-s, Q, j) for Q, d in per_Q.items() for j, s in enumerate(d["s"])))
    s_max = -allsv[0][0] if allsv else 0.0
    kept = [(Q, j) for (ms, Q, j) in allsv[:chi] if -ms > cutoff * s_max]
    # a set of (near-)degenerate values is never split at the cut: values
    # within DEGENERATE_REL of the last kept one are dropped with it
    n = len(kept)
    while 1 < n < len(allsv) and -allsv[n][0] >= (1.0 - DEGENERATE_REL) * (-allsv[n - 1][0]):
        n -= 1
    kept = kept[:n]
    kept_set = set(kept)
    discarded = [-ms for (ms, Q, j) in allsv if (Q, j) not in kept_set]
    tot = sum(ms * ms for (ms, _, _) in allsv)
    trunc_err = float(sum(x * x for x in discarded) / tot) if tot > 0 else 0.0
    if discarded and kept:
        s_last = min(per_Q[Q]["s"][j] for Q, j in kept)
        gap = float((s_last - max(discarded)) / s_max)
    else:
        gap = float("inf")
    kept_per_Q = {}
    for Q, j in kept:
        kept_per_Q.setdefault(Q, []).append(j)
    new_leg = Leg({Q: len(v) for Q, v in kept_per_Q.items()}, IN)
    ntot = F_left.size
    k_off = new_leg.offsets()
    P = np.zeros((ntot, new_leg.size))
    Pt = np.zeros((new_leg.size, ntot))
    blocks = {}
    for Q, js in kept_per_Q.items():
        js = sorted(js)
        d = per_Q[Q]
        sq = np.sqrt(d["s"][js])
        Pq = d["Rd"].T @ d["V"][:, js] / sq
        Ptq = (d["U"][:, js] / sq).T @ d["Ru"]
        for k in range(len(js)):
            row = Ptq[k]
            i = int(np.argmax(np.abs(row)))
            if row[i] < 0:
                Ptq[k] *= -1.0
                Pq[:, k] *= -1.0
        r0 = offL[Q]
        P[r0:r0 + d["n"], k_off[Q]:k_off[Q] + len(js)] = Pq
        Pt[k_off[Q]:k_off[Q] + len(js), r0:r0 + d["n"]] = Ptq
        blocks[Q] = (Pq, Ptq)
    svals = {Q: d["s"].copy() for Q, d in per_Q.items()}
    return dict(P=P, Pt=Pt, new_leg=new_leg, kept={Q: len(v) for Q, v in kept_per_Q.items()},
                svals=svals, trunc_err=trunc_err, gap=gap, s_max=s_max, per_Q=per_Q, blocks=blocks)


def renormalise(w, T, a, P, Pt):
    """C1' = (C1 T1) P,  T4' = P~ (T4 a) P,  C4' = P~ (C4 T3); each then
    scaled to unit Frobenius norm.  Leg orders: C1'[k, x1], T4'[k_lo, r, k_hi],
    C4'[x3, k]."""
    Fd, pd = _fat(w, "diff")
    nX = Leg(w.chi, IN).size
    nD = Leg(w.dd, IN).size
    CT = np.einsum("ab,bux->aux", T["C1"], T["T1"])
    CTm = CT.reshape(nX * nD, nX)[pd]
    C1n = P.T @ CTm
    # T4' = P~ (T4 a) P with the fat bonds unfused: rows of P and columns of
    # P~ back in (chi, D2) product order; the pairwise contractions take P~
    # first, so that no (chi D2)^2 D2 array is formed (84 GB at D = 8,
    # chi = 200)
    k = P.shape[1]
    P3 = np.zeros((nX * nD, k))
    P3[pd] = P
    P3 = P3.reshape(nX, nD, k)                 # [y, d, k]
    Pt3 = np.zeros((k, nX * nD))
    Pt3[:, pd] = Pt
    Pt3 = Pt3.reshape(k, nX, nD)               # [h, x, u]
    Z1 = np.einsum("hxu,ylx->huyl", Pt3, T["T4"], optimize=True)
    Z2 = np.einsum("huyl,lurd->hyrd", Z1, a, optimize=True)
    T4n = np.einsum("hyrd,ydk->krh", Z2, P3, optimize=True)
    C4T3 = np.einsum("pq,zDp->zqD", T["C4"], T["T3"]).reshape(nX, nX * nD)[:, pd]
    C4n = C4T3 @ Pt.T
    norms = [np.linalg.norm(C1n), np.linalg.norm(T4n), np.linalg.norm(C4n)]
    return C1n / norms[0], T4n / norms[1], C4n / norms[2], norms


def left_column(C1n, T4n, C4n):
    """Gauge-invariant left column L[x1, r, x3] = C1'[k1, x1] T4'[k2, r, k1] C4'[x3, k2]."""
    return np.einsum("ax,bra,zb->xrz", C1n, T4n, C4n)


def ctm_left_move(w, T, a, chi):
    """One CTM left move on dense tensors; returns every intermediate."""
    corners = enlarged_corners(w, T, a)
    (M1, M2, M3, M4), Fd, Fs = corner_matrices(w, corners)
    Hu, Hd = halves(M1, M2, M3, M4)
    pr = projectors(Hu, Hd, Fd, Fs, chi)
    C1n, T4n, C4n, norms = renormalise(w, T, a, pr["P"], pr["Pt"])
    return dict(corners=corners, mats=(M1, M2, M3, M4), F_left=Fd, F_top=Fs,
                Hu=Hu, Hd=Hd, proj=pr, C1=C1n, T4=T4n, C4=C4n, norms=norms,
                Pi=pr["P"] @ pr["Pt"], L=left_column(C1n, T4n, C4n))


# --------------------------------------------------------------------------
# Integer bookkeeping by brute force (Sec. 2: pairs of blocks with identical
# labels on the contracted legs; results grouped by output labels)
# --------------------------------------------------------------------------

class Struct:
    """Legs plus an explicit list of present blocks (charge tuples)."""

    def __init__(self, legs, blocks):
        self.legs = list(legs)
        self.blocks = sorted(set(tuple(b) for b in blocks))

    @classmethod
    def allowed(cls, legs, flux):
        return cls(legs, allowed_blocks(legs, flux))

    def nnz(self):
        return int(sum(np.prod(block_shape(self.legs, b)) for b in self.blocks))


def pair_table(SA, SB, conA, conB):
    """All (A block, B block) pairs with identical charges on the contracted
    legs; output blocks are their free-charge tuples (A free legs, then B free
    legs); flops = sum over pairs of 2*m*n*k."""
    freeA = [i for i in range(len(SA.legs)) if i not in conA]
    freeB = [j for j in range(len(SB.legs)) if j not in conB]
    pairs, outs, flops = [], {}, 0
    for ta in SA.blocks:
        for tb in SB.blocks:
            if all(ta[i] == tb[j] for i, j in zip(conA, conB)):
                o = tuple(ta[i] for i in freeA) + tuple(tb[j] for j in freeB)
                m = int(np.prod([SA.legs[i].dim(ta[i]) for i in freeA]))
                k = int(np.prod([SA.legs[i].dim(ta[i]) for i in conA]))
                n = int(np.prod([SB.legs[j].dim(tb[j]) for j in freeB]))
                pairs.append((ta, tb))
                outs.setdefault(o, []).append((ta, tb))
                flops += 2 * m * n * k
    out_legs = [SA.legs[i] for i in freeA] + [SB.legs[j] for j in freeB]
    return dict(pairs=pairs, outputs=outs, flops=flops,
                out=Struct(out_legs, list(outs.keys())))


def double_layer_table(w):
    """Outer products of the double layer: A blocks paired on the physical
    charge (K = size of that sector)."""
    SA = Struct.allowed(w.A_legs, w.flux_A)
    pairs = [(ta, tb) for ta in SA.blocks for tb in SA.blocks if ta[0] == tb[0]]
    outs = set()
    for ta, tb in pairs:
        outs.add(tuple(ta[i] - tb[i] for i in range(1, 5)))
    return dict(n_pairs=len(pairs), n_out=len(outs), A_blocks=len(SA.blocks), A_nnz=SA.nnz(),
                a=Struct.allowed(w.a_legs, 0))


def corner_tables(w, which=1):
    """Pair tables of the three steps of one enlarged corner.

    C~1 = ((C1 T1) T4) a ; C~2 = ((C2 T1) T2) a ;
    C~3 = ((C3 T3) T2) a ; C~4 = ((C4 T3) T4) a .
    """
    C = Struct.allowed(w.C_legs, 0)
    T = {k: Struct.allowed(v, 0) for k, v in w.T_legs.items()}
    a = Struct.allowed(w.a_legs, 0)
    if which == 1:
        # C1[xa,xb].T1[xb,u,x1] -> [xa,u,x1]; .T4[y,l,xa] -> [u,x1,y,l]; .a[l,u,r,d] over (l,u)
        s1 = pair_table(C, T["T1"], [1], [0])
        s2 = pair_table(s1["out"], T["T4"], [0], [2])
        s3 = pair_table(s2["out"], a, [3, 0], [0, 1])
    elif which == 2:
        # C2[xb,xc].T1[x1,u,xb] over xb -> [xc,x1,u]; .T2[xc,r,x2] -> [x1,u,r,x2]; .a over (u,r)
        s1 = pair_table(C, T["T1"], [0], [2])
        s2 = pair_table(s1["out"], T["T2"], [0], [0])
        s3 = pair_table(s2["out"], a, [1, 2], [1, 2])
    elif which == 3:
        # C3[xe,xf].T3[xf,d,x3] -> [xe,d,x3]; .T2[x2,r,xe] -> [d,x3,x2,r]; .a over (r,d)
        s1 = pair_table(C, T["T3"], [1], [0])
        s2 = pair_table(s1["out"], T["T2"], [0], [2])
        s3 = pair_table(s2["out"], a, [3, 0], [2, 3])
    else:
        # C4[xc,xd].T3[x3,d,xc] over xc -> [xd,x3,d]; .T4[xd,l,x4] -> [x3,d,l,x4]; .a over (l,d)
        s1 = pair_table(C, T["T3"], [0], [2])
        s2 = pair_table(s1["out"], T["T4"], [0], [0])
        s3 = pair_table(s2["out"], a, [2, 1], [0, 3])
    return [s1, s2, s3]


def fused_sectors(w, rule):
    F, _ = _fat(w, rule)
    return F.sectors()


def corner_output_struct(w, which):
    """Block structure of an enlarged corner as produced by its third step.

    Leg orders: C~1 [x1, x4, r, d], C~2 [x1, x2, l, d], C~3 [x3, x2, l, u],
    C~4 [x3, x4, u, r] (free legs of the chi-side operand, then of a)."""
    return corner_tables(w, which)[2]["out"]


def projector_structs(w, kept):
    """P[chi(out), D2(in), k(in)] and P~[k(out), chi(in), D2(out)] as block
    structures (all blocks of charge-conserving labels for the kept sectors)."""
    k_in = Leg(kept, IN)
    k_out = Leg(kept, OUT)
    P = Struct.allowed([Leg(w.chi, OUT), Leg(w.dd, IN), k_in], 0)
    Pt = Struct.allowed([k_out, Leg(w.chi, IN), Leg(w.dd, OUT)], 0)
    return P, Pt


def move_tables(w, kept):
    """Pair tables of every block-sparse contraction of one left move.

    corners: three steps each for C~1..C~4;
    halves:  H_u = C~1 . C~2 over the top bond, H_d = C~4 . C~3 over the
             bottom bond;
    renorm:  C1' = (C1 T1) . P ;  X1 = P~ . T4 ;  X2 = X1 . a ;
             T4' = X2 . P ;  C4' = (C4 T3) . P~ ,
             with C1 T1 and C4 T3 reused from the first corner steps (the
             order fixes which block pairs exist, hence the flop count; the
             dense result of renormalise() does not depend on it).
    """
    corners = {c: corner_tables(w, c) for c in (1, 2, 3, 4)}
    c1 = corners[1][2]["out"]   # [x1, x4, r, d]
    c2 = corners[2][2]["out"]   # [x1, x2, l, d]
    c3 = corners[3][2]["out"]   # [x3, x2, l, u]
    c4 = corners[4][2]["out"]   # [x3, x4, u, r]
    hu = pair_table(c1, c2, [0, 2], [0, 2])   # -> [x4, d, x2, d2]
    hd = pair_table(c4, c3, [0, 3], [0, 2])   # -> [x4, u, x2, u3]
    P, Pt = projector_structs(w, kept)
    CT = corners[1][0]["out"]                 # [xa, u, x1]
    C4T3 = corners[4][0]["out"]               # [xd, x3, d]
    r_c1 = pair_table(CT, P, [0, 1], [0, 1])  # -> [x1, k]
    T4s = Struct.allowed(w.T_legs["T4"], 0)   # [y, l, x]
    a = Struct.allowed(w.a_legs, 0)
    r_x1 = pair_table(Pt, T4s, [1], [2])                # -> [k_hi, u, y, l]
    r_x2 = pair_table(r_x1["out"], a, [1, 3], [1, 0])   # -> [k_hi, y, r, d]
    r_t4 = pair_table(r_x2["out"], P, [1, 3], [0, 1])   # -> [k_hi, r, k_lo]
    r_c4 = pair_table(C4T3, Pt, [0, 2], [1, 2])         # -> [x3, k]
    return dict(corners=corners, hu=hu, hd=hd,
                renorm=dict(C1=r_c1, X1=r_x1, X2=r_x2, T4=r_t4, C4=r_c4))


def move_gemm_flops(w, kept):
    """Useful flops (sum over matched block pairs of 2 m n k) of the GEMM
    phases of one left move: corners, halves and renormalisation.  The FP64
    product M = R_u R_d^T belongs to the projector stage and is not counted."""
    t = move_tables(w, kept)
    corners = sum(s["flops"] for c in t["corners"].values() for s in c)
    halves_ = t["hu"]["flops"] + t["hd"]["flops"]
    renorm = sum(v["flops"] for v in t["renorm"].values())
    return dict(corners=corners, halves=halves_, renorm=renorm,
                total=corners + halves_ + renorm)
