"""SU(2) reduced tensors expanded into dense FP64 arrays.

TEST INFRASTRUCTURE ONLY: used by tests/ to check the library's SU(2)
reduced path; never by the product library.

A symmetric tensor is a sum of blocks t_i = m_i (x) c_i, a dense reduced
tensor times a generalised Clebsch-Gordan tensor (Sec. 2, Eq. tensor-cgc).
Here every block carries one spin per leg and one coupling tree, and c_i is
the canonical basis tensor of that tree:

* the incoming legs, in leg order, are coupled left to right by ordinary
  Clebsch-Gordan coefficients, j_1 x j_2 -> k_2, k_2 x j_3 -> k_3, ... -> K;
* the outgoing legs likewise -> K (the same total spin: the tensor is
  invariant, no quantum-number shift, Sec. 2);
* c[m_1..m_R] = sum_M C_in(m_in; K M) C_out(m_out; K M).

Spins are stored doubled (tj = 2j).  Leg states are ordered by (j, copy a,
m ascending).  Expanding an SU(2) tensor gives a U(1)-symmetric tensor in the
charge 2m (the abelian counterpart of Sec. 2's rank-2 example).
"""
import itertools
from fractions import Fraction
from functools import lru_cache

import numpy as np

from . import u1

IN, OUT = +1, -1


@lru_cache(maxsize=None)
def cg(tj1, tm1, tj2, tm2, tJ, tM):
    """<j1 m1; j2 m2 | J M> (Condon-Shortley), arguments doubled, exact
    (sympy) then rounded to FP64."""
    if tm1 + tm2 != tM:
        return 0.0
    if not (abs(tj1 - tj2) <= tJ <= tj1 + tj2) or (tj1 + tj2 + tJ) % 2:
        return 0.0
    if abs(tm1) > tj1 or abs(tm2) > tj2 or abs(tM) > tJ:
        return 0.0
    from sympy.physics.quantum.cg import CG
    from sympy import Rational
    h = lambda x: Rational(x, 2)
    return float(CG(h(tj1), h(tm1), h(tj2), h(tm2), h(tJ), h(tM)).doit())


def ms(tj):
    return list(range(-tj, tj + 1, 2))


class Leg:
    """SU(2) leg: multiplets {tj: n} (n copies of spin tj/2) and a direction."""

    def __init__(self, sectors, direction):
        items = sorted((int(t), int(n)) for t, n in dict(sectors).items() if int(n) > 0)
        self.tjs = [t for t, _ in items]
        self.mult = [n for _, n in items]
        self.dir = int(direction)

    def sectors(self):
        return dict(zip(self.tjs, self.mult))

    def n(self, tj):
        return self.sectors().get(tj, 0)

    @property
    def size(self):
        return int(sum(n * (t + 1) for t, n in zip(self.tjs, self.mult)))

    @property
    def reduced_size(self):
        return int(sum(self.mult))

    def offsets(self):
        """Offset of the first state of each spin sector."""
        out, o = {}, 0
        for t, n in zip(self.tjs, self.mult):
            out[t] = o
            o += n * (t + 1)
        return out

    def states(self):
        """(tj, a, tm) of every state in order."""
        return [(t, a, m) for t, n in zip(self.tjs, self.mult) for a in range(n) for m in ms(t)]

    def u1_leg(self):
        """The abelian leg this one expands to: charge 2m, dims summed over j."""
        sec = {}
        for t, n in zip(self.tjs, self.mult):
            for m in ms(t):
                sec[m] = sec.get(m, 0) + n
        return u1.Leg(sec, self.dir)

    def u1_perm(self):
        """perm[k] = SU(2)-order index of the k-th state in U(1) order
        (charge ascending, then SU(2) order)."""
        st = self.states()
        return np.array(sorted(range(len(st)), key=lambda i: (st[i][2], i)), dtype=np.int64)


def chains(tjs):
    """All coupling chains of spins tjs (left to right): lists
    [k_1=tj_1, k_2, ..., k_r]; an empty list of spins gives [[0]]."""
    if not tjs:
        return [[0]]
    out = [[tjs[0]]]
    for t in tjs[1:]:
        nxt = []
        for c in out:
            k = c[-1]
            for K in range(abs(k - t), k + t + 1, 2):
                nxt.append(c + [K])
        out = nxt
    return out


def blocks(legs):
    """Canonical block list: (spins per leg, tree) lexicographic, where tree
    = (in-chain intermediates k_2..k_{r-1}, out-chain intermediates, K)."""
    ins = [i for i, l in enumerate(legs) if l.dir == IN]
    outs = [i for i, l in enumerate(legs) if l.dir == OUT]
    res = []
    for tj in itertools.product(*[l.tjs for l in legs]):
        ci = chains([tj[i] for i in ins])
        co = chains([tj[i] for i in outs])
        for a in ci:
            for b in co:
                if a[-1] != b[-1]:
                    continue
                tree = tuple(a[1:-1]) + tuple(b[1:-1]) + (a[-1],)
                res.append((tuple(tj), tree))
    return sorted(res)


def _chain_tensor(tjs, chain):
    """C(m_1..m_r; K M) as an array [m_1, ..., m_r, M] for one chain; for no
    spins, the scalar state K = M = 0 as an array [M] = [1]."""
    if not tjs:
        return np.ones(1)
    K = chain[-1]
    C = np.zeros([t + 1 for t in tjs] + [K + 1])
    for mm in itertools.product(*[ms(t) for t in tjs]):
        val, mu = 1.0, mm[0]
        for s in range(1, len(tjs)):
            nmu = mu + mm[s]
            val *= cg(chain[s - 1], mu, tjs[s], mm[s], chain[s], nmu)
            if val == 0.0:
                break
            mu = nmu
        if val != 0.0 and abs(mu) <= K:
            idx = tuple((m + t) // 2 for m, t in zip(mm, tjs)) + ((mu + K) // 2,)
            C[idx] = val
    return C


def _chain(tjs, mid, K):
    if not tjs:
        return [0]
    if len(tjs) == 1:
        return [tjs[0]]
    return [tjs[0]] + list(mid) + [K]


def cgc_tensor(legs, tj, tree):
    """Canonical basis tensor c[m_1..m_R] of block (tj, tree)."""
    ins = [i for i, l in enumerate(legs) if l.dir == IN]
    outs = [i for i, l in enumerate(legs) if l.dir == OUT]
    K = tree[-1]
    ni_mid, no_mid = max(0, len(ins) - 2), max(0, len(outs) - 2)
    tin = [tj[i] for i in ins]
    tout = [tj[i] for i in outs]
    Cin = _chain_tensor(tin, _chain(tin, tree[:ni_mid], K))
    Cout = _chain_tensor(tout, _chain(tout, tree[ni_mid:ni_mid + no_mid], K))
    # c[m_in, m_out] = sum_M Cin[m_in, M] Cout[m_out, M]
    cc = Cin.reshape(-1, K + 1) @ Cout.reshape(-1, K + 1).T
    cc = cc.reshape([t + 1 for t in tin] + [t + 1 for t in tout])
    return cc.transpose(np.argsort(ins + outs))


def nnz(legs):
    return int(sum(np.prod([l.n(t) for l, t in zip(legs, tj)]) for tj, _ in blocks(legs)))


def expand(legs, values):
    """Dense FP64 array (SU(2) state order) of the tensor whose reduced
    blocks hold `values` (canonical block order, row-major per block)."""
    values = np.asarray(values, dtype=np.float64)
    dense = np.zeros([l.size for l in legs])
    pos = 0
    for tj, tree in blocks(legs):
        shp = [l.n(t) for l, t in zip(legs, tj)]
        k = int(np.prod(shp))
        m = values[pos:pos + k].reshape(shp)
        pos += k
        c = cgc_tensor(legs, tj, tree)
        # t[(a_1,m_1),...] = m[a_1..] c[m_1..]
        t = np.multiply.outer(m, c)                       # [a_1..a_R, m_1..m_R]
        R = len(legs)
        t = t.transpose([x for i in range(R) for x in (i, R + i)])
        t = t.reshape([s * (tt + 1) for s, tt in zip(shp, tj)])
        sl = tuple(slice(l.offsets()[t_], l.offsets()[t_] + l.n(t_) * (t_ + 1)) for l, t_ in zip(legs, tj))
        dense[sl] += t
    if pos != values.size:
        raise ValueError(f"expand: {values.size} values for {pos} reduced entries")
    return dense


def to_u1(dense, legs):
    """Re-order every leg into the U(1) state order; returns (array, U(1) legs)."""
    out = dense
    for ax, l in enumerate(legs):
        out = np.take(out, l.u1_perm(), axis=ax)
    return out, [l.u1_leg() for l in legs]


def wigner_d(tj, beta):
    """Real Wigner small-d matrix d^j_{m'm}(beta) (rotation about y), states
    m ascending, from the standard closed form."""
    from math import factorial, cos, sin
    j = Fraction(tj, 2)
    mlist = ms(tj)
    d = np.zeros((tj + 1, tj + 1))
    for a, tmp in enumerate(mlist):
        for b, tm in enumerate(mlist):
            mp, m = Fraction(tmp, 2), Fraction(tm, 2)
            pref = (factorial(int(j + mp)) * factorial(int(j - mp)) * factorial(int(j + m)) * factorial(int(j - m))) ** 0.5
            s = 0.0
            for k in range(0, tj + 1):
                n1, n2, n3, n4 = j + m - k, k, j - k - mp, k - m + mp
                if min(n1, n2, n3, n4) < 0:
                    continue
                num = (-1) ** int(k - m + mp)
                den = factorial(int(n1)) * factorial(int(n2)) * factorial(int(n3)) * factorial(int(n4))
                s += num / den * cos(beta / 2) ** int(2 * j + m - mp - 2 * k) * sin(beta / 2) ** int(mp - m + 2 * k)
            d[a, b] = pref * s
    return d


def rotate(dense, legs, beta):
    """Apply the y-rotation d(beta) to every leg of a dense SU(2)-ordered tensor."""
    out = dense
    for ax, l in enumerate(legs):
        D = np.zeros((l.size, l.size))
        o = 0
        for t, n in zip(l.tjs, l.mult):
            d = wigner_d(t, beta)
            for a in range(n):
                D[o:o + t + 1, o:o + t + 1] = d
                o += t + 1
        out = np.moveaxis(np.tensordot(D, out, axes=([1], [ax])), 0, ax)
    return out


def reduce(legs, dense):
    """Reduced block values (canonical order, row-major per block) of a dense
    SU(2)-ordered tensor: each block is the projection onto its basis tensor,
    m[a..] = sum_m c[m..] t[(a,m)..] / <c, c>.  Inverse of `expand` on
    invariant tensors."""
    dense = np.asarray(dense, dtype=np.float64)
    R = len(legs)
    out = []
    for tj, tree in blocks(legs):
        shp = [l.n(t) for l, t in zip(legs, tj)]
        sl = tuple(slice(l.offsets()[t], l.offsets()[t] + l.n(t) * (t + 1)) for l, t in zip(legs, tj))
        sub = dense[sl].reshape([x for s, t in zip(shp, tj) for x in (s, t + 1)])
        sub = sub.transpose(list(range(0, 2 * R, 2)) + list(range(1, 2 * R, 2)))   # [a.., m..]
        c = cgc_tensor(legs, tj, tree)
        m = np.tensordot(sub, c, axes=(list(range(R, 2 * R)), list(range(R)))) / np.sum(c * c)
        out.append(m.reshape(-1))
    return np.concatenate(out) if out else np.zeros(0)


def invariant_count(tjs):
    """Number of independent invariant tensors on legs of spins tjs: the
    multiplicity of total spin 0 in their product, from S^z state counts
    (states with total M = 0 minus those with M = 1, in doubled units 0 and 2)."""
    counts = {0: 1}
    for t in tjs:
        nxt = {}
        for M, c in counts.items():
            for m in ms(t):
                nxt[M + m] = nxt.get(M + m, 0) + c
        counts = nxt
    return counts.get(0, 0) - counts.get(2, 0)


def fuse(la, lb, direction):
    """Multiplets of the product of two legs (j_a x j_b -> J for every pair)."""
    sec = {}
    for ta, na in zip(la.tjs, la.mult):
        for tb, nb in zip(lb.tjs, lb.mult):
            for J in range(abs(ta - tb), ta + tb + 1, 2):
                sec[J] = sec.get(J, 0) + na * nb
    return Leg(sec, direction)


def fusion_isometry(la, lb, fdir):
    """Unitary F[a, b, f] fusing legs la, lb into one multiplet leg f (dir
    fdir): f's spin-J multiplets are the pairs (multiplet of la with spin ja,
    multiplet of lb with spin jb) with J in ja x jb, ordered by (ja, jb), then
    row-major (i_a, i_b).  Its reduced block (ja, jb, J) is
    sqrt((2J+1)/(2K+1)) times the placement of those pairs, K the root of the
    block's tree.  Returns (legs, reduced values)."""
    nJ, base = {}, {}
    for ja in la.tjs:
        for jb in lb.tjs:
            for J in range(abs(ja - jb), ja + jb + 1, 2):
                base[(ja, jb, J)] = nJ.get(J, 0)
                nJ[J] = nJ.get(J, 0) + la.n(ja) * lb.n(jb)
    lf = Leg(nJ, fdir)
    legs = [la, lb, lf]
    vals = []
    for (ja, jb, J), tree in blocks(legs):
        m = np.zeros((la.n(ja), lb.n(jb), lf.n(J)))
        w = np.sqrt((J + 1) / (tree[-1] + 1))
        for x in range(la.n(ja)):
            for y in range(lb.n(jb)):
                m[x, y, base[(ja, jb, J)] + x * lb.n(jb) + y] = w
        vals.append(m.ravel())
    return legs, np.concatenate(vals)


def double_layer(A_legs, A_values):
    """a[L, U, R, D] = sum_s A[s, l, u, r, d] A*[s, l', u', r', d'] with each
    (ket, bra) pair fused into one multiplet leg (Sec. 3.2's rank-4 double
    layer).  A* is A (real) with every leg reversed, so the bra leg of a bond
    runs opposite to its ket leg; the fusion tensor of a bond with ket leg v
    has legs (v reversed, v, fused with v's direction).  Returns (a legs,
    reduced values, dense a in SU(2) state order)."""
    A = expand(A_legs, A_values)
    a8 = np.einsum("sabcd,sefgh->aebfcgdh", A, A)      # [l, l', u, u', r, r', d, d']
    out, a_legs = a8, []
    for v in A_legs[1:]:
        Fl, Fv = fusion_isometry(Leg(v.sectors(), -v.dir), Leg(v.sectors(), v.dir), v.dir)
        F = expand(Fl, Fv)                             # [ket, bra, fused]
        out = np.tensordot(out, F, axes=([0, 1], [0, 1]))   # consumes the leading pair, appends fused
        a_legs.append(Fl[2])
    return a_legs, reduce(a_legs, out), out
