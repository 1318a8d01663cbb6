"""Thin Python binding over libsymten's C ABI: argument marshalling only.

Every step of the hot path (block enumeration, planning, gathers, sector
GEMMs, projectors, normalisation) runs inside libsymten; this module only
converts Python lists and numpy arrays to the C types of include/symten.h.
"""
import ctypes as C

import numpy as np

from . import _lib
from ._lib import check, lib, SymtenError, PREC

IN, OUT = 1, -1


def _stream(stream):
    """A HIP stream handle: the caller's, else torch's current stream when a
    GPU is visible, else the default stream."""
    if stream is not None:
        return C.c_void_p(int(stream))
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return C.c_void_p(0)


def _ints(xs):
    xs = [int(x) for x in xs]
    return (C.c_int * max(1, len(xs)))(*xs)


def _prec(p):
    return PREC[p] if isinstance(p, str) else int(p)


class Tensor:
    """Handle to a libsymten tensor (owns the handle, shares the storage)."""

    def __init__(self, handle):
        self._h = C.c_void_p(handle) if not isinstance(handle, C.c_void_p) else handle

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().symten_destroy(h)
            except Exception:
                pass
            self._h = None

    @staticmethod
    def _desc(legs, flux, dtype, group="u1"):
        """legs: list of (sectors dict {label: dim}, direction); labels are
        U(1) charges, for group "su2" doubled spins, for group "z2" parities."""
        dirs = [int(d) for _, d in legs]
        nsec = [len(s) for s, _ in legs]
        labels = [int(q) for s, _ in legs for q in s]
        dims = [int(s[q]) for s, _ in legs for q in s]
        keep = (_ints(dirs), _ints(nsec), _ints(labels), _ints(dims))
        dt = _lib.F64 if dtype in ("f64", _lib.F64) else _lib.F32
        g = {"u1": _lib.U1, "su2": _lib.SU2, "z2": _lib.Z2}.get(group, group)
        if g not in (_lib.U1, _lib.SU2, _lib.Z2):
            raise ValueError(f"unknown symmetry group {group!r}")
        d = _lib.Desc(g, len(legs), keep[0], keep[1], keep[2], keep[3], int(flux), dt)
        return d, keep

    @classmethod
    def create(cls, legs, flux=0, dtype="f32", stream=None, group="u1"):
        d, keep = cls._desc(legs, flux, dtype, group)
        h = C.c_void_p()
        check(lib().symten_create(C.byref(h), C.byref(d), _stream(stream)))
        return cls(h)

    @classmethod
    def meta(cls, legs, flux=0, dtype="f32", group="u1"):
        d, keep = cls._desc(legs, flux, dtype, group)
        h = C.c_void_p()
        check(lib().symten_create_meta(C.byref(h), C.byref(d)))
        return cls(h)

    # ---- metadata -------------------------------------------------------
    @property
    def rank(self):
        r = C.c_int()
        check(lib().symten_rank(self._h, C.byref(r)))
        return r.value

    @property
    def flux(self):
        r = C.c_int()
        check(lib().symten_flux(self._h, C.byref(r)))
        return r.value

    @property
    def dtype(self):
        r = C.c_int()
        check(lib().symten_dtype(self._h, C.byref(r)))
        return "f64" if r.value == _lib.F64 else "f32"

    def legs(self):
        out = []
        for l in range(self.rank):
            d, n = C.c_int(), C.c_int()
            check(lib().symten_leg_info(self._h, l, C.byref(d), C.byref(n), None, None))
            lab = (C.c_int * max(1, n.value))()
            dim = (C.c_int * max(1, n.value))()
            check(lib().symten_leg_info(self._h, l, None, None, lab, dim))
            out.append(({int(lab[i]): int(dim[i]) for i in range(n.value)}, d.value))
        return out

    @property
    def num_blocks(self):
        n = C.c_int64()
        check(lib().symten_num_blocks(self._h, C.byref(n)))
        return n.value

    @property
    def nnz(self):
        n = C.c_int64()
        check(lib().symten_nnz(self._h, C.byref(n)))
        return n.value

    def blocks(self):
        """[(labels tuple, shape tuple, offset, strides tuple)] in canonical order."""
        R = self.rank
        out = []
        lab = (C.c_int * R)()
        shp = (C.c_int * R)()
        st = (C.c_int64 * R)()
        off = C.c_int64()
        for i in range(self.num_blocks):
            check(lib().symten_block_info(self._h, i, lab, shp, C.byref(off), st))
            out.append((tuple(lab), tuple(shp), off.value, tuple(st)))
        return out

    def trees(self):
        """SU(2) coupling-tree labels of every block (empty tuples for U(1))."""
        R = self.rank
        buf = (C.c_int * R)()
        n = C.c_int()
        out = []
        for i in range(self.num_blocks):
            check(lib().symten_block_tree(self._h, i, C.byref(n), buf))
            out.append(tuple(buf[k] for k in range(n.value)))
        return out

    def to_u1(self, stream=None):
        """SU(2) tensor -> U(1) tensor of its S^z components (library expansion)."""
        h = C.c_void_p()
        check(lib().symten_su2_to_u1(C.byref(h), self._h, _stream(stream)))
        return Tensor(h)

    def device_ptr(self):
        p, n = C.c_void_p(), C.c_int64()
        check(lib().symten_device_ptr(self._h, C.byref(p), C.byref(n)))
        return p.value, n.value

    @property
    def nbytes(self):
        n = C.c_int64()
        check(lib().symten_nbytes(self._h, C.byref(n)))
        return n.value

    # ---- data -------------------------------------------------------------
    def upload(self, values, stream=None):
        v = np.ascontiguousarray(values, dtype=np.float64)
        check(lib().symten_upload(self._h, v.ctypes.data_as(C.POINTER(C.c_double)), v.size, _stream(stream)))
        return self

    def download(self, stream=None):
        v = np.empty(self.nnz, dtype=np.float64)
        check(lib().symten_download(self._h, v.ctypes.data_as(C.POINTER(C.c_double)), v.size, _stream(stream)))
        return v

    def block_dict(self, stream=None):
        """{labels: ndarray} of the blocks, downloaded."""
        vals = self.download(stream)
        out, pos = {}, 0
        for lab, shp, _, _ in self.blocks():
            n = int(np.prod(shp))
            out[lab] = vals[pos:pos + n].reshape(shp)
            pos += n
        return out


# Callback objects handed to the library stay referenced for the life of the
# process: a buffer may outlive the registration that made it.
_ALLOC_KEEP = []
_ALLOC_ATEXIT = []


def set_allocator(alloc, free):
    """Device memory from alloc(nbytes) -> int address, released by free(address, nbytes).

    Both None: back to the library's own caching pool.  Buffers made under an
    earlier registration are kept, not freed, once another one is made.
    """
    if alloc is None and free is None:
        check(lib().symten_set_allocator(None, None, None))
        return
    if alloc is None or free is None:
        raise ValueError("alloc and free come as a pair")
    a = _lib.ALLOC_FN(lambda n, ctx: alloc(n) or None)
    f = _lib.FREE_FN(lambda ptr, n, ctx: free(ptr, n))
    _ALLOC_KEEP.append((a, f))
    check(lib().symten_set_allocator(C.cast(a, C.c_void_p), C.cast(f, C.c_void_p), None))
    if not _ALLOC_ATEXIT:
        # Before the interpreter (and torch) shut down, stop handing buffers
        # back to Python callables.
        import atexit
        atexit.register(lambda: lib().symten_set_allocator(None, None, None))
        _ALLOC_ATEXIT.append(True)


def use_torch_allocator(device=None, stream=None):
    """Route libsymten's device memory through torch's caching allocator.

    Blocks are tied to `stream` (default: torch's current stream now), so the
    library's calls should be issued on that stream.
    """
    import torch
    dev = torch.cuda.current_device() if device is None else torch.device(device).index
    st = torch.cuda.current_stream(dev) if stream is None else stream
    set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n, dev, st),
                  lambda ptr, n: torch.cuda.caching_allocator_delete(ptr))


def su2_cg(tj1, tm1, tj2, tm2, tJ, tM):
    """The library's Clebsch-Gordan coefficient, arguments doubled."""
    v = C.c_double()
    check(lib().symten_su2_cg(tj1, tm1, tj2, tm2, tJ, tM, C.byref(v)))
    return v.value


def contract(A, B, legsA, legsB, out_perm=None, prec="f32", stream=None):
    h = C.c_void_p()
    perm = _ints(out_perm) if out_perm is not None else None
    check(lib().symten_contract(C.byref(h), A._h, B._h, len(legsA), _ints(legsA), _ints(legsB), perm,
                                _prec(prec), _stream(stream)))
    return Tensor(h)


def contract_noalloc(out, A, B, legsA, legsB, out_perm=None, prec="f32", stream=None):
    """symten_contract written into the existing tensor `out` (the output's
    legs, contiguous blocks) through the library's fixed work area, with no
    device allocation; returns `out`."""
    perm = _ints(out_perm) if out_perm is not None else None
    check(lib().symten_contract_noalloc(out._h, A._h, B._h, len(legsA), _ints(legsA), _ints(legsB), perm,
                                        _prec(prec), _stream(stream)))
    return out


def match_blocks(A, B, legsA, legsB, pair_cap=None, out_cap=None, stream=None):
    """Sector matching of the contraction on the device (symten_match_blocks)
    into torch-allocated device buffers; waits for the stream and returns
    (pairs, out_labels, counts): pairs an int64 array of rows (A block,
    B block, output block, flops), out_labels the output label tuples (A's
    open legs then B's, unpermuted), counts (A blocks, B blocks, pairs,
    output blocks, status)."""
    import numpy as np
    import torch
    na, nb = A.num_blocks, B.num_blocks
    ro = A.rank + B.rank - 2 * len(legsA)
    pair_cap = na * nb if pair_cap is None else int(pair_cap)
    out_cap = max(1, pair_cap) if out_cap is None else int(out_cap)
    pairs = torch.zeros((max(1, pair_cap), 3), dtype=torch.int64, device="cuda")
    outl = torch.zeros((max(1, out_cap), max(1, ro)), dtype=torch.int32, device="cuda")
    counts = torch.zeros(5, dtype=torch.int64, device="cuda")
    check(lib().symten_match_blocks(A._h, B._h, len(legsA), _ints(legsA), _ints(legsB), C.c_void_p(pairs.data_ptr()),
                                    pair_cap, C.c_void_p(outl.data_ptr()), out_cap, C.c_void_p(counts.data_ptr()),
                                    _stream(stream)))
    check(lib().symten_sync(_stream(stream)))
    cnt = counts.cpu().numpy()
    raw = pairs.cpu().numpy()[:min(int(cnt[2]), pair_cap)]
    i32 = raw[:, :2].copy().view(np.int32)          # (a_block, b_block), (out_block, pad)
    rows = np.stack([i32[:, 0], i32[:, 1], i32[:, 2], raw[:, 2]], axis=1) if len(raw) else np.zeros((0, 4), np.int64)
    return rows.astype(np.int64), outl.cpu().numpy()[:min(int(cnt[3]), out_cap), :ro], cnt


def eigh(mats, k, stream=None):
    """FP64 symmetric eigensolver of the projector stage (symten_eigh) on
    torch float64 device matrices (square, symmetric, contiguous; read
    column by column).  k: eigenvectors wanted per matrix (an int or one per
    matrix).  Returns [(w ascending, Z with the eigenvector of the j-th
    largest eigenvalue in column j)], torch device tensors."""
    import torch
    count = len(mats)
    ks = [int(k)] * count if isinstance(k, int) else [int(x) for x in k]
    ws = [torch.empty(m.shape[0], dtype=torch.float64, device=m.device) for m in mats]
    zs = [torch.zeros((max(x, 1), m.shape[0]), dtype=torch.float64, device=m.device) for m, x in zip(mats, ks)]
    P = C.c_void_p
    n = (C.c_int * count)(*[m.shape[0] for m in mats])
    A = (P * count)(*[m.data_ptr() for m in mats])
    W = (P * count)(*[x.data_ptr() for x in ws])
    Z = (P * count)(*[z.data_ptr() for z in zs])
    check(lib().symten_eigh(count, n, A, n, W, (C.c_int * count)(*ks), Z, _stream(stream)))
    check(lib().symten_sync(_stream(stream)))
    # zs rows are columns of the column-major n x k result
    return [(w, z[:x].T) for w, z, x in zip(ws, zs, ks)]


def eigh_max_order():
    n = C.c_int()
    check(lib().symten_eigh_max_order(C.byref(n)))
    return int(n.value)


def plan_info(A, B, legsA, legsB, out_perm=None):
    """Host-only planning; returns (stats dict, metadata-only output Tensor)."""
    st = _lib.PlanStats()
    h = C.c_void_p()
    perm = _ints(out_perm) if out_perm is not None else None
    check(lib().symten_plan_info(A._h, B._h, len(legsA), _ints(legsA), _ints(legsB), perm, C.byref(st),
                                 C.byref(h)))
    return st.to_dict(), Tensor(h)


def double_layer(A, stream=None):
    h = C.c_void_p()
    check(lib().symten_double_layer(C.byref(h), A._h, _stream(stream)))
    return Tensor(h)


def double_layer_op(A, op, stream=None):
    """Double layer with the one-site operator op[s_bra, s_ket] between the
    layers (a d x d array over A's physical states in charge order)."""
    o = np.ascontiguousarray(np.asarray(op, dtype=np.float64))
    h = C.c_void_p()
    check(lib().symten_double_layer_op(C.byref(h), A._h, o.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream)))
    return Tensor(h)


def enlarged_corner(which, Cc, Ta, Tb, a, prec="f32", stream=None):
    h = C.c_void_p()
    st = _lib.PlanStats()
    check(lib().symten_enlarged_corner(C.byref(h), int(which), Cc._h, Ta._h, Tb._h, a._h, _prec(prec),
                                       C.byref(st), _stream(stream)))
    return Tensor(h), st.to_dict()


def enlarged_corner_single_layer(which, Cc, Ta, Tb, A, prec="f32", stream=None):
    """The enlarged corner with A and A* absorbed separately (same result as
    enlarged_corner with a = double_layer(A))."""
    h = C.c_void_p()
    st = _lib.PlanStats()
    check(lib().symten_enlarged_corner_single_layer(C.byref(h), int(which), Cc._h, Ta._h, Tb._h, A._h, _prec(prec),
                                                    C.byref(st), _stream(stream)))
    return Tensor(h), st.to_dict()


def enlarged_corners_batched(Cs, Tas, Tbs, As, prec="bf16x3", use_graph=False, stream=None):
    n = len(Cs)
    arr = lambda xs: (C.c_void_p * n)(*[x._h for x in xs])
    outs = (C.c_void_p * n)()
    st = _lib.PlanStats()
    check(lib().symten_enlarged_corners_batched(n, outs, arr(Cs), arr(Tas), arr(Tbs), arr(As), _prec(prec),
                                                int(bool(use_graph)), C.byref(st), _stream(stream)))
    return [Tensor(C.c_void_p(outs[i])) for i in range(n)], st.to_dict()


def sync(stream=None):
    check(lib().symten_sync(_stream(stream)))


def profile_begin():
    """Bracket every gather / grouped-GEMM launch with HIP events from now on."""
    check(lib().symten_profile_begin())


def profile_end():
    """Stop timing; returns one dict per kernel (launches, ms, flops, bytes)."""
    cap = 256
    buf = (_lib.KernelStat * cap)()
    n = C.c_int()
    check(lib().symten_profile_end(buf, cap, C.byref(n)))
    return [buf[i].to_dict() for i in range(min(cap, n.value))]


class CtmEnv:
    """CTM environment C1..C4, T1..T4 (clockwise bonds) with one-move updates."""

    def __init__(self, Cs, Ts):
        # the caller's tensors by slot (0..3: C1..C4, 4..7: T1..T4), held
        # while the environment may use them
        self._keep = list(Cs) + list(Ts)
        h = C.c_void_p()
        check(lib().ctm_env_create(C.byref(h), (C.c_void_p * 4)(*[c._h for c in Cs]),
                                   (C.c_void_p * 4)(*[t._h for t in Ts])))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().ctm_env_destroy(h)
            except Exception:
                pass
            self._h = None

    def get(self, k):
        """k = 0..3: C1..C4, 4..7: T1..T4."""
        h = C.c_void_p()
        check(lib().ctm_env_get(self._h, int(k), C.byref(h)))
        return Tensor(h)

    def set(self, k, t):
        """Replace tensor k (0..3: C1..C4, 4..7: T1..T4)."""
        check(lib().ctm_env_set(self._h, int(k), t._h))
        self._keep[int(k)] = t

    def move(self, a, chi, prec="f32", direction=0, stats=True, stream=None):
        st = _lib.MoveStats() if stats else None
        check(lib().ctm_move(self._h, a._h, int(direction), int(chi), _prec(prec),
                             C.byref(st) if stats else None, _stream(stream)))
        return st.to_dict() if stats else None

    def site_partition(self, a, block=1, stream=None):
        """(kappa, [Z_00, Z_b0, Z_0b, Z_bb]) of a classical model on a
        block x block patch (block 1 or 2), FP64."""
        k = C.c_double()
        z = (C.c_double * 4)()
        check(lib().ctm_site_partition(self._h, a._h, int(block), C.byref(k), z, _stream(stream)))
        return k.value, list(z)

    def expectation(self, a, sites, n, m, stream=None):
        """Z_nm(sites) / Z_nm(a) with the n x m patch's site tensors replaced
        (row-major list), FP64."""
        hs = (C.c_void_p * (n * m))(*[t._h for t in sites])
        v = C.c_double()
        check(lib().ctm_expectation(self._h, a._h, int(n), int(m), hs, C.byref(v), _stream(stream)))
        return v.value

    def heisenberg_bond_energy(self, A, stream=None):
        """(e_h, e_v): <S_i . S_j> on a horizontal and a vertical bond, FP64."""
        eh, ev = C.c_double(), C.c_double()
        check(lib().ctm_heisenberg_bond_energy(self._h, A._h, C.byref(eh), C.byref(ev), _stream(stream)))
        return eh.value, ev.value

    def run(self, a, chi, chi_max=None, prec="f64", block=1, max_steps=15, tol=1e-8, stream=None):
        """CTM steps with the error estimate of Sec. 3: returns a dict with
        kappa, err_steps, err_chi, error, steps, total_steps, chi, levels.
        chi_max None: chi stays fixed."""
        o = _lib.RunOpts(int(chi), int(chi if chi_max is None else chi_max), _prec(prec), int(block),
                         int(max_steps), float(tol))
        r = _lib.RunResult()
        check(lib().ctm_run(self._h, a._h, C.byref(o), C.byref(r), _stream(stream)))
        return r.to_dict()

    def singular_values(self):
        n = C.c_int64()
        check(lib().ctm_move_singular_values(self._h, None, 0, C.byref(n)))
        buf = (C.c_double * max(1, n.value))()
        check(lib().ctm_move_singular_values(self._h, buf, n.value, C.byref(n)))
        return np.array(buf[:n.value])

    def projectors(self):
        p, pt = C.c_void_p(), C.c_void_p()
        check(lib().ctm_move_projectors(self._h, C.byref(p), C.byref(pt)))
        return Tensor(p), Tensor(pt)


class CtmCell:
    """Environment of a unit cell of Lx x Ly sites: sites[x][y] = (Cs, Ts),
    the four corners and four edges of site (x, y) (x to the right, y down)."""

    def __init__(self, sites):
        self.Lx, self.Ly = len(sites), len(sites[0])
        cs = [c for col in sites for (Cs, _) in col for c in Cs]
        ts = [t for col in sites for (_, Ts) in col for t in Ts]
        n = 4 * self.Lx * self.Ly
        self._h = C.c_void_p()
        check(lib().ctm_cell_create(C.byref(self._h), self.Lx, self.Ly, (C.c_void_p * n)(*[c._h for c in cs]),
                                    (C.c_void_p * n)(*[t._h for t in ts])))
        self._keep = cs + ts

    def __del__(self):
        try:
            if self._h:
                lib().ctm_env_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def get(self, x, y, k):
        """Tensor k (0..3: C1..C4, 4..7: T1..T4) of site (x, y)."""
        h = C.c_void_p()
        check(lib().ctm_cell_get(self._h, int(x), int(y), int(k), C.byref(h)))
        return Tensor(h)

    def move(self, a, chi, prec="f64", direction=0, stream=None):
        """a[x][y]: the site tensors."""
        flat = [t for col in a for t in col]
        check(lib().ctm_cell_move(self._h, (C.c_void_p * len(flat))(*[t._h for t in flat]), int(direction), int(chi),
                                  _prec(prec), _stream(stream)))

    def site_partition(self, x, y, a, block=1, stream=None):
        k = C.c_double()
        z = (C.c_double * 4)()
        check(lib().ctm_cell_site_partition(self._h, int(x), int(y), a._h, int(block), C.byref(k), z,
                                            _stream(stream)))
        return k.value, list(z)

    def singular_values(self):
        n = C.c_int64()
        check(lib().ctm_move_singular_values(self._h, None, 0, C.byref(n)))
        buf = (C.c_double * max(1, n.value))()
        check(lib().ctm_move_singular_values(self._h, buf, n.value, C.byref(n)))
        return np.array(buf[:n.value])
