"""Test helper: the same seeded workload built twice, once as dense oracle
arrays and once as libsymten device tensors.  The only shared piece is the
seeded draw from ``synth``."""
import numpy as np

import paper_1808_10804_amd as st
from oracle import u1
from oracle.u1 import Workload
from synth import draw, TENSOR_INDEX

NAMES = ["A", "C1", "C2", "C3", "C4", "T1", "T2", "T3", "T4"]


def values(w, seed, batch=None):
    key = (lambda n: (seed, TENSOR_INDEX[n])) if batch is None else (lambda n: (seed, batch, TENSOR_INDEX[n]))
    return {n: draw(key(n), w.nnz_of(n)) for n in NAMES}


def oracle_side(cfgd, seed, batch=None):
    w = Workload(cfgd["phys"], cfgd["virt"], cfgd["chi"], cfgd["flux"])
    vals = values(w, seed, batch)
    T = w.dense_tensors(vals)
    a, _ = u1.double_layer(T["A"], w.A_legs)
    return w, T, a, vals


def device_side(cfgd, seed, dtype, batch=None):
    """Device tensors with the workload's legs, filled with the same draws.
    Legs come from the descriptor of the workload (sector dicts and
    directions), not from the oracle's arithmetic."""
    phys, virt, chi, flux = cfgd["phys"], cfgd["virt"], cfgd["chi"], cfgd["flux"]
    legs = {"A": ([(phys, 1), (virt, 1), (virt, 1), (virt, -1), (virt, -1)], flux)}
    out = {"A": st.Tensor.create(*legs["A"], dtype=dtype)}
    a_probe = st.double_layer(out["A"])      # its legs give the D2 sectors
    dd = a_probe.legs()[0][0]
    for c in ("C1", "C2", "C3", "C4"):
        legs[c] = ([(chi, 1), (chi, -1)], 0)
    legs["T1"] = ([(chi, 1), (dd, -1), (chi, -1)], 0)
    legs["T4"] = ([(chi, 1), (dd, -1), (chi, -1)], 0)
    legs["T2"] = ([(chi, 1), (dd, 1), (chi, -1)], 0)
    legs["T3"] = ([(chi, 1), (dd, 1), (chi, -1)], 0)
    for n in NAMES[1:]:
        out[n] = st.Tensor.create(legs[n][0], flux=legs[n][1], dtype=dtype)
    key = (lambda n: (seed, TENSOR_INDEX[n])) if batch is None else (lambda n: (seed, batch, TENSOR_INDEX[n]))
    for n in NAMES:
        out[n].upload(draw(key(n), out[n].nnz))
    out["a"] = st.double_layer(out["A"])
    return out


def to_dense(t, legs_oracle=None):
    """Embed a device tensor's blocks into a dense array using the oracle's
    leg offsets (charges ascending)."""
    legs = t.legs()
    L = [u1.Leg(s, d) for s, d in legs] if legs_oracle is None else legs_oracle
    dense = np.zeros([l.size for l in L])
    for lab, blk in t.block_dict().items():
        dense[u1.block_slices(L, lab)] = blk
    return dense


def rel(x, y):
    den = np.linalg.norm(y)
    return np.linalg.norm(x - y) / (den if den > 0 else 1.0)


def from_dense(dense, legs, flux=0, dtype="f64", group="u1"):
    """Device tensor with abelian legs [(sectors, dir)] (U(1) charges or Z2
    parities) holding the blocks of a dense array laid out with the oracle's
    leg offsets."""
    t = st.Tensor.create(legs, flux=flux, dtype=dtype, group=group)
    L = [u1.Leg(s, d) for s, d in legs]
    parts = [np.asarray(dense[u1.block_slices(L, lab)]).ravel() for lab, _, _, _ in t.blocks()]
    t.upload(np.concatenate(parts) if parts else np.zeros(0))
    return t
