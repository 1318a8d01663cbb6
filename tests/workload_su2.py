"""Test helper for SU(2) workloads: seeded reduced values, expanded by the
oracle into dense arrays on one side and uploaded as libsymten SU(2) tensors
on the other.  The only shared piece is the seeded draw from ``synth``."""
import numpy as np

import paper_1808_10804_amd as st
from oracle import su2
from synth import draw, TENSOR_INDEX

IN, OUT = 1, -1


def corner_legs(chi, dd):
    """Legs of C1, T1, T4 and the (random) double-layer tensor a, in the
    clockwise convention of the U(1) workload."""
    return {"C1": [(chi, IN), (chi, OUT)], "T1": [(chi, IN), (dd, OUT), (chi, OUT)],
            "T4": [(chi, IN), (dd, OUT), (chi, OUT)], "a": [(dd, IN), (dd, IN), (dd, OUT), (dd, OUT)]}


def su2_values(legs, seed):
    return {n: draw((seed, TENSOR_INDEX[n]), su2.nnz([su2.Leg(s, d) for s, d in spec]))
            for n, spec in legs.items()}


def device(legs, vals, dtype):
    out = {}
    for n, spec in legs.items():
        out[n] = st.Tensor.create(spec, dtype=dtype, group="su2")
        out[n].upload(vals[n])
    return out


def dense(legs, vals):
    return {n: su2.expand([su2.Leg(s, d) for s, d in spec], vals[n]) for n, spec in legs.items()}


def reduced_full(t):
    """Device SU(2) tensor -> values for every canonical block of its legs
    (blocks the tensor does not hold are zero)."""
    legs = [su2.Leg(s, d) for s, d in t.legs()]
    have = {}
    vals = t.download()
    pos = 0
    for (lab, shp, _, _), tr in zip(t.blocks(), t.trees()):
        n = int(np.prod(shp))
        have[(lab, tr)] = vals[pos:pos + n]
        pos += n
    out = []
    for tj, tr in su2.blocks(legs):
        n = int(np.prod([l.n(x) for l, x in zip(legs, tj)]))
        out.append(have.get((tj, tr), np.zeros(n)))
    return (np.concatenate(out) if out else np.zeros(0)), legs
