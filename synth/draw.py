"""Counter-free seeded Gaussian draws.

Every tensor of a workload gets its own numpy PCG64 stream, keyed by
(workload seed, tensor index[, batch index]), so that a consumer can draw a
tensor's values knowing only how many it needs.
"""
import numpy as np

# Fixed tensor order of a workload: site tensor, four corners, four edges.
# "a" is drawn directly only where a workload takes a random double-layer tensor.
TENSOR_INDEX = {"A": 0, "C1": 1, "C2": 2, "C3": 3, "C4": 4,
                "T1": 5, "T2": 6, "T3": 7, "T4": 8, "a": 9}
# the tensors of a U(1) workload, which builds a from A
SITE_AND_ENV = ("A", "C1", "C2", "C3", "C4", "T1", "T2", "T3", "T4")


def draw(key, n):
    """Return ``n`` standard normal float64 values for the stream ``key``.

    ``key`` is a tuple of non-negative ints, e.g. ``(seed, TENSOR_INDEX['T1'])``
    or ``(seed, batch, TENSOR_INDEX['C1'])``.
    """
    ss = np.random.SeedSequence([int(k) for k in key])
    rng = np.random.Generator(np.random.PCG64(ss))
    return rng.standard_normal(int(n))
