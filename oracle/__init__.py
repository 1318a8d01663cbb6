"""Plain FP64 dense CPU oracle for the symmetric CTM hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, call,
link or execute anything in this package; only ``tests/``, the smoke check
and the CPU-baseline leg of the benchmark use it.  It shares no code with the
HIP path: the only common input is the seeded Gaussian generator in ``synth``.

What it computes follows the paper's definitions directly: a symmetric tensor
is a direct sum of charge blocks (Sec. 2, Eq. tensor-blocks), blocks that
break the charge addition rule are identically zero (Sec. 2, the rank-2
example), and a block-sparse contraction is nothing but the contraction of
those blocks (Sec. 2, the contraction rule r_k = m_t . m_s).  The oracle
therefore embeds every tensor into a full FP64 array and contracts densely
with numpy, so that a reader can check each step against the definitions by
eye.  Integer bookkeeping (allowed blocks, matched pairs, output blocks,
useful flops) is computed by brute force over all label tuples.
"""
