"""Writes cfg4_leftmove.npz: the dense FP64 oracle's left move of the
D = 8, chi = 200 U(1) workload (seeded Gaussian draws of the shared input
recipe), reduced to what a device move is compared with:

  - the kept states per fused charge, the relative gap at the cut, the
    truncation error and s_max;
  - every singular value of the cut, sector by sector (descending);
  - the gauge-invariant left column L[x1, r, x3] = C1'[k, x1] T4'[k', r, k]
    C4'[x3, k'] as random projections G[i, j, r] = sum U1[i, x1] L[x1, r, x3]
    U3[j, x3] (U1, U3 seeded standard normal, 16 x chi each) and as 16 full
    r-slices L[x1, :, x3] at seeded (x1, x3).

Only the oracle and the seeded input recipe are used.  Run from the
repository root:  python tests/golden/make_cfg4_move.py  (a few minutes on
eight cores, about 16 GB of memory).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import u1  # noqa: E402
from synth import config, draw, TENSOR_INDEX, SITE_AND_ENV  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg4_leftmove.npz")
PROJ_SEED = 4040
NPROJ = 16
NSLICE = 16


def main():
    t0 = time.time()
    c = config(4)
    w = u1.Workload(c["phys"], c["virt"], c["chi"], c["flux"])
    vals = {n: draw((c["seed"], TENSOR_INDEX[n]), w.nnz_of(n)) for n in SITE_AND_ENV}
    T = w.dense_tensors(vals)
    a, _ = u1.double_layer(T["A"], w.A_legs)
    mv = u1.ctm_left_move(w, T, a, c["chi_target"])
    pr = mv["proj"]
    L = mv["L"]
    nx = L.shape[0]
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([PROJ_SEED])))
    U1 = rng.standard_normal((NPROJ, nx))
    U3 = rng.standard_normal((NPROJ, L.shape[2]))
    G = np.einsum("ia,arb,jb->ijr", U1, L, U3, optimize=True)
    xs = rng.integers(0, nx, size=NSLICE)
    zs = rng.integers(0, L.shape[2], size=NSLICE)
    slices = np.stack([L[x, :, z] for x, z in zip(xs, zs)])
    sec = sorted(pr["svals"])
    np.savez_compressed(
        OUT,
        kept_q=np.array(sorted(pr["kept"]), dtype=np.int64),
        kept_n=np.array([pr["kept"][q] for q in sorted(pr["kept"])], dtype=np.int64),
        sv_q=np.array(sec, dtype=np.int64),
        sv_n=np.array([len(pr["svals"][q]) for q in sec], dtype=np.int64),
        sv=np.concatenate([pr["svals"][q] for q in sec]),
        gap=pr["gap"], trunc_err=pr["trunc_err"], s_max=pr["s_max"],
        proj_seed=PROJ_SEED, U1=U1, U3=U3, G=G, slice_x1=xs, slice_x3=zs, slices=slices,
        L_norm=np.linalg.norm(L), seed=c["seed"], chi=c["chi_target"])
    print(f"wrote {OUT} in {time.time() - t0:.0f} s: kept {pr['kept']}, gap {pr['gap']:.3e}, "
          f"trunc_err {pr['trunc_err']:.4e}")


if __name__ == "__main__":
    main()
