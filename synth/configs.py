"""Workload descriptions shaped like the paper's square-lattice Heisenberg runs.

Charges are integers in units of 2*S^z (U(1)); SU(2) labels are 2j.  A
sector list is a dict {label: reduced dimension}.  The physical leg of the
spin-1/2 site carries charges -1 and +1; the virtual legs carry even
charges, so the only parity-consistent total charge of a site tensor is odd
(+1 here: the per-site charge the paper removes with its remover tensor,
Sec. 3.1).
"""
import numpy as np


def binomial_sectors(total, nsec):
    """Split ``total`` states over ``nsec`` charge sectors {-2h..2h} (step 2)
    with binomial(nsec-1) weights, rounding by largest remainder.

    Ties in the remainder go first to the sector nearest the centre, then to
    the lower charge.  Example: (64, 5) -> {-4:4,-2:16,0:24,2:16,4:4};
    (200, 7) -> {-6:3,-4:19,-2:47,0:62,2:47,4:19,6:3}.
    """
    from math import comb
    n = nsec - 1
    w = [comb(n, k) for k in range(nsec)]
    raw = [total * x / 2 ** n for x in w]
    base = [int(np.floor(r)) for r in raw]
    rem = total - sum(base)
    h = n // 2
    order = sorted(range(nsec), key=lambda k: (-(raw[k] - base[k]), abs(k - h), k))
    for k in order[:rem]:
        base[k] += 1
    charges = [2 * (k - h) for k in range(nsec)]
    return {q: d for q, d in zip(charges, base) if d > 0}


def virtual_sectors_for_D(D):
    """Virtual-leg sectors on charges {-2,0,2} for bond dimension D (4..8)."""
    table = {4: (1, 2, 1), 5: (1, 3, 1), 6: (1, 4, 1), 7: (2, 3, 2), 8: (2, 4, 2)}
    a, b, c = table[D]
    return {-2: a, 0: b, 2: c}


PHYS_U1 = {-1: 1, 1: 1}

CONFIGS = {
    1: dict(name="u1_corner_D4_chi16_f64", group="U1", phys=PHYS_U1, flux=1,
            virt={-2: 1, 0: 2, 2: 1}, chi={-2: 4, 0: 8, 2: 4}, chi_target=16,
            prec="f64", seed=1809,
            what="one enlarged corner C1.T1.T4.a"),
    2: dict(name="u1_leftmove_D6_chi64_f32", group="U1", phys=PHYS_U1, flux=1,
            virt={-2: 1, 0: 4, 2: 1}, chi=binomial_sectors(64, 5), chi_target=64,
            prec="f32", seed=1810,
            what="full CTM left move"),
    3: dict(name="su2_move_D10_chi100_f32", group="SU2", phys={1: 1}, flux=0,
            virt={0: 1, 1: 3, 2: 1}, chi={0: 11, 1: 13, 2: 13, 3: 6}, chi_target=100,
            # multiplets of the fused (ket, bra) leg of the double layer
            dd={0: 11, 1: 12, 2: 12, 3: 6, 4: 1},
            prec="f32", seed=1811,
            what="SU(2) reduced CTM move"),
    4: dict(name="u1_move_D8_chi200_sweep", group="U1", phys=PHYS_U1, flux=1,
            virt={-2: 2, 0: 4, 2: 2}, chi=binomial_sectors(200, 7), chi_target=200,
            prec="sweep", seed=1812,
            what="one CTM move, GEMMs in f64/f32/bf16/bf16x3"),
    6: dict(name="z2_leftmove_D6_chi64_f32", group="Z2", phys={0: 1, 1: 1}, flux=0,
            virt={0: 3, 1: 3}, chi={0: 32, 1: 32}, chi_target=64,
            prec="f32", seed=1814,
            what="full CTM left move, Z2 parities (the D = 6, chi = 64 move of config 2 with charges mod 2)"),
    5: dict(name="u1_batched64_corners", group="U1", phys=PHYS_U1, flux=1,
            batch=64, D_choices=(4, 5, 6, 7, 8), chi_range=(32, 160),
            prec="bf16x3", seed=1813,
            what="64 independent enlarged corners in one launch"),
}


def config(i):
    return dict(CONFIGS[i])


def batched_draws(seed=1813, batch=64, D_choices=(4, 5, 6, 7, 8), chi_range=(32, 160)):
    """Seeded (D, chi) draws of the batched workload, with their sector lists.

    chi sectors: binomial over 5 charge sectors if chi < 100, else over 7.
    """
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 999])))
    out = []
    for b in range(batch):
        D = int(rng.choice(D_choices))
        chi = int(rng.integers(chi_range[0], chi_range[1] + 1))
        nsec = 5 if chi < 100 else 7
        out.append(dict(D=D, chi_total=chi, virt=virtual_sectors_for_D(D),
                        chi=binomial_sectors(chi, nsec)))
    return out
