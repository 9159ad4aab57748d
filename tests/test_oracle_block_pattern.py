"""The structural zeros of the block lines (CPU only).

The GPU eliminations skip the products with entries of a line's lower and
upper 3x3 blocks that are zero by construction: in the (p, T, w) order of a
block (w the velocity normal to the line's faces), the lower block couples
the w row to w only, and the upper block couples p to p and T, T to T, and w
to p and w (the direction operators of Appendix B, eqs. (dr), (dtheta),
(dphi): advection and conduction of p and T, the divergence of w in the p
and T rows, the pressure gradient and the viscous term in the w row).  The
oracle builds its line blocks by probing the direction operators, so its
blocks must vanish wherever that pattern has a zero, for every direction,
on sectors with walls and on the sphere, with rotation, pi_inf and gravity
switched on, and away from the boundary rows as at them.
"""
import numpy as np
import pytest

import oracle
from helpers import AIR, grid_of, random_state, random_wall, small_sector, small_sphere
from paper_2004_13887_amd import inputs as I

# bit 3 r + c: entry (r, c) may be non-zero
NZ_L = 0x137  # (0,0) (0,1) (0,2) (1,1) (1,2) (2,2)
NZ_U = 0x153  # (0,0) (0,1) (1,1) (2,0) (2,2)


def _mask(bits):
    return np.array([[(bits >> (3 * r + c)) & 1 for c in range(3)] for r in range(3)], dtype=bool)


ROT = oracle.Material(*I.MaterialSpec(cp=1.6, cv=1.0, pi_inf=2500.0, mu=1.0, prandtl=1.0,
                                      omega=0.7, g_r=3.0).astuple())


@pytest.mark.parametrize("which", ["sector", "sphere"])
@pytest.mark.parametrize("mat", ["air", "rotating"])
def test_block_lines_vanish_off_the_pattern(which, mat):
    spec = small_sector() if which == "sector" else small_sphere()
    g = grid_of(spec)
    U, tau = random_state(spec, 21)
    wall = random_wall(spec, 22, 0.3) if which == "sector" else None
    m = AIR if mat == "air" else ROT
    zl, zu = ~_mask(NZ_L), ~_mask(NZ_U)
    seen_l, seen_u = np.zeros((3, 3), bool), np.zeros((3, 3), bool)
    for d in range(3):
        n_a, n_b = [(spec.nt, spec.np), (spec.nr, spec.np), (spec.nr, spec.nt)][d]
        for a in sorted({0, n_a // 2, n_a - 1}):
            for b in sorted({0, n_b // 2, n_b - 1}):
                L, D, Uu, idx, fid, cyc = oracle.line_blocks(g, m, U, tau, d, -1, a, b, wall=wall)
                # block order (p, T, normal velocity)
                assert list(fid[:3]) == [0, 4, d + 1], fid[:3]
                assert np.all(L[:, zl] == 0.0), (d, a, b, np.argwhere(L[:, zl] != 0.0)[:3])
                assert np.all(Uu[:, zu] == 0.0), (d, a, b, np.argwhere(Uu[:, zu] != 0.0)[:3])
                seen_l |= np.any(L != 0.0, axis=0)
                seen_u |= np.any(Uu != 0.0, axis=0)
    # the pattern is tight: every entry it keeps is non-zero somewhere
    assert np.array_equal(seen_l, _mask(NZ_L)), seen_l.astype(int)
    assert np.array_equal(seen_u, _mask(NZ_U)), seen_u.astype(int)
