"""Byte and flop accounting of one Dslash application per lattice site.

TEST INFRASTRUCTURE ONLY.  Section 1 of the paper prices the Wilson Dslash
at 2880 bytes read or written and 1632 flops per site, and the staggered
D_KS at 1584 bytes and 570 flops.  The formulas below derive those numbers
from the field sizes: a Wilson spinor is 4 spins x 3 colours complex, a
staggered field is 3 colours complex, a link is a 3x3 complex matrix; each
of the 8 hops reads one neighbour field and one link, and one field is
written.
"""

from __future__ import annotations

WILSON_COMPLEX = 12      # 4 spins x 3 colours
STAGGERED_COMPLEX = 3    # 3 colours
LINK_COMPLEX_FULL = 9    # 3x3
LINK_COMPLEX_TWO_ROWS = 6


def field_bytes(n_complex: int, real_bytes: int) -> int:
    return 2 * n_complex * real_bytes


def paper_bytes(spinor_b: int, link_b: int) -> int:
    """8 neighbour reads + 8 link reads + 1 write, no reuse (the paper's count)."""
    return 8 * spinor_b + 8 * link_b + spinor_b


def compulsory_eo_bytes(spinor_b: int, link_b: int) -> int:
    """One even-odd hop with each input field, each link and each output
    touched once: 1 input + 8 links + 1 output per output site."""
    return spinor_b + 8 * link_b + spinor_b


# flop counts of the pieces of one hop (real adds and multiplies)
CMUL, CADD = 6, 2
SU3_MATVEC = 9 * CMUL + 6 * CADD          # 66
HALF_SPINOR_PROJECT = 6 * CADD            # 12


def wilson_flops(convention: str = "standard") -> int:
    """Standard count: project (12) + two SU(3) matvecs (132) per hop, and
    seven 24-flop accumulations.  The paper's count adds a complex scalar
    multiply of the half spinor (36) and accumulates all eight hops."""
    if convention == "standard":
        return 8 * (HALF_SPINOR_PROJECT + 2 * SU3_MATVEC) + 7 * 12 * CADD
    if convention == "paper":
        return 8 * (HALF_SPINOR_PROJECT + 2 * SU3_MATVEC + 6 * CMUL + 12 * CADD)
    raise ValueError(convention)


def staggered_flops() -> int:
    return 8 * SU3_MATVEC + 7 * STAGGERED_COMPLEX * CADD
