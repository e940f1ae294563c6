"""The accounting formulas reproduce the per-site numbers the paper prints
(section 1): Wilson Dslash 2880 B / 1632 flop, staggered 1584 B / 570 flop."""

import json
import os

from oracle import accounting as A

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_accounting.json")))


def test_wilson_paper_numbers():
    b = GOLD["precision_bytes_per_real"]
    spinor = A.field_bytes(A.WILSON_COMPLEX, b)
    link = A.field_bytes(A.LINK_COMPLEX_FULL, b)
    w = GOLD["wilson_dslash"]
    assert A.paper_bytes(spinor, link) == w["bytes_per_site"]
    assert A.wilson_flops("paper") == w["flops_per_site"]
    assert abs(w["flops_per_site"] / w["bytes_per_site"] - w["flops_per_byte_approx"]) < 0.01


def test_staggered_paper_numbers():
    b = GOLD["precision_bytes_per_real"]
    s = GOLD["staggered_dks"]
    vec = A.field_bytes(A.STAGGERED_COMPLEX, b)
    link = A.field_bytes(A.LINK_COMPLEX_FULL, b)
    assert A.paper_bytes(vec, link) == s["bytes_per_site"]
    assert A.staggered_flops() == s["flops_per_site"]
    # the paper quotes 570/1584 = 0.3598 as "~0.35"
    assert abs(s["flops_per_site"] / s["bytes_per_site"] - s["flops_per_byte_approx"]) < 0.01


def test_compulsory_eo_bytes():
    # one input spinor, eight links, one output spinor per output site
    assert A.compulsory_eo_bytes(192, 144) == 1536
    assert A.compulsory_eo_bytes(192, 96) == 1152
    assert A.compulsory_eo_bytes(96, 48) == 576
    assert A.wilson_flops("standard") == 1320
