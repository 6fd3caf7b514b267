"""The paper's Taylor-bubble runs (Sec. 4.4) at tube diameter 32, all four
variants: the Reynolds number of the rising bubble against the paper's table,
and the variants in the paper's order (OM > OM3 > NBRC > NBKC)."""
import pytest

from paper_2207_13962_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_taylor_bubble_reynolds_as_in_the_paper():
    from paper_2207_13962_amd.validation import PAPER_TAYLOR_RE, taylor_reynolds
    re = {}
    for v in (I.NBRC, I.NBKC, I.OM, I.OM3):
        r = taylor_reynolds(32, variant=v)
        assert r["status"] == 0
        re[v] = r["Re"]
        paper = PAPER_TAYLOR_RE[32][v]
        # the paper's own runs differ from each other by up to 15 % across
        # variants; the same setup here lands within 5 % of each
        assert abs(re[v] - paper) <= 0.05 * paper, (I.VARIANT_NAMES[v], re[v], paper)
    assert re[I.OM] > re[I.OM3] > re[I.NBRC] > re[I.NBKC]
