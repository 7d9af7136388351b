"""The oracle against sizes printed in the paper (tests/golden/paper_sizes.txt)."""
import os
from math import comb

import pytest

from oracle import compressed as Z

HERE = os.path.dirname(os.path.abspath(__file__))


def rows():
    out = []
    with open(os.path.join(HERE, "golden", "paper_sizes.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                out.append([x.strip() for x in line.split("|")])
    return out


def N(p):
    return comb(p + 3, 3) if p >= 0 else 0


@pytest.mark.parametrize("p", [2, 4, 6, 8, 12])
def test_paper_sizes(p):
    seen = set()
    for name, kernel, formula in rows():
        seen.add(name)
        if name == "kept_count":
            c = int(formula.split("p-")[1].rstrip(")"))
            assert len(Z.kept(kernel, 0.0, p)) == N(p) - N(p - c)
        elif name == "fft_sizes":
            want = tuple(eval(term.replace("2p", f"2*{p}")) for term in formula.split(","))
            assert Z.fft_grid(kernel, 0.0, p) == want
    assert seen == {"kept_count", "fft_sizes"}
