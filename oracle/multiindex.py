"""Multi-index sets (Sec. 2 preliminaries; Def. bnu; Lemma max_prod_nice).

M(p) is the set of 3-multi-indices of total order <= p.  The paper's count of it
is printed as a binomial with the wrong upper argument (eq. np-count); the set
has C(p+3, 3) elements, which is what is used here.
"""
from __future__ import annotations

from math import comb, factorial
from functools import lru_cache

import numpy as np

D = 3


def n_full(p: int) -> int:
    """|M(p)| = C(p + 3, 3)."""
    return comb(p + D, D) if p >= 0 else 0


@lru_cache(maxsize=None)
def graded_order(p: int) -> tuple:
    """Multi-indices of M(p) in a graded monomial ordering nu (Def. bnu).

    Degree first; within a degree, lexicographic in (m_z, m_y, m_x) ascending, i.e.
    the z entry varies slowest.  This is the degree-lexicographic ordering used in
    the proof of Lemma max_prod_nice with k = z, so that c*e_z is the last index of
    M(c) and the kept set becomes {m : m_z < c}.
    """
    out = []
    for deg in range(p + 1):
        block = []
        for mz in range(deg + 1):
            for my in range(deg - mz + 1):
                mx = deg - mz - my
                block.append((mx, my, mz))
        block.sort(key=lambda m: (m[2], m[1], m[0]))
        out.extend(block)
    return tuple(out)


def index_of(p: int) -> dict:
    return {m: i for i, m in enumerate(graded_order(p))}


def kept_set(p: int, c: int) -> list:
    """{m in M(p) : m_z < c}: the stored indices j when the compressed axis is z
    (Lemma max_prod_nice).  Returned in the graded order."""
    return [m for m in graded_order(p) if m[2] < c]


def mfact(m) -> int:
    return factorial(m[0]) * factorial(m[1]) * factorial(m[2])


def mpow(v: np.ndarray, m) -> np.ndarray:
    """v^m for points v [..., 3]."""
    return v[..., 0] ** m[0] * v[..., 1] ** m[1] * v[..., 2] ** m[2]


def madd(a, b):
    return (a[0] + b[0], a[1] + b[1], a[2] + b[2])


def msub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def morder(m) -> int:
    return m[0] + m[1] + m[2]


def mge(a, b) -> bool:
    return a[0] >= b[0] and a[1] >= b[1] and a[2] >= b[2]
