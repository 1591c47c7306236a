"""CPU bound on the magnitudes inside the library's FP64 forward transform
(moduli below 2^50), for every thread geometry the kernels and the autotuner
use and for the split N = 32768 form, propagated stage by stage with exact
rationals.  A butterfly takes |x|, |y| <= B to |x +- t| <= B + q (1/2 + B 2^-52),
the bound on t = y w - k q with the rounded quotient k = rint(y fl(w/q))
(checked pointwise in test_fp64_arith).  Moduli below 2^47 are never reduced
inside the transform; moduli in [2^47, 2^50) are rounded into
[-q/2 - 1, q/2 + 1] at the start of every pass but the first.  Inputs reach
at most 2q + 64 in magnitude (a residue below q plus the cached Enc(0)'s
coefficient below q plus an error), and moduli of 2^47 and above get inputs
of at most q + 64 (reduced messages, canonical residues plus an error).  The
products and sums of the FP64 butterfly are exact while every value stays
below 2^53; the tests also pin the tighter 2^52 below 2^47 that the
canonicalisation's fast path assumes."""
from fractions import Fraction as F

import pytest

# (log N, log T): the default geometry of each ring degree, the autotuner's
# 8- and 32-per-thread forms, and the half transforms of the split N = 32768
GEOMS = [(12, 8), (12, 9), (12, 7), (13, 9), (13, 10), (13, 8), (14, 10), (14, 9)]


def passes(log_n, log_t):
    """Stages per pass, as the kernels' Geom splits them."""
    log_r = log_n - log_t
    npass = (log_n + log_r - 1) // log_r
    return [log_n // npass + (1 if p < log_n % npass else 0) for p in range(npass)]


def stage(b, q):
    return b + q * (F(1, 2) + b / 2 ** 52)


def max_bound(ks, q, b0, reduce_passes, split_first=False):
    b, top = F(b0), F(b0)
    if split_first:                       # the pairing stage of N = 32768
        b = stage(b, q)
        if reduce_passes:
            b = F(q, 2) + 1
        top = max(top, b)
    for p, k in enumerate(ks):
        if reduce_passes and p > 0:
            b = F(q, 2) + 1
        for _ in range(k):
            b = stage(b, q)
            top = max(top, b)
    return top


@pytest.mark.parametrize("log_n,log_t", GEOMS)
def test_moduli_below_2_47_stay_below_2_52(log_n, log_t):
    q = 2 ** 47 - 1
    ks = passes(log_n, log_t)
    assert sum(ks) == log_n and max(ks) <= log_n - log_t
    assert max_bound(ks, q, 2 * q + 64, False) < 2 ** 52
    if (log_n, log_t) == (14, 10):        # split N = 32768: pairing stage, then 14-stage halves
        assert max_bound(ks, q, 2 * q + 64, False, split_first=True) < 2 ** 52


@pytest.mark.parametrize("log_n,log_t", GEOMS)
def test_moduli_below_2_50_stay_below_2_53(log_n, log_t):
    q = 2 ** 50 - 1
    ks = passes(log_n, log_t)
    top = max_bound(ks, q, q + 64, True)
    assert top < 2 ** 53
    if (log_n, log_t) == (14, 10):
        assert max_bound(ks, q, q + 64, True, split_first=True) < 2 ** 53


def test_bound_is_tight_enough_to_matter():
    """The first pass of the 32-per-thread N = 8192 form (five stages from
    q + 64 at q near 2^50) is the worst case: above 2^52, so the 2^53 limit,
    not the tighter one, is what holds there."""
    q = 2 ** 50 - 1
    top = max_bound(passes(13, 8), q, q + 64, True)
    assert 2 ** 52 < top < 2 ** 53
