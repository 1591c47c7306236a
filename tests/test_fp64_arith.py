"""CPU check of the exact FP64 modular multiplication used by the library's
forward NTT for moduli below 2^50 (IEEE doubles; FMA emulated exactly with
rationals): t = r + l equals y w - k q exactly, with |t| <= q (1/2 + |y| 2^-52),
and a whole transform run with these butterflies stays below 2^52 and matches
the oracle's NTT."""
import random
from fractions import Fraction as F

import numpy as np
import pytest


def fma(a, b, c):
    return float(F(a) * F(b) + F(c))


def fp_mulmod(y, w, wq, q):
    k = float(np.rint(y * wq))
    h = y * w
    l = fma(y, w, -h)
    r = fma(-k, q, h)
    return r + l, k


@pytest.mark.parametrize("bits,bound_mult", [(30, 30), (40, 30), (46, 30), (47, 24), (50, 5)])
def test_fp_mulmod_exact_and_bounded(bits, bound_mult):
    rng = random.Random(bits)
    for _ in range(4000):
        q = rng.randrange(2 ** (bits - 1), 2 ** bits) | 1
        w = rng.randrange(q)
        wq = float(F(w, q))
        lim = min(bound_mult * q, 2 ** 53 - 1)
        y = float(rng.randrange(-lim, lim))
        t, k = fp_mulmod(y, float(w), wq, float(q))
        assert F(t) == F(int(y)) * w - F(int(k)) * q
        assert abs(t) <= q * (0.5 + abs(y) * 2.0 ** -52) + 1e-6


def _brv(x, b):
    r = 0
    for _ in range(b):
        r = (r << 1) | (x & 1)
        x >>= 1
    return r


@pytest.mark.parametrize("log_n,bits,passes,reduce", [(8, 40, (4, 4), False), (9, 46, (3, 3, 3), False),
                                                      (8, 50, (4, 4), True)])
def test_fp_transform_matches_oracle(orc, log_n, bits, passes, reduce):
    n = 1 << log_n
    q = orc.choose_moduli(log_n, (bits,))[0]
    psi = orc.find_psi(q, log_n)
    tw = [pow(psi, _brv(k, log_n), q) for k in range(n)]
    rng = np.random.default_rng(log_n)
    a = [int(v) for v in rng.integers(0, q, size=n)]
    x = [float(v) for v in a]
    stage = 0
    for K in passes:
        if reduce:
            x = [float(v - np.rint(v * (1.0 / q)) * q) for v in x]
        for _ in range(K):
            t = n >> (stage + 1)
            for g in range(1 << stage):
                w = tw[(1 << stage) + g]
                wq = float(F(w, q))
                for j in range(2 * g * t, 2 * g * t + t):
                    tt, _ = fp_mulmod(x[j + t], float(w), wq, float(q))
                    xa = x[j]
                    x[j], x[j + t] = xa + tt, xa - tt
                    assert abs(x[j]) < 2 ** 52 and abs(x[j + t]) < 2 ** 52
            stage += 1
    assert [int(v) % q for v in x] == [int(v) for v in orc.ntt_forward(a, log_n, q, psi)]
