"""Pins of the oracle's batch (slot) encoding for BFV and BGV plaintexts
(Scheme Flexibility section: encodings come from those schemes' papers).  The
encoding is pinned to things other than its own NTT:

  * brute force: every slot equals the plaintext polynomial evaluated at
    zeta^(e_j) with Python integers, and zeta is a primitive 2N-th root;
  * the exponents are the N odd residues mod 2N;
  * multiplication: the negacyclic product of two encodings (mod t) encodes
    the slot-wise product;
  * the automorphism X -> X^3 rotates both halves by one slot, X -> X^-1
    swaps them;
  * a constant vector encodes to the constant polynomial; round trips."""
import numpy as np
import pytest

from test_oracle_scheme import negacyclic


def evaluate(m, x, t):
    """m(x) mod t by Horner's rule with Python integers."""
    acc = 0
    for c in reversed([int(v) for v in m]):
        acc = (acc * x + c) % t
    return acc


def automorphism(m, g, t):
    """m(X^g) in Z_t[X]/(X^N + 1), g odd."""
    n = len(m)
    out = [0] * n
    for i, c in enumerate(m):
        k = (i * g) % (2 * n)
        if k < n:
            out[k] = (out[k] + int(c)) % t
        else:
            out[k - n] = (out[k - n] - int(c)) % t
    return out


def centred(v, t):
    v = [int(x) % t for x in v]
    return np.array([x - t if x > t // 2 else x for x in v], dtype=np.int64)


@pytest.mark.parametrize("log_n,t", [(3, 17), (4, 97), (5, 193), (6, 257)])
def test_batch_brute_force(orc, log_n, t):
    n = 1 << log_n
    exps = orc.batch_exponents(log_n)
    assert sorted(exps) == list(range(1, 2 * n, 2))
    zeta = orc.batch_zeta(log_n, t)
    assert pow(zeta, n, t) == t - 1                      # primitive 2N-th root
    rng = np.random.default_rng(log_n)
    v = rng.integers(-t, 2 * t, size=n)
    m = orc.batch_encode(log_n, t, v)
    assert m.min() >= 0 and m.max() < t
    for j, e in enumerate(exps):
        assert evaluate(m, pow(zeta, e, t), t) == int(v[j]) % t, j
    # decoding is evaluation too, from any representatives of the coefficients
    m2 = [int(c) + t * int(k) for c, k in zip(rng.integers(0, t, size=n), rng.integers(-3, 3, size=n))]
    want = centred([evaluate(m2, pow(zeta, e, t), t) for e in exps], t)
    assert np.array_equal(orc.batch_decode(log_n, t, m2), want)


@pytest.mark.parametrize("log_n,t", [(5, 193), (12, 65537)])
def test_batch_product_is_slotwise(orc, log_n, t):
    n = 1 << log_n
    rng = np.random.default_rng(7)
    a = rng.integers(0, t, size=n)
    b = rng.integers(0, t, size=n)
    ma, mb = orc.batch_encode(log_n, t, a), orc.batch_encode(log_n, t, b)
    prod = np.array([int(x) % t for x in negacyclic(ma, mb)], dtype=np.int64)
    ab = [(int(x) * int(y)) % t for x, y in zip(a, b)]
    assert np.array_equal(prod, orc.batch_encode(log_n, t, ab))


@pytest.mark.parametrize("log_n,t", [(5, 193), (13, 65537)])
def test_batch_rotations_and_constants(orc, log_n, t):
    n = 1 << log_n
    h = n // 2
    rng = np.random.default_rng(9)
    v = rng.integers(-(t // 2), t // 2 + 1, size=n)
    m = orc.batch_encode(log_n, t, v)
    rot = orc.batch_decode(log_n, t, automorphism(m, 3, t))
    assert np.array_equal(rot, np.concatenate([np.roll(v[:h], -1), np.roll(v[h:], -1)]))
    swap = orc.batch_decode(log_n, t, automorphism(m, 2 * n - 1, t))
    assert np.array_equal(swap, np.concatenate([v[h:], v[:h]]))
    const = orc.batch_encode(log_n, t, np.full(n, 5))
    assert const[0] == 5 and not const[1:].any()
    assert np.array_equal(orc.batch_decode(log_n, t, m), v)


def test_batch_rejects_unsuitable_t(orc):
    for log_n, t in ((4, 96), (4, 65), (12, 257)):       # not prime; not prime; 257 != 1 mod 8192
        with pytest.raises(ValueError):
            orc.batch_encode(log_n, t, [0] * (1 << log_n))
