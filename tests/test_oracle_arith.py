"""Pins of the oracle's number theory and NTT against independent routes:
sympy's primality test and root enumeration, the NTT's defining sum, and the
negacyclic product computed by numpy.convolve (the RNS/DFT structure of the
Theoretical Analysis section; moduli and roots are readings where the paper is
silent)."""
import random

import numpy as np
import pytest
import sympy


def brv(x, bits):
    r = 0
    for _ in range(bits):
        r = (r << 1) | (x & 1)
        x >>= 1
    return r


def test_is_prime_matches_sympy(orc):
    rng = random.Random(1)
    cases = [0, 1, 2, 3, 4, 561, 1105, 1729, 3215031751, 2152302898747, 3474749660383,
             341550071728321, 3825123056546413051, (1 << 61) - 1, (1 << 64) - 59, (1 << 64) - 1,
             1152921504606830593, 1099511480321]
    cases += [rng.getrandbits(64) | 1 for _ in range(3000)]
    cases += [rng.getrandbits(40) | 1 for _ in range(1000)]
    for n in cases:
        assert orc.is_prime(n) == sympy.isprime(n), n


def _moduli_by_sympy(log_n, bits):
    two_n = 2 << log_n
    out = []
    for b in bits:
        c = ((2 ** b - 1) // two_n) * two_n + 1
        while not (sympy.isprime(c) and c not in out):
            c -= two_n
        out.append(c)
    return out


@pytest.mark.parametrize("log_n,bits", [(12, (30, 30, 30)), (13, (60, 40, 40, 60)),
                                        (14, (60, 50, 50, 50, 50, 50, 50, 60)),
                                        (15, (55,) * 15), (4, (10, 10, 12))])
def test_moduli_rule(orc, log_n, bits):
    got = orc.choose_moduli(log_n, bits)
    assert got == _moduli_by_sympy(log_n, bits)
    for q, b in zip(got, bits):
        assert q < 2 ** b and q % (2 << log_n) == 1
    assert len(set(got)) == len(got)


def test_moduli_small_configs_known_values(orc):
    # values of the moduli rule for the N=4096 and N=8192 parameter sets,
    # independently reproduced above with sympy
    assert orc.choose_moduli(12, (30, 30, 30)) == [1073692673, 1073668097, 1073651713]
    assert orc.choose_moduli(13, (60, 40, 40, 60)) == [1152921504606830593, 1099511480321,
                                                        1099510890497, 1152921504606748673]


@pytest.mark.parametrize("log_n,q", [(3, 17), (4, 97), (4, 193), (5, 193), (6, 257), (7, 7681)])
def test_psi_is_smallest_primitive_root_bruteforce(orc, log_n, q):
    n = 1 << log_n
    roots = [x for x in range(1, q) if pow(x, n, q) == q - 1]   # order exactly 2N
    assert len(roots) == n
    assert orc.find_psi(q, log_n) == min(roots)


@pytest.mark.parametrize("log_n,bits", [(12, (30, 30, 30)), (13, (60, 40, 40, 60)), (15, (55,) * 3)])
def test_psi_order_large(orc, log_n, bits):
    n = 1 << log_n
    for q in orc.choose_moduli(log_n, bits):
        psi = orc.find_psi(q, log_n)
        assert pow(psi, n, q) == q - 1
        assert pow(psi, 2 * n, q) == 1
        # primitive 2N-th roots are exactly the x with x^N = -1; psi is among them
        # and the sympy n-th root enumeration lists none smaller
        cands = sympy.nthroot_mod(q - 1, n, q, all_roots=True) if log_n <= 12 else None
        if cands is not None:
            assert psi == min(cands)


def _direct_ntt(a, q, psi, log_n):
    n = 1 << log_n
    return [sum(int(a[i]) * pow(psi, (2 * brv(k, log_n) + 1) * i, q) for i in range(n)) % q
            for k in range(n)]


def _direct_intt(ah, q, psi, log_n):
    n = 1 << log_n
    pinv = pow(psi, -1, q)
    ninv = pow(n, -1, q)
    return [ninv * sum(int(ah[k]) * pow(pinv, (2 * brv(k, log_n) + 1) * i, q) for k in range(n)) % q
            for i in range(n)]


@pytest.mark.parametrize("log_n", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("qbits", [17, 30, 40, 55, 60])
def test_ntt_matches_definition(orc, log_n, qbits):
    q = orc.choose_moduli(log_n, (qbits,))[0]
    psi = orc.find_psi(q, log_n)
    rng = random.Random(log_n * 100 + qbits)
    a = [rng.randrange(q) for _ in range(1 << log_n)]
    got = orc.ntt_forward(a, log_n, q, psi)
    assert [int(x) for x in got] == _direct_ntt(a, q, psi, log_n)
    back = orc.ntt_inverse(got, log_n, q, psi)
    assert [int(x) for x in back] == a
    assert [int(x) for x in orc.ntt_inverse(a, log_n, q, psi)] == _direct_intt(a, q, psi, log_n)


def _negacyclic_numpy(a, b):
    """Schoolbook negacyclic product of small integer polynomials via numpy.convolve."""
    n = len(a)
    c = np.convolve(np.asarray(a, dtype=np.int64), np.asarray(b, dtype=np.int64))
    out = c[:n].copy()
    out[: n - 1] -= c[n:]
    return out


@pytest.mark.parametrize("log_n", [2, 4, 6, 8, 10])
@pytest.mark.parametrize("qbits", [30, 40, 60])
def test_ntt_product_is_negacyclic_schoolbook(orc, log_n, qbits):
    n = 1 << log_n
    q = orc.choose_moduli(log_n, (qbits,))[0]
    psi = orc.find_psi(q, log_n)
    rng = np.random.default_rng(log_n + qbits)
    a = rng.integers(-1000, 1000, size=n)
    b = rng.integers(-1000, 1000, size=n)
    ah = orc.ntt_forward([x % q for x in a.tolist()], log_n, q, psi)
    bh = orc.ntt_forward([x % q for x in b.tolist()], log_n, q, psi)
    prod = [(int(x) * int(y)) % q for x, y in zip(ah, bh)]
    c = orc.ntt_inverse(prod, log_n, q, psi)
    want = [int(v) % q for v in _negacyclic_numpy(a, b)]
    assert [int(x) for x in c] == want


def test_ntt_large_roundtrip_and_linearity(orc):
    log_n = 13
    for q in orc.choose_moduli(log_n, (60, 40)):
        psi = orc.find_psi(q, log_n)
        rng = random.Random(q)
        a = [rng.randrange(q) for _ in range(1 << log_n)]
        b = [rng.randrange(q) for _ in range(1 << log_n)]
        fa = orc.ntt_forward(a, log_n, q, psi)
        fb = orc.ntt_forward(b, log_n, q, psi)
        fab = orc.ntt_forward([(x + y) % q for x, y in zip(a, b)], log_n, q, psi)
        assert all(int(z) == (int(x) + int(y)) % q for x, y, z in zip(fa, fb, fab))
        assert [int(x) for x in orc.ntt_inverse(fa, log_n, q, psi)] == a
        # spot-check outputs against the defining sum
        for k in (0, 1, 777, (1 << log_n) - 1):
            e = 2 * brv(k, log_n) + 1
            want = sum(a[i] * pow(psi, e * i, q) for i in range(1 << log_n)) % q
            assert int(fa[k]) == want


def test_mulmod_powmod(orc):
    rng = random.Random(7)
    for _ in range(2000):
        q = rng.getrandbits(62) | 1
        a, b = rng.randrange(q), rng.randrange(q)
        assert orc.lib().oracle_mulmod(a, b, q) == (a * b) % q
        e = rng.getrandbits(64)
        assert orc.lib().oracle_powmod(a, e, q) == pow(a, e, q)


def test_paper_chain_is_881_bits(orc):
    """The paper's coefficient modulus (System Implementation section): 16
    primes near 2^55, the last near 2^56, 881 bits in all (the standard's
    maximum at N = 32768); each prime is = 1 mod 2N and they are distinct."""
    from paper_2408_07304_amd.workloads import P32768_Q16
    qs = orc.choose_moduli(P32768_Q16.log_n, P32768_Q16.bits)
    assert len(set(qs)) == 16
    Q = 1
    for q in qs:
        assert q % (2 * P32768_Q16.n) == 1 and orc.is_prime(q)
        Q *= q
    assert Q.bit_length() == 881
    assert [q.bit_length() for q in qs] == [55] * 15 + [56]
