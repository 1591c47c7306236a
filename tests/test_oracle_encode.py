"""Pins of the oracle's CKKS encoding and decoding (the paper takes both from
the CKKS paper; Scheme Flexibility section).  The oracle sums the canonical
embedding's defining series; here it is checked against closed forms, against
an independent route through numpy's FFT, and for invertibility and linearity."""
import numpy as np
import pytest

from paper_2408_07304_amd.workloads import P4096, P8192


def params(orc, ps):
    return orc.Params(ps.log_n, ps.bits, ps.scale, ps.seed)


def slot_exps(n):
    r = np.zeros(n // 2, dtype=np.int64)
    g = 1
    for j in range(n // 2):
        r[j] = g
        g = g * 5 % (2 * n)
    return r


def encode_by_numpy_fft(z, n, scale):
    """Independent route: the N/2-point DFT of the slots placed at positions
    k_j = (5^j mod 2N - 1)/4, twisted by zeta^-i; real and imaginary parts give
    the two halves of the coefficient vector."""
    h = n // 2
    r = slot_exps(n)
    Z = np.zeros(h, dtype=np.complex128)
    Z[(r - 1) // 4] = scale * np.asarray(z, dtype=np.float64)
    w = np.fft.fft(Z) * (2.0 / n)
    w *= np.exp(-1j * np.pi * np.arange(h) / n)
    return np.concatenate([w.real, w.imag])


@pytest.mark.parametrize("ps", [P4096, P8192], ids=["n4096", "n8192"])
def test_constant_slots_encode_to_constant_polynomial(orc, ps):
    P = params(orc, ps)
    for c in (0.0, 1.0, -0.375, 0.123456789):
        m, fr = orc.encode(P, np.full(P.n // 2, c))
        want = np.zeros(P.n, dtype=np.int64)
        want[0] = int(np.rint(c * P.scale))
        assert np.array_equal(m, want)


@pytest.mark.parametrize("ps", [P4096, P8192], ids=["n4096", "n8192"])
def test_cosine_slots_encode_to_x_minus_x_pow(orc, ps):
    """z_j = 2 cos(pi r_j / N) is the evaluation of X - X^(N-1) at zeta^(r_j)."""
    P = params(orc, ps)
    r = slot_exps(P.n)
    z = 2 * np.cos(np.pi * r / P.n)
    m, _ = orc.encode(P, z)
    want = np.zeros(P.n, dtype=np.int64)
    want[1] = int(P.scale)
    want[-1] = -int(P.scale)
    assert np.array_equal(m, want)
    dz = orc.decode(P, want)
    assert np.abs(dz - z).max() < 1e-12


@pytest.mark.parametrize("ps", [P4096, P8192], ids=["n4096", "n8192"])
def test_encode_matches_numpy_fft_route(orc, ps):
    P = params(orc, ps)
    rng = np.random.default_rng(3)
    z = rng.uniform(-1, 1, size=P.n // 2)
    m, fr = orc.encode(P, z)
    x_oracle = m.astype(np.float64) + fr
    x_fft = encode_by_numpy_fft(z, P.n, P.scale)
    err = np.abs(x_fft - x_oracle).max()
    assert err < 1e-13 * P.scale * np.log2(P.n)
    # integers agree except where the value sits within err of a half-integer
    tie = np.abs(np.abs(fr) - 0.5) <= 4 * err + 1e-9
    assert np.array_equal(m[~tie], np.rint(x_fft).astype(np.int64)[~tie])


@pytest.mark.parametrize("ps", [P4096, P8192], ids=["n4096", "n8192"])
def test_encode_decode_roundtrip_and_linearity(orc, ps):
    P = params(orc, ps)
    rng = np.random.default_rng(4)
    z1 = rng.uniform(-1, 1, size=P.n // 2)
    z2 = rng.uniform(-1, 1, size=P.n // 2)
    m1, _ = orc.encode(P, z1)
    m2, _ = orc.encode(P, z2)
    m12, _ = orc.encode(P, z1 + z2)
    assert np.abs(m12 - m1 - m2).max() <= 1
    bound = 8 * np.sqrt(P.n / 24) / P.scale + 1e-15
    assert np.abs(orc.decode(P, m1) - z1).max() < bound
    # fewer slots than N/2: zero padding
    zs = z1[:17]
    ms, _ = orc.encode(P, zs)
    back = orc.decode(P, ms)
    assert np.abs(back[:17] - zs).max() < bound and np.abs(back[17:]).max() < bound


def test_decode_of_constant(orc):
    P = params(orc, P4096)
    m = np.zeros(P.n, dtype=np.int64)
    m[0] = int(0.75 * P.scale)
    assert np.abs(orc.decode(P, m) - 0.75).max() < 1e-15
