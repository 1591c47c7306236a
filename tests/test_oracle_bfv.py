"""Pins of the oracle's BFV functions (Scheme Flexibility section, Eq. 12):
the scale Delta = floor(Q/t) by its definition, decoding's rounding boundary
at Delta/2, and Zinc and vanilla encryptions of scaled plaintexts decrypting
and decoding to the message (Zinc works on BFV without modification)."""
import numpy as np
import pytest

from paper_2408_07304_amd.workloads import P4096, P8192

TS = [257, 65537, (1 << 20) + 7]


@pytest.fixture(scope="module", params=[P4096, P8192], ids=["n4096", "n8192"])
def setup(request, orc):
    ps = request.param
    P = orc.Params(ps.log_n, ps.bits, ps.scale, ps.seed)
    sh, pk = orc.keygen(P)
    return P, sh, pk, orc.zinc_precompute(P, pk)


def test_delta_and_unit_plaintext(orc, setup):
    P = setup[0]
    Q = 1
    for q in P.data_moduli:
        Q *= int(q)
    for t in TS:
        d = orc.bfv_delta(P, t)
        assert d * t <= Q < (d + 1) * t
        one = np.zeros(P.n, dtype=np.int64)
        one[3] = 1
        pt = orc.bfv_encode(P, t, one)
        for l, q in enumerate(P.data_moduli):
            assert int(pt[l][3]) == d % int(q) and int(pt[l].astype(object).sum()) == d % int(q)


def test_decode_rounds_at_half_delta(orc, setup):
    """Delta m + v decodes to m for |v| < Delta/2 and to m + 1 past it."""
    P = setup[0]
    t = 65537
    d = orc.bfv_delta(P, t)
    m = np.array([5, -7, 0, 32768] + [1] * (P.n - 4), dtype=np.int64)
    for v, shift in ((d // 2 - d // 100, 0), (-(d // 2) + d // 100, 0), (d // 2 + d // 100, 1)):
        x = [(d * (int(a) % t) + v) for a in m]
        pt = np.array([[xi % int(q) for xi in x] for q in P.data_moduli], dtype=np.uint64)
        got = orc.bfv_decode(P, t, pt)
        want = np.array([((int(a) + shift) % t) for a in m], dtype=np.int64)
        want = np.where(want > t // 2, want - t, want)
        assert np.array_equal(got, want), v


@pytest.mark.parametrize("t", TS)
def test_zinc_and_vanilla_encrypt_bfv_plaintexts(orc, setup, t):
    P, sh, pk, zero = setup
    rng = np.random.default_rng(t)
    m = rng.integers(-(t // 2), t // 2 + 1, size=P.n)
    pt = orc.bfv_encode(P, t, m)
    for ct_id in (4, 2 ** 40 + 1):
        for ct in (orc.encrypt_zinc(P, zero, pt, ct_id), orc.encrypt_vanilla(P, pk, pt, ct_id)):
            assert np.array_equal(orc.bfv_decode(P, t, orc.decrypt(P, sh, ct)), m)
