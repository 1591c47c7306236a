"""Pins of the oracle's BGV form (Scheme Flexibility section, Eq. 13: the
errors of the key, of Enc and of Zinc's e' are scaled by the plaintext modulus
t), against exact identities with every noise polynomial recomputed by numpy's
negacyclic convolution:

  * Gen:    INTT(pk1 + pk2 s_hat) = t e;
  * Enc:    Dec(c) - m = t (e u + e1 + e2 s);
  * Enc_z:  Dec(c') - m = t (e u0 + e10 + e1' + (e20 + e2') s);
  * decoding: decode(decrypt(encrypt(encode(m)))) = m, for Zinc and vanilla."""
import numpy as np
import pytest

from paper_2408_07304_amd.workloads import P4096, P8192

from test_oracle_scheme import negacyclic, residues


@pytest.fixture(scope="module", params=[(P4096, 65537), (P8192, 257)], ids=["n4096_t65537", "n8192_t257"])
def bgv(request, orc):
    ps, t = request.param
    P = orc.Params(ps.log_n, ps.bits, ps.scale, ps.seed, bgv_t=t)
    sh, pk = orc.keygen(P)
    zero = orc.zinc_precompute(P, pk)
    s = orc.sample_ternary(P.seed, orc.KEY_ID, orc.TAG_SK, P.n)
    e = orc.sample_gaussian(P.seed, orc.KEY_ID, orc.TAG_EPK, P.n)
    return P, t, sh, pk, zero, s, e


def test_bgv_key_identity(orc, bgv):
    P, t, sh, pk, zero, s, e = bgv
    for l, q in enumerate(P.moduli):
        x = [(int(a) + int(b) * int(c)) % q for a, b, c in zip(pk[0, l], pk[1, l], sh[l])]
        assert np.array_equal(orc.ntt_inverse(x, P.log_n, q, P.psi[l]), residues(t * e, [q])[0])


def test_bgv_vanilla_and_zinc_identities(orc, bgv):
    P, t, sh, pk, zero, s, e = bgv
    rng = np.random.default_rng(t)
    m = rng.integers(-(t // 2), t // 2 + 1, size=P.n)
    pt = orc.bgv_encode(P, t, m)
    mr = np.array([int(x) % t for x in m], dtype=np.int64)        # the encoded representative
    ct_id = 17
    u = orc.sample_ternary(P.seed, ct_id, orc.TAG_U, P.n)
    e1 = orc.sample_gaussian(P.seed, ct_id, orc.TAG_E1, P.n)
    e2 = orc.sample_gaussian(P.seed, ct_id, orc.TAG_E2, P.n)
    v = t * (negacyclic(e, u) + e1 + negacyclic(e2, s))
    assert np.array_equal(orc.decrypt(P, sh, orc.encrypt_vanilla(P, pk, pt, ct_id)), residues(mr + v, P.data_moduli))
    u0 = orc.sample_ternary(P.seed, orc.ZERO_ID, orc.TAG_U, P.n)
    e10 = orc.sample_gaussian(P.seed, orc.ZERO_ID, orc.TAG_E1, P.n)
    e20 = orc.sample_gaussian(P.seed, orc.ZERO_ID, orc.TAG_E2, P.n)
    e1z = orc.sample_gaussian(P.seed, ct_id, orc.TAG_E1Z, P.n)
    e2z = orc.sample_gaussian(P.seed, ct_id, orc.TAG_E2Z, P.n)
    vz = t * (negacyclic(e, u0) + e10 + e1z + negacyclic(e20 + e2z, s))
    assert np.array_equal(orc.decrypt(P, sh, orc.encrypt_zinc(P, zero, pt, ct_id)), residues(mr + vz, P.data_moduli))


def test_bgv_round_trip(orc, bgv):
    P, t, sh, pk, zero, s, e = bgv
    rng = np.random.default_rng(t + 1)
    m = rng.integers(-(t // 2), t // 2 + 1, size=P.n)
    pt = orc.bgv_encode(P, t, m)
    for ct in (orc.encrypt_zinc(P, zero, pt, 3), orc.encrypt_vanilla(P, pk, pt, 3)):
        assert np.array_equal(orc.bgv_decode(P, t, orc.decrypt(P, sh, ct)), m)
