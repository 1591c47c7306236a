"""The element-wise steps alone (zinc_elementwise_zinc: Algorithm 1's
additions; zinc_elementwise_vanilla: Eq. 8's products and additions), bit-exact
against the oracle's element-wise functions on random canonical residues, at
the residue extremes, in place, and composed with transforms of the samples
into whole encryptions."""
import numpy as np
import pytest

import paper_2408_07304_amd as zinc
from gpu_util import empty_u64, from_dev, gpu_ctx, oracle_keys, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

NAMES = ["n4096", "n8192", "n16384", "n32768"]


def _random_residues(P, rng, shape_lead):
    out = np.empty(shape_lead + (P.L, P.n), dtype=np.uint64)
    for l, q in enumerate(P.data_moduli):
        out[..., l, :] = rng.integers(0, q, size=shape_lead + (P.n,), dtype=np.uint64)
    return out


@pytest.mark.parametrize("name", NAMES)
def test_elementwise_bit_exact(name):
    import oracle
    torch_cuda()
    c = gpu_ctx(name)
    P, sh, pk, zero = oracle_keys(name)
    rng = np.random.default_rng(31)
    B = 3
    hat = _random_residues(P, rng, (B, 2))
    uhat = _random_residues(P, rng, (B,))
    hat[1] = np.array(P.data_moduli, dtype=np.uint64)[None, :, None] - 1      # every residue q - 1
    uhat[1] = np.array(P.data_moduli, dtype=np.uint64)[:, None] - 1
    out = empty_u64(B, 2, P.L, P.n)
    c.elementwise_zinc(to_dev(hat), out)
    gz = from_dev(out)
    c.elementwise_vanilla(to_dev(uhat), to_dev(hat), out)
    gv = from_dev(out)
    for b in range(B):
        assert np.array_equal(gz[b], oracle.elementwise_zinc(P, zero, hat[b])), b
        assert np.array_equal(gv[b], oracle.elementwise_vanilla(P, pk, uhat[b], hat[b])), b
    # in place
    d = to_dev(hat)
    c.elementwise_zinc(d, d)
    assert np.array_equal(from_dev(d), gz)
    d = to_dev(hat)
    c.elementwise_vanilla(to_dev(uhat), d, d)
    assert np.array_equal(from_dev(d), gv)


@pytest.mark.parametrize("name", ["n4096", "n8192"])
def test_elementwise_composes_to_encryption(name):
    """Fed with the transforms of one ciphertext's samples (oracle-made), the
    element-wise steps give that ciphertext exactly."""
    import oracle
    torch_cuda()
    c = gpu_ctx(name)
    P, sh, pk, zero = oracle_keys(name)
    rng = np.random.default_rng(32)
    m = rng.integers(-(2 ** 20), 2 ** 20, size=P.n)
    pt = oracle.to_rns(P, m)
    ct_id = 99

    def transform(poly):
        return np.stack([oracle.ntt_forward([int(x) % q for x in poly], P.log_n, q, P.psi[l])
                         for l, q in enumerate(P.data_moduli)])

    e1z = oracle.sample_gaussian(P.seed, ct_id, oracle.TAG_E1Z, P.n)
    e2z = oracle.sample_gaussian(P.seed, ct_id, oracle.TAG_E2Z, P.n)
    hat = np.stack([transform(m + e1z), transform(e2z)])[None]
    out = empty_u64(1, 2, P.L, P.n)
    c.elementwise_zinc(to_dev(hat), out)
    assert np.array_equal(from_dev(out)[0], oracle.encrypt_zinc(P, zero, pt, ct_id))

    u = oracle.sample_ternary(P.seed, ct_id, oracle.TAG_U, P.n)
    e1 = oracle.sample_gaussian(P.seed, ct_id, oracle.TAG_E1, P.n)
    e2 = oracle.sample_gaussian(P.seed, ct_id, oracle.TAG_E2, P.n)
    hat = np.stack([transform(m + e1), transform(e2)])[None]
    c.elementwise_vanilla(to_dev(transform(u)[None]), to_dev(hat), out)
    assert np.array_equal(from_dev(out)[0], oracle.encrypt_vanilla(P, pk, pt, ct_id))


def test_elementwise_state_errors():
    torch_cuda()
    from paper_2408_07304_amd.workloads import P4096
    fresh = zinc.context_for(P4096)
    buf = empty_u64(1, 2, P4096.limbs, P4096.n)
    with pytest.raises(zinc.ZincError) as e:
        fresh.elementwise_vanilla(buf[:, 0], buf, buf)
    assert e.value.status == zinc.ZINC_E_STATE
    fresh.keygen()
    with pytest.raises(zinc.ZincError) as e:
        fresh.elementwise_zinc(buf, buf)
    assert e.value.status == zinc.ZINC_E_STATE
    fresh.close()
