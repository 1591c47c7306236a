"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Bit-exact: tables, samplers, NTT/INTT, keys, the cached Enc(0), vanilla (Eq. 8)
and Zinc (Algorithm 1) ciphertexts from a shared integer plaintext,
decryption, homomorphic addition; the fused encode+encrypt launch equals
encode followed by encrypt.  Within tolerance: FP64 encoding (integer
coefficients equal except inside the rounding-tie window, where they may
differ by one, and no more such coefficients than the rounding model allows;
see gpu_util.check_encoding) and decoding (2^-20 in message units)."""
import os

import numpy as np
import pytest

import oracle
import paper_2408_07304_amd as zinc
from gpu_util import (centred, check_encoding, check_fused, empty_u64, from_dev, gpu_ctx, ids, oracle_keys, to_dev,
                      torch_cuda)
from paper_2408_07304_amd import PKG
from paper_2408_07304_amd.workloads import (PARAM_SETS, TABLE2, W_LARGE, W_MAIN, W_MIXED, W_SMALL, dataset_rows,
                                            make_slots)

pytestmark = pytest.mark.gpu

NAMES = ["n4096", "n8192", "n16384", "n32768", "n32768_q16"]
TUNE_CACHE = os.path.join(PKG, "tuning_cache.txt")
SCHEMES = [zinc.ZINC_SCHEME_VANILLA, zinc.ZINC_SCHEME_ZINC]


def say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.mark.parametrize("name", NAMES)
def test_tables_match_oracle(name):
    c = gpu_ctx(name)
    P, sh, pk, zero = oracle_keys(name)
    info = c.info()
    assert info["moduli"] == P.moduli
    assert info["psi"] == P.psi
    assert info["cdt"] == [int(x) for x in P.cdt]
    assert info["limbs"] == P.L and info["n"] == P.n


@pytest.mark.parametrize("name", NAMES)
def test_samplers_bit_exact(name):
    c = gpu_ctx(name)
    P = oracle_keys(name)[0]
    idv = [0, 1, 12345, 2 ** 40 + 7, zinc.ZINC_ZERO_ID, zinc.ZINC_KEY_ID]
    d_ids = ids(idv)
    out = empty_u64(len(idv), P.n)
    say(f"{name} sample ternary/gauss")
    for kind, tag, fn in ((zinc.SAMPLE_TERNARY, oracle.TAG_U, oracle.sample_ternary),
                          (zinc.SAMPLE_GAUSSIAN, oracle.TAG_E1Z, oracle.sample_gaussian)):
        c.sample(kind, tag, 0, d_ids, out)
        got = from_dev(out, np.int64)
        for i, cid in enumerate(idv):
            assert np.array_equal(got[i], fn(P.seed, cid, tag, P.n)), (kind, cid)
    say(f"{name} sample uniform")
    for limb in range(P.M):
        c.sample(zinc.SAMPLE_UNIFORM, oracle.TAG_A, limb, d_ids[:2], out[:2])
        got = from_dev(out[:2])
        for i, cid in enumerate(idv[:2]):
            assert np.array_equal(got[i], oracle.sample_uniform(P.seed, cid, oracle.TAG_A, limb, P.n,
                                                                P.moduli[limb]))


@pytest.mark.parametrize("name", NAMES)
def test_ntt_bit_exact(name):
    c = gpu_ctx(name)
    P = oracle_keys(name)[0]
    rng = np.random.default_rng(7)
    for limb, q in enumerate(P.moduli):
        a = rng.integers(0, q, size=(3, P.n), dtype=np.uint64)
        a[0, :] = 0
        a[0, 0] = 1                      # delta: transform is all ones
        a[1, :] = q - 1                  # maximal residues
        d = to_dev(a)
        say(f"{name} ntt limb {limb}")
        c.ntt_forward(limb, d)
        got = from_dev(d)
        for i in range(3):
            assert np.array_equal(got[i], oracle.ntt_forward(a[i], P.log_n, q, P.psi[limb])), (limb, i)
        assert np.all(got[0] == 1)
        c.ntt_inverse(limb, d)
        assert np.array_equal(from_dev(d), a)
        b = rng.integers(0, q, size=(2, P.n), dtype=np.uint64)
        d = to_dev(b)
        c.ntt_inverse(limb, d)
        got = from_dev(d)
        for i in range(2):
            assert np.array_equal(got[i], oracle.ntt_inverse(b[i], P.log_n, q, P.psi[limb]))


@pytest.mark.parametrize("name", NAMES)
def test_keys_and_cache_bit_exact(name):
    c = gpu_ctx(name)
    P, sh, pk, zero = oracle_keys(name)
    dsk, dpk, dz = empty_u64(P.M, P.n), empty_u64(2, P.M, P.n), empty_u64(2, P.L, P.n)
    c.export_keys(dsk, dpk, dz)
    assert np.array_equal(from_dev(dsk), sh)
    assert np.array_equal(from_dev(dpk), pk)
    assert np.array_equal(from_dev(dz), zero)


def _plaintexts(P, count, seed):
    """Integer plaintexts: small signed coefficients and uniformly random residues."""
    rng = np.random.default_rng(seed)
    pts = []
    for i in range(count):
        if i % 2 == 0:
            m = rng.integers(-(2 ** 40), 2 ** 40, size=P.n)
            pts.append(oracle.to_rns(P, m))
        else:
            pts.append(np.stack([rng.integers(0, q, size=P.n, dtype=np.uint64) for q in P.data_moduli]))
    return np.stack(pts)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("name", NAMES)
def test_encrypt_from_plaintext_bit_exact(name, scheme):
    c = gpu_ctx(name)
    P, sh, pk, zero = oracle_keys(name)
    B = 5
    pt = _plaintexts(P, B, 11 + scheme)
    idv = [3, 0, 99, 2 ** 33 + 1, 7]
    out = empty_u64(B, 2, P.L, P.n)
    say(f"{name} encrypt scheme={scheme} from plaintext")
    if scheme == zinc.ZINC_SCHEME_ZINC:
        c.encrypt(to_dev(pt), ids(idv), out)
    else:
        c.encrypt_vanilla(to_dev(pt), ids(idv), out)
    got = from_dev(out)
    for i in range(B):
        want = (oracle.encrypt_zinc(P, zero, pt[i], idv[i]) if scheme == zinc.ZINC_SCHEME_ZINC
                else oracle.encrypt_vanilla(P, pk, pt[i], idv[i]))
        assert np.array_equal(got[i], want), (i, idv[i])


@pytest.mark.parametrize("name", NAMES)
def test_encode_within_tie_window(name):
    c = gpu_ctx(name)
    P = oracle_keys(name)[0]
    w = {"n4096": W_SMALL, "n8192": W_MAIN, "n16384": W_LARGE, "n32768": W_MIXED, "n32768_q16": W_MIXED}[name]
    z = make_slots(w, 3, PARAM_SETS[name])
    z[2, 100:] = 0.0                                     # also a partly empty vector
    out = empty_u64(3, P.L, P.n)
    say(f"{name} encode")
    c.encode(to_dev(z), out)
    got = from_dev(out)
    gs, ms, frs = [], [], []
    for i in range(3):
        m, fr = oracle.encode(P, z[i])
        g = centred(got[i, 0], P.moduli[0])
        gs.append(g)
        ms.append(m)
        frs.append(fr)
        for l in range(1, P.L):     # every limb holds the same integer
            assert np.array_equal(got[i, l], oracle.to_rns(P, g, P.L)[l])
    mism = check_encoding(P.n, np.stack(gs), np.stack(ms), np.stack(frs), name)
    say(f"{name} encode: {mism} of {3 * P.n} coefficients rounded the other way")


@pytest.mark.parametrize("name", NAMES)
def test_encode_exact_at_moderate_magnitude(name):
    """Slot vectors scaled so that the coefficients have rms min(2^32, q_0/64)
    (within the centred range of limb 0): the tie window is then below 10^-4,
    so the whole transform (slot order, twist, unscrambling, every twiddle) is
    checked coefficient by coefficient at every ring degree, including those
    where full-size coefficients leave the window wider than the rounding
    grid.  (Uniform slots on [-a, a] give coefficients of rms
    a Delta / sqrt(3 N).)"""
    c = gpu_ctx(name)
    P = oracle_keys(name)[0]
    rng = np.random.default_rng(17)
    target = min(2.0 ** 32, P.moduli[0] / 64)
    z = rng.uniform(-1, 1, size=(2, P.n // 2)) * (target * np.sqrt(3 * P.n) / P.scale)
    z[1, 5:] = 0.0
    z[1, :5] = [target / P.scale, -1.5 / P.scale, 0.5 / P.scale, 2.5 / P.scale, 1.0 / P.scale]
    out = empty_u64(2, P.L, P.n)
    say(f"{name} encode at 2^32")
    c.encode(to_dev(z), out)
    got = from_dev(out)
    for i in range(2):
        m, fr = oracle.encode(P, z[i])
        g = centred(got[i, 0], P.moduli[0])
        mism = check_encoding(P.n, g, m, fr, (name, i))
        assert mism <= 2, (name, i, mism)


SPARSE_COUNTS = (1, 2, 3, 4, 5)     # the encoding kernel: up to three values summed directly, more transformed


@pytest.mark.parametrize("name", NAMES)
def test_encode_sparse_slot_vectors(name):
    """The encoding kernel sums slot vectors of at most three values term by
    term instead of transforming them.  Vectors of one to five values (up to
    the threshold and past it) against the
    oracle's encoding under check_encoding's rules, at unit magnitude and with
    coefficients of rms about min(2^32, q_0/64), where the tie window is far
    below the rounding grid."""
    c = gpu_ctx(name)
    P = oracle_keys(name)[0]
    rng = np.random.default_rng(29)
    for n in SPARSE_COUNTS:
        z = rng.uniform(-1, 1, size=(2, n))
        z[1] *= min(2.0 ** 32, P.moduli[0] / 64) * P.n / (2.0 * P.scale * np.sqrt(n))
        out = empty_u64(2, P.L, P.n)
        say(f"{name} encode {n} slot values")
        c.encode(to_dev(z), out)
        got = from_dev(out)
        for i in range(2):
            m, fr = oracle.encode(P, z[i])
            g = centred(got[i, 0], P.moduli[0])
            for l in range(1, P.L):
                assert np.array_equal(got[i, l], oracle.to_rns(P, g, P.L)[l]), (n, i, l)
            check_encoding(P.n, g, m, fr, (name, n, i))


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("name", NAMES)
def test_fused_sparse_rows_against_oracle(name, scheme):
    """Fused encryption of rows of one, three and four values (Table 2's rows
    hold 1 to 16; the fused kernels transform every vector) against the
    oracle's Algorithm 1 / Eq. 8 of the same slots."""
    c = gpu_ctx(name)
    P, sh, pk, zero = oracle_keys(name)
    key = zero if scheme == zinc.ZINC_SCHEME_ZINC else pk
    rng = np.random.default_rng(31 + scheme)
    for n in (1, 3, 4):
        z = rng.uniform(-1, 1, size=(3, n))
        cid = [5 * n, 5 * n + 1, 2 ** 40 + n]
        out = empty_u64(3, 2, P.L, P.n)
        say(f"{name} scheme={scheme} fused rows of {n} values")
        c.encrypt_slots(scheme, to_dev(z), ids(cid), out)
        got = from_dev(out)
        for i in range(3):
            check_fused(c, P, scheme, key, z[i], cid[i], got[i], (name, scheme, n, i))


@pytest.mark.parametrize("name", ["n4096", "n8192", "n16384"])
def test_small_batch_limb_split_equals_full_launch(name):
    """A batch of fewer ciphertexts than half the device's CUs spreads each
    ciphertext's data limbs over several workgroups (each draws the same noise
    and encodes the same message); its ciphertexts equal those of a batch large
    enough to take one workgroup per ciphertext, from slots and from
    plaintexts, for both schemes, and the first one equals the oracle's."""
    c = gpu_ctx(name)
    P, sh, pk, zero = oracle_keys(name)
    rng = np.random.default_rng(37)
    big_b = 300
    z = rng.uniform(-1, 1, size=(big_b, P.n // 2))
    pt = _plaintexts(P, 4, 43)
    for scheme in SCHEMES:
        key = zero if scheme == zinc.ZINC_SCHEME_ZINC else pk
        big = empty_u64(big_b, 2, P.L, P.n)
        small = empty_u64(3, 2, P.L, P.n)
        say(f"{name} scheme={scheme}: {big_b} slot vectors in one launch, then 3 alone")
        c.encrypt_slots(scheme, to_dev(z), ids(range(big_b)), big)
        c.encrypt_slots(scheme, to_dev(z[:3]), ids(range(3)), small)
        got_big, got_small = from_dev(big), from_dev(small)
        assert np.array_equal(got_big[:3], got_small), (name, scheme)
        check_fused(c, P, scheme, key, z[0], 0, got_small[0], (name, scheme, "split"))
        # plaintext path: 4 alone (split) against the same 4 inside a batch of big_b
        pts = np.concatenate([pt, np.repeat(pt[:1], big_b - 4, axis=0)])
        enc = c.encrypt if scheme == zinc.ZINC_SCHEME_ZINC else c.encrypt_vanilla
        outb = empty_u64(big_b, 2, P.L, P.n)
        outs = empty_u64(4, 2, P.L, P.n)
        enc(to_dev(pts), ids(range(100, 100 + big_b)), outb)
        enc(to_dev(pt), ids(range(100, 104)), outs)
        assert np.array_equal(from_dev(outb)[:4], from_dev(outs)), (name, scheme, "pt")


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("name", NAMES)
def test_fused_equals_encode_then_encrypt(name, scheme):
    c = gpu_ctx(name)
    P = oracle_keys(name)[0]
    z = make_slots(W_SMALL if name == "n4096" else W_MAIN, 6, PARAM_SETS[name])
    B = z.shape[0]
    d_ids = ids(range(40, 40 + B))
    f = empty_u64(B, 2, P.L, P.n)
    u = empty_u64(B, 2, P.L, P.n)
    pt = empty_u64(B, P.L, P.n)
    say(f"{name} fused vs unfused scheme={scheme}")
    c.encrypt_slots(scheme, to_dev(z), d_ids, f)
    c.encode(to_dev(z), pt)
    if scheme == zinc.ZINC_SCHEME_ZINC:
        c.encrypt(pt, d_ids, u)
    else:
        c.encrypt_vanilla(pt, d_ids, u)
    assert np.array_equal(from_dev(f), from_dev(u))
    # fewer slots than N/2 take the same path with zero padding
    zs = np.ascontiguousarray(z[:, :33])
    c.encrypt_slots(scheme, to_dev(zs), d_ids, f)
    c.encode(to_dev(zs), pt)
    (c.encrypt if scheme == zinc.ZINC_SCHEME_ZINC else c.encrypt_vanilla)(pt, d_ids, u)
    assert np.array_equal(from_dev(f), from_dev(u))


@pytest.mark.parametrize("name", NAMES)
def test_decrypt_bit_exact(name):
    c = gpu_ctx(name)
    P, sh, pk, zero = oracle_keys(name)
    pt = _plaintexts(P, 3, 5)
    cts = np.stack([oracle.encrypt_zinc(P, zero, pt[0], 1), oracle.encrypt_vanilla(P, pk, pt[1], 2),
                    oracle.encrypt_zinc(P, zero, pt[2], 3)])
    out = empty_u64(3, P.L, P.n)
    say(f"{name} decrypt")
    c.decrypt(to_dev(cts), out)
    got = from_dev(out)
    for i in range(3):
        assert np.array_equal(got[i], oracle.decrypt(P, sh, cts[i]))


@pytest.mark.parametrize("name", NAMES)
def test_decode_parity(name):
    c = gpu_ctx(name)
    P = oracle_keys(name)[0]
    rng = np.random.default_rng(9)
    z = rng.uniform(-1, 1, size=(2, P.n // 2))
    ms = [oracle.encode(P, z[i])[0] for i in range(2)]
    pt = np.stack([oracle.to_rns(P, m) for m in ms])
    out = torch_cuda().empty((2, P.n // 2), dtype=torch_cuda().float64, device="cuda")
    say(f"{name} decode")
    c.decode(to_dev(pt), out)
    got = from_dev(out, np.float64)
    for i in range(2):
        assert np.abs(got[i] - oracle.decode(P, ms[i])).max() <= 2.0 ** -20
    assert c.device_errors() == 0


def noise_bound(n, scale):
    return (20 * n * 3.2 + 6 * (n / 24) ** 0.5) / scale


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("name", NAMES)
def test_round_trip_within_noise_bound(name, scheme):
    c = gpu_ctx(name)
    P = oracle_keys(name)[0]
    B = 4
    z = np.random.default_rng(13).uniform(-1, 1, size=(B, P.n // 2))
    ct = empty_u64(B, 2, P.L, P.n)
    pt = empty_u64(B, P.L, P.n)
    torch = torch_cuda()
    zz = torch.empty((B, P.n // 2), dtype=torch.float64, device="cuda")
    say(f"{name} round trip scheme={scheme}")
    c.encrypt_slots(scheme, to_dev(z), ids(range(B)), ct)
    c.decrypt(ct, pt)
    c.decode(pt, zz)
    err = np.abs(from_dev(zz, np.float64) - z).max()
    assert err < noise_bound(P.n, P.scale), err
    assert c.device_errors() == 0


@pytest.mark.parametrize("name", NAMES)
def test_add_bit_exact(name):
    c = gpu_ctx(name)
    P, sh, pk, zero = oracle_keys(name)
    pt = _plaintexts(P, 2, 3)
    a = np.stack([oracle.encrypt_zinc(P, zero, pt[0], 10)] * 2)
    b = np.stack([oracle.encrypt_vanilla(P, pk, pt[1], 11), oracle.encrypt_zinc(P, zero, pt[1], 12)])
    out = empty_u64(2, 2, P.L, P.n)
    say(f"{name} add")
    c.add(to_dev(a), to_dev(b), out)
    got = from_dev(out)
    for i in range(2):
        assert np.array_equal(got[i], oracle.add(P, a[i], b[i]))


@pytest.mark.parametrize("scheme", SCHEMES)
def test_ciphertext_independent_of_batch_position(scheme):
    c = gpu_ctx("n8192")
    P = oracle_keys("n8192")[0]
    z = make_slots(W_MAIN, 9)
    idv = list(range(500, 509))
    big = empty_u64(9, 2, P.L, P.n)
    one = empty_u64(1, 2, P.L, P.n)
    say(f"batch invariance scheme={scheme}")
    c.encrypt_slots(scheme, to_dev(z), ids(idv), big)
    c.encrypt_slots(scheme, to_dev(z[4:5]), ids(idv[4:5]), one)
    assert np.array_equal(from_dev(big)[4], from_dev(one)[0])
    again = empty_u64(9, 2, P.L, P.n)
    c.encrypt_slots(scheme, to_dev(z), ids(idv), again)          # repeat run: deterministic
    assert np.array_equal(from_dev(big), from_dev(again))


def test_state_and_range_errors():
    torch_cuda()
    ps = PARAM_SETS["n4096"]
    c = zinc.context_for(ps)
    z = to_dev(np.zeros((1, ps.slots)))
    ct = empty_u64(1, 2, ps.limbs, ps.n)
    pt = empty_u64(1, ps.limbs, ps.n)
    with pytest.raises(zinc.ZincError) as e:
        c.encrypt_slots(zinc.ZINC_SCHEME_VANILLA, z, ids([0]), ct)
    assert e.value.status == zinc.ZINC_E_STATE
    with pytest.raises(zinc.ZincError) as e:
        c.precompute()
    assert e.value.status == zinc.ZINC_E_STATE
    c.keygen()
    with pytest.raises(zinc.ZincError) as e:
        c.encrypt(pt, ids([0]), ct)
    assert e.value.status == zinc.ZINC_E_STATE
    c.precompute()
    with pytest.raises(zinc.ZincError) as e:
        c.encode(to_dev(np.zeros((1, ps.slots + 1))), pt)
    assert e.value.status == zinc.ZINC_E_RANGE
    with pytest.raises(zinc.ZincError) as e:
        c.encrypt_slots(7, z, ids([0]), ct)
    assert e.value.status == zinc.ZINC_E_INVAL
    # a slot value whose scaled magnitude reaches 2^62 sets the device flag
    assert c.device_errors() == 0
    huge = np.full((1, ps.slots), 2.0 ** 40)       # coefficient 0 = Delta * 2^40 = 2^65
    huge[0, 1] = np.nan
    say("range flag")
    c.encode(to_dev(huge), pt)
    assert c.device_errors() & 1
    assert c.device_errors() == 0          # read-and-clear
    c.close()


def _check_one(c, P, scheme, key, z, cid, got, where):
    mism = check_fused(c, P, scheme, key, z, cid, got, where)
    if mism:
        say(f"  {where}: {mism} of {P.n} coefficients of c1's message rounded the other way")


def _check_fused_against_oracle(name, w, picks, scheme):
    """Full-size batch in the launch configuration the benchmark times; sampled
    ciphertexts checked one by one against the oracle: c2 bit-exact, c1 equal
    up to NTT(delta) with delta in {-1, 0, 1} under the encoding rule of
    gpu_util.check_encoding."""
    c = gpu_ctx(name)
    P, sh, pk, zero = oracle_keys(name)
    z = make_slots(w)
    B = z.shape[0]
    ct = empty_u64(B, 2, P.L, P.n)
    # the kernel form the benchmark runs: its autotuning, from the committed cache
    default = c.get_tuning()
    tuned = c.autotune(batch=B, cache_path=TUNE_CACHE)
    say(f"{name} full batch B={B} scheme={scheme} form {tuned}")
    try:
        c.encrypt_slots(scheme, to_dev(z), ids(range(B)), ct)
    finally:
        c.set_tuning(*default["tile"], default["ntt_fp64_mask"], default["reg_epilogue"])
    torch = torch_cuda()
    sel = from_dev(ct[torch.tensor(picks, device="cuda")].contiguous())
    got = {i: sel[k] for k, i in enumerate(picks)}
    key = zero if scheme == zinc.ZINC_SCHEME_ZINC else pk
    for i in picks:
        _check_one(c, P, scheme, key, z[i], i, got[i], i)
    return got


# the special-prime form too: the benchmark times it on this batch
@pytest.mark.parametrize("scheme", SCHEMES + [zinc.ZINC_SCHEME_VANILLA_SP])
def test_full_batch_n8192_sampled(scheme):
    _check_fused_against_oracle("n8192", W_MAIN, [0, 1, 511, 1023], scheme)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_full_batch_n16384_sampled(scheme):
    _check_fused_against_oracle("n16384", W_LARGE, [0, 4095], scheme)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_full_batch_n4096(scheme):
    _check_fused_against_oracle("n4096", W_SMALL, list(range(0, 64, 9)), scheme)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_table2_shapes_at_paper_parameters(scheme):
    """The paper's parameters (N = 32768, 16 primes, Delta = 2^55) on rows of
    the shapes of its evaluation datasets (16, 1 and 3 values per row, padded
    with zeros to N/2 slots): sampled ciphertexts against the oracle as in the
    full-batch tests."""
    c = gpu_ctx("n32768_q16")
    P, sh, pk, zero = oracle_keys("n32768_q16")
    key = zero if scheme == zinc.ZINC_SCHEME_ZINC else pk
    for d in TABLE2:
        z = dataset_rows(d, 0, 3)
        ct = empty_u64(3, 2, P.L, P.n)
        first = 1000 * len(d.name)
        say(f"table-2 shape {d.name} ({d.slots} values per row) scheme={scheme}")
        c.encrypt_slots(scheme, to_dev(z), ids(range(first, first + 3)), ct)
        got = from_dev(ct)
        for i in range(3):
            _check_one(c, P, scheme, key, z[i], first + i, got[i], (d.name, i))


@pytest.mark.parametrize("scheme", SCHEMES + [zinc.ZINC_SCHEME_VANILLA_SP])
def test_table2_hg38_launch_configuration(scheme):
    """hg38's shape at the paper's parameters in the launch configuration the
    benchmark times (the whole dataset's rows, launches of 1,024 rows into one
    reused buffer): the first full launch and the ragged last one (632 rows,
    identifiers up to 34,423), sampled rows against the oracle."""
    torch = torch_cuda()
    c = gpu_ctx("n32768_q16")
    P, sh, pk, zero = oracle_keys("n32768_q16")
    key = zero if scheme == zinc.ZINC_SCHEME_ZINC else pk
    d = next(x for x in TABLE2 if x.name == "hg38")
    chunk = 1024
    rows = dataset_rows(d, 0, d.rows)
    ids_all = ids(range(d.rows))
    z_all = to_dev(rows)
    ct = empty_u64(chunk, 2, P.L, P.n)
    last = (d.rows - 1) // chunk * chunk
    for s0, picks in ((0, [0, 511, 1023]), (last, [0, d.rows - 1 - last])):
        n = min(chunk, d.rows - s0)
        say(f"hg38 rows {s0}..{s0 + n - 1} scheme={scheme}")
        c.encrypt_slots(scheme, z_all[s0:s0 + n], ids_all[s0:s0 + n], ct[:n])
        sel = from_dev(ct[torch.tensor(picks, device="cuda")].contiguous())
        for k, i in enumerate(picks):
            _check_one(c, P, scheme, key, rows[s0 + i], s0 + i, sel[k], s0 + i)
    del ct
