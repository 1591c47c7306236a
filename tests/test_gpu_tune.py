"""Tuning (zinc_set_tuning, zinc_autotune): every form of the fused kernel
(thread geometry, register or natural-order epilogue) and every choice of NTT
arithmetic must give ciphertexts bit-identical to the default configuration
(which the parity tests tie to the oracle), and the autotuner's cache must
reproduce its choice without timing."""
import numpy as np
import pytest

import paper_2408_07304_amd as zinc
from gpu_util import empty_u64, from_dev, gpu_ctx, ids, to_dev, torch_cuda
from paper_2408_07304_amd.workloads import PARAM_SETS

pytestmark = pytest.mark.gpu

# (coefficients per thread, register epilogue) forms per ring degree
FORMS = {"n4096": ((16, 0), (16, 1), (8, 0), (8, 1), (32, 0)), "n8192": ((16, 0), (16, 1), (8, 0), (8, 1), (32, 0)),
         "n16384": ((16, 0), (16, 1), (32, 0)), "n32768": ((16, 0),)}


def say(msg):
    print(f"[gpu] {msg}", flush=True)


def _encrypt(c, scheme, z, first_id=5):
    b = z.shape[0]
    out = empty_u64(b, 2, c.L, c.n)
    c.encrypt_slots(scheme, to_dev(z), ids(np.arange(first_id, first_id + b, dtype=np.uint64)), out)
    return from_dev(out)


@pytest.mark.parametrize("name", ["n4096", "n8192", "n16384"])
def test_every_tile_and_arithmetic_is_bit_identical(name):
    torch_cuda()
    c = gpu_ctx(name)
    ps = PARAM_SETS[name]
    default = c.get_tuning()
    rng = np.random.default_rng(21)
    z = rng.uniform(-1, 1, size=(5, ps.slots))
    z[3, ps.slots // 3:] = 0.0                       # a partly empty plaintext
    masks = sorted({default["ntt_fp64_mask"], 0})
    try:
        ref = {s: _encrypt(c, s, z) for s in (zinc.ZINC_SCHEME_VANILLA, zinc.ZINC_SCHEME_ZINC)}
        for mask in masks:
            for tile, reg in FORMS[name]:
                say(f"{name} tile {tile} register epilogue {reg} fp64 mask {mask:#x}")
                c.set_tuning(tile, tile, mask, 3 * reg)
                assert c.info()["tile"] == [tile, tile] and c.info()["reg_epilogue"] == 3 * reg
                for s in (zinc.ZINC_SCHEME_VANILLA, zinc.ZINC_SCHEME_ZINC):
                    assert np.array_equal(_encrypt(c, s, z), ref[s]), (tile, reg, mask, s)
    finally:
        c.set_tuning(*default["tile"], default["ntt_fp64_mask"], default["reg_epilogue"])


def test_set_tuning_rejects_unavailable_choices():
    torch_cuda()
    for name, bad in (("n16384", (8, 16, None, 0)), ("n32768", (32, 16, None, 0)), ("n8192", (16, 16, 1 << 0, 0)),
                      ("n32768", (16, 16, None, 1)), ("n16384", (32, 16, None, 1)), ("n8192", (16, 16, None, 4))):
        c = gpu_ctx(name)
        d = c.get_tuning()
        mask = d["ntt_fp64_mask"] if bad[2] is None else bad[2]       # limb 0 of n8192 is a 60-bit modulus
        with pytest.raises(zinc.ZincError) as e:
            c.set_tuning(bad[0], bad[1], mask, bad[3])
        assert e.value.status == zinc.ZINC_E_INVAL
        assert c.get_tuning() == d


def test_autotune_and_cache(tmp_path):
    torch_cuda()
    c = gpu_ctx("n8192")
    d = c.get_tuning()
    path = str(tmp_path / "tune.txt")
    try:
        r = c.autotune(batch=128, cache_path=path)
        say(f"autotune n8192: {r}")
        chosen = {"tile": r["tile"], "ntt_fp64_mask": r["ntt_fp64_mask"], "reg_epilogue": r["reg_epilogue"]}
        assert not r["from_cache"] and r["n_timed"] >= 2 * len(FORMS["n8192"])
        for s in (0, 1):
            assert (r["tile"][s], (r["reg_epilogue"] >> s) & 1) in FORMS["n8192"]
        assert min(r["best_ms"]) > 0 and min(r["default_ms"]) > 0
        assert r["best_ms"][0] <= r["default_ms"][0] * 1.05 and r["best_ms"][1] <= r["default_ms"][1] * 1.05
        assert c.get_tuning() == chosen
        c.set_tuning(*d["tile"], d["ntt_fp64_mask"], d["reg_epilogue"])
        again = c.autotune(batch=128, cache_path=path)
        assert again["from_cache"] and again["n_timed"] == 0
        assert {"tile": again["tile"], "ntt_fp64_mask": again["ntt_fp64_mask"],
                "reg_epilogue": again["reg_epilogue"]} == chosen
        assert c.get_tuning() == chosen
        lines = open(path).read().splitlines()
        assert len(lines) == 1 and lines[0].startswith("zinc-tune-2 ")
        # the tuned configuration still encrypts identically
        ps = PARAM_SETS["n8192"]
        z = np.random.default_rng(22).uniform(-1, 1, size=(3, ps.slots))
        tuned = _encrypt(c, zinc.ZINC_SCHEME_ZINC, z)
        c.set_tuning(*d["tile"], d["ntt_fp64_mask"], d["reg_epilogue"])
        assert np.array_equal(tuned, _encrypt(c, zinc.ZINC_SCHEME_ZINC, z))
    finally:
        c.set_tuning(*d["tile"], d["ntt_fp64_mask"], d["reg_epilogue"])
