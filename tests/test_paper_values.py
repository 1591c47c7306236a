"""The workload constants and the benchmark's context numbers against the
values the paper prints (tests/golden/paper_values.json, each entry cited):
the N = 32768 parameter set, the chi width, the dataset shapes of the
Experimental Setup section and the SEAL timings of Table 2."""
import json
import os

import pytest

import bench
import paper_2408_07304_amd as zinc
from paper_2408_07304_amd.workloads import P32768_Q16, TABLE2

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_paper_parameter_set(orc):
    g = GOLDEN
    assert 1 << P32768_Q16.log_n == g["ring_degree"]["value"]
    assert sum(P32768_Q16.bits) == g["coeff_modulus_bits_total"]["value"]
    assert set(P32768_Q16.bits[:-1]) == {g["coeff_modulus_prime_bits"]["middle"]}
    assert P32768_Q16.bits[-1] == g["coeff_modulus_prime_bits"]["last"]
    assert P32768_Q16.scale == 2.0 ** g["scale_log2"]["value"]
    # the primes the moduli rule picks have exactly those sizes, 881 bits in all
    qs = orc.choose_moduli(P32768_Q16.log_n, P32768_Q16.bits)
    assert sum(q.bit_length() for q in qs) == g["coeff_modulus_bits_total"]["value"]


def test_chi_width(orc):
    import inspect
    sigma = GOLDEN["chi_sigma"]["value"]
    assert inspect.signature(orc.Params.__init__).parameters["sigma"].default == sigma
    assert inspect.signature(zinc.Context.__init__).parameters["sigma"].default == sigma
    assert (orc.cdt_table() == orc.cdt_table(sigma)).all()


@pytest.mark.parametrize("name", ["covid19", "bitcoin", "hg38"])
def test_dataset_shapes_and_table2(name):
    d = {x.name: x for x in TABLE2}[name]
    g = GOLDEN["datasets"][name]
    assert d.rows == g["rows"]
    if g["values_per_row"] is not None:
        assert d.slots == g["values_per_row"]
    t2 = GOLDEN["table2_total_seconds"][name]
    assert bench.PAPER_TABLE2_S[name] == {"ckks": t2["ckks"], "zinc": t2["zinc"]}
