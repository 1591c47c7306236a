"""Seeded synthetic workloads (parameter sets and input generators).

This module holds no arithmetic of the encryption method: only the parameter
sets of the benchmark configurations and seeded generators of the plaintext
slot vectors, ciphertext identifiers, mixed-batch item lists and serving
arrival traces.  Both the GPU path and the CPU oracle are fed from here.

The paper's own evaluation datasets (U.S. Covid-19 statistics, Bitcoin trade
volume, the hg38 table; Experimental Setup section) are not available; the
synthetic inputs below stand in for them.  Values are uniform on [-1, 1) or a
clipped standard normal, the distributions of the benchmark configurations.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class ParamSet:
    name: str
    log_n: int
    bits: tuple            # moduli bit sizes; the last modulus is the special prime
    scale: float           # Delta
    seed: int = 0          # scheme randomness seed (Philox key)

    @property
    def n(self) -> int:
        return 1 << self.log_n

    @property
    def slots(self) -> int:
        return self.n // 2

    @property
    def n_moduli(self) -> int:
        return len(self.bits)

    @property
    def limbs(self) -> int:
        return len(self.bits) - 1


# N = 4096: two 30-bit data primes plus one 30-bit special prime, Delta = 2^25.
P4096 = ParamSet("n4096", 12, (30, 30, 30), 2.0 ** 25)
# N = 8192: [60, 40, 40 | 60], Delta = 2^40.
P8192 = ParamSet("n8192", 13, (60, 40, 40, 60), 2.0 ** 40)
# N = 16384: [60, 50 x 6 | 60], Delta = 2^50.
P16384 = ParamSet("n16384", 14, (60, 50, 50, 50, 50, 50, 50, 60), 2.0 ** 50)
# N = 32768: 15 x 55-bit primes (14 data limbs + special), Delta = 2^55
# (the paper's ring degree and scale; System Implementation section).
P32768 = ParamSet("n32768", 15, (55,) * 15, 2.0 ** 55)

# The paper's own parameters (System Implementation section): N = 32768 and a
# 881-bit chain of 16 primes near 2^55, the last near 2^56 (15 data limbs plus
# the special prime here), Delta = 2^55.
P32768_Q16 = ParamSet("n32768_q16", 15, (55,) * 15 + (56,), 2.0 ** 55)

PARAM_SETS = {p.name: p for p in (P4096, P8192, P16384, P32768, P32768_Q16)}


@dataclass(frozen=True)
class Workload:
    name: str
    params: tuple          # one ParamSet, or several for the mixed batch
    batch: int
    dist: str              # "uniform" on [-1,1) or "gauss_clip8"
    data_seed: int


W_SMALL = Workload("n4096_b64", (P4096,), 64, "uniform", 0)
W_MAIN = Workload("n8192_b1024", (P8192,), 1024, "uniform", 2)
W_LARGE = Workload("n16384_b4096", (P16384,), 4096, "gauss_clip8", 3)
W_MIXED = Workload("mixed_b2048", (P4096, P8192, P16384, P32768), 2048, "uniform", 4)
WORKLOADS = {w.name: w for w in (W_SMALL, W_MAIN, W_LARGE, W_MIXED)}


@dataclass(frozen=True)
class DatasetShape:
    """Shape of one of the paper's evaluation datasets (Experimental Setup
    section): one ciphertext per row, `slots` values per row.  The datasets
    themselves are not available; rows are filled with uniform [-1, 1)
    values (their value distributions are not stated either)."""
    name: str
    rows: int
    slots: int
    data_seed: int


# 341 days x 16 metrics; 1,086 trade volumes; 34,424 rows whose attribute count
# the paper does not give (three are named: transcription positions, coding
# regions, number of exons), read here as 3 values per row.
TABLE2 = (DatasetShape("covid19", 341, 16, 6), DatasetShape("bitcoin", 1086, 1, 7),
          DatasetShape("hg38", 34424, 3, 8))


def dataset_rows(d: DatasetShape, first: int, count: int) -> np.ndarray:
    """float64 [count][d.slots] values of rows first .. first + count - 1."""
    rng = np.random.default_rng([d.data_seed, first])
    return rng.uniform(-1.0, 1.0, size=(count, d.slots))


def slot_values(rng: np.random.Generator, count: int, n_slots: int, dist: str) -> np.ndarray:
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, size=(count, n_slots))
    if dist == "gauss_clip8":
        return np.clip(rng.standard_normal(size=(count, n_slots)), -8.0, 8.0)
    raise ValueError(dist)


def make_slots(w: Workload, count: int | None = None, params: ParamSet | None = None) -> np.ndarray:
    """float64 [count][N/2] slot vectors of a single-parameter workload."""
    p = params or w.params[0]
    rng = np.random.default_rng(w.data_seed)
    return slot_values(rng, w.batch if count is None else count, p.slots, w.dist)


def make_ct_ids(count: int, first: int = 0) -> np.ndarray:
    return np.arange(first, first + count, dtype=np.uint64)


@dataclass
class MixedBatch:
    """Items of a mixed batch: per item its parameter-set index, slot offset
    (in float64 elements), ciphertext offset (in uint64 words) and ct_id."""
    params: tuple
    ctx_idx: np.ndarray
    slot_off: np.ndarray
    ct_off: np.ndarray
    ct_id: np.ndarray
    slots: np.ndarray          # flat float64
    ct_words: int


def make_mixed(w: Workload = W_MIXED, count: int | None = None) -> MixedBatch:
    """Mixed batch: each plaintext draws its parameter set uniformly from
    w.params; slots are uniform on [-1, 1) (N/2 of them)."""
    rng = np.random.default_rng(w.data_seed)
    b = w.batch if count is None else count
    idx = rng.integers(0, len(w.params), size=b)
    slot_off = np.zeros(b, dtype=np.uint64)
    ct_off = np.zeros(b, dtype=np.uint64)
    chunks = []
    so = co = 0
    for i in range(b):
        p = w.params[int(idx[i])]
        slot_off[i] = so
        ct_off[i] = co
        chunks.append(slot_values(rng, 1, p.slots, w.dist)[0])
        so += p.slots
        co += 2 * p.limbs * p.n
    return MixedBatch(w.params, idx.astype(np.uint32), slot_off, ct_off,
                      np.arange(b, dtype=np.uint64), np.concatenate(chunks), co)


@dataclass
class Trace:
    """Open-loop arrival trace of a serving workload.  Per request: arrival
    (ns after the start), parameter-set index, plaintext count, offset of its
    first slot vector in `slots` (float64 elements; plaintext k follows at
    + k*N/2), first ct_id (plaintext k gets ct_id + k; identifiers are
    consecutive over the trace) and offset of its first ciphertext in a buffer
    of ct_words uint64 holding every output in request order."""
    params: tuple
    arrival_ns: np.ndarray
    ctx_idx: np.ndarray
    n_pt: np.ndarray
    slot_off: np.ndarray
    ct_id: np.ndarray
    ct_off: np.ndarray
    ct_words: int
    slots: np.ndarray          # flat float64 slot pool

    def __len__(self) -> int:
        return len(self.n_pt)

    @property
    def plaintexts(self) -> int:
        return int(self.n_pt.sum())


def make_trace(n_requests: int, rate_per_s: float, params: tuple = W_MIXED.params, seed: int = 5,
               max_count: int = 64, pool: int | None = None) -> Trace:
    """Poisson arrivals at rate_per_s (exponential gaps), request size uniform
    on {1..max_count}, parameter set uniform over `params`, slots uniform on
    [-1, 1).  pool=None gives every plaintext its own slot vector; otherwise
    each parameter set has a pool of `pool` (>= max_count) slot vectors and a
    request reads `count` consecutive ones from a uniformly drawn start."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    arrival_ns = np.round(np.cumsum(gaps) * 1e9).astype(np.uint64)
    pidx = rng.integers(0, len(params), size=n_requests).astype(np.uint32)
    cnt = rng.integers(1, max_count + 1, size=n_requests).astype(np.uint32)
    ct_id = np.zeros(n_requests, dtype=np.uint64)
    ct_id[1:] = np.cumsum(cnt[:-1], dtype=np.uint64)
    words = np.array([2 * p.limbs * p.n for p in params], dtype=np.uint64)
    per_req = cnt.astype(np.uint64) * words[pidx]
    ct_off = np.zeros(n_requests, dtype=np.uint64)
    ct_off[1:] = np.cumsum(per_req[:-1], dtype=np.uint64)
    slot_off = np.zeros(n_requests, dtype=np.uint64)
    if pool is None:
        sizes = cnt.astype(np.uint64) * np.array([p.slots for p in params], dtype=np.uint64)[pidx]
        slot_off[1:] = np.cumsum(sizes[:-1], dtype=np.uint64)
        slots = rng.uniform(-1.0, 1.0, size=int(sizes.sum()))
    else:
        if pool < max_count:
            raise ValueError("pool must hold at least max_count slot vectors")
        base = np.cumsum([0] + [pool * p.slots for p in params])
        slots = rng.uniform(-1.0, 1.0, size=int(base[-1]))
        start = rng.integers(0, pool - cnt + 1)
        per = np.array([p.slots for p in params], dtype=np.uint64)[pidx]
        slot_off = np.asarray(base[:-1], dtype=np.uint64)[pidx] + start.astype(np.uint64) * per
    return Trace(params, arrival_ns, pidx, cnt, slot_off, ct_id, ct_off, int(per_req.sum()), slots)


def trace_requests(tr: Trace) -> np.ndarray:
    """Requests of a trace as a structured array (ctx_idx, n_pt, slot_off,
    ct_off, ct_id), the field layout of the library's request records."""
    dt = np.dtype([("ctx_idx", "<u4"), ("n_pt", "<u4"), ("slot_off", "<u8"), ("ct_off", "<u8"),
                   ("ct_id", "<u8")])
    out = np.zeros(len(tr), dtype=dt)
    out["ctx_idx"], out["n_pt"], out["slot_off"] = tr.ctx_idx, tr.n_pt, tr.slot_off
    out["ct_off"], out["ct_id"] = tr.ct_off, tr.ct_id
    return out
