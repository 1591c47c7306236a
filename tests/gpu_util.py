"""Helpers shared by the GPU tests: device buffers for uint64 data (carried in
int64 torch tensors) and cached contexts / oracle key material per parameter
set."""
import functools

import numpy as np
import pytest

import paper_2408_07304_amd as zinc
from paper_2408_07304_amd.workloads import PARAM_SETS


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_dev(a):
    torch = torch_cuda()
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a.copy()).to("cuda")


def from_dev(t, dtype=np.uint64):
    torch_cuda().cuda.synchronize()
    a = t.cpu().numpy()
    return a.view(dtype) if a.dtype == np.int64 and dtype == np.uint64 else a


def empty_u64(*shape):
    torch = torch_cuda()
    return torch.empty(shape, dtype=torch.int64, device="cuda")


def ids(values):
    return to_dev(np.asarray(values, dtype=np.uint64))


@functools.lru_cache(maxsize=None)
def gpu_ctx(name):
    ps = PARAM_SETS[name]
    print(f"[gpu] context {name} keygen+precompute", flush=True)
    c = zinc.context_for(ps)
    c.keygen()
    c.precompute()
    torch_cuda().cuda.synchronize()
    return c


@functools.lru_cache(maxsize=None)
def oracle_keys(name):
    import oracle
    ps = PARAM_SETS[name]
    P = oracle.Params(ps.log_n, ps.bits, ps.scale, ps.seed)
    sh, pk = oracle.keygen(P)
    zero = oracle.zinc_precompute(P, pk)
    return P, sh, pk, zero
