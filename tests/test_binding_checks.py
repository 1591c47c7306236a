"""CPU checks of the Python binding's argument checks: every buffer must be a
contiguous torch tensor in GPU memory, of the dtype the call takes (int64
carrying uint64 data, or float64) and at least as long as the call's batch
implies.  A host tensor, a wrong dtype or a short buffer raises before
anything reaches the library, so no kernel can run off the end of a buffer.
These run without a GPU: the checks need only a context's sizes."""
import numpy as np
import pytest
import torch

import paper_2408_07304_amd as zinc


class _Meta:
    """Stands in for a device tensor: the attributes the checks read, with
    device 'cuda', and no memory behind it (the checks reject it or, in the
    passing case, the call is never made)."""

    def __init__(self, shape, dtype=torch.int64, device="cuda", contiguous=True):
        self.shape = tuple(shape)
        self.ndim = len(self.shape)
        self.dtype = dtype
        self.device = torch.device(device)
        self._contig = contiguous

    def numel(self):
        return int(np.prod(self.shape)) if self.shape else 1

    def is_contiguous(self):
        return self._contig

    def data_ptr(self):
        return 0x1000


@pytest.fixture
def meta_tensor():
    return _Meta


def _ctx(n=4096, L=2, M=3):
    c = object.__new__(zinc.Context)
    c.handle = None
    c.n, c.L, c.M = n, L, M
    return c


def test_host_tensor_is_rejected():
    c = _ctx()
    pt = torch.zeros((1, c.L, c.n), dtype=torch.int64)            # host memory
    with pytest.raises(ValueError, match="GPU memory"):
        c.encrypt(pt, torch.zeros(1, dtype=torch.int64), torch.zeros((1, 2, c.L, c.n), dtype=torch.int64))


def test_non_tensor_is_rejected():
    c = _ctx()
    with pytest.raises(TypeError, match="torch tensor"):
        c.decrypt(np.zeros((1, 2, c.L, c.n), dtype=np.int64), np.zeros((1, c.L, c.n), dtype=np.int64))


@pytest.mark.parametrize("call", ["encrypt", "encrypt_vanilla", "encrypt_vanilla_sp"])
def test_encrypt_buffers_checked(meta_tensor, call):
    c = _ctx()
    pt, ids_, ct = meta_tensor((2, c.L, c.n)), meta_tensor((2,)), meta_tensor((2, 2, c.L, c.n))
    fn = getattr(c, call)
    with pytest.raises(TypeError, match="int64"):
        fn(meta_tensor((2, c.L, c.n), torch.float64), ids_, ct)
    with pytest.raises(ValueError, match="needs"):
        fn(pt, meta_tensor((1,)), ct)                                   # one identifier for two plaintexts
    with pytest.raises(ValueError, match="needs"):
        fn(pt, ids_, meta_tensor((2, 2, c.L, c.n - 1)))                 # output one row short
    with pytest.raises(ValueError, match="contiguous"):
        fn(meta_tensor((2, c.L, c.n), contiguous=False), ids_, ct)
    with pytest.raises(ValueError, match="GPU memory"):
        fn(pt, meta_tensor((2,), device="cpu"), ct)


def test_slot_calls_checked(meta_tensor):
    c = _ctx()
    z, ids_ = meta_tensor((3, 100), torch.float64), meta_tensor((3,))
    with pytest.raises(TypeError, match="float64"):
        c.encrypt_slots(1, meta_tensor((3, 100), torch.float32), ids_, meta_tensor((3, 2, c.L, c.n)))
    with pytest.raises(ValueError, match="needs"):
        c.encrypt_slots(1, z, ids_, meta_tensor((2, 2, c.L, c.n)))     # output for two of three
    with pytest.raises(ValueError, match=r"\[batch\]\[n_slots\]"):
        c.encode(meta_tensor((300,), torch.float64), meta_tensor((3, c.L, c.n)))
    with pytest.raises(ValueError, match="needs"):
        c.encode(z, meta_tensor((3, c.L, c.n - 1)))
    with pytest.raises(TypeError, match="float64"):
        c.decode(meta_tensor((3, c.L, c.n)), meta_tensor((3, c.n // 2)))      # decode writes float64
    with pytest.raises(ValueError, match="needs"):
        c.decode(meta_tensor((3, c.L, c.n)), meta_tensor((3, c.n // 2 - 1), torch.float64))


def test_other_calls_checked(meta_tensor):
    c = _ctx()
    ct, pt = meta_tensor((2, 2, c.L, c.n)), meta_tensor((2, c.L, c.n))
    short_ct = meta_tensor((2, 2, c.L, c.n - 1))
    with pytest.raises(ValueError, match="needs"):
        c.decrypt(short_ct, pt)
    with pytest.raises(ValueError, match="needs"):
        c.add(ct, short_ct, ct)
    with pytest.raises(ValueError, match="needs"):
        c.elementwise_zinc(ct, short_ct)
    with pytest.raises(ValueError, match="needs"):
        c.elementwise_vanilla(meta_tensor((2, c.L, c.n - 1)), ct, ct)
    with pytest.raises(ValueError, match="needs"):
        c.ntt_forward(0, meta_tensor((2, c.n - 1)))
    with pytest.raises(ValueError, match="needs"):
        c.sample(0, 4, 0, meta_tensor((2,)), meta_tensor((2, c.n - 1)))
    with pytest.raises(ValueError, match="needs"):
        c.bfv_encode(257, meta_tensor((2, c.n)), meta_tensor((2, c.L, c.n - 1)))
    with pytest.raises(ValueError, match="needs"):
        c.bfv_decode(257, pt, meta_tensor((2, c.n - 1)))
    with pytest.raises(ValueError, match="needs"):
        c.bgv_encode(meta_tensor((2, c.n - 1)), pt)
    with pytest.raises(ValueError, match="needs"):
        c.batch_encode(65537, meta_tensor((2, c.n)), meta_tensor((2, c.n - 1)))
    with pytest.raises(ValueError, match="needs"):
        c.export_keys(sk=meta_tensor((c.M, c.n - 1)))
    with pytest.raises(ValueError, match="leading batch"):
        c.decrypt(meta_tensor(()), pt)


def test_server_and_plan_buffers_checked(meta_tensor):
    with pytest.raises(TypeError, match="float64"):
        zinc._server_config(1, 4, 8, 1 << 20, meta_tensor((10,), torch.int64), None)
    with pytest.raises(ValueError, match="GPU memory"):
        zinc._server_config(1, 4, 8, 1 << 20, meta_tensor((10,), torch.float64), meta_tensor((10,), device="cpu"))
    cfg = zinc._server_config(1, 4, 8, 1 << 20, meta_tensor((10,), torch.float64), meta_tensor((7,)), True)
    assert (cfg.slots_len, cfg.ct_len, cfg.retain_outputs) == (10, 7, 1)
