"""Python binding of libzinc (include/zinc.h): batched CKKS vanilla encryption
(Eq. 8) and Zinc encryption (Algorithm 1) on MI355X.

Argument marshalling only: every step runs in the HIP library.  Device
buffers are torch tensors (uint64 data is carried in int64 tensors); streams
are torch streams.  Importing this package does not load the library; the
first call does, and raises if libzinc.so has not been built.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libzinc.so")

ZINC_OK = 0
ZINC_E_INVAL, ZINC_E_PARAM, ZINC_E_STATE, ZINC_E_NOMEM, ZINC_E_HIP, ZINC_E_RANGE = -1, -2, -3, -4, -5, -6
ZINC_KEY_ID = (1 << 64) - 1
ZINC_ZERO_ID = (1 << 64) - 2
ZINC_MAX_MODULI = 32
ZINC_SCHEME_VANILLA, ZINC_SCHEME_ZINC, ZINC_SCHEME_VANILLA_SP = 0, 1, 2
SAMPLE_TERNARY, SAMPLE_GAUSSIAN, SAMPLE_UNIFORM = 0, 1, 2

_STATUS_NAMES = {-1: "ZINC_E_INVAL", -2: "ZINC_E_PARAM", -3: "ZINC_E_STATE", -4: "ZINC_E_NOMEM",
                 -5: "ZINC_E_HIP", -6: "ZINC_E_RANGE"}


class ZincError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class zinc_params(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("n_moduli", ctypes.c_uint32),
                ("bit_sizes", ctypes.POINTER(ctypes.c_uint32)), ("moduli", ctypes.POINTER(ctypes.c_uint64)),
                ("scale", ctypes.c_double), ("sigma", ctypes.c_double), ("seed", ctypes.c_uint64)]


class zinc_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("log_n", ctypes.c_uint32), ("n_moduli", ctypes.c_uint32),
                ("limbs", ctypes.c_uint32), ("moduli", ctypes.c_uint64 * ZINC_MAX_MODULI),
                ("psi", ctypes.c_uint64 * ZINC_MAX_MODULI), ("scale", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("cdt", ctypes.c_uint64 * 38),
                ("plaintext_bytes", ctypes.c_size_t), ("ciphertext_bytes", ctypes.c_size_t),
                ("keyed", ctypes.c_int), ("precomputed", ctypes.c_int), ("ntt_fp64_mask", ctypes.c_uint32),
                ("tile", ctypes.c_uint32 * 2), ("reg_epilogue", ctypes.c_uint32), ("bgv_t", ctypes.c_uint64)]


class zinc_tuning(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_uint32 * 2), ("ntt_fp64_mask", ctypes.c_uint32), ("reg_epilogue", ctypes.c_uint32)]


class zinc_tune_result(ctypes.Structure):
    _fields_ = [("chosen", zinc_tuning), ("from_cache", ctypes.c_uint32), ("n_timed", ctypes.c_uint32),
                ("best_ms", ctypes.c_double * 2), ("default_ms", ctypes.c_double * 2)]


class zinc_item(ctypes.Structure):
    _fields_ = [("ctx_idx", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("slot_off", ctypes.c_uint64),
                ("ct_off", ctypes.c_uint64), ("ct_id", ctypes.c_uint64)]


class zinc_server_config(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int), ("n_streams", ctypes.c_uint32), ("max_batch", ctypes.c_uint32),
                ("retain_outputs", ctypes.c_uint32), ("hbm_budget", ctypes.c_uint64), ("d_slots", ctypes.c_void_p),
                ("d_ct", ctypes.c_void_p), ("slots_len", ctypes.c_uint64), ("ct_len", ctypes.c_uint64)]


class zinc_request(ctypes.Structure):
    _fields_ = [("ctx_idx", ctypes.c_uint32), ("n_pt", ctypes.c_uint32), ("slot_off", ctypes.c_uint64),
                ("ct_off", ctypes.c_uint64), ("ct_id", ctypes.c_uint64)]


class zinc_request_times(ctypes.Structure):
    _fields_ = [("submit_ns", ctypes.c_uint64), ("admit_ns", ctypes.c_uint64), ("launch_ns", ctypes.c_uint64),
                ("done_ns", ctypes.c_uint64), ("batch", ctypes.c_uint32), ("stream", ctypes.c_uint32),
                ("dev_start_ns", ctypes.c_uint64), ("dev_end_ns", ctypes.c_uint64)]


# numpy layouts of zinc_request and zinc_request_times (arrays of requests)
REQUEST_FIELDS = [("ctx_idx", "<u4"), ("n_pt", "<u4"), ("slot_off", "<u8"), ("ct_off", "<u8"), ("ct_id", "<u8")]
TIMES_FIELDS = [("submit_ns", "<u8"), ("admit_ns", "<u8"), ("launch_ns", "<u8"), ("done_ns", "<u8"),
                ("batch", "<u4"), ("stream", "<u4"), ("dev_start_ns", "<u8"), ("dev_end_ns", "<u8")]

_lib = None
_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32
_SIGS = {
    "zinc_last_error": (ctypes.c_char_p, []),
    "zinc_ctx_create": (ctypes.c_int, [ctypes.POINTER(zinc_params), ctypes.POINTER(_vp)]),
    "zinc_ctx_destroy": (ctypes.c_int, [_vp]),
    "zinc_ctx_info": (ctypes.c_int, [_vp, ctypes.POINTER(zinc_info)]),
    "zinc_keygen": (ctypes.c_int, [_vp, _vp]),
    "zinc_precompute": (ctypes.c_int, [_vp, _vp]),
    "zinc_encode": (ctypes.c_int, [_vp, _vp, _u32, _u32, _vp, _vp]),
    "zinc_encrypt_vanilla": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp, _vp]),
    "zinc_encrypt": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp, _vp]),
    "zinc_encrypt_vanilla_sp": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp, _vp]),
    "zinc_encrypt_vanilla_sp_noalloc": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp, _vp]),
    "zinc_bfv_encode": (ctypes.c_int, [_vp, ctypes.c_uint64, _vp, _u32, _vp, _vp]),
    "zinc_bfv_decode": (ctypes.c_int, [_vp, ctypes.c_uint64, _vp, _u32, _vp, _vp]),
    "zinc_set_bgv": (ctypes.c_int, [_vp, ctypes.c_uint64]),
    "zinc_batch_encode": (ctypes.c_int, [_vp, ctypes.c_uint64, _vp, _u32, _vp, _vp]),
    "zinc_batch_decode": (ctypes.c_int, [_vp, ctypes.c_uint64, _vp, _u32, _vp, _vp]),
    "zinc_bgv_encode": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp]),
    "zinc_bgv_decode": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp]),
    "zinc_encrypt_slots": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _u32, _u32, _vp, _vp, _vp]),
    "zinc_decrypt": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp]),
    "zinc_decode": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp]),
    "zinc_add": (ctypes.c_int, [_vp, _vp, _vp, _u32, _vp, _vp]),
    "zinc_elementwise_zinc": (ctypes.c_int, [_vp, _vp, _u32, _vp, _vp]),
    "zinc_elementwise_vanilla": (ctypes.c_int, [_vp, _vp, _vp, _u32, _vp, _vp]),
    "zinc_device_errors": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_uint32)]),
    "zinc_plan_create": (ctypes.c_int, [ctypes.POINTER(_vp), _u32, ctypes.POINTER(zinc_item), _u32,
                                        ctypes.c_int, ctypes.POINTER(_vp)]),
    "zinc_plan_launch": (ctypes.c_int, [_vp, _vp, ctypes.c_uint64, _vp, ctypes.c_uint64, _vp]),
    "zinc_plan_destroy": (ctypes.c_int, [_vp]),
    "zinc_server_create": (ctypes.c_int, [ctypes.POINTER(_vp), _u32, ctypes.POINTER(zinc_server_config),
                                          ctypes.POINTER(_vp)]),
    "zinc_server_submit": (ctypes.c_int, [_vp, ctypes.POINTER(zinc_request), ctypes.POINTER(ctypes.c_uint64)]),
    "zinc_server_progress": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_uint32)]),
    "zinc_server_query": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(zinc_request_times)]),
    "zinc_server_output": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(_vp)]),
    "zinc_server_read_output": (ctypes.c_int, [_vp, ctypes.c_uint64, _vp, ctypes.c_uint64, _vp]),
    "zinc_server_release": (ctypes.c_int, [_vp, ctypes.c_uint64]),
    "zinc_server_drain": (ctypes.c_int, [_vp]),
    "zinc_server_destroy": (ctypes.c_int, [_vp]),
    "zinc_serve_trace": (ctypes.c_int, [ctypes.POINTER(_vp), _u32, ctypes.POINTER(zinc_server_config), _vp, _vp,
                                        _u32, _vp]),
    "zinc_set_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(zinc_tuning)]),
    "zinc_get_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(zinc_tuning)]),
    "zinc_autotune": (ctypes.c_int, [_vp, _u32, ctypes.c_char_p, ctypes.POINTER(zinc_tune_result)]),
    "zinc_ntt_forward": (ctypes.c_int, [_vp, _u32, _vp, _u32, _vp]),
    "zinc_ntt_inverse": (ctypes.c_int, [_vp, _u32, _vp, _u32, _vp]),
    "zinc_sample": (ctypes.c_int, [_vp, ctypes.c_int, _u32, _u32, _vp, _u32, _vp, _vp]),
    "zinc_export_keys": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "zinc_butterfly_rate": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint64, _u32, ctypes.POINTER(ctypes.c_double)]),
}
EXPORTED = tuple(_SIGS)


def load_library(path: str = LIB_PATH):
    """Load libzinc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # One HIP runtime per process: torch brings its own libamdhip64
        # (soname libamdhip64.so.7).  Importing torch first makes the dynamic
        # loader resolve libzinc's dependency to that same, already-loaded
        # runtime instead of mapping a second copy from /opt/rocm.
        import torch  # noqa: F401
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with `python -m paper_2408_07304_amd.build` "
                              "(or __graft_entry__.build()); there is no fallback path")
        L = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return load_library().zinc_last_error().decode()


def _check(status: int):
    if status != ZINC_OK:
        raise ZincError(status, last_error())


def _buf(t, name: str, dtype: str, numel: int):
    """Device pointer of `t` after checking that it is a contiguous torch
    tensor in GPU memory of dtype `dtype` ("int64" carries uint64 data,
    "float64") holding at least `numel` elements.  A host tensor, a wrong dtype
    or a short buffer would let the kernels read or write outside it, so each
    raises here, before anything reaches the library."""
    import torch
    if not all(hasattr(t, a) for a in ("data_ptr", "device", "dtype", "numel", "is_contiguous")):
        raise TypeError(f"{name} must be a torch tensor in GPU memory, not {type(t).__name__}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be in GPU memory (it is on {t.device})")
    if t.dtype != getattr(torch, dtype):
        raise TypeError(f"{name} must be torch.{dtype} (it is {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements; the call needs {numel}")
    return t.data_ptr()


def _opt_buf(t, name: str, dtype: str, numel: int):
    return None if t is None else _buf(t, name, dtype, numel)


def _batch(t, name: str) -> int:
    """Leading dimension of a batched buffer (the batch size the call takes)."""
    if getattr(t, "ndim", 0) < 1:
        raise ValueError(f"{name} must have a leading batch dimension")
    return int(t.shape[0])


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _u64_tensor(values, device):
    import numpy as np
    import torch
    a = np.asarray(values, dtype=np.uint64).view(np.int64)
    return torch.from_numpy(a.copy()).to(device)


class Context:
    """One parameter set (ring degree, moduli chain, scale, seed) with its
    device-resident tables, keys and Zinc cache.  Every method checks its
    buffers (GPU memory, dtype, contiguity, length) against the sizes the
    call implies; uint64 data travels in int64 tensors."""

    def __init__(self, log_n: int, bits=None, scale: float = 2.0 ** 40, seed: int = 0, moduli=None,
                 sigma: float = 3.2):
        lib = load_library()
        p = zinc_params()
        p.log_n = log_n
        count = len(moduli) if moduli is not None else len(bits)
        p.n_moduli = count
        self._bits = (ctypes.c_uint32 * count)(*(bits or [0] * count))
        self._mods = (ctypes.c_uint64 * count)(*(moduli or [0] * count))
        p.bit_sizes = self._bits if bits is not None else None
        p.moduli = self._mods if moduli is not None else None
        p.scale = scale
        p.sigma = sigma
        p.seed = seed
        h = _vp()
        _check(lib.zinc_ctx_create(ctypes.byref(p), ctypes.byref(h)))
        self.handle = h.value
        inf = self.info()
        self.n, self.log_n, self.M, self.L = inf["n"], inf["log_n"], inf["n_moduli"], inf["limbs"]
        self.moduli, self.psi, self.scale, self.seed = inf["moduli"], inf["psi"], inf["scale"], inf["seed"]

    def close(self):
        if getattr(self, "handle", None):
            load_library().zinc_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # element counts per batch entry
    @property
    def pt_words(self) -> int:
        return self.L * self.n

    @property
    def ct_words(self) -> int:
        return 2 * self.L * self.n

    def info(self) -> dict:
        i = zinc_info()
        _check(load_library().zinc_ctx_info(self.handle, ctypes.byref(i)))
        M = i.n_moduli
        return {"n": i.n, "log_n": i.log_n, "n_moduli": M, "limbs": i.limbs,
                "moduli": [int(x) for x in i.moduli[:M]], "psi": [int(x) for x in i.psi[:M]],
                "scale": i.scale, "seed": int(i.seed), "cdt": [int(x) for x in i.cdt],
                "plaintext_bytes": int(i.plaintext_bytes), "ciphertext_bytes": int(i.ciphertext_bytes),
                "keyed": bool(i.keyed), "precomputed": bool(i.precomputed),
                "ntt_fp64_mask": int(i.ntt_fp64_mask), "tile": [int(i.tile[0]), int(i.tile[1])],
                "reg_epilogue": int(i.reg_epilogue), "bgv_t": int(i.bgv_t)}

    # -- tuning (speed only; results are identical for every choice) ---------
    def set_tuning(self, tile_vanilla: int, tile_zinc: int, ntt_fp64_mask: int, reg_epilogue: int = 0):
        t = zinc_tuning()
        t.tile[0], t.tile[1], t.ntt_fp64_mask = int(tile_vanilla), int(tile_zinc), int(ntt_fp64_mask)
        t.reg_epilogue = int(reg_epilogue)
        _check(load_library().zinc_set_tuning(self.handle, ctypes.byref(t)))

    def get_tuning(self) -> dict:
        t = zinc_tuning()
        _check(load_library().zinc_get_tuning(self.handle, ctypes.byref(t)))
        return {"tile": [int(t.tile[0]), int(t.tile[1])], "ntt_fp64_mask": int(t.ntt_fp64_mask),
                "reg_epilogue": int(t.reg_epilogue)}

    def autotune(self, batch: int = 512, cache_path: str | None = None) -> dict:
        r = zinc_tune_result()
        _check(load_library().zinc_autotune(self.handle, int(batch),
                                            cache_path.encode() if cache_path else None, ctypes.byref(r)))
        return {"tile": [int(r.chosen.tile[0]), int(r.chosen.tile[1])],
                "ntt_fp64_mask": int(r.chosen.ntt_fp64_mask), "reg_epilogue": int(r.chosen.reg_epilogue),
                "from_cache": bool(r.from_cache),
                "n_timed": int(r.n_timed), "best_ms": [r.best_ms[0], r.best_ms[1]],
                "default_ms": [r.default_ms[0], r.default_ms[1]]}

    # -- the scheme ---------------------------------------------------------
    def keygen(self, stream=None):
        _check(load_library().zinc_keygen(self.handle, _stream(stream)))

    def precompute(self, stream=None):
        _check(load_library().zinc_precompute(self.handle, _stream(stream)))

    def _slots(self, slots):
        """(pointer, n_slots, batch) of a [batch][n_slots] float64 slot buffer."""
        if getattr(slots, "ndim", 0) != 2:
            raise ValueError("slots must be a [batch][n_slots] tensor")
        b, ns = int(slots.shape[0]), int(slots.shape[1])
        return _buf(slots, "slots", "float64", b * ns), ns, b

    def encode(self, slots, out, stream=None):
        ps, ns, b = self._slots(slots)
        _check(load_library().zinc_encode(self.handle, ps, ns, b, _buf(out, "out", "int64", b * self.pt_words),
                                          _stream(stream)))
        return out

    def _encrypt_pt(self, fn, pt, ct_ids, out, stream):
        b = _batch(pt, "pt")
        _check(fn(self.handle, _buf(pt, "pt", "int64", b * self.pt_words), b, _buf(ct_ids, "ct_ids", "int64", b),
                  _buf(out, "out", "int64", b * self.ct_words), _stream(stream)))
        return out

    def encrypt_vanilla(self, pt, ct_ids, out, stream=None):
        return self._encrypt_pt(load_library().zinc_encrypt_vanilla, pt, ct_ids, out, stream)

    def encrypt_vanilla_sp(self, pt, ct_ids, out, stream=None):
        """Vanilla with division by the special prime (a SEAL-style baseline)."""
        return self._encrypt_pt(load_library().zinc_encrypt_vanilla_sp, pt, ct_ids, out, stream)

    def encrypt_vanilla_sp_noalloc(self, pt, ct_ids, out, stream=None):
        """encrypt_vanilla_sp with the library's static scratch (no allocation;
        calls overlapping on one GPU race)."""
        return self._encrypt_pt(load_library().zinc_encrypt_vanilla_sp_noalloc, pt, ct_ids, out, stream)

    def encrypt(self, pt, ct_ids, out, stream=None):
        return self._encrypt_pt(load_library().zinc_encrypt, pt, ct_ids, out, stream)

    def encrypt_slots(self, scheme: int, slots, ct_ids, out, stream=None):
        ps, ns, b = self._slots(slots)
        _check(load_library().zinc_encrypt_slots(self.handle, scheme, ps, ns, b, _buf(ct_ids, "ct_ids", "int64", b),
                                                 _buf(out, "out", "int64", b * self.ct_words), _stream(stream)))
        return out

    def bfv_encode(self, t: int, m, out, stream=None):
        """BFV plaintexts (int64 [batch][N] in Z_t) -> Delta * m residues."""
        b = _batch(m, "m")
        _check(load_library().zinc_bfv_encode(self.handle, int(t), _buf(m, "m", "int64", b * self.n), b,
                                              _buf(out, "out", "int64", b * self.pt_words), _stream(stream)))
        return out

    def bfv_decode(self, t: int, pt, out, stream=None):
        """Decrypted residues -> BFV plaintexts (int64, centred mod t)."""
        b = _batch(pt, "pt")
        _check(load_library().zinc_bfv_decode(self.handle, int(t), _buf(pt, "pt", "int64", b * self.pt_words), b,
                                              _buf(out, "out", "int64", b * self.n), _stream(stream)))
        return out

    def set_bgv(self, t: int):
        """BGV form (errors scaled by t) from the next keygen; t = 1 undoes it."""
        _check(load_library().zinc_set_bgv(self.handle, int(t)))

    def bgv_encode(self, m, out, stream=None):
        """BGV plaintexts (int64 [batch][N]) -> residues of m mod t."""
        b = _batch(m, "m")
        _check(load_library().zinc_bgv_encode(self.handle, _buf(m, "m", "int64", b * self.n), b,
                                              _buf(out, "out", "int64", b * self.pt_words), _stream(stream)))
        return out

    def bgv_decode(self, pt, out, stream=None):
        """Decrypted residues -> BGV plaintexts (int64, centred mod t)."""
        b = _batch(pt, "pt")
        _check(load_library().zinc_bgv_decode(self.handle, _buf(pt, "pt", "int64", b * self.pt_words), b,
                                              _buf(out, "out", "int64", b * self.n), _stream(stream)))
        return out

    def batch_encode(self, t: int, slots, out, stream=None):
        """Slot values (int64 [batch][N]) -> BFV/BGV plaintext coefficients in [0, t)."""
        b = _batch(slots, "slots")
        _check(load_library().zinc_batch_encode(self.handle, int(t), _buf(slots, "slots", "int64", b * self.n), b,
                                                _buf(out, "out", "int64", b * self.n), _stream(stream)))
        return out

    def batch_decode(self, t: int, m, out, stream=None):
        """Plaintext coefficients (int64 [batch][N]) -> slot values, centred mod t."""
        b = _batch(m, "m")
        _check(load_library().zinc_batch_decode(self.handle, int(t), _buf(m, "m", "int64", b * self.n), b,
                                                _buf(out, "out", "int64", b * self.n), _stream(stream)))
        return out

    def decrypt(self, ct, out, stream=None):
        b = _batch(ct, "ct")
        _check(load_library().zinc_decrypt(self.handle, _buf(ct, "ct", "int64", b * self.ct_words), b,
                                           _buf(out, "out", "int64", b * self.pt_words), _stream(stream)))
        return out

    def decode(self, pt, out, stream=None):
        b = _batch(pt, "pt")
        _check(load_library().zinc_decode(self.handle, _buf(pt, "pt", "int64", b * self.pt_words), b,
                                          _buf(out, "out", "float64", b * (self.n // 2)), _stream(stream)))
        return out

    def add(self, a, b_, out, stream=None):
        b = _batch(a, "a")
        w = b * self.ct_words
        _check(load_library().zinc_add(self.handle, _buf(a, "a", "int64", w), _buf(b_, "b", "int64", w), b,
                                       _buf(out, "out", "int64", w), _stream(stream)))
        return out

    def elementwise_zinc(self, hat, out, stream=None):
        """Algorithm 1's additions alone: out = hat + Enc(0) (NTT domain)."""
        b = _batch(hat, "hat")
        w = b * self.ct_words
        _check(load_library().zinc_elementwise_zinc(self.handle, _buf(hat, "hat", "int64", w), b,
                                                    _buf(out, "out", "int64", w), _stream(stream)))
        return out

    def elementwise_vanilla(self, uhat, hat, out, stream=None):
        """Eq. 8's products and additions alone: out = pk * uhat + hat."""
        b = _batch(hat, "hat")
        w = b * self.ct_words
        _check(load_library().zinc_elementwise_vanilla(self.handle, _buf(uhat, "uhat", "int64", b * self.pt_words),
                                                       _buf(hat, "hat", "int64", w), b,
                                                       _buf(out, "out", "int64", w), _stream(stream)))
        return out

    def device_errors(self) -> int:
        f = ctypes.c_uint32()
        _check(load_library().zinc_device_errors(self.handle, ctypes.byref(f)))
        return int(f.value)

    # -- kernel-level entry points -----------------------------------------
    def ntt_forward(self, limb: int, poly, stream=None):
        b = _batch(poly, "poly")
        _check(load_library().zinc_ntt_forward(self.handle, limb, _buf(poly, "poly", "int64", b * self.n), b,
                                               _stream(stream)))
        return poly

    def ntt_inverse(self, limb: int, poly, stream=None):
        b = _batch(poly, "poly")
        _check(load_library().zinc_ntt_inverse(self.handle, limb, _buf(poly, "poly", "int64", b * self.n), b,
                                               _stream(stream)))
        return poly

    def sample(self, kind: int, tag: int, limb: int, ct_ids, out, stream=None):
        b = _batch(ct_ids, "ct_ids")
        _check(load_library().zinc_sample(self.handle, kind, tag, limb, _buf(ct_ids, "ct_ids", "int64", b), b,
                                          _buf(out, "out", "int64", b * self.n), _stream(stream)))
        return out

    def export_keys(self, sk=None, pk=None, zero=None, stream=None):
        n = self.n
        _check(load_library().zinc_export_keys(self.handle, _opt_buf(sk, "sk", "int64", self.M * n),
                                               _opt_buf(pk, "pk", "int64", 2 * self.M * n),
                                               _opt_buf(zero, "zero", "int64", self.ct_words), _stream(stream)))


class Plan:
    """A mixed-shape batch over several contexts (zinc_plan_*)."""

    def __init__(self, ctxs, items, scheme: int):
        lib = load_library()
        arr = (_vp * len(ctxs))(*[c.handle for c in ctxs])
        its = (zinc_item * len(items))()
        for i, (ci, so, co, cid) in enumerate(items):
            its[i].ctx_idx, its[i].slot_off, its[i].ct_off, its[i].ct_id = int(ci), int(so), int(co), int(cid)
        h = _vp()
        _check(lib.zinc_plan_create(arr, len(ctxs), its, len(items), scheme, ctypes.byref(h)))
        self.handle = h.value
        self._ctxs = list(ctxs)

    def launch(self, slots, ct, stream=None):
        """Encrypt every item: `slots` is the float64 slot buffer and `ct` the
        int64 output buffer the items' offsets index (the library checks that
        both reach every item); None for both on an empty plan."""
        ps = _opt_buf(slots, "slots", "float64", 0)
        pc = _opt_buf(ct, "ct", "int64", 0)
        _check(load_library().zinc_plan_launch(self.handle, ps, 0 if slots is None else slots.numel(), pc,
                                               0 if ct is None else ct.numel(), _stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            load_library().zinc_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _server_config(scheme, n_streams, max_batch, hbm_budget, slots, ct, retain_outputs=False):
    return zinc_server_config(int(scheme), int(n_streams), int(max_batch), int(bool(retain_outputs)),
                              int(hbm_budget), _buf(slots, "slots", "float64", 1),
                              _opt_buf(ct, "ct", "int64", 1), slots.numel(), 0 if ct is None else ct.numel())


class Server:
    """Admission and continuous batching over resident contexts (zinc_server_*).
    `slots` is the base of every request's slot vectors; `ct` the base of their
    outputs, or None for the server's own arena, where outputs are discarded on
    completion or, with retain_outputs, kept until release()."""

    def __init__(self, ctxs, scheme: int, slots, ct=None, n_streams: int = 4, max_batch: int = 512,
                 hbm_budget: int = 8 << 30, retain_outputs: bool = False):
        lib = load_library()
        arr = (_vp * len(ctxs))(*[c.handle for c in ctxs])
        cfg = _server_config(scheme, n_streams, max_batch, hbm_budget, slots, ct, retain_outputs)
        h = _vp()
        _check(lib.zinc_server_create(arr, len(ctxs), ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h.value
        self._keep = (list(ctxs), slots, ct)

    def submit(self, ctx_idx: int, n_pt: int, slot_off: int, ct_id: int, ct_off: int = 0) -> int:
        r = zinc_request(int(ctx_idx), int(n_pt), int(slot_off), int(ct_off), int(ct_id))
        t = ctypes.c_uint64()
        _check(load_library().zinc_server_submit(self.handle, ctypes.byref(r), ctypes.byref(t)))
        return t.value

    def progress(self) -> int:
        n = ctypes.c_uint32()
        _check(load_library().zinc_server_progress(self.handle, ctypes.byref(n)))
        return n.value

    def query(self, ticket: int):
        """None while the request runs, else its times as a dict."""
        done = ctypes.c_int()
        t = zinc_request_times()
        _check(load_library().zinc_server_query(self.handle, int(ticket), ctypes.byref(done), ctypes.byref(t)))
        if not done.value:
            return None
        return {name: getattr(t, name) for name, _ in zinc_request_times._fields_}

    def output_ptr(self, ticket: int) -> int:
        """Device address of a completed request's retained ciphertexts."""
        p = _vp()
        _check(load_library().zinc_server_output(self.handle, int(ticket), ctypes.byref(p)))
        return int(p.value)

    def read_output(self, ticket: int, out, stream=None):
        """Copy a completed request's retained ciphertexts (n_pt * 2 * L * N
        uint64 words) into the int64 tensor `out`, on `stream`."""
        _check(load_library().zinc_server_read_output(self.handle, int(ticket), _buf(out, "out", "int64", 1),
                                                      out.numel(), _stream(stream)))
        return out

    def release(self, ticket: int):
        _check(load_library().zinc_server_release(self.handle, int(ticket)))

    def drain(self):
        _check(load_library().zinc_server_drain(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            load_library().zinc_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve_trace(ctxs, scheme: int, requests, arrival_ns, slots, ct=None, n_streams: int = 4,
                max_batch: int = 512, hbm_budget: int = 8 << 30):
    """Open-loop replay (zinc_serve_trace).  `requests` is a numpy array with
    the fields of REQUEST_FIELDS, `arrival_ns` uint64 nanoseconds after the
    start; returns a numpy array with the fields of TIMES_FIELDS."""
    import numpy as np
    req = np.ascontiguousarray(requests, dtype=np.dtype(REQUEST_FIELDS))
    arr_ns = np.ascontiguousarray(arrival_ns, dtype=np.uint64)
    if req.shape != arr_ns.shape or req.ndim != 1:
        raise ValueError("requests and arrival_ns must be 1-D of equal length")
    times = np.zeros(len(req), dtype=np.dtype(TIMES_FIELDS))
    lib = load_library()
    arr = (_vp * len(ctxs))(*[c.handle for c in ctxs])
    cfg = _server_config(scheme, n_streams, max_batch, hbm_budget, slots, ct)
    _check(lib.zinc_serve_trace(arr, len(ctxs), ctypes.byref(cfg), req.ctypes.data, arr_ns.ctypes.data,
                                len(req), times.ctypes.data))
    return times


def butterfly_rate(arith: int, q: int, reps: int = 9) -> float:
    """Peak forward-transform butterflies per second of this GPU (arith 0:
    integer Shoup, 1: exact FP64) for modulus q (zinc_butterfly_rate)."""
    r = ctypes.c_double()
    _check(load_library().zinc_butterfly_rate(int(arith), int(q), int(reps), ctypes.byref(r)))
    return r.value


def context_for(ps) -> Context:
    """Context of a workloads.ParamSet."""
    return Context(ps.log_n, list(ps.bits), ps.scale, ps.seed)
