"""CPU checks of the C-ABI library: it loads, exports every function declared
in include/zinc.h, and its host-side argument and parameter validation
rejects bad input before touching the GPU."""
import ctypes
import os
import re

import pytest

import paper_2408_07304_amd as zinc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "zinc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(zinc_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(zinc.LIB_PATH):
        pytest.fail("libzinc.so is not built (run __graft_entry__.build())")
    return zinc.load_library()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(zinc.EXPORTED)


def _params(log_n=13, bits=(60, 40, 40, 60), scale=2.0 ** 40, sigma=3.2, moduli=None):
    p = zinc.zinc_params()
    p.log_n = log_n
    p.n_moduli = len(moduli) if moduli is not None else len(bits)
    if moduli is not None:
        arr = (ctypes.c_uint64 * len(moduli))(*moduli)
        p.moduli = arr
        p._keep = arr
    else:
        arr = (ctypes.c_uint32 * len(bits))(*bits)
        p.bit_sizes = arr
        p._keep = arr
    p.scale = scale
    p.sigma = sigma
    p.seed = 0
    return p


@pytest.mark.parametrize("kw,code", [
    (dict(log_n=11), zinc.ZINC_E_PARAM),
    (dict(log_n=16), zinc.ZINC_E_PARAM),
    (dict(log_n=15, bits=(55,) * 40), zinc.ZINC_E_PARAM),                         # more than 32 moduli
    (dict(bits=(60,)), zinc.ZINC_E_PARAM),
    (dict(bits=(61, 40, 60)), zinc.ZINC_E_PARAM),
    (dict(bits=(10, 40, 60)), zinc.ZINC_E_PARAM),
    (dict(scale=0.0), zinc.ZINC_E_PARAM),
    (dict(scale=float("inf")), zinc.ZINC_E_PARAM),
    (dict(scale=2.0 ** 62), zinc.ZINC_E_PARAM),
    (dict(sigma=3.3), zinc.ZINC_E_PARAM),
    (dict(moduli=(1152921504606830593, 1152921504606830593)), zinc.ZINC_E_PARAM),   # duplicate
    (dict(moduli=(1152921504606830591, 1099511480321)), zinc.ZINC_E_PARAM),         # not 1 mod 2N
    (dict(moduli=(1099511480321 + 16384, 1099511480321)), zinc.ZINC_E_PARAM),       # composite
])
def test_ctx_create_rejects_bad_parameters(lib, kw, code):
    h = ctypes.c_void_p()
    p = _params(**kw)
    assert lib.zinc_ctx_create(ctypes.byref(p), ctypes.byref(h)) == code
    assert h.value is None
    assert lib.zinc_last_error().decode()


def test_null_arguments_are_rejected(lib):
    h = ctypes.c_void_p()
    assert lib.zinc_ctx_create(None, ctypes.byref(h)) == zinc.ZINC_E_INVAL
    for name in ("zinc_keygen", "zinc_precompute"):
        assert getattr(lib, name)(None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_encode(None, None, 1, 1, None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_encrypt(None, None, 1, None, None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_encrypt_vanilla(None, None, 1, None, None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_encrypt_slots(None, 1, None, 1, 1, None, None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_decrypt(None, None, 1, None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_decode(None, None, 1, None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_add(None, None, None, 1, None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_ctx_destroy(None) == zinc.ZINC_E_INVAL
    assert lib.zinc_elementwise_zinc(None, None, 1, None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_elementwise_vanilla(None, None, None, 1, None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_bfv_encode(None, 257, None, 1, None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_bfv_decode(None, 257, None, 1, None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_set_bgv(None, 257) == zinc.ZINC_E_INVAL
    assert lib.zinc_batch_encode(None, 65537, None, 1, None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_batch_decode(None, 65537, None, 1, None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_bgv_encode(None, None, 1, None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_bgv_decode(None, None, 1, None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_encrypt_vanilla_sp(None, None, 1, None, None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_set_tuning(None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_get_tuning(None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_autotune(None, 1, None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_server_create(None, 0, None, ctypes.byref(h)) == zinc.ZINC_E_INVAL
    assert lib.zinc_server_submit(None, None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_server_progress(None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_server_query(None, 0, None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_server_drain(None) == zinc.ZINC_E_INVAL
    assert lib.zinc_server_output(None, 0, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_server_read_output(None, 0, None, 0, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_server_release(None, 0) == zinc.ZINC_E_INVAL
    assert lib.zinc_plan_launch(None, None, 0, None, 0, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_server_destroy(None) == zinc.ZINC_OK
    assert lib.zinc_serve_trace(None, 0, None, None, None, 0, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_ctx_info(None, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_ntt_forward(None, 0, None, 1, None) == zinc.ZINC_E_INVAL
    assert lib.zinc_sample(None, 0, 1, 0, None, 1, None, None) == zinc.ZINC_E_INVAL
    assert "null" in lib.zinc_last_error().decode()


def test_single_hip_runtime_in_process(lib):
    """The binding loads torch's HIP runtime first, so the process maps exactly
    one libamdhip64 (two runtimes in one process cannot share a device)."""
    maps = {ln.split()[-1] for ln in open("/proc/self/maps") if "libamdhip64" in ln}
    assert len(maps) == 1, maps


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structures have the sizes and field offsets the C
    compiler gives the header's structures."""
    import subprocess
    structs = {"zinc_params": zinc.zinc_params, "zinc_info": zinc.zinc_info, "zinc_item": zinc.zinc_item,
               "zinc_server_config": zinc.zinc_server_config, "zinc_request": zinc.zinc_request,
               "zinc_request_times": zinc.zinc_request_times, "zinc_tuning": zinc.zinc_tuning,
               "zinc_tune_result": zinc.zinc_tune_result}
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "zinc.h"', "int main(void) {"]
    for name, cls in structs.items():
        src.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            src.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    src.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(root, "include"), str(c), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        n, f, v = line.split()
        got[(n, f)] = int(v)
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)
