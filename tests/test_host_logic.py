"""Host-side logic of the library checked on the CPU by a small C++ program
(tests/host/host_logic_test.cpp) linked against the built libzinc.so: the
serving budget's first-fit arena under random allocation and release, the
mixed-plan unit tables, and the chi sampler's bucket table against the count
it stands for; and the kernels' LDS index layouts (tests/host/layout_test.cpp)."""
import os
import subprocess

import paper_2408_07304_amd as zinc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_logic(tmp_path):
    zinc.load_library()                      # the library must be built
    exe = tmp_path / "host_logic_test"
    src = os.path.join(ROOT, "tests", "host", "host_logic_test.cpp")
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc"
    subprocess.run([hipcc, "-std=c++17", "-O1", "-I", os.path.join(ROOT, "include"), "-I",
                    os.path.join(zinc.PKG, "csrc"), src, "-L", zinc.PKG, "-lzinc", f"-Wl,-rpath,{zinc.PKG}",
                    "-o", str(exe)], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr


def test_barrier_free_layouts(tmp_path):
    """The LDS index layouts behind the barrier-free exchanges, checked by brute
    force over every thread and register (tests/host/layout_test.cpp): the
    layouts are the kernels' own host/device functions, compiled as HIP source
    and evaluated on the CPU."""
    exe = tmp_path / "layout_test"
    src = os.path.join(ROOT, "tests", "host", "layout_test.cpp")
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc"
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-std=c++17", "-O1", "-I",
                    os.path.join(ROOT, "include"), "-I", os.path.join(zinc.PKG, "csrc"), src, "-o", str(exe)],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr
