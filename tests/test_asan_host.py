"""The host-side C-ABI layer (api.cpp, autotune.cpp, exact.cpp, the host parts of mft64.hip,
noalloc.hip, sweeps64.hip and relay.hip) built
with AddressSanitizer, linked with the ordinary device objects, and driven by a C harness through every entry point's argument checks
and the pilot-beam planner (no GPU needed). Sanitizers apply to host code only here."""

import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_1806_06467_amd")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"   # the harness links the same (clang) sanitizer runtime


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="needs hipcc and clang")
def test_host_abi_under_address_sanitizer(tmp_path):
    build = os.path.join(PKG, "_build")
    dev_objs = [os.path.join(build, o) for o in ("train.o", "sweeps.o", "sweeps_mr.o", "mft.o")]
    if not all(os.path.exists(o) for o in dev_objs):
        pytest.skip("library not built (run __graft_entry__.build())")
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address"]
    objs = []
    for src in ("api.cpp", "autotune.cpp", "exact.cpp", "mft64.hip", "noalloc.hip", "sweeps64.hip", "relay.hip"):
        obj = str(tmp_path / (src + ".o"))
        subprocess.run([HIPCC] + flags + ["-c", os.path.join(PKG, "csrc", src), "-o", obj], check=True,
                       capture_output=True)
        objs.append(obj)
    lib = str(tmp_path / "libfresnel_asan.so")
    subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
                    "-o", lib] + objs + dev_objs, check=True, capture_output=True)
    exe = str(tmp_path / "host_abi")
    subprocess.run([CLANG, "-g", "-fsanitize=address", "-o", exe, os.path.join(HERE, "asan", "host_abi.c"),
                    lib, "-lm"], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               LD_LIBRARY_PATH=str(tmp_path) + ":/opt/rocm/lib:" + os.environ.get("LD_LIBRARY_PATH", ""))
    p = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=120)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "ok" in p.stdout
