"""AddressSanitizer and UndefinedBehaviorSanitizer builds (CPU only):
the oracle with gcc, and the library with its host code instrumented
(hipcc, sanitizers on the host side only; device code unchanged), each
driven through its entry points by a small C program under tests/sanitize/.
The builds are cached under _build/ by a hash of their sources."""
import hashlib
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "_build", "sanitize")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
CSRC = os.path.join(ROOT, "paper_1801_08361_amd", "csrc")
HIP_SOURCES = ["forest.hip", "relocalise.hip", "mlp.hip", "verify.hip", "collab.hip", "train.hip", "prof.hip"]


def _digest(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    os.makedirs(BUILD, exist_ok=True)
    src = [os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c")]
    exe = os.path.join(BUILD, f"oracle_driver_{_digest(src + [os.path.join(ROOT, 'oracle', 'oracle.h')])}")
    if not os.path.exists(exe):
        _run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
              "-fno-sanitize-recover=all", "-ffp-contract=off", "-I", os.path.join(ROOT, "oracle"), *src,
              "-o", exe, "-lm"])
    r = _run([exe, str(tmp_path / "ckpt.bin")], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert "oracle sanitizer run ok" in r.stdout


def test_library_host_code_under_asan_ubsan(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("hipcc / clang not found")
    found = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                           text=True).stdout.strip()
    if not os.path.isabs(found) or not os.path.exists(found):
        pytest.skip("clang's AddressSanitizer runtime not found")
    rt = os.path.dirname(found)
    os.makedirs(BUILD, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in HIP_SOURCES]
    deps = srcs + [os.path.join(CSRC, "common.h"), os.path.join(CSRC, "mlp_dev.h"),
                   os.path.join(ROOT, "include", "reloc.h"), os.path.join(ROOT, "tests", "sanitize", "host_driver.c")]
    tag = _digest(deps)
    out = os.path.join(BUILD, f"lib_{tag}")
    so = os.path.join(out, "libreloc_san.so")
    exe = os.path.join(out, "host_driver")
    if not os.path.exists(exe):
        os.makedirs(out, exist_ok=True)
        objs = []
        for s in srcs:
            o = os.path.join(out, os.path.basename(s).replace(".hip", ".o"))
            _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off",
                  "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero", "-fhip-fp32-correctly-rounded-divide-sqrt",
                  "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                  "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-c", s, "-o", o])
            objs.append(o)
        _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-Xarch_host", "-fsanitize=address",
              "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", "-o", so])
        _run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-shared-libsan", "-fno-omit-frame-pointer",
              "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "sanitize", "host_driver.c"),
              "-L", out, "-lreloc_san", f"-Wl,-rpath,{out}", f"-Wl,-rpath,{rt}", "-lm", "-o", exe])
    # leaks are not checked here: the HIP runtime keeps allocations until exit
    r = _run([exe, str(tmp_path)], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert "host sanitizer run ok" in r.stdout
