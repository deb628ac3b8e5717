"""Host address / undefined-behaviour sanitizer builds (CPU only).

* The FP64 oracle (oracle/sre2_oracle.c) with gcc's AddressSanitizer and
  UndefinedBehaviorSanitizer (leak checks on), driven over every entry point
  on small states and its argument checks (tests/sanitize/oracle_driver.c).
* The host code of libsre2 (argument checks, workspace sizing, contexts, the
  allocation-free call's layout, server and simulator setup) built with the
  host sanitizers only (every -fsanitize= behind -Xarch_host; device code is
  not instrumented), linked against test stand-ins for the kernel launchers
  (tests/sanitize/stub_launchers.hip) and driven by
  tests/sanitize/abi_driver.cpp.  No device is touched.
A sanitizer report makes the run fail (UB aborts: -fno-sanitize-recover).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2512_24685_amd", "csrc")


def _run(exe, env_extra):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0 and "ok: 0 failures" in r.stdout, out[-4000:]


def test_oracle_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_san")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    os.path.join(ROOT, "oracle", "sre2_oracle.c"),
                    os.path.join(SAN, "oracle_driver.c"), "-o", exe, "-lm"], check=True)
    _run(exe, {"ASAN_OPTIONS": "detect_leaks=1", "OMP_NUM_THREADS": "2"})


def test_host_abi_under_asan_ubsan(tmp_path):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    srcs = [os.path.join(CSRC, f) for f in ("sre2_api.hip", "sre2_noalloc.hip", "sre2_server.hip",
                                            "sre2_sim.hip", "sre2_queries.hip")]
    srcs += [os.path.join(SAN, "stub_launchers.hip"), os.path.join(SAN, "abi_driver.cpp")]
    procs, objs = [], []
    for s in srcs:
        o = str(tmp_path / (os.path.basename(s) + ".o"))
        lang = ["-x", "hip"] if s.endswith(".cpp") else []
        procs.append(subprocess.Popen(["hipcc", *flags, *host_san, *lang, "-c", s, "-o", o],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        objs.append(o)
    for p in procs:
        out = p.communicate(timeout=600)[0]
        assert p.returncode == 0, out.decode(errors="replace")[-3000:]
    exe = str(tmp_path / "abi_san")
    link = ["hipcc", "--offload-arch=gfx950", "-fno-gpu-sanitize", "-fsanitize=address,undefined"]
    subprocess.run([*link, *objs, "-o", exe], check=True)
    # the HIP runtime keeps some allocations until exit: leaks are not checked
    _run(exe, {"ASAN_OPTIONS": "detect_leaks=0"})
