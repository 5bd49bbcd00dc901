"""The ring pipeline's host code (dispatcher thread, producers, reader,
counters) under the host sanitizers, in dry-run mode so that no device is
needed: pipeline.hip is compiled with ThreadSanitizer, then with
AddressSanitizer + UndefinedBehaviorSanitizer (host pass only; device code is
built as usual), linked with the library's other objects, and the stress
program tests/native/pipeline_stress.cpp runs several producer threads, a
reader and a counter poller against the dispatcher."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2307_12988_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2307_12988_amd", "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")

def _objects():
    """The library's other objects, as its build leaves them."""
    srcs = sorted(f[:-4] for f in os.listdir(CSRC) if f.endswith(".hip") and f != "pipeline.hip")
    objs = [os.path.join(BUILD, o + ".o") for o in srcs]
    if not all(os.path.exists(o) for o in objs):
        from paper_2307_12988_amd import build as b
        b.build()
    return objs


@pytest.mark.parametrize("kind", ["thread", "address,undefined"])
def test_pipeline_host_code_under_sanitizers(kind, tmp_path):
    san = "-fsanitize=" + kind
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    pobj = str(tmp_path / "pipeline.o")
    sobj = str(tmp_path / "stress.o")
    exe = str(tmp_path / "stress")
    cmds = [
        [HIPCC] + common + inc + ["-Xarch_host", san, "-c", os.path.join(CSRC, "pipeline.hip"),
                                  "-o", pobj],
        [HIPCC] + common + inc + ["-Xarch_host", san, "-x", "hip", "-c",
                                  os.path.join(ROOT, "tests", "native", "pipeline_stress.cpp"),
                                  "-o", sobj],
        [HIPCC, "--offload-arch=gfx950", "-Xarch_host", san, "-o", exe, sobj, pobj] + _objects(),
    ]
    for c in cmds:
        r = subprocess.run(c, capture_output=True, text=True)
        assert r.returncode == 0, " ".join(c) + "\n" + r.stdout + r.stderr
    env = dict(os.environ)
    env["TSAN_OPTIONS"] = "halt_on_error=1 second_deadlock_stack=1"
    env["ASAN_OPTIONS"] = "detect_leaks=0 halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1 print_stacktrace=1"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr
    assert "runtime error" not in r.stderr, r.stderr
