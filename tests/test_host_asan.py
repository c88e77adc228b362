"""AddressSanitizer build of the library's host code (CPU only).

Every library source is compiled with hipcc with the sanitizer on the host
pass only (device code is untouched), linked with the host driver
tests/host_asan/driver.cpp, and run: geometry construction and queries,
plans over many option sets and workloads, workspace queries, argument and
device-error paths, batch setup and the destroy calls, with heap-overflow,
use-after-free and leak detection.  No GPU is used (none is needed for these
paths; device calls fail cleanly where there is none).
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2109_02842_amd", "csrc")
sys.path.insert(0, ROOT)


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_host_code_under_address_sanitizer(tmp_path):
    from paper_2109_02842_amd import build as b
    cc = _hipcc()
    if cc is None:
        pytest.skip("hipcc not available")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = [f for f in b.CFLAGS if f != "-O3"] + ["-O1", "-g"] + san
    objs = []
    procs = []
    for src in b.SOURCES + ["../../tests/host_asan/driver.cpp"]:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([cc] + flags + ["-c", os.path.join(SRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out
    exe = str(tmp_path / "host_asan")
    res = subprocess.run([cc, f"--offload-arch={b.ARCH}"] + san + ["-o", exe] + objs, capture_output=True, text=True)
    assert res.returncode == 0, res.stdout + res.stderr
    supp = tmp_path / "lsan.supp"
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libamd_comgr\nleak:libdrm\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               LSAN_OPTIONS=f"suppressions={supp}", HIP_VISIBLE_DEVICES=os.environ.get("HIP_VISIBLE_DEVICES", ""))
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = run.stdout + run.stderr
    assert "AddressSanitizer" not in out and "LeakSanitizer" not in out, out[-4000:]
    assert run.returncode == 0, out[-4000:]
    assert "0 failures" in out
