"""The oracle (C) and the library's host-side builders and encoder
(host_tables.cpp) built with AddressSanitizer and UndefinedBehaviorSanitizer
by the host compilers and run over seeded random strips: no out-of-bounds
access, leak or undefined behaviour may show.  CPU only; nothing here is GPU
code."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _have(compiler, flags, tmp):
    src = os.path.join(tmp, "probe.c")
    with open(src, "w") as f:
        f.write("int main(void) { return 0; }\n")
    r = subprocess.run([compiler, *flags, "-x", "c", src, "-o", os.path.join(tmp, "probe")], capture_output=True)
    return r.returncode == 0


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    return r.returncode, r.stdout + r.stderr


@pytest.fixture(scope="module")
def tmpdir_san(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("san"))
    if not shutil.which("gcc") or not shutil.which("g++") or not _have("gcc", SAN, d):
        pytest.skip("no sanitizer runtime for the host compilers")
    return d


def test_oracle_under_sanitizers(tmpdir_san):
    exe = os.path.join(tmpdir_san, "oracle_san")
    r = subprocess.run(["gcc", *SAN, "-std=c99", os.path.join(ROOT, "oracle", "fptc_oracle.c"),
                        os.path.join(HERE, "oracle_driver.c"), "-lm", "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    rc, out = _run(exe)
    assert rc == 0 and "ok" in out, out[-4000:]


def test_host_encoder_under_sanitizers(tmpdir_san):
    exe = os.path.join(tmpdir_san, "host_san")
    r = subprocess.run(["g++", *SAN, "-std=c++17", "-pthread", f"-I{os.path.join(ROOT, 'include')}",
                        os.path.join(ROOT, "paper_2605_01086_amd", "csrc", "host_tables.cpp"),
                        os.path.join(HERE, "host_driver.cpp"), "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    rc, out = _run(exe)
    assert rc == 0 and "ok" in out, out[-4000:]
