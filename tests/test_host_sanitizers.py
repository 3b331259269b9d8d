"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (with leak
checking): every unit rebuilt with the sanitizers on its host pass only (-Xarch_host before
each flag; device code as built for the product), linked into a program of its own
(host_sanitize_check.cpp) that drives descriptor validation, workspace sizing and the error
paths of the entry points -- all of which return before touching a device, so no GPU is
needed.  Every check must return what the header states, with no sanitizer report."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CLANG = "/opt/rocm/llvm/bin/clang++"
HOST_SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
            "-fno-omit-frame-pointer", "-g"]


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not os.path.exists(CLANG) or not (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc")):
        pytest.skip("no ROCm compiler")
    import sys
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    from paper_2503_10263_amd import build as B
    d = tmp_path_factory.mktemp("host_san")
    extra = [x for flag in HOST_SAN for x in ("-Xarch_host", flag)]
    lib = B.build(out=str(d / "libkarl.so"), extra=extra)
    exe = str(d / "host_sanitize_check")
    subprocess.run([CLANG, "-std=c++17"] + HOST_SAN + ["-I", os.path.join(ROOT, "include"), "-o", exe,
                    os.path.join(HERE, "host_sanitize_check.cpp"), f"-L{d}", "-lkarl",
                    f"-Wl,-rpath,{d}"], check=True)
    assert os.path.exists(lib)
    return exe


@pytest.mark.slow
def test_host_code_clean_under_sanitizers(checker):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([checker], env=env, capture_output=True, text=True, timeout=300)
    assert p.returncode == 0, p.stdout[-3000:] + p.stderr[-3000:]
    assert "runtime error" not in p.stderr and "Sanitizer" not in p.stderr, p.stderr[-3000:]
    lines = p.stdout.splitlines()
    assert lines[-1] == "0 failed" and sum(l.startswith("ok") for l in lines) >= 30, p.stdout
