"""The host-side ABI checks (tests/test_abi_host.py) under AddressSanitizer
and UndefinedBehaviorSanitizer: the library's host code is rebuilt with both
(build.py --host-sanitizers), loaded through QIHT_LIB_PATH in a child
process with the shared ASan runtime preloaded, and any report ends the
child with a failure.  CPU only: no kernel runs."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.timeout(600)
def test_abi_host_checks_under_asan_and_ubsan(tmp_path):
    from paper_1802_04907_amd import build
    try:
        build.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    rt = build.sanitizer_runtime()
    if rt is None:
        pytest.skip("no shared ASan runtime in this ROCm")
    lib = build.build_host_sanitized()
    env = dict(os.environ)
    env.update({
        "QIHT_LIB_PATH": lib,
        "LD_PRELOAD": rt,
        "ASAN_OPTIONS": f"detect_leaks=0:halt_on_error=1:log_path={tmp_path}/asan",
        "UBSAN_OPTIONS": f"halt_on_error=1:print_stacktrace=1:log_path={tmp_path}/ubsan",
    })
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi_host.py"),
                        "-q", "-p", "no:cacheprovider"], cwd=str(tmp_path), env=env,
                       capture_output=True, text=True, timeout=500)
    reports = sorted(p for p in os.listdir(tmp_path) if p.startswith(("asan", "ubsan")))
    text = "".join(open(os.path.join(tmp_path, p)).read()[:4000] for p in reports)
    assert r.returncode == 0 and not reports, f"{r.stdout[-2000:]}\n{r.stderr[-2000:]}\n{text}"
    assert " passed" in r.stdout
