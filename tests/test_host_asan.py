"""The library's host code under the address sanitiser (CPU only).

build() also links libcfr_asan.so: the same host sources compiled with the
sanitiser on the host side only, linked with the ordinary kernel object.
A child process preloads the sanitiser's runtime, loads that build through
CFR_LIBRARY and drives every host entry point that reads caller arrays or
builds host images (tests/asan_host_paths.py).  Any invalid read or write
aborts it with a sanitiser report."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2605_14277_amd"))


def test_host_paths_under_address_sanitizer():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "_cfr_build", os.path.join(ROOT, "paper_2605_14277_amd", "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    rt = b.asan_runtime()
    if rt is None or not os.path.exists(b.LIB_ASAN):
        pytest.skip("address-sanitised build not present (run build())")
    env = dict(os.environ)
    env["LD_PRELOAD"] = rt
    env["CFR_LIBRARY"] = b.LIB_ASAN
    # the interpreter and torch leak by design; report memory errors only
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["HIP_VISIBLE_DEVICES"] = ""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "asan_host_paths.py")],
                       env=env, capture_output=True, text=True, timeout=600)
    assert "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "host paths clean" in r.stdout
