"""CPU checks of the serving loop's host core (admission, cancellation, poll, injected
allocation failures) behind a fake executor, built with sanitizers.

The queue and the device-memory ledger in ``csrc/serve_core.cpp`` hold no HIP code, so
they are compiled here with g++ together with ``tests/native/serve_core_check.cpp`` twice:
with AddressSanitizer + UndefinedBehaviorSanitizer (leak checking on, every report fatal)
and with ThreadSanitizer.  The library links the same source file, so what these runs
check is what ``rpa_submit``/``rpa_poll``/``rpa_finalize`` use.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2505_06021_amd", "csrc")
CHECK = os.path.join(ROOT, "tests", "native", "serve_core_check.cpp")

SANITIZERS = {
    "asan_ubsan": (["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                   {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
                    "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}),
    # GCC 11's TSan does not intercept the steady-clock condition waits; this build waits
    # on the system clock (serve_core.cpp, RPA_WAIT_ON_SYSTEM_CLOCK)
    "tsan": (["-fsanitize=thread", "-DRPA_WAIT_ON_SYSTEM_CLOCK"], {"TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1"}),
}


@pytest.mark.parametrize("kind", sorted(SANITIZERS))
def test_serve_core_under_sanitizer(kind, tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    flags, env_extra = SANITIZERS[kind]
    exe = str(tmp_path / f"serve_core_check_{kind}")
    cmd = (["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread"] + flags +
           [f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}",
            os.path.join(CSRC, "serve_core.cpp"), CHECK, "-o", exe])
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=240)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "all ok" in r.stdout, out[-6000:]
    for name in ("ledger", "fault_plan", "admission_order", "poll_semantics", "cancel_at_shutdown",
                 "alloc_failure", "progress_without_notify", "two_pollers",
                 "destructor_destroys_unpolled", "no_starvation", "stress"):
        assert f"ok {name}" in r.stdout, out[-6000:]
