"""The oracle under gcc's AddressSanitizer and UndefinedBehaviorSanitizer:
oracle/sanitize_check.c drives every exported routine of crk_oracle.c on
small meshes (Euler 1D/2D of degree 1..4 and 8 with every volume flux, both
limiters and walls; GLM-MHD in both interface forms; the semi-discrete
operator, the RKFR step, diagnostics, labels, the MLP) in one executable
built with both sanitizers, aborting on the first report and checking for
leaks at exit.  The sanitizer runtimes are linked statically so that the
executable does not depend on the order of preloaded libraries."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


def _sanitizers_available(tmp_path):
    src = tmp_path / "probe.c"
    src.write_text("int main(void) { return 0; }\n")
    r = subprocess.run(["gcc", "-fsanitize=address,undefined", "-static-libasan", "-static-libubsan", str(src),
                        "-o", str(tmp_path / "probe")], capture_output=True)
    return r.returncode == 0


def test_oracle_clean_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None or not _sanitizers_available(tmp_path):
        pytest.skip("gcc with the address and undefined-behaviour sanitizers is not available")
    exe = tmp_path / "sanitize_check"
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-static-libasan", "-static-libubsan", "-I", ORACLE, "-o", str(exe),
           os.path.join(ORACLE, "sanitize_check.c"), "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitize: ok" in r.stdout
