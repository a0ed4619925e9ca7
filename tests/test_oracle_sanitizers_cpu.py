"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer:
a driver (tests/oracle_sanitize_driver.c) calls every entry point on small
grids with every boundary kind; any out-of-bounds access, use after free,
leak or undefined operation aborts it.  Host code only (gcc)."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "drv")
        cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "oracle"),
               os.path.join(HERE, "oracle_sanitize_driver.c"),
               os.path.join(ROOT, "oracle", "lbm_oracle.c"), "-lm", "-o", exe]
        subprocess.run(cmd, check=True, capture_output=True, timeout=300)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        assert r.returncode == 0, r.stderr[-4000:]
        assert "all entry points ran" in r.stdout
