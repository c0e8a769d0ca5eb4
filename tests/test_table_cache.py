"""The step-table cache shared by threads (csrc/table_cache.h): a host-only
C++ harness built with g++ and ThreadSanitizer, eight threads over eleven
keys in a four-entry cache; values stay intact while held and are destroyed
exactly once after their last holder."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("sanitize", ["thread", "address"])
def test_table_cache_under_threads(tmp_path, sanitize):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "table_cache_threads"
    src = os.path.join(HERE, "native", "table_cache_threads.cpp")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", f"-fsanitize={sanitize}",
                           "-pthread", src, "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(r.stdout, r.stderr[-2000:])
    assert r.returncode == 0, r.stderr[-2000:]
    assert "WARNING: ThreadSanitizer" not in r.stderr
