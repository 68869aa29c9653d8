"""Run inside test_sanitizers' subprocess only: checks that the sanitizer
build of the library is the one loaded and that the sanitizer runtime is in
the process (CPU).  Skipped in an ordinary run."""
import os

import pytest


@pytest.mark.skipif(not os.environ.get("HPM_LIBRARY"), reason="only under the sanitizer run")
def test_the_sanitized_library_is_loaded():
    from paper_2507_04130_amd import hpm as hb
    hb.load()
    assert hb.LIB_PATH == os.environ["HPM_LIBRARY"]
    maps = open("/proc/self/maps").read()
    assert os.environ["HPM_LIBRARY"] in maps
    assert "libclang_rt.asan" in maps
