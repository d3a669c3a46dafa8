"""The library's build flags (paper_2210_07580_amd/build.py): every HIP
source is compiled with the packed-FP32 instructions switched off, and the
checking variant scopes each sanitizer flag to the host half of the
compilation (the gfx950 code is never instrumented)."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2210_07580_amd import build as B  # noqa: E402


def test_packed_fp32_instructions_are_switched_off():
    f = B.FLAGS
    i = f.index("-packed-fp32-ops")
    assert f[i - 1] == "-Xclang" and f[i - 2] == "-target-feature" and f[i - 3] == "-Xclang"
    assert "--offload-arch=gfx950" in f


def test_sanitizer_flags_are_host_only():
    flags = B._host_sanitizer_flags("undefined")
    assert len(flags) % 2 == 0
    for scope, flag in zip(flags[0::2], flags[1::2]):
        assert scope == "-Xarch_host", (scope, flag)
    assert "-fsanitize=undefined" in flags[1::2]
    assert not any(f.startswith("-fsanitize") for f in B.FLAGS)


def test_only_the_host_undefined_behaviour_build_is_offered():
    with pytest.raises(ValueError):
        B._sanitizer_runtime("address")
