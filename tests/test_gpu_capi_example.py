"""The plain C user of the library (tests/capi/example.c, built by the
package build) runs on the GPU: exact-root parity in both precision forms,
one-launch binning equal to pr_density, and the backward closed form."""
from __future__ import annotations

import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

BINARY = os.path.join(os.path.dirname(os.path.abspath(__file__)), "capi", "capi_example")


def test_c_program_through_the_abi():
    if not os.path.exists(BINARY):
        pytest.fail("tests/capi/capi_example is not built (run __graft_entry__.build())")
    r = subprocess.run([BINARY], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().endswith("ok")
