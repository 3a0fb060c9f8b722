"""The C ABI used from plain C (tests/c_abi/rtm_c_demo.c, built by build()):
hipMalloc'd buffers, the probed gradient with fused and with separate
imaging, the device status query and a host-side rejection."""
import os
import subprocess

import pytest

from gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "rtm_c_demo")


def test_plain_c_client():
    require_gpu()
    if not os.path.exists(EXE):
        pytest.fail("tests/c_abi/rtm_c_demo is not built (run __graft_entry__.build())")
    p = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    say("  " + (p.stdout.strip() or p.stderr.strip()))
    assert p.returncode == 0, p.stderr
