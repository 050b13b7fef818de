"""The C ABI from a plain C program on the GPU (tests/c/ngf_c_check.c), with
no Python or torch in the caller: a two-level registration of a synthetic
pair from host arrays, then at its result the level form of the
differentiation and the batched evaluation from device buffers, the
iteration log of a registration and an L-BFGS checkpoint replayed."""

import subprocess
import sys

import pytest

from test_capi import _build_c_check

pytestmark = pytest.mark.gpu


def test_c_caller_registers_on_the_gpu(tmp_path):
    exe = _build_c_check(tmp_path)
    print("[c-abi] running the C registration", flush=True)
    r = subprocess.run([exe, "gpu"], capture_output=True, text=True, timeout=120)
    sys.stdout.write(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "gpu registration ok" in r.stdout
    assert "gpu device forms ok" in r.stdout
    assert "iteration log and checkpoint ok" in r.stdout
