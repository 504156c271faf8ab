"""The C ABI from a plain C program (paper_2512_14414_amd/csrc/c_abi_check.c,
built by build.py next to the library): the Neel state's energy per site,
-1/2, an invalid chi refused with CTM_EINVAL, and a second context on a
caller allocator (hipMalloc/hipFree) with the same energy and every block
handed back, without Python in the process."""
import os
import subprocess

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BIN = os.path.join(ROOT, "paper_2512_14414_amd", "c_abi_check")

pytestmark = pytest.mark.gpu


def test_c_program_on_the_c_abi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    assert os.access(BIN, os.X_OK), "c_abi_check is not built (run build())"
    r = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr
    assert "E = -0.500000000000000" in r.stdout
    assert "all back" in r.stdout
