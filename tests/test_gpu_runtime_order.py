"""The Python binding in a process that loads the library before torch:
the library links the system HIP runtime and torch carries its own copy;
loaded the other way round, the library's first device query reported no
device.  The load now brings torch in first.  Runs in a fresh process (the
small exponential's entry point, not a cooperative launch) and checks the
result against the oracle's Taylor exponential."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import krylov, phi

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import json, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from paper_2410_14917_amd import _lib
_lib.load()                                   # before any import of torch here
import paper_2410_14917_amd as kp
rng = np.random.default_rng(5)
m = 64
H = np.triu(rng.standard_normal((m + 1, m)), -1)
H[np.arange(m), np.arange(m)] -= 2.0
with kp.Context() as ctx:
    F = ctx.expm_hbar(H, m, 40.0 / m)
print(json.dumps(F.tolist()))
"""


def test_library_loaded_before_torch():
    print("runtime order: fresh process, library loaded first", flush=True)
    res = subprocess.run([sys.executable, "-c", SCRIPT, ROOT], capture_output=True, text=True,
                         timeout=180)
    sys.stdout.write(res.stderr[-2000:])
    assert res.returncode == 0
    F = np.array(json.loads(res.stdout.strip().splitlines()[-1]))
    rng = np.random.default_rng(5)
    m = 64
    H = np.triu(rng.standard_normal((m + 1, m)), -1)
    H[np.arange(m), np.arange(m)] -= 2.0
    ref = phi.expm_taylor((40.0 / m) * krylov.hbar(H, m))[:, 0]
    assert np.linalg.norm(F - ref) / np.linalg.norm(ref) <= 1e-12
