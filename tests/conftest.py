import os
import shutil
import subprocess
import sys
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


@pytest.fixture(scope="session")
def rocrand_philox():
    """Philox4x32-10 blocks from rocRAND's independent engine, built for the
    host from its open-source header. rows: [k0, k1, c0, c1, c2, c3] with
    c1 < 2^30 (the engine's offset is 4*(c1:c0) in 64 bits)."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "prr")
    subprocess.check_call([hipcc, "-O1", "-o", exe,
                           os.path.join(HERE, "philox_ref", "rocrand_philox_ref.cpp")], cwd=d)

    def run(rows):
        inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True,
                             check=True).stdout
        return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()],
                        dtype=np.uint64)

    yield run
    shutil.rmtree(d, ignore_errors=True)
