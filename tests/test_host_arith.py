"""Host builds of the library's exact wide arithmetic, checked on the CPU.

The reference design's rows (Eq. (2)) whose numerator rf z* M exceeds 128
bits take a 192-by-128-bit division.  No input small enough for a test reaches
it on the GPU, so the same routine (a __host__ __device__ function of the
library's device header) is compiled for the host here and compared with
Python's exact integers.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def wide_div_exe(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    exe = tmp_path_factory.mktemp("hostarith") / "wide_div_check"
    subprocess.check_call([HIPCC, "--offload-host-only", "-O2", "-std=c++17", "-o", str(exe),
                           os.path.join(HERE, "host", "wide_div_check.cpp")])
    return str(exe)


def test_ceil_div_192_by_128(wide_div_exe):
    rng = np.random.default_rng(3)
    m = 2**64 - 1
    cases = [(1, 1, 1), (5, 12, 17), (2**62 - 1, 2**93 - 1, 2**93 - 1),
             (2**62 - 1, (2**62 - 1) * (2**31 - 1), 2**31 * (2**62 - 1)), (3, 2**64 + 5, 7),
             (2**63, 2**64, 2**65)]
    for _ in range(3000):
        a = int(rng.integers(1, 2**62))
        d = int(rng.integers(1, 2**62)) * int(rng.integers(1, 2**31))
        qmax = (d << 64) // a  # quotient below 2^64
        q = int(rng.integers(0, 2**62)) * int(rng.integers(1, 2**31)) % max(qmax, 1)
        cases.append((a, q, d))
    text = "".join(f"{a} {q >> 64} {q & m} {d >> 64} {d & m}\n" for a, q, d in cases)
    out = subprocess.run([wide_div_exe], input=text, capture_output=True, text=True,
                         check=True).stdout.split()
    assert len(out) == len(cases)
    wide = 0
    for (a, q, d), got in zip(cases, out):
        assert int(got) == -(-(a * q) // d), (a, q, d)
        wide += a * q >= 2**128
    assert wide > 100  # most cases need the 192-bit product
