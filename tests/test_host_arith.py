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


@pytest.fixture(scope="module")
def window_scan_exe(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    exe = tmp_path_factory.mktemp("hostscan") / "window_scan_check"
    subprocess.check_call([HIPCC, "--offload-host-only", "-O2", "-std=c++17", "-o", str(exe),
                           os.path.join(HERE, "host", "window_scan_check.cpp")])
    return str(exe)


def _window_scan(exe, budget, n3, wins):
    text = f"{budget} {len(n3)}\n" + "".join(f"{a} {w}\n" for a, w in zip(n3, wins))
    out = subprocess.run([exe], input=text, capture_output=True, text=True,
                         check=True).stdout.split()
    return np.array(out, dtype=np.int64).reshape(-1, 3)


def test_window_prefix_never_wraps(window_scan_exe):
    """The sampling scan splits a group's long rows when every part window
    requested up to and including the group fits the budget.  With the
    counts clamped, that decision equals the one taken on exact (unbounded)
    prefixes, and the bin-3 offsets below stay exact, even where the raw
    window counts would wrap a 32-bit field many times over."""
    rng = np.random.default_rng(11)
    cases = []
    for budget in (1024, 8192):
        # huge counts from the start: the unclamped field wraps after two groups
        cases.append((budget, [5] * 3000, [2**31 + 7] * 3000))
        # small counts that fill the budget, then counts that would wrap
        w = [int(x) for x in rng.integers(0, 40, 2500)] + [2**32 - 1] * 2000
        cases.append((budget, [int(x) for x in rng.integers(0, 9, len(w))], w))
        # a sum of 2^32 exactly early on, then zeros and small counts
        w = [2**30] * 4 + [0] * 1500 + [int(x) for x in rng.integers(0, 3, 1500)]
        cases.append((budget, [1] * len(w), w))
        # wraps inside one chunk, no split after the first overflowing group
        w = [int(x) for x in rng.integers(0, 2**32, 5000)]
        cases.append((budget, [int(x) for x in rng.integers(0, 1000, 5000)], w))
    nsplit = 0
    for budget, n3, wins in cases:
        got = _window_scan(window_scan_exe, budget, n3, wins)
        wp = np.concatenate([[0], np.cumsum(np.array(wins, dtype=object))[:-1]])
        o3 = np.concatenate([[0], np.cumsum(np.array(n3, dtype=np.int64))[:-1]])
        split = [int(w != 0 and p + w <= budget) for p, w in zip(wp, wins)]
        assert np.array_equal(got[:, 2], split), budget
        assert np.array_equal(got[:, 0], o3 % 2**32), budget
        # where a group is split, its window offset is the exact prefix
        for g, s in enumerate(split):
            if s:
                assert got[g, 1] == wp[g]
        nsplit += sum(split)
    assert nsplit > 200  # the cases do exercise the split decision
