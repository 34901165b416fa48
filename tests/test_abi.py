"""The C-ABI library loads and exports every symbol include/ssp.h declares.

CPU-only: no compute call is made here (there is no GPU in this process).
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ssp.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"SSP_API\s+[^;(]*?\b(ssp_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2207_13848_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        from paper_2207_13848_amd import build
        build.build()
    return _native.load()


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("ssp_predict_structure", "ssp_exact_structure", "ssp_reference_estimate",
                     "ssp_create", "ssp_destroy"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2207_13848_amd import _native
    out = subprocess.check_output(["nm", "-D", "--defined-only", _native.LIB_PATH], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for name in _declared():
        assert name in exported, f"{name} declared in ssp.h but not exported"
        assert hasattr(lib, name)
    assert set(_native.EXPORTED) == set(_declared())


def test_header_compiles_as_c():
    # the header is plain C: no HIP or torch types in the signatures
    src = '#include "ssp.h"\nint main(void){ ssp_stats s; (void)s; return (int)sizeof(ssp_stats); }\n'
    r = subprocess.run(["gcc", "-x", "c", "-std=c99", "-Wall", "-Werror", "-fsyntax-only",
                        "-I", os.path.join(ROOT, "include"), "-"], input=src, text=True,
                       capture_output=True)
    assert r.returncode == 0, r.stderr


def test_stats_layout_matches_header(lib):
    from paper_2207_13848_amd import _native
    assert ctypes.sizeof(_native.SspStats) == 64
    assert ctypes.sizeof(_native.SspCsr) == 40


def test_strings(lib):
    assert lib.ssp_version().decode().startswith("ssp ")
    assert lib.ssp_status_string(0) == b"ok"
    assert lib.ssp_status_string(-2) == b"A.ncols != B.nrows"
    assert lib.ssp_last_error(None) == b""


def test_null_handle_is_rejected(lib):
    from paper_2207_13848_amd import _native
    a = _native.SspCsr(0, 0, 0, None, None)
    assert lib.ssp_predict_structure(None, ctypes.byref(a), ctypes.byref(a), 0.5, 1, None, None,
                                     None, None) == -1
    assert lib.ssp_exact_structure(None, ctypes.byref(a), ctypes.byref(a), None, None, None) == -1
    assert lib.ssp_destroy(None) == -1
    assert lib.ssp_create(None, 0, 0) == -1


def test_create_without_a_gpu_reports_no_device(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib.ssp_create(ctypes.byref(h), 0, 0) == -7
    assert not h.value


def test_product_path_does_not_touch_the_oracle():
    # the package and its C sources never name the CPU oracle
    pkg = os.path.join(ROOT, "paper_2207_13848_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), f"{f} mentions the oracle"
                assert "workloads" not in text, f"{f} imports the input generators"


def test_default_tuning_matches_the_documented_defaults():
    import paper_2207_13848_amd as ssp
    assert ssp.default_tuning() == {"bin_max": [128, 1024, 8192], "hash_mult": 2, "long_len": 16,
                                    "big3": 1, "split_target": 1 << 19, "est_max_rf": 1 << 48}
