"""Tuning changes speed only: predictions, statistics and exact counts are the
same under every tuning the library accepts, including the autotuner's pick."""
import numpy as np
import pytest

import workloads
from tests.test_gpu_batch import _cases, _mixed_inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2207_13848_amd as m
    return m


# (est_max_rf 0: every row's ceiling by the 128-bit division; 1000: the long
# rows by it, the others by the estimate)
VARIANTS = [
    dict(bin_max=[64, 512, 4096], hash_mult=4, long_len=16, big3=0, split_target=1 << 15,
         est_max_rf=0),
    dict(bin_max=[32, 256, 2048], hash_mult=8, long_len=128, big3=1, split_target=1 << 19,
         est_max_rf=1000),
    dict(bin_max=[1, 1, 1], hash_mult=2, long_len=8, big3=1, split_target=1 << 12,
         est_max_rf=1 << 48),
    dict(bin_max=[128, 1024, 8192], hash_mult=2, long_len=1024, big3=0, split_target=1 << 40,
         est_max_rf=1),
]


def _run_batch(ssp, h, inputs):
    cases = _cases(ssp, inputs)
    ssp.predict_batch(cases, handle=h)
    torch.cuda.synchronize()
    return [(c.pred.clone(), c.stats.clone(), None if c.row_flop is None else c.row_flop.clone())
            for c in cases]


def test_outputs_do_not_depend_on_tuning(ssp):
    inputs = _mixed_inputs(n_extra=4)
    h = ssp.Handle(0)
    base = _run_batch(ssp, h, inputs)
    A, B = inputs[9][0], inputs[9][1]  # split long rows
    Ad, Bd = ssp.DeviceCSR.from_csr(A, "cuda:0"), ssp.DeviceCSR.from_csr(B, "cuda:0")
    ex0, st0 = ssp.exact_structure(Ad, Bd, handle=h)
    R = workloads.rmat(1 << 16, 16, 3)
    Rd = ssp.DeviceCSR.from_csr(R, "cuda:0")
    exr0, _ = ssp.exact_structure(Rd, Rd, handle=h)
    torch.cuda.synchronize()
    for v in VARIANTS:
        ssp.set_tuning(v, handle=h)
        assert ssp.get_tuning(handle=h) == v
        got = _run_batch(ssp, h, inputs)
        for i, (a, b) in enumerate(zip(base, got)):
            assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), f"{v}: case {i}"
            if a[2] is not None:
                assert torch.equal(a[2], b[2])
        ex, st = ssp.exact_structure(Ad, Bd, handle=h)
        exr, _ = ssp.exact_structure(Rd, Rd, handle=h)
        torch.cuda.synchronize()
        assert torch.equal(ex, ex0) and torch.equal(st, st0) and torch.equal(exr, exr0), f"{v}"
    h.close()


def test_set_tuning_rejects_values_outside_the_limits(ssp):
    h = ssp.Handle(0)
    good = ssp.default_tuning()
    bad = [dict(good, hash_mult=3), dict(good, bin_max=[256, 1024, 8192]),
           dict(good, bin_max=[128, 2048, 8192]), dict(good, bin_max=[128, 1024, 16384]),
           dict(good, bin_max=[512, 256, 8192], hash_mult=2), dict(good, long_len=4),
           dict(good, long_len=2048), dict(good, big3=2), dict(good, split_target=100),
           dict(good, est_max_rf=(1 << 48) + 1)]
    for b in bad:
        with pytest.raises(ssp.SspError) as ei:
            ssp.set_tuning(b, handle=h)
        assert ei.value.status == -1, b
    assert ssp.get_tuning(handle=h) == good
    h.close()


def test_autotune_keeps_results(ssp):
    inputs = [x for x in _mixed_inputs() if x[0].nrows > 0][:6]
    h = ssp.Handle(0)
    base = _run_batch(ssp, h, inputs)
    cases = _cases(ssp, inputs)
    r = ssp.autotune(cases, reps=2, handle=h)
    print("autotune", r, flush=True)
    assert ssp.get_tuning(handle=h) == r["tuning"]
    assert r["best_ms"] > 0 and r["default_ms"] > 0
    got = _run_batch(ssp, h, inputs)
    for a, b in zip(base, got):
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    h.close()
