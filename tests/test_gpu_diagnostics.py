"""Measurement diagnostics of the library: the step-latency floor and the
vector FMA rate (used by the benchmark to put the kernels' times in context)."""
import pytest

from paper_1710_09799_amd import mln

pytestmark = pytest.mark.gpu


def test_step_floor_grows_with_the_chain():
    f0 = mln.step_floor(228, 512, 2000, 0)
    f128 = mln.step_floor(228, 512, 2000, 128)
    print(f"step floor: exchange + barrier {f0:.3f} us, + 128 dependent FMAs {f128:.3f} us")
    assert 0.0 < f0 < f128 < 10.0


def test_fma_rate_plain_fp32_outruns_fp64():
    r32, r64 = mln.fma_rate(False), mln.fma_rate(True)
    print(f"plain FMA rate: FP32 {r32:.1f} TFLOP/s, FP64 {r64:.1f} TFLOP/s")
    assert 0.0 < r64 < r32 < 157.3 * 1.05


def test_diagnostics_reject_bad_arguments():
    L = mln.load()
    import ctypes
    v = ctypes.c_double()
    assert L.mln_measure_step_floor(0, 512, 10, 0, ctypes.byref(v)) == -1
    assert L.mln_measure_step_floor(1, 100, 10, 0, ctypes.byref(v)) == -1
    assert L.mln_measure_step_floor(1, 512, 10, 7, ctypes.byref(v)) == -1
    assert L.mln_measure_fma_rate(0, None) == -1
