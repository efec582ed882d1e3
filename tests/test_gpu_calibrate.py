"""The matrix-rate calibration (spider_measure_matrix_rate): argument checks on the
host, and on the GPU self-consistent, physically plausible figures for the sparse
(smfmac 16x16x64) and dense (mfma 16x16x32) fp16 instructions."""
import ctypes
import math

import pytest

import paper_2506_22035_amd as sp


@pytest.mark.parametrize("sparse,waves,iters", [(1, 0, 10), (1, 5, 10), (0, 2, 0), (2, 2, 10), (1, 2, 10 ** 7 + 1)])
def test_rejects_out_of_range_arguments_before_any_device_work(sparse, waves, iters):
    out = ctypes.c_double()
    st = sp.lib().spider_measure_matrix_rate(sparse, waves, iters, None, ctypes.byref(out), None, None)
    assert st == 1
    assert "spider_measure_matrix_rate" in sp.lib().spider_last_error().decode()


def test_rejects_a_null_result_pointer():
    assert sp.lib().spider_measure_matrix_rate(1, 2, 10, None, None, None, None) == 1


@pytest.mark.gpu
@pytest.mark.parametrize("sparse", [True, False])
@pytest.mark.parametrize("waves", [1, 2, 4])
def test_rates_are_consistent_and_plausible(sparse, waves):
    m = sp.measure_matrix_rate(sparse, waves, 4000)
    t, g, c = m["TFLOPs"], m["clock_GHz"], m["cycles_per_instruction"]
    print("%s waves/SIMD %d: %.1f TFLOP/s at %.3f GHz, %.2f cycles per instruction"
          % ("sparse" if sparse else "dense", waves, t, g, c))
    assert all(math.isfinite(v) and v > 0 for v in (t, g, c))
    assert 0.3 < g < 3.5
    # a 16 x 16 x 32 multiply-add instruction occupies a SIMD's matrix pipe for at
    # least 4 cycles, and the whole chip cannot exceed 4x its published dense peak
    assert c >= 4.0
    assert t < 4 * 2500.0
