"""Measured ceilings (scdg_probe_mfma, scdg_probe_hbm_read): plausible values
against the vendor peaks, and argument checks before any launch."""
import ctypes as C

import pytest
import torch

from paper_1911_02366_amd import _lib as L
from paper_1911_02366_amd import probe

pytestmark = pytest.mark.gpu


def test_mfma_probe_is_near_the_vendor_peak():
    f64 = probe.mfma_tflops("fp64", iters=4000)
    f32 = probe.mfma_tflops("fp32", iters=4000)
    print(f"FP64 {f64:.1f} TF/s, FP32 {f32:.1f} TF/s", flush=True)
    # vendor dense peaks 78.6 (FP64) and 157.3 (FP32) TFLOP/s; a probe cannot beat
    # them by more than clock variation and should reach most of them
    assert 0.5 * 78.6 <= f64 <= 1.15 * 78.6
    assert 0.5 * 157.3 <= f32 <= 1.15 * 157.3


def test_hbm_probe_is_near_the_vendor_peak():
    gbs = probe.hbm_read_gbs(1 << 30)
    print(f"read {gbs:.0f} GB/s", flush=True)
    assert 0.5 * 8000 <= gbs <= 1.1 * 8000


def test_probe_argument_errors():
    lib = L.load()
    out = C.c_double()
    s = torch.cuda.current_stream().cuda_stream
    assert lib.scdg_probe_mfma(2, 100, s, C.byref(out)) == -1
    assert lib.scdg_probe_mfma(0, 0, s, C.byref(out)) == -1
    assert lib.scdg_probe_mfma(0, (1 << 20) + 1, s, C.byref(out)) == -1
    assert lib.scdg_probe_mfma(0, 100, s, None) == -1
    assert lib.scdg_probe_hbm_read(1 << 20, s, C.byref(out)) == -1          # below 64 MiB
    assert lib.scdg_probe_hbm_read((64 << 20) + 8, s, C.byref(out)) == -1   # not a multiple of 16
    assert lib.scdg_probe_hbm_read(17 << 30, s, C.byref(out)) == -1
    with pytest.raises(ValueError):
        probe.mfma_tflops("bf16")
