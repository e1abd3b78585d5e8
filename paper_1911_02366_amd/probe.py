"""Measured ceilings beside the vendor peaks: matrix-core throughput and HBM
streaming-read bandwidth, from the library's probe kernels (scdg_probe_*)."""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L


def _stream(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def mfma_tflops(precision: str = "fp64", iters: int = 20000, stream=None) -> float:
    """Dense TFLOP/s of back-to-back 16x16x4 MFMAs (precision "fp64" or "fp32")."""
    if precision not in ("fp64", "fp32"):
        raise ValueError(precision)
    out = C.c_double(0.0)
    st = L.load().scdg_probe_mfma(0 if precision == "fp64" else 1, int(iters), _stream(stream), C.byref(out))
    if st != 0:
        raise L.ScdgError(st, "scdg_probe_mfma")
    return out.value


def hbm_read_gbs(nbytes: int = 4 << 30, stream=None) -> float:
    """GB/s (1e9 bytes/s) of a streaming read of an nbytes device buffer."""
    out = C.c_double(0.0)
    st = L.load().scdg_probe_hbm_read(int(nbytes), _stream(stream), C.byref(out))
    if st != 0:
        raise L.ScdgError(st, "scdg_probe_hbm_read")
    return out.value
