"""The allocation-free Newton-matrix product (scdg_dg_jacobian_apply_noalloc)
against the allocating one (scdg_dg_jacobian_apply), through the C ABI: the
same kernels on the same FP64 inputs, so the results must agree to the FP64
parity bar (they are expected bit for bit).  Two calls in a row, the second on
a smaller mesh (the shared scratch array then holds the first call's larger
gradient), then a mesh above the array's size, which must be refused before
any device work."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_common import DEV, to_np
from paper_1911_02366_amd import DgResidual
from paper_1911_02366_amd import _lib as L
from workload import dgsem as wd
from workload.physics import FlowParams

pytestmark = pytest.mark.gpu


def _inputs(k, n, seed):
    q = wd.taylor_green_state(wd.Mesh(k, n), FlowParams(0.1, 1600.0), seed)
    v = np.random.default_rng(seed + 50).standard_normal(q.shape)
    return (torch.tensor(q.reshape(-1), device=DEV).contiguous(),
            torch.tensor(v.reshape(-1), device=DEV).contiguous())


def _both(lib, k, n, seed, inv_dt):
    print(f"no-alloc product: K={k} N={n} seed={seed} inv_dt={inv_dt}", flush=True)
    dg = DgResidual(k, n, mach=0.1, reynolds=1600.0)
    q, v = _inputs(k, n, seed)
    ref = torch.empty_like(q)
    got = torch.full_like(q, float("nan"))
    assert lib.scdg_dg_jacobian_apply(dg.handle, C.c_void_p(q.data_ptr()), C.c_void_p(v.data_ptr()),
                                      C.c_double(inv_dt), C.c_void_p(ref.data_ptr())) == L.SCDG_OK
    assert lib.scdg_dg_jacobian_apply_noalloc(dg.handle, C.c_void_p(q.data_ptr()), C.c_void_p(v.data_ptr()),
                                              C.c_double(inv_dt), C.c_void_p(got.data_ptr())) == L.SCDG_OK
    torch.cuda.synchronize()
    r, g = to_np(ref), to_np(got)
    dg.close()
    return r, g


def test_noalloc_matches_allocating_product():
    lib = L.load()
    for k, n, seed, inv_dt in ((4, 5, 1, 200.0), (2, 3, 2, 0.0)):      # second call: smaller input
        r, g = _both(lib, k, n, seed, inv_dt)
        assert np.all(np.isfinite(g))
        err = float(np.abs(g - r).max() / np.abs(r).max())
        print(f"  max rel difference {err:.2e}", flush=True)
        assert err <= 1e-13


def test_noalloc_refuses_a_mesh_above_the_scratch_size():
    lib = L.load()
    dg = DgResidual(16, 5, mach=0.1, reynolds=1600.0)     # 884 736 nodes: 106 MB of gradient
    q = torch.zeros(dg.n_dof, dtype=torch.float64, device=DEV)
    out = torch.empty_like(q)
    st = lib.scdg_dg_jacobian_apply_noalloc(dg.handle, C.c_void_p(q.data_ptr()), C.c_void_p(q.data_ptr()),
                                            C.c_double(1.0), C.c_void_p(out.data_ptr()))
    assert st == -8      # SCDG_ERR_UNSUPPORTED
    dg.close()
