"""GPU parity of the learned-guess network kernels (scdg_mlp_*, scdg_guess_*)
against the FP64 oracle (oracle/mlp.py), on seeded inputs.

Tolerance: the kernels store FP32 and accumulate dot products of length K in
FP32 on the matrix cores; the oracle evaluates the same FP32 inputs in FP64.
The rounding error of a length-K FP32 dot product is at most about K u sum|a b|
(u = 2^-24, K <= 1250 gives 7.5e-5 of sum|a b|) and typically sqrt(K) u; the
tests ask for 2e-5 norm-wise and 2e-4 of the largest magnitude element-wise.
"""
import numpy as np
import pytest
import torch

from gpu_common import DEV, to_np
from oracle import mlp as om
from paper_1911_02366_amd import ScdgError
from paper_1911_02366_amd.mlp import Mlp

pytestmark = pytest.mark.gpu

SHAPES = [(6, 5, 2, 4, 3), (70, 33, 3, 45, 130), (1250, 256, 2, 625, 300)]


def _setup(shape, seed):
    n_in, n_h, n_l, n_out, batch = shape
    net = Mlp(n_in, n_h, n_l, n_out, max_batch=batch)
    w = net.init_params(seed, DEV)
    rng = np.random.default_rng(seed + 1)
    x = rng.standard_normal((batch, n_in)).astype(np.float32)
    t = rng.standard_normal((batch, n_out)).astype(np.float32)
    return net, w, x, t


def _close(got, want, norm_tol=2e-5, elem_tol=2e-4):
    got = np.asarray(got, dtype=np.float64).reshape(-1)
    want = np.asarray(want, dtype=np.float64).reshape(-1)
    scale = max(np.abs(want).max(), 1e-30)
    assert np.linalg.norm(got - want) <= norm_tol * max(np.linalg.norm(want), 1e-30)
    assert np.abs(got - want).max() <= elem_tol * scale


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_backward_match_oracle(shape):
    print(f"mlp shape {shape}", flush=True)
    n_in, n_h, n_l, n_out, batch = shape
    net, w, x, t = _setup(shape, 3)
    xd = torch.tensor(x.reshape(-1), device=DEV)
    td = torch.tensor(t.reshape(-1), device=DEV)
    y = net.forward(w, xd, batch)
    dy = torch.empty_like(y)
    loss = net.mse(y, td, batch * n_out, dy=dy)
    dx = torch.empty_like(xd)
    dw = net.backward(w, xd, dy, batch, dx=dx)
    torch.cuda.synchronize()
    sh = (n_in, n_h, n_l, n_out)
    y_o, acts = om.forward(to_np(w), x, sh)
    _close(to_np(y), y_o)
    # the loss and its gradient are taken at the kernel's own y (FP32)
    loss_o, dy_o = om.mse(to_np(y).reshape(batch, n_out), t)
    assert abs(float(loss) - loss_o) <= 1e-6 * loss_o
    _close(to_np(dy), dy_o, 1e-6, 1e-6)
    dw_o, dx_o = om.backward(to_np(w), acts, to_np(dy).reshape(batch, n_out), sh)
    lay, _ = om.layout(*sh)
    dwn = to_np(dw)
    for off, fi, fo, bo in lay:
        _close(dwn[off:off + fi * fo], dw_o[off:off + fi * fo])
        _close(dwn[bo:bo + fo], dw_o[bo:bo + fo])
    _close(to_np(dx), dx_o)
    net.close()


def test_adam_matches_oracle():
    net = Mlp(30, 20, 2, 10, max_batch=4)
    n = net.n_params
    rng = np.random.default_rng(4)
    w, g = rng.standard_normal(n).astype(np.float32), rng.standard_normal(n).astype(np.float32)
    m1 = (0.1 * rng.standard_normal(n)).astype(np.float32)
    m2 = (0.1 * rng.random(n)).astype(np.float32)
    wd, gd, m1d, m2d = (torch.tensor(a, device=DEV) for a in (w, g, m1, m2))
    for step in (1, 7):
        net.adam(wd, gd, m1d, m2d, lr=1e-3, step=step)
        # the kernel receives lr, beta1, beta2 and eps as FP32 values: give the oracle the same
        f = lambda v: float(np.float32(v))
        w, m1, m2 = om.adam(w, g, m1, m2, f(1e-3), step, f(0.9), f(0.999), f(1e-8))
        _close(to_np(wd), w, 1e-6, 1e-6)
        _close(to_np(m1d), m1, 1e-6, 1e-6)
        _close(to_np(m2d), m2, 1e-6, 1e-6)
        w, m1, m2 = to_np(wd), to_np(m1d), to_np(m2d)
    net.close()


def test_gather_is_exact_and_backward_needs_matching_forward():
    net = Mlp(8, 4, 1, 3, max_batch=16)
    src = torch.arange(40 * 8, dtype=torch.float32, device=DEV)
    idx = torch.tensor([5, 0, 39, 5, 17], dtype=torch.int32, device=DEV)
    out = net.gather(src, 8, idx, 5)
    want = to_np(src).reshape(40, 8)[[5, 0, 39, 5, 17]]
    np.testing.assert_array_equal(to_np(out).reshape(5, 8), want)
    w = net.init_params(0, DEV)
    x = torch.zeros(16 * 8, dtype=torch.float32, device=DEV)
    net.forward(w, x, 16)
    with pytest.raises(ScdgError):
        net.backward(w, x, torch.zeros(8 * 3, dtype=torch.float32, device=DEV), 8)
    with pytest.raises(ScdgError):
        net.forward(w, torch.zeros(17 * 8, dtype=torch.float32, device=DEV), 17)
    net.close()


def test_guess_maps_match_oracle():
    n_elem, dpe = 27, 5 * 64
    net = Mlp(2 * dpe, 16, 1, dpe, max_batch=n_elem)
    net3 = Mlp(3 * dpe, 16, 1, dpe, max_batch=n_elem)    # with the residual block
    rng = np.random.default_rng(8)
    base = np.tile([1.0, 0.1, -0.2, 0.05, 71.9], n_elem * dpe // 5)
    q = base + 1e-2 * rng.standard_normal(n_elem * dpe)
    dq_prev = 1e-4 * rng.standard_normal(n_elem * dpe)
    dq = dq_prev * (1 + 0.01 * rng.standard_normal(n_elem * dpe))
    r = 3.0 * rng.standard_normal(n_elem * dpe)
    qd, dpd, dqd, rd = (torch.tensor(a, device=DEV) for a in (q, dq_prev, dq, r))
    stats = net.guess_stats(qd, dpd, dqd, rd)
    np.testing.assert_allclose(to_np(stats), np.concatenate(om.field_stats(q, dq_prev, dq, r)), rtol=1e-12,
                               atol=0)
    s_np = to_np(net.guess_stats(qd, dpd))            # without dq: rc = rp; without r: rr = 1
    np.testing.assert_array_equal(s_np[15:20], s_np[10:15])
    np.testing.assert_array_equal(s_np[20:], np.ones(5))
    sv = to_np(stats)
    so = (sv[:5], sv[5:10], sv[10:15], sv[15:20], sv[20:])   # the same statistics on both sides
    x = to_np(net.features(qd, dpd, stats, n_elem))
    np.testing.assert_array_equal(x, om.features(q, dq_prev, so, n_elem).astype(np.float32).reshape(-1))
    x3 = to_np(net3.features(qd, dpd, stats, n_elem, r=rd))
    np.testing.assert_array_equal(x3, om.features(q, dq_prev, so, n_elem, r).astype(np.float32).reshape(-1))
    with pytest.raises(ScdgError):
        net3.features(qd, dpd, stats, n_elem)          # a residual block needs r
    net3.close()
    t = to_np(net.target(dqd, dpd, stats, n_elem))
    np.testing.assert_array_equal(t, om.target(dq, dq_prev, so, n_elem).astype(np.float32).reshape(-1))
    y = torch.tensor(t, device=DEV)
    back = to_np(net.apply(dpd, y, stats, n_elem))
    np.testing.assert_allclose(back, om.apply(dq_prev, t, so, n_elem), rtol=1e-15, atol=0)
    net.close()


def test_training_steps_follow_oracle():
    shape = (12, 24, 2, 6, 40)
    n_in, n_h, n_l, n_out, batch = shape
    net, w, x, t = _setup(shape, 9)
    xd = torch.tensor(x.reshape(-1), device=DEV)
    td = torch.tensor(t.reshape(-1), device=DEV)
    m1 = torch.zeros_like(w)
    m2 = torch.zeros_like(w)
    dy = torch.empty(batch * n_out, dtype=torch.float32, device=DEV)
    wo = to_np(w).astype(np.float64)
    m1o, m2o = np.zeros_like(wo), np.zeros_like(wo)
    sh = shape[:4]
    losses = []
    for step in range(1, 21):
        y = net.forward(w, xd, batch)
        loss = net.mse(y, td, batch * n_out, dy=dy)
        dw = net.backward(w, xd, dy, batch)
        net.adam(w, dw, m1, m2, lr=3e-3, step=step)
        losses.append(float(loss))
        yo, acts = om.forward(wo, x, sh)
        _, dyo = om.mse(yo, t)
        dwo, _ = om.backward(wo, acts, dyo, sh)
        wo, m1o, m2o = om.adam(wo, dwo, m1o, m2o, 3e-3, step)
    _close(to_np(w), wo, 1e-4, 1e-3)
    assert losses[-1] < losses[0]
    net.close()


def test_bitwise_repeatable():
    shape = (1250, 256, 2, 625, 200)
    outs = []
    for _ in range(2):
        net, w, x, t = _setup(shape, 12)
        xd = torch.tensor(x.reshape(-1), device=DEV)
        y = net.forward(w, xd, 200)
        dy = torch.empty_like(y)
        net.mse(y, torch.tensor(t.reshape(-1), device=DEV), y.numel(), dy=dy)
        dw = net.backward(w, xd, dy, 200)
        outs.append((to_np(y).copy(), to_np(dw).copy()))
        net.close()
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    np.testing.assert_array_equal(outs[0][1], outs[1][1])


# ---------------------------------------------------------------- bfloat16 compute mode
# Both sides round the same FP32 operands to bfloat16 (ties to even), so for a
# single linear map (the operands are the inputs themselves) the only
# difference left is FP32 versus FP64 accumulation of exact products: the FP32
# tolerances above apply.  Between layers the kernel rounds its own FP32
# activations and gradients while the oracle rounds its FP64 ones cast to FP32;
# the two FP32 values can differ in the last bits, which moves a bfloat16
# rounding across a tie in a small fraction of the elements (about 1e-3 of
# them); each such element changes one product operand by one bfloat16 step
# (2^-8 relative).  The multi-layer bound is therefore norm-wise 2e-3 and
# element-wise 2e-2 of the largest magnitude.

@pytest.mark.parametrize("shape", [(70, 1, 0, 45, 130), (1250, 1, 0, 625, 300)])
def test_bf16_linear_map_matches_oracle(shape):
    print(f"bf16 linear map {shape}", flush=True)
    n_in, n_h, n_l, n_out, batch = shape
    net, w, x, t = _setup(shape, 5)
    net.set_compute("bf16")
    xd = torch.tensor(x.reshape(-1), device=DEV)
    td = torch.tensor(t.reshape(-1), device=DEV)
    y = net.forward(w, xd, batch)
    dy = torch.empty_like(y)
    net.mse(y, td, batch * n_out, dy=dy)
    dx = torch.empty_like(xd)
    dw = net.backward(w, xd, dy, batch, dx=dx)
    torch.cuda.synchronize()
    sh = (n_in, n_h, n_l, n_out)
    y_o, acts = om.forward(to_np(w), x, sh, bf16=True)
    _close(to_np(y), y_o)
    y_32, _ = om.forward(to_np(w), x, sh)
    assert np.linalg.norm(to_np(y) - y_32.reshape(-1)) > 1e-4 * np.linalg.norm(y_32)   # the rounding is active
    dw_o, dx_o = om.backward(to_np(w), acts, to_np(dy).reshape(batch, n_out), sh, bf16=True)
    off, fi, fo, bo = om.layout(*sh)[0][0]
    _close(to_np(dw)[off:off + fi * fo], dw_o[off:off + fi * fo])
    _close(to_np(dw)[bo:bo + fo], dw_o[bo:bo + fo])
    _close(to_np(dx), dx_o)
    net.close()


def test_bf16_network_matches_oracle():
    shape = (1250, 256, 2, 625, 300)
    n_in, n_h, n_l, n_out, batch = shape
    net, w, x, t = _setup(shape, 6)
    net.set_compute("bf16")
    xd = torch.tensor(x.reshape(-1), device=DEV)
    td = torch.tensor(t.reshape(-1), device=DEV)
    y = net.forward(w, xd, batch)
    dy = torch.empty_like(y)
    net.mse(y, td, batch * n_out, dy=dy)
    dw = net.backward(w, xd, dy, batch)
    torch.cuda.synchronize()
    sh = (n_in, n_h, n_l, n_out)
    y_o, acts = om.forward(to_np(w), x, sh, bf16=True)
    _close(to_np(y), y_o, 2e-3, 2e-2)
    dw_o, _ = om.backward(to_np(w), acts, to_np(dy).reshape(batch, n_out), sh, bf16=True)
    for off, fi, fo, bo in om.layout(*sh)[0]:
        _close(to_np(dw)[off:off + fi * fo], dw_o[off:off + fi * fo], 2e-3, 2e-2)
        _close(to_np(dw)[bo:bo + fo], dw_o[bo:bo + fo], 2e-3, 2e-2)
    # switching back gives the FP32 products again
    net.set_compute("fp32")
    y32 = net.forward(w, xd, batch)
    y_32o, _ = om.forward(to_np(w), x, sh)
    _close(to_np(y32), y_32o)
    with pytest.raises(ScdgError):
        net._ok(net.lib.scdg_mlp_set_compute(net.handle, 2), "scdg_mlp_set_compute")
    net.close()


def test_bf16_training_reduces_loss_like_fp32():
    rng = np.random.default_rng(8)
    n_in, n_out, batch = 40, 20, 256
    x = rng.standard_normal((batch, n_in)).astype(np.float32)
    proj = rng.standard_normal((n_in, n_out)) / np.sqrt(n_in)
    t = np.tanh(x @ proj).astype(np.float32)
    xd, td = torch.tensor(x.reshape(-1), device=DEV), torch.tensor(t.reshape(-1), device=DEV)
    final = {}
    for mode in ("fp32", "bf16"):
        net = Mlp(n_in, 64, 2, n_out, max_batch=batch)
        net.set_compute(mode)
        w = net.init_params(9, DEV)
        m1, m2 = torch.zeros_like(w), torch.zeros_like(w)
        losses = []
        for step in range(1, 301):
            y = net.forward(w, xd, batch)
            dy = torch.empty_like(y)
            losses.append(float(net.mse(y, td, batch * n_out, dy=dy)))
            dw = net.backward(w, xd, dy, batch)
            net.adam(w, dw, m1, m2, 3e-3, step)
        final[mode] = (losses[0], losses[-1])
        net.close()
    print("training losses", final, flush=True)
    for first, last in final.values():
        assert last < 0.1 * first
    assert final["bf16"][1] < 2.0 * final["fp32"][1] + 1e-3
