"""Plain FP64 reference of the learned-initial-guess network (test oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper has no learned component; this is the reference for an addition to
its Newton-Krylov loop (Section 2.2): a per-element multilayer perceptron
that predicts the Newton increment of the next implicit step from the
element's state and its previous increment.

Network: a_0 = x, a_l = tanh(a_{l-1} W_l + b_l) for the hidden layers,
y = a_L W_out + b_out (rows are samples).  Parameters live in one flat
vector, layer after layer, W_l [fan_in x fan_out] row-major then b_l.
Gradients follow the chain rule written out per layer; Adam is the update of
Kingma and Ba (2015) with bias correction.  The BF16 compute mode rounds both
operands of every matrix product to bfloat16 (a storage format with FP32's
exponent range and an 8-bit significand); everything else stays exact.
"""
from __future__ import annotations

import numpy as np


def layout(n_in: int, n_hidden: int, n_layers: int, n_out: int):
    """[(w_offset, fan_in, fan_out, b_offset)] per layer and the parameter count."""
    out, off = [], 0
    for layer in range(n_layers + 1):
        fi = n_in if layer == 0 else n_hidden
        fo = n_out if layer == n_layers else n_hidden
        out.append((off, fi, fo, off + fi * fo))
        off += fi * fo + fo
    return out, off


def _unpack(w, shape):
    lay, n = layout(*shape)
    assert w.size == n
    return [(w[o:o + fi * fo].reshape(fi, fo), w[bo:bo + fo]) for o, fi, fo, bo in lay]


def bf16_round(a) -> np.ndarray:
    """Nearest bfloat16 of each value taken as FP32 (ties to even), as FP64.

    bfloat16 keeps the sign, the 8 exponent bits and the 7 leading mantissa
    bits of an FP32 number; rounding to nearest-even adds 0x7FFF plus the
    lowest kept bit to the FP32 bit pattern and clears the 16 dropped bits
    (finite inputs)."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _operand(bf16: bool):
    """How a matrix-product operand enters: as is (FP64), or as the nearest
    bfloat16 of its FP32 value (the BF16 compute mode)."""
    return bf16_round if bf16 else (lambda t: t)


def forward(w: np.ndarray, x: np.ndarray, shape, bf16: bool = False):
    """y and the list of activations a_0 = x, a_1, ..., a_L (FP64).  bf16: both
    operands of every product rounded to bfloat16, the rest in FP64."""
    layers = _unpack(np.asarray(w, dtype=np.float64), shape)
    op = _operand(bf16)
    a = [np.asarray(x, dtype=np.float64)]
    for i, (wl, bl) in enumerate(layers):
        z = op(a[-1]) @ op(wl) + bl
        if i < len(layers) - 1:
            a.append(np.tanh(z))
        else:
            return z, a
    raise AssertionError("unreachable")


def backward(w: np.ndarray, acts, dy: np.ndarray, shape, bf16: bool = False):
    """dLoss/dw (flat) and dLoss/dx given dLoss/dy and the forward activations
    (bf16: product operands rounded as in forward)."""
    layers = _unpack(np.asarray(w, dtype=np.float64), shape)
    op = _operand(bf16)
    lay, n = layout(*shape)
    dw = np.zeros(n)
    dz = np.asarray(dy, dtype=np.float64)
    for i in range(len(layers) - 1, -1, -1):
        wl, _ = layers[i]
        o, fi, fo, bo = lay[i]
        dw[o:o + fi * fo] = (op(acts[i]).T @ op(dz)).reshape(-1)
        dw[bo:bo + fo] = dz.sum(axis=0)
        da = op(dz) @ op(wl).T              # dLoss / d a_{i}
        if i > 0:
            dz = da * (1.0 - acts[i] ** 2)  # through a_i = tanh(z_i)
        else:
            dx = da
    return dw, dx


def mse(y: np.ndarray, t: np.ndarray):
    """mean((y - t)^2) and its gradient 2 (y - t) / n."""
    d = np.asarray(y, dtype=np.float64) - np.asarray(t, dtype=np.float64)
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam(w, g, m1, m2, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step; returns new (w, m1, m2)."""
    w, g, m1, m2 = (np.asarray(a, dtype=np.float64) for a in (w, g, m1, m2))
    m1 = beta1 * m1 + (1.0 - beta1) * g
    m2 = beta2 * m2 + (1.0 - beta2) * g * g
    mhat = m1 / (1.0 - beta1 ** step)
    vhat = m2 / (1.0 - beta2 ** step)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m1, m2


# --------------------------------------------------------------------------
# maps between DG vectors (natural DOF order, 5 variables per node) and the
# network's features and targets
# --------------------------------------------------------------------------

def field_stats(q: np.ndarray, dq_prev: np.ndarray, dq: np.ndarray | None = None,
                r: np.ndarray | None = None):
    """Per-variable mean and population standard deviation of q, root mean
    square rp of dq_prev, rc of dq - dq_prev (rc = rp without dq) and rr of the
    residual r (1 without r) over all nodes; a zero spread becomes 1."""
    qv = np.asarray(q, dtype=np.float64).reshape(-1, 5)
    dv = np.asarray(dq_prev, dtype=np.float64).reshape(-1, 5)
    mean = qv.mean(axis=0)
    std = qv.std(axis=0)
    std = np.where((std > 0) & (std > 1e-12 * np.abs(mean)), std, 1.0)
    rms = np.sqrt((dv * dv).mean(axis=0))
    rms = np.where(rms > 0, rms, 1.0)
    if dq is None:
        rc = rms.copy()
    else:
        cv = np.asarray(dq, dtype=np.float64).reshape(-1, 5) - dv
        rc = np.sqrt((cv * cv).mean(axis=0))
        rc = np.where(rc > 0, rc, 1.0)
    if r is None:
        rr = np.ones(5)
    else:
        rv = np.asarray(r, dtype=np.float64).reshape(-1, 5)
        rr = np.sqrt((rv * rv).mean(axis=0))
        rr = np.where(rr > 0, rr, 1.0)
    return mean, std, rms, rc, rr


def features(q, dq_prev, stats, n_elem: int, r=None):
    """Rows [ (Q_e - mean) / std , dQprev_e / rp ( , R_e / rr ) ] per element
    (the residual block when r is given)."""
    mean, std, rms, _, rr = stats
    qv = np.asarray(q, dtype=np.float64).reshape(n_elem, -1, 5)
    dv = np.asarray(dq_prev, dtype=np.float64).reshape(n_elem, -1, 5)
    blocks = [((qv - mean) / std).reshape(n_elem, -1), (dv / rms).reshape(n_elem, -1)]
    if r is not None:
        blocks.append((np.asarray(r, dtype=np.float64).reshape(n_elem, -1, 5) / rr).reshape(n_elem, -1))
    return np.concatenate(blocks, axis=1)


def target(dq, dq_prev, stats, n_elem: int):
    """(dQ_e - dQprev_e) / rc: the correction to the previous increment."""
    rms = stats[3]
    d = (np.asarray(dq, dtype=np.float64) - np.asarray(dq_prev, dtype=np.float64)).reshape(n_elem, -1, 5)
    return (d / rms).reshape(n_elem, -1)


def apply(dq_prev, y, stats, n_elem: int):
    """dQprev_e + rc y_e."""
    rms = stats[3]
    dv = np.asarray(dq_prev, dtype=np.float64).reshape(n_elem, -1, 5)
    return (dv + rms * np.asarray(y, dtype=np.float64).reshape(n_elem, -1, 5)).reshape(-1)


# --------------------------------------------------------------------------
# condensed-residual loss of a predicted increment
# --------------------------------------------------------------------------

def condensed_loss(s: np.ndarray, bnode_dofs: np.ndarray, y, t, rc):
    """||S P_b (rc (y - t))||^2 and its gradient with respect to y.

    A guess x0 for the condensed system S Q_b = b_S (eq. SC_step1) starts GMRES
    at the residual b_S - S x0_b = S (Q_b - x0_b): the error of the guess's
    boundary part weighted by S.  y and t are the network's normalised output
    and target as natural vectors (variable fastest), rc the five scales that
    map them back (target: (dQ - dQprev) / rc), s the dense condensed matrix in
    the boundary-vector order and bnode_dofs[node, v] (dof_maps) the natural
    index of each boundary slot.  The gradient is the chain rule written out:
    2 rc P_b^T S^T S e, zero on interior DOFs."""
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    t = np.asarray(t, dtype=np.float64).reshape(-1)
    w = np.tile(np.asarray(rc, dtype=np.float64), y.size // 5)
    idx = np.asarray(bnode_dofs, dtype=np.int64).reshape(-1)
    e = (w * (y - t))[idx]
    r = np.asarray(s, dtype=np.float64) @ e
    g = np.zeros_like(y)
    g[idx] = 2.0 * (np.asarray(s, dtype=np.float64).T @ r)
    return float(r @ r), w * g
