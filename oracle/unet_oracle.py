"""CPU float64 oracle of the learned warm start's network pieces.

TEST INFRASTRUCTURE ONLY (same rule as cgd_oracle.py: only the tests, the
smoke check and the benchmark's CPU leg use it; it shares no code with the
HIP library).

The warm start is not part of the paper: the network approximates one
backward-Euler pseudo-step of the method, e^{n+1} ~ f(e^n), and its output
seeds the CG solve of that step.  This module holds the definitions the GPU
kernels are checked against:

- 3x3x3 cross-correlation with zero padding, channels last:
  out[z,y,x,o] = b[o] + sum_{dz,dy,dx,i} in[z+dz, y+dy, x+dx, i] w[o, t, i],
  t = (dz+1)*9 + (dy+1)*3 + (dx+1); and its two gradients
  d_in[v, i] = sum_{t,o} d_out[v - off(t), o] w[o, t, i],
  d_w[o, t, i] = sum_v d_out[v, o] in[v + off(t), i], d_b[o] = sum_v d_out[v, o];
- 2x2x2 average pooling, nearest 2x upsampling, channel concatenation, the
  1x1x1 head and ReLU;
- the whole 3-level U-Net (16/32/64 channels) with the residual output
  y = x + head(...), written layer by layer;
- one step of the Adam optimiser (Kingma and Ba, "Adam: a method for
  stochastic optimization", ICLR 2015, Algorithm 1), which trains it.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def conv3_fwd(x, w, b=None):
    """x [D,H,W,Ci], w [Co,27,Ci], b [Co] -> [D,H,W,Co] (float64)."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    D, H, W, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    out = np.zeros((D, H, W, w.shape[0]))
    for t, (dz, dy, dx) in enumerate(TAPS):
        sl = xp[1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :]
        out += sl @ w[:, t, :].T
    if b is not None:
        out += np.asarray(b, dtype=np.float64)
    return out


def conv3_dgrad(dout, w):
    """Gradient of conv3_fwd with respect to its input."""
    dout = np.asarray(dout, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    D, H, W, _ = dout.shape
    dxp = np.zeros((D + 2, H + 2, W + 2, w.shape[2]))
    for t, (dz, dy, dx) in enumerate(TAPS):
        dxp[1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :] += dout @ w[:, t, :]
    return dxp[1:-1, 1:-1, 1:-1, :]


def conv3_wgrad(x, dout):
    """Gradients of conv3_fwd with respect to w [Co,27,Ci] and b [Co]."""
    x = np.asarray(x, dtype=np.float64)
    dout = np.asarray(dout, dtype=np.float64)
    D, H, W, Ci = x.shape
    Co = dout.shape[3]
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    g = dout.reshape(-1, Co)
    dw = np.zeros((Co, 27, Ci))
    for t, (dz, dy, dx) in enumerate(TAPS):
        sl = xp[1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :].reshape(-1, Ci)
        dw[:, t, :] = g.T @ sl
    return dw, g.sum(axis=0)


def avgpool2(x):
    D, H, W, C = x.shape
    return x.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(1, 3, 5))


def avgpool2_bwd(dout):
    return np.repeat(np.repeat(np.repeat(dout, 2, 0), 2, 1), 2, 2) / 8.0


def up2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 0), 2, 1), 2, 2)


def up2_bwd(dout):
    D, H, W, C = dout.shape
    return dout.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(1, 3, 5))


def relu(x):
    return np.maximum(x, 0.0)


# The network: names of the parameter tensors, in order, with their shapes.
def unet_layers(c=16):
    """(name, c_in, c_out) of the 3x3x3 convolutions, then the 1x1x1 head."""
    return [("e1a", 1, c), ("e1b", c, c), ("e2a", c, 2 * c), ("e2b", 2 * c, 2 * c),
            ("e3a", 2 * c, 4 * c), ("e3b", 4 * c, 4 * c), ("u2", 4 * c, 2 * c),
            ("d2a", 4 * c, 2 * c), ("d2b", 2 * c, 2 * c), ("u1", 2 * c, c),
            ("d1a", 2 * c, c), ("d1b", c, c)]


def _same(a):
    return a


def unet_forward(x, params, c=16, x_res=None, rnd=_same):
    """x [D,H,W,1] -> y [D,H,W,1] = x + head(U(x)).  params: name -> (w, b),
    with w [Co,27,Ci] for the 3x3x3 layers and w [1,Ci] for 'head'.
    x_res, when given, replaces x as the residual term (y = x_res + head(U(x))).
    rnd: applied to every stored intermediate tensor (layer outputs and
    pooled tensors); the identity by default, a rounding function to model
    an implementation that stores them at reduced precision."""
    P = params
    L = lambda name, t: rnd(relu(conv3_fwd(t, *P[name])))
    pool = lambda t: rnd(avgpool2(t))
    e1 = L("e1b", L("e1a", x))
    e2 = L("e2b", L("e2a", pool(e1)))
    e3 = L("e3b", L("e3a", pool(e2)))
    u2 = L("u2", up2(e3))
    d2 = L("d2b", L("d2a", np.concatenate([u2, e2], axis=3)))
    u1 = L("u1", up2(d2))
    d1 = L("d1b", L("d1a", np.concatenate([u1, e1], axis=3)))
    hw, hb = P["head"]
    base = x if x_res is None else np.asarray(x_res, dtype=np.float64)
    return base + (d1 @ np.asarray(hw, dtype=np.float64).T + hb)


def head_fwd(d1, hw, hb):
    """1x1x1 head: d1 [D,H,W,C], hw [1,C] or [C], hb scalar -> [D,H,W,1]."""
    hw = np.asarray(hw, dtype=np.float64).reshape(1, -1)
    return d1 @ hw.T + np.asarray(hb, dtype=np.float64).reshape(1)


def unet_loss_and_grads(x, target, params, c=16, x_res=None, rnd=_same):
    """Mean-squared error of the residual U-Net against `target` and its
    gradients with respect to every parameter, by reverse-mode chain rule
    through the layers of unet_forward (written out one layer at a time).

    x, target: [D,H,W,1]; x_res and rnd as in unet_forward (rnd also applies
    to every stored gradient tensor: each layer's gradient at its output
    before the convolution, and each input gradient).  Returns (loss, grads)
    with grads[name] = (dw, db) in the shapes of params[name]."""
    P = params
    x = np.asarray(x, dtype=np.float64)
    conv = lambda name, t: rnd(relu(conv3_fwd(t, *P[name])))
    # forward, keeping every activation
    a1 = conv("e1a", x)
    e1 = conv("e1b", a1)
    p1 = rnd(avgpool2(e1))
    a2 = conv("e2a", p1)
    e2 = conv("e2b", a2)
    p2 = rnd(avgpool2(e2))
    a3 = conv("e3a", p2)
    e3 = conv("e3b", a3)
    q3 = up2(e3)
    u2 = conv("u2", q3)
    c2 = np.concatenate([u2, e2], axis=3)
    a4 = conv("d2a", c2)
    d2 = conv("d2b", a4)
    q2 = up2(d2)
    u1 = conv("u1", q2)
    c1 = np.concatenate([u1, e1], axis=3)
    a5 = conv("d1a", c1)
    d1 = conv("d1b", a5)
    hw, hb = P["head"]
    y = (x if x_res is None else np.asarray(x_res, dtype=np.float64)) + head_fwd(d1, hw, hb)
    diff = y - np.asarray(target, dtype=np.float64)
    n = diff.size
    loss = float((diff ** 2).sum() / n)

    G = {}
    g_y = 2.0 * diff / n                                   # dL/dy  [.., 1]
    G["head"] = ((g_y.reshape(-1, 1) * d1.reshape(-1, d1.shape[3])).sum(0).reshape(np.shape(hw)),
                 np.asarray(g_y.sum()).reshape(np.shape(hb)))
    g = g_y @ np.asarray(hw, dtype=np.float64).reshape(1, -1)   # dL/d d1

    def back(name, t_in, t_out, g_out):
        """Through relu(conv(name, t_in)) = t_out: records the parameter
        gradients and returns dL/d t_in."""
        g_pre = rnd(g_out * (t_out > 0))
        dw, db = conv3_wgrad(t_in, g_pre)
        G[name] = (dw, db)
        return rnd(conv3_dgrad(g_pre, P[name][0]))

    g = back("d1b", a5, d1, g)
    g = back("d1a", c1, a5, g)
    g_u1, g_e1 = g[..., :u1.shape[3]], g[..., u1.shape[3]:]
    g = back("u1", q2, u1, g_u1)
    g = up2_bwd(g)                                          # dL/d d2
    g = back("d2b", a4, d2, g)
    g = back("d2a", c2, a4, g)
    g_u2, g_e2 = g[..., :u2.shape[3]], g[..., u2.shape[3]:]
    g = back("u2", q3, u2, g_u2)
    g = up2_bwd(g)                                          # dL/d e3
    g = back("e3b", a3, e3, g)
    g = back("e3a", p2, a3, g)
    g = g_e2 + avgpool2_bwd(g)                              # dL/d e2 (skip + pool)
    g = back("e2b", a2, e2, g)
    g = back("e2a", p1, a2, g)
    g = g_e1 + avgpool2_bwd(g)                              # dL/d e1
    g = back("e1b", a1, e1, g)
    back("e1a", x, a1, g)
    return loss, G


def init_params(rng, c=16):
    """He-normal 3x3x3 weights, zero biases, zero head (so the untrained net
    is the identity map x -> x)."""
    P = {}
    for name, ci, co in unet_layers(c):
        P[name] = (rng.standard_normal((co, 27, ci)) * np.sqrt(2.0 / (27 * ci)), np.zeros(co))
    P["head"] = (np.zeros((1, c)), np.zeros(1))
    return P


def flatten_params(P, c=16):
    """Parameters in the library's flat order: per layer w [Co,27,Ci] then b,
    then the head's w [C] and b."""
    parts = []
    for name, _, _ in unet_layers(c):
        parts += [np.ravel(P[name][0]), np.ravel(P[name][1])]
    parts += [np.ravel(P["head"][0]), np.ravel(P["head"][1])]
    return np.concatenate(parts)


def unflatten_params(v, c=16):
    v = np.asarray(v, dtype=np.float64)
    P, o = {}, 0
    for name, ci, co in unet_layers(c):
        w = v[o:o + co * 27 * ci].reshape(co, 27, ci)
        o += co * 27 * ci
        P[name] = (w, v[o:o + co])
        o += co
    P["head"] = (v[o:o + c].reshape(1, c), v[o + c:o + c + 1])
    assert o + c + 1 == v.size
    return P


def bf16_round(a):
    """Round float32 values to bfloat16 (8 significand bits), to nearest with
    ties to even, returned as float32.  Finite inputs only."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).reshape(np.shape(a))


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Step t (1, 2, ...) of Adam, Kingma and Ba (2015), Algorithm 1, in float64.

    m <- beta1 m + (1 - beta1) g;  v <- beta2 v + (1 - beta2) g^2;
    m_hat = m / (1 - beta1^t);  v_hat = v / (1 - beta2^t);
    params <- params - lr m_hat / (sqrt(v_hat) + eps).
    Returns (params, m, v) as new arrays.
    """
    g = np.asarray(grads, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    p = np.asarray(params, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps)
    return p, m, v
