"""Training and evaluation of the learned initial guess (UNet) on the GPU.

Training pairs come from the method itself: a snapshot is deposited
(cgd_deposit) and then diffused one backward-Euler pseudo-step at a time
(cgd_diffuse with one step of pseudo-time dtau = T / n_steps, i.e. bandwidth
b / sqrt(n_steps)), which yields e^0, e^1, ..., e^n; the network learns
e^n -> e^{n+1} (cgd_unet_train_step).  Everything runs in the library's
kernels; this module only sequences the calls.
"""
from __future__ import annotations

import math
import time

from . import HexMesh, UNet, deposit, diffuse, coarse_grain


def step_fields(mesh: HexMesh, pos, values, bandwidth, n_steps, rtol=1e-7):
    """[e^0, ..., e^n] of one snapshot (single field), float32 [cells] each."""
    field = deposit(mesh, pos, values)
    out = [field[0].clone()]
    b1 = bandwidth / math.sqrt(n_steps)
    for _ in range(n_steps):
        diffuse(mesh, field, b1, 1, rtol=rtol)
        out.append(field[0].clone())
    return out


def train(net: UNet, mesh: HexMesh, snapshots, n_snapshots, bandwidth, n_steps, lr=1e-3, lr_final=1e-4,
          rtol=1e-7, log_every=0, log=print):
    """Adam on the pairs of n_snapshots consecutive snapshots (advancing the
    sequence), learning rate decayed geometrically from lr to lr_final.
    Returns the losses that were read back (every log_every pairs, and the last)."""
    total = n_snapshots * n_steps
    losses = []
    k = 0
    for j in range(n_snapshots):
        pos, vals = snapshots.current()
        fields = step_fields(mesh, pos, vals, bandwidth, n_steps, rtol)
        for n in range(n_steps):
            rate = lr * (lr_final / lr) ** (k / max(1, total - 1))
            read = (log_every and k % log_every == 0) or k == total - 1
            loss = net.train_step(fields[n], fields[n + 1], rate, sync=bool(read))
            if read:
                losses.append((k, loss))
                if log_every and log:
                    log(f"[train] pair {k}/{total} loss {loss:.4e} lr {rate:.2e}")
            k += 1
        snapshots.advance()
    return losses


def evaluate(mesh: HexMesh, net: UNet, snapshots, n_snapshots, bandwidth, n_steps, rtol=1e-6,
             cases=((0, 0), (1, 0), (3, 0)), keep_fields=None):
    """Coarse-grains n_snapshots consecutive snapshots once per case
    (x0_mode, precond): x0_mode 0 zero guess, 1 previous step, 3 network;
    precond 0 polynomial-preconditioned CG, 1 plain CG.  Returns, per case,
    the CG iterations per step summed over snapshots, the wall time in ms
    (whole cgd_coarse_grain calls, synchronised), the fallbacks and the
    fields of the first keep_fields snapshots (all if None)."""
    import torch
    res = {c: {"iters": [0] * n_steps, "ms": 0.0, "fallbacks": 0, "fields": []} for c in cases}
    for j in range(n_snapshots):
        pos, vals = snapshots.current()
        for c in cases:
            m, pc = c
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f, st = coarse_grain(mesh, pos, vals, bandwidth, n_steps, rtol=rtol, x0_mode=m, stats=True,
                                 model=net if m == 3 else None, precond=pc)
            torch.cuda.synchronize()
            r = res[c]
            r["ms"] += 1e3 * (time.perf_counter() - t0)
            for s in range(n_steps):
                r["iters"][s] += st.iters[s][0]
            r["fallbacks"] += st.n_fallback
            if keep_fields is None or j < keep_fields:
                r["fields"].append(f[0].clone())
        snapshots.advance()
    return res
