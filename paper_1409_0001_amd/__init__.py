"""MI355X-native diffusion-based coarse graining (Sun & Xiao).

Thin Python binding over the libcgd C-ABI (include/cgd.h).  It only checks
and marshals arguments: every step of the method runs in the library's HIP
kernels.  torch tensors provide device memory and the current stream.

    import paper_1409_0001_amd as cgd
    mesh = cgd.HexMesh((256, 256, 512), lo=(0, 0, 0), hi=(1, 1, 2))
    field, stats = cgd.coarse_grain(mesh, pos, values, bandwidth=4/256, n_steps=4)

There is no CPU fallback: the calls raise if libcgd.so is missing or no GPU
is visible.
"""
from __future__ import annotations

import ctypes
import dataclasses

from . import _abi

load = _abi.load


class CgdError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = _abi.load()
        name = lib.cgd_status_string(status).decode()
        msg = lib.cgd_last_error().decode()
        super().__init__(f"{where}: {name} ({status}): {msg}")
        self.status = status


@dataclasses.dataclass
class Stats:
    status: int
    iters: list           # [n_steps][F]
    rel_res: list         # [n_steps][F]
    mass_before: list     # [F]
    mass_after: list      # [F]
    frac_bits: list       # [F]
    n_dropped: int
    n_nonfinite: int
    n_fallback: int = 0   # x0_mode 3: solves whose learned guess was rejected


def _stats(st: _abi.SolveStats, F: int, n_steps: int, status: int) -> Stats:
    return Stats(status=status, n_fallback=int(st.n_fallback),
                 iters=[[st.iters[s][f] for f in range(F)] for s in range(n_steps)],
                 rel_res=[[st.rel_res[s][f] for f in range(F)] for s in range(n_steps)],
                 mass_before=[st.mass_before[f] for f in range(F)],
                 mass_after=[st.mass_after[f] for f in range(F)],
                 frac_bits=[st.frac_bits[f] for f in range(F)],
                 n_dropped=int(st.n_dropped), n_nonfinite=int(st.n_nonfinite))


def _check(status: int, where: str, allow=(_abi.OK, _abi.NOT_CONVERGED, _abi.WARMSTART_FALLBACK)):
    if status not in allow:
        raise CgdError(status, where)
    return status


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("paper_1409_0001_amd needs a visible HIP GPU (no CPU fallback)")
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype, shape, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor on the GPU")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Mesh:
    """Owner of a cgd_mesh handle (device topology + workspace)."""

    def __init__(self, handle):
        self._h = handle
        lib = _abi.load()
        self.cells = int(lib.cgd_mesh_num_cells(handle))
        self.kind = int(lib.cgd_mesh_kind(handle))

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            _abi.load().cgd_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HexMesh(Mesh):
    """Uniform hex mesh of the box [lo, hi] with shape = (nx, ny, nz) cells."""

    def __init__(self, shape, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
        _torch()
        lib = _abi.load()
        lo_a = (ctypes.c_double * 3)(*[float(v) for v in lo])
        hi_a = (ctypes.c_double * 3)(*[float(v) for v in hi])
        h = _abi.c_mesh()
        _check(lib.cgd_mesh_create_hex(int(shape[0]), int(shape[1]), int(shape[2]), lo_a, hi_a,
                                       ctypes.byref(h)), "cgd_mesh_create_hex", allow=(0,))
        self.shape = tuple(int(s) for s in shape)
        self.lo = tuple(float(v) for v in lo)
        self.hi = tuple(float(v) for v in hi)
        super().__init__(h)


class TetMesh(Mesh):
    """Tetrahedral mesh from host arrays xyz float64 [V, 3] and tets int32
    [T, 4], with an optional cell-wise diffusivity (float32 [T], >= 0; None:
    1 everywhere)."""

    def __init__(self, xyz, tets, diffusivity=None):
        import numpy as np
        _torch()
        lib = _abi.load()
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        if xyz.ndim != 2 or xyz.shape[1] != 3 or tets.ndim != 2 or tets.shape[1] != 4:
            raise ValueError("xyz must be [V, 3] and tets [T, 4]")
        h = _abi.c_mesh()
        if diffusivity is None:
            _check(lib.cgd_mesh_create_tet(xyz.shape[0], xyz.ctypes.data, tets.shape[0], tets.ctypes.data,
                                           ctypes.byref(h)), "cgd_mesh_create_tet", allow=(0,))
        else:
            d = np.ascontiguousarray(diffusivity, dtype=np.float32).ravel()
            if d.shape[0] != tets.shape[0]:
                raise ValueError("diffusivity must have one value per tet")
            _check(lib.cgd_mesh_create_tet_d(xyz.shape[0], xyz.ctypes.data, tets.shape[0], tets.ctypes.data,
                                             d.ctypes.data, ctypes.byref(h)), "cgd_mesh_create_tet_d", allow=(0,))
        super().__init__(h)
        self.nnz = int(lib.cgd_mesh_nnz(h))


class RectMesh(Mesh):
    """Stretched (rectilinear) hex mesh from its node coordinates per axis
    (float64, strictly increasing) and an optional cell-wise diffusivity
    (float32 [nz * ny * nx], x fastest; None: 1 everywhere).  periodic:
    three booleans, one per axis (Section 3.1)."""

    def __init__(self, x_edges, y_edges, z_edges, diffusivity=None, periodic=(False, False, False)):
        import numpy as np
        _torch()
        lib = _abi.load()
        e = [np.ascontiguousarray(v, dtype=np.float64) for v in (x_edges, y_edges, z_edges)]
        if any(v.ndim != 1 or v.size < 2 for v in e):
            raise ValueError("edges must be 1-D with at least two nodes each")
        n = [v.size - 1 for v in e]
        d = None
        if diffusivity is not None:
            d = np.ascontiguousarray(diffusivity, dtype=np.float32).ravel()
            if d.size != n[0] * n[1] * n[2]:
                raise ValueError("diffusivity must hold one value per cell")
        h = _abi.c_mesh()
        _check(lib.cgd_mesh_create_rect(n[0], n[1], n[2], e[0].ctypes.data, e[1].ctypes.data, e[2].ctypes.data,
                                        d.ctypes.data if d is not None else None,
                                        sum(1 << a for a in range(3) if periodic[a]), ctypes.byref(h)),
               "cgd_mesh_create_rect", allow=(0,))
        super().__init__(h)
        self.shape = tuple(n)
        self.nnz = int(lib.cgd_mesh_nnz(h))


_SCHEMES = {"be": 0, "cn": 1}


def _opts(rtol, max_iter, x0_mode, x0, check_every, model=None, precond=0, scheme="be"):
    o = _abi.SolverOpts()
    if scheme not in _SCHEMES:
        raise ValueError(f"scheme must be 'be' (backward Euler) or 'cn' (Crank-Nicolson), not {scheme!r}")
    o.scheme = _SCHEMES[scheme]
    o.precond = int(precond)
    o.rtol = float(rtol)
    o.max_iter = int(max_iter)
    o.x0_mode = int(x0_mode)
    o.x0 = x0.data_ptr() if x0 is not None else None
    o.check_every = int(check_every)
    o.model = model.handle if model is not None else None
    return o


def velocity_from_momentum(eps, mom, eps_min=1e-6, stream=None):
    """Momentum-consistent velocity (Section 6: diffuse the momentum, not the
    velocity): mom [n_comp, cells] (diffused eps U) becomes U = mom / eps
    where eps [cells] > eps_min, 0 elsewhere, in place.  Returns mom."""
    torch = _torch()
    lib = _abi.load()
    cells = int(eps.shape[-1])
    p_eps = _dev(eps, torch.float32, (cells,), "eps")
    p_mom = _dev(mom, torch.float32, (int(mom.shape[0]), cells), "mom")
    _check(lib.cgd_velocity_from_momentum(cells, int(mom.shape[0]), p_eps, p_mom, float(eps_min),
                                          _stream_ptr(stream)), "cgd_velocity_from_momentum")
    return mom


def locate(mesh: Mesh, pos, cell=None, stream=None):
    """Host cell of each particle centroid (int32 [N]; -1 when dropped)."""
    torch = _torch()
    n = int(pos.shape[0])
    p_pos = _dev(pos, torch.float32, (n, 3), "pos")
    if cell is None:
        cell = torch.empty((n,), dtype=torch.int32, device=pos.device)
    p_cell = _dev(cell, torch.int32, (n,), "cell")
    _check(_abi.load().cgd_locate(mesh.handle, n, p_pos, p_cell, _stream_ptr(stream)), "cgd_locate",
           allow=(0,))
    return cell


def deposit(mesh: Mesh, pos, values, field=None, acc=None, stats=False, stream=None, frac_bits=None):
    """Particle centroid method (bit-exact).  pos [N, 3] f32, values [F, N] f32.

    frac_bits: None (automatic fixed-point scales) or a list of F ints, -1 for
    automatic or a scale 0..62 to force; a list is overwritten with the
    scales used.  Returns field [F, cells] (and Stats when stats=True, which
    synchronises)."""
    torch = _torch()
    lib = _abi.load()
    n = int(pos.shape[0])
    F = int(values.shape[0])
    p_pos = _dev(pos, torch.float32, (n, 3), "pos")
    p_val = _dev(values, torch.float32, (F, n), "values")
    if field is None:
        field = torch.empty((F, mesh.cells), dtype=torch.float32, device=pos.device)
    p_field = _dev(field, torch.float32, (F, mesh.cells), "field")
    p_acc = _dev(acc, torch.int64, (F, mesh.cells), "acc") if acc is not None else None
    fb = None
    if frac_bits is not None:
        if len(frac_bits) != F:
            raise ValueError(f"frac_bits needs {F} entries")
        fb = (ctypes.c_int32 * F)(*[int(v) for v in frac_bits])
    st = _abi.SolveStats() if stats else None
    rc = lib.cgd_deposit(mesh.handle, n, p_pos, F, p_val, p_field, p_acc, fb,
                         ctypes.byref(st) if st is not None else None, _stream_ptr(stream))
    if fb is not None and rc >= 0 and isinstance(frac_bits, list):
        frac_bits[:] = list(fb)
    _check(rc, "cgd_deposit", allow=(0,) if not stats else (0, _abi.E_NONFINITE))
    if stats:
        return field, _stats(st, F, 0, rc)
    return field


def diffuse(mesh: Mesh, field, bandwidth, n_steps, rtol=1e-6, max_iter=1000, x0_mode=0, x0=None,
            check_every=4, stats=False, stream=None, model=None, precond=0, scheme="be"):
    """Diffuses field [F, cells] in place for T = bandwidth^2 / 4 in n_steps
    backward-Euler ("be") or Crank-Nicolson ("cn") steps.  x0_mode 3 seeds
    every step with model(e^n) (a UNet made for this mesh's grid).  Returns
    (field, Stats or None)."""
    torch = _torch()
    lib = _abi.load()
    F = int(field.shape[0])
    p_field = _dev(field, torch.float32, (F, mesh.cells), "field")
    if x0 is not None:
        _dev(x0, torch.float32, (F, mesh.cells), "x0")
    o = _opts(rtol, max_iter, x0_mode, x0, check_every, model, precond, scheme)
    st = _abi.SolveStats() if stats else None
    rc = lib.cgd_diffuse(mesh.handle, F, p_field, float(bandwidth), int(n_steps), ctypes.byref(o),
                         ctypes.byref(st) if st is not None else None, _stream_ptr(stream))
    _check(rc, "cgd_diffuse")
    return field, (_stats(st, F, n_steps, rc) if stats else None)


def coarse_grain(mesh: Mesh, pos, values, bandwidth, n_steps, rtol=1e-6, max_iter=1000, x0_mode=0,
                 check_every=4, field=None, stats=False, stream=None, model=None, precond=0, scheme="be"):
    """The whole method (Section 2.6): PCM deposition, then diffusion.
    Returns (field [F, cells], Stats or None)."""
    torch = _torch()
    lib = _abi.load()
    n = int(pos.shape[0])
    F = int(values.shape[0])
    p_pos = _dev(pos, torch.float32, (n, 3), "pos")
    p_val = _dev(values, torch.float32, (F, n), "values")
    if field is None:
        field = torch.empty((F, mesh.cells), dtype=torch.float32, device=pos.device)
    p_field = _dev(field, torch.float32, (F, mesh.cells), "field")
    o = _opts(rtol, max_iter, x0_mode, None, check_every, model, precond, scheme)
    st = _abi.SolveStats() if stats else None
    rc = lib.cgd_coarse_grain(mesh.handle, n, p_pos, F, p_val, float(bandwidth), int(n_steps),
                              ctypes.byref(o), p_field, ctypes.byref(st) if st is not None else None,
                              _stream_ptr(stream))
    _check(rc, "cgd_coarse_grain")
    return field, (_stats(st, F, n_steps, rc) if stats else None)


def coarse_grain_batched(mesh: HexMesh, offsets, pos, values, bandwidth, n_steps, rtol=1e-6, max_iter=1000,
                         fields=None, return_iters=False, stream=None, precond=0, scheme="be", stats=False):
    """All snapshots at once.  offsets: host int64 [S + 1]; pos [N, 3]; values
    [F, N].  Returns fields [S, F, cells], then the iterations [S, F, n_steps]
    when return_iters, then a list of S Stats when stats."""
    import numpy as np
    torch = _torch()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    n_snap = len(off) - 1
    n = int(pos.shape[0])
    F = int(values.shape[0])
    if off[-1] != n:
        raise ValueError("offsets[-1] must equal the number of particles")
    p_pos = _dev(pos, torch.float32, (n, 3), "pos")
    p_val = _dev(values, torch.float32, (F, n), "values")
    if fields is None:
        fields = torch.empty((n_snap, F, mesh.cells), dtype=torch.float32, device=pos.device)
    p_f = _dev(fields, torch.float32, (n_snap, F, mesh.cells), "fields")
    o = _opts(rtol, max_iter, 0, None, 4, precond=precond, scheme=scheme)
    want = return_iters or stats
    st = (_abi.SolveStats * n_snap)() if want else None
    rc = _abi.load().cgd_coarse_grain_batched(mesh.handle, n_snap, off.ctypes.data, p_pos, F, p_val,
                                              float(bandwidth), int(n_steps), ctypes.byref(o), p_f,
                                              st, _stream_ptr(stream))
    # with stats, skipped non-finite particles are reported per snapshot
    _check(rc, "cgd_coarse_grain_batched",
           allow=(_abi.OK, _abi.NOT_CONVERGED, _abi.E_NONFINITE) if stats else (_abi.OK, _abi.NOT_CONVERGED))
    out = [fields]
    if return_iters:
        out.append(np.array([[[st[j].iters[k][f] for k in range(n_steps)] for f in range(F)]
                             for j in range(n_snap)], dtype=np.int32))
    if stats:
        out.append([_stats(st[j], F, n_steps, int(st[j].status)) for j in range(n_snap)])
    return out[0] if len(out) == 1 else tuple(out)


def autotune_batched(mesh: HexMesh, n_rhs: int):
    """Times the batched solver's tile candidates; returns (chosen, [ms per candidate])."""
    _torch()
    ms = (ctypes.c_double * 16)()
    chosen = ctypes.c_int32()
    nc = ctypes.c_int32()
    _check(_abi.load().cgd_autotune_batched(mesh.handle, int(n_rhs), ctypes.byref(chosen), ms,
                                            ctypes.byref(nc)), "cgd_autotune_batched", allow=(0,))
    return chosen.value, [ms[i] for i in range(nc.value)]


TIMING_KINDS = {0: "cg_sweep1", 1: "cg_sweep2", 2: "deposit", 3: "pcg_spmv_sweep", 4: "pcg_update_sweep",
                5: "cg_precond_pass1", 6: "cg_precond_pass_mid", 7: "cg_precond_pass_last",
                8: "cg_first_sweep1", 9: "cg_first_sweep2", 10: "cg_first_precond_pass1",
                11: "cg_first_precond_pass_mid", 12: "cg_first_precond_pass_last",
                13: "deposit_bin", 14: "deposit_scatter", 15: "deposit_accum",
                16: "pcg_poly_pass_bv", 17: "pcg_poly_pass_factor"}


def timing_enable(mesh: Mesh, on: bool = True):
    """Brackets the timed kernels of later calls on this mesh with HIP events."""
    _check(_abi.load().cgd_timing_enable(mesh.handle, int(bool(on))), "cgd_timing_enable", allow=(0,))


def timing_read(mesh: Mesh, reset: bool = False) -> dict:
    """{kind name: (launches, total_ms, algorithmic bytes per launch)}."""
    t = _abi.KernelTiming()
    _check(_abi.load().cgd_timing_read(mesh.handle, ctypes.byref(t), int(bool(reset))),
           "cgd_timing_read", allow=(0,))
    return {name: (int(t.launches[k]), float(t.total_ms[k]), float(t.bytes_per_launch[k]))
            for k, name in TIMING_KINDS.items()}


class UNet:
    """Learned initial guess f(e^n) ~ e^{n+1} for an (nx, ny, nz) hex grid
    (include/cgd.h documents the network).  Parameters and gradients are flat
    float32 numpy arrays in the library's order."""

    def __init__(self, shape, seed=0):
        _torch()
        h = _abi.c_unet()
        _check(_abi.load().cgd_unet_create(int(shape[0]), int(shape[1]), int(shape[2]), int(seed),
                                           ctypes.byref(h)), "cgd_unet_create", allow=(0,))
        self._h = h
        self.shape = tuple(int(v) for v in shape)
        self.cells = self.shape[0] * self.shape[1] * self.shape[2]
        self.n_params = int(_abi.load().cgd_unet_num_params(h))

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            _abi.load().cgd_unet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        import numpy as np
        v = np.empty(self.n_params, dtype=np.float32)
        _check(_abi.load().cgd_unet_get_params(self._h, v.ctypes.data, v.size), "cgd_unet_get_params", allow=(0,))
        return v

    def set_params(self, v):
        import numpy as np
        v = np.ascontiguousarray(v, dtype=np.float32)
        if v.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {v.size}")
        _check(_abi.load().cgd_unet_set_params(self._h, v.ctypes.data, v.size), "cgd_unet_set_params", allow=(0,))

    def get_grads(self):
        import numpy as np
        v = np.empty(self.n_params, dtype=np.float32)
        _check(_abi.load().cgd_unet_get_grads(self._h, v.ctypes.data, v.size), "cgd_unet_get_grads", allow=(0,))
        return v

    def forward(self, x, y=None, stream=None):
        """y = f(x) for one field x: float32 [cells] on the GPU."""
        torch = _torch()
        px = _dev(x, torch.float32, (self.cells,), "x")
        if y is None:
            y = torch.empty_like(x)
        py = _dev(y, torch.float32, (self.cells,), "y")
        _check(_abi.load().cgd_unet_forward(self._h, px, py, _stream_ptr(stream)), "cgd_unet_forward", allow=(0,))
        return y

    def loss_grad(self, x, target, stream=None):
        """Loss (float) and, on the device, its gradient (get_grads copies it)."""
        torch = _torch()
        px = _dev(x, torch.float32, (self.cells,), "x")
        pt = _dev(target, torch.float32, (self.cells,), "target")
        loss = ctypes.c_double()
        _check(_abi.load().cgd_unet_loss_grad(self._h, px, pt, ctypes.byref(loss), _stream_ptr(stream)),
               "cgd_unet_loss_grad", allow=(0,))
        return loss.value

    def train_step(self, x, target, lr, sync=True, stream=None):
        """One Adam step on (x, target); returns the loss before the step when sync."""
        torch = _torch()
        px = _dev(x, torch.float32, (self.cells,), "x")
        pt = _dev(target, torch.float32, (self.cells,), "target")
        loss = ctypes.c_double()
        _check(_abi.load().cgd_unet_train_step(self._h, px, pt, float(lr), ctypes.byref(loss) if sync else None,
                                               _stream_ptr(stream)), "cgd_unet_train_step", allow=(0,))
        return loss.value if sync else None


def _bf16(t, shape, name):
    torch = _torch()
    return _dev(t, torch.bfloat16, shape, name)


def conv3_forward(x, w, bias=None, relu=False, stream=None):
    """3x3x3 zero-padded convolution: x bf16 [nz, ny, nx, ci], w bf16 [co, 27, ci],
    bias float32 [co] or None -> y bf16 [nz, ny, nx, co]."""
    torch = _torch()
    nz, ny, nx, ci = (int(v) for v in x.shape)
    co = int(w.shape[0])
    px = _bf16(x, (nz, ny, nx, ci), "x")
    pw = _bf16(w, (co, 27, ci), "w")
    pb = _dev(bias, torch.float32, (co,), "bias") if bias is not None else None
    y = torch.empty((nz, ny, nx, co), dtype=torch.bfloat16, device=x.device)
    _check(_abi.load().cgd_conv3_forward(nx, ny, nz, ci, co, px, pw, pb, int(bool(relu)),
                                         ctypes.c_void_p(y.data_ptr()), _stream_ptr(stream)),
           "cgd_conv3_forward", allow=(0,))
    return y


def conv3_dgrad(g, w, stream=None):
    """Input gradient of conv3_forward: g bf16 [nz, ny, nx, co], w [co, 27, ci] -> bf16 [.., ci]."""
    torch = _torch()
    nz, ny, nx, co = (int(v) for v in g.shape)
    ci = int(w.shape[2])
    pg = _bf16(g, (nz, ny, nx, co), "g")
    pw = _bf16(w, (co, 27, ci), "w")
    dx = torch.empty((nz, ny, nx, ci), dtype=torch.bfloat16, device=g.device)
    _check(_abi.load().cgd_conv3_dgrad(nx, ny, nz, ci, co, pg, pw, ctypes.c_void_p(dx.data_ptr()),
                                       _stream_ptr(stream)), "cgd_conv3_dgrad", allow=(0,))
    return dx


def conv3_wgrad(x, g, stream=None):
    """Weight and bias gradients of conv3_forward: float32 dw [co, 27, ci], db [co]."""
    torch = _torch()
    nz, ny, nx, ci = (int(v) for v in x.shape)
    co = int(g.shape[3])
    px = _bf16(x, (nz, ny, nx, ci), "x")
    pg = _bf16(g, (nz, ny, nx, co), "g")
    dw = torch.empty((co, 27, ci), dtype=torch.float32, device=x.device)
    db = torch.empty((co,), dtype=torch.float32, device=x.device)
    _check(_abi.load().cgd_conv3_wgrad(nx, ny, nz, ci, co, px, pg, ctypes.c_void_p(dw.data_ptr()),
                                       ctypes.c_void_p(db.data_ptr()), _stream_ptr(stream)),
           "cgd_conv3_wgrad", allow=(0,))
    return dw, db
