"""GPU checks of the batched path (many snapshots x fields in one persistent
launch under a hipGraph) against the CPU oracle and the single-snapshot path.
"""
import os

import numpy as np
import pytest

from oracle import cgd_oracle as O
from paper_1409_0001_amd import inputs

pytestmark = pytest.mark.gpu

REL_L2 = 1e-5


def _t(a, torch):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _batch(shape, counts, seed):
    box = inputs.HexBox((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), shape)
    parts = [inputs.uniform_bed(box, n, 4, seed=seed + j) for j, n in enumerate(counts)]
    pos = np.concatenate([p.pos for p in parts]) if parts else np.zeros((0, 3), np.float32)
    vals = np.concatenate([p.values for p in parts], axis=1)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return box, parts, pos, vals, off


@pytest.mark.parametrize("shape", [(64, 40, 24), (128, 32, 20)])
def test_batched_matches_oracle_and_single_path(gpu_lib, shape):
    import torch
    cgd = gpu_lib
    counts = [20_000, 0, 7_000, 33_000, 1]
    box, parts, pos, vals, off = _batch(shape, counts, seed=71)
    b, steps = 4.0 / shape[0], 4
    print(f"case: batched {shape} snapshots {counts}", flush=True)
    mesh = cgd.HexMesh(shape, box.lo, box.hi)
    fields, iters = cgd.coarse_grain_batched(mesh, off, _t(pos, torch), _t(vals, torch), b, steps, rtol=1e-7,
                                             return_iters=True)
    out = fields.cpu().numpy()
    for j, p in enumerate(parts):
        dep = O.deposit_hex(p.pos, p.values, box.lo, box.hi, shape)
        ref = O.diffuse_hex_dct(dep["field64"], box.lo, box.hi, shape, b, steps)
        single, _ = cgd.coarse_grain(mesh, _t(p.pos, torch), _t(p.values, torch), b, steps, rtol=1e-7)
        single = single.cpu().numpy()
        for f in range(4):
            if counts[j] == 0:
                assert not out[j, f].any()
                continue
            assert rel_l2(out[j, f], ref[f]) <= REL_L2, (j, f, rel_l2(out[j, f], ref[f]))
            assert rel_l2(out[j, f], single[f]) <= REL_L2
    assert (iters[[0, 2, 3]] >= 1).all()


def test_batched_plain_and_preconditioned_cg_agree(gpu_lib):
    """Both solvers of the batched launch meet the oracle gate; the default
    polynomial-preconditioned CG needs at most 0.6 of plain CG's iterations
    (condition number 13 -> 2.1 at dtau / h^2 = 1)."""
    import torch
    cgd = gpu_lib
    shape = (128, 24, 40)
    counts = [30_000, 12_000, 50_000]
    box, parts, pos, vals, off = _batch(shape, counts, seed=77)
    b, steps = 4.0 / shape[0], 4
    mesh = cgd.HexMesh(shape, box.lo, box.hi)
    out = {}
    for pc in (0, 1):
        f, it = cgd.coarse_grain_batched(mesh, off, _t(pos, torch), _t(vals, torch), b, steps, rtol=1e-7,
                                         return_iters=True, precond=pc)
        out[pc] = (f.cpu().numpy(), it)
    for j, p in enumerate(parts):
        dep = O.deposit_hex(p.pos, p.values, box.lo, box.hi, shape)
        ref = O.diffuse_hex_dct(dep["field64"], box.lo, box.hi, shape, b, steps)
        for pc in (0, 1):
            for f in range(4):
                assert rel_l2(out[pc][0][j, f], ref[f]) <= REL_L2, (pc, j, f)
    print("iterations preconditioned", out[0][1].sum(), "plain", out[1][1].sum(), flush=True)
    assert out[0][1].sum() <= 0.6 * out[1][1].sum()


def test_batched_conserves_each_snapshot(gpu_lib):
    """Each snapshot's total (eq. conserve) survives the batched deposit and
    diffusion; the single-snapshot deposit of the same particles is
    bit-exact against the oracle."""
    import torch
    cgd = gpu_lib
    shape = (64, 16, 8)
    counts = [5_000, 12_000, 3]
    box, parts, pos, vals, off = _batch(shape, counts, seed=81)
    mesh = cgd.HexMesh(shape, box.lo, box.hi)
    fields = cgd.coarse_grain_batched(mesh, off, _t(pos, torch), _t(vals, torch), 0.1, 2, rtol=1e-7)
    out = fields.cpu().numpy().astype(np.float64)
    V = O.hex_cell_volume(box.lo, box.hi, shape)
    for j, p in enumerate(parts):
        dep = cgd.deposit(mesh, _t(p.pos, torch), _t(p.values, torch)).cpu().numpy().astype(np.float64)
        ref = O.deposit_hex(p.pos, p.values, box.lo, box.hi, shape)
        assert np.array_equal(dep.astype(np.float32).view(np.uint32), ref["field32"].view(np.uint32))
        for f in range(4):
            m_in = ref["field64"][f].sum() * V
            scale = np.abs(ref["field64"][f]).sum() * V
            assert abs(out[j, f].sum() * V - m_in) <= 1e-5 * scale


@pytest.mark.parametrize("F", [4, 1])
def test_batched_tiled_and_direct_deposits_agree_bitwise(gpu_lib, F, monkeypatch):
    """The tiled deposit (particles bucketed by tile of every snapshot, sums
    in LDS) and the direct one (int64 atomics) are both exact, and the solve
    is deterministic, so the batched results agree bit for bit; snapshots
    span many tiles, one is empty and one holds a single particle.  F = 4:
    96 tiles of 4096 cells per snapshot, records stored from registers; F = 1:
    24 tiles of 16384, records ordered by tile in LDS first."""
    import torch
    cgd = gpu_lib
    shape = (128, 64, 48)
    counts = [60_000, 0, 1, 25_000, 90_000]
    box, parts, pos, vals, off = _batch(shape, counts, seed=97)
    vals = np.ascontiguousarray(vals[:F])
    print(f"case: batched tiled vs direct deposit {shape} F={F} snapshots {counts}", flush=True)
    mesh = cgd.HexMesh(shape, box.lo, box.hi)
    dpos, dvals = _t(pos, torch), _t(vals, torch)
    monkeypatch.delenv("CGD_DEPOSIT_DIRECT", raising=False)
    tiled = cgd.coarse_grain_batched(mesh, off, dpos, dvals, 4.0 / shape[0], 2, rtol=1e-7).clone()
    monkeypatch.setenv("CGD_DEPOSIT_DIRECT", "1")
    direct = cgd.coarse_grain_batched(mesh, off, dpos, dvals, 4.0 / shape[0], 2, rtol=1e-7)
    assert torch.equal(tiled.view(torch.int32), direct.view(torch.int32))
    assert not tiled[1].any()


@pytest.mark.parametrize("cfg", [None, 8])
def test_graph_replays_equal_eager(gpu_lib, cfg, monkeypatch):
    """The captured graph, replayed several times with eager work and
    synchronisations in between, gives the eager result bit for bit (the
    autotuner's pick, and the per-launch candidate, whose graph replays
    the iteration budgets of the eager run before it)."""
    import torch
    cgd = gpu_lib
    if cfg is not None:
        monkeypatch.setenv("CGD_BATCHED_CFG", str(cfg))
    shape = (128, 24, 16)
    counts = [9_000, 15_000, 4_000]
    box, parts, pos, vals, off = _batch(shape, counts, seed=91)
    mesh = cgd.HexMesh(shape, box.lo, box.hi)
    dpos, dvals = _t(pos, torch), _t(vals, torch)
    os.environ["CGD_NO_GRAPH"] = "1"
    try:
        eager = cgd.coarse_grain_batched(mesh, off, dpos, dvals, 0.04, 3, rtol=1e-7).clone()
    finally:
        del os.environ["CGD_NO_GRAPH"]
    out = torch.empty_like(eager)
    for rep in range(4):
        out.fill_(float("nan"))
        cgd.coarse_grain_batched(mesh, off, dpos, dvals, 0.04, 3, rtol=1e-7, fields=out)
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int32), eager.view(torch.int32)), rep
        assert torch.isfinite(junk)


def test_autotune_reports_candidates(gpu_lib):
    cgd = gpu_lib
    mesh = cgd.HexMesh((128, 64, 32))
    chosen, ms = cgd.autotune_batched(mesh, 32)
    # persistent launch: 4 tile shapes at degree 2, 2 at degree 4, 2 at degree
    # 12; then the per-launch solver over groups of fields
    assert len(ms) == 9 and all(t > 0 for t in ms)
    assert chosen == int(np.argmin(ms))


# persistent: degree 2 (four tile shapes), degrees 4 and 12 (two each); 8: per-launch
@pytest.mark.parametrize("cfg", [0, 1, 2, 3, 4, 5, 6, 7, 8])
def test_batched_candidates_match_oracle(gpu_lib, cfg, monkeypatch):
    """Every preconditioner degree of the persistent solver reaches the same
    fields: forced candidates against the float64 oracle on 128 x 20 x 24
    (ragged row groups and tiles)."""
    import torch
    cgd = gpu_lib
    shape = (128, 20, 24)
    box = inputs.HexBox((0.0, 0.0, 0.0), (1.0, 20 / 128, 24 / 128), shape)
    snaps = [inputs.uniform_bed(box, 3000 + 500 * j, 2, seed=90 + j, diam=0.01) for j in range(3)]
    off = np.concatenate([[0], np.cumsum([len(p.pos) for p in snaps])]).astype(np.int64)
    pos = torch.from_numpy(np.concatenate([p.pos for p in snaps])).cuda()
    vals = torch.from_numpy(np.concatenate([p.values for p in snaps], axis=1)).cuda()
    mesh = cgd.HexMesh(shape, box.lo, box.hi)
    monkeypatch.setenv("CGD_BATCHED_CFG", str(cfg))
    b, steps = 4.0 / 128, 4
    print(f"case: batched candidate {cfg}, {shape}", flush=True)
    out, iters = cgd.coarse_grain_batched(mesh, off, pos, vals, b, steps, rtol=1e-7, return_iters=True)
    o = out.cpu().numpy()
    for j, p in enumerate(snaps):
        dep = O.deposit_hex(p.pos, p.values, box.lo, box.hi, shape)
        ref = O.diffuse_hex_dct(dep["field64"], box.lo, box.hi, shape, b, steps)
        for f in range(2):
            assert rel_l2(o[j, f], ref[f]) <= 1e-5, (cfg, j, f, rel_l2(o[j, f], ref[f]))
    print("iterations per step", iters.reshape(-1, steps).mean(axis=0), flush=True)


def test_batched_any_width(gpu_lib):
    """A grid width the persistent launch does not cover (nx = 96): the
    autotuner has only the per-launch solver, which meets the oracle."""
    import torch
    cgd = gpu_lib
    shape = (96, 20, 12)
    counts = [4_000, 7_000]
    box, parts, pos, vals, off = _batch(shape, counts, seed=93)
    mesh = cgd.HexMesh(shape, box.lo, box.hi)
    chosen, ms = cgd.autotune_batched(mesh, 8)
    assert len(ms) == 1 and chosen == 0
    b, steps = 4.0 / 96, 3
    out = cgd.coarse_grain_batched(mesh, off, _t(pos, torch), _t(vals, torch), b, steps, rtol=1e-7).cpu().numpy()
    for j, p in enumerate(parts):
        dep = O.deposit_hex(p.pos, p.values, box.lo, box.hi, shape)
        ref = O.diffuse_hex_dct(dep["field64"], box.lo, box.hi, shape, b, steps)
        for f in range(4):
            assert rel_l2(out[j, f], ref[f]) <= REL_L2, (j, f, rel_l2(out[j, f], ref[f]))


def test_per_launch_budget_miss_reruns(gpu_lib, monkeypatch):
    """The per-launch candidate's graph replays the iteration budget of the
    run before it; a call whose data needs more (same buffers, new values)
    finds a right-hand side unconverged after the replay and is run again
    with read-backs: the result still meets the oracle and no status says
    not converged."""
    import torch
    cgd = gpu_lib
    monkeypatch.setenv("CGD_BATCHED_CFG", "8")
    shape = (64, 16, 12)
    box = inputs.HexBox((0.0, 0.0, 0.0), (1.0, 0.25, 0.1875), shape)
    # one particle at every cell centre: with equal values the deposited
    # field is constant, an eigenvector of the operator, solved in one iteration
    idx = np.indices(shape[::-1]).reshape(3, -1)[::-1].T.astype(np.float64)
    h = (np.asarray(box.hi) - np.asarray(box.lo)) / np.asarray(shape)
    centres = (np.asarray(box.lo) + (idx + 0.5) * h).astype(np.float32)
    n = len(centres)
    pos = np.concatenate([centres, centres])
    off = np.array([0, n, 2 * n], dtype=np.int64)
    mesh = cgd.HexMesh(shape, box.lo, box.hi)
    dpos = _t(pos, torch)
    dvals = torch.full((1, 2 * n), 0.5, dtype=torch.float32, device="cuda")
    b, steps = 4.0 / 64, 2
    _, it1 = cgd.coarse_grain_batched(mesh, off, dpos, dvals, b, steps, rtol=1e-6, return_iters=True)
    _, it2 = cgd.coarse_grain_batched(mesh, off, dpos, dvals, b, steps, rtol=1e-6, return_iters=True)
    assert it1.max() == 1 and np.array_equal(it1, it2), (it1, it2)
    rv = np.random.default_rng(94).random((1, 2 * n)).astype(np.float32)
    dvals.copy_(torch.from_numpy(rv))
    out, it3 = cgd.coarse_grain_batched(mesh, off, dpos, dvals, b, steps, rtol=1e-6, return_iters=True)
    assert it3.max() >= 2
    o = out.cpu().numpy()
    for j in range(2):
        dep = O.deposit_hex(pos[off[j]:off[j + 1]], rv[:, off[j]:off[j + 1]], box.lo, box.hi, shape)
        ref = O.diffuse_hex_dct(dep["field64"], box.lo, box.hi, shape, b, steps)
        assert rel_l2(o[j, 0], ref[0]) <= REL_L2, (j, rel_l2(o[j, 0], ref[0]))


def test_batched_invalid(gpu_lib):
    import torch
    cgd = gpu_lib
    pos = torch.rand((10, 3), device="cuda")
    vals = torch.rand((1, 10), device="cuda")
    mesh = cgd.HexMesh((64, 8, 8))
    with pytest.raises(cgd.CgdError):
        cgd.coarse_grain_batched(mesh, [0, 6, 4, 10], pos, vals, 0.1, 2)  # decreasing offsets


@pytest.mark.parametrize("cfg,precond", [(None, 0), (1, 0), (1, 1), (4, 0), (4, 1), (6, 0), (6, 1), (8, 0), (8, 1)])
def test_batched_crank_nicolson_matches_oracle_and_graph_key(gpu_lib, cfg, precond, monkeypatch):
    """Crank-Nicolson in the persistent launch (the x updates carry the
    extrapolation) against the oracle's CN closed form, after a backward-Euler
    call with the same arguments: the captured graph must not be replayed
    across schemes.  The autotuner's pick and forced candidates of degree 2,
    4 and 12, each preconditioned and plain (plain CG runs the degree-2
    kernel of the same tile shape: the S2_FIRST x update with xb * b)."""
    import torch
    cgd = gpu_lib
    if cfg is not None:
        monkeypatch.setenv("CGD_BATCHED_CFG", str(cfg))
    shape = (64, 40, 36)
    counts = [15_000, 9_000, 1]
    box, parts, pos, vals, off = _batch(shape, counts, seed=91)
    b, steps = 4.0 / shape[0], 3
    print(f"case: batched CN {shape} snapshots {counts}", flush=True)
    mesh = cgd.HexMesh(shape, box.lo, box.hi)
    args = (mesh, off, _t(pos, torch), _t(vals, torch), b, steps)
    print(f"  candidate {cfg}, precond {precond}", flush=True)
    be = cgd.coarse_grain_batched(*args, rtol=1e-7, precond=precond).cpu().numpy()
    cn = cgd.coarse_grain_batched(*args, rtol=1e-7, scheme="cn", precond=precond).cpu().numpy()
    for j, p in enumerate(parts):
        dep = O.deposit_hex(p.pos, p.values, box.lo, box.hi, shape)
        ref_cn = O.diffuse_hex_dct(dep["field64"], box.lo, box.hi, shape, b, steps, scheme="cn")
        ref_be = O.diffuse_hex_dct(dep["field64"], box.lo, box.hi, shape, b, steps)
        for f in range(4):
            assert rel_l2(cn[j, f], ref_cn[f]) <= REL_L2, (j, f, rel_l2(cn[j, f], ref_cn[f]))
            assert rel_l2(be[j, f], ref_be[f]) <= REL_L2, (j, f)


def test_batched_stats_per_snapshot(gpu_lib):
    """Per-snapshot statistics of the batched call: the fixed-point scales of
    the oracle's deposit, dropped and non-finite particles of each snapshot
    (planted in one of them), mass before diffusion equal to the oracle's
    deposited mass (float32 field, float64 sums), mass after within the
    stopping rule's bound, residuals at or below rtol, and iterations that
    agree with the iteration output."""
    import torch
    cgd = gpu_lib
    shape = (64, 24, 20)
    counts = [9_000, 4_000, 0, 6_000]
    box, parts, pos, vals, off = _batch(shape, counts, seed=95)
    pos = pos.copy()
    vals = vals.copy()
    k = int(off[1]) + 10  # snapshot 1: three particles outside the box, one non-finite position
    pos[k:k + 3, 0] = 1.5
    pos[k + 3, 2] = np.nan
    parts[1].pos[10:13, 0] = 1.5
    parts[1].pos[13, 2] = np.nan
    b, steps, rtol = 4.0 / shape[0], 3, 1e-7
    print(f"case: batched stats {shape} snapshots {counts}", flush=True)
    mesh = cgd.HexMesh(shape, box.lo, box.hi)
    fields, iters, sts = cgd.coarse_grain_batched(mesh, off, _t(pos, torch), _t(vals, torch), b, steps,
                                                  rtol=rtol, return_iters=True, stats=True)
    V = O.hex_cell_volume(box.lo, box.hi, shape)
    for j, p in enumerate(parts):
        st = sts[j]
        dep = O.deposit_hex(p.pos, p.values, box.lo, box.hi, shape)
        assert st.frac_bits == dep["S"], (j, st.frac_bits, dep["S"])
        assert st.n_dropped == dep["n_dropped"] and st.n_nonfinite == dep["n_nonfinite"], j
        assert st.status == (-2 if j == 1 else 0), (j, st.status)
        for f in range(4):
            m32 = float(dep["field32"][f].astype(np.float64).sum() * V)
            assert st.mass_before[f] == pytest.approx(m32, rel=1e-12, abs=1e-300), (j, f)
            scale = float(np.abs(dep["field32"][f].astype(np.float64)).sum() * V)
            assert abs(st.mass_after[f] - st.mass_before[f]) <= 1e-5 * scale + 1e-300, (j, f)
            for s_ in range(steps):
                assert st.iters[s_][f] == iters[j, f, s_]
                assert st.rel_res[s_][f] <= rtol, (j, f, s_, st.rel_res[s_][f])
    assert sts[2].n_dropped == 0 and all(m == 0 for m in sts[2].mass_before)
