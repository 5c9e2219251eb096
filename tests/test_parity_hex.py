"""GPU parity of the hex path against the CPU oracle (through the C-ABI).

Deposition: bit-exact (int64 sums and float32 fields).  Diffusion: relative
L2 <= 1e-5 per field against the float64 oracle (the accuracy target of this
path); the GPU solves to rtol 1e-7 at small sizes and 1e-6 on the dense bed.
"""
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
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_deposit_tiny_bit_exact(gpu_lib):
    import torch
    cgd = gpu_lib
    w = inputs.tiny()
    print(f"case: {w.name}", flush=True)
    mesh = cgd.HexMesh(w.box.shape, w.box.lo, w.box.hi)
    pos, vals = _t(w.particles.pos, torch), _t(w.particles.values, torch)
    acc = torch.empty((1, mesh.cells), dtype=torch.int64, device="cuda")
    field, st = cgd.deposit(mesh, pos, vals, acc=acc, stats=True)
    ref = O.deposit_hex(w.particles.pos, w.particles.values, w.box.lo, w.box.hi, w.box.shape)
    assert st.frac_bits[0] == ref["S"][0]
    assert np.array_equal(acc.cpu().numpy(), ref["acc"])
    assert np.array_equal(field.cpu().numpy().view(np.uint32), ref["field32"].view(np.uint32))
    assert st.n_dropped == 0 and st.n_nonfinite == 0
    # shuffled particle order and a second run: bitwise identical
    perm = np.random.default_rng(5).permutation(len(w.particles.pos))
    field2 = cgd.deposit(mesh, _t(w.particles.pos[perm], torch), _t(w.particles.values[:, perm], torch))
    field3 = cgd.deposit(mesh, pos, vals)
    torch.cuda.synchronize()
    assert torch.equal(field2.view(torch.int32), field.view(torch.int32))
    assert torch.equal(field3.view(torch.int32), field.view(torch.int32))


@pytest.mark.parametrize("F", [2, 3])
def test_deposit_many_tiles_clustered_bit_exact(gpu_lib, F):
    """The dense-bed recipe on 96 x 80 x 200 (1.5M cells; tiles of 8192
    cells at F = 2 and, rounded down to a power of two, 4096 at F = 3; the
    upper tiles empty): the tiled deposit's fields and accumulators are
    bit-identical to the oracle's."""
    import torch
    cgd = gpu_lib
    w = inputs.dense_bed(n_particles=400_000, shape=(96, 80, 200), n_fields=F)
    print(f"case: {w.name}", flush=True)
    mesh = cgd.HexMesh(w.box.shape, w.box.lo, w.box.hi)
    acc = torch.empty((F, mesh.cells), dtype=torch.int64, device="cuda")
    field, st = cgd.deposit(mesh, _t(w.particles.pos, torch), _t(w.particles.values, torch), acc=acc, stats=True)
    ref = O.deposit_hex(w.particles.pos, w.particles.values, w.box.lo, w.box.hi, w.box.shape)
    assert st.frac_bits[:F] == ref["S"]
    assert np.array_equal(acc.cpu().numpy(), ref["acc"])
    assert np.array_equal(field.cpu().numpy().view(np.uint32), ref["field32"].view(np.uint32))


def test_deposit_dense_bed_single_field_many_tiles_bit_exact(gpu_lib):
    """The dense-bed recipe at one field, the benchmarked deposit: tiles of
    16384 cells (the largest LDS tile) on 128 x 128 x 256 = 256 tiles, 2.5M
    particles (the dense bed's per-volume density), 70 % of them packed in
    the bottom quarter and the rest in clumps, so tiles (here one z-plane
    each) range from nearly empty to crowded.  Accumulators and float32 field bit-identical to the oracle's
    (eq. pcm-k; eq. conserve holds exactly in the integers)."""
    import torch
    cgd = gpu_lib
    w = inputs.dense_bed(n_particles=2_500_000, shape=(128, 128, 256), n_fields=1)
    print(f"case: {w.name}", flush=True)
    mesh = cgd.HexMesh(w.box.shape, w.box.lo, w.box.hi)
    acc = torch.empty((1, mesh.cells), dtype=torch.int64, device="cuda")
    field, st = cgd.deposit(mesh, _t(w.particles.pos, torch), _t(w.particles.values, torch), acc=acc, stats=True)
    ref = O.deposit_hex(w.particles.pos, w.particles.values, w.box.lo, w.box.hi, w.box.shape)
    a = acc.cpu().numpy()
    assert st.frac_bits[0] == ref["S"][0]
    assert np.array_equal(a, ref["acc"])
    assert np.array_equal(field.cpu().numpy().view(np.uint32), ref["field32"].view(np.uint32))
    occupied = np.add.reduceat((a[0] != 0).astype(np.int64), np.arange(0, mesh.cells, 16384))
    assert occupied.min() < 100 and occupied.max() > 8000  # nearly empty and crowded tiles both present
    assert int(a.sum()) == int(O.quantise(w.particles.values[0], ref["S"][0]).sum())


@pytest.mark.parametrize("shape,cpt,F", [((64, 64, 64), 32, 1), ((64, 64, 64), 16, 1), ((64, 64, 64), 16, 4),
                                         ((60, 61, 67), 16, 2), ((64, 64, 65), 16, 1),
                                         ((64, 64, 64), 128, 1), ((64, 64, 64), 128, 4), ((64, 64, 65), 128, 3)])
def test_deposit_tile_counts_bit_exact(gpu_lib, shape, cpt, F, monkeypatch):
    """Tiles forced small (CGD_DEPOSIT_CPT) to reach the bucketing passes'
    tile limits on small grids: 8,192 tiles (32-bit counters), 16,384 (two
    16-bit counters per word), a ragged 15,327 at two fields and 16,384 at
    four, and 16,640 (beyond both: the direct path); and the scatter's: 2,048
    tiles at one and four fields (records ordered in LDS, the most tiles it
    takes) and a ragged 2,080 at three (beyond it: stored from registers).  Clustered particles
    (the dense-bed recipe), so that some tiles take thousands of one block's
    particles; accumulators and fields bit-identical to the oracle's."""
    import torch
    cgd = gpu_lib
    monkeypatch.setenv("CGD_DEPOSIT_CPT", str(cpt))
    w = inputs.dense_bed(n_particles=300_000, shape=shape, n_fields=F)
    print(f"case: {w.name}, {cpt} cells per tile", flush=True)
    mesh = cgd.HexMesh(w.box.shape, w.box.lo, w.box.hi)
    acc = torch.empty((F, mesh.cells), dtype=torch.int64, device="cuda")
    field, st = cgd.deposit(mesh, _t(w.particles.pos, torch), _t(w.particles.values, torch), acc=acc, stats=True)
    ref = O.deposit_hex(w.particles.pos, w.particles.values, w.box.lo, w.box.hi, w.box.shape)
    assert st.frac_bits[:F] == ref["S"]
    assert np.array_equal(acc.cpu().numpy(), ref["acc"])
    assert np.array_equal(field.cpu().numpy().view(np.uint32), ref["field32"].view(np.uint32))
    a = acc.cpu().numpy()[0]
    per_tile = np.add.reduceat((a != 0).astype(np.int64), np.arange(0, mesh.cells, cpt))
    assert per_tile.max() == cpt and per_tile.min() == 0  # crowded and empty tiles


@pytest.mark.parametrize("path", ["tiled", "direct"])
def test_deposit_forced_frac_bits(gpu_lib, path, monkeypatch):
    """cgd_deposit's frac_bits: a forced scale for one field, automatic for
    the other, against the oracle with the same scales (signed values, two
    fields, ragged grid); the scales used come back through the array, and
    scales outside -1..62 are refused before anything is enqueued."""
    import torch
    cgd = gpu_lib
    if path == "direct":
        monkeypatch.setenv("CGD_DEPOSIT_DIRECT", "1")
    box = inputs.HexBox((-0.3, 0.1, 2.0), (0.7, 0.35, 2.9), (37, 29, 11))
    p = inputs.uniform_bed(box, 30_000, 2, seed=23)
    print(f"case: forced frac_bits, {path} deposit", flush=True)
    mesh = cgd.HexMesh(box.shape, box.lo, box.hi)
    auto = O.deposit_hex(p.pos, p.values, box.lo, box.hi, box.shape)["S"]
    forced = [auto[0] - 9, -1]
    acc = torch.empty((2, mesh.cells), dtype=torch.int64, device="cuda")
    fb = list(forced)
    field = cgd.deposit(mesh, _t(p.pos, torch), _t(p.values, torch), acc=acc, frac_bits=fb)
    torch.cuda.synchronize()
    ref = O.deposit_hex(p.pos, p.values, box.lo, box.hi, box.shape, force_bits=forced)
    assert fb == [auto[0] - 9, auto[1]] == ref["S"]
    assert np.array_equal(acc.cpu().numpy(), ref["acc"])
    assert np.array_equal(field.cpu().numpy().view(np.uint32), ref["field32"].view(np.uint32))
    # a coarser scale changes the sums (so the forced value really was used)
    assert not np.array_equal(ref["acc"][0], O.deposit_hex(p.pos, p.values, box.lo, box.hi, box.shape)["acc"][0])
    for bad in ([63, -1], [-2, -1]):
        with pytest.raises(cgd.CgdError):
            cgd.deposit(mesh, _t(p.pos, torch), _t(p.values, torch), frac_bits=bad)


@pytest.mark.parametrize("F", [4, 1])
@pytest.mark.parametrize("path", ["tiled", "direct"])
def test_deposit_signed_multifield_ragged_and_dropped(gpu_lib, path, F, monkeypatch):
    """Both deposit paths: tile-bucketed sums in LDS (default) and direct
    device-wide atomics (CGD_DEPOSIT_DIRECT); at one field the tiled path's
    records are ordered by tile in LDS before they are stored, at four they
    are stored from registers (16-byte records plus a value array)."""
    import torch
    cgd = gpu_lib
    if path == "direct":
        monkeypatch.setenv("CGD_DEPOSIT_DIRECT", "1")
    box = inputs.HexBox((-0.3, 0.1, 2.0), (0.7, 0.35, 2.9), (37, 29, 11))
    rng = np.random.default_rng(21)
    n = 50_000
    p = inputs.uniform_bed(box, n, 4, seed=22)
    pos = p.pos.copy()
    pos[:50] += 0.5   # some outside the box
    pos[50, 1] = np.nan
    vals = p.values[:F].copy()
    vals[min(2, F - 1), 60] = np.inf
    print(f"case: ragged 37x29x11, F={F}, dropped/non-finite, {path} deposit", flush=True)
    mesh = cgd.HexMesh(box.shape, box.lo, box.hi)
    acc = torch.empty((F, mesh.cells), dtype=torch.int64, device="cuda")
    field, st = cgd.deposit(mesh, _t(pos, torch), _t(vals, torch), acc=acc, stats=True)
    ref = O.deposit_hex(pos, vals, box.lo, box.hi, box.shape)
    assert st.status == -2  # CGD_E_NONFINITE reported, field still written
    assert st.frac_bits[:F] == ref["S"]
    assert st.n_dropped == ref["n_dropped"]
    assert np.array_equal(acc.cpu().numpy(), ref["acc"])
    assert np.array_equal(field.cpu().numpy().view(np.uint32), ref["field32"].view(np.uint32))


@pytest.mark.parametrize("shape,lo,hi,b,steps", [
    ((24, 24, 24), (0, 0, 0), (1, 1, 1), 0.05, 4),            # the tiny workload
    ((37, 29, 11), (-0.3, 0.1, 2.0), (0.7, 0.35, 2.9), 0.06, 3),  # ragged tiles, non-cubic cells
    ((130, 9, 70), (0, 0, 0), (1.3, 0.09, 0.7), 0.04, 2),    # two x segments, thin y
    ((1, 1, 1), (0, 0, 0), (1, 1, 1), 0.3, 2),               # one cell: A = I
    ((64, 1, 1), (0, 0, 0), (1, 1, 1), 0.1, 4),              # 1-D
])
@pytest.mark.parametrize("precond", [0, 1])  # polynomial-preconditioned CG, plain CG
def test_coarse_grain_matches_oracle(gpu_lib, shape, lo, hi, b, steps, precond):
    import torch
    cgd = gpu_lib
    box = inputs.HexBox(lo, hi, shape)
    n = 20_000
    p = inputs.uniform_bed(box, n, 2, seed=31, diam=0.01)
    print(f"case: coarse_grain {shape} b={b} steps={steps} precond={precond}", flush=True)
    mesh = cgd.HexMesh(shape, lo, hi)
    field, st = cgd.coarse_grain(mesh, _t(p.pos, torch), _t(p.values, torch), b, steps,
                                 rtol=1e-7, stats=True, precond=precond)
    out = field.cpu().numpy()
    ref, dep = O.coarse_grain_hex(p.pos, p.values, lo, hi, shape, b, steps, solver="direct")
    for f in range(2):
        assert rel_l2(out[f], ref[f]) <= REL_L2, (f, rel_l2(out[f], ref[f]))
        V = O.hex_cell_volume(lo, hi, shape)
        mb, ma = st.mass_before[f], st.mass_after[f]
        assert abs(ma - mb) <= 1e-5 * abs(dep["field64"][f]).sum() * V
    assert st.status == 0
    assert all(st.iters[s][f] >= 1 for s in range(steps) for f in range(2)) or shape == (1, 1, 1)


def test_tiny_workload_and_determinism(gpu_lib):
    import torch
    cgd = gpu_lib
    w = inputs.tiny()
    print(f"case: {w.name} end to end", flush=True)
    mesh = cgd.HexMesh(w.box.shape, w.box.lo, w.box.hi)
    pos, vals = _t(w.particles.pos, torch), _t(w.particles.values, torch)
    f1, st = cgd.coarse_grain(mesh, pos, vals, w.bandwidth, w.n_steps, rtol=w.rtol, stats=True)
    f2, _ = cgd.coarse_grain(mesh, pos, vals, w.bandwidth, w.n_steps, rtol=w.rtol)
    torch.cuda.synchronize()
    assert torch.equal(f1.view(torch.int32), f2.view(torch.int32))  # deterministic reductions
    ref, _ = O.coarse_grain_hex(w.particles.pos, w.particles.values, w.box.lo, w.box.hi,
                                w.box.shape, w.bandwidth, w.n_steps, solver="direct")
    assert rel_l2(f1.cpu().numpy()[0], ref[0]) <= REL_L2
    assert max(r[0] for r in st.rel_res) <= w.rtol


def test_multifield_equals_single_field_bitwise(gpu_lib):
    import torch
    cgd = gpu_lib
    box = inputs.HexBox((0, 0, 0), (1, 1, 1), (48, 40, 36))
    p = inputs.uniform_bed(box, 30_000, 4, seed=41)
    mesh = cgd.HexMesh(box.shape, box.lo, box.hi)
    print("case: F=4 vs four F=1 solves", flush=True)
    vals = _t(p.values, torch)
    f4, _ = cgd.coarse_grain(mesh, _t(p.pos, torch), vals, 0.08, 4, rtol=1e-7)
    for f in range(4):
        f1, _ = cgd.coarse_grain(mesh, _t(p.pos, torch), vals[f:f + 1].contiguous(), 0.08, 4, rtol=1e-7)
        assert torch.equal(f1[0].view(torch.int32), f4[f].view(torch.int32))
    ref, _ = O.coarse_grain_hex(p.pos, p.values, box.lo, box.hi, box.shape, 0.08, 4)
    out = f4.cpu().numpy()
    for f in range(4):
        assert rel_l2(out[f], ref[f]) <= REL_L2


@pytest.mark.parametrize("mode", [1, 2])
def test_initial_guess_modes(gpu_lib, mode):
    import torch
    cgd = gpu_lib
    w = inputs.tiny()
    mesh = cgd.HexMesh(w.box.shape, w.box.lo, w.box.hi)
    print(f"case: x0_mode={mode}", flush=True)
    field = cgd.deposit(mesh, _t(w.particles.pos, torch), _t(w.particles.values, torch))
    x0 = field.clone() if mode == 2 else None
    out, st = cgd.diffuse(mesh, field, w.bandwidth, w.n_steps, rtol=1e-7, x0_mode=mode, x0=x0,
                          stats=True)
    ref, _ = O.coarse_grain_hex(w.particles.pos, w.particles.values, w.box.lo, w.box.hi,
                                w.box.shape, w.bandwidth, w.n_steps, solver="direct")
    assert rel_l2(out.cpu().numpy()[0], ref[0]) <= REL_L2


def test_zero_field_and_no_particles(gpu_lib):
    import torch
    cgd = gpu_lib
    mesh = cgd.HexMesh((16, 8, 4))
    pos = torch.zeros((0, 3), dtype=torch.float32, device="cuda")
    vals = torch.zeros((2, 0), dtype=torch.float32, device="cuda")
    print("case: no particles", flush=True)
    field, st = cgd.coarse_grain(mesh, pos, vals, 0.2, 3, stats=True)
    assert torch.count_nonzero(field).item() == 0
    for mode in (1,):
        z = torch.zeros((1, mesh.cells), dtype=torch.float32, device="cuda")
        out, _ = cgd.diffuse(mesh, z, 0.2, 2, x0_mode=mode)
        assert torch.count_nonzero(out).item() == 0


def test_not_converged_and_invalid_args(gpu_lib):
    import torch
    cgd = gpu_lib
    w = inputs.tiny()
    mesh = cgd.HexMesh(w.box.shape, w.box.lo, w.box.hi)
    field = cgd.deposit(mesh, _t(w.particles.pos, torch), _t(w.particles.values, torch))
    print("case: max_iter=1", flush=True)
    _, st = cgd.diffuse(mesh, field, w.bandwidth, 2, rtol=1e-12, max_iter=1, stats=True)
    assert st.status == 1  # CGD_NOT_CONVERGED
    assert all(it[0] == 1 for it in st.iters)
    with pytest.raises(cgd.CgdError):
        cgd.diffuse(mesh, field, -1.0, 2)
    with pytest.raises(cgd.CgdError):
        cgd.diffuse(mesh, field, 0.1, 0)
    with pytest.raises(cgd.CgdError):
        cgd.HexMesh((0, 4, 4))
    with pytest.raises(cgd.CgdError):
        cgd.HexMesh((4, 4, 4), lo=(0, 0, 0), hi=(1, 0, 1))


def test_nan_field_is_breakdown(gpu_lib):
    import torch
    cgd = gpu_lib
    mesh = cgd.HexMesh((16, 16, 16))
    f = torch.ones((1, mesh.cells), dtype=torch.float32, device="cuda")
    f[0, 7] = float("nan")
    print("case: NaN field", flush=True)
    with pytest.raises(cgd.CgdError) as e:
        cgd.diffuse(mesh, f, 0.2, 2)
    assert e.value.status == -5


def test_dense_bed_reduced_against_dct(gpu_lib):
    """The dense-bed recipe at 1/64 of the cells and particles."""
    import torch
    cgd = gpu_lib
    w = inputs.dense_bed(n_particles=20_000_000 // 64, shape=(64, 64, 128), n_fields=4)
    print(f"case: {w.name}", flush=True)
    mesh = cgd.HexMesh(w.box.shape, w.box.lo, w.box.hi)
    out, st = cgd.coarse_grain(mesh, _t(w.particles.pos, torch), _t(w.particles.values, torch),
                               w.bandwidth, w.n_steps, rtol=w.rtol, stats=True)
    dep = O.deposit_hex(w.particles.pos, w.particles.values, w.box.lo, w.box.hi, w.box.shape)
    ref = O.diffuse_hex_dct(dep["field64"], w.box.lo, w.box.hi, w.box.shape, w.bandwidth, w.n_steps)
    o = out.cpu().numpy()
    for f in range(4):
        assert rel_l2(o[f], ref[f]) <= REL_L2, (f, rel_l2(o[f], ref[f]))
    # plain CG reaches the same result in more iterations: at dtau/h^2 = 1 the
    # polynomial preconditioner takes the condition number from 13 to 3.8,
    # and the CG bound from ~25 to ~12 iterations per step at rtol 1e-6
    out1, st1 = cgd.coarse_grain(mesh, _t(w.particles.pos, torch), _t(w.particles.values, torch),
                                 w.bandwidth, w.n_steps, rtol=w.rtol, stats=True, precond=1)
    o1 = out1.cpu().numpy()
    for f in range(4):
        assert rel_l2(o1[f], ref[f]) <= REL_L2
    it0 = sum(sum(r) for r in st.iters)
    it1 = sum(sum(r) for r in st1.iters)
    print(f"iterations: preconditioned {st.iters}, plain {st1.iters}", flush=True)
    assert it0 <= 0.7 * it1, (it0, it1)


@pytest.mark.parametrize("deg", [3, 4, 8, 12])
@pytest.mark.parametrize("shape,zc", [((64, 37, 100), 16), ((128, 20, 70), 13), ((256, 13, 40), 7),
                                      ((40, 37, 60), 16), ((100, 21, 50), 9), ((200, 13, 40), 7)])
def test_lds_preconditioner_matches_oracle(gpu_lib, shape, zc, deg, monkeypatch):
    """The degree-3/4 preconditioning sweep with its powers of A in LDS
    (one wave per x-row: nx = 64, 128, 256, and partial rows of 40, 100 and
    200 cells at 1, 2 and 4 cells per lane, the lanes beyond the row idle),
    and degrees 8 and 12 as two and
    three passes of quadratic factors, forced onto small grids with ragged
    row groups (ny not a multiple of 8) and a ragged last z chunk: the result
    matches the float64 DCT solution, and the higher degree takes fewer
    iterations than degree 2.  At dtau / h^2 = 1 (spectrum [1, 13]) the
    degree-8 and degree-12 polynomials bring every step to rtol 1e-6 in at
    most 3 and 2 iterations (a float32 model of the method on 48^3 takes 3
    and 2; a wrong factor would cost iterations)."""
    import torch
    cgd = gpu_lib
    nx, ny, nz = shape
    lo, hi = (0.0, 0.0, 0.0), (nx / 64.0, ny / 64.0, nz / 64.0)
    box = inputs.HexBox(lo, hi, shape)
    p = inputs.uniform_bed(box, 50_000, 2, seed=77, diam=0.01)
    b, steps = 4.0 / 64.0, 4  # dtau / h^2 = 1, as on the dense bed
    print(f"case: lds preconditioner degree {deg}, {shape}, zc {zc}", flush=True)
    mesh = cgd.HexMesh(shape, lo, hi)
    pos, vals = _t(p.pos, torch), _t(p.values, torch)
    monkeypatch.setenv("CGD_HEX_PRECOND_DEG", "2")
    f2, st2 = cgd.coarse_grain(mesh, pos, vals, b, steps, rtol=1e-6, stats=True)
    monkeypatch.setenv("CGD_HEX_PRECOND_DEG", str(deg))
    monkeypatch.setenv("CGD_HEX_LDS_ZC", str(zc))
    f4, st4 = cgd.coarse_grain(mesh, pos, vals, b, steps, rtol=1e-6, stats=True)
    dep = O.deposit_hex(p.pos, p.values, lo, hi, shape)
    ref = O.diffuse_hex_dct(dep["field64"], lo, hi, shape, b, steps)
    o = f4.cpu().numpy()
    for f in range(2):
        assert rel_l2(o[f], ref[f]) <= REL_L2, (f, rel_l2(o[f], ref[f]))
    assert st4.status == 0
    it2 = sum(sum(r) for r in st2.iters)
    it4 = sum(sum(r) for r in st4.iters)
    print(f"iterations: degree 2 {st2.iters}, degree {deg} {st4.iters}", flush=True)
    assert it4 < it2, (it2, it4)
    if deg >= 8:
        assert max(max(r[:2]) for r in st4.iters[:steps]) <= (3 if deg == 8 else 2), st4.iters


@pytest.mark.parametrize("shape", [(200, 160, 256), (96, 128, 320), (512, 96, 128), (300, 200, 64)])
def test_any_width_picks_lds_degree_by_default(gpu_lib, shape):
    """Rows that are not 64, 128 or 256 cells wide (200 cells at 4 per lane,
    96 at 2) and rows wider than a wave covers (512, 300: solved with x and y
    exchanged, the field transposed in and out) on grids large enough to
    fill the machine: the default choice is the LDS polynomial
    preconditioner (degree 12 at dtau / h^2 = 1, 2 iterations per step, as
    on the 256-wide dense bed), and the result matches the float64 DCT
    solution."""
    import torch
    cgd = gpu_lib
    nx, ny, nz = shape
    lo, hi = (0.0, 0.0, 0.0), (nx / 256.0, ny / 256.0, nz / 256.0)
    box = inputs.HexBox(lo, hi, shape)
    p = inputs.uniform_bed(box, 1_000_000, 1, seed=78, diam=0.003)
    b, steps = 4.0 / 256.0, 4  # dtau / h^2 = 1
    print(f"case: any width default degree {shape}", flush=True)
    mesh = cgd.HexMesh(shape, lo, hi)
    out, st = cgd.coarse_grain(mesh, _t(p.pos, torch), _t(p.values, torch), b, steps, rtol=1e-6, stats=True)
    dep = O.deposit_hex(p.pos, p.values, lo, hi, shape)
    ref = O.diffuse_hex_dct(dep["field64"], lo, hi, shape, b, steps)
    assert rel_l2(out.cpu().numpy()[0], ref[0]) <= REL_L2
    print(f"iterations {st.iters}", flush=True)
    assert st.status == 0
    assert max(r[0] for r in st.iters) <= 2, st.iters


@pytest.mark.parametrize("deg", [2, 12])
def test_wide_rows_exchanged_match_oracle(gpu_lib, deg, monkeypatch):
    """Rows of 300 cells (wider than a wave covers) over 20 rows: the solve
    runs with x and y exchanged (forced degree, z chunks of 4), two fields,
    ragged 64 x 64 transpose tiles; against the float64 DCT solution, and
    against the same grid solved without the exchange (edge loads, degree 1
    sweeps) within the solver tolerance."""
    import torch
    cgd = gpu_lib
    shape = (300, 20, 17)
    lo, hi = (0.0, 0.0, 0.0), (300 / 64.0, 20 / 64.0, 17 / 64.0)
    box = inputs.HexBox(lo, hi, shape)
    p = inputs.uniform_bed(box, 60_000, 2, seed=79, diam=0.01)
    b, steps = 4.0 / 64.0, 3
    print(f"case: wide rows exchanged degree {deg}", flush=True)
    mesh = cgd.HexMesh(shape, lo, hi)
    pos, vals = _t(p.pos, torch), _t(p.values, torch)
    monkeypatch.setenv("CGD_HEX_PRECOND_DEG", str(deg))
    monkeypatch.setenv("CGD_HEX_LDS_ZC", "4")
    out, st = cgd.coarse_grain(mesh, pos, vals, b, steps, rtol=1e-7, stats=True)
    monkeypatch.setenv("CGD_HEX_NO_SWAP", "1")
    out2, st2 = cgd.coarse_grain(mesh, pos, vals, b, steps, rtol=1e-7, stats=True)
    dep = O.deposit_hex(p.pos, p.values, lo, hi, shape)
    ref = O.diffuse_hex_dct(dep["field64"], lo, hi, shape, b, steps)
    o, o2 = out.cpu().numpy(), out2.cpu().numpy()
    for f in range(2):
        assert rel_l2(o[f], ref[f]) <= REL_L2, (f, rel_l2(o[f], ref[f]))
        assert rel_l2(o2[f], ref[f]) <= REL_L2, (f, rel_l2(o2[f], ref[f]))
        m0 = (dep["field64"][f]).sum()
        assert abs(o[f].astype(np.float64).sum() - m0) <= 1e-5 * np.abs(dep["field64"][f]).sum()
    print(f"iterations: exchanged {st.iters}, not {st2.iters}", flush=True)
    assert sum(sum(r) for r in st.iters) < sum(sum(r) for r in st2.iters)


@pytest.mark.parametrize("precond", [0, 1])
def test_repeated_calls_with_iteration_budgets(gpu_lib, precond, monkeypatch):
    """A coarse-graining call with the parameters of the previous one on the
    mesh enqueues the iterations that call took per step without read-backs:
    plus one, and exactly those once two budgeted calls in a row have taken
    them (the step's last test then made after its last iteration, summed in
    the order of the kernel that would have made it).  Bit for bit the same
    fields, iteration counts and residuals as the call with read-backs
    (CGD_NO_BUDGET), both when the budget suffices (the same
    input again, with and without the spare iteration) and when it does not
    (a rougher input after the smooth ones, with no spare iteration left:
    the call goes round again with read-backs, and the spare iteration
    comes back for the calls after it, until twice as many calls in a row
    have repeated the counts)."""
    import torch
    cgd = gpu_lib
    shape = (64, 48, 40)
    lo, hi = (0.0, 0.0, 0.0), (1.0, 0.75, 0.625)
    box = inputs.HexBox(lo, hi, shape)
    smooth = inputs.uniform_bed(box, 400_000, 2, seed=81, diam=0.01)
    rough = inputs.uniform_bed(box, 3_000, 2, seed=82, diam=0.01)
    b, steps = 4.0 / 64.0, 4
    print(f"case: iteration budgets precond {precond}", flush=True)

    def run(p, budget):
        if budget:
            monkeypatch.delenv("CGD_NO_BUDGET", raising=False)
        else:
            monkeypatch.setenv("CGD_NO_BUDGET", "1")
        out, st = cgd.coarse_grain(mesh, _t(p.pos, torch), _t(p.values, torch), b, steps, rtol=1e-6, stats=True,
                                   precond=precond)
        return out.cpu().numpy(), [list(r) for r in st.iters], st.status, [list(r) for r in st.rel_res]

    mesh = cgd.HexMesh(shape, lo, hi)
    ref_s = run(smooth, False)
    ref_r = run(rough, False)
    mesh.close()
    mesh = cgd.HexMesh(shape, lo, hi)
    first = run(smooth, True)            # learns the budgets
    again = run(smooth, True)            # within them, one spare iteration per step
    steady = [run(smooth, True) for _ in range(3)]  # the counts repeat: no spare iteration from the third
    after = run(rough, True)             # beyond them (more iterations): the call is redone with read-backs
    back = [run(smooth, True) for _ in range(6)]  # a spare iteration again, none from the sixth
    after2 = run(rough, True)            # beyond them again
    for got, ref in ((first, ref_s), (again, ref_s), *((x, ref_s) for x in steady), (after, ref_r),
                     *((x, ref_s) for x in back), (after2, ref_r)):
        assert np.array_equal(got[0].view(np.uint32), ref[0].view(np.uint32))
        assert got[1] == ref[1] and got[2] == ref[2] == 0
        assert got[3] == ref[3]  # float64 relative residuals, exactly
    print(f"iterations: smooth {ref_s[1]}, rough {ref_r[1]}", flush=True)
    if precond == 1:  # plain CG: the rough input takes more iterations, so its call ran out of budget
        assert sum(map(sum, ref_r[1])) > sum(map(sum, ref_s[1])) + steps

