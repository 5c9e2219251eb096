"""GPU parity of the unstructured (tet) path against the CPU oracle.

Point location and deposition are bit-exact (cell ids, int64 sums, float32
fields); the diffused field is within relative L2 1e-5 of the float64 oracle
at sizes the oracle solves directly.  At the full 100^3 x 6 mesh the check is
per step, through properties that hold at any size: the residual of each
backward-Euler solve in the oracle's own float64 operator, and the error that
residual leaves, found by solving the error equation in float64.
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
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("order", ["spatial", "input"])
@pytest.mark.parametrize("n_hex,jitter", [(6, 0.2), (9, 0.0)])
def test_locate_and_deposit_bit_exact(gpu_lib, n_hex, jitter, order, monkeypatch):
    """Location and deposition bit for bit against the oracle, with the
    particles taken in a coarse spatial order (the default from 4,096
    particles) and in input order."""
    import torch
    cgd = gpu_lib
    if order == "input":
        monkeypatch.setenv("CGD_TET_INPUT_ORDER", "1")
    xyz, tets = inputs.kuhn_tet_mesh(n_hex, jitter, seed=51)
    rng = np.random.default_rng(52)
    pos = rng.random((20_000, 3)).astype(np.float32)
    # on vertices, on the hex grid planes, on the main diagonal and outside
    pos[:50] = xyz[rng.integers(0, len(xyz), 50)].astype(np.float32)
    pos[50:100, 0] = np.float32(0.5)
    pos[100:150, 1] = pos[100:150, 0]
    pos[150:155] = [[1.5, 0.5, 0.5], [-0.1, 0.2, 0.3], [0.5, 0.5, 2.0], [np.nan, 0.1, 0.1], [0.2, np.inf, 0.3]]
    vals = np.stack([np.full(len(pos), 3.3e-8, np.float32), rng.normal(size=len(pos)).astype(np.float32)])
    print(f"case: tet {n_hex}^3x6 jitter {jitter} {order} order", flush=True)
    mesh = cgd.TetMesh(xyz, tets)
    assert mesh.cells == len(tets)
    P, N, _ = O.tet_faces(tets)
    assert mesh.nnz == len(tets) + 2 * len(P)
    cell = cgd.locate(mesh, _t(pos, torch)).cpu().numpy()
    ref_cell = O.locate_tets(xyz, tets, pos.astype(np.float64))
    assert np.array_equal(cell, ref_cell)
    acc = torch.empty((2, mesh.cells), dtype=torch.int64, device="cuda")
    field, st = cgd.deposit(mesh, _t(pos, torch), _t(vals, torch), acc=acc, stats=True)
    ref = O.deposit_tet(xyz, tets, pos, vals, cells=ref_cell)
    assert st.n_dropped == ref["n_dropped"]
    assert st.frac_bits[:2] == ref["S"]
    assert np.array_equal(acc.cpu().numpy(), ref["acc"])
    assert np.array_equal(field.cpu().numpy().view(np.uint32), ref["field32"].view(np.uint32))


def test_locate_non_convex_mesh_bit_exact(gpu_lib):
    """An L-shaped mesh (the Kuhn tets of hexes with x > 1/2 and y > 1/2
    removed): walks that leave the mesh through the notch fall back to the
    exhaustive test; points in the notch are outside."""
    import torch
    cgd = gpu_lib
    n = 8
    xyz, tets = inputs.kuhn_tet_mesh(n, 0.2, seed=55)
    cen = xyz[tets].mean(axis=1)
    keep = ~((cen[:, 0] > 0.5) & (cen[:, 1] > 0.5))
    tets = np.ascontiguousarray(tets[keep])
    used = np.unique(tets)
    remap = -np.ones(len(xyz), dtype=np.int64)
    remap[used] = np.arange(len(used))
    xyz = np.ascontiguousarray(xyz[used])
    tets = remap[tets].astype(np.int32)
    rng = np.random.default_rng(56)
    pos = rng.random((20_000, 3)).astype(np.float32)
    pos[:40] = xyz[rng.integers(0, len(xyz), 40)].astype(np.float32)
    print("case: tet L-shaped 8^3x6", flush=True)
    mesh = cgd.TetMesh(xyz, tets)
    cell = cgd.locate(mesh, _t(pos, torch)).cpu().numpy()
    ref = O.locate_tets(xyz, tets, pos.astype(np.float64))
    assert np.array_equal(cell, ref)
    assert (ref < 0).sum() > 3000  # the notch is a quarter of the box


@pytest.mark.parametrize("n_hex,jitter,steps", [(8, 0.2, 4), (5, 0.0, 2), (12, 0.2, 1)])
def test_coarse_grain_tet_matches_oracle(gpu_lib, n_hex, jitter, steps):
    import torch
    cgd = gpu_lib
    xyz, tets = inputs.kuhn_tet_mesh(n_hex, jitter, seed=53)
    rng = np.random.default_rng(54)
    pos = rng.random((30_000, 3)).astype(np.float32)
    vals = np.stack([np.full(len(pos), 3.3e-8, np.float32), rng.normal(size=len(pos)).astype(np.float32)])
    b = 4.0 / n_hex
    print(f"case: tet coarse_grain {n_hex}^3x6 jitter {jitter} steps {steps}", flush=True)
    mesh = cgd.TetMesh(xyz, tets)
    out, st = cgd.coarse_grain(mesh, _t(pos, torch), _t(vals, torch), b, steps, rtol=1e-7, stats=True)
    dep = O.deposit_tet(xyz, tets, pos, vals)
    ref = O.diffuse_tet(dep["field64"], xyz, tets, b, steps, solver="direct")
    o = out.cpu().numpy()
    V, _ = O.tet_volumes(xyz, tets)
    for f in range(2):
        assert rel_l2(o[f], ref[f]) <= REL_L2, (f, rel_l2(o[f], ref[f]))
        # conservation (eq. conserve) up to the solver tolerance
        m0 = (dep["field64"][f] * V).sum()
        assert abs(st.mass_after[f] - m0) <= 1e-5 * np.abs(dep["field64"][f] * V).sum()
    assert st.status == 0


@pytest.mark.parametrize("deg", ["0", "2", "8", "16"])
@pytest.mark.parametrize("scheme", ["be", "cn"])
def test_tet_polynomial_degrees_match_oracle(gpu_lib, deg, scheme, monkeypatch):
    """The Chebyshev polynomial preconditioner of the Jacobi-scaled operator
    at forced degrees (0: Jacobi) on 6,000 jittered tets (23 full blocks of
    rows and a ragged one), two fields, both schemes, against the oracle's
    direct solve; mass conserved."""
    import torch
    cgd = gpu_lib
    n_hex, steps = 10, 3
    xyz, tets = inputs.kuhn_tet_mesh(n_hex, 0.2, seed=57)
    rng = np.random.default_rng(58)
    pos = rng.random((20_000, 3)).astype(np.float32)
    vals = np.stack([np.full(len(pos), 3.3e-8, np.float32), rng.normal(size=len(pos)).astype(np.float32)])
    b = 4.0 / n_hex
    print(f"case: tet polynomial degree {deg} {scheme}", flush=True)
    mesh = cgd.TetMesh(xyz, tets)
    monkeypatch.setenv("CGD_TET_DEGREE", deg)
    out, st = cgd.coarse_grain(mesh, _t(pos, torch), _t(vals, torch), b, steps, rtol=1e-7, stats=True,
                               scheme=scheme)
    dep = O.deposit_tet(xyz, tets, pos, vals)
    ref = O.diffuse_tet(dep["field64"], xyz, tets, b, steps, solver="direct", scheme=scheme)
    o = out.cpu().numpy()
    V, _ = O.tet_volumes(xyz, tets)
    for f in range(2):
        assert rel_l2(o[f], ref[f]) <= REL_L2, (f, rel_l2(o[f], ref[f]))
        m0 = (dep["field64"][f] * V).sum()
        assert abs(st.mass_after[f] - m0) <= 1e-5 * np.abs(dep["field64"][f] * V).sum()
    assert st.status == 0
    assert max(max(r) for r in st.rel_res) <= 1e-7, st.rel_res
    # more degree, fewer iterations (a float64 model of the same CG on this
    # mesh takes 71 / 26 / 9 / 5 at dtau / h^2 = 4/3, 52 / 19 / 7 / 4 at 2/3)
    its = max(max(r) for r in st.iters)
    assert its <= {"0": 100, "2": 36, "8": 13, "16": 8}[deg], st.iters


@pytest.mark.parametrize("precond,scheme", [(0, "be"), (1, "be"), (0, "cn")])
def test_tet_repeated_calls_with_iteration_budgets(gpu_lib, precond, scheme, monkeypatch):
    """A repeated coarse-graining call on a tet mesh enqueues the previous
    call's iterations per step without read-backs (plus one until the
    counts repeat; the last iteration leaves out the next preconditioner,
    whose first pass would only make the step end's check).  Fields,
    iteration counts and residuals are bit for bit those of the calls with
    read-backs (CGD_NO_BUDGET), under the polynomial and Jacobi, whether the
    budget suffices or a rougher input runs out of it and is redone."""
    import torch
    cgd = gpu_lib
    xyz, tets = inputs.kuhn_tet_mesh(12, 0.2, seed=63)
    rng = np.random.default_rng(64)
    smooth = rng.random((200_000, 3)).astype(np.float32)
    rough = rng.random((300, 3)).astype(np.float32)
    vs = np.full((1, len(smooth)), 2.0e-7, np.float32)
    vr = rng.normal(size=(1, len(rough))).astype(np.float32)
    b, steps = 4.0 / 12, 3
    print(f"case: tet iteration budgets precond={precond} {scheme}", flush=True)

    def run(mesh, p, v, budget):
        if budget:
            monkeypatch.delenv("CGD_NO_BUDGET", raising=False)
        else:
            monkeypatch.setenv("CGD_NO_BUDGET", "1")
        out, st = cgd.coarse_grain(mesh, _t(p, torch), _t(v, torch), b, steps, rtol=1e-7, stats=True,
                                   precond=precond, scheme=scheme)
        return out.cpu().numpy(), [list(r) for r in st.iters], st.status, [list(r) for r in st.rel_res]

    mesh = cgd.TetMesh(xyz, tets)
    ref_s = run(mesh, smooth, vs, False)
    ref_r = run(mesh, rough, vr, False)
    mesh.close()
    mesh = cgd.TetMesh(xyz, tets)
    calls = [(run(mesh, smooth, vs, True), ref_s) for _ in range(5)]
    calls.append((run(mesh, rough, vr, True), ref_r))
    calls += [(run(mesh, smooth, vs, True), ref_s) for _ in range(6)]
    calls.append((run(mesh, rough, vr, True), ref_r))
    for got, ref in calls:
        assert np.array_equal(got[0].view(np.uint32), ref[0].view(np.uint32))
        assert got[1] == ref[1] and got[2] == ref[2] == 0
        assert got[3] == ref[3]
    print(f"iterations: smooth {ref_s[1]}, rough {ref_r[1]}", flush=True)


def test_tet_default_preconditioner_iterations(gpu_lib):
    """162,000 jittered tets at dtau / h^2 = 1 (the unstructured workload's
    ratio), rtol 1e-6: the default polynomial preconditioner takes at most 12
    iterations per step where Jacobi takes over 40, and both fields agree
    with the oracle's float64 CG to 1e-5."""
    import torch
    cgd = gpu_lib
    n_hex, steps = 30, 4
    xyz, tets = inputs.kuhn_tet_mesh(n_hex, 0.2, seed=59)
    rng = np.random.default_rng(60)
    pos = rng.random((400_000, 3)).astype(np.float32)
    vals = np.full((1, len(pos)), 3.3e-8, np.float32)
    b = 4.0 / n_hex
    print("case: tet default preconditioner 30^3x6", flush=True)
    mesh = cgd.TetMesh(xyz, tets)
    out, st = cgd.coarse_grain(mesh, _t(pos, torch), _t(vals, torch), b, steps, rtol=1e-6, stats=True)
    jac, sj = cgd.coarse_grain(mesh, _t(pos, torch), _t(vals, torch), b, steps, rtol=1e-6, stats=True,
                               precond=1)
    dep = O.deposit_tet(xyz, tets, pos, vals)
    ref = O.diffuse_tet(dep["field64"], xyz, tets, b, steps, solver="cg", rtol=1e-11)
    print(f"iterations: polynomial {st.iters}, Jacobi {sj.iters}", flush=True)
    assert max(r[0] for r in st.iters) <= 12, st.iters
    assert min(r[0] for r in sj.iters) >= 40, sj.iters
    # each step's statistics land in its own row: the recorded residual of
    # every step meets rtol, and a step's count matches a one-step call
    assert max(r[0] for r in st.rel_res) <= 1e-6 and max(r[0] for r in sj.rel_res) <= 1e-6, (st.rel_res,
                                                                                              sj.rel_res)
    field, _ = cgd.deposit(mesh, _t(pos, torch), _t(vals, torch), stats=True)
    _, s1 = cgd.diffuse(mesh, field, b / np.sqrt(steps), 1, rtol=1e-6, stats=True)
    assert s1.iters[0] == st.iters[0] and s1.rel_res[0] == st.rel_res[0], (s1, st)
    assert rel_l2(out.cpu().numpy()[0], ref[0]) <= REL_L2
    assert rel_l2(jac.cpu().numpy()[0], ref[0]) <= REL_L2
    assert st.status == 0 and sj.status == 0


@pytest.mark.parametrize("precond", [0, 1])
@pytest.mark.parametrize("scheme", ["be", "cn"])
def test_tet_cellwise_diffusivity_matches_oracle(gpu_lib, precond, scheme):
    """Section 5.2's local diffusion constant on tets: D = 0 in the tets
    whose centroid has x < 0.25 (PCM there) and D = 1 + 3 [y > 0.5] elsewhere
    (a fourfold jump), the face flux scaled by the harmonic mean of the two
    tets' D.  Against the oracle's direct solve with the same D, under the
    default polynomial preconditioner and Jacobi, both schemes; frozen tets
    keep their deposited values and the total is conserved."""
    import torch
    cgd = gpu_lib
    n_hex, steps = 9, 3
    xyz, tets = inputs.kuhn_tet_mesh(n_hex, 0.2, seed=61)
    c = xyz[tets].mean(axis=1)
    frozen = c[:, 0] < 0.25
    D = np.where(frozen, 0.0, 1.0 + 3.0 * (c[:, 1] > 0.5)).astype(np.float32)
    rng = np.random.default_rng(62)
    pos = rng.random((25_000, 3)).astype(np.float32)
    vals = np.stack([np.full(len(pos), 3.3e-8, np.float32), rng.normal(size=len(pos)).astype(np.float32)])
    b = 4.0 / n_hex
    print(f"case: tet diffusivity precond={precond} {scheme}", flush=True)
    mesh = cgd.TetMesh(xyz, tets, diffusivity=D)
    out, st = cgd.coarse_grain(mesh, _t(pos, torch), _t(vals, torch), b, steps, rtol=1e-7, stats=True,
                               precond=precond, scheme=scheme)
    dep = O.deposit_tet(xyz, tets, pos, vals)
    ref = O.diffuse_tet(dep["field64"], xyz, tets, b, steps, solver="direct", scheme=scheme,
                        diffusivity=D.astype(np.float64))
    o = out.cpu().numpy()
    V, _ = O.tet_volumes(xyz, tets)
    assert frozen.sum() > 0
    for f in range(2):
        assert rel_l2(o[f], ref[f]) <= REL_L2, (f, rel_l2(o[f], ref[f]))
        pcm = dep["field64"][f][frozen]
        assert np.abs(o[f][frozen] - pcm).max() <= 1e-5 * np.abs(dep["field64"][f]).max()
        m0 = (dep["field64"][f] * V).sum()
        assert abs(st.mass_after[f] - m0) <= 1e-5 * np.abs(dep["field64"][f] * V).sum()
    assert st.status == 0
    # D = 1 everywhere: the same mesh as without a diffusivity, bit for bit
    if precond == 0 and scheme == "be":
        m1 = cgd.TetMesh(xyz, tets, diffusivity=np.ones(len(tets), np.float32))
        m0 = cgd.TetMesh(xyz, tets)
        a1, _ = cgd.coarse_grain(m1, _t(pos, torch), _t(vals, torch), b, steps, rtol=1e-7, stats=True)
        a0, _ = cgd.coarse_grain(m0, _t(pos, torch), _t(vals, torch), b, steps, rtol=1e-7, stats=True)
        assert torch.equal(a1.view(torch.int32), a0.view(torch.int32))
    for bad in (-1.0, float("nan"), float("inf")):
        Db = D.copy()
        Db[3] = bad
        with pytest.raises(cgd.CgdError):
            cgd.TetMesh(xyz, tets, diffusivity=Db)
    # D = 0 everywhere: no face carries flux, every tet keeps its deposited
    # value (the degenerate operator M, solved without a polynomial)
    if precond == 0 and scheme == "be":
        mz = cgd.TetMesh(xyz, tets, diffusivity=np.zeros(len(tets), np.float32))
        oz, sz = cgd.coarse_grain(mz, _t(pos, torch), _t(vals, torch), b, steps, rtol=1e-7, stats=True)
        assert sz.status == 0
        for f in range(2):
            d = dep["field64"][f]
            assert np.abs(oz.cpu().numpy()[f] - d).max() <= 1e-6 * np.abs(d).max()


def test_tet_invalid_meshes(gpu_lib):
    cgd = gpu_lib
    xyz, tets = inputs.kuhn_tet_mesh(2, 0.0)
    bad = tets.copy()
    bad[3, [1, 2]] = bad[3, [2, 1]]  # negative orientation
    with pytest.raises(cgd.CgdError):
        cgd.TetMesh(xyz, bad)
    bad = tets.copy()
    bad[0, 0] = len(xyz)  # vertex id out of range
    with pytest.raises(cgd.CgdError):
        cgd.TetMesh(xyz, bad)
    with pytest.raises(cgd.CgdError):
        cgd.TetMesh(xyz, np.concatenate([tets, tets[:1]]))  # a face shared by three tets


def _check_location_by_definition(xyz, tets, pos, cell):
    """Checks a located cell for every particle against the definition of
    point location (the oracle's point_in_tets predicate: each face's float64
    orientation on its vertices in increasing id order; inside means no face
    puts the point strictly on the far side; lowest id on ties), vectorised
    over (particle, cell) pairs:
      - the cell contains the particle;
      - a particle strictly inside its cell (every face value at least 1e-9
        of the opposite vertex's, far beyond float64 rounding) lies in no
        other tet of a conforming mesh, so the cell is the lowest containing id;
      - the rest, near a face, edge or vertex, are located again by the
        oracle's own search and must agree.
    Returns the mask of particles near a face."""
    xyz = np.asarray(xyz, dtype=np.float64)
    T = np.asarray(tets, dtype=np.int64)[cell]
    p = np.asarray(pos, dtype=np.float64)
    assert O.point_in_tets(xyz, tets, p, cell).all()
    margin = np.full(len(p), np.inf)
    for opp, (i, j, k) in enumerate(((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2))):
        f = np.sort(T[:, [i, j, k]], axis=1)
        a, b, c = xyz[f[:, 0]], xyz[f[:, 1]], xyz[f[:, 2]]
        sp_ = O._orient(a, b, c, p)
        sd = O._orient(a, b, c, xyz[T[:, opp]])
        margin = np.minimum(margin, sp_ * np.sign(sd) / np.abs(sd))
    assert (margin >= 0).all()
    near = margin < 1e-9
    if near.any():
        assert np.array_equal(cell[near], O.locate_tets(xyz, tets, p[near]))
    return near


def test_unstructured_full_size_per_step_residuals(gpu_lib):
    """The unstructured workload at full size: 100^3 hexes x 6 jittered tets,
    5M particles, b = 0.04, 4 steps, CG rtol 1e-6 with the default
    (polynomial) preconditioner."""
    import scipy.sparse as sp
    import torch
    cgd = gpu_lib
    xyz, tets, parts, b, steps, rtol = inputs.unstructured()
    print("case: unstructured 6M tets, 5M particles", flush=True)
    mesh = cgd.TetMesh(xyz, tets)
    pos = _t(parts.pos, torch)
    vals = _t(parts.values, torch)
    # point location of every particle against the definition (the lowest
    # id among the tets whose closed set contains the centroid)
    cell = cgd.locate(mesh, pos).cpu().numpy()
    assert (cell >= 0).all()
    near = _check_location_by_definition(xyz, tets, parts.pos, cell)
    print(f"{int(near.sum())} particles near a face located by the oracle's search", flush=True)
    sample = np.random.default_rng(55).choice(len(parts.pos), 1000, replace=False)
    ref_cell = O.locate_tets(xyz, tets, parts.pos[sample].astype(np.float64))
    assert np.array_equal(cell[sample], ref_cell)
    # deposition: the oracle's fixed-point sums over the cells just shown to
    # be the definition's, bit for bit
    acc = torch.empty((1, mesh.cells), dtype=torch.int64, device="cuda")
    field, st = cgd.deposit(mesh, pos, vals, acc=acc, stats=True)
    want, S = O.deposit_cells(cell, cell >= 0, parts.values, mesh.cells)
    assert st.frac_bits[0] == S[0]
    assert np.array_equal(acc.cpu().numpy(), want)
    # diffusion one step at a time (b / 2 per call gives the same dtau)
    K, V = O.tet_tpfa(xyz, tets)
    dtau = b * b / 4.0 / steps
    A = (sp.diags(V) + dtau * K).tocsr()
    e = field.cpu().numpy()[0].astype(np.float64)
    for s in range(steps):
        _, st = cgd.diffuse(mesh, field, b / np.sqrt(steps), 1, rtol=rtol, stats=True)
        x = field.cpu().numpy()[0].astype(np.float64)
        rhs = V * e
        r = rhs - A @ x
        res = np.linalg.norm(r) / np.linalg.norm(rhs)
        # the solver meets rtol on its float32 operator; the float64 residual
        # also carries the float32 rounding of A and b (cell volumes span 27x)
        assert res <= 20 * rtol, (s, res)
        # error of this step's solve: A d = r solved in float64 (30 CG
        # iterations fix d to far better than the 1e-5 being tested)
        d, _ = O.cg(A, r, rtol=1e-4, maxiter=60)
        assert np.linalg.norm(d) / np.linalg.norm(x) <= REL_L2, (s, np.linalg.norm(d) / np.linalg.norm(x))
        assert abs((V * x).sum() - (V * e).sum()) <= 1e-5 * (V * np.abs(e)).sum()
        e = x
