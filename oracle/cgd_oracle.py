"""CPU FP64 oracle for diffusion-based coarse graining (Sun & Xiao).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this module: only the tests, the smoke check and the benchmark's CPU-baseline
leg use it.  It shares no code with the HIP library (no kernels, helpers,
constants or pre/post-processing); both sides only receive the same seeded
inputs.

What it computes, step by step, in float64 (Section 2.6, "Overview of
Proposed Diffusion-Based Coarse Graining Method", and Section 3.1):

1. particle centroid method (Section 2.2, eq. pcm-k): each particle's value
   goes to the cell that contains its centroid; the cell value is the sum
   divided by the cell volume.  Sums are taken in 64-bit fixed point so that
   they are exact and order-free (conservation, eq. conserve).
2. diffusion of that field for pseudo-time T = b^2/4 (Section 3.2.1: the
   Green's function of the unit-diffusivity heat equation at time T equals
   the Gaussian kernel of eq. hi with b = sqrt(4T)), with zero-flux walls
   (Section 3.2.2), discretised by the second-order central finite-volume
   Laplacian (Section 5.1) and integrated by backward Euler in n equal
   pseudo-steps, or by the paper's Crank-Nicolson scheme (Section 5.1).

Readings of points the paper leaves open (each has a line in the design
notes): backward Euler by default, Crank-Nicolson as an option; T split into
equal steps; the system is taken in symmetric form (M + dtau K) x = M eps;
ties at cell faces go to the upper cell, points on the upper wall to the
last cell; out-of-box or non-finite particles are not deposited.

Second routes kept here as pins for the first (they share nothing with it):
the DCT-II closed form of the same discrete problem on uniform hex grids,
the Thomas algorithm in 1-D, and the Gaussian kernel of eqs. superpo/hi with
the image kernels of eqs. hi-bound / wall-ext for axis-aligned boxes.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.special import erf

# ---------------------------------------------------------------------------
# 1. Particle centroid method on a uniform hex grid (Section 2.2, eq. pcm-k)
# ---------------------------------------------------------------------------


def hex_spacing(lo, hi, shape):
    """Cell widths h_a = (hi_a - lo_a) / N_a, float64."""
    return tuple((float(hi[a]) - float(lo[a])) / int(shape[a]) for a in range(3))


def hex_cell_volume(lo, hi, shape):
    """V_c = h_x * h_y * h_z, evaluated left to right in float64."""
    hx, hy, hz = hex_spacing(lo, hi, shape)
    return (hx * hy) * hz


def bin_hex(pos, lo, hi, shape):
    """Host cell of each centroid (Section 2.2: the cell the centroid falls in).

    u_a = (x_a - lo_a) * s_a with s_a = N_a / (hi_a - lo_a); i_a = floor(u_a),
    clamped to [0, N_a - 1] for points on the closed box's faces.  Returns
    (cell index int64 with x fastest, mask of deposited particles,
    number of non-finite particles).  Points outside the closed box and
    non-finite points are not deposited.
    """
    x = np.asarray(pos, dtype=np.float64)
    finite = np.isfinite(x).all(axis=1)
    inside = finite.copy()
    idx = []
    for a in range(3):
        lo_a, hi_a, n_a = float(lo[a]), float(hi[a]), int(shape[a])
        s_a = n_a / (hi_a - lo_a)
        xa = np.where(finite, x[:, a], lo_a)
        inside &= (xa >= lo_a) & (xa <= hi_a)
        u = (xa - lo_a) * s_a
        i = np.floor(u)
        i = np.clip(i, 0, n_a - 1).astype(np.int64)
        idx.append(i)
    nx, ny, _ = shape
    cell = idx[0] + nx * (idx[1] + ny * idx[2])
    return cell, inside, int((~finite).sum())


def frac_bits(values_row, n_particles):
    """Fixed-point scale S for one field: S = 62 - e_max - e_N.

    max |v| <= 2^e_max (frexp exponent), e_N = ceil(log2 N).  Then the sum of
    all |q| = |rint(v 2^S)| stays below 2^62, so int64 sums never overflow.
    All-zero values give S = 0.  Non-finite values are left out of the max
    (they are not deposited).
    """
    v = np.asarray(values_row, dtype=np.float64)
    v = v[np.isfinite(v)]
    m = float(np.max(np.abs(v))) if v.size else 0.0
    if m == 0.0:
        return 0
    _, e_max = math.frexp(m)
    e_n = 0 if n_particles <= 1 else int(math.ceil(math.log2(n_particles)))
    return 62 - e_max - e_n


def quantise(values_row, S):
    """q = rint(v * 2^S), round half to even, as int64 (exact scaling)."""
    return np.rint(np.ldexp(np.asarray(values_row, dtype=np.float64), S)).astype(np.int64)


def deposit_cells(cell, mask, values, n_cells, force_bits=None):
    """Fixed-point PCM sums: acc[f, k] = sum over particles in cell k of q_f.

    Returns (acc int64 [F, n_cells], S list).  Integer sums: exact, so the
    result does not depend on the particle order (eq. conserve holds exactly
    in the integers).  A particle whose value of field f is not finite is
    left out of field f.  force_bits: None, or per field a scale to use
    instead of frac_bits (None or -1 in an entry: the automatic one).
    """
    values = np.atleast_2d(values)
    F, n = values.shape
    acc = np.zeros((F, n_cells), dtype=np.int64)
    Ss = []
    for f in range(F):
        forced = None if force_bits is None else force_bits[f]
        S = frac_bits(values[f], n) if forced is None or forced < 0 else int(forced)
        Ss.append(S)
        sel = np.nonzero(mask & np.isfinite(values[f]))[0]
        q = quantise(values[f, sel], S)
        np.add.at(acc[f], cell[sel], q)
    return acc, Ss


def finalise(acc, S, volume):
    """eps_k = (acc_k * 2^-S) / V_k in float64 (eq. pcm-k), and its float32 rounding."""
    f64 = np.ldexp(acc.astype(np.float64), -S) / volume
    return f64, f64.astype(np.float32)


def deposit_hex(pos, values, lo, hi, shape, force_bits=None):
    """Particle centroid method on a uniform hex grid.

    Returns dict with acc [F, cells] int64, S per field, field64 / field32
    [F, cells] (densities: sum of values in the cell over the cell volume),
    and counts of dropped / non-finite particles.  force_bits: see
    deposit_cells.
    """
    values = np.atleast_2d(values)
    nx, ny, nz = shape
    cell, mask, n_nonfinite = bin_hex(pos, lo, hi, shape)
    acc, Ss = deposit_cells(cell, mask, values, nx * ny * nz, force_bits)
    V = hex_cell_volume(lo, hi, shape)
    f64 = np.empty(acc.shape, dtype=np.float64)
    f32 = np.empty(acc.shape, dtype=np.float32)
    for f in range(acc.shape[0]):
        f64[f], f32[f] = finalise(acc[f], Ss[f], V)
    return dict(acc=acc, S=Ss, field64=f64, field32=f32, cell=cell, mask=mask,
                n_dropped=int((~mask).sum()), n_nonfinite=n_nonfinite)


# ---------------------------------------------------------------------------
# 2. Finite-volume Laplacian with zero-flux walls (Sections 3.2.2, 5.1)
# ---------------------------------------------------------------------------


def hex_laplacian(shape, lo, hi):
    """K with (K e)_k = sum over interior faces f of k of (A_f / d_f)(e_k - e_nb).

    Central two-point flux between cell centres; wall faces carry no flux
    (zero-gradient Neumann condition), so they add nothing.  K is symmetric
    and its columns sum to zero.  Cells are numbered x fastest.
    """
    nx, ny, nz = shape
    hx, hy, hz = hex_spacing(lo, hi, shape)
    areas = (hy * hz, hx * hz, hx * hy)
    dists = (hx, hy, hz)
    n = nx * ny * nz
    idx = np.arange(n).reshape(nz, ny, nx)
    rows, cols, vals = [], [], []
    diag = np.zeros(n)
    for a, (sl_lo, sl_hi) in enumerate((
            ((slice(None), slice(None), slice(0, -1)), (slice(None), slice(None), slice(1, None))),
            ((slice(None), slice(0, -1), slice(None)), (slice(None), slice(1, None), slice(None))),
            ((slice(0, -1), slice(None), slice(None)), (slice(1, None), slice(None), slice(None))))):
        coef = areas[a] / dists[a]
        p = idx[sl_lo].ravel()
        q = idx[sl_hi].ravel()
        rows += [p, q]
        cols += [q, p]
        vals += [np.full(p.size, -coef), np.full(q.size, -coef)]
        np.add.at(diag, p, coef)
        np.add.at(diag, q, coef)
    rows.append(np.arange(n))
    cols.append(np.arange(n))
    vals.append(diag)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def pseudo_time(bandwidth):
    """T = b^2 / 4, from b = sqrt(4T) (Section 3.2.1)."""
    return bandwidth * bandwidth / 4.0


def cg(A, b, rtol=1e-12, maxiter=10000, x0=None):
    """Textbook conjugate gradients in float64 (Hestenes-Stiefel).

    Stops when ||r||_2 <= rtol ||b||_2.  Returns (x, iterations).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x
    bnorm = math.sqrt(float(b @ b))
    if bnorm == 0.0:
        return np.zeros_like(b), 0
    p = r.copy()
    rr = float(r @ r)
    for it in range(1, maxiter + 1):
        Ap = A @ p
        alpha = rr / float(p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        rr_new = float(r @ r)
        if math.sqrt(rr_new) <= rtol * bnorm:
            return x, it
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, maxiter


def backward_euler(M_diag, K, eps0, T, n_steps, solver="cg", rtol=1e-12):
    """n_steps backward-Euler steps of dtau = T / n_steps for M de/dtau = -K e.

    Each step solves (M + dtau K) e^{n+1} = M e^n.  eps0 is [cells] or
    [F, cells]; returns the same shape in float64.
    """
    dtau = T / n_steps
    A = (sp.diags(M_diag) + dtau * K).tocsr()
    eps = np.atleast_2d(np.asarray(eps0, dtype=np.float64)).copy()
    lu = spla.splu(A.tocsc()) if solver == "direct" else None
    for f in range(eps.shape[0]):
        e = eps[f]
        for _ in range(n_steps):
            rhs = M_diag * e
            e = lu.solve(rhs) if lu is not None else cg(A, rhs, rtol)[0]
        eps[f] = e
    return eps.reshape(np.shape(eps0))


def crank_nicolson(M_diag, K, eps0, T, n_steps, solver="cg", rtol=1e-12):
    """n_steps Crank-Nicolson steps of dtau = T / n_steps for M de/dtau = -K e
    (the paper's time integrator, Section 5.1).

    Each step solves (M + dtau/2 K) e^{n+1} = (M - dtau/2 K) e^n, the
    trapezoidal rule in pseudo-time.  Shapes as in backward_euler.
    """
    dtau = T / n_steps
    Md = sp.diags(M_diag)
    A = (Md + (0.5 * dtau) * K).tocsr()
    B = (Md - (0.5 * dtau) * K).tocsr()
    eps = np.atleast_2d(np.asarray(eps0, dtype=np.float64)).copy()
    lu = spla.splu(A.tocsc()) if solver == "direct" else None
    for f in range(eps.shape[0]):
        e = eps[f]
        for _ in range(n_steps):
            rhs = B @ e
            e = lu.solve(rhs) if lu is not None else cg(A, rhs, rtol)[0]
        eps[f] = e
    return eps.reshape(np.shape(eps0))


def _integrator(scheme):
    if scheme == "be":
        return backward_euler
    if scheme == "cn":
        return crank_nicolson
    raise ValueError(f"scheme must be 'be' or 'cn', not {scheme!r}")


def diffuse_hex(field, lo, hi, shape, bandwidth, n_steps, solver="cg", rtol=1e-12, scheme="be"):
    """Diffuse cell fields [F, cells] on the hex grid for T = b^2/4
    (scheme "be": backward Euler, "cn": Crank-Nicolson)."""
    n = shape[0] * shape[1] * shape[2]
    V = hex_cell_volume(lo, hi, shape)
    K = hex_laplacian(shape, lo, hi)
    return _integrator(scheme)(np.full(n, V), K, field, pseudo_time(bandwidth), n_steps, solver, rtol)


def coarse_grain_hex(pos, values, lo, hi, shape, bandwidth, n_steps, solver="cg", rtol=1e-12, scheme="be"):
    """Full method on a uniform hex grid: PCM, then n_steps pseudo-steps."""
    dep = deposit_hex(pos, values, lo, hi, shape)
    out = diffuse_hex(dep["field64"], lo, hi, shape, bandwidth, n_steps, solver, rtol, scheme)
    return out, dep


# ---------------------------------------------------------------------------
# Stretched (rectilinear) hex grids with a cell-wise diffusivity (Sections 4.2
# and 5.2: stretched meshes; a small local diffusion constant degenerates the
# method to PCM there while keeping conservation)
# ---------------------------------------------------------------------------


def rect_bin(pos, edges):
    """Host cell on a rectilinear grid (Section 2.2): along each axis the
    index i with e_i <= x < e_{i+1} (the upper cell at an interior face), a
    point on the upper wall in the last cell.  edges: three increasing float64
    arrays of N_a + 1 node coordinates.  Returns (cell int64 with x fastest,
    mask of deposited particles, number of non-finite particles); points
    outside the closed box and non-finite points are not deposited."""
    x = np.asarray(pos, dtype=np.float64)
    finite = np.isfinite(x).all(axis=1)
    inside = finite.copy()
    idx = []
    for a in range(3):
        e = np.asarray(edges[a], dtype=np.float64)
        n_a = len(e) - 1
        xa = np.where(finite, x[:, a], e[0])
        inside &= (xa >= e[0]) & (xa <= e[-1])
        i = np.searchsorted(e, xa, side="right") - 1
        idx.append(np.clip(i, 0, n_a - 1).astype(np.int64))
    nx, ny = len(edges[0]) - 1, len(edges[1]) - 1
    cell = idx[0] + nx * (idx[1] + ny * idx[2])
    return cell, inside, int((~finite).sum())


def rect_volumes(edges):
    """V_ijk = hx_i * hy_j * hz_k, evaluated left to right in float64 [cells]."""
    hx, hy, hz = (np.diff(np.asarray(e, dtype=np.float64)) for e in edges)
    return ((hx[None, None, :] * hy[None, :, None]) * hz[:, None, None]).ravel()


def face_diffusivity(da, db):
    """Diffusivity at the face between cells with da and db: the harmonic
    mean 2 da db / (da + db), 0 when either is 0 (no flux through a face of
    a cell that does not diffuse)."""
    da = np.asarray(da, dtype=np.float64)
    db = np.asarray(db, dtype=np.float64)
    den = da + db
    return np.where((da > 0) & (db > 0), 2.0 * da * db / np.where(den > 0, den, 1.0), 0.0)


def rect_laplacian(edges, diffusivity=None, periodic=(False, False, False)):
    """K with (K e)_k = sum over the interior faces f of k of
    D_f (A_f / d_f)(e_k - e_nb): A_f the face area, d_f the distance between
    the two cell centres, D_f = face_diffusivity of the two cells (1 when
    diffusivity is None).  Wall faces carry no flux (Section 3.2.2), except
    on a periodic axis (Section 3.1: periodic conditions there), where the
    first and last cells share a face at distance (h_first + h_last) / 2
    (for two cells on that axis, a second face between the same pair)."""
    h = [np.diff(np.asarray(e, dtype=np.float64)) for e in edges]
    nx, ny, nz = (len(v) for v in h)
    n = nx * ny * nz
    D = np.ones(n) if diffusivity is None else np.asarray(diffusivity, dtype=np.float64).ravel()
    idx = lambda i, j, k: i + nx * (j + ny * k)
    rows, cols, vals = [], [], []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                me = idx(i, j, k)
                for a, (ii, jj, kk) in enumerate(((i + 1, j, k), (i, j + 1, k), (i, j, k + 1))):
                    if ii >= nx or jj >= ny or kk >= nz:
                        if not periodic[a] or (nx, ny, nz)[a] < 2:
                            continue
                        ii, jj, kk = ii % nx, jj % ny, kk % nz  # the face across the periodic boundary
                    nb = idx(ii, jj, kk)
                    if a == 0:
                        area, dist = h[1][j] * h[2][k], 0.5 * (h[0][i] + h[0][ii])
                    elif a == 1:
                        area, dist = h[0][i] * h[2][k], 0.5 * (h[1][j] + h[1][jj])
                    else:
                        area, dist = h[0][i] * h[1][j], 0.5 * (h[2][k] + h[2][kk])
                    w = float(face_diffusivity(D[me], D[nb])) * area / dist
                    rows += [me, nb, me, nb]
                    cols += [nb, me, me, nb]
                    vals += [-w, -w, w, w]
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def deposit_rect(pos, values, edges):
    """Particle centroid method on a rectilinear grid: fixed-point sums as
    deposit_hex, divided by each cell's own volume."""
    values = np.atleast_2d(values)
    cell, mask, n_nonfinite = rect_bin(pos, edges)
    V = rect_volumes(edges)
    acc, Ss = deposit_cells(cell, mask, values, V.size)
    f64 = np.empty(acc.shape, dtype=np.float64)
    f32 = np.empty(acc.shape, dtype=np.float32)
    for f in range(acc.shape[0]):
        f64[f], f32[f] = finalise(acc[f], Ss[f], V)
    return dict(acc=acc, S=Ss, field64=f64, field32=f32, cell=cell, mask=mask,
                n_dropped=int((~mask).sum()), n_nonfinite=n_nonfinite)


def diffuse_rect(field, edges, bandwidth, n_steps, diffusivity=None, solver="cg", rtol=1e-12, scheme="be",
                 periodic=(False, False, False)):
    """Diffuse cell fields [F, cells] on a rectilinear grid for T = b^2/4
    (with the cell-wise diffusivity scaling the face fluxes)."""
    K = rect_laplacian(edges, diffusivity, periodic)
    return _integrator(scheme)(rect_volumes(edges), K, field, pseudo_time(bandwidth), n_steps, solver, rtol)


def coarse_grain_rect(pos, values, edges, bandwidth, n_steps, diffusivity=None, solver="cg", rtol=1e-12,
                      scheme="be", periodic=(False, False, False)):
    """Full method on a rectilinear grid: PCM, then n_steps pseudo-steps."""
    dep = deposit_rect(pos, values, edges)
    out = diffuse_rect(dep["field64"], edges, bandwidth, n_steps, diffusivity, solver, rtol, scheme, periodic)
    return out, dep


def velocity_from_momentum(eps, mom, eps_min):
    """Momentum-consistent velocity (Section 6: diffuse the momentum, not the
    velocity): U = (eps U) / eps for each component where eps > eps_min, 0
    elsewhere.  eps [cells] and mom [n_comp, cells] are diffused fields."""
    eps = np.asarray(eps, dtype=np.float64)
    mom = np.atleast_2d(np.asarray(mom, dtype=np.float64))
    ok = eps > eps_min
    return np.where(ok[None, :], mom / np.where(ok, eps, 1.0)[None, :], 0.0)


# ---------------------------------------------------------------------------
# Second route on uniform hex grids: DCT-II diagonalisation (closed form)
# ---------------------------------------------------------------------------


def neumann_eigenvalues(n, h):
    """Eigenvalues (4/h^2) sin^2(pi k / 2n) of the 1-D cell-centred
    zero-flux Laplacian; eigenvectors cos(pi k (i + 1/2) / n)."""
    k = np.arange(n)
    return (4.0 / (h * h)) * np.sin(np.pi * k / (2.0 * n)) ** 2


def diffuse_hex_dct(field, lo, hi, shape, bandwidth, n_steps, scheme="be"):
    """Exact result of diffuse_hex, by the DCT-II closed form.

    field [..., cells] (x fastest).  Backward Euler:
    e^n = IDCT[ DCT(e^0) (1 + dtau lam)^-n ]; Crank-Nicolson: each mode is
    multiplied by (1 - dtau lam / 2) / (1 + dtau lam / 2) per step.
    """
    from scipy.fft import dctn, idctn
    nx, ny, nz = shape
    hx, hy, hz = hex_spacing(lo, hi, shape)
    dtau = pseudo_time(bandwidth) / n_steps
    lam = (neumann_eigenvalues(nz, hz)[:, None, None] + neumann_eigenvalues(ny, hy)[None, :, None]
           + neumann_eigenvalues(nx, hx)[None, None, :])
    if scheme == "be":
        damp = (1.0 + dtau * lam) ** (-n_steps)
    elif scheme == "cn":
        damp = ((1.0 - 0.5 * dtau * lam) / (1.0 + 0.5 * dtau * lam)) ** n_steps
    else:
        raise ValueError(f"scheme must be 'be' or 'cn', not {scheme!r}")
    f = np.atleast_2d(np.asarray(field, dtype=np.float64))
    out = np.empty_like(f)
    for i in range(f.shape[0]):
        c = dctn(f[i].reshape(nz, ny, nx), type=2, norm="ortho", workers=-1)
        c *= damp
        out[i] = idctn(c, type=2, norm="ortho", workers=-1).ravel()
    return out.reshape(np.shape(field))


# ---------------------------------------------------------------------------
# 1-D: Thomas algorithm (textbook tridiagonal elimination)
# ---------------------------------------------------------------------------


def thomas(a, b, c, d):
    """Solve a tridiagonal system: a sub-diagonal (a[0] unused), b diagonal,
    c super-diagonal (c[-1] unused), right-hand side d."""
    n = len(d)
    cp = np.zeros(n)
    dp = np.zeros(n)
    cp[0] = c[0] / b[0]
    dp[0] = d[0] / b[0]
    for i in range(1, n):
        m = b[i] - a[i] * cp[i - 1]
        cp[i] = c[i] / m if i < n - 1 else 0.0
        dp[i] = (d[i] - a[i] * dp[i - 1]) / m
    x = np.zeros(n)
    x[-1] = dp[-1]
    for i in range(n - 2, -1, -1):
        x[i] = dp[i] - cp[i] * x[i + 1]
    return x


def diffuse_1d_thomas(field, length, bandwidth, n_steps, scheme="be"):
    """1-D zero-flux diffusion of a cell field by Thomas solves: backward
    Euler ("be") or Crank-Nicolson ("cn", whose right-hand side is the
    explicit half step e_i + c/2 (e_i-1 - 2 e_i + e_i+1), a missing wall
    neighbour taken as e_i)."""
    if scheme not in ("be", "cn"):
        raise ValueError(f"scheme must be 'be' or 'cn', not {scheme!r}")
    n = len(field)
    h = length / n
    c = pseudo_time(bandwidth) / n_steps / (h * h)
    ci = 0.5 * c if scheme == "cn" else c
    a = np.full(n, -ci)
    cc = np.full(n, -ci)
    b = np.full(n, 1.0 + 2.0 * ci)
    b[0] -= ci
    b[-1] -= ci
    e = np.asarray(field, dtype=np.float64).copy()
    for _ in range(n_steps):
        if scheme == "cn":
            left = np.concatenate(([e[0]], e[:-1]))
            right = np.concatenate((e[1:], [e[-1]]))
            d = e + 0.5 * c * (left - 2.0 * e + right)
        else:
            d = e
        e = thomas(a, b, cc, d)
    return e


# ---------------------------------------------------------------------------
# Gaussian kernel averaging (Section 2.5, eqs. superpo, hi, hi-bound, wall-ext)
# ---------------------------------------------------------------------------


def gaussian_kernel(r2, bandwidth):
    """h = (b^2 pi)^(-3/2) exp(-r^2 / b^2)  (eq. hi)."""
    b2 = bandwidth * bandwidth
    return (b2 * math.pi) ** -1.5 * np.exp(-np.asarray(r2) / b2)


def _images_1d(x, lo, hi, n_images, bandwidth):
    """Positions of a point and its mirror images across two parallel walls.

    Reflections across lo and hi repeated: x + 2mL and 2lo - x + 2mL for
    |m| <= n_images (orthogonal walls: eq. wall-ext truncated).  With
    n_images None, enough images are kept that every dropped one lies more
    than 7 b outside the box (its weight inside is below 1e-21)."""
    L = hi - lo
    if n_images is None:
        n_images = int(math.ceil(7.0 * bandwidth / (2.0 * L))) + 1
    out = []
    for m in range(-n_images, n_images + 1):
        out.append(x + 2 * m * L)
        out.append(2 * lo - x + 2 * m * L)
    return out


def kernel_point_values(pos, values, centres, bandwidth, box_lo=None, box_hi=None, n_images=None):
    """eps(x) = sum_i V_i h~_i(x) at the given points (eqs. superpo, hi-bound).

    With box_lo/box_hi the image kernels of the axis-aligned walls are added
    (per axis: the particle and its mirror images), so the total is conserved.
    Brute force over all particles: small inputs only.
    """
    pos = np.asarray(pos, dtype=np.float64)
    vals = np.asarray(values, dtype=np.float64)
    cen = np.asarray(centres, dtype=np.float64)
    b2 = bandwidth * bandwidth
    norm1 = (b2 * math.pi) ** -0.5
    out = np.zeros(len(cen))
    for i in range(len(pos)):
        fac = np.ones(len(cen))
        for a in range(3):
            if box_lo is None:
                srcs = [pos[i, a]]
            else:
                srcs = _images_1d(pos[i, a], box_lo[a], box_hi[a], n_images, bandwidth)
            g = np.zeros(len(cen))
            for s in srcs:
                g += norm1 * np.exp(-((cen[:, a] - s) ** 2) / b2)
            fac *= g
        out += vals[i] * fac
    return out


def kernel_cell_average_1d(x_p, edges, bandwidth, lo=None, hi=None, n_images=None):
    """Cell average of the 1-D Gaussian factor (with wall images) over cells
    [edges[k], edges[k+1]]:  (1/dx) * 1/2 [erf((a2-c)/b) - erf((a1-c)/b)]."""
    edges = np.asarray(edges, dtype=np.float64)
    srcs = [x_p] if lo is None else _images_1d(x_p, lo, hi, n_images, bandwidth)
    tot = np.zeros(len(edges) - 1)
    for c in srcs:
        e = erf((edges - c) / bandwidth)
        tot += 0.5 * (e[1:] - e[:-1])
    return tot / np.diff(edges)


def kernel_cell_average_hex(pos, values, lo, hi, shape, bandwidth, n_images=None):
    """Cell-averaged Gaussian-kernel field with wall images on a hex grid
    (the paper's benchmark in Section 5.2 is this cell integral).  The 3-D
    kernel factorises, so the cell average is a product of 1-D averages."""
    nx, ny, nz = shape
    edges = [np.linspace(lo[a], hi[a], shape[a] + 1) for a in range(3)]
    pos = np.asarray(pos, dtype=np.float64)
    vals = np.asarray(values, dtype=np.float64)
    out = np.zeros((nz, ny, nx))
    for i in range(len(pos)):
        gx = kernel_cell_average_1d(pos[i, 0], edges[0], bandwidth, lo[0], hi[0], n_images)
        gy = kernel_cell_average_1d(pos[i, 1], edges[1], bandwidth, lo[1], hi[1], n_images)
        gz = kernel_cell_average_1d(pos[i, 2], edges[2], bandwidth, lo[2], hi[2], n_images)
        out += vals[i] * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    return out.ravel()


def numerical_diffusion_gamma(eps_num, eps_ana):
    """gamma = A_diffu / A_total (Section 5.2).  Both curves carry the same
    area, so the area lost around the peak equals the area gained in the
    tails: gamma = (1/2) ||num - ana||_1 / ||ana||_1."""
    eps_num = np.asarray(eps_num, dtype=np.float64)
    eps_ana = np.asarray(eps_ana, dtype=np.float64)
    return 0.5 * np.abs(eps_num - eps_ana).sum() / np.abs(eps_ana).sum()


# ---------------------------------------------------------------------------
# Unstructured tetrahedral meshes: two-point-flux FV (Sections 2.1 item 4, 4.3)
# ---------------------------------------------------------------------------


def tet_volumes(xyz, tets):
    """|det[b - a, c - a, d - a]| / 6 per tet, float64."""
    p = np.asarray(xyz, dtype=np.float64)[np.asarray(tets)]
    e1 = p[:, 1] - p[:, 0]
    e2 = p[:, 2] - p[:, 0]
    e3 = p[:, 3] - p[:, 0]
    det = (e1[:, 0] * (e2[:, 1] * e3[:, 2] - e2[:, 2] * e3[:, 1])
           - e1[:, 1] * (e2[:, 0] * e3[:, 2] - e2[:, 2] * e3[:, 0])
           + e1[:, 2] * (e2[:, 0] * e3[:, 1] - e2[:, 1] * e3[:, 0]))
    return np.abs(det) / 6.0, det


def tet_faces(tets):
    """Interior faces as (tet P, tet N, sorted vertex triple) by matching the
    sorted vertex triples of all tet faces; boundary faces are unmatched."""
    tets = np.asarray(tets, dtype=np.int64)
    nt = len(tets)
    tri = np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]],
                          tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]])
    owner = np.tile(np.arange(nt), 4)
    tri = np.sort(tri, axis=1)
    order = np.lexsort((tri[:, 2], tri[:, 1], tri[:, 0]))
    ts = tri[order]
    same = (ts[1:] == ts[:-1]).all(axis=1)
    i = np.nonzero(same)[0]
    P = owner[order[i]]
    N = owner[order[i + 1]]
    return P, N, ts[i]


def tet_tpfa(xyz, tets, diffusivity=None):
    """Two-point-flux FV Laplacian K on a tet mesh and cell volumes.

    Interior face f between P and N: a_f = D_f |A_f| / |c_N - c_P| (face
    area over the distance between tet centroids, times the face
    diffusivity D_f = face_diffusivity(D_P, D_N), the harmonic mean of the
    two cells' diffusivities (Section 5.2's local diffusion constant); D = 1
    when diffusivity is None).  Boundary faces carry no flux.  No
    non-orthogonal correction.  Returns (K csr, V [tets]).
    """
    xyz = np.asarray(xyz, dtype=np.float64)
    V, _ = tet_volumes(xyz, tets)
    P, N, tri = tet_faces(tets)
    c = xyz[np.asarray(tets)].mean(axis=1)
    a = xyz[tri[:, 0]]
    u = xyz[tri[:, 1]] - a
    w = xyz[tri[:, 2]] - a
    area = 0.5 * np.linalg.norm(np.cross(u, w), axis=1)
    dist = np.linalg.norm(c[N] - c[P], axis=1)
    coef = area / dist
    if diffusivity is not None:
        D = np.asarray(diffusivity, dtype=np.float64)
        coef = coef * face_diffusivity(D[P], D[N])
    n = len(V)
    diag = np.zeros(n)
    np.add.at(diag, P, coef)
    np.add.at(diag, N, coef)
    K = sp.csr_matrix((np.concatenate([-coef, -coef, diag]),
                       (np.concatenate([P, N, np.arange(n)]),
                        np.concatenate([N, P, np.arange(n)]))), shape=(n, n))
    return K, V


def _orient(a, b, c, p):
    """det[b - a, c - a, p - a] in float64, one fixed expression."""
    u = b - a
    v = c - a
    w = p - a
    return (u[..., 0] * (v[..., 1] * w[..., 2] - v[..., 2] * w[..., 1])
            - u[..., 1] * (v[..., 0] * w[..., 2] - v[..., 2] * w[..., 0])
            + u[..., 2] * (v[..., 0] * w[..., 1] - v[..., 1] * w[..., 0]))


def point_in_tets(xyz, tets, p, cand):
    """Which candidate tets contain point p (inclusive of faces).

    Each face is evaluated on its vertices in increasing global-id order, so
    the two tets sharing a face compute the identical value; the opposite
    vertex's side fixes the sign.  p is inside when no face puts it strictly
    on the far side.
    """
    xyz = np.asarray(xyz, dtype=np.float64)
    T = np.asarray(tets, dtype=np.int64)[cand]
    inside = np.ones(len(cand), dtype=bool)
    for opp, (i, j, k) in enumerate(((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2))):
        f = np.sort(T[:, [i, j, k]], axis=1)
        a, b, c = xyz[f[:, 0]], xyz[f[:, 1]], xyz[f[:, 2]]
        sp_ = _orient(a, b, c, np.broadcast_to(p, a.shape))
        sd = _orient(a, b, c, xyz[T[:, opp]])
        inside &= (sp_ * np.sign(sd)) >= 0
    return inside


def locate_tets(xyz, tets, pos, bucket=None):
    """Containing tet of each point, lowest tet id on ties; -1 if none.

    Candidate tets come from a uniform bucket grid over tet bounding boxes
    (a generic search that knows nothing of how the mesh was built).
    """
    xyz = np.asarray(xyz, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int64)
    pos = np.asarray(pos, dtype=np.float64)
    lo = xyz.min(axis=0)
    hi = xyz.max(axis=0)
    nt = len(tets)
    nb = bucket or max(1, int(round((nt / 6) ** (1 / 3))))
    width = (hi - lo) / nb
    tb = xyz[tets]
    bmin = np.clip(np.floor((tb.min(axis=1) - lo) / width).astype(np.int64), 0, nb - 1)
    bmax = np.clip(np.floor((tb.max(axis=1) - lo) / width).astype(np.int64), 0, nb - 1)
    keys, owners = [], []
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                ix = bmin[:, 0] + dx
                iy = bmin[:, 1] + dy
                iz = bmin[:, 2] + dz
                ok = (ix <= bmax[:, 0]) & (iy <= bmax[:, 1]) & (iz <= bmax[:, 2])
                keys.append((ix + nb * (iy + nb * iz))[ok])
                owners.append(np.nonzero(ok)[0])
    keys = np.concatenate(keys)
    owners = np.concatenate(owners)
    order = np.lexsort((owners, keys))
    keys = keys[order]
    owners = owners[order]
    start = np.searchsorted(keys, np.arange(nb ** 3))
    end = np.searchsorted(keys, np.arange(nb ** 3), side="right")
    out = np.full(len(pos), -1, dtype=np.int64)
    pb = np.clip(np.floor((pos - lo) / width).astype(np.int64), 0, nb - 1)
    pk = pb[:, 0] + nb * (pb[:, 1] + nb * pb[:, 2])
    for i in range(len(pos)):
        cand = owners[start[pk[i]]:end[pk[i]]]
        if cand.size == 0:
            continue
        hit = point_in_tets(xyz, tets, pos[i], cand)
        if hit.any():
            out[i] = cand[hit].min()
    return out


def deposit_tet(xyz, tets, pos, values, cells=None):
    """PCM on a tet mesh: locate centroids, fixed-point sums, divide by V."""
    values = np.atleast_2d(values)
    if cells is None:
        cells = locate_tets(xyz, tets, pos)
    mask = cells >= 0
    V, _ = tet_volumes(xyz, tets)
    acc, Ss = deposit_cells(np.where(mask, cells, 0), mask, values, len(tets))
    f64 = np.empty(acc.shape)
    f32 = np.empty(acc.shape, dtype=np.float32)
    for f in range(acc.shape[0]):
        f64[f], f32[f] = finalise(acc[f], Ss[f], V)
    return dict(acc=acc, S=Ss, field64=f64, field32=f32, cell=cells,
                n_dropped=int((~mask).sum()))


def diffuse_tet(field, xyz, tets, bandwidth, n_steps, solver="cg", rtol=1e-12, scheme="be", diffusivity=None):
    """Diffusion of tet-cell fields with the TPFA Laplacian (scheme "be":
    backward Euler, "cn": Crank-Nicolson), with a cell-wise diffusivity
    scaling the face fluxes when given."""
    K, V = tet_tpfa(xyz, tets, diffusivity)
    return _integrator(scheme)(V, K, field, pseudo_time(bandwidth), n_steps, solver, rtol)
