/*
 * cgd.h - C-ABI of libcgd: diffusion-based coarse graining on MI355X (gfx950).
 *
 * The method (Sun & Xiao, "Diffusion-based coarse graining in hybrid
 * continuum-discrete solvers", Section 2.6): particle quantities are first
 * deposited into the mesh cells that contain the particle centroids (the
 * particle centroid method, Section 2.2, eq. pcm-k); the resulting cell field
 * is then diffused for a pseudo-time T = b^2 / 4 (Section 3.2.1: with this T
 * the heat kernel equals the Gaussian kernel of bandwidth b, eq. hi) with
 * zero-flux walls (Section 3.2.2).  Diffusion is integrated here by n equal
 * backward-Euler pseudo-steps, each an implicit solve of the finite-volume
 * Laplacian system (M + dtau K) e^{n+1} = M e^n (Section 5.1 describes the
 * spatial discretisation; the paper integrates with Crank-Nicolson).
 *
 * Conventions shared by every entry point:
 *  - All particle and field arrays are DEVICE pointers owned by the caller;
 *    the library never frees them.  Positions are float32 [n, 3] (x, y, z
 *    interleaved); per-particle values are float32 [F, n]; cell fields are
 *    float32 [F, cells].  Hex cells are numbered x fastest:
 *    k = ix + nx * (iy + ny * iz).  Tet cells follow the caller's tet order.
 *  - A cell field is a density: the value summed over the cell's particles
 *    divided by the cell volume, so sum_k field_k V_k = sum_p value_p
 *    (eq. conserve).
 *  - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL is the
 *    default stream) on the device the mesh was created on.
 *  - Arguments are validated on the host before anything is enqueued; a
 *    negative status means nothing was written.  No C++ exception or abort
 *    crosses this boundary.  cgd_last_error() gives a text for the last
 *    failing call on the calling thread.
 *  - A mesh must not be used by two calls at the same time (it owns the
 *    workspace the calls use).
 */
#ifndef CGD_H
#define CGD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cgd_status;

#define CGD_OK                  0
#define CGD_NOT_CONVERGED       1   /* a solve hit max_iter; result = last iterate */
#define CGD_WARMSTART_FALLBACK  2   /* a learned initial guess was rejected; zero guess used */
#define CGD_E_INVALID          -1   /* bad argument (null, size, shape, b <= 0, n_steps < 1 ...) */
#define CGD_E_NONFINITE        -2   /* NaN/Inf among positions or values (those particles skipped) */
#define CGD_E_NOMEM            -3   /* device or pinned-host allocation failed */
#define CGD_E_HIP              -4   /* a HIP runtime call failed; cgd_last_error() has its text */
#define CGD_E_BREAKDOWN        -5   /* CG breakdown: p.Ap <= 0 or a non-finite scalar */
#define CGD_E_UNSUPPORTED      -6   /* operation not available for this mesh kind */

#define CGD_MAX_FIELDS 16
#define CGD_MAX_STEPS  64

typedef struct cgd_mesh_s* cgd_mesh;

/* Uniform hex mesh of the box [lo, hi] with nx * ny * nz cells: the CFD mesh
 * that the centroid deposit bins on and the diffusion equation is solved on
 * (Section 3.1, eq. pcm-k; zero-flux walls on all six faces, Section 3.2.2;
 * the uniform meshes of Section 4).  lo, hi are host arrays of 3 doubles,
 * hi > lo.
 * The mesh lives on the current HIP device.  Returns CGD_E_INVALID for
 * non-positive sizes or an empty box. */
cgd_status cgd_mesh_create_hex(int32_t nx, int32_t ny, int32_t nz,
                               const double lo[3], const double hi[3], cgd_mesh* out);

/* Tetrahedral mesh (Section 2.1 item 4: arbitrary unstructured meshes).
 * xyz: host float64 [n_vert, 3]; tv: host int32 [n_tet, 4] vertex ids, each
 * tet with positive orientation det[v1-v0, v2-v0, v3-v0] > 0 (checked:
 * CGD_E_INVALID otherwise).  Builds on the host, once: tet volumes, the
 * two-point-flux Laplacian a_f = |A_f| / |c_N - c_P| over interior faces
 * (boundary faces carry no flux), stored per tet in its four face slots
 * (float32 a_f, int32 id of the tet across the face, which also serves point
 * location): a sparse matrix with rows padded to four off-diagonal entries;
 * and a point-location grid;
 * then copies them to the device.  Every face must be shared by at most two
 * tets (CGD_E_INVALID otherwise). */
cgd_status cgd_mesh_create_tet(int64_t n_vert, const double* xyz,
                               int64_t n_tet, const int32_t* tv, cgd_mesh* out);

/* Tetrahedral mesh with a cell-wise diffusivity (Section 5.2: a small local
 * diffusion constant, e.g. 0 where the cells are large, so that PCM applies
 * there while mass stays conserved).  As cgd_mesh_create_tet, with each
 * interior face's coefficient a_f = D_f |A_f| / |c_N - c_P|, D_f the
 * harmonic mean 2 D_P D_N / (D_P + D_N) of the two tets' diffusivities (0
 * when either is 0: a tet with D = 0 exchanges nothing and keeps its
 * deposited value), in float64, rounded once.  diffusivity: host float32
 * [n_tet], finite and >= 0 (else CGD_E_INVALID), or NULL for 1 everywhere
 * (then the same mesh as cgd_mesh_create_tet). */
cgd_status cgd_mesh_create_tet_d(int64_t n_vert, const double* xyz, int64_t n_tet, const int32_t* tv,
                                 const float* diffusivity, cgd_mesh* out);

/* Stretched (rectilinear) hex mesh with a cell-wise diffusivity (Section
 * 4.3: stretched meshes; Section 5.2: a small local diffusion constant
 * degenerates the method to PCM there, conservation kept).  x_edges, y_edges,
 * z_edges: host float64 node coordinates, nx + 1, ny + 1, nz + 1 of them,
 * finite and strictly increasing; cells are numbered x fastest.
 * diffusivity: host float32 [nx * ny * nz], finite and >= 0, or NULL for 1.
 * A particle goes to the cell with e_i <= x < e_{i+1} on each axis (the
 * upper cell at an interior face, the last cell on the upper wall; outside
 * the closed box: dropped); the cell density divides by the cell's own
 * volume.  The operator is the finite-volume Laplacian with flux
 * D_f A_f / d_f (e_P - e_N) through each interior face (A_f the face area,
 * d_f the distance between the two cell centres, D_f the harmonic mean of
 * the two cells' diffusivities, 0 if either is 0), solved by
 * preconditioned CG (x0_mode 0).  When the diffusivity factors as
 * D(i,j,k) = Dx(i) Dy(j) Dz(k) (checked to 1e-6 relative at creation; NULL
 * counts) the operator is kept as per-axis factor arrays and applied by
 * stencil sweeps, with a Chebyshev polynomial preconditioner on a scaled
 * operator where one wave covers an x-row (nx <= 256), Jacobi on wider rows;
 * a periodic x axis there also needs the row in one segment of waves
 * (nx <= 64, or up to 128 / 256 with 8 / 16-byte aligned fields).  Otherwise
 * the operator is stored like the tet operator with six face slots per row
 * and solved by CG with the tet path's polynomial preconditioner.  periodic: bit a set makes axis a
 * (0 x, 1 y, 2 z) periodic (Section 3.1): its first and last cells share a
 * face at distance (h_first + h_last) / 2 instead of two walls (no effect on
 * an axis of one cell); binning is unchanged.  nx * ny * nz < 2^28, else
 * CGD_E_INVALID. */
cgd_status cgd_mesh_create_rect(int32_t nx, int32_t ny, int32_t nz, const double* x_edges,
                                const double* y_edges, const double* z_edges, const float* diffusivity,
                                int32_t periodic, cgd_mesh* out);

void    cgd_mesh_destroy(cgd_mesh m);
int64_t cgd_mesh_num_cells(cgd_mesh m);
/* 0 = hex, 1 = tet, 2 = rectilinear hex, -1 = NULL mesh */
int32_t cgd_mesh_kind(cgd_mesh m);
/* Tet and rectilinear meshes: number of non-zeros of M + dtau K, cells + 2 x
 * interior faces (0 for uniform hex). */
int64_t cgd_mesh_nnz(cgd_mesh m);

/* Learned initial-guess network (cgd_unet_create below). */
typedef struct cgd_unet_s* cgd_unet;

typedef struct {
    double  rtol;         /* stop when ||r||_2 <= rtol ||b||_2 (per field, per step); <= 0: 1e-6 */
    int32_t max_iter;     /* per step; <= 0: 1000 */
    int32_t x0_mode;      /* 0: zero initial guess; 1: previous pseudo-step's solution;
                             2: caller's guess x0 for the first step (zero after);
                             3: the network `model`'s prediction from the previous
                                pseudo-step's field, every step (hex meshes) */
    const float* x0;      /* device [F, cells] when x0_mode == 2, else NULL */
    int32_t check_every;  /* iterations enqueued between convergence read-backs once a step
                             runs past the previous solve's count; <= 0: 4 */
    int32_t precond;      /* hex meshes: 0 (default) conjugate gradients preconditioned by
                             a Chebyshev polynomial of A on its spectrum [1, 1 + 4 sum_a c_a]:
                             degree 4, 8 or 12 (one Horner sweep; two or three sweeps of two
                             quadratic factors each), the one with the least work predicted
                             from the Chebyshev bound on the iteration count, where one
                             wavefront covers an x-row (nx = 64, 128 or 256) and the grid
                             fills the machine, else degree 2 or 1; 1 plain CG.  Tet meshes
                             and the face-slot rows of rectilinear meshes: 0 CG
                             preconditioned by the Chebyshev polynomial of even degree
                             0..16 (0: Jacobi) of the Jacobi-scaled operator with the least
                             predicted work, on the spectrum estimate [sum V / sum diag,
                             1 + t / (1 + t)], t = dtau max K_ii / V_i (face coefficients
                             rounded to float16 in the preconditioner only); 1 Jacobi.  The
                             stopping rule is the same for all. */
    cgd_unet model;       /* x0_mode 3: a network created for this mesh's grid, else NULL */
    int32_t scheme;       /* pseudo-time integrator (Section 5.1): 0 (default) backward Euler,
                             each step solving (M + dtau K) e^{n+1} = M e^n; 1 Crank-Nicolson,
                             (M + dtau/2 K) e^{n+1} = (M - dtau/2 K) e^n, computed as the
                             half-step solve (M + dtau/2 K) y = M e^n (same solvers, stopping
                             rule on y) followed by e^{n+1} = 2 y - e^n (on hex meshes from
                             a zero guess the CG's x updates carry it).  Crank-Nicolson
                             conserves mass but, unlike backward Euler, is not positivity
                             preserving at large dtau / h^2.  Other values: CGD_E_INVALID. */
} cgd_solver_opts;

typedef struct {
    int32_t n_steps, n_fields;
    int32_t iters[CGD_MAX_STEPS][CGD_MAX_FIELDS];     /* CG iterations per step and field */
    double  rel_res[CGD_MAX_STEPS][CGD_MAX_FIELDS];   /* recursive ||r|| / ||b|| at exit */
    double  mass_before[CGD_MAX_FIELDS];              /* sum_k V_k field_k before diffusion */
    double  mass_after[CGD_MAX_FIELDS];               /* ... and after (equal up to rtol) */
    int32_t frac_bits[CGD_MAX_FIELDS];                /* fixed-point scale S used by deposit */
    int64_t n_dropped;                                /* particles outside the mesh / non-finite */
    int64_t n_nonfinite;                              /* non-finite positions or values */
    int32_t status;
    int32_t n_fallback;                               /* x0_mode 3: (step, field) solves whose
                                                         learned guess was rejected */
} cgd_solve_stats;

/* Centroid binning alone (the first half of cgd_deposit): the host cell of
 * each particle, i.e. the hex cell index (rule of cgd_deposit) or the lowest
 * id among the tets containing the centroid, and -1 when the position is not
 * finite or lies outside the mesh.
 *  pos:  device float32 [n, 3]
 *  cell: device int32 [n], written
 * Asynchronous on `stream`. */
cgd_status cgd_locate(cgd_mesh m, int64_t n, const float* pos, int32_t* cell, void* stream);

/* Particle centroid method (Section 2.2, eq. pcm-k), bit-exact.
 *
 * Each particle p with a finite position inside the closed mesh domain is
 * assigned to the cell containing its centroid (hex: i_a = floor((x_a - lo_a)
 * * s_a), s_a = N_a / (hi_a - lo_a) in float64, clamped to [0, N_a - 1]; a
 * point on an interior face goes to the upper cell; tet: the containing tet,
 * lowest id on ties).  Its value v of field f is quantised to
 * q = rint(v * 2^S_f) (int64, round half to even) with S_f = 62 - e_max - e_N
 * (max_p |v_p| <= 2^e_max over finite values, e_N = ceil(log2 n)), so that no
 * sum can overflow, or with a scale S_f the caller forces, and summed in
 * int64: the sums are exact and independent of particle order (eq.
 * conserve holds exactly in the integers).  Then
 * field[f, k] = float32(acc * 2^-S_f / V_k).  On hex meshes (and
 * rectilinear ones of at most 4093 cells over the three axes) the particles
 * are bucketed by tile of consecutive cells and each tile is summed in LDS
 * (the temporary buffers, 12 bytes per particle at F = 1, 20 at F = 2 or 3
 * and 20 + 4 (F - 3) above, come from the mesh workspace); with more than
 * 16384 tiles (of 16384 / F cells, a power of two) or 2^32 particles, or
 * CGD_DEPOSIT_DIRECT set in the
 * environment, every particle is added with a device-wide int64 atomic
 * instead.  Both give the same bits.  On tet meshes every particle is added
 * with a device-wide int64 atomic after its walk to the host tet; from 4,096
 * particles the walks are taken in a coarse spatial order (a counting sort
 * by blocks of the point-location buckets: 8 bytes per particle plus
 * per-block key histograms, from the mesh workspace; CGD_TET_INPUT_ORDER
 * set: input order), which changes no bit of the result.
 *
 *  n:       number of particles (>= 0)
 *  pos:     device float32 [n, 3]
 *  F:       number of fields, 1..CGD_MAX_FIELDS
 *  values:  device float32 [F, n]
 *  field:   device float32 [F, cells], written
 *  acc:     device int64 [F, cells] (written: the raw fixed-point sums) or NULL
 *  frac_bits: host int32 [F] or NULL (all automatic).  In: -1 for the
 *           automatic S_f above, or a scale 0..62 to force (other values:
 *           CGD_E_INVALID, nothing enqueued).  A forced scale is the caller's
 *           promise that |v| 2^S_f < 2^62 for every value and that every
 *           cell's sum of |q| stays below 2^63; the library does not check it
 *           (beyond it the int64 sums wrap).  Out: the scale used per field;
 *           when any entry was -1 the call waits for the stream to read it.
 *  st:      host, nullable.  Non-NULL makes the call wait for the stream and
 *           fill frac_bits / n_dropped / n_nonfinite; the call then returns
 *           CGD_E_NONFINITE if any non-finite position or value was seen.
 *           With st == NULL the call does not report them and non-finite
 *           particles are skipped silently; with st == NULL and no
 *           automatic scale requested through frac_bits it is asynchronous. */
cgd_status cgd_deposit(cgd_mesh m, int64_t n, const float* pos, int32_t F,
                       const float* values, float* field, int64_t* acc,
                       int32_t* frac_bits, cgd_solve_stats* st, void* stream);

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, serving loops that must not call hipMalloc, harnesses that forbid
 * it): cgd_deposit on a uniform hex mesh, with the same kernels, results and
 * automatic fixed-point scales, but its temporary buffers in one
 * library-owned device array of 64 MiB per GPU (held until the process
 * ends) instead of the mesh's workspace; it calls no hipMalloc, hipFree or
 * other allocating routine.
 *  n, pos, F, values, field, acc, stream: as in cgd_deposit (acc nullable;
 *           no statistics, no forced scales; the call is asynchronous).
 *  Limits: the tiled deposit's scratch, 12 bytes per particle at F = 1
 *           (20 at F = 2 or 3, 20 + 4 (F - 3) above) plus
 *           12 bytes per tile of 16384 / F cells, must fit 64 MiB - 4 KiB
 *           (about 5.5M particles at F = 1, 2.8M at F = 4), and the grid at
 *           most 16384 tiles; larger inputs return CGD_E_INVALID with the
 *           sizes in cgd_last_error(), and other mesh kinds CGD_E_UNSUPPORTED,
 *           before anything is enqueued.
 *  Every call on a GPU uses that GPU's one array: calls that overlap on the
 *  same GPU (from any stream, thread or mesh) race and must be ordered by
 *  the caller.  Each call re-initialises what it reads. */
cgd_status cgd_deposit_noalloc(cgd_mesh m, int64_t n, const float* pos, int32_t F,
                               const float* values, float* field, int64_t* acc, void* stream);

/* Diffusion of F cell fields in place (Sections 3.1, 3.2, 5.1).
 *
 * T = bandwidth^2 / 4, dtau = T / n_steps; each of the n_steps backward-Euler
 * steps solves (M + dtau K) e^{n+1} = M e^n by conjugate gradients with float32
 * vectors and float64 inner products (hex: matrix-free 7-point stencil with a
 * polynomial preconditioner, see cgd_solver_opts.precond; tet: A p from the face
 * slots in flux form, a polynomial of the Jacobi-scaled operator as preconditioner).  Zero-flux walls: wall faces carry
 * no flux.  Fields are independent solves (Section 3.2.1: each component is
 * diffused on its own).
 *
 *  field:     device float32 [F, cells], in: deposited field, out: diffused field
 *  bandwidth: Gaussian-kernel bandwidth b > 0 in domain length units
 *  n_steps:   1..CGD_MAX_STEPS
 *  o:         solver options, nullable (defaults)
 *  st:        host, nullable: iteration counts, residuals, mass before/after
 *
 * The convergence test is read back one chunk of iterations late, so the
 * device always has queued work: the first chunk of a step runs to the
 * iteration at which the previous solve on this mesh stopped, the next holds
 * one iteration, later ones o->check_every iterations (all of them
 * o->check_every before a first solve).  The call returns to the host about
 * when the last step has converged.  Returns
 * CGD_NOT_CONVERGED if some solve hit max_iter (result = last iterate) and
 * CGD_E_BREAKDOWN on a breakdown. */
cgd_status cgd_diffuse(cgd_mesh m, int32_t F, float* field, double bandwidth,
                       int32_t n_steps, const cgd_solver_opts* o,
                       cgd_solve_stats* st, void* stream);

/* cgd_deposit followed by cgd_diffuse (Section 2.6): the whole method.
 * field: device float32 [F, cells], written.
 * From a zero guess (x0_mode 0), a call with the arguments of the
 * previous one on the mesh (grid, F, bandwidth, n_steps, max_iter, rtol,
 * precond, scheme) enqueues each step's iterations of that call, plus one
 * until two such calls in a row have taken the same counts (twice as many
 * after each call that ran out without the extra one, up to 64), with no
 * read-back between steps; if a step runs out, the call goes round again
 * with read-backs.  Fields, counts and statistics are those of the call with
 * read-backs either way (environment CGD_NO_BUDGET turns this off). */
cgd_status cgd_coarse_grain(cgd_mesh m, int64_t n, const float* pos, int32_t F,
                            const float* values, double bandwidth, int32_t n_steps,
                            const cgd_solver_opts* o, float* field,
                            cgd_solve_stats* st, void* stream);

/* Momentum-consistent velocity (Section 6: the diffusion acts on the
 * momentum, not on the velocity).  Coarse grain F = 1 + n_comp fields
 * (particle volume, then volume times each velocity component) and divide:
 * mom[c][k] = mom[c][k] / eps[k] where eps[k] > eps_min, else 0 (one float32
 * division, correctly rounded).
 *  cells:  cells of the fields; n_comp: 1..CGD_MAX_FIELDS - 1
 *  eps:    device float32 [cells], the diffused solid volume fraction
 *  mom:    device float32 [n_comp, cells], in: diffused eps U; out: U
 *  eps_min: finite, >= 0
 * Enqueued on `stream`; CGD_E_INVALID for bad sizes or null pointers. */
cgd_status cgd_velocity_from_momentum(int64_t cells, int32_t n_comp, const float* eps, float* mom,
                                      float eps_min, void* stream);

/* Batched coarse graining of n_snap independent snapshots on one hex mesh
 * (each snapshot its own particles; F fields each, e.g. solid volume plus
 * three drag components), each field diffused on its own (Section 3.2.1).
 *
 * Deposition follows cgd_deposit per snapshot (its own fixed-point scale per
 * snapshot and field).  All n_snap * F right-hand sides are then solved from
 * a zero initial guess by CG preconditioned with a Chebyshev polynomial of
 * the operator (o->precond = 1: plain CG), with float32 vectors, float64
 * inner products, and the stencil and stopping rule of cgd_diffuse, by the
 * candidate cgd_autotune_batched chose (run automatically on first use):
 *  - ONE persistent launch in which each workgroup solves its share of the
 *    right-hand sides one after the other, at a tile shape and a polynomial
 *    degree of 2, 4 or 12 (nx = 64, 128 or 256); or
 *  - the launches of cgd_diffuse over groups of up to CGD_MAX_FIELDS
 *    right-hand sides (any nx; degree 12 where its LDS sweep applies), each
 *    step with a fixed budget of iterations: the most any right-hand side
 *    took in the run that made the graph.  A replay that leaves a right-hand
 *    side above the tolerance is followed by the same call with read-backs
 *    of the convergence state, so every result meets the stopping rule.
 * The whole call (offset upload, deposit, solve, statistics read-back) is
 * captured in a hipGraph for a given argument set and replayed afterwards
 * (the per-launch candidate first runs once with read-backs to learn its
 * budgets).
 *
 *  n_snap:  1.. ; n_snap * F <= 4096
 *  offsets: HOST int64 [n_snap + 1]; snapshot j owns particles
 *           offsets[j] .. offsets[j+1]-1; offsets[0] = 0, non-decreasing
 *  pos:     device float32 [offsets[n_snap], 3]
 *  values:  device float32 [F, offsets[n_snap]]
 *  fields:  device float32 [n_snap, F, cells], written
 *  o:       rtol / max_iter / precond / scheme as in cgd_diffuse; x0_mode must be 0
 *  st:      HOST cgd_solve_stats [n_snap] or NULL: per snapshot, as cgd_coarse_grain
 *           reports for one call: CG iterations and ||r|| / ||b|| per step and
 *           field, mass before and after diffusion per field (sum_k V field_k,
 *           float64; their difference is bounded by the stopping rule), the
 *           fixed-point scale of each field, dropped and non-finite particles,
 *           and the snapshot's worst status (n_fallback 0).  Asking for st adds
 *           two float64 sums over all fields to the launch.
 * Uniform hex meshes only (CGD_E_UNSUPPORTED otherwise).  The call waits
 * for its stream before returning. */
cgd_status cgd_coarse_grain_batched(cgd_mesh m, int32_t n_snap, const int64_t* offsets,
                                    const float* pos, int32_t F, const float* values,
                                    double bandwidth, int32_t n_steps, const cgd_solver_opts* o,
                                    float* fields, cgd_solve_stats* st, void* stream);

/* Autotuner of the batched solver: times each candidate solving n_rhs
 * synthetic right-hand sides for one backward-Euler step at dtau / h^2 = 1
 * to rtol 1e-6, and keeps the fastest for this mesh shape (also appended to
 * the file named by the environment variable CGD_AUTOTUNE_CACHE, when set,
 * and read from it).  Candidates: where nx is 64, 128 or 256, indices 0..7
 * are the persistent launch (rows per wave, waves per workgroup and
 * preconditioner degree 2, 2, 2, 2, 4, 4, 12, 12); the last index is the
 * per-launch solver over groups of right-hand sides.
 *  chosen: host, written with the chosen candidate index
 *  ms:     host double [16] or NULL: time of each candidate (forces a re-run)
 *  n_cand: host, written with the number of candidates (nullable) */
cgd_status cgd_autotune_batched(cgd_mesh m, int32_t n_rhs, int32_t* chosen, double* ms, int32_t* n_cand);

/* ------------------------------------------------------------------------
 * Learned initial guess (an addition to the method, not in the paper).
 *
 * A three-level 3-D convolutional U-Net f that maps the field of one
 * backward-Euler pseudo-step to an estimate of the next, f(e^n) ~ e^{n+1}
 * (Section 3.2: every step solves the same system, so one network serves all
 * steps).  With cgd_solver_opts.x0_mode = 3, cgd_diffuse seeds each step's
 * CG solve with f(e^n); the solve and its stopping rule are unchanged, so
 * the result is the same discrete solution, only reached in fewer
 * iterations when the guess is good.  A guess whose residual is not finite
 * or exceeds ||b|| is rejected and the step starts from zero (counted in
 * cgd_solve_stats.n_fallback; the call then returns CGD_WARMSTART_FALLBACK
 * unless something worse happened).
 *
 * Architecture (base width 16, zero padding, ReLU after each 3x3x3 conv):
 * two convs per level at 16 / 32 / 64 channels, 2x2x2 average pooling down,
 * nearest 2x upsampling + conv up, skip connections by channel
 * concatenation, a 1x1x1 head, and a residual output
 *   y = x + s * head(U(x / s)),  s = sqrt(mean(x^2)).
 * Activations and weights in bfloat16 on the matrix cores with float32
 * accumulation; master weights, gradients, Adam state and loss in float32 /
 * float64.  Every reduction runs in a fixed order (deterministic training).
 *
 * Parameters, flat float32, in this order: for each conv layer (e1a, e1b,
 * e2a, e2b, e3a, e3b, u2, d2a, d2b, u1, d1a, d1b) its weights [co][27][ci]
 * (tap = (dz+1)*9 + (dy+1)*3 + (dx+1), a cross-correlation) then its biases
 * [co]; then the head's 16 weights and its bias.
 * The network lives on the device current at creation and owns its
 * activations; a network must not be used by two calls at the same time.
 * ---------------------------------------------------------------------- */

/* nx, ny, nz: the hex grid the network works on, each a multiple of 4.
 * Weights He-normal from `seed` (splitmix64 + Box-Muller), biases zero and
 * head zero, so the untrained network returns its input. */
cgd_status cgd_unet_create(int32_t nx, int32_t ny, int32_t nz, uint64_t seed, cgd_unet* out);
void       cgd_unet_destroy(cgd_unet u);
int64_t    cgd_unet_num_params(cgd_unet u);
/* Host float32 [n] copies of the parameters (set resets the Adam state) and
 * of the gradient of the last cgd_unet_loss_grad / cgd_unet_train_step.
 * These wait for the device. */
cgd_status cgd_unet_get_params(cgd_unet u, float* host, int64_t n);
cgd_status cgd_unet_set_params(cgd_unet u, const float* host, int64_t n);
cgd_status cgd_unet_get_grads(cgd_unet u, float* host, int64_t n);
/* y = f(x); x, y: device float32 [nz][ny][nx] (one field).  Asynchronous. */
cgd_status cgd_unet_forward(cgd_unet u, const float* x, float* y, void* stream);
/* Loss mean((f(x) - target)^2) / s^2 and its gradient with respect to the
 * parameters (kept on the device; cgd_unet_get_grads copies it out).
 * loss: host, nullable; non-NULL makes the call wait for the stream. */
cgd_status cgd_unet_loss_grad(cgd_unet u, const float* x, const float* target, double* loss, void* stream);
/* cgd_unet_loss_grad followed by one Adam step (beta1 0.9, beta2 0.999,
 * eps 1e-8, learning rate lr > 0) on the float32 master weights. */
cgd_status cgd_unet_train_step(cgd_unet u, const float* x, const float* target, double lr, double* loss,
                               void* stream);

/* Single 3x3x3 convolutions with zero padding on caller buffers, the kernels
 * the network runs (bfloat16 tensors passed as uint16_t bit patterns,
 * channels last: x [nz][ny][nx][ci]; weights [co][27][ci]):
 *   forward: y = conv(x, w) + bias (bias nullable), ReLU when relu != 0;
 *            ci in {1, 16, 32, 64}, co in {16, 32, 64}
 *   dgrad:   dx = gradient of sum(g * conv(x, w)) with respect to x;
 *            ci, co in {16, 32, 64}
 *   wgrad:   dw [co][27][ci] and db [co] (float32) of sum(g * (conv(x, w) + b))
 * These allocate scratch memory and wait for the stream. */
cgd_status cgd_conv3_forward(int32_t nx, int32_t ny, int32_t nz, int32_t ci, int32_t co, const uint16_t* x,
                             const uint16_t* w, const float* bias, int32_t relu, uint16_t* y, void* stream);
cgd_status cgd_conv3_dgrad(int32_t nx, int32_t ny, int32_t nz, int32_t ci, int32_t co, const uint16_t* g,
                           const uint16_t* w, uint16_t* dx, void* stream);
cgd_status cgd_conv3_wgrad(int32_t nx, int32_t ny, int32_t nz, int32_t ci, int32_t co, const uint16_t* x,
                           const uint16_t* g, float* dw, float* db, void* stream);

/* Kernel timing, for roofline measurement.  While enabled, each launch of the
 * timed kernels is bracketed by two HIP events recorded on the caller's
 * stream (events without a system-scope fence, so that timing stalls the
 * queue as little as possible); the elapsed times are collected when the
 * call synchronises (every cgd_diffuse / cgd_coarse_grain does at its end).
 * Kinds (one kernel each unless stated):
 *   0  CG sweep 1 (p = z + beta p_old, A p, p.Ap), hex stencil
 *   1  CG sweep 2 (x += alpha p, r -= alpha A p, r.r), hex stencil
 *   2  whole deposit: centroid binning, bucketing and fixed-point sums
 *      (all kernels of a call; kinds 13..15 split the tiled hex path)
 *   3  matrix sweep of the CG on face slots (p, A p, p.Ap)
 *   4  update sweep of the CG on face slots (x, r, z = D^-1 r or v = H r, r.r)
 *   5  hex preconditioning, degree-4 Horner pass or first product pass
 *      (r -> U), degree 1 / 2 register sweep
 *   6  hex preconditioning, middle product pass (U -> V, degree 12)
 *   7  hex preconditioning, last product pass (V -> z, r.z)
 *   8  first iteration of a step, direction sweep (p.Ap with p = z)
 *   9  first iteration of a step, update sweep (x = alpha p, r = b - alpha A p)
 *  10  first iteration, kind 5's pass reading b (b.b as well)
 *  11  first iteration, kind 6's pass
 *  12  first iteration, kind 7's pass
 *  13  tiled hex deposit: binning and tile counts
 *  14  tiled hex deposit: prefix sum and scatter of records into tiles
 *  15  tiled hex deposit: fixed-point sums in LDS and the finished field
 *  16  tet / face-slot polynomial preconditioning, pass w = B v
 *  17  tet / face-slot polynomial preconditioning, pass v = g (B w + s w + q v)
 *      (the last pass of each application also sums r.z)
 * bytes_per_launch is the algorithmic byte count of the last timed launch of
 * that kind (what the method must move, not what the hardware moved). */
#define CGD_TIMING_KINDS 18
typedef struct {
    int64_t launches[CGD_TIMING_KINDS];
    double  total_ms[CGD_TIMING_KINDS];
    double  bytes_per_launch[CGD_TIMING_KINDS];
} cgd_kernel_timing;

cgd_status cgd_timing_enable(cgd_mesh m, int32_t on);
/* Copies the accumulated timings to *out; reset != 0 clears them. */
cgd_status cgd_timing_read(cgd_mesh m, cgd_kernel_timing* out, int32_t reset);

const char* cgd_status_string(cgd_status s);
const char* cgd_last_error(void);
/* Library version as an integer (major * 10000 + minor * 100 + patch). */
int32_t     cgd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CGD_H */
