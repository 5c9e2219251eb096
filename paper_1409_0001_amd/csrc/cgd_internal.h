// Internal declarations of libcgd (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

#include "../../include/cgd.h"
#include "hex_bin.h"

namespace cgd {

// Thread-local error text for cgd_last_error().
void set_error(const std::string& msg);

#define CGD_HIP_TRY(expr)                                                        \
    do {                                                                         \
        hipError_t e__ = (expr);                                                 \
        if (e__ != hipSuccess) {                                                 \
            ::cgd::set_error(std::string(#expr) + ": " + hipGetErrorString(e__)); \
            return CGD_E_HIP;                                                    \
        }                                                                        \
    } while (0)

// Per-field CG state kept on the device.  Each field is written only by
// the first block of a kernel and read only by later kernels (the two rr
// slots alternate by iteration parity so that a kernel never reads a slot
// its own first block is writing).
struct CgField {
    double bb;         // ||b||^2 of the current step
    double rr_par[2];  // ||r_k||^2, slot k % 2
    double rho_par[2]; // preconditioned CG: r_k . z_k, slot k % 2
    int32_t done;      // 1 once converged / stopped
    int32_t status;    // CGD_OK, CGD_NOT_CONVERGED or CGD_E_BREAKDOWN
};

// Counters the deposit kernels fill (device).
struct DepositInfo {
    uint32_t maxbits[CGD_MAX_FIELDS];       // max |v| bit pattern over finite values
    int32_t force_s[CGD_MAX_FIELDS];        // fixed-point scale set by the caller; -1: automatic
    unsigned long long nonfinite_val[CGD_MAX_FIELDS];
    unsigned long long dropped;             // non-finite or outside the domain
    unsigned long long nonfinite_pos;
};

// Fixed-point scales a deposit call is asked to use: s[f] in 0..62 forces
// S_f, -1 leaves it to the rule of frac_bits_of.
struct ScaleForce {
    int32_t s[CGD_MAX_FIELDS];
};

struct HexGeom {
    int32_t nx, ny, nz;
    double lo[3], hi[3];
    double s[3];   // N_a / (hi_a - lo_a)
    double h[3];   // (hi_a - lo_a) / N_a
    double vol;    // (h_x h_y) h_z
};

// The CG iterations each pseudo-step of a coarse-graining call from a zero
// guess took (largest over the fields), with the parameters that determine
// them; a later call with the same parameters enqueues that many iterations
// (plus one until the counts repeat) per step without reading convergence
// back between steps.
struct IterBudget {
    bool valid = false;
    int32_t F = 0, n_steps = 0, max_iter = 0, precond = 0, scheme = 0;
    double bandwidth = 0.0, rtol = 0.0;
    int32_t iters[CGD_MAX_STEPS] = {};
    int32_t repeats = 0;  // calls in a row, each budgeted, that took exactly these iterations
    int32_t steady = 2;   // repeats after which the spare iteration is dropped (doubled by each miss without it)
};

struct TetData;  // defined in tet.cpp
struct RectOp;   // below

// Event-pair timing of selected kernels (cgd_timing_enable).
struct Timing {
    bool on = false;
    std::vector<hipEvent_t> pool;          // free events
    std::vector<hipEvent_t> used;          // recorded pairs (start, end)
    std::vector<int> kinds;                // kind of each closed pair
    std::vector<int> first;                // index in `used` of each closed pair's start event
    std::vector<double> bytes;             // algorithmic bytes of each pair
    std::vector<int64_t> tags;             // caller's label of each pair
    int64_t launches[CGD_TIMING_KINDS] = {};
    double total_ms[CGD_TIMING_KINDS] = {};
    double bytes_per_launch[CGD_TIMING_KINDS] = {};
};

// Records the start event of a timed launch (no-op when timing is off).
// Returns an opaque index to pass to timing_end.
int timing_begin(Timing* t, hipStream_t s);
// tag: caller's label of the launch, passed back to the filter of timing_collect.
void timing_end(Timing* t, int idx, int kind, double bytes, hipStream_t s, int64_t tag = -1);
// Adds the elapsed times of the recorded pairs (the stream must be
// synchronised); pairs whose tag the filter rejects (launches that found
// nothing to do) are dropped.
void timing_collect(Timing* t, const std::function<bool(int64_t)>& keep = nullptr);

// Device workspace owned by a mesh, grown on demand.
struct Workspace {
    void* ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace cgd

struct cgd_mesh_s {
    int32_t kind;     // 0 hex, 1 tet
    int32_t device;
    int64_t cells;
    cgd::HexGeom hex;
    cgd::TetData* tet = nullptr;
    cgd::RectOp* rop = nullptr;    // rectilinear grids with a separable diffusivity: the sweeps' operator
    cgd::Workspace ws;
    void* pinned = nullptr;        // small pinned host buffer for read-backs
    size_t pinned_bytes = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    cgd::Timing timing;
    int32_t cg_hint = -1;          // iteration at which the last CG solve on this mesh stopped (-1: none yet)
    cgd::IterBudget budget;        // iterations per step of the last coarse-graining call
};

namespace cgd {

// Grows m->ws to at least `bytes`.  Synchronises the device before freeing.
cgd_status ensure_workspace(cgd_mesh m, size_t bytes);
cgd_status ensure_pinned(cgd_mesh m, size_t bytes);

// deposit.hip
// temp: deposit_hex_temp_bytes(m, n, F) bytes of device scratch for the tiled
// path (nullptr or 0 bytes: the direct path, which needs acc).  On the tiled
// path acc may be nullptr (the accumulators are then not written out).
// timing: the mesh's timing records, or nullptr for no events at all.
cgd_status deposit_hex(cgd_mesh m, int64_t n, const float* pos, int32_t F, const float* values,
                       float* field, int64_t* acc, DepositInfo* info_dev, void* temp, const ScaleForce& fs,
                       Timing* timing, hipStream_t s);
// (also the tiled path of rectilinear meshes, which tiles the same way)
size_t deposit_hex_temp_bytes(const cgd_mesh m, int64_t n, int32_t F);
// Edges (all three axes) of the largest rectilinear grid the tiled deposit
// takes (it holds them in LDS); larger grids use the direct path.
constexpr int kRectTiledEdges = 4096;
// Clears a deposit's counters and sets its forced scales (enqueued on s).
void deposit_info_init(DepositInfo* info, const ScaleForce& fs, hipStream_t s);

// Tiled deposit of one or several snapshots on a mesh's hex grid (device
// pointers; the counters are cleared by the caller).  The fields of snapshot
// j are those a deposit of snapshot j alone gives.
struct TiledDeposit {
    const float* pos;              // [total][3]
    const float* values;           // [F][total]
    int64_t total;                 // particles of all snapshots
    int64_t max_n;                 // particles of the largest snapshot
    const int64_t* off;            // [n_snap + 1] particle offsets; nullptr: one snapshot
    int32_t n_snap, F;
    uint32_t* maxbits;             // [n_snap][F] max |v| bit patterns
    const int32_t* force_s;        // nullable: [F] scales forced by the caller (-1: automatic)
    unsigned long long* nf_val;    // field f's non-finite values are counted at nf_val[f * nf_val_stride]
    int32_t nf_val_stride;
    int32_t cnt_jstride;           // snapshot j's counts sit at dropped / nf_pos / nf_val + j * cnt_jstride
    unsigned long long* dropped;   // particles outside the box or with a non-finite coordinate
    unsigned long long* nf_pos;    // ... of those, the non-finite ones
    float* field;                  // [n_snap][F][cells]
    long long* acc;                // nullable: [n_snap][F][cells] int64 accumulators
    void* temp;                    // tiled_deposit_temp_bytes
    int32_t rect = 0;              // 1: the mesh's rectilinear edges locate (rl), each cell
    RectLoc rl = {};               //    divides by its own volume (vcell [cells])
    const double* vcell = nullptr;
};
// Bytes of `temp`; 0 when the grid or the particle count rules the tiled
// deposit out (then the direct atomic deposit is used).
size_t tiled_deposit_temp_bytes(int64_t cells, int64_t total, int32_t n_snap, int32_t F);
cgd_status tiled_deposit(cgd_mesh m, const TiledDeposit& d, Timing* timing, hipStream_t s);

// cg_hex.hip
struct DiffuseArgs {
    int32_t F;
    float* field;
    double bandwidth;
    int32_t n_steps;
    double rtol;
    int32_t max_iter;
    int32_t x0_mode;
    const float* x0;
    int32_t check_every;
    int32_t precond;  // hex: 0 polynomial-preconditioned CG, 1 plain CG
    cgd_unet model;   // x0_mode 3
    int32_t scheme;   // 0 backward Euler, 1 Crank-Nicolson (half-step solve, then 2 y - e)
};
// fixed: nullptr, or per step the iterations to enqueue without host
// read-backs (a step whose fields have not converged within it ends with
// CGD_NOT_CONVERGED, as one that reaches max_iter).
cgd_status diffuse_hex(cgd_mesh m, const DiffuseArgs& a, cgd_solve_stats* st, hipStream_t s,
                       const int* fixed = nullptr);
// The device work of diffuse_hex, enqueued on s with its workspace at `base`
// (diffuse_hex_workspace(m, a.F) bytes, laid out as the mesh workspace: the
// small region, partial sums, then the vectors).  fixed: nullptr for the
// look-ahead loop with host read-backs (uses the mesh's pinned buffer), or a
// budget of iterations per step enqueued without any host interaction (the
// launches of a field that has converged return at once; a field not
// converged within its budget is settled by k_cg_step_end as not converged),
// which may be captured in a graph.  sums: the mass before and after.  The
// statistics stay in the small region at `base`.
// ro: nullptr for the uniform grid's operator, or a rectilinear grid's
// (the field then holds M^1/2 e; RectOp's preconditioner).  geom: the grid
// to solve on in place of the mesh's (the same cells in another layout).
cgd_status diffuse_hex_enqueue(cgd_mesh m, const DiffuseArgs& a, char* base, const int* fixed, bool sums,
                               hipStream_t s, const RectOp* ro = nullptr, const HexGeom* geom = nullptr);

// A rectilinear grid whose diffusivity is a product of per-axis factors
// (D_ijk = Dx_i Dy_j Dz_k), periodic axes included.  The solve runs on
// A = I + dtau M^-1/2 K M^-1/2 for x~ = M^1/2 x, whose entries are products
// of per-axis factors (stencil::Geom).  Its preconditioner is
// S p(S A S) S with S a diagonal scaling that is itself a product of
// per-axis factors, chosen per dtau so that S A S has a diagonal close to 1
// (rect_op_prepare), and p the Chebyshev polynomial on S A S's spectrum.
struct RectOp {
    // dtau-free per-axis data from the mesh: cell widths, diffusivity
    // factors, face weights of M^-1/2 K M^-1/2 ([n + 1], 0 at walls) and its
    // diagonal sums
    std::vector<double> h[3], fac[3], gf[3], sd[3];
    // device arrays of A (dtau-free): face weights g [n + 1], diagonal sums
    // s, diffusivity factors d, identity factors e (ones), and the change of
    // variable's factors in (sqrt h) and out (1 / sqrt h) [n each]
    float* g[3];
    float* s[3];
    float* d[3];
    float* e[3];
    float* win[3];
    float* wout[3];
    // device arrays of S A S for the last prepared dtau: the same four
    // factors with S folded in, and S's own factors sg [n each]
    float* pg[3];
    float* ps[3];
    float* pd[3];
    float* pe[3];
    float* psg[3];
    float* dev = nullptr;    // A's arrays
    float* pdev = nullptr;   // S A S's arrays
    float* host = nullptr;   // pinned staging of S A S's arrays
    size_t pfloats = 0;
    int per = 0;             // bit a: axis a periodic (and of at least two cells)
    double dtau = -1.0;      // dtau S A S was formed for (-1: none yet)
    double lmin = 1.0, lmax = 1.0;  // bounds of S A S's spectrum
};

// Whether the hex sweeps on g cover an x-row with one x segment of waves
// (the condition for a periodic x axis), for a field at `field`.
bool hex_one_x_segment(const HexGeom& g, const float* field);

// Forms S A S's device arrays and spectrum bounds for dtau (no work when
// dtau is the one of the last call; otherwise synchronises the stream once
// before the staging buffer is rewritten).
cgd_status rect_op_prepare(cgd_mesh m, double dtau, hipStream_t s);

// mom[c][k] /= eps[k] where eps[k] > eps_min, else 0 (cg_common.hip).
void velocity_from_momentum(int64_t cells, int n_comp, const float* eps, float* mom, float eps_min,
                            hipStream_t s);

// Bytes of workspace the hex diffusion needs for F fields.
size_t diffuse_hex_workspace(const cgd_mesh m, int32_t F);

// ceil(log2 n) for n >= 2, 0 for n <= 1 (the e_N of the fixed-point scale).
int ceil_log2_count(int64_t n);

// Resets the counters (and records the forced scales), clears acc [F, cells]
// and computes max |v| per field.
void deposit_prologue(int64_t n, int32_t F, const float* values, int64_t* acc, int64_t cells,
                      DepositInfo* info, const ScaleForce& fs, hipStream_t s);

#ifdef __HIPCC__
// Fixed-point scale S = 62 - e_max - e_N, max |v| = m 2^e_max, m in [0.5, 1).
__device__ inline int frac_bits_of(uint32_t maxbits, int e_n) {
    if (maxbits == 0u) return 0;
    int e;
    (void)frexp((double)__uint_as_float(maxbits), &e);
    return 62 - e - e_n;
}
// The scale in use: the caller's, else the automatic one.
__device__ inline int frac_bits_used(uint32_t maxbits, int32_t force, int e_n) {
    return force >= 0 ? force : frac_bits_of(maxbits, e_n);
}
#endif

// Host cell of each particle (-1: outside / non-finite); device int32 [n].
cgd_status locate_hex(cgd_mesh m, int64_t n, const float* pos, int32_t* cell, hipStream_t s);
cgd_status locate_tet(cgd_mesh m, int64_t n, const float* pos, int32_t* cell, hipStream_t s);

// unet.hip: y = f(x) for one field on the network's grid (asynchronous);
// whether the network was made for this grid and device.
namespace unet {
cgd_status unet_guess(cgd_unet u, const float* x, float* y, hipStream_t s);
bool unet_matches(cgd_unet u, int nx, int ny, int nz, int device);
}  // namespace unet

// batched.hip
cgd_status coarse_grain_batched(cgd_mesh m, int32_t n_snap, const int64_t* offsets, const float* pos, int32_t F,
                                const float* values, const DiffuseArgs& da, float* fields, cgd_solve_stats* st_out,
                                hipStream_t s);
cgd_status autotune_batched(cgd_mesh m, int n_rhs, int* chosen, double* ms_out, int* n_cand);
void destroy_batched(cgd_mesh m);

#ifdef __HIPCC__
// atomicMax of a value that only grows, skipped when the value there is
// already at least v (the load may be stale, never larger than the true
// value, so a skipped update was never needed): one same-address atomic per
// block would otherwise serialise thousands of blocks.
__device__ inline void atomic_max_if_larger(uint32_t* p, uint32_t v) {
    if (v > __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(p, v);
}
#endif

// tet.cpp / tet.hip
// temp (rectilinear meshes): deposit_hex_temp_bytes(m, n, F) bytes for the
// tiled path, as deposit_hex; nullptr for the direct path.  Tet meshes:
// deposit_tet_temp_bytes(m, n) bytes for the particles' spatial ordering
// (nullptr: located in input order).
size_t deposit_tet_temp_bytes(const cgd_mesh m, int64_t n);
cgd_status deposit_tet(cgd_mesh m, int64_t n, const float* pos, int32_t F, const float* values,
                       float* field, int64_t* acc, DepositInfo* info_dev, void* temp, const ScaleForce& fs,
                       hipStream_t s);
// fixed: iterations per step (no read-backs) or nullptr (read-backs).
cgd_status diffuse_tet(cgd_mesh m, const DiffuseArgs& a, cgd_solve_stats* st, hipStream_t s,
                       const int* fixed = nullptr);
// Whether diffuse_tet takes the uniform grid's sweeps with per-axis factors.
bool rect_fast_path(const cgd_mesh m, const DiffuseArgs& a);
void destroy_tet_data(cgd_mesh m);
int64_t tet_nnz(cgd_mesh m);

}  // namespace cgd
