// Backward-Euler diffusion on uniform hex grids by conjugate gradients with a
// matrix-free 7-point stencil (Sections 3.2 and 5.1).
//
// Each pseudo-step solves A x = b with A = I + dtau K / V (the finite-volume
// Laplacian K divided by the uniform cell volume, so that A stays symmetric
// positive definite): (A p)_k = p_k + sum_a c_a (2 p_k - p_k-1 - p_k+1) with
// c_a = dtau / h_a^2, where a missing neighbour at a wall is replaced by p_k
// itself (zero flux through wall faces, Section 3.2.2).
//
// One CG iteration is two streaming sweeps over the grid, 32 bytes per cell:
//   sweep 1: p = r + beta p_old (also recomputed at neighbours), A p, p.Ap
//            reads r, p_old; writes p
//   sweep 2: x += alpha p, r -= alpha A p (A p recomputed), r.r
//            reads p, x, r; writes x, r
// Each sweep is followed by a one-block finisher per field that reduces the
// float64 block partials in a fixed order (deterministic) and updates the
// field's alpha / beta / convergence state on the device.
//
// Sweep layout: a wave owns 64 consecutive x (one lane each) times TY rows
// of y, and marches over a chunk of z planes keeping the planes z-1, z, z+1
// in registers.  x-neighbours come from lane shuffles (the two wave-edge
// lanes load theirs), y-neighbours from the wave's own rows plus one halo row
// on each side.  Blocks of 4 waves are spread so that consecutive tiles land
// on the same XCD (workgroups are dealt round-robin over the 8 XCDs), which
// keeps halo rows in that XCD's L2.
#include <algorithm>

#include "cgd_internal.h"

namespace cgd {
namespace {

constexpr int kWaves = 4;
constexpr int kBlock = 64 * kWaves;

enum Mode { S1_FIRST = 0, S1 = 1, S2_FIRST = 2, S2 = 3, S_RES = 4 };

struct SweepArgs {
    const float* B;     // right-hand side of the step (zero-guess first iteration: p = b)
    float* R;           // residual
    const float* Pold;  // previous direction (sweep 1)
    float* Pnew;        // new direction (sweep 1 writes, sweep 2 reads)
    float* X;           // iterate
    const CgField* st;
    double* partials;   // [F][2][bpf]
    int64_t cells;
    int nx, ny, nz;
    float cx, cy, cz;
    int xsegs, ygroups, zc;
    int wpf, bpf, nblocks;
    int beta_zero;
};

template <int MODE>
__device__ __forceinline__ float load_p(const SweepArgs& a, size_t i, float beta) {
    if constexpr (MODE == S1_FIRST || MODE == S2_FIRST) {
        return a.B[i];
    } else if constexpr (MODE == S1) {
        float r = a.R[i];
        return a.beta_zero ? r : fmaf(beta, a.Pold[i], r);
    } else if constexpr (MODE == S2) {
        return a.Pnew[i];
    } else {
        return a.X[i];
    }
}

template <int TY, int MODE>
__global__ __launch_bounds__(kBlock) void k_sweep(SweepArgs a) {
    int b = blockIdx.x;
    if ((a.nblocks & 7) == 0) b = (b & 7) * (a.nblocks >> 3) + (b >> 3);
    const int f = b / a.bpf;
    const int blk = b - f * a.bpf;
    const CgField* stf = a.st + f;
    if (stf->done) return;  // uniform over the block

    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int w = blk * kWaves + wave;
    double acc0 = 0.0, acc1 = 0.0;

    if (w < a.wpf) {
        const float alpha = (float)stf->alpha;
        const float beta = (float)stf->beta;
        const int xs = w % a.xsegs;
        const int t = w / a.xsegs;
        const int yg = t % a.ygroups;
        const int zci = t / a.ygroups;
        const int x = xs * 64 + lane;
        const bool xin = x < a.nx;
        const bool has_l = x > 0, has_r = x + 1 < a.nx;
        const int y0 = yg * TY;
        const int zb = zci * a.zc;
        const int ze = min(zb + a.zc, a.nz);
        const size_t plane = (size_t)a.nx * a.ny;
        const size_t fo = (size_t)f * a.cells + x;
        const float cx = a.cx, cy = a.cy, cz = a.cz;

        auto idx = [&](int z, int y) -> size_t { return fo + (size_t)z * plane + (size_t)y * a.nx; };
        auto ld = [&](int z, int y) -> float {
            return (xin && y >= 0 && y < a.ny) ? load_p<MODE>(a, idx(z, y), beta) : 0.f;
        };

        float pm[TY], pc[TY], pn[TY];
#pragma unroll
        for (int j = 0; j < TY; ++j) {
            pm[j] = zb > 0 ? ld(zb - 1, y0 + j) : 0.f;
            pc[j] = ld(zb, y0 + j);
        }
        for (int z = zb; z < ze; ++z) {
            const bool has_zu = z + 1 < a.nz, has_zd = z > 0;
#pragma unroll
            for (int j = 0; j < TY; ++j) pn[j] = has_zu ? ld(z + 1, y0 + j) : 0.f;
            const float hlo = ld(z, y0 - 1);
            const float hhi = ld(z, y0 + TY);
#pragma unroll
            for (int j = 0; j < TY; ++j) {
                const int y = y0 + j;
                const float c = pc[j];
                float l = __shfl_up(c, 1);
                float r = __shfl_down(c, 1);
                if (lane == 0 && has_l && y < a.ny) l = load_p<MODE>(a, idx(z, y) - 1, beta);
                if (lane == 63 && has_r && y < a.ny) r = load_p<MODE>(a, idx(z, y) + 1, beta);
                l = has_l ? l : c;
                r = has_r ? r : c;
                const float yl = y > 0 ? (j > 0 ? pc[j - 1] : hlo) : c;
                const float yh = y + 1 < a.ny ? (j + 1 < TY ? pc[j + 1] : hhi) : c;
                const float zl = has_zd ? pm[j] : c;
                const float zh = has_zu ? pn[j] : c;
                const float c2 = c + c;
                float Ap = fmaf(cx, (c2 - l) - r, c);
                Ap = fmaf(cy, (c2 - yl) - yh, Ap);
                Ap = fmaf(cz, (c2 - zl) - zh, Ap);
                if (xin && y < a.ny) {
                    const size_t i = idx(z, y);
                    if constexpr (MODE == S1_FIRST) {
                        acc0 = fma((double)c, (double)Ap, acc0);
                        acc1 = fma((double)c, (double)c, acc1);
                    } else if constexpr (MODE == S1) {
                        a.Pnew[i] = c;
                        acc0 = fma((double)c, (double)Ap, acc0);
                    } else if constexpr (MODE == S2_FIRST) {
                        const float xn = alpha * c;
                        const float rn = fmaf(-alpha, Ap, c);
                        a.X[i] = xn;
                        a.R[i] = rn;
                        acc0 = fma((double)rn, (double)rn, acc0);
                    } else if constexpr (MODE == S2) {
                        const float xn = fmaf(alpha, c, a.X[i]);
                        const float rn = fmaf(-alpha, Ap, a.R[i]);
                        a.X[i] = xn;
                        a.R[i] = rn;
                        acc0 = fma((double)rn, (double)rn, acc0);
                    } else {  // S_RES: r = b - A x0
                        const float bv = a.B[i];
                        const float rn = bv - Ap;
                        a.R[i] = rn;
                        acc0 = fma((double)rn, (double)rn, acc0);
                        acc1 = fma((double)bv, (double)bv, acc1);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < TY; ++j) {
                pm[j] = pc[j];
                pc[j] = pn[j];
            }
        }
    }

    // block reduction of the float64 partials, fixed order
    for (int o = 32; o > 0; o >>= 1) {
        acc0 += __shfl_xor(acc0, o);
        acc1 += __shfl_xor(acc1, o);
    }
    __shared__ double s0[kWaves], s1[kWaves];
    if (lane == 0) {
        s0[wave] = acc0;
        s1[wave] = acc1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t0 = 0.0, t1 = 0.0;
#pragma unroll
        for (int i = 0; i < kWaves; ++i) {
            t0 += s0[i];
            t1 += s1[i];
        }
        a.partials[((size_t)f * 2 + 0) * a.bpf + blk] = t0;
        a.partials[((size_t)f * 2 + 1) * a.bpf + blk] = t1;
    }
}

enum Finish { F1_FIRST = 0, F1 = 1, F2 = 2, F_RES = 3 };

struct FinishArgs {
    const double* partials;
    int bpf;
    CgField* st;
    int* ndone;
    int step;
    double rtol2;
    int max_iter;
    int32_t* iters;    // [CGD_MAX_STEPS][CGD_MAX_FIELDS]
    double* relres;    // [CGD_MAX_STEPS][CGD_MAX_FIELDS]
    int32_t* status;   // [CGD_MAX_STEPS][CGD_MAX_FIELDS], final status of each solve
};

// Sums one field's partials in a fixed order: thread t adds t, t+256, ...,
// then a fixed shuffle tree and a fixed sum over the 4 waves.
__device__ inline double block_sum_fixed(const double* p, int n) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kBlock) s += p[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    __shared__ double sh[kWaves];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) t += sh[i];
    __syncthreads();
    return t;
}

__device__ inline void mark_done(CgField& s, const FinishArgs& a, int f) {
    s.done = 1;
    a.status[a.step * CGD_MAX_FIELDS + f] = s.status;
    atomicAdd(a.ndone, 1);
}

template <int KIND>
__global__ __launch_bounds__(kBlock) void k_finish(FinishArgs a) {
    const int f = blockIdx.x;
    CgField* st = a.st + f;
    if (KIND != F1_FIRST && KIND != F_RES && st->done) return;
    const double s0 = block_sum_fixed(a.partials + ((size_t)f * 2 + 0) * a.bpf, a.bpf);
    double s1 = 0.0;
    if (KIND == F1_FIRST || KIND == F_RES) s1 = block_sum_fixed(a.partials + ((size_t)f * 2 + 1) * a.bpf, a.bpf);
    if (threadIdx.x != 0) return;
    CgField s = *st;
    if constexpr (KIND == F1_FIRST) {
        // s0 = b.Ab, s1 = b.b
        s.bb = s1;
        s.rr = s1;
        if (s1 == 0.0) {
            s.alpha = 0.0;  // b = 0: x = 0, detected as converged after sweep 2
        } else if (!(s0 > 0.0) || !isfinite(s0) || !isfinite(s1)) {
            s.alpha = 0.0;
            s.status = CGD_E_BREAKDOWN;
        } else {
            s.alpha = s1 / s0;
        }
    } else if constexpr (KIND == F1) {
        if (!(s0 > 0.0) || !isfinite(s0)) {
            s.status = CGD_E_BREAKDOWN;
            s.alpha = 0.0;
            mark_done(s, a, f);
        } else {
            s.alpha = s.rr / s0;
        }
    } else if constexpr (KIND == F_RES) {
        // s0 = r.r, s1 = b.b
        s.bb = s1;
        s.rr = s0;
        s.beta = 0.0;
        if (!isfinite(s0) || !isfinite(s1)) {
            s.status = CGD_E_BREAKDOWN;
            mark_done(s, a, f);
        } else if (s0 <= a.rtol2 * s1) {
            mark_done(s, a, f);  // the initial guess already meets the tolerance
        }
        a.relres[a.step * CGD_MAX_FIELDS + f] = s1 > 0.0 ? sqrt(s0 / s1) : 0.0;
        a.iters[a.step * CGD_MAX_FIELDS + f] = 0;
    } else {  // F2: s0 = r_new . r_new
        s.iter += 1;
        const double rel = s.bb > 0.0 ? sqrt(s0 / s.bb) : 0.0;
        a.iters[a.step * CGD_MAX_FIELDS + f] = s.iter;
        a.relres[a.step * CGD_MAX_FIELDS + f] = rel;
        if (!isfinite(s0)) {
            s.status = CGD_E_BREAKDOWN;
            mark_done(s, a, f);
        } else if (s.status != CGD_OK || s0 <= a.rtol2 * s.bb) {
            mark_done(s, a, f);
        } else if (s.iter >= a.max_iter) {
            s.status = CGD_NOT_CONVERGED;
            mark_done(s, a, f);
        } else {
            s.beta = s0 / s.rr;
            s.rr = s0;
        }
    }
    *st = s;
}

__global__ void k_step_init(CgField* st, int F, int* ndone, int32_t* status_row) {
    int f = threadIdx.x;
    if (f < F) {
        CgField s = {};
        s.status = CGD_OK;
        st[f] = s;
        status_row[f] = CGD_OK;
    }
    if (threadIdx.x == 0) *ndone = 0;
}

// x0 paths: a field whose right-hand side is zero has solution zero.
__global__ void k_zero_if_rhs_zero(float* X, int64_t cells, const CgField* st) {
    const int f = blockIdx.y;
    if (st[f].bb != 0.0) return;
    float* x = X + (size_t)f * cells;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < cells;
         k += (int64_t)gridDim.x * blockDim.x)
        x[k] = 0.f;
}

// Sum of each field (float64), for the mass statistics.
__global__ __launch_bounds__(kBlock) void k_field_sum(const float* v, int64_t cells, double* partials, int bpf) {
    const int f = blockIdx.y;
    double s = 0.0;
    const float* p = v + (size_t)f * cells;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < cells;
         k += (int64_t)gridDim.x * blockDim.x)
        s += (double)p[k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    __shared__ double sh[kWaves];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < kWaves; ++i) t += sh[i];
        partials[(size_t)f * bpf + blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_sum_finish(const double* partials, int bpf, double* out) {
    const int f = blockIdx.x;
    double t = block_sum_fixed(partials + (size_t)f * bpf, bpf);
    if (threadIdx.x == 0) out[f] = t;
}

// ---------------------------------------------------------------- host side

struct Plan {
    int ty, zc, xsegs, ygroups, zchunks, wpf, bpf, nblocks;
};

Plan make_plan(const HexGeom& g, int F, int ty, int zc) {
    Plan p;
    p.ty = ty;
    p.zc = std::max(1, std::min(zc, g.nz));
    p.xsegs = (g.nx + 63) / 64;
    p.ygroups = (g.ny + ty - 1) / ty;
    p.zchunks = (g.nz + p.zc - 1) / p.zc;
    p.wpf = p.xsegs * p.ygroups * p.zchunks;
    p.bpf = (p.wpf + kWaves - 1) / kWaves;
    p.nblocks = p.bpf * F;
    return p;
}

// Default tiling: TY = 8 rows and a z chunk that gives about 16 waves per
// compute unit (256 CUs), but never fewer than 8 planes per chunk.
Plan default_plan(const HexGeom& g, int F) {
    const int ty = g.ny >= 8 ? 8 : 4;
    const int64_t cols = (int64_t)((g.nx + 63) / 64) * ((g.ny + ty - 1) / ty) * F;
    const int64_t target_waves = 4096;
    int64_t chunks = std::max<int64_t>(1, target_waves / std::max<int64_t>(1, cols));
    int zc = (int)std::max<int64_t>(8, (g.nz + chunks - 1) / chunks);
    return make_plan(g, F, ty, zc);
}

template <int MODE>
void launch_sweep_mode(const Plan& p, const SweepArgs& a, hipStream_t s) {
    switch (p.ty) {
        case 4: hipLaunchKernelGGL((k_sweep<4, MODE>), dim3(p.nblocks), dim3(kBlock), 0, s, a); break;
        case 8: hipLaunchKernelGGL((k_sweep<8, MODE>), dim3(p.nblocks), dim3(kBlock), 0, s, a); break;
        default: hipLaunchKernelGGL((k_sweep<16, MODE>), dim3(p.nblocks), dim3(kBlock), 0, s, a); break;
    }
}

void launch_sweep(int mode, const Plan& p, const SweepArgs& a, hipStream_t s) {
    switch (mode) {
        case S1_FIRST: launch_sweep_mode<S1_FIRST>(p, a, s); break;
        case S1: launch_sweep_mode<S1>(p, a, s); break;
        case S2_FIRST: launch_sweep_mode<S2_FIRST>(p, a, s); break;
        case S2: launch_sweep_mode<S2>(p, a, s); break;
        default: launch_sweep_mode<S_RES>(p, a, s); break;
    }
}

void launch_finish(int kind, int F, const FinishArgs& a, hipStream_t s) {
    switch (kind) {
        case F1_FIRST: hipLaunchKernelGGL(k_finish<F1_FIRST>, dim3(F), dim3(kBlock), 0, s, a); break;
        case F1: hipLaunchKernelGGL(k_finish<F1>, dim3(F), dim3(kBlock), 0, s, a); break;
        case F2: hipLaunchKernelGGL(k_finish<F2>, dim3(F), dim3(kBlock), 0, s, a); break;
        default: hipLaunchKernelGGL(k_finish<F_RES>, dim3(F), dim3(kBlock), 0, s, a); break;
    }
}

// Layout of the small region at the start of the workspace (bytes).
constexpr size_t kOffState = 0;                     // CgField[CGD_MAX_FIELDS]
constexpr size_t kOffNdone = 4096;                  // int
constexpr size_t kOffIters = 8192;                  // int32 [STEPS][FIELDS]
constexpr size_t kOffRelres = kOffIters + 4096;     // double [STEPS][FIELDS]
constexpr size_t kOffStatus = kOffRelres + 8192;    // int32 [STEPS][FIELDS]
constexpr size_t kOffSums = kOffStatus + 4096;      // double [2][FIELDS]
constexpr size_t kSmallFixed = 64 * 1024;           // partials follow

// Layout of the pinned host buffer (bytes).
constexpr size_t kPinFlags = 0;                     // int[2]
constexpr size_t kPinIters = 4096;
constexpr size_t kPinRelres = kPinIters + 4096;
constexpr size_t kPinStatus = kPinRelres + 8192;
constexpr size_t kPinSums = kPinStatus + 4096;
constexpr size_t kPinBytes = kPinSums + 4096;

size_t small_bytes(int F, int bpf) {
    size_t b = kSmallFixed + (size_t)F * 2 * (size_t)bpf * sizeof(double);
    return (b + 255) & ~(size_t)255;
}

}  // namespace

size_t diffuse_hex_workspace(const cgd_mesh m, int32_t F) {
    Plan p = default_plan(m->hex, F);
    return small_bytes(F, p.bpf) + 4 * (size_t)F * m->cells * sizeof(float);
}

cgd_status diffuse_hex(cgd_mesh m, const DiffuseArgs& da, cgd_solve_stats* out, hipStream_t s) {
    const HexGeom& g = m->hex;
    const int F = da.F;
    const int64_t cells = m->cells;
    Plan p = default_plan(g, F);
    if (const char* e = getenv("CGD_HEX_TILE")) {  // "TY,ZC" for tuning runs
        int ty = 0, zc = 0;
        if (sscanf(e, "%d,%d", &ty, &zc) == 2 && (ty == 4 || ty == 8 || ty == 16) && zc > 0)
            p = make_plan(g, F, ty, zc);
    }
    const size_t small = small_bytes(F, p.bpf);
    cgd_status rc = ensure_workspace(m, small + 4 * (size_t)F * cells * sizeof(float));
    if (rc != CGD_OK) return rc;
    rc = ensure_pinned(m, kPinBytes);
    if (rc != CGD_OK) return rc;

    char* base = static_cast<char*>(m->ws.ptr);
    CgField* d_state = reinterpret_cast<CgField*>(base + kOffState);
    int* d_ndone = reinterpret_cast<int*>(base + kOffNdone);
    int32_t* d_iters = reinterpret_cast<int32_t*>(base + kOffIters);
    double* d_relres = reinterpret_cast<double*>(base + kOffRelres);
    int32_t* d_status = reinterpret_cast<int32_t*>(base + kOffStatus);
    double* d_sums = reinterpret_cast<double*>(base + kOffSums);
    double* d_partials = reinterpret_cast<double*>(base + kSmallFixed);
    float* W0 = reinterpret_cast<float*>(base + small);
    float* R = W0 + (size_t)F * cells;
    float* PA = R + (size_t)F * cells;
    float* PB = PA + (size_t)F * cells;
    char* pin = static_cast<char*>(m->pinned);

    const double T = da.bandwidth * da.bandwidth / 4.0;
    const double dtau = T / da.n_steps;
    SweepArgs a = {};
    a.cells = cells;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.cx = (float)(dtau / (g.h[0] * g.h[0]));
    a.cy = (float)(dtau / (g.h[1] * g.h[1]));
    a.cz = (float)(dtau / (g.h[2] * g.h[2]));
    a.xsegs = p.xsegs;
    a.ygroups = p.ygroups;
    a.zc = p.zc;
    a.wpf = p.wpf;
    a.bpf = p.bpf;
    a.nblocks = p.nblocks;
    a.st = d_state;
    a.partials = d_partials;
    a.R = R;

    FinishArgs fa = {};
    fa.partials = d_partials;
    fa.bpf = p.bpf;
    fa.st = d_state;
    fa.ndone = d_ndone;
    fa.rtol2 = da.rtol * da.rtol;
    fa.max_iter = da.max_iter;
    fa.iters = d_iters;
    fa.relres = d_relres;
    fa.status = d_status;

    int* pinned_flags = reinterpret_cast<int*>(pin + kPinFlags);
    const int chunk = std::max(1, da.check_every);
    const int sum_bpf = (int)std::min<int64_t>(1024, (cells + kBlock - 1) / kBlock);

    if (out) {  // mass before diffusion
        hipLaunchKernelGGL(k_field_sum, dim3(sum_bpf, F), dim3(kBlock), 0, s, da.field, cells, d_partials, sum_bpf);
        hipLaunchKernelGGL(k_sum_finish, dim3(F), dim3(kBlock), 0, s, d_partials, sum_bpf, d_sums);
    }

    float* cur = da.field;  // b of the current step
    float* nxt = W0;        // x of the current step
    for (int step = 0; step < da.n_steps; ++step) {
        fa.step = step;
        a.B = cur;
        a.X = nxt;
        hipLaunchKernelGGL(k_step_init, dim3(1), dim3(64), 0, s, d_state, F, d_ndone, d_status + step * CGD_MAX_FIELDS);
        const bool use_x0 = (da.x0_mode == 1) || (da.x0_mode == 2 && step == 0);
        int it;  // index of the next iteration to enqueue
        if (!use_x0) {
            launch_sweep(S1_FIRST, p, a, s);
            launch_finish(F1_FIRST, F, fa, s);
            launch_sweep(S2_FIRST, p, a, s);
            launch_finish(F2, F, fa, s);
            it = 1;
        } else {
            const float* x0 = da.x0_mode == 1 ? cur : da.x0;
            CGD_HIP_TRY(hipMemcpyAsync(nxt, x0, (size_t)F * cells * sizeof(float), hipMemcpyDeviceToDevice, s));
            launch_sweep(S_RES, p, a, s);
            launch_finish(F_RES, F, fa, s);
            it = 0;
        }
        // Iterations are enqueued `chunk` at a time; the number of converged
        // fields is copied back after each chunk and checked one chunk later,
        // so the device always has queued work while the host waits.
        int slot = 0;
        bool have_prev = false;
        for (;;) {
            const int todo = std::min(chunk, da.max_iter - it);
            for (int c = 0; c < todo; ++c, ++it) {
                if (!use_x0) {
                    a.Pold = it == 1 ? cur : ((it & 1) ? PB : PA);
                    a.Pnew = (it & 1) ? PA : PB;
                    a.beta_zero = 0;
                } else {
                    a.Pold = (it & 1) ? PA : PB;
                    a.Pnew = (it & 1) ? PB : PA;
                    a.beta_zero = it == 0;
                }
                int t1 = timing_begin(&m->timing, s);
                launch_sweep(S1, p, a, s);
                timing_end(&m->timing, t1, 0, 12.0 * (double)F * cells, s);
                launch_finish(F1, F, fa, s);
                int t2 = timing_begin(&m->timing, s);
                launch_sweep(S2, p, a, s);
                timing_end(&m->timing, t2, 1, 20.0 * (double)F * cells, s);
                launch_finish(F2, F, fa, s);
            }
            CGD_HIP_TRY(hipMemcpyAsync(&pinned_flags[slot], d_ndone, sizeof(int), hipMemcpyDeviceToHost, s));
            CGD_HIP_TRY(hipEventRecord(m->ev[slot], s));
            if (have_prev) {
                CGD_HIP_TRY(hipEventSynchronize(m->ev[slot ^ 1]));
                if (pinned_flags[slot ^ 1] >= F) break;
            }
            if (it >= da.max_iter) {
                CGD_HIP_TRY(hipEventSynchronize(m->ev[slot]));
                break;
            }
            have_prev = true;
            slot ^= 1;
        }
        if (use_x0) {
            int blocks = (int)std::min<int64_t>(2048, (cells + kBlock - 1) / kBlock);
            hipLaunchKernelGGL(k_zero_if_rhs_zero, dim3(blocks, F), dim3(kBlock), 0, s, nxt, cells, d_state);
        }
        std::swap(cur, nxt);
    }
    if (cur != da.field) {
        CGD_HIP_TRY(hipMemcpyAsync(da.field, cur, (size_t)F * cells * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
    if (out) {
        hipLaunchKernelGGL(k_field_sum, dim3(sum_bpf, F), dim3(kBlock), 0, s, da.field, cells, d_partials, sum_bpf);
        hipLaunchKernelGGL(k_sum_finish, dim3(F), dim3(kBlock), 0, s, d_partials, sum_bpf, d_sums + CGD_MAX_FIELDS);
    }
    CGD_HIP_TRY(hipGetLastError());
    int32_t* h_iters = reinterpret_cast<int32_t*>(pin + kPinIters);
    double* h_rel = reinterpret_cast<double*>(pin + kPinRelres);
    int32_t* h_status = reinterpret_cast<int32_t*>(pin + kPinStatus);
    double* h_sums = reinterpret_cast<double*>(pin + kPinSums);
    CGD_HIP_TRY(hipMemcpyAsync(h_status, d_status, 4096, hipMemcpyDeviceToHost, s));
    if (out) {
        CGD_HIP_TRY(hipMemcpyAsync(h_iters, d_iters, 4096, hipMemcpyDeviceToHost, s));
        CGD_HIP_TRY(hipMemcpyAsync(h_rel, d_relres, 8192, hipMemcpyDeviceToHost, s));
        CGD_HIP_TRY(hipMemcpyAsync(h_sums, d_sums, 2 * CGD_MAX_FIELDS * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    CGD_HIP_TRY(hipStreamSynchronize(s));
    timing_collect(&m->timing);
    cgd_status worst = CGD_OK;
    for (int st = 0; st < da.n_steps; ++st)
        for (int f = 0; f < F; ++f) {
            int32_t v = h_status[st * CGD_MAX_FIELDS + f];
            if (v == CGD_E_BREAKDOWN) {
                set_error("CG breakdown in pseudo-step " + std::to_string(st) + ", field " + std::to_string(f));
                worst = CGD_E_BREAKDOWN;
            } else if (v == CGD_NOT_CONVERGED && worst == CGD_OK) {
                worst = CGD_NOT_CONVERGED;
            }
        }
    if (out) {
        out->n_steps = da.n_steps;
        out->n_fields = F;
        for (int st = 0; st < da.n_steps; ++st)
            for (int f = 0; f < F; ++f) {
                out->iters[st][f] = h_iters[st * CGD_MAX_FIELDS + f];
                out->rel_res[st][f] = h_rel[st * CGD_MAX_FIELDS + f];
            }
        for (int f = 0; f < F; ++f) {
            out->mass_before[f] = h_sums[f] * g.vol;
            out->mass_after[f] = h_sums[CGD_MAX_FIELDS + f] * g.vol;
        }
        out->status = worst;
    }
    return worst;
}

}  // namespace cgd
