// Batched coarse graining: many independent snapshots and fields on one hex
// mesh (Section 3.2.1: each field component is diffused on its own).
//
// Deposition is segmented by snapshot (each snapshot and field gets its own
// fixed-point scale, exactly as a single-snapshot deposit would).  The
// diffusion of all right-hand sides (snapshots x fields) is ONE persistent
// launch: each workgroup runs every pseudo-step of the zero-guess CG of its
// right-hand sides (dealt statically, blockIdx.x + i * gridDim.x) alone,
// with workgroup-level reductions only (no grid-wide synchronisation, so no
// co-residency is assumed).  Its waves
// use the same stencil tiles as the per-launch solver.  The whole call
// (offset upload, deposit, solve, status read-back) is captured once in a
// hipGraph per argument set and replayed.  The tile shape (rows per wave,
// waves per workgroup) and the preconditioner's degree (2 in registers, 4
// through the LDS sweep of precond_lds.h) come from an autotuner that times
// every candidate on the device and caches the choice per mesh shape (and in
// the file named by CGD_AUTOTUNE_CACHE, when set).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "cg_common.h"
#include "hex_bin.h"
#include "precond_lds.h"
#include "stencil_tile.h"

namespace cgd {
namespace {

using namespace stencil;

constexpr int kDBlock = 256;
constexpr int kItems = 16;                  // particles per thread per deposit block
constexpr int kChunk = kDBlock * kItems;    // particles per deposit block
constexpr int kMaxRhs = 4096;

// ---------------------------------------------------------------- deposit

struct BDep {
    const int64_t* off;       // [n_snap + 1] device
    const float* pos;
    const float* values;      // [F][total]
    int64_t total;
    int n_snap, F;
    uint32_t* maxbits;        // [n_snap][F]
    unsigned long long* acc;  // [n_snap][F][cells]
    float* fields;            // [n_snap][F][cells]
    unsigned long long* counters;  // [n_snap][2]: dropped, non-finite (positions and values)
    int64_t cells;
    double vol;
    HexBin g;
};

__device__ inline int e_n_of(int64_t n) { return n <= 1 ? 0 : 64 - __clzll((unsigned long long)(n - 1)); }

__global__ void k_bdep_init(BDep d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d.n_snap * d.F) d.maxbits[i] = 0u;
    if (i < 2 * d.n_snap) d.counters[i] = 0ull;
}

__global__ void k_bzero(unsigned long long* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// grid: (chunks, n_snap * F); block (c, j * F + f) covers particles
// [off[j] + c * kChunk, ...) of snapshot j.
__global__ __launch_bounds__(kDBlock) void k_babsmax(BDep d) {
    const int j = blockIdx.y / d.F, f = blockIdx.y % d.F;
    const int64_t p0 = d.off[j], p1 = d.off[j + 1];
    const int64_t b = p0 + (int64_t)blockIdx.x * kChunk;
    uint32_t m = 0u;
    unsigned long long bad = 0ull;
    const uint32_t* v = reinterpret_cast<const uint32_t*>(d.values + (size_t)f * d.total);
    for (int t = 0; t < kItems; ++t) {
        const int64_t i = b + (int64_t)t * kDBlock + threadIdx.x;
        if (i < p1) {
            const uint32_t a = v[i] & 0x7fffffffu;
            if (a >= 0x7f800000u) ++bad;
            else m = a > m ? a : m;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t mo = __shfl_xor(m, o);
        m = mo > m ? mo : m;
        bad += __shfl_xor(bad, o);
    }
    if ((threadIdx.x & 63) == 0) {
        if (m) atomic_max_if_larger(&d.maxbits[j * d.F + f], m);
        if (bad) atomicAdd(&d.counters[2 * j + 1], bad);
    }
}

__global__ __launch_bounds__(kDBlock) void k_bdeposit(BDep d) {
    const int j = blockIdx.y;
    const int64_t p0 = d.off[j], p1 = d.off[j + 1];
    const int e_n = e_n_of(p1 - p0);
    __shared__ int S[CGD_MAX_FIELDS];
    if (threadIdx.x < d.F) S[threadIdx.x] = frac_bits_of(d.maxbits[j * d.F + threadIdx.x], e_n);
    __syncthreads();
    const int64_t b = p0 + (int64_t)blockIdx.x * kChunk;
    unsigned long long dropped = 0ull, nf = 0ull;
    for (int t = 0; t < kItems; ++t) {
        const int64_t i = b + (int64_t)t * kDBlock + threadIdx.x;
        if (i >= p1) break;
        bool nonfinite;
        const int64_t k = hex_cell(d.g, d.pos[3 * i], d.pos[3 * i + 1], d.pos[3 * i + 2], &nonfinite);
        if (k < 0) {
            ++dropped;
            nf += nonfinite ? 1ull : 0ull;
            continue;
        }
        for (int f = 0; f < d.F; ++f) {
            const float v = d.values[(size_t)f * d.total + i];
            if (!isfinite(v)) continue;
            const long long q = __double2ll_rn(ldexp((double)v, S[f]));
            if (q != 0) atomicAdd(&d.acc[((size_t)j * d.F + f) * d.cells + k], (unsigned long long)q);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        dropped += __shfl_xor(dropped, o);
        nf += __shfl_xor(nf, o);
    }
    if ((threadIdx.x & 63) == 0 && dropped) {
        atomicAdd(&d.counters[2 * j], dropped);
        if (nf) atomicAdd(&d.counters[2 * j + 1], nf);
    }
}

__global__ __launch_bounds__(kDBlock) void k_bfinalize(BDep d) {
    const int jf = blockIdx.y;
    const int j = jf / d.F;
    const int S = frac_bits_of(d.maxbits[jf], e_n_of(d.off[j + 1] - d.off[j]));
    const long long* a = reinterpret_cast<const long long*>(d.acc) + (size_t)jf * d.cells;
    float* out = d.fields + (size_t)jf * d.cells;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < d.cells; k += (int64_t)gridDim.x * blockDim.x)
        out[k] = (float)(ldexp((double)a[k], -S) / d.vol);
}

// ---------------------------------------------------------------- solver

struct BSolve {
    float* fields;      // [n_rhs][cells]: in deposited, out diffused
    float* ws;          // [grid][5][cells]
    int pcg;            // 1: preconditioned CG (degree 2: Geom c0, c1, c2; degree 4: cp)
    PrecondCoef pc;     // degree-4 polynomial's Horner levels (configurations with DEG = 4)
    PrecondCoef pp[3];  // degree-12 polynomial's three product passes (DEG = 12)
    int n_rhs;
    int64_t cells;
    Geom g;
    int xsegs, ygroups;
    int n_steps;
    double rtol2;
    int max_iter;
    int32_t* iters;     // [n_rhs][n_steps]
    double* relres;     // [n_rhs][n_steps]: recursive ||r|| / ||b|| at exit
    int32_t* status;    // [n_rhs]
};

// Mass of each right-hand side, sum_k V field_k, in float64 (one workgroup
// per right-hand side, every sum in one fixed order).
__global__ __launch_bounds__(1024) void k_bmass(const float* __restrict__ fields, int64_t cells, double vol,
                                                 double* __restrict__ out) {
    const float* f = fields + (size_t)blockIdx.x * cells;
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < cells; k += 1024) s += (double)f[k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    __shared__ double sh[16];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < 16; ++i) t += sh[i];
        out[blockIdx.x] = t * vol;
    }
}

// A value every lane of the wave holds identically, handed to the compiler as
// a wave-uniform (scalar) value so that branches on it are scalar branches.
__device__ inline double wave_uniform(double v) {
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Workgroup-wide float64 sums of two values in one fixed order; every thread
// returns the same pair, as wave-uniform values.
template <int NW>
__device__ inline void wg_sum2(double& a, double& b, double (*sh)[2]) {
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[w][0] = a;
        sh[w][1] = b;
    }
    __syncthreads();
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        s0 += sh[i][0];
        s1 += sh[i][1];
    }
    __syncthreads();
    a = wave_uniform(s0);
    b = wave_uniform(s1);
}

template <int VEC, int TY, int NW, int MODE>
__device__ inline void wg_sweep(const BSolve& a, const Ptrs& p, float alpha, float beta, double& s0, double& s1,
                                double (*sh)[2]) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    double acc0 = 0.0, acc1 = 0.0;
    const int tiles = a.xsegs * a.ygroups;
    for (int t = wave; t < tiles; t += NW)
        tile_sweep<VEC, TY, MODE, false>(p, a.g, 0, t % a.xsegs, t / a.xsegs, 0, a.g.nz, lane, alpha, beta, acc0,
                                         acc1);
    wg_sum2<NW>(acc0, acc1, sh);  // includes the barrier that publishes this sweep's writes
    s0 = acc0;
    s1 = acc1;
}

// z = M r over the workgroup's grid (one wave per row), r.z (and r.r when FIRST).
template <int VEC, int TY, int NW, bool FIRST>
__device__ inline void wg_precond(const BSolve& a, const Ptrs& p, double& s0, double& s1, double (*sh)[2]) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    double acc0 = 0.0, acc1 = 0.0;
    for (int t = wave; t < a.ygroups; t += NW)
        tile_precond2<VEC, TY, FIRST>(p, a.g, 0, t, 0, a.g.nz, lane, acc0, acc1);
    wg_sum2<NW>(acc0, acc1, sh);
    s0 = acc0;
    s1 = acc1;
}

// z = p(A) r with the degree-4 polynomial, tile by tile (8 rows of y, all of
// z) through the LDS sweep of precond_lds.h; r.z (and r.r when FIRST).
template <int VEC, int NW, bool FIRST>
__device__ inline void wg_precond_lds(float* lds, const BSolve& a, const Ptrs& p, double& s0, double& s1,
                                      double (*sh)[2]) {
    double acc0 = 0.0, acc1 = 0.0;
    const int tiles = (a.g.ny + 7) / 8;
    for (int t = 0; t < tiles; ++t)
        precond_lds_tile<VEC, 4, 8, NW, FIRST, true>(lds, FIRST ? p.B : p.R, p.Z, a.g, a.pc, a.g.ny, a.g.nz, 8 * t, 0,
                                               a.g.nz, acc0, acc1);
    wg_sum2<NW>(acc0, acc1, sh);
    s0 = acc0;
    s1 = acc1;
}

// One product pass over all tiles of the workgroup's grid.  Not inlined, so
// that each pass's tile gets its own register allocation instead of sharing
// the persistent kernel's (which spilled when all three were inlined).
template <int VEC, int NW, bool FIRST, int FORM>
__device__ __attribute__((noinline)) void wg_prod_pass(float* lds, const BSolve& a, const float* src, float* dst,
                                                       const PrecondCoef& pc, const float* r, double* acc) {
    double acc0 = 0.0, acc1 = 0.0;
    const int tiles = (a.g.ny + 7) / 8;
    for (int t = 0; t < tiles; ++t)
        precond_lds_tile<VEC, 4, 8, NW, FIRST, false, FORM>(lds, src, dst, a.g, pc, a.g.ny, a.g.nz, 8 * t, 0, a.g.nz,
                                                            acc0, acc1, r);
    acc[0] = acc0;
    acc[1] = acc1;
}

// z = p(A) r with the degree-12 polynomial: three product passes over all
// tiles (r -> U -> V -> z, two quadratic factors each), a barrier between
// passes publishing each pass's output; r.z from the last pass (r read for the
// output rows through the LDS side channel), r.r from the first when FIRST.
template <int VEC, int NW, bool FIRST>
__device__ inline void wg_precond_prod(float* lds, const BSolve& a, const Ptrs& p, double& s0, double& s1,
                                       double (*sh)[2]) {
    double first[2], mid[2], last[2];
    const float* r = FIRST ? p.B : p.R;
    wg_prod_pass<VEC, NW, FIRST, 1>(lds, a, r, p.U, a.pp[0], r, first);
    __syncthreads();
    wg_prod_pass<VEC, NW, false, 1>(lds, a, p.U, p.V, a.pp[1], r, mid);
    __syncthreads();
    wg_prod_pass<VEC, NW, false, 2>(lds, a, p.V, p.Z, a.pp[2], r, last);
    double acc0 = last[0], acc1 = first[1];
    wg_sum2<NW>(acc0, acc1, sh);
    s0 = acc0;
    s1 = acc1;
}

template <int VEC, int TY, int NW, int DEG, bool FIRST>
__device__ inline void wg_precondition(float* lds, const BSolve& a, const Ptrs& p, double& s0, double& s1,
                                       double (*sh)[2]) {
    if constexpr (DEG == 12) wg_precond_prod<VEC, NW, FIRST>(lds, a, p, s0, s1, sh);
    else if constexpr (DEG == 4) wg_precond_lds<VEC, NW, FIRST>(lds, a, p, s0, s1, sh);
    else wg_precond<VEC, TY, NW, FIRST>(a, p, s0, s1, sh);
}

// Right-hand sides are dealt to workgroups statically (rhs = blockIdx.x,
// blockIdx.x + gridDim.x, ...), so every loop of this kernel is controlled by
// wave-uniform values: no lane of a wave ever waits at a barrier for another
// lane of the same wave that took a different path.
template <int VEC, int TY, int NW, int DEG>
__global__ __launch_bounds__(64 * NW) void k_batched_cg(BSolve a) {
    __shared__ double sh[NW][2];
    __shared__ __align__(16) float lds[DEG == 12 ? precond_lds_floats<VEC, 4, 8, 2>()
                                                 : (DEG == 4 ? precond_lds_floats<VEC, 4, 8>() : 4)];
    const size_t cells = (size_t)a.cells;
    float* W0 = a.ws + (size_t)blockIdx.x * 5 * cells;
    float* R = W0 + cells;
    float* PA = R + cells;
    float* PB = PA + cells;
    float* Z = PB + cells;
    for (int rhs = blockIdx.x; rhs < a.n_rhs; rhs += gridDim.x) {
        float* field = a.fields + (size_t)rhs * cells;
        float* cur = field;
        float* nxt = W0;
        int worst = CGD_OK;
        for (int step = 0; step < a.n_steps; ++step) {
            if (DEG >= 4 || a.pcg) {  // degree-4 and -12 configurations run preconditioned CG only
                // preconditioned CG from x = 0: z = M b, p = z, x = alpha p, r = b - alpha A p
                Ptrs p{cur, R, nullptr, PA, nxt, Z};
                // degree 12's intermediates: both p buffers are free before
                // sweep 1 of the first iteration
                p.U = PA;
                p.V = PB;
                Ptrs q = p;  // the direction sweeps read z through Ptrs::R
                q.R = Z;
                double rho, bb, pap, rr, dummy;
                wg_precondition<VEC, TY, NW, DEG, true>(lds, a, p, rho, bb, sh);
                wg_sweep<VEC, TY, NW, S1_B0>(a, q, 0.f, 0.f, pap, dummy, sh);
                bool broken = !isfinite(bb) || !isfinite(pap) || !isfinite(rho) || (bb > 0.0 && !(pap > 0.0));
                float alpha = (broken || bb == 0.0) ? 0.f : (float)(rho / pap);
                wg_sweep<VEC, TY, NW, S2P_FIRST>(a, p, alpha, 0.f, rr, dummy, sh);
                int k = 1;
                int st = CGD_OK;
                for (;;) {
                    if (broken || !isfinite(rr)) {
                        st = CGD_E_BREAKDOWN;
                        break;
                    }
                    if (rr <= a.rtol2 * bb) break;
                    if (k >= a.max_iter) {
                        st = CGD_NOT_CONVERGED;
                        break;
                    }
                    double rho_new;
                    q.Pold = (k & 1) ? PA : PB;
                    q.Pnew = (k & 1) ? PB : PA;
                    // degree 12's intermediates: the p buffer sweep 1 is about
                    // to write, and b's buffer (dead after the first iteration;
                    // it becomes the next step's iterate)
                    p.U = q.Pnew;
                    p.V = cur;
                    wg_precondition<VEC, TY, NW, DEG, false>(lds, a, p, rho_new, dummy, sh);
                    wg_sweep<VEC, TY, NW, S1>(a, q, 0.f, (float)(rho_new / rho), pap, dummy, sh);
                    if (!(pap > 0.0) || !isfinite(pap)) {
                        broken = true;
                        continue;
                    }
                    alpha = (float)(rho_new / pap);
                    p.Pnew = q.Pnew;
                    wg_sweep<VEC, TY, NW, S2>(a, p, alpha, 0.f, rr, dummy, sh);
                    rho = rho_new;
                    ++k;
                }
                if (threadIdx.x == 0) {
                    a.iters[(size_t)rhs * a.n_steps + step] = k;
                    a.relres[(size_t)rhs * a.n_steps + step] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
                }
                if (st == CGD_E_BREAKDOWN || (st == CGD_NOT_CONVERGED && worst == CGD_OK)) worst = st;
                float* t = cur;
                cur = nxt;
                nxt = t;
                continue;
            }
            if constexpr (DEG >= 4) continue;
            Ptrs p{cur, R, nullptr, nullptr, nxt, nullptr};
            double bab, bb, rr, dummy;
            wg_sweep<VEC, TY, NW, S1_FIRST>(a, p, 0.f, 0.f, bab, bb, sh);
            bool broken = !isfinite(bb) || !isfinite(bab) || (bb > 0.0 && !(bab > 0.0));
            const float alpha0 = (broken || bb == 0.0) ? 0.f : (float)(bb / bab);
            wg_sweep<VEC, TY, NW, S2_FIRST>(a, p, alpha0, 0.f, rr, dummy, sh);
            double rr_prev = bb;
            int k = 1;
            int st = CGD_OK;
            for (;;) {
                if (broken || !isfinite(rr)) {
                    st = CGD_E_BREAKDOWN;
                    break;
                }
                if (rr <= a.rtol2 * bb) break;
                if (k >= a.max_iter) {
                    st = CGD_NOT_CONVERGED;
                    break;
                }
                p.Pold = k == 1 ? cur : ((k & 1) ? PB : PA);
                p.Pnew = (k & 1) ? PA : PB;
                const float beta = (float)(rr / rr_prev);
                double pap;
                wg_sweep<VEC, TY, NW, S1>(a, p, 0.f, beta, pap, dummy, sh);
                if (!(pap > 0.0) || !isfinite(pap)) {
                    broken = true;
                    continue;
                }
                const float alpha = (float)(rr / pap);
                double rr_new;
                wg_sweep<VEC, TY, NW, S2>(a, p, alpha, 0.f, rr_new, dummy, sh);
                rr_prev = rr;
                rr = rr_new;
                ++k;
            }
            if (threadIdx.x == 0) {
                a.iters[(size_t)rhs * a.n_steps + step] = k;
                a.relres[(size_t)rhs * a.n_steps + step] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
            }
            if (st == CGD_E_BREAKDOWN || (st == CGD_NOT_CONVERGED && worst == CGD_OK)) worst = st;
            float* t = cur;
            cur = nxt;
            nxt = t;
        }
        if (cur != field) {  // odd number of steps: the result is in the scratch vector
            for (size_t i = threadIdx.x; i < cells; i += blockDim.x) field[i] = cur[i];
            __syncthreads();
        }
        if (threadIdx.x == 0) a.status[rhs] = worst;
    }
}

// Fills n_rhs synthetic right-hand sides (a hash of the index, values in
// [0, 1)) for autotuning.
__global__ void k_fill_synthetic(float* f, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t h = (uint32_t)i * 2654435761u;
        h ^= h >> 15;
        h *= 2246822519u;
        h ^= h >> 13;
        f[i] = (float)(h >> 8) * (1.0f / 16777216.0f);
    }
}

// ---------------------------------------------------------------- configs

struct Cfg {
    int vec, ty, nw, deg;
    const void* fn;
};

// The degree-12 polynomial's three product passes (two quadratic factors
// each, the overall scale on the last).
void fill_prod12(BSolve& a) {
    double qs[6], qq[6], qg[6], scale;
    poly_precond_quadratics(a.g.cx, a.g.cy, a.g.cz, 12, qs, qq, qg, &scale);
    for (int i = 0; i < 3; ++i)
        precond_coef_fill_quadratics(a.pp[i], a.g.cx, a.g.cy, a.g.cz, qs + 2 * i, qq + 2 * i, qg + 2 * i,
                                     i == 2 ? scale : 1.0);
}

template <int VEC, int TY, int NW, int DEG>
Cfg make_cfg() {
    return Cfg{VEC, TY, NW, DEG, reinterpret_cast<const void*>(&k_batched_cg<VEC, TY, NW, DEG>)};
}

// Tile shapes of the CG sweeps (rows per wave, waves per workgroup) and the
// preconditioner degree: 2 in registers (rows per wave small enough that its
// queues fit without spilling at 16 waves), 4 through the LDS sweep (16
// waves, 8 rows of y per tile), or 12 as three LDS product passes.
std::vector<Cfg> candidates(int vec) {
    if (vec == 4)
        return {make_cfg<4, 1, 8, 2>(), make_cfg<4, 1, 16, 2>(), make_cfg<4, 2, 8, 2>(), make_cfg<4, 2, 12, 2>(),
                make_cfg<4, 1, 16, 4>(), make_cfg<4, 2, 16, 4>(), make_cfg<4, 1, 16, 12>(), make_cfg<4, 2, 16, 12>()};
    if (vec == 2)
        return {make_cfg<2, 2, 8, 2>(), make_cfg<2, 2, 16, 2>(), make_cfg<2, 4, 8, 2>(), make_cfg<2, 4, 12, 2>(),
                make_cfg<2, 2, 16, 4>(), make_cfg<2, 4, 16, 4>(), make_cfg<2, 2, 16, 12>(), make_cfg<2, 4, 16, 12>()};
    return {make_cfg<1, 4, 8, 2>(), make_cfg<1, 4, 16, 2>(), make_cfg<1, 8, 8, 2>(), make_cfg<1, 8, 16, 2>(),
            make_cfg<1, 4, 16, 4>(), make_cfg<1, 8, 16, 4>(), make_cfg<1, 4, 16, 12>(), make_cfg<1, 8, 16, 12>()};
}

int batched_vec(const HexGeom& g) {
    if (g.nx == 256) return 4;
    if (g.nx == 128) return 2;
    return g.nx == 64 ? 1 : 0;  // 0: unsupported width
}

// Resident workgroups of a configuration on this device.
int grid_for(const Cfg& c, int n_rhs) {
    int dev = 0, cus = 256, per = 1;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, c.fn, 64 * c.nw, 0) != hipSuccess || per < 1) per = 1;
    return std::max(1, std::min(n_rhs, cus * per));
}

cgd_status launch_solver(const Cfg& c, const BSolve& a, int grid, hipStream_t s) {
    void* args[] = {const_cast<BSolve*>(&a)};
    CGD_HIP_TRY(hipLaunchKernel(c.fn, dim3(grid), dim3(64 * c.nw), args, 0, s));
    return CGD_OK;
}

std::mutex g_tune_mu;
std::map<std::string, int> g_tune;  // shape key -> candidate index

std::string tune_key(const HexGeom& g, int n_rhs) {
    char name[64] = "gpu";
    hipDeviceProp_t prop;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        snprintf(name, sizeof name, "%s", prop.gcnArchName);
    for (char* q = name; *q; ++q)
        if (*q == ' ' || *q == ':') *q = '_';
    return std::string(name) + "/" + std::to_string(g.nx) + "x" + std::to_string(g.ny) + "x" +
           std::to_string(g.nz) + "/rhs" + std::to_string(std::min(n_rhs, 1024));
}

void load_tune_file() {
    const char* path = getenv("CGD_AUTOTUNE_CACHE");
    if (!path) return;
    FILE* fp = fopen(path, "r");
    if (!fp) return;
    char key[256];
    int idx;
    double ms;
    while (fscanf(fp, "%255s %d %lf", key, &idx, &ms) == 3) g_tune[key] = idx;
    fclose(fp);
}

void save_tune_file(const std::string& key, int idx, double ms) {
    const char* path = getenv("CGD_AUTOTUNE_CACHE");
    if (!path) return;
    FILE* fp = fopen(path, "a");
    if (!fp) return;
    fprintf(fp, "%s %d %.4f\n", key.c_str(), idx, ms);
    fclose(fp);
}

}  // namespace

// Workspace of the batched call: a small region (fixed part, then the
// per-right-hand-side arrays at 256-byte aligned offsets), then
// max(int64 accumulators, solver scratch).
// Byte offsets of the per-call arrays, in the device workspace and, from
// `status` on, mirrored in pinned host memory after kPinBytes: status
// [n_rhs] then iters [n_rhs][n_steps] (int32), counters [n_snap][2] (dropped,
// non-finite), maxbits [n_rhs], relres [n_rhs][n_steps], mass [2][n_rhs]
// (before, after diffusion).
struct BLayout {
    size_t maxbits, off, status, counters, relres, mass, small;
};

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static BLayout batched_layout_at(size_t start, int n_rhs, int n_snap, int n_steps) {
    BLayout L;
    L.off = start;
    L.status = align256(L.off + 8 * ((size_t)n_snap + 1));
    L.counters = align256(L.status + 4 * (size_t)n_rhs * (1 + n_steps));
    L.maxbits = align256(L.counters + 16 * (size_t)n_snap);
    L.relres = align256(L.maxbits + 4 * (size_t)n_rhs);
    L.mass = align256(L.relres + 8 * (size_t)n_rhs * n_steps);
    L.small = align256(L.mass + 16 * (size_t)n_rhs) + 4096;
    return L;
}

static BLayout batched_layout(int n_rhs, int n_snap, int n_steps) {
    return batched_layout_at(kSmallFixed, n_rhs, n_snap, n_steps);
}

struct BatchedGraph {
    std::string key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<int> budget;  // per-launch candidate: iterations per step in the captured solve
};

}  // namespace cgd

namespace cgd {

static std::mutex g_graph_mu;
static std::map<cgd_mesh, BatchedGraph> g_graphs;

void destroy_batched(cgd_mesh m) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(m);
    if (it == g_graphs.end()) return;
    if (it->second.exec) (void)hipGraphExecDestroy(it->second.exec);
    if (it->second.graph) (void)hipGraphDestroy(it->second.graph);
    g_graphs.erase(it);
}

// Right-hand sides per call of the per-launch candidate's solver.
constexpr int kGroup = CGD_MAX_FIELDS;

// Statistics of one group's solve (the small region of its workspace: int32
// iters / status and double relres, [step][CGD_MAX_FIELDS]) into the batched
// arrays (iters, relres [rhs][n_steps]; status [rhs], the worst over steps).
__global__ void k_gather_group(const int32_t* __restrict__ g_iters, const double* __restrict__ g_relres,
                               const int32_t* __restrict__ g_status, int r0, int nf, int n_steps,
                               int32_t* __restrict__ iters, double* __restrict__ relres, int32_t* __restrict__ status) {
    const int f = threadIdx.x;
    if (f >= nf) return;
    int worst = CGD_OK;
    for (int st = 0; st < n_steps; ++st) {
        iters[(size_t)(r0 + f) * n_steps + st] = g_iters[st * CGD_MAX_FIELDS + f];
        relres[(size_t)(r0 + f) * n_steps + st] = g_relres[st * CGD_MAX_FIELDS + f];
        const int v = g_status[st * CGD_MAX_FIELDS + f];
        if (v == CGD_E_BREAKDOWN || (v == CGD_NOT_CONVERGED && worst == CGD_OK)) worst = v;
    }
    status[r0 + f] = worst;
}

// The per-launch candidate: the single-call solver of cg_hex.hip (degree 12
// by default on these grids: three LDS product passes, two iterations per
// step at dtau / h^2 = 1) over groups of up to CGD_MAX_FIELDS right-hand
// sides, each launch covering all of the group's fields.  fixed: iterations
// per step (capturable) or nullptr (host read-backs).  Its workspace starts at
// `base` (diffuse_hex_workspace(m, kGroup) bytes).
static cgd_status solve_grouped(cgd_mesh m, float* fields, int n_rhs, const DiffuseArgs& da, char* base,
                                const int* fixed, int32_t* iters, double* relres, int32_t* status, hipStream_t q) {
    const bool timing = m->timing.on;
    m->timing.on = false;  // no events inside the batched call (it may be captured)
    cgd_status rc = CGD_OK;
    for (int r0 = 0; r0 < n_rhs && rc == CGD_OK; r0 += kGroup) {
        DiffuseArgs dg = da;
        dg.F = std::min(kGroup, n_rhs - r0);
        dg.field = fields + (size_t)r0 * m->cells;
        dg.x0_mode = 0;
        dg.x0 = nullptr;
        dg.model = nullptr;
        rc = diffuse_hex_enqueue(m, dg, base, fixed, false, q);
        if (rc == CGD_OK) {
            hipLaunchKernelGGL(k_gather_group, dim3(1), dim3(64), 0, q, reinterpret_cast<int32_t*>(base + kOffIters),
                               reinterpret_cast<double*>(base + kOffRelres),
                               reinterpret_cast<int32_t*>(base + kOffStatus), r0, dg.F, da.n_steps, iters, relres,
                               status);
            rc = hipGetLastError() == hipSuccess ? CGD_OK : CGD_E_HIP;
        }
    }
    m->timing.on = timing;
    return rc;
}

// Times each candidate on min(n_rhs, resident) synthetic right-hand sides
// (one backward-Euler step at dtau / h^2 = 1, solved to rtol 1e-6) and
// returns the fastest.  Candidates 0..7: the persistent launch (nx = 64, 128
// or 256 only); the last: the per-launch solver over groups of fields.
cgd_status autotune_batched(cgd_mesh m, int n_rhs, int* chosen, double* ms_out, int* n_cand) {
    const HexGeom& g = m->hex;
    const int vec = batched_vec(g);
    const std::vector<Cfg> cs = vec ? candidates(vec) : std::vector<Cfg>();
    const int nc = (int)cs.size() + 1;
    const int c_launch = (int)cs.size();
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        static bool loaded = false;
        if (!loaded) {
            load_tune_file();
            loaded = true;
        }
        auto it = g_tune.find(tune_key(g, n_rhs));
        if (it != g_tune.end() && it->second >= 0 && it->second < nc && !ms_out) {
            *chosen = it->second;
            if (n_cand) *n_cand = nc;
            return CGD_OK;
        }
    }
    int gmax = std::min(n_rhs, 4 * kGroup);
    for (const Cfg& c : cs) gmax = std::max(gmax, grid_for(c, n_rhs));
    const int nr = std::min(n_rhs, gmax);
    const size_t cells = (size_t)m->cells;
    CGD_HIP_TRY(hipDeviceSynchronize());
    const BLayout L = batched_layout(nr, 1, 1);
    const size_t small = L.small;
    const size_t scratch_bytes = std::max((size_t)gmax * 5 * cells * 4, diffuse_hex_workspace(m, kGroup));
    cgd_status rc = ensure_workspace(m, small + (size_t)nr * cells * 4 + scratch_bytes);
    if (rc != CGD_OK) return rc;
    rc = ensure_pinned(m, kPinBytes);
    if (rc != CGD_OK) return rc;
    char* base = static_cast<char*>(m->ws.ptr);
    float* fields = reinterpret_cast<float*>(base + small);
    float* scratch = fields + (size_t)nr * cells;
    int32_t* status = reinterpret_cast<int32_t*>(base + L.status);
    int32_t* iters = status + nr;
    double* relres = reinterpret_cast<double*>(base + L.relres);
    hipStream_t s = nullptr;
    CGD_HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    hipEvent_t e0, e1;
    CGD_HIP_TRY(hipEventCreate(&e0));
    CGD_HIP_TRY(hipEventCreate(&e1));
    BSolve a = {};
    a.fields = fields;
    a.ws = scratch;
    a.n_rhs = nr;
    a.cells = (int64_t)cells;
    a.g.nx = g.nx;
    a.g.ny = g.ny;
    a.g.nz = g.nz;
    a.g.cx = a.g.cy = a.g.cz = 1.0f;
    a.pcg = 1;  // the default solver is what gets tuned
    poly_precond_coeffs(1.0, 1.0, 1.0, 2, &a.g.c0, &a.g.c1, &a.g.c2);
    {
        double c4[8];
        poly_precond_coeffs_n(1.0, 1.0, 1.0, 4, c4);
        precond_coef_fill(a.pc, a.g.cx, a.g.cy, a.g.cz, c4, 4);
        fill_prod12(a);
    }
    // time to solution (rtol 1e-6), so that candidates of different
    // preconditioner degree compare fairly
    a.n_steps = 1;
    a.rtol2 = 1e-12;
    a.max_iter = 100;
    a.iters = iters;
    a.relres = relres;
    a.status = status;
    // the per-launch candidate: the same step (dtau = h_x^2, so c_x = 1)
    DiffuseArgs dl = {};
    dl.bandwidth = 2.0 * g.h[0];
    dl.n_steps = 1;
    dl.rtol = 1e-6;
    dl.max_iter = 100;
    dl.check_every = 4;
    double best = 1e30;
    int best_i = 0;
    for (int i = 0; i < nc; ++i) {
        double ms_best = 1e30;
        for (int rep = 0; rep < 3; ++rep) {
            hipLaunchKernelGGL(k_fill_synthetic, dim3(2048), dim3(256), 0, s, fields, (int64_t)(nr * cells));
            CGD_HIP_TRY(hipEventRecord(e0, s));
            if (i == c_launch) {
                rc = solve_grouped(m, fields, nr, dl, reinterpret_cast<char*>(scratch), nullptr, iters, relres,
                                   status, s);
            } else {
                const Cfg& c = cs[i];
                a.xsegs = 1;
                a.ygroups = (g.ny + c.ty - 1) / c.ty;
                rc = launch_solver(c, a, grid_for(c, nr), s);
            }
            if (rc != CGD_OK) break;
            CGD_HIP_TRY(hipEventRecord(e1, s));
            CGD_HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            CGD_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) ms_best = std::min(ms_best, (double)ms);
        }
        if (rc != CGD_OK) break;
        if (ms_out) ms_out[i] = ms_best;
        if (ms_best < best) {
            best = ms_best;
            best_i = i;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    if (rc != CGD_OK) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        const std::string key = tune_key(g, n_rhs);
        g_tune[key] = best_i;
        save_tune_file(key, best_i, best);
    }
    *chosen = best_i;
    if (n_cand) *n_cand = nc;
    return CGD_OK;
}

cgd_status coarse_grain_batched(cgd_mesh m, int32_t n_snap, const int64_t* offsets, const float* pos, int32_t F,
                                const float* values, const DiffuseArgs& da, float* fields, cgd_solve_stats* st_out,
                                hipStream_t s) {
    const HexGeom& g = m->hex;
    const int n_rhs = n_snap * F;
    const int64_t total = offsets[n_snap];
    const size_t cells = (size_t)m->cells;
    int ci = 0;
    cgd_status rc = autotune_batched(m, n_rhs, &ci, nullptr, nullptr);
    if (rc != CGD_OK) return rc;
    const int vec = batched_vec(g);
    const std::vector<Cfg> cands = vec ? candidates(vec) : std::vector<Cfg>();
    const int c_launch = (int)cands.size();
    if (const char* e = getenv("CGD_BATCHED_CFG")) {  // a fixed candidate, for tests and tuning runs
        const int v = atoi(e);
        if (v >= 0 && v <= c_launch) ci = v;
    }
    const bool per_launch = ci == c_launch;
    Cfg c = {};
    if (!per_launch) {
        c = cands[ci];
        if (da.precond != 0 && c.deg >= 4) {
            // plain CG: the degree-2 configuration of the same shape (else the
            // 16-wave one), whose kernel carries the unpreconditioned path
            int alt = -1;
            for (int i = 0; i < (int)cands.size(); ++i)
                if (cands[i].deg == 2 && cands[i].ty == c.ty && cands[i].nw == c.nw) alt = i;
            if (alt < 0)
                for (int i = 0; i < (int)cands.size(); ++i)
                    if (cands[i].deg == 2 && cands[i].nw == 16) alt = i;
            ci = alt;
            c = cands[ci];
        }
    }
    const int grid = per_launch ? 0 : grid_for(c, n_rhs);
    const BLayout L = batched_layout(n_rhs, n_snap, da.n_steps);
    const size_t small = L.small;
    // deposit: the tiled path's bucketed records, else int64 accumulators
    const size_t tile_bytes = tiled_deposit_temp_bytes((int64_t)cells, total, n_snap, F);
    const bool tiled = tile_bytes > 0;
    const size_t dep_bytes = tiled ? tile_bytes : (size_t)n_rhs * cells * 8;
    const size_t solver_bytes = per_launch ? diffuse_hex_workspace(m, std::min(kGroup, n_rhs))
                                           : (size_t)grid * 5 * cells * 4;
    rc = ensure_workspace(m, small + std::max(dep_bytes, solver_bytes));
    if (rc != CGD_OK) return rc;
    // the same arrays in pinned host memory, after the region the other calls use
    const BLayout P = batched_layout_at(kPinBytes, n_rhs, n_snap, da.n_steps);
    rc = ensure_pinned(m, P.small);
    if (rc != CGD_OK) return rc;

    char* base = static_cast<char*>(m->ws.ptr);
    char* pin = static_cast<char*>(m->pinned);
    unsigned long long* d_counters = reinterpret_cast<unsigned long long*>(base + L.counters);
    uint32_t* d_maxbits = reinterpret_cast<uint32_t*>(base + L.maxbits);
    int64_t* d_off = reinterpret_cast<int64_t*>(base + L.off);
    int32_t* d_status = reinterpret_cast<int32_t*>(base + L.status);
    int32_t* d_iters = d_status + n_rhs;
    double* d_relres = reinterpret_cast<double*>(base + L.relres);
    double* d_mass = reinterpret_cast<double*>(base + L.mass);
    void* big = base + small;
    int64_t* h_off = reinterpret_cast<int64_t*>(pin + P.off);
    int32_t* h_status = reinterpret_cast<int32_t*>(pin + P.status);
    int32_t* h_iters = h_status + n_rhs;
    unsigned long long* h_counters = reinterpret_cast<unsigned long long*>(pin + P.counters);
    uint32_t* h_maxbits = reinterpret_cast<uint32_t*>(pin + P.maxbits);
    double* h_relres = reinterpret_cast<double*>(pin + P.relres);
    double* h_mass = reinterpret_cast<double*>(pin + P.mass);
    memcpy(h_off, offsets, 8 * ((size_t)n_snap + 1));
    const bool want_mass = st_out != nullptr;

    BDep d = {};
    d.off = d_off;
    d.pos = pos;
    d.values = values;
    d.total = total;
    d.n_snap = n_snap;
    d.F = F;
    d.maxbits = d_maxbits;
    d.acc = static_cast<unsigned long long*>(big);
    d.fields = fields;
    d.counters = d_counters;
    d.cells = (int64_t)cells;
    d.vol = g.vol;
    for (int a = 0; a < 3; ++a) {
        d.g.lo[a] = g.lo[a];
        d.g.hi[a] = g.hi[a];
        d.g.s[a] = g.s[a];
    }
    d.g.n[0] = g.nx;
    d.g.n[1] = g.ny;
    d.g.n[2] = g.nz;
    int64_t max_n = 0;
    for (int j = 0; j < n_snap; ++j) max_n = std::max(max_n, offsets[j + 1] - offsets[j]);
    const int chunks = (int)std::max<int64_t>(1, (max_n + kChunk - 1) / kChunk);

    // Crank-Nicolson: the half-step solve, its extrapolation carried by the
    // x updates (every right-hand side starts from a zero guess)
    const double dtau = da.bandwidth * da.bandwidth / 4.0 / da.n_steps * (da.scheme == 1 ? 0.5 : 1.0);
    BSolve a = {};
    a.fields = fields;
    a.g.xs1 = da.scheme == 1 ? 1.f : 0.f;
    a.g.xb = da.scheme == 1 ? -1.f : 0.f;
    a.ws = static_cast<float*>(big);
    a.n_rhs = n_rhs;
    a.cells = (int64_t)cells;
    a.g.nx = g.nx;
    a.g.ny = g.ny;
    a.g.nz = g.nz;
    a.g.cx = (float)(dtau / (g.h[0] * g.h[0]));
    a.g.cy = (float)(dtau / (g.h[1] * g.h[1]));
    a.g.cz = (float)(dtau / (g.h[2] * g.h[2]));
    a.pcg = da.precond == 0 ? 1 : 0;
    poly_precond_coeffs(a.g.cx, a.g.cy, a.g.cz, 2, &a.g.c0, &a.g.c1, &a.g.c2);
    {
        double c4[8];
        poly_precond_coeffs_n(a.g.cx, a.g.cy, a.g.cz, 4, c4);
        precond_coef_fill(a.pc, a.g.cx, a.g.cy, a.g.cz, c4, 4);
        fill_prod12(a);
    }
    a.xsegs = 1;
    a.ygroups = per_launch ? 1 : (g.ny + c.ty - 1) / c.ty;
    a.n_steps = da.n_steps;
    a.rtol2 = da.rtol * da.rtol;
    a.max_iter = da.max_iter;
    a.iters = d_iters;
    a.relres = d_relres;
    a.status = d_status;

    // everything the call does, in stream order; budget: the per-launch
    // solver's iterations per step (nullptr: host read-backs, not capturable)
    auto enqueue_all = [&](hipStream_t q, const int* budget) -> cgd_status {
        CGD_HIP_TRY(hipMemcpyAsync(d_off, h_off, 8 * ((size_t)n_snap + 1), hipMemcpyHostToDevice, q));
        hipLaunchKernelGGL(k_bdep_init, dim3((std::max(n_rhs, 2 * n_snap) + 255) / 256), dim3(256), 0, q, d);
        if (tiled) {
            TiledDeposit td = {};
            td.pos = pos;
            td.values = values;
            td.total = total;
            td.max_n = max_n;
            td.off = d_off;
            td.n_snap = n_snap;
            td.F = F;
            td.maxbits = d_maxbits;
            // per snapshot: one count of non-finite positions and values
            td.nf_val = d_counters + 1;
            td.nf_val_stride = 0;
            td.cnt_jstride = 2;
            td.dropped = d_counters;
            td.nf_pos = d_counters + 1;
            td.field = fields;
            td.acc = nullptr;
            td.temp = big;
            cgd_status r = tiled_deposit(m, td, nullptr, q);
            if (r != CGD_OK) return r;
        } else {
            hipLaunchKernelGGL(k_bzero, dim3(8192), dim3(256), 0, q, d.acc, (int64_t)(n_rhs * cells));
            if (total > 0) {
                hipLaunchKernelGGL(k_babsmax, dim3(chunks, n_rhs), dim3(kDBlock), 0, q, d);
                hipLaunchKernelGGL(k_bdeposit, dim3(chunks, n_snap), dim3(kDBlock), 0, q, d);
            }
            hipLaunchKernelGGL(k_bfinalize, dim3(512, n_rhs), dim3(kDBlock), 0, q, d);
        }
        if (want_mass) hipLaunchKernelGGL(k_bmass, dim3(n_rhs), dim3(1024), 0, q, fields, a.cells, g.vol, d_mass);
        cgd_status r = per_launch ? solve_grouped(m, fields, n_rhs, da, static_cast<char*>(big), budget, d_iters,
                                                  d_relres, d_status, q)
                                  : launch_solver(c, a, grid, q);
        if (r != CGD_OK) return r;
        if (want_mass)
            hipLaunchKernelGGL(k_bmass, dim3(n_rhs), dim3(1024), 0, q, fields, a.cells, g.vol, d_mass + n_rhs);
        // status, iters, counters, maxbits, relres (and mass) in one copy
        const size_t upto = want_mass ? L.mass + 16 * (size_t)n_rhs : L.relres + 8 * (size_t)n_rhs * da.n_steps;
        CGD_HIP_TRY(hipMemcpyAsync(pin + P.status, base + L.status, upto - L.status, hipMemcpyDeviceToHost, q));
        return CGD_OK;
    };
    // the per-launch solver's iterations per step of a finished eager run:
    // the most any right-hand side took (the budget of the captured graph)
    auto budget_of = [&]() {
        std::vector<int> b(da.n_steps, 1);
        for (int r = 0; r < n_rhs; ++r)
            for (int k = 0; k < da.n_steps; ++k) b[k] = std::max(b[k], (int)h_iters[(size_t)r * da.n_steps + k]);
        return b;
    };
    auto not_converged = [&]() {
        for (int r = 0; r < n_rhs; ++r)
            if (h_status[r] == CGD_NOT_CONVERGED) return true;
        return false;
    };

    const bool use_graph = getenv("CGD_NO_GRAPH") == nullptr;
    if (use_graph) {
        char keybuf[512];
        snprintf(keybuf, sizeof keybuf, "%p %p %p %d %d %lld %d %d %.17g %.17g %d %d %p %zu %p %d %d %d",
                 (const void*)pos, (const void*)values, (void*)fields, n_snap, F, (long long)total, chunks,
                 da.n_steps, da.bandwidth, da.rtol, da.max_iter, ci, m->ws.ptr, m->ws.bytes, m->pinned, a.pcg,
                 (int)tiled, da.scheme * 2 + (int)want_mass);
        std::lock_guard<std::mutex> lk(g_graph_mu);
        BatchedGraph& bg = g_graphs[m];
        auto drop = [&]() {
            if (bg.exec) (void)hipGraphExecDestroy(bg.exec);
            if (bg.graph) (void)hipGraphDestroy(bg.graph);
            bg.exec = nullptr;
            bg.graph = nullptr;
            bg.key.clear();
        };
        auto capture = [&](const int* budget) -> cgd_status {
            hipStream_t cap = nullptr;
            CGD_HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            CGD_HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
            cgd_status r = enqueue_all(cap, budget);
            hipGraph_t graph = nullptr;
            hipError_t ee = hipStreamEndCapture(cap, &graph);
            (void)hipStreamDestroy(cap);
            if (r != CGD_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return r;
            }
            if (ee != hipSuccess) {
                set_error(std::string("batched graph capture failed: ") + hipGetErrorString(ee));
                return CGD_E_HIP;
            }
            bg.graph = graph;
            CGD_HIP_TRY(hipGraphInstantiate(&bg.exec, graph, nullptr, nullptr, 0));
            bg.key = keybuf;
            return CGD_OK;
        };
        if (bg.key != keybuf || !bg.exec) {
            drop();
            if (per_launch) {
                // one eager run with read-backs learns the iterations per step;
                // the graph captured after it replays them as fixed budgets
                rc = enqueue_all(s, nullptr);
                if (rc != CGD_OK) return rc;
                CGD_HIP_TRY(hipStreamSynchronize(s));
                bg.budget = budget_of();
                rc = capture(bg.budget.data());
                if (rc != CGD_OK) return rc;
            } else {
                rc = capture(nullptr);
                if (rc != CGD_OK) return rc;
                CGD_HIP_TRY(hipGraphLaunch(bg.exec, s));
                CGD_HIP_TRY(hipStreamSynchronize(s));
            }
        } else {
            CGD_HIP_TRY(hipGraphLaunch(bg.exec, s));
            CGD_HIP_TRY(hipStreamSynchronize(s));
            if (per_launch && not_converged()) {
                // a right-hand side needed more iterations than the budget:
                // the call again with read-backs, and a new graph next time
                drop();
                rc = enqueue_all(s, nullptr);
                if (rc != CGD_OK) return rc;
                CGD_HIP_TRY(hipStreamSynchronize(s));
                bg.budget = budget_of();
            }
        }
    } else {
        rc = enqueue_all(s, nullptr);
        if (rc != CGD_OK) return rc;
        CGD_HIP_TRY(hipStreamSynchronize(s));
    }
    cgd_status worst = CGD_OK;
    for (int r = 0; r < n_rhs; ++r) {
        if (h_status[r] == CGD_E_BREAKDOWN) {
            set_error("CG breakdown in right-hand side " + std::to_string(r));
            worst = CGD_E_BREAKDOWN;
        } else if (h_status[r] == CGD_NOT_CONVERGED && worst == CGD_OK) {
            worst = CGD_NOT_CONVERGED;
        }
    }
    unsigned long long nonfinite = 0;
    for (int j = 0; j < n_snap; ++j) nonfinite += h_counters[2 * j + 1];
    if (st_out) {
        for (int j = 0; j < n_snap; ++j) {
            cgd_solve_stats& st = st_out[j];
            memset(&st, 0, sizeof st);
            st.n_steps = da.n_steps;
            st.n_fields = F;
            const int e_n = ceil_log2_count(offsets[j + 1] - offsets[j]);
            int32_t sworst = CGD_OK;
            for (int f = 0; f < F; ++f) {
                const int r = j * F + f;
                for (int k = 0; k < da.n_steps; ++k) {
                    st.iters[k][f] = h_iters[(size_t)r * da.n_steps + k];
                    st.rel_res[k][f] = h_relres[(size_t)r * da.n_steps + k];
                }
                st.mass_before[f] = h_mass[r];
                st.mass_after[f] = h_mass[n_rhs + r];
                int S = 0;
                if (const uint32_t mb = h_maxbits[r]) {
                    float mv;
                    memcpy(&mv, &mb, 4);
                    int e;
                    (void)frexp((double)mv, &e);
                    S = 62 - e - e_n;
                }
                st.frac_bits[f] = S;
                if (h_status[r] == CGD_E_BREAKDOWN) sworst = CGD_E_BREAKDOWN;
                else if (h_status[r] == CGD_NOT_CONVERGED && sworst == CGD_OK) sworst = CGD_NOT_CONVERGED;
            }
            st.n_dropped = (int64_t)h_counters[2 * j];
            st.n_nonfinite = (int64_t)h_counters[2 * j + 1];
            if (sworst == CGD_OK && st.n_nonfinite) sworst = CGD_E_NONFINITE;
            st.status = sworst;
        }
    }
    if (worst == CGD_OK && nonfinite) {
        set_error("non-finite particle positions or values were skipped");
        worst = CGD_E_NONFINITE;
    }
    return worst;
}

}  // namespace cgd
