// Backward-Euler diffusion on uniform hex grids by conjugate gradients with a
// matrix-free 7-point stencil (Sections 3.2 and 5.1).
//
// Each pseudo-step solves A x = b with A = I + dtau K / V (the finite-volume
// Laplacian K divided by the uniform cell volume, so that A stays symmetric
// positive definite): (A p)_k = p_k + sum_a c_a (2 p_k - p_k-1 - p_k+1) with
// c_a = dtau / h_a^2, where a missing neighbour at a wall is replaced by p_k
// itself (zero flux through wall faces, Section 3.2.2).  Crank-Nicolson
// (Section 5.1) runs the same solve with dtau / 2 and takes 2 x - b: from a
// zero guess the x updates carry it, after a guess a pass sets it.
//
// One CG iteration k is two streaming sweeps over the grid, 32 bytes per cell:
//   sweep 1: p = r + beta p_old (also recomputed at neighbours), A p, p.Ap
//            reads r, p_old; writes p
//   sweep 2: x += alpha p, r -= alpha A p (A p recomputed), r.r
//            reads p, x, r; writes x, r
// Global scalars need no extra launches: every block of a sweep first sums
// the float64 block partials of the sweep before it, in one fixed order, so
// all blocks obtain bit-identical alpha / beta; the first block also records
// the convergence state for later kernels and for the host.
//
// Sweep layout: a wave owns 64 * VEC consecutive x (VEC per lane) times TY
// rows of y and marches over a chunk of z planes, keeping planes z-1, z, z+1
// (with one halo row on each side) in registers.  x-neighbours come from lane
// shuffles.  Blocks of 4 waves are spread so that consecutive tiles land on
// the same XCD (workgroups are dealt round-robin over the 8 XCDs), which
// keeps halo rows in that XCD's L2.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "cg_common.h"
#include "precond_lds.h"
#include "stencil_tile.h"

namespace cgd {
namespace {

constexpr int kWaves = kCgWaves;
constexpr int kBlock = kCgBlock;

using namespace stencil;

struct SweepArgs {
    Ptrs p;
    Geom g;
    CgCtl c;
    // Block partial sums, [F][2][pstride] each; a sweep writes one entry per
    // block (bpf of its own plan) and the next sweep's prologue adds the
    // bpf_in entries the producing sweep wrote (each kind of sweep has its
    // own tile plan).
    double* P1;         // slot 0 p.Ap, slot 1 b.b
    double* P2;         // r.r of r_k in slot k % 2
    double* P3;         // preconditioned CG: r.z of r_k in slot k % 2
    int pstride, bpf_in;
    int pcg;            // 1: preconditioned CG (the S1 modes read z; alpha, beta from r.z)
    int x0_zero;        // the step started from a zero initial guess
    int64_t cells;
    int nx, ny, nz;
    int xsegs, ygroups, zc;
    int wpf, bpf, nblocks;
    int k;              // iteration index within the step
    PrecondCoef pc;     // k_precond_lds: Horner levels of M = sum_j cp[j] A^j, or the first product pass
    PrecondCoef pc2;    // the last product pass (degrees 8 and 12)
    PrecondCoef pcm;    // the middle product pass (degree 12)
    int rect;           // the rectilinear operator (Geom's per-axis factors; register sweeps only)
};

// One sweep over all fields: each wave takes one tile (stencil_tile.h).
template <int VEC, int TY, int MODE, bool EDGE, bool RECT = false>
__global__ __launch_bounds__(kBlock) void k_sweep(SweepArgs a) {
    int b = blockIdx.x;
    if ((a.nblocks & 7) == 0) b = (b & 7) * (a.nblocks >> 3) + (b >> 3);
    const int f = b / a.bpf;
    const int blk = b - f * a.bpf;
    CgField* stf = a.c.st + f;
    if constexpr (MODE == S2 || MODE == S2_FIRST || MODE == S2P_FIRST) post_ndone(a.c);
    // S2_FIRST / S2P_FIRST must write x and r even when their first block
    // flags a breakdown.
    if (MODE != S2_FIRST && MODE != S2P_FIRST && stf->done) return;  // uniform over the block

    __shared__ double sh[kWaves];
    const bool lead = blk == 0 && threadIdx.x == 0;
    float alpha = 0.f, beta = 0.f;
    if constexpr (MODE == SZ || MODE == SZ2) {
        // preconditioned CG: convergence test on r_k . r_k from the previous
        // sweep 2 (or, at k = 0, the residual sweep, which also gave b.b)
        const double rrk = block_sum_fixed(a.P2 + ((size_t)f * 2 + (a.k & 1)) * a.pstride, a.bpf_in, sh);
        double bb;
        if (a.k == 0) bb = block_sum_fixed(a.P1 + ((size_t)f * 2 + 1) * a.pstride, a.bpf_in, sh);
        else bb = stf->bb;
        if (lead) {
            stf->rr_par[a.k & 1] = rrk;
            if (a.k == 0) stf->bb = bb;
        }
        if (check_stop(a.c, f, a.k, rrk, bb, lead)) return;
    } else if ((MODE == S1 || MODE == S1_B0) && a.pcg) {
        // rho_k = r_k . z_k from the preconditioning sweep
        const double rho = block_sum_fixed(a.P3 + ((size_t)f * 2 + (a.k & 1)) * a.pstride, a.bpf_in, sh);
        double bb = 0.0;
        // zero initial guess: b.b comes from the first preconditioning sweep
        // (a warm start had it from the residual sweep, in the SZ prologue)
        const bool need_bb = MODE == S1_B0 && a.x0_zero;
        if (need_bb) bb = block_sum_fixed(a.P1 + ((size_t)f * 2 + 1) * a.pstride, a.bpf_in, sh);
        if (lead) {
            stf->rho_par[a.k & 1] = rho;
            if (need_bb) {
                stf->bb = bb;
                stf->rr_par[0] = bb;
            }
        }
        if (MODE == S1) beta = (float)(rho / stf->rho_par[(a.k - 1) & 1]);
    } else if constexpr (MODE == S1 || MODE == S1_B0) {
        // r_k . r_k from the previous sweep 2 (or the residual sweep)
        const double rrk = block_sum_fixed(a.P2 + ((size_t)f * 2 + (a.k & 1)) * a.pstride, a.bpf_in, sh);
        double bb;
        if constexpr (MODE == S1_B0) bb = block_sum_fixed(a.P1 + ((size_t)f * 2 + 1) * a.pstride, a.bpf_in, sh);
        else bb = stf->bb;
        if (lead) {
            stf->rr_par[a.k & 1] = rrk;
            if (MODE == S1_B0) stf->bb = bb;
        }
        if (check_stop(a.c, f, a.k, rrk, bb, lead)) return;
        if constexpr (MODE == S1) beta = (float)(rrk / stf->rr_par[(a.k - 1) & 1]);
    } else if constexpr (MODE == S2P_FIRST) {
        // preconditioned CG, zero initial guess: alpha = rho_0 / p.Ap; b = 0 or
        // a breakdown gives alpha = 0, i.e. x = 0 and r = b
        const double pap = block_sum_fixed(a.P1 + ((size_t)f * 2 + 0) * a.pstride, a.bpf_in, sh);
        const double bb = stf->bb, rho = stf->rho_par[0];
        const bool broken = !isfinite(bb) || !isfinite(pap) || !isfinite(rho) || (bb > 0.0 && !(pap > 0.0));
        if (lead && broken) finish_field(a.c, f, CGD_E_BREAKDOWN);
        alpha = (broken || bb == 0.0) ? 0.f : (float)(rho / pap);
    } else if constexpr (MODE == S2 || MODE == S2_FIRST) {
        const double pap = block_sum_fixed(a.P1 + ((size_t)f * 2 + 0) * a.pstride, a.bpf_in, sh);
        if constexpr (MODE == S2_FIRST) {
            const double bb = block_sum_fixed(a.P1 + ((size_t)f * 2 + 1) * a.pstride, a.bpf_in, sh);
            const bool broken = !isfinite(bb) || !isfinite(pap) || (bb > 0.0 && !(pap > 0.0));
            if (lead) {
                stf->bb = bb;
                stf->rr_par[0] = bb;
                if (broken) finish_field(a.c, f, CGD_E_BREAKDOWN);
            }
            // b = 0 or a breakdown: alpha = 0 gives x = 0, r = b
            alpha = (broken || bb == 0.0) ? 0.f : (float)(bb / pap);
        } else {
            const double rrk = a.pcg ? stf->rho_par[a.k & 1] : stf->rr_par[a.k & 1];
            if (!(pap > 0.0) || !isfinite(pap)) {
                if (lead) finish_field(a.c, f, CGD_E_BREAKDOWN);
                return;
            }
            alpha = (float)(rrk / pap);
        }
    }

    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int w = blk * kWaves + wave;
    double acc0 = 0.0, acc1 = 0.0;

    if (w < a.wpf) {
        const int xs = w % a.xsegs;
        const int t = w / a.xsegs;
        const int yg = t % a.ygroups;
        const int zci = t / a.ygroups;
        const int zb = zci * a.zc;
        const int ze = min(zb + a.zc, a.nz);
        if constexpr (MODE == SZ2_FIRST || MODE == SZ2) {
            if constexpr (!EDGE)
                tile_precond2<VEC, TY, MODE == SZ2_FIRST, RECT>(a.p, a.g, (size_t)f * a.cells, yg, zb, ze, lane, acc0,
                                                                acc1);
        } else {
            tile_sweep<VEC, TY, MODE, EDGE, RECT>(a.p, a.g, (size_t)f * a.cells, xs, yg, zb, ze, lane, alpha, beta,
                                                  acc0, acc1);
        }
    }

    // block reduction of the float64 partials, fixed order
    constexpr bool kTwo = (MODE == S1_FIRST || MODE == S_RES || MODE == SZ_FIRST || MODE == SZ2_FIRST);
    for (int o = 32; o > 0; o >>= 1) {
        acc0 += __shfl_xor(acc0, o);
        if (kTwo) acc1 += __shfl_xor(acc1, o);
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
        // where each mode's sums go (see SweepArgs)
        if constexpr (MODE == S1_FIRST || MODE == S1 || MODE == S1_B0) {
            a.P1[((size_t)f * 2 + 0) * a.pstride + blk] = t0;
            if (MODE == S1_FIRST) a.P1[((size_t)f * 2 + 1) * a.pstride + blk] = t1;
        } else if constexpr (MODE == S2_FIRST || MODE == S2 || MODE == S2P_FIRST) {
            a.P2[((size_t)f * 2 + ((a.k + 1) & 1)) * a.pstride + blk] = t0;
        } else if constexpr (MODE == SZ_FIRST || MODE == SZ || MODE == SZ2_FIRST || MODE == SZ2) {
            a.P3[((size_t)f * 2 + (a.k & 1)) * a.pstride + blk] = t0;
            if (MODE == SZ_FIRST || MODE == SZ2_FIRST) a.P1[((size_t)f * 2 + 1) * a.pstride + blk] = t1;
        } else {  // S_RES: r_0 . r_0 and b . b
            a.P2[((size_t)f * 2 + 0) * a.pstride + blk] = t0;
            a.P1[((size_t)f * 2 + 1) * a.pstride + blk] = t1;
        }
    }
}

// Direction sweep of preconditioned CG with the rows shared through LDS:
// p = z + beta p_old, A p and p.Ap, writing p; when B0, p = z, which is not
// written again (the caller uses z's buffer as p).  A block of NW
// waves owns NW - 2 rows of y (one wave per x-row, nx = 64 VEC; the first
// and last wave carry the halo rows) and marches over its z chunk; each row
// is loaded once, so the halo costs 2 / (NW - 2) in L2 reads instead of the
// register sweep's 2 / TY.  At step t every wave forms p of its row at plane
// t from the loads issued one step earlier, keeps it in a 3-plane register
// ring and in LDS (3 plane slots), and after one barrier forms A p at plane
// t - 1 from its own planes t - 2 .. t, the rows above and below from LDS
// and the x-neighbours by DPP shifts.  Rows and planes beyond a wall take the
// cell itself.
template <int VEC, int NW, bool B0, bool PART = false>
__global__ __launch_bounds__(NW * 64) void k_dir_lds(SweepArgs a) {
    constexpr int NT = NW * 64;
    constexpr int NXR = 64 * VEC;
    constexpr int TY = NW - 2;
    __shared__ double sh[NW];
    __shared__ __align__(16) float lds[3 * NW * NXR];

    int b = blockIdx.x;
    if ((a.nblocks & 7) == 0) b = (b & 7) * (a.nblocks >> 3) + (b >> 3);
    const int f = b / a.bpf;
    const int blk = b - f * a.bpf;
    CgField* stf = a.c.st + f;
    if (stf->done) return;  // uniform over the block
    const bool lead = blk == 0 && threadIdx.x == 0;
    float beta = 0.f;
    {
        // rho_k = r_k . z_k from the preconditioning sweep
        const double rho = block_sum_nt<NT>(a.P3 + ((size_t)f * 2 + (a.k & 1)) * a.pstride, a.bpf_in, sh);
        double bb = 0.0;
        // zero initial guess: b.b comes from the first preconditioning sweep
        const bool need_bb = B0 && a.x0_zero;
        if (need_bb) bb = block_sum_nt<NT>(a.P1 + ((size_t)f * 2 + 1) * a.pstride, a.bpf_in, sh);
        if (lead) {
            stf->rho_par[a.k & 1] = rho;
            if (need_bb) {
                stf->bb = bb;
                stf->rr_par[0] = bb;
            }
        }
        if (!B0) beta = (float)(rho / stf->rho_par[(a.k - 1) & 1]);
    }

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // rows of nx <= NXR cells: lanes from nx / VEC on load the row's last
    // cells, store nothing and add nothing; the last real lane has the wall
    const int nx = a.nx;
    const int ny = a.ny, nz = a.nz;
    const int x0 = lane * VEC;
    const bool xin = x0 < nx;
    const int yg = blk % a.ygroups, zci = blk / a.ygroups;
    const int y0 = yg * TY, zb = zci * a.zc, ze = min(zb + a.zc, nz);
    const size_t plane = (size_t)nx * ny;
    const size_t fo = (size_t)f * a.cells + (xin ? x0 : nx - VEC);
    const Geom& g = a.g;

    const int yw = y0 - 1 + w;  // this wave's row
    const bool in_dom = yw >= 0 && yw < ny;
    const bool owner = w >= 1 && w <= TY && yw < ny;
    const bool has_yd = yw > 0, has_yu = yw + 1 < ny;
    const int yc = yw < 0 ? 0 : (yw >= ny ? ny - 1 : yw);
    const float* zsrc = a.p.R + fo + (size_t)yc * nx;  // the S1 modes read z through Ptrs::R
    const float* psrc = a.p.Pold + fo + (size_t)yc * nx;
    float* pdst = a.p.Pnew + fo + (size_t)yc * nx;
    auto row = [&](int q, int wr) -> float* { return lds + ((q % 3) * NW + wr) * NXR + x0; };
    auto ld = [](const float* r) { return ldv<VEC>(static_cast<const float*>(__builtin_assume_aligned(r, 4 * VEC))); };
    const float cx = g.cx, cy = g.cy, cz = g.cz;
    const float d_in = 1.f + 2.f * (cx + cy + cz);

    // planes of p needed: zb - 1 .. ze (within the grid); A p at zb .. ze - 1
    const int t0 = max(0, zb - 1);
    const int tl = min(nz - 1, ze);
    Vec<VEC> zr, pr;  // loads of the next plane
    auto load = [&](int t) {
        const size_t o = (size_t)min(t, tl) * plane;
        zr = ldv<VEC>(zsrc + o);
        if constexpr (!B0) pr = ldv<VEC>(psrc + o);
    };
    Vec<VEC> ring[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int e = 0; e < VEC; ++e) ring[i].f[e] = 0.f;
    double acc = 0.0;
    load(t0);

    // step t: p of plane t, then A p of plane t - 1 (ring slot of plane t0 + s is s mod 3)
    auto step = [&](auto S_, int t) {
        constexpr int S = decltype(S_)::value;
        Vec<VEC> pv;
#pragma unroll
        for (int e = 0; e < VEC; ++e) pv.f[e] = 0.f;
        if (t <= tl) {
            pv = zr;
            if constexpr (!B0) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) pv.f[e] = fmaf(beta, pr.f[e], zr.f[e]);
            }
            load(t + 1);
            if (in_dom) {
                stv<VEC>(row(t, w), pv);
                // B0: p_0 = z_0, which the caller keeps in place of p
                if (!B0 && owner && xin && t >= zb && t < ze) stv<VEC>(pdst + (size_t)t * plane, pv);
            }
        }
        ring[S % 3] = pv;
        lds_barrier();
        const int q = t - 1;
        if (owner && xin && q >= zb && q < ze) {
            const Vec<VEC>& c = ring[(S + 2) % 3];   // plane q
            const Vec<VEC>& zl = ring[(S + 1) % 3];  // plane q - 1
            const Vec<VEC>& zh = ring[S % 3];        // plane q + 1
            Vec<VEC> ys = ld(row(q, has_yd ? w - 1 : w));
            {
                const Vec<VEC> yh = ld(row(q, has_yu ? w + 1 : w));
#pragma unroll
                for (int e = 0; e < VEC; ++e) ys.f[e] += yh.f[e];
            }
            float lft, rgt;
            x_neighbours<VEC>(c, lft, rgt);
            if constexpr (PART) rgt = x0 + VEC >= nx ? c.f[VEC - 1] : rgt;  // a row shorter than the wave
            const bool hzd = q > 0, hzu = q + 1 < nz;
            const float czd = hzd ? cz : 0.f, czu = hzu ? cz : 0.f;
            const float dq = d_in - (hzd ? 0.f : cz) - (hzu ? 0.f : cz);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const float l = e > 0 ? c.f[e - 1] : lft;
                const float r = e + 1 < VEC ? c.f[e + 1] : rgt;
                float v = dq * c.f[e];
                v = fmaf(-cx, l + r, v);
                v = fmaf(-cy, ys.f[e], v);
                v = fmaf(-czd, zl.f[e], v);
                v = fmaf(-czu, zh.f[e], v);
                acc = fma((double)c.f[e], (double)v, acc);
            }
        }
    };
    for (int t = t0; t <= tl + 1; t += 3) {
        step(std::integral_constant<int, 0>{}, t);
        if (t + 1 > tl + 1) break;
        step(std::integral_constant<int, 1>{}, t + 1);
        if (t + 2 > tl + 1) break;
        step(std::integral_constant<int, 2>{}, t + 2);
    }

    // block reduction, fixed order: p.Ap into P1 slot 0
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) sh[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double u = 0.0;
#pragma unroll
        for (int i = 0; i < NW; ++i) u += sh[i];
        a.P1[((size_t)f * 2 + 0) * a.pstride + blk] = u;
    }
}

// The degree-D preconditioning sweep of preconditioned CG (precond_lds.h):
// convergence test first (as the register sweeps' SZ prologue), then one tile
// per block, then the block's r.z (and b.b) partials.  FORM 1, 3 and 2 are
// the passes of the product form: the first (r -> src of the next pass) has
// the convergence test and b.b, the middle ones neither, the last (-> z) the
// r.z partials.
template <int VEC, int D, int TY, int NW, bool FIRST, int FORM, bool RECT, bool PART>
__device__ __forceinline__ void precond_block(const SweepArgs& a, const Geom& g, const PrecondCoef& pc,
                                              const float* src, float* dst) {
    constexpr int NT = NW * 64;
    __shared__ double sh[NW];
    __shared__ __align__(16) float lds[precond_lds_floats<VEC, D, TY, FORM, RECT>()];

    int b = blockIdx.x;
    if ((a.nblocks & 7) == 0) b = (b & 7) * (a.nblocks >> 3) + (b >> 3);
    const int f = b / a.bpf;
    const int blk = b - f * a.bpf;
    CgField* stf = a.c.st + f;
    if (stf->done) return;  // uniform over the block
    const bool lead = blk == 0 && threadIdx.x == 0;
    if constexpr (!FIRST && (FORM == 0 || FORM == 1)) {
        // convergence test on r_k . r_k from the previous sweep 2 (or, at
        // k = 0, the residual sweep, which also gave b.b)
        const double rrk = block_sum_nt<NT>(a.P2 + ((size_t)f * 2 + (a.k & 1)) * a.pstride, a.bpf_in, sh);
        double bb;
        if (a.k == 0) bb = block_sum_nt<NT>(a.P1 + ((size_t)f * 2 + 1) * a.pstride, a.bpf_in, sh);
        else bb = stf->bb;
        if (lead) {
            stf->rr_par[a.k & 1] = rrk;
            if (a.k == 0) stf->bb = bb;
        }
        if (check_stop(a.c, f, a.k, rrk, bb, lead)) return;
    }

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int yg = blk % a.ygroups, zci = blk / a.ygroups;
    const int zb = zci * a.zc;
    double acc0 = 0.0, acc1 = 0.0;
    const size_t fo = (size_t)f * a.cells;
    const float* rsrc = FIRST ? a.p.B : a.p.R;  // r_k (b at a zero first guess)
    constexpr int TF = FORM == 3 ? 1 : FORM;  // a middle pass is a first pass without the partials
    // RECT: S on the input of the first pass and on the output of the last
    constexpr bool SIN = RECT && (FORM == 0 || FORM == 1), SOUT = RECT && (FORM == 0 || FORM == 2);
    precond_lds_tile<VEC, D, TY, NW, FIRST && (FORM == 0 || FORM == 1), false, TF, RECT, SIN, SOUT, PART>(
        lds, src + fo, dst + fo, g, pc, a.ny, a.nz, yg * TY, zb, min(zb + a.zc, a.nz), acc0, acc1, rsrc + fo);
    if constexpr (FORM == 3) return;

    // block reduction of the float64 partials, fixed order
    constexpr bool kRz = FORM == 0 || FORM == 2, kBb = FIRST && (FORM == 0 || FORM == 1);
    for (int o = 32; o > 0; o >>= 1) {
        if (kRz) acc0 += __shfl_xor(acc0, o);
        if (kBb) acc1 += __shfl_xor(acc1, o);
    }
    __shared__ double s0[NW], s1[NW];
    if (lane == 0) {
        s0[w] = acc0;
        s1[w] = acc1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double u0 = 0.0, u1 = 0.0;
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            u0 += s0[i];
            u1 += s1[i];
        }
        if (kRz) a.P3[((size_t)f * 2 + (a.k & 1)) * a.pstride + blk] = u0;
        if (kBb) a.P1[((size_t)f * 2 + 1) * a.pstride + blk] = u1;
    }
}

// Uniform grids: the Horner pass (FORM 0, coefficients pc) or the product
// form's passes r -> U (FORM 1, pc), U -> V (FORM 3, pcm; degree 12) and
// V -> z (FORM 2, pc2).  At 2 cells per lane (LDS for two blocks per CU) the
// middle pass, the first pass of later iterations and the last pass are
// held to 64 VGPRs so that two blocks share a CU: the 128^3 batched launch
// went from 3,224 to 3,388 fields/s with the first two (no spills), and to
// 3,455 with the last pass too once its loaders keep one plane in flight
// instead of two (5 registers spilled; with two planes it spilled 15 and
// the launch fell to 3,168).  The first iteration's first pass would spill.
template <int VEC, int D, int TY, int NW, bool FIRST, int FORM = 0, bool PART = false>
__global__ __launch_bounds__(NW * 64, (VEC <= 2 && (FORM == 3 || FORM == 2 || (FORM == 1 && !FIRST))) ? 8 : 1) void k_precond_lds(SweepArgs a) {
    const float* rsrc = FIRST ? a.p.B : a.p.R;
    const float* src = FORM == 2 ? a.p.V : (FORM == 3 ? a.p.U : rsrc);
    float* dst = FORM == 1 ? a.p.U : (FORM == 3 ? a.p.V : a.p.Z);
    precond_block<VEC, D, TY, NW, FIRST, FORM, false, PART>(a, a.g, FORM == 2 ? a.pc2 : (FORM == 3 ? a.pcm : a.pc),
                                                            src, dst);
}

// Rectilinear grids: one pass of D = 2 levels of the polynomial in S A S
// (per-axis factors in gp) with its own coefficients and buffers (the Horner
// pass of degree 2, or one quadratic factor of the product form).
template <int VEC, bool FIRST, int FORM, bool PART>
__global__ __launch_bounds__(16 * 64) void k_precond_rect(SweepArgs a, Geom gp, PrecondCoef pc, const float* src,
                                                          float* dst) {
    precond_block<VEC, 2, 8, 16, FIRST, FORM, true, PART>(a, gp, pc, src, dst);
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

// Learned initial guess (x0_mode 3): after the residual sweep, a field
// whose guess residual is not finite or exceeds ||b|| (||r0||^2 > ||b||^2)
// restarts from zero.  One block per field sums the two partial arrays of
// the residual sweep in the fixed order; on rejection the r.r partials are
// replaced by the b.b partials, so the following sweeps see r = b.
__global__ __launch_bounds__(kBlock) void k_warm_check(const double* P1, double* P2, int pstride, int bpf,
                                                       int32_t* fb_row) {
    const int f = blockIdx.x;
    __shared__ double sh[kWaves];
    double* rr_p = P2 + ((size_t)f * 2 + 0) * pstride;
    const double* bb_p = P1 + ((size_t)f * 2 + 1) * pstride;
    const double rr = block_sum_fixed(rr_p, bpf, sh);
    const double bb = block_sum_fixed(bb_p, bpf, sh);
    const bool fb = !(rr <= bb);
    if (threadIdx.x == 0) fb_row[f] = fb ? 1 : 0;
    if (fb)
        for (int i = threadIdx.x; i < bpf; i += kBlock) rr_p[i] = bb_p[i];
}

// ... and its vectors become x = 0, r = b.
__global__ void k_warm_reset(float* X, float* R, const float* B, int64_t cells, const int32_t* fb_row) {
    const int f = blockIdx.y;
    if (!fb_row[f]) return;
    const size_t o = (size_t)f * cells;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < cells;
         k += (int64_t)gridDim.x * blockDim.x) {
        X[o + k] = 0.f;
        R[o + k] = B[o + k];
    }
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
    __shared__ double sh[kWaves];
    double t = block_sum_fixed(partials + (size_t)f * bpf, bpf, sh);
    if (threadIdx.x == 0) out[f] = t;
}

// ---------------------------------------------------------------- host side

struct Plan {
    int vec, ty, zc, xsegs, ygroups, zchunks, wpf, bpf, nblocks;
    bool edge;
};

// VEC: cells per lane.  A wave covers a whole x-row when nx <= 64 * VEC and
// nx is a multiple of VEC (the lanes beyond the row idle), for VEC in {4, 2,
// 1}; wider rows, and rows of 65..256 cells that no VEC divides, run with
// VEC = 1 and edge loads over several x segments.
int pick_vec(int nx) {
    if (nx <= 64) return 1;
    if (nx <= 128) return nx % 2 == 0 ? 2 : 1;
    if (nx <= 256) return nx % 4 == 0 ? 4 : 1;
    return 1;
}

bool ty_supported(int vec, int ty) {
    if (vec == 4) return ty == 2 || ty == 4;
    return ty == 4 || ty == 8;
}

Plan make_plan(const HexGeom& g, int F, int vec, int ty, int zc) {
    Plan p;
    p.vec = vec;
    p.edge = (vec == 1 && g.nx > 64);
    p.ty = ty;
    p.zc = std::max(1, std::min(zc, g.nz));
    p.xsegs = (g.nx + 64 * vec - 1) / (64 * vec);
    p.ygroups = (g.ny + ty - 1) / ty;
    p.zchunks = (g.nz + p.zc - 1) / p.zc;
    p.wpf = p.xsegs * p.ygroups * p.zchunks;
    p.bpf = (p.wpf + kWaves - 1) / kWaves;
    p.nblocks = p.bpf * F;
    return p;
}

// Default tiling: about 4096 waves in flight (16 per compute unit) with
// z chunks of at least 2 planes (a chunk re-reads its two halo planes, so
// small grids trade that for filling the machine: 128^3 runs 23 % faster
// with 2-plane chunks than with 8).
Plan default_plan(const HexGeom& g, int F, int vec) {
    const int ty = vec == 4 ? 2 : (vec == 2 ? 4 : (g.ny >= 8 ? 8 : 4));
    const int64_t cols = (int64_t)((g.nx + 64 * vec - 1) / (64 * vec)) * ((g.ny + ty - 1) / ty) * F;
    const int64_t target_waves = 4096;
    int64_t chunks = std::max<int64_t>(1, target_waves / std::max<int64_t>(1, cols));
    int zc = (int)std::max<int64_t>(2, (g.nz + chunks - 1) / chunks);
    return make_plan(g, F, vec, ty, zc);
}

// The rectilinear operator's sweeps: the modes of Jacobi-preconditioned CG
// from a zero guess (the SZ modes form z = r / diag(A)).
template <int VEC, int TY, bool EDGE>
void launch_sweep_rect(int mode, const Plan& p, const SweepArgs& a, hipStream_t s) {
    const dim3 grid(p.nblocks), block(kBlock);
    switch (mode) {
        case S1: hipLaunchKernelGGL((k_sweep<VEC, TY, S1, EDGE, true>), grid, block, 0, s, a); break;
        case S1_B0: hipLaunchKernelGGL((k_sweep<VEC, TY, S1_B0, EDGE, true>), grid, block, 0, s, a); break;
        case S2: hipLaunchKernelGGL((k_sweep<VEC, TY, S2, EDGE, true>), grid, block, 0, s, a); break;
        case S2P_FIRST: hipLaunchKernelGGL((k_sweep<VEC, TY, S2P_FIRST, EDGE, true>), grid, block, 0, s, a); break;
        case SZ_FIRST: hipLaunchKernelGGL((k_sweep<VEC, TY, SZ_FIRST, EDGE, true>), grid, block, 0, s, a); break;
        case SZ: hipLaunchKernelGGL((k_sweep<VEC, TY, SZ, EDGE, true>), grid, block, 0, s, a); break;
        default: break;  // not used on rectilinear grids
    }
}

template <int VEC, int TY, bool EDGE>
void launch_sweep_t(int mode, const Plan& p, const SweepArgs& a, hipStream_t s) {
    if (a.rect) return launch_sweep_rect<VEC, TY, EDGE>(mode, p, a, s);
    const dim3 grid(p.nblocks), block(kBlock);
    switch (mode) {
        case S1_FIRST: hipLaunchKernelGGL((k_sweep<VEC, TY, S1_FIRST, EDGE>), grid, block, 0, s, a); break;
        case S1: hipLaunchKernelGGL((k_sweep<VEC, TY, S1, EDGE>), grid, block, 0, s, a); break;
        case S1_B0: hipLaunchKernelGGL((k_sweep<VEC, TY, S1_B0, EDGE>), grid, block, 0, s, a); break;
        case S2_FIRST: hipLaunchKernelGGL((k_sweep<VEC, TY, S2_FIRST, EDGE>), grid, block, 0, s, a); break;
        case S2: hipLaunchKernelGGL((k_sweep<VEC, TY, S2, EDGE>), grid, block, 0, s, a); break;
        case SZ_FIRST: hipLaunchKernelGGL((k_sweep<VEC, TY, SZ_FIRST, EDGE>), grid, block, 0, s, a); break;
        case SZ: hipLaunchKernelGGL((k_sweep<VEC, TY, SZ, EDGE>), grid, block, 0, s, a); break;
        case S2P_FIRST: hipLaunchKernelGGL((k_sweep<VEC, TY, S2P_FIRST, EDGE>), grid, block, 0, s, a); break;
        case SZ2_FIRST: hipLaunchKernelGGL((k_sweep<VEC, TY, SZ2_FIRST, EDGE>), grid, block, 0, s, a); break;
        case SZ2: hipLaunchKernelGGL((k_sweep<VEC, TY, SZ2, EDGE>), grid, block, 0, s, a); break;
        default: hipLaunchKernelGGL((k_sweep<VEC, TY, S_RES, EDGE>), grid, block, 0, s, a); break;
    }
}

void launch_sweep(int mode, const Plan& p, const SweepArgs& a, hipStream_t s) {
    if (p.vec == 4) {
        if (p.ty == 2) launch_sweep_t<4, 2, false>(mode, p, a, s);
        else launch_sweep_t<4, 4, false>(mode, p, a, s);
    } else if (p.vec == 2) {
        if (p.ty == 4) launch_sweep_t<2, 4, false>(mode, p, a, s);
        else launch_sweep_t<2, 8, false>(mode, p, a, s);
    } else if (p.edge) {
        if (p.ty == 4) launch_sweep_t<1, 4, true>(mode, p, a, s);
        else launch_sweep_t<1, 8, true>(mode, p, a, s);
    } else {
        if (p.ty == 4) launch_sweep_t<1, 4, false>(mode, p, a, s);
        else launch_sweep_t<1, 8, false>(mode, p, a, s);
    }
}

// LDS preconditioning sweep: TY = 8 rows per block of 16 waves (at most
// one row per wave and level, so a level costs one LDS round trip).
constexpr int kLdsTY = 8, kLdsNW = 16;

constexpr int lds_precond_bytes(int vec, int deg) {
    return (deg == 4 ? lds_level_base<4, kLdsTY>(4)
                     : (deg == 2 ? lds_level_base<2, kLdsTY>(2) : lds_level_base<3, kLdsTY>(3))) *
           64 * vec * 4;
}

template <int VEC, bool FIRST, bool PART>
void launch_precond_rect_p(int form, const Plan& q, const SweepArgs& a, const Geom& gp, const PrecondCoef& pc,
                           const float* src, float* dst, hipStream_t s) {
    const dim3 grid(q.nblocks), block(kLdsNW * 64);
    switch (form) {
        case 0: hipLaunchKernelGGL((k_precond_rect<VEC, FIRST, 0, PART>), grid, block, 0, s, a, gp, pc, src, dst); break;
        case 1: hipLaunchKernelGGL((k_precond_rect<VEC, FIRST, 1, PART>), grid, block, 0, s, a, gp, pc, src, dst); break;
        case 2: hipLaunchKernelGGL((k_precond_rect<VEC, FIRST, 2, PART>), grid, block, 0, s, a, gp, pc, src, dst); break;
        default: hipLaunchKernelGGL((k_precond_rect<VEC, FIRST, 3, PART>), grid, block, 0, s, a, gp, pc, src, dst); break;
    }
}

// PART: rows shorter than the wave's 64 VEC cells
template <int VEC, bool FIRST>
void launch_precond_rect_v(int form, const Plan& q, const SweepArgs& a, const Geom& gp, const PrecondCoef& pc,
                           const float* src, float* dst, hipStream_t s) {
    if (a.nx != 64 * VEC) launch_precond_rect_p<VEC, FIRST, true>(form, q, a, gp, pc, src, dst, s);
    else launch_precond_rect_p<VEC, FIRST, false>(form, q, a, gp, pc, src, dst, s);
}

// One pass of the rectilinear preconditioner (FORM 0: the degree-2 Horner
// pass; 1, 3, 2: first, middle and last factor of the product form).
void launch_precond_rect(int vec, bool first, int form, const Plan& q, const SweepArgs& a, const Geom& gp,
                         const PrecondCoef& pc, const float* src, float* dst, hipStream_t s) {
    if (vec == 4) {
        if (first) launch_precond_rect_v<4, true>(form, q, a, gp, pc, src, dst, s);
        else launch_precond_rect_v<4, false>(form, q, a, gp, pc, src, dst, s);
    } else if (vec == 2) {
        if (first) launch_precond_rect_v<2, true>(form, q, a, gp, pc, src, dst, s);
        else launch_precond_rect_v<2, false>(form, q, a, gp, pc, src, dst, s);
    } else {
        if (first) launch_precond_rect_v<1, true>(form, q, a, gp, pc, src, dst, s);
        else launch_precond_rect_v<1, false>(form, q, a, gp, pc, src, dst, s);
    }
}

template <int VEC, int D, int FORM>
void launch_precond_lds_v(bool first, const Plan& q, const SweepArgs& a, hipStream_t s) {
    const dim3 grid(q.nblocks), block(kLdsNW * 64);
    const bool part = a.nx != 64 * VEC;  // rows shorter than the wave covers
    if (first && part) hipLaunchKernelGGL((k_precond_lds<VEC, D, kLdsTY, kLdsNW, true, FORM, true>), grid, block, 0, s, a);
    else if (first) hipLaunchKernelGGL((k_precond_lds<VEC, D, kLdsTY, kLdsNW, true, FORM, false>), grid, block, 0, s, a);
    else if (part) hipLaunchKernelGGL((k_precond_lds<VEC, D, kLdsTY, kLdsNW, false, FORM, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_precond_lds<VEC, D, kLdsTY, kLdsNW, false, FORM, false>), grid, block, 0, s, a);
}

template <int D, int FORM>
void launch_precond_lds_d(int vec, bool first, const Plan& q, const SweepArgs& a, hipStream_t s) {
    if (vec == 4) launch_precond_lds_v<4, D, FORM>(first, q, a, s);
    else if (vec == 2) launch_precond_lds_v<2, D, FORM>(first, q, a, s);
    else launch_precond_lds_v<1, D, FORM>(first, q, a, s);
}

// Degree 3 or 4: one Horner pass; degree 8: two product passes (r -> U,
// V = U -> z); degree 12: three (r -> U -> V -> z).
void launch_precond_lds(int deg, int vec, bool first, const Plan& q, const SweepArgs& a, hipStream_t s) {
    if (deg == 8 || deg == 12) {
        launch_precond_lds_d<4, 1>(vec, first, q, a, s);
        if (deg == 12) launch_precond_lds_d<4, 3>(vec, first, q, a, s);
        launch_precond_lds_d<4, 2>(vec, first, q, a, s);
    } else if (deg == 4) {
        launch_precond_lds_d<4, 0>(vec, first, q, a, s);
    } else {
        launch_precond_lds_d<3, 0>(vec, first, q, a, s);
    }
}

// Degree of the LDS polynomial preconditioner with the least predicted work:
// for degree m the residual polynomial keeps the preconditioned spectrum in
// [1 - e, 1 + e], e = 1 / T_{m+1}(sig(0)), so CG needs about
// k = log(1 / rtol) / log(1 / rho) iterations, rho = (sqrt(K) - 1) / (sqrt(K) + 1),
// K = (1 + e) / (1 - e); an iteration costs sweeps 1 and 2 plus one pass of
// the LDS tile per 4 degrees, each pass about 0.43 of the two sweeps.  (The
// textbook bound has log(2 / rtol); without the 2 the count matches the
// measured iterations per step on the dense bed for degrees 4, 8 and 12 at
// dtau / h^2 = 1 (5, 3, 2) and 1/2 (4, 2, 2), where the 2 overcounts degree
// 4 at 1 and degree 8 at 1/2 by one.)
int lds_degree(double cx, double cy, double cz, double rtol) {
    const double lmax = 1.0 + 4.0 * (cx + cy + cz);
    const double s0 = (lmax + 1.0) / std::max(lmax - 1.0, 1e-12);
    const double th = std::acosh(std::max(s0, 1.0 + 1e-12));
    const double want = std::log(1.0 / std::max(rtol, 1e-300));
    int best = 4;
    double best_cost = 1e300;
    for (int m : {4, 8, 12}) {
        const double e = 1.0 / std::cosh(std::min((m + 1) * th, 700.0));
        const double K = (1.0 + e) / std::max(1.0 - e, 1e-300);
        const double rho = (std::sqrt(K) - 1.0) / (std::sqrt(K) + 1.0);
        // one iteration only where the bound says so with a margin: at
        // e near rtol the first iterate misses by a hair and takes a second
        const double x = rho > 0.0 ? want / std::log(1.0 / rho) : 0.0;
        const double k = x <= 0.8 ? 1.0 : std::max(2.0, std::ceil(x));
        const double cost = k * (1.0 + 0.43 * (m / 4));
        if (cost < best_cost * (1.0 - 1e-9)) {
            best_cost = cost;
            best = m;
        }
    }
    return best;
}

// Degree of the rectilinear operator's polynomial preconditioner on
// [lmin, lmax] with the least predicted work, as lds_degree: degree m costs
// m / 2 passes of the D = 2 tile (one for m = 2), each about 0.37 of the two
// sweeps.  Degree 1 (Jacobi) is not a candidate: its register pass costs
// about as much as a tile pass.
int rect_degree(double lmin, double lmax, double rtol) {
    const double s0 = (lmax + lmin) / std::max(lmax - lmin, 1e-12 * lmax);
    const double th = std::acosh(std::max(s0, 1.0 + 1e-12));
    const double want = std::log(1.0 / std::max(rtol, 1e-300));
    int best = 2;
    double best_cost = 1e300;
    for (int m = 2; m <= 12; m += 2) {
        const double e = 1.0 / std::cosh(std::min((m + 1) * th, 700.0));
        const double K = (1.0 + e) / std::max(1.0 - e, 1e-300);
        const double rho = (std::sqrt(K) - 1.0) / (std::sqrt(K) + 1.0);
        const double x = rho > 0.0 ? want / std::log(1.0 / rho) : 0.0;
        const double k = x <= 0.8 ? 1.0 : std::max(2.0, std::ceil(x));
        const double cost = k * (1.0 + 0.37 * (m == 2 ? 1 : m / 2));
        if (cost < best_cost * (1.0 - 1e-9)) {
            best_cost = cost;
            best = m;
        }
    }
    return best;
}

// Tiling of the LDS preconditioning sweep: ceil(ny / TY) row groups times z
// chunks sized to give every compute unit its share of blocks (as many as
// its 160 KB of LDS holds).  zc_raw: the chunk depth that fills the machine,
// before the floor of 2 D planes (a chunk recomputes 2 D halo planes).  The
// sweep is used when zc_raw >= D (D = 4 for degree 8, which runs two passes
// of the degree-4 tile): at 128^3 (zc 8) degree 8 takes 1.12 ms per field,
// degree 4 1.44 and degree 2 in registers 2.57 (before the later sweep
// changes); at 256 x 256 x 512 (zc 64) 4.80, 5.83 and 10.31.
Plan lds_plan(const HexGeom& g, int F, int vec, int deg, int zc_force, int* zc_raw, int zc_max) {
    Plan p = {};
    p.vec = vec;
    p.ty = kLdsTY;
    p.xsegs = 1;
    p.ygroups = (g.ny + kLdsTY - 1) / kLdsTY;
    const int per_cu = std::max(1, std::min(2048 / (kLdsNW * 64), (160 * 1024) / lds_precond_bytes(vec, deg)));
    const int64_t want_blocks = (int64_t)256 * per_cu;
    const int64_t cols = (int64_t)p.ygroups * F;
    *zc_raw = (int)std::max<int64_t>(1, ((int64_t)g.nz * cols + want_blocks - 1) / want_blocks);
    p.zc = zc_force > 0 ? zc_force : std::max(*zc_raw, 2 * deg);
    p.zc = std::max(1, std::min({p.zc, g.nz, zc_max}));
    p.zchunks = (g.nz + p.zc - 1) / p.zc;
    p.bpf = p.ygroups * p.zchunks;
    p.wpf = p.bpf * kLdsNW;
    p.nblocks = p.bpf * F;
    return p;
}

template <int VEC, int NW>
void launch_dir_lds_v(bool b0, const Plan& q, const SweepArgs& a, hipStream_t s) {
    const dim3 grid(q.nblocks), block(NW * 64);
    const bool part = a.nx != 64 * VEC;  // rows shorter than the wave covers
    if (b0 && part) hipLaunchKernelGGL((k_dir_lds<VEC, NW, true, true>), grid, block, 0, s, a);
    else if (b0) hipLaunchKernelGGL((k_dir_lds<VEC, NW, true, false>), grid, block, 0, s, a);
    else if (part) hipLaunchKernelGGL((k_dir_lds<VEC, NW, false, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_dir_lds<VEC, NW, false, false>), grid, block, 0, s, a);
}

template <int NW>
void launch_dir_lds_nw(int vec, bool b0, const Plan& q, const SweepArgs& a, hipStream_t s) {
    if (vec == 4) launch_dir_lds_v<4, NW>(b0, q, a, s);
    else if (vec == 2) launch_dir_lds_v<2, NW>(b0, q, a, s);
    else launch_dir_lds_v<1, NW>(b0, q, a, s);
}

void launch_dir_lds(int nw, int vec, bool b0, const Plan& q, const SweepArgs& a, hipStream_t s) {
    if (nw == 16) launch_dir_lds_nw<16>(vec, b0, q, a, s);
    else launch_dir_lds_nw<8>(vec, b0, q, a, s);
}

// Tiling of the LDS direction sweep: NW - 2 rows per block, z chunks that
// give every compute unit its resident blocks (by threads and LDS).
Plan dir_plan(const HexGeom& g, int F, int vec, int nw, int zc_force) {
    Plan p = {};
    p.vec = vec;
    p.ty = nw - 2;
    p.xsegs = 1;
    p.ygroups = (g.ny + p.ty - 1) / p.ty;
    const int lds = 3 * nw * 64 * vec * 4;
    const int per_cu = std::max(1, std::min(2048 / (nw * 64), (160 * 1024) / lds));
    const int64_t want = (int64_t)256 * per_cu;
    const int64_t cols = (int64_t)p.ygroups * F;
    int zc = (int)std::max<int64_t>(1, ((int64_t)g.nz * cols + want - 1) / want);
    zc = std::max(zc, 8);
    if (zc_force > 0) zc = zc_force;
    p.zc = std::max(1, std::min(zc, g.nz));
    p.zchunks = (g.nz + p.zc - 1) / p.zc;
    p.bpf = p.ygroups * p.zchunks;
    p.wpf = p.bpf * nw;
    p.nblocks = p.bpf * F;
    return p;
}

size_t small_bytes(int F, int bpf) {
    size_t b = kSmallFixed + 3 * (size_t)F * 2 * (size_t)bpf * sizeof(double);
    return (b + 255) & ~(size_t)255;
}

}  // namespace

// Largest partial count any plan can use for this mesh (VEC = 1, TY = 4, one
// plane per chunk), so the workspace never has to grow between plans.
static size_t max_bpf(const HexGeom& g, int F) {
    Plan p = make_plan(g, F, 1, 4, 1);
    return (size_t)p.bpf;
}

bool hex_one_x_segment(const HexGeom& g, const float* field) {
    int vec = pick_vec(g.nx);
    if ((uintptr_t)field % (4 * vec)) vec = 1;
    return g.nx <= 64 * vec;
}

// Rows wider than a wave covers (nx > 64 VEC) while the y rows fit one: the
// uniform grid is solved with x and y exchanged, the field transposed into
// a seventh workspace vector and back (16 bytes per cell, about 3 % of a
// solve at 256 x 256 x 512), so that the LDS tiles apply.
static bool fits_one_wave(int n) { return n <= 64 * pick_vec(n); }
static bool swap_xy(const HexGeom& g) { return !fits_one_wave(g.nx) && fits_one_wave(g.ny); }

static HexGeom swapped_xy(const HexGeom& g) {
    HexGeom t = g;
    t.nx = g.ny;
    t.ny = g.nx;
    std::swap(t.lo[0], t.lo[1]);
    std::swap(t.hi[0], t.hi[1]);
    std::swap(t.s[0], t.s[1]);
    std::swap(t.h[0], t.h[1]);
    return t;
}

// out[f][z][x][y] = in[f][z][y][x] for an nx-wide, ny-tall plane: 64 x 64
// tiles through LDS (one padding column against bank conflicts), coalesced
// on both sides.  Grid: (ceil(nx / 64), ceil(ny / 64), nz * F).
__global__ __launch_bounds__(256) void k_transpose_xy(const float* __restrict__ in, float* __restrict__ out, int nx,
                                                      int ny) {
    __shared__ float t[64][65];
    const size_t po = (size_t)blockIdx.z * nx * ny;
    const int x0 = blockIdx.x * 64, y0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int y = y0 + r, x = x0 + tx;
        if (y < ny && x < nx) t[r][tx] = in[po + (size_t)y * nx + x];
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int x = x0 + r, y = y0 + tx;
        if (x < nx && y < ny) out[po + (size_t)x * ny + y] = t[tx][r];
    }
}

static void transpose_xy(const float* in, float* out, int nx, int ny, int64_t planes, hipStream_t s) {
    const dim3 grid((nx + 63) / 64, (ny + 63) / 64, (unsigned)planes);
    hipLaunchKernelGGL(k_transpose_xy, grid, dim3(256), 0, s, in, out, nx, ny);
}

size_t diffuse_hex_workspace(const cgd_mesh m, int32_t F) {
    const HexGeom& g = m->hex;
    const bool sw = swap_xy(g);
    const size_t bpf = sw ? std::max(max_bpf(g, F), max_bpf(swapped_xy(g), F)) : max_bpf(g, F);
    return small_bytes(F, (int)bpf) + (sw ? 7 : 6) * (size_t)F * m->cells * sizeof(float);
}

cgd_status diffuse_hex(cgd_mesh m, const DiffuseArgs& da, cgd_solve_stats* out, hipStream_t s, const int* fixed) {
    cgd_status rc = ensure_workspace(m, diffuse_hex_workspace(m, da.F));
    if (rc != CGD_OK) return rc;
    rc = ensure_pinned(m, kPinBytes);
    if (rc != CGD_OK) return rc;
    char* base = static_cast<char*>(m->ws.ptr);
    const HexGeom& g = m->hex;
    if (swap_xy(g) && (da.x0_mode == 0 || da.x0_mode == 1) && !getenv("CGD_HEX_NO_SWAP")) {
        // the seventh vector, after the six the solve uses
        const size_t bpf = std::max(max_bpf(g, da.F), max_bpf(swapped_xy(g), da.F));
        float* T = reinterpret_cast<float*>(base + small_bytes(da.F, (int)bpf)) + 6 * (size_t)da.F * m->cells;
        const HexGeom gs = swapped_xy(g);
        const int64_t planes = (int64_t)da.F * g.nz;
        transpose_xy(da.field, T, g.nx, g.ny, planes, s);
        DiffuseArgs d2 = da;
        d2.field = T;
        rc = diffuse_hex_enqueue(m, d2, base, fixed, out != nullptr, s, nullptr, &gs);
        if (rc != CGD_OK) return rc;
        transpose_xy(T, da.field, gs.nx, gs.ny, planes, s);
        CGD_HIP_TRY(hipGetLastError());
    } else {
        rc = diffuse_hex_enqueue(m, da, base, fixed, out != nullptr, s, nullptr);
        if (rc != CGD_OK) return rc;
    }
    return cg_finish_call(m, da.F, da.n_steps, m->hex.vol, s, out, da.x0_mode == 3);
}

cgd_status diffuse_hex_enqueue(cgd_mesh m, const DiffuseArgs& da, char* base, const int* fixed, bool sums,
                               hipStream_t s, const RectOp* ro, const HexGeom* geom) {
    const HexGeom& g = geom ? *geom : m->hex;
    const int F = da.F;
    const int64_t cells = m->cells;
    // vector width: rows must be 16 / 8 byte aligned in every buffer touched
    int vec = pick_vec(g.nx);
    const uintptr_t align = (uintptr_t)da.field | (uintptr_t)(da.x0_mode == 2 ? da.x0 : nullptr);
    if (align % (4 * vec)) vec = 1;
    // Tile plans: p for the update sweeps (sweep 2, residual), p1 for the
    // direction sweeps (sweep 1), pz for the preconditioning sweeps.  With
    // 4 cells per lane, sweep 1 takes z chunks twice as deep and the
    // preconditioning sweep 4 rows per wave (its two halo rows then cost 1.5x
    // instead of 2x in loads); both measured faster on the dense bed.
    Plan p = default_plan(g, F, vec);
    Plan p1 = vec == 4 ? make_plan(g, F, vec, p.ty, 2 * p.zc) : p;
    Plan pz = vec == 4 ? make_plan(g, F, vec, 4, p.zc) : p;
    auto tile_env = [&](const char* name, Plan& q) {  // "TY,ZC" for tuning runs
        if (const char* e = getenv(name)) {
            int ty = 0, zc = 0;
            if (sscanf(e, "%d,%d", &ty, &zc) == 2 && ty_supported(vec, ty) && zc > 0) q = make_plan(g, F, vec, ty, zc);
        }
    };
    tile_env("CGD_HEX_TILE", p);
    tile_env("CGD_HEX_TILE", p1);
    tile_env("CGD_HEX_TILE", pz);
    tile_env("CGD_HEX_TILE1", p1);
    tile_env("CGD_HEX_TILE2", p);
    tile_env("CGD_HEX_TILEZ", pz);
    const size_t small = small_bytes(F, (int)max_bpf(g, F));
    CgCtl ctl = {};
    ctl.st = reinterpret_cast<CgField*>(base + kOffState);
    ctl.ndone = reinterpret_cast<int*>(base + kOffNdone);
    ctl.iters = reinterpret_cast<int32_t*>(base + kOffIters);
    ctl.relres = reinterpret_cast<double*>(base + kOffRelres);
    ctl.status = reinterpret_cast<int32_t*>(base + kOffStatus);
    ctl.rtol2 = da.rtol * da.rtol;
    ctl.step = 0;
    double* d_sums = reinterpret_cast<double*>(base + kOffSums);
    const size_t pmax = (size_t)F * 2 * max_bpf(g, F);
    double* d_P1 = reinterpret_cast<double*>(base + kSmallFixed);
    double* d_P2 = d_P1 + pmax;
    double* d_P3 = d_P2 + pmax;
    float* W0 = reinterpret_cast<float*>(base + small);
    float* R = W0 + (size_t)F * cells;
    float* PA = R + (size_t)F * cells;
    float* PB = PA + (size_t)F * cells;
    float* Z = PB + (size_t)F * cells;
    float* PV = Z + (size_t)F * cells;  // the degree-12 preconditioner's middle-pass output

    const double T = da.bandwidth * da.bandwidth / 4.0;
    // Crank-Nicolson solves with half the step and extrapolates (below)
    const double dtau = T / da.n_steps * (da.scheme == 1 ? 0.5 : 1.0);
    SweepArgs a = {};
    a.cells = cells;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.g.nx = g.nx;
    a.g.ny = g.ny;
    a.g.nz = g.nz;
    a.g.cx = (float)(dtau / (g.h[0] * g.h[0]));
    a.g.cy = (float)(dtau / (g.h[1] * g.h[1]));
    a.g.cz = (float)(dtau / (g.h[2] * g.h[2]));
    Geom gp = {};  // the rectilinear preconditioner's S A S (prepared for this dtau)
    if (ro) {
        // the rectilinear operator A (per-axis factors)
        if ((ro->per & 1) && p.xsegs != 1) {
            set_error("cgd_diffuse: a periodic x axis needs the row in one x segment");
            return CGD_E_UNSUPPORTED;
        }
        a.rect = 1;
        a.g.dt = (float)dtau;
        a.g.per = ro->per;
        for (int ax = 0; ax < 3; ++ax) {
            a.g.rg[ax] = ro->g[ax];
            a.g.rs[ax] = ro->s[ax];
            a.g.rd[ax] = ro->d[ax];
            a.g.re[ax] = ro->e[ax];
        }
        gp = a.g;
        for (int ax = 0; ax < 3; ++ax) {
            gp.rg[ax] = ro->pg[ax];
            gp.rs[ax] = ro->ps[ax];
            gp.rd[ax] = ro->pd[ax];
            gp.re[ax] = ro->pe[ax];
            gp.rsg[ax] = ro->psg[ax];
        }
    }
    a.pstride = (int)max_bpf(g, F);
    a.c = ctl;
    a.P1 = d_P1;
    a.P2 = d_P2;
    a.P3 = d_P3;
    a.p.R = R;
    a.p.Z = Z;
    // Preconditioned CG (default) with the Chebyshev polynomial preconditioner
    // of poly_precond_coeffs: degree 2 where one wave covers a row (the sweep
    // keeps two halo rows and planes, tile_precond2; condition number 13 ->
    // 2.1 at dtau / h^2 = 1), degree 1 otherwise (13 -> 3.8).
    // Where the grid fills the machine with z chunks of at least D planes
    // (lds_plan), the degree rises to 4, 8 or 12, applied by k_precond_lds
    // (below).
    const bool pcg = da.precond == 0 || ro;  // the rectilinear operator runs preconditioned CG only
    const bool row_wave = !p.edge && p.xsegs == 1;  // one wave per x-row (possibly partial)
    const int deg = (pcg && row_wave && !ro) ? 2 : 1;  // rectilinear: Jacobi (the SZ modes)
    a.pcg = pcg ? 1 : 0;
    poly_precond_coeffs(a.g.cx, a.g.cy, a.g.cz, deg, &a.g.c0, &a.g.c1, &a.g.c2);
    const int mode_z_first = deg == 2 ? SZ2_FIRST : SZ_FIRST;
    const int mode_z = deg == 2 ? SZ2 : SZ;
    int deg_lds = 0;
    if (deg == 2 && !ro) {
        // Degree 4, 8 or 12 (one Horner pass; two or three passes of two
        // quadratic factors) where the LDS tile applies, by predicted cost
        // (lds_degree).  At dtau / h^2 = 1: 5, 3 and 2 iterations per step;
        // on the 256 x 256 x 512 grid 5.83, 4.90 and 3.89 ms per field.
        // CGD_HEX_PRECOND_DEG (3, 4, 8 or 12) overrides.
        int want = lds_degree(a.g.cx, a.g.cy, a.g.cz, da.rtol), zc_force = 0, zc_raw = 0;
        if (const char* e = getenv("CGD_HEX_PRECOND_DEG")) want = atoi(e);
        if (const char* e = getenv("CGD_HEX_LDS_ZC")) zc_force = atoi(e);
        if (want == 3 || want == 4 || want == 8 || want == 12) {
            // degrees 8 and 12 run as two and three passes of the degree-4 tile
            const int dt = want >= 8 ? 4 : want;
            Plan pl = lds_plan(g, F, p.vec, dt, zc_force, &zc_raw, 1 << 30);
            if ((zc_force > 0 || zc_raw >= dt) && (size_t)pl.bpf <= max_bpf(g, F)) {
                deg_lds = want;
                pz = pl;
                if (want >= 8) {
                    double qs[6], qq[6], qg[6], scale;
                    const int nf = poly_precond_quadratics(a.g.cx, a.g.cy, a.g.cz, want, qs, qq, qg, &scale);
                    precond_coef_fill_quadratics(a.pc, a.g.cx, a.g.cy, a.g.cz, qs, qq, qg, 1.0);
                    if (nf == 6) precond_coef_fill_quadratics(a.pcm, a.g.cx, a.g.cy, a.g.cz, qs + 2, qq + 2, qg + 2, 1.0);
                    precond_coef_fill_quadratics(a.pc2, a.g.cx, a.g.cy, a.g.cz, qs + nf - 2, qq + nf - 2, qg + nf - 2,
                                                 scale);
                } else {
                    double c[8];
                    poly_precond_coeffs_n(a.g.cx, a.g.cy, a.g.cz, want, c);
                    precond_coef_fill(a.pc, a.g.cx, a.g.cy, a.g.cz, c, want);
                }
            }
        }
    }

    // The rectilinear operator where one wave covers an x-row: S p(S A S) S
    // with the Chebyshev polynomial p on S A S's spectrum [lmin, lmax]
    // (RectOp), in passes of the LDS tile with D = 2 levels
    // (k_precond_rect): degree 2 by Horner in one pass, or m / 2 passes of
    // one quadratic factor each, by predicted cost (rect_degree); elsewhere
    // Jacobi (the SZ modes).  CGD_HEX_PRECOND_DEG (2, 4, ..., 12; 1 for
    // Jacobi) and CGD_HEX_LDS_ZC override.
    int deg_rect = 0;
    PrecondCoef rect_pc[6];
    if (ro && row_wave) {
        int want = rect_degree(ro->lmin, ro->lmax, da.rtol), zc_force = 0, zc_raw = 0;
        if (const char* e = getenv("CGD_HEX_PRECOND_DEG")) want = atoi(e);
        if (const char* e = getenv("CGD_HEX_LDS_ZC")) zc_force = atoi(e);
        if (want >= 2 && want <= 12 && want % 2 == 0) {
            Plan pl = lds_plan(g, F, p.vec, 2, zc_force, &zc_raw, kRectZMax - 8);  // plane table's bound
            if ((zc_force > 0 || zc_raw >= 2) && (size_t)pl.bpf <= max_bpf(g, F)) {
                deg_rect = want;
                pz = pl;
                if (want == 2) {
                    double c[8];
                    poly_precond_coeffs_iv(ro->lmin, ro->lmax, 2, c);
                    precond_coef_fill(rect_pc[0], 0.f, 0.f, 0.f, c, 2);
                } else {
                    double qs[6], qq[6], qg[6], scale;
                    const int nf = poly_precond_quadratics_iv(ro->lmin, ro->lmax, want, qs, qq, qg, &scale);
                    for (int k = 0; k < nf; ++k)
                        precond_coef_fill_quadratics(rect_pc[k], 0.f, 0.f, 0.f, qs + k, qq + k, qg + k,
                                                     k == nf - 1 ? scale : 1.0, 2);
                }
            }
        }
    }

    // Preconditioned CG where one wave covers an x-row: the direction sweep
    // shares its rows through LDS (k_dir_lds, 16 waves: 14 rows per block, so
    // the two halo rows cost 1/7 of a row per output row in L2 reads).  On
    // the 256 x 256 x 512 grid it takes 82 us against 84.5 with 8 waves and
    // 98.5 for the register sweep; at 128^3 both LDS widths are within 1 %.
    // CGD_HEX_DIR (0: the register sweep), CGD_HEX_DIR_NW (8 or 16 waves)
    // and CGD_HEX_DIR_ZC override.
    int dir_nw = 0;
    if (pcg && row_wave && !ro) {
        dir_nw = 16;
        int zc_force = 0;
        if (const char* e = getenv("CGD_HEX_DIR")) dir_nw = atoi(e) ? 16 : 0;
        if (const char* e = getenv("CGD_HEX_DIR_NW")) dir_nw = dir_nw ? (atoi(e) == 16 ? 16 : 8) : 0;
        if (const char* e = getenv("CGD_HEX_DIR_ZC")) zc_force = atoi(e);
        if (dir_nw) {
            Plan pd = dir_plan(g, F, p.vec, dir_nw, zc_force);
            if ((size_t)pd.bpf <= max_bpf(g, F)) p1 = pd;
            else dir_nw = 0;
        }
    }

    // One sweep: its own plan, and the block count of the sweep whose
    // partial sums its prologue adds.
    auto set_plan = [&](int mode) -> const Plan& {
        const bool is_z = mode == SZ_FIRST || mode == SZ || mode == SZ2_FIRST || mode == SZ2;
        const bool is_1 = mode == S1_FIRST || mode == S1 || mode == S1_B0;
        const Plan& q = is_z ? pz : (is_1 ? p1 : p);
        a.xsegs = q.xsegs;
        a.ygroups = q.ygroups;
        a.zc = q.zc;
        a.wpf = q.wpf;
        a.bpf = q.bpf;
        a.nblocks = q.nblocks;
        if (is_z) a.bpf_in = p.bpf;                   // r.r (and b.b) of sweep 2 / the residual sweep
        else if (is_1) a.bpf_in = a.pcg ? pz.bpf : p.bpf;  // r.z of the preconditioning sweep, or r.r
        else a.bpf_in = p1.bpf;                       // p.Ap (and b.b) of sweep 1
        return q;
    };
    auto launch = [&](int mode) {
        const bool is_z = mode == SZ_FIRST || mode == SZ || mode == SZ2_FIRST || mode == SZ2;
        const bool is_1 = mode == S1_FIRST || mode == S1 || mode == S1_B0;
        const Plan& q = set_plan(mode);
        if (is_z && deg_lds) launch_precond_lds(deg_lds, p.vec, mode == mode_z_first, q, a, s);
        else if (is_1 && dir_nw) launch_dir_lds(dir_nw, p.vec, mode == S1_B0, q, a, s);
        else launch_sweep(mode, q, a, s);
    };
    // The preconditioning step z = M r with every pass timed on its own:
    // kinds 5 / 6 / 7 (10 / 11 / 12 in a step's first iteration, which reads
    // b) for the first, middle and last pass; 8 bytes per cell and pass (read
    // its input, write its output), plus the last product pass's read of r.
    auto launch_precond_timed = [&](bool first, int64_t tag) {
        const int mode = first ? mode_z_first : mode_z;
        const double cb = (double)F * cells;
        const int k0 = first ? 10 : 5;
        if (deg_rect) {
            // pass k reads the previous pass's output (r or b first) and
            // writes U, V, U, ... (z last); the middle passes share a kind
            const Plan& q = set_plan(mode);
            const int np = deg_rect == 2 ? 1 : deg_rect / 2;
            const float* in = first ? a.p.B : a.p.R;
            for (int k = 0; k < np; ++k) {
                const int form = np == 1 ? 0 : (k == 0 ? 1 : (k == np - 1 ? 2 : 3));
                float* out = k == np - 1 ? a.p.Z : ((k & 1) ? a.p.V : a.p.U);
                const int t = timing_begin(&m->timing, s);
                launch_precond_rect(p.vec, first, form, q, a, gp, rect_pc[k], in, out, s);
                const int kind = np == 1 ? k0 : (k == 0 ? k0 : (k == np - 1 ? k0 + 2 : k0 + 1));
                timing_end(&m->timing, t, kind, (form == 2 ? 12.0 : 8.0) * cb, s, tag);
                in = out;
            }
        } else if (deg_lds == 8 || deg_lds == 12) {
            const Plan& q = set_plan(mode);
            int t = timing_begin(&m->timing, s);
            launch_precond_lds_d<4, 1>(p.vec, first, q, a, s);
            timing_end(&m->timing, t, k0, 8.0 * cb, s, tag);
            if (deg_lds == 12) {
                t = timing_begin(&m->timing, s);
                launch_precond_lds_d<4, 3>(p.vec, first, q, a, s);
                timing_end(&m->timing, t, k0 + 1, 8.0 * cb, s, tag);
            }
            t = timing_begin(&m->timing, s);
            launch_precond_lds_d<4, 2>(p.vec, first, q, a, s);
            timing_end(&m->timing, t, k0 + 2, 12.0 * cb, s, tag);
        } else {
            int t = timing_begin(&m->timing, s);
            launch(mode);
            timing_end(&m->timing, t, k0, 8.0 * cb, s, tag);
        }
    };

    const int sum_bpf = (int)std::min<int64_t>(1024, (cells + kBlock - 1) / kBlock);
    double* d_sum_part = d_P2;  // free outside the solves

    if (sums) {  // mass before diffusion
        hipLaunchKernelGGL(k_field_sum, dim3(sum_bpf, F), dim3(kBlock), 0, s, da.field, cells, d_sum_part, sum_bpf);
        hipLaunchKernelGGL(k_sum_finish, dim3(F), dim3(kBlock), 0, s, d_sum_part, sum_bpf, d_sums);
    }

    if (da.x0_mode == 3) CGD_HIP_TRY(hipMemsetAsync(base + kOffFallback, 0, 4096, s));

    float* cur = da.field;  // b of the current step
    float* nxt = W0;        // x of the current step
    for (int step = 0; step < da.n_steps; ++step) {
        a.c.step = step;
        a.p.B = cur;
        a.p.X = nxt;
        hipLaunchKernelGGL(k_cg_step_init, dim3(1), dim3(64), 0, s, ctl.st, F, ctl.ndone,
                           ctl.status + step * CGD_MAX_FIELDS);
        const bool use_x0 = (da.x0_mode == 1) || (da.x0_mode == 2 && step == 0) || da.x0_mode == 3;
        a.x0_zero = use_x0 ? 0 : 1;
        // Crank-Nicolson from a zero guess: the x updates carry the
        // extrapolation (x = 2 y - b at every iterate); from a guess, a pass
        // after the solve does
        const bool cn_fused = da.scheme == 1 && !use_x0;
        a.g.xs1 = cn_fused ? 1.f : 0.f;
        a.g.xb = cn_fused ? -1.f : 0.f;
        int it0;
        a.k = 0;
        if (!use_x0 && pcg) {
            it0 = 0;  // iteration 0 (z = M b, p = z, x = alpha p) is enqueued by the loop
        } else if (!use_x0) {
            launch(S1_FIRST);
            launch(S2_FIRST);
            it0 = 1;
        } else {
            if (da.x0_mode == 3) {
                for (int f = 0; f < F; ++f) {
                    cgd_status rg = unet::unet_guess(da.model, cur + (size_t)f * cells, nxt + (size_t)f * cells, s);
                    if (rg != CGD_OK) return rg;
                }
            } else {
                const float* x0 = da.x0_mode == 1 ? cur : da.x0;
                CGD_HIP_TRY(hipMemcpyAsync(nxt, x0, (size_t)F * cells * sizeof(float), hipMemcpyDeviceToDevice, s));
            }
            launch(S_RES);
            if (da.x0_mode == 3) {
                int32_t* fb_row = reinterpret_cast<int32_t*>(base + kOffFallback) + step * CGD_MAX_FIELDS;
                hipLaunchKernelGGL(k_warm_check, dim3(F), dim3(kBlock), 0, s, d_P1, d_P2, a.pstride, p.bpf, fb_row);
                const int blocks = (int)std::min<int64_t>(2048, (cells + kBlock - 1) / kBlock);
                hipLaunchKernelGGL(k_warm_reset, dim3(blocks, F), dim3(kBlock), 0, s, nxt, R, cur, cells, fb_row);
            }
            it0 = 0;
        }
        auto enqueue_pcg = [&](int it, int* host_flags) {
            // iteration it: z = M r (convergence test first), p = z + beta p_old, x, r update
            const bool first = it == 0 && !use_x0;
            const int64_t tag = (int64_t)step * 65536 + it;
            // Buffers: z of iteration it in zb, p_old and p in Pold / Pnew.
            // With the LDS direction sweep, p_0 = z_0 stays in Z (S1_B0 only
            // reads it), z_1 goes to PA and p_1 to PB; from iteration 2 on z
            // is in Z and p alternates between PA and PB.  Otherwise p_0 is a
            // copy of z_0 in PA.
            float* zb = Z;
            float* pold = (it & 1) ? PA : PB;
            float* pnew = (it & 1) ? PB : PA;
            if (dir_nw && it == 0) {
                pnew = Z;
            } else if (dir_nw && it == 1) {
                zb = PA;
                pold = Z;
            }
            a.k = it;
            a.p.R = R;
            a.p.Z = zb;
            // the product form's intermediate: a p buffer that holds nothing
            // live until sweep 1 writes p_new into it
            a.p.U = it == 0 ? (dir_nw ? PA : PB) : pnew;
            a.p.V = (deg_lds == 12 || deg_rect >= 6) ? PV : a.p.U;
            launch_precond_timed(first, tag);
            a.p.Z = Z;
            a.p.R = zb;
            a.p.Pold = pold;
            a.p.Pnew = pnew;
            // direction sweep: reads z and p_old, writes p (12 bytes per
            // cell); p_0 = z_0 reads z only, and is written only by the
            // register sweep
            const double b1 = it == 0 ? (dir_nw ? 4.0 : 8.0) : 12.0;
            int t1 = timing_begin(&m->timing, s);
            launch(it == 0 ? S1_B0 : S1);
            timing_end(&m->timing, t1, it == 0 ? 8 : 0, b1 * (double)F * cells, s, tag);
            a.p.R = R;
            a.c.host_flags = host_flags;
            // update sweep: reads p, x, r, writes x, r (20); from a zero
            // guess reads p, b, writes x, r (16)
            int t2 = timing_begin(&m->timing, s);
            launch(first ? S2P_FIRST : S2);
            timing_end(&m->timing, t2, first ? 9 : 1, (first ? 16.0 : 20.0) * (double)F * cells, s, tag);
            a.c.host_flags = nullptr;
        };
        auto enqueue = [&](int it, int* host_flags) {
            if (pcg) return enqueue_pcg(it, host_flags);
            int mode1 = S1;
            if (!use_x0) {
                a.p.Pold = it == 1 ? cur : ((it & 1) ? PB : PA);
                a.p.Pnew = (it & 1) ? PA : PB;
            } else {
                a.p.Pold = (it & 1) ? PA : PB;
                a.p.Pnew = (it & 1) ? PB : PA;
                if (it == 0) mode1 = S1_B0;
            }
            a.k = it;
            const int64_t tag = (int64_t)step * 65536 + it;
            int t1 = timing_begin(&m->timing, s);
            launch(mode1);
            timing_end(&m->timing, t1, 0, 12.0 * (double)F * cells, s, tag);
            a.c.host_flags = host_flags;
            int t2 = timing_begin(&m->timing, s);
            launch(S2);
            timing_end(&m->timing, t2, 1, 20.0 * (double)F * cells, s, tag);
            a.c.host_flags = nullptr;
        };
        int it_end = it0;
        if (fixed) {
            // a fixed budget of iterations, with no read-back (the launches of
            // a field that has converged return at once)
            it_end = std::max(it0, std::min(fixed[step], da.max_iter));
            for (int it = it0; it < it_end; ++it) enqueue(it, nullptr);
        } else {
            cgd_status rc2 = cg_lookahead_loop(m, F, it0, da.max_iter, da.check_every, ctl.ndone, s, enqueue, &it_end);
            if (rc2 != CGD_OK) return rc2;
        }
        CgCtl c2 = ctl;
        c2.step = step;
        // the test of iteration it_end's first kernel, in its summation order:
        // an LDS preconditioning pass (1024 threads) or a register sweep
        if (pcg && (deg_lds || deg_rect)) {
            static_assert(kLdsNW * 64 == 1024, "LDS passes sum with 1024 threads");
            hipLaunchKernelGGL(k_cg_step_end<1024>, dim3(F), dim3(1024), 0, s, c2,
                               d_P2 + (size_t)(it_end & 1) * a.pstride, (size_t)2 * a.pstride, p.bpf, it_end);
        } else {
            hipLaunchKernelGGL(k_cg_step_end<kBlock>, dim3(F), dim3(kBlock), 0, s, c2,
                               d_P2 + (size_t)(it_end & 1) * a.pstride, (size_t)2 * a.pstride, p.bpf, it_end);
        }
        if (use_x0) {
            int blocks = (int)std::min<int64_t>(2048, (cells + kBlock - 1) / kBlock);
            hipLaunchKernelGGL(k_zero_if_rhs_zero, dim3(blocks, F), dim3(kBlock), 0, s, nxt, cells, ctl.st);
        }
        if (da.scheme == 1 && !cn_fused) cn_extrapolate(nxt, cur, (int64_t)F * cells, s);
        std::swap(cur, nxt);
    }
    if (cur != da.field) {
        CGD_HIP_TRY(hipMemcpyAsync(da.field, cur, (size_t)F * cells * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
    if (sums) {
        hipLaunchKernelGGL(k_field_sum, dim3(sum_bpf, F), dim3(kBlock), 0, s, da.field, cells, d_sum_part, sum_bpf);
        hipLaunchKernelGGL(k_sum_finish, dim3(F), dim3(kBlock), 0, s, d_sum_part, sum_bpf, d_sums + CGD_MAX_FIELDS);
    }
    CGD_HIP_TRY(hipGetLastError());
    return CGD_OK;
}

}  // namespace cgd
