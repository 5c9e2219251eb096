// Unstructured tetrahedral meshes: centroid location + fixed-point deposit
// (Section 2.2 on arbitrary cells) and backward-Euler diffusion with the
// two-point-flux finite-volume Laplacian by CG over a sparse operator with
// rows padded to a tet's four face slots, preconditioned by a Chebyshev
// polynomial of the Jacobi-scaled operator (or Jacobi alone) (Sections 2.1
// item 4, 4.3, 5.1).
//
// Point location: a tet contains the point when, for each face, the float64
// orientation of the point relative to the face (evaluated on the face's
// vertices in increasing global-id order, so both tets sharing a face compute
// the identical number) is not strictly on the opposite side from the tet's
// fourth vertex; the result is the lowest containing id.  The search walks
// from the seed tet of the point's bucket across faces the point lies
// strictly beyond (orientation walk over face neighbours).  A tet that has
// the point strictly inside all four faces is the only tet containing it (a
// conforming mesh), so the walk's answer is the definition's.  When the walk
// meets a zero orientation (the point on a face, edge or vertex), leaves the
// mesh, or exceeds a step limit, the bucket's tets are tested in ascending
// id order and the first hit is returned (the same definition, exhaustively).
//
// Crank-Nicolson (Section 5.1): the same solve with dtau / 2, then x = 2 x - e.
//
// Diffusion step: (M + dtau K) x = M e with M = diag(V), K the two-point-flux
// Laplacian; CG with z = D^-1 r (Jacobi, D = diag(M + dtau K)) or z = p(B) H r
// (the polynomial preconditioner below: sweep 2 then writes v = H r to z and
// the passes turn it into z).  A p is
// evaluated in flux form, (A p)_i = V_i p_i + dtau sum_f a_f (p_i - p_j), from
// the four face slots of row i (one 16-byte load of neighbour ids, one of
// a_f): each face's flux enters its two rows with opposite signs, so A keeps
// the conservation of the continuous operator in float32 (a constant p has
// no flux at all), which the assembled diagonal K_ii = sum a_f does not.
// One iteration k is two sweeps:
//   sweep 1: p = z + beta p_old (recomputed at the neighbours it gathers),
//            q = A p, p.q;  writes p, q
//   sweep 2: x += alpha p, r -= alpha q, z = D^-1 r; r.z and r.r;
//            writes x, r, z
// Scalars come from the previous sweep's float64 block partials, summed by
// every block in one fixed order (cg_common.h).
#pragma clang fp contract(off)

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "cg_common.h"
#include "hex_bin.h"
#include "tet_data.h"

namespace cgd {
namespace {

constexpr int kBlock = kCgBlock;
constexpr int kWaves = kCgWaves;

// det[b - a, c - a, p - a], the same expression for every caller
__device__ inline double orient(const double* a, const double* b, const double* c, const double* p) {
    const double u0 = b[0] - a[0], u1 = b[1] - a[1], u2 = b[2] - a[2];
    const double v0 = c[0] - a[0], v1 = c[1] - a[1], v2 = c[2] - a[2];
    const double w0 = p[0] - a[0], w1 = p[1] - a[1], w2 = p[2] - a[2];
    return u0 * (v1 * w2 - v2 * w1) - u1 * (v0 * w2 - v2 * w0) + u2 * (v0 * w1 - v1 * w0);
}

__device__ inline bool tet_contains(const double* __restrict__ xyz, const int32_t* __restrict__ tv, int t,
                                    const double* p) {
    const int4 v4 = *reinterpret_cast<const int4*>(tv + (size_t)t * 4);
    const int ids[4] = {v4.x, v4.y, v4.z, v4.w};
    for (int j = 0; j < 4; ++j) {
        int f[3], k = 0;
        for (int i = 0; i < 4; ++i)
            if (i != j) f[k++] = ids[i];
        // sort the three ids
        if (f[0] > f[1]) { int tmp = f[0]; f[0] = f[1]; f[1] = tmp; }
        if (f[1] > f[2]) { int tmp = f[1]; f[1] = f[2]; f[2] = tmp; }
        if (f[0] > f[1]) { int tmp = f[0]; f[0] = f[1]; f[1] = tmp; }
        const double* a = xyz + 3 * (size_t)f[0];
        const double* b = xyz + 3 * (size_t)f[1];
        const double* c = xyz + 3 * (size_t)f[2];
        const double sp = orient(a, b, c, p);
        const double sd = orient(a, b, c, xyz + 3 * (size_t)ids[j]);
        const double sg = sd > 0.0 ? 1.0 : (sd < 0.0 ? -1.0 : 0.0);
        if (!(sp * sg >= 0.0)) return false;
    }
    return true;
}

struct LocArgs {
    const double* xyz;
    const int32_t* tv;
    const double* bbox;
    const int64_t* bstart;
    const int32_t* blist;
    const int32_t* bseed;
    const int32_t* nbr;
    int32_t nb[3];
    double glo[3], ghi[3], ginv[3];
};

constexpr int kWalkSteps = 64;

// One step of the walk: 1 if the point is strictly inside all four faces of
// t, 0 if it is on a face (some orientation zero, none negative), else -1
// with *exit the local index of the first face the point lies beyond.
__device__ inline int walk_test(const double* __restrict__ xyz, const int32_t* __restrict__ tv, int t, const double* p,
                                int* exit) {
    const int4 v4 = *reinterpret_cast<const int4*>(tv + (size_t)t * 4);
    const int ids[4] = {v4.x, v4.y, v4.z, v4.w};
    bool zero = false;
    for (int j = 0; j < 4; ++j) {
        int f[3], k = 0;
        for (int i = 0; i < 4; ++i)
            if (i != j) f[k++] = ids[i];
        if (f[0] > f[1]) { int tmp = f[0]; f[0] = f[1]; f[1] = tmp; }
        if (f[1] > f[2]) { int tmp = f[1]; f[1] = f[2]; f[2] = tmp; }
        if (f[0] > f[1]) { int tmp = f[0]; f[0] = f[1]; f[1] = tmp; }
        const double* a = xyz + 3 * (size_t)f[0];
        const double* b = xyz + 3 * (size_t)f[1];
        const double* c = xyz + 3 * (size_t)f[2];
        const double sp = orient(a, b, c, p);
        const double sd = orient(a, b, c, xyz + 3 * (size_t)ids[j]);
        const double v = sp * (sd > 0.0 ? 1.0 : (sd < 0.0 ? -1.0 : 0.0));
        if (!(v >= 0.0)) {
            *exit = j;
            return -1;
        }
        if (v == 0.0) zero = true;
    }
    return zero ? 0 : 1;
}

// Containing tet of a point, -1 when none (outside the mesh or non-finite).
__device__ inline int locate(const LocArgs& g, const double* p) {
    int bi[3];
    for (int a = 0; a < 3; ++a) {
        if (!(p[a] >= g.glo[a] && p[a] <= g.ghi[a])) return -1;
        int b = (int)floor((p[a] - g.glo[a]) * g.ginv[a]);
        bi[a] = b < 0 ? 0 : (b >= g.nb[a] ? g.nb[a] - 1 : b);
    }
    const size_t bk = (size_t)bi[0] + (size_t)g.nb[0] * ((size_t)bi[1] + (size_t)g.nb[1] * bi[2]);
    int t = g.bseed[bk];
    if (t < 0) return -1;  // no tet's bounding box reaches this bucket
    for (int step = 0; step < kWalkSteps; ++step) {
        int exit = -1;
        const int r = walk_test(g.xyz, g.tv, t, p, &exit);
        if (r > 0) return t;
        if (r == 0) break;  // on a face: several tets may contain the point
        const int tn = g.nbr[(size_t)t * 4 + exit];
        if (tn == t) break;  // a boundary face: walked out of the mesh
        t = tn;
    }
    const int64_t e = g.bstart[bk + 1];
    for (int64_t i = g.bstart[bk]; i < e; ++i) {
        const int t = g.blist[i];
        const double* bb = g.bbox + (size_t)t * 6;
        if (p[0] < bb[0] || p[1] < bb[1] || p[2] < bb[2] || p[0] > bb[3] || p[1] > bb[4] || p[2] > bb[5]) continue;
        if (tet_contains(g.xyz, g.tv, t, p)) return t;
    }
    return -1;
}

struct TetLoc {
    LocArgs g;
    __device__ int operator()(const double* p) const { return locate(g, p); }
};

// perm (nullable): the order in which the threads take the particles (the
// spatial ordering below), so that the threads of a wave walk nearby tets.
template <class Loc>
__global__ __launch_bounds__(kBlock) void k_locate_deposit_tet(const float* __restrict__ pos,
                                                               const float* __restrict__ values, int64_t n, int F,
                                                               Loc loc, int e_n, unsigned long long* __restrict__ acc,
                                                               int64_t cells, DepositInfo* info, int32_t* cell_out,
                                                               const int32_t* __restrict__ perm) {
    __shared__ int S[CGD_MAX_FIELDS];
    if (threadIdx.x < F) S[threadIdx.x] = frac_bits_used(info->maxbits[threadIdx.x], info->force_s[threadIdx.x], e_n);
    __syncthreads();
    unsigned long long dropped = 0ull, nfpos = 0ull;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int64_t q = perm ? (int64_t)perm[i] : i;
        const double p[3] = {(double)pos[3 * q], (double)pos[3 * q + 1], (double)pos[3 * q + 2]};
        int t = -1;
        if (isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2])) {
            t = loc(p);
        } else {
            ++nfpos;
        }
        if (cell_out) cell_out[q] = t;
        if (t < 0) {
            ++dropped;
            continue;
        }
        for (int f = 0; f < F; ++f) {
            const float v = values[(size_t)f * n + q];
            if (!isfinite(v)) continue;
            const long long qv = __double2ll_rn(ldexp((double)v, S[f]));
            if (qv != 0) atomicAdd(&acc[(size_t)f * cells + t], (unsigned long long)qv);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        dropped += __shfl_xor(dropped, o);
        nfpos += __shfl_xor(nfpos, o);
    }
    if ((threadIdx.x & 63) == 0 && dropped) {
        atomicAdd(&info->dropped, dropped);
        if (nfpos) atomicAdd(&info->nonfinite_pos, nfpos);
    }
}

// Spatial ordering of the particles for the walk: key = the walk's bucket
// coordinates shifted right by `shift` (a block of 8^shift buckets), sorted by
// counting with per-block histograms in LDS (no global atomics): each of
// nblk blocks counts its contiguous run of particles into LDS and stores the
// row hist[block][key]; the rows are scanned per key over the blocks and the
// key totals over the keys; the scatter then ranks each block's particles
// with LDS atomics on base[key] + hist[block][key].  The order within a key
// is arbitrary, which the integer sums do not see.  Points outside the
// bucket grid or non-finite take the last key.
constexpr int kOrderThreads = 1024;
constexpr int kOrderMaxKeys = 16383;  // LDS counters of a block: 64 KB with the last key

struct OrderArgs {
    const float* pos;
    int64_t n;
    int32_t* key;     // [n]
    int32_t* hist;    // [nblk][nkey + 1]: per-block counts, then their exclusive scan over the blocks
    int32_t* total;   // [nkey + 1]: key totals, then their exclusive scan (the keys' first slots)
    int32_t* perm;    // [n]
    int32_t* seg;     // [kOrderSegs][nkey + 1]: per-segment sums of hist, then their scan
    int64_t per;      // particles per block
    int nblk;
    int nb[3], sb[3], shift, nkey;
    double glo[3], ghi[3], ginv[3];
};

__device__ inline int order_key(const OrderArgs& a, const float* pq) {
    int k = 0, mul = 1;
    for (int d = 0; d < 3; ++d) {
        const double p = (double)pq[d];
        if (!(p >= a.glo[d] && p <= a.ghi[d])) return a.nkey;
        int b = (int)floor((p - a.glo[d]) * a.ginv[d]);
        b = b < 0 ? 0 : (b >= a.nb[d] ? a.nb[d] - 1 : b);
        k += (b >> a.shift) * mul;
        mul *= a.sb[d];
    }
    return k;
}

__global__ __launch_bounds__(kOrderThreads) void k_order_count(OrderArgs a) {
    __shared__ int32_t h[kOrderMaxKeys + 1];
    const int nk = a.nkey + 1;
    for (int k = threadIdx.x; k < nk; k += kOrderThreads) h[k] = 0;
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * a.per, e = min(b + a.per, a.n);
    for (int64_t q = b + threadIdx.x; q < e; q += kOrderThreads) {
        const int k = order_key(a, a.pos + 3 * q);
        a.key[q] = k;
        atomicAdd(&h[k], 1);
    }
    __syncthreads();
    int32_t* row = a.hist + (size_t)blockIdx.x * nk;
    for (int k = threadIdx.x; k < nk; k += kOrderThreads) row[k] = h[k];
}

// per key: exclusive scan of its counts over the blocks, and the total, in
// three coalesced passes over kOrderSegs segments of blocks (thread per key
// and segment): segment sums; their scan per key (and the total); each
// segment's run from its offset.
constexpr int kOrderSegs = 16;

__global__ __launch_bounds__(kBlock) void k_order_segsum(OrderArgs a) {
    const int nk = a.nkey + 1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x, sg = blockIdx.y;
    if (k >= nk) return;
    const int per = (a.nblk + kOrderSegs - 1) / kOrderSegs;
    const int b0 = sg * per, b1 = min(b0 + per, a.nblk);
    int32_t run = 0;
    for (int b = b0; b < b1; ++b) run += a.hist[(size_t)b * nk + k];
    a.seg[(size_t)sg * nk + k] = run;
}

__global__ __launch_bounds__(kBlock) void k_order_segscan(OrderArgs a) {
    const int nk = a.nkey + 1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nk) return;
    int32_t run = 0;
    for (int sg = 0; sg < kOrderSegs; ++sg) {
        const int32_t v = a.seg[(size_t)sg * nk + k];
        a.seg[(size_t)sg * nk + k] = run;
        run += v;
    }
    a.total[k] = run;
}

__global__ __launch_bounds__(kBlock) void k_order_colscan(OrderArgs a) {
    const int nk = a.nkey + 1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x, sg = blockIdx.y;
    if (k >= nk) return;
    const int per = (a.nblk + kOrderSegs - 1) / kOrderSegs;
    const int b0 = sg * per, b1 = min(b0 + per, a.nblk);
    int32_t run = a.seg[(size_t)sg * nk + k];
    for (int b = b0; b < b1; ++b) {
        int32_t* c = a.hist + (size_t)b * nk + k;
        const int32_t v = *c;
        *c = run;
        run += v;
    }
}

// Exclusive scan of count[0..m) in place, one block of 1024 threads, each
// owning a contiguous run.
__global__ __launch_bounds__(1024) void k_order_scan(int32_t* count, int m) {
    __shared__ int32_t part[1024];
    const int per = (m + 1023) / 1024;
    const int b = threadIdx.x * per, e = min(b + per, m);
    int32_t s = 0;
    for (int i = b; i < e; ++i) s += count[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int32_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int32_t run = part[threadIdx.x] - s;
    for (int i = b; i < e; ++i) {
        const int32_t c = count[i];
        count[i] = run;
        run += c;
    }
}

__global__ __launch_bounds__(kOrderThreads) void k_order_scatter(OrderArgs a) {
    __shared__ int32_t h[kOrderMaxKeys + 1];
    const int nk = a.nkey + 1;
    const int32_t* row = a.hist + (size_t)blockIdx.x * nk;
    for (int k = threadIdx.x; k < nk; k += kOrderThreads) h[k] = a.total[k] + row[k];
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * a.per, e = min(b + a.per, a.n);
    for (int64_t q = b + threadIdx.x; q < e; q += kOrderThreads) a.perm[atomicAdd(&h[a.key[q]], 1)] = (int32_t)q;
}

__global__ __launch_bounds__(kBlock) void k_finalize_vol(const long long* __restrict__ acc, float* __restrict__ field,
                                                         int64_t cells, const double* __restrict__ vol, int e_n,
                                                         const DepositInfo* info) {
    const int f = blockIdx.y;
    const int S = frac_bits_used(info->maxbits[f], info->force_s[f], e_n);
    const long long* a = acc + (size_t)f * cells;
    float* out = field + (size_t)f * cells;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < cells; k += (int64_t)gridDim.x * blockDim.x)
        out[k] = (float)(ldexp((double)a[k], -S) / vol[k]);
}

// ---------------------------------------------------------------- PCG

enum TMode { T1_FIRST = 0, T1 = 1, T2_FIRST = 2, T2 = 3 };

struct TetArgs {
    const int4* col;      // [n]: neighbour across each face slot (own id in a boundary slot)
    const float4* kf;     // [n]: a_f per face slot (0 in a boundary slot)
    const int2* col2;     // [n]: slots 5 and 6 (rectilinear hexes)
    const float2* kf2;
    const float* volf;    // V (float)
    const float* dinv;    // 1 / (V + dtau K_ii)
    const float* B;       // e^n (the step's input field)
    float* R;
    float* Z;             // D^-1 r
    float* X;
    const float* Pold;
    float* Pnew;
    float* Q;
    CgCtl c;
    double* P1;           // [F][3][bpf]: p.q, r.z (k = 0), r.r (k = 0)
    double* P2;           // [F][2][2][bpf]: parity, (r.z, r.r)
    int n;                // rows
    int bpf, nblocks, nchunks;
    float dtau;
    int k;
};

// POLY (first iteration only): z_0 was formed by the polynomial passes, which
// also wrote r_0 = M e, b.b and r.z; the sweep reads z_0 from Z.
template <int MODE, int NS, bool POLY = false>
__global__ __launch_bounds__(kBlock) void k_tet_sweep(TetArgs a) {
    int b = blockIdx.x;
    if ((a.nblocks & 7) == 0) b = (b & 7) * (a.nblocks >> 3) + (b >> 3);
    const int f = b / a.bpf;
    const int blk = b - f * a.bpf;
    CgField* stf = a.c.st + f;
    if constexpr (MODE == T2 || MODE == T2_FIRST) post_ndone(a.c);
    if (MODE != T2_FIRST && stf->done) return;

    __shared__ double sh[kWaves];
    const bool lead = blk == 0 && threadIdx.x == 0;
    float alpha = 0.f, beta = 0.f;
    if constexpr (MODE == T1) {
        const double* p2 = a.P2 + ((size_t)f * 4 + (a.k & 1) * 2) * a.bpf;
        const double rz = block_sum_fixed(p2, a.bpf, sh);
        const double rr = block_sum_fixed(p2 + a.bpf, a.bpf, sh);
        if (lead) stf->rr_par[a.k & 1] = rz;
        if (check_stop(a.c, f, a.k, rr, stf->bb, lead)) return;
        beta = (float)(rz / stf->rr_par[(a.k - 1) & 1]);
    } else if constexpr (MODE == T2 || MODE == T2_FIRST) {
        const double* p1 = a.P1 + (size_t)f * 3 * a.bpf;
        const double pq = block_sum_fixed(p1, a.bpf, sh);
        if constexpr (MODE == T2_FIRST) {
            const double rz = block_sum_fixed(p1 + a.bpf, a.bpf, sh);
            const double bb = block_sum_fixed(p1 + 2 * a.bpf, a.bpf, sh);
            const bool broken = !isfinite(bb) || !isfinite(pq) || !isfinite(rz) || (bb > 0.0 && !(pq > 0.0));
            if (lead) {
                stf->bb = bb;
                stf->rr_par[0] = rz;
                if (broken) finish_field(a.c, f, CGD_E_BREAKDOWN);
            }
            alpha = (broken || bb == 0.0) ? 0.f : (float)(rz / pq);
        } else {
            if (!(pq > 0.0) || !isfinite(pq)) {
                if (lead) finish_field(a.c, f, CGD_E_BREAKDOWN);
                return;
            }
            alpha = (float)(stf->rr_par[a.k & 1] / pq);
        }
    }

    const size_t fo = (size_t)f * a.n;
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;

    if constexpr (MODE == T1_FIRST || MODE == T1) {
        // p at a row: z = D^-1 M e on the first iteration, else z + beta p_old
        auto pval = [&](int j) -> float {
            if constexpr (MODE == T1_FIRST && POLY) return a.Z[fo + j];
            else if constexpr (MODE == T1_FIRST) return a.dinv[j] * (a.volf[j] * a.B[fo + j]);
            else return fmaf(beta, a.Pold[fo + j], a.Z[fo + j]);
        };
        for (int chunk = blk; chunk < a.nchunks; chunk += a.bpf) {
            const int i = chunk * kBlock + threadIdx.x;
            if (i >= a.n) continue;
            const int4 c = a.col[i];
            const float4 w = a.kf[i];
            const float pi = pval(i);
            const float p0 = pval(c.x), p1 = pval(c.y), p2 = pval(c.z), p3 = pval(c.w);
            float fl = w.x * (pi - p0);
            fl = fmaf(w.y, pi - p1, fl);
            fl = fmaf(w.z, pi - p2, fl);
            fl = fmaf(w.w, pi - p3, fl);
            if constexpr (NS == 6) {
                const int2 c2 = a.col2[i];
                const float2 w2 = a.kf2[i];
                const float p4 = pval(c2.x), p5 = pval(c2.y);
                fl = fmaf(w2.x, pi - p4, fl);
                fl = fmaf(w2.y, pi - p5, fl);
            }
            const float q = fmaf(a.dtau, fl, a.volf[i] * pi);
            a.Pnew[fo + i] = pi;
            a.Q[fo + i] = q;
            acc0 = fma((double)pi, (double)q, acc0);
            if constexpr (MODE == T1_FIRST && !POLY) {
                const float r = a.volf[i] * a.B[fo + i];
                a.R[fo + i] = r;
                acc1 = fma((double)r, (double)pi, acc1);  // r.z with z = p
                acc2 = fma((double)r, (double)r, acc2);
            }
        }
    } else {
        for (int chunk = blk; chunk < a.nchunks; chunk += a.bpf) {
            const int i = chunk * kBlock + threadIdx.x;
            if (i >= a.n) continue;
            const float p = a.Pnew[fo + i];
            const float q = a.Q[fo + i];
            const float x = MODE == T2_FIRST ? alpha * p : fmaf(alpha, p, a.X[fo + i]);
            const float r = fmaf(-alpha, q, a.R[fo + i]);
            const float z = a.dinv[i] * r;
            a.X[fo + i] = x;
            a.R[fo + i] = r;
            a.Z[fo + i] = z;
            acc0 = fma((double)r, (double)z, acc0);
            acc1 = fma((double)r, (double)r, acc1);
        }
    }
    const double t0 = block_reduce_fixed(acc0, sh);
    const double t1 = block_reduce_fixed(acc1, sh);
    const double t2 = (MODE == T1_FIRST && !POLY) ? block_reduce_fixed(acc2, sh) : 0.0;
    if (threadIdx.x == 0) {
        if constexpr (MODE == T1_FIRST || MODE == T1) {
            double* p1 = a.P1 + (size_t)f * 3 * a.bpf;
            p1[blk] = t0;
            if (MODE == T1_FIRST && !POLY) {
                p1[a.bpf + blk] = t1;
                p1[2 * a.bpf + blk] = t2;
            }
        } else {
            double* p2 = a.P2 + ((size_t)f * 4 + ((a.k + 1) & 1) * 2) * a.bpf;
            p2[blk] = t0;
            p2[a.bpf + blk] = t1;
        }
    }
}

__global__ void k_tet_dinv(const float* volf, const float* kdiag, float dtau, float* dinv, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        dinv[i] = (float)(1.0 / ((double)volf[i] + (double)dtau * (double)kdiag[i]));
}

// ------------------------------------------------ polynomial preconditioner
//
// z = p(B) h r with B = H A~, A~ = M + dtau K~ and H = diag(A~)^-1, where K~
// is K with its face coefficients rounded to float16 after division by their
// maximum (symmetric: both rows of a face hold the same rounding), so that
// p(B) H = H^1/2 p(H^1/2 A~ H^1/2) H^1/2 is symmetric.  p is the Chebyshev
// polynomial of even degree m that makes 1 - l p(l) smallest on [lmin, lmax]
// (the spectrum estimate of B, from dtau once per call), evaluated as a product of
// m / 2 quadratic factors g_k (B^2 + s_k B + q_k), each in two passes:
//   pass 1: w = B v                 (v gathered at the face neighbours)
//   pass 2: v = g_k ((1 + s_k) w - h kappa sum_f a~_f w_j + q_k v)
// with (B v)_i = v_i - h_i kappa sum_f a~_f v_j, kappa = dtau amax.  The last
// pass 2 carries the leading coefficient and sums r.z.  For even m the
// residual polynomial 1 - l p(l) is below 1 for every l > 0, so p > 0 on any
// positive spectrum: a poor estimate costs iterations, never definiteness.

typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

struct ChebArgs {
    const int4* col;
    const int2* col2;
    const f16x4* kh;
    const f16x2* kh2;
    const float* h;       // 1 / (V + kappa sum a~)
    const float* R;       // r (last pass: r.z)
    const float* G;       // gathered input: v (pass 1) or w (pass 2)
    const float* V;       // pass 2: the factor's input v (own row)
    float* out;
    double* part;         // last pass: r.z partial of block blk of field f at part[f * pstride + blk]
    size_t pstride;
    const double* rrp;    // first pass (nullable): r.r partials of sweep 2 at rrp[f * pstride + blk],
    int kcheck;           // tested as the convergence check of iteration kcheck
    CgCtl c;
    float kappa, c1, cq, gk;
    int n, bpf, nblocks, nchunks;
};

template <int NS, int STAGE>  // STAGE 0: pass 1; 1: pass 2; 2: the last pass 2
__global__ __launch_bounds__(kBlock) void k_tet_cheb(ChebArgs a) {
    int b = blockIdx.x;
    if ((a.nblocks & 7) == 0) b = (b & 7) * (a.nblocks >> 3) + (b >> 3);
    const int f = b / a.bpf;
    const int blk = b - f * a.bpf;
    CgField* stf = a.c.st + f;
    if (stf->done) return;
    __shared__ double sh[kWaves];
    if constexpr (STAGE == 0) {
        // the next iteration's convergence check, made here so that a
        // converged field skips the polynomial as well (every block sums the
        // partials in the same order and takes the same decision)
        if (a.rrp) {
            const double rr = block_sum_fixed(a.rrp + (size_t)f * a.pstride, a.bpf, sh);
            if (check_stop(a.c, f, a.kcheck, rr, stf->bb, blk == 0 && threadIdx.x == 0)) return;
        }
    }
    const size_t fo = (size_t)f * a.n;
    const float* g = a.G + fo;
    double acc = 0.0;
    for (int chunk = blk; chunk < a.nchunks; chunk += a.bpf) {
        const int i = chunk * kBlock + threadIdx.x;
        if (i >= a.n) continue;
        const int4 c = a.col[i];
        const f16x4 w = a.kh[i];
        float s = (float)w.x * g[c.x];
        s = fmaf((float)w.y, g[c.y], s);
        s = fmaf((float)w.z, g[c.z], s);
        s = fmaf((float)w.w, g[c.w], s);
        if constexpr (NS == 6) {
            const int2 c2 = a.col2[i];
            const f16x2 w2 = a.kh2[i];
            s = fmaf((float)w2.x, g[c2.x], s);
            s = fmaf((float)w2.y, g[c2.y], s);
        }
        const float hk = a.h[i] * a.kappa;
        float o;
        if constexpr (STAGE == 0) {
            o = fmaf(-hk, s, g[i]);
        } else {
            o = a.gk * fmaf(a.cq, a.V[fo + i], fmaf(a.c1, g[i], -hk * s));
        }
        a.out[fo + i] = o;
        if constexpr (STAGE == 2) acc = fma((double)a.R[fo + i], (double)o, acc);
    }
    if constexpr (STAGE == 2) {
        const double t = block_reduce_fixed(acc, sh);
        if (threadIdx.x == 0) a.part[(size_t)f * a.pstride + blk] = t;
    }
}

// h = 1 / (V + kappa sum_f a~_f)
__global__ void k_tet_hinv(const float* volf, const float* kdh, float kappa, float* h, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        h[i] = (float)(1.0 / ((double)volf[i] + (double)kappa * (double)kdh[i]));
}

// First iteration of a step: r_0 = M e, v = h r_0 (the polynomial's input),
// b.b partials into the slot sweep 2 of the first iteration reads.
__global__ __launch_bounds__(kBlock) void k_tet_cheb_init(TetArgs a) {
    int b = blockIdx.x;
    if ((a.nblocks & 7) == 0) b = (b & 7) * (a.nblocks >> 3) + (b >> 3);
    const int f = b / a.bpf;
    const int blk = b - f * a.bpf;
    const size_t fo = (size_t)f * a.n;
    double acc = 0.0;
    for (int chunk = blk; chunk < a.nchunks; chunk += a.bpf) {
        const int i = chunk * kBlock + threadIdx.x;
        if (i >= a.n) continue;
        const float r = a.volf[i] * a.B[fo + i];
        a.R[fo + i] = r;
        a.Z[fo + i] = a.dinv[i] * r;
        acc = fma((double)r, (double)r, acc);
    }
    __shared__ double sh[kWaves];
    const double t = block_reduce_fixed(acc, sh);
    if (threadIdx.x == 0) a.P1[(size_t)f * 3 * a.bpf + 2 * a.bpf + blk] = t;
}

__global__ __launch_bounds__(kBlock) void k_tet_mass(const float* e, const double* vol, int n, double* part, int bpf) {
    const int f = blockIdx.y;
    __shared__ double sh[kWaves];
    double s = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        s += vol[i] * (double)e[(size_t)f * n + i];
    const double t = block_reduce_fixed(s, sh);
    if (threadIdx.x == 0) part[(size_t)f * bpf + blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_tet_sum_finish(const double* part, int bpf, double* out) {
    __shared__ double sh[kWaves];
    const double t = block_sum_fixed(part + (size_t)blockIdx.x * bpf, bpf, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

struct TetPlan {
    int bpf, nblocks, nchunks;
};

// Blocks per field: every block of a sweep sums all bpf partials of the
// previous one, so bpf stays near the number that fills the machine.
// Measured on 6M tets: 512 / 1024 / 2048 / 4096 give 32.6 / 31.2 / 32.1 /
// 36.8 ms per field.  CGD_TET_BPF overrides the default.
TetPlan tet_plan(int n, int F) {
    TetPlan p;
    int bpf_max = 1024;
    if (const char* e = getenv("CGD_TET_BPF")) bpf_max = std::max(8, std::min(8192, atoi(e)));
    p.nchunks = (n + kBlock - 1) / kBlock;
    p.bpf = std::min(p.nchunks, bpf_max);
    p.nblocks = p.bpf * F;
    return p;
}

template <typename T>
cgd_status upload(const std::vector<T>& h, T** d) {
    if (h.empty()) {
        *d = nullptr;
        return CGD_OK;
    }
    hipError_t e = hipMalloc(d, h.size() * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error(std::string("tet mesh device allocation failed: ") + hipGetErrorString(e));
        return CGD_E_NOMEM;
    }
    CGD_HIP_TRY(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return CGD_OK;
}

size_t tet_small(int F, int bpf) {
    size_t b = kSmallFixed + (size_t)F * 7 * (size_t)bpf * sizeof(double);
    return (b + 255) & ~(size_t)255;
}

// Degree of the polynomial preconditioner with the least predicted work, as
// for the hex stencil: degree m keeps the spectrum of p(B) B in [1 - e,
// 1 + e], e = 1 / T_{m+1}(sig(0)) on [lmin, lmax]; CG needs about
// log(1 / rtol) / log(1 / rho) iterations, rho = (sqrt(K) - 1) / (sqrt(K) + 1),
// K = (1 + e) / (1 - e) (K = lmax / lmin for Jacobi, m = 0).  An iteration
// costs the two sweeps plus m passes, each pass about kPassCost of the two
// sweeps' bytes (28 + 12 bytes per row against 52 + 32 with four slots).
int tet_degree(double lmin, double lmax, double rtol, int ns) {
    const double kPassCost = ns == 6 ? 44.0 / 100.0 : 40.0 / 84.0;
    const double s0 = (lmax + lmin) / std::max(lmax - lmin, 1e-12 * lmax);
    const double th = std::acosh(std::max(s0, 1.0 + 1e-12));
    const double want = std::log(1.0 / std::max(rtol, 1e-300));
    int best = 0;
    double best_cost = 1e300;
    for (int m = 0; m <= 16; m += 2) {
        const double e = m == 0 ? 0.0 : 1.0 / std::cosh(std::min((m + 1) * th, 700.0));
        const double K = m == 0 ? lmax / lmin : (1.0 + e) / std::max(1.0 - e, 1e-300);
        const double rho = (std::sqrt(K) - 1.0) / (std::sqrt(K) + 1.0);
        const double x = rho > 0.0 ? want / std::log(1.0 / rho) : 0.0;
        const double k = std::max(1.0, std::ceil(x));
        const double cost = k * (1.0 + kPassCost * m);
        if (cost < best_cost * (1.0 - 1e-9)) {
            best_cost = cost;
            best = m;
        }
    }
    return best;
}

}  // namespace

cgd_status cheb_operator_setup(TetData* t, const std::vector<float>& kface, const std::vector<float>& kface2,
                               const std::vector<double>& vol) {
    const size_t n = vol.size();
    double amax = 0.0;
    for (float v : kface) amax = std::max(amax, (double)v);
    for (float v : kface2) amax = std::max(amax, (double)v);
    std::vector<_Float16> kh(kface.size()), kh2(kface2.size());
    std::vector<float> kdh(n, 0.f);
    const float inv = amax > 0.0 ? (float)(1.0 / amax) : 0.f;
    for (size_t i = 0; i < n; ++i) {
        float sum = 0.f;
        for (int j = 0; j < 4; ++j) {
            kh[i * 4 + j] = (_Float16)(kface[i * 4 + j] * inv);
            sum += (float)kh[i * 4 + j];
        }
        if (!kface2.empty()) {
            for (int j = 0; j < 2; ++j) {
                kh2[i * 2 + j] = (_Float16)(kface2[i * 2 + j] * inv);
                sum += (float)kh2[i * 2 + j];
            }
        }
        kdh[i] = sum;
    }
    double sv = 0.0, sk = 0.0, kv = 0.0;
    for (size_t i = 0; i < n; ++i) {
        sv += vol[i];
        sk += amax * (double)kdh[i];
        kv = std::max(kv, amax * (double)kdh[i] / vol[i]);
    }
    t->amax = amax;
    t->sum_v = sv;
    t->sum_k = sk;
    t->kv_max = kv;
    cgd_status rc = upload(kh, &t->kh);
    if (rc == CGD_OK) rc = upload(kh2, &t->kh2);
    if (rc == CGD_OK) rc = upload(kdh, &t->kdh);
    return rc;
}

void destroy_tet_data(cgd_mesh m) {
    if (RectOp* ro = m->rop) {
        if (ro->dev) (void)hipFree(ro->dev);
        if (ro->pdev) (void)hipFree(ro->pdev);
        if (ro->host) (void)hipHostFree(ro->host);
        delete ro;
        m->rop = nullptr;
    }
    TetData* t = m->tet;
    if (!t) return;
    void* ptrs[] = {t->xyz,   t->tv,     t->vol,   t->volf,  t->bbox, t->kface, t->kdiag,
                    t->bstart, t->blist, t->bseed, t->nbr,  t->nbr2, t->kface2, t->redges,
                    t->kh,     t->kh2,   t->kdh};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete t;
    m->tet = nullptr;
}

int64_t tet_nnz(cgd_mesh m) { return m->tet ? m->tet->nnz : 0; }

namespace {
template <class Loc>
__global__ __launch_bounds__(kBlock) void k_locate_tet(const float* __restrict__ pos, int64_t n, Loc loc,
                                                       int32_t* __restrict__ cell) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const double p[3] = {(double)pos[3 * q], (double)pos[3 * q + 1], (double)pos[3 * q + 2]};
        cell[q] = (isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2])) ? loc(p) : -1;
    }
}

RectLoc rect_loc(const TetData* t) {
    RectLoc r;
    r.e = t->redges;
    for (int a = 0; a < 3; ++a) r.n[a] = t->rdim[a];
    return r;
}

LocArgs loc_args(const TetData* t) {
    LocArgs g;
    g.xyz = t->xyz;
    g.tv = t->tv;
    g.bbox = t->bbox;
    g.bstart = t->bstart;
    g.blist = t->blist;
    g.bseed = t->bseed;
    g.nbr = t->nbr;
    for (int a = 0; a < 3; ++a) {
        g.nb[a] = t->nb[a];
        g.glo[a] = t->glo[a];
        g.ghi[a] = t->ghi[a];
        g.ginv[a] = t->ginv[a];
    }
    return g;
}
}  // namespace

cgd_status locate_tet(cgd_mesh m, int64_t n, const float* pos, int32_t* cell, hipStream_t s) {
    if (n > 0) {
        const int blocks = (int)std::min<int64_t>(16384, (n + kBlock - 1) / kBlock);
        if (m->tet->ns == 6)
            hipLaunchKernelGGL(k_locate_tet<RectLoc>, dim3(blocks), dim3(kBlock), 0, s, pos, n, rect_loc(m->tet), cell);
        else
            hipLaunchKernelGGL(k_locate_tet<TetLoc>, dim3(blocks), dim3(kBlock), 0, s, pos, n,
                               TetLoc{loc_args(m->tet)}, cell);
    }
    CGD_HIP_TRY(hipGetLastError());
    return CGD_OK;
}

size_t diffuse_tet_workspace(const cgd_mesh m, int32_t F) {
    const TetPlan p = tet_plan(m->tet->n_tet, F);
    // 7 vectors per field (x, r, p twice, q, z, the preconditioner's w) and
    // D^-1 (or the preconditioner's h)
    return tet_small(F, p.bpf) + (7 * (size_t)F + 1) * (size_t)m->tet->n_tet * sizeof(float) + 256;
}

namespace {
// Key layout of the spatial ordering: the smallest shift that leaves at
// least 256 particles per key on average and at most kOrderMaxKeys keys;
// blocks of at least 8192 particles, at most 512 blocks.
OrderArgs order_layout(const TetData* t, int64_t n) {
    OrderArgs a = {};
    a.n = n;
    for (int sh = 0;; ++sh) {
        int64_t k = 1;
        for (int d = 0; d < 3; ++d) k *= ((t->nb[d] - 1) >> sh) + 1;
        if ((k * 256 <= n && k < kOrderMaxKeys) || sh >= 10) {
            a.shift = sh;
            break;
        }
    }
    a.nkey = 1;
    for (int d = 0; d < 3; ++d) {
        a.nb[d] = t->nb[d];
        a.sb[d] = ((t->nb[d] - 1) >> a.shift) + 1;
        a.nkey *= a.sb[d];
        a.glo[d] = t->glo[d];
        a.ghi[d] = t->ghi[d];
        a.ginv[d] = t->ginv[d];
    }
    a.nblk = (int)std::max<int64_t>(1, std::min<int64_t>(512, n / 8192));
    a.per = (n + a.nblk - 1) / a.nblk;
    return a;
}
}  // namespace

size_t deposit_tet_temp_bytes(const cgd_mesh m, int64_t n) {
    const TetData* t = m->tet;
    if (!t || t->ns != 4 || n < 4096 || n > INT32_MAX || getenv("CGD_TET_INPUT_ORDER")) return 0;
    const OrderArgs a = order_layout(t, n);
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t nk = (size_t)a.nkey + 1;
    return 2 * al((size_t)n * 4) + al(nk * 4) + al((size_t)a.nblk * nk * 4) + al((size_t)kOrderSegs * nk * 4);
}

cgd_status deposit_tet(cgd_mesh m, int64_t n, const float* pos, int32_t F, const float* values, float* field,
                       int64_t* acc, DepositInfo* info, void* temp, const ScaleForce& fs, hipStream_t s) {
    const TetData* t = m->tet;
    const int64_t cells = t->n_tet;
    const int e_n = ceil_log2_count(n);
    if (t->ns == 6 && temp && deposit_hex_temp_bytes(m, n, F) > 0 &&
        (int64_t)t->rdim[0] + t->rdim[1] + t->rdim[2] + 3 <= kRectTiledEdges) {
        // rectilinear: the hex grid's tiled deposit with the edges' binning
        // and each cell's own volume (the same cells, sums and roundings)
        TiledDeposit d = {};
        d.pos = pos;
        d.values = values;
        d.total = n;
        d.max_n = n;
        d.n_snap = 1;
        d.F = F;
        d.maxbits = info->maxbits;
        d.force_s = info->force_s;
        d.nf_val = info->nonfinite_val;
        d.nf_val_stride = 1;
        d.dropped = &info->dropped;
        d.nf_pos = &info->nonfinite_pos;
        d.field = field;
        d.acc = reinterpret_cast<long long*>(acc);
        d.temp = temp;
        d.rect = 1;
        d.rl = rect_loc(t);
        d.vcell = t->vol;
        deposit_info_init(info, fs, s);
        return tiled_deposit(m, d, &m->timing, s);
    }
    deposit_prologue(n, F, values, acc, cells, info, fs, s);
    if (n > 0) {
        const int blocks = (int)std::min<int64_t>(16384, (n + kBlock - 1) / kBlock);
        int tm = timing_begin(&m->timing, s);
        int32_t* perm = nullptr;
        if (t->ns == 4 && temp && deposit_tet_temp_bytes(m, n) > 0) {
            // the particles in the order of a coarse bucket key
            OrderArgs o = order_layout(t, n);
            char* tb = static_cast<char*>(temp);
            auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
            const size_t nb4 = al((size_t)n * 4), nk = (size_t)o.nkey + 1;
            o.pos = pos;
            o.key = reinterpret_cast<int32_t*>(tb);
            o.perm = reinterpret_cast<int32_t*>(tb + nb4);
            o.total = reinterpret_cast<int32_t*>(tb + 2 * nb4);
            o.hist = reinterpret_cast<int32_t*>(tb + 2 * nb4 + al(nk * 4));
            o.seg = reinterpret_cast<int32_t*>(tb + 2 * nb4 + al(nk * 4) + al((size_t)o.nblk * nk * 4));
            const unsigned kb = (unsigned)((nk + kBlock - 1) / kBlock);
            hipLaunchKernelGGL(k_order_count, dim3(o.nblk), dim3(kOrderThreads), 0, s, o);
            hipLaunchKernelGGL(k_order_segsum, dim3(kb, kOrderSegs), dim3(kBlock), 0, s, o);
            hipLaunchKernelGGL(k_order_segscan, dim3(kb), dim3(kBlock), 0, s, o);
            hipLaunchKernelGGL(k_order_colscan, dim3(kb, kOrderSegs), dim3(kBlock), 0, s, o);
            hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(1024), 0, s, o.total, (int)nk);
            hipLaunchKernelGGL(k_order_scatter, dim3(o.nblk), dim3(kOrderThreads), 0, s, o);
            perm = o.perm;
        }
        if (t->ns == 6)
            hipLaunchKernelGGL(k_locate_deposit_tet<RectLoc>, dim3(blocks), dim3(kBlock), 0, s, pos, values, n, F,
                               rect_loc(t), e_n, reinterpret_cast<unsigned long long*>(acc), cells, info, nullptr,
                               nullptr);
        else
            hipLaunchKernelGGL(k_locate_deposit_tet<TetLoc>, dim3(blocks), dim3(kBlock), 0, s, pos, values, n, F,
                               TetLoc{loc_args(t)}, e_n, reinterpret_cast<unsigned long long*>(acc), cells, info,
                               nullptr, perm);
        timing_end(&m->timing, tm, 2, (12.0 + 12.0 * F) * (double)n, s);
    }
    const int blocks = (int)std::min<int64_t>(8192, (cells + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_finalize_vol, dim3(blocks, F), dim3(kBlock), 0, s, reinterpret_cast<const long long*>(acc),
                       field, cells, t->vol, e_n, info);
    CGD_HIP_TRY(hipGetLastError());
    return CGD_OK;
}

namespace {
// The change of variable of the rectilinear fast path: field *= fx_i fy_j fz_k
// (sqrt of the cell widths going in, their reciprocals coming out).
__global__ __launch_bounds__(kBlock) void k_rect_scale(float* __restrict__ field, int64_t cells, int nx, int ny,
                                                      const float* __restrict__ fx, const float* __restrict__ fy,
                                                      const float* __restrict__ fz) {
    float* f = field + (size_t)blockIdx.y * cells;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(c % nx);
        const int64_t r = c / nx;
        const int j = (int)(r % ny);
        const int k = (int)(r / ny);
        f[c] *= (fx[i] * fy[j]) * fz[k];
    }
}
}  // namespace

// The scaling S of the rectilinear preconditioner and the bounds of S A S's
// spectrum.  A's diagonal d_ijk = 1 + dtau (Dy Dz sx_i + Dx Dz sy_j + Dx Dy
// sz_k) is a sum of products of per-axis factors; S^2 = mu^2 / (dx_i dy_j
// dz_k), where dx_i is the mean of d over j and k (and so on) and mu the mean
// of d over all cells, which is exactly 1 / d when d itself is a product of
// per-axis factors.  Every mean is a product of per-axis means.  Since K is
// positive semi-definite, S A S >= S^2, so lmin = min S^2 = the product of
// the per-axis minima; lmax is the largest Gershgorin row sum of S A S, a max
// over the cells of ex_i E_jk + hx_i P_jk + Dx_i Q_jk (nonnegative terms),
// one pass over the cells.
cgd_status rect_op_prepare(cgd_mesh m, double dtau, hipStream_t s) {
    RectOp* ro = m->rop;
    if (ro->dtau == dtau) return CGD_OK;
    const int n[3] = {m->hex.nx, m->hex.ny, m->hex.nz};
    auto mean = [](const std::vector<double>& v) {
        double t = 0.0;
        for (double x : v) t += x;
        return t / (double)v.size();
    };
    double mD[3], ms[3];
    for (int a = 0; a < 3; ++a) {
        mD[a] = mean(ro->fac[a]);
        ms[a] = mean(ro->sd[a]);
    }
    const double mu = 1.0 + dtau * (ms[0] * mD[1] * mD[2] + mD[0] * ms[1] * mD[2] + mD[0] * mD[1] * ms[2]);
    const double mu23 = std::cbrt(mu * mu);
    std::vector<double> sig2[3];
    for (int a = 0; a < 3; ++a) {
        const int b = (a + 1) % 3, c = (a + 2) % 3;
        sig2[a].resize(n[a]);
        for (int i = 0; i < n[a]; ++i) {
            // mean over the other two axes of d at index i on axis a
            const double da = 1.0 + dtau * (ro->sd[a][i] * mD[b] * mD[c] + ro->fac[a][i] * (ms[b] * mD[c] + mD[b] * ms[c]));
            sig2[a][i] = mu23 / da;
        }
    }
    // S A S's per-axis factors; h_a = s'_a + g'_a(lower) + g'_a(upper) for the Gershgorin sums
    std::vector<double> gs[3], ss[3], ds[3], hs[3];
    double lmin = 1.0;
    for (int a = 0; a < 3; ++a) {
        const int na = n[a];
        gs[a].assign(na + 1, 0.0);
        ss[a].resize(na);
        ds[a].resize(na);
        hs[a].resize(na);
        double mn = sig2[a][0];
        for (int i = 0; i < na; ++i) {
            ss[a][i] = sig2[a][i] * ro->sd[a][i];
            ds[a][i] = sig2[a][i] * ro->fac[a][i];
            mn = std::min(mn, sig2[a][i]);
        }
        for (int i = 1; i < na; ++i) gs[a][i] = std::sqrt(sig2[a][i - 1] * sig2[a][i]) * ro->gf[a][i];
        if ((ro->per >> a) & 1) gs[a][0] = gs[a][na] = std::sqrt(sig2[a][na - 1] * sig2[a][0]) * ro->gf[a][0];
        for (int i = 0; i < na; ++i) hs[a][i] = ss[a][i] + gs[a][i] + gs[a][i + 1];
        lmin *= mn;
    }
    double lmax = 0.0;
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j) {
            const double E = sig2[1][j] * sig2[2][k];
            const double P = dtau * ds[1][j] * ds[2][k];
            const double Q = dtau * (ds[2][k] * hs[1][j] + ds[1][j] * hs[2][k]);
            double rmax = 0.0;
            for (int i = 0; i < n[0]; ++i) rmax = std::max(rmax, sig2[0][i] * E + hs[0][i] * P + ds[0][i] * Q);
            lmax = std::max(lmax, rmax);
        }
    // stage and upload (the previous call's copy and kernels must be done
    // with the staging buffer and the device arrays' old contents)
    CGD_HIP_TRY(hipStreamSynchronize(s));
    float* h = ro->host;
    size_t o = 0;
    for (int a = 0; a < 3; ++a) {
        const int na = n[a];
        for (int i = 0; i <= na; ++i) h[o++] = (float)gs[a][i];
        for (int i = 0; i < na; ++i) h[o++] = (float)ss[a][i];
        for (int i = 0; i < na; ++i) h[o++] = (float)ds[a][i];
        for (int i = 0; i < na; ++i) h[o++] = (float)sig2[a][i];
        for (int i = 0; i < na; ++i) h[o++] = (float)std::sqrt(sig2[a][i]);
    }
    CGD_HIP_TRY(hipMemcpyAsync(ro->pdev, h, o * sizeof(float), hipMemcpyHostToDevice, s));
    ro->dtau = dtau;
    ro->lmin = lmin;
    ro->lmax = std::max(lmax, lmin * (1.0 + 1e-6));
    return CGD_OK;
}

// Rectilinear grid with a separable diffusivity: the uniform grid's sweeps
// on A = I + dtau M^-1/2 K M^-1/2 for x~ = M^1/2 x (the same system as
// (M + dtau K) x = M e, scaled symmetrically), preconditioned by
// S p(S A S) S (RectOp); the stopping rule applies to the scaled residual.
static cgd_status diffuse_rect_fast(cgd_mesh m, const DiffuseArgs& da, cgd_solve_stats* out, hipStream_t s,
                                    const int* fixed) {
    const TetData* t = m->tet;
    RectOp* ro = m->rop;
    const int F = da.F;
    const int n = t->n_tet;
    cgd_status rc = ensure_workspace(m, diffuse_hex_workspace(m, F));
    if (rc != CGD_OK) return rc;
    rc = ensure_pinned(m, kPinBytes);
    if (rc != CGD_OK) return rc;
    const double T = da.bandwidth * da.bandwidth / 4.0;
    rc = rect_op_prepare(m, T / da.n_steps * (da.scheme == 1 ? 0.5 : 1.0), s);
    if (rc != CGD_OK) return rc;
    char* base = static_cast<char*>(m->ws.ptr);
    double* d_sums = reinterpret_cast<double*>(base + kOffSums);
    double* d_mpart = reinterpret_cast<double*>(base + kSmallFixed);  // free outside the solve
    const int mbpf = std::min(1024, (n + kBlock - 1) / kBlock);
    if (out) {
        hipLaunchKernelGGL(k_tet_mass, dim3(mbpf, F), dim3(kBlock), 0, s, da.field, t->vol, n, d_mpart, mbpf);
        hipLaunchKernelGGL(k_tet_sum_finish, dim3(F), dim3(kBlock), 0, s, d_mpart, mbpf, d_sums);
    }
    const int sblocks = std::min(4096, (n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_rect_scale, dim3(sblocks, F), dim3(kBlock), 0, s, da.field, (int64_t)n, m->hex.nx,
                       m->hex.ny, ro->win[0], ro->win[1], ro->win[2]);
    rc = diffuse_hex_enqueue(m, da, base, fixed, false, s, ro);
    if (rc != CGD_OK) return rc;
    hipLaunchKernelGGL(k_rect_scale, dim3(sblocks, F), dim3(kBlock), 0, s, da.field, (int64_t)n, m->hex.nx,
                       m->hex.ny, ro->wout[0], ro->wout[1], ro->wout[2]);
    if (out) {
        hipLaunchKernelGGL(k_tet_mass, dim3(mbpf, F), dim3(kBlock), 0, s, da.field, t->vol, n, d_mpart, mbpf);
        hipLaunchKernelGGL(k_tet_sum_finish, dim3(F), dim3(kBlock), 0, s, d_mpart, mbpf, d_sums + CGD_MAX_FIELDS);
    }
    return cg_finish_call(m, F, da.n_steps, 1.0, s, out, false);
}

// Per-axis factors of a rectilinear grid's operator (RectOp), when the
// diffusivity is a product of per-axis factors (checked on every cell to a
// relative 1e-6); otherwise the mesh keeps the face-slot rows only.  A
// periodic axis of at least two cells gets the face between its last and
// first cells (weights g[0] = g[n], in both cells' diagonal sums).
static cgd_status build_rect_op(cgd_mesh m, const int32_t dims[3], const double* const edges[3], const float* D,
                                int32_t periodic) {
    const int nx = dims[0], ny = dims[1], nz = dims[2];
    std::vector<double> fac[3];
    for (int a = 0; a < 3; ++a) fac[a].assign(dims[a], 1.0);
    if (D) {
        int64_t k0 = -1;
        const int64_t n = (int64_t)nx * ny * nz;
        for (int64_t k = 0; k < n && k0 < 0; ++k)
            if (D[k] > 0.f) k0 = k;
        if (k0 < 0) {
            fac[0].assign(nx, 0.0);  // no diffusion anywhere
        } else {
            const int i0 = (int)(k0 % nx), j0 = (int)((k0 / nx) % ny), z0 = (int)(k0 / ((int64_t)nx * ny));
            auto at = [&](int i, int j, int k) { return (double)D[i + (int64_t)nx * (j + (int64_t)ny * k)]; };
            const double d0 = at(i0, j0, z0);
            for (int i = 0; i < nx; ++i) fac[0][i] = at(i, j0, z0);
            for (int j = 0; j < ny; ++j) fac[1][j] = at(i0, j, z0) / d0;
            for (int k = 0; k < nz; ++k) fac[2][k] = at(i0, j0, k) / d0;
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j) {
                    const double yz = fac[1][j] * fac[2][k];
                    for (int i = 0; i < nx; ++i) {
                        const double want = at(i, j, k), got = fac[0][i] * yz;
                        if (!(std::fabs(got - want) <= 1e-6 * std::fabs(want))) return CGD_OK;  // not separable
                    }
                }
        }
    }
    RectOp* ro = new (std::nothrow) RectOp();
    if (!ro) return CGD_E_NOMEM;
    m->rop = ro;
    size_t pfloats = 0;
    std::vector<float> hA;  // A's arrays, in RectOp's order
    for (int a = 0; a < 3; ++a) {
        const int na = dims[a];
        std::vector<double>& h = ro->h[a];
        std::vector<double>& gf = ro->gf[a];
        std::vector<double>& sd = ro->sd[a];
        h.resize(na);
        gf.assign(na + 1, 0.0);
        sd.assign(na, 0.0);
        for (int i = 0; i < na; ++i) h[i] = edges[a][i + 1] - edges[a][i];
        for (int i = 0; i + 1 < na; ++i) {
            const double da = fac[a][i], db = fac[a][i + 1];
            const double hm = (da > 0.0 && db > 0.0) ? 2.0 * da * db / (da + db) : 0.0;
            const double df = 0.5 * (h[i] + h[i + 1]);
            gf[i + 1] = hm / (df * std::sqrt(h[i] * h[i + 1]));
            sd[i] += hm / (df * h[i]);
            sd[i + 1] += hm / (df * h[i + 1]);
        }
        if (((periodic >> a) & 1) && na >= 2) {
            const int l = na - 1;
            const double da = fac[a][l], db = fac[a][0];
            const double hm = (da > 0.0 && db > 0.0) ? 2.0 * da * db / (da + db) : 0.0;
            const double df = 0.5 * (h[l] + h[0]);
            gf[0] = gf[na] = hm / (df * std::sqrt(h[l] * h[0]));
            sd[l] += hm / (df * h[l]);
            sd[0] += hm / (df * h[0]);
            ro->per |= 1 << a;
        }
        ro->fac[a] = fac[a];
        for (int i = 0; i <= na; ++i) hA.push_back((float)gf[i]);
        for (int i = 0; i < na; ++i) hA.push_back((float)sd[i]);
        for (int i = 0; i < na; ++i) hA.push_back((float)fac[a][i]);
        for (int i = 0; i < na; ++i) hA.push_back(1.f);
        for (int i = 0; i < na; ++i) hA.push_back((float)std::sqrt(h[i]));
        for (int i = 0; i < na; ++i) hA.push_back((float)(1.0 / std::sqrt(h[i])));
        pfloats += (size_t)na + 1 + 4 * (size_t)na;
    }
    ro->pfloats = pfloats;
    cgd_status rc = upload(hA, &ro->dev);
    if (rc != CGD_OK) return rc;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&ro->pdev), pfloats * sizeof(float));
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&ro->host), pfloats * sizeof(float), hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error(std::string("cgd_mesh_create_rect: allocation failed: ") + hipGetErrorString(e));
        return CGD_E_NOMEM;
    }
    float* p = ro->dev;
    float* pp = ro->pdev;
    for (int a = 0; a < 3; ++a) {
        const int na = dims[a];
        ro->g[a] = p;
        p += na + 1;
        ro->s[a] = p;
        p += na;
        ro->d[a] = p;
        p += na;
        ro->e[a] = p;
        p += na;
        ro->win[a] = p;
        p += na;
        ro->wout[a] = p;
        p += na;
        ro->pg[a] = pp;
        pp += na + 1;
        ro->ps[a] = pp;
        pp += na;
        ro->pd[a] = pp;
        pp += na;
        ro->pe[a] = pp;
        pp += na;
        ro->psg[a] = pp;
        pp += na;
    }
    HexGeom& hg = m->hex;
    hg.nx = nx;
    hg.ny = ny;
    hg.nz = nz;
    for (int a = 0; a < 3; ++a) {
        hg.lo[a] = edges[a][0];
        hg.hi[a] = edges[a][dims[a]];
        hg.h[a] = (hg.hi[a] - hg.lo[a]) / dims[a];
        hg.s[a] = dims[a] / (hg.hi[a] - hg.lo[a]);
    }
    hg.vol = (hg.h[0] * hg.h[1]) * hg.h[2];
    return CGD_OK;
}

// The per-axis factor sweeps apply: a rectilinear grid with a separable
// diffusivity, the default preconditioner and a zero guess (a periodic x axis
// also needs the row in one x segment; otherwise the face-slot rows).
bool rect_fast_path(const cgd_mesh m, const DiffuseArgs& da) {
    return m->kind == 2 && m->rop && da.precond == 0 && da.x0_mode == 0 && !getenv("CGD_RECT_SLOTS") &&
           (!(m->rop->per & 1) || hex_one_x_segment(m->hex, da.field));
}

cgd_status diffuse_tet(cgd_mesh m, const DiffuseArgs& da, cgd_solve_stats* out, hipStream_t s, const int* fixed) {
    if (da.x0_mode != 0) {
        set_error("cgd_diffuse: tet meshes support x0_mode 0 only");
        return CGD_E_UNSUPPORTED;
    }
    if (rect_fast_path(m, da)) return diffuse_rect_fast(m, da, out, s, fixed);
    const TetData* t = m->tet;
    const int F = da.F;
    const int n = t->n_tet;
    const TetPlan p = tet_plan(n, F);
    const size_t small = tet_small(F, p.bpf);
    cgd_status rc = ensure_workspace(m, diffuse_tet_workspace(m, F));
    if (rc != CGD_OK) return rc;
    rc = ensure_pinned(m, kPinBytes);
    if (rc != CGD_OK) return rc;
    char* base = static_cast<char*>(m->ws.ptr);
    CgCtl ctl = {};
    ctl.st = reinterpret_cast<CgField*>(base + kOffState);
    ctl.ndone = reinterpret_cast<int*>(base + kOffNdone);
    ctl.iters = reinterpret_cast<int32_t*>(base + kOffIters);
    ctl.relres = reinterpret_cast<double*>(base + kOffRelres);
    ctl.status = reinterpret_cast<int32_t*>(base + kOffStatus);
    ctl.rtol2 = da.rtol * da.rtol;
    ctl.step = 0;
    double* d_sums = reinterpret_cast<double*>(base + kOffSums);
    double* d_P1 = reinterpret_cast<double*>(base + kSmallFixed);
    double* d_P2 = d_P1 + (size_t)F * 3 * p.bpf;
    float* W0 = reinterpret_cast<float*>(base + small);
    const size_t fn = (size_t)F * n;
    float* R = W0 + fn;
    float* PA = R + fn;
    float* PB = PA + fn;
    float* Q = PB + fn;
    float* Z = Q + fn;
    float* Wv = Z + fn;
    float* dinv = Wv + fn;

    // Crank-Nicolson solves with half the step, then extrapolates (below)
    const double dtau = da.bandwidth * da.bandwidth / 4.0 / da.n_steps * (da.scheme == 1 ? 0.5 : 1.0);
    const int eblocks = std::min(4096, (n + kBlock - 1) / kBlock);
    // Preconditioner: the Chebyshev polynomial of B = H A~ on [lmin, lmax]
    // with lmin the Rayleigh quotient of a constant field (sum V / sum
    // diag A~: the slowest modes of the mass-plus-diffusion operator are the
    // smooth ones) and lmax Gershgorin's bound 1 + t / (1 + t), t = dtau max
    // K~_ii / V_i; Jacobi (degree 0) where the cost model prefers it or
    // precond = 1.  CGD_TET_DEGREE forces an even degree 0..16.
    const double kappa = dtau * t->amax;
    const double lmin = t->sum_v / (t->sum_v + dtau * t->sum_k);
    const double tmx = dtau * t->kv_max;
    const double lmax = 1.0 + tmx / (1.0 + tmx);
    int deg = da.precond == 1 || !(t->amax > 0.0) ? 0 : tet_degree(lmin, lmax, da.rtol, t->ns);
    if (const char* e = getenv("CGD_TET_DEGREE")) deg = std::max(0, std::min(16, atoi(e))) & ~1;
    if (!(t->amax > 0.0)) deg = 0;
    double qs[8], qq[8], qg[8], lead = 1.0;
    const int nq = deg > 0 ? poly_precond_quadratics_iv(lmin, lmax, deg, qs, qq, qg, &lead) : 0;
    if (deg > 0)
        hipLaunchKernelGGL(k_tet_hinv, dim3(eblocks), dim3(kBlock), 0, s, t->volf, t->kdh, (float)kappa, dinv, n);
    else
        hipLaunchKernelGGL(k_tet_dinv, dim3(eblocks), dim3(kBlock), 0, s, t->volf, t->kdiag, (float)dtau, dinv,
                           n);

    TetArgs a = {};
    a.col = reinterpret_cast<const int4*>(t->nbr);
    a.kf = reinterpret_cast<const float4*>(t->kface);
    a.col2 = reinterpret_cast<const int2*>(t->nbr2);
    a.kf2 = reinterpret_cast<const float2*>(t->kface2);
    a.volf = t->volf;
    a.dinv = dinv;
    a.dtau = (float)dtau;
    a.Z = Z;
    a.c = ctl;
    a.P1 = d_P1;
    a.P2 = d_P2;
    a.n = n;
    a.bpf = p.bpf;
    a.nblocks = p.nblocks;
    a.nchunks = p.nchunks;
    a.R = R;
    a.Q = Q;
    const int mbpf = std::min(1024, (n + kBlock - 1) / kBlock);
    double* d_mpart = d_P2;  // free outside the solves
    if (out) {
        hipLaunchKernelGGL(k_tet_mass, dim3(mbpf, F), dim3(kBlock), 0, s, da.field, t->vol, n, d_mpart, mbpf);
        hipLaunchKernelGGL(k_tet_sum_finish, dim3(F), dim3(kBlock), 0, s, d_mpart, mbpf, d_sums);
    }
    // sweep 1, one field: ids, a_f, z, p_old, V; writes p, q (6 face slots: 16 more)
    const double b1 = (t->ns == 6 ? 68.0 : 52.0) * n;
    const double b2 = 32.0 * n;  // sweep 2, one field: p, q, x, r, D^-1; writes x, r, z
    const dim3 grid(p.nblocks), block(kBlock);
    auto sweep = [&](int mode) {
        if (t->ns == 6) {
            switch (mode) {
                case T1_FIRST: hipLaunchKernelGGL((k_tet_sweep<T1_FIRST, 6>), grid, block, 0, s, a); break;
                case T2_FIRST: hipLaunchKernelGGL((k_tet_sweep<T2_FIRST, 6>), grid, block, 0, s, a); break;
                case T1: hipLaunchKernelGGL((k_tet_sweep<T1, 6>), grid, block, 0, s, a); break;
                default: hipLaunchKernelGGL((k_tet_sweep<T2, 6>), grid, block, 0, s, a); break;
            }
        } else {
            switch (mode) {
                case T1_FIRST: hipLaunchKernelGGL((k_tet_sweep<T1_FIRST, 4>), grid, block, 0, s, a); break;
                case T2_FIRST: hipLaunchKernelGGL((k_tet_sweep<T2_FIRST, 4>), grid, block, 0, s, a); break;
                case T1: hipLaunchKernelGGL((k_tet_sweep<T1, 4>), grid, block, 0, s, a); break;
                default: hipLaunchKernelGGL((k_tet_sweep<T2, 4>), grid, block, 0, s, a); break;
            }
        }
    };
    // z = p(B) h r from v = h r in Z (sweep 2 or the step's first kernel
    // wrote it); the last pass sums r.z into part (field stride pstride)
    ChebArgs ca = {};
    ca.col = a.col;
    ca.col2 = a.col2;
    ca.kh = reinterpret_cast<const f16x4*>(t->kh);
    ca.kh2 = reinterpret_cast<const f16x2*>(t->kh2);
    ca.h = dinv;
    ca.R = R;
    ca.c = ctl;
    ca.kappa = (float)kappa;
    ca.n = n;
    ca.bpf = p.bpf;
    ca.nblocks = p.nblocks;
    ca.nchunks = p.nchunks;
    // pass 1: ids, a~, h, v; writes w.  pass 2: the same with w, plus v; writes v (+ r in the last)
    const double slot_b = t->ns == 6 ? 36.0 : 24.0;
    const double bp1 = (slot_b + 12.0) * n, bp2 = (slot_b + 16.0) * n;
    // rrp / kcheck: sweep 2's r.r partials and the iteration they decide
    // (the first pass makes the check, so a converged field skips the passes)
    auto cheb = [&](double* part, size_t pstride, int64_t tag, const double* rrp, int kcheck) {
        ca.part = part;
        ca.pstride = pstride;
        for (int k = 0; k < nq; ++k) {
            const bool last = k + 1 == nq;
            ca.rrp = k == 0 ? rrp : nullptr;
            ca.kcheck = kcheck;
            ca.G = Z;
            ca.out = Wv;
            int t1 = timing_begin(&m->timing, s);
            if (t->ns == 6) hipLaunchKernelGGL((k_tet_cheb<6, 0>), grid, block, 0, s, ca);
            else hipLaunchKernelGGL((k_tet_cheb<4, 0>), grid, block, 0, s, ca);
            timing_end(&m->timing, t1, 16, bp1 * F, s, tag);
            ca.G = Wv;
            ca.V = Z;
            ca.out = Z;
            ca.c1 = (float)(1.0 + qs[k]);
            ca.cq = (float)qq[k];
            ca.gk = (float)(qg[k] * (last ? lead : 1.0));
            int t2 = timing_begin(&m->timing, s);
            if (t->ns == 6) {
                if (last) hipLaunchKernelGGL((k_tet_cheb<6, 2>), grid, block, 0, s, ca);
                else hipLaunchKernelGGL((k_tet_cheb<6, 1>), grid, block, 0, s, ca);
            } else {
                if (last) hipLaunchKernelGGL((k_tet_cheb<4, 2>), grid, block, 0, s, ca);
                else hipLaunchKernelGGL((k_tet_cheb<4, 1>), grid, block, 0, s, ca);
            }
            timing_end(&m->timing, t2, 17, (bp2 + (last ? 4.0 * n : 0.0)) * F, s, tag);
        }
    };
    float* cur = da.field;
    float* nxt = W0;
    for (int step = 0; step < da.n_steps; ++step) {
        a.c.step = step;
        ca.c.step = step;  // the passes record a converged check in this step's row
        a.B = cur;
        a.X = nxt;
        hipLaunchKernelGGL(k_cg_step_init, dim3(1), dim3(64), 0, s, ctl.st, F, ctl.ndone,
                           ctl.status + step * CGD_MAX_FIELDS);
        a.k = 0;
        a.Pnew = PA;
        a.Pold = PB;
        if (nq > 0) {
            // r_0 = M e, v = h r_0, b.b; z_0 and r.z from the passes; then
            // the direction sweep with p = z_0
            hipLaunchKernelGGL(k_tet_cheb_init, grid, block, 0, s, a);
            cheb(d_P1 + p.bpf, (size_t)3 * p.bpf, (int64_t)step * 65536, nullptr, 0);
            if (t->ns == 6) hipLaunchKernelGGL((k_tet_sweep<T1_FIRST, 6, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_tet_sweep<T1_FIRST, 4, true>), grid, block, 0, s, a);
        } else {
            sweep(T1_FIRST);
        }
        sweep(T2_FIRST);
        if (nq > 0)
            cheb(d_P2 + (size_t)2 * p.bpf, (size_t)4 * p.bpf, (int64_t)step * 65536 + 1, d_P2 + (size_t)3 * p.bpf,
                 1);
        bool next_cheb = true;  // an iteration ends with the next one's preconditioner (and its check)
        auto enqueue = [&](int it, int* host_flags) {
            a.k = it;
            a.Pold = (it & 1) ? PA : PB;
            a.Pnew = (it & 1) ? PB : PA;
            const int64_t tag = (int64_t)step * 65536 + it;
            int t1 = timing_begin(&m->timing, s);
            sweep(T1);
            timing_end(&m->timing, t1, 3, b1 * F, s, tag);
            a.c.host_flags = host_flags;
            int t2 = timing_begin(&m->timing, s);
            sweep(T2);
            timing_end(&m->timing, t2, 4, b2 * F, s, tag);
            a.c.host_flags = nullptr;
            // sweep 2 of iteration it wrote v = h r and r.r for parity (it + 1) & 1
            // (tagged with the iteration it serves, so that it is timed only when that one ran)
            if (nq > 0 && next_cheb)
                cheb(d_P2 + (size_t)((it + 1) & 1) * 2 * p.bpf, (size_t)4 * p.bpf, tag + 1,
                     d_P2 + ((size_t)((it + 1) & 1) * 2 + 1) * p.bpf, it + 1);
        };
        int it_end = 1;
        if (fixed) {
            // a fixed budget of iterations, with no read-back; the last one
            // leaves out the next preconditioner, whose first pass would only
            // make the check that the step end makes from the same partials
            it_end = std::max(1, std::min(fixed[step], da.max_iter));
            for (int it = 1; it < it_end; ++it) {
                next_cheb = it + 1 < it_end;
                enqueue(it, nullptr);
            }
        } else {
            rc = cg_lookahead_loop(m, F, 1, da.max_iter, da.check_every, ctl.ndone, s, enqueue, &it_end);
            if (rc != CGD_OK) return rc;
        }
        CgCtl c2 = ctl;
        c2.step = step;
        // r.r of the last sweep 2: parity (it_end & 1), second slot, summed
        // as the check of the passes and sweeps (256 threads)
        hipLaunchKernelGGL(k_cg_step_end<kCgBlock>, dim3(F), dim3(kCgBlock), 0, s, c2,
                           d_P2 + ((size_t)(it_end & 1) * 2 + 1) * p.bpf, (size_t)4 * p.bpf, p.bpf, it_end);
        if (da.scheme == 1) cn_extrapolate(nxt, cur, (int64_t)fn, s);
        std::swap(cur, nxt);
    }
    if (cur != da.field)
        CGD_HIP_TRY(hipMemcpyAsync(da.field, cur, fn * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (out) {
        hipLaunchKernelGGL(k_tet_mass, dim3(mbpf, F), dim3(kBlock), 0, s, da.field, t->vol, n, d_mpart, mbpf);
        hipLaunchKernelGGL(k_tet_sum_finish, dim3(F), dim3(kBlock), 0, s, d_mpart, mbpf, d_sums + CGD_MAX_FIELDS);
    }
    return cg_finish_call(m, F, da.n_steps, 1.0, s, out);
}

}  // namespace cgd

using namespace cgd;

extern "C" cgd_status cgd_mesh_create_tet(int64_t n_vert, const double* xyz, int64_t n_tet, const int32_t* tv,
                                          cgd_mesh* out) {
    return cgd_mesh_create_tet_d(n_vert, xyz, n_tet, tv, nullptr, out);
}

extern "C" cgd_status cgd_mesh_create_tet_d(int64_t n_vert, const double* xyz, int64_t n_tet, const int32_t* tv,
                                            const float* diffusivity, cgd_mesh* out) {
    if (!out || !xyz || !tv) {
        set_error("cgd_mesh_create_tet: null pointer");
        return CGD_E_INVALID;
    }
    *out = nullptr;
    TetHost h;
    cgd_status rc;
    try {
        rc = build_tet_host(n_vert, xyz, n_tet, tv, diffusivity, &h);
    } catch (const std::bad_alloc&) {
        set_error("cgd_mesh_create_tet: host allocation failed");
        return CGD_E_NOMEM;
    }
    if (rc != CGD_OK) return rc;
    cgd_mesh m = new (std::nothrow) cgd_mesh_s();
    if (!m) return CGD_E_NOMEM;
    m->kind = 1;
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        set_error("cgd_mesh_create_tet: no HIP device");
        return CGD_E_HIP;
    }
    m->cells = h.n_tet;
    m->tet = new (std::nothrow) TetData();
    if (!m->tet) {
        delete m;
        return CGD_E_NOMEM;
    }
    TetData* t = m->tet;
    t->n_tet = h.n_tet;
    t->n_vert = h.n_vert;
    t->nnz = h.nnz;
    for (int a = 0; a < 3; ++a) {
        t->nb[a] = h.nb[a];
        t->glo[a] = h.glo[a];
        t->ghi[a] = h.ghi[a];
        t->ginv[a] = h.ginv[a];
    }
    std::vector<double> hx(xyz, xyz + n_vert * 3);
    std::vector<int32_t> htv(tv, tv + n_tet * 4);
    std::vector<float> volf(h.vol.size());
    for (size_t i = 0; i < volf.size(); ++i) volf[i] = (float)h.vol[i];
    std::vector<cgd_status> st = {upload(hx, &t->xyz),         upload(htv, &t->tv),       upload(h.vol, &t->vol),
                                  upload(volf, &t->volf),      upload(h.bbox, &t->bbox),  upload(h.kface, &t->kface),
                                  upload(h.kdiag, &t->kdiag),
                                  upload(h.bstart, &t->bstart), upload(h.blist, &t->blist),
                                  upload(h.bseed, &t->bseed),   upload(h.nbr, &t->nbr),
                                  cheb_operator_setup(t, h.kface, {}, h.vol)};
    for (cgd_status r : st) {
        if (r != CGD_OK) {
            cgd_mesh_destroy(m);
            return r;
        }
    }
    for (int i = 0; i < 2; ++i) {
        if (hipEventCreateWithFlags(&m->ev[i], hipEventDisableTiming) != hipSuccess) {
            cgd_mesh_destroy(m);
            set_error("cgd_mesh_create_tet: hipEventCreate failed");
            return CGD_E_HIP;
        }
    }
    *out = m;
    return CGD_OK;
}

// Rectilinear (stretched) hex meshes with a cell-wise diffusivity: the padded
// rows of the tet solver with 6 face slots.  Face coefficient between cells a
// and b along an axis: D_f A_f / d_f with A_f the face area, d_f the distance
// between the two cell centres and D_f = 2 D_a D_b / (D_a + D_b) (0 when
// either is 0), evaluated in float64 and rounded once; volumes
// (hx_i hy_j) hz_k in float64.  On a periodic axis the first and last cells
// share a face at distance (h_first + h_last) / 2 (Section 3.1).
extern "C" cgd_status cgd_mesh_create_rect(int32_t nx, int32_t ny, int32_t nz, const double* x_edges,
                                           const double* y_edges, const double* z_edges, const float* diffusivity,
                                           int32_t periodic, cgd_mesh* out) {
    if (!out || !x_edges || !y_edges || !z_edges) {
        set_error("cgd_mesh_create_rect: null pointer");
        return CGD_E_INVALID;
    }
    *out = nullptr;
    const int32_t dims[3] = {nx, ny, nz};
    const double* edges[3] = {x_edges, y_edges, z_edges};
    if (nx < 1 || ny < 1 || nz < 1 || (int64_t)nx * ny * nz >= (int64_t(1) << 28)) {
        set_error("cgd_mesh_create_rect: need n_a >= 1 and nx * ny * nz < 2^28");
        return CGD_E_INVALID;
    }
    if (periodic & ~7) {
        set_error("cgd_mesh_create_rect: periodic is a mask of bits 0 (x), 1 (y), 2 (z)");
        return CGD_E_INVALID;
    }
    for (int a = 0; a < 3; ++a) {
        for (int i = 0; i <= dims[a]; ++i) {
            if (!std::isfinite(edges[a][i]) || (i > 0 && !(edges[a][i] > edges[a][i - 1]))) {
                set_error("cgd_mesh_create_rect: edges must be finite and strictly increasing");
                return CGD_E_INVALID;
            }
        }
    }
    const int64_t n = (int64_t)nx * ny * nz;
    std::vector<double> hw[3], hd, vol, redges;
    std::vector<float> volf, kface, kface2, kdiag, D;
    std::vector<int32_t> nbr, nbr2;
    try {
        if (diffusivity) {
            D.assign(diffusivity, diffusivity + n);
            for (float d : D) {
                if (!std::isfinite(d) || d < 0.f) {
                    set_error("cgd_mesh_create_rect: diffusivity must be finite and >= 0");
                    return CGD_E_INVALID;
                }
            }
        }
        for (int a = 0; a < 3; ++a) {
            for (int i = 0; i < dims[a]; ++i) hw[a].push_back(edges[a][i + 1] - edges[a][i]);
            redges.insert(redges.end(), edges[a], edges[a] + dims[a] + 1);
        }
        vol.resize(n);
        volf.resize(n);
        kface.assign((size_t)n * 4, 0.f);
        kface2.assign((size_t)n * 2, 0.f);
        kdiag.assign(n, 0.f);
        nbr.resize((size_t)n * 4);
        nbr2.resize((size_t)n * 2);
    } catch (const std::bad_alloc&) {
        set_error("cgd_mesh_create_rect: host allocation failed");
        return CGD_E_NOMEM;
    }
    auto dcell = [&](int64_t k) { return D.empty() ? 1.0 : (double)D[k]; };
    int64_t faces = 0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int64_t me = i + (int64_t)nx * (j + (int64_t)ny * k);
                vol[me] = (hw[0][i] * hw[1][j]) * hw[2][k];
                volf[me] = (float)vol[me];
                const int c[3] = {i, j, k};
                const int64_t stride[3] = {1, nx, (int64_t)nx * ny};
                double diag = 0.0;
                for (int a = 0; a < 3; ++a) {
                    const double area = hw[(a + 1) % 3][c[(a + 1) % 3]] * hw[(a + 2) % 3][c[(a + 2) % 3]];
                    for (int side = 0; side < 2; ++side) {  // 0: lower neighbour, 1: upper
                        const int slot = 2 * a + side;
                        int cn = c[a] + (side ? 1 : -1);
                        if ((cn < 0 || cn >= dims[a]) && ((periodic >> a) & 1) && dims[a] >= 2)
                            cn = (cn + dims[a]) % dims[a];  // the face across the periodic boundary
                        int64_t nb = me;
                        double w = 0.0;
                        if (cn >= 0 && cn < dims[a]) {
                            nb = me + (int64_t)(cn - c[a]) * stride[a];
                            const double da = dcell(me), db = dcell(nb);
                            const double df = (da > 0.0 && db > 0.0) ? 2.0 * da * db / (da + db) : 0.0;
                            w = df * area / (0.5 * (hw[a][c[a]] + hw[a][cn]));
                            if (side) ++faces;
                        }
                        if (slot < 4) {
                            nbr[(size_t)me * 4 + slot] = (int32_t)nb;
                            kface[(size_t)me * 4 + slot] = (float)w;
                        } else {
                            nbr2[(size_t)me * 2 + slot - 4] = (int32_t)nb;
                            kface2[(size_t)me * 2 + slot - 4] = (float)w;
                        }
                        diag += w;
                    }
                }
                kdiag[me] = (float)diag;
            }
    cgd_mesh m = new (std::nothrow) cgd_mesh_s();
    if (!m) return CGD_E_NOMEM;
    m->kind = 2;
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        set_error("cgd_mesh_create_rect: no HIP device");
        return CGD_E_HIP;
    }
    m->cells = n;
    m->tet = new (std::nothrow) TetData();
    if (!m->tet) {
        delete m;
        return CGD_E_NOMEM;
    }
    TetData* t = m->tet;
    t->n_tet = (int32_t)n;
    t->nnz = n + 2 * faces;
    t->ns = 6;
    for (int a = 0; a < 3; ++a) t->rdim[a] = dims[a];
    std::vector<cgd_status> st = {upload(vol, &t->vol),       upload(volf, &t->volf),   upload(kface, &t->kface),
                                  upload(kface2, &t->kface2), upload(kdiag, &t->kdiag), upload(nbr, &t->nbr),
                                  upload(nbr2, &t->nbr2),     upload(redges, &t->redges),
                                  cheb_operator_setup(t, kface, kface2, vol)};
    for (cgd_status r : st) {
        if (r != CGD_OK) {
            cgd_mesh_destroy(m);
            return r;
        }
    }
    for (int i = 0; i < 2; ++i) {
        if (hipEventCreateWithFlags(&m->ev[i], hipEventDisableTiming) != hipSuccess) {
            cgd_mesh_destroy(m);
            set_error("cgd_mesh_create_rect: hipEventCreate failed");
            return CGD_E_HIP;
        }
    }
    {
        cgd_status r = build_rect_op(m, dims, edges, diffusivity, periodic);
        if (r != CGD_OK) {
            cgd_mesh_destroy(m);
            return r;
        }
    }
    *out = m;
    return CGD_OK;
}
