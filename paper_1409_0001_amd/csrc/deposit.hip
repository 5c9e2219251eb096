// Particle centroid method on uniform hex grids (Section 2.2, eq. pcm-k),
// bit-exact through 64-bit fixed point.
//
// Direct pipeline (all on the caller's stream, no host synchronisation; the
// tiled pipeline below replaces the last three steps):
//   k_dep_init   reset the per-call counters
//   k_zero64     clear the int64 accumulators
//   k_absmax     max |v| per field over finite values -> fixed-point scale S_f
//   k_deposit    centroid binning in float64 + int64 atomic adds of rint(v 2^S_f)
//   k_finalize   field = float32((acc * 2^-S_f) / V)
//
// The bin index and the quantised value are integers decided by float64
// arithmetic that is written so that no operation can be contracted or
// reordered: (x - lo) * s, floor, clamp; ldexp + round-half-even.
#pragma clang fp contract(off)

#include <stdlib.h>

#include <algorithm>

#include "cgd_internal.h"
#include "hex_bin.h"

namespace cgd {
namespace {

constexpr int kBlock = 256;

__global__ void k_dep_init(DepositInfo* info, ScaleForce fs) {
    int t = threadIdx.x;
    if (t < CGD_MAX_FIELDS) {
        info->maxbits[t] = 0u;
        info->force_s[t] = fs.s[t];
        info->nonfinite_val[t] = 0ull;
    }
    if (t == 0) {
        info->dropped = 0ull;
        info->nonfinite_pos = 0ull;
    }
}

__global__ void k_zero64(unsigned long long* __restrict__ p, int64_t n) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0ull;
}

// Max |v| over finite values of each field, as an unsigned bit pattern
// (for non-negative floats the integer order equals the float order).
__global__ void k_absmax(const float* __restrict__ values, int64_t n, DepositInfo* info) {
    const int f = blockIdx.y;
    const uint32_t* v = reinterpret_cast<const uint32_t*>(values + (size_t)f * n);
    uint32_t m = 0u;
    unsigned long long bad = 0ull;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t a = v[i] & 0x7fffffffu;
        if (a >= 0x7f800000u) {
            ++bad;
        } else {
            m = a > m ? a : m;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t mo = __shfl_xor(m, o);
        m = mo > m ? mo : m;
        bad += __shfl_xor(bad, o);
    }
    __shared__ uint32_t sm[kBlock / 64];
    __shared__ unsigned long long sb[kBlock / 64];
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sm[w] = m;
        sb[w] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t mm = 0u;
        unsigned long long bb = 0ull;
        for (int i = 0; i < kBlock / 64; ++i) {
            mm = sm[i] > mm ? sm[i] : mm;
            bb += sb[i];
        }
        if (mm) atomic_max_if_larger(&info->maxbits[f], mm);
        if (bb) atomicAdd(&info->nonfinite_val[f], bb);
    }
}

__global__ __launch_bounds__(kBlock) void k_deposit_hex(
    const float* __restrict__ pos, const float* __restrict__ values, int64_t n, int F, HexBin g,
    int e_n, unsigned long long* __restrict__ acc, int64_t cells, DepositInfo* info) {
    __shared__ int S[CGD_MAX_FIELDS];
    if (threadIdx.x < F) S[threadIdx.x] = frac_bits_used(info->maxbits[threadIdx.x], info->force_s[threadIdx.x], e_n);
    __syncthreads();
    unsigned long long dropped = 0ull, nfpos = 0ull;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        bool nf;
        int64_t k = hex_cell(g, pos[3 * p], pos[3 * p + 1], pos[3 * p + 2], &nf);
        if (k < 0) {
            ++dropped;
            nfpos += nf ? 1ull : 0ull;
            continue;
        }
        for (int f = 0; f < F; ++f) {
            float v = values[(size_t)f * n + p];
            if (!isfinite(v)) continue;
            long long q = __double2ll_rn(ldexp((double)v, S[f]));
            if (q != 0) atomicAdd(&acc[(size_t)f * cells + k], (unsigned long long)q);
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

// ---------------------------------------------------------------- tiled deposit
// The cells of a grid are cut into tiles of `cpt` consecutive indices.  The
// particles are bucketed by tile (a counting sort over fixed chunks of
// particles per block), then one workgroup per tile adds its particles'
// fixed-point values in LDS and writes the tile's finished field (and
// accumulators): every int64 sum stays exact, and the device-wide atomics on
// the accumulators of the direct path are replaced by LDS atomics.  A
// bucketed record is 8 bytes, (cell within the tile, bits of the first
// field's value); further fields' values follow in their own arrays, and the
// values are quantised in the accumulate pass.  Several snapshots on the
// same grid (particle ranges off[j] .. off[j + 1]) are deposited together:
// snapshot j's tiles are numbered j * ntiles + t, and its fixed-point scales
// come from its own max |v| and particle count, so each snapshot's result is
// the one a deposit of that snapshot alone gives.

constexpr int kTBlock = 1024;
constexpr int kTPer = 16;                  // particles per thread and pass, held in registers
constexpr int kTChunk = kTBlock * 16;      // particles per block and chunk of the bucketing passes
constexpr int kTPass = kTChunk / (kTBlock * kTPer);  // register passes per chunk
constexpr int kBPer = 4;                   // particles per thread and register pass of the counting pass
constexpr int kTileWords = 16384;          // int64 LDS accumulators of one tile workgroup (128 KB)
constexpr int kMaxTiles = 8192;            // LDS tile counters of the bucketing passes (per snapshot)
constexpr int kMaxTilesPacked = 2 * kMaxTiles;  // ... as 16-bit halves of the same words (PACK)
constexpr int kPackMaxChunks = 3;          // chunks per block with 16-bit counters (3 x 16384 < 2^16)
constexpr int kRectEdges = kRectTiledEdges;  // rectilinear grids: edges of all three axes held in LDS

struct TileArgs {
    const float* pos;
    const float* values;   // [F][total]
    int64_t total;
    const int64_t* off;    // [n_snap + 1] particle offsets; nullptr: one snapshot [0, total)
    int n_snap, F;
    HexBin g;
    int64_t cells;         // of one snapshot's grid
    int cpt, ntiles;       // cells per tile, tiles per snapshot
    int cpt_log2;          // cpt = 2^cpt_log2
    int nsub;              // kTChunk-particle chunks per block of the scatter
    int nsub_bin;          // ... and of the counting pass
    int32_t* cellbuf;      // [total]: host cell of each particle (-1: dropped)
    uint32_t* counts;      // [n_snap * ntiles]: particles per tile
    uint32_t* offsets;     // [n_snap * ntiles + 1]
    uint32_t* cursor;      // [n_snap * ntiles]
    // Tile-bucketed records [total]: F = 1: (cell within its tile, bits of
    // field 0's value), 8 bytes; F >= 2: (cell, fields 0, 1, 2), 16 bytes
    // (one scattered write per particle instead of one per field).
    uint2* rec;
    uint4* rec4;
    float* rv;             // [F - 3][total]: values of fields 3.. (F >= 4), tile-bucketed
    uint32_t* maxbits;     // [n_snap][F]
    const int32_t* force_s;  // nullable: [F] scales forced by the caller
    unsigned long long* nf_val;  // snapshot j's non-finite values of field f counted at
                                 // nf_val[j * cnt_jstride + f * nf_val_stride]
    int nf_val_stride;
    int cnt_jstride;       // snapshot stride of the three counters (dropped, nf_pos, nf_val)
    unsigned long long* dropped;
    unsigned long long* nf_pos;
    float* field;          // [n_snap][F][cells]
    long long* acc;        // nullable, [n_snap][F][cells]
    double vol;
    int rect;              // 1: rectilinear edges (rl) locate, vcell [cells] holds each cell's volume
    RectLoc rl;
    const double* vcell;
};

// Per-block tile counters in LDS: one 32-bit word per tile, or (PACK, for
// up to twice the tiles in the same words) two 16-bit counters per word, tile
// t in half t & 1 of word t >> 1; a block's chunk has fewer than 2^16
// particles then, so no half carries into the other.
template <bool PACK>
__device__ inline uint32_t hist_add(uint32_t* h, int t) {  // returns the count before
    if constexpr (PACK) {
        const int sh = (t & 1) << 4;
        return (atomicAdd(&h[t >> 1], 1u << sh) >> sh) & 0xFFFFu;
    } else {
        return atomicAdd(&h[t], 1u);
    }
}
template <bool PACK>
__device__ inline uint32_t hist_get(const uint32_t* h, int t) {
    if constexpr (PACK) return (h[t >> 1] >> ((t & 1) << 4)) & 0xFFFFu;
    else return h[t];
}
template <bool PACK>
__device__ inline int hist_words(int ntiles) { return PACK ? (ntiles + 1) >> 1 : ntiles; }

__device__ inline void snap_range(const TileArgs& a, int j, int64_t& s0, int64_t& s1) {
    s0 = a.off ? a.off[j] : 0;
    s1 = a.off ? a.off[j + 1] : a.total;
}

__device__ inline int e_n_dev(int64_t n) { return n <= 1 ? 0 : 64 - __clzll((unsigned long long)(n - 1)); }

__global__ void k_tile_clear(TileArgs a) {
    const int nt = a.n_snap * a.ntiles;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += gridDim.x * blockDim.x) a.counts[t] = 0u;
}

// Pass 1 (grid: blocks x snapshots): host cells (stored), dropped counts,
// particles per tile, and the max |v| / non-finite count of every field over
// the block's chunk of nsub_bin * kTChunk particles (the values of the direct
// path's k_absmax, folded into this pass).
// RECT: the host cell by the rectilinear edges (RectLoc's definition), from
// a copy of the edges in LDS: per axis the largest i < n with e_i <= x by
// binary lifting (steps of decreasing powers of two, the same count for
// every lane), the kBPer particles of a thread interleaved.
template <bool RECT, bool PACK>
__global__ __launch_bounds__(kTBlock) void k_tile_bin(TileArgs a) {
    __shared__ uint32_t hist[kMaxTiles];
    __shared__ double redge[RECT ? kRectEdges : 1];
    __shared__ uint32_t bmax[CGD_MAX_FIELDS];
    __shared__ unsigned long long bbad[CGD_MAX_FIELDS];
    const int j = blockIdx.y;
    int64_t s0, s1;
    snap_range(a, j, s0, s1);
    const int64_t cb = s0 + (int64_t)blockIdx.x * a.nsub_bin * kTChunk;
    if (cb >= s1) return;  // the whole block: beyond its snapshot's particles
    const int64_t ce = min(cb + (int64_t)a.nsub_bin * kTChunk, s1);
    for (int t = threadIdx.x; t < hist_words<PACK>(a.ntiles); t += kTBlock) hist[t] = 0u;
    if (threadIdx.x < CGD_MAX_FIELDS) {
        bmax[threadIdx.x] = 0u;
        bbad[threadIdx.x] = 0ull;
    }
    if constexpr (RECT) {
        const int ne = a.rl.n[0] + a.rl.n[1] + a.rl.n[2] + 3;  // <= kRectEdges (host)
        for (int i = threadIdx.x; i < ne; i += kTBlock) redge[i] = a.rl.e[i];
    }
    __syncthreads();
    unsigned long long dropped = 0ull, nfpos = 0ull;
    const int npass = a.nsub_bin * (kTChunk / (kTBlock * kBPer));
    // Software pipeline: the positions of pass sub + 1 are loaded before the
    // cell ids of pass sub are stored (loads and stores share one counter, so
    // loads issued after the stores would wait for them), and every load is
    // unconditional (clamped index) so that none is sunk into a branch.
    float px[kBPer], py[kBPer], pz[kBPer];
    auto load = [&](int sub) {
        const int64_t p0 = cb + (int64_t)sub * (kTBlock * kBPer) + threadIdx.x;
#pragma unroll
        for (int i = 0; i < kBPer; ++i) {
            const int64_t p = min(p0 + (int64_t)i * kTBlock, ce - 1);
            px[i] = a.pos[3 * p];
            py[i] = a.pos[3 * p + 1];
            pz[i] = a.pos[3 * p + 2];
        }
    };
    load(0);
    for (int sub = 0; sub < npass; ++sub) {
        const int64_t p0 = cb + (int64_t)sub * (kTBlock * kBPer) + threadIdx.x;
        int32_t k[kBPer];
        bool nf[kBPer];
        if constexpr (RECT) {
            // a non-finite coordinate on any axis counts as non-finite; a
            // point outside the closed box on any axis is dropped
            double p[kBPer][3];
            bool in[kBPer];
            int id[kBPer];
#pragma unroll
            for (int i = 0; i < kBPer; ++i) {
                p[i][0] = (double)px[i];
                p[i][1] = (double)py[i];
                p[i][2] = (double)pz[i];
                nf[i] = !(isfinite(p[i][0]) && isfinite(p[i][1]) && isfinite(p[i][2]));
                in[i] = !nf[i];
                id[i] = 0;
            }
            int off = 0, mul = 1;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const int na = a.rl.n[ax];
                const double* e = redge + off;
                int ia[kBPer];
#pragma unroll
                for (int i = 0; i < kBPer; ++i) {
                    in[i] = in[i] && p[i][ax] >= e[0] && p[i][ax] <= e[na];
                    ia[i] = 0;
                }
                for (int step = na > 1 ? 1 << (31 - __clz(na - 1)) : 0; step > 0; step >>= 1) {
#pragma unroll
                    for (int i = 0; i < kBPer; ++i) {
                        const int c = ia[i] + step;
                        ia[i] = (c < na && e[min(c, na - 1)] <= p[i][ax]) ? c : ia[i];
                    }
                }
#pragma unroll
                for (int i = 0; i < kBPer; ++i) id[i] += mul * ia[i];
                off += na + 1;
                mul *= na;
            }
#pragma unroll
            for (int i = 0; i < kBPer; ++i) k[i] = in[i] ? id[i] : -1;
        } else {
#pragma unroll
            for (int i = 0; i < kBPer; ++i) k[i] = (int32_t)hex_cell(a.g, px[i], py[i], pz[i], &nf[i]);
        }
        if (sub + 1 < npass) load(sub + 1);
#pragma unroll
        for (int i = 0; i < kBPer; ++i) {
            const int64_t p = p0 + (int64_t)i * kTBlock;
            if (p >= ce) continue;
            a.cellbuf[p] = k[i];
            if (k[i] < 0) {
                ++dropped;
                nfpos += nf[i] ? 1ull : 0ull;
            } else {
                (void)hist_add<PACK>(hist, k[i] >> a.cpt_log2);
            }
        }
    }
    for (int f = 0; f < a.F; ++f) {
        const uint32_t* v = reinterpret_cast<const uint32_t*>(a.values + (size_t)f * a.total);
        uint32_t m = 0u;
        unsigned long long bad = 0ull;
        for (int sub = 0; sub < npass; ++sub) {
            const int64_t p0 = cb + (int64_t)sub * (kTBlock * kBPer) + threadIdx.x;
            uint32_t x[kBPer];
#pragma unroll
            for (int i = 0; i < kBPer; ++i) {
                const int64_t p = p0 + (int64_t)i * kTBlock;
                const uint32_t raw = v[min(p, ce - 1)];  // unconditional: no load in a branch
                x[i] = p < ce ? raw & 0x7fffffffu : 0u;
            }
#pragma unroll
            for (int i = 0; i < kBPer; ++i) {
                if (x[i] >= 0x7f800000u) {
                    ++bad;
                } else {
                    m = x[i] > m ? x[i] : m;
                }
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const uint32_t mo = __shfl_xor(m, o);
            m = mo > m ? mo : m;
            bad += __shfl_xor(bad, o);
        }
        if ((threadIdx.x & 63) == 0) {
            if (m) atomicMax(&bmax[f], m);
            if (bad) atomicAdd(&bbad[f], bad);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        dropped += __shfl_xor(dropped, o);
        nfpos += __shfl_xor(nfpos, o);
    }
    if ((threadIdx.x & 63) == 0 && dropped) {
        atomicAdd(a.dropped + (size_t)j * a.cnt_jstride, dropped);
        if (nfpos) atomicAdd(a.nf_pos + (size_t)j * a.cnt_jstride, nfpos);
    }
    __syncthreads();
    uint32_t* counts = a.counts + (size_t)j * a.ntiles;
    for (int t = threadIdx.x; t < a.ntiles; t += kTBlock)
        if (const uint32_t c = hist_get<PACK>(hist, t)) atomicAdd(&counts[t], c);
    if (threadIdx.x < a.F) {
        const int f = threadIdx.x;
        if (bmax[f]) atomic_max_if_larger(&a.maxbits[j * a.F + f], bmax[f]);
        if (bbad[f]) atomicAdd(&a.nf_val[(size_t)j * a.cnt_jstride + f * a.nf_val_stride], bbad[f]);
    }
}

// Pass 2: offsets = exclusive prefix sum of the counts of all tiles (one
// block): each thread sums a run of consecutive tiles, a wave scan by
// shuffles and the wave totals give each run's start.
__global__ __launch_bounds__(kTBlock) void k_tile_scan(TileArgs a) {
    __shared__ uint32_t wsum[kTBlock / 64];
    const int nt = a.n_snap * a.ntiles;
    const int per = (nt + kTBlock - 1) / kTBlock;
    const int t0 = min((int)threadIdx.x * per, nt), t1 = min(t0 + per, nt);
    uint32_t s = 0u;
    for (int t = t0; t < t1; ++t) s += a.counts[t];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = s;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = 0u, total = 0u;
    for (int w = 0; w < kTBlock / 64; ++w) {
        const uint32_t v = wsum[w];
        before += w < wave ? v : 0u;
        total += v;
    }
    if (threadIdx.x == 0) a.offsets[nt] = total;
    uint32_t run = before + incl - s;
    for (int t = t0; t < t1; ++t) {
        a.offsets[t] = run;
        a.cursor[t] = run;
        run += a.counts[t];
    }
}

// Pass 3 (grid: blocks x snapshots): each block counts its chunk of
// nsub * kTChunk particles per tile, reserves one range per tile, then
// writes the particles' records there, a register pass of kTPer particles
// per thread at a time (R16: 16-byte records, in two halves of the pass so
// that the three values' registers fit).
template <bool R16, bool PACK>
__global__ __launch_bounds__(kTBlock) void k_tile_scatter(TileArgs a) {
    __shared__ uint32_t hist[kMaxTiles];
    __shared__ uint32_t base[PACK ? kMaxTilesPacked : kMaxTiles];
    const int j = blockIdx.y;
    int64_t s0, s1;
    snap_range(a, j, s0, s1);
    const int64_t cb = s0 + (int64_t)blockIdx.x * a.nsub * kTChunk;
    if (cb >= s1) return;  // the whole block: beyond its snapshot's particles
    const int64_t ce = min(cb + (int64_t)a.nsub * kTChunk, s1);
    const int64_t c0 = cb + threadIdx.x;
    const int nw = hist_words<PACK>(a.ntiles);
    for (int t = threadIdx.x; t < nw; t += kTBlock) hist[t] = 0u;
    __syncthreads();
    const int npass = a.nsub * kTPass;
    for (int sub = 0; sub < npass; ++sub) {
        const int64_t p0 = c0 + (int64_t)sub * (kTBlock * kTPer);
        int32_t kk[kTPer];
#pragma unroll
        for (int i = 0; i < kTPer; ++i) {
            const int64_t p = p0 + (int64_t)i * kTBlock;
            kk[i] = p < ce ? a.cellbuf[p] : -1;
        }
#pragma unroll
        for (int i = 0; i < kTPer; ++i)
            if (kk[i] >= 0) (void)hist_add<PACK>(hist, kk[i] >> a.cpt_log2);
    }
    __syncthreads();
    // (one cursor atomic in flight per thread: issuing all of a thread's
    // together congested the tile cursors, 173 -> 224 us on the dense bed)
    uint32_t* cursor = a.cursor + (size_t)j * a.ntiles;
    for (int w = threadIdx.x; w < nw; w += kTBlock) {
        constexpr int TW = PACK ? 2 : 1;  // tiles per counter word
        for (int h = 0; h < TW; ++h) {
            const int t = w * TW + h;
            if (t >= a.ntiles) break;
            const uint32_t c = hist_get<PACK>(hist, t);
            base[t] = c ? atomicAdd(&cursor[t], c) : 0u;
        }
        hist[w] = 0u;  // reused as the in-block rank counter
    }
    __syncthreads();
    constexpr int NP = R16 ? kTPer / 2 : kTPer;  // particles per thread in one write pass
    for (int sub = 0; sub < npass * (kTPer / NP); ++sub) {
        const int64_t p0 = c0 + (int64_t)sub * (kTBlock * NP);
        int32_t kk[NP];
        float v0[NP], v1[NP], v2[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int64_t p = p0 + (int64_t)i * kTBlock;
            kk[i] = p < ce ? a.cellbuf[p] : -1;
            v0[i] = p < ce ? a.values[p] : 0.f;
            if constexpr (R16) {
                v1[i] = p < ce ? a.values[(size_t)a.total + p] : 0.f;
                v2[i] = (p < ce && a.F > 2) ? a.values[(size_t)2 * a.total + p] : 0.f;
            }
        }
        uint32_t slot[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            if (kk[i] < 0) continue;
            const int t = kk[i] >> a.cpt_log2;
            slot[i] = base[t] + hist_add<PACK>(hist, t);
            const uint32_t cl = (uint32_t)(kk[i] & (a.cpt - 1));
            if constexpr (R16)
                a.rec4[slot[i]] = make_uint4(cl, __float_as_uint(v0[i]), __float_as_uint(v1[i]), __float_as_uint(v2[i]));
            else
                a.rec[slot[i]] = make_uint2(cl, __float_as_uint(v0[i]));
        }
        for (int f = 3; f < a.F; ++f) {
            const float* vf = a.values + (size_t)f * a.total;
            float v[NP];
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const int64_t p = p0 + (int64_t)i * kTBlock;
                v[i] = p < ce ? vf[p] : 0.f;
            }
            float* rvf = a.rv + (size_t)(f - 3) * a.total;
#pragma unroll
            for (int i = 0; i < NP; ++i)
                if (kk[i] >= 0) rvf[slot[i]] = v[i];
        }
    }
}

// Pass 3 for F <= 4 on grids of at most kStageMaxTiles tiles, staged in LDS
// (grid: blocks x snapshots, C particles per block).  A block's run of
// records in a tile is short (about 8 on the dense bed), so records written
// straight from the particles' registers reach each cache line one at a time
// and lines left partly written in L2 go to HBM piecewise (2.5 bytes written
// per record byte).  Here the block ranks its particles per tile with LDS
// atomics, prefix-sums the counts, places every record at its tile's
// block-local position in LDS, reserves one range per tile from the cursors,
// and then writes the staged records in order: consecutive lanes store
// consecutive records of a run.  The cell ids and values are read once.
// NV fields: the 8-byte record at NV = 1, the 16-byte record (fields 0..2)
// above, and at NV = 4 field 3's value in its own staged array.  C is as
// large as the LDS allows: 16384 at NV = 1, 8192 at 2 or 3, 4096 at 4.
constexpr int kStageMaxTiles = 2 * kTBlock;  // the prefix sum takes two tiles per thread
template <int NV>
struct StageRec { using T = uint4; };
template <>
struct StageRec<1> { using T = uint2; };
template <int C, int NV>
__global__ __launch_bounds__(kTBlock) void k_tile_scatter_staged(TileArgs a) {
    static_assert(C % kTBlock == 0 && NV >= 1 && NV <= 4, "whole passes, at most four fields");
    constexpr int P = C / kTBlock;  // particles per thread
    using Rec = typename StageRec<NV>::T;
    __shared__ Rec stage[C];                        // (cell, value bits), tile by tile
    __shared__ uint32_t stage3[NV == 4 ? C : 1];    // field 3's value bits, in the same order
    __shared__ uint32_t hist[kStageMaxTiles];       // the block's particles per tile
    __shared__ uint32_t loc[kStageMaxTiles];        // block-local start of each tile's run
    __shared__ uint32_t base[kStageMaxTiles];       // its start in the tile's global range
    __shared__ uint32_t wsum[kTBlock / 64];
    const int j = blockIdx.y;
    int64_t s0, s1;
    snap_range(a, j, s0, s1);
    const int64_t cb = s0 + (int64_t)blockIdx.x * C;
    if (cb >= s1) return;  // the whole block: beyond its snapshot's particles
    const int64_t ce = min(cb + (int64_t)C, s1);
    const int nt = a.ntiles;  // <= kStageMaxTiles (host)
    for (int t = threadIdx.x; t < nt; t += kTBlock) hist[t] = 0u;
    int32_t kk[P];
    uint32_t vv[NV][P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const int64_t p = cb + threadIdx.x + (int64_t)i * kTBlock;
        kk[i] = p < ce ? a.cellbuf[p] : -1;
#pragma unroll
        for (int f = 0; f < NV; ++f) vv[f][i] = p < ce ? __float_as_uint(a.values[(size_t)f * a.total + p]) : 0u;
    }
    __syncthreads();
    uint32_t rank[P];
#pragma unroll
    for (int i = 0; i < P; ++i) rank[i] = kk[i] >= 0 ? atomicAdd(&hist[kk[i] >> a.cpt_log2], 1u) : 0u;
    __syncthreads();
    // exclusive prefix sum of the counts: tiles 2 tid and 2 tid + 1 per thread,
    // a wave scan by shuffles, then the wave totals
    const int t0 = 2 * (int)threadIdx.x;
    const uint32_t h0 = t0 < nt ? hist[t0] : 0u, h1 = t0 + 1 < nt ? hist[t0 + 1] : 0u;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = h0 + h1;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    uint32_t* cursor = a.cursor + (size_t)j * nt;
    for (int t = threadIdx.x; t < nt; t += kTBlock) {
        const uint32_t c = hist[t];
        base[t] = c ? atomicAdd(&cursor[t], c) : 0u;
    }
    __syncthreads();
    uint32_t before = 0u, total = 0u;
    for (int w = 0; w < kTBlock / 64; ++w) {
        const uint32_t s = wsum[w];
        before += w < wave ? s : 0u;
        total += s;
    }
    const uint32_t ex = before + incl - (h0 + h1);
    if (t0 < nt) loc[t0] = ex;
    if (t0 + 1 < nt) loc[t0 + 1] = ex + h0;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < P; ++i) {
        if (kk[i] < 0) continue;
        const uint32_t k = loc[kk[i] >> a.cpt_log2] + rank[i];  // < total <= C
        if constexpr (NV == 1) {
            stage[k] = make_uint2((uint32_t)kk[i], vv[0][i]);
        } else {
            stage[k] = make_uint4((uint32_t)kk[i], vv[0][i], vv[1][i], NV > 2 ? vv[NV > 2 ? 2 : 0][i] : 0u);
            if constexpr (NV == 4) stage3[k] = vv[3][i];
        }
    }
    __syncthreads();
    const uint32_t mask = (uint32_t)a.cpt - 1u;
    for (uint32_t k = threadIdx.x; k < total; k += kTBlock) {
        const Rec e = stage[k];
        const uint32_t t = e.x >> a.cpt_log2;
        const uint32_t g = base[t] + (k - loc[t]);
        if constexpr (NV == 1) {
            a.rec[g] = make_uint2(e.x & mask, e.y);
        } else {
            a.rec4[g] = make_uint4(e.x & mask, e.y, e.z, e.w);
            if constexpr (NV == 4) a.rv[g] = __uint_as_float(stage3[k]);
        }
    }
}

__device__ inline long long quantise(float v, int S) {
    return isfinite(v) ? __double2ll_rn(ldexp((double)v, S)) : 0ll;
}

// Pass 4: one workgroup per tile (of all snapshots): exact int64 sums in LDS
// of the quantised values rint(v 2^S_f), then the tile's
// field = float32((acc 2^-S_f) / V) (and the accumulators when asked for).
// R16: the records hold the cell and fields 0..2.
template <bool R16>
__global__ __launch_bounds__(kTBlock) void k_tile_accum(TileArgs a) {
    __shared__ unsigned long long lacc[kTileWords];
    __shared__ int S[CGD_MAX_FIELDS];
    const int T = blockIdx.x;
    const int j = T / a.ntiles, t = T - j * a.ntiles;
    const int64_t c0 = (int64_t)t * a.cpt;
    const int nc = (int)min<int64_t>(a.cpt, a.cells - c0);
    for (int i = threadIdx.x; i < a.F * a.cpt; i += kTBlock) lacc[i] = 0ull;
    if (threadIdx.x < a.F) {
        int64_t s0, s1;
        snap_range(a, j, s0, s1);
        S[threadIdx.x] = frac_bits_used(a.maxbits[j * a.F + threadIdx.x], a.force_s ? a.force_s[threadIdx.x] : -1,
                                        e_n_dev(s1 - s0));
    }
    __syncthreads();
    const uint32_t r0 = a.offsets[T], r1 = a.offsets[T + 1];
    const int S0 = S[0];
    constexpr int U = 4;  // records per thread whose loads are in flight together
    for (uint32_t r = r0 + threadIdx.x; r < r1; r += U * kTBlock) {
        uint4 e[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t rr = r + u * kTBlock;
            if constexpr (R16) {
                e[u] = rr < r1 ? a.rec4[rr] : make_uint4(0u, 0u, 0u, 0u);
            } else {
                const uint2 e2 = rr < r1 ? a.rec[rr] : make_uint2(0u, 0u);
                e[u] = make_uint4(e2.x, e2.y, 0u, 0u);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long q = quantise(__uint_as_float(e[u].y), S0);
            if (q != 0) atomicAdd(&lacc[e[u].x], (unsigned long long)q);
            if constexpr (R16) {
                const long long q1 = quantise(__uint_as_float(e[u].z), S[1]);
                if (q1 != 0) atomicAdd(&lacc[a.cpt + e[u].x], (unsigned long long)q1);
                if (a.F > 2) {
                    const long long q2 = quantise(__uint_as_float(e[u].w), S[2]);
                    if (q2 != 0) atomicAdd(&lacc[2 * a.cpt + e[u].x], (unsigned long long)q2);
                }
            }
        }
        for (int f = 3; f < a.F; ++f) {
            float v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t rr = r + u * kTBlock;
                v[u] = rr < r1 ? a.rv[(size_t)(f - 3) * a.total + rr] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const long long q = quantise(v[u], S[f]);
                if (q != 0) atomicAdd(&lacc[f * a.cpt + e[u].x], (unsigned long long)q);
            }
        }
    }
    __syncthreads();
    for (int f = 0; f < a.F; ++f) {
        const size_t o = ((size_t)j * a.F + f) * a.cells + c0;
        for (int i = threadIdx.x; i < nc; i += kTBlock) {
            const long long v = (long long)lacc[f * a.cpt + i];
            a.field[o + i] = (float)(ldexp((double)v, -S[f]) / (a.vcell ? a.vcell[c0 + i] : a.vol));
            if (a.acc) a.acc[o + i] = v;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_locate_hex(const float* __restrict__ pos, int64_t n, HexBin g,
                                                       int32_t* __restrict__ cell) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        bool nf;
        const int64_t k = hex_cell(g, pos[3 * p], pos[3 * p + 1], pos[3 * p + 2], &nf);
        cell[p] = (int32_t)k;
    }
}

__global__ __launch_bounds__(kBlock) void k_finalize(const long long* __restrict__ acc,
                                                     float* __restrict__ field, int64_t cells,
                                                     double vol, int e_n, const DepositInfo* info) {
    const int f = blockIdx.y;
    const int S = frac_bits_used(info->maxbits[f], info->force_s[f], e_n);
    const long long* a = acc + (size_t)f * cells;
    float* out = field + (size_t)f * cells;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < cells; k += stride) {
        double d = ldexp((double)a[k], -S);
        out[k] = (float)(d / vol);
    }
}

}  // namespace

void deposit_prologue(int64_t n, int32_t F, const float* values, int64_t* acc, int64_t cells,
                      DepositInfo* info, const ScaleForce& fs, hipStream_t s) {
    hipLaunchKernelGGL(k_dep_init, dim3(1), dim3(64), 0, s, info, fs);
    const int64_t words = (int64_t)F * cells;
    int zblocks = (int)std::min<int64_t>(8192, std::max<int64_t>(1, (words + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_zero64, dim3(zblocks), dim3(kBlock), 0, s, reinterpret_cast<unsigned long long*>(acc),
                       words);
    if (n > 0) {
        int blocks = (int)std::min<int64_t>(4096, (n + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_absmax, dim3(blocks, F), dim3(kBlock), 0, s, values, n, info);
    }
}

int ceil_log2_count(int64_t n) {
    if (n <= 1) return 0;
    return 64 - __builtin_clzll((unsigned long long)(n - 1));
}

static HexBin hex_bin(const cgd_mesh m) {
    HexBin g;
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = m->hex.lo[a];
        g.hi[a] = m->hex.hi[a];
        g.s[a] = m->hex.s[a];
    }
    g.n[0] = m->hex.nx;
    g.n[1] = m->hex.ny;
    g.n[2] = m->hex.nz;
    return g;
}

cgd_status locate_hex(cgd_mesh m, int64_t n, const float* pos, int32_t* cell, hipStream_t s) {
    if (n > 0) {
        const int blocks = (int)std::min<int64_t>(16384, (n + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_locate_hex, dim3(blocks), dim3(kBlock), 0, s, pos, n, hex_bin(m), cell);
    }
    CGD_HIP_TRY(hipGetLastError());
    return CGD_OK;
}

// Tiling of the tiled deposit (tiles of a power-of-two number of cells, so
// that tile and cell-in-tile are a shift and a mask); false when the direct
// (atomic) path is used: more tiles per grid than the bucketing passes count
// in LDS, more particles than 32-bit offsets hold, or CGD_DEPOSIT_DIRECT set.
// Up to kMaxTiles tiles the counters are 32-bit words, up to
// kMaxTilesPacked 16-bit halves (the bucketing passes' PACK variant).
// CGD_DEPOSIT_CPT forces a smaller power-of-two tile (at least 16 cells), so
// that tests reach many tiles on small grids.
static bool tile_plan(int64_t cells, int64_t total, int32_t F, int* cpt, int* ntiles) {
    if (getenv("CGD_DEPOSIT_DIRECT") || total <= 0 || total >= (int64_t)UINT32_MAX) return false;
    int c = kTileWords;  // the largest power of two with F * c <= kTileWords
    while (c * F > kTileWords) c >>= 1;
    if (const char* e = getenv("CGD_DEPOSIT_CPT")) {
        const int w = atoi(e);
        if (w >= 16 && (w & (w - 1)) == 0 && w < c) c = w;
    }
    const int64_t t = (cells + c - 1) / c;
    if (t > kMaxTilesPacked) return false;
    *cpt = c;
    *ntiles = (int)t;
    return true;
}

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// Record bytes per particle (8 at F = 1, 16 above) and the fields kept in
// separate value arrays (3.. at F >= 4).
static size_t rec_bytes(int F) { return F == 1 ? 8 : 16; }
static size_t rv_fields(int F) { return F > 3 ? (size_t)(F - 3) : 0; }

size_t tiled_deposit_temp_bytes(int64_t cells, int64_t total, int32_t n_snap, int32_t F) {
    int cpt, nt;
    if (!tile_plan(cells, total, F, &cpt, &nt)) return 0;
    return al256(4 * (size_t)total) + al256(rec_bytes(F) * total) + al256(4 * rv_fields(F) * total) +
           al256(4 * (3 * (size_t)n_snap * nt + 1));
}

void deposit_info_init(DepositInfo* info, const ScaleForce& fs, hipStream_t s) {
    hipLaunchKernelGGL(k_dep_init, dim3(1), dim3(64), 0, s, info, fs);
}

size_t deposit_hex_temp_bytes(const cgd_mesh m, int64_t n, int32_t F) {
    return tiled_deposit_temp_bytes(m->cells, n, 1, F);
}

// kTChunk-particle chunks per block of a bucketing pass: one (longer chunks
// measured slower on the dense bed and on the batched launch); an
// environment override for tuning runs.
static int tile_nsub(const char* env) {
    if (const char* e = getenv(env)) return std::max(1, atoi(e));
    return 1;
}

cgd_status tiled_deposit(cgd_mesh m, const TiledDeposit& d, Timing* timing, hipStream_t s) {
    int cpt = 0, nt = 0;
    if (!d.temp || !tile_plan(m->cells, d.total, d.F, &cpt, &nt)) {
        set_error("tiled deposit: no tiling for this grid and particle count");
        return CGD_E_INVALID;
    }
    char* t = static_cast<char*>(d.temp);
    TileArgs a = {};
    a.pos = d.pos;
    a.values = d.values;
    a.total = d.total;
    a.off = d.off;
    a.n_snap = d.n_snap;
    a.F = d.F;
    a.g = hex_bin(m);
    a.cells = m->cells;
    a.cpt = cpt;
    a.cpt_log2 = __builtin_ctz((unsigned)cpt);
    a.ntiles = nt;
    a.nsub = tile_nsub("CGD_DEPOSIT_NSUB");
    a.nsub_bin = tile_nsub("CGD_DEPOSIT_BIN_NSUB");
    const bool pack = nt > kMaxTiles;
    if (pack) {  // 16-bit counters: fewer than 2^16 particles per block
        a.nsub = std::min(a.nsub, kPackMaxChunks);
        a.nsub_bin = std::min(a.nsub_bin, kPackMaxChunks);
    }
    a.cellbuf = reinterpret_cast<int32_t*>(t);
    t += al256(4 * (size_t)d.total);
    a.rec = reinterpret_cast<uint2*>(t);
    a.rec4 = reinterpret_cast<uint4*>(t);
    t += al256(rec_bytes(d.F) * d.total);
    a.rv = reinterpret_cast<float*>(t);
    t += al256(4 * rv_fields(d.F) * d.total);
    const int all = d.n_snap * nt;
    a.counts = reinterpret_cast<uint32_t*>(t);
    a.offsets = a.counts + all;
    a.cursor = a.offsets + all + 1;
    a.maxbits = d.maxbits;
    a.force_s = d.force_s;
    a.nf_val = d.nf_val;
    a.nf_val_stride = d.nf_val_stride;
    a.cnt_jstride = d.cnt_jstride;
    a.dropped = d.dropped;
    a.nf_pos = d.nf_pos;
    a.field = d.field;
    a.acc = d.acc;
    a.vol = m->hex.vol;
    a.rect = d.rect;
    a.rl = d.rl;
    a.vcell = d.vcell;
    hipLaunchKernelGGL(k_tile_clear, dim3((all + 255) / 256), dim3(256), 0, s, a);
    const int64_t bchunk = (int64_t)a.nsub_bin * kTChunk, schunk = (int64_t)a.nsub * kTChunk;
    const int cblocks = (int)std::max<int64_t>(1, (d.max_n + bchunk - 1) / bchunk);
    const int sblocks = (int)std::max<int64_t>(1, (d.max_n + schunk - 1) / schunk);
    // Timed as a whole (kind 2: 12 bytes of position and 12 per field and
    // particle, the direct path's count) and per stage (kinds 13..15, each
    // with the bytes it must move: binning reads positions and values and
    // writes the host cell; the scatter reads cell and values and writes the
    // records and the values of fields 3..; the accumulation reads them and
    // writes the field, 4 bytes per cell and field).
    const double np_ = (double)d.total;
    int tm = timing ? timing_begin(timing, s) : -1;
    int t13 = timing ? timing_begin(timing, s) : -1;
    if (d.rect) {
        if (pack) hipLaunchKernelGGL((k_tile_bin<true, true>), dim3(cblocks, d.n_snap), dim3(kTBlock), 0, s, a);
        else hipLaunchKernelGGL((k_tile_bin<true, false>), dim3(cblocks, d.n_snap), dim3(kTBlock), 0, s, a);
    } else {
        if (pack) hipLaunchKernelGGL((k_tile_bin<false, true>), dim3(cblocks, d.n_snap), dim3(kTBlock), 0, s, a);
        else hipLaunchKernelGGL((k_tile_bin<false, false>), dim3(cblocks, d.n_snap), dim3(kTBlock), 0, s, a);
    }
    if (timing) timing_end(timing, t13, 13, (12.0 + 4.0 * d.F + 4.0) * np_, s);
    int t14 = timing ? timing_begin(timing, s) : -1;
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(kTBlock), 0, s, a);
    if (nt <= kStageMaxTiles && d.F <= 4 && a.nsub == 1) {
        // staged in LDS: C = 16384 / 8192 / 4096 particles per block at F = 1 / 2..3 / 4
        const int c = d.F == 1 ? kTChunk : (d.F <= 3 ? kTChunk / 2 : kTChunk / 4);
        const dim3 g((unsigned)std::max<int64_t>(1, (d.max_n + c - 1) / c), d.n_snap);
        if (d.F == 1) hipLaunchKernelGGL((k_tile_scatter_staged<kTChunk, 1>), g, dim3(kTBlock), 0, s, a);
        else if (d.F == 2) hipLaunchKernelGGL((k_tile_scatter_staged<kTChunk / 2, 2>), g, dim3(kTBlock), 0, s, a);
        else if (d.F == 3) hipLaunchKernelGGL((k_tile_scatter_staged<kTChunk / 2, 3>), g, dim3(kTBlock), 0, s, a);
        else hipLaunchKernelGGL((k_tile_scatter_staged<kTChunk / 4, 4>), g, dim3(kTBlock), 0, s, a);
    } else if (d.F >= 2) {
        if (pack) hipLaunchKernelGGL((k_tile_scatter<true, true>), dim3(sblocks, d.n_snap), dim3(kTBlock), 0, s, a);
        else hipLaunchKernelGGL((k_tile_scatter<true, false>), dim3(sblocks, d.n_snap), dim3(kTBlock), 0, s, a);
    } else {
        if (pack) hipLaunchKernelGGL((k_tile_scatter<false, true>), dim3(sblocks, d.n_snap), dim3(kTBlock), 0, s, a);
        else hipLaunchKernelGGL((k_tile_scatter<false, false>), dim3(sblocks, d.n_snap), dim3(kTBlock), 0, s, a);
    }
    const double recb = (double)rec_bytes(d.F) + 4.0 * (double)rv_fields(d.F);  // bytes written per particle
    if (timing) timing_end(timing, t14, 14, (4.0 + 4.0 * d.F + recb) * np_, s);
    int t15 = timing ? timing_begin(timing, s) : -1;
    if (d.F >= 2) hipLaunchKernelGGL(k_tile_accum<true>, dim3(all), dim3(kTBlock), 0, s, a);
    else hipLaunchKernelGGL(k_tile_accum<false>, dim3(all), dim3(kTBlock), 0, s, a);
    if (timing)
        timing_end(timing, t15, 15,
                   recb * np_ + (4.0 * d.F + (d.vcell ? 8.0 : 0.0)) * (double)m->cells * d.n_snap,
                   s);
    if (timing) timing_end(timing, tm, 2, (12.0 + 12.0 * d.F) * np_, s);
    CGD_HIP_TRY(hipGetLastError());
    return CGD_OK;
}

cgd_status deposit_hex(cgd_mesh m, int64_t n, const float* pos, int32_t F, const float* values,
                       float* field, int64_t* acc, DepositInfo* info, void* temp, const ScaleForce& fs,
                       Timing* timing, hipStream_t s) {
    const int64_t cells = m->cells;
    const int e_n = ceil_log2_count(n);
    const HexBin g = hex_bin(m);
    if (temp && deposit_hex_temp_bytes(m, n, F) > 0) {
        TiledDeposit d = {};
        d.pos = pos;
        d.values = values;
        d.total = n;
        d.max_n = n;
        d.off = nullptr;
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
        deposit_info_init(info, fs, s);
        return tiled_deposit(m, d, timing, s);
    }
    deposit_prologue(n, F, values, acc, cells, info, fs, s);
    if (n > 0) {
        int dblocks = (int)std::min<int64_t>(16384, (n + kBlock - 1) / kBlock);
        int t = timing ? timing_begin(timing, s) : -1;
        hipLaunchKernelGGL(k_deposit_hex, dim3(dblocks), dim3(kBlock), 0, s, pos, values, n, F, g,
                           e_n, reinterpret_cast<unsigned long long*>(acc), cells, info);
        if (timing) timing_end(timing, t, 2, (12.0 + 12.0 * F) * (double)n, s);
    }
    {
        int blocks = (int)std::min<int64_t>(8192, (cells + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_finalize, dim3(blocks, F), dim3(kBlock), 0, s,
                           reinterpret_cast<const long long*>(acc), field, cells, m->hex.vol, e_n,
                           info);
    }
    CGD_HIP_TRY(hipGetLastError());
    return CGD_OK;
}

}  // namespace cgd
