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

__global__ void k_dep_init(DepositInfo* info) {
    int t = threadIdx.x;
    if (t < CGD_MAX_FIELDS) {
        info->maxbits[t] = 0u;
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
        if (mm) atomicMax(&info->maxbits[f], mm);
        if (bb) atomicAdd(&info->nonfinite_val[f], bb);
    }
}

__global__ __launch_bounds__(kBlock) void k_deposit_hex(
    const float* __restrict__ pos, const float* __restrict__ values, int64_t n, int F, HexBin g,
    int e_n, unsigned long long* __restrict__ acc, int64_t cells, DepositInfo* info) {
    __shared__ int S[CGD_MAX_FIELDS];
    if (threadIdx.x < F) S[threadIdx.x] = frac_bits_of(info->maxbits[threadIdx.x], e_n);
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
// The cells are cut into tiles of `cpt` consecutive indices.  The particles
// are bucketed by tile (a counting sort over fixed chunks of particles per
// block), then one workgroup per tile adds its particles' fixed-point values
// in LDS and writes the tile's finished field (and accumulators): every int64
// sum stays exact, and the device-wide atomics on the accumulators of the
// direct path are replaced by LDS atomics.  A bucketed record is 8 bytes,
// (cell within the tile, bits of the first field's value); further fields'
// values follow in their own arrays, and the values are quantised in the
// accumulate pass.

constexpr int kTBlock = 1024;
constexpr int kTPer = 16;                  // particles per thread and pass, held in registers
constexpr int kTChunk = kTBlock * 16;      // particles per block and chunk of the bucketing passes
constexpr int kTPass = kTChunk / (kTBlock * kTPer);  // register passes per chunk
constexpr int kBPer = 4;                   // particles per thread and register pass of the counting pass
constexpr int kTileWords = 16384;          // int64 LDS accumulators of one tile workgroup (128 KB)
constexpr int kMaxTiles = 8192;            // LDS tile counters of the bucketing passes

struct TileArgs {
    const float* pos;
    const float* values;
    int64_t n;
    int F;
    HexBin g;
    int e_n;
    int64_t cells;
    int cpt, ntiles;
    int cpt_log2;       // cpt = 2^cpt_log2
    int nsub;           // kTChunk-particle passes per block of the scatter
    int nsub_bin;       // ... and of the counting pass
    int32_t* cellbuf;   // [n]: host cell of each particle (-1: dropped)
    uint32_t* counts;   // [ntiles]: particles per tile
    uint32_t* offsets;  // [ntiles + 1]
    uint32_t* cursor;   // [ntiles]
    uint2* rec;         // [n]: (cell within its tile, bits of field 0's value), tile-bucketed
    float* rv;          // [F - 1][n]: values of fields 1.., tile-bucketed
    float* field;
    long long* acc;     // nullable
    double vol;
    DepositInfo* info;
};

__global__ void k_tile_clear(TileArgs a) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < a.ntiles; t += gridDim.x * blockDim.x) a.counts[t] = 0u;
}

// Pass 1: host cells (stored), dropped counts, particles per tile, and the
// max |v| / non-finite count of every field over the block's chunk of
// nsub_bin * kTChunk particles (the values of the direct path's k_absmax,
// folded into this pass).
__global__ __launch_bounds__(kTBlock) void k_tile_bin(TileArgs a) {
    __shared__ uint32_t hist[kMaxTiles];
    __shared__ uint32_t bmax[CGD_MAX_FIELDS];
    __shared__ unsigned long long bbad[CGD_MAX_FIELDS];
    for (int t = threadIdx.x; t < a.ntiles; t += kTBlock) hist[t] = 0u;
    if (threadIdx.x < CGD_MAX_FIELDS) {
        bmax[threadIdx.x] = 0u;
        bbad[threadIdx.x] = 0ull;
    }
    __syncthreads();
    unsigned long long dropped = 0ull, nfpos = 0ull;
    const int npass = a.nsub_bin * (kTChunk / (kTBlock * kBPer));
    for (int sub = 0; sub < npass; ++sub) {
        const int64_t p0 = ((int64_t)blockIdx.x * npass + sub) * (kTBlock * kBPer) + threadIdx.x;
        float px[kBPer], py[kBPer], pz[kBPer];
#pragma unroll
        for (int i = 0; i < kBPer; ++i) {
            const int64_t p = min(p0 + (int64_t)i * kTBlock, a.n - 1);
            px[i] = a.pos[3 * p];
            py[i] = a.pos[3 * p + 1];
            pz[i] = a.pos[3 * p + 2];
        }
#pragma unroll
        for (int i = 0; i < kBPer; ++i) {
            const int64_t p = p0 + (int64_t)i * kTBlock;
            if (p >= a.n) continue;
            bool nf;
            const int32_t k = (int32_t)hex_cell(a.g, px[i], py[i], pz[i], &nf);
            a.cellbuf[p] = k;
            if (k < 0) {
                ++dropped;
                nfpos += nf ? 1ull : 0ull;
            } else {
                atomicAdd(&hist[k >> a.cpt_log2], 1u);
            }
        }
    }
    for (int f = 0; f < a.F; ++f) {
        const uint32_t* v = reinterpret_cast<const uint32_t*>(a.values + (size_t)f * a.n);
        uint32_t m = 0u;
        unsigned long long bad = 0ull;
        for (int sub = 0; sub < npass; ++sub) {
            const int64_t p0 = ((int64_t)blockIdx.x * npass + sub) * (kTBlock * kBPer) + threadIdx.x;
            uint32_t x[kBPer];
#pragma unroll
            for (int i = 0; i < kBPer; ++i) {
                const int64_t p = p0 + (int64_t)i * kTBlock;
                x[i] = p < a.n ? v[p] & 0x7fffffffu : 0u;
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
        atomicAdd(&a.info->dropped, dropped);
        if (nfpos) atomicAdd(&a.info->nonfinite_pos, nfpos);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < a.ntiles; t += kTBlock)
        if (hist[t]) atomicAdd(&a.counts[t], hist[t]);
    if (threadIdx.x < a.F) {
        if (bmax[threadIdx.x]) atomicMax(&a.info->maxbits[threadIdx.x], bmax[threadIdx.x]);
        if (bbad[threadIdx.x]) atomicAdd(&a.info->nonfinite_val[threadIdx.x], bbad[threadIdx.x]);
    }
}

// Pass 2: offsets = exclusive prefix sum of the counts (one block).
__global__ __launch_bounds__(kTBlock) void k_tile_scan(TileArgs a) {
    __shared__ uint32_t part[kTBlock];
    const int per = (a.ntiles + kTBlock - 1) / kTBlock;
    const int t0 = threadIdx.x * per, t1 = min(t0 + per, a.ntiles);
    uint32_t s = 0u;
    for (int t = t0; t < t1; ++t) s += a.counts[t];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0u;
        for (int i = 0; i < kTBlock; ++i) {
            const uint32_t v = part[i];
            part[i] = run;
            run += v;
        }
        a.offsets[a.ntiles] = run;
    }
    __syncthreads();
    uint32_t run = part[threadIdx.x];
    for (int t = t0; t < t1; ++t) {
        a.offsets[t] = run;
        a.cursor[t] = run;
        run += a.counts[t];
    }
}

// Pass 3: each block counts its chunk of nsub * kTChunk particles per tile,
// reserves one range per tile, then writes the particles' records there, a
// register pass of kTPer particles per thread at a time.
// Longer chunks give longer runs of consecutive slots per block and tile,
// which the L2 merges into whole lines before they are written back.
__global__ __launch_bounds__(kTBlock) void k_tile_scatter(TileArgs a) {
    __shared__ uint32_t hist[kMaxTiles];
    __shared__ uint32_t base[kMaxTiles];
    const int64_t c0 = (int64_t)blockIdx.x * a.nsub * kTChunk + threadIdx.x;
    for (int t = threadIdx.x; t < a.ntiles; t += kTBlock) hist[t] = 0u;
    __syncthreads();
    const int npass = a.nsub * kTPass;
    for (int sub = 0; sub < npass; ++sub) {
        const int64_t p0 = c0 + (int64_t)sub * (kTBlock * kTPer);
        int32_t kk[kTPer];
#pragma unroll
        for (int i = 0; i < kTPer; ++i) {
            const int64_t p = p0 + (int64_t)i * kTBlock;
            kk[i] = p < a.n ? a.cellbuf[p] : -1;
        }
#pragma unroll
        for (int i = 0; i < kTPer; ++i)
            if (kk[i] >= 0) atomicAdd(&hist[kk[i] >> a.cpt_log2], 1u);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < a.ntiles; t += kTBlock) {
        const uint32_t c = hist[t];
        base[t] = c ? atomicAdd(&a.cursor[t], c) : 0u;
        hist[t] = 0u;  // reused as the in-block rank counter
    }
    __syncthreads();
    for (int sub = 0; sub < npass; ++sub) {
        const int64_t p0 = c0 + (int64_t)sub * (kTBlock * kTPer);
        int32_t kk[kTPer];
        float v0[kTPer];
#pragma unroll
        for (int i = 0; i < kTPer; ++i) {
            const int64_t p = p0 + (int64_t)i * kTBlock;
            kk[i] = p < a.n ? a.cellbuf[p] : -1;
            v0[i] = p < a.n ? a.values[p] : 0.f;
        }
        uint32_t slot[kTPer];
#pragma unroll
        for (int i = 0; i < kTPer; ++i) {
            if (kk[i] < 0) continue;
            const int t = kk[i] >> a.cpt_log2;
            slot[i] = base[t] + atomicAdd(&hist[t], 1u);
            a.rec[slot[i]] = make_uint2((uint32_t)(kk[i] & (a.cpt - 1)), __float_as_uint(v0[i]));
        }
        for (int f = 1; f < a.F; ++f) {
            const float* vf = a.values + (size_t)f * a.n;
            float v[kTPer];
#pragma unroll
            for (int i = 0; i < kTPer; ++i) {
                const int64_t p = p0 + (int64_t)i * kTBlock;
                v[i] = p < a.n ? vf[p] : 0.f;
            }
            float* rvf = a.rv + (size_t)(f - 1) * a.n;
#pragma unroll
            for (int i = 0; i < kTPer; ++i)
                if (kk[i] >= 0) rvf[slot[i]] = v[i];
        }
    }
}

__device__ inline long long quantise(float v, int S) {
    return isfinite(v) ? __double2ll_rn(ldexp((double)v, S)) : 0ll;
}

// Pass 4: one workgroup per tile: exact int64 sums in LDS of the quantised
// values rint(v 2^S_f), then the tile's field = float32((acc 2^-S_f) / V)
// (and the accumulators when asked for).
__global__ __launch_bounds__(kTBlock) void k_tile_accum(TileArgs a) {
    __shared__ unsigned long long lacc[kTileWords];
    __shared__ int S[CGD_MAX_FIELDS];
    const int t = blockIdx.x;
    const int64_t c0 = (int64_t)t * a.cpt;
    const int nc = (int)min<int64_t>(a.cpt, a.cells - c0);
    for (int i = threadIdx.x; i < a.F * a.cpt; i += kTBlock) lacc[i] = 0ull;
    if (threadIdx.x < a.F) S[threadIdx.x] = frac_bits_of(a.info->maxbits[threadIdx.x], a.e_n);
    __syncthreads();
    const uint32_t r0 = a.offsets[t], r1 = a.offsets[t + 1];
    const int S0 = S[0];
    constexpr int U = 4;  // records per thread whose loads are in flight together
    for (uint32_t r = r0 + threadIdx.x; r < r1; r += U * kTBlock) {
        uint2 e[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint32_t rr = r + j * kTBlock;
            e[j] = rr < r1 ? a.rec[rr] : make_uint2(0u, 0u);
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const long long q = quantise(__uint_as_float(e[j].y), S0);
            if (q != 0) atomicAdd(&lacc[e[j].x], (unsigned long long)q);
        }
        for (int f = 1; f < a.F; ++f) {
            float v[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const uint32_t rr = r + j * kTBlock;
                v[j] = rr < r1 ? a.rv[(size_t)(f - 1) * a.n + rr] : 0.f;
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const long long q = quantise(v[j], S[f]);
                if (q != 0) atomicAdd(&lacc[f * a.cpt + e[j].x], (unsigned long long)q);
            }
        }
    }
    __syncthreads();
    for (int f = 0; f < a.F; ++f) {
        float* out = a.field + (size_t)f * a.cells + c0;
        for (int i = threadIdx.x; i < nc; i += kTBlock) {
            const long long v = (long long)lacc[f * a.cpt + i];
            out[i] = (float)(ldexp((double)v, -S[f]) / a.vol);
            if (a.acc) a.acc[(size_t)f * a.cells + c0 + i] = v;
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
    const int S = frac_bits_of(info->maxbits[f], e_n);
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
                      DepositInfo* info, hipStream_t s) {
    hipLaunchKernelGGL(k_dep_init, dim3(1), dim3(64), 0, s, info);
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
// (atomic) path is used:
// more tiles than the bucketing passes count in LDS, more particles than
// 32-bit offsets hold, or CGD_DEPOSIT_DIRECT set.
bool tile_plan(int64_t cells, int64_t n, int32_t F, int* cpt, int* ntiles) {
    if (getenv("CGD_DEPOSIT_DIRECT") || n <= 0 || n >= (int64_t)UINT32_MAX) return false;
    int c = kTileWords;  // the largest power of two with F * c <= kTileWords
    while (c * F > kTileWords) c >>= 1;
    const int64_t t = (cells + c - 1) / c;
    if (t > kMaxTiles) return false;
    *cpt = c;
    *ntiles = (int)t;
    return true;
}

size_t deposit_hex_temp_bytes(const cgd_mesh m, int64_t n, int32_t F) {
    int cpt, nt;
    if (!tile_plan(m->cells, n, F, &cpt, &nt)) return 0;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return al(4 * (size_t)n) + al(8 * (size_t)n) + al(4 * (size_t)(F - 1) * n) + al(4 * (3 * (size_t)nt + 1));
}

// kTChunk-particle passes per scatter block: as long as the grid still
// gives every compute unit several blocks.
static int scatter_nsub(const char* env, int64_t n) {
    if (const char* e = getenv(env)) return std::max(1, atoi(e));
    int nsub = 1;
    while (nsub < 8 && (n + 2 * nsub * (int64_t)kTChunk - 1) / (2 * nsub * (int64_t)kTChunk) >= 1024) nsub *= 2;
    return nsub;
}

cgd_status deposit_hex(cgd_mesh m, int64_t n, const float* pos, int32_t F, const float* values,
                       float* field, int64_t* acc, DepositInfo* info, void* temp, hipStream_t s) {
    const int64_t cells = m->cells;
    const int e_n = ceil_log2_count(n);
    const HexBin g = hex_bin(m);
    int cpt = 0, nt = 0;
    if (temp && tile_plan(cells, n, F, &cpt, &nt)) {
        auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
        char* t = static_cast<char*>(temp);
        TileArgs a = {};
        a.pos = pos;
        a.values = values;
        a.n = n;
        a.F = F;
        a.g = g;
        a.e_n = e_n;
        a.cells = cells;
        a.cpt = cpt;
        a.cpt_log2 = __builtin_ctz((unsigned)cpt);
        a.ntiles = nt;
        a.nsub = scatter_nsub("CGD_DEPOSIT_NSUB", n);
        a.nsub_bin = scatter_nsub("CGD_DEPOSIT_BIN_NSUB", n);
        a.cellbuf = reinterpret_cast<int32_t*>(t);
        t += al(4 * (size_t)n);
        a.rec = reinterpret_cast<uint2*>(t);
        t += al(8 * (size_t)n);
        a.rv = reinterpret_cast<float*>(t);
        t += al(4 * (size_t)(F - 1) * n);
        a.counts = reinterpret_cast<uint32_t*>(t);
        a.offsets = a.counts + nt;
        a.cursor = a.offsets + nt + 1;
        a.field = field;
        a.acc = reinterpret_cast<long long*>(acc);
        a.vol = m->hex.vol;
        a.info = info;
        hipLaunchKernelGGL(k_dep_init, dim3(1), dim3(64), 0, s, info);
        hipLaunchKernelGGL(k_tile_clear, dim3((nt + 255) / 256), dim3(256), 0, s, a);
        const int cblocks = (int)((n + (int64_t)a.nsub_bin * kTChunk - 1) / ((int64_t)a.nsub_bin * kTChunk));
        int tm = timing_begin(&m->timing, s);
        hipLaunchKernelGGL(k_tile_bin, dim3(cblocks), dim3(kTBlock), 0, s, a);
        hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(kTBlock), 0, s, a);
        const int sblocks = (int)((n + (int64_t)a.nsub * kTChunk - 1) / ((int64_t)a.nsub * kTChunk));
        hipLaunchKernelGGL(k_tile_scatter, dim3(sblocks), dim3(kTBlock), 0, s, a);
        hipLaunchKernelGGL(k_tile_accum, dim3(nt), dim3(kTBlock), 0, s, a);
        timing_end(&m->timing, tm, 2, (12.0 + 12.0 * F) * (double)n, s);
        CGD_HIP_TRY(hipGetLastError());
        return CGD_OK;
    }
    deposit_prologue(n, F, values, acc, cells, info, s);
    if (n > 0) {
        int dblocks = (int)std::min<int64_t>(16384, (n + kBlock - 1) / kBlock);
        int t = timing_begin(&m->timing, s);
        hipLaunchKernelGGL(k_deposit_hex, dim3(dblocks), dim3(kBlock), 0, s, pos, values, n, F, g,
                           e_n, reinterpret_cast<unsigned long long*>(acc), cells, info);
        timing_end(&m->timing, t, 2, (12.0 + 12.0 * F) * (double)n, s);
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
