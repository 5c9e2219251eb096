// Particle centroid method on uniform hex grids (Section 2.2, eq. pcm-k),
// bit-exact through 64-bit fixed point.
//
// Pipeline (all on the caller's stream, no host synchronisation):
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

cgd_status deposit_hex(cgd_mesh m, int64_t n, const float* pos, int32_t F, const float* values,
                       float* field, int64_t* acc, DepositInfo* info, hipStream_t s) {
    const int64_t cells = m->cells;
    const int e_n = ceil_log2_count(n);
    const HexBin g = hex_bin(m);
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
