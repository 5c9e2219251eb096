// Learned initial guess for the backward-Euler solves: a three-level 3-D
// convolutional U-Net that maps the field of one pseudo-step, e^n, to an
// estimate of the next, e^{n+1}.  The network is an addition to the method
// (the paper diffuses from the previous field only); the CG solve it seeds
// is unchanged, so the result is the same discrete solution whatever the
// guess (Section 3.2 defines the system, Section 5.1 the discretisation).
//
// Network (base width C = 16, zero padding, ReLU after every 3x3x3 conv):
//   level 0: e1a 1->16, e1b 16->16                      (nx, ny, nz)
//   level 1: avg-pool 2, e2a 16->32, e2b 32->32          (n / 2)
//   level 2: avg-pool 2, e3a 32->64, e3b 64->64          (n / 4)
//   level 1: nearest-up 2 + u2 64->32, concat e2, d2a 64->32, d2b 32->32
//   level 0: nearest-up 2 + u1 32->16, concat e1, d1a 32->16, d1b 16->16
//   head: y = x + s * (hw . d1 + hb), inputs scaled by 1/s, s = rms(x).
//
// Arithmetic: activations and weights in bfloat16, products on the matrix
// cores (v_mfma_f32_16x16x32_bf16) with float32 accumulation; head, loss,
// gradients of the weights, Adam moments and master weights in float32; the
// normalisation and the loss in float64 sums.  Every reduction runs in one
// fixed order, so a training step is deterministic.
//
// Layout: activations channels-last [z][y][x][c] (x fastest among the
// voxels, as the cell fields), weights canonical [co][tap][ci] with
// tap = (dz+1)*9 + (dy+1)*3 + (dx+1).
//
// Convolution (forward and input-gradient): implicit GEMM per brick of
// 16 x 4 x 4 output voxels and 256 threads.  The input brick with its
// one-voxel halo (18 x 6 x 6) is staged in LDS, 16 or 32 channels per pass;
// nearest upsampling and channel concatenation are applied while staging,
// so neither is ever materialised.  Each wave owns 4 rows of 16 voxels; an
// MFMA multiplies 16 output channels (rows, weights from L1/L2) by 16 voxels
// (columns, from LDS) over 32 reduction values (one tap x 32 channels, or
// two taps x 16 channels).  The epilogue adds the bias and applies ReLU
// (forward) or the ReLU mask of the layer below (input gradient), and stores
// four bfloat16 channels per lane.  The input gradient of a layer is the
// same convolution with the taps mirrored and the channel roles swapped.
//
// Weight gradient: per brick of 16 x 4 x 2 voxels, the gradient at the
// output (LDS, [voxel][co]) times the staged input (LDS, with halo), with
// voxels as the reduction dimension; each block walks several bricks and
// writes its partial sums, which a second kernel adds in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "cgd_internal.h"

namespace cgd {
namespace unet {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBase = 16;   // channels at level 0
constexpr int kLayers = 12;
constexpr int kThreads = 256;

// forward / input-gradient brick
constexpr int BX = 16, BY = 4, BZ = 4;
constexpr int HX = BX + 2, HY = BY + 2;
constexpr int kRowsPerWave = BY * BZ / 4;
// weight-gradient brick
constexpr int WBZ = 2;
constexpr int WV = BX * BY * WBZ;  // 128 voxels = 4 reduction chunks of 32
constexpr int kTilesPerWave = 8;
constexpr int kTilesPerGroup = 4 * kTilesPerWave;

__device__ inline int tap_dz(int t) { return t / 9 - 1; }
__device__ inline int tap_dy(int t) { return (t / 3) % 3 - 1; }
__device__ inline int tap_dx(int t) { return t % 3 - 1; }

__device__ inline bool bf16_pos(uint16_t b) { return !(b & 0x8000u) && b != 0; }

__device__ inline uint16_t bf16_bits(float f) {
    bf16 h = (bf16)f;
    return __builtin_bit_cast(uint16_t, h);
}
__device__ inline float bf16_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Input of a convolution: channels [0, ca) from tensor a (optionally read
// through nearest 2x upsampling, i.e. from a grid of half the size), then
// channels [ca, ca + cb) from tensor b.  lda / ldb: elements per voxel.
struct Src {
    const bf16* a;
    int ca, lda, upa;
    const bf16* b;
    int cb, ldb;
};

// 8 channels c..c+7 (c a multiple of 8) of voxel (x, y, z) of the virtual input.
__device__ inline uint4 load_src8(const Src& s, int c, int x, int y, int z, int nx, int ny) {
    if (c < s.ca) {
        if (s.upa) {
            x >>= 1;
            y >>= 1;
            z >>= 1;
            nx >>= 1;
            ny >>= 1;
        }
        const size_t v = ((size_t)z * ny + y) * nx + x;
        return *reinterpret_cast<const uint4*>(s.a + v * s.lda + c);
    }
    const size_t v = ((size_t)z * ny + y) * nx + x;
    return *reinterpret_cast<const uint4*>(s.b + v * s.ldb + (c - s.ca));
}

// Stages channels [pass*CC, pass*CC + CC) of the (BX+2) x (BY+2) x HZ halo
// brick whose first interior voxel is (x0, y0, z0); voxels outside the grid
// read as zero (the zero padding).  Record stride CC + 8 elements.
template <int CC, int HZ>
__device__ inline void stage_halo(uint4* lds, const Src& s, int pass, int x0, int y0, int z0, int nx, int ny,
                                  int nz) {
    constexpr int G8 = CC / 8, RSU = G8 + 1, HV = HX * HY * HZ;
    for (int i = threadIdx.x; i < HV * G8; i += kThreads) {
        const int hv = i / G8, j = i - hv * G8;
        const int hx = hv % HX, t = hv / HX, hy = t % HY, hz = t / HY;
        const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if ((unsigned)gx < (unsigned)nx && (unsigned)gy < (unsigned)ny && (unsigned)gz < (unsigned)nz)
            v = load_src8(s, pass * CC + 8 * j, gx, gy, gz, nx, ny);
        lds[hv * RSU + j] = v;
    }
}

// Single-channel input (the first layer): one bfloat16 per halo voxel.
template <int HZ>
__device__ inline void stage_halo1(uint16_t* lds, const Src& s, int x0, int y0, int z0, int nx, int ny, int nz) {
    constexpr int HV = HX * HY * HZ;
    const uint16_t* a = reinterpret_cast<const uint16_t*>(s.a);
    for (int hv = threadIdx.x; hv < HV; hv += kThreads) {
        const int hx = hv % HX, t = hv / HX, hy = t % HY, hz = t / HY;
        const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
        uint16_t v = 0;
        if ((unsigned)gx < (unsigned)nx && (unsigned)gy < (unsigned)ny && (unsigned)gz < (unsigned)nz)
            v = a[(((size_t)gz * ny + gy) * nx + gx) * s.lda];
        lds[hv] = v;
    }
}

// Kernel-layout geometry of a weight tensor for a given channels-per-pass CC:
// [co][pass][KT][CC]; taps past 26 are zero padding.
__host__ __device__ constexpr int kt_of(int cc) { return cc == 1 ? 32 : (cc == 16 ? 28 : 27); }

struct ConvArgs {
    Src src;
    const bf16* w;       // [CO][NP][KT][CC]
    const float* bias;   // [CO] or null
    bf16* out;           // [voxel][ldo], channels [0, CO)
    int ldo;
    const bf16* mask_a;  // input gradient: ReLU mask of channels [0, mca) (ld ldma) ...
    int mca, ldma;
    const bf16* mask_b;  // ... and of channels [mca, CO) (ld ldmb)
    int ldmb;
    int relu;
    int nx, ny, nz, bnx, bny;
};

// One 3x3x3 convolution (see the file comment).  CC: input channels per LDS
// pass (1, 16 or 32); CO: output channels; NP: passes (CI = NP * CC).
template <int CC, int CO, int NP>
__global__ __launch_bounds__(kThreads) void k_conv(ConvArgs a) {
    constexpr int NT = CO / 16;
    constexpr int KT = kt_of(CC);
    constexpr int NCH = CC == 1 ? 1 : (CC == 16 ? 14 : 27);
    constexpr int RSU = CC == 1 ? 1 : CC / 8 + 1;
    constexpr int HV = HX * HY * (BZ + 2);
    constexpr int LDS_U4 = CC == 1 ? (HV * 2 + 15) / 16 : HV * RSU;
    __shared__ uint4 lds[LDS_U4];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, xl = lane & 15;
    int b = blockIdx.x;
    const int bx = b % a.bnx;
    b /= a.bnx;
    const int by = b % a.bny, bz = b / a.bny;
    const int x0 = bx * BX, y0 = by * BY, z0 = bz * BZ;

    f32x4 acc[kRowsPerWave][NT];
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[r][t] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int p = 0; p < NP; ++p) {
        if (p) __syncthreads();
        if constexpr (CC == 1)
            stage_halo1<BZ + 2>(reinterpret_cast<uint16_t*>(lds), a.src, x0, y0, z0, a.nx, a.ny, a.nz);
        else
            stage_halo<CC, BZ + 2>(lds, a.src, p, x0, y0, z0, a.nx, a.ny, a.nz);
        __syncthreads();

        if constexpr (CC == 1) {
            // K = 32 taps (27 real): lane group g holds taps 8g .. 8g+7
            bf16x8 af[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t)
                af[t] = *reinterpret_cast<const bf16x8*>(a.w + (size_t)(16 * t + xl) * KT + 8 * g);
            const uint16_t* l16 = reinterpret_cast<const uint16_t*>(lds);
#pragma unroll
            for (int r = 0; r < kRowsPerWave; ++r) {
                const int row = wave * kRowsPerWave + r;
                const int ty = row % BY, tz = row / BY;
                bf16x8 bfr;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int tap = min(8 * g + e, 26);  // padded taps carry zero weights
                    const int hv = ((tz + 1 + tap_dz(tap)) * HY + ty + 1 + tap_dy(tap)) * HX + xl + 1 + tap_dx(tap);
                    bfr[e] = __builtin_bit_cast(bf16, l16[hv]);
                }
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[t], bfr, acc[r][t], 0, 0, 0);
            }
        } else {
            const bf16x8* l8 = reinterpret_cast<const bf16x8*>(lds);
            for (int kc = 0; kc < NCH; ++kc) {
                int tap, ch;
                if constexpr (CC == 32) {
                    tap = kc;
                    ch = 8 * g;
                } else {
                    tap = 2 * kc + (g >> 1);
                    ch = 8 * (g & 1);
                }
                bf16x8 af[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    af[t] = *reinterpret_cast<const bf16x8*>(a.w + ((size_t)(16 * t + xl) * NP + p) * KT * CC +
                                                             tap * CC + ch);
                const int tp = min(tap, 26);  // tap 27 (CC = 16 padding) has zero weights
                const int dz = tap_dz(tp), dy = tap_dy(tp), dx = tap_dx(tp);
#pragma unroll
                for (int r = 0; r < kRowsPerWave; ++r) {
                    const int row = wave * kRowsPerWave + r;
                    const int ty = row % BY, tz = row / BY;
                    const int hv = ((tz + 1 + dz) * HY + ty + 1 + dy) * HX + xl + 1 + dx;
                    const bf16x8 bfr = l8[hv * RSU + (ch >> 3)];
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[t], bfr, acc[r][t], 0, 0, 0);
                }
            }
        }
    }

    // epilogue: lane holds channels 16t + 4g + (0..3) of voxel x0 + xl
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) {
        const int row = wave * kRowsPerWave + r;
        const int x = x0 + xl, y = y0 + row % BY, z = z0 + row / BY;
        if (x >= a.nx || y >= a.ny || z >= a.nz) continue;
        const size_t v = ((size_t)z * a.ny + y) * a.nx + x;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int co = 16 * t + 4 * g;
            float o[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = acc[r][t][e] + (a.bias ? a.bias[co + e] : 0.f);
            if (a.relu) {
#pragma unroll
                for (int e = 0; e < 4; ++e) o[e] = fmaxf(o[e], 0.f);
            }
            if (a.mask_a) {
                const bf16* mp = co < a.mca ? a.mask_a + v * a.ldma + co : a.mask_b + v * a.ldmb + (co - a.mca);
                const uint2 m = *reinterpret_cast<const uint2*>(mp);
                const uint16_t mb[4] = {(uint16_t)(m.x & 0xFFFFu), (uint16_t)(m.x >> 16), (uint16_t)(m.y & 0xFFFFu),
                                        (uint16_t)(m.y >> 16)};
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (!bf16_pos(mb[e])) o[e] = 0.f;
            }
            uint2 st;
            st.x = (uint32_t)bf16_bits(o[0]) | ((uint32_t)bf16_bits(o[1]) << 16);
            st.y = (uint32_t)bf16_bits(o[2]) | ((uint32_t)bf16_bits(o[3]) << 16);
            *reinterpret_cast<uint2*>(a.out + v * a.ldo + co) = st;
        }
    }
}

struct WgArgs {
    Src src;
    const bf16* g;  // [voxel][ldg]: gradient at the conv output (before ReLU), CO channels
    int ldg;
    float* part;    // [gridDim.x][NP * T][16 * 16]
    int nx, ny, nz, bnx, bny, nbricks;
    int np;
};

// Weight gradient partial sums (see the file comment).  Tiles: CC >= 16:
// (tap, ci-tile, co-tile), T = 27 * (CC/16) * (CO/16), D[co][ci]; CC = 1:
// (tap-tile, co-tile), T = 2 * (CO/16), D[co][tap].  blockIdx.y: group of
// kTilesPerGroup tiles, blockIdx.z: input pass.
template <int CC, int CO>
__global__ __launch_bounds__(kThreads) void k_wgrad(WgArgs a) {
    constexpr int NCOT = CO / 16;
    constexpr int NCIT = CC == 1 ? 2 : CC / 16;
    constexpr int T = CC == 1 ? NCIT * NCOT : 27 * NCIT * NCOT;
    constexpr int RSU = CC == 1 ? 1 : CC / 8 + 1;
    constexpr int RS = RSU * 8;
    constexpr int HV = HX * HY * (WBZ + 2);
    constexpr int LDS_U4 = CC == 1 ? (HV * 2 + 15) / 16 : HV * RSU;
    constexpr int RSG = CO + 8;
    __shared__ uint4 xs[LDS_U4];
    __shared__ uint4 gs[WV * RSG / 8];
    const uint16_t* x16 = reinterpret_cast<const uint16_t*>(xs);
    const uint16_t* g16 = reinterpret_cast<const uint16_t*>(gs);

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, xl = lane & 15;
    const int pass = blockIdx.z;
    const int t_begin = blockIdx.y * kTilesPerGroup;

    f32x4 acc[kTilesPerWave];
#pragma unroll
    for (int j = 0; j < kTilesPerWave; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int br = blockIdx.x; br < a.nbricks; br += gridDim.x) {
        int b = br;
        const int bx = b % a.bnx;
        b /= a.bnx;
        const int by = b % a.bny, bz = b / a.bny;
        const int x0 = bx * BX, y0 = by * BY, z0 = bz * WBZ;
        __syncthreads();  // the previous brick's reads are done
        if constexpr (CC == 1)
            stage_halo1<WBZ + 2>(reinterpret_cast<uint16_t*>(xs), a.src, x0, y0, z0, a.nx, a.ny, a.nz);
        else
            stage_halo<CC, WBZ + 2>(xs, a.src, pass, x0, y0, z0, a.nx, a.ny, a.nz);
        for (int i = threadIdx.x; i < WV * CO / 8; i += kThreads) {
            const int vi = i / (CO / 8), j = i - vi * (CO / 8);
            const int x = x0 + (vi & 15), y = y0 + ((vi >> 4) & 3), z = z0 + (vi >> 6);
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (x < a.nx && y < a.ny && z < a.nz)
                v = *reinterpret_cast<const uint4*>(a.g + (((size_t)z * a.ny + y) * a.nx + x) * a.ldg + 8 * j);
            gs[vi * (RSG / 8) + j] = v;
        }
        __syncthreads();

#pragma unroll 1
        for (int c = 0; c < WV / 32; ++c) {
            const int vi0 = 32 * c + 8 * g;  // this lane's 8 voxels: vi0 .. vi0 + 7 (one half row)
            const int row = vi0 >> 4, xo = vi0 & 15;
            const int ty = row & 3, tz = row >> 2;
            bf16x8 af[NCOT];
#pragma unroll
            for (int ct = 0; ct < NCOT; ++ct)
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    af[ct][e] = __builtin_bit_cast(bf16, g16[(vi0 + e) * RSG + 16 * ct + xl]);
#pragma unroll
            for (int j = 0; j < kTilesPerWave; ++j) {
                const int tile = t_begin + wave + 4 * j;
                if (tile >= T) continue;  // uniform over the wave
                const int cot = tile % NCOT;
                bf16x8 bfr;
                if constexpr (CC == 1) {
                    const int tap = 16 * (tile / NCOT) + xl;
                    const int tp = min(tap, 26);
                    const int hv0 = ((tz + 1 + tap_dz(tp)) * HY + ty + 1 + tap_dy(tp)) * HX + xo + 1 + tap_dx(tp);
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        bfr[e] = __builtin_bit_cast(bf16, tap < 27 ? x16[hv0 + e] : (uint16_t)0);
                } else {
                    const int rest = tile / NCOT;
                    const int cit = rest % NCIT, tap = rest / NCIT;
                    const int hv0 = ((tz + 1 + tap_dz(tap)) * HY + ty + 1 + tap_dy(tap)) * HX + xo + 1 + tap_dx(tap);
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        bfr[e] = __builtin_bit_cast(bf16, x16[(hv0 + e) * RS + 16 * cit + xl]);
                }
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[cot], bfr, acc[j], 0, 0, 0);
            }
        }
    }

    const size_t npt = (size_t)a.np * T;
#pragma unroll
    for (int j = 0; j < kTilesPerWave; ++j) {
        const int tile = t_begin + wave + 4 * j;
        if (tile >= T) continue;
        float* o = a.part + ((size_t)blockIdx.x * npt + (size_t)pass * T + tile) * 256;
#pragma unroll
        for (int e = 0; e < 4; ++e) o[(4 * g + e) * 16 + xl] = acc[j][e];
    }
}

// Weight gradient for CC in {16, 32}: the same brick, partial-sum layout and
// tile numbering as k_wgrad, with wide LDS reads.  The input halo is staged
// transposed, XT[ci][hz][hy][e] with the x of halo voxel hx at element
// e = hx + 7 (so interior x lands 16-byte aligned at e = x + 8), and the
// output gradient as GT[co][v].  A lane's 8 consecutive voxels are then one
// 16-byte read; the taps dx = -1 and +1 are the aligned read shifted by one
// element either way, built from the neighbouring aligned chunk with
// v_alignbyte.  A wave owns whole tap rows (dz, dy) of one channel tile
// (a unit) and multiplies the three dx fragments, read once, by every output
// channel tile.
constexpr int kXRow = 32;                       // elements per (hz, hy) row of XT
constexpr int kXStride = 4 * HY * kXRow + 8;    // per channel (padding shifts banks by 4)
constexpr int kGStride = WV + 8;                // per output channel of GT

__device__ inline uint32_t align2(uint32_t hi, uint32_t lo) { return __builtin_amdgcn_alignbyte(hi, lo, 2); }

template <int CC, int CO>
__global__ __launch_bounds__(kThreads) void k_wgrad2(WgArgs a) {
    constexpr int NCOT = CO / 16;
    constexpr int NCIT = CC / 16;
    constexpr int UPW = NCOT == 1 ? 4 : (NCOT == 2 ? 2 : 1);  // units per wave
    constexpr int UNITS = 9 * NCIT;
    __shared__ uint4 xs[CC * kXStride / 8];
    __shared__ uint4 gs[CO * kGStride / 8];
    uint16_t* x16 = reinterpret_cast<uint16_t*>(xs);
    uint16_t* g16 = reinterpret_cast<uint16_t*>(gs);

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, xl = lane & 15;
    const int pass = blockIdx.z;
    const int u0 = (blockIdx.y * 4 + wave) * UPW;

    f32x4 acc[UPW][3][NCOT];
#pragma unroll
    for (int i = 0; i < UPW; ++i)
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int t = 0; t < NCOT; ++t) acc[i][d][t] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int br = blockIdx.x; br < a.nbricks; br += gridDim.x) {
        int b = br;
        const int bx = b % a.bnx;
        b /= a.bnx;
        const int by = b % a.bny, bz = b / a.bny;
        const int x0 = bx * BX, y0 = by * BY, z0 = bz * WBZ;
        __syncthreads();  // the previous brick's reads are done
        // input: quads of 4 halo voxels along x (e = 4q .. 4q+3, q = 1..6) x 8 channels
        for (int i = threadIdx.x; i < (WBZ + 2) * HY * 6 * (CC / 8); i += kThreads) {
            int r = i;
            const int j = r % (CC / 8);
            r /= CC / 8;
            const int q = 1 + r % 6;
            r /= 6;
            const int hy = r % HY, hz = r / HY;
            uint32_t w[4][4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int hx = 4 * q + k - 7;
                const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
                uint4 v = make_uint4(0u, 0u, 0u, 0u);
                if (hx >= 0 && hx < HX && (unsigned)gx < (unsigned)a.nx && (unsigned)gy < (unsigned)a.ny &&
                    (unsigned)gz < (unsigned)a.nz)
                    v = load_src8(a.src, pass * CC + 8 * j, gx, gy, gz, a.nx, a.ny);
                w[k][0] = v.x;
                w[k][1] = v.y;
                w[k][2] = v.z;
                w[k][3] = v.w;
            }
            // channel c = 2m + h of voxel k sits in half h of w[k][m]
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int m = c >> 1, sh = 16 * (c & 1);
                uint2 o;
                o.x = ((w[0][m] >> sh) & 0xFFFFu) | (((w[1][m] >> sh) & 0xFFFFu) << 16);
                o.y = ((w[2][m] >> sh) & 0xFFFFu) | (((w[3][m] >> sh) & 0xFFFFu) << 16);
                *reinterpret_cast<uint2*>(x16 + (size_t)(8 * j + c) * kXStride + (hz * HY + hy) * kXRow + 4 * q) = o;
            }
        }
        // output gradient: quads of 4 voxels x 8 channels
        for (int i = threadIdx.x; i < (WV / 4) * (CO / 8); i += kThreads) {
            const int j = i % (CO / 8), vq = i / (CO / 8);
            uint32_t w[4][4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int vi = 4 * vq + k;
                const int x = x0 + (vi & 15), y = y0 + ((vi >> 4) & 3), z = z0 + (vi >> 6);
                uint4 v = make_uint4(0u, 0u, 0u, 0u);
                if (x < a.nx && y < a.ny && z < a.nz)
                    v = *reinterpret_cast<const uint4*>(a.g + (((size_t)z * a.ny + y) * a.nx + x) * a.ldg + 8 * j);
                w[k][0] = v.x;
                w[k][1] = v.y;
                w[k][2] = v.z;
                w[k][3] = v.w;
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int m = c >> 1, sh = 16 * (c & 1);
                uint2 o;
                o.x = ((w[0][m] >> sh) & 0xFFFFu) | (((w[1][m] >> sh) & 0xFFFFu) << 16);
                o.y = ((w[2][m] >> sh) & 0xFFFFu) | (((w[3][m] >> sh) & 0xFFFFu) << 16);
                *reinterpret_cast<uint2*>(g16 + (size_t)(8 * j + c) * kGStride + 4 * vq) = o;
            }
        }
        __syncthreads();

#pragma unroll 1
        for (int c = 0; c < WV / 32; ++c) {
            const int vi0 = 32 * c + 8 * g;  // this lane's 8 voxels (one half row)
            const int row = vi0 >> 4, xo = vi0 & 15;
            const int ty = row & 3, tz = row >> 2;
            bf16x8 af[NCOT];
#pragma unroll
            for (int t = 0; t < NCOT; ++t)
                af[t] = *reinterpret_cast<const bf16x8*>(g16 + (size_t)(16 * t + xl) * kGStride + vi0);
#pragma unroll
            for (int i = 0; i < UPW; ++i) {
                const int u = u0 + i;
                if (u >= UNITS) continue;  // uniform over the wave
                const int cit = u % NCIT, tr = u / NCIT;
                const int dz = tr / 3 - 1, dy = tr % 3 - 1;
                const uint16_t* rowp = x16 + (size_t)(16 * cit + xl) * kXStride +
                                       ((tz + 1 + dz) * HY + ty + 1 + dy) * kXRow + xo;
                const uint4 A = *reinterpret_cast<const uint4*>(rowp);
                const uint4 B = *reinterpret_cast<const uint4*>(rowp + 8);
                const uint4 C = *reinterpret_cast<const uint4*>(rowp + 16);
                uint4 fm, fp;  // dx = -1: elements xo+7 .. xo+14; dx = +1: xo+9 .. xo+16
                fm.x = align2(B.x, A.w);
                fm.y = align2(B.y, B.x);
                fm.z = align2(B.z, B.y);
                fm.w = align2(B.w, B.z);
                fp.x = align2(B.y, B.x);
                fp.y = align2(B.z, B.y);
                fp.z = align2(B.w, B.z);
                fp.w = align2(C.x, B.w);
                const bf16x8 bm = __builtin_bit_cast(bf16x8, fm);
                const bf16x8 b0 = __builtin_bit_cast(bf16x8, B);
                const bf16x8 bp = __builtin_bit_cast(bf16x8, fp);
#pragma unroll
                for (int t = 0; t < NCOT; ++t) {
                    acc[i][0][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[t], bm, acc[i][0][t], 0, 0, 0);
                    acc[i][1][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[t], b0, acc[i][1][t], 0, 0, 0);
                    acc[i][2][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[t], bp, acc[i][2][t], 0, 0, 0);
                }
            }
        }
    }

    // tile numbering of k_wgrad: tile = (tap * NCIT + cit) * NCOT + cot, tap = tr * 3 + dx + 1
    constexpr int T = 27 * NCIT * NCOT;
    const size_t npt = (size_t)a.np * T;
#pragma unroll
    for (int i = 0; i < UPW; ++i) {
        const int u = u0 + i;
        if (u >= UNITS) continue;
        const int cit = u % NCIT, tr = u / NCIT;
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int t = 0; t < NCOT; ++t) {
                const int tile = ((tr * 3 + d) * NCIT + cit) * NCOT + t;
                float* o = a.part + ((size_t)blockIdx.x * npt + (size_t)pass * T + tile) * 256;
#pragma unroll
                for (int e = 0; e < 4; ++e) o[(4 * g + e) * 16 + xl] = acc[i][d][t][e];
            }
    }
}

// Sums the weight-gradient partials of nblk blocks and writes dW in the
// canonical layout [co][tap][ci].  A block takes 32 consecutive outputs; its
// 8 thread rows each add the partials b = r, r + 8, ... in increasing b, and
// row 0 adds the 8 row sums in order (a fixed order for every run).
constexpr int kRedCols = 32, kRedRows = kThreads / kRedCols;

__device__ inline float reduce_rows_fixed(const float* part, int nblk, size_t total, size_t idx, bool valid,
                                          float (*sh)[kRedCols]) {
    const int c = threadIdx.x % kRedCols, r = threadIdx.x / kRedCols;
    float s = 0.f;
    if (valid) {
#pragma unroll 4
        for (int b = r; b < nblk; b += kRedRows) s += part[(size_t)b * total + idx];
    }
    sh[r][c] = s;
    __syncthreads();
    float t = 0.f;
    if (r == 0)
        for (int i = 0; i < kRedRows; ++i) t += sh[i][c];
    return t;
}

__global__ __launch_bounds__(kThreads) void k_wgrad_reduce(const float* part, int nblk, int cc, int co_n, int np,
                                                          int ci_n, float* dw) {
    __shared__ float sh[kRedRows][kRedCols];
    const int ncot = co_n / 16;
    const int ncit = cc == 1 ? 2 : cc / 16;
    const int T = cc == 1 ? ncit * ncot : 27 * ncit * ncot;
    const int total = np * T * 256;
    const int idx = blockIdx.x * kRedCols + threadIdx.x % kRedCols;
    const float s = reduce_rows_fixed(part, nblk, total, idx, idx < total, sh);
    if (threadIdx.x >= kRedCols || idx >= total) return;
    const int ptile = idx >> 8, i = (idx >> 4) & 15, jc = idx & 15;
    const int pass = ptile / T, tile = ptile % T;
    const int co = 16 * (tile % ncot) + i;
    if (cc == 1) {
        const int tap = 16 * (tile / ncot) + jc;
        if (tap < 27) dw[(size_t)co * 27 + tap] = s;
    } else {
        const int rest = tile / ncot;
        const int cit = rest % ncit, tap = rest / ncit;
        const int ci = pass * cc + 16 * cit + jc;
        dw[((size_t)co * 27 + tap) * ci_n + ci] = s;
    }
}

// Bias gradient: per-block channel sums of g [voxel][ldg] (CO channels) ...
template <int CO>
__global__ __launch_bounds__(kThreads) void k_bias_part(const bf16* g, int ldg, int64_t nvox, float* part) {
    constexpr int G8 = CO / 8, VL = kThreads / G8;
    const int j = threadIdx.x % G8, vl = threadIdx.x / G8;
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int64_t v = (int64_t)blockIdx.x * VL + vl; v < nvox; v += (int64_t)gridDim.x * VL) {
        const uint4 q = *reinterpret_cast<const uint4*>(g + v * ldg + 8 * j);
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            s[2 * e] += bf16_float((uint16_t)(w[e] & 0xFFFFu));
            s[2 * e + 1] += bf16_float((uint16_t)(w[e] >> 16));
        }
    }
    __shared__ float sh[kThreads][9];
#pragma unroll
    for (int e = 0; e < 8; ++e) sh[threadIdx.x][e] = s[e];
    __syncthreads();
    if (threadIdx.x < CO) {
        const int c = threadIdx.x, jj = c / 8, e = c % 8;
        float t = 0.f;
        for (int l = 0; l < VL; ++l) t += sh[l * G8 + jj][e];
        part[(size_t)blockIdx.x * CO + c] = t;
    }
}

// ... added over the blocks (fixed order, as k_wgrad_reduce).
__global__ __launch_bounds__(kThreads) void k_bias_reduce(const float* part, int nblk, int co_n, float* db) {
    __shared__ float sh[kRedRows][kRedCols];
    const int idx = blockIdx.x * kRedCols + threadIdx.x % kRedCols;
    const float s = reduce_rows_fixed(part, nblk, co_n, idx, idx < co_n, sh);
    if (threadIdx.x < kRedCols && idx < co_n) db[idx] = s;
}

// Sum of nblk float64 values in a fixed order: thread t adds t, t + 256, ...,
// then a fixed shuffle tree and the 4 wave sums in order.  Valid in thread 0.
__device__ inline double block_sum_f64(const double* p, int nblk, size_t stride, double* sh) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kThreads) s += p[(size_t)b * stride];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    return ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// 2x2x2 average pooling (fine grid nx, ny, nz; C channels).
__global__ void k_pool2(const bf16* in, int C, int nx, int ny, int nz, bf16* out) {
    const int mx = nx / 2, my = ny / 2, mz = nz / 2, G8 = C / 8;
    const int64_t total = (int64_t)mx * my * mz * G8;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(i % G8);
        const int64_t V = i / G8;
        const int X = (int)(V % mx), Y = (int)((V / mx) % my), Z = (int)(V / ((int64_t)mx * my));
        float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int c = 0; c < 8; ++c) {
            const int x = 2 * X + (c & 1), y = 2 * Y + ((c >> 1) & 1), z = 2 * Z + (c >> 2);
            const uint4 q = *reinterpret_cast<const uint4*>(in + (((size_t)z * ny + y) * nx + x) * C + 8 * j);
            const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                s[2 * e] += bf16_float((uint16_t)(w[e] & 0xFFFFu));
                s[2 * e + 1] += bf16_float((uint16_t)(w[e] >> 16));
            }
        }
        uint4 o;
        uint32_t* ow = reinterpret_cast<uint32_t*>(&o);
#pragma unroll
        for (int e = 0; e < 4; ++e)
            ow[e] = (uint32_t)bf16_bits(s[2 * e] * 0.125f) | ((uint32_t)bf16_bits(s[2 * e + 1] * 0.125f) << 16);
        *reinterpret_cast<uint4*>(out + (size_t)V * C + 8 * j) = o;
    }
}

// Gradient through a pooling: out[v] = (skip[v] + gp[parent(v)] / 8) * [act[v] > 0]
// on the fine grid (skip: the gradient arriving through the skip connection,
// ld lds_; C channels).
__global__ void k_pool_bwd(const bf16* skip, int lds_, const bf16* gp, const bf16* act, int C, int nx, int ny, int nz,
                           bf16* out) {
    const int G8 = C / 8, mx = nx / 2, my = ny / 2;
    const int64_t total = (int64_t)nx * ny * nz * G8;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(i % G8);
        const int64_t v = i / G8;
        const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((int64_t)nx * ny));
        const size_t V = ((size_t)(z >> 1) * my + (y >> 1)) * mx + (x >> 1);
        const uint4 qs = *reinterpret_cast<const uint4*>(skip + (size_t)v * lds_ + 8 * j);
        const uint4 qp = *reinterpret_cast<const uint4*>(gp + V * C + 8 * j);
        const uint4 qa = *reinterpret_cast<const uint4*>(act + (size_t)v * C + 8 * j);
        const uint32_t ws[4] = {qs.x, qs.y, qs.z, qs.w}, wp[4] = {qp.x, qp.y, qp.z, qp.w},
                       wa[4] = {qa.x, qa.y, qa.z, qa.w};
        uint4 o;
        uint32_t* ow = reinterpret_cast<uint32_t*>(&o);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            uint32_t r = 0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint16_t bs = (uint16_t)(ws[e] >> (16 * h)), bp = (uint16_t)(wp[e] >> (16 * h)),
                               ba = (uint16_t)(wa[e] >> (16 * h));
                const float val = bf16_pos(ba) ? bf16_float(bs) + 0.125f * bf16_float(bp) : 0.f;
                r |= (uint32_t)bf16_bits(val) << (16 * h);
            }
            ow[e] = r;
        }
        *reinterpret_cast<uint4*>(out + (size_t)v * C + 8 * j) = o;
    }
}

// Gradient through a nearest upsampling: out[V] = sum of the 8 children of
// gup (fine grid 2mx x 2my x 2mz), times [act[V] > 0] (coarse grid).
__global__ void k_up_bwd(const bf16* gup, const bf16* act, int C, int mx, int my, int mz, bf16* out) {
    const int G8 = C / 8, nx = 2 * mx, ny = 2 * my;
    const int64_t total = (int64_t)mx * my * mz * G8;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(i % G8);
        const int64_t V = i / G8;
        const int X = (int)(V % mx), Y = (int)((V / mx) % my), Z = (int)(V / ((int64_t)mx * my));
        float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int c = 0; c < 8; ++c) {
            const int x = 2 * X + (c & 1), y = 2 * Y + ((c >> 1) & 1), z = 2 * Z + (c >> 2);
            const uint4 q = *reinterpret_cast<const uint4*>(gup + (((size_t)z * ny + y) * nx + x) * C + 8 * j);
            const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                s[2 * e] += bf16_float((uint16_t)(w[e] & 0xFFFFu));
                s[2 * e + 1] += bf16_float((uint16_t)(w[e] >> 16));
            }
        }
        const uint4 qa = *reinterpret_cast<const uint4*>(act + (size_t)V * C + 8 * j);
        const uint32_t wa[4] = {qa.x, qa.y, qa.z, qa.w};
        uint4 o;
        uint32_t* ow = reinterpret_cast<uint32_t*>(&o);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float v0 = bf16_pos((uint16_t)(wa[e] & 0xFFFFu)) ? s[2 * e] : 0.f;
            const float v1 = bf16_pos((uint16_t)(wa[e] >> 16)) ? s[2 * e + 1] : 0.f;
            ow[e] = (uint32_t)bf16_bits(v0) | ((uint32_t)bf16_bits(v1) << 16);
        }
        *reinterpret_cast<uint4*>(out + V * C + 8 * j) = o;
    }
}

// Normalisation: s = sqrt(mean(x^2)) from float64 block partials in a fixed
// order; sc[0] = s, sc[1] = 1 / s (0 when s = 0).
__global__ __launch_bounds__(kThreads) void k_sumsq_part(const float* x, int64_t n, double* part) {
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = x[i];
        s += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    __shared__ double sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

__global__ __launch_bounds__(kThreads) void k_norm_finish(const double* part, int nblk, int64_t n, float* sc) {
    __shared__ double sh[4];
    const double s = block_sum_f64(part, nblk, 1, sh);
    if (threadIdx.x != 0) return;
    const double rms = sqrt(s / (double)n);
    const float sf = (float)rms;
    sc[0] = sf;
    sc[1] = (sf > 0.f && isfinite(sf)) ? 1.f / sf : 0.f;
}

__global__ void k_prep_input(const float* x, const float* sc, int64_t n, bf16* x0) {
    const float inv = sc[1];
    uint16_t* o = reinterpret_cast<uint16_t*>(x0);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        o[i] = bf16_bits(x[i] * inv);
}

// Head (1x1x1 conv of d1, 16 channels) and residual.  Inference (t == null):
// y = x + s * h.  Training: loss = mean((x/s + h - t/s)^2), gradient at the
// head input gd1 = gy * hw * [d1 > 0] with gy = 2 (x/s + h - t/s) / n, and
// per-block float64 partials [18]: loss sum, d/dhw (16), d/dhb.
struct HeadArgs {
    const bf16* d1;
    const float* x;
    const float* t;
    const float* sc;
    const float* hw;  // [16] then hb
    float* y;
    bf16* gd1;
    double* part;
    int64_t n;
};

__global__ __launch_bounds__(kThreads) void k_head(HeadArgs a) {
    float hw[kBase];
#pragma unroll
    for (int c = 0; c < kBase; ++c) hw[c] = a.hw[c];
    const float hb = a.hw[kBase];
    const float s = a.sc[0], inv = a.sc[1];
    const bool train = a.t != nullptr;
    double acc[kBase + 2];
#pragma unroll
    for (int c = 0; c < kBase + 2; ++c) acc[c] = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += (int64_t)gridDim.x * blockDim.x) {
        const uint4 q0 = *reinterpret_cast<const uint4*>(a.d1 + v * kBase);
        const uint4 q1 = *reinterpret_cast<const uint4*>(a.d1 + v * kBase + 8);
        const uint32_t w[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
        uint16_t db[kBase];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            db[2 * e] = (uint16_t)(w[e] & 0xFFFFu);
            db[2 * e + 1] = (uint16_t)(w[e] >> 16);
        }
        float h = hb;
#pragma unroll
        for (int c = 0; c < kBase; ++c) h += hw[c] * bf16_float(db[c]);
        const float xv = a.x[v];
        if (!train) {
            a.y[v] = xv + s * h;
            continue;
        }
        const float diff = (xv * inv + h) - a.t[v] * inv;
        const float gy = 2.f * diff / (float)a.n;
        acc[0] += (double)diff * (double)diff;
        uint4 o0, o1;
        uint32_t* ow0 = reinterpret_cast<uint32_t*>(&o0);
        uint32_t* ow1 = reinterpret_cast<uint32_t*>(&o1);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            uint32_t r = 0;
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const int c = 2 * e + hh;
                const float dv = bf16_float(db[c]);
                acc[1 + c] += (double)(gy * dv);
                r |= (uint32_t)bf16_bits(bf16_pos(db[c]) ? gy * hw[c] : 0.f) << (16 * hh);
            }
            if (e < 4) ow0[e] = r;
            else ow1[e - 4] = r;
        }
        acc[kBase + 1] += (double)gy;
        *reinterpret_cast<uint4*>(a.gd1 + v * kBase) = o0;
        *reinterpret_cast<uint4*>(a.gd1 + v * kBase + 8) = o1;
    }
    if (!train) return;
    __shared__ double sh[4][kBase + 2];
#pragma unroll
    for (int c = 0; c < kBase + 2; ++c) {
        double t = acc[c];
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][c] = t;
    }
    __syncthreads();
    if (threadIdx.x < kBase + 2) {
        const int c = threadIdx.x;
        a.part[(size_t)blockIdx.x * (kBase + 2) + c] = ((sh[0][c] + sh[1][c]) + sh[2][c]) + sh[3][c];
    }
}

// Sums the head partials (one block per value, fixed order): loss (double),
// gradient of hw and hb.
__global__ __launch_bounds__(kThreads) void k_head_finish(const double* part, int nblk, int64_t n, float* ghead,
                                                         double* loss) {
    __shared__ double sh[4];
    const int c = blockIdx.x;
    const double s = block_sum_f64(part + c, nblk, kBase + 2, sh);
    if (threadIdx.x != 0) return;
    if (c == 0) *loss = s / (double)n;
    else ghead[c - 1] = (float)s;
}

// Adam step on the float32 master weights.
__global__ void k_adam(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

// Master weights [co][27][ci] -> bfloat16 kernel layouts: forward
// wk [co][pass][KT][cc] and, when wd is given, input-gradient
// wd [ci][pass'][KT'][ccd] with the taps mirrored (tap -> 26 - tap).
__global__ void k_prep_w(const float* w, int ci_n, int co_n, bf16* wk, int cc, int np, bf16* wd, int ccd, int npd) {
    const int kt = kt_of(cc), ktd = kt_of(ccd);
    const int total = co_n * 27 * ci_n;
    uint16_t* wk16 = reinterpret_cast<uint16_t*>(wk);
    uint16_t* wd16 = reinterpret_cast<uint16_t*>(wd);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int ci = i % ci_n, tap = (i / ci_n) % 27, co = i / (27 * ci_n);
        const uint16_t b = bf16_bits(w[i]);
        wk16[(((size_t)co * np + ci / cc) * kt + tap) * cc + ci % cc] = b;
        if (wd) wd16[(((size_t)ci * npd + co / ccd) * ktd + (26 - tap)) * ccd + co % ccd] = b;
    }
}

// ------------------------------------------------------------------ host

struct Tensor {
    bf16* p = nullptr;
    int c = 0;   // channels (= elements per voxel)
    int lev = 0;
};

struct Layer {
    const char* name;
    int ci_a, ci_b, co, lev, up;
    int64_t w_off, b_off;
    int cc, np;    // forward kernel layout
    int ccd, npd;  // input-gradient layout (ccd = 0: none)
    bf16* wk = nullptr;
    bf16* wd = nullptr;
};

int cc_of(int ci) { return ci == 1 ? 1 : std::min(ci, 32); }

}  // namespace unet
}  // namespace cgd

struct cgd_unet_s {
    int device = 0;
    int n[3][3];         // [level][axis] grid sizes
    int64_t nvox[3];
    int64_t n_params = 0;
    int64_t head_off = 0;
    int64_t adam_t = 0;
    cgd::unet::Layer L[cgd::unet::kLayers];
    void* arena = nullptr;
    float *params, *grads, *adam_m, *adam_v;
    float* sc;           // [2]: s, 1/s
    double* loss;        // [1]
    double* dpart;       // float64 partials
    float* fpart;        // float32 partials (weight / bias gradients)
    size_t fpart_floats = 0;
    cgd::unet::Tensor x0, act[cgd::unet::kLayers], p1, p2;
    // gradients (see backward())
    cgd::unet::Tensor gd1, ga5, gc1, gq2, gd2, ga4, gc2, gq3, ge3, ga3, gp2, ge2, ga2, gp1, ge1, ga1;
};

namespace cgd {
namespace unet {

namespace {

enum { E1A, E1B, E2A, E2B, E3A, E3B, U2, D2A, D2B, U1, D1A, D1B };

int grid_blocks(int64_t work, int per_block = kThreads, int cap = 4096) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(cap, (work + per_block - 1) / per_block));
}

template <int CC, int CO, int NP>
void launch_conv_t(const ConvArgs& a, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL((k_conv<CC, CO, NP>), dim3(nblocks), dim3(kThreads), 0, s, a);
}

// Enqueues one convolution; returns false for an unsupported shape.
bool launch_conv(int cc, int co, int np, ConvArgs a, hipStream_t s) {
    a.bnx = (a.nx + BX - 1) / BX;
    a.bny = (a.ny + BY - 1) / BY;
    const int bnz = (a.nz + BZ - 1) / BZ;
    const int nb = a.bnx * a.bny * bnz;
#define CGD_CONV_CASE(C1, C2, C3) \
    if (cc == C1 && co == C2 && np == C3) return launch_conv_t<C1, C2, C3>(a, nb, s), true;
    CGD_CONV_CASE(1, 16, 1)
    CGD_CONV_CASE(16, 16, 1)
    CGD_CONV_CASE(16, 32, 1)
    CGD_CONV_CASE(16, 64, 1)
    CGD_CONV_CASE(32, 16, 1)
    CGD_CONV_CASE(32, 32, 1)
    CGD_CONV_CASE(32, 64, 1)
    CGD_CONV_CASE(32, 16, 2)
    CGD_CONV_CASE(32, 32, 2)
    CGD_CONV_CASE(32, 64, 2)
#undef CGD_CONV_CASE
    return false;
}

int wgrad_tiles(int cc, int co) { return cc == 1 ? 2 * (co / 16) : 27 * (cc / 16) * (co / 16); }

// Blocks along x of a weight-gradient launch (partials per block), chosen so
// that about 1024 blocks run in all.
int wgrad_nblk(int64_t nbricks, int groups, int np) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(nbricks, 1024 / std::max(1, groups * np)));
}

// Block groups along y of a weight-gradient launch: k_wgrad (CC = 1) takes
// kTilesPerGroup tiles per group, k_wgrad2 four waves of whole tap-row units.
int wgrad_groups(int cc, int co) {
    if (cc == 1) return (wgrad_tiles(cc, co) + kTilesPerGroup - 1) / kTilesPerGroup;
    const int ncot = co / 16, units = 9 * (cc / 16);
    const int upw = ncot == 1 ? 4 : (ncot == 2 ? 2 : 1);
    return (units + 4 * upw - 1) / (4 * upw);
}

size_t wgrad_part_floats(int nx, int ny, int nz, int cc, int co, int np) {
    const int64_t nbr = (int64_t)((nx + BX - 1) / BX) * ((ny + BY - 1) / BY) * ((nz + WBZ - 1) / WBZ);
    const int T = wgrad_tiles(cc, co);
    const int groups = wgrad_groups(cc, co);
    return (size_t)wgrad_nblk(nbr, groups, np) * np * T * 256;
}

template <int CC, int CO>
void launch_wgrad_t(const WgArgs& a, dim3 grid, hipStream_t s) {
    hipLaunchKernelGGL((k_wgrad<CC, CO>), grid, dim3(kThreads), 0, s, a);
}

template <int CC, int CO>
void launch_wgrad2_t(const WgArgs& a, dim3 grid, hipStream_t s) {
    hipLaunchKernelGGL((k_wgrad2<CC, CO>), grid, dim3(kThreads), 0, s, a);
}

// Weight and bias gradients of one convolution into dw [co][27][ci], db [co].
bool launch_wgrad(int cc, int co, int np, const Src& src, const bf16* g, int ldg, int nx, int ny, int nz, float* part,
                  float* dw, float* db, hipStream_t s) {
    WgArgs a = {};
    a.src = src;
    a.g = g;
    a.ldg = ldg;
    a.part = part;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.bnx = (nx + BX - 1) / BX;
    a.bny = (ny + BY - 1) / BY;
    a.nbricks = a.bnx * a.bny * ((nz + WBZ - 1) / WBZ);
    a.np = np;
    const int T = wgrad_tiles(cc, co);
    const int groups = wgrad_groups(cc, co);
    const int nblk = wgrad_nblk(a.nbricks, groups, np);
    const dim3 grid(nblk, groups, np);
    bool ok = true;
    if (cc == 1 && co == 16) launch_wgrad_t<1, 16>(a, grid, s);
    else if (cc == 16 && co == 16) launch_wgrad2_t<16, 16>(a, grid, s);
    else if (cc == 16 && co == 32) launch_wgrad2_t<16, 32>(a, grid, s);
    else if (cc == 16 && co == 64) launch_wgrad2_t<16, 64>(a, grid, s);
    else if (cc == 32 && co == 16) launch_wgrad2_t<32, 16>(a, grid, s);
    else if (cc == 32 && co == 32) launch_wgrad2_t<32, 32>(a, grid, s);
    else if (cc == 32 && co == 64) launch_wgrad2_t<32, 64>(a, grid, s);
    else ok = false;
    if (!ok) return false;
    const int ci_n = cc == 1 ? 1 : cc * np;
    const int total = np * T * 256;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((total + kRedCols - 1) / kRedCols), dim3(kThreads), 0, s, part, nblk, cc,
                       co, np, ci_n, dw);
    // bias: partials reuse the start of `part` (the reduce above has read it: same stream)
    const int64_t nvox = (int64_t)nx * ny * nz;
    const int bnb = grid_blocks(nvox / 8 + 1, kThreads, 1024);
    if (co == 16) hipLaunchKernelGGL(k_bias_part<16>, dim3(bnb), dim3(kThreads), 0, s, g, ldg, nvox, part);
    else if (co == 32) hipLaunchKernelGGL(k_bias_part<32>, dim3(bnb), dim3(kThreads), 0, s, g, ldg, nvox, part);
    else hipLaunchKernelGGL(k_bias_part<64>, dim3(bnb), dim3(kThreads), 0, s, g, ldg, nvox, part);
    hipLaunchKernelGGL(k_bias_reduce, dim3((co + kRedCols - 1) / kRedCols), dim3(kThreads), 0, s, part, bnb, co, db);
    return true;
}

Src src1(const Tensor& t, int up = 0) {
    Src s = {};
    s.a = t.p;
    s.ca = t.c;
    s.lda = t.c;
    s.upa = up;
    return s;
}
Src src2(const Tensor& a, const Tensor& b) {
    Src s = src1(a);
    s.b = b.p;
    s.cb = b.c;
    s.ldb = b.c;
    return s;
}

// Input of each layer, as the forward pass reads it.
Src layer_src(const cgd_unet_s* u, int l) {
    switch (l) {
        case E1A: return src1(u->x0);
        case E2A: return src1(u->p1);
        case E3A: return src1(u->p2);
        case U2: return src1(u->act[E3B], 1);
        case D2A: return src2(u->act[U2], u->act[E2B]);
        case U1: return src1(u->act[D2B], 1);
        case D1A: return src2(u->act[U1], u->act[E1B]);
        default: return src1(u->act[l - 1]);
    }
}

ConvArgs conv_args_at(const cgd_unet_s* u, int lev) {
    ConvArgs a = {};
    a.nx = u->n[lev][0];
    a.ny = u->n[lev][1];
    a.nz = u->n[lev][2];
    return a;
}

cgd_status forward(cgd_unet_s* u, const float* x, hipStream_t s) {
    const int64_t n0 = u->nvox[0];
    const int nb = grid_blocks(n0, kThreads, 1024);
    hipLaunchKernelGGL(k_sumsq_part, dim3(nb), dim3(kThreads), 0, s, x, n0, u->dpart);
    hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(kThreads), 0, s, u->dpart, nb, n0, u->sc);
    hipLaunchKernelGGL(k_prep_input, dim3(grid_blocks(n0)), dim3(kThreads), 0, s, x, u->sc, n0, u->x0.p);
    for (int l = 0; l < kLayers; ++l) {
        const Layer& L = u->L[l];
        if (l == E2A)
            hipLaunchKernelGGL(k_pool2, dim3(grid_blocks(u->nvox[1] * 2)), dim3(kThreads), 0, s, u->act[E1B].p, kBase,
                               u->n[0][0], u->n[0][1], u->n[0][2], u->p1.p);
        if (l == E3A)
            hipLaunchKernelGGL(k_pool2, dim3(grid_blocks(u->nvox[2] * 4)), dim3(kThreads), 0, s, u->act[E2B].p,
                               2 * kBase, u->n[1][0], u->n[1][1], u->n[1][2], u->p2.p);
        ConvArgs a = conv_args_at(u, L.lev);
        a.src = layer_src(u, l);
        a.w = L.wk;
        a.bias = u->params + L.b_off;
        a.out = u->act[l].p;
        a.ldo = L.co;
        a.relu = 1;
        if (!launch_conv(L.cc, L.co, L.np, a, s)) {
            set_error(std::string("unet: no convolution kernel for layer ") + L.name);
            return CGD_E_INVALID;
        }
    }
    return CGD_OK;
}

// One input-gradient convolution of layer l: out = conv(g, wd) masked by the
// ReLU pattern of the tensors given (mask_b may be null when mca == out channels).
void dgrad(cgd_unet_s* u, int l, const Tensor& g, int ldg, const Tensor& out, const Tensor* ma, int mca,
           const Tensor* mb, hipStream_t s) {
    const Layer& L = u->L[l];
    ConvArgs a = conv_args_at(u, L.lev);
    a.src = {};
    a.src.a = g.p;
    a.src.ca = L.co;
    a.src.lda = ldg;
    a.w = L.wd;
    a.out = out.p;
    a.ldo = out.c;
    if (ma) {
        a.mask_a = ma->p;
        a.mca = mca;
        a.ldma = ma->c;
        a.mask_b = mb ? mb->p : nullptr;
        a.ldmb = mb ? mb->c : 0;
    }
    launch_conv(L.ccd, L.ci_a + L.ci_b, L.npd, a, s);
}

void wgrad(cgd_unet_s* u, int l, const bf16* g, int ldg, hipStream_t s) {
    const Layer& L = u->L[l];
    launch_wgrad(L.cc, L.co, L.np, layer_src(u, l), g, ldg, u->n[L.lev][0], u->n[L.lev][1], u->n[L.lev][2], u->fpart,
                 u->grads + L.w_off, u->grads + L.b_off, s);
}

// Backward pass after forward(): gradients of the loss against `t` into u->grads.
void backward(cgd_unet_s* u, const float* x, const float* t, hipStream_t s) {
    const int64_t n0 = u->nvox[0];
    const int nb = grid_blocks(n0, kThreads, 1024);
    HeadArgs h = {};
    h.d1 = u->act[D1B].p;
    h.x = x;
    h.t = t;
    h.sc = u->sc;
    h.hw = u->params + u->head_off;
    h.gd1 = u->gd1.p;
    h.part = u->dpart;
    h.n = n0;
    hipLaunchKernelGGL(k_head, dim3(nb), dim3(kThreads), 0, s, h);
    hipLaunchKernelGGL(k_head_finish, dim3(kBase + 2), dim3(kThreads), 0, s, u->dpart, nb, n0, u->grads + u->head_off,
                       u->loss);

    Tensor* A = u->act;
    auto up_bwd = [&](const Tensor& gup, const Tensor& act, const Tensor& out, int lev) {
        hipLaunchKernelGGL(k_up_bwd, dim3(grid_blocks(u->nvox[lev] * act.c / 8)), dim3(kThreads), 0, s, gup.p, act.p,
                           act.c, u->n[lev][0], u->n[lev][1], u->n[lev][2], out.p);
    };
    auto pool_bwd = [&](const bf16* skip, int ldsk, const Tensor& gp, const Tensor& act, const Tensor& out, int lev) {
        hipLaunchKernelGGL(k_pool_bwd, dim3(grid_blocks(u->nvox[lev] * act.c / 8)), dim3(kThreads), 0, s, skip, ldsk,
                           gp.p, act.p, act.c, u->n[lev][0], u->n[lev][1], u->n[lev][2], out.p);
    };

    wgrad(u, D1B, u->gd1.p, kBase, s);
    dgrad(u, D1B, u->gd1, kBase, u->ga5, &A[D1A], kBase, nullptr, s);
    wgrad(u, D1A, u->ga5.p, kBase, s);
    dgrad(u, D1A, u->ga5, kBase, u->gc1, &A[U1], kBase, &A[E1B], s);  // [u1 | e1] channels
    wgrad(u, U1, u->gc1.p, 2 * kBase, s);                                // first 16 channels of gc1
    dgrad(u, U1, u->gc1, 2 * kBase, u->gq2, nullptr, 0, nullptr, s);
    up_bwd(u->gq2, A[D2B], u->gd2, 1);
    wgrad(u, D2B, u->gd2.p, 2 * kBase, s);
    dgrad(u, D2B, u->gd2, 2 * kBase, u->ga4, &A[D2A], 2 * kBase, nullptr, s);
    wgrad(u, D2A, u->ga4.p, 2 * kBase, s);
    dgrad(u, D2A, u->ga4, 2 * kBase, u->gc2, &A[U2], 2 * kBase, &A[E2B], s);  // [u2 | e2]
    wgrad(u, U2, u->gc2.p, 4 * kBase, s);
    dgrad(u, U2, u->gc2, 4 * kBase, u->gq3, nullptr, 0, nullptr, s);
    up_bwd(u->gq3, A[E3B], u->ge3, 2);
    wgrad(u, E3B, u->ge3.p, 4 * kBase, s);
    dgrad(u, E3B, u->ge3, 4 * kBase, u->ga3, &A[E3A], 4 * kBase, nullptr, s);
    wgrad(u, E3A, u->ga3.p, 4 * kBase, s);
    dgrad(u, E3A, u->ga3, 4 * kBase, u->gp2, nullptr, 0, nullptr, s);
    pool_bwd(u->gc2.p + 2 * kBase, 4 * kBase, u->gp2, A[E2B], u->ge2, 1);
    wgrad(u, E2B, u->ge2.p, 2 * kBase, s);
    dgrad(u, E2B, u->ge2, 2 * kBase, u->ga2, &A[E2A], 2 * kBase, nullptr, s);
    wgrad(u, E2A, u->ga2.p, 2 * kBase, s);
    dgrad(u, E2A, u->ga2, 2 * kBase, u->gp1, nullptr, 0, nullptr, s);
    pool_bwd(u->gc1.p + kBase, 2 * kBase, u->gp1, A[E1B], u->ge1, 0);
    wgrad(u, E1B, u->ge1.p, kBase, s);
    dgrad(u, E1B, u->ge1, kBase, u->ga1, &A[E1A], kBase, nullptr, s);
    wgrad(u, E1A, u->ga1.p, kBase, s);
}

void prep_weights(cgd_unet_s* u, hipStream_t s) {
    for (int l = 0; l < kLayers; ++l) {
        const Layer& L = u->L[l];
        const int ci = L.ci_a + L.ci_b;
        hipLaunchKernelGGL(k_prep_w, dim3(grid_blocks((int64_t)L.co * 27 * ci)), dim3(kThreads), 0, s,
                           u->params + L.w_off, ci, L.co, L.wk, L.cc, L.np, L.wd, L.ccd, L.npd);
    }
}

// splitmix64 + Box-Muller, for the initial weights (host).
struct HostRng {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    double normal() {
        const double u1 = uniform(), u2 = uniform();
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    }
};

struct DevGuard {
    int prev = -1;
    explicit DevGuard(int d) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != d) (void)hipSetDevice(d);
    }
    ~DevGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

cgd_status unet_guess(cgd_unet u, const float* x, float* y, hipStream_t s) {
    cgd_status rc = forward(u, x, s);
    if (rc != CGD_OK) return rc;
    HeadArgs h = {};
    h.d1 = u->act[D1B].p;
    h.x = x;
    h.sc = u->sc;
    h.hw = u->params + u->head_off;
    h.y = y;
    h.n = u->nvox[0];
    hipLaunchKernelGGL(k_head, dim3(grid_blocks(u->nvox[0], kThreads, 1024)), dim3(kThreads), 0, s, h);
    CGD_HIP_TRY(hipGetLastError());
    return CGD_OK;
}

bool unet_matches(cgd_unet u, int nx, int ny, int nz, int device) {
    return u && u->n[0][0] == nx && u->n[0][1] == ny && u->n[0][2] == nz && u->device == device;
}

}  // namespace unet
}  // namespace cgd

using namespace cgd;
using namespace cgd::unet;

extern "C" {

cgd_status cgd_unet_create(int32_t nx, int32_t ny, int32_t nz, uint64_t seed, cgd_unet* out) {
    if (!out) {
        set_error("cgd_unet_create: out is NULL");
        return CGD_E_INVALID;
    }
    *out = nullptr;
    if (nx < 4 || ny < 4 || nz < 4 || nx % 4 || ny % 4 || nz % 4 || (int64_t)nx * ny * nz > (int64_t)1 << 30) {
        set_error("cgd_unet_create: each grid size must be a positive multiple of 4 (and nx*ny*nz <= 2^30)");
        return CGD_E_INVALID;
    }
    auto* u = new (std::nothrow) cgd_unet_s();
    if (!u) return CGD_E_NOMEM;
    if (hipGetDevice(&u->device) != hipSuccess) {
        delete u;
        set_error("cgd_unet_create: no HIP device");
        return CGD_E_HIP;
    }
    for (int lev = 0; lev < 3; ++lev) {
        u->n[lev][0] = nx >> lev;
        u->n[lev][1] = ny >> lev;
        u->n[lev][2] = nz >> lev;
        u->nvox[lev] = (int64_t)u->n[lev][0] * u->n[lev][1] * u->n[lev][2];
    }
    const int C = kBase;
    const struct {
        const char* name;
        int ci_a, ci_b, co, lev, up;
    } spec[kLayers] = {{"e1a", 1, 0, C, 0, 0},         {"e1b", C, 0, C, 0, 0},
                       {"e2a", C, 0, 2 * C, 1, 0},     {"e2b", 2 * C, 0, 2 * C, 1, 0},
                       {"e3a", 2 * C, 0, 4 * C, 2, 0}, {"e3b", 4 * C, 0, 4 * C, 2, 0},
                       {"u2", 4 * C, 0, 2 * C, 1, 1},  {"d2a", 2 * C, 2 * C, 2 * C, 1, 0},
                       {"d2b", 2 * C, 0, 2 * C, 1, 0}, {"u1", 2 * C, 0, C, 0, 1},
                       {"d1a", C, C, C, 0, 0},         {"d1b", C, 0, C, 0, 0}};
    int64_t off = 0;
    size_t wbytes = 0;
    for (int l = 0; l < kLayers; ++l) {
        Layer& L = u->L[l];
        L.name = spec[l].name;
        L.ci_a = spec[l].ci_a;
        L.ci_b = spec[l].ci_b;
        L.co = spec[l].co;
        L.lev = spec[l].lev;
        L.up = spec[l].up;
        const int ci = L.ci_a + L.ci_b;
        L.w_off = off;
        off += (int64_t)L.co * 27 * ci;
        L.b_off = off;
        off += L.co;
        L.cc = cc_of(ci);
        L.np = L.cc == 1 ? 1 : ci / L.cc;
        L.ccd = l == E1A ? 0 : std::min(L.co, 32);
        L.npd = L.ccd ? L.co / L.ccd : 0;
        wbytes += (size_t)L.co * L.np * kt_of(L.cc) * L.cc * 2;
        if (L.ccd) wbytes += (size_t)ci * L.npd * kt_of(L.ccd) * L.ccd * 2;
    }
    u->head_off = off;
    off += C + 1;
    u->n_params = off;

    // activation and gradient tensors: (pointer, channels, level)
    struct TD {
        Tensor* t;
        int c, lev;
    } tds[] = {{&u->x0, 1, 0},          {&u->act[E1A], C, 0},     {&u->act[E1B], C, 0},     {&u->p1, C, 1},
               {&u->act[E2A], 2 * C, 1}, {&u->act[E2B], 2 * C, 1}, {&u->p2, 2 * C, 2},      {&u->act[E3A], 4 * C, 2},
               {&u->act[E3B], 4 * C, 2}, {&u->act[U2], 2 * C, 1},  {&u->act[D2A], 2 * C, 1}, {&u->act[D2B], 2 * C, 1},
               {&u->act[U1], C, 0},      {&u->act[D1A], C, 0},     {&u->act[D1B], C, 0},     {&u->gd1, C, 0},
               {&u->ga5, C, 0},          {&u->gc1, 2 * C, 0},      {&u->gq2, 2 * C, 0},      {&u->gd2, 2 * C, 1},
               {&u->ga4, 2 * C, 1},      {&u->gc2, 4 * C, 1},      {&u->gq3, 4 * C, 1},      {&u->ge3, 4 * C, 2},
               {&u->ga3, 4 * C, 2},      {&u->gp2, 2 * C, 2},      {&u->ge2, 2 * C, 1},      {&u->ga2, 2 * C, 1},
               {&u->gp1, C, 1},          {&u->ge1, C, 0},          {&u->ga1, C, 0}};
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t fpart = 0;
    for (int l = 0; l < kLayers; ++l) {
        const Layer& L = u->L[l];
        fpart = std::max(fpart, wgrad_part_floats(u->n[L.lev][0], u->n[L.lev][1], u->n[L.lev][2], L.cc, L.co, L.np));
    }
    fpart = std::max<size_t>(fpart, 1024 * 64);
    u->fpart_floats = fpart;
    size_t bytes = 4 * al((size_t)off * 4) + al(2 * 4) + al(8) + al(4096 * 8 * (kBase + 2)) + al(fpart * 4) + al(wbytes);
    for (auto& td : tds) bytes += al((size_t)u->nvox[td.lev] * td.c * 2);
    if (hipMalloc(&u->arena, bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete u;
        set_error("cgd_unet_create: device allocation of " + std::to_string(bytes) + " bytes failed");
        return CGD_E_NOMEM;
    }
    char* p = static_cast<char*>(u->arena);
    auto take = [&](size_t b) {
        char* r = p;
        p += al(b);
        return r;
    };
    u->params = reinterpret_cast<float*>(take((size_t)off * 4));
    u->grads = reinterpret_cast<float*>(take((size_t)off * 4));
    u->adam_m = reinterpret_cast<float*>(take((size_t)off * 4));
    u->adam_v = reinterpret_cast<float*>(take((size_t)off * 4));
    u->sc = reinterpret_cast<float*>(take(2 * 4));
    u->loss = reinterpret_cast<double*>(take(8));
    u->dpart = reinterpret_cast<double*>(take(4096 * 8 * (kBase + 2)));
    u->fpart = reinterpret_cast<float*>(take(fpart * 4));
    char* wbase = take(wbytes);
    for (int l = 0; l < kLayers; ++l) {
        Layer& L = u->L[l];
        const int ci = L.ci_a + L.ci_b;
        L.wk = reinterpret_cast<bf16*>(wbase);
        wbase += (size_t)L.co * L.np * kt_of(L.cc) * L.cc * 2;
        if (L.ccd) {
            L.wd = reinterpret_cast<bf16*>(wbase);
            wbase += (size_t)ci * L.npd * kt_of(L.ccd) * L.ccd * 2;
        }
    }
    for (auto& td : tds) {
        td.t->p = reinterpret_cast<bf16*>(take((size_t)u->nvox[td.lev] * td.c * 2));
        td.t->c = td.c;
        td.t->lev = td.lev;
    }
    // zero everything once: padding taps of the kernel layouts, Adam moments
    if (hipMemset(u->arena, 0, bytes) != hipSuccess) {
        (void)hipFree(u->arena);
        delete u;
        set_error("cgd_unet_create: hipMemset failed");
        return CGD_E_HIP;
    }
    // He-normal weights, zero biases and head: the untrained net is x -> x
    std::vector<float> h(off, 0.f);
    HostRng rng{seed};
    for (int l = 0; l < kLayers; ++l) {
        const Layer& L = u->L[l];
        const int ci = L.ci_a + L.ci_b;
        const double sd = std::sqrt(2.0 / (27.0 * ci));
        for (int64_t i = 0; i < (int64_t)L.co * 27 * ci; ++i) h[L.w_off + i] = (float)(sd * rng.normal());
    }
    cgd_status rc = cgd_unet_set_params(u, h.data(), off);
    if (rc != CGD_OK) {
        cgd_unet_destroy(u);
        return rc;
    }
    *out = u;
    return CGD_OK;
}

void cgd_unet_destroy(cgd_unet u) {
    if (!u) return;
    DevGuard dg(u->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(u->arena);
    delete u;
}

int64_t cgd_unet_num_params(cgd_unet u) { return u ? u->n_params : 0; }

cgd_status cgd_unet_set_params(cgd_unet u, const float* host, int64_t n) {
    if (!u || !host || n != u->n_params) {
        set_error("cgd_unet_set_params: NULL argument or n != cgd_unet_num_params");
        return CGD_E_INVALID;
    }
    DevGuard dg(u->device);
    CGD_HIP_TRY(hipDeviceSynchronize());
    CGD_HIP_TRY(hipMemcpy(u->params, host, (size_t)n * 4, hipMemcpyHostToDevice));
    CGD_HIP_TRY(hipMemset(u->adam_m, 0, (size_t)n * 4));
    CGD_HIP_TRY(hipMemset(u->adam_v, 0, (size_t)n * 4));
    u->adam_t = 0;
    prep_weights(u, nullptr);
    CGD_HIP_TRY(hipGetLastError());
    CGD_HIP_TRY(hipDeviceSynchronize());
    return CGD_OK;
}

cgd_status cgd_unet_get_params(cgd_unet u, float* host, int64_t n) {
    if (!u || !host || n != u->n_params) {
        set_error("cgd_unet_get_params: NULL argument or n != cgd_unet_num_params");
        return CGD_E_INVALID;
    }
    DevGuard dg(u->device);
    CGD_HIP_TRY(hipDeviceSynchronize());
    CGD_HIP_TRY(hipMemcpy(host, u->params, (size_t)n * 4, hipMemcpyDeviceToHost));
    return CGD_OK;
}

cgd_status cgd_unet_get_grads(cgd_unet u, float* host, int64_t n) {
    if (!u || !host || n != u->n_params) {
        set_error("cgd_unet_get_grads: NULL argument or n != cgd_unet_num_params");
        return CGD_E_INVALID;
    }
    DevGuard dg(u->device);
    CGD_HIP_TRY(hipDeviceSynchronize());
    CGD_HIP_TRY(hipMemcpy(host, u->grads, (size_t)n * 4, hipMemcpyDeviceToHost));
    return CGD_OK;
}

cgd_status cgd_unet_forward(cgd_unet u, const float* x, float* y, void* stream) {
    if (!u || !x || !y) {
        set_error("cgd_unet_forward: NULL argument");
        return CGD_E_INVALID;
    }
    DevGuard dg(u->device);
    return unet_guess(u, x, y, static_cast<hipStream_t>(stream));
}

cgd_status cgd_unet_loss_grad(cgd_unet u, const float* x, const float* target, double* loss, void* stream) {
    if (!u || !x || !target) {
        set_error("cgd_unet_loss_grad: NULL argument");
        return CGD_E_INVALID;
    }
    DevGuard dg(u->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    cgd_status rc = forward(u, x, s);
    if (rc != CGD_OK) return rc;
    backward(u, x, target, s);
    CGD_HIP_TRY(hipGetLastError());
    if (loss) {
        CGD_HIP_TRY(hipMemcpyAsync(loss, u->loss, 8, hipMemcpyDeviceToHost, s));
        CGD_HIP_TRY(hipStreamSynchronize(s));
    }
    return CGD_OK;
}

cgd_status cgd_unet_train_step(cgd_unet u, const float* x, const float* target, double lr, double* loss,
                               void* stream) {
    if (!u || !x || !target || !(lr > 0.0) || !std::isfinite(lr)) {
        set_error("cgd_unet_train_step: NULL argument or lr not positive");
        return CGD_E_INVALID;
    }
    DevGuard dg(u->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    cgd_status rc = forward(u, x, s);
    if (rc != CGD_OK) return rc;
    backward(u, x, target, s);
    u->adam_t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float bc1 = (float)(1.0 - std::pow(b1, (double)u->adam_t));
    const float bc2 = (float)(1.0 - std::pow(b2, (double)u->adam_t));
    hipLaunchKernelGGL(k_adam, dim3(grid_blocks(u->n_params)), dim3(kThreads), 0, s, u->params, u->adam_m, u->adam_v,
                       u->grads, u->n_params, (float)lr, (float)b1, (float)b2, 1e-8f, bc1, bc2);
    prep_weights(u, s);
    CGD_HIP_TRY(hipGetLastError());
    if (loss) {
        CGD_HIP_TRY(hipMemcpyAsync(loss, u->loss, 8, hipMemcpyDeviceToHost, s));
        CGD_HIP_TRY(hipStreamSynchronize(s));
    }
    return CGD_OK;
}

// ---- single convolutions on caller buffers (bfloat16 passed as uint16_t)

static bool conv_shape_ok(int32_t nx, int32_t ny, int32_t nz, int32_t ci, int32_t co) {
    const bool ci_ok = ci == 1 || ci == 16 || ci == 32 || ci == 64;
    const bool co_ok = co == 16 || co == 32 || co == 64;
    return nx > 0 && ny > 0 && nz > 0 && ci_ok && co_ok && (int64_t)nx * ny * nz <= ((int64_t)1 << 30);
}

cgd_status cgd_conv3_forward(int32_t nx, int32_t ny, int32_t nz, int32_t ci, int32_t co, const uint16_t* x,
                             const uint16_t* w, const float* bias, int32_t relu, uint16_t* y, void* stream) {
    if (!x || !w || !y || !conv_shape_ok(nx, ny, nz, ci, co)) {
        set_error("cgd_conv3_forward: NULL argument or unsupported shape (ci in {1,16,32,64}, co in {16,32,64})");
        return CGD_E_INVALID;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int cc = cc_of(ci), np = cc == 1 ? 1 : ci / cc;
    const size_t wkb = (size_t)co * np * kt_of(cc) * cc * 2;
    void* wk = nullptr;
    CGD_HIP_TRY(hipMalloc(&wk, wkb + (size_t)co * 27 * ci * 4));
    float* w32 = reinterpret_cast<float*>(static_cast<char*>(wk) + wkb);
    cgd_status rc = CGD_OK;
    do {
        if (hipMemsetAsync(wk, 0, wkb, s) != hipSuccess) { rc = CGD_E_HIP; break; }
        // bf16 -> f32 is exact; the prep kernel rounds back to the same bits
        std::vector<uint16_t> hw((size_t)co * 27 * ci);
        std::vector<float> hf(hw.size());
        if (hipMemcpyAsync(hw.data(), w, hw.size() * 2, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) { rc = CGD_E_HIP; break; }
        for (size_t i = 0; i < hw.size(); ++i) {
            uint32_t b = (uint32_t)hw[i] << 16;
            std::memcpy(&hf[i], &b, 4);
        }
        if (hipMemcpyAsync(w32, hf.data(), hf.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess) { rc = CGD_E_HIP; break; }
        hipLaunchKernelGGL(k_prep_w, dim3(grid_blocks((int64_t)co * 27 * ci)), dim3(kThreads), 0, s, w32, ci, co,
                           reinterpret_cast<bf16*>(wk), cc, np, (bf16*)nullptr, 16, 1);
        ConvArgs a = {};
        a.src.a = reinterpret_cast<const bf16*>(x);
        a.src.ca = ci;
        a.src.lda = ci;
        a.w = reinterpret_cast<const bf16*>(wk);
        a.bias = bias;
        a.out = reinterpret_cast<bf16*>(y);
        a.ldo = co;
        a.relu = relu ? 1 : 0;
        a.nx = nx;
        a.ny = ny;
        a.nz = nz;
        if (!launch_conv(cc, co, np, a, s)) { rc = CGD_E_INVALID; break; }
        if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess) rc = CGD_E_HIP;
    } while (0);
    (void)hipFree(wk);
    if (rc == CGD_E_HIP) set_error("cgd_conv3_forward: HIP error");
    return rc;
}

cgd_status cgd_conv3_dgrad(int32_t nx, int32_t ny, int32_t nz, int32_t ci, int32_t co, const uint16_t* g,
                           const uint16_t* w, uint16_t* dx, void* stream) {
    if (!g || !w || !dx || ci == 1 || !conv_shape_ok(nx, ny, nz, ci, co)) {
        set_error("cgd_conv3_dgrad: NULL argument or unsupported shape (ci in {16,32,64}, co in {16,32,64})");
        return CGD_E_INVALID;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int ccd = std::min(co, 32), npd = co / ccd;
    const int cc = cc_of(ci), np = ci / cc;
    const size_t wkb = (size_t)co * np * kt_of(cc) * cc * 2;
    const size_t wdb = (size_t)ci * npd * kt_of(ccd) * ccd * 2;
    void* buf = nullptr;
    CGD_HIP_TRY(hipMalloc(&buf, wkb + wdb + (size_t)co * 27 * ci * 4));
    bf16* wk = reinterpret_cast<bf16*>(buf);
    bf16* wd = reinterpret_cast<bf16*>(static_cast<char*>(buf) + wkb);
    float* w32 = reinterpret_cast<float*>(static_cast<char*>(buf) + wkb + wdb);
    cgd_status rc = CGD_OK;
    do {
        if (hipMemsetAsync(buf, 0, wkb + wdb, s) != hipSuccess) { rc = CGD_E_HIP; break; }
        std::vector<uint16_t> hw((size_t)co * 27 * ci);
        std::vector<float> hf(hw.size());
        if (hipMemcpyAsync(hw.data(), w, hw.size() * 2, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) { rc = CGD_E_HIP; break; }
        for (size_t i = 0; i < hw.size(); ++i) {
            uint32_t b = (uint32_t)hw[i] << 16;
            std::memcpy(&hf[i], &b, 4);
        }
        if (hipMemcpyAsync(w32, hf.data(), hf.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess) { rc = CGD_E_HIP; break; }
        hipLaunchKernelGGL(k_prep_w, dim3(grid_blocks((int64_t)co * 27 * ci)), dim3(kThreads), 0, s, w32, ci, co, wk,
                           cc, np, wd, ccd, npd);
        ConvArgs a = {};
        a.src.a = reinterpret_cast<const bf16*>(g);
        a.src.ca = co;
        a.src.lda = co;
        a.w = wd;
        a.out = reinterpret_cast<bf16*>(dx);
        a.ldo = ci;
        a.nx = nx;
        a.ny = ny;
        a.nz = nz;
        if (!launch_conv(ccd, ci, npd, a, s)) { rc = CGD_E_INVALID; break; }
        if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess) rc = CGD_E_HIP;
    } while (0);
    (void)hipFree(buf);
    if (rc == CGD_E_HIP) set_error("cgd_conv3_dgrad: HIP error");
    return rc;
}

cgd_status cgd_conv3_wgrad(int32_t nx, int32_t ny, int32_t nz, int32_t ci, int32_t co, const uint16_t* x,
                           const uint16_t* g, float* dw, float* db, void* stream) {
    if (!x || !g || !dw || !db || !conv_shape_ok(nx, ny, nz, ci, co)) {
        set_error("cgd_conv3_wgrad: NULL argument or unsupported shape (ci in {1,16,32,64}, co in {16,32,64})");
        return CGD_E_INVALID;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int cc = cc_of(ci), np = cc == 1 ? 1 : ci / cc;
    const size_t pf = std::max<size_t>(wgrad_part_floats(nx, ny, nz, cc, co, np), 1024 * 64);
    void* part = nullptr;
    CGD_HIP_TRY(hipMalloc(&part, pf * 4));
    Src src = {};
    src.a = reinterpret_cast<const bf16*>(x);
    src.ca = ci;
    src.lda = ci;
    cgd_status rc = CGD_OK;
    if (!launch_wgrad(cc, co, np, src, reinterpret_cast<const bf16*>(g), co, nx, ny, nz, static_cast<float*>(part), dw,
                      db, s))
        rc = CGD_E_INVALID;
    else if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess)
        rc = CGD_E_HIP;
    (void)hipFree(part);
    if (rc == CGD_E_HIP) set_error("cgd_conv3_wgrad: HIP error");
    return rc;
}

}  // extern "C"
