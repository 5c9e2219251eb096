// Pieces shared by the hex (stencil) and tet (CSR) conjugate-gradient solvers.
#pragma once

#include <algorithm>
#include <functional>
#include <string>
#include <vector>

#include "cgd_internal.h"

namespace cgd {

constexpr int kCgWaves = 4;
constexpr int kCgBlock = 64 * kCgWaves;

// Layout of the small region at the start of a mesh workspace (bytes).
constexpr size_t kOffState = 0;                   // CgField[CGD_MAX_FIELDS]
constexpr size_t kOffNdone = 4096;                // int[2]: fields finished, largest stopping iteration
constexpr size_t kOffIters = 8192;                // int32 [STEPS][FIELDS]
constexpr size_t kOffRelres = kOffIters + 4096;   // double [STEPS][FIELDS]
constexpr size_t kOffStatus = kOffRelres + 8192;  // int32 [STEPS][FIELDS]
constexpr size_t kOffSums = kOffStatus + 4096;    // double [2][FIELDS]
constexpr size_t kOffFallback = kOffSums + 4096;  // int32 [STEPS][FIELDS]: learned guess rejected
constexpr size_t kOffDeposit = 48 * 1024;         // DepositInfo
constexpr size_t kSmallFixed = 64 * 1024;         // partial sums follow

// Layout of the pinned host buffer (bytes).
constexpr size_t kPinFlags = 0;  // int[2][2]: read-back slot, (fields finished, largest stopping iteration)
constexpr size_t kPinIters = 4096;
constexpr size_t kPinRelres = kPinIters + 4096;
constexpr size_t kPinStatus = kPinRelres + 8192;
constexpr size_t kPinSums = kPinStatus + 4096;
constexpr size_t kPinDeposit = kPinSums + 4096;
constexpr size_t kPinFallback = kPinDeposit + 4096;
constexpr size_t kPinBytes = kPinFallback + 4096;

// Convergence bookkeeping written by the first block of a sweep.
struct CgCtl {
    CgField* st;       // [F]
    int* ndone;
    int* host_flags;   // nullable: the launch that ends a read-back chunk copies ndone[0..1] here (pinned host memory)
    int32_t* iters;    // [CGD_MAX_STEPS][CGD_MAX_FIELDS]
    double* relres;
    int32_t* status;
    double rtol2;
    int step;
};

#ifdef __HIPCC__
// The last sweep of a read-back chunk hands the host the finished-field count
// and the largest stopping iteration (written by the convergence tests of
// earlier launches), in place of a device-to-host copy after it.  Called
// before any early return, so a launch whose fields are all done still posts.
__device__ inline void post_ndone(const CgCtl& c) {
    if (c.host_flags && blockIdx.x == 0 && threadIdx.x == 0) {
        const int n0 = __atomic_load_n(c.ndone, __ATOMIC_RELAXED);
        const int n1 = __atomic_load_n(c.ndone + 1, __ATOMIC_RELAXED);
        c.host_flags[0] = n0;
        c.host_flags[1] = n1;
    }
}

// Sum of n float64 values by a block of NT threads in one fixed order
// (thread t adds t, t + NT, ...; then a fixed shuffle tree and a fixed sum
// over the NT / 64 waves).  Every thread of the block returns the same value,
// bit for bit, in every block; the order depends on NT.
template <int NT>
__device__ inline double block_sum_nt(const double* p, int n, double* sh) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) s += p[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) t += sh[i];
    __syncthreads();
    return t;
}

// The same by a block of kCgBlock threads.
__device__ inline double block_sum_fixed(const double* p, int n, double* sh) {
    return block_sum_nt<kCgBlock>(p, n, sh);
}

// Block-wide float64 sum in fixed order; the result is valid in thread 0.
__device__ inline double block_reduce_fixed(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kCgWaves; ++i) t += sh[i];
    }
    __syncthreads();
    return t;
}

__device__ inline void finish_field(const CgCtl& c, int f, int status) {
    c.st[f].status = status;
    c.st[f].done = 1;
    c.status[c.step * CGD_MAX_FIELDS + f] = status;
    atomicAdd(c.ndone, 1);
}

// Records iteration k's residual and, when it meets the tolerance or is not
// finite, stops the field.  Returns true when the field stops.
__device__ inline bool check_stop(const CgCtl& c, int f, int k, double rrk, double bb, bool lead) {
    const bool broken = !isfinite(rrk) || !isfinite(bb);
    const bool conv = !broken && rrk <= c.rtol2 * bb;
    if (lead) {
        c.iters[c.step * CGD_MAX_FIELDS + f] = k;
        c.relres[c.step * CGD_MAX_FIELDS + f] = bb > 0.0 ? sqrt(rrk / bb) : 0.0;
        if (broken || conv) {
            atomicMax(c.ndone + 1, k);
            finish_field(c, f, broken ? CGD_E_BREAKDOWN : CGD_OK);
        }
    }
    return broken || conv;
}

__global__ void k_cg_step_init(CgField* st, int F, int* ndone, int32_t* status_row);
// Settles the fields still running after k_end iterations, from the r.r
// partial sums of the last sweep (rr_part: [F][slot stride] with stride):
// the test that iteration k_end's first kernel would have made, summed in
// its order (NT: that kernel's block size; launch with NT threads), and
// CGD_NOT_CONVERGED where it fails.  Instantiated for NT = 256 and 1024.
template <int NT>
__global__ void k_cg_step_end(CgCtl c, const double* rr_part, size_t field_stride, int bpf, int k_end);

// Crank-Nicolson from its half-step solve (Section 5.1): with
// (M + dtau/2 K) y = M e, the step (M + dtau/2 K) e' = (M - dtau/2 K) e has
// e' = 2 y - e.  Overwrites y [n] with 2 y - e (one rounding per element).
void cn_extrapolate(float* y, const float* e, int64_t n, hipStream_t s);
#endif

// Host: coefficients of the polynomial preconditioner M = c0 I + c1 A + c2 A^2
// of degree 1 or 2 for the hex operator A = I + sum_a c_a L_a, whose
// spectrum lies in [1, lmax], lmax = 1 + 4 sum_a c_a (the constant field
// gives exactly 1).  1 - lambda M(lambda) is the Chebyshev polynomial
// T_{deg+1} scaled to that interval, so the preconditioned condition number
// is (1 + e) / (1 - e) with e = 1 / T_{deg+1}((lmax + 1) / (lmax - 1)).
void poly_precond_coeffs(double cx, double cy, double cz, int deg, float* c0, float* c1, float* c2);
// The same polynomial for any degree 1..6: c[0..deg] (float64).
void poly_precond_coeffs_n(double cx, double cy, double cz, int deg, double* c);
// The even-degree polynomial of poly_precond_coeffs_n as a product of
// quadratic factors: p(l) = scale prod_k g_k (l^2 + s_k l + q_k), k < deg / 2,
// each g_k scaling its factor to at most 1 on the spectrum [1, 1 + 4 (cx +
// cy + cz)].  Returns the number of factors.  The roots are in closed form
// (those of T_{deg+1}(sig(l)) = T_{deg+1}(sig(0)) other than l = 0).
int poly_precond_quadratics(double cx, double cy, double cz, int deg, double* s, double* q, double* g,
                            double* scale);
// The same two for an operator whose spectrum lies in [lmin, lmax].
void poly_precond_coeffs_iv(double lmin, double lmax, int deg, double* c);
int poly_precond_quadratics_iv(double lmin, double lmax, int deg, double* s, double* q, double* g, double* scale);

// Host: enqueues iterations through `enqueue(it)` until the device reports
// all F fields stopped (read back one chunk late, so the device always has
// queued work) or max_iter iterations are queued.  The first chunk runs to
// the iteration at which the previous solve on this mesh stopped
// (m->cg_hint) and the next holds one iteration, so a solve that stops where
// the last one did leaves one iteration of empty launches; later chunks, and
// every chunk before a first solve, hold `chunk` iterations.  The stopping
// iteration read back becomes the new hint.  Returns the index of the next
// iteration that would have been enqueued.
cgd_status cg_lookahead_loop(cgd_mesh m, int F, int it0, int max_iter, int chunk, const int* d_ndone,
                             hipStream_t s, const std::function<void(int, int*)>& enqueue, int* it_end);

// Host: after the steps, copies statuses / iterations / residuals back,
// fills `out`, drops timing pairs of launches that found nothing to do, and
// returns the worst status.  warm: the steps were seeded by the learned
// guess, whose rejections (kOffFallback) are counted and reported as
// CGD_WARMSTART_FALLBACK when nothing worse happened.
cgd_status cg_finish_call(cgd_mesh m, int F, int n_steps, double vol_scale, hipStream_t s,
                          cgd_solve_stats* out, bool warm = false);

}  // namespace cgd
