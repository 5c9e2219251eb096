// Shared CG bookkeeping kernels and host loops (see cg_common.h).
#include <algorithm>
#include <cmath>

#include "cg_common.h"

namespace cgd {

__global__ void k_cg_step_init(CgField* st, int F, int* ndone, int32_t* status_row) {
    int f = threadIdx.x;
    if (f < F) {
        CgField s = {};
        s.status = CGD_OK;
        st[f] = s;
        status_row[f] = CGD_OK;
    }
    if (threadIdx.x == 0) {
        ndone[0] = 0;
        ndone[1] = 0;
    }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_cg_step_end(CgCtl c, const double* rr_part, size_t field_stride, int bpf,
                                                   int k_end) {
    const int f = blockIdx.x;
    CgField* stf = c.st + f;
    if (stf->done) return;
    __shared__ double sh[NT / 64];
    const double rrk = block_sum_nt<NT>(rr_part + (size_t)f * field_stride, bpf, sh);
    if (threadIdx.x != 0) return;
    if (!check_stop(c, f, k_end, rrk, stf->bb, true)) finish_field(c, f, CGD_NOT_CONVERGED);
}
template __global__ void k_cg_step_end<kCgBlock>(CgCtl, const double*, size_t, int, int);
template __global__ void k_cg_step_end<1024>(CgCtl, const double*, size_t, int, int);

__global__ __launch_bounds__(kCgBlock) void k_cn_extrapolate(float* __restrict__ y, const float* __restrict__ e,
                                                            int64_t n) {
    const int64_t n4 = n / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((reinterpret_cast<uintptr_t>(y) | reinterpret_cast<uintptr_t>(e)) % 16 == 0) {
        float4* y4 = reinterpret_cast<float4*>(y);
        const float4* e4 = reinterpret_cast<const float4*>(e);
        for (int64_t k = i; k < n4; k += stride) {
            float4 a = y4[k];
            const float4 b = e4[k];
            a.x = fmaf(2.f, a.x, -b.x);
            a.y = fmaf(2.f, a.y, -b.y);
            a.z = fmaf(2.f, a.z, -b.z);
            a.w = fmaf(2.f, a.w, -b.w);
            y4[k] = a;
        }
        const int64_t t = 4 * n4 + i;  // the at most 3 elements past the last whole float4
        if (t < n) y[t] = fmaf(2.f, y[t], -e[t]);
        return;
    }
    for (int64_t k = i; k < n; k += stride) y[k] = fmaf(2.f, y[k], -e[k]);
}

void cn_extrapolate(float* y, const float* e, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    const int64_t blocks = std::min<int64_t>(4096, (n / 4 + kCgBlock - 1) / kCgBlock + 1);
    hipLaunchKernelGGL(k_cn_extrapolate, dim3((unsigned)blocks), dim3(kCgBlock), 0, s, y, e, n);
}

__global__ __launch_bounds__(kCgBlock) void k_velocity_from_momentum(int64_t cells, int n_comp,
                                                                    const float* __restrict__ eps,
                                                                    float* __restrict__ mom, float eps_min) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < cells; k += stride) {
        const float e = eps[k];
        const bool ok = e > eps_min;
        for (int c = 0; c < n_comp; ++c) {
            float* m = mom + (size_t)c * cells + k;
            *m = ok ? *m / e : 0.f;
        }
    }
}

void velocity_from_momentum(int64_t cells, int n_comp, const float* eps, float* mom, float eps_min,
                            hipStream_t s) {
    if (cells <= 0) return;
    const int64_t blocks = std::min<int64_t>(8192, (cells + kCgBlock - 1) / kCgBlock);
    hipLaunchKernelGGL(k_velocity_from_momentum, dim3((unsigned)blocks), dim3(kCgBlock), 0, s, cells, n_comp, eps,
                       mom, eps_min);
}

void poly_precond_coeffs(double cx, double cy, double cz, int deg, float* c0, float* c1, float* c2) {
    // with s = lmax + 1 and d = lmax - 1 (finite as d -> 0, where M tends to a
    // multiple of the identity):
    //   degree 1 (T_2): c0 = 8 s / (2 s^2 - d^2), c1 = -8 / (2 s^2 - d^2)
    //   degree 2 (T_3): c0 = 2 (12 s^2 - 3 d^2) / (4 s^3 - 3 s d^2),
    //                   c1 = -48 / (4 s^2 - 3 d^2), c2 = 32 / (4 s^3 - 3 s d^2)
    const double lmax = 1.0 + 4.0 * (cx + cy + cz);
    const double sp = lmax + 1.0, dm = lmax - 1.0;
    if (deg == 1) {
        const double den = 2.0 * sp * sp - dm * dm;
        *c0 = (float)(8.0 * sp / den);
        *c1 = (float)(-8.0 / den);
        *c2 = 0.f;
    } else {
        const double den3 = 4.0 * sp * sp * sp - 3.0 * sp * dm * dm;
        *c0 = (float)(2.0 * (12.0 * sp * sp - 3.0 * dm * dm) / den3);
        *c1 = (float)(-48.0 / (4.0 * sp * sp - 3.0 * dm * dm));
        *c2 = (float)(32.0 / den3);
    }
}

void poly_precond_coeffs_n(double cx, double cy, double cz, int deg, double* c) {
    poly_precond_coeffs_iv(1.0, 1.0 + 4.0 * (cx + cy + cz), deg, c);
}

void poly_precond_coeffs_iv(double lmin, double lmax, int deg, double* c) {
    // p(l) = (1 - T_m(sig(l)) / T_m(sig(0))) / l with m = deg + 1 and
    // sig(l) = (s - 2 l) / d, s = lmax + lmin, d = lmax - lmin, built from
    // T_{n+1} = 2 sig T_n - T_{n-1} on monomial coefficient arrays in l.
    constexpr int kMax = 8;
    const double sp = lmax + lmin, dm = std::max(lmax - lmin, 1e-12 * sp);
    const int m = std::min(deg, kMax - 2) + 1;
    double t0[kMax + 1] = {1.0}, t1[kMax + 1] = {sp / dm, -2.0 / dm};
    for (int n = 1; n < m; ++n) {
        double t2[kMax + 1] = {0.0};
        for (int j = 0; j <= n; ++j) {
            t2[j] += 2.0 * (sp / dm) * t1[j];
            t2[j + 1] += 2.0 * (-2.0 / dm) * t1[j];
        }
        for (int j = 0; j <= n - 1; ++j) t2[j] -= t0[j];
        for (int j = 0; j <= kMax; ++j) {
            t0[j] = t1[j];
            t1[j] = t2[j];
        }
    }
    // t1 = T_m(sig(l)); T_m(sig(0)) = t1[0]; 1 - t1 / t1[0] has no constant term
    for (int j = 0; j < m; ++j) c[j] = -t1[j + 1] / t1[0];
}

int poly_precond_quadratics(double cx, double cy, double cz, int deg, double* s, double* q, double* g,
                            double* scale) {
    return poly_precond_quadratics_iv(1.0, 1.0 + 4.0 * (cx + cy + cz), deg, s, q, g, scale);
}

int poly_precond_quadratics_iv(double lmin, double lmax, int deg, double* s, double* q, double* g, double* scale) {
    // p(l) = lead prod_k (l^2 + s_k l + q_k): the roots of p are the l != 0
    // with T_n(sig(l)) = T_n(sig(0)), n = deg + 1, i.e. sig = cosh(theta + 2 pi i k / n),
    // theta = acosh(sig(0)), k = 1 .. deg, in conjugate pairs (k, n - k);
    // l = (sp - sig dm) / 2.  lead is the l^deg coefficient of
    // -(T_n(sig(l)) - T_n(sig(0))) / (T_n(sig(0)) l): -2^(n-1) (-2 / dm)^n / cosh(n theta).
    const double sp = lmax + lmin, dm = std::max(lmax - lmin, 1e-12 * sp);
    const int m = deg & ~1, n = m + 1;
    const double th = std::acosh(sp / dm);
    double lead = -std::pow(2.0, n - 1) * std::pow(-2.0 / dm, n) / std::cosh(n * th);
    const double kPi = 3.14159265358979323846;
    for (int k = 1; k <= m / 2; ++k) {
        const double a = 2.0 * kPi * k / n;
        // sig = cosh(th) cos(a) + i sinh(th) sin(a)
        const double sr = std::cosh(th) * std::cos(a), si = std::sinh(th) * std::sin(a);
        const double lr = (sp - sr * dm) / 2.0, li = -si * dm / 2.0;
        s[k - 1] = -2.0 * lr;
        q[k - 1] = lr * lr + li * li;
        // the factor is positive and convex on the spectrum [lmin, lmax]: its
        // maximum there is at an end point
        const double f1 = lmin * lmin + s[k - 1] * lmin + q[k - 1], f2 = lmax * lmax + s[k - 1] * lmax + q[k - 1];
        g[k - 1] = 1.0 / std::max(f1, f2);
        lead /= g[k - 1];
    }
    *scale = lead;
    return m / 2;
}

cgd_status cg_lookahead_loop(cgd_mesh m, int F, int it0, int max_iter, int chunk, const int* d_ndone,
                             hipStream_t s, const std::function<void(int, int*)>& enqueue, int* it_end) {
    int* pinned_flags = reinterpret_cast<int*>(static_cast<char*>(m->pinned) + kPinFlags);
    int it = it0;
    int slot = 0;
    bool have_prev = false;
    chunk = std::max(1, chunk);
    const bool hinted = m->cg_hint >= it0;
    for (int n = 0;; ++n) {
        int size = chunk;
        if (hinted && n == 0) size = m->cg_hint - it0 + 1;
        else if (hinted && n == 1) size = 1;
        const int todo = std::min(size, max_iter - it);
        // the chunk's last iteration posts ndone to this slot itself
        for (int c = 0; c < todo; ++c, ++it) enqueue(it, c + 1 == todo ? &pinned_flags[2 * slot] : nullptr);
        if (todo <= 0)
            CGD_HIP_TRY(hipMemcpyAsync(&pinned_flags[2 * slot], d_ndone, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
        CGD_HIP_TRY(hipEventRecord(m->ev[slot], s));
        if (have_prev) {
            CGD_HIP_TRY(hipEventSynchronize(m->ev[slot ^ 1]));
            if (pinned_flags[2 * (slot ^ 1)] >= F) {
                m->cg_hint = pinned_flags[2 * (slot ^ 1) + 1];
                break;
            }
        }
        if (it >= max_iter) {
            CGD_HIP_TRY(hipEventSynchronize(m->ev[slot]));
            break;
        }
        have_prev = true;
        slot ^= 1;
    }
    *it_end = it;
    return CGD_OK;
}

cgd_status cg_finish_call(cgd_mesh m, int F, int n_steps, double vol_scale, hipStream_t s,
                          cgd_solve_stats* out, bool warm) {
    char* base = static_cast<char*>(m->ws.ptr);
    char* pin = static_cast<char*>(m->pinned);
    int32_t* h_iters = reinterpret_cast<int32_t*>(pin + kPinIters);
    double* h_rel = reinterpret_cast<double*>(pin + kPinRelres);
    int32_t* h_status = reinterpret_cast<int32_t*>(pin + kPinStatus);
    double* h_sums = reinterpret_cast<double*>(pin + kPinSums);
    CGD_HIP_TRY(hipGetLastError());
    CGD_HIP_TRY(hipMemcpyAsync(h_status, base + kOffStatus, 4096, hipMemcpyDeviceToHost, s));
    CGD_HIP_TRY(hipMemcpyAsync(h_iters, base + kOffIters, 4096, hipMemcpyDeviceToHost, s));
    int32_t* h_fb = reinterpret_cast<int32_t*>(pin + kPinFallback);
    if (warm) CGD_HIP_TRY(hipMemcpyAsync(h_fb, base + kOffFallback, 4096, hipMemcpyDeviceToHost, s));
    if (out) {
        CGD_HIP_TRY(hipMemcpyAsync(h_rel, base + kOffRelres, 8192, hipMemcpyDeviceToHost, s));
        CGD_HIP_TRY(hipMemcpyAsync(h_sums, base + kOffSums, 2 * CGD_MAX_FIELDS * sizeof(double),
                                   hipMemcpyDeviceToHost, s));
    }
    CGD_HIP_TRY(hipStreamSynchronize(s));
    {
        // an enqueued iteration did work iff its index is below the step's
        // final iteration count (largest over the fields)
        std::vector<int> ran(n_steps, 0);
        for (int st = 0; st < n_steps; ++st)
            for (int f = 0; f < F; ++f) ran[st] = std::max(ran[st], (int)h_iters[st * CGD_MAX_FIELDS + f]);
        timing_collect(&m->timing, [&](int64_t tag) {
            if (tag < 0) return true;  // not a CG iteration
            const int st = (int)(tag / 65536), it = (int)(tag % 65536);
            return st < n_steps && it < ran[st];
        });
    }
    cgd_status worst = CGD_OK;
    for (int st = 0; st < n_steps; ++st)
        for (int f = 0; f < F; ++f) {
            int32_t v = h_status[st * CGD_MAX_FIELDS + f];
            if (v == CGD_E_BREAKDOWN) {
                set_error("CG breakdown in pseudo-step " + std::to_string(st) + ", field " + std::to_string(f));
                worst = CGD_E_BREAKDOWN;
            } else if (v == CGD_NOT_CONVERGED && worst == CGD_OK) {
                worst = CGD_NOT_CONVERGED;
            }
        }
    int n_fallback = 0;
    if (warm)
        for (int st = 0; st < n_steps; ++st)
            for (int f = 0; f < F; ++f) n_fallback += h_fb[st * CGD_MAX_FIELDS + f] != 0;
    if (n_fallback > 0 && worst == CGD_OK) worst = CGD_WARMSTART_FALLBACK;
    if (out) {
        out->n_fallback = n_fallback;
        out->n_steps = n_steps;
        out->n_fields = F;
        for (int st = 0; st < n_steps; ++st)
            for (int f = 0; f < F; ++f) {
                out->iters[st][f] = h_iters[st * CGD_MAX_FIELDS + f];
                out->rel_res[st][f] = h_rel[st * CGD_MAX_FIELDS + f];
            }
        for (int f = 0; f < F; ++f) {
            out->mass_before[f] = h_sums[f] * vol_scale;
            out->mass_after[f] = h_sums[CGD_MAX_FIELDS + f] * vol_scale;
        }
        out->status = worst;
    }
    return worst;
}

}  // namespace cgd
