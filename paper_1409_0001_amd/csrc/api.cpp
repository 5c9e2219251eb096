// C-ABI entry points of libcgd: argument validation, mesh objects and their
// workspace, and the order of device work.  No exception crosses the ABI.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>

#include "cg_common.h"
#include "tet_data.h"

namespace cgd {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

cgd_status ensure_workspace(cgd_mesh m, size_t bytes) {
    if (m->ws.bytes >= bytes) return CGD_OK;
    if (m->ws.ptr) {
        CGD_HIP_TRY(hipDeviceSynchronize());
        CGD_HIP_TRY(hipFree(m->ws.ptr));
        m->ws.ptr = nullptr;
        m->ws.bytes = 0;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("workspace allocation of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
        return CGD_E_NOMEM;
    }
    m->ws.ptr = p;
    m->ws.bytes = bytes;
    return CGD_OK;
}

cgd_status ensure_pinned(cgd_mesh m, size_t bytes) {
    if (m->pinned_bytes >= bytes) return CGD_OK;
    if (m->pinned) {
        CGD_HIP_TRY(hipDeviceSynchronize());
        CGD_HIP_TRY(hipHostFree(m->pinned));
        m->pinned = nullptr;
        m->pinned_bytes = 0;
    }
    void* p = nullptr;
    hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error(std::string("pinned host allocation failed: ") + hipGetErrorString(e));
        return CGD_E_NOMEM;
    }
    memset(p, 0, bytes);
    m->pinned = p;
    m->pinned_bytes = bytes;
    return CGD_OK;
}

// Timing events carry no system-scope fence: they only bracket kernels on
// the device's clock, and a fence would flush the L2 and stall the queue at
// every record (about 10 us per timed kernel).
int timing_begin(Timing* t, hipStream_t s) {
    if (!t->on) return -1;
    hipEvent_t e[2];
    for (int i = 0; i < 2; ++i) {
        if (t->pool.empty()) {
            if (hipEventCreateWithFlags(&e[i], hipEventDisableSystemFence) != hipSuccess) return -1;
        } else {
            e[i] = t->pool.back();
            t->pool.pop_back();
        }
    }
    (void)hipEventRecord(e[0], s);
    t->used.push_back(e[0]);
    t->used.push_back(e[1]);
    return (int)t->used.size() - 2;
}

void timing_end(Timing* t, int idx, int kind, double bytes, hipStream_t s, int64_t tag) {
    if (idx < 0) return;
    (void)hipEventRecord(t->used[idx + 1], s);
    t->kinds.push_back(kind);
    t->first.push_back(idx);  // pairs may nest, so they close out of order
    t->bytes.push_back(bytes);
    t->tags.push_back(tag);
}

void timing_collect(Timing* t, const std::function<bool(int64_t)>& keep) {
    for (size_t p = 0; p < t->kinds.size(); ++p) {
        float ms = 0.f;
        if (keep && !keep(t->tags[p])) continue;
        if (hipEventElapsedTime(&ms, t->used[t->first[p]], t->used[t->first[p] + 1]) == hipSuccess) {
            int k = t->kinds[p];
            t->launches[k] += 1;
            t->total_ms[k] += ms;
            t->bytes_per_launch[k] = t->bytes[p];
        }
    }
    for (hipEvent_t e : t->used) t->pool.push_back(e);
    t->used.clear();
    t->kinds.clear();
    t->first.clear();
    t->bytes.clear();
    t->tags.clear();
}

// Device of the mesh made current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev) {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Workspace use of a deposit: the counters sit at kOffDeposit (a part of
// the small region the diffusion does not use); from kSmallFixed on, either
// the bucketing scratch of the tiled hex deposit or the int64 accumulators
// of the direct path (when the caller passes none).  The diffusion that
// follows in cgd_coarse_grain reuses that memory only after the deposit's
// last kernel has read it, in stream order.
static cgd_status deposit_buffers(cgd_mesh m, int64_t n, int32_t F, int64_t* user_acc, int64_t** acc,
                                  DepositInfo** info, void** temp) {
    const size_t tiled = m->kind != 1 ? deposit_hex_temp_bytes(m, n, F) : 0;
    size_t acc_bytes = (user_acc || tiled) ? 0 : ((size_t)F * m->cells * sizeof(int64_t) + 255) & ~(size_t)255;
    // tet meshes: the particles' spatial ordering after the accumulators
    const size_t order = m->kind == 1 ? deposit_tet_temp_bytes(m, n) : 0;
    size_t need = kSmallFixed + acc_bytes + tiled + order;
    size_t diff = m->kind == 0 ? diffuse_hex_workspace(m, F) : diffuse_tet_workspace(m, F);
    cgd_status rc = ensure_workspace(m, need > diff ? need : diff);
    if (rc != CGD_OK) return rc;
    char* base = static_cast<char*>(m->ws.ptr);
    *info = reinterpret_cast<DepositInfo*>(base + kOffDeposit);
    *temp = tiled ? base + kSmallFixed : (order ? base + kSmallFixed + acc_bytes : nullptr);
    *acc = user_acc ? user_acc : (tiled ? nullptr : reinterpret_cast<int64_t*>(base + kSmallFixed));
    return CGD_OK;
}

}  // namespace cgd

using namespace cgd;

extern "C" {

const char* cgd_last_error(void) { return g_last_error.c_str(); }

int32_t cgd_version(void) { return 100; }

const char* cgd_status_string(cgd_status s) {
    switch (s) {
        case CGD_OK: return "CGD_OK";
        case CGD_NOT_CONVERGED: return "CGD_NOT_CONVERGED";
        case CGD_WARMSTART_FALLBACK: return "CGD_WARMSTART_FALLBACK";
        case CGD_E_INVALID: return "CGD_E_INVALID";
        case CGD_E_NONFINITE: return "CGD_E_NONFINITE";
        case CGD_E_NOMEM: return "CGD_E_NOMEM";
        case CGD_E_HIP: return "CGD_E_HIP";
        case CGD_E_BREAKDOWN: return "CGD_E_BREAKDOWN";
        case CGD_E_UNSUPPORTED: return "CGD_E_UNSUPPORTED";
        default: return "unknown cgd_status";
    }
}

cgd_status cgd_mesh_create_hex(int32_t nx, int32_t ny, int32_t nz, const double lo[3],
                               const double hi[3], cgd_mesh* out) {
    if (!out || !lo || !hi) {
        set_error("cgd_mesh_create_hex: null pointer");
        return CGD_E_INVALID;
    }
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) {
        set_error("cgd_mesh_create_hex: sizes must be >= 1");
        return CGD_E_INVALID;
    }
    for (int a = 0; a < 3; ++a) {
        if (!isfinite(lo[a]) || !isfinite(hi[a]) || !(hi[a] > lo[a])) {
            set_error("cgd_mesh_create_hex: need finite lo < hi on every axis");
            return CGD_E_INVALID;
        }
    }
    if ((int64_t)nx * ny * nz > (int64_t)1 << 33) {
        set_error("cgd_mesh_create_hex: too many cells");
        return CGD_E_INVALID;
    }
    cgd_mesh m = new (std::nothrow) cgd_mesh_s();
    if (!m) return CGD_E_NOMEM;
    m->kind = 0;
    if (hipGetDevice(&m->device) != hipSuccess) {
        set_error("cgd_mesh_create_hex: no HIP device");
        delete m;
        return CGD_E_HIP;
    }
    m->cells = (int64_t)nx * ny * nz;
    HexGeom& g = m->hex;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    const int32_t n[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = lo[a];
        g.hi[a] = hi[a];
        g.s[a] = (double)n[a] / (hi[a] - lo[a]);
        g.h[a] = (hi[a] - lo[a]) / (double)n[a];
    }
    g.vol = (g.h[0] * g.h[1]) * g.h[2];
    for (int i = 0; i < 2; ++i) {
        if (hipEventCreateWithFlags(&m->ev[i], hipEventDisableTiming) != hipSuccess) {
            set_error("cgd_mesh_create_hex: hipEventCreate failed");
            cgd_mesh_destroy(m);
            return CGD_E_HIP;
        }
    }
    *out = m;
    return CGD_OK;
}

void cgd_mesh_destroy(cgd_mesh m) {
    if (!m) return;
    DeviceGuard dg(m->device);
    (void)hipDeviceSynchronize();
    if (m->ws.ptr) (void)hipFree(m->ws.ptr);
    if (m->pinned) (void)hipHostFree(m->pinned);
    for (int i = 0; i < 2; ++i)
        if (m->ev[i]) (void)hipEventDestroy(m->ev[i]);
    destroy_batched(m);
    for (hipEvent_t e : m->timing.pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : m->timing.used) (void)hipEventDestroy(e);
    destroy_tet_data(m);
    delete m;
}

int64_t cgd_mesh_num_cells(cgd_mesh m) { return m ? m->cells : 0; }

int32_t cgd_mesh_kind(cgd_mesh m) { return m ? m->kind : -1; }

int64_t cgd_mesh_nnz(cgd_mesh m) { return m ? tet_nnz(m) : 0; }

cgd_status cgd_timing_enable(cgd_mesh m, int32_t on) {
    if (!m) {
        set_error("cgd_timing_enable: null mesh");
        return CGD_E_INVALID;
    }
    m->timing.on = on != 0;
    return CGD_OK;
}

cgd_status cgd_timing_read(cgd_mesh m, cgd_kernel_timing* out, int32_t reset) {
    if (!m || !out) {
        set_error("cgd_timing_read: null argument");
        return CGD_E_INVALID;
    }
    DeviceGuard dg(m->device);
    if (!m->timing.used.empty()) {
        CGD_HIP_TRY(hipDeviceSynchronize());
        timing_collect(&m->timing);
    }
    for (int k = 0; k < CGD_TIMING_KINDS; ++k) {
        out->launches[k] = m->timing.launches[k];
        out->total_ms[k] = m->timing.total_ms[k];
        out->bytes_per_launch[k] = m->timing.bytes_per_launch[k];
        if (reset) {
            m->timing.launches[k] = 0;
            m->timing.total_ms[k] = 0.0;
        }
    }
    return CGD_OK;
}

static cgd_status check_common(cgd_mesh m, int32_t F, const char* who) {
    if (!m) {
        set_error(std::string(who) + ": null mesh");
        return CGD_E_INVALID;
    }
    if (F < 1 || F > CGD_MAX_FIELDS) {
        set_error(std::string(who) + ": F must be in 1.." + std::to_string(CGD_MAX_FIELDS));
        return CGD_E_INVALID;
    }
    return CGD_OK;
}

// frac_bits: host [F] or NULL; in: -1 (automatic) or a forced scale 0..62
// (validated by the caller), out: the scale used.  The call waits for the
// stream when st is given or some scale was automatic.
static cgd_status do_deposit(cgd_mesh m, int64_t n, const float* pos, int32_t F, const float* values,
                             float* field, int64_t* acc, int32_t* frac_bits, cgd_solve_stats* st, hipStream_t s) {
    int64_t* acc_buf;
    DepositInfo* info;
    void* temp;
    ScaleForce fs;
    bool need_auto = false;
    for (int f = 0; f < CGD_MAX_FIELDS; ++f) fs.s[f] = (frac_bits && f < F) ? frac_bits[f] : -1;
    for (int f = 0; f < F; ++f) need_auto = need_auto || fs.s[f] < 0;
    cgd_status rc = deposit_buffers(m, n, F, acc, &acc_buf, &info, &temp);
    if (rc != CGD_OK) return rc;
    if (m->kind == 0)
        rc = deposit_hex(m, n, pos, F, values, field, acc_buf, info, temp, fs, &m->timing, s);
    else
        rc = deposit_tet(m, n, pos, F, values, field, acc_buf, info, temp, fs, s);
    if (rc != CGD_OK || !(st || (frac_bits && need_auto))) return rc;
    cgd_status prc = ensure_pinned(m, kPinBytes);
    if (prc != CGD_OK) return prc;
    DepositInfo* h = reinterpret_cast<DepositInfo*>(static_cast<char*>(m->pinned) + kPinDeposit);
    CGD_HIP_TRY(hipMemcpyAsync(h, info, sizeof(DepositInfo), hipMemcpyDeviceToHost, s));
    CGD_HIP_TRY(hipStreamSynchronize(s));
    const int e_n = ceil_log2_count(n);
    unsigned long long nf = h->nonfinite_pos;
    for (int f = 0; f < F; ++f) {
        uint32_t mb = h->maxbits[f];
        int S = 0;
        if (fs.s[f] >= 0) {
            S = fs.s[f];
        } else if (mb) {
            float mv;
            memcpy(&mv, &mb, 4);
            int e;
            (void)frexp((double)mv, &e);
            S = 62 - e - e_n;
        }
        if (st) st->frac_bits[f] = S;
        if (frac_bits) frac_bits[f] = S;
        nf += h->nonfinite_val[f];
    }
    if (!st) return CGD_OK;
    st->n_dropped = (int64_t)h->dropped;
    st->n_nonfinite = (int64_t)nf;
    if (nf) {
        set_error("non-finite particle positions or values were skipped");
        return CGD_E_NONFINITE;
    }
    return CGD_OK;
}

cgd_status cgd_locate(cgd_mesh m, int64_t n, const float* pos, int32_t* cell, void* stream) {
    if (!m || n < 0 || (n > 0 && (!pos || !cell))) {
        set_error("cgd_locate: need a mesh, n >= 0 and non-null pos / cell");
        return CGD_E_INVALID;
    }
    if (reinterpret_cast<uintptr_t>(pos) % 4 || reinterpret_cast<uintptr_t>(cell) % 4) {
        set_error("cgd_locate: misaligned pointer");
        return CGD_E_INVALID;
    }
    DeviceGuard dg(m->device);
    if (dg.err != hipSuccess) {
        set_error(std::string("cgd_locate: ") + hipGetErrorString(dg.err));
        return CGD_E_HIP;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    return m->kind == 0 ? locate_hex(m, n, pos, cell, s) : locate_tet(m, n, pos, cell, s);
}

cgd_status cgd_deposit(cgd_mesh m, int64_t n, const float* pos, int32_t F, const float* values,
                       float* field, int64_t* acc, int32_t* frac_bits, cgd_solve_stats* st, void* stream) {
    cgd_status rc = check_common(m, F, "cgd_deposit");
    if (rc != CGD_OK) return rc;
    if (n < 0 || (n > 0 && (!pos || !values)) || !field) {
        set_error("cgd_deposit: need n >= 0 and non-null pos/values (n > 0) and field");
        return CGD_E_INVALID;
    }
    if (frac_bits) {
        for (int f = 0; f < F; ++f) {
            if (frac_bits[f] < -1 || frac_bits[f] > 62) {
                set_error("cgd_deposit: frac_bits entries must be -1 (automatic) or a scale in 0..62");
                return CGD_E_INVALID;
            }
        }
    }
    if (reinterpret_cast<uintptr_t>(acc) % 8 || reinterpret_cast<uintptr_t>(pos) % 4 ||
        reinterpret_cast<uintptr_t>(values) % 4 || reinterpret_cast<uintptr_t>(field) % 4) {
        set_error("cgd_deposit: misaligned pointer");
        return CGD_E_INVALID;
    }
    DeviceGuard dg(m->device);
    if (dg.err != hipSuccess) {
        set_error(std::string("cgd_deposit: ") + hipGetErrorString(dg.err));
        return CGD_E_HIP;
    }
    if (st) memset(st, 0, sizeof(*st));
    return do_deposit(m, n, pos, F, values, field, acc, frac_bits, st, static_cast<hipStream_t>(stream));
}

static cgd_status fill_opts(const cgd_solver_opts* o, int32_t F, float* field, double bandwidth,
                            int32_t n_steps, DiffuseArgs* a, const char* who) {
    if (!field) {
        set_error(std::string(who) + ": null field");
        return CGD_E_INVALID;
    }
    if (!(bandwidth > 0.0) || !isfinite(bandwidth)) {
        set_error(std::string(who) + ": bandwidth must be finite and > 0");
        return CGD_E_INVALID;
    }
    if (n_steps < 1 || n_steps > CGD_MAX_STEPS) {
        set_error(std::string(who) + ": n_steps must be in 1.." + std::to_string(CGD_MAX_STEPS));
        return CGD_E_INVALID;
    }
    a->F = F;
    a->field = field;
    a->bandwidth = bandwidth;
    a->n_steps = n_steps;
    a->rtol = (o && o->rtol > 0.0) ? o->rtol : 1e-6;
    a->max_iter = (o && o->max_iter > 0) ? o->max_iter : 1000;
    a->x0_mode = o ? o->x0_mode : 0;
    a->x0 = o ? o->x0 : nullptr;
    a->check_every = (o && o->check_every > 0) ? o->check_every : 4;
    a->model = o ? o->model : nullptr;
    a->precond = o ? o->precond : 0;
    a->scheme = o ? o->scheme : 0;
    if (a->scheme < 0 || a->scheme > 1) {
        set_error(std::string(who) + ": scheme must be 0 (backward Euler) or 1 (Crank-Nicolson)");
        return CGD_E_INVALID;
    }
    if (a->precond < 0 || a->precond > 1) {
        set_error(std::string(who) + ": precond must be 0 (default preconditioner) or 1 (none)");
        return CGD_E_INVALID;
    }
    if (a->x0_mode < 0 || a->x0_mode > 3 || (a->x0_mode == 2 && !a->x0) || (a->x0_mode == 3 && !a->model) ||
        !isfinite(a->rtol)) {
        set_error(std::string(who) + ": bad solver options (x0_mode 0..3, x0 needed for mode 2, model for mode 3)");
        return CGD_E_INVALID;
    }
    return CGD_OK;
}

static cgd_status do_diffuse(cgd_mesh m, const DiffuseArgs& a, cgd_solve_stats* st, hipStream_t s) {
    if (a.x0_mode == 3 &&
        (m->kind != 0 || !unet::unet_matches(a.model, m->hex.nx, m->hex.ny, m->hex.nz, m->device))) {
        set_error("x0_mode 3: the network must be created for this hex mesh's grid, on its device");
        return CGD_E_INVALID;
    }
    if (m->kind == 0) return diffuse_hex(m, a, st, s);
    return diffuse_tet(m, a, st, s);
}

cgd_status cgd_diffuse(cgd_mesh m, int32_t F, float* field, double bandwidth, int32_t n_steps,
                       const cgd_solver_opts* o, cgd_solve_stats* st, void* stream) {
    cgd_status rc = check_common(m, F, "cgd_diffuse");
    if (rc != CGD_OK) return rc;
    DiffuseArgs a;
    rc = fill_opts(o, F, field, bandwidth, n_steps, &a, "cgd_diffuse");
    if (rc != CGD_OK) return rc;
    DeviceGuard dg(m->device);
    if (dg.err != hipSuccess) {
        set_error(std::string("cgd_diffuse: ") + hipGetErrorString(dg.err));
        return CGD_E_HIP;
    }
    if (st) memset(st, 0, sizeof(*st));
    return do_diffuse(m, a, st, static_cast<hipStream_t>(stream));
}

cgd_status cgd_coarse_grain(cgd_mesh m, int64_t n, const float* pos, int32_t F, const float* values,
                            double bandwidth, int32_t n_steps, const cgd_solver_opts* o, float* field,
                            cgd_solve_stats* st, void* stream) {
    cgd_status rc = check_common(m, F, "cgd_coarse_grain");
    if (rc != CGD_OK) return rc;
    if (n < 0 || (n > 0 && (!pos || !values))) {
        set_error("cgd_coarse_grain: need n >= 0 and non-null pos/values when n > 0");
        return CGD_E_INVALID;
    }
    DiffuseArgs a;
    rc = fill_opts(o, F, field, bandwidth, n_steps, &a, "cgd_coarse_grain");
    if (rc != CGD_OK) return rc;
    if (a.x0_mode == 2) {
        set_error("cgd_coarse_grain: x0_mode 2 needs cgd_diffuse");
        return CGD_E_INVALID;
    }
    DeviceGuard dg(m->device);
    if (dg.err != hipSuccess) {
        set_error(std::string("cgd_coarse_grain: ") + hipGetErrorString(dg.err));
        return CGD_E_HIP;
    }
    if (st) memset(st, 0, sizeof(*st));
    hipStream_t s = static_cast<hipStream_t>(stream);
    // Every mesh kind, from a zero guess: a call with the parameters of the
    // previous one on this mesh enqueues, per step, the iterations that call
    // took plus a margin of one, with no read-back between steps (launches
    // after a field has converged return at once, so the result is the same).
    // Once hb.steady budgeted calls in a row (2 at first) have taken exactly
    // the previous counts, the margin is dropped (the spare iteration's five
    // empty launches cost about 12 us per step on a 256 x 256 x 512 grid).  A
    // step that runs out of its budget (its residual checked after the last
    // iteration) sends the call round again with read-backs, and the margin
    // returns until the counts repeat; a miss without the margin doubles
    // hb.steady (at most 64), so that inputs whose counts rise every few
    // calls do not pay a rerun each time.
    IterBudget& hb = m->budget;
    const bool budgeted = a.x0_mode == 0 && !getenv("CGD_NO_BUDGET");
    const bool have = budgeted && hb.valid && hb.F == F && hb.n_steps == a.n_steps && hb.max_iter == a.max_iter &&
                      hb.precond == a.precond && hb.scheme == a.scheme && hb.bandwidth == a.bandwidth &&
                      hb.rtol == a.rtol;
    const int margin = hb.repeats >= hb.steady ? 0 : 1;
    int bud[CGD_MAX_STEPS];
    for (int i = 0; i < a.n_steps; ++i) bud[i] = have ? std::max(1, hb.iters[i] + margin) : 0;
    for (int round = have ? 0 : 1; round < 2; ++round) {
        rc = do_deposit(m, n, pos, F, values, field, nullptr, nullptr, st, s);
        cgd_status dep_rc = rc;
        if (rc < 0 && rc != CGD_E_NONFINITE) return rc;
        if (round == 0) {
            rc = m->kind == 0 ? diffuse_hex(m, a, st, s, bud) : diffuse_tet(m, a, st, s, bud);
            if (rc == CGD_NOT_CONVERGED) {
                hb.valid = false;
                if (margin == 0) hb.steady = std::min(64, 2 * hb.steady);
                if (st) memset(st, 0, sizeof(*st));
                continue;
            }
        } else {
            rc = do_diffuse(m, a, st, s);
        }
        if (rc < 0) return rc;
        if (budgeted) {
            // this call's iterations per step (cg_finish_call left them in the pinned buffer)
            hb.valid = rc == CGD_OK;
            const int32_t* it = reinterpret_cast<const int32_t*>(static_cast<char*>(m->pinned) + kPinIters);
            bool same = round == 0 && rc == CGD_OK;  // a budgeted call that did not run out
            for (int i = 0; i < a.n_steps; ++i) {
                int v = 0;
                for (int f = 0; f < F; ++f) v = std::max(v, (int)it[i * CGD_MAX_FIELDS + f]);
                same = same && v == hb.iters[i];
                hb.iters[i] = v;
            }
            hb.repeats = same ? hb.repeats + 1 : 0;
            hb.F = F;
            hb.n_steps = a.n_steps;
            hb.max_iter = a.max_iter;
            hb.precond = a.precond;
            hb.scheme = a.scheme;
            hb.bandwidth = a.bandwidth;
            hb.rtol = a.rtol;
        }
        if (dep_rc == CGD_E_NONFINITE) return dep_rc;
        return rc;
    }
    return rc;
}

cgd_status cgd_coarse_grain_batched(cgd_mesh m, int32_t n_snap, const int64_t* offsets, const float* pos,
                                    int32_t F, const float* values, double bandwidth, int32_t n_steps,
                                    const cgd_solver_opts* o, float* fields, cgd_solve_stats* st, void* stream) {
    cgd_status rc = check_common(m, F, "cgd_coarse_grain_batched");
    if (rc != CGD_OK) return rc;
    if (m->kind != 0) {
        set_error("cgd_coarse_grain_batched: hex meshes only");
        return CGD_E_UNSUPPORTED;
    }
    if (n_snap < 1 || (int64_t)n_snap * F > 4096 || !offsets) {
        set_error("cgd_coarse_grain_batched: need 1 <= n_snap, n_snap * F <= 4096 and offsets");
        return CGD_E_INVALID;
    }
    if (offsets[0] != 0) {
        set_error("cgd_coarse_grain_batched: offsets[0] must be 0");
        return CGD_E_INVALID;
    }
    for (int j = 0; j < n_snap; ++j) {
        if (offsets[j + 1] < offsets[j]) {
            set_error("cgd_coarse_grain_batched: offsets must not decrease");
            return CGD_E_INVALID;
        }
    }
    if (offsets[n_snap] > 0 && (!pos || !values)) {
        set_error("cgd_coarse_grain_batched: null pos / values");
        return CGD_E_INVALID;
    }
    DiffuseArgs a;
    rc = fill_opts(o, F, fields, bandwidth, n_steps, &a, "cgd_coarse_grain_batched");
    if (rc != CGD_OK) return rc;
    if (a.x0_mode != 0) {
        set_error("cgd_coarse_grain_batched: x0_mode must be 0");
        return CGD_E_INVALID;
    }
    if (reinterpret_cast<uintptr_t>(fields) % 16 || reinterpret_cast<uintptr_t>(pos) % 4 ||
        reinterpret_cast<uintptr_t>(values) % 4) {
        set_error("cgd_coarse_grain_batched: fields must be 16-byte aligned, pos / values 4-byte aligned");
        return CGD_E_INVALID;
    }
    DeviceGuard dg(m->device);
    if (dg.err != hipSuccess) {
        set_error(std::string("cgd_coarse_grain_batched: ") + hipGetErrorString(dg.err));
        return CGD_E_HIP;
    }
    return coarse_grain_batched(m, n_snap, offsets, pos, F, values, a, fields, st,
                                static_cast<hipStream_t>(stream));
}

cgd_status cgd_autotune_batched(cgd_mesh m, int32_t n_rhs, int32_t* chosen, double* ms, int32_t* n_cand) {
    if (!m || m->kind != 0 || n_rhs < 1 || !chosen) {
        set_error("cgd_autotune_batched: need a hex mesh, n_rhs >= 1 and chosen");
        return CGD_E_INVALID;
    }
    DeviceGuard dg(m->device);
    int c = 0, nc = 0;
    cgd_status rc = autotune_batched(m, n_rhs, &c, ms, &nc);
    if (rc != CGD_OK) return rc;
    *chosen = c;
    if (n_cand) *n_cand = nc;
    return CGD_OK;
}

cgd_status cgd_velocity_from_momentum(int64_t cells, int32_t n_comp, const float* eps, float* mom,
                                      float eps_min, void* stream) {
    if (cells < 0 || n_comp < 1 || n_comp > CGD_MAX_FIELDS - 1 || (cells > 0 && (!eps || !mom)) ||
        !isfinite(eps_min) || eps_min < 0.f) {
        set_error("cgd_velocity_from_momentum: need cells >= 0, 1 <= n_comp < CGD_MAX_FIELDS, eps, mom and a "
                  "finite eps_min >= 0");
        return CGD_E_INVALID;
    }
    velocity_from_momentum(cells, n_comp, eps, mom, eps_min, static_cast<hipStream_t>(stream));
    CGD_HIP_TRY(hipGetLastError());
    return CGD_OK;
}

}  // extern "C"
