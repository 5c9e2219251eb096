// One wave's tile of a 7-point-stencil CG sweep on a uniform hex grid (used
// by the per-launch sweeps of cg_hex.hip and the persistent batched solver).
//
// The operator is A = I + dtau K / V: (A p)_k = p_k + sum_a c_a (2 p_k -
// p_k-1 - p_k+1), c_a = dtau / h_a^2, with a missing neighbour at a wall
// replaced by p_k itself (zero flux through wall faces).
//
// A wave owns 64 * VEC consecutive x (VEC per lane) times TY rows of y and
// marches over the planes [zb, ze), keeping planes z-1, z, z+1 (with one halo
// row on each side) in registers; x-neighbours come from lane shuffles.
// Every load is issued unconditionally at a clamped, in-bounds address and
// out-of-range values are replaced afterwards, so the loads of a plane are
// issued together.  EDGE: the row is wider than one wave (VEC = 1), so lanes
// 0 and 63 also load the cell beyond the wave's ends (every other lane loads
// its own cell at that instruction).
#pragma once

#include <hip/hip_runtime.h>

namespace cgd {
namespace stencil {

//   S1_FIRST  p = b;                 b.Ab and b.b
//   S1        p = r + beta p_old;    writes p; p.Ap
//   S1_B0     p = r;                 writes p; p.Ap
//   S2_FIRST  x = alpha b, r = b - alpha A b;  r.r
//   S2        x += alpha p, r -= alpha A p;   r.r
//   S_RES     r = b - A x;           r.r and b.b
// Preconditioned CG (z = M r with a polynomial M = c0 I + c1 A + c2 A^2; the
// S1 modes then read z through Ptrs::R):
//   SZ_FIRST  z = M b;               writes z; b.z and b.b   (degree 1)
//   SZ        z = M r;               writes z; r.z           (degree 1)
//   S2P_FIRST x = alpha p, r = b - alpha A p;  r.r   (zero initial guess)
//   SZ2_FIRST, SZ2: as SZ_FIRST, SZ with the degree-2 polynomial (tile_precond2)
enum Mode {
    S1_FIRST = 0, S1 = 1, S2_FIRST = 2, S2 = 3, S_RES = 4, S1_B0 = 5,
    SZ_FIRST = 6, SZ = 7, S2P_FIRST = 8, SZ2_FIRST = 9, SZ2 = 10
};

struct Ptrs {
    const float* B;     // right-hand side of the step
    float* R;           // residual (the S1 modes of preconditioned CG: z)
    const float* Pold;  // previous direction
    float* Pnew;        // new direction
    float* X;           // iterate
    float* Z;           // preconditioned residual (SZ modes)
    float* U;           // product-form preconditioner: output of its first pass
    float* V;           // ... input of its last pass (U, or the middle pass's output)
};

struct Geom {
    int nx, ny, nz;
    float cx, cy, cz;
    float c0, c1, c2;   // preconditioner M = c0 I + c1 A + c2 A^2
    // Crank-Nicolson folded into the x updates of a zero-guess solve: x
    // advances by (1 + xs1) alpha p from xb b, so that with xs1 = 1, xb = -1
    // the iterate is 2 y - b when y solves the half step (0, 0: plain x)
    float xs1, xb;
    // Rectilinear grids with a separable diffusivity (RECT kernels): the
    // operator is A = S (I + dt M^-1/2 K M^-1/2) S (M the cell volumes, K the
    // finite-volume Laplacian with harmonic-mean face diffusivities, S a
    // diagonal scaling that is a product of per-axis factors: the identity
    // for the CG sweeps, a preconditioner's scaling in the polynomial
    // passes), whose entries are products of per-axis factors.  Per axis a
    // with n cells: rg[a] [n + 1] face weights (0 at a wall), rs[a] [n] the
    // cell's own diagonal sum over its two faces, rd[a] [n] the diffusivity
    // factor, re[a] [n] the identity's factor (all with S folded in), rsg[a]
    // [n] S's own factors (polynomial passes only).  Cell (i, j, k):
    //   (A v) = (ex ey ez + dt (Dy Dz sx_i + Dx (Dz sy_j + Dy sz_k))) v
    //           - dt Dy Dz (gx_i v_{i-1} + gx_{i+1} v_{i+1})
    //           - dt Dx Dz (gy_j v_{j-1} + gy_{j+1} v_{j+1})
    //           - dt Dx Dy (gz_k v_{k-1} + gz_{k+1} v_{k+1})
    const float* rg[3];
    const float* rs[3];
    const float* rd[3];
    const float* re[3];
    const float* rsg[3];
    float dt;
    // RECT: bit a set when axis a is periodic (its first and last cells are
    // neighbours through a face of weight rg[a][0] = rg[a][n]); a periodic
    // x axis needs the row in one x segment
    int per;
};

// RECT: the x factors of a lane's VEC cells (dt folded into the weights),
// loaded once per tile; lane cells beyond the grid take the last cell's.
template <int VEC>
struct RectX {
    float gl[VEC], gr[VEC], s[VEC], d[VEC], e[VEC];
};

template <int VEC>
__device__ __forceinline__ RectX<VEC> rect_x(const Geom& g, int x0) {
    RectX<VEC> X;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        const int i = min(x0 + e, g.nx - 1);
        X.gl[e] = g.dt * g.rg[0][i];
        X.gr[e] = g.dt * g.rg[0][i + 1];
        X.s[e] = g.dt * g.rs[0][i];
        X.d[e] = g.rd[0][i];
        X.e[e] = g.re[0][i];
    }
    return X;
}

// RECT: the y and z factors of one row at one plane (wave-uniform values).
struct RectYZ {
    float e, dyz, a, bd, bu, cd, cu;
};

// The factors of one row (y) or one plane (z): lower and upper face
// weights, diagonal sum, diffusivity factor, identity factor.
struct RectA {
    float gd, gu, s, d, e;
};

__device__ __forceinline__ RectA rect_a(const Geom& g, int axis, int i, int n) {
    i = min(max(i, 0), n - 1);
    return RectA{g.rg[axis][i], g.rg[axis][i + 1], g.rs[axis][i], g.rd[axis][i], g.re[axis][i]};
}

__device__ __forceinline__ RectYZ rect_yz(const Geom& g, const RectA& Y, const RectA& Z) {
    RectYZ r;
    r.e = Y.e * Z.e;
    r.dyz = Y.d * Z.d;
    r.a = g.dt * fmaf(Z.d, Y.s, Y.d * Z.s);
    r.bd = g.dt * Z.d * Y.gd;
    r.bu = g.dt * Z.d * Y.gu;
    r.cd = g.dt * Y.d * Z.gd;
    r.cu = g.dt * Y.d * Z.gu;
    return r;
}

__device__ __forceinline__ RectYZ rect_yz(const Geom& g, int y, int z) {
    return rect_yz(g, rect_a(g, 1, y, g.ny), rect_a(g, 2, z, g.nz));
}

// RECT: the diagonal of A at one cell.
template <int VEC>
__device__ __forceinline__ float rect_diag(const RectX<VEC>& X, int e, const RectYZ& q) {
    return fmaf(q.dyz, X.s[e], fmaf(X.d[e], q.a, X.e[e] * q.e));
}

// RECT: (A v) at one cell (a neighbour across a wall has weight 0, so any
// finite value may stand there).
template <int VEC>
__device__ __forceinline__ float rect_cell(const RectX<VEC>& X, int e, const RectYZ& q, float c, float l, float r,
                                           float yl, float yh, float zl, float zh) {
    const float d = rect_diag<VEC>(X, e, q);
    const float nxv = fmaf(X.gl[e], l, X.gr[e] * r);
    const float nyz = fmaf(q.bd, yl, fmaf(q.bu, yh, fmaf(q.cd, zl, q.cu * zh)));
    return fmaf(d, c, -fmaf(X.d[e], nyz, q.dyz * nxv));
}

template <int VEC>
struct Vec {
    float f[VEC];
};

template <int VEC>
__device__ __forceinline__ Vec<VEC> ldv(const float* q) {
    Vec<VEC> v;
    if constexpr (VEC == 4) {
        const float4 t = *reinterpret_cast<const float4*>(q);
        v.f[0] = t.x; v.f[1] = t.y; v.f[2] = t.z; v.f[3] = t.w;
    } else if constexpr (VEC == 2) {
        const float2 t = *reinterpret_cast<const float2*>(q);
        v.f[0] = t.x; v.f[1] = t.y;
    } else {
        v.f[0] = *q;
    }
    return v;
}

template <int VEC>
__device__ __forceinline__ void stv(float* q, const Vec<VEC>& v) {
    if constexpr (VEC == 4) {
        *reinterpret_cast<float4*>(q) = make_float4(v.f[0], v.f[1], v.f[2], v.f[3]);
    } else if constexpr (VEC == 2) {
        *reinterpret_cast<float2*>(q) = make_float2(v.f[0], v.f[1]);
    } else {
        *q = v.f[0];
    }
}

// The direction vector at VEC consecutive cells starting at i (an in-bounds
// address; the caller clamps).
template <int VEC, int MODE>
__device__ __forceinline__ Vec<VEC> load_p(const Ptrs& p, size_t i, float beta) {
    if constexpr (MODE == S1_FIRST || MODE == S2_FIRST || MODE == SZ_FIRST) {
        return ldv<VEC>(p.B + i);
    } else if constexpr (MODE == SZ) {
        return ldv<VEC>(p.R + i);
    } else if constexpr (MODE == S1) {
        Vec<VEC> r = ldv<VEC>(p.R + i);
        const Vec<VEC> q = ldv<VEC>(p.Pold + i);
#pragma unroll
        for (int e = 0; e < VEC; ++e) r.f[e] = fmaf(beta, q.f[e], r.f[e]);
        return r;
    } else if constexpr (MODE == S1_B0) {
        return ldv<VEC>(p.R + i);
    } else if constexpr (MODE == S2 || MODE == S2P_FIRST) {
        return ldv<VEC>(p.Pnew + i);
    } else {
        return ldv<VEC>(p.X + i);
    }
}

// One wave: x segment xs, row group yg (rows yg*TY ...), planes [zb, ze) of
// the field starting at element fo.  Adds this wave's dot products to acc0 /
// acc1 (see Mode).
template <int VEC, int TY, int MODE, bool EDGE, bool RECT = false>
__device__ __forceinline__ void tile_sweep(const Ptrs& p, const Geom& g, size_t fo, int xs, int yg, int zb, int ze,
                                           int lane, float alpha, float beta, double& acc0, double& acc1) {
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int x0 = xs * 64 * VEC + lane * VEC;
    const bool xin = x0 < nx;
    const int xc = xin ? x0 : nx - VEC;
    const bool wall_l = x0 == 0;
    const bool wall_r = x0 + VEC >= nx;
    const int y0 = yg * TY;
    const size_t plane = (size_t)nx * ny;
    const size_t base = fo + xc;
    const float cx = g.cx, cy = g.cy, cz = g.cz;
    int eoff = 0;
    if constexpr (EDGE) eoff = (lane == 0 && x0 > 0) ? -1 : ((lane == 63 && x0 + 1 < nx) ? 1 : 0);

    // Rows and planes beyond the grid: clamped, or on a periodic axis the
    // neighbours of the first and last (-1 -> n - 1, n -> 0; anything
    // further is clamped: only out-of-range rows and planes use it)
    const int per = RECT ? g.per : 0;
    auto at = [&](int z, int y) -> size_t {
        z = z < 0 ? ((per & 4) && z == -1 ? nz - 1 : 0) : (z >= nz ? ((per & 4) && z == nz ? 0 : nz - 1) : z);
        y = y < 0 ? ((per & 2) && y == -1 ? ny - 1 : 0) : (y >= ny ? ((per & 2) && y == ny ? 0 : ny - 1) : y);
        return base + (size_t)z * plane + (size_t)y * nx;
    };

    if constexpr (RECT && (MODE == SZ_FIRST || MODE == SZ)) {
        // Jacobi on the rectilinear operator: z = r / diag(A), pointwise
        // (no neighbours); r.z (and b.b)
        const RectX<VEC> X = rect_x<VEC>(g, x0);
        RectA Y[TY];
#pragma unroll
        for (int j = 0; j < TY; ++j) Y[j] = rect_a(g, 1, y0 + j, ny);
        for (int z = zb; z < ze; ++z) {
            Vec<VEC> rv[TY];
#pragma unroll
            for (int j = 0; j < TY; ++j) rv[j] = load_p<VEC, MODE>(p, at(z, y0 + j), beta);
            const RectA Z = rect_a(g, 2, z, nz);
#pragma unroll
            for (int j = 0; j < TY; ++j) {
                const int y = y0 + j;
                const RectYZ q = rect_yz(g, Y[j], Z);
                Vec<VEC> zv;
                // any positive diagonal preconditions CG: the hardware
                // reciprocal (1 ulp) in place of a division
#pragma unroll
                for (int e = 0; e < VEC; ++e) zv.f[e] = rv[j].f[e] * __builtin_amdgcn_rcpf(rect_diag<VEC>(X, e, q));
                if (xin && y < ny) {
                    stv<VEC>(p.Z + at(z, y), zv);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        acc0 = fma((double)rv[j].f[e], (double)zv.f[e], acc0);
                        if (MODE == SZ_FIRST) acc1 = fma((double)rv[j].f[e], (double)rv[j].f[e], acc1);
                    }
                }
            }
        }
        return;
    }

    Vec<VEC> pm[TY], pc[TY + 2], pn[TY + 2];
    float ec[TY], en[TY];
#pragma unroll
    for (int j = 0; j < TY; ++j) pm[j] = load_p<VEC, MODE>(p, at(zb - 1, y0 + j), beta);
#pragma unroll
    for (int j = 0; j < TY + 2; ++j) pc[j] = load_p<VEC, MODE>(p, at(zb, y0 - 1 + j), beta);
    if constexpr (EDGE) {
#pragma unroll
        for (int j = 0; j < TY; ++j) ec[j] = load_p<1, MODE>(p, at(zb, y0 + j) + eoff, beta).f[0];
    }
    RectX<VEC> X;
    RectA Y[TY];
    if constexpr (RECT) {
        X = rect_x<VEC>(g, x0);
#pragma unroll
        for (int j = 0; j < TY; ++j) Y[j] = rect_a(g, 1, y0 + j, ny);
    }
    for (int z = zb; z < ze; ++z) {
#pragma unroll
        for (int j = 0; j < TY + 2; ++j) pn[j] = load_p<VEC, MODE>(p, at(z + 1, y0 - 1 + j), beta);
        RectA Z;
        if constexpr (RECT) Z = rect_a(g, 2, z, nz);
        if constexpr (EDGE) {
#pragma unroll
            for (int j = 0; j < TY; ++j) en[j] = load_p<1, MODE>(p, at(z + 1, y0 + j) + eoff, beta).f[0];
        }
        const bool has_zd = z > 0 || (per & 4), has_zu = z + 1 < nz || (per & 4);
#pragma unroll
        for (int j = 0; j < TY; ++j) {
            const int y = y0 + j;
            const bool valid = xin && y < ny;
            const size_t i = at(z, y);
            const Vec<VEC>& c = pc[j + 1];
            const bool has_yd = y > 0 || (per & 2), has_yu = y + 1 < ny || (per & 2);
            float lft = __shfl_up(c.f[VEC - 1], 1);
            float rgt = __shfl_down(c.f[0], 1);
            if constexpr (EDGE) {
                lft = lane == 0 ? ec[j] : lft;
                rgt = lane == 63 ? ec[j] : rgt;
            }
            bool wl = wall_l, wr = wall_r;
            if constexpr (RECT) {
                if (per & 1) {
                    // periodic x (one segment, nx a multiple of VEC): the
                    // row's last cell (lane (nx - 1) / VEC) is the first
                    // cell's left neighbour, the first cell (lane 0) the last
                    // cell's right neighbour
                    const float last =
                        __int_as_float(__builtin_amdgcn_readlane(__float_as_int(c.f[VEC - 1]), (nx - 1) / VEC));
                    const float first = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(c.f[0]), 0));
                    lft = x0 == 0 ? last : lft;
                    rgt = x0 + VEC >= nx ? first : rgt;
                    wl = wr = false;
                }
            }
            Vec<VEC> ap;
            RectYZ q;
            if constexpr (RECT) q = rect_yz(g, Y[j], Z);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const float ce = c.f[e];
                float l = e > 0 ? c.f[e - 1] : (wl ? ce : lft);
                float r = e + 1 < VEC ? c.f[e + 1] : (wr ? ce : rgt);
                const float yl = has_yd ? pc[j].f[e] : ce;
                const float yh = has_yu ? pc[j + 2].f[e] : ce;
                const float zl = has_zd ? pm[j].f[e] : ce;
                const float zh = has_zu ? pn[j + 1].f[e] : ce;
                if constexpr (RECT) {
                    ap.f[e] = rect_cell<VEC>(X, e, q, ce, l, r, yl, yh, zl, zh);
                } else {
                    const float c2 = ce + ce;
                    float v = fmaf(cx, (c2 - l) - r, ce);
                    v = fmaf(cy, (c2 - yl) - yh, v);
                    ap.f[e] = fmaf(cz, (c2 - zl) - zh, v);
                }
            }
            if constexpr (MODE == S1_FIRST) {
                if (valid) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        acc0 = fma((double)c.f[e], (double)ap.f[e], acc0);
                        acc1 = fma((double)c.f[e], (double)c.f[e], acc1);
                    }
                }
            } else if constexpr (MODE == S1 || MODE == S1_B0) {
                if (valid) {
                    stv<VEC>(p.Pnew + i, c);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) acc0 = fma((double)c.f[e], (double)ap.f[e], acc0);
                }
            } else if constexpr (MODE == S2_FIRST) {
                Vec<VEC> xn, rn;
                const float ax = fmaf(g.xs1, alpha, alpha);
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    xn.f[e] = fmaf(ax, c.f[e], g.xb * c.f[e]);
                    rn.f[e] = fmaf(-alpha, ap.f[e], c.f[e]);
                }
                if (valid) {
                    stv<VEC>(p.X + i, xn);
                    stv<VEC>(p.R + i, rn);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) acc0 = fma((double)rn.f[e], (double)rn.f[e], acc0);
                }
            } else if constexpr (MODE == S2) {
                Vec<VEC> xv = ldv<VEC>(p.X + i);
                Vec<VEC> rv = ldv<VEC>(p.R + i);
                const float ax = fmaf(g.xs1, alpha, alpha);
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    xv.f[e] = fmaf(ax, c.f[e], xv.f[e]);
                    rv.f[e] = fmaf(-alpha, ap.f[e], rv.f[e]);
                }
                if (valid) {
                    stv<VEC>(p.X + i, xv);
                    stv<VEC>(p.R + i, rv);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) acc0 = fma((double)rv.f[e], (double)rv.f[e], acc0);
                }
            } else if constexpr (MODE == SZ_FIRST || MODE == SZ) {
                Vec<VEC> zv;
#pragma unroll
                for (int e = 0; e < VEC; ++e) zv.f[e] = fmaf(g.c1, ap.f[e], g.c0 * c.f[e]);
                if (valid) {
                    stv<VEC>(p.Z + i, zv);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        acc0 = fma((double)c.f[e], (double)zv.f[e], acc0);
                        if (MODE == SZ_FIRST) acc1 = fma((double)c.f[e], (double)c.f[e], acc1);
                    }
                }
            } else if constexpr (MODE == S2P_FIRST) {
                const Vec<VEC> bv = ldv<VEC>(p.B + i);
                Vec<VEC> xn, rn;
                const float ax = fmaf(g.xs1, alpha, alpha);
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    xn.f[e] = fmaf(ax, c.f[e], g.xb * bv.f[e]);
                    rn.f[e] = fmaf(-alpha, ap.f[e], bv.f[e]);
                }
                if (valid) {
                    stv<VEC>(p.X + i, xn);
                    stv<VEC>(p.R + i, rn);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) acc0 = fma((double)rn.f[e], (double)rn.f[e], acc0);
                }
            } else {  // S_RES: r = b - A x0
                const Vec<VEC> bv = ldv<VEC>(p.B + i);
                Vec<VEC> rn;
#pragma unroll
                for (int e = 0; e < VEC; ++e) rn.f[e] = bv.f[e] - ap.f[e];
                if (valid) {
                    stv<VEC>(p.R + i, rn);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        acc0 = fma((double)rn.f[e], (double)rn.f[e], acc0);
                        acc1 = fma((double)bv.f[e], (double)bv.f[e], acc1);
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < TY; ++j) pm[j] = pc[j + 1];
#pragma unroll
        for (int j = 0; j < TY + 2; ++j) pc[j] = pn[j];
        if constexpr (EDGE) {
#pragma unroll
            for (int j = 0; j < TY; ++j) ec[j] = en[j];
        }
    }
}

// (A v) along one row of VEC-wide lanes: c the row itself, yl / yh the rows
// below / above in the same plane, zl / zh the same row in the planes below /
// above; a missing neighbour (wall) is replaced by the cell itself.  The row
// is covered by one wave (x-neighbours of the end elements from the adjacent
// lanes; walls at lanes 0 and 63).
template <int VEC, bool RECT = false>
__device__ __forceinline__ Vec<VEC> apply_row(const Geom& g, const Vec<VEC>& c, const Vec<VEC>& yl,
                                              const Vec<VEC>& yh, const Vec<VEC>& zl, const Vec<VEC>& zh,
                                              bool hyd, bool hyu, bool hzd, bool hzu, bool wall_l, bool wall_r,
                                              const RectX<VEC>* X = nullptr, const RectYZ* q = nullptr) {
    const float lft = __shfl_up(c.f[VEC - 1], 1);
    const float rgt = __shfl_down(c.f[0], 1);
    Vec<VEC> out;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        const float ce = c.f[e];
        const float l = e > 0 ? c.f[e - 1] : (wall_l ? ce : lft);
        const float r = e + 1 < VEC ? c.f[e + 1] : (wall_r ? ce : rgt);
        const float ylo = hyd ? yl.f[e] : ce;
        const float yhi = hyu ? yh.f[e] : ce;
        const float zlo = hzd ? zl.f[e] : ce;
        const float zhi = hzu ? zh.f[e] : ce;
        if constexpr (RECT) {
            out.f[e] = rect_cell<VEC>(*X, e, *q, ce, l, r, ylo, yhi, zlo, zhi);
        } else {
            const float c2 = ce + ce;
            float v = fmaf(g.cx, (c2 - l) - r, ce);
            v = fmaf(g.cy, (c2 - ylo) - yhi, v);
            out.f[e] = fmaf(g.cz, (c2 - zlo) - zhi, v);
        }
    }
    return out;
}

// The same product with the x-neighbours of the lane's end cells given
// (lft, rgt: already the cell itself at a wall).
template <int VEC>
__device__ __forceinline__ Vec<VEC> apply_row_lr(const Geom& g, const Vec<VEC>& c, float lft, float rgt,
                                                 const Vec<VEC>& yl, const Vec<VEC>& yh, const Vec<VEC>& zl,
                                                 const Vec<VEC>& zh) {
    Vec<VEC> out;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        const float ce = c.f[e];
        const float l = e > 0 ? c.f[e - 1] : lft;
        const float r = e + 1 < VEC ? c.f[e + 1] : rgt;
        const float c2 = ce + ce;
        float v = fmaf(g.cx, (c2 - l) - r, ce);
        v = fmaf(g.cy, (c2 - yl.f[e]) - yh.f[e], v);
        out.f[e] = fmaf(g.cz, (c2 - zl.f[e]) - zh.f[e], v);
    }
    return out;
}

// Preconditioning sweep of degree 2: z = c0 r + c1 A r + c2 A (A r), both
// products matrix-free.  The wave marches over z keeping r for planes z ..
// z+2 with two halo rows on each side and A r for planes z-1 .. z+1 with one
// halo row: when plane z+2 of r arrives, A r of plane z+1 is formed, and then
// A (A r) of plane z.  Values at clamped rows or planes beyond a wall are
// never used (the wall rule substitutes the cell itself).  One wave covers a
// row (nx <= 64 VEC, a multiple of VEC; lanes beyond it load the row's last
// cells and store and add nothing).  FIRST: the input is b (zero initial
// guess) and b.b is accumulated as well.
template <int VEC, int TY, bool FIRST, bool RECT = false>
__device__ __forceinline__ void tile_precond2(const Ptrs& p, const Geom& g, size_t fo, int yg, int zb, int ze,
                                              int lane, double& acc0, double& acc1) {
    constexpr int RR = TY + 4;  // rows of r: y0 - 2 .. y0 + TY + 1
    constexpr int RA = TY + 2;  // rows of A r: y0 - 1 .. y0 + TY
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int x0 = lane * VEC;
    const bool xin = x0 < nx;
    const bool wall_l = x0 == 0, wall_r = x0 + VEC >= nx;
    const int y0 = yg * TY;
    const size_t plane = (size_t)nx * ny;
    const size_t base = fo + (xin ? x0 : nx - VEC);
    const float* src = FIRST ? p.B : p.R;
    auto at = [&](int z, int y) -> size_t {
        z = z < 0 ? 0 : (z >= nz ? nz - 1 : z);
        y = y < 0 ? 0 : (y >= ny ? ny - 1 : y);
        return base + (size_t)z * plane + (size_t)y * nx;
    };
    auto load_plane = [&](Vec<VEC>* dst, int z) {
#pragma unroll
        for (int i = 0; i < RR; ++i) dst[i] = ldv<VEC>(src + at(z, y0 - 2 + i));
    };
    RectX<VEC> X;
    if constexpr (RECT) X = rect_x<VEC>(g, x0);
    // A r for the RA rows of plane q, from r planes q-1 (lo), q (c), q+1 (hi)
    auto ar_plane = [&](Vec<VEC>* dst, const Vec<VEC>* lo, const Vec<VEC>* c, const Vec<VEC>* hi, int q) {
        const bool hzd = q > 0, hzu = q + 1 < nz;
#pragma unroll
        for (int jj = 0; jj < RA; ++jj) {
            const int y = y0 - 1 + jj;
            RectYZ yz;
            if constexpr (RECT) yz = rect_yz(g, y, q);
            dst[jj] = apply_row<VEC, RECT>(g, c[jj + 1], c[jj], c[jj + 2], lo[jj + 1], hi[jj + 1], y > 0, y + 1 < ny,
                                           hzd, hzu, wall_l, wall_r, &X, &yz);
        }
    };

    Vec<VEC> r0[RR], r1[RR], r2[RR];  // r of planes z, z+1, z+2 (in the loop)
    Vec<VEC> a0[RA], a1[RA], a2[RA];  // A r of planes z-1, z, z+1
    {
        Vec<VEC> rm[RR];
        load_plane(rm, zb - 2);
        load_plane(r0, zb - 1);
        load_plane(r1, zb);
        load_plane(r2, zb + 1);
        ar_plane(a0, rm, r0, r1, zb - 1);
        ar_plane(a1, r0, r1, r2, zb);
        // shift so that r0, r1 hold planes zb, zb + 1
#pragma unroll
        for (int i = 0; i < RR; ++i) {
            r0[i] = r1[i];
            r1[i] = r2[i];
        }
    }
    for (int z = zb; z < ze; ++z) {
        load_plane(r2, z + 2);
        ar_plane(a2, r0, r1, r2, z + 1);
        const bool hzd = z > 0, hzu = z + 1 < nz;
#pragma unroll
        for (int j = 0; j < TY; ++j) {
            const int y = y0 + j;
            RectYZ yz;
            if constexpr (RECT) yz = rect_yz(g, y, z);
            const Vec<VEC> aar = apply_row<VEC, RECT>(g, a1[j + 1], a1[j], a1[j + 2], a0[j + 1], a2[j + 1], y > 0,
                                                      y + 1 < ny, hzd, hzu, wall_l, wall_r, &X, &yz);
            const Vec<VEC>& rv = r0[j + 2];
            Vec<VEC> zv;
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                zv.f[e] = fmaf(g.c2, aar.f[e], fmaf(g.c1, a1[j + 1].f[e], g.c0 * rv.f[e]));
            if (xin && y < ny) {
                stv<VEC>(p.Z + at(z, y), zv);
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    acc0 = fma((double)rv.f[e], (double)zv.f[e], acc0);
                    if (FIRST) acc1 = fma((double)rv.f[e], (double)rv.f[e], acc1);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < RR; ++i) {
            r0[i] = r1[i];
            r1[i] = r2[i];
        }
#pragma unroll
        for (int jj = 0; jj < RA; ++jj) {
            a0[jj] = a1[jj];
            a1[jj] = a2[jj];
        }
    }
}

}  // namespace stencil
}  // namespace cgd
