// Polynomial preconditioning sweep of a uniform hex grid with the powers of
// A in LDS: one block's tile (TY rows of y, planes [zb, ze)), shared by the
// per-launch solver (cg_hex.hip) and the persistent batched one
// (batched.hip).  Requires nx = 64 VEC (one wave per x-row).
#pragma once

#include "stencil_tile.h"

namespace cgd {
namespace stencil {

// LDS barrier that waits only for this wave's LDS operations, so global
// loads issued ahead (the prefetched planes) stay in flight across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// x-neighbours of a lane's end cells across the wave (DPP wave shifts): the
// last cell of the lane below and the first cell of the lane above; lanes 0
// and 63 keep their own end cell (the wall rule).
template <int VEC>
__device__ __forceinline__ void x_neighbours(const Vec<VEC>& c, float& lft, float& rgt) {
    lft = __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(c.f[0]), __float_as_int(c.f[VEC - 1]),
                                                     0x138 /* wave_shr:1 */, 0xf, 0xf, false));
    rgt = __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(c.f[VEC - 1]), __float_as_int(c.f[0]),
                                                     0x130 /* wave_shl:1 */, 0xf, 0xf, false));
}

// z = p(A) r with p(l) = sum_j cp[j] l^j,
// evaluated by Horner's rule, u_D = cp[D] r, u_j = cp[j] r + A u_{j+1},
// z = u_0, every product matrix-free.  A block of NW waves owns TY rows of y
// (one wave per x-row, nx = 64 VEC) and marches over its z chunk.  u_{D-j}
// is needed up to D - j rows and planes away from the block's output, so
// wave w handles the row y0 - D + w at every level whose extent holds it.
// At step t, level j forms u_{D-j} of plane q = t - j: the row's own values
// of the previous level at planes q-1, q, q+1 come from the wave's
// registers (it formed them at steps t-2, t-1, t), the rows above and below
// at plane q from LDS, where their waves wrote them at step t-1, and the
// x-neighbours from DPP shifts.  LDS holds three planes of r and of level 1
// (level 2 reads its own row's level-1 planes there, which saves a register
// ring) and two of each higher level (written at steps of one parity, read
// at the next), so a step needs one barrier.  The steps are unrolled by 6 so
// that every register ring (r: 6 planes, levels >= 2: 3 planes) is indexed
// at compile time.  r enters LDS through the waves that
// own no output row: they keep P planes of loads in flight and never store,
// while the output waves only store, so neither kind waits for the other's
// memory operations.  Rows and planes beyond a wall take the cell itself
// (the wall rule): rows by pointing at the cell's own row, planes through
// per-plane coefficients.  FIRST: the input is b (zero initial guess) and
// b.b is accumulated as well.

// Coefficients of the Horner levels, formed on the host so that a kernel
// picks them with scalar selects (the vector unit would otherwise recompute
// the wall-dependent diagonal at every level and step): level j = 1..D forms
// u = cr r + ca A u_prev, ca = cp[D] at j = 1 and 1 above, as
// u = kd c + cr r + nkx (x-neighbours) + nky (y-neighbours) + nkz (z-neighbours)
// with kd[w] = ca (1 + 2 (cx + cy + cz) - cz [no plane below] - cz [no plane
// above]), w = (no plane below) + 2 (no plane above), and nk = -ca c (stored
// negated so that every term is one multiply-add with a scalar operand); a
// missing plane also drops its nkz term.
// The rectilinear operator (RECT tiles) has per-cell coefficients, formed
// in the tile from the per-axis factors; a level there is u = gg (A u_prev)
// + gs u_prev + cr (extra term), with gg and gs below.
constexpr int kPcMaxD = 4;
struct PrecondCoef {
    float kd[kPcMaxD][4];
    float nkx[kPcMaxD], nky[kPcMaxD], nkz[kPcMaxD], cr[kPcMaxD];
    float gg[kPcMaxD], gs[kPcMaxD];
};

// cp: the D + 1 polynomial coefficients (float64, from poly_precond_coeffs_n).
inline void precond_coef_fill(PrecondCoef& pc, float cx, float cy, float cz, const double* cp, int D) {
    pc = PrecondCoef{};
    const float d_in = 1.f + 2.f * (cx + cy + cz);
    for (int j = 1; j <= D && j <= kPcMaxD; ++j) {
        const float ca = j == 1 ? (float)cp[D] : 1.f;
        for (int w = 0; w < 4; ++w) pc.kd[j - 1][w] = ca * (d_in - ((w & 1) ? cz : 0.f) - ((w & 2) ? cz : 0.f));
        pc.nkx[j - 1] = -(ca * cx);
        pc.nky[j - 1] = -(ca * cy);
        pc.nkz[j - 1] = -(ca * cz);
        pc.cr[j - 1] = (float)cp[D - j];
        pc.gg[j - 1] = ca;
        pc.gs[j - 1] = 0.f;
    }
}

// One pass of the product form of the preconditioner (FORM 1 and 2 below):
// levels 1..4 apply two quadratic factors to the pass's input v,
// u1 = A v, u2 = g1 (A u1 + s1 u1 + q1 v), u3 = A u2, u4 = g2 last (A u3 +
// s2 u3 + q2 u2), in the coefficients above (kd folds s and the walls; cr
// weights the level's extra term: v at level 2, u2 at level 4, none at odd
// levels).  s, q, g: the pass's two factors (poly_precond_quadratics); last:
// the polynomial's overall scale on the final pass, else 1.  D = 2: one
// factor per pass (levels 1 and 2).
inline void precond_coef_fill_quadratics(PrecondCoef& pc, float cx, float cy, float cz, const double* s,
                                         const double* q, const double* g, double last, int D = 4) {
    pc = PrecondCoef{};
    const double d_in = 1.0 + 2.0 * ((double)cx + (double)cy + (double)cz);
    for (int j = 1; j <= D; ++j) {
        const bool even = (j & 1) == 0;
        const int k = (j - 1) / 2;
        const double gg = even ? g[k] * (j == D ? last : 1.0) : 1.0;
        const double sh = even ? s[k] : 0.0;
        for (int w = 0; w < 4; ++w)
            pc.kd[j - 1][w] = (float)(gg * (d_in - ((w & 1) ? cz : 0.0) - ((w & 2) ? cz : 0.0) + sh));
        pc.nkx[j - 1] = (float)(-gg * cx);
        pc.nky[j - 1] = (float)(-gg * cy);
        pc.nkz[j - 1] = (float)(-gg * cz);
        pc.cr[j - 1] = even ? (float)(gg * q[k]) : 0.f;
        pc.gg[j - 1] = (float)gg;
        pc.gs[j - 1] = (float)(gg * sh);
    }
}

// First LDS row of level j (rows of TY + 2 (D - i) per plane; 3 planes for
// levels 0 and 1, 2 planes above).
template <int D, int TY>
__host__ __device__ constexpr int lds_level_base(int j) {
    int rows = 0;
    for (int i = 0; i < j; ++i) rows += (i <= 1 ? 3 : 2) * (TY + 2 * (D - i));
    return rows;
}

// RECT tiles: the z factors of every plane a block touches (its chunk and
// D halo planes each side) sit in an LDS table of kZtStride floats per
// plane, so the march reads them from LDS; the host keeps chunks of such
// tiles to at most kRectZMax - 2 D planes.
constexpr int kRectZMax = 264, kZtStride = 8;

// LDS floats a tile needs: levels 0..D-1 (precond_lds_tile's `lds`), for
// FORM 2 two planes of the output rows of r, and RECT's plane table.
template <int VEC, int D, int TY, int FORM = 0, bool RECT = false>
__host__ __device__ constexpr int precond_lds_floats() {
    return (lds_level_base<D, TY>(D) + (FORM == 2 ? 2 * TY : 0)) * 64 * VEC + (RECT ? kRectZMax * kZtStride : 0);
}

// lds: precond_lds_floats<VEC, D, TY, FORM>() floats of LDS, 16-byte aligned.
// FORM 0: z = p(A) r by Horner (src = r); acc0 = r.z (and acc1 = b.b when
// FIRST).  FORM 1 and 2 (D = 4, or D = 2 for one factor): one pass of the
// product form (src = the pass's input v; dst = its output); FORM 1 adds
// acc1 = v.v when FIRST (v = b), FORM 2 adds acc0 = r.dst with r read from
// side_field (the loaders feed the output rows of r through LDS).  RECT: the
// rectilinear operator of Geom (per-cell coefficients from per-axis
// factors; walls have zero face weights) with the levels' gg, gs.  PART:
// the row is shorter than the wave's 64 VEC cells (the last real lane takes
// the wall).  SIN /
// SOUT (RECT): the input is multiplied by the scaling S (Geom::rsg) as it
// enters LDS / the output by S before it is stored, so that the passes
// apply S p(A) S; FIRST then takes b.b from the loaders' unscaled rows, and
// FORM 0's r.z is (S r).p(A)(S r).
template <int VEC, int D, int TY, int NW, bool FIRST, bool PF = false, int FORM = 0, bool RECT = false,
          bool SIN = false, bool SOUT = false, bool PART = false>
__device__ inline void precond_lds_tile(float* __restrict__ lds, const float* __restrict__ src_field,
                                        float* __restrict__ dst_field, const Geom& g, const PrecondCoef& pc, int ny, int nz,
                                        int y0, int zb, int ze, double& acc0, double& acc1,
                                        const float* __restrict__ side_field = nullptr) {
    static_assert(FORM == 0 || D == 4 || D == 2, "the product form runs one or two quadratic factors per pass");
    constexpr int NXR = 64 * VEC;
    constexpr int E0 = TY + 2 * D;
    constexpr int NL = NW - TY;                  // waves owning no output row: the loaders
    constexpr int RPL = (E0 + NL - 1) / NL;      // rows of r per loader
    constexpr int P = (VEC <= 2 && FORM == 2) ? 1 : 2;  // planes of r in flight per loader
    static_assert(E0 <= NW, "one row per wave covers every level");
    static_assert(RPL <= 2, "loaders hold at most two rows");
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // A row of nx <= NXR cells (nx a multiple of VEC): lanes from nx / VEC
    // on hold copies of the row's last cells, are never stored and add
    // nothing to the sums; the last real lane takes the wall (or periodic)
    // rule on its right
    const int nx = g.nx;
    const int x0 = lane * VEC;
    const bool xin = x0 < nx;
    const int xg = xin ? x0 : nx - VEC;  // the column this lane loads
    const size_t plane = (size_t)nx * ny;

    // this wave's row; it is in level j's extent (extent row w - j) iff
    // j <= w < TY + 2 D - j
    // RECT: periodic axes (Geom::per): a row or plane beyond the grid is a
    // real one, wrapped (the rows of a wave's extent and the planes of a
    // chunk's halo compute like any other; only output rows are stored)
    const int per = RECT ? g.per : 0;
    const int yw = y0 - D + w;
    const int ywr = (per & 2) ? ((yw % ny) + ny) % ny : min(max(yw, 0), ny - 1);  // the row's data
    const bool in_dom = w < E0 && ((per & 2) || (yw >= 0 && yw < ny));
    const bool has_yd = yw > 0 || (per & 2), has_yu = yw + 1 < ny || (per & 2);
    auto wrapz = [&](int q) { return (per & 4) ? (q < 0 ? q + nz : (q >= nz ? q - nz : q)) : q; };
    const bool owner = w >= D && w < D + TY;  // an output row (written if yw < ny)
    const int li = w < D ? w : w - TY;        // loader index (non-owners)

    auto ld = [](const float* r) {  // row starts are 16-byte aligned: one LDS access per row
        return ldv<VEC>(static_cast<const float*>(__builtin_assume_aligned(r, 4 * VEC)));
    };
    const float* src = src_field + xg;
    auto ysrc = [&](int e) {  // clamped (or wrapped) row of extent row e of level 0
        const int y = (per & 2) ? ((y0 - D + e) % ny + ny) % ny : min(max(y0 - D + e, 0), ny - 1);
        return (size_t)y * nx;
    };

    // FORM 2: r of output row i at plane q in side slot q & 1, written by
    // loader i at step q + D - 1 (loaded one step earlier) and read by the
    // owner of the row at step q + D
    float* side_lds = lds + lds_level_base<D, TY>(D) * NXR;
    const float* side = FORM == 2 ? side_field + xg : nullptr;
    const size_t side_y = (size_t)min(y0 + (li < TY ? li : 0), ny - 1) * nx;
    auto side_load = [&](int q) { return ldv<VEC>(side + (size_t)min(max(q, 0), nz - 1) * plane + side_y); };

    const int t0 = (per & 4) ? zb - D : max(0, zb - D);
    const int tl = (per & 4) ? ze + D - 1 : min(nz, ze + D) - 1;  // last plane of r needed
    const int t1 = ze - 1 + D;           // last step (plane ze - 1 of z completes)
    // LDS slot of level j's plane q: (q - t0) mod 3 for levels 0 and 1, mod 2
    // above.  Relative to the chunk's first plane t0, so that in the step
    // loop (t = t0 + 6 k + S) every slot is a compile-time constant
    // (rowk in step), with no index arithmetic per access.
    auto row = [&](int j, int q, int e) -> float* {  // level j, plane q, extent row e
        const int slot = j <= 1 ? (q - t0 + 12) % 3 : ((q - t0 + 12) & 1);  // q >= t0 - D - 1
        return lds + (lds_level_base<D, TY>(j) + slot * (TY + 2 * (D - j)) + e) * NXR + x0;
    };
    auto row0 = [&](int q, int e) -> float* { return row(0, q, e); };
    (void)g;
    // RECT: this lane's x factors and this wave's row factors, for every
    // level, and the plane table (planes t0 .. tl: face weights below and
    // above, diagonal sum, diffusivity, identity factor, S), filled here and
    // first read after the barrier that ends the set-up below
    RectX<VEC> X;
    RectA Yw;
    float sgx[VEC], sgy = 1.f;  // S of this lane's cells on x, of this wave's row on y
    float* ztab = lds + (lds_level_base<D, TY>(D) + (FORM == 2 ? 2 * TY : 0)) * NXR;
    if constexpr (RECT) {
        X = rect_x<VEC>(g, x0);
        Yw = rect_a(g, 1, ywr, ny);
        for (int i = threadIdx.x; i < (tl - t0 + 1) * kZtStride; i += NW * 64) {
            const int q = wrapz(t0 + i / kZtStride), f = i % kZtStride;
            float v = 0.f;
            if (f == 0) v = g.rg[2][q];
            else if (f == 1) v = g.rg[2][q + 1];
            else if (f == 2) v = g.rs[2][q];
            else if (f == 3) v = g.rd[2][q];
            else if (f == 4) v = g.re[2][q];
            else if (f == 5) v = (SIN || SOUT) ? g.rsg[2][q] : 1.f;
            ztab[i] = v;
        }
    }
    if constexpr (SIN || SOUT) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) sgx[e] = g.rsg[0][xg + e];
        sgy = g.rsg[1][ywr];
    }
    // SIN: S on the y axis of the loader's rows (fixed for the march)
    float sgl[2] = {1.f, 1.f};
    // SIN: a row of the input entering LDS at plane q (extent row e, the
    // loader's row i): b.b over the output cells from the unscaled values,
    // then the scaling (S on z from the table, or from memory during the
    // set-up, before the table is complete)
    auto scale_in = [&](Vec<VEC>& v, int e, int i, int q, bool setup) {
        if constexpr (SIN) {
            const int y = y0 - D + e;
            if (FIRST && xin && e >= D && e < D + TY && y < ny && q >= zb && q < ze) {
#pragma unroll
                for (int k = 0; k < VEC; ++k) acc1 = fma((double)v.f[k], (double)v.f[k], acc1);
            }
            const int qc = min(max(q, t0), tl);  // a plane beyond tl holds tl's values (unused)
            const float sz = setup ? g.rsg[2][wrapz(qc)] : ztab[(qc - t0) * kZtStride + 5];
            const float syz = sgl[i] * sz;
#pragma unroll
            for (int k = 0; k < VEC; ++k) v.f[k] *= sgx[k] * syz;
        }
    };

    // r of this row, plane t0 + s at slot s mod RK: Horner (FORM 0) weights r
    // at every level (planes t - 1 .. t - D); the product form only at level 2
    constexpr int RK = FORM == 0 ? 6 : 3;
    Vec<VEC> rk[RK];
    Vec<VEC> lv[D > 2 ? D - 2 : 1][3];      // level j >= 2's u of this row, plane t0 + s at slot s mod 3
    Vec<VEC> u1;                            // level 1's u of this row formed at the current step
#pragma unroll
    for (int i = 0; i < RK; ++i)
#pragma unroll
        for (int e = 0; e < VEC; ++e) rk[i].f[e] = 0.f;
#pragma unroll
    for (int j = 0; j < D - 2; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int e = 0; e < VEC; ++e) lv[j][i].f[e] = 0.f;
#pragma unroll
    for (int e = 0; e < VEC; ++e) u1.f[e] = 0.f;

    // one step at t = t0 + S (mod 6); LOADER: the wave feeds r into LDS
    auto step = [&](auto S_, auto LOADER_, int t, Vec<VEC> (&pf)[P][RPL], Vec<VEC>& sr) {
        constexpr int S = decltype(S_)::value;
        constexpr bool LOADER = decltype(LOADER_)::value;
        // level j's row e at plane t + k, and the side slot of plane t + k:
        // t - t0 is S mod 6, so the slots fold to constants once the level
        // loop is unrolled
        auto rowk = [&](int j, int k, int e) -> float* {
            const int slot = j <= 1 ? (S + k + 12) % 3 : ((S + k + 12) & 1);
            return lds + (lds_level_base<D, TY>(j) + slot * (TY + 2 * (D - j)) + e) * NXR + x0;
        };
        auto side_rowk = [&](int k, int i) -> float* {
            return side_lds + (((S + k + 12) & 1) * TY + i) * NXR + x0;
        };
        if constexpr (LOADER && FORM == 2) {
            // side channel: output row li of r at plane t + 1 - D (in flight
            // since the previous step) into LDS, then the load of the next plane
            if (li < TY) stv<VEC>(side_rowk(1 - D, li), sr);
            sr = side_load(t + 2 - D);
        }
        if constexpr (LOADER) {
            // plane t + 1 (in flight since step t + 1 - P) into LDS, then
            // the load of plane t + 1 + P into the freed buffer
            constexpr int B = (S + 1) % P;
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const int e = li + NL * i;
                if (e < E0) {
                    scale_in(pf[B][i], e, i, t + 1, false);
                    stv<VEC>(rowk(0, 1, e), pf[B][i]);
                }
            }
            const int tn = min(t + 1 + P, tl);
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const int e = min(li + NL * i, E0 - 1);
                pf[B][i] = ldv<VEC>(src + (size_t)wrapz(tn) * plane + ysrc(e));
            }
        }
        if (w < E0) rk[S % RK] = ld(rowk(0, 0, w));  // own row of r at plane t (written at step t - 1)

        // Level j's rows y - 1 and y + 1 (level j - 1 at plane t - j, this
        // row itself at a wall) and level 2's planes q, q - 1 of level 1 were
        // all written at earlier steps.  PF: each level issues the next
        // level's LDS reads before its own arithmetic, so they are in flight
        // while it computes (faster in the persistent batched kernel at
        // nx = 128, slower at nx = 256, where it costs registers).  Level 2's
        // plane q + 1 of level 1 is the u that level 1 has just formed in
        // this wave (u1).
        auto go_of = [&](int j) {
            const int q = t - j;
            if (per & 4) return in_dom && j <= w && w < E0 - j && q >= zb - (D - j) && q < ze + (D - j);
            return in_dom && j <= w && w < E0 - j && q >= max(0, zb - (D - j)) && q < min(nz, ze + (D - j));
        };
        auto ys_rows = [&](int j, Vec<VEC>& yd, Vec<VEC>& yu) {
            yd = ld(rowk(j - 1, -j, has_yd ? w - j : w - j + 1));
            yu = ld(rowk(j - 1, -j, has_yu ? w - j + 2 : w - j + 1));
        };
        Vec<VEC> yd, yu, c2, zl2;
        if (PF && go_of(1)) ys_rows(1, yd, yu);
#pragma unroll
        for (int j = 1; j <= D; ++j) {
            const int q = t - j;
            const bool go = go_of(j);
            Vec<VEC> ydn, yun;
            if (PF && j < D && go_of(j + 1)) {
                ys_rows(j + 1, ydn, yun);
                if (j == 1) {
                    c2 = ld(rowk(1, -2, w - 1));
                    zl2 = ld((t - 2 > 0 || (per & 4)) ? rowk(1, -3, w - 1) : rowk(1, -2, w - 1));
                }
            }
            if (!PF && go) {
                // the same reads, issued just before their use
                ys_rows(j, yd, yu);
                if (j == 2) {
                    c2 = ld(rowk(1, -j, w - 1));
                    zl2 = ld((q > 0 || (per & 4)) ? rowk(1, -j - 1, w - 1) : rowk(1, -j, w - 1));
                }
            }
            if (go) {
                // previous level's u of this row at planes q - 1, q, q + 1:
                // r from the register ring, level 1 from LDS and u1, level >= 2
                // from its register ring
                Vec<VEC> c, zl, zh;
                if (j == 1) {
                    c = rk[((S - j) % RK + RK) % RK];
                    zl = rk[((S - j - 1) % RK + RK) % RK];
                    zh = rk[((S - j + 1) % RK + RK) % RK];
                } else if (j == 2) {
                    c = c2;
                    zl = zl2;
                    zh = u1;  // formed at this step when q + 1 < nz; else weighted by zero
                } else {
                    const int jr = j >= 3 ? j - 3 : 0;  // ring of level j - 1
                    c = lv[jr][((S - j) % 3 + 3) % 3];
                    zl = lv[jr][((S - j - 1) % 3 + 3) % 3];
                    zh = lv[jr][((S - j + 1) % 3 + 3) % 3];
                }
                // level 0 (r or v) of this row at plane q (FORM 1, 2: used at
                // levels 1 and 2 only, planes the 3-plane ring holds)
                const Vec<VEC>& rq = rk[((S - j) % RK + RK) % RK];
                // the level's extra term: r (FORM 0), v at level 2 and u2 at
                // level 4 (FORM 1, 2), none at odd levels of FORM 1, 2
                const Vec<VEC>& ex = (FORM != 0 && j == 4) ? lv[0][((S - 4) % 3 + 3) % 3] : rq;
                const bool has_ex = FORM == 0 || (j % 2) == 0;
                Vec<VEC> ys = yd;
#pragma unroll
                for (int e = 0; e < VEC; ++e) ys.f[e] += yu.f[e];
                float lft, rgt;
                x_neighbours<VEC>(c, lft, rgt);
                if constexpr (PART) rgt = x0 + VEC >= nx ? c.f[VEC - 1] : rgt;  // the row's last cell: wall
                if (per & 1) {
                    // periodic x: the row's end cells are neighbours
                    const float last =
                        __int_as_float(__builtin_amdgcn_readlane(__float_as_int(c.f[VEC - 1]), (nx - 1) / VEC));
                    const float first = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(c.f[0]), 0));
                    lft = lane == 0 ? last : lft;
                    rgt = x0 + VEC >= nx ? first : rgt;
                }
                // u = cp[D-j] r + ca A u_prev (ca = cp[D] at j = 1, else 1), with
                // ca folded into the stencil's coefficients (PrecondCoef).
                // Interior planes of a grid with h_x = h_y take the fast path:
                // loop-invariant scalar coefficients, 7 operations per cell;
                // wall planes and h_x != h_y the general one (8, with the
                // wall's coefficients selected per plane).
                const bool hzd = q > 0, hzu = q + 1 < nz;
                const float cr = pc.cr[j - 1];
                Vec<VEC> u;
                if constexpr (RECT) {
                    // u = gg (A c) + gs c + cr ex with A's coefficients of
                    // this row at plane q (gg folded into the row-and-plane
                    // products); a wall's face weight is zero, so whatever
                    // finite value stands beyond it drops out
                    const float* zt = ztab + (q - t0) * kZtStride;
                    const float4 z4 = *reinterpret_cast<const float4*>(zt);  // gd, gu, s, d
                    const RectYZ yz = rect_yz(g, Yw, RectA{z4.x, z4.y, z4.z, z4.w, zt[4]});
                    const float gg = pc.gg[j - 1], gs = pc.gs[j - 1];
                    const float nbd = -gg * yz.bd, nbu = -gg * yz.bu, ncd = -gg * yz.cd, ncu = -gg * yz.cu;
                    const float ge = gg * yz.e, gdyz = gg * yz.dyz, ga = gg * yz.a;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const float l = e > 0 ? c.f[e - 1] : lft;
                        const float r = e + 1 < VEC ? c.f[e + 1] : rgt;
                        const float xs = fmaf(X.gl[e], l, X.gr[e] * r);
                        const float yzs = fmaf(nbd, yd.f[e], fmaf(nbu, yu.f[e], fmaf(ncd, zl.f[e], ncu * zh.f[e])));
                        const float kdc = fmaf(X.e[e], ge, fmaf(X.s[e], gdyz, fmaf(X.d[e], ga, gs)));
                        float v = has_ex ? fmaf(kdc, c.f[e], cr * ex.f[e]) : kdc * c.f[e];
                        v = fmaf(-gdyz, xs, v);
                        u.f[e] = fmaf(X.d[e], yzs, v);
                    }
                } else if (hzd && hzu && pc.nkx[j - 1] == pc.nky[j - 1]) {
                    const float kd = pc.kd[j - 1][0], nkx = pc.nkx[j - 1], nkz = pc.nkz[j - 1];
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const float l = e > 0 ? c.f[e - 1] : lft;
                        const float r = e + 1 < VEC ? c.f[e + 1] : rgt;
                        float v = has_ex ? fmaf(kd, c.f[e], cr * ex.f[e]) : kd * c.f[e];
                        v = fmaf(nkx, (l + r) + ys.f[e], v);
                        v = fmaf(nkz, zl.f[e], v);
                        u.f[e] = fmaf(nkz, zh.f[e], v);
                    }
                } else {
                    const float kd = pc.kd[j - 1][(hzd ? 0 : 1) + (hzu ? 0 : 2)];
                    const float nkzd = hzd ? pc.nkz[j - 1] : 0.f, nkzu = hzu ? pc.nkz[j - 1] : 0.f;
                    const float nkx = pc.nkx[j - 1], nky = pc.nky[j - 1];
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const float l = e > 0 ? c.f[e - 1] : lft;
                        const float r = e + 1 < VEC ? c.f[e + 1] : rgt;
                        float v = has_ex ? fmaf(kd, c.f[e], cr * ex.f[e]) : kd * c.f[e];
                        v = fmaf(nkx, l + r, v);
                        v = fmaf(nky, ys.f[e], v);
                        v = fmaf(nkzd, zl.f[e], v);
                        u.f[e] = fmaf(nkzu, zh.f[e], v);
                    }
                }
                if (j == 1) u1 = u;
                if (FIRST && FORM == 1 && !SIN && j == 1 && owner && xin && yw < ny && q >= zb && q < ze) {
                    // b.b over the output cells, from this row's b at plane q
#pragma unroll
                    for (int e = 0; e < VEC; ++e) acc1 = fma((double)c.f[e], (double)c.f[e], acc1);
                }
                if (j < D) stv<VEC>(rowk(j, -j, w - j), u);
                // levels >= 2 keep their planes in a register ring; a slot
                // not written here keeps an older, finite plane that is only
                // ever read with a zero coefficient (beyond a wall)
                if (j >= 2 && j < D) lv[j >= 2 ? j - 2 : 0][((S - j) % 3 + 3) % 3] = u;
                if (j == D && owner && xin && yw < ny && q >= zb && q < ze) {
                    // output of plane q complete: store it and add r.z (and b.b)
                    Vec<VEC> us = u;
                    if constexpr (SOUT) {
                        const float syz = sgy * ztab[(q - t0) * kZtStride + 5];
#pragma unroll
                        for (int e = 0; e < VEC; ++e) us.f[e] *= sgx[e] * syz;
                    }
                    stv<VEC>(dst_field + xg + (size_t)q * plane + (size_t)yw * nx, us);
                    if constexpr (FORM == 2) {
                        const Vec<VEC> rr = ld(side_rowk(-j, w - D));
#pragma unroll
                        for (int e = 0; e < VEC; ++e) acc0 = fma((double)rr.f[e], (double)us.f[e], acc0);
                    }
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        if (FORM == 0) acc0 = fma((double)rq.f[e], (double)u.f[e], acc0);
                        if (FIRST && FORM == 0 && !SIN) acc1 = fma((double)rq.f[e], (double)rq.f[e], acc1);
                    }
                }
            }
            if (PF && j < D) {
                yd = ydn;
                yu = yun;
            }
        }
        lds_barrier();
    };

    auto run = [&](auto LOADER_) {
        constexpr bool LOADER = decltype(LOADER_)::value;
        Vec<VEC> pf[P][RPL];
        Vec<VEC> sr;  // FORM 2 loaders: the side plane in flight (plane t + 1 - D at step t)
        if constexpr (LOADER && FORM == 2) sr = side_load(t0 + 1 - D);
        if constexpr (LOADER) {
            // planes t0 .. t0 + P - 1 in flight; plane t0 into LDS; t0 + P replaces it
#pragma unroll
            for (int s = 0; s < P; ++s)
#pragma unroll
                for (int i = 0; i < RPL; ++i) {
                    const int e = min(li + NL * i, E0 - 1);
                    pf[s][i] = ldv<VEC>(src + (size_t)wrapz(min(t0 + s, tl)) * plane + ysrc(e));
                }
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const int e = li + NL * i;
                if constexpr (SIN) sgl[i] = g.rsg[1][ysrc(min(e, E0 - 1)) / nx];
                if (e < E0) {
                    scale_in(pf[0][i], e, i, t0, true);
                    stv<VEC>(row0(t0, e), pf[0][i]);
                }
            }
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const int e = min(li + NL * i, E0 - 1);
                pf[0][i] = ldv<VEC>(src + (size_t)wrapz(min(t0 + P, tl)) * plane + ysrc(e));
            }
        }
        lds_barrier();
        for (int t = t0; t <= t1; t += 6) {
            step(std::integral_constant<int, 0>{}, LOADER_, t, pf, sr);
            if (t + 1 > t1) break;
            step(std::integral_constant<int, 1>{}, LOADER_, t + 1, pf, sr);
            if (t + 2 > t1) break;
            step(std::integral_constant<int, 2>{}, LOADER_, t + 2, pf, sr);
            if (t + 3 > t1) break;
            step(std::integral_constant<int, 3>{}, LOADER_, t + 3, pf, sr);
            if (t + 4 > t1) break;
            step(std::integral_constant<int, 4>{}, LOADER_, t + 4, pf, sr);
            if (t + 5 > t1) break;
            step(std::integral_constant<int, 5>{}, LOADER_, t + 5, pf, sr);
        }
    };
    if (owner) run(std::false_type{});
    else run(std::true_type{});

}

}  // namespace stencil
}  // namespace cgd
