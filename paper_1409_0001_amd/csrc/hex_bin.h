// Centroid binning on uniform and rectilinear hex grids (Section 2.2: the
// host cell is the cell that contains the particle centroid).  Shared by the
// single and the batched deposit and the point location.  The function body is compiled without floating-point
// contraction so that the float64 expression is exactly (x - lo) * s.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cgd {

struct HexBin {
    double lo[3], hi[3], s[3];
    int32_t n[3];
};

// Host cell of one centroid; -1 if the point is not finite or outside the
// closed box.  u = (x - lo) * s, i = floor(u), clamped to [0, N-1].  The axes
// are tested in order x, y, z and *nonfinite tells whether the first failing
// axis was a non-finite coordinate.  Written without branches: every axis is
// evaluated, the clamp is done in float64 (identical to clamping the integer
// floor) and the in-range value is converted to int32 natively.
__device__ inline int64_t hex_cell(const HexBin& g, float fx, float fy, float fz, bool* nonfinite) {
#pragma clang fp contract(off)
    const float xs[3] = {fx, fy, fz};
    int32_t idx[3];
    bool done = false, nf = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double x = (double)xs[a];
        const bool fin = isfinite(x);
        const bool in = x >= g.lo[a] && x <= g.hi[a];
        nf = nf || (!done && !fin);
        done = done || !fin || !in;
        const double u = (x - g.lo[a]) * g.s[a];
        const double c = fmin(fmax(floor(u), 0.0), (double)(g.n[a] - 1));
        idx[a] = (int32_t)c;
    }
    *nonfinite = nf;
    if (done) return -1;
    return idx[0] + (int64_t)g.n[0] * (idx[1] + (int64_t)g.n[1] * idx[2]);
}

// Rectilinear hexes (Section 2.2 with the cell given by the edges): along
// each axis the largest i < N with e_i <= x (the upper cell at an interior
// face, the last cell on the upper wall); -1 outside the closed box.
struct RectLoc {
    const double* e;  // x edges, then y, then z
    int n[3];
    __device__ int operator()(const double* p) const {
        const double* ea = e;
        int id[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int na = n[a];
            if (!(p[a] >= ea[0] && p[a] <= ea[na])) return -1;
            int lo = 0, hi = na - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (ea[mid] <= p[a]) lo = mid;
                else hi = mid - 1;
            }
            id[a] = lo;
            ea += na + 1;
        }
        return id[0] + n[0] * (id[1] + n[1] * id[2]);
    }
};

}  // namespace cgd
