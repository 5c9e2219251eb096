// Centroid binning on a uniform hex grid (Section 2.2: the host cell is the
// cell that contains the particle centroid).  Shared by the single and the
// batched deposit.  The function body is compiled without floating-point
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
// closed box.  u = (x - lo) * s, i = floor(u), clamped to [0, N-1].
__device__ inline int64_t hex_cell(const HexBin& g, float fx, float fy, float fz, bool* nonfinite) {
#pragma clang fp contract(off)
    const float xs[3] = {fx, fy, fz};
    int64_t idx[3];
    *nonfinite = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double x = (double)xs[a];
        if (!isfinite(x)) {
            *nonfinite = true;
            return -1;
        }
        if (!(x >= g.lo[a] && x <= g.hi[a])) return -1;
        double u = (x - g.lo[a]) * g.s[a];
        int64_t i = (int64_t)floor(u);
        i = i < 0 ? 0 : i;
        i = i > g.n[a] - 1 ? g.n[a] - 1 : i;
        idx[a] = i;
    }
    return idx[0] + (int64_t)g.n[0] * (idx[1] + (int64_t)g.n[1] * idx[2]);
}


}  // namespace cgd
