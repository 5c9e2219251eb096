// Host-side construction of a tetrahedral mesh (done once per mesh).
//
// The paper's method needs, on an arbitrary unstructured mesh, only the cell
// volumes and the immediate face neighbours (Section 2.5.1 contrasts this
// with the kernel method's non-local search; Section 4.3 runs it on
// unstructured meshes).  From the vertex coordinates and the tet -> vertex
// table this builds:
//   - volumes V = det[v1-v0, v2-v0, v3-v0] / 6 (positive orientation required)
//   - interior faces by matching the sorted vertex triples of all tet faces
//   - the two-point-flux Laplacian K: a_f = D_f |A_f| / |c_N - c_P| between
//     the centroids of the two tets of each interior face (D_f the harmonic
//     mean of the two tets' diffusivities, 1 without them); boundary faces
//     carry no flux.  K is stored as a sparse matrix with rows padded to the four
//     face slots a tet has: row t's off-diagonal entries are -a_f at columns
//     nbr[t][j] (float32 values, int32 columns; a boundary slot holds the
//     tet's own id and 0), the diagonal K_tt = sum of the tet's a_f
//   - per-tet bounding boxes and a uniform bucket grid listing, for every
//     bucket, the tets whose bounding box overlaps it, and per bucket a seed
//     tet for point location by walking across the face slots
#pragma clang fp contract(off)

#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "tet_data.h"

namespace cgd {

namespace {

struct Face {
    int32_t v[3];
    int32_t tet;
    int32_t j;  // local index of the vertex opposite the face
};

// det[b - a, c - a, p - a] (the device's orientation expression)
inline double orient_h(const double* a, const double* b, const double* c, const double* p) {
    const double u0 = b[0] - a[0], u1 = b[1] - a[1], u2 = b[2] - a[2];
    const double v0 = c[0] - a[0], v1 = c[1] - a[1], v2 = c[2] - a[2];
    const double w0 = p[0] - a[0], w1 = p[1] - a[1], w2 = p[2] - a[2];
    return u0 * (v1 * w2 - v2 * w1) - u1 * (v0 * w2 - v2 * w0) + u2 * (v0 * w1 - v1 * w0);
}

// Whether p lies in the closed tet t (each face evaluated on its vertices in
// increasing id order, as on the device).
bool contains_h(const double* xyz, const int32_t* tv, int32_t t, const double* p) {
    const int32_t* ids = tv + (size_t)t * 4;
    for (int j = 0; j < 4; ++j) {
        int32_t f[3], k = 0;
        for (int i = 0; i < 4; ++i)
            if (i != j) f[k++] = ids[i];
        std::sort(f, f + 3);
        const double sp = orient_h(xyz + 3 * (size_t)f[0], xyz + 3 * (size_t)f[1], xyz + 3 * (size_t)f[2], p);
        const double sd = orient_h(xyz + 3 * (size_t)f[0], xyz + 3 * (size_t)f[1], xyz + 3 * (size_t)f[2],
                                   xyz + 3 * (size_t)ids[j]);
        const double sg = sd > 0.0 ? 1.0 : (sd < 0.0 ? -1.0 : 0.0);
        if (!(sp * sg >= 0.0)) return false;
    }
    return true;
}

inline double det3(const double* a, const double* b, const double* c, const double* d) {
    const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    const double e3[3] = {d[0] - a[0], d[1] - a[1], d[2] - a[2]};
    return e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
           e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
}

}  // namespace

cgd_status build_tet_host(int64_t n_vert, const double* xyz, int64_t n_tet, const int32_t* tv, const float* D,
                          TetHost* out) {
    if (n_vert < 4 || n_tet < 1 || n_tet > (int64_t)INT32_MAX / 8 || n_vert > INT32_MAX) {
        set_error("cgd_mesh_create_tet: need n_vert >= 4 and 1 <= n_tet < 2^28");
        return CGD_E_INVALID;
    }
    if (D) {
        for (int64_t t = 0; t < n_tet; ++t) {
            if (!(D[t] >= 0.f) || !isfinite(D[t])) {
                set_error("cgd_mesh_create_tet_d: diffusivity must be finite and >= 0 (tet " + std::to_string(t) +
                          ")");
                return CGD_E_INVALID;
            }
        }
    }
    const int32_t nt = (int32_t)n_tet;
    out->n_vert = n_vert;
    out->n_tet = nt;
    out->vol.resize(nt);
    out->bbox.resize((size_t)nt * 6);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < n_vert * 3; ++i) {
        if (!isfinite(xyz[i])) {
            set_error("cgd_mesh_create_tet: non-finite vertex coordinate");
            return CGD_E_INVALID;
        }
    }
    std::vector<double> cen((size_t)nt * 3);
    for (int32_t t = 0; t < nt; ++t) {
        const int32_t* v = tv + (size_t)t * 4;
        for (int j = 0; j < 4; ++j) {
            if (v[j] < 0 || v[j] >= n_vert) {
                set_error("cgd_mesh_create_tet: vertex id out of range in tet " + std::to_string(t));
                return CGD_E_INVALID;
            }
        }
        const double* p[4] = {xyz + 3 * (size_t)v[0], xyz + 3 * (size_t)v[1], xyz + 3 * (size_t)v[2],
                              xyz + 3 * (size_t)v[3]};
        const double d = det3(p[0], p[1], p[2], p[3]);
        if (!(d > 0.0)) {
            set_error("cgd_mesh_create_tet: tet " + std::to_string(t) + " is not positively oriented");
            return CGD_E_INVALID;
        }
        out->vol[t] = fabs(d) / 6.0;
        for (int a = 0; a < 3; ++a) {
            double mn = p[0][a], mx = p[0][a];
            for (int j = 1; j < 4; ++j) {
                mn = std::min(mn, p[j][a]);
                mx = std::max(mx, p[j][a]);
            }
            out->bbox[(size_t)t * 6 + a] = mn;
            out->bbox[(size_t)t * 6 + 3 + a] = mx;
            lo[a] = std::min(lo[a], mn);
            hi[a] = std::max(hi[a], mx);
            cen[(size_t)t * 3 + a] = (((p[0][a] + p[1][a]) + p[2][a]) + p[3][a]) / 4.0;
        }
    }

    // faces: the face opposite vertex j of each tet, vertex ids sorted
    std::vector<Face> faces((size_t)nt * 4);
    for (int32_t t = 0; t < nt; ++t) {
        const int32_t* v = tv + (size_t)t * 4;
        for (int j = 0; j < 4; ++j) {
            Face& f = faces[(size_t)t * 4 + j];
            int k = 0;
            for (int i = 0; i < 4; ++i)
                if (i != j) f.v[k++] = v[i];
            std::sort(f.v, f.v + 3);
            f.tet = t;
            f.j = j;
        }
    }
    std::sort(faces.begin(), faces.end(), [](const Face& a, const Face& b) {
        if (a.v[0] != b.v[0]) return a.v[0] < b.v[0];
        if (a.v[1] != b.v[1]) return a.v[1] < b.v[1];
        if (a.v[2] != b.v[2]) return a.v[2] < b.v[2];
        return a.tet < b.tet;
    });
    // face slots: the tet across each face and the face's coefficient a_f;
    // a boundary face keeps the tet's own id and a_f = 0 (no flux)
    out->nbr.resize((size_t)nt * 4);
    for (int32_t t = 0; t < nt; ++t)
        for (int j = 0; j < 4; ++j) out->nbr[(size_t)t * 4 + j] = t;
    out->kface.assign((size_t)nt * 4, 0.f);
    std::vector<double> diag(nt, 0.0);
    int64_t n_int = 0;
    const size_t nf = faces.size();
    for (size_t i = 0; i < nf;) {
        size_t j = i + 1;
        while (j < nf && faces[j].v[0] == faces[i].v[0] && faces[j].v[1] == faces[i].v[1] &&
               faces[j].v[2] == faces[i].v[2])
            ++j;
        if (j - i > 2) {
            set_error("cgd_mesh_create_tet: a face is shared by more than two tets");
            return CGD_E_INVALID;
        }
        if (j - i == 2) {
            const int32_t P = faces[i].tet, N = faces[i + 1].tet;
            const double* a = xyz + 3 * (size_t)faces[i].v[0];
            const double* b = xyz + 3 * (size_t)faces[i].v[1];
            const double* c = xyz + 3 * (size_t)faces[i].v[2];
            const double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
            const double w[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
            const double cr[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
            const double area = 0.5 * sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
            const double dc[3] = {cen[(size_t)N * 3] - cen[(size_t)P * 3], cen[(size_t)N * 3 + 1] - cen[(size_t)P * 3 + 1],
                                  cen[(size_t)N * 3 + 2] - cen[(size_t)P * 3 + 2]};
            const double dist = sqrt(dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2]);
            double af = area / dist;
            if (D) {
                // the face diffusivity: harmonic mean of the two cells' D,
                // 0 when either is 0 (Section 5.2's local diffusion constant)
                const double da = (double)D[P], db = (double)D[N];
                af = af * ((da > 0.0 && db > 0.0) ? 2.0 * da * db / (da + db) : 0.0);
            }
            out->nbr[(size_t)P * 4 + faces[i].j] = N;
            out->nbr[(size_t)N * 4 + faces[i + 1].j] = P;
            out->kface[(size_t)P * 4 + faces[i].j] = (float)af;
            out->kface[(size_t)N * 4 + faces[i + 1].j] = (float)af;
            diag[P] += af;
            diag[N] += af;
            ++n_int;
        }
        i = j;
    }
    out->n_interior_faces = n_int;
    out->nnz = (int64_t)nt + 2 * n_int;
    out->kdiag.resize(nt);
    for (int32_t t = 0; t < nt; ++t) out->kdiag[t] = (float)diag[t];

    // bucket grid over the vertex bounding box: about one tet-sized cell per
    // 6 tets; every tet is listed in each bucket its bounding box overlaps
    const double span[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
    const double vol_box = std::max(span[0], 1e-300) * std::max(span[1], 1e-300) * std::max(span[2], 1e-300);
    const double cell = cbrt(vol_box / std::max(1.0, nt / 6.0));
    int64_t nbt = 1;
    for (int a = 0; a < 3; ++a) {
        int n = (int)std::max(1.0, std::min(1024.0, round(span[a] / cell)));
        out->nb[a] = n;
        out->glo[a] = lo[a];
        out->ghi[a] = hi[a];
        out->ginv[a] = span[a] > 0 ? n / span[a] : 0.0;
        nbt *= n;
    }
    auto bucket_range = [&](int32_t t, int a, int* i0, int* i1) {
        const double mn = out->bbox[(size_t)t * 6 + a], mx = out->bbox[(size_t)t * 6 + 3 + a];
        int b0 = (int)floor((mn - lo[a]) * out->ginv[a]);
        int b1 = (int)floor((mx - lo[a]) * out->ginv[a]);
        *i0 = std::max(0, std::min(out->nb[a] - 1, b0));
        *i1 = std::max(0, std::min(out->nb[a] - 1, b1));
    };
    std::vector<int64_t> cnt(nbt + 1, 0);
    for (int32_t t = 0; t < nt; ++t) {
        int r0[3], r1[3];
        for (int a = 0; a < 3; ++a) bucket_range(t, a, &r0[a], &r1[a]);
        for (int z = r0[2]; z <= r1[2]; ++z)
            for (int y = r0[1]; y <= r1[1]; ++y)
                for (int x = r0[0]; x <= r1[0]; ++x) cnt[(size_t)x + out->nb[0] * ((size_t)y + (size_t)out->nb[1] * z) + 1]++;
    }
    for (int64_t b = 0; b < nbt; ++b) cnt[b + 1] += cnt[b];
    if (cnt[nbt] > INT32_MAX) {
        set_error("cgd_mesh_create_tet: point-location grid too large");
        return CGD_E_INVALID;
    }
    out->bstart.assign(cnt.begin(), cnt.end());
    out->blist.assign(cnt[nbt], 0);
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int32_t t = 0; t < nt; ++t) {  // ascending tet ids within each bucket
        int r0[3], r1[3];
        for (int a = 0; a < 3; ++a) bucket_range(t, a, &r0[a], &r1[a]);
        for (int z = r0[2]; z <= r1[2]; ++z)
            for (int y = r0[1]; y <= r1[1]; ++y)
                for (int x = r0[0]; x <= r1[0]; ++x)
                    out->blist[pos[(size_t)x + out->nb[0] * ((size_t)y + (size_t)out->nb[1] * z)]++] = t;
    }
    int64_t maxb = 0;
    for (int64_t b = 0; b < nbt; ++b) maxb = std::max<int64_t>(maxb, cnt[b + 1] - cnt[b]);
    out->max_bucket = maxb;
    // walk seeds: per bucket, the first listed tet that contains the bucket's
    // centre (else the first listed tet; -1 for an empty bucket)
    out->bseed.assign(nbt, -1);
    for (int z = 0; z < out->nb[2]; ++z)
        for (int y = 0; y < out->nb[1]; ++y)
            for (int x = 0; x < out->nb[0]; ++x) {
                const size_t b = (size_t)x + out->nb[0] * ((size_t)y + (size_t)out->nb[1] * z);
                if (cnt[b] == cnt[b + 1]) continue;
                const double c[3] = {lo[0] + (x + 0.5) * (span[0] / out->nb[0]),
                                     lo[1] + (y + 0.5) * (span[1] / out->nb[1]),
                                     lo[2] + (z + 0.5) * (span[2] / out->nb[2])};
                int32_t seed = out->blist[cnt[b]];
                for (int64_t k = cnt[b]; k < cnt[b + 1]; ++k) {
                    const int32_t t = out->blist[k];
                    const double* bb = &out->bbox[(size_t)t * 6];
                    if (c[0] < bb[0] || c[1] < bb[1] || c[2] < bb[2] || c[0] > bb[3] || c[1] > bb[4] || c[2] > bb[5])
                        continue;
                    if (contains_h(xyz, tv, t, c)) {
                        seed = t;
                        break;
                    }
                }
                out->bseed[b] = seed;
            }
    return CGD_OK;
}

}  // namespace cgd
