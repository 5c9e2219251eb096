// Tetrahedral mesh data: host build products and their device copies.
#pragma once

#include <vector>

#include "cgd_internal.h"

namespace cgd {

struct TetHost {
    int64_t n_vert = 0;
    int32_t n_tet = 0;
    int64_t n_interior_faces = 0;
    int64_t nnz = 0;              // non-zeros of K: n_tet + 2 * n_interior_faces
    int64_t max_bucket = 0;
    std::vector<double> vol;      // [n_tet]
    std::vector<double> bbox;     // [n_tet][6]: min xyz, max xyz
    std::vector<float> kface;     // [n_tet][4]: a_f of the face opposite vertex j (0: boundary face)
    std::vector<float> kdiag;     // [n_tet]: K_ii = sum of the tet's a_f
    int32_t nb[3] = {1, 1, 1};    // bucket grid
    double glo[3] = {0, 0, 0}, ghi[3] = {0, 0, 0}, ginv[3] = {0, 0, 0};
    std::vector<int64_t> bstart;  // [nb + 1]
    std::vector<int32_t> blist;   // tets per bucket, ascending ids
    std::vector<int32_t> bseed;   // [nb]: walk start per bucket (-1: empty bucket)
    std::vector<int32_t> nbr;     // [n_tet][4]: tet across the face opposite vertex j (own id: boundary)
};

struct TetData {
    int32_t n_tet = 0;
    int64_t n_vert = 0;
    int64_t nnz = 0;
    int32_t nb[3] = {1, 1, 1};
    double glo[3], ghi[3], ginv[3];
    double* xyz = nullptr;      // [n_vert][3]
    int32_t* tv = nullptr;      // [n_tet][4]
    double* vol = nullptr;      // [n_tet]
    float* volf = nullptr;      // [n_tet]
    double* bbox = nullptr;     // [n_tet][6]
    float* kface = nullptr;     // [n_tet][4]
    float* kdiag = nullptr;
    int64_t* bstart = nullptr;
    int32_t* blist = nullptr;
    int32_t* bseed = nullptr;
    int32_t* nbr = nullptr;     // [n_tet][4]: the padded rows' column indices
    // Rectilinear hex meshes use the same padded rows with 6 face slots: the
    // first four in nbr / kface (-x, +x, -y, +y), the last two here (-z, +z).
    int32_t ns = 4;             // face slots per row: 4 (tets) or 6 (rectilinear hexes)
    int32_t* nbr2 = nullptr;    // [n][2]
    float* kface2 = nullptr;    // [n][2]
    int32_t rdim[3] = {0, 0, 0};
    double* redges = nullptr;   // node coordinates: x (rdim[0] + 1), then y, then z
    // Operator of the polynomial preconditioner: face coefficients a_f / amax
    // in float16 (one rounding per face, shared by its two rows, so the
    // operator stays symmetric) and their float sum per row.
    _Float16* kh = nullptr;     // [n][4]
    _Float16* kh2 = nullptr;    // [n][2] (6 face slots)
    float* kdh = nullptr;       // [n]
    double amax = 0.0;          // largest a_f
    double sum_v = 0.0;         // sum of V
    double sum_k = 0.0;         // sum of amax * kdh
    double kv_max = 0.0;        // max of amax * kdh / V
};

// Fills the preconditioner's operator fields of t from the float face
// coefficients (kface2 empty for 4 slots) and the volumes, and uploads them.
cgd_status cheb_operator_setup(TetData* t, const std::vector<float>& kface, const std::vector<float>& kface2,
                               const std::vector<double>& vol);

// D: cell-wise diffusivity [n_tet] (nullable: 1 everywhere).
cgd_status build_tet_host(int64_t n_vert, const double* xyz, int64_t n_tet, const int32_t* tv, const float* D,
                          TetHost* out);

size_t diffuse_tet_workspace(const cgd_mesh m, int32_t F);

}  // namespace cgd
