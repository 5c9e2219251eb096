// Placeholder for the unstructured path until its kernels exist.
#include "cgd_internal.h"

namespace cgd {
cgd_status deposit_tet(cgd_mesh, int64_t, const float*, int32_t, const float*, float*, int64_t*,
                       DepositInfo*, hipStream_t) {
    set_error("tet meshes are not available");
    return CGD_E_UNSUPPORTED;
}
cgd_status diffuse_tet(cgd_mesh, const DiffuseArgs&, cgd_solve_stats*, hipStream_t) {
    set_error("tet meshes are not available");
    return CGD_E_UNSUPPORTED;
}
void destroy_tet_data(cgd_mesh) {}
int64_t tet_nnz(cgd_mesh) { return 0; }
}  // namespace cgd

extern "C" cgd_status cgd_mesh_create_tet(int64_t, const double*, int64_t, const int32_t*, cgd_mesh* out) {
    if (out) *out = nullptr;
    cgd::set_error("tet meshes are not available");
    return CGD_E_UNSUPPORTED;
}
