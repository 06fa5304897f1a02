// Sparse (CSR) s-step SGD path.
#include "internal.hpp"
#include "misc.hpp"

namespace casgd {

casgd_status sparse_workspace_size(const casgd_matrix* X, int32_t b, int32_t s, int32_t lanes,
                                   size_t* bytes) {
    (void)X; (void)b; (void)s; (void)lanes; (void)bytes;
    set_error("the CSR path is not available in this build");
    return CASGD_EUNSUPPORTED;
}

casgd_status sparse_fit(const casgd_matrix* X, const float* y, float* x_lanes,
                        const double* lambdas_host, int32_t L, double eta, int32_t b, int32_t s,
                        uint64_t seed, uint64_t outer_begin, int64_t n_outer,
                        const casgd_opts* opts, void* ws, size_t ws_bytes, void* stream) {
    (void)X; (void)y; (void)x_lanes; (void)lambdas_host; (void)L; (void)eta; (void)b; (void)s;
    (void)seed; (void)outer_begin; (void)n_outer; (void)opts; (void)ws; (void)ws_bytes;
    (void)stream;
    set_error("the CSR path is not available in this build");
    return CASGD_EUNSUPPORTED;
}

}  // namespace casgd
