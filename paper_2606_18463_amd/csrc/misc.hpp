// Host launchers of the auxiliary kernels (sampling, storage conversion, loss,
// column statistics) and of the sparse path.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/casgd.h"

namespace casgd {

casgd_status run_sample(uint64_t seed, uint64_t t0, int64_t count, int64_t m, int64_t* out,
                        hipStream_t st);
casgd_status run_quantize(const float* src, int64_t m, int64_t n, int64_t ld_src, int dtype,
                          void* dst, int64_t ld_dst, float* row_scale, const float* col_scale,
                          hipStream_t st);
constexpr int kLossBlocks = 256;     // partial sums per weight vector
constexpr int kStatRowBlocks = 64;   // row blocks of the column statistics
casgd_status run_loss(const casgd_matrix* X, const float* y, const float* xs, int64_t count,
                      int64_t x_stride, int loss, double* out, double* partial, hipStream_t st);
casgd_status run_colstats(const casgd_matrix* X, float* stats, double* partial, hipStream_t st);

casgd_status run_mlp_features(const float* stats, int64_t N, const float* norm, float* feats,
                              hipStream_t st);
casgd_status run_mlp_forward(const float* params, const float* feats, int64_t N, float* out,
                             float* pre, hipStream_t st);
size_t mlp_loss_ws(int P);
casgd_status run_mlp_loss_grad(const float* out, const int64_t* seg_off, int P, int64_t N,
                               const float* t_d, const float* t_eta, float w_eta, double* loss,
                               float* g_out, double* terms, hipStream_t st);
size_t mlp_backward_ws(int64_t N);
casgd_status run_mlp_backward(const float* params, const float* feats, const float* pre,
                              const float* g_out, int64_t N, float* grad, float* partial,
                              hipStream_t st);
casgd_status run_adam(float* p, const float* g, float* m1, float* m2, int count, int64_t t,
                      float lr, float b1, float b2, float eps, hipStream_t st);
casgd_status run_feature_norm(const float* stats, int64_t N, float* norm, hipStream_t st);
casgd_status run_mlp_apply(const float* out, int64_t N, float* q, float* eta, hipStream_t st);
casgd_status run_jacobi_target(const float* h, int64_t n, float* t_d, float* q, hipStream_t st);
size_t hess_ws(const casgd_matrix* X);
casgd_status run_hess_diag(const casgd_matrix* X, const float* x, double lambda, float* hdiag,
                           void* ws, hipStream_t st);

casgd_status sparse_workspace_size(const casgd_matrix* X, int32_t b, int32_t s, int32_t lanes,
                                   size_t* bytes);
casgd_status sparse_prepare(const casgd_matrix* X, int32_t b, int32_t s, int32_t lanes, void* ws,
                            size_t ws_bytes, void* stream);
casgd_status sparse_fit(const casgd_matrix* X, const float* y, float* x_lanes,
                        const double* lambdas_host, int32_t L, double eta, int32_t b, int32_t s,
                        uint64_t seed, uint64_t outer_begin, int64_t n_outer,
                        const casgd_opts* opts, void* ws, size_t ws_bytes, void* stream);

}  // namespace casgd
