// Learned diagonal preconditioner: a 4 -> 64 -> 2 MLP over per-column
// statistics (forward, loss gradient, backward, Adam), and the diagonal of
// the logistic-loss Hessian used to build its training targets.
//
// Parameters (FP32, 450 floats): W1[64][4], b1[64], W2[2][64], b2[2].
// Row r of the network's input is one column of one problem:
//   pre = W1 f + b1, h = relu(pre), o = W2 h + b2.
// o[0] predicts log d_k (a per-feature step scale), o[1] is averaged over the
// problem's columns into its log step size.
// Every reduction runs in a fixed order: per-block partial sums, then an
// ordered sum of the partials.
#include "internal.hpp"
#include "misc.hpp"

namespace casgd {

constexpr int kIn = 4, kHid = 64, kOut = 2;
constexpr int kW1 = 0, kB1 = kW1 + kHid * kIn, kW2 = kB1 + kHid, kB2 = kW2 + kOut * kHid,
              kParams = kB2 + kOut;
static_assert(kParams == 450, "parameter layout");
constexpr int kRowsPerBlock = 64;

// f = (log(1 + |stat|) - mu) / sd
__global__ void k_mlp_features(const float* stats, int64_t N, const float* norm, float* feats) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N * kIn) return;
    const int c = (int)(i % kIn);
    feats[i] = (log1pf(fabsf(stats[i])) - norm[c]) / norm[kIn + c];
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float* params, const float* feats,
                                                     int64_t N, float* out, float* pre_out) {
    __shared__ float P[kParams];
    for (int q = threadIdx.x; q < kParams; q += blockDim.x) P[q] = params[q];
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    float f[kIn];
#pragma unroll
    for (int c = 0; c < kIn; ++c) f[c] = feats[r * kIn + c];
    float o[kOut] = {P[kB2], P[kB2 + 1]};
    for (int j = 0; j < kHid; ++j) {
        float p = P[kB1 + j];
#pragma unroll
        for (int c = 0; c < kIn; ++c) p = fmaf(P[kW1 + j * kIn + c], f[c], p);
        if (pre_out) pre_out[r * kHid + j] = p;
        const float h = fmaxf(p, 0.f);
#pragma unroll
        for (int q = 0; q < kOut; ++q) o[q] = fmaf(P[kW2 + q * kHid + j], h, o[q]);
    }
#pragma unroll
    for (int q = 0; q < kOut; ++q) out[r * kOut + q] = o[q];
}

// Loss over P problems (rows seg_off[p] .. seg_off[p+1]-1):
//   L = mean_rows (o0 - t_d)^2 + w_eta * mean_p (mean_rows(p) o1 - t_eta[p])^2
// writes dL/do (N x 2) and L (FP64). One block per problem computes the
// problem's mean of o1 and its loss terms; block 0 of a second kernel sums
// the per-problem terms in order.
__global__ __launch_bounds__(256) void k_mlp_loss_problem(const float* out, const int64_t* seg_off,
                                                          int P, int64_t N, const float* t_d,
                                                          const float* t_eta, float w_eta,
                                                          float* g_out, double* terms) {
    const int p = blockIdx.x;
    const int64_t r0 = seg_off[p], r1 = seg_off[p + 1];
    __shared__ double s1[256], s0[256];
    double a1 = 0.0, a0 = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        a1 += out[r * kOut + 1];
        const double e = (double)out[r * kOut] - (double)t_d[r];
        a0 += e * e;
    }
    s1[threadIdx.x] = a1;
    s0[threadIdx.x] = a0;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s1[threadIdx.x] += s1[threadIdx.x + w];
            s0[threadIdx.x] += s0[threadIdx.x + w];
        }
        __syncthreads();
    }
    const double cnt = (double)(r1 - r0);
    const double mean1 = cnt > 0 ? s1[0] / cnt : 0.0;
    const double e1 = mean1 - (double)t_eta[p];
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        g_out[r * kOut] = (float)(2.0 * ((double)out[r * kOut] - (double)t_d[r]) / (double)N);
        g_out[r * kOut + 1] = (float)(w_eta * 2.0 * e1 / ((double)P * cnt));
    }
    if (threadIdx.x == 0) {
        terms[2 * p] = s0[0];
        terms[2 * p + 1] = e1 * e1;
    }
}

__global__ void k_mlp_loss_total(const double* terms, int P, int64_t N, float w_eta, double* loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.0, c = 0.0;
    for (int p = 0; p < P; ++p) {
        a += terms[2 * p];
        c += terms[2 * p + 1];
    }
    *loss = a / (double)N + (double)w_eta * c / (double)P;
}

// Backward over a block of kRowsPerBlock rows: g_pre = (W2^T g_o) * [pre > 0],
// then thread q sums parameter q's gradient over the block's rows in order.
__global__ __launch_bounds__(256) void k_mlp_backward(const float* params, const float* feats,
                                                      const float* pre, const float* g_out,
                                                      int64_t N, float* partial) {
    __shared__ float W2[kOut * kHid];
    __shared__ float gp[kRowsPerBlock][kHid + 1];
    __shared__ float hh[kRowsPerBlock][kHid + 1];
    __shared__ float ff[kRowsPerBlock][kIn];
    __shared__ float go[kRowsPerBlock][kOut];
    for (int q = threadIdx.x; q < kOut * kHid; q += blockDim.x) W2[q] = params[kW2 + q];
    const int64_t r0 = (int64_t)blockIdx.x * kRowsPerBlock;
    const int nr = (int)min<int64_t>(kRowsPerBlock, N - r0);
    for (int q = threadIdx.x; q < kRowsPerBlock * kOut; q += blockDim.x) {
        const int rr = q / kOut, o = q % kOut;
        go[rr][o] = rr < nr ? g_out[(r0 + rr) * kOut + o] : 0.f;
    }
    for (int q = threadIdx.x; q < kRowsPerBlock * kIn; q += blockDim.x) {
        const int rr = q / kIn, c = q % kIn;
        ff[rr][c] = rr < nr ? feats[(r0 + rr) * kIn + c] : 0.f;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kRowsPerBlock * kHid; q += blockDim.x) {
        const int rr = q / kHid, j = q % kHid;
        float p = 0.f, g = 0.f;
        if (rr < nr) {
            p = pre[(r0 + rr) * kHid + j];
            g = W2[j] * go[rr][0] + W2[kHid + j] * go[rr][1];
        }
        hh[rr][j] = fmaxf(p, 0.f);
        gp[rr][j] = p > 0.f ? g : 0.f;
    }
    __syncthreads();
    float* out = partial + (int64_t)blockIdx.x * kParams;
    for (int q = threadIdx.x; q < kParams; q += blockDim.x) {
        float a = 0.f;
        if (q < kB1) {                       // W1[j][c]
            const int j = q / kIn, c = q % kIn;
            for (int rr = 0; rr < nr; ++rr) a = fmaf(gp[rr][j], ff[rr][c], a);
        } else if (q < kW2) {                // b1[j]
            const int j = q - kB1;
            for (int rr = 0; rr < nr; ++rr) a += gp[rr][j];
        } else if (q < kB2) {                // W2[o][j]
            const int o = (q - kW2) / kHid, j = (q - kW2) % kHid;
            for (int rr = 0; rr < nr; ++rr) a = fmaf(go[rr][o], hh[rr][j], a);
        } else {                             // b2[o]
            const int o = q - kB2;
            for (int rr = 0; rr < nr; ++rr) a += go[rr][o];
        }
        out[q] = a;
    }
}

__global__ void k_mlp_grad_sum(const float* partial, int nblk, float* grad) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= kParams) return;
    float a = 0.f;
    for (int k = 0; k < nblk; ++k) a += partial[(int64_t)k * kParams + q];
    grad[q] = a;
}

// Adam (Kingma and Ba, 2015) with bias correction; t counts from 1.
__global__ void k_adam(float* p, const float* g, float* m1, float* m2, int count, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const float gq = g[q];
    const float a = b1 * m1[q] + (1.f - b1) * gq;
    const float v = b2 * m2[q] + (1.f - b2) * gq * gq;
    m1[q] = a;
    m2[q] = v;
    p[q] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// Diagonal of the Hessian of the mean logistic loss plus lambda at x:
//   H_kk = m^-1 sum_i s(z_i)(1 - s(z_i)) a_ik^2 + lambda,  z_i = a_i^T x.
// Pass 1 (k_logit_weight): w_i = s(z_i)(1 - s(z_i)) (one wave per row).
// Pass 2 (k_hess_diag): thread per column, row blocks as partials, ordered sum.
template <int DT>
__global__ __launch_bounds__(256) void k_logit_weight(const void* Xv, const float* scale, int64_t m,
                                                      int64_t n, int64_t ld, const float* x,
                                                      float* w) {
    using T = typename Store<DT>::T;
    constexpr int VEC = Store<DT>::kVec;
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= m) return;
    const T* row = static_cast<const T*>(Xv) + i * ld;
    float z = 0.f;
    for (int64_t c = (int64_t)lane * VEC; c < n; c += 64 * VEC) {
        const V16 v = load_v16<DT>(row, c, n);
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            if (c + e < n) z = fmaf(v16_elem<DT>(v, e), x[c + e], z);
    }
    z = group_sum<64>(z);
    if (scale) z *= scale[i];
    if (lane == 0) {
        const double sg = 1.0 / (1.0 + exp(-(double)z));
        w[i] = (float)(sg * (1.0 - sg));
    }
}

template <int DT>
__global__ __launch_bounds__(256) void k_hess_partial(const void* X, const float* scale, int64_t m,
                                                      int64_t n, int64_t ld, const float* w,
                                                      double* partial) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const int64_t rows = (m + gridDim.y - 1) / gridDim.y;
    const int64_t i0 = (int64_t)blockIdx.y * rows, i1 = min(m, i0 + rows);
    double a = 0.0;
    for (int64_t i = i0; i < i1; ++i) {
        float v;
        if constexpr (DT == DT_F32) v = static_cast<const float*>(X)[i * ld + k];
        else if constexpr (DT == DT_BF16) v = bf16_to_float(static_cast<const uint16_t*>(X)[i * ld + k]);
        else if constexpr (DT == DT_F16) v = f16_to_float(static_cast<const uint16_t*>(X)[i * ld + k]);
        else v = e4m3_to_float(static_cast<const uint8_t*>(X)[i * ld + k]);
        if (scale) v *= scale[i];
        a += (double)w[i] * (double)v * (double)v;
    }
    partial[(int64_t)blockIdx.y * n + k] = a;
}

__global__ void k_hess_final(const double* partial, int nrb, int64_t m, int64_t n, double lambda,
                             float* hdiag) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double a = 0.0;
    for (int rb = 0; rb < nrb; ++rb) a += partial[(int64_t)rb * n + k];
    hdiag[k] = (float)(a / (double)m + lambda);
}

// ------------------------------------------- single-workgroup reductions
// The per-problem post-processing below reduces over at most a few hundred
// thousand values, so one 1024-thread workgroup does it: every thread sums a
// fixed stride in FP64, then a fixed-shape tree over LDS.
constexpr int kRedThreads = 1024;

__device__ double block_sum_f64(double v, double* lds) {
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();
    return r;
}

// norm[c] = mean_k log(1 + |stats[k][c]|), norm[4 + c] = max(sample std, 1e-6).
__global__ __launch_bounds__(kRedThreads) void k_feature_norm(const float* stats, int64_t N,
                                                               float* norm) {
    __shared__ double lds[kRedThreads];
    for (int c = 0; c < kIn; ++c) {
        double a = 0.0;
        for (int64_t k = threadIdx.x; k < N; k += kRedThreads)
            a += log1p(fabs((double)stats[k * kIn + c]));
        const double mu = block_sum_f64(a, lds) / (double)N;
        double q = 0.0;
        for (int64_t k = threadIdx.x; k < N; k += kRedThreads) {
            const double v = log1p(fabs((double)stats[k * kIn + c])) - mu;
            q += v * v;
        }
        const double var = block_sum_f64(q, lds) / (double)(N > 1 ? N - 1 : 1);
        if (threadIdx.x == 0) {
            norm[c] = (float)mu;
            norm[kIn + c] = (float)fmax(sqrt(var), 1e-6);
        }
    }
}

// q_k = exp(clamp(out[k][0] - mean_k out[k][0], -20, 20) / 2), the column scale
// sqrt(d_k); eta = exp(mean_k out[k][1]).
__global__ __launch_bounds__(kRedThreads) void k_mlp_apply(const float* out, int64_t N, float* q,
                                                            float* eta) {
    __shared__ double lds[kRedThreads];
    double a0 = 0.0, a1 = 0.0;
    for (int64_t k = threadIdx.x; k < N; k += kRedThreads) {
        a0 += (double)out[k * kOut];
        a1 += (double)out[k * kOut + 1];
    }
    const double mu0 = block_sum_f64(a0, lds) / (double)N;
    const double mu1 = block_sum_f64(a1, lds) / (double)N;
    for (int64_t k = threadIdx.x; k < N; k += kRedThreads)
        q[k] = (float)exp(0.5 * fmin(fmax((double)out[k * kOut] - mu0, -20.0), 20.0));
    if (threadIdx.x == 0) eta[0] = (float)exp(mu1);
}

// t_d = -log h + mean_k log h_k (centred); q = exp(t_d / 2) when q is not null.
__global__ __launch_bounds__(kRedThreads) void k_jacobi_target(const float* h, int64_t n,
                                                                float* t_d, float* q) {
    __shared__ double lds[kRedThreads];
    double a = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += kRedThreads) a += log((double)h[k]);
    const double mu = block_sum_f64(a, lds) / (double)n;
    for (int64_t k = threadIdx.x; k < n; k += kRedThreads) {
        const double t = mu - log((double)h[k]);
        t_d[k] = (float)t;
        if (q) q[k] = (float)exp(0.5 * t);
    }
}

// ------------------------------------------------------------------ host

casgd_status run_mlp_features(const float* stats, int64_t N, const float* norm, float* feats,
                              hipStream_t st) {
    const int64_t tot = N * kIn;
    if (tot == 0) return CASGD_OK;
    hipLaunchKernelGGL(k_mlp_features, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                       stats, N, norm, feats);
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

casgd_status run_mlp_forward(const float* params, const float* feats, int64_t N, float* out,
                             float* pre, hipStream_t st) {
    if (N == 0) return CASGD_OK;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, params,
                       feats, N, out, pre);
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

size_t mlp_loss_ws(int P) { return (size_t)P * 2 * sizeof(double); }

casgd_status run_mlp_loss_grad(const float* out, const int64_t* seg_off, int P, int64_t N,
                               const float* t_d, const float* t_eta, float w_eta, double* loss,
                               float* g_out, double* terms, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_loss_problem, dim3(P), dim3(256), 0, st, out, seg_off, P, N, t_d,
                       t_eta, w_eta, g_out, terms);
    CASGD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_mlp_loss_total, dim3(1), dim3(64), 0, st, terms, P, N, w_eta, loss);
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

size_t mlp_backward_ws(int64_t N) {
    const int64_t nblk = (N + kRowsPerBlock - 1) / kRowsPerBlock;
    return (size_t)std::max<int64_t>(nblk, 1) * kParams * sizeof(float);
}

casgd_status run_mlp_backward(const float* params, const float* feats, const float* pre,
                              const float* g_out, int64_t N, float* grad, float* partial,
                              hipStream_t st) {
    const int nblk = (int)((N + kRowsPerBlock - 1) / kRowsPerBlock);
    if (nblk > 0) {
        hipLaunchKernelGGL(k_mlp_backward, dim3(nblk), dim3(256), 0, st, params, feats, pre, g_out,
                           N, partial);
        CASGD_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_mlp_grad_sum, dim3((kParams + 255) / 256), dim3(256), 0, st, partial,
                       nblk, grad);
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

casgd_status run_adam(float* p, const float* g, float* m1, float* m2, int count, int64_t t,
                      float lr, float b1, float b2, float eps, hipStream_t st) {
    const float c1 = 1.f - (float)std::pow((double)b1, (double)t);
    const float c2 = 1.f - (float)std::pow((double)b2, (double)t);
    hipLaunchKernelGGL(k_adam, dim3((count + 255) / 256), dim3(256), 0, st, p, g, m1, m2, count, lr,
                       b1, b2, eps, c1, c2);
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

size_t hess_ws(const casgd_matrix* X) {
    return (size_t)kStatRowBlocks * X->n * sizeof(double) + (size_t)X->m * sizeof(float) + 256;
}

casgd_status run_hess_diag(const casgd_matrix* X, const float* x, double lambda, float* hdiag,
                           void* ws, hipStream_t st) {
    double* partial = static_cast<double*>(ws);
    float* w = reinterpret_cast<float*>(static_cast<char*>(ws) +
                                        (((size_t)kStatRowBlocks * X->n * sizeof(double) + 255) &
                                         ~(size_t)255));
    const dim3 g1((unsigned)((X->m + 3) / 4)), g2((unsigned)((X->n + 255) / 256), kStatRowBlocks);
    switch (X->dtype) {
        case DT_F32:
            hipLaunchKernelGGL(k_logit_weight<DT_F32>, g1, dim3(256), 0, st, X->values, X->row_scale,
                               X->m, X->n, X->ld, x, w);
            hipLaunchKernelGGL(k_hess_partial<DT_F32>, g2, dim3(256), 0, st, X->values,
                               X->row_scale, X->m, X->n, X->ld, w, partial);
            break;
        case DT_BF16:
            hipLaunchKernelGGL(k_logit_weight<DT_BF16>, g1, dim3(256), 0, st, X->values,
                               X->row_scale, X->m, X->n, X->ld, x, w);
            hipLaunchKernelGGL(k_hess_partial<DT_BF16>, g2, dim3(256), 0, st, X->values,
                               X->row_scale, X->m, X->n, X->ld, w, partial);
            break;
        case DT_F16:
            hipLaunchKernelGGL(k_logit_weight<DT_F16>, g1, dim3(256), 0, st, X->values,
                               X->row_scale, X->m, X->n, X->ld, x, w);
            hipLaunchKernelGGL(k_hess_partial<DT_F16>, g2, dim3(256), 0, st, X->values,
                               X->row_scale, X->m, X->n, X->ld, w, partial);
            break;
        default:
            hipLaunchKernelGGL(k_logit_weight<DT_FP8>, g1, dim3(256), 0, st, X->values,
                               X->row_scale, X->m, X->n, X->ld, x, w);
            hipLaunchKernelGGL(k_hess_partial<DT_FP8>, g2, dim3(256), 0, st, X->values,
                               X->row_scale, X->m, X->n, X->ld, w, partial);
            break;
    }
    CASGD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_hess_final, dim3((unsigned)((X->n + 255) / 256)), dim3(256), 0, st,
                       partial, kStatRowBlocks, X->m, X->n, lambda, hdiag);
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

casgd_status run_feature_norm(const float* stats, int64_t N, float* norm, hipStream_t st) {
    hipLaunchKernelGGL(k_feature_norm, dim3(1), dim3(kRedThreads), 0, st, stats, N, norm);
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

casgd_status run_mlp_apply(const float* out, int64_t N, float* q, float* eta, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_apply, dim3(1), dim3(kRedThreads), 0, st, out, N, q, eta);
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

casgd_status run_jacobi_target(const float* h, int64_t n, float* t_d, float* q, hipStream_t st) {
    hipLaunchKernelGGL(k_jacobi_target, dim3(1), dim3(kRedThreads), 0, st, h, n, t_d, q);
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

}  // namespace casgd
