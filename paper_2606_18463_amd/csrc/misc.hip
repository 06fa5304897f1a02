// Auxiliary kernels: sampling, storage conversion (Table 1 storage slot),
// logistic loss on snapshots and per-column statistics.
#include "internal.hpp"
#include "misc.hpp"

namespace casgd {

// ---------------------------------------------------------------- sampling
__global__ void k_sample(uint64_t seed, uint64_t t0, int64_t count, uint64_t m, int64_t* out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < count) out[q] = sample_row(seed, t0 + (uint64_t)q, m);
}

casgd_status run_sample(uint64_t seed, uint64_t t0, int64_t count, int64_t m, int64_t* out,
                        hipStream_t st) {
    if (count == 0) return CASGD_OK;
    const int64_t grid = (count + 255) / 256;
    hipLaunchKernelGGL(k_sample, dim3((unsigned)grid), dim3(256), 0, st, seed, t0, count,
                       (uint64_t)m, out);
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

// ------------------------------------------------------ storage conversion
// One workgroup per row. FP8: amax over the row, scale = amax/448 and
// inv = 448/amax in FP32, codes = e4m3(x * inv).
__global__ __launch_bounds__(256) void k_quantize(const float* src, int64_t n, int64_t ld_src,
                                                  int dtype, void* dst, int64_t ld_dst,
                                                  float* row_scale, const float* col_scale) {
    const int64_t i = blockIdx.x;
    const float* row = src + i * ld_src;
    // value of column k: row[k] (times col_scale[k] if given, rounded to FP32)
    auto val = [&](int64_t k) { return col_scale ? row[k] * col_scale[k] : row[k]; };
    __shared__ float s_red[4];
    float inv = 1.0f, scale = 1.0f;
    if (dtype == DT_FP8) {
        float a = 0.f;
        for (int64_t k = threadIdx.x; k < n; k += 256) a = fmaxf(a, fabsf(val(k)));
        for (int off = 32; off > 0; off >>= 1) a = fmaxf(a, __shfl_xor(a, off, 64));
        if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = a;
        __syncthreads();
        const float amax = fmaxf(fmaxf(s_red[0], s_red[1]), fmaxf(s_red[2], s_red[3]));
        if (amax > 0.f) {
            scale = amax / 448.0f;
            inv = 448.0f / amax;
        }
    }
    if (row_scale && threadIdx.x == 0) row_scale[i] = scale;
    for (int64_t k = threadIdx.x; k < ld_dst; k += 256) {
        const float v = k < n ? val(k) : 0.0f;
        switch (dtype) {
            case DT_F32: static_cast<float*>(dst)[i * ld_dst + k] = v; break;
            case DT_BF16:
                static_cast<uint16_t*>(dst)[i * ld_dst + k] = (uint16_t)float_to_bf16(v);
                break;
            case DT_F16:
                static_cast<uint16_t*>(dst)[i * ld_dst + k] = (uint16_t)float_to_f16(v);
                break;
            default:
                static_cast<uint8_t*>(dst)[i * ld_dst + k] =
                    k < n ? (uint8_t)float_to_e4m3(v * inv) : (uint8_t)0;
                break;
        }
    }
}

casgd_status run_quantize(const float* src, int64_t m, int64_t n, int64_t ld_src, int dtype,
                          void* dst, int64_t ld_dst, float* row_scale, const float* col_scale,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_quantize, dim3((unsigned)m), dim3(256), 0, st, src, n, ld_src, dtype, dst,
                       ld_dst, row_scale, col_scale);
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

// --------------------------------------------------------------- loss
__device__ __forceinline__ double softplus(double v) {
    return (v > 0 ? v : 0.0) + log1p(exp(-fabs(v)));
}

// L(z, y) of Sec. 2.1 in FP64: logistic through the stable softplus, linear
// (z - y)^2 / 2, Poisson exp(z) - y z.
__device__ __forceinline__ double glm_loss(double z, double y, int loss) {
    if (loss == LOSS_LINEAR) return 0.5 * (z - y) * (z - y);
    if (loss == LOSS_POISSON) return exp(z) - y * z;
    return softplus(-y * z);
}

template <int DT>
__global__ __launch_bounds__(256) void k_loss_dense(const void* Xv, const float* scale,
                                                    int64_t m, int64_t n, int64_t ld,
                                                    const float* y, const float* xs,
                                                    int64_t x_stride, int loss, double* partial) {
    using T = typename Store<DT>::T;
    constexpr int VEC = Store<DT>::kVec;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t k = blockIdx.y;
    const float* x = xs + k * x_stride;
    const T* X = static_cast<const T*>(Xv);
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 4 + w; i < m; i += (int64_t)gridDim.x * 4) {
        const T* row = X + i * ld;
        float z = 0.f;
        for (int64_t c = (int64_t)lane * VEC; c < n; c += 64 * VEC) {
            const V16 v = load_v16<DT>(row, c, n);
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                if (c + e < n) z = fmaf(v16_elem<DT>(v, e), x[c + e], z);
        }
        z = group_sum<64>(z);
        if (scale) z *= scale[i];
        acc += glm_loss((double)z, (double)y[i], loss);
    }
    __shared__ double s[4];
    if (lane == 0) s[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[k * gridDim.x + blockIdx.x] = ((s[0] + s[1]) + s[2]) + s[3];
}

__global__ __launch_bounds__(256) void k_loss_csr(const int64_t* rp, const int32_t* ci,
                                                  const float* va, int64_t m, const float* y,
                                                  const float* xs, int64_t x_stride, int loss,
                                                  double* partial) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t k = blockIdx.y;
    const float* x = xs + k * x_stride;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 4 + w; i < m; i += (int64_t)gridDim.x * 4) {
        float z = 0.f;
        for (int64_t p = rp[i] + lane; p < rp[i + 1]; p += 64) z = fmaf(va[p], x[ci[p]], z);
        z = group_sum<64>(z);
        acc += glm_loss((double)z, (double)y[i], loss);
    }
    __shared__ double s[4];
    if (lane == 0) s[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[k * gridDim.x + blockIdx.x] = ((s[0] + s[1]) + s[2]) + s[3];
}

__global__ void k_loss_final(const double* partial, int64_t count, int nblk, int64_t m,
                             double* out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    double t = 0.0;
    for (int j = 0; j < nblk; ++j) t += partial[k * nblk + j];
    out[k] = t / (double)m;
}

casgd_status run_loss(const casgd_matrix* X, const float* y, const float* xs, int64_t count,
                      int64_t x_stride, int loss, double* out, double* partial, hipStream_t st) {
    const dim3 grid(kLossBlocks, (unsigned)count);
    if (X->layout == CASGD_CSR) {
        hipLaunchKernelGGL(k_loss_csr, grid, dim3(256), 0, st, X->row_ptr, X->col_idx,
                           static_cast<const float*>(X->values), X->m, y, xs, x_stride, loss, partial);
    } else {
        switch (X->dtype) {
            case DT_F32:
                hipLaunchKernelGGL(k_loss_dense<DT_F32>, grid, dim3(256), 0, st, X->values,
                                   X->row_scale, X->m, X->n, X->ld, y, xs, x_stride, loss, partial);
                break;
            case DT_BF16:
                hipLaunchKernelGGL(k_loss_dense<DT_BF16>, grid, dim3(256), 0, st, X->values,
                                   X->row_scale, X->m, X->n, X->ld, y, xs, x_stride, loss, partial);
                break;
            case DT_F16:
                hipLaunchKernelGGL(k_loss_dense<DT_F16>, grid, dim3(256), 0, st, X->values,
                                   X->row_scale, X->m, X->n, X->ld, y, xs, x_stride, loss, partial);
                break;
            default:
                hipLaunchKernelGGL(k_loss_dense<DT_FP8>, grid, dim3(256), 0, st, X->values,
                                   X->row_scale, X->m, X->n, X->ld, y, xs, x_stride, loss, partial);
                break;
        }
    }
    CASGD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_loss_final, dim3((unsigned)((count + 63) / 64)), dim3(64), 0, st,
                       partial, count, kLossBlocks, X->m, out);
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

// ------------------------------------------------------- column statistics
template <int DT>
__device__ __forceinline__ float load_elem(const void* X, int64_t off) {
    if constexpr (DT == DT_F32) return static_cast<const float*>(X)[off];
    else if constexpr (DT == DT_BF16) return bf16_to_float(static_cast<const uint16_t*>(X)[off]);
    else if constexpr (DT == DT_F16) return f16_to_float(static_cast<const uint16_t*>(X)[off]);
    else return e4m3_to_float(static_cast<const uint8_t*>(X)[off]);
}

// Thread per column, workgroup rows split into kStatRowBlocks row blocks;
// partial (s1, s2, count, max) per (row block, column) in FP64.
template <int DT>
__global__ __launch_bounds__(256) void k_colstats_dense(const void* X, const float* scale,
                                                        int64_t m, int64_t n, int64_t ld,
                                                        double* partial) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const int64_t rows = (m + gridDim.y - 1) / gridDim.y;
    const int64_t i0 = (int64_t)blockIdx.y * rows, i1 = min(m, i0 + rows);
    double s1 = 0.0, s2 = 0.0, cnt = 0.0, mx = 0.0;
    for (int64_t i = i0; i < i1; ++i) {
        float v = load_elem<DT>(X, i * ld + k);
        if (scale) v *= scale[i];
        const double d = v;
        s1 += d;
        s2 += d * d;
        cnt += (v != 0.f) ? 1.0 : 0.0;
        mx = fmax(mx, fabs(d));
    }
    double* p = partial + ((int64_t)blockIdx.y * n + k) * 4;
    p[0] = s1;
    p[1] = s2;
    p[2] = cnt;
    p[3] = mx;
}

__global__ void k_colstats_final(const double* partial, int nrb, int64_t m, int64_t n,
                                 float* stats) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double s1 = 0.0, s2 = 0.0, cnt = 0.0, mx = 0.0;
    for (int rb = 0; rb < nrb; ++rb) {
        const double* p = partial + ((int64_t)rb * n + k) * 4;
        s1 += p[0];
        s2 += p[1];
        cnt += p[2];
        mx = fmax(mx, p[3]);
    }
    const double mean = s1 / (double)m;
    stats[k * 4 + 0] = (float)mean;
    stats[k * 4 + 1] = (float)fmax(0.0, s2 / (double)m - mean * mean);
    stats[k * 4 + 2] = (float)(cnt / (double)m);
    stats[k * 4 + 3] = (float)mx;
}

// CSR: the same partial sums, by row block, scattered per column. A workgroup
// owns a row block and a column window; each thread scans the rows of the
// block and accumulates the entries that fall in its own column, so no two
// threads write the same partial.
__global__ __launch_bounds__(256) void k_colstats_csr(const int64_t* rp, const int32_t* ci,
                                                      const float* va, int64_t m, int64_t n,
                                                      double* partial) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t rows = (m + gridDim.y - 1) / gridDim.y;
    const int64_t i0 = (int64_t)blockIdx.y * rows, i1 = min(m, i0 + rows);
    const int64_t kw0 = (int64_t)blockIdx.x * 256;
    double s1 = 0.0, s2 = 0.0, cnt = 0.0, mx = 0.0;
    for (int64_t i = i0; i < i1; ++i) {
        // entries of row i inside [kw0, kw0+256): binary search for the start
        int64_t lo = rp[i], hi = rp[i + 1];
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (ci[mid] < kw0) lo = mid + 1; else hi = mid;
        }
        for (int64_t p = lo; p < rp[i + 1] && ci[p] < kw0 + 256; ++p) {
            if (ci[p] == k) {
                const double d = va[p];
                s1 += d;
                s2 += d * d;
                cnt += (va[p] != 0.f) ? 1.0 : 0.0;
                mx = fmax(mx, fabs(d));
            }
        }
    }
    if (k >= n) return;
    double* p = partial + ((int64_t)blockIdx.y * n + k) * 4;
    p[0] = s1;
    p[1] = s2;
    p[2] = cnt;
    p[3] = mx;
}

casgd_status run_colstats(const casgd_matrix* X, float* stats, double* partial, hipStream_t st) {
    const dim3 grid((unsigned)((X->n + 255) / 256), kStatRowBlocks);
    if (X->layout == CASGD_CSR) {
        hipLaunchKernelGGL(k_colstats_csr, grid, dim3(256), 0, st, X->row_ptr, X->col_idx,
                           static_cast<const float*>(X->values), X->m, X->n, partial);
    } else {
        switch (X->dtype) {
            case DT_F32:
                hipLaunchKernelGGL(k_colstats_dense<DT_F32>, grid, dim3(256), 0, st, X->values,
                                   X->row_scale, X->m, X->n, X->ld, partial);
                break;
            case DT_BF16:
                hipLaunchKernelGGL(k_colstats_dense<DT_BF16>, grid, dim3(256), 0, st, X->values,
                                   X->row_scale, X->m, X->n, X->ld, partial);
                break;
            case DT_F16:
                hipLaunchKernelGGL(k_colstats_dense<DT_F16>, grid, dim3(256), 0, st, X->values,
                                   X->row_scale, X->m, X->n, X->ld, partial);
                break;
            default:
                hipLaunchKernelGGL(k_colstats_dense<DT_FP8>, grid, dim3(256), 0, st, X->values,
                                   X->row_scale, X->m, X->n, X->ld, partial);
                break;
        }
    }
    CASGD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_colstats_final, dim3((unsigned)((X->n + 255) / 256)), dim3(256), 0, st,
                       partial, kStatRowBlocks, X->m, X->n, stats);
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

}  // namespace casgd
