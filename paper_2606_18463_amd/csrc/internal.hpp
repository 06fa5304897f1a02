// Host-side internals of libcasgd shared between translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/casgd.h"
#include "dense.hpp"

namespace casgd {

void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
casgd_status hip_fail(hipError_t e, const char* what);

#define CASGD_HIP(call)                                   \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

int dtype_bytes(int dtype);
int dtype_vec(int dtype);          // elements per 16-byte vector
int slice_width_of(int dtype);     // columns per update / margin slice


// Workspace layout of one dense problem (byte offsets, 256-byte aligned).
struct DenseLayout {
    int sb, ts, ntiles, needed, gt, bt, gna, ksplit, nslices, t128, n128;
    int sk_nslots;      // partial slots of the stand-alone K-split Gram region (0: none)
    int64_t kchunk, ldy, ldg;
    size_t off_flags, off_tilecnt, off_G0, off_G1, off_Gpart, off_rp0, off_rp1, off_c, off_r, off_pub,
        off_Y[3], off_yI[3], off_sI[3], total;
    size_t total_sk;    // total plus the K-split Gram region (epoch line + slots)
};

bool dense_layout(int64_t n, int dtype, int b, int s, DenseLayout* L);
// Binds the workspace; the K-split Gram region is used when ws_bytes holds it.
void dense_bind(const DenseLayout& L, void* ws, size_t ws_bytes, Dense* P);

// Tuning knobs chosen by the host (or the autotuner).
struct FitPlan {
    int exec_mode;      // 1 persistent, 2 stream-ordered
    int variant;        // 1 redundant recurrence (one barrier/outer), 2 single recurrence group
    int grid;           // persistent grid size
    int recur64;        // FP64 recurrence
    int gram128;        // Gram units are 128 x 128 LDS tiles
    unsigned long long spin;
};

// Gram unit kind: 128 x 128 LDS tiles when asked for (gram_tile 128), or
// automatically when there are enough of them for the workgroups that build
// the Gram (see choose_gram128).
bool choose_gram128(const Dense& P, int dtype, int gram_tile, int gram_workgroups);

casgd_status plan_fit(const Dense& P, int dtype, const casgd_opts* o, int64_t H, FitPlan* plan);
casgd_status run_fit(const Dense& P, int dtype, uint64_t h0, int64_t H, const FitPlan& plan,
                     hipStream_t st);
casgd_status run_gather(const Dense& P, int dtype, uint64_t h, hipStream_t st);
casgd_status run_gram(const Dense& P, int dtype, float* Gout, uint64_t h, hipStream_t st);
casgd_status run_margin(const Dense& P, int dtype, uint64_t h, float* rp_out, hipStream_t st);
casgd_status run_margin_reduce(const Dense& P, const float* rp, uint64_t h, float* r_out,
                               hipStream_t st);
casgd_status run_recurrence(const Dense& P, const float* G, const float* rp, uint64_t h,
                            const float* r_in, const float* y_in, float* c, float* delta_out,
                            bool fp64, hipStream_t st);
casgd_status run_recurrence_multi(const Dense& P, const float* G, const float* r, const float* y,
                                  float* c, float* delta_out, bool fp64, unsigned long long spin,
                                  hipStream_t st);
casgd_status run_update(const Dense& P, int dtype, const float* c, uint64_t h, hipStream_t st);
casgd_status check_loss(int loss);
casgd_status check_dense(const casgd_matrix* X);
casgd_status check_bs(int32_t b, int32_t s);
casgd_status check_ws(const void* ws, size_t ws_bytes, size_t need);
casgd_status make_dense(const casgd_matrix* X, const float* y, float* x, double eta,
                        double lambda, int32_t b, int32_t s, uint64_t seed, const casgd_opts* o,
                        void* ws, size_t ws_bytes, Dense* P, DenseLayout* L, bool need_ws);
casgd_status run_zero(unsigned* p, int64_t words, hipStream_t st);
casgd_status run_fit_batch(const Dense* table_dev, const int2* wgmap_dev, int grid, int dtype,
                           size_t lds, unsigned long long spin, bool generic, hipStream_t st);
int batch_max_grid(int dtype, size_t lds, bool generic);
casgd_status launch_fit_f32(const Dense& P, const FitPlan& plan, hipStream_t st);
casgd_status launch_fit_bf16(const Dense& P, const FitPlan& plan, hipStream_t st);
casgd_status launch_fit_f16(const Dense& P, const FitPlan& plan, hipStream_t st);
casgd_status launch_fit_fp8(const Dense& P, const FitPlan& plan, hipStream_t st);
const void* batch_kernel_f32(bool generic);
const void* batch_kernel_bf16(bool generic);
const void* batch_kernel_f16(bool generic);
const void* batch_kernel_fp8(bool generic);
int fit_max_grid_f32(const Dense& P, int recur64);
int fit_max_grid_bf16(const Dense& P, int recur64);
int fit_max_grid_f16(const Dense& P, int recur64);
int fit_max_grid_fp8(const Dense& P, int recur64);
size_t fit_lds(const Dense& P, int dtype, int recur64);

int device_cus();

}  // namespace casgd
