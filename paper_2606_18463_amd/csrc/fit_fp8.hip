// Fused persistent fit and batched launch for fp8 storage.
#include "fit.hpp"

namespace casgd {

casgd_status launch_fit_fp8(const Dense& P, const FitPlan& plan, hipStream_t st) {
    return plan.recur64 ? launch_fit_t<DT_FP8, double>(P, plan, st)
                        : launch_fit_t<DT_FP8, float>(P, plan, st);
}

int fit_max_grid_fp8(const Dense& P, int recur64) {
    return recur64 ? fit_max_grid<DT_FP8, double>(P) : fit_max_grid<DT_FP8, float>(P);
}

const void* batch_kernel_fp8(bool generic) { return batch_kernel_t<DT_FP8>(generic); }

}  // namespace casgd
