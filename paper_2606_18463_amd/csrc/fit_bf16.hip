// Fused persistent fit and batched launch for bf16 storage.
#include "fit.hpp"

namespace casgd {

casgd_status launch_fit_bf16(const Dense& P, const FitPlan& plan, hipStream_t st) {
    return plan.recur64 ? launch_fit_t<DT_BF16, double>(P, plan, st)
                        : launch_fit_t<DT_BF16, float>(P, plan, st);
}

int fit_max_grid_bf16(const Dense& P, int recur64) {
    return recur64 ? fit_max_grid<DT_BF16, double>(P) : fit_max_grid<DT_BF16, float>(P);
}

const void* batch_kernel_bf16(bool generic) { return batch_kernel_t<DT_BF16>(generic); }

}  // namespace casgd
