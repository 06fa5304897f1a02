// Fused persistent fit and batched launch for f32 storage.
#include "fit.hpp"

namespace casgd {

casgd_status launch_fit_f32(const Dense& P, const FitPlan& plan, hipStream_t st) {
    return plan.recur64 ? launch_fit_t<DT_F32, double>(P, plan, st)
                        : launch_fit_t<DT_F32, float>(P, plan, st);
}

int fit_max_grid_f32(const Dense& P, int recur64) {
    return recur64 ? fit_max_grid<DT_F32, double>(P) : fit_max_grid<DT_F32, float>(P);
}

const void* batch_kernel_f32(bool generic) { return batch_kernel_t<DT_F32>(generic); }

}  // namespace casgd
