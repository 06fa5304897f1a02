// Fused persistent fit for f32 storage.
#include "fit.hpp"

namespace casgd {

casgd_status launch_fit_f32(const Dense& P, const FitPlan& plan, hipStream_t st) {
    return plan.recur64 ? launch_fit_t<DT_F32, double>(P, plan, st)
                        : launch_fit_t<DT_F32, float>(P, plan, st);
}

int fit_max_grid_f32(const Dense& P, int recur64) {
    return recur64 ? fit_max_grid<DT_F32, double>(P) : fit_max_grid<DT_F32, float>(P);
}

}  // namespace casgd
