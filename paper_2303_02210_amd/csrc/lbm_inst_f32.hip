// lbm_inst_f32.hip -- the step, init, mass, finalize and batch kernels
// instantiated for float storage (one translation unit per storage type so
// that they compile in parallel).
#include "lbm_step.hpp"

namespace lbm {

#define LBM_INSTANTIATE(S)                                                              \
    template hipError_t launch_step<S>(const StepArgs<S> &, dim3, int, int, hipStream_t);    \
    template hipError_t launch_step_vec<S>(const StepArgs<S> &, dim3, int, int, hipStream_t);    \
    template hipError_t launch_step_staged<S>(const StepArgs<S> &, dim3, hipStream_t);          \
    template hipError_t launch_step7<S>(const StepArgs<S> &, dim3, int, int, int, hipStream_t); \
    template hipError_t launch_init<S>(const InitArgs<S> &, dim3, int, hipStream_t);    \
    template hipError_t launch_mass<S>(const MassArgs<S> &, dim3, int, hipStream_t);    \
    template hipError_t launch_finalize<S>(const FinalizeArgs<S> &, hipStream_t);           \
    template hipError_t launch_step_batch<S>(BatchRep<S> *const *, const TileRef *,           \
                                             const int32_t *, int, int, int, int, int, int, int, \
                                             int, GridBar *, hipStream_t);                  \
    template int batch_coop_grid<S>(int, int, int, int, int, int);                           \
    template hipError_t launch_plan_batch<S>(const PlanJob *, int, hipStream_t);             \
    template hipError_t launch_finalize_batch<S>(BatchRep<S> *const *, int, int, hipStream_t); \
    template hipError_t launch_batch_advance<S>(BatchRep<S> *const *, int, int, hipStream_t);

LBM_INSTANTIATE(float)

}  // namespace lbm
