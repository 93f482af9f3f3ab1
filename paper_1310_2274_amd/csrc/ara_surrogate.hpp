// ara_surrogate.hpp -- launchers of the surrogate kernels (ara_surrogate.hip).
#pragma once

#include "ara_internal.hpp"
#include "ara_mlp.hpp"

namespace ara {

hipError_t sur_launch_tuplegen(int64_t n, uint32_t seed, float* out, hipStream_t s);
hipError_t sur_launch_init(float* P, uint32_t seed, hipStream_t s);
hipError_t sur_launch_train_step(const float* tuples, int64_t n_tuples, int64_t pa, int64_t pc, int64_t row0,
                                 int32_t batch, float* P, float* m, float* v, float* gpart, float* lpart, float* grad,
                                 float* loss_acc, float lr, int64_t step, bool update, hipStream_t s);
hipError_t sur_launch_build_frag(const float* P, MlpFrag* F, hipStream_t s);
hipError_t sur_launch_calib(const float* tuples, int64_t n, const MlpFrag* F, const float* bias, unsigned int* cnt,
                            unsigned long long* sum, unsigned int* maxbits, hipStream_t s);
hipError_t sur_launch_eval(const double* a, const double* b, const double* u, int64_t n, const MlpFrag* F,
                           const uint32_t* mask, const float* bias, double* x, int32_t* used, hipStream_t s);

}  // namespace ara
