// The 1-64-64-1 CDF network of the learned bucket path: launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gs {

constexpr int kMlpParams = 4353;

hipError_t mlp_init(float *params, uint64_t seed, hipStream_t st);
// Training: two launches per step (batch/32 work-groups, then the ordered
// reduction and Adam); losses[0], losses[1] get the mean loss of the first and
// the last step.  `gate` (may be null): skip when *gate != 0.
hipError_t mlp_train(float *params, float *m, float *v, const float *su, const float *stgt, int64_t S,
                     int steps, int batch, float lr, uint64_t seed, int full_batch, float *partial,
                     float *losses, const unsigned *gate, hipStream_t st);
hipError_t mlp_loss_grad(const float *params, const float *u, const float *t, int batch, float *partial,
                         float *grad, float *loss, hipStream_t st);
// knots > 0: y[i] = net(i / knots) for i < count; else y[i] = net(u[i]).
hipError_t mlp_forward(const float *params, const float *u, int64_t count, float *y, int64_t knots,
                       const unsigned *gate, hipStream_t st);
int mlp_samples_per_group();

}  // namespace gs
