// Learned-limiter training: launchers (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hy_mlp.h"

namespace hy {

constexpr int TRAIN_BLOCKS = 256;

hipError_t launch_coarsen4(const float *U, int64_t vs, int ndim, const int nf[3], float gm1, float *Wc, float *sub,
                           hipStream_t s);
hipError_t launch_samples(const float *Wc, const float *sub, int ndim, const int nc[3], float *x, float *t,
                          hipStream_t s);
hipError_t launch_train_grad(const MlpDevice *m, const float *x, const float *t, const int *idx, int64_t batch,
                             float *partial, float *loss_partial, int nblocks, float *grad, float *loss, hipStream_t s);
hipError_t launch_adam(MlpDevice *m, const float *grad, float *m1, float *m2, float lr, double b1, double b2,
                       float eps, int step, hipStream_t s);

}  // namespace hy
