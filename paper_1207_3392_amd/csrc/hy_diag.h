// Diagnostic reductions (internal; defined in reduce.hip).
#pragma once

#include "hy_internal.h"

namespace hy {

// Kinetic energy per component: totals[5 + q] = dv * sum over cells of
// S_q^2 / (2 D), fixed-order FP64 trees (the chunks of the conserved totals).
template <typename T>
hipError_t launch_kinetic(const T *u, int64_t ncell, int64_t vstride, int ndim, double dv,
                          double *partials, int nblocks, DevCtl *ctl, hipStream_t s);

}  // namespace hy
