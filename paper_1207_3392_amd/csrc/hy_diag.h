// Diagnostic reductions (internal; defined in reduce.hip and spectrum.hip).
#pragma once

#include "hy_internal.h"

namespace hy {

// Kinetic energy per component: totals[5 + q] = dv * sum over cells of
// S_q^2 / (2 D), fixed-order FP64 trees (the chunks of the conserved totals).
template <typename T>
hipError_t launch_kinetic(const T *u, int64_t ncell, int64_t vstride, int ndim, double dv,
                          double *partials, int nblocks, DevCtl *ctl, hipStream_t s);

// Kinetic-energy spectrum of a 2D N x N patch (N a power of two, 2..8192)
// on a square box of side box: the shell sums e[0 .. spectrum_shells(n) - 1]
// are left in device memory inside the workspace (*e_dev points at them).
constexpr int SPEC_MAX_SHELLS = 5794;  // spectrum_shells(8192)
int spectrum_shells(int n);
size_t spectrum_workspace_bytes(int n);
template <typename T>
hipError_t launch_spectrum(const T *u, int64_t vstride, int n, double box, void *ws, double **e_dev, DevCtl *ctl,
                           hipStream_t s);

}  // namespace hy
