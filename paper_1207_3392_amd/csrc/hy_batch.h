// Batched 1D tubes: device records and launchers (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hy {

constexpr int BATCH_NMAX = 6144;  // cells per tube (LDS-resident); up to 6, 12 or 24 per thread

struct TubeDesc {
    int n;
    int bclo, bchi;
    float idx;    // 1 / dx
    float gamma;
    float theta;
    int64_t off;  // first cell in the concatenated state arrays
};

struct TubeStatus {
    int steps;
    int err;      // bit 0: rho <= 0, p <= 0 or non-finite met; bit 1: stopped early (dt not > 0 or step cap)
    double t;
};

struct BatchCtl {
    unsigned next;  // queue head
    int solver;
    int max_steps;
    int pad;
    double t_end;
    double cfl;
};

hipError_t launch_batch_reset(BatchCtl *ctl, hipStream_t s);
// bt = threads per workgroup: 256, 512 or 1024 (4096 / bt cells per thread
// when the longest tube has at most 4096 cells, else BATCH_NMAX / bt)
bool batch_bt_supported(int bt);
hipError_t launch_batch(const TubeDesc *tubes, const int *order, float *U, int64_t ntot, BatchCtl *ctl,
                        TubeStatus *status, int ntubes, int nmax, int nblocks, int bt, hipStream_t s);
size_t batch_lds_bytes(int nmax);
hipError_t prepare_batch(int nmax);
int batch_blocks_per_cu(int nmax, int bt);

}  // namespace hy
