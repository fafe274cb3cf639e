// kernels.h -- launch wrappers of the gfx950 kernels (internal to libdilbm).
#pragma once

#include <hip/hip_runtime.h>

#include "dilbm_internal.h"

namespace dilbm {

// addr: 0 = one buffer resource per population buffer (buffer under 4 GB), 1 = 32-bit
// offsets from a plane base (plane under 2 GB), 2 = 64-bit addresses; open: some member has
// open ends in x (the instance with the inlet / outlet columns)
hipError_t launch_collide(int shape, int storage, int addr, bool open, int grid,
                          hipStream_t stream, const SolveDesc *descs, const int32_t *tile_solve,
                          const BatchHeader *hdr, int k);
// blocks of the collide instance resident on one CU at once (0 on error)
int collide_blocks_per_cu(int shape, int storage, int addr, bool open);
hipError_t launch_fields(int shape, int storage, int64_t ntiles, hipStream_t stream,
                         const SolveDesc *desc, int p, Region region, double *rho, double *ux,
                         double *uy);
hipError_t launch_bodies(bool bin_only, int grid, hipStream_t stream, const SolveDesc *descs,
                         const int32_t *body_solve, const BatchHeader *hdr, int k);
hipError_t launch_set_pops(int storage, int64_t count, hipStream_t stream, const SolveDesc *desc,
                           int p, const double *fin);
hipError_t launch_get_pops(int storage, int64_t count, hipStream_t stream, const SolveDesc *desc,
                           int p, double *fout);
// every population of both buffers at the rest state of step desc->step0 (count = 9 nx ny)
hipError_t launch_rest_pops(int storage, int64_t count, hipStream_t stream,
                            const SolveDesc *desc);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t stream);
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t stream);
hipError_t launch_zero_bytes(void *p, int64_t bytes, hipStream_t stream);

}  // namespace dilbm
