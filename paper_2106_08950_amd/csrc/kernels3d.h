// kernels3d.h -- launch wrappers of the three-dimensional gfx950 kernels (internal to
// libdilbm).
#pragma once

#include <hip/hip_runtime.h>

#include "dilbm3d_internal.h"

namespace dilbm {

// Every kernel takes `step`, the solve's step count: the populations after step t are
// stored in the moving reference frame V_t.
// one step's collide over all tiles of the solve (parity p); tile_x is the tile width
// (64: tiles of 64 x 4 x 1 nodes, chunked persistent grid; 256: 256 x 1 x 1, one block
// per tile)
// q: the lattice, 19 (D3Q19) or 27 (D3Q27); h: FP16 population storage; open: the
// instance with open ends in x (desc->xbc)
hipError_t launch3_collide(int q, bool h, bool open, int tile_x, int grid, hipStream_t stream,
                           const Desc3 *desc, int p, int64_t step);
// blocks of the collide kernel resident on one CU at once (0 on error)
int collide3_blocks_per_cu(int q, bool h, bool open, int tile_x);
// a batch's collide: members' descriptors descs[], tile_solve[t] the member of
// concatenated tile t, k steps since the batch call began (tile_x and the instance shared)
hipError_t launch3_collide_batch(int q, bool h, bool open, int tile_x, int grid,
                                 hipStream_t stream, const Desc3 *descs,
                                 const int32_t *tile_solve, int64_t total_tiles, int k);
int collide3_batch_blocks_per_cu(int q, bool h, bool open, int tile_x);
// a batch's sphere step: body_solve[g] the member of concatenated sphere g
hipError_t launch3_bodies_batch(int total_bodies, int tile_x, hipStream_t stream,
                                const Desc3 *descs, const int32_t *body_solve, int k);
// rho and corrected u of parity p's state into [nz][ny][nx] device arrays (the boundary
// state on the planes of open ends)
hipError_t launch3_fields(int q, bool h, int tile_x, int64_t ntiles, hipStream_t stream,
                          const Desc3 *desc, int p, int64_t step, double *rho, double *ux,
                          double *uy, double *uz);
// the sphere step of parity p (or, bin_only, the binning of parity p's state) into the
// lists of tiles tile_x wide (64 or 256)
hipError_t launch3_bodies(bool bin_only, int nbodies, int tile_x, hipStream_t stream,
                          const Desc3 *desc, int p);
// populations in / out of parity p's buffer (count = q nx ny nz), device FP64 arrays
hipError_t launch3_set_pops(int q, bool h, int64_t count, hipStream_t stream,
                            const Desc3 *desc, int p, int64_t step, const double *fin);
hipError_t launch3_get_pops(int q, bool h, int64_t count, hipStream_t stream,
                            const Desc3 *desc, int p, int64_t step, double *fout);
// the fluid at rest in both buffers (count = q nx ny nz)
hipError_t launch3_rest_pops(int q, bool h, int64_t count, hipStream_t stream,
                             const Desc3 *desc, int64_t step);

}  // namespace dilbm
