// kernels.h -- host-callable launchers of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "layout.h"

namespace su3hb {

// checkerboard slice update (one colour, one direction, all replicas);
// waves = minimum waves per SIMD the kernel was built for (2, or 3 for D = 4)
hipError_t launch_update(int D, int prec, int waves, dim3 grid, dim3 block, hipStream_t st,
                         const UpdateArgs &a);

// LDS one block of such a launch needs (static + dynamic) and the device's
// per-block limit; the caller refuses launches that would not fit
hipError_t update_lds(int D, int prec, int waves, dim3 block, const UpdateArgs &a, size_t *need, size_t *limit);

// persistent cooperative batch sweep: n_sweeps x 2D slices with a grid barrier
// persistent batch sweeps: kPersistentThreads per block, a.barrier zeroed beforehand
hipError_t launch_update_persistent(int D, int prec, int blocks, hipStream_t st, const UpdateArgs &a, int n_sweeps);
hipError_t persistent_max_blocks(int D, int prec, int *blocks_per_cu);

// plaquettes: per-block partial sums, then one block per replica finalises
hipError_t launch_plaquette(int D, int prec, dim3 grid, dim3 block, hipStream_t st, const PlaqArgs &a);
hipError_t launch_plaquette_finalize(hipStream_t st, const RepDesc *reps, int nrep, int D,
                                     const double *partials, double *out, double *series,
                                     uint32_t *series_cursor);

// fused measurement: sums the per-block plaquette class partials (nc = 1 for
// one layer, 3 for two) the parity-1 update slices wrote, normalises like the
// plaquette path
hipError_t launch_measure_finalize(hipStream_t st, const double *meas, int D, uint32_t nblocks, int nc, double V,
                                   int nlat, double beta0, double beta1, double *out, double *series,
                                   uint32_t *cursor);

// start configuration of one replica: mode 1 ordered, 2 Haar
hipError_t launch_start(int D, int prec, hipStream_t st, void *links, const RepDesc *reps, int r,
                        uint32_t nthreads, int mode);

// canonical FP64 [layer][site][mu][3][3] <-> internal storage, for the sites
// [c0, c0 + count) of the flat (layer * V + site) range of replica r
hipError_t launch_pack(int D, int prec, hipStream_t st, const void *links, const RepDesc *reps, int r,
                       uint64_t c0, uint32_t count, double *dst);
hipError_t launch_unpack(int D, int prec, hipStream_t st, void *links, const RepDesc *reps, int r,
                         uint64_t c0, uint32_t count, const double *src);
// max over matrices of max(|U U^dag - 1|, |det U - 1|) as the bits of a
// non-negative double (Inf for non-finite input), folded into *maxdef
hipError_t launch_validate(hipStream_t st, const double *src, uint64_t nmat, unsigned long long *maxdef);

// write one replica descriptor (by value) to device memory
hipError_t launch_rep_set(hipStream_t st, const RepDesc &r, RepDesc *dst);

// statistics slots and counters
hipError_t launch_stats_zero(hipStream_t st, StatSlot *slots);
hipError_t launch_stats_reduce(hipStream_t st, const StatSlot *slots, StatSlot *out);
hipError_t launch_counter_add(hipStream_t st, uint32_t *ctr, uint32_t add);
hipError_t launch_counter_set(hipStream_t st, uint32_t *ctr, uint32_t value);
hipError_t launch_u32_zero(hipStream_t st, uint32_t *p, int n);
hipError_t launch_u64_zero(hipStream_t st, unsigned long long *p, int n);

}  // namespace su3hb
