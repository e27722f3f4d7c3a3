/*
 * vplbm_probes.h — measurement probes beside the VP-LBM library (libvplbm_probes.so).
 *
 * These calls do not advance any simulation.  They time kernels that reproduce how the step
 * kernels of libvplbm.so move memory, with the per-node update of Section 2 (Eqs. 8-18)
 * replaced by a trivial one, and two plain ceilings of the GPU.  They give the figures the step
 * kernels are measured against: the time their access pattern alone takes, the copy bandwidth,
 * and the rate at which the vector ALUs issue FP32 FMAs.
 *
 * Conventions: every call returns 0 or a negative code (-1 bad argument, -2 allocation failed,
 * -3 a HIP call failed) and then vplbm_probe_last_error() holds a message.  Each call allocates
 * and frees its own device memory on the current device, runs on a stream of its own, and
 * returns when its work is done.  Host pointers are written only on success.
 */
#ifndef VPLBM_PROBES_H
#define VPLBM_PROBES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The step's access pattern on an nx x ny lattice of binary32 populations (nine planes in, nine
   out, x fastest, rows padded to 64 elements, one mask byte per node; every edge periodic), with
   `steps_per_launch` updates per launch:
     1: one node per thread in 128 x 2 workgroups: nine shifted loads, the mask byte, nine
        non-temporal stores (the access pattern of the one-step kernel);
     2, 3: tile_w x tile_h tiles of 512 threads.  The first phase updates the tile and a halo of
        steps_per_launch - 1 nodes from global memory into an LDS tile; with 3, a middle phase
        updates the tile and a one-node halo in place in LDS; the last phase pulls from LDS and
        stores the tile with non-temporal stores (the two-step kernel's pattern and its
        three-step kernel's).  Tiles: 128 x 8, 64 x 8, 128 x 16 for 2; 64 x 14, 128 x 8, 128 x 6,
        64 x 8 for 3.  nx must be a multiple of tile_w and ny of tile_h.
   Each node's update halves its nine values and adds a multiple of its mask byte, so every byte
   loaded is used.  Workgroups map to tiles as in the step kernels (each XCD takes a contiguous
   range).  `launches` timed launches follow launches / 8 + 1 untimed ones; *us_per_launch is
   their mean duration (HIP events around the timed launches).  nx, ny >= 8, and the nine planes
   of a buffer hold fewer than 2^31 elements (rows padded to 64). */
int vplbm_probe_pattern(int32_t nx, int32_t ny, int32_t steps_per_launch, int32_t tile_w,
                        int32_t tile_h, int32_t launches, double *us_per_launch);

/* Copy of `bytes` bytes (a multiple of 16, at least 1 MiB) from one device buffer to another with
   16-byte loads and stores (four per thread), `reps` times after one untimed copy:
   *gbs = 2 * bytes / the mean copy time (bytes read plus bytes written, in 1e9 bytes per second). */
int vplbm_probe_copy(uint64_t bytes, int32_t reps, double *gbs);

/* Independent FP32 FMA chains (eight per lane, no packed FP32): 2048 workgroups of 256 threads
   run `reps` rounds of 1024 FMAs per chain.  *lane_fma_per_s = lane FMAs per second, the issue
   rate one VALU instruction per lane per cycle gives (each wave64 instruction counted once per
   lane). */
int vplbm_probe_fma(int32_t reps, double *lane_fma_per_s);

/* Message of the calling thread's last failed probe call. */
const char *vplbm_probe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VPLBM_PROBES_H */
