// Kernel argument records and host-side launchers of the VP-LBM library (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"

namespace vplbm {

constexpr int kMaxBodies = 8;
constexpr int kRingWidth = 1 + 2 * kMaxBodies;   // mass, (fx, fy) per body
constexpr int kBlock = 256;                      // threads per workgroup (4 wave64)
constexpr int kBlock2 = 512;                     // the two-step kernel's workgroup (8 wave64)
// Per-step reductions go through kSub sub-slots: workgroup b adds its partials into sub-slot
// b % kSub, so no address takes more than 1/kSub of the atomics (device-scope FP64 atomics to
// one address serialize).  The next launch's first workgroups (or the fold kernel at observation
// time) sum the sub-slots in a fixed order into the ring.  Steps use kAccSets sets of sub-slots
// round-robin, so that a launch of up to kMaxSteps steps can fold the kMaxSteps steps before it
// while it adds into its own and clears those of the next launch.
constexpr int kSub = 64;
constexpr int kMaxSteps = 3;                     // steps per launch, at most
constexpr int kAccSets = 16;                     // >= 3 kMaxSteps, a power of two
static_assert(kAccSets >= 3 * kMaxSteps && (kAccSets & (kAccSets - 1)) == 0, "reduction sets");

struct BodyParams {          // as given by the caller (vplbm_body), device copy
    int kind;                // 0 disk, 1 rect, 2 outside of a disk
    double cx, cy, r, hx, hy, ux, uy, omega, ax, ay, freq;
};

// Everything one launch of the step kernel needs.  Passed by value (kernel arguments).
struct StepArgs {
    const void *src;         // post-collision planes of the previous step
    void *dst;               // planes this step writes
    const uint8_t *mask;     // body id per node (pitch = geometry pitch)
    const BodyState *bodies; // body state at this step's time
    const uint8_t *mask2;    // two- and three-step launches: mask and body states of the second
    const BodyState *bodies2;//   step (the same arrays as mask / bodies unless bodies move)
    const uint8_t *mask3;    // three-step launches: those of the third step
    const BodyState *bodies3;
    double *ring;            // [ring_len][kRingWidth] per-step observables
    double *acc;             // [kAccSets][kSub][kRingWidth] per-step partial sums
    unsigned *status;        // bit 0: non-finite or non-positive density seen
    const long long *t_base; // step counter on the device
    Geom g;
    Outlet outlet;           // convective outlet state (prev = nullptr: none)
    int t_off;               // this launch's step = *t_base + t_off
    int ring_len;
    int reduce;              // 1: accumulate mass and body forces into the ring
    int ntx;                 // tiles along x
    int bx_log2, by;         // workgroup = (1 << bx_log2) x by threads
    int rows;                // each thread updates `rows` nodes, by rows apart
    int nt_store;            // 1: non-temporal population stores (buffers larger than the cache)
    NodeParams p;
};

struct TileShape {
    int bx_log2, by, rows, ntx, nty;   // a tile is (1 << bx_log2) x (by * rows) nodes
};
TileShape tile_shape(int nx, int ny, int elem_bytes);

hipError_t launch_step(int storage, const StepArgs &a, hipStream_t st);
// Steps *t_base + t_off and the one after in one launch, from a.src into a.dst; the second step
// takes its mask and body states from a.mask2 / a.bodies2 (the convective outlet included).
hipError_t launch_step2(int storage, const StepArgs &a, hipStream_t st);
// Steps *t_base + t_off .. + 2 in one launch (binary32 storage, the convective outlet included);
// the second and third steps take a.mask2 / a.bodies2 and a.mask3 / a.bodies3.
bool step3_supported(int storage);
hipError_t launch_step3(int storage, const StepArgs &a, hipStream_t st);

// Per-node density and penalized velocity of the current state into dense FP64 arrays.
hipError_t launch_readback(int storage, const StepArgs &a, double *rho, double *ux, double *uy,
                           hipStream_t st);

// f = f^eq(rho, u): from dense device fields (rho/ux/uy) if given, else (rho0, u0) with u_s in
// solid nodes.
hipError_t launch_init(int storage, const StepArgs &a, const double *rho, const double *ux,
                       const double *uy, double rho0, double ux0, double uy0, hipStream_t st);

// Dense FP64 [9][ny][nx] <-> the storage planes of a.dst (encode) / a.src (decode).
hipError_t launch_encode(int storage, const StepArgs &a, const double *pop, hipStream_t st);
hipError_t launch_decode(int storage, const StepArgs &a, double *pop, hipStream_t st);

// Body states at time *t_base + t_off.
hipError_t launch_bodies(const BodyParams *params, BodyState *state, int nbodies,
                         const long long *t_base, int t_off, hipStream_t st);

// Moving bodies before a launch of nsteps (1 to 3) steps, in one launch: for step s of the launch
// (time *t_base + t_off + s) the body states into state[s] and the swept boxes re-rasterized into
// mask[s].  box[k] = (x0, y0, w, h) of body k (w = 0: none, e.g. a static body); box_start holds
// the prefix sums of the box areas (box_start[kMaxBodies] = all of them).  Every box lies inside
// the lattice.
struct PlaceArgs {
    const BodyParams *params;
    int nbodies;
    int nsteps;
    uint8_t *mask[kMaxSteps];
    BodyState *state[kMaxSteps];
    const long long *t_base;
    int t_off;
    Geom g;
    int box[kMaxBodies][4];
    int box_start[kMaxBodies + 1];
};
hipError_t launch_place(const PlaceArgs &a, hipStream_t st);

// Rasterize the bodies into the mask over the rectangle [x0, x0+w) x [y0, y0+h).
hipError_t launch_mask(uint8_t *mask, const Geom &g, const BodyParams *params,
                       const BodyState *state, int nbodies, int x0, int y0, int w, int h,
                       hipStream_t st);

hipError_t launch_advance(long long *t_base, long long n, hipStream_t st);
// Convergence residual of the state a.src against the velocity snapshot snap ([2][ny*nx] FP64):
// out[0] = sum over fluid nodes of |u - u_snap|^2, out[1] = sum of |u|^2 (fixed summation
// order); the snapshot becomes u.  part holds residual_parts(g) x 2 doubles.
int residual_parts(const Geom &g);
hipError_t launch_residual(int storage, const StepArgs &a, double *snap, double *part, double *out,
                           hipStream_t st);
// Momentum exchange of the state a.src: out[2k], out[2k+1] += body k's (fx, fy) (out zeroed).
hipError_t launch_momentum_exchange(int storage, const StepArgs &a, double *out, hipStream_t st);
// Convective outlet: prev = the last column's populations 3, 6, 7 of the state a.src.
hipError_t launch_outlet_init(int storage, const StepArgs &a, void *prev, hipStream_t st);
// Sum the sub-slots of steps *t_base - 2 and *t_base - 1 into their ring entries.
hipError_t launch_fold(const StepArgs &a, hipStream_t st);
hipError_t launch_fill_f64(double *p, size_t n, double v, hipStream_t st);
hipError_t launch_fill_u32(unsigned *p, size_t n, unsigned v, hipStream_t st);

}  // namespace vplbm
