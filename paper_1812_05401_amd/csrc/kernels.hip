// HIP kernels of the VP-LBM library for gfx950 (MI355X).
//
// The step is one fused pass: per node 9 pulled population loads, a 1-byte mask load, the
// moments / penalization / collision in registers, 9 coalesced stores, and the FP64 per-step
// reductions (wave64 shuffles, one LDS hop, FP64 atomics into sub-slots that a later launch folds
// into a device ring).  One step per launch it is bound by HBM bandwidth; the two-step kernel
// keeps the first of two steps in LDS and moves the planes once per two steps.  Nothing here is a
// dense contraction, so there is no MFMA.
#include <stdlib.h>

#include "kernels.hpp"

namespace vplbm {

// ---- the fused step --------------------------------------------------------------------------

// Sub-slots [kSub][kRingWidth] of step t: one of kAccSets sets, used round-robin by step.
__device__ __forceinline__ double *acc_set(const StepArgs &a, long long t)
{
    return a.acc + (size_t)(t & (kAccSets - 1)) * kSub * kRingWidth;
}

// Sum value q of the sub-slots of steps t - kMaxSteps .. t - 1 (those that exist) into their ring
// entries, with one wave: lane l adds sub-slots l, l + 64, ... in order, then a fixed butterfly
// adds the lanes, so a result does not depend on which workgroup folds or when.  One memory round
// trip for all of them.  Nothing is cleared, so folding a step again gives the same value: a step
// is folded by the next launch, and again by later ones while it is among their last kMaxSteps.
// The fold always takes the shuffle form of the wave sum, so that every fold of a step (by any
// kernel class, or by an observation) writes the same value.
__device__ __forceinline__ void fold_recent(const StepArgs &a, long long t, int q)
{
    const int lane = threadIdx.x & 63;
    double v[kMaxSteps];
#pragma unroll
    for (int d = 0; d < kMaxSteps; d++) v[d] = 0.0;
    for (int b = lane; b < kSub; b += 64) {
#pragma unroll
        for (int d = 0; d < kMaxSteps; d++) v[d] += acc_set(a, t - 1 - d)[b * kRingWidth + q];
    }
#pragma unroll
    for (int d = 0; d < kMaxSteps; d++) {
        const double sum = wave_sum<false>(v[d]);
        if (lane == 0 && t >= 1 + d) a.ring[(size_t)((t - 1 - d) % a.ring_len) * kRingWidth + q] = sum;
    }
}

// Start of a launch that computes steps t .. t + n - 1 (1 <= n <= kMaxSteps): workgroup q's first
// wave folds value q of steps t - kMaxSteps .. t - 1, and workgroup b zeroes sub-slot b of the
// sets of steps t + n .. t + n + kMaxSteps - 1, which the next launch accumulates into.  The sets
// one launch folds, writes and clears span at most 3 kMaxSteps consecutive steps, so with
// kAccSets >= 3 kMaxSteps they are distinct.  Step s is first folded by a launch starting at most
// kMaxSteps steps after s; the launch that clears its set for step s + kAccSets starts at least
// kAccSets - 2 kMaxSteps + 1 steps after s, later in stream order, so every fold of s sees its
// complete sums.
__device__ __forceinline__ void reduction_prologue(const StepArgs &a, long long t, int n)
{
    if (threadIdx.x < 64)
        for (int q = blockIdx.x; q < kRingWidth; q += gridDim.x) fold_recent(a, t, q);
    if (threadIdx.x < kMaxSteps * kRingWidth) {
        double *set = acc_set(a, t + n + threadIdx.x / kRingWidth);
        const int q = threadIdx.x % kRingWidth;
        for (int b = blockIdx.x; b < kSub; b += gridDim.x) set[b * kRingWidth + q] = 0.0;
    }
}

// A workgroup's partial sums of step t (rows of per-wave partials, added in a fixed order) into
// its sub-slot of the step's set: threads 0 .. kRingWidth - 1, after the barrier that completes
// the rows.
__device__ __forceinline__ void add_partials(const StepArgs &a, long long t, const double *rows, int nrows)
{
    if (threadIdx.x < kRingWidth) {
        double v = 0.0;
        for (int w = 0; w < nrows; w++) v += rows[w * kRingWidth + threadIdx.x];   // fixed order
        double *slot = acc_set(a, t) + (blockIdx.x & (kSub - 1)) * kRingWidth;
        if (v != 0.0) unsafeAtomicAdd(slot + threadIdx.x, v);
    }
}

template <int S, bool NT>
__global__ __launch_bounds__(kBlock) void step_kernel(StepArgs a)
{
    using C = Codec<S>;
    using T = typename C::real;
    constexpr bool DPP = wave_sum_dpp<T>();
    using E = typename C::elem;
    // Per-wave partial sums: each wave writes only its own row (LDS accesses of one wave are in
    // order), so the workgroup needs a single barrier, before the rows are added.
    __shared__ double wave_acc[kBlock / 64][kRingWidth];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long t = *a.t_base + a.t_off;
    if (a.reduce) {
        if (lane < kRingWidth) wave_acc[wave][lane] = 0.0;
        reduction_prologue(a, t, 1);   // earlier steps' partials are complete (kernel boundary)
    }
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int x = ((tile % a.ntx) << a.bx_log2) + (threadIdx.x & ((1 << a.bx_log2) - 1));
    const int y0 = (tile / a.ntx) * a.by * a.rows + (threadIdx.x >> a.bx_log2);
    const E *__restrict__ src = static_cast<const E *>(a.src);
    E *__restrict__ dst = static_cast<E *>(a.dst);
    bool bad = false;
    double mass = 0.0;                          // this thread's nodes, FP64
    for (int r = 0; r < a.rows; r++) {
        const int y = y0 + r * a.by;
        const bool active = (x < a.g.nx) & (y < a.g.ny);
        double fx_d = 0.0, fy_d = 0.0;
        int id = 0;
        if (active) {
            const Macro<T> m = update_node<S, NT, mask_first_one_step<S, NT>()>(
                src, dst, a.mask, a.bodies, a.g, a.outlet, a.p, x, y, id, (unsigned)t);
            const double rho_d = 1.0 + double(m.drho);
            mass += rho_d;
            fx_d = double(m.fx);
            fy_d = double(m.fy);
            bad |= !(rho_d > 0.0 && rho_d < 1e30);   // also catches NaN
        }
        if (a.reduce) wave_forces<DPP>(wave_acc[wave], fx_d, fy_d, id);
    }
    if (a.reduce) {
        const double mw = wave_sum<DPP>(mass);
        if (lane == 0) wave_acc[wave][0] = mw;
        if (__ballot(bad) && lane == 0) atomicOr(a.status, 1u);
        __syncthreads();
        add_partials(a, t, &wave_acc[0][0], kBlock / 64);
    }
}

// ---- two steps per launch ----------------------------------------------------------------------
// Steps t and t + 1 of a TW x TH tile in one launch.  Phase 1 computes step t on the tile and its
// one-node halo, from the planes in global memory, and keeps the result in LDS in the storage
// format, rounded exactly as a store to global memory would round it; phase 2 computes step t + 1
// of the tile from LDS and stores it.  Each node's arithmetic is the one-step kernel's, so the
// populations are bitwise those of two one-step launches, with one read and one write of the
// planes instead of two of each.  The halo is computed twice (by this tile and its neighbour):
// (TW + 2)(TH + 2) / (TW TH) of the nodes in phase 1.  Phase 1 takes the mask and body states of
// step t, phase 2 those of step t + 1 (where bodies move, the host rebuilds two masks).  The
// convective outlet's step-t values stay in LDS: phase 1 reads the previous ones from global
// memory and keeps what it records for its own rows, phase 2 applies the outlet rule with them and
// records step t + 1 for the next launch.
// Tiles (measured): 128 x 8 for FP32 (47 KB of LDS, three workgroups per CU); 64 x 8 for the
// FP64-arithmetic formats (F64: 48 KB; F32D: 24 KB, 25-36% faster than 128 x 8 under its 94
// VGPRs); for 2-byte storage 128 x 16 on large lattices (42 KB: less halo, 10-13% faster at
// 8192 x 2048) and 128 x 8 on smaller ones, whose taller tiles would not fill the chip.
// CONV: the lattice has a convective outlet (a separate instantiation: the outlet code in the
// loops costs the 16-bit kernels about 20% even where it is skipped).
template <int S, int TW, int TH, bool NT, bool CONV>
__global__ __launch_bounds__(kBlock2) void step2_kernel(StepArgs a)
{
    using C = Codec<S>;
    using T = typename C::real;
    using E = typename C::elem;
    constexpr int EW = TW + 2, EN = EW * (TH + 2);
    constexpr int NW = kBlock2 / 64;
    constexpr bool MF = mask_first_two_step<S, NT>();   // mask byte loaded before the populations
    constexpr bool DPP = wave_sum_dpp<T>();
    static_assert((TW * TH) % kBlock2 == 0, "phase 2 gives every thread the same number of nodes");
    __shared__ E mid[9 * EN];                      // step t on the tile and its halo
    __shared__ double wave_acc[2][NW][kRingWidth]; // per-wave partials of steps t and t + 1
    __shared__ T outl[3][TH];                      // convective outlet: step t's recorded values
    constexpr int odirs[3] = {3, 6, 7};            // the directions entering from x = nx
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long t = *a.t_base + a.t_off;
    const Geom &g = a.g;
    if (a.reduce) {
        if (lane < kRingWidth) {
            wave_acc[0][wave][lane] = 0.0;
            wave_acc[1][wave][lane] = 0.0;
        }
        reduction_prologue(a, t, 2);
    }
    const int ntx = (g.nx + TW - 1) / TW;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int x0 = (tile % ntx) * TW, y0 = (tile / ntx) * TH;
    const E *__restrict__ src = static_cast<const E *>(a.src);
    E *__restrict__ dst = static_cast<E *>(a.dst);
    // Phase 1 reads the outlet and records nothing.  (Without a convective outlet prev is null at
    // run time; making it null at compile time changes the schedule and costs 5-8%, measured.)
    const Outlet out1{a.outlet.prev, nullptr, a.outlet.u};
    bool bad = false;
    double mass = 0.0;

    // A tile two or more nodes from every edge: every node of phase 1 (the halo included) pulls
    // by plain shifts and needs no wrap, and so does every node of phase 2 (same loads, same
    // values, fewer instructions).
    const bool inner = (x0 >= 2) & (x0 + TW + 2 <= g.nx) & (y0 >= 2) & (y0 + TH + 2 <= g.ny);

    // Phase 1.  Halo nodes across a periodic edge are the wrapped nodes; halo positions outside
    // a non-periodic edge (and beyond a ragged tile) are skipped: no phase-2 pull reads them.
    for (int it = 0; it < (EN + kBlock2 - 1) / kBlock2; it++) {
        const int e = threadIdx.x + it * kBlock2;
        const int lx = e % EW - 1, ly = e / EW - 1;
        const int ux = x0 + lx, uy = y0 + ly;     // unwrapped
        int x = ux, y = uy;
        bool live = e < EN, own;
        if (inner) {
            own = live & (lx >= 0) & (lx < TW) & (ly >= 0) & (ly < TH);
        } else {
            if (x < 0 || x >= g.nx) {
                if (g.xper && x >= -1 && x <= g.nx) x += x < 0 ? g.nx : -g.nx;
                else live = false;
            }
            if (y < 0 || y >= g.ny) {
                if (g.yper && y >= -1 && y <= g.ny) y += y < 0 ? g.ny : -g.ny;
                else live = false;
            }
            own = live & (lx >= 0) & (lx < TW) & (ly >= 0) & (ly < TH) & (ux < g.nx) & (uy < g.ny);
        }
        double fx_d = 0.0, fy_d = 0.0;
        int id = 0;
        if (live) {
            if constexpr (MF) id = *at(a.mask, unsigned(y * g.pitch + x));
            T f[9];
            if (inner) pull_interior<S>(src, x, y, g, f);
            else pull<S>(src, x, y, g, out1, f);
            if (CONV && x == g.nx - 1 && own)
                for (int k = 0; k < 3; k++) outl[k][ly] = f[odirs[k]];
            const Macro<T> m = MF ? relax_node_id(f, id, a.bodies, g, a.p, x, y)
                                  : relax_node(f, a.mask, a.bodies, g, a.p, x, y, id);
            store_node<S>(mid, EN, unsigned(e), f, unsigned(y * g.pitch + x), (unsigned)t);
            if (own) {
                const double rho_d = 1.0 + double(m.drho);
                mass += rho_d;
                fx_d = double(m.fx);
                fy_d = double(m.fy);
                bad |= !(rho_d > 0.0 && rho_d < 1e30);
            } else {
                id = 0;                           // another tile's node: not in this tile's sums
            }
        }
        if (a.reduce) wave_forces<DPP>(wave_acc[0][wave], fx_d, fy_d, id);
    }
    if (a.reduce) {
        const double mw = wave_sum<DPP>(mass);
        if (lane == 0) wave_acc[0][wave][0] = mw;
    }
    mass = 0.0;
    __syncthreads();                              // the tile of step t is complete
    if (a.reduce) add_partials(a, t, &wave_acc[0][0][0], NW);

    // Phase 2.
    for (int it = 0; it < TW * TH / kBlock2; it++) {
        const int j = threadIdx.x + it * kBlock2;
        const int x = x0 + j % TW, y = y0 + j / TW;
        double fx_d = 0.0, fy_d = 0.0;
        int id = 0;
        if ((x < g.nx) & (y < g.ny)) {
            if constexpr (MF) id = *at(a.mask2, unsigned(y * g.pitch + x));
            T f[9];
            if (inner) pull_tile_shifts<S>(mid, EN, EW, x, y, x0, y0, f);
            else pull_tile<S>(mid, EN, EW, x, y, x0, y0, g, f);
            if (CONV && x == g.nx - 1) {
                // the outlet rule of pull, with step t's values from LDS
                const T u = T(a.outlet.u);
                T *next = static_cast<T *>(a.outlet.next);
                for (int k = 0; k < 3; k++) {
                    int pa;
                    const unsigned jn = tile_source(odirs[k], g.nx - 2, y, x0, y0, EW, g, pa);
                    const T nb = C::load(mid + pa * EN, jn, weight<T>(odirs[k]));
                    f[odirs[k]] = (outl[k][y - y0] + u * nb) / (T(1) + u);
                }
                for (int k = 0; k < 3; k++) next[k * g.ny + y] = f[odirs[k]];
            }
            const Macro<T> m = MF ? relax_node_id(f, id, a.bodies2, g, a.p, x, y)
                                  : relax_node(f, a.mask2, a.bodies2, g, a.p, x, y, id);
            const unsigned i = y * g.pitch + x;
            store_node<S, NT>(dst, g.plane, i, f, i, (unsigned)(t + 1));
            const double rho_d = 1.0 + double(m.drho);
            mass += rho_d;
            fx_d = double(m.fx);
            fy_d = double(m.fy);
            bad |= !(rho_d > 0.0 && rho_d < 1e30);
        }
        if (a.reduce) wave_forces<DPP>(wave_acc[1][wave], fx_d, fy_d, id);
    }
    if (a.reduce) {
        const double mw = wave_sum<DPP>(mass);
        if (lane == 0) wave_acc[1][wave][0] = mw;
        if (__ballot(bad) && lane == 0) atomicOr(a.status, 1u);
        __syncthreads();
        add_partials(a, t + 1, &wave_acc[1][0][0], NW);
    }
}

// ---- three steps per launch --------------------------------------------------------------------
// Steps t, t + 1 and t + 2 of a TW x TH tile in one launch.  Phase 1 computes step t on the tile
// and a two-node halo from the planes in global memory into LDS; phase 2 computes step t + 1 on
// the tile and a one-node halo from LDS, keeps its results in registers until every thread has
// made its pulls, then writes them over the same slots; phase 3 computes step t + 2 of the tile
// from LDS and stores it.  Each node's arithmetic is the one-step kernel's and every value kept in
// LDS is rounded as a store to global memory would round it, so the populations are bitwise those
// of three one-step launches, with one read and one write of the planes per three updates.  A halo
// position across a periodic edge holds the wrapped node; one beyond a non-periodic edge or a
// ragged tile is skipped (no later pull reads it).  The phases take the masks and body states of
// their own steps (a.mask, a.mask2, a.mask3).  CONV (an instantiation of its own): the lattice
// has a convective outlet; phase 1 reads the previous launch's records from global memory and
// keeps the values it records at x = nx - 1 for the tile's rows and a one-row halo in LDS, phase 2
// applies the outlet rule with them and keeps its own for the tile's rows, and phase 3 applies it
// with those and records its values in global memory for the next launch.  Only tiles that reach
// the last column take this code.  Tiles: 64 x 14 for binary32 (46 KB of LDS, three workgroups per
// CU; the phases cover 1224, 1056 and 896 nodes, 1.18 computed per update).  Measured at
// 8192 x 2048: 111 us per step, against 113 for 64 x 12, 116 for 64 x 16, 118 for 32 x 24, 123 for
// 128 x 6 and 64 x 10, 127 for 128 x 10, 137 for 128 x 8 (two workgroups per CU) and 151 for
// 256 x 4: the VALUs bound this kernel, and taller tiles recompute less halo.  Inner tiles load and
// the last phase stores through buffer resources (pull_interior_buf, store_node_buf), which keep
// the plane offsets out of the vector ALUs.
template <int S, int TW, int TH, bool NT, bool CONV>
__global__ __launch_bounds__(kBlock2) void step3_kernel(StepArgs a)
{
    using C = Codec<S>;
    using T = typename C::real;
    using E = typename C::elem;
    constexpr int EW = TW + 4, EN = EW * (TH + 4);       // phase 1: the tile and two halo rings
    constexpr int MW = TW + 2, MN = MW * (TH + 2);       // phase 2: the tile and one halo ring
    constexpr int NW = kBlock2 / 64;
    constexpr int R1 = (EN + kBlock2 - 1) / kBlock2;
    constexpr int R2 = (MN + kBlock2 - 1) / kBlock2;
    constexpr int R3 = (TW * TH + kBlock2 - 1) / kBlock2;
    constexpr bool MF = false;   // mask byte after the populations (mask first: 87 VGPRs without NT)
    constexpr bool DPP = wave_sum_dpp<T>();
    __shared__ E mid[9 * EN];                           // steps t, then t + 1, on the tile
    __shared__ double wave_acc[3][NW][kRingWidth];      // per-wave partials of the three steps
    // convective outlet: the values steps t and t + 1 record at x = nx - 1, rows y0 - 1 ..
    // y0 + TH (unwrapped) and y0 .. y0 + TH - 1
    __shared__ T outl1[CONV ? 3 : 1][TH + 2];
    __shared__ T outl2[CONV ? 3 : 1][TH];
    constexpr int odirs[3] = {3, 6, 7};                 // the directions entering from x = nx
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long t = *a.t_base + a.t_off;
    const Geom &g = a.g;
    if (a.reduce) {
        if (lane < kRingWidth)
            for (int k = 0; k < 3; k++) wave_acc[k][wave][lane] = 0.0;
        reduction_prologue(a, t, 3);
    }
    const int ntx = (g.nx + TW - 1) / TW;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int x0 = (tile % ntx) * TW, y0 = (tile / ntx) * TH;
    const E *__restrict__ src = static_cast<const E *>(a.src);
    // the source and destination planes as buffers (the host keeps three-step lattices below 4 GB)
    const unsigned bytes = 9u * unsigned(g.plane) * unsigned(sizeof(E));
    const __amdgpu_buffer_rsrc_t rsrc = buffer_over(const_cast<void *>(a.src), bytes);
    const __amdgpu_buffer_rsrc_t rdst = buffer_over(a.dst, bytes);
    const Outlet none{nullptr, nullptr, 0.0};
    const Outlet out1{a.outlet.prev, nullptr, a.outlet.u};   // step t reads the outlet, records here
    bool bad = false;
    double mass = 0.0;
    // A tile three or more nodes from every edge: every node of every phase pulls by plain shifts
    // and needs no wrap.
    const bool inner = (x0 >= 3) & (x0 + TW + 3 <= g.nx) & (y0 >= 3) & (y0 + TH + 3 <= g.ny);
    // The lattice node at unwrapped position (ux, uy), h or fewer nodes outside the tile: live
    // unless beyond a non-periodic edge or more than h beyond the lattice (a ragged tile).
    auto locate = [&](int ux, int uy, int h, int &x, int &y) -> bool {
        x = ux;
        y = uy;
        bool live = true;
        if (x < 0 || x >= g.nx) {
            if (g.xper && x >= -h && x < g.nx + h) x += x < 0 ? g.nx : -g.nx;
            else live = false;
        }
        if (y < 0 || y >= g.ny) {
            if (g.yper && y >= -h && y < g.ny + h) y += y < 0 ? g.ny : -g.ny;
            else live = false;
        }
        return live;
    };
    auto in_tile = [&](int ux, int uy) -> bool {
        return (ux >= x0) & (ux < x0 + TW) & (uy >= y0) & (uy < y0 + TH) & (ux < g.nx) & (uy < g.ny);
    };

    // Phase 1: step t.
    for (int it = 0; it < R1; it++) {
        const int e = threadIdx.x + it * kBlock2;
        const int ux = x0 + e % EW - 2, uy = y0 + e / EW - 2;
        int x = ux, y = uy;
        const bool live = (e < EN) && (inner || locate(ux, uy, 2, x, y));
        double fx_d = 0.0, fy_d = 0.0;
        int id = 0;
        if (live) {
            if constexpr (MF) id = *at(a.mask, unsigned(y * g.pitch + x));
            T f[9];
            if (inner) pull_interior_buf<S>(rsrc, g.plane, g.pitch, unsigned(y * g.pitch + x), f);
            else pull<S>(src, x, y, g, CONV ? out1 : none, f);
            if (CONV && !inner && x == g.nx - 1 && uy >= y0 - 1 && uy <= y0 + TH)
                for (int q = 0; q < 3; q++) outl1[q][uy - y0 + 1] = f[odirs[q]];
            const Macro<T> m = MF ? relax_node_id(f, id, a.bodies, g, a.p, x, y)
                                  : relax_node(f, a.mask, a.bodies, g, a.p, x, y, id);
            store_node<S>(mid, EN, unsigned(e), f, unsigned(y * g.pitch + x), (unsigned)t);
            if (in_tile(ux, uy)) {
                const double rho_d = 1.0 + double(m.drho);
                mass += rho_d;
                fx_d = double(m.fx);
                fy_d = double(m.fy);
                bad |= !(rho_d > 0.0 && rho_d < 1e30);
            } else {
                id = 0;                           // another tile's node: not in this tile's sums
            }
        }
        if (a.reduce) wave_forces<DPP>(wave_acc[0][wave], fx_d, fy_d, id);
    }
    if (a.reduce) {
        const double mw = wave_sum<DPP>(mass);
        if (lane == 0) wave_acc[0][wave][0] = mw;
    }
    mass = 0.0;
    __syncthreads();                              // the tile of step t is complete
    if (a.reduce) add_partials(a, t, &wave_acc[0][0][0], NW);

    // Phase 2: step t + 1, from LDS into registers, then over the same slots.
    T res[R2][9];
    int slot[R2];                                 // -1: no node
    unsigned node[R2];
#pragma unroll
    for (int it = 0; it < R2; it++) {
        const int j = threadIdx.x + it * kBlock2;
        const int ux = x0 + j % MW - 1, uy = y0 + j / MW - 1;
        int x = ux, y = uy;
        const bool live = (j < MN) && (inner || locate(ux, uy, 1, x, y));
        slot[it] = live ? (j / MW + 1) * EW + j % MW + 1 : -1;
        node[it] = unsigned(y * g.pitch + x);
        double fx_d = 0.0, fy_d = 0.0;
        int id = 0;
        if (live) {
            if constexpr (MF) id = *at(a.mask2, node[it]);
            if (inner) pull_tile_shifts<S, 2>(mid, EN, EW, ux, uy, x0, y0, res[it]);
            else pull_tile<S, 2>(mid, EN, EW, ux, uy, x0, y0, g, res[it]);
            if (CONV && !inner && x == g.nx - 1) {
                // the outlet rule of pull, with step t's records and neighbours from LDS
                const T u = T(a.outlet.u);
                for (int q = 0; q < 3; q++) {
                    int pa;
                    const unsigned jn = tile_source<2>(odirs[q], g.nx - 2, uy, x0, y0, EW, g, pa);
                    const T nb = C::load(mid + pa * EN, jn, weight<T>(odirs[q]));
                    res[it][odirs[q]] = (outl1[q][uy - y0 + 1] + u * nb) / (T(1) + u);
                }
                if (uy >= y0 && uy < y0 + TH)
                    for (int q = 0; q < 3; q++) outl2[q][uy - y0] = res[it][odirs[q]];
            }
            const Macro<T> m = MF ? relax_node_id(res[it], id, a.bodies2, g, a.p, x, y)
                                  : relax_node(res[it], a.mask2, a.bodies2, g, a.p, x, y, id);
            if (in_tile(ux, uy)) {
                const double rho_d = 1.0 + double(m.drho);
                mass += rho_d;
                fx_d = double(m.fx);
                fy_d = double(m.fy);
                bad |= !(rho_d > 0.0 && rho_d < 1e30);
            } else {
                id = 0;
            }
        }
        if (a.reduce) wave_forces<DPP>(wave_acc[1][wave], fx_d, fy_d, id);
    }
    if (a.reduce) {
        const double mw = wave_sum<DPP>(mass);
        if (lane == 0) wave_acc[1][wave][0] = mw;
    }
    mass = 0.0;
    __syncthreads();                              // every phase-2 pull has read step t
    if (a.reduce) add_partials(a, t + 1, &wave_acc[1][0][0], NW);
#pragma unroll
    for (int it = 0; it < R2; it++)
        if (slot[it] >= 0) store_node<S>(mid, EN, unsigned(slot[it]), res[it], node[it], (unsigned)(t + 1));
    __syncthreads();                              // the tile of step t + 1 is complete

    // Phase 3: step t + 2 of the tile, to global memory.
#pragma unroll
    for (int it = 0; it < R3; it++) {
        const int j = threadIdx.x + it * kBlock2;
        const int x = x0 + j % TW, y = y0 + j / TW;
        double fx_d = 0.0, fy_d = 0.0;
        int id = 0;
        if ((j < TW * TH) & (x < g.nx) & (y < g.ny)) {
            if constexpr (MF) id = *at(a.mask3, unsigned(y * g.pitch + x));
            T f[9];
            if (inner) pull_tile_shifts<S, 2>(mid, EN, EW, x, y, x0, y0, f);
            else pull_tile<S, 2>(mid, EN, EW, x, y, x0, y0, g, f);
            if (CONV && !inner && x == g.nx - 1) {
                // the outlet rule with step t + 1's records; this step's go to global memory
                const T u = T(a.outlet.u);
                T *next = static_cast<T *>(a.outlet.next);
                for (int q = 0; q < 3; q++) {
                    int pa;
                    const unsigned jn = tile_source<2>(odirs[q], g.nx - 2, y, x0, y0, EW, g, pa);
                    const T nb = C::load(mid + pa * EN, jn, weight<T>(odirs[q]));
                    f[odirs[q]] = (outl2[q][y - y0] + u * nb) / (T(1) + u);
                }
                for (int q = 0; q < 3; q++) next[q * g.ny + y] = f[odirs[q]];
            }
            const Macro<T> m = MF ? relax_node_id(f, id, a.bodies3, g, a.p, x, y)
                                  : relax_node(f, a.mask3, a.bodies3, g, a.p, x, y, id);
            store_node_buf<S, NT>(rdst, g.plane, y * g.pitch + x, f);
            const double rho_d = 1.0 + double(m.drho);
            mass += rho_d;
            fx_d = double(m.fx);
            fy_d = double(m.fy);
            bad |= !(rho_d > 0.0 && rho_d < 1e30);
        }
        if (a.reduce) wave_forces<DPP>(wave_acc[2][wave], fx_d, fy_d, id);
    }
    if (a.reduce) {
        const double mw = wave_sum<DPP>(mass);
        if (lane == 0) wave_acc[2][wave][0] = mw;
        if (__ballot(bad) && lane == 0) atomicOr(a.status, 1u);
        __syncthreads();
        add_partials(a, t + 2, &wave_acc[2][0][0], NW);
    }
}

__global__ void fold_kernel(StepArgs a)
{
    const long long t = *a.t_base;
    for (int q = 0; q < kRingWidth; q++) fold_recent(a, t, q);
}

hipError_t launch_fold(const StepArgs &a, hipStream_t st)
{
    fold_kernel<<<1, 64, 0, st>>>(a);
    return hipGetLastError();
}

TileShape tile_shape(int nx, int ny, int elem_bytes)
{
    TileShape t;
    int bx_log2 = 7;                            // 128 x 2 by default (measured best)
    while (bx_log2 > 6 && (1 << (bx_log2 - 1)) >= nx) bx_log2--;
    if (const char *e = getenv("VPLBM_TILE_BX_LOG2")) {   // tuning override: 6, 7 or 8
        int v = atoi(e);
        if (v >= 6 && v <= 8) bx_log2 = v;
    }
    t.bx_log2 = bx_log2;
    t.by = kBlock >> bx_log2;
    t.ntx = (nx + (1 << bx_log2) - 1) >> bx_log2;
    // Enough workgroups to fill the chip a few times over (256 CUs x 8 resident x 4), then
    // several rows per thread, which cuts the per-workgroup reduction work.
    const long long one_row_tiles = (long long)t.ntx * ((ny + t.by - 1) / t.by);
    int rows = (int)(one_row_tiles / 8192);
    rows = rows < 1 ? 1 : (rows > 8 ? 8 : rows);
    if (elem_bytes >= 4) rows = 1;              // measured: one row is best for FP32/FP64
    if (const char *e = getenv("VPLBM_ROWS")) {   // tuning override: 1..16
        int v = atoi(e);
        if (v >= 1 && v <= 16) rows = v;
    }
    t.rows = rows;
    t.nty = (ny + t.by * rows - 1) / (t.by * rows);
    return t;
}

hipError_t launch_step(int storage, const StepArgs &a, hipStream_t st)
{
    const dim3 grid(a.ntx * ((a.g.ny + a.by * a.rows - 1) / (a.by * a.rows))), block(kBlock);
#define VPLBM_STEP(S)                                                                             \
    (a.nt_store ? step_kernel<S, true><<<grid, block, 0, st>>>(a)                                   \
                : step_kernel<S, false><<<grid, block, 0, st>>>(a))
    switch (storage) {
    case kF64: VPLBM_STEP(kF64); break;
    case kF32: VPLBM_STEP(kF32); break;
    case kF16S: VPLBM_STEP(kF16S); break;
    case kBF16S: VPLBM_STEP(kBF16S); break;
    case kF32D: VPLBM_STEP(kF32D); break;
    case kF16SR: VPLBM_STEP(kF16SR); break;
    case kBF16SR: VPLBM_STEP(kBF16SR); break;
    default: return hipErrorInvalidValue;
    }
#undef VPLBM_STEP
    return hipGetLastError();
}

template <int S, int TW, int TH>
static void launch2(const StepArgs &a, hipStream_t st)
{
    const dim3 grid(((a.g.nx + TW - 1) / TW) * ((a.g.ny + TH - 1) / TH)), block(kBlock2);
    if (a.outlet.prev) {
        if (a.nt_store) step2_kernel<S, TW, TH, true, true><<<grid, block, 0, st>>>(a);
        else step2_kernel<S, TW, TH, false, true><<<grid, block, 0, st>>>(a);
    } else {
        if (a.nt_store) step2_kernel<S, TW, TH, true, false><<<grid, block, 0, st>>>(a);
        else step2_kernel<S, TW, TH, false, false><<<grid, block, 0, st>>>(a);
    }
}

bool step3_supported(int storage) { return storage == kF32; }

hipError_t launch_step3(int storage, const StepArgs &a, hipStream_t st)
{
    constexpr int TW = 64, TH = 14;
    if (storage != kF32) return hipErrorInvalidValue;
    const dim3 grid(((a.g.nx + TW - 1) / TW) * ((a.g.ny + TH - 1) / TH)), block(kBlock2);
    if (a.outlet.prev) {   // convective outlet: an instantiation of its own
        if (a.nt_store) step3_kernel<kF32, TW, TH, true, true><<<grid, block, 0, st>>>(a);
        else step3_kernel<kF32, TW, TH, false, true><<<grid, block, 0, st>>>(a);
    } else {
        if (a.nt_store) step3_kernel<kF32, TW, TH, true, false><<<grid, block, 0, st>>>(a);
        else step3_kernel<kF32, TW, TH, false, false><<<grid, block, 0, st>>>(a);
    }
    return hipGetLastError();
}

hipError_t launch_step2(int storage, const StepArgs &a, hipStream_t st)
{
    // 2-byte storage: tall tiles once there are enough of them (4 M nodes and up)
    const bool tall = (long long)((a.g.nx + 127) / 128) * ((a.g.ny + 15) / 16) >= 2048;
#define VPLBM_STEP2(S) (tall ? launch2<S, 128, 16>(a, st) : launch2<S, 128, 8>(a, st))
    switch (storage) {
    case kF64: launch2<kF64, 64, 8>(a, st); break;
    case kF32: launch2<kF32, 128, 8>(a, st); break;
    case kF32D: launch2<kF32D, 64, 8>(a, st); break;
    case kF16S: VPLBM_STEP2(kF16S); break;
    case kBF16S: VPLBM_STEP2(kBF16S); break;
    case kF16SR: VPLBM_STEP2(kF16SR); break;
    case kBF16SR: VPLBM_STEP2(kBF16SR); break;
    default: return hipErrorInvalidValue;
    }
#undef VPLBM_STEP2
    return hipGetLastError();
}

// ---- observation -------------------------------------------------------------------------------

template <int S>
__global__ __launch_bounds__(kBlock) void readback_kernel(StepArgs a, double *rho, double *ux,
                                                           double *uy)
{
    using C = Codec<S>;
    using E = typename C::elem;
    const int node = blockIdx.x * kBlock + threadIdx.x;
    if (node >= a.g.nx * a.g.ny) return;
    const int x = node % a.g.nx, y = node / a.g.nx;
    int id;
    const auto m = observe_node<S>(static_cast<const E *>(a.src), a.mask, a.bodies, a.g, a.outlet, a.p, x, y, id);
    rho[node] = 1.0 + double(m.drho);
    ux[node] = double(m.ux);
    uy[node] = double(m.uy);
}

// Convergence residual, node part: at every fluid node, |u - u_snap|^2 and |u|^2 of the velocity
// the next step would take; the snapshot becomes u at every node.  Per-workgroup sums (waves in
// order) go to part[blockIdx.x][2], so the result does not depend on scheduling.
template <int S>
__global__ __launch_bounds__(kBlock) void residual_kernel(StepArgs a, double *snap, double *part)
{
    using C = Codec<S>;
    using E = typename C::elem;
    __shared__ double wsum[kBlock / 64][2];
    const int n = a.g.nx * a.g.ny;
    const int node = blockIdx.x * kBlock + threadIdx.x;
    double d2 = 0.0, u2 = 0.0;
    if (node < n) {
        const int x = node % a.g.nx, y = node / a.g.nx;
        int id;
        const auto m = observe_node<S>(static_cast<const E *>(a.src), a.mask, a.bodies, a.g, a.outlet, a.p, x, y, id);
        const double ux = double(m.ux), uy = double(m.uy);
        if (id == 0) {
            const double dx = ux - snap[node], dy = uy - snap[n + node];
            d2 = dx * dx + dy * dy;
            u2 = ux * ux + uy * uy;
        }
        snap[node] = ux;
        snap[n + node] = uy;
    }
    d2 = wave_sum(d2);
    u2 = wave_sum(u2);
    if ((threadIdx.x & 63) == 0) {
        wsum[threadIdx.x >> 6][0] = d2;
        wsum[threadIdx.x >> 6][1] = u2;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double v = 0.0;
        for (int w = 0; w < kBlock / 64; w++) v += wsum[w][threadIdx.x];
        part[2 * blockIdx.x + threadIdx.x] = v;
    }
}

// Sum part[nparts][2] in a fixed order into out[2] (one wave: lane l takes parts l, l + 64, ...).
__global__ void residual_fold_kernel(const double *part, int nparts, double *out)
{
    double d2 = 0.0, u2 = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 64) {
        d2 += part[2 * i];
        u2 += part[2 * i + 1];
    }
    d2 = wave_sum(d2);
    u2 = wave_sum(u2);
    if (threadIdx.x == 0) {
        out[0] = d2;
        out[1] = u2;
    }
}

template <int S>
__global__ __launch_bounds__(kBlock) void init_kernel(StepArgs a, const double *rho_f,
                                                       const double *ux_f, const double *uy_f,
                                                       double rho0, double ux0, double uy0)
{
    using C = Codec<S>;
    using T = typename C::real;
    using E = typename C::elem;
    const int node = blockIdx.x * kBlock + threadIdx.x;
    if (node >= a.g.nx * a.g.ny) return;
    const int x = node % a.g.nx, y = node / a.g.nx;
    const int i = y * a.g.pitch + x;
    T drho, ux, uy;
    if (rho_f) {
        drho = T(rho_f[node] - 1.0);
        ux = T(ux_f[node]);
        uy = T(uy_f[node]);
    } else {
        drho = T(rho0 - 1.0);
        ux = T(ux0);
        uy = T(uy0);
        const int id = a.mask[i];
        if (id) solid_velocity(a.bodies[id - 1], x, y, ux, uy);
    }
    T f[9];
    equilibrium(drho, ux, uy, f);
    E *dst = static_cast<E *>(a.dst);
#pragma unroll
    for (int k = 0; k < 9; k++) C::store(dst + k * a.g.plane, i, f[k], weight<T>(k));
}

template <int S>
__global__ __launch_bounds__(kBlock) void encode_kernel(StepArgs a, const double *pop)
{
    using C = Codec<S>;
    using E = typename C::elem;
    const int node = blockIdx.x * kBlock + threadIdx.x;
    const int n = a.g.nx * a.g.ny;
    if (node >= n) return;
    const int x = node % a.g.nx, y = node / a.g.nx;
    const int i = y * a.g.pitch + x;
    E *dst = static_cast<E *>(a.dst);
#pragma unroll
    for (int k = 0; k < 9; k++) C::encode(dst + k * a.g.plane, i, pop[(size_t)k * n + node], weight<double>(k));
}

template <int S>
__global__ __launch_bounds__(kBlock) void decode_kernel(StepArgs a, double *pop)
{
    using C = Codec<S>;
    using E = typename C::elem;
    const int node = blockIdx.x * kBlock + threadIdx.x;
    const int n = a.g.nx * a.g.ny;
    if (node >= n) return;
    const int x = node % a.g.nx, y = node / a.g.nx;
    const int i = y * a.g.pitch + x;
    const E *src = static_cast<const E *>(a.src);
#pragma unroll
    for (int k = 0; k < 9; k++) pop[(size_t)k * n + node] = C::decode(src + k * a.g.plane, i, weight<double>(k));
}

#define VPLBM_DISPATCH(storage, kern, ...)                                                        \
    switch (storage) {                                                                           \
    case kF64: kern<kF64><<<grid, block, 0, st>>>(__VA_ARGS__); break;                          \
    case kF32: kern<kF32><<<grid, block, 0, st>>>(__VA_ARGS__); break;                          \
    case kF16S: kern<kF16S><<<grid, block, 0, st>>>(__VA_ARGS__); break;                        \
    case kBF16S: kern<kBF16S><<<grid, block, 0, st>>>(__VA_ARGS__); break;                      \
    case kF32D: kern<kF32D><<<grid, block, 0, st>>>(__VA_ARGS__); break;                        \
    case kF16SR: kern<kF16SR><<<grid, block, 0, st>>>(__VA_ARGS__); break;                      \
    case kBF16SR: kern<kBF16SR><<<grid, block, 0, st>>>(__VA_ARGS__); break;                    \
    default: return hipErrorInvalidValue;                                                        \
    }

static dim3 node_grid(const Geom &g) { return dim3((g.nx * g.ny + kBlock - 1) / kBlock); }

hipError_t launch_readback(int storage, const StepArgs &a, double *rho, double *ux, double *uy,
                           hipStream_t st)
{
    const dim3 grid = node_grid(a.g), block(kBlock);
    VPLBM_DISPATCH(storage, readback_kernel, a, rho, ux, uy);
    return hipGetLastError();
}

int residual_parts(const Geom &g) { return (g.nx * g.ny + kBlock - 1) / kBlock; }

hipError_t launch_residual(int storage, const StepArgs &a, double *snap, double *part, double *out,
                           hipStream_t st)
{
    const dim3 grid = node_grid(a.g), block(kBlock);
    VPLBM_DISPATCH(storage, residual_kernel, a, snap, part);
    residual_fold_kernel<<<1, 64, 0, st>>>(part, (int)grid.x, out);
    return hipGetLastError();
}

hipError_t launch_init(int storage, const StepArgs &a, const double *rho, const double *ux,
                       const double *uy, double rho0, double ux0, double uy0, hipStream_t st)
{
    const dim3 grid = node_grid(a.g), block(kBlock);
    VPLBM_DISPATCH(storage, init_kernel, a, rho, ux, uy, rho0, ux0, uy0);
    return hipGetLastError();
}

hipError_t launch_encode(int storage, const StepArgs &a, const double *pop, hipStream_t st)
{
    const dim3 grid = node_grid(a.g), block(kBlock);
    VPLBM_DISPATCH(storage, encode_kernel, a, pop);
    return hipGetLastError();
}

hipError_t launch_decode(int storage, const StepArgs &a, double *pop, hipStream_t st)
{
    const dim3 grid = node_grid(a.g), block(kBlock);
    VPLBM_DISPATCH(storage, decode_kernel, a, pop);
    return hipGetLastError();
}

// Momentum exchange over the fluid-solid links of the current (post-collision) state: for a fluid
// node x_f and a solid node x_s = x_f + xi_a of body k, streaming carries xi_a (g_a(x_f) +
// g_abar(x_s)) into the body.  Links through a periodic edge wrap; through other edges they do
// not exist.  out[2k], out[2k+1] accumulate body k's (fx, fy) in FP64.
template <int S>
__global__ __launch_bounds__(kBlock) void momentum_exchange_kernel(StepArgs a, double *out)
{
    using C = Codec<S>;
    using E = typename C::elem;
    constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    __shared__ double acc[2 * kMaxBodies];
    if (threadIdx.x < 2 * kMaxBodies) acc[threadIdx.x] = 0.0;
    __syncthreads();
    const int node = blockIdx.x * kBlock + threadIdx.x;
    const Geom &g = a.g;
    if (node < g.nx * g.ny) {
        const int x = node % g.nx, y = node / g.nx;
        const E *src = static_cast<const E *>(a.src);
        if (a.mask[y * g.pitch + x] == 0) {
#pragma unroll
            for (int d = 1; d < 9; d++) {
                int xs = x + cx[d], ys = y + cy[d];
                if (xs < 0 || xs >= g.nx) {
                    if (!g.xper) continue;
                    xs += xs < 0 ? g.nx : -g.nx;
                }
                if (ys < 0 || ys >= g.ny) {
                    if (!g.yper) continue;
                    ys += ys < 0 ? g.ny : -g.ny;
                }
                const int id = a.mask[ys * g.pitch + xs];
                if (!id) continue;
                const double m = C::decode(src + d * g.plane, y * g.pitch + x, weight<double>(d)) +
                                 C::decode(src + opp[d] * g.plane, ys * g.pitch + xs, weight<double>(opp[d]));
                atomicAdd(&acc[2 * (id - 1)], cx[d] * m);
                atomicAdd(&acc[2 * (id - 1) + 1], cy[d] * m);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * kMaxBodies && acc[threadIdx.x] != 0.0) unsafeAtomicAdd(out + threadIdx.x, acc[threadIdx.x]);
}

hipError_t launch_momentum_exchange(int storage, const StepArgs &a, double *out, hipStream_t st)
{
    const dim3 grid = node_grid(a.g), block(kBlock);
    VPLBM_DISPATCH(storage, momentum_exchange_kernel, a, out);
    return hipGetLastError();
}

template <int S>
__global__ void outlet_init_kernel(StepArgs a, void *prev)
{
    using C = Codec<S>;
    using T = typename C::real;
    using E = typename C::elem;
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= a.g.ny) return;
    constexpr int dirs[3] = {3, 6, 7};
    const E *src = static_cast<const E *>(a.src);
    T *p = static_cast<T *>(prev);
#pragma unroll
    for (int k = 0; k < 3; k++)
        p[k * a.g.ny + y] = C::load(src + dirs[k] * a.g.plane, y * a.g.pitch + a.g.nx - 1, weight<T>(dirs[k]));
}

hipError_t launch_outlet_init(int storage, const StepArgs &a, void *prev, hipStream_t st)
{
    const dim3 grid((a.g.ny + 255) / 256), block(256);
    VPLBM_DISPATCH(storage, outlet_init_kernel, a, prev);
    return hipGetLastError();
}

// ---- obstacles ---------------------------------------------------------------------------------

// State of a body at time t: centre c0 + a sin(2 pi f t), velocity U + 2 pi f a cos(2 pi f t).
// FP64 without contraction; every kernel that places bodies uses this one function.
__device__ __forceinline__ BodyState body_state_at(const BodyParams &b, double t)
{
#pragma clang fp contract(off)
    const double two_pi = 6.283185307179586;
    const double ph = two_pi * b.freq * t;
    const double sn = sin(ph), cs = cos(ph);
    BodyState o;
    o.cx = b.cx + b.ax * sn;
    o.cy = b.cy + b.ay * sn;
    o.vx = b.ux + b.ax * two_pi * b.freq * cs;
    o.vy = b.uy + b.ay * two_pi * b.freq * cs;
    o.omega = b.omega;
    return o;
}

// Body id of node (x, y): node-centre inclusion in FP64 without contraction, so that the decision
// is the correctly rounded one; the lowest-index body containing the node owns it.
__device__ __forceinline__ uint8_t rasterize_node(int x, int y, const BodyParams *p,
                                                  const BodyState *s, int nb)
{
#pragma clang fp contract(off)
    int id = 0;
    for (int k = 0; k < nb && id == 0; k++) {
        const double dx = double(x) - s[k].cx, dy = double(y) - s[k].cy;
        const double d2 = dx * dx + dy * dy;
        const double r2 = p[k].r * p[k].r;
        bool inside;
        if (p[k].kind == 0) inside = d2 <= r2;
        else if (p[k].kind == 1) inside = fabs(dx) <= p[k].hx && fabs(dy) <= p[k].hy;
        else inside = d2 >= r2;
        if (inside) id = k + 1;
    }
    return (uint8_t)id;
}

__global__ void bodies_kernel(const BodyParams *p, BodyState *s, int nb, const long long *t_base,
                              int t_off)
{
    const int k = threadIdx.x;
    if (k >= nb) return;
    s[k] = body_state_at(p[k], double(*t_base + t_off));
}

__global__ __launch_bounds__(kBlock) void mask_kernel(uint8_t *mask, Geom g, const BodyParams *p,
                                                      const BodyState *s, int nb, int x0, int y0,
                                                      int w, int h)
{
    const int node = blockIdx.x * kBlock + threadIdx.x;
    if (node >= w * h) return;
    const int x = x0 + node % w, y = y0 + node / w;
    if (x < 0 || x >= g.nx || y < 0 || y >= g.ny) return;
    mask[y * g.pitch + x] = rasterize_node(x, y, p, s, nb);
}

// Moving bodies before a launch of a.nsteps (1 to 3) steps: for each step s, the body states at
// time *t_base + t_off + s into a.state[s] and the swept boxes of the moving bodies re-rasterized
// into a.mask[s], in one launch.  Every workgroup computes the states it needs into LDS (a few
// FP64 sines per body); workgroup 0 also stores them.  The box nodes of all steps are spread over
// the grid.  Boxes may overlap: such a node is written more than once with the same id.
__global__ __launch_bounds__(kBlock) void place_kernel(PlaceArgs a)
{
    __shared__ BodyState st[kMaxSteps][kMaxBodies];
    __shared__ BodyParams bp[kMaxBodies];
    const int nb = a.nbodies;
    if ((int)threadIdx.x < nb) bp[threadIdx.x] = a.params[threadIdx.x];
    __syncthreads();
    if ((int)threadIdx.x < a.nsteps * nb) {
        const int sidx = threadIdx.x / nb, k = threadIdx.x % nb;
        const BodyState o = body_state_at(bp[k], double(*a.t_base + a.t_off + sidx));
        st[sidx][k] = o;
        if (blockIdx.x == 0) a.state[sidx][k] = o;
    }
    __syncthreads();
    const int total = a.box_start[kMaxBodies];
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.nsteps * total; i += gridDim.x * kBlock) {
        const int sidx = i / total, j = i % total;
        int k = 0;
        while (j >= a.box_start[k + 1]) k++;
        const int* b = a.box[k];
        const int e = j - a.box_start[k];
        const int x = b[0] + e % b[2], y = b[1] + e / b[2];
        a.mask[sidx][y * a.g.pitch + x] = rasterize_node(x, y, bp, st[sidx], nb);
    }
}

hipError_t launch_bodies(const BodyParams *params, BodyState *state, int nbodies,
                         const long long *t_base, int t_off, hipStream_t st)
{
    bodies_kernel<<<1, 64, 0, st>>>(params, state, nbodies, t_base, t_off);
    return hipGetLastError();
}

hipError_t launch_place(const PlaceArgs &a, hipStream_t st)
{
    const int total = a.nsteps * a.box_start[kMaxBodies];
    if (total <= 0) {
        // no swept box: only the states (bodies that move without changing the mask)
        place_kernel<<<1, kBlock, 0, st>>>(a);
        return hipGetLastError();
    }
    int blocks = (total + kBlock - 1) / kBlock;
    blocks = blocks > 1024 ? 1024 : blocks;
    place_kernel<<<blocks, kBlock, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_mask(uint8_t *mask, const Geom &g, const BodyParams *params,
                       const BodyState *state, int nbodies, int x0, int y0, int w, int h,
                       hipStream_t st)
{
    if (w <= 0 || h <= 0) return hipSuccess;
    const dim3 grid((w * h + kBlock - 1) / kBlock), block(kBlock);
    mask_kernel<<<grid, block, 0, st>>>(mask, g, params, state, nbodies, x0, y0, w, h);
    return hipGetLastError();
}

// ---- small helpers (fill kernels rather than memsets so they can sit in captured graphs) -----

__global__ void advance_kernel(long long *t, long long n) { *t += n; }

__global__ void fill_f64_kernel(double *p, size_t n, double v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_u32_kernel(unsigned *p, size_t n, unsigned v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_advance(long long *t_base, long long n, hipStream_t st)
{
    advance_kernel<<<1, 1, 0, st>>>(t_base, n);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, size_t n, double v, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const size_t blocks = (n + kBlock - 1) / kBlock;
    fill_f64_kernel<<<dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(kBlock), 0, st>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned *p, size_t n, unsigned v, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const size_t blocks = (n + kBlock - 1) / kBlock;
    fill_u32_kernel<<<dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(kBlock), 0, st>>>(p, n, v);
    return hipGetLastError();
}

}  // namespace vplbm
