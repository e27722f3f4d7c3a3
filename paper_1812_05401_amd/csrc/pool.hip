// Serving pool: many resident VP-LBM simulations advanced together by a batched step kernel
// replayed from a captured HIP graph (see the pool section of include/vplbm.h).
//
// Device side.  A descriptor per slot (buffers, geometry, parameters, admission step, target) and
// a table of tiles covering every resident simulation.  One workgroup per tile.  Binary32
// simulations take three steps per launch on 64 x 14 tiles, the first two kept in LDS as in the
// single-simulation three-step kernel; the other formats two steps per launch on 64 x 8 tiles, the
// first kept in LDS as in the two-step kernel.  Each tile runs the same per-node update as the
// single-simulation step, so a simulation's fields do not depend on its co-residents or on the
// launch shape.  All resident simulations advance together, so a simulation's
// steps done are the pool's step counter (on the device) minus its admission step: no per-step
// bookkeeping launch is needed.  On a simulation's final step each tile writes its FP64 partial
// sums (mass, body forces) to its own slot, summed in a fixed order inside the tile; at
// retirement a fold kernel adds the tiles in tile order, so the final observables are bitwise
// independent of the mix.
//
// Early stop: for simulations that ask for it, the graph ends with a residual check (a per-tile
// kernel and a per-slot fold) that lowers the simulation's target on the device once its
// velocity change is below the tolerance.
//
// Host side.  Between graph replays: retire finished, failed and cancelled simulations (fold,
// copy results, free memory), admit queued requests first come first served while the memory
// budget, the slots and the resident-node cap allow, rebuild the tile table.  The graph reads the
// tables from device memory; it is captured again only when the tile count outgrows its grid or
// the residual check is switched on or off.
#include <math.h>
#include <stddef.h>
#include <string.h>

#include <deque>
#include <map>
#include <mutex>
#include <unordered_set>
#include <vector>

#include "internal.hpp"
#include "pool_policy.hpp"

using namespace vplbm;

namespace vplbm {

constexpr int kPoolTileW = 64, kPoolTileH = 8;   // 512 nodes: one per thread of kBlock2
constexpr int kPoolEW = kPoolTileW + 2, kPoolEN = kPoolEW * (kPoolTileH + 2);
// binary32: three steps per launch on 64 x 14 tiles, an LDS tile with a two-node halo
constexpr int kPool3H = 14;
constexpr int kPool3EW = kPoolTileW + 4, kPool3EN = kPool3EW * (kPool3H + 4);
constexpr int kPoolMaxSlots = 1024;
static_assert(kPoolTileW * kPoolTileH == kBlock2, "one node per thread in the second step");

struct PoolSim {
    void *buf[2];
    const uint8_t *mask;
    const BodyState *bodies;
    double *partials;        // [ntiles][kRingWidth] of the final step
    Geom g;
    NodeParams p;
    int storage;
    int ntx, ntiles;
    int th;                  // tile height (the tile width is kPoolTileW)
    int spk;                 // steps per kernel launch: 3 for binary32, else 2
    int nt;                  // 1: non-temporal population stores (the resident buffers exceed the cache)
    int conv;                // 1: convective outlet at x = nx - 1
    double ou;               // its convection speed (the inlet speed)
    void *outlet[2];         // its recorded values (3 x ny, compute type) per buffer parity
    int active;
    int spl;                 // steps per graph replay (the pool's steps_per_launch)
    long long t0, target;    // pool step at admission; steps to run
    unsigned status;
    double obs[kRingWidth];  // folded final observables
    // early stop (tol > 0): residual checks at done >= next_check, every `every` steps
    double tol, residual;
    long long every, next_check;
    int have_snap;
    double *snap;            // [2][ny*nx] velocity at the last check
    double *rpart;           // [ntiles][2] residual partial sums
};

struct TileRef {
    int slot, tile;
};

// Buffer holding a simulation's state after `done` steps.  Each graph replay of spl steps runs
// ceil(spl / spk) launches of the simulation's kernel from the replay's start, spk steps each and
// what remains last; a simulation is admitted at a replay boundary, and a launch moves its state
// to the other buffer however many steps it takes (fewer when the simulation has fewer left).
__host__ __device__ inline int pool_buf(long long done, int spl, int spk)
{
    const long long launches = (done / spl) * ((spl + spk - 1) / spk) + ((done % spl) + spk - 1) / spk;
    return (int)(launches & 1);
}

// The final step's per-tile sums (mass, body forces): wave shuffles, then the waves in order,
// into the tile's slot of the simulation's partials.  Called by every thread of the workgroup.
template <bool DPP>
__device__ __forceinline__ void pool_tile_partials(const PoolSim &d, int tile, double rho, double fx,
                                                   double fy, int id, double (*part)[kRingWidth])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < kRingWidth) part[wave][lane] = 0.0;
    const double mw = wave_sum<DPP>(rho);
    if (lane == 0) part[wave][0] = mw;
    unsigned long long solid = __ballot(id != 0);
    while (solid) {
        const int lead = __ffsll((unsigned long long)solid) - 1;
        const int b = __shfl(id, lead, 64);
        const bool mine = id == b;
        const double sx = wave_sum<DPP>(mine ? -fx : 0.0);
        const double sy = wave_sum<DPP>(mine ? -fy : 0.0);
        if (lane == 0) {
            part[wave][1 + 2 * (b - 1)] = sx;
            part[wave][2 + 2 * (b - 1)] = sy;
        }
        solid &= ~__ballot(mine);
    }
    __syncthreads();
    if (threadIdx.x < kRingWidth) {
        double v = 0.0;
        for (int w = 0; w < kBlock2 / 64; w++) v += part[w][threadIdx.x];
        d.partials[(size_t)tile * kRingWidth + threadIdx.x] = v;
    }
}

// One tile of one simulation for `nsteps` (1 or 2) steps from `done`: the node arithmetic of the
// single-simulation kernels (update_node, or the two-step form with the first step kept in LDS),
// so a simulation's fields do not depend on the launch shape or its co-residents.  CONV: the
// simulation has a convective outlet; as in the single-simulation two-step kernel, the first step
// reads the previous values from global memory and keeps what it records for the tile's rows in
// LDS (outl, 3 x kPoolTileH values), and the second applies the outlet rule with them and records
// its own for the next launch.
template <int S, bool CONV>
__device__ __forceinline__ void pool_tile(const PoolSim &d, int tile, long long done, int nsteps,
                                          unsigned char *lds, double (*part)[kRingWidth],
                                          double *outl_lds, unsigned *status)
{
    using C = Codec<S>;
    using T = typename C::real;
    using E = typename C::elem;
    constexpr int odirs[3] = {3, 6, 7};           // the directions entering from x = nx
    const Geom &g = d.g;
    const int b = pool_buf(done, d.spl, d.spk);
    // selects rather than indexing: the kernel holds d in registers, not in memory
    const E *__restrict__ src = static_cast<const E *>(b ? d.buf[1] : d.buf[0]);
    E *__restrict__ dst = static_cast<E *>(b ? d.buf[0] : d.buf[1]);
    const Outlet none{nullptr, nullptr, 0.0};
    void *const oprev = b ? d.outlet[1] : d.outlet[0];
    void *const onext = b ? d.outlet[0] : d.outlet[1];
    const Outlet one{CONV ? oprev : nullptr, CONV ? onext : nullptr, d.ou};
    const Outlet out1{CONV ? oprev : nullptr, nullptr, d.ou};
    T *outl = reinterpret_cast<T *>(outl_lds);
    const int x0 = (tile % d.ntx) * kPoolTileW, y0 = (tile / d.ntx) * kPoolTileH;
    const int x = x0 + (threadIdx.x % kPoolTileW), y = y0 + (threadIdx.x / kPoolTileW);
    const bool active = (x < g.nx) & (y < g.ny);
    double rho = 0.0, fx = 0.0, fy = 0.0;
    int id = 0;
    bool bad = false;
    if (nsteps == 1) {
        if (active) {
            const auto m = update_node<S>(src, dst, d.mask, d.bodies, g, CONV ? one : none, d.p, x, y, id,
                                          (unsigned)done);
            rho = 1.0 + double(m.drho);
            fx = double(m.fx);
            fy = double(m.fy);
            bad = !(rho > 0.0 && rho < 1e30);
        }
    } else {
        E *mid = reinterpret_cast<E *>(lds);
        for (int it = 0; it < (kPoolEN + kBlock2 - 1) / kBlock2; it++) {
            const int e = threadIdx.x + it * kBlock2;
            const int lx = e % kPoolEW - 1, ly = e / kPoolEW - 1;
            int hx = x0 + lx, hy = y0 + ly;
            bool live = e < kPoolEN;
            if (hx < 0 || hx >= g.nx) {
                if (g.xper && hx >= -1 && hx <= g.nx) hx += hx < 0 ? g.nx : -g.nx;
                else live = false;
            }
            if (hy < 0 || hy >= g.ny) {
                if (g.yper && hy >= -1 && hy <= g.ny) hy += hy < 0 ? g.ny : -g.ny;
                else live = false;
            }
            if (live) {
                T f[9];
                int hid;
                const bool own = (lx >= 0) & (lx < kPoolTileW) & (ly >= 0) & (ly < kPoolTileH) &
                                 (x0 + lx < g.nx) & (y0 + ly < g.ny);
                pull<S>(src, hx, hy, g, CONV ? out1 : none, f);
                if (CONV && hx == g.nx - 1 && own)
                    for (int k = 0; k < 3; k++) outl[k * kPoolTileH + ly] = f[odirs[k]];
                const auto m = relax_node(f, d.mask, d.bodies, g, d.p, hx, hy, hid);
                store_node<S>(mid, kPoolEN, unsigned(e), f, unsigned(hy * g.pitch + hx), (unsigned)done);
                const double r1 = 1.0 + double(m.drho);
                bad |= own && !(r1 > 0.0 && r1 < 1e30);
            }
        }
        __syncthreads();
        if (active) {
            T f[9];
            pull_tile<S>(mid, kPoolEN, kPoolEW, x, y, x0, y0, g, f);
            if (CONV && x == g.nx - 1) {
                // the outlet rule of pull, with the first step's values from LDS
                const T u = T(d.ou);
                T *next = static_cast<T *>(onext);
                for (int k = 0; k < 3; k++) {
                    int pa;
                    const unsigned jn = tile_source(odirs[k], g.nx - 2, y, x0, y0, kPoolEW, g, pa);
                    const T nb = C::load(mid + pa * kPoolEN, jn, weight<T>(odirs[k]));
                    f[odirs[k]] = (outl[k * kPoolTileH + (y - y0)] + u * nb) / (T(1) + u);
                }
                for (int k = 0; k < 3; k++) next[k * g.ny + y] = f[odirs[k]];
            }
            const auto m = relax_node(f, d.mask, d.bodies, g, d.p, x, y, id);
            const unsigned i = y * g.pitch + x;
            store_node<S>(dst, g.plane, i, f, i, (unsigned)(done + 1));
            rho = 1.0 + double(m.drho);
            fx = double(m.fx);
            fy = double(m.fy);
            bad |= !(rho > 0.0 && rho < 1e30);
        }
    }
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(status, 1u);
    if (done + nsteps == d.target) pool_tile_partials<wave_sum_dpp<T>()>(d, tile, rho, fx, fy, id, part);
}

// The lattice node at unwrapped position (ux, uy) of a tile, h or fewer nodes outside it: live
// unless beyond a non-periodic edge or more than h beyond the lattice (a ragged tile); a position
// across a periodic edge is the wrapped node.
__device__ __forceinline__ bool pool_locate(const Geom &g, int ux, int uy, int h, int &x, int &y)
{
    x = ux;
    y = uy;
    if (x < 0 || x >= g.nx) {
        if (g.xper && x >= -h && x < g.nx + h) x += x < 0 ? g.nx : -g.nx;
        else return false;
    }
    if (y < 0 || y >= g.ny) {
        if (g.yper && y >= -h && y < g.ny + h) y += y < 0 ? g.ny : -g.ny;
        else return false;
    }
    return true;
}

// pull_interior_buf and store_node_buf (binary32) for the pool, with each plane's scalar offset
// passed through readfirstlane.  The offsets are uniform over the workgroup (the simulation's
// pitch and plane size); stated so, the compiler keeps them in scalar registers instead of
// wrapping each buffer access in a loop over distinct lane values.
__device__ __forceinline__ void pool_pull_buf(__amdgpu_buffer_rsrc_t r, unsigned plane, unsigned pitch,
                                              unsigned i, float f[9])
{
    const int v = int(i * 4u);
    const int P = int(pitch);
    const int shift[9] = {0, -1, -P, 1, P, -P - 1, -P + 1, P + 1, P - 1};
#pragma unroll
    for (int a = 0; a < 9; a++) {
        const int so = __builtin_amdgcn_readfirstlane(int((unsigned(a) * plane + unsigned(shift[a])) * 4u));
        f[a] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, v, so, 0));
    }
}

template <bool NT>
__device__ __forceinline__ void pool_store_buf(__amdgpu_buffer_rsrc_t r, unsigned plane, unsigned i,
                                               const float f[9])
{
#pragma unroll
    for (int k = 0; k < 9; k++) {
        const int so = __builtin_amdgcn_readfirstlane(int(unsigned(k) * plane * 4u));
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(f[k]), r, int(i * 4u), so, NT ? 2 : 0);   // 2: nt
    }
}

// First phase of a multi-step launch on a 64 x kPool3H tile: step `step` on the tile and a halo
// of H nodes, from the planes in global memory into the LDS tile, whose slots are laid out with a
// two-node halo (kPool3EW per row) whatever H is.  Returns whether an own node went bad.  CONV:
// the convective outlet reads the previous records `prev` and the values this step records at
// x = nx - 1 go to rec1 for rows y0 - 1 .. y0 + kPool3H (3 x (kPool3H + 2), unwrapped rows).
template <int S, int H, bool inner, bool CONV = false>
__device__ __forceinline__ bool pool_first_phase(const PoolSim &d, const typename Codec<S>::elem *src,
                                                 __amdgpu_buffer_rsrc_t rsrc,
                                                 typename Codec<S>::elem *mid, int x0, int y0,
                                                 unsigned step, void *prev = nullptr,
                                                 typename Codec<S>::real *rec1 = nullptr)
{
    using T = typename Codec<S>::real;
    constexpr int W1 = kPoolTileW + 2 * H, N1 = W1 * (kPool3H + 2 * H);
    constexpr int odirs[3] = {3, 6, 7};           // the directions entering from x = nx
    const Geom &g = d.g;
    const Outlet none{nullptr, nullptr, 0.0};
    const Outlet out1{prev, nullptr, d.ou};
    bool bad = false;
    for (int e = threadIdx.x; e < N1; e += kBlock2) {
        const int ux = x0 + e % W1 - H, uy = y0 + e / W1 - H;
        int x = ux, y = uy;
        if (!inner && !pool_locate(g, ux, uy, H, x, y)) continue;
        T f[9];
        int id;
        if constexpr (inner) pool_pull_buf(rsrc, g.plane, g.pitch, unsigned(y * g.pitch + x), f);
        else pull<S>(src, x, y, g, CONV ? out1 : none, f);
        if (CONV && x == g.nx - 1 && uy >= y0 - 1 && uy <= y0 + kPool3H)
            for (int q = 0; q < 3; q++) rec1[q * (kPool3H + 2) + (uy - y0 + 1)] = f[odirs[q]];
        const auto m = relax_node(f, d.mask, d.bodies, g, d.p, x, y, id);
        store_node<S>(mid, kPool3EN, unsigned((uy - y0 + 2) * kPool3EW + (ux - x0 + 2)), f,
                      unsigned(y * g.pitch + x), step);
        const bool own = (ux >= x0) & (ux < x0 + kPoolTileW) & (uy >= y0) & (uy < y0 + kPool3H) &
                         (ux < g.nx) & (uy < g.ny);
        const double r1 = 1.0 + double(m.drho);
        bad |= own && !(r1 > 0.0 && r1 < 1e30);
    }
    return bad;
}

// One 64 x kPool3H tile of a binary32 simulation for k (1 to 3) steps from `done`, as the
// single-simulation kernels compute them: for k = 3 step done on the tile and a two-node halo into
// LDS, step done + 1 on the tile and a one-node halo in place (its results held in registers
// until every pull is made), step done + 2 of the tile to global memory; for k = 2 the first
// phase with a one-node halo and the last; for k = 1 the last alone, from global memory.  On the
// simulation's final step the tile's FP64 sums go to its slot of the partials (per-wave rows
// added in order, rows in order).  inner: the tile lies three or more nodes from every edge of a
// simulation whose planes span less than 4 GB (pool3_inner); then every phase pulls by plain
// shifts, the first through a buffer resource, and the last stores through one, as the
// single-simulation three-step kernel does for its inner tiles.  CONV (edge tiles only): the
// convective outlet, its recorded values passed from phase to phase in LDS (outl_lds) as in the
// single-simulation three-step kernel, the last phase writing them for the next launch.
template <int S, bool inner, bool CONV>
__device__ __forceinline__ void pool_tile3(const PoolSim &d, int tile, long long done, int k,
                                           unsigned char *lds, double (*part)[kRingWidth],
                                           double *outl_lds, unsigned *status)
{
    using C = Codec<S>;
    using T = typename C::real;
    using E = typename C::elem;
    constexpr int TW = kPoolTileW, TH = kPool3H, EW = kPool3EW, EN = kPool3EN;
    constexpr bool DPP = wave_sum_dpp<T>();
    const Geom &g = d.g;
    const int b = pool_buf(done, d.spl, d.spk);
    // selects rather than indexing: the kernel holds d in registers, not in memory
    const E *__restrict__ src = static_cast<const E *>(b ? d.buf[1] : d.buf[0]);
    E *__restrict__ dst = static_cast<E *>(b ? d.buf[0] : d.buf[1]);
    const Outlet none{nullptr, nullptr, 0.0};
    void *const oprev = b ? d.outlet[1] : d.outlet[0];
    void *const onext = b ? d.outlet[0] : d.outlet[1];
    constexpr int odirs[3] = {3, 6, 7};           // the directions entering from x = nx
    T *rec1 = reinterpret_cast<T *>(outl_lds);     // first phase's records, rows y0 - 1 .. y0 + TH
    T *rec2 = rec1 + 3 * (TH + 2);                 // middle phase's records, rows y0 .. y0 + TH - 1
    const int x0 = (tile % d.ntx) * TW, y0 = (tile / d.ntx) * TH;
    E *mid = reinterpret_cast<E *>(lds);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool final_step = done + k == d.target;             // uniform over the workgroup
    if (final_step && lane < kRingWidth) part[wave][lane] = 0.0;
    const unsigned long long pbytes = 9ull * (unsigned long long)g.plane * sizeof(E);
    const __amdgpu_buffer_rsrc_t rsrc = buffer_over(const_cast<E *>(src), unsigned(pbytes));
    const __amdgpu_buffer_rsrc_t rdst = buffer_over(dst, unsigned(pbytes));
    bool bad = false;
    if (k == 3) {
        bad |= pool_first_phase<S, 2, inner, CONV>(d, src, rsrc, mid, x0, y0, (unsigned)done, oprev, rec1);
        __syncthreads();
        constexpr int MW = TW + 2, MN = MW * (TH + 2), R2 = (MN + kBlock2 - 1) / kBlock2;
        T res[R2][9];
        int slot[R2];
        unsigned node[R2];
#pragma unroll
        for (int it = 0; it < R2; it++) {
            const int j = threadIdx.x + it * kBlock2;
            const int ux = x0 + j % MW - 1, uy = y0 + j / MW - 1;
            int x = ux, y = uy;
            slot[it] = -1;
            node[it] = 0;
            if (j < MN && (inner || pool_locate(g, ux, uy, 1, x, y))) {
                int id;
                if constexpr (inner) pull_tile_shifts<S, 2>(mid, EN, EW, ux, uy, x0, y0, res[it]);
                else pull_tile<S, 2>(mid, EN, EW, ux, uy, x0, y0, g, res[it]);
                if (CONV && x == g.nx - 1) {
                    // the outlet rule of pull, with the first phase's records and neighbours
                    const T u = T(d.ou);
                    for (int q = 0; q < 3; q++) {
                        int pa;
                        const unsigned jn = tile_source<2>(odirs[q], g.nx - 2, uy, x0, y0, EW, g, pa);
                        const T nb = C::load(mid + pa * EN, jn, weight<T>(odirs[q]));
                        res[it][odirs[q]] = (rec1[q * (TH + 2) + (uy - y0 + 1)] + u * nb) / (T(1) + u);
                    }
                    if (uy >= y0 && uy < y0 + TH)
                        for (int q = 0; q < 3; q++) rec2[q * TH + (uy - y0)] = res[it][odirs[q]];
                }
                const auto m = relax_node(res[it], d.mask, d.bodies, g, d.p, x, y, id);
                slot[it] = (j / MW + 1) * EW + j % MW + 1;
                node[it] = unsigned(y * g.pitch + x);
                const bool own = (ux >= x0) & (ux < x0 + TW) & (uy >= y0) & (uy < y0 + TH) &
                                 (ux < g.nx) & (uy < g.ny);
                const double r1 = 1.0 + double(m.drho);
                bad |= own && !(r1 > 0.0 && r1 < 1e30);
            }
        }
        __syncthreads();                          // every middle-phase pull has read step done
#pragma unroll
        for (int it = 0; it < R2; it++)
            if (slot[it] >= 0) store_node<S>(mid, EN, unsigned(slot[it]), res[it], node[it], (unsigned)(done + 1));
        __syncthreads();
    } else if (k == 2) {
        bad |= pool_first_phase<S, 1, inner, CONV>(d, src, rsrc, mid, x0, y0, (unsigned)done, oprev, rec1);
        __syncthreads();
    }
    constexpr int R3 = (TW * TH + kBlock2 - 1) / kBlock2;
#pragma unroll
    for (int it = 0; it < R3; it++) {
        const int j = threadIdx.x + it * kBlock2;
        const int x = x0 + j % TW, y = y0 + j / TW;
        double rho = 0.0, fx = 0.0, fy = 0.0;
        int id = 0;
        if ((j < TW * TH) & (x < g.nx) & (y < g.ny)) {
            Macro<T> m;
            if (k == 1) {
                const Outlet one{oprev, onext, d.ou};
                m = update_node<S>(src, dst, d.mask, d.bodies, g, CONV ? one : none, d.p, x, y, id,
                                   (unsigned)done);
            } else {
                T f[9];
                if constexpr (inner) pull_tile_shifts<S, 2>(mid, EN, EW, x, y, x0, y0, f);
                else pull_tile<S, 2>(mid, EN, EW, x, y, x0, y0, g, f);
                if (CONV && x == g.nx - 1) {
                    // the outlet rule with the previous phase's records; this step's go to memory
                    const T u = T(d.ou);
                    T *next = static_cast<T *>(onext);
                    for (int q = 0; q < 3; q++) {
                        int pa;
                        const unsigned jn = tile_source<2>(odirs[q], g.nx - 2, y, x0, y0, EW, g, pa);
                        const T nb = C::load(mid + pa * EN, jn, weight<T>(odirs[q]));
                        const T pr = k == 3 ? rec2[q * TH + (y - y0)] : rec1[q * (TH + 2) + (y - y0 + 1)];
                        f[odirs[q]] = (pr + u * nb) / (T(1) + u);
                    }
                    for (int q = 0; q < 3; q++) next[q * g.ny + y] = f[odirs[q]];
                }
                m = relax_node(f, d.mask, d.bodies, g, d.p, x, y, id);
                const unsigned i = y * g.pitch + x;
                if constexpr (!inner) store_node<S>(dst, g.plane, i, f, i, (unsigned)(done + k - 1));
                else if (d.nt) pool_store_buf<true>(rdst, g.plane, i, f);
                else pool_store_buf<false>(rdst, g.plane, i, f);
            }
            rho = 1.0 + double(m.drho);
            fx = double(m.fx);
            fy = double(m.fy);
            bad |= !(rho > 0.0 && rho < 1e30);
        }
        if (final_step) {
            // this round's nodes into the wave's row (lane 0 of the wave adds, in round order)
            const double mw = wave_sum<DPP>(rho);
            if (lane == 0) part[wave][0] += mw;
            unsigned long long solid = __ballot(id != 0);
            while (solid) {
                const int lead = __ffsll((unsigned long long)solid) - 1;
                const int bb = __shfl(id, lead, 64);
                const bool mine = id == bb;
                const double sx = wave_sum<DPP>(mine ? -fx : 0.0);
                const double sy = wave_sum<DPP>(mine ? -fy : 0.0);
                if (lane == 0) {
                    part[wave][1 + 2 * (bb - 1)] += sx;
                    part[wave][2 + 2 * (bb - 1)] += sy;
                }
                solid &= ~__ballot(mine);
            }
        }
    }
    if (__ballot(bad) && lane == 0) atomicOr(status, 1u);
    if (final_step) {
        __syncthreads();
        if (threadIdx.x < kRingWidth) {
            double v = 0.0;
            for (int w = 0; w < kBlock2 / 64; w++) v += part[w][threadIdx.x];
            d.partials[(size_t)tile * kRingWidth + threadIdx.x] = v;
        }
    }
}

// Whether binary32 tile `tile` of d takes pool_tile3's inner form.
__device__ __forceinline__ bool pool3_inner(const PoolSim &d, int tile)
{
    const Geom &g = d.g;
    const int x0 = (tile % d.ntx) * kPoolTileW, y0 = (tile / d.ntx) * kPool3H;
    return (x0 >= 3) & (x0 + kPoolTileW + 3 <= g.nx) & (y0 >= 3) & (y0 + kPool3H + 3 <= g.ny) &
           (9ull * (unsigned long long)g.plane * 4ull <= 0xFFFFFFFFull);
}

// Storage formats by kernel: class 1 computes in FP64 (F64, F32D), class 0 in FP32 with 2-byte
// storage, both two steps per launch; class 2 is binary32 storage, three steps per launch.  Each
// class has a kernel of its own, so the FP32 formats are not held to the FP64 path's registers
// and LDS: measured 4 waves per SIMD with one kernel for all.
__host__ __device__ inline int pool_class(int storage, int conv)
{
    return storage == kF64 || storage == kF32D ? 1 : (storage == kF32 ? 2 : 0);
}

// Tile height and steps per kernel launch of a storage format's class.
__host__ __device__ inline int pool_tile_h(int storage, int conv) { return pool_class(storage, conv) == 2 ? kPool3H : kPoolTileH; }
__host__ __device__ inline int pool_spk(int storage, int conv) { return pool_class(storage, conv) == 2 ? 3 : 2; }

// pool_tile with or without the convective outlet (a separate instantiation, as in the
// single-simulation two-step kernel).
template <int S>
__device__ __forceinline__ void pool_tile2(const PoolSim &d, int tile, long long done, int nsteps,
                                           unsigned char *lds, double (*part)[kRingWidth], double *outl,
                                           unsigned *status)
{
    if (d.conv) pool_tile<S, true>(d, tile, done, nsteps, lds, part, outl, status);
    else pool_tile<S, false>(d, tile, done, nsteps, lds, part, outl, status);
}

// Steps t_off .. t_off + nsteps - 1 of the graph replay (nsteps up to the class's steps per
// launch), for every resident simulation of class CLASS: workgroup w (< *ntiles) updates tile
// entry w (tiles of the other classes return at once); a simulation with fewer steps left takes
// those.  The host writes the table in XCD order (upload_tables), so the entry is found without
// first reading the tile count: the two loads are issued together, and a workgroup starts with
// two dependent loads (its entry, then its simulation's descriptor) before its populations.
template <int CLASS>
__global__ __launch_bounds__(kBlock2) void pool_step_kernel(PoolSim *sims, const TileRef *tiles,
                                                            const int *ntiles,
                                                            const long long *t_base, int t_off,
                                                            int nsteps)
{
    // the LDS tile in the class's widest storage format
    __shared__ __align__(16) unsigned char lds[CLASS == 2 ? 9 * kPool3EN * 4 : 9 * kPoolEN * (CLASS ? 8 : 4)];
    __shared__ double part[kBlock2 / 64][kRingWidth];
    // convective outlet records: pool_tile's 3 x kPoolTileH values of T, pool_tile3's
    // 3 x (2 kPool3H + 2) binary32 values
    constexpr int kOutl = CLASS == 2 ? (3 * (2 * kPool3H + 2) + 1) / 2 : 3 * kPoolTileH;
    __shared__ double outl[kOutl];
    const int n = *ntiles;
    const TileRef tr = tiles[blockIdx.x];                     // the table spans the grid
    if ((int)blockIdx.x >= n) return;                         // uniform over the workgroup
    // A local copy of the descriptor: its fields are read once into scalar registers (read through
    // the pointer, they were read again after stores that might alias it: measured 16% of the
    // kernel's time).  The status flag is written through the pointer.
    const PoolSim d = sims[tr.slot];
    unsigned *status = &sims[tr.slot].status;
    const long long done = *t_base + t_off - d.t0;
    if (!d.active || done < 0 || done >= d.target) return;    // uniform over the workgroup
    if (pool_class(d.storage, d.conv) != CLASS) return;
    const int k = d.target - done < nsteps ? int(d.target - done) : nsteps;
    if constexpr (CLASS == 2) {
        if (pool3_inner(d, tr.tile)) pool_tile3<kF32, true, false>(d, tr.tile, done, k, lds, part, outl, status);
        else if (d.conv) pool_tile3<kF32, false, true>(d, tr.tile, done, k, lds, part, outl, status);
        else pool_tile3<kF32, false, false>(d, tr.tile, done, k, lds, part, outl, status);
    } else if constexpr (CLASS == 1) {
        if (d.storage == kF64) pool_tile2<kF64>(d, tr.tile, done, k, lds, part, outl, status);
        else pool_tile2<kF32D>(d, tr.tile, done, k, lds, part, outl, status);
    } else {
        switch (d.storage) {
        case kF16S: pool_tile2<kF16S>(d, tr.tile, done, k, lds, part, outl, status); break;
        case kF16SR: pool_tile2<kF16SR>(d, tr.tile, done, k, lds, part, outl, status); break;
        case kBF16SR: pool_tile2<kBF16SR>(d, tr.tile, done, k, lds, part, outl, status); break;
        default: pool_tile2<kBF16S>(d, tr.tile, done, k, lds, part, outl, status); break;
        }
    }
}

// Final observables of the simulation in `slot`: value q (workgroup q) of its tiles' partial
// sums.  Thread j adds tiles j, j + 256, ... in order, a fixed butterfly adds each wave's lanes and
// thread 0 the four waves in order, so the result depends only on the simulation's own tiles.
constexpr int kFoldBlock = 256;
__global__ __launch_bounds__(kFoldBlock) void pool_fold_kernel(PoolSim *sims, int slot)
{
    __shared__ double ws[kFoldBlock / 64];
    const int q = blockIdx.x;
    const int nt = sims[slot].ntiles;
    const double *part = sims[slot].partials;
    double v = 0.0;
    for (int t = threadIdx.x; t < nt; t += kFoldBlock) v += part[(size_t)t * kRingWidth + q];
    v = wave_sum<false>(v);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) sims[slot].obs[q] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

// Whether a simulation checks its residual after this launch (the same test in both kernels).
__device__ __forceinline__ bool residual_due(const PoolSim &d, long long done)
{
    return d.active && d.tol > 0.0 && done >= d.next_check && done < d.target;
}

// Residual check, node part, on the state after the launch's steps: |u - u_snap|^2 and |u|^2 at
// a fluid node; the snapshot becomes u.
template <int S>
__device__ __forceinline__ void pool_residual_node(const PoolSim &d, int parity, int x, int y,
                                                   double &d2, double &u2)
{
    using E = typename Codec<S>::elem;
    const Outlet o{d.conv ? d.outlet[parity] : nullptr, nullptr, d.ou};   // read, not recorded
    int id;
    const auto m = observe_node<S>(static_cast<const E *>(d.buf[parity]), d.mask, d.bodies, d.g, o, d.p, x, y, id);
    const size_t n = (size_t)d.g.nx * d.g.ny, i = (size_t)y * d.g.nx + x;
    const double ux = double(m.ux), uy = double(m.uy);
    if (id == 0) {
        const double dx = ux - d.snap[i], dy = uy - d.snap[n + i];
        d2 = dx * dx + dy * dy;
        u2 = ux * ux + uy * uy;
    }
    d.snap[i] = ux;
    d.snap[n + i] = uy;
}

// One workgroup per tile, as the step kernel; per-tile sums (waves in a fixed order).
__global__ __launch_bounds__(kBlock2) void pool_residual_kernel(PoolSim *sims, const TileRef *tiles,
                                                                const int *ntiles,
                                                                const long long *t_base, int t_off)
{
    __shared__ double part[kBlock2 / 64][2];
    const int n = *ntiles;
    if ((int)blockIdx.x >= n) return;                         // uniform over the workgroup
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const TileRef tr = tiles[blockIdx.x];                     // the table is in XCD order
    const PoolSim &d = sims[tr.slot];
    const long long done = *t_base + t_off - d.t0;
    if (!residual_due(d, done)) return;                       // uniform over the workgroup
    const int x = (tr.tile % d.ntx) * kPoolTileW + lane;
    const int y0 = (tr.tile / d.ntx) * d.th;
    double d2 = 0.0, u2 = 0.0;
    const int parity = pool_buf(done, d.spl, d.spk);
    for (int r = wave; r < d.th; r += kBlock2 / 64) {          // rows of the tile, in order
        const int y = y0 + r;
        if (x >= d.g.nx || y >= d.g.ny) continue;
        double a2 = 0.0, b2 = 0.0;
        switch (d.storage) {
        case kF64: pool_residual_node<kF64>(d, parity, x, y, a2, b2); break;
        case kF32: pool_residual_node<kF32>(d, parity, x, y, a2, b2); break;
        case kF16S: pool_residual_node<kF16S>(d, parity, x, y, a2, b2); break;
        case kF32D: pool_residual_node<kF32D>(d, parity, x, y, a2, b2); break;
        case kF16SR: pool_residual_node<kF16SR>(d, parity, x, y, a2, b2); break;
        case kBF16SR: pool_residual_node<kBF16SR>(d, parity, x, y, a2, b2); break;
        default: pool_residual_node<kBF16S>(d, parity, x, y, a2, b2); break;
        }
        d2 += a2;
        u2 += b2;
    }
    d2 = wave_sum(d2);
    u2 = wave_sum(u2);
    if (lane == 0) {
        part[wave][0] = d2;
        part[wave][1] = u2;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double v = 0.0;
        for (int w = 0; w < kBlock2 / 64; w++) v += part[w][threadIdx.x];
        d.rpart[2 * tr.tile + threadIdx.x] = v;
    }
}

// Residual check, decision: workgroup s (one wave) folds slot s's tile sums in a fixed order;
// below the tolerance the simulation gets one more step, whose observables the step kernel
// reduces.
__global__ void pool_residual_fold_kernel(PoolSim *sims, const long long *t_base, int t_off)
{
    PoolSim &d = sims[blockIdx.x];
    const long long done = *t_base + t_off - d.t0;
    if (!residual_due(d, done)) return;                       // uniform over the workgroup
    double d2 = 0.0, u2 = 0.0;
    for (int t = threadIdx.x; t < d.ntiles; t += 64) {
        d2 += d.rpart[2 * t];
        u2 += d.rpart[2 * t + 1];
    }
    d2 = wave_sum(d2);
    u2 = wave_sum(u2);
    if (threadIdx.x == 0) {
        double r = u2 > 0.0 ? sqrt(d2 / u2) : (d2 > 0.0 ? INFINITY : 0.0);
        if (!d.have_snap) r = INFINITY;
        d.residual = r;
        d.have_snap = 1;
        d.next_check = done + d.every;
        if (r < d.tol) d.target = done + 1;
    }
}

__global__ void pool_advance_kernel(long long *t, long long n) { *t += n; }

}  // namespace vplbm

namespace {

struct Request {
    int64_t id = -1;
    vplbm_config cfg{};
    std::vector<vplbm_body> bodies;
    int64_t nsteps = 0;
    int keep_fields = 0;
    double tol = 0.0;
    int64_t every = 0;
    bool cancel = false;
    double residual = INFINITY;
    int state = VPLBM_QUEUED;
    int slot = -1;
    uint64_t bytes = 0;
    int64_t done = 0;
    vplbm_obs obs{};
    std::vector<double> rho, ux, uy;
    // device memory while resident
    void *buf[2] = {nullptr, nullptr};
    uint8_t *mask = nullptr;
    BodyParams *params = nullptr;
    BodyState *state_dev = nullptr;
    double *partials = nullptr;
    double *snap = nullptr;
    double *rpart = nullptr;
    void *outlet[2] = {nullptr, nullptr};
};

int pool_geometry(const vplbm_config &c, Geom &g, int &ntx, int &ntiles)
{
    g.nx = c.nx;
    g.ny = c.ny;
    g.pitch = (c.nx + 63) / 64 * 64;
    g.plane = g.pitch * c.ny;
    g.xper = c.bc_xlo == VPLBM_PERIODIC;
    g.yper = c.bc_ylo == VPLBM_PERIODIC;
    g.inlet = c.bc_xlo == VPLBM_VELOCITY;
    const int th = pool_tile_h(c.storage, c.bc_xhi == VPLBM_CONVECTIVE);
    ntx = (c.nx + kPoolTileW - 1) / kPoolTileW;
    ntiles = ntx * ((c.ny + th - 1) / th);
    return VPLBM_OK;
}

uint64_t bytes_needed(const vplbm_config &c, bool stop = false)
{
    Geom g;
    int ntx, ntiles;
    pool_geometry(c, g, ntx, ntiles);
    const uint64_t pop = (uint64_t)9 * g.plane * elem_bytes(c.storage);
    const uint64_t residual = stop ? 2 * (uint64_t)g.nx * g.ny * sizeof(double) + (uint64_t)ntiles * 2 * sizeof(double) : 0;
    const uint64_t outlet = c.bc_xhi == VPLBM_CONVECTIVE ? 2 * 3 * (uint64_t)g.ny * sizeof(double) : 0;
    return 2 * pop + (uint64_t)g.pitch * g.ny + sizeof(BodyParams) * kMaxBodies +
           sizeof(BodyState) * kMaxBodies + (uint64_t)ntiles * kRingWidth * sizeof(double) + residual +
           outlet;
}

std::mutex g_pool_mu;
std::unordered_set<const void *> g_pools;

}  // namespace

struct vplbm_pool_s {
    vplbm_pool_config cfg{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    int grid_cap = 0;                     // workgroups per launch in the captured graph
    bool graph_checks = false;            // the graph ends with the residual-check kernels
    int graph_classes = 0;                // storage classes the graph has step kernels for
    PoolSim *d_sims = nullptr;
    TileRef *d_tiles = nullptr;
    int *d_ntiles = nullptr;
    long long *d_t = nullptr;             // pool step counter (steps every resident sim has run)
    long long *d_zero = nullptr;
    double *staging = nullptr;
    size_t staging_bytes = 0;
    int tile_cap = 0;
    int ntiles = 0;
    long long t_host = 0;                 // host copy of *d_t after the last finished chunk
    std::vector<PoolSim> h_sims;
    std::vector<int64_t> slot_req;        // request id per slot (-1 free)
    std::map<int64_t, Request> reqs;
    std::deque<int64_t> queue;
    int64_t next_id = 0;
    uint64_t used = 0;
    bool in_flight = false;
    int32_t finished = 0;
    uint64_t max_nodes = 0;               // admission cap on resident lattice nodes (0: none)
    uint64_t resident_nodes = 0;
};

namespace {

bool pool_valid(const void *p)
{
    if (!p) return false;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    return g_pools.count(p) != 0;
}

void free_request_memory(vplbm_pool p, Request &r)
{
    void *ptrs[] = {r.buf[0], r.buf[1], r.mask, r.params, r.state_dev, r.partials, r.snap, r.rpart,
                    r.outlet[0], r.outlet[1]};
    for (void *q : ptrs)
        if (q) (void)hipFreeAsync(q, p->stream);
    r.outlet[0] = r.outlet[1] = nullptr;
    r.snap = nullptr;
    r.rpart = nullptr;
    r.buf[0] = r.buf[1] = nullptr;
    r.mask = nullptr;
    r.params = nullptr;
    r.state_dev = nullptr;
    r.partials = nullptr;
}

int ensure_pool_staging(vplbm_pool p, size_t bytes)
{
    if (p->staging_bytes >= bytes) return VPLBM_OK;
    HIP_TRY(hipStreamSynchronize(p->stream));
    if (p->staging) HIP_TRY(hipFree(p->staging));
    p->staging = nullptr;
    p->staging_bytes = 0;
    if (hipMalloc(&p->staging, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(VPLBM_ENOMEM, "cannot allocate %zu bytes of staging memory", bytes);
    }
    p->staging_bytes = bytes;
    return VPLBM_OK;
}

long long steps_done(const vplbm_pool p, const PoolSim &d)
{
    const long long n = p->t_host - d.t0;
    return n < d.target ? n : d.target;
}

// Copy a finished (or failed) simulation's results to the host and release its slot and memory.
int retire(vplbm_pool p, int slot)
{
    Request &r = p->reqs[p->slot_req[slot]];
    PoolSim &d = p->h_sims[slot];
    const long long done = steps_done(p, d);
    r.done = done;
    r.residual = d.residual;
    memset(&r.obs, 0, sizeof r.obs);
    r.obs.step = done - 1;
    r.obs.nbodies = (int32_t)r.bodies.size();
    r.obs.status = (d.status & 1u) ? 1 : 0;
    const bool cancelled = r.cancel && done < d.target && !r.obs.status;
    if (done == d.target) {
        pool_fold_kernel<<<kRingWidth, kFoldBlock, 0, p->stream>>>(p->d_sims, slot);
        HIP_TRY(hipGetLastError());
        const char *dev_obs = reinterpret_cast<const char *>(p->d_sims + slot) + offsetof(PoolSim, obs);
        HIP_TRY(hipMemcpyAsync(d.obs, dev_obs, sizeof d.obs, hipMemcpyDeviceToHost, p->stream));
    }
    if (r.keep_fields) {
        const size_t n = (size_t)d.g.nx * d.g.ny;
        int rc = ensure_pool_staging(p, 3 * n * sizeof(double));
        if (rc) return rc;
        r.rho.resize(n);
        r.ux.resize(n);
        r.uy.resize(n);
        StepArgs a{};
        const int pb = pool_buf(done, d.spl, d.spk);
        a.src = d.buf[pb];                          // the state after `done` steps
        a.outlet.prev = d.conv ? d.outlet[pb] : nullptr;
        a.outlet.u = d.ou;
        a.mask = d.mask;
        a.bodies = d.bodies;
        a.t_base = p->d_zero;
        a.g = d.g;
        a.p = d.p;
        HIP_TRY(launch_readback(d.storage, a, p->staging, p->staging + n, p->staging + 2 * n, p->stream));
        HIP_TRY(hipMemcpyAsync(r.rho.data(), p->staging, n * sizeof(double), hipMemcpyDeviceToHost, p->stream));
        HIP_TRY(hipMemcpyAsync(r.ux.data(), p->staging + n, n * sizeof(double), hipMemcpyDeviceToHost, p->stream));
        HIP_TRY(hipMemcpyAsync(r.uy.data(), p->staging + 2 * n, n * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    }
    HIP_TRY(hipStreamSynchronize(p->stream));
    if (done == d.target) {
        r.obs.mass = d.obs[0];
        for (int k = 0; k < kMaxBodies; k++) {
            r.obs.fx[k] = d.obs[1 + 2 * k];
            r.obs.fy[k] = d.obs[2 + 2 * k];
        }
    }
    r.state = r.obs.status ? VPLBM_FAILED : (cancelled ? VPLBM_CANCELLED : VPLBM_DONE);
    host_log("pool %p: retire request %lld (%s) after %lld steps", (void *)p, (long long)r.id,
        r.state == VPLBM_DONE ? "done" : r.state == VPLBM_FAILED ? "failed" : "cancelled", done);
    free_request_memory(p, r);
    p->used -= r.bytes;
    p->resident_nodes -= (uint64_t)r.cfg.nx * r.cfg.ny;
    r.slot = -1;
    p->slot_req[slot] = -1;
    memset(&p->h_sims[slot], 0, sizeof(PoolSim));
    p->finished++;
    return VPLBM_OK;
}

// Allocate and initialise a queued request in a free slot.  Returns 1 if admitted, 0 if it does
// not fit the budget now, 2 if the device refused its memory, < 0 on error.
int admit(vplbm_pool p, Request &r, int slot)
{
    const uint64_t nodes = (uint64_t)r.cfg.nx * r.cfg.ny;
    const AdmissionState st{p->used, p->cfg.budget_bytes, p->resident_nodes, p->max_nodes, 1};
    if (!may_admit(st, r.bytes, nodes)) return 0;
    PoolSim d{};
    pool_geometry(r.cfg, d.g, d.ntx, d.ntiles);
    const int conv = r.cfg.bc_xhi == VPLBM_CONVECTIVE ? 1 : 0;
    const size_t pop = (size_t)9 * d.g.plane * elem_bytes(r.cfg.storage);
    struct { void **ptr; size_t n; } allocs[] = {
        {&r.buf[0], pop}, {&r.buf[1], pop}, {(void **)&r.mask, (size_t)d.g.pitch * d.g.ny},
        {(void **)&r.params, sizeof(BodyParams) * kMaxBodies},
        {(void **)&r.state_dev, sizeof(BodyState) * kMaxBodies},
        {(void **)&r.partials, (size_t)d.ntiles * kRingWidth * sizeof(double)},
        {(void **)&r.snap, r.tol > 0.0 ? 2 * (size_t)d.g.nx * d.g.ny * sizeof(double) : 0},
        {(void **)&r.rpart, r.tol > 0.0 ? (size_t)d.ntiles * 2 * sizeof(double) : 0},
        {&r.outlet[0], conv ? 3 * (size_t)d.g.ny * sizeof(double) : 0},
        {&r.outlet[1], conv ? 3 * (size_t)d.g.ny * sizeof(double) : 0},
    };
    for (auto &a : allocs) {
        if (a.n == 0) continue;
        if (hipMallocAsync(a.ptr, a.n, p->stream) != hipSuccess) {
            (void)hipGetLastError();
            free_request_memory(p, r);
            return 2;   // the device is fuller than the budget says
        }
    }
    BodyParams hp[kMaxBodies];
    memset(hp, 0, sizeof hp);
    const int nb = (int)r.bodies.size();
    for (int k = 0; k < nb; k++) {
        const vplbm_body &b = r.bodies[k];
        hp[k].kind = b.kind; hp[k].cx = b.cx; hp[k].cy = b.cy; hp[k].r = b.r; hp[k].hx = b.hx;
        hp[k].hy = b.hy; hp[k].ux = b.ux; hp[k].uy = b.uy; hp[k].omega = b.omega;
    }
    HIP_TRY(hipMemcpyAsync(r.params, hp, sizeof hp, hipMemcpyHostToDevice, p->stream));
    HIP_TRY(launch_bodies(r.params, r.state_dev, nb, p->d_zero, 0, p->stream));
    HIP_TRY(launch_mask(r.mask, d.g, r.params, r.state_dev, nb, 0, 0, d.g.nx, d.g.ny, p->stream));
    d.buf[0] = r.buf[0];
    d.buf[1] = r.buf[1];
    d.mask = r.mask;
    d.bodies = r.state_dev;
    d.partials = r.partials;
    d.p = node_params(r.cfg);
    d.storage = r.cfg.storage;
    d.conv = conv;
    d.ou = r.cfg.u_in_x;
    d.outlet[0] = r.outlet[0];
    d.outlet[1] = r.outlet[1];
    d.th = pool_tile_h(d.storage, conv);
    d.spk = pool_spk(d.storage, conv);
    d.active = 1;
    d.spl = p->cfg.steps_per_launch;
    d.t0 = p->t_host;
    d.target = r.nsteps;
    d.tol = r.tol;
    d.every = r.every;
    d.next_check = r.every;
    d.residual = INFINITY;
    d.snap = r.snap;
    d.rpart = r.rpart;
    StepArgs a{};
    a.dst = d.buf[0];
    a.mask = d.mask;
    a.bodies = d.bodies;
    a.g = d.g;
    a.p = d.p;
    HIP_TRY(launch_init(d.storage, a, nullptr, nullptr, nullptr, r.cfg.rho0, r.cfg.ux0, r.cfg.uy0, p->stream));
    if (conv) {   // the previous-step outlet values start as the initial state's last column
        a.src = d.buf[0];
        HIP_TRY(launch_outlet_init(d.storage, a, d.outlet[0], p->stream));
    }
    // the body table copy above reads `hp` from the stack: let it land before returning
    HIP_TRY(hipStreamSynchronize(p->stream));
    p->h_sims[slot] = d;
    r.slot = slot;
    r.state = VPLBM_RUNNING;
    p->used += r.bytes;
    p->resident_nodes += nodes;
    host_log("pool %p: admit request %lld (%dx%d, %lld steps) in slot %d, %llu bytes; resident %llu nodes",
        (void *)p, (long long)r.id, r.cfg.nx, r.cfg.ny, (long long)r.nsteps, slot,
        (unsigned long long)r.bytes, (unsigned long long)p->resident_nodes);
    return 1;
}

int ensure_pool_graph(vplbm_pool p)
{
    bool checks = false;
    int classes = 0;                      // bit c: a simulation of class c is resident
    for (const PoolSim &d : p->h_sims) {
        checks |= d.active && d.tol > 0.0;
        if (d.active) classes |= 1 << pool_class(d.storage, d.conv);
    }
    if (!classes) classes = 1;
    if (p->graph && p->grid_cap >= p->ntiles && p->grid_cap <= 8 * (p->ntiles > 4096 ? p->ntiles : 4096) &&
        p->graph_checks == checks && p->graph_classes == classes)
        return VPLBM_OK;
    if (p->graph) {
        HIP_TRY(hipGraphExecDestroy(p->graph));
        p->graph = nullptr;
    }
    int cap = 4096;
    while (cap < p->ntiles) cap *= 2;
    // every workgroup reads its table entry before it compares its index with the tile count
    if (cap > p->tile_cap) return fail(VPLBM_EHIP, "tile table (%d entries) shorter than the grid (%d)", p->tile_cap, cap);
    p->grid_cap = cap;
    host_log("pool %p: capture the step graph (%d workgroups per launch, %d steps, residual checks %d)",
        (void *)p, cap, p->cfg.steps_per_launch, (int)checks);
    if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    // Each class's launches from the replay's start: spk steps each (2, or 3 for binary32), what
    // remains last (pool_buf counts launches this way).  The classes advance the same steps.
    const int spl = p->cfg.steps_per_launch;
    for (int j = 0; j < spl && e == hipSuccess; j += 2) {
        const int nsteps = spl - j >= 2 ? 2 : 1;
        if (classes & 1) {
            pool_step_kernel<0><<<dim3(cap), dim3(kBlock2), 0, p->cap_stream>>>(p->d_sims, p->d_tiles, p->d_ntiles, p->d_t, j, nsteps);
            e = hipGetLastError();
        }
        if (e == hipSuccess && (classes & 2)) {
            pool_step_kernel<1><<<dim3(cap), dim3(kBlock2), 0, p->cap_stream>>>(p->d_sims, p->d_tiles, p->d_ntiles, p->d_t, j, nsteps);
            e = hipGetLastError();
        }
    }
    for (int j = 0; j < spl && e == hipSuccess && (classes & 4); j += 3) {
        const int nsteps = spl - j >= 3 ? 3 : spl - j;
        pool_step_kernel<2><<<dim3(cap), dim3(kBlock2), 0, p->cap_stream>>>(p->d_sims, p->d_tiles, p->d_ntiles, p->d_t, j, nsteps);
        e = hipGetLastError();
    }
    if (e == hipSuccess && checks) {
        const int n = p->cfg.steps_per_launch;
        pool_residual_kernel<<<dim3(cap), dim3(kBlock2), 0, p->cap_stream>>>(p->d_sims, p->d_tiles, p->d_ntiles, p->d_t, n);
        e = hipGetLastError();
        if (e == hipSuccess) {
            pool_residual_fold_kernel<<<dim3(p->cfg.max_slots), dim3(64), 0, p->cap_stream>>>(p->d_sims, p->d_t, n);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess) {
        pool_advance_kernel<<<1, 1, 0, p->cap_stream>>>(p->d_t, p->cfg.steps_per_launch);
        e = hipGetLastError();
    }
    p->graph_checks = checks;
    p->graph_classes = classes;
    hipError_t e2 = hipStreamEndCapture(p->cap_stream, &graph);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(VPLBM_EHIP, "pool graph capture failed: %s", hipGetErrorString(e));
    }
    HIP_TRY(e2);
    e = hipGraphInstantiate(&p->graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIP_TRY(e);
    return VPLBM_OK;
}

// Entry b of the device tile table: the tile that workgroup b of a launch over n tiles takes.
// Workgroups are dealt to the 8 XCDs round-robin; each XCD takes one contiguous range of the
// tiles (in simulation and tile order), so tiles that share cache lines through the x-shifted
// pulls stay in one L2.  The kernels then read entry blockIdx.x directly.
int xcd_entry(int b, int n)
{
    const int q = n >> 3, r = n & 7;
    const int xcd = b & 7, j = b >> 3;
    return xcd < r ? xcd * (q + 1) + j : r * (q + 1) + (xcd - r) * q + j;
}

int upload_tables(vplbm_pool p)
{
    std::vector<TileRef> tiles;
    uint64_t pop_bytes = 0;   // both population buffers of every resident simulation
    for (int s = 0; s < p->cfg.max_slots; s++) {
        const PoolSim &d = p->h_sims[s];
        if (!d.active) continue;
        for (int t = 0; t < d.ntiles; t++) tiles.push_back({s, t});
        pop_bytes += (uint64_t)2 * 9 * d.g.plane * elem_bytes(d.storage);
    }
    // Non-temporal stores once the resident populations exceed what the cache keeps (the rule of
    // a single simulation, applied to the whole pool: every launch reads them all again).
    for (int s = 0; s < p->cfg.max_slots; s++)
        if (p->h_sims[s].active) p->h_sims[s].nt = pop_bytes > ((uint64_t)192 << 20) ? 1 : 0;
    if ((int)tiles.size() > p->tile_cap) {
        HIP_TRY(hipStreamSynchronize(p->stream));
        if (p->d_tiles) HIP_TRY(hipFree(p->d_tiles));
        p->d_tiles = nullptr;
        int cap = p->tile_cap ? p->tile_cap : 4096;
        while (cap < (int)tiles.size()) cap *= 2;
        if (hipMalloc(&p->d_tiles, sizeof(TileRef) * cap) != hipSuccess) {
            (void)hipGetLastError();
            p->tile_cap = 0;
            return fail(VPLBM_ENOMEM, "cannot allocate the tile table");
        }
        p->tile_cap = cap;
        if (p->graph) {   // the graph holds the table pointer: capture again
            HIP_TRY(hipGraphExecDestroy(p->graph));
            p->graph = nullptr;
        }
    }
    const int n = (int)tiles.size();
    p->ntiles = n;
    std::vector<TileRef> order(n);
    for (int b = 0; b < n; b++) order[b] = tiles[xcd_entry(b, n)];
    if (n) HIP_TRY(hipMemcpyAsync(p->d_tiles, order.data(), sizeof(TileRef) * n, hipMemcpyHostToDevice, p->stream));
    HIP_TRY(hipMemcpyAsync(p->d_ntiles, &n, sizeof n, hipMemcpyHostToDevice, p->stream));
    HIP_TRY(hipMemcpyAsync(p->d_sims, p->h_sims.data(), sizeof(PoolSim) * p->cfg.max_slots, hipMemcpyHostToDevice, p->stream));
    // The host copies above read memory that changes on the next call: finish them.
    HIP_TRY(hipStreamSynchronize(p->stream));
    return VPLBM_OK;
}

}  // namespace

extern "C" {

int vplbm_pool_bytes_needed(const vplbm_config *cfg, uint64_t *bytes)
{
    int rc = check_config(cfg);
    if (rc) return rc;
    if (!bytes) return fail(VPLBM_EINVAL, "bytes is NULL");
    *bytes = bytes_needed(*cfg);
    return VPLBM_OK;
}

int vplbm_pool_create(const vplbm_pool_config *cfg, vplbm_pool *out)
{
    if (!out) return fail(VPLBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(VPLBM_EINVAL, "config is NULL");
    if (cfg->abi_version != VPLBM_ABI_VERSION) return fail(VPLBM_EINVAL, "abi_version %u, library is %d", cfg->abi_version, VPLBM_ABI_VERSION);
    if (cfg->max_slots < 1 || cfg->max_slots > kPoolMaxSlots) return fail(VPLBM_EINVAL, "max_slots must be in [1, %d]", kPoolMaxSlots);
    if (cfg->steps_per_launch < 1 || cfg->steps_per_launch > 4096) return fail(VPLBM_EINVAL, "steps_per_launch must be in [1, 4096]");
    if (cfg->budget_bytes == 0) return fail(VPLBM_EINVAL, "budget_bytes must be > 0");
    vplbm_pool p = new vplbm_pool_s();
    p->cfg = *cfg;
    if (cfg->stream) {
        p->stream = (hipStream_t)cfg->stream;
    } else {
        if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess) {
            delete p;
            return fail(VPLBM_EHIP, "cannot create a stream");
        }
        p->own_stream = true;
    }
    p->h_sims.assign(cfg->max_slots, PoolSim{});
    memset(p->h_sims.data(), 0, sizeof(PoolSim) * cfg->max_slots);
    p->slot_req.assign(cfg->max_slots, -1);
    hipError_t e = hipMalloc(&p->d_sims, sizeof(PoolSim) * cfg->max_slots);
    if (e == hipSuccess) e = hipMalloc(&p->d_ntiles, sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&p->d_zero, sizeof(long long));
    if (e == hipSuccess) e = hipMalloc(&p->d_t, sizeof(long long));
    if (e == hipSuccess) e = hipMemsetAsync(p->d_zero, 0, sizeof(long long), p->stream);
    if (e == hipSuccess) e = hipMemsetAsync(p->d_t, 0, sizeof(long long), p->stream);
    if (e == hipSuccess) e = hipMemsetAsync(p->d_ntiles, 0, sizeof(int), p->stream);
    if (e == hipSuccess) e = hipMemsetAsync(p->d_sims, 0, sizeof(PoolSim) * cfg->max_slots, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (p->d_sims) (void)hipFree(p->d_sims);
        if (p->d_ntiles) (void)hipFree(p->d_ntiles);
        if (p->d_zero) (void)hipFree(p->d_zero);
        if (p->d_t) (void)hipFree(p->d_t);
        if (p->own_stream) (void)hipStreamDestroy(p->stream);
        delete p;
        return fail(VPLBM_ENOMEM, "cannot allocate the pool tables: %s", hipGetErrorString(e));
    }
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        g_pools.insert(p);
    }
    *out = p;
    return VPLBM_OK;
}

int vplbm_pool_submit(vplbm_pool p, const vplbm_config *cfg, const vplbm_body *bodies,
                      int32_t nbodies, int64_t nsteps, int32_t keep_fields, int64_t *id)
{
    if (!pool_valid(p)) return fail(VPLBM_EINVAL, "invalid pool");
    if (!id) return fail(VPLBM_EINVAL, "id is NULL");
    int rc = check_config(cfg);
    if (rc) return rc;
    rc = check_bodies(bodies, nbodies);
    if (rc) return rc;
    for (int k = 0; k < nbodies; k++)
        if (bodies[k].freq != 0.0 && (bodies[k].ax != 0.0 || bodies[k].ay != 0.0))
            return fail(VPLBM_EINVAL, "pool simulations take static bodies only (body %d moves)", k);
    if (nsteps < 1) return fail(VPLBM_EINVAL, "nsteps must be >= 1");
    const uint64_t need = bytes_needed(*cfg);
    if (need > p->cfg.budget_bytes)
        return fail(VPLBM_EBUDGET, "simulation needs %llu bytes, pool budget is %llu", (unsigned long long)need, (unsigned long long)p->cfg.budget_bytes);
    Request r;
    r.id = p->next_id++;
    r.cfg = *cfg;
    r.bodies.assign(bodies, bodies + nbodies);
    r.nsteps = nsteps;
    r.keep_fields = keep_fields ? 1 : 0;
    r.bytes = need;
    p->reqs[r.id] = r;
    p->queue.push_back(r.id);
    *id = r.id;
    return VPLBM_OK;
}

int vplbm_pool_set_stop(vplbm_pool p, int64_t id, double tol, int64_t every)
{
    if (!pool_valid(p)) return fail(VPLBM_EINVAL, "invalid pool");
    auto it = p->reqs.find(id);
    if (it == p->reqs.end()) return fail(VPLBM_EINVAL, "unknown request %lld", (long long)id);
    Request &r = it->second;
    if (r.state != VPLBM_QUEUED) return fail(VPLBM_ESTATE, "request %lld is no longer queued", (long long)id);
    if (!(tol > 0.0) || !isfinite(tol)) return fail(VPLBM_EINVAL, "tol must be finite and > 0");
    if (every < 1) return fail(VPLBM_EINVAL, "every must be >= 1");
    const uint64_t need = bytes_needed(r.cfg, true);
    if (need > p->cfg.budget_bytes)
        return fail(VPLBM_EBUDGET, "simulation with a residual snapshot needs %llu bytes, pool budget is %llu",
                    (unsigned long long)need, (unsigned long long)p->cfg.budget_bytes);
    r.tol = tol;
    r.every = every;
    r.bytes = need;
    return VPLBM_OK;
}

int vplbm_pool_cancel(vplbm_pool p, int64_t id)
{
    if (!pool_valid(p)) return fail(VPLBM_EINVAL, "invalid pool");
    auto it = p->reqs.find(id);
    if (it == p->reqs.end()) return fail(VPLBM_EINVAL, "unknown request %lld", (long long)id);
    Request &r = it->second;
    if (r.state == VPLBM_QUEUED) {
        for (auto q = p->queue.begin(); q != p->queue.end(); ++q)
            if (*q == id) {
                p->queue.erase(q);
                break;
            }
        memset(&r.obs, 0, sizeof r.obs);
        r.obs.step = -1;
        r.obs.nbodies = (int32_t)r.bodies.size();
        r.done = 0;
        r.state = VPLBM_CANCELLED;
        r.keep_fields = 0;
        p->finished++;
        return VPLBM_OK;
    }
    if (r.state == VPLBM_RUNNING) {
        r.cancel = true;
        return VPLBM_OK;
    }
    return fail(VPLBM_ESTATE, "request %lld has already finished", (long long)id);
}

int vplbm_pool_set_admission(vplbm_pool p, uint64_t max_resident_nodes)
{
    if (!pool_valid(p)) return fail(VPLBM_EINVAL, "invalid pool");
    p->max_nodes = max_resident_nodes;
    return VPLBM_OK;
}

int vplbm_pool_residual(vplbm_pool p, int64_t id, double *residual)
{
    if (!pool_valid(p)) return fail(VPLBM_EINVAL, "invalid pool");
    if (!residual) return fail(VPLBM_EINVAL, "residual is NULL");
    auto it = p->reqs.find(id);
    if (it == p->reqs.end()) return fail(VPLBM_EINVAL, "unknown request %lld", (long long)id);
    const Request &r = it->second;
    *residual = r.state == VPLBM_RUNNING ? p->h_sims[r.slot].residual : r.residual;
    return VPLBM_OK;
}

int vplbm_pool_advance(vplbm_pool p, int32_t *running, int32_t *queued, int32_t *finished_total)
{
    if (!pool_valid(p)) return fail(VPLBM_EINVAL, "invalid pool");
    if (p->in_flight) {
        HIP_TRY(hipStreamSynchronize(p->stream));
        p->in_flight = false;
        p->t_host += p->cfg.steps_per_launch;
        HIP_TRY(hipMemcpy(p->h_sims.data(), p->d_sims, sizeof(PoolSim) * p->cfg.max_slots, hipMemcpyDeviceToHost));
    }
    bool changed = false;
    for (int s = 0; s < p->cfg.max_slots; s++) {
        PoolSim &d = p->h_sims[s];
        if (!d.active) continue;
        const long long done = steps_done(p, d);
        p->reqs[p->slot_req[s]].done = done;
        if (done >= d.target || (d.status & 1u) || p->reqs[p->slot_req[s]].cancel) {
            int rc = retire(p, s);
            if (rc) return rc;
            changed = true;
        }
    }
    // First come, first served: the head of the queue waits for room rather than being passed.
    while (!p->queue.empty()) {
        int slot = -1;
        for (int s = 0; s < p->cfg.max_slots; s++)
            if (p->slot_req[s] < 0) { slot = s; break; }
        if (slot < 0) break;
        Request &r = p->reqs[p->queue.front()];
        int rc = admit(p, r, slot);
        if (rc < 0) return rc;
        if (rc == 2) {
            // The device refused the memory.  With simulations resident, retirements will free
            // some: wait.  With none, nothing ever will: the request fails instead of blocking
            // the queue for good.
            bool resident = false;
            for (int s = 0; s < p->cfg.max_slots; s++) resident |= p->h_sims[s].active != 0;
            if (!fail_when_refused(resident)) break;
            memset(&r.obs, 0, sizeof r.obs);
            r.obs.step = -1;
            r.obs.nbodies = (int32_t)r.bodies.size();
            r.obs.status = 2;
            r.done = 0;
            r.state = VPLBM_FAILED;
            r.keep_fields = 0;
            p->finished++;
            host_log("pool %p: request %lld failed: the device refused %llu bytes with nothing resident",
                (void *)p, (long long)r.id, (unsigned long long)r.bytes);
            p->queue.pop_front();
            changed = true;
            continue;
        }
        if (rc == 0) break;
        p->slot_req[slot] = r.id;
        p->queue.pop_front();
        changed = true;
    }
    int nrun = 0;
    for (int s = 0; s < p->cfg.max_slots; s++) nrun += p->h_sims[s].active ? 1 : 0;
    if (changed) {
        int rc = upload_tables(p);
        if (rc) return rc;
    }
    if (nrun > 0) {
        int rc = ensure_pool_graph(p);
        if (rc) return rc;
        HIP_TRY(hipGraphLaunch(p->graph, p->stream));
        p->in_flight = true;
    }
    if (running) *running = nrun;
    if (queued) *queued = (int32_t)p->queue.size();
    if (finished_total) *finished_total = p->finished;
    return VPLBM_OK;
}

int vplbm_pool_status(vplbm_pool p, int64_t id, int32_t *state, int64_t *steps_done)
{
    if (!pool_valid(p)) return fail(VPLBM_EINVAL, "invalid pool");
    auto it = p->reqs.find(id);
    if (it == p->reqs.end()) return fail(VPLBM_EINVAL, "unknown request %lld", (long long)id);
    if (state) *state = it->second.state;
    if (steps_done) *steps_done = it->second.done;
    return VPLBM_OK;
}

int vplbm_pool_result(vplbm_pool p, int64_t id, vplbm_obs *out, double *rho, double *ux, double *uy)
{
    if (!pool_valid(p)) return fail(VPLBM_EINVAL, "invalid pool");
    auto it = p->reqs.find(id);
    if (it == p->reqs.end()) return fail(VPLBM_EINVAL, "unknown request %lld", (long long)id);
    Request &r = it->second;
    if (r.state != VPLBM_DONE && r.state != VPLBM_FAILED && r.state != VPLBM_CANCELLED)
        return fail(VPLBM_ESTATE, "request %lld has not finished", (long long)id);
    if ((rho || ux || uy) && !r.keep_fields) return fail(VPLBM_EINVAL, "request %lld did not keep its fields", (long long)id);
    if (out) *out = r.obs;
    const size_t n = r.rho.size();
    if (rho) memcpy(rho, r.rho.data(), n * sizeof(double));
    if (ux) memcpy(ux, r.ux.data(), n * sizeof(double));
    if (uy) memcpy(uy, r.uy.data(), n * sizeof(double));
    p->reqs.erase(it);
    return VPLBM_OK;
}

int vplbm_pool_destroy(vplbm_pool p)
{
    if (!p) return VPLBM_OK;
    if (!pool_valid(p)) return fail(VPLBM_EINVAL, "invalid pool");
    (void)hipStreamSynchronize(p->stream);
    for (auto &kv : p->reqs) free_request_memory(p, kv.second);
    (void)hipStreamSynchronize(p->stream);
    if (p->graph) (void)hipGraphExecDestroy(p->graph);
    void *ptrs[] = {p->d_sims, p->d_tiles, p->d_ntiles, p->d_zero, p->d_t, p->staging};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->own_stream) (void)hipStreamDestroy(p->stream);
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        g_pools.erase(p);
    }
    delete p;
    return VPLBM_OK;
}

}  // extern "C"
