// HIP kernels of the VP-LBM library for gfx950 (MI355X).
//
// The step is one fused, memory-bound pass: per node 9 pulled population loads, a 1-byte mask
// load, the moments / penalization / collision in registers, 9 coalesced stores, and the FP64
// per-step reductions (wave64 shuffles, one LDS hop, FP64 atomics into sub-slots that the next
// step folds into a device ring).  Nothing here is a dense contraction, so there is no MFMA; the
// roofline is HBM bandwidth.
#include <stdlib.h>

#include "kernels.hpp"

namespace vplbm {

// ---- the fused step --------------------------------------------------------------------------

// Sum value q of the sub-slots [kSub][kRingWidth] of step t into ring entry t, with one wave:
// lane l adds sub-slots l, l + 64, ... in order, then a fixed butterfly adds the lanes, so the
// result does not depend on which workgroup folds or when.  One memory round trip, not kSub.
__device__ __forceinline__ void fold_value(const StepArgs &a, long long t, int q, bool clear)
{
    double *acc = a.acc + (size_t)(t & 1) * kSub * kRingWidth;
    const int lane = threadIdx.x & 63;
    double v = 0.0;
    for (int b = lane; b < kSub; b += 64) v += acc[b * kRingWidth + q];
    v = wave_sum(v);
    if (lane == 0) a.ring[(size_t)(t % a.ring_len) * kRingWidth + q] = v;
    if (clear)
        for (int b = lane; b < kSub; b += 64) acc[b * kRingWidth + q] = 0.0;
}

// Body forces of one row of nodes: only waves holding solid nodes do any work, one pass per
// body id present in the wave; lane 0 adds the wave's sums into the wave's own LDS partials.
__device__ __forceinline__ void wave_forces(double *wave_acc, double fx, double fy, int id)
{
    unsigned long long solid = __ballot(id != 0);
    while (solid) {
        const int lead = __ffsll((unsigned long long)solid) - 1;
        const int k = __shfl(id, lead, 64);
        const bool mine = id == k;
        const double sx = wave_sum(mine ? -fx : 0.0);
        const double sy = wave_sum(mine ? -fy : 0.0);
        if ((threadIdx.x & 63) == 0) {
            wave_acc[1 + 2 * (k - 1)] += sx;
            wave_acc[2 + 2 * (k - 1)] += sy;
        }
        solid &= ~__ballot(mine);
    }
}

template <int S, bool NT>
__global__ __launch_bounds__(kBlock) void step_kernel(StepArgs a)
{
    using C = Codec<S>;
    using T = typename C::real;
    using E = typename C::elem;
    // Per-wave partial sums: each wave writes only its own row (LDS accesses of one wave are in
    // order), so the workgroup needs a single barrier, before the rows are added.
    __shared__ double wave_acc[kBlock / 64][kRingWidth];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long t = *a.t_base + a.t_off;
    if (a.reduce) {
        if (lane < kRingWidth) wave_acc[wave][lane] = 0.0;
        // The previous step's partials are complete (kernel boundary): fold and clear them.
        // Workgroup q's first wave folds value q (all of them if the grid is smaller).
        if (t >= 1 && wave == 0)
            for (int q = blockIdx.x; q < kRingWidth; q += gridDim.x) fold_value(a, t - 1, q, true);
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
            const Macro<T> m = update_node<S, NT>(src, dst, a.mask, a.bodies, a.g, a.outlet, a.p, x, y, id,
                                                  (unsigned)t);
            const double rho_d = 1.0 + double(m.drho);
            mass += rho_d;
            fx_d = double(m.fx);
            fy_d = double(m.fy);
            bad |= !(rho_d > 0.0 && rho_d < 1e30);   // also catches NaN
        }
        if (a.reduce) wave_forces(wave_acc[wave], fx_d, fy_d, id);
    }
    if (a.reduce) {
        const double mw = wave_sum(mass);
        if (lane == 0) wave_acc[wave][0] = mw;
        if (__ballot(bad) && lane == 0) atomicOr(a.status, 1u);
        __syncthreads();
        if (threadIdx.x < kRingWidth) {
            double v = 0.0;
            for (int w = 0; w < kBlock / 64; w++) v += wave_acc[w][threadIdx.x];   // fixed order
            double *slot = a.acc + ((size_t)(t & 1) * kSub + (blockIdx.x & (kSub - 1))) * kRingWidth;
            if (v != 0.0) unsafeAtomicAdd(slot + threadIdx.x, v);
        }
    }
}

__global__ void fold_kernel(StepArgs a)
{
    const long long t = *a.t_base;
    if (t >= 1)
        for (int q = 0; q < kRingWidth; q++) fold_value(a, t - 1, q, false);
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
    using T = typename C::real;
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
    using T = typename C::real;
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

__global__ void bodies_kernel(const BodyParams *p, BodyState *s, int nb, const long long *t_base,
                              int t_off)
{
#pragma clang fp contract(off)
    const int k = threadIdx.x;
    if (k >= nb) return;
    const double t = double(*t_base + t_off);
    const double two_pi = 6.283185307179586;
    const BodyParams b = p[k];
    const double ph = two_pi * b.freq * t;
    const double sn = sin(ph), cs = cos(ph);
    BodyState o;
    o.cx = b.cx + b.ax * sn;
    o.cy = b.cy + b.ay * sn;
    o.vx = b.ux + b.ax * two_pi * b.freq * cs;
    o.vy = b.uy + b.ay * two_pi * b.freq * cs;
    o.omega = b.omega;
    s[k] = o;
}

// Node-centre inclusion in FP64 without contraction, so that the decision for a node is the
// correctly rounded one: the lowest-index body containing the node owns it.
__global__ __launch_bounds__(kBlock) void mask_kernel(uint8_t *mask, Geom g, const BodyParams *p,
                                                      const BodyState *s, int nb, int x0, int y0,
                                                      int w, int h)
{
#pragma clang fp contract(off)
    const int node = blockIdx.x * kBlock + threadIdx.x;
    if (node >= w * h) return;
    const int x = x0 + node % w, y = y0 + node / w;
    if (x < 0 || x >= g.nx || y < 0 || y >= g.ny) return;
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
    mask[y * g.pitch + x] = (uint8_t)id;
}

hipError_t launch_bodies(const BodyParams *params, BodyState *state, int nbodies,
                         const long long *t_base, int t_off, hipStream_t st)
{
    bodies_kernel<<<1, 64, 0, st>>>(params, state, nbodies, t_base, t_off);
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
