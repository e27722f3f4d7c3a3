// Per-node device code of the VP-LBM step (arXiv:1812.05401, Section 2) for gfx950.
//
// One node = pull 9 populations (left side of Eqs. 2/10), apply the edge rules, take the moments
// (Eqs. 8-9), solve the penalized velocity and force (Eqs. 17-18), collide, store 9 populations.
//
// Collision.  Eq. 14 relaxes every even non-conserved moment (e, eps, p_xx, p_xy) with s_n and
// both odd non-conserved moments (q_x, q_y) with s_q; the conserved moments come out the same for
// any of their rates because the Lu term adds exactly the force to the momentum.  So the MRT of
// Eqs. 10-16 is a two-relaxation-time collision: the symmetric half (f_a + f_abar)/2 of every
// opposite pair relaxes with s+ = s_n, the antisymmetric half with s- = s_q, and the forcing term
// splits as (1 - s+/2) F+ + (1 - s-/2) F-.  The SRT of Eqs. 2 and 7 is the case s+ = s- = 1/tau,
// as the paper states for equal rates.  This form needs no 9x9 products.
//
// Shifted arithmetic.  Every kernel works on h_a = f_a - w_a, the deviation from the rest state
// (rho = 1, u = 0), never on f itself: rho = 1 + sum h, j = sum xi h (sum xi w = 0), and the
// collision, forcing, edge rules and Zou-He inlet are affine in f with w-preserving maps, so they
// carry over to h with the equilibrium h^eq = w (drho + rho (3c + 4.5c^2 - 1.5u^2)).  In FP32 the
// h are about 1e3 times smaller than f, and so are their rounding errors; rounding f ~ w every
// step (which a uniform region repeats with the same sign) is what drifts the mass of long FP32
// runs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vplbm {

enum Storage { kF64 = 0, kF32 = 1, kF16S = 2, kBF16S = 3, kF32D = 4, kF16SR = 5, kBF16SR = 6 };

// ---- storage codecs --------------------------------------------------------------------------
// load/store move h = f - w_a in the compute type `real`; encode/decode move f in FP64 (host
// checkpoints, the momentum exchange).  F64 keeps f itself.  F32, F32D, F16S and BF16S keep h, so
// the stored numbers are the small deviations from rest and the format's relative precision
// applies to them rather than to f.  A decode/encode round trip gives back the stored bits: h + w
// in FP64 is off by at most half an FP64 ulp of w (2^-57), below half an ulp of any h that binary16
// or bfloat16 can hold and of any binary32 h above about 2^-33.  F32D computes in
// FP64: with only the storage rounded to binary32, long runs keep FP64's mass and forces, and the
// FP64 arithmetic costs this memory-bound step about a tenth of its time.
// store_nt: the same value with a non-temporal store, for grids whose buffers do not fit in the
// Infinity Cache (the next step's reads come from HBM anyway, so the writes need not be cached).
template <int S> struct Codec;

// Element i of a population plane, addressed as the plane's base (uniform over the wave, held in
// scalar registers) plus a 32-bit byte offset: the form of a global load or store with a scalar
// base, which needs no 64-bit address arithmetic per lane.  Planes stay below 2^31 elements
// (create rejects larger lattices), so the offset fits.
template <typename E> __device__ __forceinline__ const E *at(const E *plane, unsigned i)
{
    return reinterpret_cast<const E *>(reinterpret_cast<const char *>(plane) + i * (unsigned)sizeof(E));
}
template <typename E> __device__ __forceinline__ E *at(E *plane, unsigned i)
{
    return reinterpret_cast<E *>(reinterpret_cast<char *>(plane) + i * (unsigned)sizeof(E));
}

template <> struct Codec<kF64> {
    using elem = double;
    using real = double;
    static constexpr bool stochastic = false;
    static __device__ __forceinline__ real load(const elem *p, unsigned i, real w) { return *at(p, i) - w; }
    static __device__ __forceinline__ void store(elem *p, unsigned i, real h, real w) { *at(p, i) = h + w; }
    static __device__ __forceinline__ void store_nt(elem *p, unsigned i, real h, real w) { __builtin_nontemporal_store(h + w, at(p, i)); }
    static __device__ __forceinline__ double decode(const elem *p, unsigned i, double) { return *at(p, i); }
    static __device__ __forceinline__ void encode(elem *p, unsigned i, double f, double) { *at(p, i) = f; }
};

// binary32 h with FP32 (F32) or FP64 (F32D) arithmetic.
template <typename R> struct CodecF32 {
    using elem = float;
    using real = R;
    static constexpr bool stochastic = false;
    static __device__ __forceinline__ real load(const elem *p, unsigned i, real) { return *at(p, i); }
    static __device__ __forceinline__ void store(elem *p, unsigned i, real h, real) { *at(p, i) = float(h); }
    static __device__ __forceinline__ void store_nt(elem *p, unsigned i, real h, real) { __builtin_nontemporal_store(float(h), at(p, i)); }
    static __device__ __forceinline__ double decode(const elem *p, unsigned i, double w) { return double(*at(p, i)) + w; }
    static __device__ __forceinline__ void encode(elem *p, unsigned i, double f, double w) { *at(p, i) = float(f - w); }
};
template <> struct Codec<kF32> : CodecF32<float> {};
template <> struct Codec<kF32D> : CodecF32<double> {};

template <> struct Codec<kF16S> {
    using elem = _Float16;
    using real = float;
    static constexpr bool stochastic = false;
    static __device__ __forceinline__ real load(const elem *p, unsigned i, real) { return (float)*at(p, i); }
    static __device__ __forceinline__ void store(elem *p, unsigned i, real h, real) { *at(p, i) = (_Float16)h; }
    static __device__ __forceinline__ void store_nt(elem *p, unsigned i, real h, real)
    {
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, (_Float16)h),
                                    reinterpret_cast<unsigned short *>(at(p, i)));
    }
    static __device__ __forceinline__ double decode(const elem *p, unsigned i, double w) { return double(*at(p, i)) + w; }
    static __device__ __forceinline__ void encode(elem *p, unsigned i, double f, double w) { *at(p, i) = (_Float16)(f - w); }
};

template <> struct Codec<kBF16S> {
    using elem = __bf16;
    using real = float;
    static constexpr bool stochastic = false;
    static __device__ __forceinline__ real load(const elem *p, unsigned i, real) { return (float)*at(p, i); }
    static __device__ __forceinline__ void store(elem *p, unsigned i, real h, real) { *at(p, i) = (__bf16)h; }
    static __device__ __forceinline__ void store_nt(elem *p, unsigned i, real h, real)
    {
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, (__bf16)h),
                                    reinterpret_cast<unsigned short *>(at(p, i)));
    }
    static __device__ __forceinline__ double decode(const elem *p, unsigned i, double w) { return double(*at(p, i)) + w; }
    static __device__ __forceinline__ void encode(elem *p, unsigned i, double f, double w) { *at(p, i) = (__bf16)(float)(f - w); }
};

// ---- stochastic rounding ---------------------------------------------------------------------
// F16SR / BF16SR store h like F16S / BF16S but round it up or down at random, with probability
// proportional to the distance to each neighbour, so the rounding error has zero mean.  Rounding
// to nearest repeats the same error at every node of a uniform region, step after step, which
// drifts the mass of long 16-bit runs; random rounding turns that drift into a random walk.
// The random bits come from a counter-based hash of (node, step): the 32-bit finalizer of
// MurmurHash3 (Appleby), then Marsaglia's xorshift32 for each further word.  Runs are
// reproducible; the bits need to be unbiased, not of cryptographic quality.
__device__ __forceinline__ unsigned mix32(unsigned h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

__device__ __forceinline__ unsigned xorshift32(unsigned x)
{
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}

// binary16 with stochastic rounding; r holds 13 random bits (bits 0..12).  Below 2^-14 the
// binary16 quantum is 2^-24: scale, add a uniform fraction, take the floor, scale back (all exact).
// Above, add the random bits under the 10 kept mantissa bits of the binary32 pattern and drop them
// (a carry moves into the exponent as it should); the result is exact in binary16.
__device__ __forceinline__ bool f16_sr_tiny(float v) { return __builtin_fabsf(v) < 6.103515625e-05f; }

__device__ __forceinline__ _Float16 f16_sr_below(float v, unsigned r)   // |v| < 2^-14
{
    const float n = __builtin_floorf(v * 16777216.0f + float(r & 0x1FFFu) * 1.220703125e-04f);
    return (_Float16)(n * 5.9604644775390625e-08f);
}

__device__ __forceinline__ _Float16 f16_sr_above(float v, unsigned r)   // |v| >= 2^-14
{
    return (_Float16)__uint_as_float((__float_as_uint(v) + (r & 0x1FFFu)) & ~0x1FFFu);
}

__device__ __forceinline__ _Float16 f16_stochastic(float v, unsigned r)
{
    return f16_sr_tiny(v) ? f16_sr_below(v, r) : f16_sr_above(v, r);
}

// bfloat16 (the top 16 bits of binary32) with stochastic rounding; r holds 16 random bits.
__device__ __forceinline__ unsigned short bf16_stochastic_bits(float v, unsigned r)
{
    return (unsigned short)((__float_as_uint(v) + (r & 0xFFFFu)) >> 16);
}

template <> struct Codec<kF16SR> : Codec<kF16S> {
    static constexpr bool stochastic = true;
    static __device__ __forceinline__ void store_raw(elem *p, unsigned i, _Float16 q) { *at(p, i) = q; }
    static __device__ __forceinline__ void store_raw_nt(elem *p, unsigned i, _Float16 q)
    {
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, q), reinterpret_cast<unsigned short *>(at(p, i)));
    }
    static __device__ __forceinline__ void store_sr(elem *p, unsigned i, real h, unsigned r) { *at(p, i) = f16_stochastic(h, r); }
    static __device__ __forceinline__ void store_sr_nt(elem *p, unsigned i, real h, unsigned r)
    {
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, f16_stochastic(h, r)),
                                    reinterpret_cast<unsigned short *>(at(p, i)));
    }
};

template <> struct Codec<kBF16SR> : Codec<kBF16S> {
    static constexpr bool stochastic = true;
    static __device__ __forceinline__ void store_sr(elem *p, unsigned i, real h, unsigned r)
    {
        *reinterpret_cast<unsigned short *>(at(p, i)) = bf16_stochastic_bits(h, r);
    }
    static __device__ __forceinline__ void store_sr_nt(elem *p, unsigned i, real h, unsigned r)
    {
        __builtin_nontemporal_store(bf16_stochastic_bits(h, r), reinterpret_cast<unsigned short *>(at(p, i)));
    }
};

// Lattice weights of Eq. 5 in the compute type.
template <typename T> struct W {
    static constexpr T rest = T(4.0 / 9.0);
    static constexpr T axis = T(1.0 / 9.0);
    static constexpr T diag = T(1.0 / 36.0);
};

template <typename T> __device__ __forceinline__ T weight(int a)
{
    return a == 0 ? W<T>::rest : (a <= 4 ? W<T>::axis : W<T>::diag);
}

// ---- geometry and edges ------------------------------------------------------------------------

struct Geom {
    int nx, ny, pitch;      // pitch: elements per row (>= nx, multiple of 64)
    int plane;              // elements per population plane
    int xper, yper;         // periodic x / y
    int inlet;              // Zou-He velocity inlet on x = 0 (then x = nx-1 is an outlet)
};

// Convective outlet on x = nx-1: the populations entering from x = nx (3, 6, 7) obey
// df/dt + U df/dx = 0, implicitly upwind: f(nx-1, t+1) = (f(nx-1, t) + U f(nx-2, t+1)) / (1 + U).
// The rule is affine with weights summing to one, so it holds for h as well.  prev holds
// h(nx-1, t) as [3][ny] in the compute type; the step writes next (the other parity).
struct Outlet {
    const void *prev;       // nullptr: zero-gradient outlet (or no outlet)
    void *next;             // nullptr: do not record (observation kernels)
    double u;               // convection speed
};

// Source of direction a at edge node (x, y) under the edge rules: a row outside the lattice
// wraps (periodic) or is replaced by the specular image in the same row (free-slip: the
// population arriving in a left with the y-mirrored direction); a column outside wraps
// (periodic) or is clamped to the edge column (outlet; at the inlet it is a placeholder that
// the inlet rule overwrites).  Mirroring keeps |xi|, so the lattice weight is unchanged.
__device__ __forceinline__ int edge_source(int a, int x, int y, const Geom &g, int &plane_dir)
{
    constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    constexpr int mirror_y[9] = {0, 1, 4, 3, 2, 8, 7, 6, 5};
    int sx = x - cx[a], sy = y - cy[a];
    plane_dir = a;
    if (sy < 0 || sy >= g.ny) {
        if (g.yper) sy += sy < 0 ? g.ny : -g.ny;
        else { sy = y; plane_dir = mirror_y[a]; }
    }
    if (sx < 0 || sx >= g.nx) {
        if (g.xper) sx += sx < 0 ? g.nx : -g.nx;
        else sx = sx < 0 ? 0 : g.nx - 1;
    }
    return sy * g.pitch + sx;
}

// Pull of a node with all eight neighbours inside the lattice (0 < x < nx-1, 0 < y < ny-1): nine
// plain shifts.  Every index below is >= pitch - 1 >= 0 there.
template <int S>
__device__ __forceinline__ void pull_interior(const typename Codec<S>::elem *__restrict__ src, int x,
                                              int y, const Geom &g, typename Codec<S>::real f[9])
{
    using C = Codec<S>;
    using T = typename C::real;
    const unsigned P = g.pitch;
    const unsigned i = y * P + x;
    f[0] = C::load(src, i, W<T>::rest);
    f[1] = C::load(src + 1 * g.plane, i - 1, W<T>::axis);
    f[2] = C::load(src + 2 * g.plane, i - P, W<T>::axis);
    f[3] = C::load(src + 3 * g.plane, i + 1, W<T>::axis);
    f[4] = C::load(src + 4 * g.plane, i + P, W<T>::axis);
    f[5] = C::load(src + 5 * g.plane, i - P - 1, W<T>::diag);
    f[6] = C::load(src + 6 * g.plane, i - P + 1, W<T>::diag);
    f[7] = C::load(src + 7 * g.plane, i + P + 1, W<T>::diag);
    f[8] = C::load(src + 8 * g.plane, i + P - 1, W<T>::diag);
}

// Pull the nine shifted populations h of node (x, y) from the post-collision planes `src`.
template <int S>
__device__ __forceinline__ void pull(const typename Codec<S>::elem *__restrict__ src, int x, int y,
                                     const Geom &g, const Outlet &o, typename Codec<S>::real f[9])
{
    using C = Codec<S>;
    using T = typename C::real;
    const bool interior = (x > 0) & (x < g.nx - 1) & (y > 0) & (y < g.ny - 1);
    if (interior) {
        pull_interior<S>(src, x, y, g, f);
    } else {
#pragma unroll
        for (int a = 0; a < 9; a++) {
            int pa;
            int j = edge_source(a, x, y, g, pa);
            f[a] = C::load(src + pa * g.plane, j, weight<T>(a));
        }
        if (o.prev && x == g.nx - 1) {
            constexpr int dirs[3] = {3, 6, 7};
            const T *prev = static_cast<const T *>(o.prev);
            const T u = T(o.u);
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const int a = dirs[k];
                int pa;
                const int j = edge_source(a, g.nx - 2, y, g, pa);
                const T nb = C::load(src + pa * g.plane, j, weight<T>(a));
                f[a] = (prev[k * g.ny + y] + u * nb) / (T(1) + u);
            }
            if (o.next) {
                T *next = static_cast<T *>(o.next);
#pragma unroll
                for (int k = 0; k < 3; k++) next[k * g.ny + y] = f[dirs[k]];
            }
        }
    }
}

// Element of a workgroup's LDS tile (see pull_tile) that direction a of node (x, y) pulls from,
// and its plane in pa: edge_source without the periodic wrap, which the tile's halo holds.  The
// tile starts H nodes before the workgroup's first node (x0, y0) in both directions; (x, y) are
// unwrapped coordinates (a halo node across a periodic edge lies outside the lattice).
template <int H = 1>
__device__ __forceinline__ unsigned tile_source(int a, int x, int y, int x0, int y0, int ew,
                                                const Geom &g, int &pa)
{
    constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    constexpr int mirror_y[9] = {0, 1, 4, 3, 2, 8, 7, 6, 5};
    int sx = x - cx[a], sy = y - cy[a];
    pa = a;
    if ((sy < 0 || sy >= g.ny) && !g.yper) { sy = y; pa = mirror_y[a]; }
    if ((sx < 0 || sx >= g.nx) && !g.xper) sx = sx < 0 ? 0 : g.nx - 1;
    return unsigned((sy - y0 + H) * ew + (sx - x0 + H));
}

// Pull the nine shifted populations h of node (x, y) from a workgroup's tile in LDS instead of the
// planes in global memory.  The tile holds the post-collision populations of the nodes
// [x0 - H, x0 + ew - H - 1] x [y0 - H, ...] in unwrapped coordinates, ew per row, `plane` elements
// per population: a periodic neighbour across an edge sits in the tile's halo, so for the tile
// only the free-slip and clamped edges of edge_source remain.  Every node the pull reads lies
// within one node of (x, y), inside the tile.
// The tile pull of a node whose nine sources are plain shifts (no free-slip or clamped edge next to
// it): every index below is >= 0, the tile having a halo.
template <int S, int H = 1>
__device__ __forceinline__ void pull_tile_shifts(const typename Codec<S>::elem *tile, unsigned plane,
                                                 int ew, int x, int y, int x0, int y0,
                                                 typename Codec<S>::real f[9])
{
    using C = Codec<S>;
    using T = typename C::real;
    const unsigned e = unsigned((y - y0 + H) * ew + (x - x0 + H));
    const unsigned E = unsigned(ew);
    f[0] = C::load(tile, e, W<T>::rest);
    f[1] = C::load(tile + 1 * plane, e - 1, W<T>::axis);
    f[2] = C::load(tile + 2 * plane, e - E, W<T>::axis);
    f[3] = C::load(tile + 3 * plane, e + 1, W<T>::axis);
    f[4] = C::load(tile + 4 * plane, e + E, W<T>::axis);
    f[5] = C::load(tile + 5 * plane, e - E - 1, W<T>::diag);
    f[6] = C::load(tile + 6 * plane, e - E + 1, W<T>::diag);
    f[7] = C::load(tile + 7 * plane, e + E + 1, W<T>::diag);
    f[8] = C::load(tile + 8 * plane, e + E - 1, W<T>::diag);
}

template <int S, int H = 1>
__device__ __forceinline__ void pull_tile(const typename Codec<S>::elem *tile, unsigned plane, int ew,
                                          int x, int y, int x0, int y0, const Geom &g,
                                          typename Codec<S>::real f[9])
{
    using C = Codec<S>;
    using T = typename C::real;
    const bool shifts = (g.xper | ((x > 0) & (x < g.nx - 1))) & (g.yper | ((y > 0) & (y < g.ny - 1)));
    if (shifts) {
        pull_tile_shifts<S, H>(tile, plane, ew, x, y, x0, y0, f);
    } else {
#pragma unroll
        for (int a = 0; a < 9; a++) {
            int pa;
            const unsigned j = tile_source<H>(a, x, y, x0, y0, ew, g, pa);
            f[a] = C::load(tile + pa * plane, j, weight<T>(a));
        }
    }
}

// Zou-He velocity inlet on the west edge: the populations entering from x < 0 (1, 5, 8) are set
// so that sum f = rho and sum xi f = rho (ux, uy), with rho from the known populations and the
// non-equilibrium parts bounced back.  On h: the known weights w0 + w2 + w4 + 2 (w3 + w6 + w7)
// sum to 1, so rho - 1 = (H + ux) / (1 - ux) with H the same combination of h, and the unknowns
// are set by the same formulas since opposite directions share a weight.
template <typename T>
__device__ __forceinline__ void zou_he_west(T h[9], T ux, T uy)
{
    T drho = (h[0] + h[2] + h[4] + T(2) * (h[3] + h[6] + h[7]) + ux) / (T(1) - ux);
    T rho = T(1) + drho;
    T half_t = T(0.5) * (h[2] - h[4]);
    T ru6 = rho * ux * T(1.0 / 6.0);
    h[1] = h[3] + T(2.0 / 3.0) * rho * ux;
    h[5] = h[7] - half_t + ru6 + T(0.5) * rho * uy;
    h[8] = h[6] + half_t + ru6 - T(0.5) * rho * uy;
}

// ---- moments and penalization ------------------------------------------------------------------

template <typename T> struct Macro {
    T drho, rho, ux, uy;   // density deviation rho - 1, density and penalized velocity (Eq. 18)
    T fx, fy;              // penalization force (Eq. 17)
};

// Eqs. 8-9 and 17-18 with dt = 1, from the shifted populations.  In a solid node (chi = 1) the
// velocity and force are taken in the algebraically equal forms u = u_s + (j/rho - u_s) k and
// f = -(j - rho u_s) c with k = 1/(1 + 1/(2 eta)) and c = 1/(eta + 1/2): the literal forms
// subtract nearly equal numbers (u - u_s is ~eta) and lose about -log10(eta) digits.
// 1/x: FP64 divides; FP32 takes the hardware reciprocal (1 ulp) and one Newton step, three
// instructions in place of the ten of a correctly rounded division (within an ulp of it).
template <typename T> __device__ __forceinline__ T reciprocal(T x) { return T(1) / x; }
template <> __device__ __forceinline__ float reciprocal<float>(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return __builtin_fmaf(__builtin_fmaf(-x, r, 1.0f), r, r);
}

template <typename T>
__device__ __forceinline__ Macro<T> moments(const T h[9], bool solid, T usx, T usy, T k_relax, T c_pen)
{
    Macro<T> m;
    T drho = (h[0] + (h[1] + h[3])) + ((h[2] + h[4]) + ((h[5] + h[7]) + (h[6] + h[8])));
    T jx = (h[1] - h[3]) + ((h[5] - h[7]) + (h[8] - h[6]));
    T jy = (h[2] - h[4]) + ((h[5] - h[7]) + (h[6] - h[8]));
    T rho = T(1) + drho;
    T inv_rho = reciprocal(rho);
    m.drho = drho;
    m.rho = rho;
    if (solid) {
        m.ux = usx + (jx * inv_rho - usx) * k_relax;
        m.uy = usy + (jy * inv_rho - usy) * k_relax;
        m.fx = -(jx - rho * usx) * c_pen;
        m.fy = -(jy - rho * usy) * c_pen;
    } else {
        m.ux = jx * inv_rho;
        m.uy = jy * inv_rho;
        m.fx = T(0);
        m.fy = T(0);
    }
    return m;
}

// ---- collision -----------------------------------------------------------------------------------

// a * b + c, rounded once.  A sum of two products is written with its fused product explicit: left
// to the compiler's contraction, either product may be fused, and the choice can differ between
// kernels that inline the same code, which would break their bitwise agreement.
template <typename T> __device__ __forceinline__ T fmadd(T a, T b, T c);
template <> __device__ __forceinline__ float fmadd<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double fmadd<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One opposite pair (a, abar) of shifted populations with lattice weight w, c = xi_a . u and
// xf = xi_a . f; q = -1.5 |u|^2.  FORCED = false drops the forcing terms, which vanish at fluid
// nodes (f = 0 there): the same result, without their arithmetic.
template <bool FORCED, typename T>
__device__ __forceinline__ void collide_pair(T &ha, T &hb, T c, T xf, T w, T drho, T rho, T q,
                                             T ufp, T sp, T sm, T kp, T km)
{
    T heq_s = w * (drho + rho * (q + T(4.5) * c * c));   // symmetric part of Eq. 4, minus w
    T heq_a = w * rho * (T(3) * c);                      // antisymmetric part of Eq. 4
    T hs = T(0.5) * (ha + hb);
    T hd = T(0.5) * (ha - hb);
    T ns = hs - sp * (hs - heq_s);
    T na = hd - sm * (hd - heq_a);
    if (FORCED) {
        T frc_s = w * (T(9) * c * xf - T(3) * ufp);      // symmetric part of Eq. 16
        T frc_a = w * (T(3) * xf);                       // antisymmetric part of Eq. 16
        ns += kp * frc_s;
        na += km * frc_a;
    }
    ha = ns + na;
    hb = ns - na;
}

// Two-rate collision with the split forcing term: sp/sm are the even/odd rates, kp = 1 - sp/2,
// km = 1 - sm/2.  In place on the shifted populations h.
template <bool FORCED, typename T>
__device__ __forceinline__ void collide(T h[9], const Macro<T> &m, T sp, T sm, T kp, T km)
{
    const T ux = m.ux, uy = m.uy, rho = m.rho, drho = m.drho;
    const T q = T(-1.5) * fmadd(ux, ux, uy * uy);
    const T ufp = FORCED ? fmadd(ux, m.fx, uy * m.fy) : T(0);
    {
        T heq0 = W<T>::rest * (drho + rho * q);
        h[0] = h[0] - sp * (h[0] - heq0);
        if (FORCED) h[0] += kp * (W<T>::rest * (T(-3) * ufp));
    }
    collide_pair<FORCED>(h[1], h[3], ux, m.fx, W<T>::axis, drho, rho, q, ufp, sp, sm, kp, km);
    collide_pair<FORCED>(h[2], h[4], uy, m.fy, W<T>::axis, drho, rho, q, ufp, sp, sm, kp, km);
    collide_pair<FORCED>(h[5], h[7], ux + uy, m.fx + m.fy, W<T>::diag, drho, rho, q, ufp, sp, sm, kp, km);
    collide_pair<FORCED>(h[6], h[8], uy - ux, m.fy - m.fx, W<T>::diag, drho, rho, q, ufp, sp, sm, kp, km);
}

// Equilibrium of Eq. 4 minus the weights (used to initialise); drho = rho - 1.
template <typename T>
__device__ __forceinline__ void equilibrium(T drho, T ux, T uy, T h[9])
{
    const T rho = T(1) + drho;
    const T q = T(-1.5) * (ux * ux + uy * uy);
    const T c[9] = {T(0), ux, uy, -ux, -uy, ux + uy, uy - ux, -ux - uy, ux - uy};
#pragma unroll
    for (int a = 0; a < 9; a++)
        h[a] = weight<T>(a) * (drho + rho * (q + T(3) * c[a] + T(4.5) * c[a] * c[a]));
}

// ---- obstacles ------------------------------------------------------------------------------------

// Per-body state at the current time, written by the body kernel: centre, translation velocity
// and angular velocity.
struct BodyState {
    double cx, cy, vx, vy, omega;
};

// Rigid-body solid velocity u_s = V + omega e_z x (x - c) at node (x, y).
template <typename T>
__device__ __forceinline__ void solid_velocity(const BodyState &b, int x, int y, T &usx, T &usy)
{
    usx = T(b.vx) - T(b.omega) * (T(y) - T(b.cy));
    usy = T(b.vy) + T(b.omega) * (T(x) - T(b.cx));
}

// ---- one lattice update ------------------------------------------------------------------------

// Relaxation, penalization and inlet parameters of one simulation (FP64; each kernel converts
// them to its compute type the same way).
struct NodeParams {
    double sp, sm, kp, km;   // even/odd relaxation rates and 1 - s/2
    double k_relax, c_pen;   // 1/(1 + 1/(2 eta)) and 1/(eta + 1/2)
    double uin_x, uin_y;     // inlet velocity
};

// Inlet rule, mask, body velocity, Eqs. 8-9 and 17-18, and the collision at node (x, y), in place
// on the pulled populations f.  Returns the moments and sets id to the node's body id.
template <typename T>
__device__ __forceinline__ Macro<T> relax_node(T f[9], const uint8_t *__restrict__ mask,
                                               const BodyState *__restrict__ bodies, const Geom &g,
                                               const NodeParams &p, int x, int y, int &id)
{
    if (g.inlet && x == 0) zou_he_west(f, T(p.uin_x), T(p.uin_y));
    id = *at(mask, unsigned(y * g.pitch + x));
    T usx = T(0), usy = T(0);
    if (id) solid_velocity(bodies[id - 1], x, y, usx, usy);
    const Macro<T> m = moments(f, id != 0, usx, usy, T(p.k_relax), T(p.c_pen));
    if (id) collide<true>(f, m, T(p.sp), T(p.sm), T(p.kp), T(p.km));   // penalized: forced
    else collide<false>(f, m, T(p.sp), T(p.sm), T(p.kp), T(p.km));     // fluid: no force
    return m;
}

// relax_node with the body id already loaded by the caller (the mask value at (x, y)).  The same
// statements, kept separate so that each form inlines and schedules as measured.
template <typename T>
__device__ __forceinline__ Macro<T> relax_node_id(T f[9], int id, const BodyState *__restrict__ bodies,
                                                  const Geom &g, const NodeParams &p, int x, int y)
{
    if (g.inlet && x == 0) zou_he_west(f, T(p.uin_x), T(p.uin_y));
    T usx = T(0), usy = T(0);
    if (id) solid_velocity(bodies[id - 1], x, y, usx, usy);
    const Macro<T> m = moments(f, id != 0, usx, usy, T(p.k_relax), T(p.c_pen));
    if (id) collide<true>(f, m, T(p.sp), T(p.sm), T(p.kp), T(p.km));
    else collide<false>(f, m, T(p.sp), T(p.sm), T(p.kp), T(p.km));
    return m;
}

// Whether a kernel loads a node's mask byte before its populations (MF) or after them.  Both give
// the same result; the order changes only how the loads overlap, and the better one was measured
// per kernel, format and lattice size:
//  * one step per launch: mask first for the 2-byte formats (4-7% faster); after the populations
//    for FP32, F32D and FP64 (mask first is up to 4% slower for FP32 and 11% for F32D);
//  * two steps per launch: mask first (2-12% faster), except for FP32 on lattices that stream from
//    HBM, where it is 5% slower.  Those are the lattices that take non-temporal stores (NT), so
//    NT selects the order for FP32.
template <int S, bool NT> constexpr bool mask_first_one_step() { return sizeof(typename Codec<S>::elem) == 2; }
template <int S, bool NT> constexpr bool mask_first_two_step() { return !(S == kF32 && NT); }

// Store the nine post-collision populations of the node with lattice index `node` (row * pitch +
// column) at element i of the planes dst, plane elements apart (the population planes in global
// memory, or a workgroup's tile in LDS).  The stochastic formats draw their bits from (node, step),
// so a value rounds the same wherever it is stored.
template <int S, bool NT = false>
__device__ __forceinline__ void store_node(typename Codec<S>::elem *__restrict__ dst, unsigned plane,
                                           unsigned i, const typename Codec<S>::real f[9],
                                           unsigned node, unsigned step)
{
    using C = Codec<S>;
    using T = typename C::real;
    if constexpr (S == kF16SR) {
        // As below, with the values under 2^-14 (rare: solid nodes at rest) redone in a
        // wave-uniform branch that only waves holding such a value take.  Selected per lane, their
        // exact-quantum rounding cost every stored value its instructions.  Same results.
        const unsigned r0 = mix32(node ^ mix32(step * 0x9e3779b9u + 0x7f4a7c15u));
        unsigned r = r0;
        _Float16 q[9];
        bool tiny = false;
#pragma unroll
        for (int k = 0; k < 9; k++) {
            if (k % 2 == 0 && k > 0) r = xorshift32(r);
            q[k] = f16_sr_above(f[k], (k % 2) ? (r >> 16) : r);
            tiny |= f16_sr_tiny(f[k]);
        }
        if (__any(tiny)) {
            r = r0;
#pragma unroll
            for (int k = 0; k < 9; k++) {
                if (k % 2 == 0 && k > 0) r = xorshift32(r);
                if (f16_sr_tiny(f[k])) q[k] = f16_sr_below(f[k], (k % 2) ? (r >> 16) : r);
            }
        }
#pragma unroll
        for (int k = 0; k < 9; k++) {
            if (NT) C::store_raw_nt(dst + k * plane, i, q[k]);
            else C::store_raw(dst + k * plane, i, q[k]);
        }
    } else if constexpr (C::stochastic) {
        // one hash per node and step, then two 16-bit words per xorshift state
        unsigned r = mix32(node ^ mix32(step * 0x9e3779b9u + 0x7f4a7c15u));
#pragma unroll
        for (int k = 0; k < 9; k++) {
            if (k % 2 == 0 && k > 0) r = xorshift32(r);
            const unsigned bits = (k % 2) ? (r >> 16) : r;
            if (NT) C::store_sr_nt(dst + k * plane, i, f[k], bits);
            else C::store_sr(dst + k * plane, i, f[k], bits);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 9; k++) {
            if (NT) C::store_nt(dst + k * plane, i, f[k], weight<T>(k));
            else C::store(dst + k * plane, i, f[k], weight<T>(k));
        }
    }
}

// A buffer resource over `bytes` bytes from p (raw, unformatted dwords): buffer stores through it
// take the per-lane byte offset in a vector register and a wave-uniform offset (a plane's start)
// in a scalar one, so they need no 64-bit address arithmetic per lane.  Accesses beyond `bytes`
// are dropped by the hardware.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_over(void *p, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(p, 0, int(bytes), 0x00020000);   // data format: 32 bit
}

// pull_interior for 4-byte storage through a buffer resource over the planes (buffer_over): every
// load takes the node's byte offset 4 i in the same vector register, and the plane's start plus
// the direction's shift, (a plane + shift) * 4, in a scalar one, so the nine loads need no vector
// address arithmetic.  Same values as pull_interior.
template <int S>
__device__ __forceinline__ void pull_interior_buf(__amdgpu_buffer_rsrc_t r, unsigned plane, unsigned pitch,
                                                  unsigned i, typename Codec<S>::real f[9])
{
    static_assert(sizeof(typename Codec<S>::elem) == 4, "binary32 storage");
    using T = typename Codec<S>::real;
    const int v = int(i * 4u);
    const int P = int(pitch);
    const int shift[9] = {0, -1, -P, 1, P, -P - 1, -P + 1, P + 1, P - 1};
#pragma unroll
    for (int a = 0; a < 9; a++)
        f[a] = T(__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                   r, v, int((unsigned(a) * plane + unsigned(shift[a])) * 4u), 0)));
}

// store_node for 4-byte storage without stochastic rounding through a buffer resource over the
// planes (buffer_over): plane k of node i at byte (k plane + i) * 4, the same values and rounding.
template <int S, bool NT>
__device__ __forceinline__ void store_node_buf(__amdgpu_buffer_rsrc_t r, unsigned plane, unsigned i,
                                               const typename Codec<S>::real f[9])
{
    static_assert(sizeof(typename Codec<S>::elem) == 4 && !Codec<S>::stochastic, "binary32 storage");
#pragma unroll
    for (int k = 0; k < 9; k++)
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(float(f[k])), r, int(i * 4u),
                                              int(unsigned(k) * plane * 4u), NT ? 2 : 0);   // 2: nt
}

// The whole step at node (x, y): pull, edges, moments and penalization, collision, store.
// Returns the moments (density, penalization force) for the reductions and the body id.
// MF: load the mask byte before the populations (see mask_first_one_step).
template <int S, bool NT = false, bool MF = false>
__device__ __forceinline__ Macro<typename Codec<S>::real>
update_node(const typename Codec<S>::elem *__restrict__ src, typename Codec<S>::elem *__restrict__ dst,
            const uint8_t *__restrict__ mask, const BodyState *__restrict__ bodies, const Geom &g,
            const Outlet &o, const NodeParams &p, int x, int y, int &id, unsigned step)
{
    using T = typename Codec<S>::real;
    T f[9];                  // shifted populations h = f - w
    if constexpr (MF) {
        const unsigned i = y * g.pitch + x;
        id = *at(mask, i);
        pull<S>(src, x, y, g, o, f);
        const Macro<T> m = relax_node_id(f, id, bodies, g, p, x, y);
        store_node<S, NT>(dst, g.plane, i, f, i, step);
        return m;
    } else {
        pull<S>(src, x, y, g, o, f);
        const Macro<T> m = relax_node(f, mask, bodies, g, p, x, y, id);
        const unsigned i = y * g.pitch + x;
        store_node<S, NT>(dst, g.plane, i, f, i, step);
        return m;
    }
}

// The moments the next step would take at node (x, y) of the state `src`, without storing
// anything: pull, edges (the convective outlet is read, not recorded), body velocity, Eqs. 8-9 and
// 17-18.  Density is 1 + drho and velocity (ux, uy) in the compute type; id is the body id.
template <int S>
__device__ __forceinline__ Macro<typename Codec<S>::real>
observe_node(const typename Codec<S>::elem *__restrict__ src, const uint8_t *__restrict__ mask,
             const BodyState *__restrict__ bodies, const Geom &g, const Outlet &o,
             const NodeParams &p, int x, int y, int &id)
{
    using T = typename Codec<S>::real;
    T f[9];
    const Outlet ro{o.prev, nullptr, o.u};
    pull<S>(src, x, y, g, ro, f);
    if (g.inlet && x == 0) zou_he_west(f, T(p.uin_x), T(p.uin_y));
    id = mask[y * g.pitch + x];
    T usx = T(0), usy = T(0);
    if (id) solid_velocity(bodies[id - 1], x, y, usx, usy);
    return moments(f, id != 0, usx, usy, T(p.k_relax), T(p.c_pen));
}

// ---- wave reductions ------------------------------------------------------------------------------

// v from another lane of the same row of 16, by a DPP lane pattern (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_double(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp(int(b), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(int(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double lane_double(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(int(b), lane);
    const int hi = __builtin_amdgcn_readlane(int(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum of v over the 64 lanes of a wave (every lane active), the same value in every lane, in a
// fixed order.  DPP = true: within each row of 16 lanes, four DPP exchanges add lane pairs, then
// quads, then half-rows (lane i with i ^ 1, with i ^ 2, with the mirrored lane of the other quad,
// with the mirrored lane of the other half-row; FP addition commutes, so both partners hold the
// same sum after each step), and the four row sums, read from lanes 0, 16, 32 and 48, are added.
// No LDS round trips: 2-3% faster FP32-arithmetic step kernels.  DPP = false: a butterfly of lane
// shuffles, kept for the FP64-arithmetic kernels, whose schedule the DPP form made slower (the
// F32D one-step kernel by 20% at 8192 x 2048, measured).
template <bool DPP = true>
__device__ __forceinline__ double wave_sum(double v)
{
    if constexpr (DPP) {
        v += dpp_double<0xB1>(v);    // quad_perm [1, 0, 3, 2]
        v += dpp_double<0x4E>(v);    // quad_perm [2, 3, 0, 1]
        v += dpp_double<0x141>(v);   // row_half_mirror
        v += dpp_double<0x140>(v);   // row_mirror
        return (lane_double(v, 0) + lane_double(v, 16)) + (lane_double(v, 32) + lane_double(v, 48));
    } else {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        return v;
    }
}

// The wave sum a kernel computing in T uses.
template <typename T> constexpr bool wave_sum_dpp() { return sizeof(T) == 4; }

// Body forces of one row of nodes: only waves holding solid nodes do any work, one pass per
// body id present in the wave; lane 0 adds the wave's sums into the wave's own LDS partials.
template <bool DPP>
__device__ __forceinline__ void wave_forces(double *wave_acc, double fx, double fy, int id)
{
    unsigned long long solid = __ballot(id != 0);
    while (solid) {
        const int lead = __ffsll((unsigned long long)solid) - 1;
        const int k = __shfl(id, lead, 64);
        const bool mine = id == k;
        const double sx = wave_sum<DPP>(mine ? -fx : 0.0);
        const double sy = wave_sum<DPP>(mine ? -fy : 0.0);
        if ((threadIdx.x & 63) == 0) {
            wave_acc[1 + 2 * (k - 1)] += sx;
            wave_acc[2 + 2 * (k - 1)] += sy;
        }
        solid &= ~__ballot(mine);
    }
}

// Map a hardware workgroup id to a logical tile so that each XCD (workgroups are dealt to the 8
// XCDs round-robin) works on one contiguous range of tiles, keeping x-neighbouring tiles, which
// share cache lines through the x-shifted pulls, in the same L2.
__device__ __forceinline__ int xcd_tile(int wg, int nwg)
{
    const int q = nwg >> 3, r = nwg & 7;
    const int xcd = wg & 7, j = wg >> 3;
    return xcd < r ? xcd * (q + 1) + j : r * (q + 1) + (xcd - r) * q + j;
}

}  // namespace vplbm
