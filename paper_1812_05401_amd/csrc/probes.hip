// Measurement probes (libvplbm_probes.so): the step kernels' memory access patterns with a trivial
// per-node update, a 16-byte copy and FP32 FMA chains.  They advance no simulation; they give the
// ceilings the step kernels of libvplbm.so are measured against.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "lattice.hpp"
#include "vplbm_probes.h"

namespace {

using vplbm::at;
using vplbm::xcd_tile;

constexpr int kCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

struct Lat {
    int nx, ny, pitch;
    unsigned plane;       // elements per plane
};

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// The trivial update: every value and the mask byte are used, nothing else is computed.
__device__ __forceinline__ void touch(float f[9], int m)
{
#pragma unroll
    for (int a = 0; a < 9; a++) f[a] = f[a] * 0.5f + float(m) * 1e-3f;
}

__device__ __forceinline__ void pull_global(const float *src, const Lat &L, int x, int y, float f[9])
{
#pragma unroll
    for (int a = 0; a < 9; a++)
        f[a] = *at(src + a * L.plane, unsigned(wrap(y - kCy[a], L.ny) * L.pitch + wrap(x - kCx[a], L.nx)));
}

// One step per launch: 128 x 2 nodes per workgroup of 256 threads, one node per thread.
__global__ __launch_bounds__(256) void pull1_probe(const float *src, float *dst, const uint8_t *mask, Lat L)
{
    const int ntx = L.nx / 128;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int x = (tile % ntx) * 128 + (threadIdx.x & 127);
    const int y = (tile / ntx) * 2 + (threadIdx.x >> 7);
    float f[9];
    pull_global(src, L, x, y, f);
    const unsigned i = unsigned(y * L.pitch + x);
    touch(f, *at(mask, i));
#pragma unroll
    for (int a = 0; a < 9; a++) __builtin_nontemporal_store(f[a], at(dst + a * L.plane, i));
}

// STEPS (2 or 3) updates per launch on a TW x TH tile with 512 threads.  The first phase covers the
// tile and a halo of STEPS - 1 nodes (EW x EH nodes) from global memory into LDS; a middle phase
// (STEPS = 3) covers the tile and a one-node halo in place, reading every pulled value into
// registers before the barrier that precedes the writes; the last phase pulls the tile from LDS
// and stores it.
template <int TW, int TH, int STEPS>
__global__ __launch_bounds__(512) void tile_probe(const float *src, float *dst, const uint8_t *mask, Lat L)
{
    constexpr int H = STEPS - 1;
    constexpr int EW = TW + 2 * H, EH = TH + 2 * H, EN = EW * EH;
    __shared__ float mid[9 * EN];
    const int ntx = L.nx / TW;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int x0 = (tile % ntx) * TW, y0 = (tile / ntx) * TH;
    for (int e = threadIdx.x; e < EN; e += 512) {
        const int x = wrap(x0 + e % EW - H, L.nx), y = wrap(y0 + e / EW - H, L.ny);
        float f[9];
        pull_global(src, L, x, y, f);
        touch(f, *at(mask, unsigned(y * L.pitch + x)));
#pragma unroll
        for (int a = 0; a < 9; a++) mid[a * EN + e] = f[a];
    }
    __syncthreads();
    if constexpr (STEPS == 3) {
        constexpr int MW = TW + 2, MN = MW * (TH + 2), R = (MN + 511) / 512;
        float g[R][9];
        int m[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int j = threadIdx.x + r * 512;
            m[r] = 0;
            if (j < MN) {
                const int lx = j % MW, ly = j / MW;          // tile coordinates + 1
                const int s = (ly + 1) * EW + lx + 1;        // its slot (halo H = 2)
#pragma unroll
                for (int a = 0; a < 9; a++) g[r][a] = mid[a * EN + s - kCy[a] * EW - kCx[a]];
                const int x = wrap(x0 + lx - 1, L.nx), y = wrap(y0 + ly - 1, L.ny);
                m[r] = *at(mask, unsigned(y * L.pitch + x));
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int j = threadIdx.x + r * 512;
            if (j < MN) {
                const int s = (j / MW + 1) * EW + j % MW + 1;
                touch(g[r], m[r]);
#pragma unroll
                for (int a = 0; a < 9; a++) mid[a * EN + s] = g[r][a];
            }
        }
        __syncthreads();
    }
    for (int j = threadIdx.x; j < TW * TH; j += 512) {
        const int lx = j % TW, ly = j / TW;
        const int s = (ly + H) * EW + lx + H;
        float f[9];
#pragma unroll
        for (int a = 0; a < 9; a++) f[a] = mid[a * EN + s - kCy[a] * EW - kCx[a]];
        const unsigned i = unsigned((y0 + ly) * L.pitch + x0 + lx);
        touch(f, *at(mask, i));
#pragma unroll
        for (int a = 0; a < 9; a++) __builtin_nontemporal_store(f[a], at(dst + a * L.plane, i));
    }
}

// Four 16-byte elements per thread, 256 apart, so that every load of a wave is one contiguous 1 KiB.
__global__ __launch_bounds__(256) void copy_probe(const float4 *src, float4 *dst, size_t n)
{
    const size_t base = blockIdx.x * (size_t)1024 + threadIdx.x;
    float4 v[4];
#pragma unroll
    for (int k = 0; k < 4; k++)
        if (base + k * 256 < n) v[k] = src[base + k * 256];
#pragma unroll
    for (int k = 0; k < 4; k++)
        if (base + k * 256 < n) dst[base + k * 256] = v[k];
}

__global__ __launch_bounds__(256) void fma_probe(float *out, int reps, float b, float c)
{
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; k++) v[k] = float(threadIdx.x + k);
    for (int r = 0; r < reps; r++) {
#pragma unroll 16
        for (int i = 0; i < 1024; i++) {
#pragma unroll
            for (int k = 0; k < 8; k++) v[k] = __builtin_fmaf(v[k], b, c);
        }
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; k++) s += v[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Device memory freed on every path out of a probe.
struct Buffers {
    void *p[3] = {nullptr, nullptr, nullptr};
    hipStream_t st = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    ~Buffers()
    {
        for (void *q : p)
            if (q) (void)hipFree(q);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (st) (void)hipStreamDestroy(st);
    }
    int setup()
    {
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)
            return fail(-3, "cannot create a stream or events");
        return 0;
    }
    int alloc(int k, size_t bytes)
    {
        if (hipMalloc(&p[k], bytes) != hipSuccess) {
            p[k] = nullptr;
            (void)hipGetLastError();
            return fail(-2, "device allocation of " + std::to_string(bytes) + " bytes failed");
        }
        return 0;
    }
    // Mean milliseconds of `n` calls of launch(i) after `warm` untimed ones.
    template <typename F> int time(F launch, int warm, int n, double *ms)
    {
        for (int i = 0; i < warm; i++) launch(i);
        if (hipEventRecord(ev[0], st) != hipSuccess) return fail(-3, "event record failed");
        for (int i = 0; i < n; i++) launch(warm + i);
        if (hipEventRecord(ev[1], st) != hipSuccess) return fail(-3, "event record failed");
        hipError_t e = hipEventSynchronize(ev[1]);
        if (e == hipSuccess) e = hipGetLastError();
        if (e != hipSuccess) return fail(-3, std::string("probe launch failed: ") + hipGetErrorString(e));
        float t = 0.f;
        if (hipEventElapsedTime(&t, ev[0], ev[1]) != hipSuccess) return fail(-3, "event timing failed");
        *ms = double(t) / n;
        return 0;
    }
};

template <int TW, int TH, int STEPS>
void launch_tile(const float *s, float *d, const uint8_t *m, const Lat &L, hipStream_t st)
{
    tile_probe<TW, TH, STEPS><<<(L.nx / TW) * (L.ny / TH), 512, 0, st>>>(s, d, m, L);
}

}  // namespace

extern "C" {

const char *vplbm_probe_last_error(void) { return g_err.c_str(); }

int vplbm_probe_pattern(int32_t nx, int32_t ny, int32_t steps_per_launch, int32_t tile_w,
                        int32_t tile_h, int32_t launches, double *us_per_launch)
{
    if (!us_per_launch) return fail(-1, "us_per_launch is NULL");
    if (nx < 8 || ny < 8) return fail(-1, "nx and ny must be at least 8");
    if (launches < 1 || launches > 100000) return fail(-1, "launches must be in [1, 100000]");
    using Launch = void (*)(const float *, float *, const uint8_t *, const Lat &, hipStream_t);
    Launch fn = nullptr;
    int tw = 128, th = 2;
    if (steps_per_launch == 1) {
        fn = [](const float *s, float *d, const uint8_t *m, const Lat &L, hipStream_t st) {
            pull1_probe<<<(L.nx / 128) * (L.ny / 2), 256, 0, st>>>(s, d, m, L);
        };
    } else {
        tw = tile_w;
        th = tile_h;
        const int k = steps_per_launch * 100000 + tile_w * 100 + tile_h;
        switch (k) {
        case 212808: fn = launch_tile<128, 8, 2>; break;
        case 206408: fn = launch_tile<64, 8, 2>; break;
        case 212816: fn = launch_tile<128, 16, 2>; break;
        case 312808: fn = launch_tile<128, 8, 3>; break;
        case 312806: fn = launch_tile<128, 6, 3>; break;
        case 306408: fn = launch_tile<64, 8, 3>; break;
        case 306414: fn = launch_tile<64, 14, 3>; break;
        default:
            return fail(-1, "no probe for " + std::to_string(steps_per_launch) + " steps per launch on " +
                                std::to_string(tile_w) + " x " + std::to_string(tile_h) + " tiles");
        }
    }
    if (nx % tw || ny % th)
        return fail(-1, "nx must be a multiple of " + std::to_string(tw) + " and ny of " + std::to_string(th));
    Lat L;
    L.nx = nx;
    L.ny = ny;
    L.pitch = (nx + 63) / 64 * 64;
    const size_t plane = (size_t)L.pitch * ny;
    if (plane * 9 >= ((size_t)1 << 31)) return fail(-1, "lattice too large for 32-bit plane offsets");
    L.plane = (unsigned)plane;
    Buffers b;
    int rc;
    if ((rc = b.setup()) || (rc = b.alloc(0, plane * 9 * sizeof(float))) ||
        (rc = b.alloc(1, plane * 9 * sizeof(float))) || (rc = b.alloc(2, plane)))
        return rc;
    if (hipMemsetAsync(b.p[0], 0, plane * 9 * sizeof(float), b.st) != hipSuccess ||
        hipMemsetAsync(b.p[1], 0, plane * 9 * sizeof(float), b.st) != hipSuccess ||
        hipMemsetAsync(b.p[2], 1, plane, b.st) != hipSuccess)
        return fail(-3, "memset failed");
    float *buf[2] = {static_cast<float *>(b.p[0]), static_cast<float *>(b.p[1])};
    const uint8_t *mask = static_cast<const uint8_t *>(b.p[2]);
    double ms = 0.0;
    rc = b.time([&](int i) { fn(buf[i & 1], buf[(i & 1) ^ 1], mask, L, b.st); }, launches / 8 + 1, launches, &ms);
    if (rc) return rc;
    *us_per_launch = ms * 1e3;
    return 0;
}

int vplbm_probe_copy(uint64_t bytes, int32_t reps, double *gbs)
{
    if (!gbs) return fail(-1, "gbs is NULL");
    if (bytes < (1u << 20) || bytes % 16) return fail(-1, "bytes must be a multiple of 16 and at least 1 MiB");
    if (reps < 1 || reps > 10000) return fail(-1, "reps must be in [1, 10000]");
    Buffers b;
    int rc;
    if ((rc = b.setup()) || (rc = b.alloc(0, bytes)) || (rc = b.alloc(1, bytes))) return rc;
    if (hipMemsetAsync(b.p[0], 0, bytes, b.st) != hipSuccess) return fail(-3, "memset failed");
    const size_t n = bytes / 16;
    const float4 *s = static_cast<const float4 *>(b.p[0]);
    float4 *d = static_cast<float4 *>(b.p[1]);
    double ms = 0.0;
    const unsigned blocks = unsigned((n + 1023) / 1024);
    rc = b.time([&](int) { copy_probe<<<blocks, 256, 0, b.st>>>(s, d, n); }, 1, reps, &ms);
    if (rc) return rc;
    *gbs = 2.0 * double(bytes) / (ms * 1e-3) / 1e9;
    return 0;
}

int vplbm_probe_fma(int32_t reps, double *lane_fma_per_s)
{
    if (!lane_fma_per_s) return fail(-1, "lane_fma_per_s is NULL");
    if (reps < 1 || reps > 1000) return fail(-1, "reps must be in [1, 1000]");
    constexpr int blocks = 2048, threads = 256;
    Buffers b;
    int rc;
    if ((rc = b.setup()) || (rc = b.alloc(0, sizeof(float) * blocks * threads))) return rc;
    float *out = static_cast<float *>(b.p[0]);
    double ms = 0.0;
    rc = b.time([&](int) { fma_probe<<<blocks, threads, 0, b.st>>>(out, reps, 0.999f, 1e-3f); }, 1, 3, &ms);
    if (rc) return rc;
    *lane_fma_per_s = double(blocks) * threads * reps * 1024.0 * 8.0 / (ms * 1e-3);
    return 0;
}

}  // extern "C"
