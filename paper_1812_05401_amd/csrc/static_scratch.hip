// The library's one entry point that allocates nothing: the momentum exchange of the paper's
// Section 3.3 written to caller-supplied device memory, asynchronously, with its partial sums in
// a file-scope device array instead of memory the library allocates.  For callers that cannot
// call hipMalloc (code under HIP graph capture, tight serving loops).
//
// The array (`scratch`) holds one row of partial sums per workgroup of the partial-sum kernel.
// Each GPU the library runs on has its own copy, at its own address, for the life of the
// process; host code reaches it only through the address hipGetSymbolAddress returns for the
// current device (the array's name is a host-side stand-in, not a device address).  Every call
// on a GPU shares that GPU's copy: calls that overlap on one GPU race.
#include <mutex>

#include "internal.hpp"
#include "kernels.hpp"
#include "static_scratch.hpp"

namespace vplbm {

// One row of kRingWidth doubles per workgroup (entries 1 .. 16: fx, fy of the 8 bodies).
__device__ __align__(256) double scratch[kScratchParts * kRingWidth];

namespace {
std::mutex g_scratch_mu;
double *g_scratch_ptr[kScratchDevices] = {nullptr};
}  // namespace

int static_scratch_init()
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices) return fail(VPLBM_EINVAL, "device %d beyond the library's %d", dev, kScratchDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return VPLBM_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return fail(VPLBM_EHIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev, hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = static_cast<double *>(p);
    return VPLBM_OK;
}

double *static_scratch(int dev)
{
    if (dev < 0 || dev >= kScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}

// Link momentum of the current state, per workgroup of kBlock nodes (one node per thread): for a
// fluid node x_f and a solid node x_s = x_f + xi_a of body k, xi_a (g_a(x_f) + g_abar(x_s)), added
// per body in a fixed order (direction by direction, the wave's lanes by a fixed butterfly, the
// waves in order) into row blockIdx.x of part.  Every row is written, so nothing needs clearing.
template <int S>
__global__ __launch_bounds__(kBlock) void exchange_parts_kernel(StepArgs a, double *part)
{
    using C = Codec<S>;
    using E = typename C::elem;
    constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    __shared__ double rows[kBlock / 64][kRingWidth];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < kRingWidth) rows[wave][lane] = 0.0;
    const Geom &g = a.g;
    const int node = blockIdx.x * kBlock + threadIdx.x;
    const bool in = node < g.nx * g.ny;
    const int x = in ? node % g.nx : 0, y = in ? node / g.nx : 0;
    const bool fluid = in && a.mask[y * g.pitch + x] == 0;
    const E *src = static_cast<const E *>(a.src);
#pragma unroll
    for (int d = 1; d < 9; d++) {
        int id = 0;
        double mx = 0.0, my = 0.0;
        if (fluid) {
            int xs = x + cx[d], ys = y + cy[d];
            bool link = true;
            if (xs < 0 || xs >= g.nx) {
                if (g.xper) xs += xs < 0 ? g.nx : -g.nx;
                else link = false;
            }
            if (ys < 0 || ys >= g.ny) {
                if (g.yper) ys += ys < 0 ? g.ny : -g.ny;
                else link = false;
            }
            if (link) id = a.mask[ys * g.pitch + xs];
            if (id) {
                const double m = C::decode(src + d * g.plane, y * g.pitch + x, weight<double>(d)) +
                                 C::decode(src + opp[d] * g.plane, ys * g.pitch + xs, weight<double>(opp[d]));
                mx = cx[d] * m;
                my = cy[d] * m;
            }
        }
        // wave_forces adds minus its arguments, per body id, in a fixed order
        wave_forces<false>(rows[wave], -mx, -my, id);
    }
    __syncthreads();
    if (threadIdx.x < kRingWidth) {
        double v = 0.0;
        for (int w = 0; w < kBlock / 64; w++) v += rows[w][threadIdx.x];
        part[(size_t)blockIdx.x * kRingWidth + threadIdx.x] = v;
    }
}

// out[2k], out[2k + 1] = body k's (fx, fy): the rows of part summed in a fixed order (lane l takes
// rows l, l + 64, ..., then a fixed butterfly), one wave per value.
__global__ void exchange_fold_kernel(const double *part, int nparts, double *out)
{
    const int q = 1 + blockIdx.x;                   // entry 1 .. 16 of a row
    double v = 0.0;
    for (int b = threadIdx.x; b < nparts; b += 64) v += part[(size_t)b * kRingWidth + q];
    v = wave_sum<false>(v);
    if (threadIdx.x == 0) out[q - 1] = v;
}

int launch_exchange_static(int storage, const StepArgs &a, double *scratch_ptr, double *out,
                           hipStream_t st)
{
    const long long nodes = (long long)a.g.nx * a.g.ny;
    const long long parts = (nodes + kBlock - 1) / kBlock;
    if (parts > kScratchParts)
        return fail(VPLBM_EINVAL, "lattice of %lld nodes: the static scratch holds the partial sums of "
                    "%lld nodes at most", nodes, (long long)kScratchParts * kBlock);
    const dim3 grid((unsigned)parts), block(kBlock);
    switch (storage) {
    case kF64: exchange_parts_kernel<kF64><<<grid, block, 0, st>>>(a, scratch_ptr); break;
    case kF32: exchange_parts_kernel<kF32><<<grid, block, 0, st>>>(a, scratch_ptr); break;
    case kF16S: exchange_parts_kernel<kF16S><<<grid, block, 0, st>>>(a, scratch_ptr); break;
    case kBF16S: exchange_parts_kernel<kBF16S><<<grid, block, 0, st>>>(a, scratch_ptr); break;
    case kF32D: exchange_parts_kernel<kF32D><<<grid, block, 0, st>>>(a, scratch_ptr); break;
    case kF16SR: exchange_parts_kernel<kF16SR><<<grid, block, 0, st>>>(a, scratch_ptr); break;
    case kBF16SR: exchange_parts_kernel<kBF16SR><<<grid, block, 0, st>>>(a, scratch_ptr); break;
    default: return fail(VPLBM_EINVAL, "unknown storage %d", storage);
    }
    HIP_TRY(hipGetLastError());
    exchange_fold_kernel<<<2 * kMaxBodies, 64, 0, st>>>(scratch_ptr, (int)parts, out);
    HIP_TRY(hipGetLastError());
    return VPLBM_OK;
}

}  // namespace vplbm
