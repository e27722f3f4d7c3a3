// The static device scratch of the allocation-free entry point (internal; see static_scratch.hip).
#pragma once

#include "kernels.hpp"

namespace vplbm {

// Rows of partial sums the static scratch holds: one per workgroup of kBlock nodes, so lattices
// of up to kScratchParts * kBlock = 16,777,216 nodes (8192 x 2048).  8.5 MiB per GPU.
constexpr int kScratchParts = 65536;
constexpr int kScratchDevices = 64;

// Look up the current device's address of the scratch array once (hipGetSymbolAddress).
int static_scratch_init();
// The address static_scratch_init recorded for device dev, or nullptr.
double *static_scratch(int dev);
// Momentum exchange of the state a.src into out[16] (device memory), partial sums in scratch_ptr.
int launch_exchange_static(int storage, const StepArgs &a, double *scratch_ptr, double *out,
                           hipStream_t st);

}  // namespace vplbm
