// Device-side helpers shared by the kernel sources (not the host code).
#pragma once

#include <hip/hip_runtime.h>

namespace dnnmg {

// The thread's index in its workgroup, opaque to the optimiser.  The batched
// kernels loop over tiles; with the plain index the compiler hoists every
// index-derived address and mask out of that loop and keeps them live across
// it, which costs tens of VGPRs.  The empty asm makes the value new in each
// tile, so it is recomputed where it is used, as in the single-flow kernels.
__device__ inline int tile_thread()
{
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

}  // namespace dnnmg
