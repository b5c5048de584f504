// Device-side helpers shared by the kernel sources (not the host code).
#pragma once

#include <hip/hip_runtime.h>

namespace dnnmg {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));

// Logistic function and tanh from the hardware exponential and reciprocal
// (tanh x = 1 - 2 / (1 + e^{2x})); absolute error ~1e-7, which is what the
// state update h' = z h + (1 - z) tanh(.) needs.
__device__ inline float sigmoid(float t) { return __builtin_amdgcn_rcpf(1.0f + __expf(-t)); }
__device__ inline float fast_tanh(float t) { return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + __expf(2.0f * t)); }
// The same on pre-activations that the packed BF16 weights have already
// multiplied by -log2(e) (the gates z and r, logistic) or by 2 log2(e) (the
// candidate state, tanh): the exponential is then the hardware's 2^x, with no
// scaling multiply.
__device__ inline float sigmoid_l2(float t) { return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t)); }
__device__ inline float tanh_l2(float t) { return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t)); }

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

// Pointer into global memory (address space 1): loads through it are global
// loads with a scalar base and a 32-bit lane offset, not flat loads, which
// would also count against the LDS wait counter.
template <typename T>
using gptr = const __attribute__((address_space(1))) T *;

// A pointer the optimiser cannot move loads through from before this point:
// keeps weight loads where they are written instead of hoisted to the top of
// a kernel, where they would hold registers through unrelated phases.  The
// pointee must be device (global) memory.
template <typename T>
__device__ inline gptr<T> pinned(const void *p)
{
    asm volatile("" : "+s"(p));
    return (gptr<T>)(p);
}

}  // namespace dnnmg
