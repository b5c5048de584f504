// Duplicate averaging, corrected velocity, FP64 right-hand side and restriction.
//
// Per patch E (one coarse element) the kernel
//   1. averages the per-patch network outputs at each of its (n+1)^2 fine
//      nodes over the 1, 2 or 4 patches that contain the node (Sec. 4.2),
//      zeroes Dirichlet nodes, and stores the corrected velocity P v + d as the
//      state for the next defect (the patch that owns a node writes it);
//   2. forms its share of b_L = P^T (1/dt) M_f (P v + d) (Alg. 2, lines 8-9) at
//      its four corners, in FP64.
// Step 2 uses exact moment tables instead of fine quadrature.  With the
// coarse map F, det J = d0 + d1 xi + d2 eta is affine, so for the coarse hat N_c
// restricted to E
//   int_E N_c (P v) dx = sum_c' v_c' [d0 M0 + d1 M1 + d2 M2]_{c c'}
//   int_E N_c d     dx = sum_l  d_l  [d0 G0 + d1 G1 + d2 G2]_{c l}
// where M_k, G_k integrate N_c N_c' {1, xi, eta} and N_c phi_l {1, xi, eta} on the
// reference square (phi_l the fine Q1 hat of patch node l).  These are the
// same integrals the fine-level 2 x 2 Gauss rule computes exactly (the
// integrands are polynomials of degree <= 3 per variable on every fine cell),
// and P^T is the evaluation of N_c at fine nodes, so the result equals the
// definition up to FP64 rounding.  A second kernel sums the four patch
// contributions at each coarse node in a fixed order (no atomics).
#include "internal.h"

namespace dnnmg {

template <int K>
__device__ inline bool dirichlet_node(unsigned dir, int I, int J, int NX, int NY)
{
    return ((dir & 1u) && I == 0) || ((dir & 2u) && I == NX) || ((dir & 4u) && J == 0) || ((dir & 8u) && J == NY);
}

// from_patches = 1: average f.dpatch (the step); 0: take f.dbar_in (stage).
template <int K, int FROM_PATCHES>
__global__ __launch_bounds__(kThreads) void k_rhs(FlowArgs single, const BatchTable *bt, RhsTables tab)
{
    constexpr int n = 1 << K;
    constexpr int nf = (n + 1) * (n + 1);
    constexpr int nout = 2 * nf;
    int blk = blockIdx.x;
    const FlowArgs f = bt ? *batch_flow(bt, kKindRhs, blk) : single;
    const int nx = f.nx, ny = f.ny, NX = nx * n, NY = ny * n;
    const int e = blk * kThreads + threadIdx.x;
    // The step's defect has already read the first-step flag (stream order).
    if (FROM_PATCHES && e == 0) *f.first_flag = 0;
    if (e >= nx * ny) return;
    const int pi = e % nx, pj = e / nx;
    const double d0 = f.geo64[4 * (size_t)e], d1 = f.geo64[4 * (size_t)e + 1], d2 = f.geo64[4 * (size_t)e + 2];
    const float2 *v2 = reinterpret_cast<const float2 *>(f.v);
    const int c00 = pj * (nx + 1) + pi;
    const float2 vc[4] = {v2[c00], v2[c00 + 1], v2[c00 + nx + 1], v2[c00 + nx + 2]};

    double acc[4][2];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c][0] = acc[c][1] = 0.0;

    for (int b = 0; b <= n; ++b) {
        for (int a = 0; a <= n; ++a) {
            const int l = b * (n + 1) + a;
            const int I = pi * n + a, J = pj * n + b;
            float dx, dy;
            if (FROM_PATCHES) {
                // containing patches in (row, column) order, as the mean is defined
                const int qj0 = (b == 0 && pj > 0) ? pj - 1 : pj, qj1 = (b == n && pj < ny - 1) ? pj + 1 : pj;
                const int qi0 = (a == 0 && pi > 0) ? pi - 1 : pi, qi1 = (a == n && pi < nx - 1) ? pi + 1 : pi;
                float sx = 0.f, sy = 0.f;
                int cnt = 0;
                for (int qj = qj0; qj <= qj1; ++qj)
                    for (int qi = qi0; qi <= qi1; ++qi) {
                        const int ll = (b - (qj - pj) * n) * (n + 1) + (a - (qi - pi) * n);
                        const float *dq = f.dpatch + ((size_t)qj * nx + qi) * nout + 2 * ll;
                        sx += dq[0];
                        sy += dq[1];
                        ++cnt;
                    }
                const float inv = cnt == 1 ? 1.0f : (cnt == 2 ? 0.5f : 0.25f);
                dx = sx * inv;
                dy = sy * inv;
                if (dirichlet_node<K>(f.dirichlet, I, J, NX, NY)) dx = dy = 0.f;
                const bool owned = (a < n || pi == nx - 1) && (b < n || pj == ny - 1);
                if (owned) {
                    const size_t fi = (size_t)J * (NX + 1) + I;
                    const float xi = a * (1.0f / n), eta = b * (1.0f / n);
                    const float n00 = (1.f - xi) * (1.f - eta), n10 = xi * (1.f - eta), n01 = (1.f - xi) * eta,
                                n11 = xi * eta;
                    const float pvx = n00 * vc[0].x + n10 * vc[1].x + n01 * vc[2].x + n11 * vc[3].x;
                    const float pvy = n00 * vc[0].y + n10 * vc[1].y + n01 * vc[2].y + n11 * vc[3].y;
                    reinterpret_cast<float2 *>(f.uprev)[fi] = make_float2(pvx + dx, pvy + dy);
                    if (f.dbar_out) reinterpret_cast<float2 *>(f.dbar_out)[fi] = make_float2(dx, dy);
                }
            } else {
                const float2 d = reinterpret_cast<const float2 *>(f.dbar_in)[(size_t)J * (NX + 1) + I];
                dx = d.x;
                dy = d.y;
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double w = d0 * tab.G[(0 * 4 + c) * nf + l] + d1 * tab.G[(1 * 4 + c) * nf + l] +
                                 d2 * tab.G[(2 * 4 + c) * nf + l];
                acc[c][0] += w * (double)dx;
                acc[c][1] += w * (double)dy;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            const double w = d0 * tab.M[(0 * 4 + c) * 4 + cc] + d1 * tab.M[(1 * 4 + c) * 4 + cc] +
                             d2 * tab.M[(2 * 4 + c) * 4 + cc];
            acc[c][0] += w * (double)vc[cc].x;
            acc[c][1] += w * (double)vc[cc].y;
        }
    double *out = f.part + 8 * (size_t)e;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        out[2 * c] = f.inv_dt64 * acc[c][0];
        out[2 * c + 1] = f.inv_dt64 * acc[c][1];
    }
}

// b_L at coarse node (i,j): the node is corner 11 of patch (i-1,j-1), corner 01
// of (i,j-1), corner 10 of (i-1,j) and corner 00 of (i,j); summed in that order.
__global__ __launch_bounds__(kThreads) void k_gather(FlowArgs single, const BatchTable *bt)
{
    int blk = blockIdx.x;
    const FlowArgs f = bt ? *batch_flow(bt, kKindGather, blk) : single;
    const int nx = f.nx, ny = f.ny;
    const int t = blk * kThreads + threadIdx.x;
    if (t >= (nx + 1) * (ny + 1)) return;
    const int i = t % (nx + 1), j = t / (nx + 1);
    double bx = 0.0, by = 0.0;
    if (i > 0 && j > 0) { const double *q = f.part + 8 * ((size_t)(j - 1) * nx + i - 1) + 6; bx += q[0]; by += q[1]; }
    if (i < nx && j > 0) { const double *q = f.part + 8 * ((size_t)(j - 1) * nx + i) + 4; bx += q[0]; by += q[1]; }
    if (i > 0 && j < ny) { const double *q = f.part + 8 * ((size_t)j * nx + i - 1) + 2; bx += q[0]; by += q[1]; }
    if (i < nx && j < ny) { const double *q = f.part + 8 * ((size_t)j * nx + i); bx += q[0]; by += q[1]; }
    f.bL[2 * (size_t)t] = bx;
    f.bL[2 * (size_t)t + 1] = by;
}

hipError_t launch_rhs(const FlowArgs &f, const BatchTable *bt, int nblocks, int K, const RhsTables &tab,
                      int from_patches, hipStream_t s)
{
    dim3 g(nblocks), b(kThreads);
#define DNNMG_RHS_CASE(KK)                                                                \
    case KK:                                                                              \
        if (from_patches) hipLaunchKernelGGL((k_rhs<KK, 1>), g, b, 0, s, f, bt, tab);     \
        else hipLaunchKernelGGL((k_rhs<KK, 0>), g, b, 0, s, f, bt, tab);                  \
        break;
    switch (K) {
        DNNMG_RHS_CASE(1)
        DNNMG_RHS_CASE(2)
        DNNMG_RHS_CASE(3)
    default: return hipErrorInvalidValue;
    }
#undef DNNMG_RHS_CASE
    return hipGetLastError();
}

hipError_t launch_gather(const FlowArgs &f, const BatchTable *bt, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather, dim3(nblocks), dim3(kThreads), 0, s, f, bt);
    return hipGetLastError();
}

}  // namespace dnnmg
