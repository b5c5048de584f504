// The fine DNN-MG step on unstructured quadrilateral meshes (explicit
// connectivity; fine nodes on curved edges moved onto the curve).
//
// Per step (Alg. 2, lines 6-9), all data addressed through the patch maps:
//   k_udefect  one thread per fine element: the element residual of the
//              defect (quad_residual: its own bilinear map and nodal P v, P p,
//              u_prev), summed per patch-local node in LDS in four colour
//              rounds (elements of one colour share no node);
//   k_unode    one thread per fine node: the patches' contributions summed in
//              patch order (node_occ), zero at Dirichlet nodes;
//   k_uinput   the network input rows [P v, D, hx, hy, aspect, area];
//   (network)  the structured path's kernels on the rows;
//   k_uaverage one thread per fine node: the mean of the patches' outputs,
//              masked; the corrected velocity P v + d is the next u_prev;
//   k_urhs     one thread per patch, FP64: its fine elements' mass products
//              (1/dt) M (P v + d), weighted by the coarse hats at the nodes,
//              give the patch's share of b^L at its four corners (R = P^T);
//   k_ugather  one thread per coarse node: the shares summed in patch order.
// Sums over shared nodes are gathers in a fixed order: no atomics, bitwise
// deterministic.  P v at a fine node is the bilinear interpolation, in the
// reference coordinates of the first patch that holds the node, of that
// patch's corner values.
#include "device.h"
#include "element.h"
#include "internal.h"

namespace dnnmg {

// Coarse hats of corners v0 (0,0), v1 (1,0), v2 (1,1), v3 (0,1) at the
// patch-local node l = b (n+1) + a.
template <typename T>
__device__ inline void corner_hats(int n, int l, T (&N)[4])
{
    const int a = l % (n + 1), b = l / (n + 1);
    const T s = (T)a / (T)n, t = (T)b / (T)n;
    N[0] = (1 - s) * (1 - t);
    N[1] = s * (1 - t);
    N[2] = s * t;
    N[3] = (1 - s) * t;
}

// ------------------------------------------------------------------ defect
template <int K>
__global__ __launch_bounds__(kThreads) void k_udefect(UArgs u)
{
    constexpr int n = 1 << K, nf = (n + 1) * (n + 1), NE = n * n, PPB = kThreads / NE;
    __shared__ float2 s_loc[PPB * nf];
    const int tid = threadIdx.x, pb = tid / NE, el = tid - pb * NE, a = el % n, b = el / n;
    const int e = blockIdx.x * PPB + pb;
    const bool valid = e < u.P;
    for (int t = tid; t < PPB * nf; t += kThreads) s_loc[t] = make_float2(0.f, 0.f);
    float R[8];
    const int l00 = b * (n + 1) + a, ls[4] = {l00, l00 + 1, l00 + n + 1, l00 + n + 2};
    if (valid) {
        const int *cn = u.corners + 4 * (size_t)e;
        const float2 *v2 = reinterpret_cast<const float2 *>(u.v);
        float2 cv[4];
        float cp[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            cv[k] = v2[cn[k]];
            cp[k] = u.p ? u.p[cn[k]] : 0.0f;
        }
        const int first = *u.first_flag;
        const float idt = first ? 0.0f : u.inv_dt;
        float x[4], y[4], vx[4], vy[4], pn[4], wx[4], wy[4];
        const double2 *rel = reinterpret_cast<const double2 *>(u.rel) + (size_t)e * nf;
        const float2 *up = reinterpret_cast<const float2 *>(u.uprev);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double2 r = rel[ls[k]];
            x[k] = (float)r.x;
            y[k] = (float)r.y;
            float N[4];
            corner_hats(n, ls[k], N);
            vx[k] = N[0] * cv[0].x + N[1] * cv[1].x + N[2] * cv[2].x + N[3] * cv[3].x;
            vy[k] = N[0] * cv[0].y + N[1] * cv[1].y + N[2] * cv[2].y + N[3] * cv[3].y;
            pn[k] = N[0] * cp[0] + N[1] * cp[1] + N[2] * cp[2] + N[3] * cp[3];
            const float2 w = first ? make_float2(0.f, 0.f) : up[u.pmap[(size_t)e * nf + ls[k]]];
            wx[k] = w.x * idt;
            wy[k] = w.y * idt;
        }
        quad_residual<HwRcp>(x, y, vx, vy, pn, wx, wy, u.nu, idt, R);
    }
    __syncthreads();
    // four rounds: elements (a, b) of one parity pair share no node
    const int colour = (a & 1) + 2 * (b & 1);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (valid && colour == c) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float2 &q = s_loc[pb * nf + ls[k]];
                q.x += R[2 * k];
                q.y += R[2 * k + 1];
            }
        }
        __syncthreads();
    }
    float2 *dl = reinterpret_cast<float2 *>(u.dloc) + (size_t)blockIdx.x * PPB * nf;
    const int nvalid = min(PPB, u.P - blockIdx.x * PPB) * nf;
    for (int t = tid; t < nvalid; t += kThreads) dl[t] = s_loc[t];
}

__global__ __launch_bounds__(kThreads) void k_unode(UArgs u, float *D)
{
    const int f = blockIdx.x * kThreads + threadIdx.x;
    if (f >= u.Fn) return;
    const float2 *dl = reinterpret_cast<const float2 *>(u.dloc);
    float2 s = make_float2(0.f, 0.f);
    for (int k = u.node_ptr[f]; k < u.node_ptr[f + 1]; ++k) {
        const float2 q = dl[u.node_occ[k]];
        s.x += q.x;
        s.y += q.y;
    }
    if (u.mask[f]) s = make_float2(0.f, 0.f);
    reinterpret_cast<float2 *>(D)[f] = s;
}

template <int K>
static void launch_udefect_k(const UArgs &u, float *D, hipStream_t s)
{
    constexpr int n = 1 << K, PPB = kThreads / (n * n);
    hipLaunchKernelGGL(k_udefect<K>, dim3((u.P + PPB - 1) / PPB), dim3(kThreads), 0, s, u);
    hipLaunchKernelGGL(k_unode, dim3((u.Fn + kThreads - 1) / kThreads), dim3(kThreads), 0, s, u, D);
}

hipError_t launch_udefect(const UArgs &u, float *D, hipStream_t s)
{
    switch (u.K) {
    case 1: launch_udefect_k<1>(u, D, s); break;
    case 2: launch_udefect_k<2>(u, D, s); break;
    case 3: launch_udefect_k<3>(u, D, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------- network input rows
// One thread per (patch, local node) writes P v and D at the node; one per
// patch writes its four features.
template <int K, typename XT>
__global__ __launch_bounds__(kThreads) void k_uinput(UArgs u)
{
    constexpr int n = 1 << K, nf = (n + 1) * (n + 1);
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (t >= (long long)u.P * (nf + 1)) return;
    const int e = (int)(t / (nf + 1)), l = (int)(t - (long long)e * (nf + 1));
    XT *x = reinterpret_cast<XT *>(u.X) + (size_t)e * u.nin;
    if (l == nf) {
        const float4 ft = reinterpret_cast<const float4 *>(u.feat)[e];
        x[4 * nf] = (XT)ft.x; x[4 * nf + 1] = (XT)ft.y; x[4 * nf + 2] = (XT)ft.z; x[4 * nf + 3] = (XT)ft.w;
        return;
    }
    const int *cn = u.corners + 4 * (size_t)e;
    const float2 *v2 = reinterpret_cast<const float2 *>(u.v);
    float N[4];
    corner_hats(n, l, N);
    const float2 c0 = v2[cn[0]], c1 = v2[cn[1]], c2 = v2[cn[2]], c3 = v2[cn[3]];
    const float2 d = reinterpret_cast<const float2 *>(u.D)[u.pmap[(size_t)e * nf + l]];
    x[2 * l] = (XT)(N[0] * c0.x + N[1] * c1.x + N[2] * c2.x + N[3] * c3.x);
    x[2 * l + 1] = (XT)(N[0] * c0.y + N[1] * c1.y + N[2] * c2.y + N[3] * c3.y);
    x[2 * nf + 2 * l] = (XT)d.x;
    x[2 * nf + 2 * l + 1] = (XT)d.y;
}

hipError_t launch_uinput(const UArgs &u, hipStream_t s)
{
    const int nf = ((1 << u.K) + 1) * ((1 << u.K) + 1);
    const long long items = (long long)u.P * (nf + 1);
    dim3 g((unsigned)((items + kThreads - 1) / kThreads)), b(kThreads);
#define DNNMG_UINPUT(KK)                                                                  \
    case KK:                                                                              \
        if (u.xfmt == 1) hipLaunchKernelGGL((k_uinput<KK, __bf16>), g, b, 0, s, u);       \
        else hipLaunchKernelGGL((k_uinput<KK, float>), g, b, 0, s, u);                    \
        break;
    switch (u.K) {
        DNNMG_UINPUT(1)
        DNNMG_UINPUT(2)
        DNNMG_UINPUT(3)
    default: return hipErrorInvalidValue;
    }
#undef DNNMG_UINPUT
    return hipGetLastError();
}

// P v (and P p) at fine node f from its first patch.
template <typename T>
__device__ inline void uprolong_node(const UArgs &u, int nf, int n, int f, T &vx, T &vy, bool want_p, T &pp)
{
    const int occ = u.node_occ[u.node_ptr[f]];
    const int e = occ / nf, l = occ - e * nf;
    const int *cn = u.corners + 4 * (size_t)e;
    T N[4];
    corner_hats(n, l, N);
    const float2 *v2 = reinterpret_cast<const float2 *>(u.v);
    vx = 0;
    vy = 0;
    T q = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float2 c = v2[cn[k]];
        vx += N[k] * (T)c.x;
        vy += N[k] * (T)c.y;
        if (want_p) q += N[k] * (T)u.p[cn[k]];
    }
    pp = q;
}

// ------------------------------------------- averaging, state, correction
__global__ __launch_bounds__(kThreads) void k_uaverage(UArgs u)
{
    const int f = blockIdx.x * kThreads + threadIdx.x;
    if (f >= u.Fn) return;
    const int n = 1 << u.K, nf = (n + 1) * (n + 1);
    const int k0 = u.node_ptr[f], k1 = u.node_ptr[f + 1];
    float2 s = make_float2(0.f, 0.f);
    for (int k = k0; k < k1; ++k) {
        const float2 q = reinterpret_cast<const float2 *>(u.dpatch)[u.node_occ[k]];
        s.x += q.x;
        s.y += q.y;
    }
    const float inv = 1.0f / (float)(k1 - k0);
    float2 d = u.mask[f] ? make_float2(0.f, 0.f) : make_float2(s.x * inv, s.y * inv);
    float vx, vy, unused;
    uprolong_node<float>(u, nf, n, f, vx, vy, false, unused);
    reinterpret_cast<float2 *>(u.uprev)[f] = make_float2(vx + d.x, vy + d.y);
    reinterpret_cast<float2 *>(u.D)[f] = d;
    if (u.dbar_out) reinterpret_cast<float2 *>(u.dbar_out)[f] = d;
    if (u.nonfinite && !(__builtin_isfinite(d.x) && __builtin_isfinite(d.y))) atomicOr(u.nonfinite, 1);
    if (f == 0) *u.first_flag = 0;   // the step's defect has read it (stream order)
}

hipError_t launch_uaverage(const UArgs &u, hipStream_t s)
{
    hipLaunchKernelGGL(k_uaverage, dim3((u.Fn + kThreads - 1) / kThreads), dim3(kThreads), 0, s, u);
    return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void k_uprolong(UArgs u)
{
    const int f = blockIdx.x * kThreads + threadIdx.x;
    if (f >= u.Fn) return;
    const int n = 1 << u.K, nf = (n + 1) * (n + 1);
    float vx, vy, q = 0.0f;
    uprolong_node<float>(u, nf, n, f, vx, vy, u.p && u.pp_out, q);
    if (u.pv_out) reinterpret_cast<float2 *>(u.pv_out)[f] = make_float2(vx, vy);
    if (u.p && u.pp_out) u.pp_out[f] = q;
}

hipError_t launch_uprolong(const UArgs &u, hipStream_t s)
{
    hipLaunchKernelGGL(k_uprolong, dim3((u.Fn + kThreads - 1) / kThreads), dim3(kThreads), 0, s, u);
    return hipGetLastError();
}

// -------------------------------------------------------- FP64 rhs shares
// One thread per patch.  For each fine element and Gauss point: det and the
// corrected velocity (P v from the corner values in FP64, plus d) at the
// point; node k of the element receives w det N_k u, which the coarse hats
// at that node carry to the patch's corners.
template <int K>
__global__ __launch_bounds__(kThreads) void k_urhs(UArgs u, const float *dbar)
{
    constexpr int n = 1 << K, nf = (n + 1) * (n + 1);
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= u.P) return;
    constexpr double g0 = 0.21132486540518711775, g1 = 0.78867513459481288225;
    const int *cn = u.corners + 4 * (size_t)e;
    const float2 *v2 = reinterpret_cast<const float2 *>(u.v);
    double cvx[4], cvy[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float2 c = v2[cn[k]];
        cvx[k] = c.x;
        cvy[k] = c.y;
    }
    const double2 *rel = reinterpret_cast<const double2 *>(u.rel) + (size_t)e * nf;
    const int *pm = u.pmap + (size_t)e * nf;
    const float2 *db = reinterpret_cast<const float2 *>(dbar);
    double b[4][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
#pragma unroll 1
    for (int el = 0; el < n * n; ++el) {
        const int a = el % n, bb = el / n, l00 = bb * (n + 1) + a;
        const int ls[4] = {l00, l00 + 1, l00 + n + 1, l00 + n + 2};
        double x[4], y[4], ux[4], uy[4], H[4][4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double2 r = rel[ls[k]];
            x[k] = r.x;
            y[k] = r.y;
            corner_hats(n, ls[k], H[k]);
            const float2 d = db[pm[ls[k]]];
            ux[k] = H[k][0] * cvx[0] + H[k][1] * cvx[1] + H[k][2] * cvx[2] + H[k][3] * cvx[3] + (double)d.x;
            uy[k] = H[k][0] * cvy[0] + H[k][1] * cvy[1] + H[k][2] * cvy[2] + H[k][3] * cvy[3] + (double)d.y;
        }
#pragma unroll 1
        for (int q = 0; q < 4; ++q) {
            const double s = (q & 1) ? g1 : g0, t = (q >> 1) ? g1 : g0;
            const double N[4] = {(1 - s) * (1 - t), s * (1 - t), (1 - s) * t, s * t};
            const double Ns[4] = {-(1 - t), 1 - t, -t, t}, Nt[4] = {-(1 - s), -s, 1 - s, s};
            double xs = 0, xt = 0, ys = 0, yt = 0, uqx = 0, uqy = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                xs += x[k] * Ns[k]; xt += x[k] * Nt[k];
                ys += y[k] * Ns[k]; yt += y[k] * Nt[k];
                uqx += N[k] * ux[k]; uqy += N[k] * uy[k];
            }
            const double wd = 0.25 * fabs(xs * yt - xt * ys);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double mx = wd * N[k] * uqx, my = wd * N[k] * uqy;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    b[c][0] += H[k][c] * mx;
                    b[c][1] += H[k][c] * my;
                }
            }
        }
    }
    double2 *out = reinterpret_cast<double2 *>(u.part) + 4 * (size_t)e;
#pragma unroll
    for (int c = 0; c < 4; ++c) out[c] = make_double2(u.inv_dt64 * b[c][0], u.inv_dt64 * b[c][1]);
}

hipError_t launch_urhs(const UArgs &u, const float *dbar, hipStream_t s)
{
    dim3 g((u.P + kThreads - 1) / kThreads), b(kThreads);
    switch (u.K) {
    case 1: hipLaunchKernelGGL(k_urhs<1>, g, b, 0, s, u, dbar); break;
    case 2: hipLaunchKernelGGL(k_urhs<2>, g, b, 0, s, u, dbar); break;
    case 3: hipLaunchKernelGGL(k_urhs<3>, g, b, 0, s, u, dbar); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void k_ugather(UArgs u)
{
    const int c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= u.Nc) return;
    const double2 *pt = reinterpret_cast<const double2 *>(u.part);
    double bx = 0.0, by = 0.0;
    for (int k = u.cnode_ptr[c]; k < u.cnode_ptr[c + 1]; ++k) {
        const double2 q = pt[u.cnode_occ[k]];
        bx += q.x;
        by += q.y;
    }
    reinterpret_cast<double2 *>(u.bL)[c] = make_double2(bx, by);
    if (u.nonfinite && !(__builtin_isfinite(bx) && __builtin_isfinite(by))) atomicOr(u.nonfinite, 2);
}

hipError_t launch_ugather(const UArgs &u, hipStream_t s)
{
    hipLaunchKernelGGL(k_ugather, dim3((u.Nc + kThreads - 1) / kThreads), dim3(kThreads), 0, s, u);
    return hipGetLastError();
}

}  // namespace dnnmg
