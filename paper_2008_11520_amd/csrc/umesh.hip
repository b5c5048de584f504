// The fine DNN-MG step on unstructured quadrilateral meshes (explicit
// connectivity; fine nodes on curved edges moved onto the curve).
//
// Per step (the fine part of Alg. 2), all data addressed through the patch maps:
//   k_udefect  one thread per fine element: the element residual of the
//              defect (quad_residual: its own bilinear map and nodal P v, P p,
//              u_prev), summed per patch-local node in LDS in four colour
//              rounds (elements of one colour share no node);
//   k_unode    one thread per fine node: the patches' contributions summed in
//              patch order (node_occ), zero at Dirichlet nodes;
//   k_uinput   the network input rows [P v, D, hx, hy, aspect, area], D
//              summed from the contributions as k_unode sums them;
//   (network)  the structured path's kernels on the rows;
//   k_uaverage one thread per fine node: the mean of the patches' outputs,
//              masked; the corrected velocity P v + d is the next u_prev;
//   k_urhs     FP64: each patch's share of b^L = R (1/dt) M (P v + d) at its
//              corners: on a patch with straight edges (the bilinear image of
//              the reference square) from exact moments of det J, as on
//              structured meshes; on one with a curved edge from its
//              hat-weighted mass rows (formed at create from the fine
//              elements' 2 x 2 Gauss points); R = P^T;
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
        const float2 *rel = reinterpret_cast<const float2 *>(u.rel) + (size_t)e * nf;
        const float2 *up = reinterpret_cast<const float2 *>(u.uprev);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float2 r = rel[ls[k]];
            x[k] = r.x;
            y[k] = r.y;
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

// D == nullptr: the element contributions only (the step: the network input
// sums them per node itself); else also the defect at the fine nodes.
template <int K>
static void launch_udefect_k(const UArgs &u, float *D, hipStream_t s)
{
    constexpr int n = 1 << K, PPB = kThreads / (n * n);
    hipLaunchKernelGGL(k_udefect<K>, dim3((u.P + PPB - 1) / PPB), dim3(kThreads), 0, s, u);
    if (D) hipLaunchKernelGGL(k_unode, dim3((u.Fn + kThreads - 1) / kThreads), dim3(kThreads), 0, s, u, D);
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
// One thread per (patch, local node) writes P v and D at the node (pairs as
// one store); one per patch writes its four features.  D comes from the
// patches' element contributions directly: the node's contributions summed
// over its gather list in patch order, as k_unode sums them (the same value
// bit for bit), zero at Dirichlet nodes.
template <typename XT>
__device__ inline void store_pair(XT *o, float a, float b)
{
    if constexpr (sizeof(XT) == 4) {
        *reinterpret_cast<float2 *>(o) = make_float2(a, b);
    } else {
        typedef __bf16 b2 __attribute__((ext_vector_type(2)));
        b2 v;
        v[0] = (__bf16)a;
        v[1] = (__bf16)b;
        *reinterpret_cast<b2 *>(o) = v;
    }
}

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
        store_pair(x + 4 * nf, ft.x, ft.y);
        store_pair(x + 4 * nf + 2, ft.z, ft.w);
        return;
    }
    const int *cn = u.corners + 4 * (size_t)e;
    const float2 *v2 = reinterpret_cast<const float2 *>(u.v);
    float N[4];
    corner_hats(n, l, N);
    const float2 c0 = v2[cn[0]], c1 = v2[cn[1]], c2 = v2[cn[2]], c3 = v2[cn[3]];
    const float2 *dl = reinterpret_cast<const float2 *>(u.dloc);
    const int a = l % (n + 1), b = l / (n + 1);
    float2 d;
    if (a > 0 && a < n && b > 0 && b < n) {
        // a node inside the patch: this patch alone holds it, no Dirichlet side
        d = dl[(size_t)e * nf + l];
    } else {
        const int f = u.pmap[(size_t)e * nf + l];
        d = make_float2(0.f, 0.f);
        for (int k = u.node_ptr[f]; k < u.node_ptr[f + 1]; ++k) {
            const float2 q = dl[u.node_occ[k]];
            d.x += q.x;
            d.y += q.y;
        }
        if (u.mask[f]) d = make_float2(0.f, 0.f);
    }
    store_pair(x + 2 * l, N[0] * c0.x + N[1] * c1.x + N[2] * c2.x + N[3] * c3.x,
               N[0] * c0.y + N[1] * c1.y + N[2] * c2.y + N[3] * c3.y);
    store_pair(x + 2 * nf + 2 * l, d.x, d.y);
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
// The patch's share of R (1/dt) M_f u at each corner c, u = P v + d, from its
// hat-weighted mass rows formed at create (static geometry, FP64):
//   sum_k M4[c][k] v_k + sum_l W[c][l] d_l.
// A workgroup takes PPB patches; thread (patch, l) reads d at node l and the
// four rows' entries l (consecutive lanes, consecutive addresses) and leaves
// the eight products in LDS; thread (patch, corner, component) then sums them
// over l in order.
// One thread per patch.  Straight edges: with u the nodal values (a, b) of
// the patch, the share at structured corner (cx, cy) is
//   d0 S0 + d1 S1 + d2 S2,  S_k = sum_b A[my_k][cy][b] sum_a A[mx_k][cx][a] u(a, b)
// ((mx, my) = (0, 0), (1, 0), (0, 1)), formed node row by node row as in the
// structured rhs; the coarse term of P v from the moment tables M likewise.
// (one wave per block: the patches are few for the chip, so small blocks
// spread them over every CU; for K <= 2 all of a patch's map entries and then
// all its corrections are loaded before any arithmetic: two memory round
// trips per patch instead of two per node row)
constexpr int kURhsThreads = 64;

template <int K>
__global__ __launch_bounds__(kURhsThreads) void k_urhs(UArgs u, const float *dbar)
{
    constexpr int n = 1 << K, nf = (n + 1) * (n + 1);
    constexpr int NA = 4 * (n + 1), NM = 48;
    constexpr bool ALL = K <= 2;
    __shared__ double s_A[NA], s_M[NM];
    const int tid = threadIdx.x;
    for (int t = tid; t < NA + NM; t += kURhsThreads) {
        if (t < NA) s_A[t] = u.tab.A[t];
        else s_M[t - NA] = u.tab.M[t - NA];
    }
    __syncthreads();
    const int e = blockIdx.x * kURhsThreads + tid;
    if (e >= u.P) return;
    const int *pm = u.pmap + (size_t)e * nf;
    const float2 *d2 = reinterpret_cast<const float2 *>(dbar);
    float2 wall[ALL ? nf : 1];
    if constexpr (ALL) {
        int f[nf];
#pragma unroll
        for (int l = 0; l < nf; ++l) f[l] = pm[l];
#pragma unroll
        for (int l = 0; l < nf; ++l) wall[l] = d2[f[l]];
    }
    const int *cn = u.corners + 4 * (size_t)e;
    const float2 *v2 = reinterpret_cast<const float2 *>(u.v);
    float2 cv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) cv[k] = v2[cn[k]];
    const int ci = u.cidx[e];
    double out[4][2];     // [corner (00, 10, 11, 01)][component]
    if (ci < 0) {
        const double *g = u.dgeo + 4 * (size_t)e;
        const double g0 = g[0], g1 = g[1], g2 = g[2];
        // S[cs][k][comp], cs the structured corner cx + 2 cy
        double S[4][3][2];
#pragma unroll
        for (int cs = 0; cs < 4; ++cs)
#pragma unroll
            for (int k = 0; k < 3; ++k) S[cs][k][0] = S[cs][k][1] = 0.0;
#pragma unroll
        for (int b = 0; b <= n; ++b) {
            float2 w[n + 1];
#pragma unroll
            for (int a = 0; a <= n; ++a) w[a] = ALL ? wall[(b * (n + 1) + a) % (ALL ? nf : 1)] : d2[pm[b * (n + 1) + a]];
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                double s0x = 0.0, s0y = 0.0, s1x = 0.0, s1y = 0.0;
#pragma unroll
                for (int a = 0; a <= n; ++a) {
                    const double a0 = s_A[(0 * 2 + cx) * (n + 1) + a], a1 = s_A[(1 * 2 + cx) * (n + 1) + a];
                    s0x += a0 * (double)w[a].x; s0y += a0 * (double)w[a].y;
                    s1x += a1 * (double)w[a].x; s1y += a1 * (double)w[a].y;
                }
#pragma unroll
                for (int cy = 0; cy < 2; ++cy) {
                    const double y0 = s_A[(0 * 2 + cy) * (n + 1) + b], y1 = s_A[(1 * 2 + cy) * (n + 1) + b];
                    double (&T)[3][2] = S[cx + 2 * cy];
                    T[0][0] += y0 * s0x; T[0][1] += y0 * s0y;
                    T[1][0] += y0 * s1x; T[1][1] += y0 * s1y;
                    T[2][0] += y1 * s0x; T[2][1] += y1 * s0y;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int cs = c ^ (c >> 1);
#pragma unroll
            for (int comp = 0; comp < 2; ++comp) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int ks = k ^ (k >> 1);
                    const double m = g0 * s_M[(0 * 4 + cs) * 4 + ks] + g1 * s_M[(1 * 4 + cs) * 4 + ks] +
                                     g2 * s_M[(2 * 4 + cs) * 4 + ks];
                    acc += m * (double)(comp ? cv[k].y : cv[k].x);
                }
                out[c][comp] = acc + g0 * S[cs][0][comp] + g1 * S[cs][1][comp] + g2 * S[cs][2][comp];
            }
        }
    } else {
        // a curved edge: the stored rows
        const double *W = u.W + (size_t)ci * 4 * nf, *M = u.M4 + 16 * (size_t)ci;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double ax = 0.0, ay = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                ax += M[4 * c + k] * (double)cv[k].x;
                ay += M[4 * c + k] * (double)cv[k].y;
            }
            out[c][0] = ax;
            out[c][1] = ay;
        }
        for (int l = 0; l < nf; ++l) {
            const float2 w = ALL ? wall[l % (ALL ? nf : 1)] : d2[pm[l]];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double r = W[c * nf + l];
                out[c][0] += r * (double)w.x;
                out[c][1] += r * (double)w.y;
            }
        }
    }
    double2 *o = reinterpret_cast<double2 *>(u.part + 8 * (size_t)e);
#pragma unroll
    for (int c = 0; c < 4; ++c) o[c] = make_double2(u.inv_dt64 * out[c][0], u.inv_dt64 * out[c][1]);
}

hipError_t launch_urhs(const UArgs &u, const float *dbar, hipStream_t s)
{
    switch (u.K) {
#define DNNMG_URHS(KK)                                                                                \
    case KK: {                                                                                        \
        hipLaunchKernelGGL(k_urhs<KK>, dim3((u.P + kURhsThreads - 1) / kURhsThreads), dim3(kURhsThreads), 0, s, \
                           u, dbar);                                                                  \
        break;                                                                                        \
    }
        DNNMG_URHS(1)
        DNNMG_URHS(2)
        DNNMG_URHS(3)
#undef DNNMG_URHS
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
