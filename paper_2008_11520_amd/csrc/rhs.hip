// Duplicate averaging, corrected velocity, FP64 right-hand side and restriction.
//
// Per patch E (one coarse element) the kernel
//   1. averages the per-patch network outputs at each of its (n+1)^2 fine
//      nodes over the 1, 2 or 4 patches that contain the node (Sec. 4.2),
//      zeroes Dirichlet nodes, and stores the corrected velocity P v + d as the
//      state for the next defect (the patch that owns a node writes it);
//   2. forms its share of b_L = P^T (1/dt) M_f (P v + d) (Alg. 2, rhs + restriction) at
//      its four corners, in FP64.
// Step 2 uses exact moment tables instead of fine quadrature.  With the
// coarse map F, det J = d0 + d1 xi + d2 eta is affine, so for the coarse hat N_c
// restricted to E
//   int_E N_c (P v) dx = sum_c' v_c' [d0 M0 + d1 M1 + d2 M2]_{c c'}
//   int_E N_c d     dx = sum_l  d_l  [d0 G0 + d1 G1 + d2 G2]_{c l}
// where M_k, G_k integrate N_c N_c' {1, xi, eta} and N_c phi_l {1, xi, eta} on the
// reference square (phi_l the fine Q1 hat of patch node l).  G_k is a tensor
// product of 1D integrals A[m][p][a] = int_0^1 L_p hat_a x^m, so the sums over
// the (n+1)^2 nodes are done as a pass along x then a pass along y.  These are the
// same integrals the fine-level 2 x 2 Gauss rule computes exactly (the
// integrands are polynomials of degree <= 3 per variable on every fine cell),
// and P^T is the evaluation of N_c at fine nodes, so the result equals the
// definition up to FP64 rounding.  A second kernel sums the four patch
// contributions at each coarse node in a fixed order (no atomics).
#include "device.h"
#include "frame.h"
#include "internal.h"

namespace dnnmg {

template <int K>
__device__ inline bool dirichlet_node(unsigned dir, int I, int J, int NX, int NY)
{
    return ((dir & 1u) && I == 0) || ((dir & 2u) && I == NX) || ((dir & 4u) && J == 0) || ((dir & 8u) && J == NY);
}

// The explicit transport term of the theta scheme at the four corners c of
// each patch E, in FP64:
//   T_c = int_E N_c (u . grad u) + nu grad N_c . grad u  dx,  u = P v + d,
// N_c the coarse hat: since the fine Q1 space holds the coarse one, the
// restriction R = P^T of the fine rows T(u) is this integral of the coarse
// hats, taken with the fine elements' 2 x 2 Gauss rule (u is bilinear on each
// fine element, the map F bilinear on E).  Per Gauss point (xi, eta) in E's
// reference square, with Cof = det J^{-T} and w = 1 / (4 n^2):
//   w [ N_c (u_x (Cof grad_ref u)_x + u_y (Cof grad_ref u)_y)
//       + (nu / det) (Cof grad_ref N_c) . (Cof grad_ref u) ].
// One item per (patch, fine element row); the rows of a patch sit on
// neighbouring lanes and are summed with a fixed butterfly.
template <int K>
__device__ __forceinline__ void transport_corners(const FlowArgs &f, int tid, int pi0, int pj0, const float2 *s_v,
                                                  const float2 *s_dbar, double *s_T)
{
    constexpr int n = 1 << K;
    constexpr int TP = kRhsFine / n, NO = kRhsFine + 1;
    constexpr int NI = TP * TP * n;
    static_assert(kThreads % n == 0, "a patch's rows on neighbouring lanes of one wave");
    constexpr double inv_n = 1.0 / n, wq = 0.25 / (n * n);
    constexpr double g0 = 0.21132486540518711775, g1 = 0.78867513459481288225;
    const double nu = f.nu64;
    const int nx = f.nx, ny = f.ny;
    for (int it0 = 0; it0 < NI; it0 += kThreads) {
        const int it = it0 + tid;
        const int b = it % n, pl = it / n;
        const int pa = pl % TP, pb = pl / TP;
        double acc[4][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
        if (it < NI && pi0 + pa < nx && pj0 + pb < ny) {
            const double *m = f.map64 + 8 * ((size_t)(pj0 + pb) * nx + pi0 + pa);
            const double exx = m[0], exy = m[1], eyx = m[2], eyy = m[3], twx = m[4], twy = m[5];
            constexpr int SV = TP + 2;     // the rhs tile's corner layout
            const int c = pb * SV + pa;
            const float2 v00 = s_v[c], v10 = s_v[c + 1], v01 = s_v[c + SV], v11 = s_v[c + SV + 1];
            // u = P v + d at fine node (a, bb) of the patch, FP64
            auto unode = [&](int a, int bb, double &ux, double &uy) {
                const double xi = a * inv_n, eta = bb * inv_n;
                const double n00 = (1.0 - xi) * (1.0 - eta), n10 = xi * (1.0 - eta), n01 = (1.0 - xi) * eta,
                             n11 = xi * eta;
                const float2 d = s_dbar[(pb * n + bb) * NO + pa * n + a];
                ux = n00 * v00.x + n10 * v10.x + n01 * v01.x + n11 * v11.x + (double)d.x;
                uy = n00 * v00.y + n10 * v10.y + n01 * v01.y + n11 * v11.y + (double)d.y;
            };
            double u0x, u0y, u2x, u2y;     // left column of the current element: rows b, b + 1
            unode(0, b, u0x, u0y);
            unode(0, b + 1, u2x, u2y);
#pragma unroll 1
            for (int a = 0; a < n; ++a) {
                double u1x, u1y, u3x, u3y;
                unode(a + 1, b, u1x, u1y);
                unode(a + 1, b + 1, u3x, u3y);
#pragma unroll 1
                for (int q = 0; q < 4; ++q) {
                        const double s = (q & 1) ? g1 : g0, t = (q >> 1) ? g1 : g0;
                        const double xi = (a + s) * inv_n, eta = (b + t) * inv_n;
                        const double xs = exx + twx * eta, ys = exy + twy * eta;
                        const double xt = eyx + twx * xi, yt = eyy + twy * xi;
                        const double det = xs * yt - xt * ys;
                        const double ux = (1.0 - t) * (u0x + (u1x - u0x) * s) + t * (u2x + (u3x - u2x) * s);
                        const double uy = (1.0 - t) * (u0y + (u1y - u0y) * s) + t * (u2y + (u3y - u2y) * s);
                        // coarse-reference derivatives (n times the fine element's)
                        const double usx = n * ((u1x - u0x) * (1.0 - t) + (u3x - u2x) * t);
                        const double usy = n * ((u1y - u0y) * (1.0 - t) + (u3y - u2y) * t);
                        const double utx = n * ((u2x - u0x) * (1.0 - s) + (u3x - u1x) * s);
                        const double uty = n * ((u2y - u0y) * (1.0 - s) + (u3y - u1y) * s);
                        // Cof grad_ref of each component
                        const double gxx = yt * usx - ys * utx, gxy = -xt * usx + xs * utx;
                        const double gyx = yt * usy - ys * uty, gyy = -xt * usy + xs * uty;
                        const double cvx = ux * gxx + uy * gxy, cvy = ux * gyx + uy * gyy;
                        const double nud = nu / det;
                        const double N[4] = {(1.0 - xi) * (1.0 - eta), xi * (1.0 - eta), (1.0 - xi) * eta, xi * eta};
                        const double Ns[4] = {-(1.0 - eta), 1.0 - eta, -eta, eta};
                        const double Nt[4] = {-(1.0 - xi), -xi, 1.0 - xi, xi};
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const double hx = yt * Ns[k] - ys * Nt[k], hy = -xt * Ns[k] + xs * Nt[k];
                            acc[k][0] += wq * (N[k] * cvx + nud * (hx * gxx + hy * gxy));
                            acc[k][1] += wq * (N[k] * cvy + nud * (hx * gyx + hy * gyy));
                        }
                    }
                u0x = u1x; u0y = u1y; u2x = u3x; u2y = u3y;
            }
        }
        // sum over the patch's n rows (lanes it - b .. it - b + n - 1)
#pragma unroll
        for (int off = 1; off < n; off <<= 1)
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int c = 0; c < 2; ++c) acc[k][c] += __shfl_xor(acc[k][c], off);
        if (it < NI && b == 0)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                s_T[8 * pl + 2 * k] = acc[k][0];
                s_T[8 * pl + 2 * k + 1] = acc[k][1];
            }
    }
}

// One workgroup per tile of kRhsFine x kRhsFine fine elements (TP x TP patches).
// FROM_PATCHES = 1: average f.dpatch and store the corrected velocity (the
// step); 2: the same step after the one-launch K = 2 kernel, which has
// averaged every node inside the tile's boundary lines already (frame.h):
// the deep nodes' corrected velocity is read from the state, the frame
// completed here; 0: take the correction from f.dbar_in (stage, state
// untouched).
// CN: the theta scheme's rhs, (1/dt) M u - (1 - theta) T(u), restricted.
// The implicit-Euler step (UB) sums the stored corrected velocity u = P v + d
// against the hat moments: P v is bilinear on the patch, so its fine
// interpolant is itself, and R (1/dt) M u needs no separate coarse term.
// The stage and the theta scheme keep d and the coarse mass term of P v.
template <int K, int FROM_PATCHES, bool OPAQUE_TID, bool CN = false>
__device__ __forceinline__ void rhs_tile(const FlowArgs &f, int blk, RhsTables tab)
{
    static_assert(FROM_PATCHES != 2 || (K == 2 && !CN && !OPAQUE_TID), "tile frame: the one-launch K = 2 step, one tile per block");
    constexpr bool UB = FROM_PATCHES != 0 && !CN;
    const int tid = OPAQUE_TID ? tile_thread() : (int)threadIdx.x;
    constexpr int n = 1 << K;
    constexpr int nf = (n + 1) * (n + 1);
    constexpr int TP = kRhsFine / n;          // patches per tile and direction
    constexpr int HP = TP + 2;                // with a ring of neighbour patches
    constexpr int NO = kRhsFine + 1;          // tile nodes per direction
    constexpr int SV = TP + 2;                // corner velocities: the tile's patches and the next column and row
    constexpr float inv_n = 1.0f / n;
    static_assert(kRhsFine == kFrameLine, "one tile shape for the frame");

    // the staged per-patch outputs (step) and, once the node pass has read
    // them, the averaged correction (or u) at the tile's nodes share one buffer
    constexpr int kStaged = FROM_PATCHES == 1 ? HP * HP * nf : 0;
    __shared__ float2 s_buf[kStaged > NO * NO ? kStaged : NO * NO];
    float2 *const s_dbar = s_buf;
    __shared__ float2 s_v[SV * SV];
    __shared__ double s_A[4 * (n + 1)];
    __shared__ double s_M[3 * 4 * 4];
    __shared__ double2 s_g[2 * TP * TP];
    __shared__ double s_T[CN ? 8 * TP * TP : 1];

    const int nx = f.nx, ny = f.ny, NX = nx * n, NY = ny * n;
    const int tiles_x = (nx + TP - 1) / TP;
    const int tx = blk % tiles_x, ty = blk / tiles_x;
    const int pi0 = tx * TP, pj0 = ty * TP;    // first patch of the tile
    const int I0 = pi0 * n, J0 = pj0 * n;      // first fine node
    // Addresses are formed from the tile's base (uniform, in scalar
    // registers) plus a 32-bit offset per thread.
    const size_t pt0 = (size_t)pj0 * nx + pi0;  // the tile's first patch
    const size_t nt0 = (size_t)J0 * (NX + 1) + I0;   // the tile's first node (rows of NX+1 nodes)
    const int up = f.upitch;                          // u_prev rows: upitch nodes
    float2 *const ut = reinterpret_cast<float2 *>(f.uprev) + (size_t)J0 * up + I0;
    // The step's defect has already read the first-step flag (stream order).
    if (FROM_PATCHES && blk == 0 && tid == 0) *f.first_flag = 0;

    // P v at tile node (li, lj) from the corners of the patch that owns it
    // (the left/lower one: that patch may lie in the next tile column or row)
    auto pv_of = [&](int li, int lj, float &px, float &py) {
        const int I = I0 + li, J = J0 + lj;
        const int pI = min(I >> K, nx - 1), pJ = min(J >> K, ny - 1);
        const int c = (pJ - pj0) * SV + (pI - pi0);
        const float2 v00 = s_v[c], v10 = s_v[c + 1], v01 = s_v[c + SV], v11 = s_v[c + SV + 1];
        const PvRow r = pv_row(v00.x, v00.y, v10.x, v10.y, v01.x, v01.y, v11.x, v11.y, (J - pJ * n) * inv_n);
        pv_at(r, (I - pI * n) * inv_n, px, py);
    };

    // ---- stage: moment tables, coarse corner velocities, the patches' map
    //      determinant coefficients, per-patch outputs (or the tile frame).
    //      Every load is issued into registers before the first LDS store, so
    //      the tile waits for one memory round trip instead of one per table.
    //      The tables are read through pinned pointers: in the batched tile
    //      loop their loads would otherwise be hoisted and held in registers.
    const gptr<double> tabA = pinned<double>(tab.A), tabM = pinned<double>(tab.M);
    constexpr int NA = 4 * (n + 1), NM = 3 * 4 * 4, NV = SV * SV, NG = 2 * TP * TP;
    static_assert(NA + NM <= kThreads, "one table entry per thread");
    constexpr int VIT = (NV + kThreads - 1) / kThreads, GIT = (NG + kThreads - 1) / kThreads;
    // (the addresses are clamped into the arrays and the loads made
    // unconditionally: a load under a condition is waited for at once)
    const double tabA_r = tabA[min(tid, NA - 1)], tabM_r = tabM[min(max(tid - NA, 0), NM - 1)];
    const float2 *vt = reinterpret_cast<const float2 *>(f.v) + (size_t)pj0 * (nx + 1) + pi0;
    const double2 *gt = reinterpret_cast<const double2 *>(f.geo64) + 2 * pt0;
    float2 v_r[VIT];
    double2 g_r[GIT];
#pragma unroll
    for (int i = 0; i < VIT; ++i) {
        const int t = min(tid + i * kThreads, NV - 1);
        const int ci = min(t % SV, nx - pi0), cj = min(t / SV, ny - pj0);
        v_r[i] = vt[cj * (nx + 1) + ci];
    }
#pragma unroll
    for (int i = 0; i < GIT; ++i) {
        // (d0, d1) and (d2, pad) of patch t / 2 of the tile
        const int t = min(tid + i * kThreads, NG - 1), pl = t >> 1;
        const int pa = min(pl % TP, nx - 1 - pi0), pb = min(pl / TP, ny - 1 - pj0);
        g_r[i] = gt[2 * (pb * nx + pa) + (t & 1)];
    }
    // tile frame (FROM_PATCHES = 2): the deep nodes' u (li, lj in 2 .. kRhsFine - 2),
    // the inner nodes' averaged d (threads < INNER) and, on the threads from
    // kThreads - EDGES on, the outputs of every patch at one boundary-line node
    typedef TileFrame<K> FR;
    constexpr int DN = kRhsFine - 3, ND = DN * DN;
    constexpr int DIT = FROM_PATCHES == 2 ? (ND + kThreads - 1) / kThreads : 1;
    static_assert(FROM_PATCHES != 2 || FR::INNER <= kThreads - FR::EDGES, "inner and edge nodes on separate threads");
    float2 du[DIT];
    float2 fin = make_float2(0.f, 0.f);
    float2 fq[4];
    if constexpr (FROM_PATCHES == 2) {
        const float2 *fr = reinterpret_cast<const float2 *>(f.frame);
#pragma unroll
        for (int i = 0; i < DIT; ++i) {
            // (a tile holds at least one patch: NX - I0, NY - J0 >= n >= 2)
            const int t = min(tid + i * kThreads, ND - 1);
            const int li = min(2 + t % DN, NX - I0), lj = min(2 + t / DN, NY - J0);
            du[i] = ut[lj * up + li];
        }
        if (tid < FR::INNER) fin = fr[(size_t)blk * FR::SIZE + 4 * FR::SIDE + tid];
        if (tid >= kThreads - FR::EDGES) {
            int li, lj;
            FR::edge_pos(tid - (kThreads - FR::EDGES), li, lj);
            const int I = I0 + li, J = J0 + lj;
            long o[4] = {0, 0, 0, 0};
            if (I <= NX && J <= NY) {
                // the node's patches in row-major order: lower left, lower,
                // left, own (own: the left/lower-owner patch of the node)
                const int pI = min(I >> K, nx - 1), pJ = min(J >> K, ny - 1);
                const int a = I - pI * n, b = J - pJ * n;
                const bool lft = a == 0 && pI > 0, low = b == 0 && pJ > 0;
                o[3] = FR::contrib(nx, pI, pJ, a, b);
                o[0] = lft && low ? FR::contrib(nx, pI - 1, pJ - 1, n, n) : o[3];
                o[1] = low ? FR::contrib(nx, pI, pJ - 1, a, n) : o[3];
                o[2] = lft ? FR::contrib(nx, pI - 1, pJ, n, b) : o[3];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) fq[q] = fr[o[q] < 0 ? 0 : o[q]];
        }
    }
    if constexpr (FROM_PATCHES == 1) {
        // per-patch outputs, 8 bytes at a time, into the staged (TP+2)^2-patch
        // layout: the tile's own patches whole (each tile row of TP patches is
        // one contiguous run of TP nf nodes), and of the ring of neighbours only
        // the nodes on the edges the tile touches (right edges of the left
        // column, left edges of the right column, top edges of the row below,
        // bottom edges of the row above, one node of each diagonal patch); the
        // rest of the ring is never read.  All of a thread's loads are issued
        // before any LDS store.
        constexpr int RW = TP * nf, NS = TP * RW, IT = (NS + kThreads - 1) / kThreads;
        constexpr int NR = 4 * TP * (n + 1) + 4;
        static_assert(NR <= kThreads, "one ring node per thread");
        float2 *sd2 = s_buf;
        const float2 *dt2 = reinterpret_cast<const float2 *>(f.dpatch) + pt0 * nf;
        const int prow = nx * nf;                  // nodes per patch row of the mesh
        const int npr = min(TP, nx - pi0), nrows = min(TP, ny - pj0);
        // With nx even and the tile full in x, every row starts on a 16-byte
        // boundary and holds an even number of nodes: 16 bytes per load.
        const bool wide = (nx & 1) == 0 && npr == TP;
        constexpr int RW4 = RW / 2, NS4 = TP * RW4, IT4 = (NS4 + kThreads - 1) / kThreads;
        static_assert(RW % 2 == 0, "whole 16-byte pieces per tile row");
        float2 tmp[IT];
        float4 tmp4[IT4];
        if (wide) {
            const float4 *dt4 = reinterpret_cast<const float4 *>(dt2);
#pragma unroll
            for (int i = 0; i < IT4; ++i) {
                const int t = tid + i * kThreads;
                const int r = t / RW4, k = t - r * RW4;
                tmp4[i] = (t < NS4 && r < nrows) ? dt4[r * (prow / 2) + k] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        } else {
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const int t = tid + i * kThreads;
                const int r = t / RW, k = t - r * RW;
                tmp[i] = (t < NS && r < nrows && k < npr * nf) ? dt2[r * prow + k] : make_float2(0.f, 0.f);
            }
        }
        float2 ring = make_float2(0.f, 0.f);
        int rdst = -1;
        if (tid < NR) {
            const int side = tid / (TP * (n + 1)), sidx = tid - side * (TP * (n + 1));
            const int r = sidx / (n + 1), m = sidx - r * (n + 1);
            int qi, qj, a, b;
            switch (side) {
            case 0: qi = -1; qj = r; a = n; b = m; break;         // left column: right edges
            case 1: qi = TP; qj = r; a = 0; b = m; break;         // right column: left edges
            case 2: qi = r; qj = -1; a = m; b = n; break;         // row below: top edges
            case 3: qi = r; qj = TP; a = m; b = 0; break;         // row above: bottom edges
            default:                                              // diagonal patches: one corner each
                qi = (sidx & 1) ? TP : -1; qj = (sidx & 2) ? TP : -1;
                a = (sidx & 1) ? 0 : n; b = (sidx & 2) ? 0 : n;
            }
            const int gi = pi0 + qi, gj = pj0 + qj;
            if (gi >= 0 && gi < nx && gj >= 0 && gj < ny) {
                ring = dt2[(qj * nx + qi) * nf + b * (n + 1) + a];
                rdst = ((qj + 1) * HP + qi + 1) * nf + b * (n + 1) + a;
            }
        }
        if (wide) {
#pragma unroll
            for (int i = 0; i < IT4; ++i) {
                const int t = tid + i * kThreads;
                const int r = t / RW4, k = t - r * RW4;
                if (t < NS4) {
                    float2 *d = sd2 + ((r + 1) * HP + 1) * nf + 2 * k;
                    d[0] = make_float2(tmp4[i].x, tmp4[i].y);
                    d[1] = make_float2(tmp4[i].z, tmp4[i].w);
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const int t = tid + i * kThreads;
                const int r = t / RW, k = t - r * RW;
                if (t < NS) sd2[((r + 1) * HP + 1) * nf + k] = tmp[i];
            }
        }
        if (rdst >= 0) sd2[rdst] = ring;
    }
    if (tid < NA) s_A[tid] = tabA_r;
    else if (tid < NA + NM) s_M[tid - NA] = tabM_r;
#pragma unroll
    for (int i = 0; i < VIT; ++i) {
        // corners beyond the mesh (tiles at its end) hold zeros
        const int t = tid + i * kThreads;
        if (t < NV) s_v[t] = (pi0 + t % SV <= nx && pj0 + t / SV <= ny) ? v_r[i] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < GIT; ++i)
        if (tid + i * kThreads < NG) s_g[tid + i * kThreads] = g_r[i];
    if constexpr (FROM_PATCHES == 2) {
#pragma unroll
        for (int i = 0; i < DIT; ++i) {
            const int t = tid + i * kThreads;
            const int li = 2 + t % DN, lj = 2 + t / DN;
            if (t < ND && I0 + li <= NX && J0 + lj <= NY) s_dbar[lj * NO + li] = du[i];
        }
    }
    __syncthreads();

    // ---- node pass: mean over the containing patches (row-major order, as
    //      the mean is defined), Dirichlet mask, corrected velocity.
    const float2 *sd2 = s_buf;
    // Any tile node (li, lj); the patch offsets are those of the staged ring.
    // Returns the node's averaged correction and sets u to the corrected
    // velocity (the step).  nonfin: this thread has averaged a correction
    // that is not finite (the step's non-finite check).
    bool nonfin = false;
    auto node = [&](int li, int lj, float2 &u) -> float2 {
        const int I = I0 + li, J = J0 + lj;
        float2 d = make_float2(0.f, 0.f);
        u = d;
        if (I <= NX && J <= NY) {
            if (FROM_PATCHES == 1) {
                // the node's own (left/lower-owner) patch, plus the patches to the
                // left, below and diagonal when the node lies on their edges;
                // summed in row-major patch order
                const int pI = min(I >> K, nx - 1), pJ = min(J >> K, ny - 1);
                const int a = I - pI * n, b = J - pJ * n;
                const bool lft = a == 0 && pI > 0, low = b == 0 && pJ > 0;
                const int hb = (pJ - pj0 + 1) * HP + (pI - pi0 + 1);   // own patch in the staged ring
                float2 acc = make_float2(0.f, 0.f);
                if (lft && low) { const float2 q = sd2[(hb - HP - 1) * nf + n * (n + 1) + n]; acc.x += q.x; acc.y += q.y; }
                if (low) { const float2 q = sd2[(hb - HP) * nf + n * (n + 1) + a]; acc.x += q.x; acc.y += q.y; }
                if (lft) { const float2 q = sd2[(hb - 1) * nf + b * (n + 1) + n]; acc.x += q.x; acc.y += q.y; }
                { const float2 q = sd2[hb * nf + b * (n + 1) + a]; acc.x += q.x; acc.y += q.y; }
                const float inv = (lft && low) ? 0.25f : ((lft || low) ? 0.5f : 1.0f);
                d = make_float2(acc.x * inv, acc.y * inv);
                if (dirichlet_node<K>(f.dirichlet, I, J, NX, NY)) d = make_float2(0.f, 0.f);
                nonfin |= !(__builtin_isfinite(d.x) && __builtin_isfinite(d.y));
                float px, py;
                pv_of(li, lj, px, py);
                u = make_float2(px + d.x, py + d.y);
                const bool owned = (li < kRhsFine || I == NX) && (lj < kRhsFine || J == NY);
                if (owned) {
                    ut[lj * up + li] = u;
                    if (f.dbar_out) (reinterpret_cast<float2 *>(f.dbar_out) + nt0)[lj * (NX + 1) + li] = d;
                }
            } else if (FROM_PATCHES == 0) {
                d = (reinterpret_cast<const float2 *>(f.dbar_in) + nt0)[lj * (NX + 1) + li];
            }
        }
        return d;
    };
    if constexpr (FROM_PATCHES == 0) {
        float2 u;
        for (int t = tid; t < NO * NO; t += kThreads) s_dbar[t] = node(t % NO, t / NO, u);
    } else if constexpr (FROM_PATCHES == 2) {
        // the frame: inner nodes take the averaged d handed over, edge nodes
        // average their patches' outputs; both store u = P v + d where they own
        // the node and put u where the FP64 pass reads it (the deep nodes' u
        // is there already)
        float2 *const dout = f.dbar_out ? reinterpret_cast<float2 *>(f.dbar_out) + nt0 : nullptr;
        if (tid < FR::INNER) {
            int li, lj;
            FR::inner_pos(tid, li, lj);
            if (I0 + li <= NX && J0 + lj <= NY) {
                float px, py;
                pv_of(li, lj, px, py);
                const float2 u = make_float2(px + fin.x, py + fin.y);
                ut[lj * up + li] = u;
                if (dout) dout[lj * (NX + 1) + li] = fin;
                s_dbar[lj * NO + li] = u;
            }
        } else if (tid >= kThreads - FR::EDGES) {
            int li, lj;
            FR::edge_pos(tid - (kThreads - FR::EDGES), li, lj);
            const int I = I0 + li, J = J0 + lj;
            if (I <= NX && J <= NY) {
                const int pI = min(I >> K, nx - 1), pJ = min(J >> K, ny - 1);
                const bool lft = I - pI * n == 0 && pI > 0, low = J - pJ * n == 0 && pJ > 0;
                float2 acc = make_float2(0.f, 0.f);
                if (lft && low) { acc.x += fq[0].x; acc.y += fq[0].y; }
                if (low) { acc.x += fq[1].x; acc.y += fq[1].y; }
                if (lft) { acc.x += fq[2].x; acc.y += fq[2].y; }
                acc.x += fq[3].x; acc.y += fq[3].y;
                const float inv = (lft && low) ? 0.25f : ((lft || low) ? 0.5f : 1.0f);
                float2 d = make_float2(acc.x * inv, acc.y * inv);
                if (dirichlet_node<K>(f.dirichlet, I, J, NX, NY)) d = make_float2(0.f, 0.f);
                nonfin |= !(__builtin_isfinite(d.x) && __builtin_isfinite(d.y));
                float px, py;
                pv_of(li, lj, px, py);
                const float2 u = make_float2(px + d.x, py + d.y);
                if ((li < kRhsFine || I == NX) && (lj < kRhsFine || J == NY)) {
                    ut[lj * up + li] = u;
                    if (dout) dout[lj * (NX + 1) + li] = d;
                }
                s_dbar[lj * NO + li] = u;
            }
        }
        if (nonfin && f.nonfinite) atomicOr(f.nonfinite, 1);
    } else {
        // the corrections (or u) are kept in registers until every thread is
        // done reading the staged outputs, then written over them
        constexpr int OIT = (TP * TP * n + kThreads - 1) / kThreads;
        float2 dreg[OIT][n];
        int dpos[OIT];
        float2 dlast = make_float2(0.f, 0.f);
        int lpos = -1;
        // the nodes (a, b), a, b < n, of the tile's own patches, one node row of
        // one patch per item: the same sums as node() with the patch known
        // (a node with I < NX, J < NY is masked only on the sides I = 0, J = 0)
        const unsigned dir = f.dirichlet;
#pragma unroll
        for (int o = 0; o < OIT; ++o) {
            const int it = tid + o * kThreads;
            dpos[o] = -1;
            const int pl = it % (TP * TP), b = it / (TP * TP);
            const int pa = pl % TP, pb = pl / TP, pi = pi0 + pa, pj = pj0 + pb;
            if (it >= TP * TP * n || pi >= nx || pj >= ny) continue;
            dpos[o] = (pb * n + b) * NO + pa * n;
            const int hb = (pb + 1) * HP + pa + 1;
            const bool low = b == 0 && pj > 0;
            const bool mrow = (dir & 4u) && pj == 0 && b == 0, mcol = (dir & 1u) && pi == 0;
            // P v along the node row (the patch owns these nodes)
            const int c = pb * SV + pa;
            const float2 v00 = s_v[c], v10 = s_v[c + 1], v01 = s_v[c + SV], v11 = s_v[c + SV + 1];
            const PvRow row = pv_row(v00.x, v00.y, v10.x, v10.y, v01.x, v01.y, v11.x, v11.y, b * inv_n);
            float2 *const urow = ut + (pb * n + b) * up + pa * n;
            float2 *const drow = f.dbar_out ? reinterpret_cast<float2 *>(f.dbar_out) + nt0 + (pb * n + b) * (NX + 1) + pa * n
                                            : nullptr;
#pragma unroll
            for (int a = 0; a < n; ++a) {
                const bool lft = a == 0 && pi > 0;
                float2 acc = make_float2(0.f, 0.f);
                if (lft && low) { const float2 q = sd2[(hb - HP - 1) * nf + n * (n + 1) + n]; acc.x += q.x; acc.y += q.y; }
                if (low) { const float2 q = sd2[(hb - HP) * nf + n * (n + 1) + a]; acc.x += q.x; acc.y += q.y; }
                if (lft) { const float2 q = sd2[(hb - 1) * nf + b * (n + 1) + n]; acc.x += q.x; acc.y += q.y; }
                { const float2 q = sd2[hb * nf + b * (n + 1) + a]; acc.x += q.x; acc.y += q.y; }
                const float inv = (lft && low) ? 0.25f : ((lft || low) ? 0.5f : 1.0f);
                float2 d = make_float2(acc.x * inv, acc.y * inv);
                if (mrow || (a == 0 && mcol)) d = make_float2(0.f, 0.f);
                nonfin |= !(__builtin_isfinite(d.x) && __builtin_isfinite(d.y));
                float px, py;
                pv_at(row, a * inv_n, px, py);
                const float2 u = make_float2(px + d.x, py + d.y);
                urow[a] = u;
                if (drow) drow[a] = d;
                dreg[o][a] = UB ? u : d;
            }
        }
        // the rest: the last node column and row of the tile's patches (the
        // tile's own last column and row, or the mesh end inside the tile)
        const int le = min(TP, nx - pi0) * n, me = min(TP, ny - pj0) * n;
        static_assert(2 * kRhsFine + 1 <= kThreads, "one last-row/column node per thread");
        if (tid < le + me + 1) {
            const int li = tid <= me ? le : tid - me - 1, lj = tid <= me ? tid : me;
            float2 u;
            const float2 d = node(li, lj, u);
            dlast = UB ? u : d;
            lpos = lj * NO + li;
        }
        __syncthreads();
#pragma unroll
        for (int o = 0; o < OIT; ++o)
            if (dpos[o] >= 0) {
#pragma unroll
                for (int a = 0; a < n; ++a) s_dbar[dpos[o] + a] = dreg[o][a];
            }
        if (lpos >= 0) s_dbar[lpos] = dlast;
        if (nonfin && f.nonfinite) atomicOr(f.nonfinite, 1);
    }
    __syncthreads();
    if constexpr (CN) {
        transport_corners<K>(f, tid, pi0, pj0, s_v, s_dbar, s_T);
        __syncthreads();
    }
    const double th_old = CN ? 1.0 - (double)f.theta : 0.0;

    // ---- FP64 share of each patch at each of its 4 corners c = (cx, cy):
    //      (1/dt) sum_k d_k sum_{a,b} A[mx_k][cx][a] A[my_k][cy][b] w(a,b),
    //      w = u (the step), or w = Dbar plus the coarse term
    //      (1/dt) sum_c' (d0 M0 + d1 M1 + d2 M2)[c][c'] v_c' (stage, theta scheme).
    //      One item per (patch, component, cx): the x pass T_m(b) = sum_a A[m][cx][a] w(a,b)
    //      and the y pass for both cy (the four items of a patch on
    //      neighbouring lanes read neighbouring LDS words).
    const float *dbar1 = reinterpret_cast<const float *>(s_dbar);
    const size_t P = (size_t)nx * ny;
    double *const pt = f.part + 2 * pt0;
    for (int it = tid; it < TP * TP * 4; it += kThreads) {
        const int cx = it & 1, comp = (it >> 1) & 1, pl = it >> 2;
        const int pi = pi0 + pl % TP, pj = pj0 + pl / TP;
        if (pi >= nx || pj >= ny) continue;
        const double2 g01 = s_g[2 * pl], g2x = s_g[2 * pl + 1];
        const double d0 = g01.x, d1 = g01.y, d2 = g2x.x;
        const int bi = (pl % TP) * n, bj = (pl / TP) * n;
        // x pass of node row b, then its terms of the y pass for both cy.  With
        // 8 or more patches per tile row (K <= 2) the two patch rows one wave
        // holds start their walk over the node rows one row apart, so that at
        // each step their reads fall in different LDS banks (patch rows lie a
        // multiple of 64 banks apart).  (At K = 3 the rotation's run-time row
        // index cost more than the conflicts it removed.)
        constexpr int RR = TP >= 8 ? 2 : 1;
        const int rot = (pl / TP) % RR;
        double S[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
#pragma unroll
        for (int b0 = 0; b0 <= n; ++b0) {
            const int b = b0 + rot > n ? b0 + rot - (n + 1) : b0 + rot;
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int a = 0; a <= n; ++a) {
                const double dv = (double)dbar1[2 * ((bj + b) * NO + bi + a) + comp];
                s0 += s_A[(0 * 2 + cx) * (n + 1) + a] * dv;
                s1 += s_A[(1 * 2 + cx) * (n + 1) + a] * dv;
            }
#pragma unroll
            for (int cy = 0; cy < 2; ++cy) {
                const double ay0 = s_A[(0 * 2 + cy) * (n + 1) + b], ay1 = s_A[(1 * 2 + cy) * (n + 1) + b];
                S[cy][0] += ay0 * s0;
                S[cy][1] += ay0 * s1;
                S[cy][2] += ay1 * s0;
            }
        }
        // this item's entry in corner plane cx (plane c = cx + 2 cy holds P pairs)
        double *const pq = pt + 2 * (size_t)cx * P + 2 * ((pl / TP) * nx + pl % TP) + comp;
        const int cb = (pl / TP) * SV + (pl % TP);
        const float *v1 = reinterpret_cast<const float *>(s_v);
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
            const double S0 = S[cy][0], S1 = S[cy][1], S2 = S[cy][2];
            const int c = cx + 2 * cy;
            double acc = d0 * S0 + d1 * S1 + d2 * S2;
            if constexpr (!UB) {
                const double vq[4] = {(double)v1[2 * cb + comp], (double)v1[2 * (cb + 1) + comp],
                                      (double)v1[2 * (cb + SV) + comp], (double)v1[2 * (cb + SV + 1) + comp]};
#pragma unroll
                for (int cc = 0; cc < 4; ++cc) {
                    const double w = d0 * s_M[(0 * 4 + c) * 4 + cc] + d1 * s_M[(1 * 4 + c) * 4 + cc] +
                                     d2 * s_M[(2 * 4 + c) * 4 + cc];
                    acc += w * vq[cc];
                }
            }
            double b = f.inv_dt64 * acc;
            if constexpr (CN) b -= th_old * s_T[8 * pl + 2 * c + comp];
            pq[4 * cy * P] = b;
        }
    }
}

// Single flow: one tile per block.  Batched: the blocks stride over the
// table's tiles of all flows, so the grid need not match the batch.
// Waves per SIMD the rhs aims at (what its LDS allows; register budget 512 /
// waves; the batched K = 3 instance needs more registers than 5 waves leave).
template <int K, bool BATCHED>
constexpr int rhs_waves() { return K == 2 ? 6 : (K == 3 && !BATCHED ? 5 : 4); }

// The theta scheme (Crank-Nicolson), single flow.
template <int K, int FROM_PATCHES>
__global__ __launch_bounds__(kThreads, 3) void k_rhs_cn(FlowArgs single, RhsTables tab)
{
    rhs_tile<K, FROM_PATCHES, false, true>(single, xcd_tile(blockIdx.x, gridDim.x), tab);
}

template <int K, int FROM_PATCHES, bool BATCHED>
__global__ __launch_bounds__(kThreads, (rhs_waves<K, BATCHED>())) void k_rhs(FlowArgs single, const BatchTable *__restrict__ bt, RhsTables tab)
{
    if constexpr (!BATCHED) {
        rhs_tile<K, FROM_PATCHES, false>(single, xcd_tile(blockIdx.x, gridDim.x), tab);
    } else if constexpr (FROM_PATCHES == 2 || K == 3) {
        // after the batched one-launch tiles, and at K = 3: one tile per
        // block, with the single-flow tile code
        const int total = bt->prefix[kKindRhs][bt->nflows];
        if ((int)blockIdx.x >= total) return;
        int blk = xcd_tile(blockIdx.x, total);
        const FlowArgs &f = *batch_flow(bt, kKindRhs, blk);
        rhs_tile<K, FROM_PATCHES, false>(f, blk, tab);
    } else {
        const int total = bt->prefix[kKindRhs][bt->nflows];
#pragma unroll 1
        for (int g = blockIdx.x; g < total; g += gridDim.x) {
            int blk = xcd_tile(g, total);
            const FlowArgs &f = *batch_flow(bt, kKindRhs, blk);
            rhs_tile<K, FROM_PATCHES, true>(f, blk, tab);
            __syncthreads();   // LDS is reused by the next tile
        }
    }
}

// b_L at coarse node (i,j): the node is corner 11 of patch (i-1,j-1), corner 01
// of (i,j-1), corner 10 of (i-1,j) and corner 00 of (i,j); summed in that order.
__device__ __forceinline__ void gather_tile(const FlowArgs &f, int blk)
{
    const int nx = f.nx, ny = f.ny;
    const int t = blk * kThreads + threadIdx.x;
    if (t >= (nx + 1) * (ny + 1)) return;
    const int i = t % (nx + 1), j = t / (nx + 1);
    // partials are stored as four corner planes of P (x, y) pairs
    const double2 *pl = reinterpret_cast<const double2 *>(f.part);
    const size_t P = (size_t)nx * ny;
    double bx = 0.0, by = 0.0;
    if (i > 0 && j > 0) { const double2 q = pl[3 * P + (size_t)(j - 1) * nx + i - 1]; bx += q.x; by += q.y; }
    if (i < nx && j > 0) { const double2 q = pl[2 * P + (size_t)(j - 1) * nx + i]; bx += q.x; by += q.y; }
    if (i > 0 && j < ny) { const double2 q = pl[1 * P + (size_t)j * nx + i - 1]; bx += q.x; by += q.y; }
    if (i < nx && j < ny) { const double2 q = pl[(size_t)j * nx + i]; bx += q.x; by += q.y; }
    reinterpret_cast<double2 *>(f.bL)[t] = make_double2(bx, by);
    if (f.nonfinite && !(__builtin_isfinite(bx) && __builtin_isfinite(by))) atomicOr(f.nonfinite, 2);
}

// Single flow: one tile per block.  Batched: the blocks stride over the
template <bool BATCHED>
__global__ __launch_bounds__(kThreads) void k_gather(FlowArgs single, const BatchTable *__restrict__ bt)
{
    if (!BATCHED) {
        gather_tile(single, blockIdx.x);
        return;
    }
    const int total = bt->prefix[kKindGather][bt->nflows];
#pragma unroll 1
    for (int g = blockIdx.x; g < total; g += gridDim.x) {
        int blk = g;
        const FlowArgs &f = *batch_flow(bt, kKindGather, blk);
        gather_tile(f, blk);
    }
}

hipError_t launch_rhs(const FlowArgs &f, const BatchTable *bt, int nblocks, int K, const RhsTables &tab,
                      int from_patches, hipStream_t s)
{
    if (bt && !from_patches) return hipErrorInvalidValue;   // batched launches are whole steps
    const bool cn = f.theta != 1.0f;
    if (cn && (bt || !f.map64)) return hipErrorInvalidValue;
    dim3 g(nblocks), b(kThreads);
    if (from_patches == 2 || (from_patches && f.frame)) {
        // after the one-launch K = 2 step: a single flow (f.frame), or a batch
        // whose flows all have their tile frame (from_patches = 2; one tile
        // per block, nblocks at least the table's tiles)
        if (K != 2 || cn || (!bt && !f.frame)) return hipErrorInvalidValue;
        if (bt) hipLaunchKernelGGL((k_rhs<2, 2, true>), g, b, 0, s, f, bt, tab);
        else hipLaunchKernelGGL((k_rhs<2, 2, false>), g, b, 0, s, f, bt, tab);
        return hipGetLastError();
    }
#define DNNMG_RHS_CASE(KK)                                                                \
    case KK:                                                                              \
        if (cn && from_patches) hipLaunchKernelGGL((k_rhs_cn<KK, 1>), g, b, 0, s, f, tab); \
        else if (cn) hipLaunchKernelGGL((k_rhs_cn<KK, 0>), g, b, 0, s, f, tab);           \
        else if (bt) hipLaunchKernelGGL((k_rhs<KK, 1, true>), g, b, 0, s, f, bt, tab);    \
        else if (from_patches) hipLaunchKernelGGL((k_rhs<KK, 1, false>), g, b, 0, s, f, bt, tab); \
        else hipLaunchKernelGGL((k_rhs<KK, 0, false>), g, b, 0, s, f, bt, tab);           \
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

__global__ void k_moment_tables(int K, double *A, double *M)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) fill_moment_tables(K, A, M);
}

hipError_t launch_moment_tables(int K, double *A, double *M, hipStream_t s)
{
    if (K < 1 || K > 3) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_moment_tables, dim3(1), dim3(64), 0, s, K, A, M);
    return hipGetLastError();
}

hipError_t launch_gather(const FlowArgs &f, const BatchTable *bt, int nblocks, hipStream_t s)
{
    if (bt) hipLaunchKernelGGL(k_gather<true>, dim3(nblocks), dim3(kThreads), 0, s, f, bt);
    else hipLaunchKernelGGL(k_gather<false>, dim3(nblocks), dim3(kThreads), 0, s, f, bt);
    return hipGetLastError();
}

}  // namespace dnnmg
