// Create-time geometry, prolongation and the fine Navier-Stokes defect on gfx950.
//
// Defect (momentum rows of the nonlinear residual of Eq. (nonlinearshort),
// implicit-Euler form, Q1/Q1):
//   D_a,c = sum_e sum_q w_q |det J_q| [ (1/dt) phi_a (u_prev - v)_c - phi_a (v.grad v_c)
//                                       - nu grad phi_a . grad v_c + p d_c phi_a ]
// evaluated on the prolongated coarse fields v = P v_L, p = P p_L (Alg. 2,
// line 6) and zeroed at Dirichlet nodes.  One workgroup owns a 16 x 16 tile of
// fine elements plus a ring of one halo element, so that the nodes on the tile
// border get every element contribution without global atomics; element
// residuals go to LDS and are summed per node in a fixed order (bitwise
// deterministic).  The tile also writes the network input rows of its patches.
//
// Fine-element geometry is taken from the coarse element's bilinear map
// F(xi,eta) = c00 + ex xi + ey eta + exy xi eta (edge vectors formed in FP64 at
// create time), so Jacobians keep full FP32 relative precision even when the
// absolute coordinates are large compared with the fine mesh width.
#include "internal.h"

namespace dnnmg {

// ---------------------------------------------------------------- geometry
// Per coarse element: FP32 map vectors for the defect, FP64 coefficients of
// det J = d0 + d1 xi + d2 eta for the right-hand side, and the four patch
// features hx, hy, hx/hy, area.  *bad is set if an element is not positively
// oriented (det J <= 0 at a corner).
__global__ __launch_bounds__(kThreads) void k_geometry(const double *__restrict__ cxy, int nx, int ny,
                                                       float *__restrict__ geo, double *__restrict__ geo64,
                                                       float *__restrict__ feat, int *__restrict__ bad)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nx * ny) return;
    int i = e % nx, j = e / nx;
    const double *c00 = cxy + 2 * (j * (nx + 1) + i);
    const double *c10 = c00 + 2;
    const double *c01 = c00 + 2 * (nx + 1);
    const double *c11 = c01 + 2;
    double exx = c10[0] - c00[0], exy_ = c10[1] - c00[1];
    double eyx = c01[0] - c00[0], eyy = c01[1] - c00[1];
    double twx = c11[0] - c10[0] - c01[0] + c00[0], twy = c11[1] - c10[1] - c01[1] + c00[1];
    float *g = geo + 6 * (size_t)e;
    g[0] = (float)exx; g[1] = (float)exy_;
    g[2] = (float)eyx; g[3] = (float)eyy;
    g[4] = (float)twx; g[5] = (float)twy;
    double d0 = exx * eyy - exy_ * eyx;      // ex x ey
    double d1 = exx * twy - exy_ * twx;      // ex x exy
    double d2 = twx * eyy - twy * eyx;       // exy x ey
    double *g64 = geo64 + 4 * (size_t)e;
    g64[0] = d0; g64[1] = d1; g64[2] = d2; g64[3] = 0.0;
    if (!(d0 > 0.0 && d0 + d1 > 0.0 && d0 + d2 > 0.0 && d0 + d1 + d2 > 0.0)) *bad = 1;
    double hx = 0.5 * (hypot(exx, exy_) + hypot(c11[0] - c01[0], c11[1] - c01[1]));
    double hy = 0.5 * (hypot(eyx, eyy) + hypot(c11[0] - c10[0], c11[1] - c10[1]));
    double ax = c11[0] - c00[0], ay = c11[1] - c00[1];
    double bx = c01[0] - c10[0], by = c01[1] - c10[1];
    float *f = feat + 4 * (size_t)e;
    f[0] = (float)hx; f[1] = (float)hy; f[2] = (float)(hx / hy); f[3] = (float)(0.5 * fabs(ax * by - ay * bx));
}

hipError_t launch_geometry(const double *cxy, int nx, int ny, float *geo, double *geo64, float *feat,
                           int *bad, hipStream_t s)
{
    int P = nx * ny;
    hipLaunchKernelGGL(k_geometry, dim3((P + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                       cxy, nx, ny, geo, geo64, feat, bad);
    return hipGetLastError();
}

// ------------------------------------------------------------ prolongation
// Bilinear interpolation of the coarse corner values of the element that
// holds fine node (I,J) (Alg. 2, line 6).
template <int K>
__device__ inline void prolong_node(const float *__restrict__ v, const float *__restrict__ p, int nx, int ny,
                                    int I, int J, float &vx, float &vy, float &pp)
{
    constexpr int n = 1 << K;
    int i = min(I >> K, nx - 1), a = I - i * n;
    int j = min(J >> K, ny - 1), b = J - j * n;
    float xi = a * (1.0f / n), eta = b * (1.0f / n);
    float n00 = (1.0f - xi) * (1.0f - eta), n10 = xi * (1.0f - eta), n01 = (1.0f - xi) * eta, n11 = xi * eta;
    int c = j * (nx + 1) + i;
    const float2 *v2 = reinterpret_cast<const float2 *>(v);
    float2 v00 = v2[c], v10 = v2[c + 1], v01 = v2[c + nx + 1], v11 = v2[c + nx + 2];
    vx = n00 * v00.x + n10 * v10.x + n01 * v01.x + n11 * v11.x;
    vy = n00 * v00.y + n10 * v10.y + n01 * v01.y + n11 * v11.y;
    pp = p ? n00 * p[c] + n10 * p[c + 1] + n01 * p[c + nx + 1] + n11 * p[c + nx + 2] : 0.0f;
}

template <int K>
__global__ __launch_bounds__(kThreads) void k_prolong(FlowArgs f, float *__restrict__ pv, float *__restrict__ pp)
{
    constexpr int n = 1 << K;
    int NX = f.nx * n, NY = f.ny * n;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (NX + 1) * (NY + 1)) return;
    int I = t % (NX + 1), J = t / (NX + 1);
    float vx, vy, q;
    prolong_node<K>(f.v, f.p, f.nx, f.ny, I, J, vx, vy, q);
    if (pv) { pv[2 * t] = vx; pv[2 * t + 1] = vy; }
    if (pp) pp[t] = q;
}

hipError_t launch_prolong(const FlowArgs &f, int K, float *pv, float *pp, hipStream_t s)
{
    int n = 1 << K;
    int Fn = (f.nx * n + 1) * (f.ny * n + 1);
    dim3 g((Fn + kThreads - 1) / kThreads), b(kThreads);
    switch (K) {
    case 1: hipLaunchKernelGGL(k_prolong<1>, g, b, 0, s, f, pv, pp); break;
    case 2: hipLaunchKernelGGL(k_prolong<2>, g, b, 0, s, f, pv, pp); break;
    case 3: hipLaunchKernelGGL(k_prolong<3>, g, b, 0, s, f, pv, pp); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ defect
// Two-point Gauss abscissae on [0,1]: 1/2 -+ 1/(2 sqrt 3).
__device__ constexpr float kG0 = 0.21132486540518711775f;
__device__ constexpr float kG1 = 0.78867513459481288225f;

int blocks_for(int kind, int nx, int ny, int K)
{
    int n = 1 << K;
    switch (kind) {
    case kKindDefect: {
        int tp = kTileFine / n;
        return ((nx + tp - 1) / tp) * ((ny + tp - 1) / tp);
    }
    case kKindNet: return (nx * ny + kNetRows - 1) / kNetRows;
    case kKindRhs: return (nx * ny + kThreads - 1) / kThreads;
    case kKindGather: return ((nx + 1) * (ny + 1) + kThreads - 1) / kThreads;
    }
    return 0;
}

template <int K>
__global__ __launch_bounds__(kThreads) void k_defect(FlowArgs single, const BatchTable *bt, int write_X)
{
    constexpr int n = 1 << K;
    constexpr int TP = kTileFine / n;           // patches per tile and direction
    constexpr int NE = kTileFine + 2;           // elements incl. one halo ring
    constexpr int NN = kTileFine + 3;           // nodes of those elements
    constexpr int NO = kTileFine + 1;           // output nodes (tile nodes)
    constexpr int nf = (n + 1) * (n + 1);
    constexpr int nin = 4 * nf + 4;

    __shared__ float s_vx[NN * NN], s_vy[NN * NN], s_p[NN * NN], s_dx[NN * NN], s_dy[NN * NN];
    __shared__ float s_R[8][NE * NE];
    __shared__ float2 s_D[NO * NO];

    int blk = blockIdx.x;
    const FlowArgs f = bt ? *batch_flow(bt, kKindDefect, blk) : single;
    const int nx = f.nx, ny = f.ny, NX = nx * n, NY = ny * n;
    const int tiles_x = (nx + TP - 1) / TP;
    const int tx = blk % tiles_x, ty = blk / tiles_x;
    const int I0 = tx * kTileFine, J0 = ty * kTileFine;
    const int tid = threadIdx.x;
    const int first = *f.first_flag;

    // 1. nodal values of P v, P p and (u_prev - P v) on the tile's nodes + halo.
    for (int t = tid; t < NN * NN; t += kThreads) {
        int I = I0 - 1 + t % NN, J = J0 - 1 + t / NN;
        float vx = 0.f, vy = 0.f, q = 0.f, dx = 0.f, dy = 0.f;
        if (I >= 0 && I <= NX && J >= 0 && J <= NY) {
            prolong_node<K>(f.v, f.p, nx, ny, I, J, vx, vy, q);
            if (!first) {
                float2 u = reinterpret_cast<const float2 *>(f.uprev)[(size_t)J * (NX + 1) + I];
                dx = u.x - vx;
                dy = u.y - vy;
            }
        }
        s_vx[t] = vx; s_vy[t] = vy; s_p[t] = q; s_dx[t] = dx; s_dy[t] = dy;
    }
    __syncthreads();

    // 2. element residuals (4 nodes x 2 components) on the tile + halo ring.
    const float inv_dt = f.inv_dt, nu = f.nu;
    for (int t = tid; t < NE * NE; t += kThreads) {
        int le = t % NE, me = t / NE;
        int eI = I0 - 1 + le, eJ = J0 - 1 + me;
        float R[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (eI >= 0 && eI < NX && eJ >= 0 && eJ < NY) {
            int ci = eI >> K, a = eI & (n - 1), cj = eJ >> K, b = eJ & (n - 1);
            const float *g = f.geo + 6 * ((size_t)cj * nx + ci);
            float exx = g[0], exy = g[1], eyx = g[2], eyy = g[3], twx = g[4], twy = g[5];
            int nd[4] = {me * NN + le, me * NN + le + 1, (me + 1) * NN + le, (me + 1) * NN + le + 1};
            float vx[4], vy[4], pq[4], dx[4], dy[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                vx[k] = s_vx[nd[k]]; vy[k] = s_vy[nd[k]]; pq[k] = s_p[nd[k]];
                dx[k] = s_dx[nd[k]]; dy[k] = s_dy[nd[k]];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float s = (q & 1) ? kG1 : kG0, tt = (q & 2) ? kG1 : kG0;
                const float xi = (a + s) * (1.0f / n), eta = (b + tt) * (1.0f / n);
                // columns of the fine-element Jacobian: d x / d s and d x / d t
                const float xs = (exx + twx * eta) * (1.0f / n), ys = (exy + twy * eta) * (1.0f / n);
                const float xt = (eyx + twx * xi) * (1.0f / n), yt = (eyy + twy * xi) * (1.0f / n);
                const float det = xs * yt - xt * ys;
                const float idet = 1.0f / det;
                const float wd = 0.25f * fabsf(det);
                const float N[4] = {(1.f - s) * (1.f - tt), s * (1.f - tt), (1.f - s) * tt, s * tt};
                const float dNs[4] = {-(1.f - tt), 1.f - tt, -tt, tt};
                const float dNt[4] = {-(1.f - s), -s, 1.f - s, s};
                float dNx[4], dNy[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    dNx[k] = (yt * dNs[k] - ys * dNt[k]) * idet;
                    dNy[k] = (-xt * dNs[k] + xs * dNt[k]) * idet;
                }
                float v0 = 0.f, v1 = 0.f, d0 = 0.f, d1 = 0.f, pp = 0.f;
                float g00 = 0.f, g01 = 0.f, g10 = 0.f, g11 = 0.f;  // g[c][k] = d v_c / d x_k
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    v0 += N[k] * vx[k]; v1 += N[k] * vy[k];
                    d0 += N[k] * dx[k]; d1 += N[k] * dy[k];
                    pp += N[k] * pq[k];
                    g00 += vx[k] * dNx[k]; g01 += vx[k] * dNy[k];
                    g10 += vy[k] * dNx[k]; g11 += vy[k] * dNy[k];
                }
                const float m0 = inv_dt * d0 - (v0 * g00 + v1 * g01);   // mass - convection, c = x
                const float m1 = inv_dt * d1 - (v0 * g10 + v1 * g11);   // c = y
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    R[2 * k] += wd * (N[k] * m0 - nu * (dNx[k] * g00 + dNy[k] * g01) + pp * dNx[k]);
                    R[2 * k + 1] += wd * (N[k] * m1 - nu * (dNx[k] * g10 + dNy[k] * g11) + pp * dNy[k]);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) s_R[r][t] = R[r];
    }
    __syncthreads();

    // 3. node sums over the (up to) four elements around each tile node, in
    //    the order (I-1,J-1), (I,J-1), (I-1,J), (I,J); Dirichlet mask.
    const unsigned dir = f.dirichlet;
    for (int t = tid; t < NO * NO; t += kThreads) {
        int li = t % NO, lj = t / NO;
        int I = I0 + li, J = J0 + lj;
        float2 d = make_float2(0.f, 0.f);
        if (I <= NX && J <= NY) {
            int e00 = lj * NE + li;                  // element (I-1, J-1) in tile-local numbering
            d.x = s_R[6][e00] + s_R[4][e00 + 1] + s_R[2][e00 + NE] + s_R[0][e00 + NE + 1];
            d.y = s_R[7][e00] + s_R[5][e00 + 1] + s_R[3][e00 + NE] + s_R[1][e00 + NE + 1];
            bool m = ((dir & 1u) && I == 0) || ((dir & 2u) && I == NX) || ((dir & 4u) && J == 0) ||
                     ((dir & 8u) && J == NY);
            if (m) d = make_float2(0.f, 0.f);
            if (f.D_out && (li < kTileFine || I == NX) && (lj < kTileFine || J == NY))
                reinterpret_cast<float2 *>(f.D_out)[(size_t)J * (NX + 1) + I] = d;
        }
        s_D[t] = d;
    }
    if (!write_X) return;
    __syncthreads();

    // 4. network input rows of the tile's patches:
    //    [P v at the (n+1)^2 patch nodes ; D at the same nodes ; features].
    for (int t = tid; t < TP * TP * nin; t += kThreads) {
        int pl = t / nin, fi = t - pl * nin;
        int pi = tx * TP + pl % TP, pj = ty * TP + pl / TP;
        if (pi >= nx || pj >= ny) continue;
        size_t e = (size_t)pj * nx + pi;
        float val;
        if (fi < 4 * nf) {
            int half = fi >= 2 * nf;
            int r = fi - half * 2 * nf;
            int l = r >> 1, c = r & 1;
            int a = l % (n + 1), b = l / (n + 1);
            int li = (pl % TP) * n + a, lj = (pl / TP) * n + b;   // output-node coordinates
            if (!half) {
                int nn = (lj + 1) * NN + (li + 1);
                val = c ? s_vy[nn] : s_vx[nn];
            } else {
                float2 d = s_D[lj * NO + li];
                val = c ? d.y : d.x;
            }
        } else {
            val = f.feat[4 * e + (fi - 4 * nf)];
        }
        f.X[e * nin + fi] = val;
    }
}

hipError_t launch_defect(const FlowArgs &f, const BatchTable *bt, int nblocks, int K, int write_X,
                         hipStream_t s)
{
    dim3 g(nblocks), b(kThreads);
    switch (K) {
    case 1: hipLaunchKernelGGL(k_defect<1>, g, b, 0, s, f, bt, write_X); break;
    case 2: hipLaunchKernelGGL(k_defect<2>, g, b, 0, s, f, bt, write_X); break;
    case 3: hipLaunchKernelGGL(k_defect<3>, g, b, 0, s, f, bt, write_X); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace dnnmg
