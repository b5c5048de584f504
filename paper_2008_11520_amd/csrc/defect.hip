// Create-time geometry, prolongation and the fine Navier-Stokes defect on gfx950.
//
// Defect (momentum rows of the nonlinear residual of Eq. (nonlinearshort),
// implicit-Euler form, Q1/Q1):
//   D_a,c = sum_e sum_q w_q |det J_q| [ (1/dt) phi_a (u_prev - v)_c - phi_a (v.grad v_c)
//                                       - nu grad phi_a . grad v_c + p d_c phi_a ]
// evaluated on the prolongated coarse fields v = P v_L, p = P p_L (Alg. 2,
// prolongation) and zeroed at Dirichlet nodes.  One workgroup owns a 32 x 32 tile of
// fine elements plus a ring of one halo element, so that the nodes on the tile
// border get every element contribution without global atomics; element
// residuals go to LDS and are summed per node in a fixed order (bitwise
// deterministic).  The tile also writes the network input rows of its patches.
//
// Fine-element geometry is taken from the coarse element's bilinear map
// F(xi,eta) = c00 + ex xi + ey eta + exy xi eta (edge vectors formed in FP64 at
// create time), so Jacobians keep full FP32 relative precision even when the
// absolute coordinates are large compared with the fine mesh width.
#include <type_traits>

#include "device.h"
#include "element.h"
#include "frame.h"
#include "fp8.h"
#include "internal.h"

namespace dnnmg {

// ---------------------------------------------------------------- geometry
// Per coarse element: FP32 map vectors for the defect, FP64 coefficients of
// det J = d0 + d1 xi + d2 eta for the right-hand side, optionally the FP64
// map vectors themselves (the Crank-Nicolson rhs), the four patch features
// hx, hy, hx/hy, area, and optionally the paper's twelve geometry inputs
// (edge lengths bottom, right, top, left; ratios h0/h1, h2/h3, h0/h2, h1/h3;
// interior angles at the corners 00, 10, 11, 01).  *bad is set if an element
// is not positively oriented (det J <= 0 at a corner).
__device__ inline double corner_angle64(double ux, double uy, double wx, double wy)
{
    return atan2(fabs(ux * wy - uy * wx), ux * wx + uy * wy);
}

__global__ __launch_bounds__(kThreads) void k_geometry(const double *__restrict__ cxy, int nx, int ny,
                                                       float *__restrict__ geo, double *__restrict__ geo64,
                                                       double *__restrict__ map64, float *__restrict__ feat,
                                                       float *__restrict__ geo12, int *__restrict__ bad)
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
    if (map64) {
        double *m = map64 + 8 * (size_t)e;
        m[0] = exx; m[1] = exy_; m[2] = eyx; m[3] = eyy; m[4] = twx; m[5] = twy; m[6] = 0.0; m[7] = 0.0;
    }
    if (!(d0 > 0.0 && d0 + d1 > 0.0 && d0 + d2 > 0.0 && d0 + d1 + d2 > 0.0)) *bad = 1;
    double hx = 0.5 * (hypot(exx, exy_) + hypot(c11[0] - c01[0], c11[1] - c01[1]));
    double hy = 0.5 * (hypot(eyx, eyy) + hypot(c11[0] - c10[0], c11[1] - c10[1]));
    double ax = c11[0] - c00[0], ay = c11[1] - c00[1];
    double bx = c01[0] - c10[0], by = c01[1] - c10[1];
    float *f = feat + 4 * (size_t)e;
    f[0] = (float)hx; f[1] = (float)hy; f[2] = (float)(hx / hy); f[3] = (float)(0.5 * fabs(ax * by - ay * bx));
    if (geo12) {
        const double rx = c11[0] - c10[0], ry = c11[1] - c10[1];   // right edge, 10 -> 11
        const double tx = c11[0] - c01[0], ty = c11[1] - c01[1];   // top edge, 01 -> 11
        const double h0 = hypot(exx, exy_), h1 = hypot(rx, ry), h2 = hypot(tx, ty), h3 = hypot(eyx, eyy);
        float *o = geo12 + 12 * (size_t)e;
        o[0] = (float)h0; o[1] = (float)h1; o[2] = (float)h2; o[3] = (float)h3;
        o[4] = (float)(h0 / h1); o[5] = (float)(h2 / h3); o[6] = (float)(h0 / h2); o[7] = (float)(h1 / h3);
        o[8] = (float)corner_angle64(exx, exy_, eyx, eyy);          // at 00: to 10 and to 01
        o[9] = (float)corner_angle64(rx, ry, -exx, -exy_);          // at 10: to 11 and to 00
        o[10] = (float)corner_angle64(-tx, -ty, -rx, -ry);          // at 11: to 01 and to 10
        o[11] = (float)corner_angle64(-eyx, -eyy, tx, ty);          // at 01: to 00 and to 11
    }
}

hipError_t launch_geometry(const double *cxy, int nx, int ny, float *geo, double *geo64, double *map64,
                           float *feat, float *geo12, int *bad, hipStream_t s)
{
    int P = nx * ny;
    hipLaunchKernelGGL(k_geometry, dim3((P + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                       cxy, nx, ny, geo, geo64, map64, feat, geo12, bad);
    return hipGetLastError();
}

// ------------------------------------------------------------ prolongation
// Bilinear interpolation of the coarse corner values of the element that
// holds fine node (I,J) (Alg. 2, prolongation).
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
int blocks_for(int kind, int nx, int ny, int K)
{
    int n = 1 << K;
    switch (kind) {
    case kKindDefect: {
        int tp = kTileFine / n;
        return ((nx + tp - 1) / tp) * ((ny + tp - 1) / tp);
    }
    case kKindNet: return (nx * ny + kNetRows - 1) / kNetRows;
    case kKindRhs: {
        int tp = kRhsFine / n;
        return ((nx + tp - 1) / tp) * ((ny + tp - 1) / tp);
    }
    case kKindGather: return ((nx + 1) * (ny + 1) + kThreads - 1) / kThreads;
    }
    return 0;
}

// ------------------------------------------------- defect + network fusion
// For K = 2 a defect tile covers 8 x 8 = 64 patches, one network tile: the
// fused step keeps the network input in LDS and runs the GRU and MLP of the
// tile right after its defect (BF16 operands, H = 64).  Layout and MFMA use
// follow the persistent network kernel (products formed transposed, so a lane
// holds one patch row and four consecutive units); wave w owns hidden tile w
// for all four row tiles and loads that tile's weight fragments itself.
constexpr int kFusedLDA = 104 + 64 + 16;       // [x | h | 8 zeros] rows (168 + 8 values), padded so that 16 rows of a fragment read fall in distinct LDS banks
constexpr int kFusedLDH = 64 + 8;

template <int HM, bool FRAME>
__device__ __forceinline__ void gru_fused(const FlowArgs &f, int tx, int ty, int tid, const NetArgs &net,
                                          __bf16 *sA, __bf16 *sR, __bf16 *sHp, __bf16 *sAm, float *s_of,
                                          float2 *s_vc)
{
    constexpr int nin = 104, nout = 50, H = 64, KC = 32, KQ = 8, KC1 = 6, TP = 8, RT = 4, HT = 4;
    constexpr int LDA = kFusedLDA, LDH = kFusedLDH;
    static_assert((nin + H) % KQ == 0 && nin + H > (KC1 - 1) * KC, "k-padding only in the last chunk");
    static_assert(LDA >= nin + H + KQ, "room for the zeros after [x | h]");
    const int nx = f.nx, ny = f.ny;
    const int wave = tid >> 6, lane = tid & 63, li = lane & 15, lq = lane >> 4;
    const int ht = wave, ucol = 16 * ht + 4 * lq;
    auto valid = [&](int r) { return tx * TP + r % TP < nx && ty * TP + r / TP < ny; };
    // This lane's rows 16 q + li are patches (2 q + li / 8, li % 8) of the
    // tile: their state and outputs are addressed from the tile's first patch
    // (a uniform 64-bit base) with 32-bit lane offsets, formed once and
    // stepped by 2 q patch rows (no 64-bit index products per access).
    // (FRAME false keeps the plain index form, which holds fewer registers
    // across the network)
    const size_t p00 = (size_t)(ty * TP) * nx + tx * TP;
    const unsigned roff = ((li >> 3) ? (unsigned)nx : 0u) + (unsigned)(li & 7);
    auto patch = [&](int r) { return (size_t)(ty * TP + r / TP) * nx + tx * TP + r % TP; };
    auto hrow = [&](int q) {
        return FRAME ? f.h + p00 * H + (roff + 2u * q * (unsigned)nx) * H + ucol : f.h + patch(16 * q + li) * H + ucol;
    };
    const gptr<bf8> B1 = pinned<bf8>(net.B1);
    const gptr<bf8> B2 = pinned<bf8>(net.B2);
    const gptr<bf8> B3 = pinned<bf8>(net.B3);
    const gptr<bf8> B4 = pinned<bf8>(net.B4);
    // the tile's state in this lane's layout (rows 16 q + li, units ucol..+3):
    // one HBM read serves the MFMA operand (BF16, next to the network input)
    // and the update.  It is waited for only after the k-chunks that hold
    // input alone.
    f4 hp[RT];
#pragma unroll
    for (int q = 0; q < RT; ++q) {
        const int r = 16 * q + li;
        hp[q] = valid(r) ? *reinterpret_cast<const f4 *>(hrow(q)) : f4{0.f, 0.f, 0.f, 0.f};
    }
    // corner velocities of the tile's patches, for the averaging after the
    // network when the outputs stay in LDS (f.frame); loaded on every launch,
    // clamped into the mesh, and stored once the input-only chunks are issued
    constexpr int SVF = TP + 1;
    float2 vc = make_float2(0.f, 0.f);
    if constexpr (FRAME) {
        const int t = min(tid, SVF * SVF - 1);
        const int ci = min(t % SVF, nx - tx * TP), cj = min(t / SVF, ny - ty * TP);
        vc = reinterpret_cast<const float2 *>(f.v)[(size_t)(ty * TP + cj) * (nx + 1) + tx * TP + ci];
    }
    // zeros after [x | h]: the lanes of the last k-chunk that lie beyond it
    // read these (the zero is formed from tile_thread(), so that it is not
    // materialised once and held in a register)
    if (tid < 64) {
        const unsigned z = (unsigned)tile_thread() >> 16;
        *reinterpret_cast<uint4 *>(&sA[tid * LDA + nin + H]) = make_uint4(z, z, z, z);
    }

    // ---- phase 1: the three gates of this wave's hidden tile, four row tiles.
    //      Weight fragments are read chunk by chunk (L2-resident; other waves
    //      cover the latency); the first chunk starts the accumulators.
    f4 az[RT], ar[RT], ah[RT];
    auto chunk = [&](int kc, bool first, bool last) {
        const bf8 wz = B1[((0 * HT + ht) * KC1 + kc) * 64 + lane];
        const bf8 wr = B1[((1 * HT + ht) * KC1 + kc) * 64 + lane];
        const bf8 wh = B1[((2 * HT + ht) * KC1 + kc) * 64 + lane];
        const int k0 = kc * KC + lq * KQ;
        const int kk = last && k0 >= nin + H ? nin + H : k0;
#pragma unroll
        for (int q = 0; q < RT; ++q) {
            const bf8 a = *reinterpret_cast<const bf8 *>(&sA[(16 * q + li) * LDA + kk]);
            const f4 z0 = {0.f, 0.f, 0.f, 0.f};
            az[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wz, a, first ? z0 : az[q], 0, 0, 0);
            ar[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wr, a, first ? z0 : ar[q], 0, 0, 0);
            ah[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, a, first ? z0 : ah[q], 0, 0, 0);
        }
    };
    // the chunks of input alone (the input rows are complete: the defect
    // phase ended with a barrier), then the state's BF16 copy joins the rows
    constexpr int KX = nin / KC;
    static_assert(KX >= 1 && KX < KC1 - 1, "input-only chunks, then chunks with the state");
    chunk(0, true, false);
#pragma unroll
    for (int kc = 1; kc < KX; ++kc) chunk(kc, false, false);
#pragma unroll
    for (int q = 0; q < RT; ++q) {
        bf4 hb;
        hb[0] = (__bf16)hp[q].x; hb[1] = (__bf16)hp[q].y; hb[2] = (__bf16)hp[q].z; hb[3] = (__bf16)hp[q].w;
        *reinterpret_cast<bf4 *>(&sA[(16 * q + li) * LDA + nin + ucol]) = hb;
    }
    if (FRAME && f.frame && tid < SVF * SVF) s_vc[tid] = vc;
    __syncthreads();
#pragma unroll 1
    for (int kc = KX; kc < KC1 - 1; ++kc) chunk(kc, false, false);
    chunk(KC1 - 1, false, true);
    bf8 w2[2];
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) w2[kc] = B2[(ht * 2 + kc) * 64 + lane];
    const f4 (&hold)[RT] = hp;
    __syncthreads();   // every wave is done with the input rows (r*h reuses them)
#pragma unroll
    for (int q = 0; q < RT; ++q) {
        const int r = 16 * q + li;
        bf4 rh;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            az[q][e] = sigmoid_l2(az[q][e]);
            rh[e] = (__bf16)(sigmoid_l2(ar[q][e]) * hold[q][e]);
        }
        *reinterpret_cast<bf4 *>(&sR[r * LDH + ucol]) = rh;
    }
    __syncthreads();

    // ---- phase 2: U_h (r*h); new state
#pragma unroll
    for (int q = 0; q < RT; ++q) {
        const int r = 16 * q + li;
        f4 au = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < 2; ++kc)
            au = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2[kc], *reinterpret_cast<const bf8 *>(&sR[r * LDH + kc * KC + lq * KQ]), au, 0, 0, 0);
        f4 hn;
        bf4 hb;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float z = az[q][e];
            // h' = z h + (1 - z) c = c + z (h - c), c the candidate state
            const float c = tanh_l2(ah[q][e] + au[e]);
            hn[e] = c + z * (hold[q][e] - c);
            hb[e] = (__bf16)hn[e];
        }
        if (valid(r)) *reinterpret_cast<f4 *>(hrow(q)) = hn;
        *reinterpret_cast<bf4 *>(&sHp[r * LDH + ucol]) = hb;
    }
    __syncthreads();

    // ---- MLP head: M2 relu(M1 h') (HM = 64) or M h' (HM = 0); wave w makes output tile w
    const __bf16 *src = sHp;
    bf8 wo[2];
    if constexpr (HM > 0) {
        bf8 w3[2];
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) w3[kc] = B3[(ht * 2 + kc) * 64 + lane];
#pragma unroll
        for (int q = 0; q < RT; ++q) {
            const int r = 16 * q + li;
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kc = 0; kc < 2; ++kc)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3[kc], *reinterpret_cast<const bf8 *>(&sHp[r * LDH + kc * KC + lq * KQ]), acc, 0, 0, 0);
            bf4 m;
#pragma unroll
            for (int e = 0; e < 4; ++e) m[e] = (__bf16)fmaxf(acc[e], 0.f);
            *reinterpret_cast<bf4 *>(&sAm[r * LDH + ucol]) = m;
        }
        __syncthreads();
        src = sAm;
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) wo[kc] = B4[(ht * 2 + kc) * 64 + lane];
    } else {
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) wo[kc] = B3[(ht * 2 + kc) * 64 + lane];
    }
    f4 acc[RT];
#pragma unroll
    for (int q = 0; q < RT; ++q) {
        const int r = 16 * q + li;
        acc[q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < 2; ++kc)
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wo[kc], *reinterpret_cast<const bf8 *>(&src[r * LDH + kc * KC + lq * KQ]), acc[q], 0, 0, 0);
    }
    // outputs to LDS (rows of nout floats) for the averaging in the tile
    // (f.frame), and/or to the per-patch outputs.  Without the MLP hidden
    // layer the products above read h' from the bytes the LDS rows take.
    const bool frame = FRAME && f.frame != nullptr;
    if constexpr (HM == 0) {
        if (frame) __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < RT; ++q) {
        const int r = 16 * q + li;
        // nout is even: the pairs (ucol, ucol+1), (ucol+2, ucol+3) are inside or outside together
        if (frame) {
            float *o = s_of + r * nout + ucol;
            if (ucol < nout) *reinterpret_cast<float2 *>(o) = make_float2(acc[q][0], acc[q][1]);
            if (ucol + 2 < nout) *reinterpret_cast<float2 *>(o + 2) = make_float2(acc[q][2], acc[q][3]);
        }
        if ((!frame || f.keep_dpatch) && valid(r)) {
            float *o = FRAME ? f.dpatch + p00 * nout + (roff + 2u * q * (unsigned)nx) * nout + ucol
                             : f.dpatch + patch(r) * nout + ucol;
            if (ucol < nout) *reinterpret_cast<float2 *>(o) = make_float2(acc[q][0], acc[q][1]);
            if (ucol + 2 < nout) *reinterpret_cast<float2 *>(o + 2) = make_float2(acc[q][2], acc[q][3]);
        }
    }
}

// Duplicate averaging (Sec. 4.2) inside the one-launch step, with the tile's
// outputs in LDS (rows of 2 nf floats, s_o) and its patches' corner
// velocities (s_vc, (TP+1)^2): every node inside the tile's boundary lines has
// all its patches here.  Deep nodes get the corrected velocity P v + d in the
// state (and d in the caller's output); inner frame nodes hand over d, the
// tile's sides hand over their outputs (frame.h) for the rhs kernel to
// complete.  The sums, the mask and P v + d are formed as the rhs kernel forms
// them, so the state and outputs match the separate-launch step bit for bit.
// The completed values are staged as a tile image in LDS (s_img, (kTileFine
// + 1)^2 nodes: u at deep nodes, d at inner ones) and then stored row by row
// with 16-byte stores: stored node by node straight from the sums, the 8-byte
// values of one store instruction would lie 32 bytes apart.
__device__ __forceinline__ void fused_average(const FlowArgs &f, int tx, int ty, int tid, const float2 *s_o,
                                              const float2 *s_vc, float2 *s_img)
{
    constexpr int K = 2, n = 1 << K, nf = (n + 1) * (n + 1), TP = kTileFine / n, SVF = TP + 1;
    constexpr float inv_n = 1.0f / n;
    typedef TileFrame<K> FR;
    static_assert(TP * TP * n == kThreads && FR::TP == TP, "one node row of one patch per thread");
    const int nx = f.nx, ny = f.ny, NX = nx * n, NY = ny * n;
    const int pi0 = tx * TP, pj0 = ty * TP, I0 = pi0 * n, J0 = pj0 * n;
    const int tiles_x = (nx + TP - 1) / TP;
    const int up = f.upitch;
    const unsigned dir = f.dirichlet;
    float2 *const fr = reinterpret_cast<float2 *>(f.frame) + (size_t)(ty * tiles_x + tx) * FR::SIZE;
    float2 *const ut = reinterpret_cast<float2 *>(f.uprev) + (size_t)J0 * up + I0;
    float2 *const dout = f.dbar_out ? reinterpret_cast<float2 *>(f.dbar_out) + (size_t)J0 * (NX + 1) + I0 : nullptr;
    bool nonfin = false;
    // the sides' outputs: wave w copies side w (slots w SIDE + lane)
    static_assert(kThreads == 4 * 64 && FR::SIDE <= 64, "one side per wave");
    {
        const int w = tid >> 6, l = tid & 63;
        if (l < FR::SIDE) {
            int pa, pb, a, b;
            FR::side_pos(w, l, pa, pb, a, b);
            if (pi0 + pa < nx && pj0 + pb < ny) fr[w * FR::SIDE + l] = s_o[(pb * TP + pa) * nf + b * (n + 1) + a];
        }
    }
    // a completed node: inner frame nodes hand over d, deep nodes store u
    constexpr int NO = kTileFine + 1;
    auto finish = [&](int li, int lj, float2 d, float px, float py) {
        if (frame_kind(li, lj) == kFrameInner) {
            s_img[lj * NO + li] = d;
        } else {
            s_img[lj * NO + li] = make_float2(px + d.x, py + d.y);
            if (dout) dout[lj * (NX + 1) + li] = d;
        }
    };
    // the nodes (a, b), a, b < n, of the tile's patches, one node row of one
    // patch per thread.  With li, lj >= 1 such a node has the patch to its
    // left exactly when a = 0 and the one below exactly when b = 0, both in
    // the tile, and no mask (masks lie on the sides I = 0, J = 0, which are
    // boundary lines).  Absent patches are read from the own patch and
    // replaced by +0 (a running sum from +0 is never -0, so adding +0 leaves
    // its bits as skipping the patch would): the sums, in row-major patch
    // order, are those of the rhs kernel.
    const bool chk = f.nonfinite != nullptr;
    {
        const int pl = tid % (TP * TP), b = tid / (TP * TP);
        const int pa = pl % TP, pb = pl / TP, pi = pi0 + pa, pj = pj0 + pb;
        const int lj = pb * n + b;
        if (pi < nx && pj < ny && lj > 0) {
            const bool low = b == 0;
            const bool rin = lj == 1 || lj == kTileFine - 1;
            const int c = pb * SVF + pa;
            const float2 v00 = s_vc[c], v10 = s_vc[c + 1], v01 = s_vc[c + SVF], v11 = s_vc[c + SVF + 1];
            const PvRow row = pv_row(v00.x, v00.y, v10.x, v10.y, v01.x, v01.y, v11.x, v11.y, b * inv_n);
            const float2 *const qo = s_o + pl * nf + b * (n + 1);              // own node row
            const float2 *const ql = s_o + (low ? pl - TP : pl) * nf + n * (n + 1);   // top row of the patch below
            const float2 z = make_float2(0.f, 0.f);
#pragma unroll
            for (int a = 0; a < n; ++a) {
                const int li = pa * n + a;
                if (a == 0 && pa == 0) continue;                               // li = 0: boundary line
                float2 acc = z;
                if (a == 0) {
                    const float2 qd = low ? s_o[(pl - TP - 1) * nf + n * (n + 1) + n] : z;
                    acc.x += qd.x; acc.y += qd.y;
                }
                {
                    const float2 q = ql[a];
                    const float2 qb = low ? q : z;
                    acc.x += qb.x; acc.y += qb.y;
                }
                if (a == 0) {
                    const float2 q = s_o[(pl - 1) * nf + b * (n + 1) + n];
                    acc.x += q.x; acc.y += q.y;
                }
                acc.x += qo[a].x; acc.y += qo[a].y;
                const float inv = a == 0 ? (low ? 0.25f : 0.5f) : (low ? 0.5f : 1.0f);
                const float2 d = make_float2(acc.x * inv, acc.y * inv);
                if (chk) nonfin |= !(__builtin_isfinite(d.x) && __builtin_isfinite(d.y));
                float px, py;
                pv_at(row, a * inv_n, px, py);
                const bool inner = rin || (a == 1 && pa == 0) || (a == n - 1 && pa == TP - 1);
                s_img[lj * NO + li] = inner ? d : make_float2(px + d.x, py + d.y);
                if (dout && !inner) dout[lj * (NX + 1) + li] = d;
            }
        }
    }
    // the mesh end inside a ragged tile: its last node column li = le and row
    // lj = me (on a full tile these are boundary lines)
    const int le = min(TP, nx - pi0) * n, me = min(TP, ny - pj0) * n;
    if (tid < le + me + 1) {
        const int li = tid <= me ? le : tid - me - 1, lj = tid <= me ? tid : me;
        if (frame_kind(li, lj) != kFrameEdge) {
            const int I = I0 + li, J = J0 + lj;
            const int pI = min(I >> K, nx - 1), pJ = min(J >> K, ny - 1);
            const int a = I - pI * n, b = J - pJ * n;
            const bool lft = a == 0 && pI > 0, low = b == 0 && pJ > 0;
            const int hb = (pJ - pj0) * TP + (pI - pi0);
            float2 acc = make_float2(0.f, 0.f);
            if (lft && low) { const float2 q = s_o[(hb - TP - 1) * nf + n * (n + 1) + n]; acc.x += q.x; acc.y += q.y; }
            if (low) { const float2 q = s_o[(hb - TP) * nf + n * (n + 1) + a]; acc.x += q.x; acc.y += q.y; }
            if (lft) { const float2 q = s_o[(hb - 1) * nf + b * (n + 1) + n]; acc.x += q.x; acc.y += q.y; }
            { const float2 q = s_o[hb * nf + b * (n + 1) + a]; acc.x += q.x; acc.y += q.y; }
            const float inv = (lft && low) ? 0.25f : ((lft || low) ? 0.5f : 1.0f);
            float2 d = make_float2(acc.x * inv, acc.y * inv);
            if (((dir & 1u) && I == 0) || ((dir & 2u) && I == NX) || ((dir & 4u) && J == 0) || ((dir & 8u) && J == NY))
                d = make_float2(0.f, 0.f);
            if (chk) nonfin |= !(__builtin_isfinite(d.x) && __builtin_isfinite(d.y));
            const int c = (pJ - pj0) * SVF + (pI - pi0);
            const float2 v00 = s_vc[c], v10 = s_vc[c + 1], v01 = s_vc[c + SVF], v11 = s_vc[c + SVF + 1];
            const PvRow row = pv_row(v00.x, v00.y, v10.x, v10.y, v01.x, v01.y, v11.x, v11.y, b * inv_n);
            float px, py;
            pv_at(row, a * inv_n, px, py);
            finish(li, lj, d, px, py);
        }
    }
    if (nonfin && f.nonfinite) atomicOr(f.nonfinite, 1);
    __syncthreads();
    // the deep rows lj = 2 .. kTileFine - 2 of the state, nodes li = 2 ..
    // kTileFine - 2 in pairs (16 bytes, aligned: state rows start on 128-byte
    // lines and li = 2 is 16 bytes in), the last one alone; nodes beyond the
    // mesh are not stored
    constexpr int DL = kTileFine - 3, PR = (DL + 1) / 2;   // deep nodes per row, stores per row
    static_assert(DL % 2 == 1, "pairs, then one node");
    const int lim = NX - I0, ljm = NY - J0;                // last tile node inside the mesh
    for (int t = tid; t < DL * PR; t += kThreads) {
        const int lj = 2 + t / PR, c = t - (t / PR) * PR, li = 2 + 2 * c;
        if (lj > ljm || li > lim) continue;
        const float2 a = s_img[lj * NO + li];
        float2 *const q = ut + lj * up + li;
        if (c < PR - 1 && li + 1 <= lim) {
            const float2 b = s_img[lj * NO + li + 1];
            *reinterpret_cast<float4 *>(q) = make_float4(a.x, a.y, b.x, b.y);
        } else {
            *q = a;
        }
    }
    // the inner frame nodes' d, in slot order
    if (tid < FR::INNER) {
        int li, lj;
        FR::inner_pos(tid, li, lj);
        if (li <= lim && lj <= ljm) fr[4 * FR::SIDE + tid] = s_img[lj * NO + li];
    }
}

// FUSED (K = 2, BF16 input): the network input stays in LDS and the tile's
// GRU and MLP run right after (gru_fused); HM is the MLP hidden width.
// CN: the theta scheme (Crank-Nicolson at f.theta = 1/2): after the first
// step the elements take element_residual_theta, with the previous corrected
// velocity itself (not divided by dt) at the nodes.  On the first step the
// previous velocity is P v, the two transport levels coincide and the mass
// term vanishes, so the implicit-Euler elements with 1/dt = 0 give the same
// defect.
// PAPER: the network input of the paper's form (Sec. 4.2): the residual at
// the patch nodes, momentum rows (D) then continuity rows, the corner
// velocities, Peclet numbers and twelve geometry values, padded with zeros to
// a multiple of 8 values.
template <int K, typename XT, bool OPAQUE_TID, bool FUSED = false, int HM = 0, bool CN = false, bool PAPER = false>
__device__ __forceinline__ void defect_tile(const FlowArgs &f, int blk, const NetArgs *net = nullptr)
{
    static_assert(!(CN && FUSED), "the theta scheme runs unfused");
    static_assert(!(PAPER && (FUSED || std::is_same<XT, uint8_t>::value)), "paper inputs: unfused, FP32 or BF16");
    const int tid = OPAQUE_TID ? tile_thread() : (int)threadIdx.x;
    constexpr int n = 1 << K;
    constexpr float inv_n = 1.0f / n;
    constexpr int TP = kTileFine / n;           // patches per tile and direction
    constexpr int NN = kTileFine + 3;           // nodes of those elements
    constexpr int CE = TP + 2;                  // coarse elements incl. halo

    constexpr int nf = (n + 1) * (n + 1), nin = PAPER ? (3 * nf + 24 + 7) / 8 * 8 : 4 * nf + 4;
    // XT = uint8_t: FP8 network input, formed in FP32 and quantised per patch
    constexpr bool FP8 = std::is_same<XT, uint8_t>::value;
    typedef typename std::conditional<FP8, float, XT>::type ST;
    constexpr int XS8 = xstride_fp8(nin);        // FP8 row stride (bytes)
    constexpr size_t kWBytes = sizeof(float2) * NN * NN;
    static_assert(!FUSED || (K == 2 && std::is_same<XT, __bf16>::value), "fused step: K = 2, BF16");
    constexpr size_t kXBytes = FUSED ? sizeof(__bf16) * 64 * kFusedLDA
                                     : (FP8 ? (size_t)TP * TP * XS8 : sizeof(ST) * TP * TP * nin);
    __shared__ CoarseRec s_c[CE * CE];
    // u_prev / dt at the nodes; once the element residuals are formed the same
    // bytes hold the tile's network-input rows
    __shared__ __align__(16) unsigned char s_wx[kWBytes > kXBytes ? kWBytes : kXBytes];
    float2 *s_w = reinterpret_cast<float2 *>(s_wx);
    ST *s_x = reinterpret_cast<ST *>(s_wx);
    __shared__ __align__(16) float2 s_acc[NN * NN];   // assembled residual at nodes

    const int nx = f.nx, ny = f.ny, NX = nx * n, NY = ny * n;
    const int tiles_x = (nx + TP - 1) / TP;
    const int tx = blk % tiles_x, ty = blk / tiles_x;
    const int ci0 = tx * TP - 1, cj0 = ty * TP - 1;   // first (halo) coarse element
    const int I0 = tx * kTileFine, J0 = ty * kTileFine;
    const int first = *f.first_flag;
    const float inv_dt = f.inv_dt, nu = f.nu;

    // 0. the previous corrected velocity on the tile's nodes + halo: issue the
    //    loads now, use them after the coarse records are formed
    //    (node t of the halo grid is row t / NN, column t % NN; thread tid
    //    takes t = tid + i kThreads, stepped by kThreads = DR rows + DC
    //    columns, with a 32-bit offset from the grid's first node)
    constexpr int NIT = (NN * NN + kThreads - 1) / kThreads;
    constexpr int DR = kThreads / NN, DC = kThreads % NN;
    float2 uq[NIT];
    if constexpr (OPAQUE_TID) {
        // (batched: the index form that keeps fewer registers live)
#pragma unroll
        for (int i = 0; i < NIT; ++i) {
            const int t = tid + i * kThreads;
            const int I = I0 - 1 + t % NN, J = J0 - 1 + t / NN;
            const bool in = t < NN * NN && !first && I >= 0 && I <= NX && J >= 0 && J <= NY;
            uq[i] = in ? reinterpret_cast<const float2 *>(f.uprev)[(size_t)J * f.upitch + I] : make_float2(0.f, 0.f);
        }
    } else {
        const int up = f.upitch;
        const float2 *const ub = reinterpret_cast<const float2 *>(f.uprev) + ((ptrdiff_t)(J0 - 1) * up + (I0 - 1));
        int row = tid / NN, col = tid - row * NN;
        unsigned off = (unsigned)row * (unsigned)up + (unsigned)col;
#pragma unroll
        for (int i = 0; i < NIT; ++i) {            // issue every load first
            const int t = tid + i * kThreads;
            const int I = I0 - 1 + col, J = J0 - 1 + row;
            const bool in = t < NN * NN && !first && I >= 0 && I <= NX && J >= 0 && J <= NY;
            uq[i] = in ? ub[off] : make_float2(0.f, 0.f);
            row += DR;
            col += DC;
            off += (unsigned)(DR * up + DC);
            if (col >= NN) {
                col -= NN;
                ++row;
                off += (unsigned)(up - NN);
            }
        }
    }

    // 1. coarse-element records.  Every record is formed from indices clamped
    //    into the mesh, with no branch, so that all of its loads (corner v
    //    and p, map coefficients) are issued before any is used; a record
    //    outside the mesh then copies the nearest element's and is never read
    //    (residuals and input rows are formed for elements inside the mesh).
    const float2 *v2 = reinterpret_cast<const float2 *>(f.v);
    const bool has_p = f.p != nullptr;
    const float *p1 = has_p ? f.p : reinterpret_cast<const float *>(f.v);   // read and discarded without p
    for (int t = tid; t < CE * CE; t += kThreads) {
        const int ci = min(max(ci0 + t % CE, 0), nx - 1), cj = min(max(cj0 + t / CE, 0), ny - 1);
        // (single flow: 32-bit offsets, 6 P and the corner count fit; the
        // batched form keeps the index form it was tuned with)
        const unsigned cjn = (unsigned)cj * (unsigned)nx;
        const unsigned c = OPAQUE_TID ? (unsigned)(cj * (nx + 1) + ci) : cjn + (unsigned)(cj + ci);
        const float2 a = v2[c], b = v2[c + 1], cc = v2[c + nx + 1], d = v2[c + nx + 2];
        const float *g = OPAQUE_TID ? f.geo + 6 * ((size_t)cj * nx + ci) : f.geo + 6u * (cjn + (unsigned)ci);
        const float g0 = g[0], g1 = g[1], g2 = g[2], g3 = g[3], g4 = g[4], g5 = g[5];
        const float pa = p1[c], pb = p1[c + 1], pc = p1[c + nx + 1], pd = p1[c + nx + 2];
        CoarseRec r;
        r.V0x = a.x; r.V1x = b.x - a.x; r.V2x = cc.x - a.x; r.V3x = d.x - b.x - cc.x + a.x;
        r.V0y = a.y; r.V1y = b.y - a.y; r.V2y = cc.y - a.y; r.V3y = d.y - b.y - cc.y + a.y;
        r.P0 = has_p ? pa : 0.f;
        r.P1 = has_p ? pb - pa : 0.f;
        r.P2 = has_p ? pc - pa : 0.f;
        r.P3 = has_p ? pd - pb - pc + pa : 0.f;
        r.exx = g0; r.exy = g1;
        r.eyx = g2; r.eyy = g3;
        r.exyx = g4; r.exyy = g5;
        s_c[t] = r;
    }

    // 2. u_prev / dt on the tile's nodes + halo (zero before the first step:
    //    u_prev is then P v, so the element code, which subtracts v / dt at
    //    each Gauss point, takes 1/dt as 0); clear the node accumulators.
    //    The theta scheme keeps u_prev itself.
    const float idt = first ? 0.0f : inv_dt;
    const bool theta_elems = CN && !first;
#pragma unroll
    for (int i = 0; i < NIT; ++i) {
        const int t = tid + i * kThreads;
        if (t >= NN * NN) break;
        const float sw = CN ? 1.0f : idt;
        s_w[t] = make_float2(uq[i].x * sw, uq[i].y * sw);
        s_acc[t] = make_float2(0.f, 0.f);
    }
    __syncthreads();

    // 3. element residuals, kept in registers (the formulas are in
    //    element.h).  The tile's own elements are taken as vertical strips of
    //    SH elements inside one coarse element; wave w holds the strips of
    //    colour w (column parity w & 1, strip-row parity w >> 1), so that the
    //    strips of one wave share no node.  The ring of halo elements around
    //    the tile, one per thread, is computed element by element.
    constexpr int SH = n < 4 ? n : 4;                      // strip height
    constexpr int NSR = kTileFine / SH;                    // strip rows per tile
    constexpr int SPL = kTileFine * NSR / kThreads;        // strips per thread
    static_assert(kTileFine == kTileElems && kThreads == 256 && NSR == 8 * SPL,
                  "strip mapping: 16 columns x 4 strip rows per wave and strip");
    const int wave = tid >> 6, lane = tid & 63;
    float S[SPL][SH + 1][4];
    int sn0[SPL];                                          // lower-left node of the strip (-1: outside the mesh)
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
        int ec, sr;
        strip_of(wave, lane, s, ec, sr);
        const int eI = I0 + ec, eJ = J0 + sr * SH;
        sn0[s] = -1;
        if (eI < NX && eJ < NY) {
            const int n0 = (sr * SH + 1) * NN + ec + 1;
            sn0[s] = n0;
            const CoarseRec &r = s_c[((eJ >> K) - cj0) * CE + ((eI >> K) - ci0)];
            if (theta_elems) {
                // element by element up the strip: corners 00, 10 on node row k, 01, 11 on row k + 1
                const float2 *w = s_w + n0;
#pragma unroll
                for (int k = 0; k < SH; ++k) {
                    float R[8];
                    element_residual_theta<K, HwRcp>(r, eI & (n - 1), (eJ & (n - 1)) + k, nu, inv_dt, f.theta,
                                                     w[k * NN], w[k * NN + 1], w[(k + 1) * NN],
                                                     w[(k + 1) * NN + 1], R);
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        S[s][k][c] = k ? S[s][k][c] + R[c] : R[c];
                        S[s][k + 1][c] = R[4 + c];
                    }
                }
            } else {
                strip_residual<K, SH, HwRcp>(r, eI & (n - 1), eJ & (n - 1), nu, idt, s_w + n0, NN, S[s]);
            }
        }
    }
    // halo ring, one element per thread (halo_of)
    constexpr int NH = 4 * (kTileFine + 1);
    float Rh[8];
    int hn0 = -1, hcol = -1;
    if (tid < NH) {
        int le, me;                                        // tile-local element (-1 .. kTileFine)
        halo_of(tid, le, me, hcol);
        const int eI = I0 + le, eJ = J0 + me;
        if (eI >= 0 && eI < NX && eJ >= 0 && eJ < NY) {
            const int n0 = (me + 1) * NN + le + 1;
            hn0 = n0;
            const CoarseRec &r = s_c[((eJ >> K) - cj0) * CE + ((eI >> K) - ci0)];
            if (theta_elems)
                element_residual_theta<K, HwRcp>(r, eI & (n - 1), eJ & (n - 1), nu, inv_dt, f.theta, s_w[n0],
                                                 s_w[n0 + 1], s_w[n0 + NN], s_w[n0 + NN + 1], Rh);
            else
                element_residual<K, HwRcp>(r, eI & (n - 1), eJ & (n - 1), nu, idt, s_w[n0], s_w[n0 + 1],
                                           s_w[n0 + NN], s_w[n0 + NN + 1], Rh);
        }
    }

    // 4. assembly in four colour rounds: round c adds the strips of wave c and
    //    the halo elements of colour c, which share no node, so every node
    //    receives its contributions without conflicts and in a fixed order.
#pragma unroll
    for (int colour = 0; colour < 4; ++colour) {
        if (wave == colour) {
#pragma unroll
            for (int s = 0; s < SPL; ++s) {
                if (sn0[s] < 0) continue;
#pragma unroll
                for (int k = 0; k <= SH; ++k) {
                    float2 *q = &s_acc[sn0[s] + k * NN];
                    q[0].x += S[s][k][0]; q[0].y += S[s][k][1];
                    q[1].x += S[s][k][2]; q[1].y += S[s][k][3];
                }
            }
        }
        if (hcol == colour && hn0 >= 0) {
            float2 *q0 = &s_acc[hn0], *q1 = &s_acc[hn0 + 1], *q2 = &s_acc[hn0 + NN], *q3 = &s_acc[hn0 + NN + 1];
            q0->x += Rh[0]; q0->y += Rh[1];
            q1->x += Rh[2]; q1->y += Rh[3];
            q2->x += Rh[4]; q2->y += Rh[5];
            q3->x += Rh[6]; q3->y += Rh[7];
        }
        __syncthreads();
    }

    // 5. Dirichlet mask on the tile's nodes (in place); a tile away from the
    //    masked sides has nothing to mask
    const unsigned dir = f.dirichlet;
    constexpr int NO = kTileFine + 1;
    const bool masked = ((dir & 1u) && I0 == 0) || ((dir & 2u) && I0 + kTileFine >= NX) ||
                        ((dir & 4u) && J0 == 0) || ((dir & 8u) && J0 + kTileFine >= NY);
    if (masked || f.D)
    for (int t = tid; t < NO * NO; t += kThreads) {
        const int li = t % NO, lj = t / NO;
        const int I = I0 + li, J = J0 + lj;
        if (I > NX || J > NY) continue;
        const bool m = ((dir & 1u) && I == 0) || ((dir & 2u) && I == NX) || ((dir & 4u) && J == 0) ||
                       ((dir & 8u) && J == NY);
        float2 &d = s_acc[(lj + 1) * NN + li + 1];
        if (m) d = make_float2(0.f, 0.f);
        // stage entry: the defect itself, written by the tile that owns the node
        if (f.D && (li < kTileFine || I == NX) && (lj < kTileFine || J == NY))
            reinterpret_cast<float2 *>(f.D)[(size_t)J * (NX + 1) + I] = d;
    }
    if (!FUSED && !f.X) return;
    __syncthreads();

    const int npr = min(TP, nx - tx * TP);            // patches of this tile row inside the mesh
    if constexpr (FP8) {
        // FP8: each patch is taken by G consecutive lanes; they form the
        // patch's values (kept in registers when few enough, else formed
        // again), reduce the row maximum with lane shuffles, then scale,
        // convert and write byte pairs into rows of xstride bytes (zero
        // beyond nin).
        uint8_t *s_q = reinterpret_cast<uint8_t *>(s_wx);
        constexpr int G = kThreads / (TP * TP);            // lanes per patch: 1, 4 or 16
        constexpr int NI = (nf + 1 + G - 1) / G;           // items (node or features) per lane
        constexpr bool KEEP = NI <= 8;
        static_assert(G * TP * TP == kThreads && (G & (G - 1)) == 0 && G <= 64, "patch lane groups");
        // item (patch pl, node l < nf): P v and D at the node; l == nf: the features
        auto node_values = [&](int pl, int l, float4 &o) {
            const int pa = pl % TP, pb = pl / TP;
            if (l == nf) {
                o = reinterpret_cast<const float4 *>(f.feat)[(size_t)(ty * TP + pb) * nx + tx * TP + pa];
                return;
            }
            const int a = l % (n + 1), b = l / (n + 1);
            const CoarseRec &r = s_c[(pb + 1) * CE + (pa + 1)];
            const float xi = a * inv_n, eta = b * inv_n;
            const float2 d = s_acc[(pb * n + b + 1) * NN + pa * n + a + 1];
            o.x = (r.V0x + r.V1x * xi) + eta * (r.V2x + r.V3x * xi);
            o.y = (r.V0y + r.V1y * xi) + eta * (r.V2y + r.V3y * xi);
            o.z = d.x;
            o.w = d.y;
        };
        const int pl = tid / G, j = tid % G;
        const int pi = tx * TP + pl % TP, pj = ty * TP + pl / TP;
        const bool pin = pi < nx && pj < ny;
        uint8_t *row = s_q + pl * XS8;
        // the bytes beyond nin (the others are all written below)
        for (int b = nin + j; b < XS8; b += G) row[b] = 0;
        float4 o[KEEP ? NI : 1];
        float m = 0.0f;
#pragma unroll
        for (int q = 0; q < NI; ++q) {
            const int l = j + q * G;
            if (l <= nf && pin) {
                float4 v;
                node_values(pl, l, v);
                if constexpr (KEEP) o[q] = v;
                m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
            }
        }
#pragma unroll
        for (int off = 1; off < G; off <<= 1) m = fmaxf(m, __shfl_xor(m, off));
        m = fmaxf(m, kFp8MinMax);
        const float rs = 448.0f / m;
        if (pin && j == 0) f.sx[(size_t)pj * nx + pi] = m / 448.0f;
#pragma unroll
        for (int q = 0; q < NI; ++q) {
            const int l = j + q * G;
            if (l > nf || !pin) continue;
            float4 v;
            if constexpr (KEEP) v = o[q];
            else node_values(pl, l, v);
            const uint32_t c = pack4_e4m3(v.x * rs, v.y * rs, v.z * rs, v.w * rs);
            if (l == nf) {
                *reinterpret_cast<uint32_t *>(row + 4 * nf) = c;      // 4 nf is a multiple of 4
            } else {
                *reinterpret_cast<uint16_t *>(row + 2 * l) = (uint16_t)c;            // P v
                *reinterpret_cast<uint16_t *>(row + 2 * nf + 2 * l) = (uint16_t)(c >> 16);   // D
            }
        }
        __syncthreads();
        constexpr int CPR = TP * XS8 / 16;                 // 16-byte pieces per tile row of patches
        for (int t = tid; t < TP * CPR; t += kThreads) {
            const int pb = t / CPR, c = t - pb * CPR;
            const int pj = ty * TP + pb;
            if (pj >= ny || c * 16 >= npr * XS8) continue;
            const uint4 v = reinterpret_cast<const uint4 *>(s_q + pb * TP * XS8)[c];
            uint8_t *dst = reinterpret_cast<uint8_t *>(f.X) + ((size_t)pj * nx + tx * TP) * XS8;
            reinterpret_cast<uint4 *>(dst)[c] = v;
        }
    } else {
        // 6. network input rows of the tile's patches, assembled in LDS, then
        //    written with full 16-byte stores (each row of TP patches is
        //    contiguous in X):
        //    X[e] = [P v at the (n+1)^2 patch nodes (x,y interleaved, x fastest) ;
        //            D at the same nodes ; hx, hy, hx/hy, area]
        //    One item is one node row b of one patch (P v along the row is
        //    linear in the node index) or, for b = n + 1, the patch features.
        constexpr int PP = TP * TP, LDX = FUSED ? kFusedLDA : nin;
        auto store2 = [](ST *o, float x, float y) {
            if constexpr (std::is_same<ST, float>::value) {
                *reinterpret_cast<float2 *>(o) = make_float2(x, y);
            } else {
                typedef __bf16 b2 __attribute__((ext_vector_type(2)));
                b2 v;
                v[0] = (__bf16)x; v[1] = (__bf16)y;
                *reinterpret_cast<b2 *>(o) = v;
            }
        };
        if constexpr (PAPER) {
            // continuity row of fine node (I, J): -(div P v, xi) over its (up to
            // four) fine elements.  On a coarse element det J div(P v) is affine
            // in the reference coordinates, c0 + c1 xi + c2 eta (the xi eta
            // terms cancel), so each element's integral against the node's hat
            // is exact in closed form: (h^2 / 4) (c0 + c1 xb + c2 eb), h = 1/n,
            // (xb, eb) the element's corner shifted by h/3 (far side 2h/3)
            // towards the node.
            auto cont_row = [&](int I, int J) -> float {
                float acc = 0.0f;
#pragma unroll
                for (int dj = 0; dj < 2; ++dj)
#pragma unroll
                    for (int di = 0; di < 2; ++di) {
                        const int eI = I - 1 + di, eJ = J - 1 + dj;
                        if (eI < 0 || eI >= NX || eJ < 0 || eJ >= NY) continue;
                        const CoarseRec &r = s_c[((eJ >> K) - cj0) * CE + ((eI >> K) - ci0)];
                        const float c0 = r.eyy * r.V1x - r.exy * r.V2x - r.eyx * r.V1y + r.exx * r.V2y;
                        const float c1 = r.exyy * r.V1x - r.exy * r.V3x - r.exyx * r.V1y + r.exx * r.V3y;
                        const float c2 = r.eyy * r.V3x - r.exyy * r.V2x - r.eyx * r.V3y + r.exyx * r.V2y;
                        const float xb = ((eI & (n - 1)) + (2 - di) * (1.0f / 3.0f)) * inv_n;
                        const float eb = ((eJ & (n - 1)) + (2 - dj) * (1.0f / 3.0f)) * inv_n;
                        acc += c0 + c1 * xb + c2 * eb;
                    }
                return -0.25f * inv_n * inv_n * acc;
            };
            const float inv_nu = 1.0f / f.nu;
            const float2 *vg = reinterpret_cast<const float2 *>(f.v);
            for (int t = tid; t < PP * (n + 2); t += kThreads) {
                const bool extra = t >= PP * (n + 1);
                const int pl = extra ? t - PP * (n + 1) : t / (n + 1), b = extra ? n + 1 : t - pl * (n + 1);
                const int pa = pl % TP, pb = pl / TP, pi = tx * TP + pa, pj = ty * TP + pb;
                if (pi >= nx || pj >= ny) continue;
                ST *o = s_x + pl * LDX;
                if (extra) {
                    // corner velocities and Peclet numbers (corners 00, 10, 01, 11),
                    // the twelve geometry values, zeros to the padded width
                    const size_t e = (size_t)pj * nx + pi;
                    const int c = pj * (nx + 1) + pi;
                    const float2 cv[4] = {vg[c], vg[c + 1], vg[c + nx + 1], vg[c + nx + 2]};
                    const float q = sqrtf(f.feat[4 * e + 3]) * inv_nu;
                    ST *x = o + 3 * nf;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        x[2 * k] = (ST)cv[k].x;
                        x[2 * k + 1] = (ST)cv[k].y;
                        x[8 + k] = (ST)(q * sqrtf(cv[k].x * cv[k].x + cv[k].y * cv[k].y));
                    }
#pragma unroll
                    for (int k = 0; k < 12; ++k) x[12 + k] = (ST)f.geo12[12 * e + k];
                    for (int k = 3 * nf + 24; k < nin; ++k) o[k] = (ST)0.0f;
                    continue;
                }
                const float2 *d = &s_acc[(pb * n + b + 1) * NN + pa * n + 1];
                const int J = pj * n + b;
#pragma unroll
                for (int a = 0; a <= n; ++a) {
                    const int l = b * (n + 1) + a;
                    const float2 dd = d[a];
                    store2(o + 2 * l, dd.x, dd.y);
                    o[2 * nf + l] = (ST)cont_row(pi * n + a, J);
                }
            }
        } else
        // (items of one patch on consecutive lanes: their LDS rows interleave
        // across the banks, where one row per lane would stride LDX apart)
        for (int t = tid; t < PP * (n + 2); t += kThreads) {
            const bool feat = t >= PP * (n + 1);
            const int pl = feat ? t - PP * (n + 1) : t / (n + 1), b = feat ? n + 1 : t - pl * (n + 1);
            const int pa = pl % TP, pb = pl / TP;
            if (tx * TP + pa >= nx || ty * TP + pb >= ny) continue;
            ST *o = s_x + pl * LDX;
            if (b == n + 1) {
                const float4 ft = reinterpret_cast<const float4 *>(f.feat)[(size_t)(ty * TP + pb) * nx + tx * TP + pa];
                store2(o + 4 * nf, ft.x, ft.y);
                store2(o + 4 * nf + 2, ft.z, ft.w);
                continue;
            }
            const CoarseRec &r = s_c[(pb + 1) * CE + (pa + 1)];
            const float eta = b * inv_n;
            const float ax = r.V0x + r.V2x * eta, bx = (r.V1x + r.V3x * eta) * inv_n;
            const float ay = r.V0y + r.V2y * eta, by = (r.V1y + r.V3y * eta) * inv_n;
            const float2 *d = &s_acc[(pb * n + b + 1) * NN + pa * n + 1];
#pragma unroll
            for (int a = 0; a <= n; ++a) {
                const int l = b * (n + 1) + a;
                store2(o + 2 * l, ax + bx * a, ay + by * a);
                const float2 dd = d[a];
                store2(o + 2 * nf + 2 * l, dd.x, dd.y);
            }
        }
        __syncthreads();
        if constexpr (FUSED) {
            // the network input rows stay in LDS; r*h, h' reuse them after phase
            // 1 and the MLP hidden layer reuses the node accumulators
            __bf16 *sA = reinterpret_cast<__bf16 *>(s_wx);
            // (the outputs' LDS rows take the input rows' bytes, the corner
            // velocities the coarse records', the averaged tile image the node
            // accumulators')
            float2 *const s_vc = reinterpret_cast<float2 *>(s_c);
            static_assert(NN * NN >= (kTileFine + 1) * (kTileFine + 1), "tile image in the node accumulators");
            // (the one-launch tiles run one per block, single-flow and batched
            // alike, so the frame code is always there; a flow without a tile
            // frame stores the per-patch outputs)
            constexpr bool FRAME = !OPAQUE_TID;
            gru_fused<HM, FRAME>(f, tx, ty, tid, *net, sA, sA, sA + 64 * kFusedLDH,
                                 reinterpret_cast<__bf16 *>(s_acc), reinterpret_cast<float *>(s_wx), s_vc);
            if (FRAME && f.frame) {
                __syncthreads();
                fused_average(f, tx, ty, tid, reinterpret_cast<const float2 *>(s_wx), s_vc, s_acc);
            }
            return;
        }
        constexpr int CPR = TP * nin * sizeof(XT) / 16;   // 16-byte pieces per tile row of patches
        for (int t = tid; t < TP * CPR; t += kThreads) {
            const int pb = t / CPR, c = t - pb * CPR;
            const int pj = ty * TP + pb;
            if (pj >= ny || c * 16 >= npr * nin * (int)sizeof(XT)) continue;
            const uint4 v = reinterpret_cast<const uint4 *>(s_x + pb * TP * nin)[c];
            XT *dst = reinterpret_cast<XT *>(f.X) + ((size_t)pj * nx + tx * TP) * nin;
            reinterpret_cast<uint4 *>(dst)[c] = v;
        }
    }
}

// Single flow: one tile per block.  Batched: the blocks stride over the
// table's tiles of all flows, so the grid need not match the batch.
// Waves per SIMD the defect aims at (register budget 512 / waves): 4, or
// what its LDS allows (K = 1 tiles hold more patches; FP32 input rows).
template <int K, typename XT>
constexpr int defect_waves()
{
    return K == 1 ? (std::is_same<XT, float>::value ? 2 : 3) : (K == 2 && std::is_same<XT, float>::value ? 3 : 4);
}

template <int K, typename XT, bool BATCHED>
__global__ __launch_bounds__(kThreads, (defect_waves<K, XT>())) void k_defect(FlowArgs single, const BatchTable *__restrict__ bt)
{
    if (!BATCHED) {
        defect_tile<K, XT, false>(single, xcd_tile(blockIdx.x, gridDim.x));
        return;
    }
    const int total = bt->prefix[kKindDefect][bt->nflows];
#pragma unroll 1
    for (int g = blockIdx.x; g < total; g += gridDim.x) {
        int blk = xcd_tile(g, total);
        const FlowArgs &f = *batch_flow(bt, kKindDefect, blk);
        defect_tile<K, XT, true>(f, blk);
        __syncthreads();   // LDS is reused by the next tile
    }
}

// The theta scheme (Crank-Nicolson) and/or the paper's network input, single flow.
// (at K = 1 the paper's wider input rows leave LDS for one workgroup fewer)
template <int K, typename XT, bool PAPER>
constexpr int defect_form_waves()
{
    return PAPER && K == 1 ? defect_waves<K, XT>() - 1 : defect_waves<K, XT>();
}

template <int K, typename XT, bool CN, bool PAPER>
__global__ __launch_bounds__(kThreads, (defect_form_waves<K, XT, PAPER>())) void k_defect_form(FlowArgs single)
{
    defect_tile<K, XT, false, false, 0, CN, PAPER>(single, xcd_tile(blockIdx.x, gridDim.x));
}

// Batched: one tile per block as in a single flow (the grid covers the
// table's tiles; blocks past them return), so the tiles take the single-flow
// code, the tile frame included, with the flow's arguments from the table.
template <bool BATCHED, int HM>
__global__ __launch_bounds__(kThreads, 4) void k_defect_net(FlowArgs single, const BatchTable *__restrict__ bt, NetArgs net)
{
    if (!BATCHED) {
        defect_tile<2, __bf16, false, true, HM>(single, xcd_tile(blockIdx.x, gridDim.x), &net);
        return;
    }
    const int total = bt->prefix[kKindDefect][bt->nflows];
    if ((int)blockIdx.x >= total) return;
    int blk = xcd_tile(blockIdx.x, total);
    const FlowArgs &f = *batch_flow(bt, kKindDefect, blk);
    defect_tile<2, __bf16, false, true, HM>(f, blk, &net);
}

bool fused_step(const NetArgs &net)
{
    return net.prec == 1 && net.K == 2 && net.H == 64 && (net.Hm == 0 || net.Hm == 64) && net.xform == 0 &&
           !net.reset_after;
}

hipError_t launch_defect_net(const FlowArgs &f, const BatchTable *bt, int nblocks, const NetArgs &net, hipStream_t s)
{
    if (!fused_step(net) || f.theta != 1.0f) return hipErrorInvalidValue;
    dim3 g(nblocks), b(kThreads);
    if (net.Hm == 64) {
        if (bt) hipLaunchKernelGGL((k_defect_net<true, 64>), g, b, 0, s, f, bt, net);
        else hipLaunchKernelGGL((k_defect_net<false, 64>), g, b, 0, s, f, bt, net);
    } else {
        if (bt) hipLaunchKernelGGL((k_defect_net<true, 0>), g, b, 0, s, f, bt, net);
        else hipLaunchKernelGGL((k_defect_net<false, 0>), g, b, 0, s, f, bt, net);
    }
    return hipGetLastError();
}

hipError_t launch_defect(const FlowArgs &f, const BatchTable *bt, int nblocks, int K, int xfmt, hipStream_t s)
{
    dim3 g(nblocks), b(kThreads);
    const bool cn = f.theta != 1.0f, paper = f.xform != 0;
    if ((cn || paper) && bt) return hipErrorInvalidValue;
    if (paper && (xfmt == 2 || !f.geo12)) return hipErrorInvalidValue;
#define DNNMG_DEFECT_LAUNCH(KK, XT)                                                           \
    if (bt) hipLaunchKernelGGL((k_defect<KK, XT, true>), g, b, 0, s, f, bt);                   \
    else if (cn) hipLaunchKernelGGL((k_defect_form<KK, XT, true, false>), g, b, 0, s, f);      \
    else hipLaunchKernelGGL((k_defect<KK, XT, false>), g, b, 0, s, f, bt);
#define DNNMG_DEFECT_PAPER(KK, XT)                                                            \
    if (cn) hipLaunchKernelGGL((k_defect_form<KK, XT, true, true>), g, b, 0, s, f);            \
    else hipLaunchKernelGGL((k_defect_form<KK, XT, false, true>), g, b, 0, s, f);
#define DNNMG_DEFECT_CASE(KK)                                                                 \
    case KK:                                                                                  \
        if (paper && xfmt == 1) { DNNMG_DEFECT_PAPER(KK, __bf16) }                            \
        else if (paper) { DNNMG_DEFECT_PAPER(KK, float) }                                     \
        else if (xfmt == 1) { DNNMG_DEFECT_LAUNCH(KK, __bf16) }                               \
        else if (xfmt == 2) { DNNMG_DEFECT_LAUNCH(KK, uint8_t) }                              \
        else { DNNMG_DEFECT_LAUNCH(KK, float) }                                               \
        break;
    switch (K) {
        DNNMG_DEFECT_CASE(1)
        DNNMG_DEFECT_CASE(2)
        DNNMG_DEFECT_CASE(3)
    default: return hipErrorInvalidValue;
    }
#undef DNNMG_DEFECT_CASE
#undef DNNMG_DEFECT_PAPER
#undef DNNMG_DEFECT_LAUNCH
    return hipGetLastError();
}

}  // namespace dnnmg
