// Fine-element residuals of the momentum defect on a coarse Q1 element
// (implicit-Euler Navier-Stokes, Q1/Q1, 2 x 2 Gauss rule): one element at a
// time, or a vertical strip of elements that share their abscissae.  Host and
// device code; the reciprocal is a parameter (the device passes the hardware
// one).
#pragma once

#include <hip/hip_runtime.h>

namespace dnnmg {

// Per coarse element, the coefficients the defect needs (LDS record):
// prolongated velocity and pressure as bilinear polynomials in the coarse
// reference coordinates, v = V0 + V1 xi + V2 eta + V3 xi eta, and the map
// vectors of F(xi, eta) = c00 + ex xi + ey eta + exy xi eta, so that
// x_xi = ex + exy eta, x_eta = ey + exy xi.  Derivatives are taken in the
// coarse reference coordinates; the fine element's own reference derivatives
// are these times 1/n, a factor the element sums apply at the end.
struct CoarseRec {
    float V0x, V1x, V2x, V3x, V0y, V1y, V2y, V3y;
    float P0, P1, P2, P3;
    float exx, exy, eyx, eyy, exyx, exyy;
};

// Device operations of the element code: the hardware reciprocal, and a
// scheduling fence that keeps the compiler from interleaving the two
// abscissa passes of a strip (which would hold both passes' coefficients in
// registers at once).
struct HwRcp {
    __device__ static float f(float x) { return __builtin_amdgcn_rcpf(x); }
    __device__ static void fence() { __builtin_amdgcn_sched_barrier(0); }
};

constexpr float kGauss0 = 0.21132486540518711775f, kGauss1 = 0.78867513459481288225f;

// At each Gauss point, with Cof = det J^{-T} (so det grad = Cof grad_ref) and
// G = Cof^T Cof:
//   mass - convection:  m_c = det (u_prev - v)_c / dt - v . (Cof grad_ref v_c)
//   pressure - viscous: Q_c = p Cof^T e_c - (nu / det) G grad_ref v_c
// and R_a,c = sum_q w_q [ N_a m_c + grad_ref N_a . Q_c ] (w_q = 1/4), with J
// and grad_ref in the coarse reference coordinates.

// Test-function sums of one component of the element residual: with the
// Gauss abscissae g0, g1 and 1 - g0 = g1,
//   R_a += 1/4 sum_q [ N_a(q) m(q) + dN_a/ds(q) Qs(q) + dN_a/dt(q) Qt(q) ]
// for nodes a = 00, 10, 01, 11 (stride 2 in R: components interleaved).
// m and Q come from coarse-reference derivatives: m carries n^2 and Q carries
// n relative to the fine element's, so those factors and the weight 1/4 go
// into the outer constants.
template <int n>
__host__ __device__ inline void element_sums(const float m[2][2], const float Qs[2][2], const float Qt[2][2], float *R)
{
    constexpr float g0 = kGauss0, g1 = kGauss1;
    constexpr float hm0 = 0.25f * g0 / (n * n), hm1 = 0.25f * g1 / (n * n);
    constexpr float h0 = 0.25f * g0 / n, h1 = 0.25f * g1 / n;
    const float mb0 = g1 * m[0][0] + g0 * m[0][1], mb1 = g1 * m[1][0] + g0 * m[1][1];   // weight 1 - t
    const float mt0 = g0 * m[0][0] + g1 * m[0][1], mt1 = g0 * m[1][0] + g1 * m[1][1];   // weight t
    const float qs0 = Qs[0][0] + Qs[1][0], qs1 = Qs[0][1] + Qs[1][1];                   // sum over s
    const float qt0 = Qt[0][0] + Qt[0][1], qt1 = Qt[1][0] + Qt[1][1];                   // sum over t
    const float Sx0 = h1 * qs0 + h0 * qs1, Sx1 = h0 * qs0 + h1 * qs1;
    const float Sy0 = h1 * qt0 + h0 * qt1, Sy1 = h0 * qt0 + h1 * qt1;
    R[0] = hm1 * mb0 + hm0 * mb1 - Sx0 - Sy0;
    R[2] = hm0 * mb0 + hm1 * mb1 + Sx0 - Sy1;
    R[4] = hm1 * mt0 + hm0 * mt1 - Sx1 + Sy0;
    R[6] = hm0 * mt0 + hm1 * mt1 + Sx1 + Sy1;
}

// One fine element: column a, row b (0 .. n-1) of coarse element r; w0..w3
// the nodal u_prev / dt at its corners 00, 10, 01, 11, idt = 1/dt (the Gauss
// point value of (u_prev - v)/dt is the interpolated nodal u_prev / dt minus
// idt times v there).  R[2 a + c] is the residual of component c at corner a.
template <int K, typename Rcp>
__host__ __device__ inline void element_residual(const CoarseRec &r, int a, int b, float nu, float idt, float2 w0,
                                                 float2 w1, float2 w2, float2 w3, float (&R)[8])
{
    constexpr int n = 1 << K;
    constexpr float inv_n = 1.0f / n, g0 = kGauss0, g1 = kGauss1;
    const float xi[2] = {(a + g0) * inv_n, (a + g1) * inv_n};
    const float eta[2] = {(b + g0) * inv_n, (b + g1) * inv_n};
    float xsx[2], xsy[2], xtx[2], xty[2];          // x_s(eta_j), x_t(xi_i)
    float vsx[2], vsy[2], vtx[2], vty[2];          // v_xi(eta_j), v_eta(xi_i) per component
    float ax_[2], ay_[2], ap[2], bp[2];            // v = ax_ + vtx eta along xi_i
    for (int j = 0; j < 2; ++j) {
        xsx[j] = r.exx + r.exyx * eta[j]; xsy[j] = r.exy + r.exyy * eta[j];
        vsx[j] = r.V1x + r.V3x * eta[j]; vsy[j] = r.V1y + r.V3y * eta[j];
    }
    for (int i = 0; i < 2; ++i) {
        xtx[i] = r.eyx + r.exyx * xi[i]; xty[i] = r.eyy + r.exyy * xi[i];
        vtx[i] = r.V2x + r.V3x * xi[i]; vty[i] = r.V2y + r.V3y * xi[i];
        ax_[i] = r.V0x + r.V1x * xi[i];
        ay_[i] = r.V0y + r.V1y * xi[i];
        ap[i] = r.P0 + r.P1 * xi[i]; bp[i] = r.P2 + r.P3 * xi[i];
    }
    // u_prev / dt at the Gauss points from the element's nodal values
    float wx[2][2], wy[2][2];
    for (int i = 0; i < 2; ++i) {
        const float sg = i ? g1 : g0;
        const float bxv = w0.x + (w1.x - w0.x) * sg, txv = w2.x + (w3.x - w2.x) * sg;
        const float byv = w0.y + (w1.y - w0.y) * sg, tyv = w2.y + (w3.y - w2.y) * sg;
        wx[i][0] = bxv + (txv - bxv) * g0; wx[i][1] = bxv + (txv - bxv) * g1;
        wy[i][0] = byv + (tyv - byv) * g0; wy[i][1] = byv + (tyv - byv) * g1;
    }
    const float g11[2] = {xtx[0] * xtx[0] + xty[0] * xty[0], xtx[1] * xtx[1] + xty[1] * xty[1]};
    const float g22[2] = {xsx[0] * xsx[0] + xsy[0] * xsy[0], xsx[1] * xsx[1] + xsy[1] * xsy[1]};
    float mx[2][2], my[2][2], Qxs[2][2], Qxt[2][2], Qys[2][2], Qyt[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            const float xs = xsx[j], ys = xsy[j], xt = xtx[i], yt = xty[i];
            const float det = xs * yt - xt * ys;
            const float vxq = ax_[i] + vtx[i] * eta[j], vyq = ay_[i] + vty[i] * eta[j];
            const float pq = ap[i] + bp[i] * eta[j];
            // det grad v_c = Cof grad_ref v_c
            const float dxx = yt * vsx[j] - ys * vtx[i], dxy = -xt * vsx[j] + xs * vtx[i];
            const float dyx = yt * vsy[j] - ys * vty[i], dyy = -xt * vsy[j] + xs * vty[i];
            mx[i][j] = det * (wx[i][j] - idt * vxq) - (vxq * dxx + vyq * dxy);
            my[i][j] = det * (wy[i][j] - idt * vyq) - (vxq * dyx + vyq * dyy);
            const float g12 = -(xs * xt + ys * yt);
            const float inv = nu * Rcp::f(det);
            Qxs[i][j] = pq * yt - inv * (g11[i] * vsx[j] + g12 * vtx[i]);
            Qxt[i][j] = -pq * ys - inv * (g12 * vsx[j] + g22[j] * vtx[i]);
            Qys[i][j] = -pq * xt - inv * (g11[i] * vsy[j] + g12 * vty[i]);
            Qyt[i][j] = pq * xs - inv * (g12 * vsy[j] + g22[j] * vty[i]);
        }
    element_sums<n>(mx, Qxs, Qxt, R);
    element_sums<n>(my, Qys, Qyt, R + 1);
}

// The same element with the time scheme's weights (Crank-Nicolson at
// theta = 1/2): the new level's convection and diffusion weighted by theta,
// the old level's (the previous corrected velocity u, nodal values w0..w3 at
// the corners 00, 10, 01, 11) by 1 - theta:
//   m_c = det (u_c - v_c) / dt - theta v . (Cof grad_ref v_c) - (1 - theta) u . (Cof grad_ref u_c)
//   Q_c = p Cof^T e_c - (nu / det) G (theta grad_ref v_c + (1 - theta) grad_ref u_c)
// with grad_ref u from the element's bilinear nodal interpolant (n times its
// fine-element derivatives, in the coarse reference coordinates).
template <int K, typename Rcp>
__host__ __device__ inline void element_residual_theta(const CoarseRec &r, int a, int b, float nu, float idt,
                                                       float theta, float2 w0, float2 w1, float2 w2, float2 w3,
                                                       float (&R)[8])
{
    constexpr int n = 1 << K;
    constexpr float inv_n = 1.0f / n, g0 = kGauss0, g1 = kGauss1;
    const float th_old = 1.0f - theta;
    const float gs[2] = {g0, g1};
    // the previous velocity's nodal values on this element
    const float u00x = w0.x, u00y = w0.y, u10x = w1.x, u10y = w1.y;
    const float u01x = w2.x, u01y = w2.y, u11x = w3.x, u11y = w3.y;
    float mx[2][2], my[2][2], Qxs[2][2], Qxt[2][2], Qys[2][2], Qyt[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            const float s = gs[i], t = gs[j];                 // fine-element coordinates
            const float xi = (a + s) * inv_n, eta = (b + t) * inv_n;
            const float xs = r.exx + r.exyx * eta, ys = r.exy + r.exyy * eta;
            const float xt = r.eyx + r.exyx * xi, yt = r.eyy + r.exyy * xi;
            const float det = xs * yt - xt * ys;
            // new level: v, its coarse-reference gradient, p
            const float vxq = (r.V0x + r.V1x * xi) + (r.V2x + r.V3x * xi) * eta;
            const float vyq = (r.V0y + r.V1y * xi) + (r.V2y + r.V3y * xi) * eta;
            const float vsx = r.V1x + r.V3x * eta, vsy = r.V1y + r.V3y * eta;
            const float vtx = r.V2x + r.V3x * xi, vty = r.V2y + r.V3y * xi;
            const float pq = (r.P0 + r.P1 * xi) + (r.P2 + r.P3 * xi) * eta;
            // old level: u and its coarse-reference gradient
            const float uxq = (1 - t) * (u00x + (u10x - u00x) * s) + t * (u01x + (u11x - u01x) * s);
            const float uyq = (1 - t) * (u00y + (u10y - u00y) * s) + t * (u01y + (u11y - u01y) * s);
            const float usx = n * ((u10x - u00x) * (1 - t) + (u11x - u01x) * t);
            const float usy = n * ((u10y - u00y) * (1 - t) + (u11y - u01y) * t);
            const float utx = n * ((u01x - u00x) * (1 - s) + (u11x - u10x) * s);
            const float uty = n * ((u01y - u00y) * (1 - s) + (u11y - u10y) * s);
            // Cof grad_ref of each component, both levels
            const float dvxx = yt * vsx - ys * vtx, dvxy = -xt * vsx + xs * vtx;
            const float dvyx = yt * vsy - ys * vty, dvyy = -xt * vsy + xs * vty;
            const float duxx = yt * usx - ys * utx, duxy = -xt * usx + xs * utx;
            const float duyx = yt * usy - ys * uty, duyy = -xt * usy + xs * uty;
            mx[i][j] = det * idt * (uxq - vxq) - theta * (vxq * dvxx + vyq * dvxy) - th_old * (uxq * duxx + uyq * duxy);
            my[i][j] = det * idt * (uyq - vyq) - theta * (vxq * dvyx + vyq * dvyy) - th_old * (uxq * duyx + uyq * duyy);
            const float g11 = xt * xt + yt * yt, g22 = xs * xs + ys * ys, g12 = -(xs * xt + ys * yt);
            const float inv = nu * Rcp::f(det);
            const float gsx = theta * vsx + th_old * usx, gtx = theta * vtx + th_old * utx;
            const float gsy = theta * vsy + th_old * usy, gty = theta * vty + th_old * uty;
            Qxs[i][j] = pq * yt - inv * (g11 * gsx + g12 * gtx);
            Qxt[i][j] = -pq * ys - inv * (g12 * gsx + g22 * gtx);
            Qys[i][j] = -pq * xt - inv * (g11 * gsy + g12 * gty);
            Qyt[i][j] = pq * xs - inv * (g12 * gsy + g22 * gty);
        }
    element_sums<n>(mx, Qxs, Qxt, R);
    element_sums<n>(my, Qys, Qyt, R + 1);
}

// A vertical strip of SH fine elements of coarse element r: column a, rows
// b0 .. b0 + SH - 1.  The same sums as element_residual, arranged so that the
// work per Gauss point shrinks: on the coarse element
//   det          = d0 + d1 xi + d2 eta                 (no xi eta term)
//   det grad v_c = B_c(xi) + C_c eta                   (no xi eta term)
//   nu g12       = G0(xi) + G1(xi) eta,  nu g22 = k0 + k1 eta + k2 eta^2
// so at a fixed abscissa xi the viscous numerators are polynomials in eta,
//   nu (g11 v_c,xi + g12 v_c,eta) = E0 + E1 eta,
//   nu (g12 v_c,xi + g22 v_c,eta) = F0 + F1 eta + F2 eta^2,
// whose coefficients are formed once per abscissa and serve the 2 SH Gauss
// points of the strip on it.  The element sums are taken one abscissa at a
// time and added straight into the strip's nodes: S[k] is node row k (0 ..
// SH) as left x, left y, right x, right y (overwritten).  w points
// at the nodal u_prev / dt of the strip's lower-left node; rows are ldw apart;
// idt = 1/dt as in element_residual.
template <int K, int SH, typename Rcp>
__host__ __device__ inline void strip_residual(const CoarseRec &r, int a, int b0, float nu, float idt, const float2 *w,
                                               int ldw, float (&S)[SH + 1][4])
{
    constexpr int n = 1 << K;
    constexpr float inv_n = 1.0f / n, g0 = kGauss0, g1 = kGauss1;
    constexpr float hm0 = 0.25f * g0 / (n * n), hm1 = 0.25f * g1 / (n * n);
    constexpr float h0 = 0.25f * g0 / n, h1 = 0.25f * g1 / n;
    // strip constants
    const float d0 = r.exx * r.eyy - r.eyx * r.exy;
    const float d1 = r.exx * r.exyy - r.exyx * r.exy;
    const float d2 = r.exyx * r.eyy - r.eyx * r.exyy;
    // det d(v_c)/dx = Bx_c + Cx_c eta, det d(v_c)/dy = By_c + Cy_c eta, Bx_c = Bx0_c + Bx1_c xi, ...
    const float Bx0x = r.eyy * r.V1x - r.exy * r.V2x, Bx1x = r.exyy * r.V1x - r.exy * r.V3x;
    const float Cxx = r.eyy * r.V3x - r.exyy * r.V2x;
    const float By0x = r.exx * r.V2x - r.eyx * r.V1x, By1x = r.exx * r.V3x - r.exyx * r.V1x;
    const float Cyx = r.exyx * r.V2x - r.eyx * r.V3x;
    const float Bx0y = r.eyy * r.V1y - r.exy * r.V2y, Bx1y = r.exyy * r.V1y - r.exy * r.V3y;
    const float Cxy = r.eyy * r.V3y - r.exyy * r.V2y;
    const float By0y = r.exx * r.V2y - r.eyx * r.V1y, By1y = r.exx * r.V3y - r.exyx * r.V1y;
    const float Cyy = r.exyx * r.V2y - r.eyx * r.V3y;
    const float Cxx2 = Cxx + idt * d2, Cyy2 = Cyy + idt * d2;
    const float nexx = nu * r.exx, nexy = nu * r.exy, nexyx = nu * r.exyx, nexyy = nu * r.exyy;
    const float k0 = nexx * r.exx + nexy * r.exy;
    const float k1 = 2.0f * (nexx * r.exyx + nexy * r.exyy);
    const float k2 = nexyx * r.exyx + nexyy * r.exyy;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float gi = i ? g1 : g0;
        const float xi = (a + gi) * inv_n;
        const float xt = r.eyx + r.exyx * xi, yt = r.eyy + r.exyy * xi;
        const float vtx = r.V2x + r.V3x * xi, vty = r.V2y + r.V3y * xi;
        const float ax = r.V0x + r.V1x * xi, ay = r.V0y + r.V1y * xi;
        const float ap = r.P0 + r.P1 * xi, bp = r.P2 + r.P3 * xi;
        const float A = d0 + d1 * xi;
        // the mass term's -v_c det / dt joins the diagonal gradient terms:
        // det (w_c - v_c / dt) - v . det grad v_c
        //   = det w_c - v_x (det dv_c/dx + [c = x] det / dt) - v_y (det dv_c/dy + [c = y] det / dt)
        const float Bxx = Bx0x + Bx1x * xi + idt * A, Byx = By0x + By1x * xi;
        const float Bxy = Bx0y + Bx1y * xi, Byy = By0y + By1y * xi + idt * A;
        // with v_c = a_c + vt_c eta and det d(v_c)/dx_k = B + C eta on this
        // abscissa, v_x (det dv_c/dx + ...) + v_y (det dv_c/dy + ...) is a
        // quadratic in eta: its coefficients once per xi, two FMAs per point
        const float q0x = ax * Bxx + ay * Byx, q2x = vtx * Cxx2 + vty * Cyx;
        const float q1x = ax * Cxx2 + vtx * Bxx + ay * Cyx + vty * Byx;
        const float q0y = ax * Bxy + ay * Byy, q2y = vtx * Cxy + vty * Cyy2;
        const float q1y = ax * Cxy + vtx * Bxy + ay * Cyy2 + vty * Byy;
        const float g11 = nu * (xt * xt + yt * yt);
        const float G0 = -(nexx * xt + nexy * yt), G1 = -(nexyx * xt + nexyy * yt);
        const float E0x = g11 * r.V1x + G0 * vtx, E1x = g11 * r.V3x + G1 * vtx;
        const float E0y = g11 * r.V1y + G0 * vty, E1y = g11 * r.V3y + G1 * vty;
        const float F0x = G0 * r.V1x + k0 * vtx, F1x = G0 * r.V3x + G1 * r.V1x + k1 * vtx, F2x = G1 * r.V3x + k2 * vtx;
        const float F0y = G0 * r.V1y + k0 * vty, F1y = G0 * r.V3y + G1 * r.V1y + k1 * vty, F2y = G1 * r.V3y + k2 * vty;
        const float hmA = i ? hm0 : hm1, hmB = i ? hm1 : hm0, hA = i ? h0 : h1, hB = i ? h1 : h0;
        // nodal values interpolated to this abscissa along the element's lower
        // and upper node rows (the upper row carries over to the next element)
        float wxl, wyl;
        {
            const float2 wl = w[0], wr = w[1];
            wxl = wl.x + (wr.x - wl.x) * gi;
            wyl = wl.y + (wr.y - wl.y) * gi;
        }
#pragma unroll
        for (int k = 0; k < SH; ++k) {
            const float2 wl = w[(k + 1) * ldw], wr = w[(k + 1) * ldw + 1];
            const float wxu = wl.x + (wr.x - wl.x) * gi, wyu = wl.y + (wr.y - wl.y) * gi;
            float m[2][2], Qs[2][2], Qt[2][2];     // [component][eta point]
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const float gj = j ? g1 : g0;
                const float eta = (b0 + k + gj) * inv_n;
                const float xs = r.exx + r.exyx * eta, ys = r.exy + r.exyy * eta;
                const float det = A + d2 * eta;
                const float inv = Rcp::f(det);
                const float pq = ap + bp * eta;
                const float cvx = q0x + (q1x + q2x * eta) * eta, cvy = q0y + (q1y + q2y * eta) * eta;
                const float wxq = wxl + (wxu - wxl) * gj;
                const float wyq = wyl + (wyu - wyl) * gj;
                m[0][j] = det * wxq - cvx;
                m[1][j] = det * wyq - cvy;
                const float T1x = E0x + E1x * eta, T1y = E0y + E1y * eta;
                const float T2x = F0x + (F1x + F2x * eta) * eta, T2y = F0y + (F1y + F2y * eta) * eta;
                Qs[0][j] = pq * yt - inv * T1x;
                Qt[0][j] = -pq * ys - inv * T2x;
                Qs[1][j] = -pq * xt - inv * T1y;
                Qt[1][j] = pq * xs - inv * T2y;
            }
            wxl = wxu;
            wyl = wyu;
            // this abscissa's share of element k's sums (element_sums split by xi)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const float mb = g1 * m[c][0] + g0 * m[c][1], mt = g0 * m[c][0] + g1 * m[c][1];
                const float sx0 = h1 * Qs[c][0] + h0 * Qs[c][1], sx1 = h0 * Qs[c][0] + h1 * Qs[c][1];
                const float qt = Qt[c][0] + Qt[c][1];
                const float r0 = hmA * mb - sx0 - hA * qt, r2 = hmB * mb + sx0 - hB * qt;
                const float r4 = hmA * mt - sx1 + hA * qt, r6 = hmB * mt + sx1 + hB * qt;
                // the first pass writes each node once before adding to it
                if (i == 0 && k == 0) {
                    S[k][c] = r0;
                    S[k][2 + c] = r2;
                } else {
                    S[k][c] += r0;
                    S[k][2 + c] += r2;
                }
                if (i == 0) {
                    S[k + 1][c] = r4;
                    S[k + 1][2 + c] = r6;
                } else {
                    S[k + 1][c] += r4;
                    S[k + 1][2 + c] += r6;
                }
            }
            Rcp::fence();
        }
    }
}

// One fine element of an unstructured mesh with its own bilinear map: node
// coordinates x, y (corners 00, 10, 01, 11, relative to any origin), nodal
// velocity v, pressure p and u_prev / dt (w), idt = 1/dt; the same terms as
// element_residual with every derivative in the element's own reference
// coordinates:
//   m_c = det (w_c - idt v_c) - v . (Cof grad_ref v_c)
//   Q_c = p Cof^T e_c - (nu / det) G grad_ref v_c
//   R[2 a + c] = 1/4 sum_q [ N_a m_c + grad_ref N_a . Q_c ].
template <typename Rcp>
__host__ __device__ inline void quad_residual(const float (&x)[4], const float (&y)[4], const float (&vx)[4],
                                              const float (&vy)[4], const float (&pn)[4], const float (&wx)[4],
                                              const float (&wy)[4], float nu, float idt, float (&R)[8])
{
    constexpr float g0 = kGauss0, g1 = kGauss1;
    for (int k = 0; k < 8; ++k) R[k] = 0.0f;
    for (int q = 0; q < 4; ++q) {
        const float s = (q & 1) ? g1 : g0, t = (q >> 1) ? g1 : g0;
        const float N[4] = {(1.0f - s) * (1.0f - t), s * (1.0f - t), (1.0f - s) * t, s * t};
        const float Ns[4] = {-(1.0f - t), 1.0f - t, -t, t};
        const float Nt[4] = {-(1.0f - s), -s, 1.0f - s, s};
        float xs = 0.f, xt = 0.f, ys = 0.f, yt = 0.f, v0 = 0.f, v1 = 0.f, pq = 0.f, w0 = 0.f, w1 = 0.f;
        float vs0 = 0.f, vt0 = 0.f, vs1 = 0.f, vt1 = 0.f;
        for (int k = 0; k < 4; ++k) {
            xs += x[k] * Ns[k]; xt += x[k] * Nt[k];
            ys += y[k] * Ns[k]; yt += y[k] * Nt[k];
            v0 += N[k] * vx[k]; v1 += N[k] * vy[k];
            pq += N[k] * pn[k];
            w0 += N[k] * wx[k]; w1 += N[k] * wy[k];
            vs0 += vx[k] * Ns[k]; vt0 += vx[k] * Nt[k];
            vs1 += vy[k] * Ns[k]; vt1 += vy[k] * Nt[k];
        }
        const float det = xs * yt - xt * ys;
        const float dxx = yt * vs0 - ys * vt0, dxy = -xt * vs0 + xs * vt0;   // det grad v_x
        const float dyx = yt * vs1 - ys * vt1, dyy = -xt * vs1 + xs * vt1;   // det grad v_y
        const float m0 = det * (w0 - idt * v0) - (v0 * dxx + v1 * dxy);
        const float m1 = det * (w1 - idt * v1) - (v0 * dyx + v1 * dyy);
        const float inv = nu * Rcp::f(det);
        const float g11 = xt * xt + yt * yt, g22 = xs * xs + ys * ys, g12 = -(xs * xt + ys * yt);
        const float Qs0 = pq * yt - inv * (g11 * vs0 + g12 * vt0), Qt0 = -pq * ys - inv * (g12 * vs0 + g22 * vt0);
        const float Qs1 = -pq * xt - inv * (g11 * vs1 + g12 * vt1), Qt1 = pq * xs - inv * (g12 * vs1 + g22 * vt1);
        for (int a = 0; a < 4; ++a) {
            R[2 * a] += 0.25f * (N[a] * m0 + Ns[a] * Qs0 + Nt[a] * Qt0);
            R[2 * a + 1] += 0.25f * (N[a] * m1 + Ns[a] * Qs1 + Nt[a] * Qt1);
        }
    }
}

// ---------------------------------------------------------------- tile partition
// A defect tile owns kT x kT fine elements (kT = 32) and computes the ring of
// halo elements around them as well (tile-local element coordinates -1 .. kT).
// The own elements are vertical strips of SH elements inside one coarse
// element; thread (wave, lane) holds strip s of its SPL strips at element
// column ec and strip row sr.  Wave w holds the strips of colour w (column
// parity w & 1, strip-row parity w >> 1), so one wave's strips share no node.
constexpr int kTileElems = 32;

__host__ __device__ inline void strip_of(int wave, int lane, int s, int &ec, int &sr)
{
    ec = 2 * (lane & 15) + (wave & 1);
    sr = 2 * ((lane >> 4) + 4 * s) + (wave >> 1);
}

// Halo element of thread t (t < 4 (kT + 1)): the left and right columns with the
// corners, then the rows below and above.  colour is the one assembly round in
// which the element shares no node with that round's strips or with the other
// halo elements of that round.
__host__ __device__ inline void halo_of(int t, int &le, int &me, int &colour)
{
    constexpr int T = kTileElems;
    if (t < 2 * (T + 2)) {
        const int side = t / (T + 2);
        le = side ? T : -1;
        me = t - side * (T + 2) - 1;
        colour = side ? ((me & 1) ? 2 : 0) : ((me & 1) ? 3 : 1);
    } else {
        const int u = t - 2 * (T + 2), side = u / T;
        le = u - side * T;
        me = side ? T : -1;
        colour = side ? ((le & 1) ? 1 : 0) : ((le & 1) ? 3 : 2);
    }
}

}  // namespace dnnmg
