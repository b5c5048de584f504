// Host check of the fine-element code shared with the defect kernels
// (paper_2008_11520_amd/csrc/element.h):
//   1. strip_residual equals the sum of element_residual over the strip's
//      elements (random coarse elements: skewed, stretched, 1e-2 .. 1e2 in size);
//   2. element_residual_theta and quad_residual (unstructured meshes) against
//      element_residual on the same element;
//   3. the tile partition (strip_of, halo_of) covers the tile's 32 x 32
//      elements and its halo ring exactly once, and within each of the four
//      assembly rounds no node receives two contributions.
// Prints one line per check and exits non-zero on a failure.
#include "element.h"

#include <cmath>
#include <cstdio>
#include <map>
#include <random>
#include <set>
#include <utility>

using namespace dnnmg;

struct HostOps {
    static float f(float x) { return 1.0f / x; }
    static void fence() {}
};

template <int K, int SH>
static double strip_vs_elements(std::mt19937 &g, int trials)
{
    constexpr int n = 1 << K;
    std::uniform_real_distribution<float> U(-1.f, 1.f);
    double worst = 0;
    for (int t = 0; t < trials; ++t) {
        CoarseRec r;
        float *v = &r.V0x;
        for (int q = 0; q < 12; ++q) v[q] = U(g) * (q % 4 == 0 ? 2.f : 0.7f);
        const float sc = std::pow(10.f, 2 * U(g));
        r.exx = sc * (1.f + 0.3f * U(g)); r.exy = sc * 0.3f * U(g);
        r.eyx = sc * 0.3f * U(g); r.eyy = sc * (1.f + 0.3f * U(g)) * (1 + 3 * (t % 2));
        r.exyx = sc * 0.2f * U(g); r.exyy = sc * 0.2f * U(g);
        const float nu = 1e-3f * (1 + 10 * (t % 3)), idt = (t % 4 == 0) ? 0.f : 200.f;
        const int a = t % n, b0 = ((t / n) % (n / SH)) * SH, ldw = 7;
        float2 w[(SH + 1) * 7];
        for (auto &x : w) { x.x = U(g) * 300; x.y = U(g) * 300; }
        float S[SH + 1][4];
        strip_residual<K, SH, HostOps>(r, a, b0, nu, idt, w, ldw, S);
        float E[SH + 1][4] = {};
        float mag = 0;
        for (int k = 0; k < SH; ++k) {
            float R[8];
            element_residual<K, HostOps>(r, a, b0 + k, nu, idt, w[k * ldw], w[k * ldw + 1], w[(k + 1) * ldw],
                                         w[(k + 1) * ldw + 1], R);
            for (int c = 0; c < 4; ++c) { E[k][c] += R[c]; E[k + 1][c] += R[4 + c]; }
            for (float x : R) mag = std::fmax(mag, std::fabs(x));
        }
        for (int k = 0; k <= SH; ++k)
            for (int c = 0; c < 4; ++c) worst = std::fmax(worst, std::fabs(S[k][c] - E[k][c]) / mag);
    }
    return worst;
}

// element_residual_theta at theta = 1 against element_residual (the same
// implicit-Euler sums, arranged differently), and at theta = 1/2 with the old
// level equal to the new one (u = v at the nodes of a bilinear v, so both
// levels' transport terms are the same and the weights must add up to one).
template <int K>
static double theta_form_vs_element_form(std::mt19937 &g, int trials)
{
    constexpr int n = 1 << K;
    std::uniform_real_distribution<float> U(-1.f, 1.f);
    double worst = 0;
    for (int t = 0; t < trials; ++t) {
        CoarseRec r;
        float *v = &r.V0x;
        for (int q = 0; q < 12; ++q) v[q] = U(g) * (q % 4 == 0 ? 2.f : 0.7f);
        const float sc = std::pow(10.f, 2 * U(g));
        r.exx = sc * (1.f + 0.3f * U(g)); r.exy = sc * 0.3f * U(g);
        r.eyx = sc * 0.3f * U(g); r.eyy = sc * (1.f + 0.3f * U(g));
        r.exyx = sc * 0.2f * U(g); r.exyy = sc * 0.2f * U(g);
        const bool same = t % 2;   // u = v at the corners (bilinear v): theta = 1/2 must equal theta = 1
        // (with u = v the mass term is left out: u - v would only hold the
        // two evaluations' rounding, amplified by 1/dt)
        const float nu = 1e-3f * (1 + 10 * (t % 3)), idt = same ? 0.f : 200.f;
        const int a = t % n, b = (t / n) % n;
        float2 u[4];
        for (int c = 0; c < 4; ++c) {
            const float xi = (a + (c & 1)) * (1.0f / n), eta = (b + (c >> 1)) * (1.0f / n);
            if (same) {
                u[c].x = (r.V0x + r.V1x * xi) + (r.V2x + r.V3x * xi) * eta;
                u[c].y = (r.V0y + r.V1y * xi) + (r.V2y + r.V3y * xi) * eta;
            } else {
                u[c].x = 2 * U(g); u[c].y = 2 * U(g);
            }
        }
        float Rt[8], Re[8];
        element_residual_theta<K, HostOps>(r, a, b, nu, idt, same ? 0.5f : 1.0f, u[0], u[1], u[2], u[3], Rt);
        float2 w[4];
        for (int c = 0; c < 4; ++c) w[c] = {u[c].x * idt, u[c].y * idt};
        element_residual<K, HostOps>(r, a, b, nu, idt, w[0], w[1], w[2], w[3], Re);
        float mag = 0;
        for (float x : Re) mag = std::fmax(mag, std::fabs(x));
        for (int c = 0; c < 8; ++c) worst = std::fmax(worst, std::fabs(Rt[c] - Re[c]) / mag);
    }
    return worst;
}

// quad_residual (an unstructured mesh's fine element with its own bilinear
// map and nodal values) against element_residual on the same fine element of
// a coarse element: node coordinates from the coarse map, nodal v and p from
// the coarse bilinear fields, random nodal u_prev / dt.
template <int K>
static double quad_vs_element(std::mt19937 &g, int trials)
{
    constexpr int n = 1 << K;
    std::uniform_real_distribution<float> U(-1.f, 1.f);
    double worst = 0;
    for (int t = 0; t < trials; ++t) {
        CoarseRec r;
        float *v = &r.V0x;
        for (int q = 0; q < 12; ++q) v[q] = U(g) * (q % 4 == 0 ? 2.f : 0.7f);
        const float sc = std::pow(10.f, 2 * U(g));
        r.exx = sc * (1.f + 0.3f * U(g)); r.exy = sc * 0.3f * U(g);
        r.eyx = sc * 0.3f * U(g); r.eyy = sc * (1.f + 0.3f * U(g));
        r.exyx = sc * 0.2f * U(g); r.exyy = sc * 0.2f * U(g);
        const float nu = 1e-3f * (1 + 10 * (t % 3)), idt = (t % 4 == 0) ? 0.f : 200.f;
        const int a = t % n, b = (t / n) % n;
        float x[4], y[4], vx[4], vy[4], pn[4], wx[4], wy[4];
        float2 w[4];
        for (int c = 0; c < 4; ++c) {
            const float xi = (a + (c & 1)) * (1.0f / n), eta = (b + (c >> 1)) * (1.0f / n);
            x[c] = r.exx * xi + r.eyx * eta + r.exyx * xi * eta;
            y[c] = r.exy * xi + r.eyy * eta + r.exyy * xi * eta;
            vx[c] = (r.V0x + r.V1x * xi) + (r.V2x + r.V3x * xi) * eta;
            vy[c] = (r.V0y + r.V1y * xi) + (r.V2y + r.V3y * xi) * eta;
            pn[c] = (r.P0 + r.P1 * xi) + (r.P2 + r.P3 * xi) * eta;
            w[c] = {U(g) * 300, U(g) * 300};
            wx[c] = w[c].x; wy[c] = w[c].y;
        }
        float Rq[8], Re[8];
        quad_residual<HostOps>(x, y, vx, vy, pn, wx, wy, nu, idt, Rq);
        element_residual<K, HostOps>(r, a, b, nu, idt, w[0], w[1], w[2], w[3], Re);
        float mag = 0;
        for (float z : Re) mag = std::fmax(mag, std::fabs(z));
        for (int c = 0; c < 8; ++c) worst = std::fmax(worst, std::fabs(Rq[c] - Re[c]) / mag);
    }
    return worst;
}

template <int SH>
static bool partition_ok(int K)
{
    constexpr int T = kTileElems, NSR = T / SH, SPL = T * NSR / 256;
    const int n = 1 << K;
    std::map<std::pair<int, int>, int> cover;
    std::map<int, std::map<std::pair<int, int>, int>> rounds;   // colour -> node -> contributions
    for (int tid = 0; tid < 256; ++tid) {
        const int wave = tid >> 6, lane = tid & 63;
        for (int s = 0; s < SPL; ++s) {
            int ec, sr;
            strip_of(wave, lane, s, ec, sr);
            if ((sr * SH) / n != (sr * SH + SH - 1) / n) return false;      // one coarse element
            for (int k = 0; k < SH; ++k) cover[{ec, sr * SH + k}]++;
            for (int dx = 0; dx < 2; ++dx)
                for (int k = 0; k <= SH; ++k) rounds[wave][{ec + dx, sr * SH + k}]++;
        }
    }
    for (int t = 0; t < 4 * (T + 1); ++t) {
        int le, me, colour;
        halo_of(t, le, me, colour);
        cover[{le, me}]++;
        for (int dx = 0; dx < 2; ++dx)
            for (int dy = 0; dy < 2; ++dy) rounds[colour][{le + dx, me + dy}]++;
    }
    if ((int)cover.size() != (T + 2) * (T + 2)) return false;
    for (auto &e : cover)
        if (e.second != 1 || e.first.first < -1 || e.first.first > T || e.first.second < -1 || e.first.second > T)
            return false;
    for (auto &r : rounds)
        for (auto &nd : r.second)
            if (nd.second != 1) return false;
    return true;
}

int main()
{
    std::mt19937 g(7);
    const double e1 = strip_vs_elements<1, 2>(g, 20000), e2 = strip_vs_elements<2, 4>(g, 20000),
                 e3 = strip_vs_elements<3, 4>(g, 20000);
    std::printf("strip vs elements, max relative difference: K=1 %.3g  K=2 %.3g  K=3 %.3g\n", e1, e2, e3);
    const double t1 = theta_form_vs_element_form<1>(g, 20000), t2 = theta_form_vs_element_form<2>(g, 20000),
                 t3 = theta_form_vs_element_form<3>(g, 20000);
    std::printf("theta form (theta = 1, and theta = 1/2 with u = v) vs element form: K=1 %.3g  K=2 %.3g  K=3 %.3g\n",
                t1, t2, t3);
    const double q1 = quad_vs_element<1>(g, 20000), q2 = quad_vs_element<2>(g, 20000),
                 q3 = quad_vs_element<3>(g, 20000);
    std::printf("unstructured fine element vs element form: K=1 %.3g  K=2 %.3g  K=3 %.3g\n", q1, q2, q3);
    const bool p1 = partition_ok<2>(1), p2 = partition_ok<4>(2), p3 = partition_ok<4>(3);
    std::printf("tile partition: K=1 %s  K=2 %s  K=3 %s\n", p1 ? "ok" : "FAIL", p2 ? "ok" : "FAIL", p3 ? "ok" : "FAIL");
    return (e1 < 1e-5 && e2 < 1e-5 && e3 < 1e-5 && t1 < 1e-5 && t2 < 1e-5 && t3 < 1e-5 && q1 < 1e-5 && q2 < 1e-5 &&
            q3 < 1e-5 && p1 && p2 && p3) ? 0 : 1;
}
