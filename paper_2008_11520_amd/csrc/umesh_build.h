// Host construction of the refined unstructured mesh (no HIP calls): the
// canonical fine node numbering of dnnmg_create_umesh, fine node coordinates
// (edges on circles refined along the arc, element interiors by the
// transfinite map of their four edge curves), the patch maps, the Dirichlet
// mask and the gather lists of the step's kernels.  A host test compares it
// with the FP64 reference implementation.
#pragma once

#include <cmath>
#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

namespace dnnmg {

struct UMeshHost {
    int nc = 0, ne = 0, E = 0, Fn = 0, K = 0, n = 0, nf = 0;
    std::vector<int> corners;           // ne x 4
    std::vector<int> pmap;              // ne x nf
    std::vector<double> fxy;            // Fn x 2
    std::vector<double> rel;            // ne x nf x 2, relative to the patch's corner v0
    std::vector<float> rel32;           // the same in FP32 (the defect's element maps)
    std::vector<unsigned char> mask;    // Fn
    std::vector<int> node_ptr, node_occ;    // Fn + 1, ne nf (patch nf + l, patch order)
    std::vector<int> cnode_ptr, cnode_occ;  // nc + 1, 4 ne (patch 4 + corner)
    std::vector<float> feat;            // ne x 4: hx, hy, hx / hy, area
    // A patch with straight edges is the bilinear image of the reference
    // square, its fine elements those of the uniform sub-squares: its mass
    // products against the coarse hats are exact moments of det J = d0 + d1 s
    // + d2 t (the structured rhs tables).  dgeo: d0, d1, d2 (and 0) per patch.
    std::vector<double> dgeo;           // ne x 4
    // A patch with a curved edge keeps its mass products weighted by its
    // coarse hats (static geometry): its share of R M_f u at corner c is
    // sum_l W[c][l] u_l, and for u = P v inside the patch sum_k M4[c][k] v_k.
    // cidx: the patch's row of W and M4, or -1 (straight edges).
    std::vector<int> cidx;              // ne
    std::vector<double> W;              // (patches with a curved edge) x 4 x nf
    std::vector<double> M4;             // (patches with a curved edge) x 4 x 4
};

namespace umesh_detail {

inline uint64_t edge_key(int a, int b)
{
    const uint32_t lo = (uint32_t)(a < b ? a : b), hi = (uint32_t)(a < b ? b : a);
    return ((uint64_t)lo << 32) | hi;
}

// Point at parameter s of the edge from node a to node b: straight, or the
// arc of circle `circ` (angle linear in s, the shorter way round).
inline void edge_point(const double *xy, int a, int b, double s, int circ, const double *circles, double *out)
{
    const double ax = xy[2 * a], ay = xy[2 * a + 1], bx = xy[2 * b], by = xy[2 * b + 1];
    if (circ < 0) {
        out[0] = ax + s * (bx - ax);
        out[1] = ay + s * (by - ay);
        return;
    }
    const double cx = circles[3 * circ], cy = circles[3 * circ + 1], r = circles[3 * circ + 2];
    const double ta = std::atan2(ay - cy, ax - cx);
    double d = std::atan2(by - cy, bx - cx) - ta;
    const double pi = 3.14159265358979323846;
    if (d > pi) d -= 2.0 * pi;
    if (d < -pi) d += 2.0 * pi;
    out[0] = cx + r * std::cos(ta + s * d);
    out[1] = cy + r * std::sin(ta + s * d);
}

}  // namespace umesh_detail

// Builds the refined mesh; returns "" or the reason the mesh is rejected.
inline std::string build_umesh(int nc, int ne, const double *xy, const int *elems, int ndir, const int *dir_edges,
                               int ncirc, const double *circles, int ncurved, const int *curved, int K,
                               UMeshHost &m)
{
    using namespace umesh_detail;
    if (nc < 4 || ne < 1) return "a mesh needs at least 4 nodes and 1 element";
    if (K < 1 || K > 3) return "K must be 1, 2 or 3";
    for (int i = 0; i < 2 * nc; ++i)
        if (!std::isfinite(xy[i])) return "node coordinates must be finite";
    m = UMeshHost();
    m.nc = nc; m.ne = ne; m.K = K; m.n = 1 << K; m.nf = (m.n + 1) * (m.n + 1);
    const int n = m.n, nf = m.nf;
    m.corners.assign(elems, elems + 4 * (size_t)ne);
    // edges in order of first appearance; each used by at most two elements,
    // in opposite directions (a consistently oriented mesh)
    struct EdgeUse { int index, uses, from; };
    std::unordered_map<uint64_t, EdgeUse> edges;
    edges.reserve(4 * (size_t)ne);
    std::vector<int> eidx(4 * (size_t)ne);
    for (int e = 0; e < ne; ++e) {
        const int *v = elems + 4 * e;
        for (int k = 0; k < 4; ++k)
            if (v[k] < 0 || v[k] >= nc) return "element node index out of range";
        for (int k = 0; k < 4; ++k)
            for (int j = k + 1; j < 4; ++j)
                if (v[k] == v[j]) return "an element repeats a node";
        const int ends[4][2] = {{v[0], v[1]}, {v[1], v[2]}, {v[3], v[2]}, {v[0], v[3]}};
        const bool ccw[4] = {true, true, false, false};   // local edge direction along the element's boundary
        for (int k = 0; k < 4; ++k) {
            const uint64_t key = edge_key(ends[k][0], ends[k][1]);
            const int from = ccw[k] ? ends[k][0] : ends[k][1];   // where the counter-clockwise walk enters it
            auto it = edges.find(key);
            if (it == edges.end()) {
                edges.emplace(key, EdgeUse{(int)edges.size(), 1, from});
                eidx[4 * e + k] = (int)edges.size() - 1;
            } else {
                if (it->second.uses >= 2) return "an edge is shared by more than two elements";
                if (it->second.from == from) return "neighbouring elements are not oriented alike";
                it->second.uses++;
                eidx[4 * e + k] = it->second.index;
            }
        }
    }
    m.E = (int)edges.size();
    m.Fn = nc + m.E * (n - 1) + ne * (n - 1) * (n - 1);
    if ((double)m.Fn * 2 > 2e9 || (double)ne * nf > 2e9) return "mesh too large";
    // curved edges: endpoints on their circle, the edge in the mesh
    std::unordered_map<uint64_t, int> curve;
    for (int k = 0; k < ncurved; ++k) {
        const int a = curved[3 * k], b = curved[3 * k + 1], c = curved[3 * k + 2];
        if (a < 0 || a >= nc || b < 0 || b >= nc || c < 0 || c >= ncirc) return "curved edge index out of range";
        if (!(circles[3 * c + 2] > 0.0)) return "circle radius must be > 0";
        for (int q : {a, b}) {
            const double d = std::hypot(xy[2 * q] - circles[3 * c], xy[2 * q + 1] - circles[3 * c + 1]);
            if (std::fabs(d - circles[3 * c + 2]) > 1e-9 * circles[3 * c + 2])
                return "a curved edge's node is not on its circle";
        }
        if (!edges.count(edge_key(a, b))) return "a curved edge is not an edge of the mesh";
        curve[edge_key(a, b)] = c;
    }
    auto curve_of = [&](int a, int b) {
        auto it = curve.find(edge_key(a, b));
        return it == curve.end() ? -1 : it->second;
    };
    // fine nodes and patch maps
    m.fxy.assign(2 * (size_t)m.Fn, 0.0);
    m.pmap.assign((size_t)ne * nf, -1);
    for (int i = 0; i < 2 * nc; ++i) m.fxy[i] = xy[i];
    const int base_in = nc + m.E * (n - 1);
    for (int e = 0; e < ne; ++e) {
        const int *v = elems + 4 * e;
        const int ends[4][2] = {{v[0], v[1]}, {v[1], v[2]}, {v[3], v[2]}, {v[0], v[3]}};
        int circ[4];
        for (int k = 0; k < 4; ++k) circ[k] = curve_of(ends[k][0], ends[k][1]);
        for (int b = 0; b <= n; ++b)
            for (int a = 0; a <= n; ++a) {
                int f, k = -1, along = 0;
                if (b == 0 && a > 0 && a < n) { k = 0; along = a; }
                else if (a == n && b > 0 && b < n) { k = 1; along = b; }
                else if (b == n && a > 0 && a < n) { k = 2; along = a; }
                else if (a == 0 && b > 0 && b < n) { k = 3; along = b; }
                if (a == 0 && b == 0) f = v[0];
                else if (a == n && b == 0) f = v[1];
                else if (a == n && b == n) f = v[2];
                else if (a == 0 && b == n) f = v[3];
                else if (k >= 0) {
                    const int p = ends[k][0], q = ends[k][1], lo = p < q ? p : q, hi = p < q ? q : p;
                    const int t = p < q ? along : n - along;
                    f = nc + eidx[4 * e + k] * (n - 1) + t - 1;
                    edge_point(xy, lo, hi, (double)t / n, circ[k], circles, &m.fxy[2 * (size_t)f]);
                } else {
                    f = base_in + e * (n - 1) * (n - 1) + (b - 1) * (n - 1) + (a - 1);
                    const double s = (double)a / n, t = (double)b / n;
                    double B[2], T[2], L[2], R[2];
                    edge_point(xy, v[0], v[1], s, circ[0], circles, B);
                    edge_point(xy, v[3], v[2], s, circ[2], circles, T);
                    edge_point(xy, v[0], v[3], t, circ[3], circles, L);
                    edge_point(xy, v[1], v[2], t, circ[1], circles, R);
                    for (int c = 0; c < 2; ++c) {
                        const double corner = (1 - s) * (1 - t) * xy[2 * v[0] + c] + s * (1 - t) * xy[2 * v[1] + c] +
                                              s * t * xy[2 * v[2] + c] + (1 - s) * t * xy[2 * v[3] + c];
                        m.fxy[2 * (size_t)f + c] = (1 - t) * B[c] + t * T[c] + (1 - s) * L[c] + s * R[c] - corner;
                    }
                }
                m.pmap[(size_t)e * nf + b * (n + 1) + a] = f;
            }
    }
    // positively oriented fine elements (det of a bilinear map is affine in
    // each variable: positive at the four corners means positive throughout)
    m.rel.assign((size_t)ne * nf * 2, 0.0);
    for (int e = 0; e < ne; ++e) {
        const double ox = xy[2 * elems[4 * e]], oy = xy[2 * elems[4 * e] + 1];
        for (int l = 0; l < nf; ++l) {
            const int f = m.pmap[(size_t)e * nf + l];
            m.rel[((size_t)e * nf + l) * 2] = m.fxy[2 * (size_t)f] - ox;
            m.rel[((size_t)e * nf + l) * 2 + 1] = m.fxy[2 * (size_t)f + 1] - oy;
        }
        for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) {
                const double *r00 = &m.rel[((size_t)e * nf + b * (n + 1) + a) * 2];
                const double *r10 = r00 + 2, *r01 = r00 + 2 * (n + 1), *r11 = r01 + 2;
                const double *P[4] = {r00, r10, r11, r01};
                for (int c = 0; c < 4; ++c) {
                    const double *o = P[c], *x1 = P[(c + 1) % 4], *x3 = P[(c + 3) % 4];
                    const double cr = (x1[0] - o[0]) * (x3[1] - o[1]) - (x1[1] - o[1]) * (x3[0] - o[0]);
                    if (!(cr > 0.0)) return "a fine element is not positively oriented";
                }
            }
    }
    m.rel32.assign(m.rel.begin(), m.rel.end());
    // Dirichlet mask
    m.mask.assign((size_t)m.Fn, 0);
    std::unordered_map<uint64_t, int> dir;
    for (int k = 0; k < ndir; ++k) {
        const int a = dir_edges[2 * k], b = dir_edges[2 * k + 1];
        if (a < 0 || a >= nc || b < 0 || b >= nc || !edges.count(edge_key(a, b)))
            return "a Dirichlet edge is not an edge of the mesh";
        dir[edge_key(a, b)] = 1;
    }
    for (int e = 0; e < ne; ++e) {
        const int *v = elems + 4 * e;
        const int ends[4][2] = {{v[0], v[1]}, {v[1], v[2]}, {v[3], v[2]}, {v[0], v[3]}};
        for (int k = 0; k < 4; ++k) {
            if (!dir.count(edge_key(ends[k][0], ends[k][1]))) continue;
            for (int t = 0; t <= n; ++t) {
                const int a = (k == 0 || k == 2) ? t : (k == 1 ? n : 0);
                const int b = (k == 1 || k == 3) ? t : (k == 2 ? n : 0);
                m.mask[m.pmap[(size_t)e * nf + b * (n + 1) + a]] = 1;
            }
        }
    }
    // gather lists (counting sort keeps patch order)
    m.node_ptr.assign((size_t)m.Fn + 1, 0);
    for (int x : m.pmap) m.node_ptr[x + 1]++;
    for (int f = 0; f < m.Fn; ++f) m.node_ptr[f + 1] += m.node_ptr[f];
    m.node_occ.assign((size_t)ne * nf, 0);
    {
        std::vector<int> at(m.node_ptr.begin(), m.node_ptr.end() - 1);
        for (int e = 0; e < ne; ++e)
            for (int l = 0; l < nf; ++l) m.node_occ[at[m.pmap[(size_t)e * nf + l]]++] = e * nf + l;
    }
    m.cnode_ptr.assign((size_t)nc + 1, 0);
    for (int i = 0; i < 4 * ne; ++i) m.cnode_ptr[elems[i] + 1]++;
    for (int c = 0; c < nc; ++c) m.cnode_ptr[c + 1] += m.cnode_ptr[c];
    m.cnode_occ.assign(4 * (size_t)ne, 0);
    {
        std::vector<int> at(m.cnode_ptr.begin(), m.cnode_ptr.end() - 1);
        for (int e = 0; e < ne; ++e)
            for (int k = 0; k < 4; ++k) m.cnode_occ[at[elems[4 * e + k]]++] = 4 * e + k;
    }
    // hat-weighted mass rows: 2 x 2 Gauss points on every fine element's own
    // bilinear map; W[c][l_j] += sum_q w |det| N_j(q) sum_k H_c(l_k) N_k(q),
    // H_c(l) the coarse hat of corner c at patch-local node l
    m.dgeo.assign(4 * (size_t)ne, 0.0);
    m.cidx.assign((size_t)ne, -1);
    int ncp = 0;
    for (int e = 0; e < ne; ++e) {
        const int *v = elems + 4 * e;
        const double *x0 = xy + 2 * v[0], *x1 = xy + 2 * v[1], *x2 = xy + 2 * v[2], *x3 = xy + 2 * v[3];
        const double exx = x1[0] - x0[0], exy = x1[1] - x0[1], eyx = x3[0] - x0[0], eyy = x3[1] - x0[1];
        const double fx = x2[0] - x1[0] - x3[0] + x0[0], fy = x2[1] - x1[1] - x3[1] + x0[1];
        double *g = &m.dgeo[4 * (size_t)e];
        g[0] = exx * eyy - eyx * exy;
        g[1] = exx * fy - fx * exy;
        g[2] = fx * eyy - eyx * fy;
        const int ends[4][2] = {{v[0], v[1]}, {v[1], v[2]}, {v[3], v[2]}, {v[0], v[3]}};
        bool curved = false;
        for (int k = 0; k < 4; ++k) curved = curved || curve_of(ends[k][0], ends[k][1]) >= 0;
        if (curved) m.cidx[e] = ncp++;
    }
    m.W.assign((size_t)ncp * 4 * nf, 0.0);
    m.M4.assign((size_t)ncp * 16, 0.0);
    {
        const double g[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
        auto hat = [&](int c, int l) {
            const double s = (double)(l % (n + 1)) / n, t = (double)(l / (n + 1)) / n;
            return c == 0 ? (1 - s) * (1 - t) : c == 1 ? s * (1 - t) : c == 2 ? s * t : (1 - s) * t;
        };
        for (int e = 0; e < ne; ++e) {
            if (m.cidx[e] < 0) continue;
            double *We = &m.W[(size_t)m.cidx[e] * 4 * nf];
            for (int b = 0; b < n; ++b)
                for (int a = 0; a < n; ++a) {
                    const int l00 = b * (n + 1) + a, ls[4] = {l00, l00 + 1, l00 + n + 1, l00 + n + 2};
                    for (int q = 0; q < 4; ++q) {
                        const double s = g[q & 1], t = g[q >> 1];
                        const double N[4] = {(1 - s) * (1 - t), s * (1 - t), (1 - s) * t, s * t};
                        const double Ns[4] = {-(1 - t), 1 - t, -t, t}, Nt[4] = {-(1 - s), -s, 1 - s, s};
                        double xs = 0, xt = 0, ys = 0, yt = 0;
                        for (int k = 0; k < 4; ++k) {
                            const double *r = &m.rel[((size_t)e * nf + ls[k]) * 2];
                            xs += r[0] * Ns[k]; xt += r[0] * Nt[k];
                            ys += r[1] * Ns[k]; yt += r[1] * Nt[k];
                        }
                        const double wd = 0.25 * std::fabs(xs * yt - xt * ys);
                        for (int c = 0; c < 4; ++c) {
                            double hq = 0.0;
                            for (int k = 0; k < 4; ++k) hq += hat(c, ls[k]) * N[k];
                            for (int j = 0; j < 4; ++j) We[(size_t)c * nf + ls[j]] += wd * N[j] * hq;
                        }
                    }
                }
            for (int c = 0; c < 4; ++c)
                for (int k = 0; k < 4; ++k) {
                    double acc = 0.0;
                    for (int l = 0; l < nf; ++l) acc += We[(size_t)c * nf + l] * hat(k, l);
                    m.M4[(size_t)m.cidx[e] * 16 + 4 * c + k] = acc;
                }
        }
    }
    // patch features from the straight corners
    m.feat.assign(4 * (size_t)ne, 0.0f);
    for (int e = 0; e < ne; ++e) {
        const double *c0 = xy + 2 * elems[4 * e], *c1 = xy + 2 * elems[4 * e + 1];
        const double *c2 = xy + 2 * elems[4 * e + 2], *c3 = xy + 2 * elems[4 * e + 3];
        const double hx = 0.5 * (std::hypot(c1[0] - c0[0], c1[1] - c0[1]) + std::hypot(c2[0] - c3[0], c2[1] - c3[1]));
        const double hy = 0.5 * (std::hypot(c3[0] - c0[0], c3[1] - c0[1]) + std::hypot(c2[0] - c1[0], c2[1] - c1[1]));
        const double area = 0.5 * std::fabs((c2[0] - c0[0]) * (c3[1] - c1[1]) - (c2[1] - c0[1]) * (c3[0] - c1[0]));
        float *o = &m.feat[4 * (size_t)e];
        o[0] = (float)hx; o[1] = (float)hy; o[2] = (float)(hx / hy); o[3] = (float)area;
    }
    return std::string();
}

}  // namespace dnnmg
