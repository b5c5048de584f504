// The tile frame that the one-launch step hands to the rhs kernel, and the
// nodal P v + d formula both kernels use, host and device (a host test
// replays the frame's index math over ragged meshes).
//
// Duplicate averaging (Sec. 4.2) needs, at a fine node, the outputs of every
// patch that holds it.  The one-launch step (K = 2) has the outputs of its
// tile's TP x TP patches in LDS, so it completes every tile node whose
// patches all lie in the tile, i.e. all but the nodes on the tile's four
// boundary lines.  Of those it writes the corrected velocity P v + d straight
// into the state (and d into the caller's output) at the "deep" nodes, which
// no other tile's defect reads: a tile's defect reads its neighbours' nodes
// up to one fine node past the shared line, so the nodes one step inside
// the lines (li or lj = 1 or kFrameLine - 1) are still being read and are
// handed over instead ("inner" frame nodes: their averaged d).  The nodes on
// the lines ("edge") are handed over as the tile's own outputs there; the
// rhs kernel adds its neighbours' and completes them.
#pragma once

#ifndef __HIP__
#include <cmath>
#ifndef DNNMG_HD
#define DNNMG_HD
#endif
#else
#include <hip/hip_runtime.h>
#ifndef DNNMG_HD
#define DNNMG_HD __host__ __device__
#endif
#endif

namespace dnnmg {

constexpr int kFrameLine = 32;   // fine elements per tile side (the defect and rhs tiles)

enum FrameKind { kFrameDeep = 0, kFrameInner = 1, kFrameEdge = 2 };

// Tile node (li, lj), 0 <= li, lj <= kFrameLine.
DNNMG_HD inline int frame_kind(int li, int lj)
{
    if (li == 0 || lj == 0 || li == kFrameLine || lj == kFrameLine) return kFrameEdge;
    if (li == 1 || lj == 1 || li == kFrameLine - 1 || lj == kFrameLine - 1) return kFrameInner;
    return kFrameDeep;
}

// Per tile: four sides of TP (n + 1) values (L: the patches of tile column 0
// at their node column a = 0; R: column TP - 1 at a = n; B: row 0 at node row
// b = 0; T: row TP - 1 at b = n; in patch order, then node order along the
// side), then the inner nodes' averaged corrections: rows lj = 1 and
// lj = kFrameLine - 1 (li = 1 .. kFrameLine - 1), then columns li = 1 and
// li = kFrameLine - 1 (lj = 2 .. kFrameLine - 2).  One float2 per slot.
template <int K>
struct TileFrame {
    static constexpr int n = 1 << K;
    static constexpr int TP = kFrameLine / n;
    static constexpr int SIDE = TP * (n + 1);
    static constexpr int RUN = kFrameLine - 1;
    static constexpr int INNER = 2 * RUN + 2 * (RUN - 2);
    static constexpr int SIZE = 4 * SIDE + INNER;

    DNNMG_HD static int inner_slot(int li, int lj)
    {
        if (lj == 1) return 4 * SIDE + li - 1;
        if (lj == kFrameLine - 1) return 4 * SIDE + RUN + li - 1;
        if (li == 1) return 4 * SIDE + 2 * RUN + lj - 2;
        return 4 * SIDE + 2 * RUN + (RUN - 2) + lj - 2;
    }
    // Inverse of inner_slot: the tile node of inner slot k (0 <= k < INNER).
    // (each coordinate by its own selects: branches that assign one or the
    // other make the compiler keep the pair in scratch memory)
    DNNMG_HD static void inner_pos(int k, int &li, int &lj)
    {
        const bool r0 = k < RUN, r1 = k < 2 * RUN, c0 = k < 3 * RUN - 2;
        li = r0 ? 1 + k : (r1 ? 1 + k - RUN : (c0 ? 1 : kFrameLine - 1));
        lj = r0 ? 1 : (r1 ? kFrameLine - 1 : (c0 ? 2 + k - 2 * RUN : 2 + k - (3 * RUN - 2)));
    }
    // The tile's boundary-line nodes, e = 0 .. 4 kFrameLine - 1: columns
    // li = 0 and li = kFrameLine (lj = 0 .. kFrameLine), then rows lj = 0 and
    // lj = kFrameLine (li = 1 .. kFrameLine - 1).
    static constexpr int EDGES = 4 * kFrameLine;
    DNNMG_HD static void edge_pos(int e, int &li, int &lj)
    {
        constexpr int NO = kFrameLine + 1;
        const bool c0 = e < NO, c1 = e < 2 * NO, r0 = e < 3 * NO - 2;
        li = c0 ? 0 : (c1 ? kFrameLine : (r0 ? 1 + e - 2 * NO : 1 + e - (3 * NO - 2)));
        lj = c0 ? e : (c1 ? e - NO : (r0 ? 0 : kFrameLine));
    }
    // Slot of the output of tile patch (pa, pb) at its node (a, b) when that
    // node lies on one of the tile's sides; -1 otherwise.
    DNNMG_HD static int side_slot(int pa, int pb, int a, int b)
    {
        if (a == 0 && pa == 0) return 0 * SIDE + pb * (n + 1) + b;
        if (a == n && pa == TP - 1) return 1 * SIDE + pb * (n + 1) + b;
        if (b == 0 && pb == 0) return 2 * SIDE + pa * (n + 1) + a;
        if (b == n && pb == TP - 1) return 3 * SIDE + pa * (n + 1) + a;
        return -1;
    }
    // Entry k < SIDE of side `side` (0 L, 1 R, 2 B, 3 T): tile patch (pa, pb)
    // and node (a, b) it holds.
    DNNMG_HD static void side_pos(int side, int k, int &pa, int &pb, int &a, int &b)
    {
        const int p = k / (n + 1), m = k - p * (n + 1);
        pa = side == 0 ? 0 : (side == 1 ? TP - 1 : p);
        pb = side < 2 ? p : (side == 2 ? 0 : TP - 1);
        a = side == 0 ? 0 : (side == 1 ? n : m);
        b = side < 2 ? m : (side == 2 ? 0 : n);
    }
    // The same for slot s < 4 SIDE.
    DNNMG_HD static void side_source(int s, int &pa, int &pb, int &a, int &b)
    {
        const int side = s / SIDE;
        side_pos(side, s - side * SIDE, pa, pb, a, b);
    }
    // Offset (in slots) in the flow's frame array of mesh patch (gi, gj)'s
    // output at node (a, b), a node on its tile's sides; -1 if it is not.
    DNNMG_HD static long contrib(int nx, int gi, int gj, int a, int b)
    {
        const int tiles_x = (nx + TP - 1) / TP;
        const int tx = gi / TP, ty = gj / TP;
        const int s = side_slot(gi - tx * TP, gj - ty * TP, a, b);
        return s < 0 ? -1 : ((long)ty * tiles_x + tx) * SIZE + s;
    }
};

// P v at a fine node of a patch from its corner velocities, along the node
// row b (eta = b / n) then across it (xi = a / n), with explicit fused
// multiply-adds so that every kernel that forms the corrected velocity rounds
// it alike.
struct PvRow {
    float lx, ly, dx, dy;
};

DNNMG_HD inline PvRow pv_row(float v00x, float v00y, float v10x, float v10y, float v01x, float v01y, float v11x,
                             float v11y, float eta)
{
    PvRow r;
    r.lx = fmaf(v01x - v00x, eta, v00x);
    r.ly = fmaf(v01y - v00y, eta, v00y);
    const float rx = fmaf(v11x - v10x, eta, v10x);
    const float ry = fmaf(v11y - v10y, eta, v10y);
    r.dx = rx - r.lx;
    r.dy = ry - r.ly;
    return r;
}

DNNMG_HD inline void pv_at(const PvRow &r, float xi, float &px, float &py)
{
    px = fmaf(r.dx, xi, r.lx);
    py = fmaf(r.dy, xi, r.ly);
}

}  // namespace dnnmg
