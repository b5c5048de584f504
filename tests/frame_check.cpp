// Host replay of the tile frame (csrc/frame.h) that the one-launch K = 2 step
// hands to the rhs kernel, over meshes of 1..26 x 1..26 coarse elements
// (full and ragged tiles):
//   - the fused pass completes every node inside a tile's boundary lines once
//     (deep nodes: the state, inner nodes: their frame slot), with every patch
//     it sums inside the tile and inside the mesh;
//   - no other tile's defect reads a deep node (the defect reads its tile's
//     nodes and one fine node past each boundary line), so writing them in
//     place does not race;
//   - every contribution the rhs kernel looks up for a boundary-line node is a
//     slot the fused pass wrote with exactly that patch's output at that node;
//   - the rhs kernel's nodal values cover every node of the tile's patches,
//     and every mesh node's state is written by exactly one tile;
//   - the inner-slot and boundary-node enumerations are bijections, and the
//     deep-node loads stay inside the state rows.
// Exit status 0 when all hold.
#include <cstdio>
#include <map>
#include <set>
#include <tuple>
#include <vector>

#include "frame.h"

using namespace dnnmg;

static int failures = 0;
#define CHECK(c, ...)                                                   \
    do {                                                                \
        if (!(c)) {                                                     \
            if (failures < 20) {                                        \
                std::printf("FAIL %s:%d: ", __FILE__, __LINE__);        \
                std::printf(__VA_ARGS__);                               \
                std::printf("\n");                                      \
            }                                                           \
            ++failures;                                                 \
        }                                                               \
    } while (0)

typedef TileFrame<2> FR;
constexpr int K = 2, n = 4, TP = FR::TP, L = kFrameLine;

int main()
{
    // enumerations
    {
        std::set<std::pair<int, int>> seen;
        for (int k = 0; k < FR::INNER; ++k) {
            int li, lj;
            FR::inner_pos(k, li, lj);
            CHECK(frame_kind(li, lj) == kFrameInner, "inner slot %d -> (%d,%d) not inner", k, li, lj);
            CHECK(FR::inner_slot(li, lj) == 4 * FR::SIDE + k, "inner slot %d round trip", k);
            seen.insert({li, lj});
        }
        int inner = 0;
        for (int lj = 0; lj <= L; ++lj)
            for (int li = 0; li <= L; ++li) inner += frame_kind(li, lj) == kFrameInner;
        CHECK((int)seen.size() == FR::INNER && inner == FR::INNER, "inner enumeration %zu / %d", seen.size(), inner);
        std::set<std::pair<int, int>> edges;
        for (int e = 0; e < FR::EDGES; ++e) {
            int li, lj;
            FR::edge_pos(e, li, lj);
            CHECK(li >= 0 && li <= L && lj >= 0 && lj <= L && frame_kind(li, lj) == kFrameEdge, "edge %d", e);
            edges.insert({li, lj});
        }
        int ne = 0;
        for (int lj = 0; lj <= L; ++lj)
            for (int li = 0; li <= L; ++li) ne += frame_kind(li, lj) == kFrameEdge;
        CHECK((int)edges.size() == FR::EDGES && ne == FR::EDGES, "edge enumeration");
    }

    long meshes = 0;
    for (int ny = 1; ny <= 26; ++ny)
        for (int nx = 1; nx <= 26; ++nx) {
            ++meshes;
            const int NX = nx * n, NY = ny * n;
            const int tiles_x = (nx + TP - 1) / TP, tiles_y = (ny + TP - 1) / TP;
            const long nslots = (long)tiles_x * tiles_y * FR::SIZE;
            // what the fused pass writes: slot -> (patch gi, gj, node a, b) for
            // side slots, (node I, J) for inner slots
            std::map<long, std::tuple<int, int, int, int>> side_src;
            std::map<long, std::pair<int, int>> inner_src;
            std::map<std::pair<int, int>, int> state_writes;   // node -> count
            std::map<std::pair<int, int>, int> deep_owner;     // node -> tile
            for (int ty = 0; ty < tiles_y; ++ty)
                for (int tx = 0; tx < tiles_x; ++tx) {
                    const int tile = ty * tiles_x + tx;
                    const int pi0 = tx * TP, pj0 = ty * TP, I0 = pi0 * n, J0 = pj0 * n;
                    const long base = (long)tile * FR::SIZE;
                    for (int s = 0; s < 4 * FR::SIDE; ++s) {
                        int pa, pb, a, b;
                        FR::side_source(s, pa, pb, a, b);
                        if (pi0 + pa < nx && pj0 + pb < ny) side_src[base + s] = {pi0 + pa, pj0 + pb, a, b};
                    }
                    // the fused pass: one node row of one patch per thread, then the mesh end
                    std::set<std::pair<int, int>> done;
                    auto complete = [&](int li, int lj) {
                        const int I = I0 + li, J = J0 + lj;
                        CHECK(I <= NX && J <= NY, "completed node outside the mesh");
                        CHECK(done.insert(std::make_pair(li, lj)).second, "node (%d,%d) of tile %d completed twice", li, lj, tile);
                        const int pI = std::min(I >> K, nx - 1), pJ = std::min(J >> K, ny - 1);
                        const int a = I - pI * n, b = J - pJ * n;
                        const bool lft = a == 0 && pI > 0, low = b == 0 && pJ > 0;
                        const int qi[4] = {pI - 1, pI, pI - 1, pI}, qj[4] = {pJ - 1, pJ - 1, pJ, pJ};
                        const bool use[4] = {lft && low, low, lft, true};
                        for (int q = 0; q < 4; ++q)
                            if (use[q])
                                CHECK(qi[q] >= pi0 && qi[q] < pi0 + TP && qj[q] >= pj0 && qj[q] < pj0 + TP &&
                                          qi[q] < nx && qj[q] < ny,
                                      "fused sum of node (%d,%d) reads patch (%d,%d) outside tile %d", I, J, qi[q],
                                      qj[q], tile);
                        if (frame_kind(li, lj) == kFrameInner) {
                            inner_src[base + FR::inner_slot(li, lj)] = {I, J};
                        } else {
                            state_writes[{I, J}]++;
                            deep_owner[{I, J}] = tile;
                        }
                    };
                    for (int tid = 0; tid < 256; ++tid) {
                        const int pl = tid % (TP * TP), b = tid / (TP * TP);
                        const int pa = pl % TP, pb = pl / TP, pi = pi0 + pa, pj = pj0 + pb;
                        const int lj = pb * n + b;
                        if (!(pi < nx && pj < ny && lj > 0)) continue;
                        for (int a = 0; a < n; ++a) {
                            const int li = pa * n + a;
                            if (li == 0 || frame_kind(li, lj) == kFrameEdge) continue;
                            complete(li, lj);
                        }
                    }
                    const int le = std::min(TP, nx - pi0) * n, me = std::min(TP, ny - pj0) * n;
                    for (int tid = 0; tid < le + me + 1; ++tid) {
                        const int li = tid <= me ? le : tid - me - 1, lj = tid <= me ? tid : me;
                        if (frame_kind(li, lj) != kFrameEdge) complete(li, lj);
                    }
                    // every node of the tile inside its boundary lines and the mesh is done
                    for (int lj = 1; lj < L; ++lj)
                        for (int li = 1; li < L; ++li)
                            if (I0 + li <= NX && J0 + lj <= NY)
                                CHECK(done.count(std::make_pair(li, lj)), "node (%d,%d) of tile %d (mesh %dx%d) not completed", li,
                                      lj, tile, nx, ny);
                }
            // deep nodes are read by no other tile's defect (nodes I0-1 .. I0+L+1)
            for (const auto &kv : deep_owner) {
                const int I = kv.first.first, J = kv.first.second;
                for (int ty = 0; ty < tiles_y; ++ty)
                    for (int tx = 0; tx < tiles_x; ++tx) {
                        const int tile = ty * tiles_x + tx;
                        if (tile == kv.second) continue;
                        const int I0 = tx * TP * n, J0 = ty * TP * n;
                        CHECK(!(I >= I0 - 1 && I <= I0 + L + 1 && J >= J0 - 1 && J <= J0 + L + 1),
                              "deep node (%d,%d) of tile %d is read by tile %d's defect", I, J, kv.second, tile);
                    }
            }
            // the rhs kernel, tile by tile
            for (int ty = 0; ty < tiles_y; ++ty)
                for (int tx = 0; tx < tiles_x; ++tx) {
                    const int tile = ty * tiles_x + tx;
                    const int pi0 = tx * TP, pj0 = ty * TP, I0 = pi0 * n, J0 = pj0 * n;
                    std::set<std::pair<int, int>> have;   // tile nodes with u in LDS
                    constexpr int DN = L - 3, ND = DN * DN;
                    for (int t = 0; t < ((ND + 255) / 256) * 256; ++t) {
                        const int tc = std::min(t, ND - 1);
                        const int lic = std::min(2 + tc % DN, NX - I0), ljc = std::min(2 + tc / DN, NY - J0);
                        CHECK(lic >= 0 && ljc >= 0 && I0 + lic <= NX && J0 + ljc <= NY, "deep load outside the state");
                        const int li = 2 + t % DN, lj = 2 + t / DN;
                        if (t < ND && I0 + li <= NX && J0 + lj <= NY) {
                            CHECK(frame_kind(li, lj) == kFrameDeep, "deep load of a frame node");
                            const std::pair<int, int> key(I0 + li, J0 + lj);
                            CHECK(deep_owner.count(key) && deep_owner[key] == tile,
                                  "deep node (%d,%d) read by tile %d was not written by it", I0 + li, J0 + lj, tile);
                            have.insert({li, lj});
                        }
                    }
                    for (int k = 0; k < FR::INNER; ++k) {
                        int li, lj;
                        FR::inner_pos(k, li, lj);
                        if (I0 + li <= NX && J0 + lj <= NY) {
                            const long slot = (long)tile * FR::SIZE + 4 * FR::SIDE + k;
                            const std::pair<int, int> key(I0 + li, J0 + lj);
                            CHECK(inner_src.count(slot) && inner_src[slot] == key,
                                  "inner slot %ld not written for its node", slot);
                            state_writes[{I0 + li, J0 + lj}]++;
                            have.insert({li, lj});
                        }
                    }
                    for (int e = 0; e < FR::EDGES; ++e) {
                        int li, lj;
                        FR::edge_pos(e, li, lj);
                        const int I = I0 + li, J = J0 + lj;
                        if (!(I <= NX && J <= NY)) continue;
                        const int pI = std::min(I >> K, nx - 1), pJ = std::min(J >> K, ny - 1);
                        const int a = I - pI * n, b = J - pJ * n;
                        const bool lft = a == 0 && pI > 0, low = b == 0 && pJ > 0;
                        const int qi[4] = {pI - 1, pI, pI - 1, pI}, qj[4] = {pJ - 1, pJ - 1, pJ, pJ};
                        const int qa[4] = {n, a, n, a}, qb[4] = {n, n, b, b};
                        const bool use[4] = {lft && low, low, lft, true};
                        for (int q = 0; q < 4; ++q) {
                            if (!use[q]) continue;
                            const long o = FR::contrib(nx, qi[q], qj[q], qa[q], qb[q]);
                            CHECK(o >= 0 && o < nslots, "edge node (%d,%d): contribution %d has no slot", I, J, q);
                            CHECK(side_src.count(o) &&
                                      side_src[o] == std::make_tuple(qi[q], qj[q], qa[q], qb[q]),
                                  "edge node (%d,%d) mesh %dx%d: slot %ld does not hold patch (%d,%d) node (%d,%d)", I,
                                  J, nx, ny, o, qi[q], qj[q], qa[q], qb[q]);
                        }
                        if ((li < L || I == NX) && (lj < L || J == NY)) state_writes[{I, J}]++;
                        have.insert({li, lj});
                    }
                    // the FP64 pass reads every node of the tile's patches
                    for (int pb = 0; pb < TP; ++pb)
                        for (int pa = 0; pa < TP; ++pa) {
                            if (pi0 + pa >= nx || pj0 + pb >= ny) continue;
                            for (int b = 0; b <= n; ++b)
                                for (int a = 0; a <= n; ++a)
                                    CHECK(have.count(std::make_pair(pa * n + a, pb * n + b)),
                                          "tile %d: node (%d,%d) of its patch (%d,%d) has no value", tile,
                                          pa * n + a, pb * n + b, pa, pb);
                        }
                }
            for (int J = 0; J <= NY; ++J)
                for (int I = 0; I <= NX; ++I) {
                    const auto it = state_writes.find({I, J});
                    CHECK(it != state_writes.end() && it->second == 1, "mesh %dx%d node (%d,%d) written %d times", nx,
                          ny, I, J, it == state_writes.end() ? 0 : it->second);
                }
        }
    std::printf("tile frame: %ld meshes, %d failures\n", meshes, failures);
    return failures ? 1 : 0;
}
