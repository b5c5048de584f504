// Host replay of the persistent network kernels' tile prefetch addresses
// (paper_2008_11520_amd/csrc/net_index.h, the functions the kernels call):
//   k_net_b16w: the copy of a 128-patch tile's input rows into LDS
//     (wide_x_piece) and the load of its FP32 state (wide_h_row), for
//     K = 1..3, H = 64/128, first half 1..64 rows, second half 0..64 rows;
//   k_net_h64 / k_net_q8p: the predicated register prefetch of a 64-patch
//     tile (tile_piece_in), for the same shapes and 0..64 rows.
// Every read must lie inside the rows of the half it reads, every LDS write
// inside the tile's LDS rows, and every row the tile stores results for must
// receive exactly its own input row and state.  Prints one line per shape
// and exits non-zero if any check fails.
#include "net_index.h"

#include <cstdio>
#include <vector>

using namespace dnnmg;

static int fails = 0;
#define CHECK(c, ...)                                                   \
    do {                                                                \
        if (!(c)) {                                                     \
            if (fails++ < 10) { std::printf("FAIL: " __VA_ARGS__); std::printf("\n"); } \
        }                                                               \
    } while (0)

static void wide(int K, int H)
{
    const int n = 1 << K, nf = (n + 1) * (n + 1), nin = 4 * nf + 4, XP = nin / 8;
    const int HT = H / 16, WPH = 8 / HT, RTW = 8 / WPH;
    const int loads = (2 * XP + 7) / 8;
    long checked = 0;
    const int fails0 = fails;
    for (int na = 1; na <= 64; ++na)
        for (int nb = 0; nb <= 64; ++nb) {
            // LDS element (start of a 16-byte piece) -> source (half, offset)
            std::vector<int> lds_half(128 * nin, -1), lds_src(128 * nin, -1);
            for (int wave = 0; wave < 8; ++wave)
                for (int i = 0; i < loads; ++i)
                    for (int lane = 0; lane < 64; ++lane) {
                        const WidePiece w = wide_x_piece(i, wave, lane, XP, na, nb);
                        const int rows = w.half ? nb : na;
                        CHECK(w.src >= 0 && w.src + 8 <= rows * nin,
                              "b16w K=%d H=%d na=%d nb=%d wave %d load %d lane %d: read [%d, %d) of %d elements",
                              K, H, na, nb, wave, i, lane, w.src, w.src + 8, rows * nin);
                        const int d = w.dst + 8 * lane;
                        CHECK(d >= 0 && d + 8 <= 128 * nin, "b16w K=%d na=%d nb=%d: LDS write at %d of %d",
                              K, na, nb, d, 128 * nin);
                        if (d < 0 || d + 8 > 128 * nin) continue;
                        if (lds_half[d] >= 0)
                            CHECK(lds_half[d] == w.half && lds_src[d] == w.src,
                                  "b16w K=%d na=%d nb=%d: LDS piece %d written twice with different data", K, na, nb, d);
                        lds_half[d] = w.half;
                        lds_src[d] = w.src;
                        ++checked;
                    }
            for (int h = 0; h < 2; ++h) {
                const int rows = h ? nb : na;
                for (int r = 0; r < rows; ++r)
                    for (int c = 0; c < XP; ++c) {
                        const int d = h * 64 * nin + r * nin + 8 * c;
                        CHECK(lds_half[d] == h && lds_src[d] == r * nin + 8 * c,
                              "b16w K=%d na=%d nb=%d: half %d row %d piece %d holds (%d, %d)",
                              K, na, nb, h, r, c, lds_half[d], lds_src[d]);
                    }
            }
            // the state: rows 16 (rt0 + q) + l of the wave's row tiles, units ucol .. ucol + 3
            for (int wave = 0; wave < 8; ++wave) {
                const int rt0 = RTW * (wave / HT);
                for (int q = 0; q < RTW; ++q)
                    for (int lane = 0; lane < 64; ++lane) {
                        const int l = lane & 15, ucol = 16 * (wave % HT) + 4 * (lane >> 4);
                        const int r = 16 * (rt0 + q) + l;
                        int half;
                        const int row = wide_h_row(r, na, nb, half);
                        const int rows = half ? nb : na;
                        const int off = row * H + ucol;
                        CHECK(row >= 0 && off + 4 <= rows * H,
                              "b16w state K=%d H=%d na=%d nb=%d: tile row %d reads [%d, %d) of %d",
                              K, H, na, nb, r, off, off + 4, rows * H);
                        if ((r & 63) < ((r >= 64) ? nb : na))
                            CHECK(half == (r >= 64) && row == (r & 63),
                                  "b16w state K=%d na=%d nb=%d: tile row %d reads half %d row %d", K, na, nb, r, half, row);
                        ++checked;
                    }
            }
        }
    std::printf("k_net_b16w K=%d H=%d: %ld prefetch addresses replayed, %d violations\n", K, H, checked,
                fails - fails0);
}

// register prefetch of a 64-row tile: pieces of per_row 16-byte pieces per row
static void predicated(const char *name, int tag, int per_row)
{
    const int threads = 512, pieces = 64 * per_row, per_thread = (pieces + threads - 1) / threads;
    long checked = 0;
    const int fails0 = fails;
    for (int rows = 0; rows <= 64; ++rows) {
        std::vector<int> seen(pieces, 0);
        for (int t = 0; t < threads; ++t)
            for (int i = 0; i < per_thread; ++i) {
                const int c = t + i * threads;
                if (!tile_piece_in(c, per_row, rows)) continue;
                CHECK(c >= 0 && c < rows * per_row, "%s %d rows=%d: piece %d of %d read", name, tag, rows, c,
                      rows * per_row);
                if (c >= 0 && c < pieces) ++seen[c];
                ++checked;
            }
        for (int c = 0; c < rows * per_row; ++c)
            CHECK(seen[c] == 1, "%s %d rows=%d: piece %d read %d times", name, tag, rows, c, seen[c]);
    }
    std::printf("%s %d (%d pieces per row): %ld predicated reads replayed, %d violations\n", name, tag, per_row,
                checked, fails - fails0);
}

int main()
{
    for (int K = 1; K <= 3; ++K)
        for (int H : {64, 128}) wide(K, H);
    for (int K = 1; K <= 3; ++K) {
        const int n = 1 << K, nin = 4 * (n + 1) * (n + 1) + 4;
        predicated("k_net_h64 input K", K, nin / 8);            // BF16 rows
        predicated("k_net_q8p input K", K, (nin + 31) / 32 * 32 / 16);  // E4M3 rows, k-chunk padded
    }
    for (int H : {64, 128}) predicated("state rows H", H, H / 4);
    if (fails) {
        std::printf("%d violations\n", fails);
        return 1;
    }
    std::printf("all prefetch addresses in bounds\n");
    return 0;
}
