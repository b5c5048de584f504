// Index math of the persistent network kernels' tile prefetch, host and
// device: the kernels call these, and a host test replays them over every
// row count to show that each read stays inside the rows of its tile.
#pragma once

#ifndef __HIP__
#include <algorithm>
#define DNNMG_HD
#else
#include <hip/hip_runtime.h>
#define DNNMG_HD __host__ __device__
#endif

namespace dnnmg {

#ifndef __HIP__
using std::min;
#endif

// One 16-byte piece of the copy of a 128-patch tile's input rows into LDS
// (k_net_b16w).  The tile is two halves of up to 64 rows each (a: na >= 1
// rows, b: nb >= 0 rows); a row is XP pieces of 8 BF16 (nin = 8 XP).  Wave
// load i of wave w moves the pieces 64 j .. 64 j + 63 of the tile's 2 XP
// groups, j = min(w + 8 i, 2 XP - 1) (waves with one load fewer repeat the
// last group); lane l moves piece p = 64 jj + l of its half, which lands at
// LDS element 8 p of that half, i.e. at (row p / XP, column p mod XP).
// Rows past a half's end take the half's last row, at the same column, and
// an empty second half reads the first half's rows: those rows' results are
// never stored, and the copy stays unconditional (so the waits for later
// loads can count past it).
struct WidePiece {
    int half;   // 0: the source is half a, 1: half b
    int src;    // BF16 element offset from that half's first input row
    int dst;    // BF16 element offset in the tile's LDS rows of the wave's 64-piece group (lane l adds 8 l)
};

DNNMG_HD inline WidePiece wide_x_piece(int i, int wave, int lane, int XP, int na, int nb)
{
    const int j = min(wave + 8 * i, 2 * XP - 1);
    const bool second = j >= XP;
    const int jj = second ? j - XP : j;
    WidePiece w;
    w.half = second && nb > 0 ? 1 : 0;
    const int nrows = w.half ? nb : na;
    const int p = 64 * jj + lane;
    const int r = p / XP;
    const int row = min(r, nrows - 1);
    w.src = row * 8 * XP + 8 * (p - r * XP);
    w.dst = (second ? 64 * 8 * XP : 0) + 512 * jj;
    return w;
}

// Row of the FP32 state that tile row r (0 .. 127) of a 128-patch tile
// reads (k_net_b16w); half tells which half it belongs to.  Rows past a
// half's end read its last row; an empty second half reads the first's.
DNNMG_HD inline int wide_h_row(int r, int na, int nb, int &half)
{
    half = r >= 64 && nb > 0 ? 1 : 0;
    return min(r & 63, (half ? nb : na) - 1);
}

// Predicate of the register prefetch of a 64-patch tile (k_net_h64,
// k_net_q8p): piece c of per_row pieces per row is read when it lies in the
// tile (c < 64 per_row) and in one of its nrows rows; other pieces are zero.
DNNMG_HD inline bool tile_piece_in(int c, int per_row, int nrows)
{
    return c < 64 * per_row && c / per_row < nrows;
}

}  // namespace dnnmg
