// Tile choice of the Ozaki purification products, used by dmp::tile_choice:
// per kind and slice range, for n in [n_lo, n_hi], the tile height (rb = 2:
// 64-row tiles, two workgroups per CU; rb = 4: 128-row tiles) and whether
// the last, partly filled round of tiles is split along the reduction.
// The first matching row wins; no match: 128-row tiles, split tail.
// Initial table (before a measured one is written by
// paper_2407_13299_amd/autotune.py --tiles): 64-row tiles and a split tail
// for every size up to S = 7.
#pragma once
namespace dmp {
struct TileRule {
    int kind;        // dmp_kind
    int s_lo, s_hi;  // slice counts
    int n_lo, n_hi;  // sizes
    int rb;          // 2 or 4
    int split_tail;  // 0 or 1
};
constexpr TileRule kTileTable[] = {
    {1, 1, 7, 1, 1 << 30, 2, 1},
    {2, 1, 7, 1, 1 << 30, 2, 1},
};
}  // namespace dmp
