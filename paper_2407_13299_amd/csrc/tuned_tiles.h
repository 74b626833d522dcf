// Tile choice of the Ozaki purification products, used by dmp::tile_choice:
// per kind and slice range, for n in [n_lo, n_hi], the tile height (rb = 2:
// 64-row tiles, two workgroups per CU; rb = 4: 128-row tiles) and whether
// the last, partly filled round of tiles is split along the reduction.
// The first matching row wins; no match: 128-row tiles, split tail.
// Written by paper_2407_13299_amd/autotune.py --tiles from these
// measurements (spectrum-controlled H, half filled, 10 iterations, median
// of interleaved rounds, ms; a non-default choice must win by 1.5%):
//   int8 S= 6 n=  256  64/whole    0.612  64/split    0.608  128/whole    0.706  128/split    0.706  -> 64/split
//   int8 S= 6 n=  384  64/whole    0.668  64/split    0.667  128/whole    0.791  128/split    0.798  -> 64/split
//   int8 S= 6 n=  512  64/whole    0.745  64/split    0.740  128/whole    0.881  128/split    0.865  -> 64/split
//   int8 S= 6 n=  640  64/whole    0.836  64/split    0.825  128/whole    0.981  128/split    1.006  -> 64/split
//   int8 S= 6 n=  768  64/whole    0.887  64/split    0.883  128/whole    1.070  128/split    1.054  -> 64/split
//   int8 S= 6 n= 1024  64/whole    0.981  64/split    0.971  128/whole    1.153  128/split    1.173  -> 64/split
//   int8 S= 6 n= 1280  64/whole    1.129  64/split    1.153  128/whole    1.372  128/split    1.391  -> 64/whole
//   int8 S= 6 n= 1536  64/whole    1.663  64/split    1.661  128/whole    1.608  128/split    1.594  -> 128/split
//   int8 S= 6 n= 1792  64/whole    2.025  64/split    1.993  128/whole    1.924  128/split    1.939  -> 128/whole
//   int8 S= 6 n= 2048  64/whole    2.940  64/split    2.861  128/whole    3.396  128/split    3.089  -> 64/split
//   int8 S= 6 n= 2560  64/whole    4.432  64/split    4.417  128/whole    4.248  128/split    4.310  -> 128/whole
//   int8 S= 6 n= 3072  64/whole    6.742  64/split    6.988  128/whole    7.199  128/split    7.011  -> 64/whole
//   int8 S= 6 n= 4096  64/whole   14.590  64/split   14.434  128/whole   14.922  128/split   14.286  -> 64/split
//   int8 S= 6 n= 6144  64/whole   44.761  64/split   44.819  128/whole   45.688  128/split   43.650  -> 128/split
//   int8 S= 6 n= 8192  64/whole  105.871  64/split  105.196  128/whole  105.699  128/split  102.064  -> 128/split
//   int8 S= 7 n=  256  64/whole    0.630  64/split    0.635  128/whole    0.762  128/split    0.758  -> 64/split
//   int8 S= 7 n=  384  64/whole    0.716  64/split    0.721  128/whole    0.868  128/split    0.869  -> 64/split
//   int8 S= 7 n=  512  64/whole    0.809  64/split    0.806  128/whole    0.981  128/split    0.982  -> 64/split
//   int8 S= 7 n=  640  64/whole    0.907  64/split    0.902  128/whole    1.110  128/split    1.106  -> 64/split
//   int8 S= 7 n=  768  64/whole    0.972  64/split    0.971  128/whole    1.213  128/split    1.207  -> 64/split
//   int8 S= 7 n= 1024  64/whole    1.081  64/split    1.095  128/whole    1.373  128/split    1.369  -> 64/split
//   int8 S= 7 n= 1280  64/whole    1.282  64/split    1.299  128/whole    1.616  128/split    1.626  -> 64/split
//   int8 S= 7 n= 1536  64/whole    1.937  64/split    1.933  128/whole    1.915  128/split    1.886  -> 128/split
//   int8 S= 7 n= 1792  64/whole    2.325  64/split    2.340  128/whole    2.240  128/split    2.272  -> 128/whole
//   int8 S= 7 n= 2048  64/whole    3.507  64/split    3.326  128/whole    4.159  128/split    3.651  -> 64/split
//   int8 S= 7 n= 2560  64/whole    5.424  64/split    5.395  128/whole    5.288  128/split    5.348  -> 128/whole
//   int8 S= 7 n= 3072  64/whole    8.228  64/split    8.595  128/whole    9.021  128/split    8.735  -> 64/whole
//   int8 S= 7 n= 4096  64/whole   17.969  64/split   17.929  128/whole   18.995  128/split   18.024  -> 64/split
//   int8 S= 7 n= 6144  64/whole   57.272  64/split   56.790  128/whole   59.581  128/split   56.685  -> 64/split
//   int8 S= 7 n= 8192  64/whole  134.236  64/split  132.963  128/whole  137.380  128/split  131.940  -> 64/split
//   int8 S= 8 n=  256  128/whole    0.796  128/split    0.794  -> 128/split
//   int8 S= 8 n=  384  128/whole    0.929  128/split    0.923  -> 128/split
//   int8 S= 8 n=  512  128/whole    1.032  128/split    1.059  -> 128/whole
//   int8 S= 8 n=  640  128/whole    1.214  128/split    1.209  -> 128/split
//   int8 S= 8 n=  768  128/whole    1.340  128/split    1.321  -> 128/split
//   int8 S= 8 n= 1024  128/whole    1.531  128/split    1.563  -> 128/whole
//   int8 S= 8 n= 1280  128/whole    1.850  128/split    1.865  -> 128/split
//   int8 S= 8 n= 1536  128/whole    2.196  128/split    2.228  -> 128/split
//   int8 S= 8 n= 1792  128/whole    2.664  128/split    2.721  -> 128/whole
//   int8 S= 8 n= 2048  128/whole    4.952  128/split    4.244  -> 128/split
//   int8 S= 8 n= 2560  128/whole    6.264  128/split    6.377  -> 128/whole
//   int8 S= 8 n= 3072  128/whole   10.621  128/split   10.082  -> 128/split
//   int8 S= 8 n= 4096  128/whole   23.162  128/split   21.521  -> 128/split
//   int8 S= 8 n= 6144  128/whole   72.447  128/split   68.611  -> 128/split
//   int8 S= 8 n= 8192  128/whole  163.768  128/split  158.550  -> 128/split
//   fp16 S= 7 n=  256  64/whole    0.909  64/split    0.914  128/whole    1.086  128/split    1.077  -> 64/split
//   fp16 S= 7 n=  384  64/whole    1.128  64/split    1.136  128/whole    1.378  128/split    1.360  -> 64/split
//   fp16 S= 7 n=  512  64/whole    1.392  64/split    1.402  128/whole    1.657  128/split    1.667  -> 64/split
//   fp16 S= 7 n=  640  64/whole    1.613  64/split    1.614  128/whole    1.941  128/split    1.933  -> 64/split
//   fp16 S= 7 n=  768  64/whole    1.826  64/split    1.837  128/whole    2.223  128/split    2.214  -> 64/split
//   fp16 S= 7 n= 1024  64/whole    2.222  64/split    2.229  128/whole    2.731  128/split    2.717  -> 64/split
//   fp16 S= 7 n= 1280  64/whole    2.727  64/split    2.751  128/whole    3.330  128/split    3.303  -> 64/split
//   fp16 S= 7 n= 1536  64/whole    3.916  64/split    3.941  128/whole    3.907  128/split    3.860  -> 128/split
//   fp16 S= 7 n= 1792  64/whole    4.574  64/split    4.620  128/whole    4.521  128/split    4.511  -> 128/split
//   fp16 S= 7 n= 2048  64/whole    8.020  64/split    6.396  128/whole    9.443  128/split    6.732  -> 64/split
//   fp16 S= 7 n= 2560  64/whole   11.944  64/split   11.921  128/whole   11.869  128/split   11.869  -> 64/split
//   fp16 S= 7 n= 3072  64/whole   18.405  64/split   18.054  128/whole   20.770  128/split   18.362  -> 64/split
//   fp16 S= 7 n= 4096  64/whole   43.159  64/split   40.743  128/whole   46.609  128/split   40.773  -> 64/split
//   fp16 S= 7 n= 6144  64/whole  141.037  64/split  136.461  128/whole  145.445  128/split  132.346  -> 128/split
//   fp16 S= 7 n= 8192  64/whole  319.432  64/split  314.532  128/whole  324.605  128/split  306.726  -> 128/split
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
    {1, 1, 6, 1, 1152, 2, 1},
    {1, 1, 6, 1153, 1408, 2, 0},
    {1, 1, 6, 1409, 1664, 4, 1},
    {1, 1, 6, 1665, 1920, 4, 0},
    {1, 1, 6, 1921, 2304, 2, 1},
    {1, 1, 6, 2305, 2816, 4, 0},
    {1, 1, 6, 2817, 3584, 2, 0},
    {1, 1, 6, 3585, 5120, 2, 1},
    {1, 1, 6, 5121, 1 << 30, 4, 1},
    {1, 7, 7, 1, 1408, 2, 1},
    {1, 7, 7, 1409, 1664, 4, 1},
    {1, 7, 7, 1665, 1920, 4, 0},
    {1, 7, 7, 1921, 2304, 2, 1},
    {1, 7, 7, 2305, 2816, 4, 0},
    {1, 7, 7, 2817, 3584, 2, 0},
    {1, 7, 7, 3585, 1 << 30, 2, 1},
    {1, 8, 12, 1, 448, 4, 1},
    {1, 8, 12, 449, 576, 4, 0},
    {1, 8, 12, 577, 896, 4, 1},
    {1, 8, 12, 897, 1152, 4, 0},
    {1, 8, 12, 1153, 1664, 4, 1},
    {1, 8, 12, 1665, 1920, 4, 0},
    {1, 8, 12, 1921, 2304, 4, 1},
    {1, 8, 12, 2305, 2816, 4, 0},
    {1, 8, 12, 2817, 1 << 30, 4, 1},
    {2, 1, 7, 1, 1408, 2, 1},
    {2, 1, 7, 1409, 1920, 4, 1},
    {2, 1, 7, 1921, 5120, 2, 1},
    {2, 1, 7, 5121, 1 << 30, 4, 1},
};
}  // namespace dmp
