// Tile choice of the Ozaki purification products, used by dmp::tile_choice:
// per kind and slice range, for n in [n_lo, n_hi], the tile height (rb = 2:
// 64-row tiles, two workgroups per CU; rb = 4: 128-row tiles) and whether
// the last, partly filled round of tiles is split along the reduction.
// The first matching row wins; no match: 128-row tiles, split tail.
// Written by paper_2407_13299_amd/autotune.py --tiles from these
// measurements (spectrum-controlled H, half filled, 10 iterations, median
// of interleaved rounds, ms; a non-default choice must win by 1.5%):
//   int8 S= 6 n=  256  64/whole    0.597  64/split    0.594  128/whole    0.704  128/split    0.713  -> 64/split
//   int8 S= 6 n=  384  64/whole    0.654  64/split    0.655  128/whole    0.794  128/split    0.803  -> 64/split
//   int8 S= 6 n=  512  64/whole    0.724  64/split    0.716  128/whole    0.883  128/split    0.887  -> 64/split
//   int8 S= 6 n=  640  64/whole    0.791  64/split    0.804  128/whole    0.984  128/split    0.989  -> 64/whole
//   int8 S= 6 n=  768  64/whole    0.851  64/split    0.849  128/whole    1.075  128/split    1.072  -> 64/split
//   int8 S= 6 n= 1024  64/whole    0.931  64/split    0.934  128/whole    1.186  128/split    1.194  -> 64/split
//   int8 S= 6 n= 1280  64/whole    1.058  64/split    1.084  128/whole    1.379  128/split    1.423  -> 64/whole
//   int8 S= 6 n= 1536  64/whole    1.585  64/split    1.576  128/whole    1.645  128/split    1.642  -> 64/split
//   int8 S= 6 n= 1792  64/whole    1.872  64/split    1.888  128/whole    1.929  128/split    1.947  -> 64/split
//   int8 S= 6 n= 2048  64/whole    2.879  64/split    2.825  128/whole    3.539  128/split    3.217  -> 64/split
//   int8 S= 6 n= 2560  64/whole    4.377  64/split    4.333  128/whole    4.519  128/split    4.636  -> 64/split
//   int8 S= 6 n= 3072  64/whole    6.491  64/split    6.437  128/whole    7.435  128/split    7.656  -> 64/split
//   int8 S= 6 n= 4096  64/whole   13.648  64/split   13.761  128/whole   15.059  128/split   14.385  -> 64/split
//   int8 S= 6 n= 6144  64/whole   42.547  64/split   42.580  128/whole   44.451  128/split   43.566  -> 64/split
//   int8 S= 6 n= 8192  64/whole   99.150  64/split   98.886  128/whole  104.963  128/split  101.593  -> 64/split
//   int8 S= 7 n=  256  64/whole    0.634  64/split    0.627  128/whole    0.753  128/split    0.762  -> 64/split
//   int8 S= 7 n=  384  64/whole    0.699  64/split    0.701  128/whole    0.862  128/split    0.862  -> 64/split
//   int8 S= 7 n=  512  64/whole    0.770  64/split    0.772  128/whole    0.974  128/split    0.983  -> 64/split
//   int8 S= 7 n=  640  64/whole    0.876  64/split    0.854  128/whole    1.107  128/split    1.111  -> 64/split
//   int8 S= 7 n=  768  64/whole    0.917  64/split    0.922  128/whole    1.196  128/split    1.210  -> 64/split
//   int8 S= 7 n= 1024  64/whole    1.015  64/split    1.018  128/whole    1.342  128/split    1.361  -> 64/split
//   int8 S= 7 n= 1280  64/whole    1.216  64/split    1.220  128/whole    1.599  128/split    1.603  -> 64/split
//   int8 S= 7 n= 1536  64/whole    1.781  64/split    1.792  128/whole    1.894  128/split    1.904  -> 64/split
//   int8 S= 7 n= 1792  64/whole    2.215  64/split    2.187  128/whole    2.320  128/split    2.356  -> 64/split
//   int8 S= 7 n= 2048  64/whole    3.361  64/split    3.267  128/whole    4.261  128/split    3.762  -> 64/split
//   int8 S= 7 n= 2560  64/whole    5.288  64/split    5.280  128/whole    5.531  128/split    5.751  -> 64/split
//   int8 S= 7 n= 3072  64/whole    7.814  64/split    7.764  128/whole    9.090  128/split    9.422  -> 64/split
//   int8 S= 7 n= 4096  64/whole   16.853  64/split   16.677  128/whole   18.817  128/split   17.757  -> 64/split
//   int8 S= 7 n= 6144  64/whole   53.058  64/split   52.626  128/whole   58.684  128/split   55.901  -> 64/split
//   int8 S= 7 n= 8192  64/whole  123.722  64/split  123.069  128/whole  134.372  128/split  130.075  -> 64/split
//   int8 S= 8 n=  256  128/whole    0.786  128/split    0.791  -> 128/split
//   int8 S= 8 n=  384  128/whole    0.913  128/split    0.913  -> 128/split
//   int8 S= 8 n=  512  128/whole    1.053  128/split    1.053  -> 128/split
//   int8 S= 8 n=  640  128/whole    1.198  128/split    1.192  -> 128/split
//   int8 S= 8 n=  768  128/whole    1.302  128/split    1.310  -> 128/split
//   int8 S= 8 n= 1024  128/whole    1.500  128/split    1.499  -> 128/split
//   int8 S= 8 n= 1280  128/whole    1.826  128/split    1.848  -> 128/split
//   int8 S= 8 n= 1536  128/whole    2.121  128/split    2.145  -> 128/split
//   int8 S= 8 n= 1792  128/whole    2.571  128/split    2.580  -> 128/split
//   int8 S= 8 n= 2048  128/whole    4.862  128/split    4.161  -> 128/split
//   int8 S= 8 n= 2560  128/whole    6.366  128/split    6.422  -> 128/split
//   int8 S= 8 n= 3072  128/whole   10.656  128/split   10.142  -> 128/split
//   int8 S= 8 n= 4096  128/whole   22.540  128/split   20.838  -> 128/split
//   int8 S= 8 n= 6144  128/whole   70.127  128/split   67.347  -> 128/split
//   int8 S= 8 n= 8192  128/whole  160.780  128/split  155.265  -> 128/split
//   fp16 S= 7 n=  256  64/whole    0.857  64/split    0.867  128/whole    1.285  128/split    1.279  -> 64/split
//   fp16 S= 7 n=  384  64/whole    1.069  64/split    1.064  128/whole    1.669  128/split    1.670  -> 64/split
//   fp16 S= 7 n=  512  64/whole    1.303  64/split    1.315  128/whole    2.053  128/split    2.058  -> 64/split
//   fp16 S= 7 n=  640  64/whole    1.513  64/split    1.520  128/whole    2.470  128/split    2.429  -> 64/split
//   fp16 S= 7 n=  768  64/whole    1.730  64/split    1.732  128/whole    2.860  128/split    2.835  -> 64/split
//   fp16 S= 7 n= 1024  64/whole    2.109  64/split    2.117  128/whole    3.569  128/split    3.534  -> 64/split
//   fp16 S= 7 n= 1280  64/whole    2.564  64/split    2.585  128/whole    4.350  128/split    4.355  -> 64/split
//   fp16 S= 7 n= 1536  64/whole    3.666  64/split    3.694  128/whole    5.108  128/split    5.083  -> 64/split
//   fp16 S= 7 n= 1792  64/whole    4.290  64/split    4.310  128/whole    5.990  128/split    5.945  -> 64/split
//   fp16 S= 7 n= 2048  64/whole    7.554  64/split    6.204  128/whole   12.686  128/split    8.687  -> 64/split
//   fp16 S= 7 n= 2560  64/whole   11.445  64/split   11.476  128/whole   16.515  128/split   16.510  -> 64/split
//   fp16 S= 7 n= 3072  64/whole   17.659  64/split   17.026  128/whole   29.899  128/split   26.545  -> 64/split
//   fp16 S= 7 n= 4096  64/whole   40.041  64/split   37.853  128/whole   68.410  128/split   58.342  -> 64/split
//   fp16 S= 7 n= 6144  64/whole  133.721  64/split  129.938  128/whole  208.507  128/split  193.344  -> 64/split
//   fp16 S= 7 n= 8192  64/whole  305.689  64/split  301.257  128/whole  467.426  128/split  448.777  -> 64/split
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
    {1, 1, 6, 1, 576, 2, 1},
    {1, 1, 6, 577, 704, 2, 0},
    {1, 1, 6, 705, 1152, 2, 1},
    {1, 1, 6, 1153, 1408, 2, 0},
    {1, 1, 6, 1409, 1 << 30, 2, 1},
    {1, 7, 7, 1, 1 << 30, 2, 1},
    {1, 8, 12, 1, 1 << 30, 4, 1},
    {2, 1, 7, 1, 1 << 30, 2, 1},
};
}  // namespace dmp
