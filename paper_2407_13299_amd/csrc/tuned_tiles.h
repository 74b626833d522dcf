// Tile choice of the Ozaki purification products, used by dmp::tile_choice:
// per kind and slice range, for n in [n_lo, n_hi], the tile height (rb = 2:
// 64-row tiles, two workgroups per CU; rb = 4: 128-row tiles) and whether
// the last, partly filled round of tiles is split along the reduction.
// The first matching row wins; no match: 128-row tiles, split tail.
// Written by paper_2407_13299_amd/autotune.py --tiles from these
// measurements (spectrum-controlled H, half filled, 10 iterations, median
// of interleaved rounds, ms; a non-default choice must win by 1.5%):
//   int8 S= 6 n=  256  64/whole    0.583  64/split    0.583  128/whole    0.694  128/split    0.702  -> 64/split
//   int8 S= 6 n=  384  64/whole    0.648  64/split    0.646  128/whole    0.789  128/split    0.792  -> 64/split
//   int8 S= 6 n=  512  64/whole    0.711  64/split    0.709  128/whole    0.879  128/split    0.880  -> 64/split
//   int8 S= 6 n=  640  64/whole    0.784  64/split    0.798  128/whole    0.984  128/split    0.987  -> 64/whole
//   int8 S= 6 n=  768  64/whole    0.846  64/split    0.843  128/whole    1.070  128/split    1.071  -> 64/split
//   int8 S= 6 n= 1024  64/whole    0.916  64/split    0.935  128/whole    1.185  128/split    1.191  -> 64/whole
//   int8 S= 6 n= 1280  64/whole    1.076  64/split    1.071  128/whole    1.365  128/split    1.380  -> 64/split
//   int8 S= 6 n= 1536  64/whole    1.564  64/split    1.573  128/whole    1.605  128/split    1.617  -> 64/split
//   int8 S= 6 n= 1792  64/whole    1.825  64/split    1.813  128/whole    1.881  128/split    1.906  -> 64/split
//   int8 S= 6 n= 2048  64/whole    2.819  64/split    2.779  128/whole    3.489  128/split    3.160  -> 64/split
//   int8 S= 6 n= 2560  64/whole    4.380  64/split    4.288  128/whole    4.476  128/split    4.557  -> 64/split
//   int8 S= 6 n= 3072  64/whole    6.466  64/split    6.730  128/whole    7.373  128/split    7.325  -> 64/whole
//   int8 S= 6 n= 4096  64/whole   13.763  64/split   13.688  128/whole   15.305  128/split   14.549  -> 64/split
//   int8 S= 6 n= 6144  64/whole   42.136  64/split   42.127  128/whole   46.480  128/split   44.155  -> 64/split
//   int8 S= 6 n= 8192  64/whole   97.529  64/split   97.768  128/whole  105.087  128/split  101.544  -> 64/split
//   int8 S= 7 n=  256  64/whole    0.609  64/split    0.609  128/whole    0.736  128/split    0.737  -> 64/split
//   int8 S= 7 n=  384  64/whole    0.679  64/split    0.687  128/whole    0.857  128/split    0.853  -> 64/split
//   int8 S= 7 n=  512  64/whole    0.756  64/split    0.764  128/whole    0.964  128/split    0.968  -> 64/split
//   int8 S= 7 n=  640  64/whole    0.842  64/split    0.845  128/whole    1.092  128/split    1.086  -> 64/split
//   int8 S= 7 n=  768  64/whole    0.907  64/split    0.913  128/whole    1.206  128/split    1.194  -> 64/split
//   int8 S= 7 n= 1024  64/whole    1.006  64/split    1.009  128/whole    1.344  128/split    1.351  -> 64/split
//   int8 S= 7 n= 1280  64/whole    1.205  64/split    1.197  128/whole    1.588  128/split    1.610  -> 64/split
//   int8 S= 7 n= 1536  64/whole    1.782  64/split    1.773  128/whole    1.896  128/split    1.898  -> 64/split
//   int8 S= 7 n= 1792  64/whole    2.132  64/split    2.137  128/whole    2.222  128/split    2.337  -> 64/split
//   int8 S= 7 n= 2048  64/whole    3.330  64/split    3.202  128/whole    4.182  128/split    3.719  -> 64/split
//   int8 S= 7 n= 2560  64/whole    5.129  64/split    5.122  128/whole    5.444  128/split    5.598  -> 64/split
//   int8 S= 7 n= 3072  64/whole    7.705  64/split    8.183  128/whole    9.024  128/split    8.893  -> 64/whole
//   int8 S= 7 n= 4096  64/whole   16.643  64/split   16.445  128/whole   19.004  128/split   17.946  -> 64/split
//   int8 S= 7 n= 6144  64/whole   51.681  64/split   51.504  128/whole   58.476  128/split   55.735  -> 64/split
//   int8 S= 7 n= 8192  64/whole  120.025  64/split  119.894  128/whole  132.941  128/split  128.970  -> 64/split
//   int8 S= 8 n=  256  64/whole    0.663  64/split    0.646  128/whole    0.788  128/split    0.797  -> 64/split
//   int8 S= 8 n=  384  64/whole    0.737  64/split    0.734  128/whole    0.920  128/split    0.914  -> 64/split
//   int8 S= 8 n=  512  64/whole    0.836  64/split    0.820  128/whole    1.045  128/split    1.068  -> 64/split
//   int8 S= 8 n=  640  64/whole    0.915  64/split    0.919  128/whole    1.187  128/split    1.184  -> 64/split
//   int8 S= 8 n=  768  64/whole    0.998  64/split    1.016  128/whole    1.299  128/split    1.297  -> 64/whole
//   int8 S= 8 n= 1024  64/whole    1.131  64/split    1.139  128/whole    1.492  128/split    1.484  -> 64/split
//   int8 S= 8 n= 1280  64/whole    1.352  64/split    1.374  128/whole    1.769  128/split    1.789  -> 64/whole
//   int8 S= 8 n= 1536  64/whole    2.077  64/split    2.072  128/whole    2.105  128/split    2.120  -> 64/split
//   int8 S= 8 n= 1792  64/whole    2.514  64/split    2.545  128/whole    2.525  128/split    2.550  -> 64/split
//   int8 S= 8 n= 2048  64/whole    3.976  64/split    3.740  128/whole    4.855  128/split    4.172  -> 64/split
//   int8 S= 8 n= 2560  64/whole    6.325  64/split    6.260  128/whole    6.292  128/split    6.437  -> 64/split
//   int8 S= 8 n= 3072  64/whole    9.507  64/split    9.838  128/whole   10.718  128/split   10.361  -> 64/whole
//   int8 S= 8 n= 4096  64/whole   20.469  64/split   20.310  128/whole   22.687  128/split   21.191  -> 64/split
//   int8 S= 8 n= 6144  64/whole   64.732  64/split   63.822  128/whole   71.347  128/split   67.338  -> 64/split
//   int8 S= 8 n= 8192  64/whole  148.407  64/split  148.838  128/whole  160.755  128/split  155.267  -> 64/split
//   fp16 S= 7 n=  256  64/whole    0.795  64/split    0.807  128/whole    1.293  128/split    1.296  -> 64/split
//   fp16 S= 7 n=  384  64/whole    0.957  64/split    0.959  128/whole    1.687  128/split    1.671  -> 64/split
//   fp16 S= 7 n=  512  64/whole    1.159  64/split    1.173  128/whole    2.070  128/split    2.071  -> 64/split
//   fp16 S= 7 n=  640  64/whole    1.321  64/split    1.327  128/whole    2.470  128/split    2.452  -> 64/split
//   fp16 S= 7 n=  768  64/whole    1.496  64/split    1.502  128/whole    2.859  128/split    2.838  -> 64/split
//   fp16 S= 7 n= 1024  64/whole    1.781  64/split    1.806  128/whole    3.560  128/split    3.539  -> 64/split
//   fp16 S= 7 n= 1280  64/whole    2.234  64/split    2.239  128/whole    4.372  128/split    4.370  -> 64/split
//   fp16 S= 7 n= 1536  64/whole    3.477  64/split    3.535  128/whole    5.157  128/split    5.068  -> 64/whole
//   fp16 S= 7 n= 1792  64/whole    4.153  64/split    4.142  128/whole    5.947  128/split    6.100  -> 64/split
//   fp16 S= 7 n= 2048  64/whole    6.834  64/split    5.866  128/whole   12.716  128/split    8.764  -> 64/split
//   fp16 S= 7 n= 2560  64/whole   10.883  64/split   10.888  128/whole   16.511  128/split   16.659  -> 64/split
//   fp16 S= 7 n= 3072  64/whole   16.716  64/split   16.933  128/whole   30.016  128/split   26.769  -> 64/split
//   fp16 S= 7 n= 4096  64/whole   38.506  64/split   37.140  128/whole   68.486  128/split   59.153  -> 64/split
//   fp16 S= 7 n= 6144  64/whole  124.385  64/split  121.336  128/whole  208.356  128/split  193.353  -> 64/split
//   fp16 S= 7 n= 8192  64/whole  285.591  64/split  282.126  128/whole  467.117  128/split  448.605  -> 64/split
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
    {1, 1, 6, 705, 896, 2, 1},
    {1, 1, 6, 897, 1152, 2, 0},
    {1, 1, 6, 1153, 2816, 2, 1},
    {1, 1, 6, 2817, 3584, 2, 0},
    {1, 1, 6, 3585, 1 << 30, 2, 1},
    {1, 7, 7, 1, 2816, 2, 1},
    {1, 7, 7, 2817, 3584, 2, 0},
    {1, 7, 7, 3585, 1 << 30, 2, 1},
    {1, 8, 8, 1, 704, 2, 1},
    {1, 8, 8, 705, 896, 2, 0},
    {1, 8, 8, 897, 1152, 2, 1},
    {1, 8, 8, 1153, 1408, 2, 0},
    {1, 8, 8, 1409, 2816, 2, 1},
    {1, 8, 8, 2817, 3584, 2, 0},
    {1, 8, 8, 3585, 1 << 30, 2, 1},
    {2, 1, 8, 1, 1408, 2, 1},
    {2, 1, 8, 1409, 1664, 2, 0},
    {2, 1, 8, 1665, 1 << 30, 2, 1},
};
}  // namespace dmp
