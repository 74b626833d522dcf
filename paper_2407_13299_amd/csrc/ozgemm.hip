// Slice-pair products of the Ozaki scheme (Sec. 2.4) on gfx950 matrix cores,
// with the FP64 summation and the purification work fused into the epilogue.
//
// A workgroup owns one 64 x 64 output tile; its four wavefronts own 32 x 32
// quadrants.  For every chunk of the reduction (32 INT8 or 16 FP16 elements)
// the S digit planes of the tile's two 32-row blocks of each operand (4 S KiB,
// contiguous runs in HBM) are staged once through double-buffered LDS and
// every wavefront forms all S (S + 1) / 2 slice pairs (i + j <= S + 1) from
// registers:
//   INT8: v_mfma_i32_32x32x32_i8, exact INT32 sums; one accumulator per
//         anti-diagonal group g = i + j (products of the same weight
//         2^-(8g - 4) add exactly), (g - 1) k 2^14 < 2^31 checked on the host;
//   FP16: v_mfma_f32_32x32x16_f16; the FP32 sum of one chunk is an integer
//         below 2^24 (16 (g - 1) 2^14 <= 2^24 for g - 1 <= 64), so it is exact,
//         and it is converted to INT32 and added to the group accumulator.
// Epilogue, per element: Horner over the groups from the smallest weight up,
//   h = G_{S+1};  h = h 2^-8 + G_g  (g = S .. 2);  C = h 2^(e_i + f_j - 12),
// which equals adding the scaled group sums smallest first (the scaling by
// powers of two is exact).  Then, by mode:
//   EPI_STORE   C (rows < M, columns < N)
//   EPI_SQUARE  X2 = P P on tiles I <= J, mirrored; tile partials of
//               tr(P - X2) and sum_ij X2_ij (delta_ij - P_ij) = tr(X2 - P^3)
//   EPI_UPDATE  P' = alpha P + beta X2 + gamma (X2 P) on tiles I <= J,
//               mirrored; tile partials of tr(P' H) and tr P'
// In the two purification modes a diagonal tile keeps only its upper
// triangle and mirrors it, so every iterate is exactly symmetric and its row
// digits also serve as its column digits.
#include "common.hpp"

namespace dmp {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Two workgroups per CU while the group accumulators, operand fragments and
// staging registers fit in 256 registers per lane; one beyond that.
template <int S, bool FP16>
struct MinBlocks { static constexpr int value = (FP16 ? S <= 5 : S <= 8) ? 2 : 1; };

template <int S, bool FP16>
__global__ __launch_bounds__(256, (MinBlocks<S, FP16>::value)) void k_ozgemm(GemmParams p) {
    constexpr int PLANE_RUN = S * kFragBytes;          // bytes of one (rb, chunk)
    constexpr int U4_PER_THREAD = S;                   // 4 runs / 256 threads
    __shared__ __align__(16) uint8_t lds[2][4][PLANE_RUN];
    __shared__ double red[4][kPartials];

    // XCD-aware block order: hardware hands consecutive blocks to the 8 XCDs
    // in turn; give every XCD one contiguous slice of the tile list.
    const int nb = gridDim.x, b = blockIdx.x;
    const int xcd = b & 7, q = nb >> 3, rem = nb & 7, loc = b >> 3;
    const int t = (xcd < rem) ? xcd * (q + 1) + loc : rem * (q + 1) + (xcd - rem) * q + loc;
    const Tile tile = p.tiles[t];
    const MatDesc& d = p.descs ? p.descs[tile.mat] : p.one;
    const DevState* st = p.states ? p.states + d.state_index : nullptr;
    if (st != nullptr && st->done) return;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int I = tile.I, J = tile.J;
    const uint8_t* a0 = d.pa + int64_t(2 * I) * d.a_rb_stride;
    const uint8_t* b0 = d.pb + int64_t(2 * J) * d.b_rb_stride;
    const int KC = d.KC;

    uint4 stage[U4_PER_THREAD];
    auto gload = [&](int kc) {
#pragma unroll
        for (int r = 0; r < U4_PER_THREAD; ++r) {
            const int qi = r * 256 + tid;                  // uint4 index in 4 runs
            const int ob = qi / (S * 64), w = qi % (S * 64);
            const uint8_t* base = ob < 2 ? a0 + int64_t(ob) * d.a_rb_stride
                                         : b0 + int64_t(ob - 2) * d.b_rb_stride;
            stage[r] = *reinterpret_cast<const uint4*>(base + int64_t(kc) * PLANE_RUN + w * 16);
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int r = 0; r < U4_PER_THREAD; ++r) {
            const int qi = r * 256 + tid;
            const int ob = qi / (S * 64), w = qi % (S * 64);
            *reinterpret_cast<uint4*>(&lds[buf][ob][w * 16]) = stage[r];
        }
    };

    v16i acc[S];
#pragma unroll
    for (int g = 0; g < S; ++g)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[g][v] = 0;

    if (KC > 0) {
        gload(0);
        lstore(0);
    }
    __syncthreads();
    for (int kc = 0; kc < KC; ++kc) {
        const int buf = kc & 1;
        if (kc + 1 < KC) gload(kc + 1);
        v4i fa[S], fb[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            fa[s] = *reinterpret_cast<const v4i*>(&lds[buf][wm][s * kFragBytes + lane * 16]);
            fb[s] = *reinterpret_cast<const v4i*>(&lds[buf][2 + wn][s * kFragBytes + lane * 16]);
        }
#pragma unroll
        for (int g = 2; g <= S + 1; ++g) {
            if constexpr (!FP16) {
#pragma unroll
                for (int i = 1; i < g; ++i) {
                    const int j = g - i;
                    if (j <= S)
                        acc[g - 2] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[i - 1], fb[j - 1],
                                                                           acc[g - 2], 0, 0, 0);
                }
            } else {
                v16f tmp;
#pragma unroll
                for (int v = 0; v < 16; ++v) tmp[v] = 0.0f;
#pragma unroll
                for (int i = 1; i < g; ++i) {
                    const int j = g - i;
                    if (j <= S)
                        tmp = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                            __builtin_bit_cast(v8h, fa[i - 1]), __builtin_bit_cast(v8h, fb[j - 1]),
                            tmp, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[g - 2][v] += int(tmp[v]);
            }
        }
        if (kc + 1 < KC) lstore(buf ^ 1);
        __syncthreads();
    }

    // ---- epilogue -----------------------------------------------------------
    const int col = J * kTile + wn * 32 + (lane & 31);
    const int row0 = I * kTile + wm * 32 + (lane >> 5) * 4;
    const int fj = d.eb[col];
    const int mode = p.mode;
    double alpha = 0.0, beta = 0.0, gamma = 0.0;
    if (mode == EPI_UPDATE) {
        alpha = st->alpha;
        beta = st->beta;
        gamma = st->gamma;
    }
    const int n = d.M;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = row0 + (v >> 2) * 8 + (v & 3);
        double h = double(acc[S - 1][v]);
#pragma unroll
        for (int g = S - 2; g >= 0; --g) h = h * 0x1p-8 + double(acc[g][v]);
        const int ei = d.ea[row];
        double c = (ei >= kNonFiniteExp || fj >= kNonFiniteExp)
                       ? __builtin_nan("")
                       : ldexp(h, ei + fj - 2 * kTopBits);
        if (mode == EPI_STORE) {
            if (row < d.M && col < d.N) d.out[int64_t(row) * d.ldc + col] = c;
            continue;
        }
        if (row >= n || col >= n) continue;
        if (I == J && row > col) continue;
        const bool diag = (row == col);
        const double mult = diag ? 1.0 : 2.0;
        const int64_t ij = int64_t(row) * n + col, ji = int64_t(col) * n + row;
        const double pij = d.P[ij];
        if (mode == EPI_SQUARE) {
            d.out[ij] = c;
            if (!diag) d.out[ji] = c;
            if (diag) s0 += pij - c;
            s1 += mult * c * ((diag ? 1.0 : 0.0) - pij);
        } else {  // EPI_UPDATE
            const double nv = alpha * pij + beta * d.X2[ij] + gamma * c;
            d.out[ij] = nv;
            if (!diag) d.out[ji] = nv;
            s0 += mult * nv * d.H[ij];
            if (diag) s1 += nv;
        }
    }
    if (mode != EPI_STORE) {
        s0 = wave_sum(s0);
        s1 = wave_sum(s1);
        if (lane == 0) {
            red[wave][0] = s0;
            red[wave][1] = s1;
        }
        __syncthreads();
        if (tid == 0) {
            p.partials[int64_t(t) * kPartials + 0] = ((red[0][0] + red[1][0]) + red[2][0]) + red[3][0];
            p.partials[int64_t(t) * kPartials + 1] = ((red[0][1] + red[1][1]) + red[2][1]) + red[3][1];
        }
    }
}

template <int S>
static void launch_s(bool fp16, const GemmParams& p, int ntiles, hipStream_t stream) {
    if (fp16)
        k_ozgemm<S, true><<<ntiles, 256, 0, stream>>>(p);
    else
        k_ozgemm<S, false><<<ntiles, 256, 0, stream>>>(p);
}

using GemmFn = void (*)(bool, const GemmParams&, int, hipStream_t);
static const GemmFn kGemm[kMaxSlices + 1] = {
    nullptr,     launch_s<1>, launch_s<2>, launch_s<3>,  launch_s<4>,  launch_s<5>, launch_s<6>,
    launch_s<7>, launch_s<8>, launch_s<9>, launch_s<10>, launch_s<11>, launch_s<12>};

int launch_ozgemm(int S, dmp_kind kind, const GemmParams& p, int ntiles, hipStream_t stream) {
    if (ntiles <= 0) return DMP_OK;
    kGemm[S](kind == DMP_OZ_FP16, p, ntiles, stream);
    DMP_CHECK_HIP(hipGetLastError());
    return DMP_OK;
}

}  // namespace dmp
