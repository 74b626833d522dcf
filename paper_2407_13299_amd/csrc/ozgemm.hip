// Slice-pair products of the Ozaki scheme (Sec. 2.4) on gfx950 matrix cores,
// with the FP64 summation and the purification work fused into the epilogue.
//
// A workgroup of 8 wavefronts owns one 128 x 64 output tile (4 x 2 quadrants
// of 32 x 32, one per wavefront), or, in the 64-row variant, 4 wavefronts own
// a 64 x 64 tile (see RB below).  The reduction runs in chunks (32 INT8 or
// 16 FP16 elements); one chunk of a 128 x 64 tile is 6 S fragment blocks of
// 1 KiB (4 row blocks of the left operand, 2 of the right, S digit planes
// each; 4 S for 64 x 64), contiguous in HBM per row block.  The fragment
// blocks go from memory straight into LDS (buffer loads with the LDS flag:
// no register staging, no LDS stores), into three LDS stages (128-row
// tiles: chunk c + 2 is loaded while chunk c is multiplied) or two (64-row
// tiles, two workgroups per CU: chunk c + 1), with one barrier per chunk.
// Every wavefront forms all S (S + 1) / 2 slice pairs (i + j <= S + 1):
//   INT8: v_mfma_i32_32x32x32_i8, exact INT32 sums; one accumulator per
//         anti-diagonal group g = i + j (products of the same weight
//         2^-(8g - 4) add exactly), (g - 1) k 2^14 < 2^31 checked on the host;
//         loop over the left slice i (inner: right slice j), so consecutive
//         MFMAs feed different accumulators;
//   FP16: v_mfma_f32_32x32x16_f16; per group and chunk the FP32 sum is an
//         integer of magnitude <= 16 (g - 1) 2^14 <= 2^24, hence exact, and is
//         converted to INT32 and added to the group accumulator.
// Epilogue, per element: Horner over the groups from the smallest weight up,
//   h = G_{S+1};  h = h 2^-8 + G_g  (g = S .. 2);  C = h 2^(e_i + f_j - 12),
// equal to adding the scaled group sums smallest first (power-of-two
// scalings are exact).  Then, by mode:
//   EPI_STORE   C (rows < M, columns < N); optionally the row and column
//               maxima of |C| (bit patterns, atomicMax) for the next splits
//   EPI_STORE_SYM  C = A B known to be symmetric (square): upper tiles only,
//               C_ij stored and mirrored (optionally its row maxima)
//   EPI_SQUARE  X2 = P P for row <= col, mirrored; tile partials of
//               tr(P - X2) and sum_ij X2_ij (delta_ij - P_ij) = tr(X2 - P^3)
//   EPI_UPDATE  P' = alpha P + beta X2 + gamma (X2 P) for row <= col,
//               mirrored; tile partials of tr(P' H) and tr P' (gamma == 0:
//               no products at all, P' = alpha P + beta X2)
// (GemmParams::upper_only: the purification modes store the upper triangle
// only; the row maxima still cover the mirror's rows)
//   EPI_SQUARE_TRS4  X2 = X X as EPI_SQUARE; partials of tr F = tr(X2 (4X -
//               3 X2)) and tr G = ||X - X2||_F^2 (TRS4, Sec. 3)
// In the purification modes only the upper triangle is computed and kept,
// so every iterate is exactly symmetric and its row digits also serve as its
// column digits.
#include "common.hpp"

namespace dmp {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

// Workgroup barrier without the memory fence __syncthreads() implies (that
// fence would also wait for the prefetch loads in flight); the signal fences
// keep the compiler from moving memory accesses across it.  Before each
// barrier the kernel waits for its own operand loads and LDS reads itself
// (ops_wait).
__device__ inline void bare_barrier() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Fourth word of a raw buffer descriptor on gfx950 (32-bit data format,
// no swizzle, no index stride).
constexpr int kBufferWord3 = 0x00020000;

typedef __attribute__((address_space(3))) uint8_t lds_u8;

// Byte offset of a shared-memory address inside the workgroup's LDS.
__device__ inline uint32_t lds_offset(const void* p) {
    return static_cast<uint32_t>(reinterpret_cast<size_t>((const lds_u8*)(p)));
}

// A raw buffer descriptor (base, no stride, ``bytes`` records) as four
// wave-uniform words, for the inline assembly below, which takes it in
// scalar registers.
__device__ inline v4i sgpr_desc(const void* base, int bytes) {
    const uint64_t b = reinterpret_cast<uint64_t>(base);
    v4i d;
    d[0] = __builtin_amdgcn_readfirstlane(int(uint32_t(b)));
    d[1] = __builtin_amdgcn_readfirstlane(int(uint32_t(b >> 32) & 0xffffu));
    d[2] = __builtin_amdgcn_readfirstlane(bytes);
    d[3] = kBufferWord3;
    return d;
}

// One 1 KiB fragment block from global memory straight into LDS (a buffer
// load with the LDS flag): lane l's 16 bytes at buffer offset voff + soff
// land at LDS byte lds + 16 l, which is exactly the fragment layout, so no
// register staging and no LDS store instruction is needed.  It is written
// as inline assembly so that the compiler's wait counting, which would
// otherwise wait for every such load before any LDS read, leaves it alone;
// the kernel waits for these loads itself (ops_wait) before the barrier
// that publishes them.  The load has no register destination; m0 holds the
// LDS address and is set right before it.  m0 is a register the compiler
// reserves; nothing else in these kernels reads it (gfx950 LDS instructions
// do not use it), which tests/test_isa_m0.py checks on the compiled code.
__device__ inline void frag_to_lds(v4i r, uint32_t lds, int voff, int soff) {
    // the operands are wave-uniform; reading them from the first lane makes
    // them scalar registers at this point even where register pressure has
    // moved them to vector registers in between
    v4i rs;
#pragma unroll
    for (int q = 0; q < 4; ++q) rs[q] = __builtin_amdgcn_readfirstlane(r[q]);
    const uint32_t ls = __builtin_amdgcn_readfirstlane(lds);
    const int ss = __builtin_amdgcn_readfirstlane(soff);
    asm volatile("s_mov_b32 m0, %0\n\tbuffer_load_dwordx4 %1, %2, %3 offen lds"
                 :: "s"(ls), "v"(voff), "s"(rs), "s"(ss) : "memory", "m0");
}

// s_waitcnt vmcnt(N) lgkmcnt(0): at most N vector-memory operations of the
// wavefront still in flight, and every LDS read returned.
template <int N>
__device__ inline void ops_wait() {
    asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)" :: "n"(N) : "memory");
}

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// TERMS > 0: the Markidis product (Sec. 4.5) on the same tiles: S = 2 FP16
// planes (high, low parts), the first TERMS of A0 B0, A0 B1, A1 B0, A1 B1
// accumulated in one FP32 accumulator, and C = acc 2^(e_i + f_j).
// PUR: the purification epilogues (EPI_SQUARE, EPI_UPDATE, EPI_SQUARE_TRS4);
// otherwise the plain ones (EPI_STORE, EPI_STORE_SYM).  Two instantiations
// keep each epilogue free of the other family's code.
// RB: 32-row blocks of the left operand per tile.  RB = 4: 128 x 64 tiles,
// 8 wavefronts, one workgroup per CU (126 KiB of LDS at S = 7).  RB = 2:
// 64 x 64 tiles, 4 wavefronts, 56 KiB, two workgroups per CU, so that one
// tile's pipeline fill and epilogue overlap another's main loop (small
// matrices, where those are a large share of a tile's time).
// PHASE: kWhole for whole tiles; the split tail (GemmParams::fix) adds two
// launches: kPiece, one block per part (its share of the chunks, group sums
// stored, no epilogue), then kFixup, one block per split tile (adds the
// parts' group sums in place of the main loop, then runs the epilogue).
// Separate instantiations keep the whole-tile kernel's registers as they are.
constexpr int kWhole = 0, kPiece = 1, kFixup = 2;
template <int S, bool FP16, int TERMS = 0, bool PUR = false, int RB = 4, int PHASE = kWhole>
__global__ __launch_bounds__(128 * RB, RB == 4 ? 1 : 2) void k_ozgemm(GemmParams p) {
    constexpr int BLOCKS = (RB + 2) * S;          // 1 KiB blocks per chunk
    constexpr int STAGE = BLOCKS * kFragBytes;
    constexpr int WAVES = 2 * RB;
    constexpr int PER = (BLOCKS + WAVES - 1) / WAVES;  // loads per wavefront per chunk
    // LDS stages: three for the 128-row tiles (one workgroup per CU) while
    // they fit, else two (the 64-row tiles keep two workgroups per CU)
    constexpr int NBUF = RB == 4 && 3 * STAGE <= 150 * 1024 ? 3 : 2;
    __shared__ __align__(16) uint8_t lds[NBUF][STAGE];
    __shared__ double red[WAVES][kPartials];

    static_assert(PHASE == kWhole || TERMS == 0, "tail split: Ozaki kinds");
    // XCD-aware block order: the hardware hands consecutive blocks to the 8
    // XCDs in turn; give every XCD one contiguous slice of the tile list.
    const int b = blockIdx.x;
    int t, part = 0;
    if constexpr (PHASE == kWhole) {
        const int nb = gridDim.x;
        const int xcd = b & 7, q = nb >> 3, rem = nb & 7, loc = b >> 3;
        t = p.spread ? b : (xcd < rem) ? xcd * (q + 1) + loc : rem * (q + 1) + (xcd - rem) * q + loc;
    } else if constexpr (PHASE == kPiece) {
        t = p.nfull + b / p.nsplit;
        part = b - (t - p.nfull) * p.nsplit;
    } else {
        t = p.nfull + b;
    }
    const Tile tile = p.tiles[t];
    const MatDesc d = p.descs ? p.descs[tile.mat] : p.one;
    const DevState* st = p.states ? p.states + d.state_index : nullptr;
    if (st != nullptr && st->done) return;
    // clock stamps (timing mode): wave-uniform, so they live in scalar
    // registers and leave the vector register budget of the loop untouched
    const bool clocked = p.clk != nullptr;
    const uint64_t clk_c = clocked ? __builtin_amdgcn_s_memtime() : 0;
    const uint64_t clk_r = clocked ? __builtin_amdgcn_s_memrealtime() : 0;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
    const int wm = wave >> 1, wn = wave & 1;
    const int I = tile.I, J = tile.J;
    // chunks of this block: all of them, or those of its part
    int KC = d.KC, kbase = 0;
    if constexpr (PHASE == kPiece) {
        kbase = int(int64_t(d.KC) * part / p.nsplit);
        KC = int(int64_t(d.KC) * (part + 1) / p.nsplit) - kbase;
    }
    const int64_t a_rb = d.a_rb_stride, b_rb = d.b_rb_stride;
    // Piece i of this thread: block i * WAVES + wave (wave-uniform), lane.
    // Block b of a chunk is digit plane b % S of operand row block b / S (left
    // operand row blocks RB I .. RB I + RB - 1, then right operand row blocks
    // 2J, 2J+1).
    // Loads are buffer loads straight into LDS: one descriptor per piece
    // holding the base of its row block (wave-uniform, scalar registers),
    // the per-chunk offset in a scalar register and the lane's 16 bytes as
    // the only vector offset.  Pieces past the last block are not loaded:
    // wavefronts [0, FULL) issue PER loads per chunk, the others PER - 1.
    constexpr int FULL = BLOCKS - (PER - 1) * WAVES;
    v4i dsc[PER];
    int poff[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int blk0 = i * WAVES + wave;
        const int blk = blk0 < BLOCKS ? blk0 : 0;
        const int ob = blk / S;
        poff[i] = (blk % S) * kFragBytes + kbase * (S * kFragBytes);
        const uint8_t* base = ob < RB ? d.pa + int64_t(RB * I + ob) * a_rb
                                      : d.pb + int64_t(2 * J + ob - RB) * b_rb;
        const int64_t rb = ob < RB ? a_rb : b_rb;   // bytes of one row block
        dsc[i] = sgpr_desc(base, int(rb));
    }
    const uint32_t lbase = lds_offset(&lds[0][0]);
    // loads of chunk kc into LDS stage ``stage``
    auto issue = [&](int kc, int stage) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int blk = i * WAVES + wave;
            if (i < PER - 1 || blk < BLOCKS)
                frag_to_lds(dsc[i], lbase + uint32_t(stage * STAGE + blk * kFragBytes), lane * 16,
                            kc * (S * kFragBytes) + poff[i]);
        }
    };
    // wait for this wavefront's loads of every chunk but the newest one
    // (and for its LDS reads), then the barrier
    const bool full = wave < FULL;
    auto publish_older = [&]() __attribute__((always_inline)) {
        if (full) ops_wait<PER>(); else ops_wait<PER - 1>();
        bare_barrier();
    };
    auto publish_all = [&]() __attribute__((always_inline)) {
        ops_wait<0>();
        bare_barrier();
    };

    static_assert(TERMS == 0 || (S == 2 && FP16), "Markidis: two FP16 planes");
    v16i acc[S];
#pragma unroll
    for (int g = 0; g < S; ++g)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[g][v] = 0;
    v16f accf;
#pragma unroll
    for (int v = 0; v < 16; ++v) accf[v] = 0.0f;

    auto compute = [&](int buf) __attribute__((always_inline)) {
        const uint8_t* sa = &lds[buf][(wm * S) * kFragBytes + lane * 16];
        const uint8_t* sb = &lds[buf][((RB + wn) * S) * kFragBytes + lane * 16];
        if constexpr (TERMS > 0) {
            const v8h a0 = __builtin_bit_cast(v8h, *reinterpret_cast<const v4i*>(sa));
            const v8h b0 = __builtin_bit_cast(v8h, *reinterpret_cast<const v4i*>(sb));
            accf = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0, b0, accf, 0, 0, 0);
            if constexpr (TERMS >= 2) {
                const v8h b1 = __builtin_bit_cast(v8h, *reinterpret_cast<const v4i*>(sb + kFragBytes));
                accf = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0, b1, accf, 0, 0, 0);
                if constexpr (TERMS >= 3) {
                    const v8h a1 = __builtin_bit_cast(v8h, *reinterpret_cast<const v4i*>(sa + kFragBytes));
                    accf = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1, b0, accf, 0, 0, 0);
                    if constexpr (TERMS >= 4)
                        accf = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1, b1, accf, 0, 0, 0);
                }
            }
        } else if constexpr (!FP16) {
            v4i fb[S];
#pragma unroll
            for (int s = 0; s < S; ++s) fb[s] = *reinterpret_cast<const v4i*>(sb + s * kFragBytes);
#pragma unroll
            for (int i = 1; i <= S; ++i) {
                const v4i fa = *reinterpret_cast<const v4i*>(sa + (i - 1) * kFragBytes);
#pragma unroll
                for (int j = 1; j <= S + 1 - i; ++j)
                    acc[i + j - 2] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa, fb[j - 1], acc[i + j - 2], 0, 0, 0);
            }
        } else {
            v4i fa[S], fb[S];
#pragma unroll
            for (int s = 0; s < S; ++s) {
                fa[s] = *reinterpret_cast<const v4i*>(sa + s * kFragBytes);
                fb[s] = *reinterpret_cast<const v4i*>(sb + s * kFragBytes);
            }
#pragma unroll
            for (int g = 2; g <= S + 1; ++g) {
                v16f tmp;
#pragma unroll
                for (int v = 0; v < 16; ++v) tmp[v] = 0.0f;
#pragma unroll
                for (int i = 1; i < g; ++i) {
                    const int j = g - i;
                    if (j <= S)
                        tmp = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(v8h, fa[i - 1]),
                                                                     __builtin_bit_cast(v8h, fb[j - 1]),
                                                                     tmp, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[g - 2][v] += int(tmp[v]);
            }
        }
    };

    // an update whose product weight is zero (a TRS4 step without the
    // second product) keeps only the elementwise part
    const bool no_product = PUR && p.mode == EPI_UPDATE && st != nullptr && st->gamma == 0.0;
    auto add_clock = [&]() __attribute__((always_inline)) {
        if (clocked) {
            const uint64_t dc = __builtin_amdgcn_s_memtime() - clk_c;
            const uint64_t dr = __builtin_amdgcn_s_memrealtime() - clk_r;
            if (threadIdx.x == 0) {
                atomicAdd(p.clk + 0, static_cast<unsigned long long>(dc));
                atomicAdd(p.clk + 1, static_cast<unsigned long long>(dr));
            }
        }
    };
    // Part u of the split tail keeps its group sums at piece u of p.fix:
    // [wavefront][group][4 x 4 values][lane], 16 bytes per lane and store.
    constexpr int64_t kPieceInts = int64_t(WAVES) * S * 16 * 64;
    if constexpr (PHASE == kFixup) {
        if (!no_product) {
            const int* src = p.fix + int64_t(b) * p.nsplit * kPieceInts +
                             int64_t(wave) * (S * 16 * 64) + lane * 4;
            for (int pt = 0; pt < p.nsplit; ++pt) {
#pragma unroll
                for (int g = 0; g < S; ++g)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const v4i x = *reinterpret_cast<const v4i*>(src + (g * 4 + q) * 256);
#pragma unroll
                        for (int e = 0; e < 4; ++e) acc[g][4 * q + e] += x[e];
                    }
                src += kPieceInts;
            }
        }
    } else {
        // Chunk c lives in LDS stage c mod NBUF.  Three stages: chunk c + 2
        // is loaded while chunk c is multiplied, and the barrier ending the
        // step publishes chunk c + 1.  Two stages: chunk c + 1 is loaded
        // while chunk c is multiplied and published at the end of the step.
        // A stage is reloaded only after the barrier that follows the last
        // reads of the chunk it held.
        if (!no_product && KC > 0) {
            if constexpr (NBUF == 3) {
                issue(0, 0);
                if (KC > 1) {
                    issue(1, 1);
                    publish_older();
                } else {
                    publish_all();
                }
                int stage = 0;
                for (int kc = 0; kc < KC; ++kc) {
                    const bool more = kc + 2 < KC;
                    if (more) issue(kc + 2, stage == 0 ? 2 : stage - 1);   // (kc + 2) mod 3
                    compute(stage);
                    __builtin_amdgcn_sched_barrier(0);   // as in the two-stage loop
                    if (more) publish_older(); else publish_all();
                    stage = stage == 2 ? 0 : stage + 1;
                }
            } else {
                issue(0, 0);
                publish_all();
                int stage = 0;
                for (int kc = 0; kc < KC; ++kc) {
                    if (kc + 1 < KC) issue(kc + 1, stage ^ 1);
                    compute(stage);
                    // keep every product of the chunk ahead of the barrier
                    // (the scheduler would otherwise move some past it, so the
                    // wave would wait at the barrier with little of its own
                    // work in the matrix core)
                    __builtin_amdgcn_sched_barrier(0);
                    publish_all();
                    stage ^= 1;
                }
            }
        }
        if constexpr (PHASE == kPiece) {
            if (!no_product) {
                int* dst = p.fix + int64_t(b) * kPieceInts + int64_t(wave) * (S * 16 * 64) + lane * 4;
#pragma unroll
                for (int g = 0; g < S; ++g)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        *reinterpret_cast<v4i*>(dst + (g * 4 + q) * 256) =
                            v4i{acc[g][4 * q], acc[g][4 * q + 1], acc[g][4 * q + 2], acc[g][4 * q + 3]};
            }
            add_clock();
            return;
        }
    }

    // ---- epilogue -----------------------------------------------------------
    const int col = J * kTileN + wn * 32 + (lane & 31);
    const int row0 = I * (32 * RB) + wm * 32 + (lane >> 5) * 4;
    const int fj = d.eb[col];
    const int mode = p.mode;
    double alpha = 0.0, beta = 0.0, gamma = 0.0;
    if (PUR && mode == EPI_UPDATE) {
        alpha = st->alpha;
        beta = st->beta;
        gamma = st->gamma;
    }
    const int n = d.M;
    double s0 = 0.0, s1 = 0.0;
    // Maxima of |output| for the next splits, as bit patterns (for
    // non-negative doubles the integer order is the numeric order, a NaN
    // above an infinity): per row, over the 32 lanes of a half-wavefront
    // (the columns of the row, reduce-scatter below); per column, over the
    // lane's 16 elements.  In the mirrored modes a column of the tile is a row of the
    // mirror, so both go to rowmax; in EPI_STORE the columns go to colmax.
    // Trace partials and the P, X2, H inputs: the purification modes only.
    constexpr bool traces = PUR;
    const bool rowmax = d.rowmax != nullptr;
    uint64_t* const colmax_dst = (!PUR && mode == EPI_STORE) ? d.colmax : d.rowmax;
    uint64_t rbits[16];   // |output| bit patterns of the lane's 16 elements
    uint64_t cmax = 0;
    auto absbits = [](double x) __attribute__((always_inline)) {
        return static_cast<uint64_t>(__double_as_longlong(x)) & 0x7fffffffffffffffull;
    };
    // The epilogue runs in three phases: the group sums of all 16 elements
    // of the lane are combined first (the accumulators are then dead), then
    // every load of the epilogue is issued, then the outputs are formed and
    // stored.  The compiler cannot tell that the output does not alias P,
    // X2, H or the exponents, so a load placed after a store would wait for
    // it and every element would pay a full memory latency.
    double hsum[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        if constexpr (TERMS > 0) {
            hsum[v] = double(accf[v]);
        } else {
            double h = double(acc[S - 1][v]);
#pragma unroll
            for (int g = S - 2; g >= 0; --g) h = h * 0x1p-8 + double(acc[g][v]);
            hsum[v] = h;
        }
    }
    // Materialise the combined sums here (an empty asm statement that takes
    // each as a register operand): otherwise the combination is sunk to its
    // uses below, past the loads, and the accumulators stay live beside them.
#pragma unroll
    for (int v = 0; v < 16; ++v) asm volatile("" : "+v"(hsum[v]));
    // The base pointers pass through the same kind of empty statement, so the
    // loads below depend on this point and are not hoisted above the main
    // loop (where their results would hold registers all along).
    const int* ea = d.ea;
    const double *Pin = d.P, *X2in = d.X2, *Hin = d.H;
    asm volatile("" : "+s"(ea), "+s"(Pin), "+s"(X2in), "+s"(Hin));
    int eiv[16];
    double pv[16], xv[16], hv[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = row0 + (v >> 2) * 8 + (v & 3);
        eiv[v] = ea[row];
        pv[v] = xv[v] = hv[v] = 0.0;
        if (traces && row < n && col < n && row <= col) {
            const int64_t ij = int64_t(row) * n + col;
            pv[v] = Pin[ij];
            if (mode == EPI_UPDATE) {
                xv[v] = X2in[ij];
                hv[v] = Hin[ij];
            }
        }
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = row0 + (v >> 2) * 8 + (v & 3);
        const double h = hsum[v];
        const int ei = eiv[v];
        constexpr int shift = TERMS > 0 ? 0 : 2 * kTopBits;
        const double c = no_product ? 0.0
                         : (ei >= kNonFiniteExp || fj >= kNonFiniteExp)
                             ? __builtin_nan("")
                             : ldexp(h, ei + fj - shift);
        uint64_t bits = 0;
        if (!PUR && mode == EPI_STORE) {
            if (row < d.M && col < d.N) {
                d.out[int64_t(row) * d.ldc + col] = c;
                bits = absbits(c);
                cmax = bits > cmax ? bits : cmax;
            }
        } else if (!PUR) {   // EPI_STORE_SYM
            if (row < n && col < n && row <= col) {
                d.out[int64_t(row) * n + col] = c;
                if (row != col) d.out[int64_t(col) * n + row] = c;
                bits = absbits(c);
                cmax = bits > cmax ? bits : cmax;
            }
        } else if (row < n && col < n && row <= col) {
            const bool diag = (row == col);
            const double mult = diag ? 1.0 : 2.0;
            const int64_t ij = int64_t(row) * n + col, ji = int64_t(col) * n + row;
            const double pij = pv[v];
            double w;
            if (mode == EPI_SQUARE) {
                w = c;
                if (diag) s0 += pij - c;
                s1 += mult * c * ((diag ? 1.0 : 0.0) - pij);
            } else if (mode == EPI_SQUARE_TRS4) {
                // tr F = sum_ij X2_ij (4 X_ij - 3 X2_ij), tr G = sum_ij (X_ij - X2_ij)^2
                w = c;
                const double r = pij - c;
                s0 += mult * c * (4.0 * pij - 3.0 * c);
                s1 += mult * r * r;
            } else {  // EPI_UPDATE
                w = alpha * pij + beta * xv[v] + gamma * c;
                s0 += mult * w * hv[v];
                if (diag) s1 += w;
            }
            d.out[ij] = w;
            if (!diag && !p.upper_only) d.out[ji] = w;
            bits = absbits(w);
            cmax = bits > cmax ? bits : cmax;      // its mirror (col, row) of row ``col``
        }
        rbits[v] = bits;
    }
    if (rowmax) {
        // Row maxima by a reduce-scatter over the 32 lanes (columns) of each
        // half-wavefront: in the step over lane bit b (16, 8, 4, 2) a lane
        // keeps half of its current values (the upper half if its bit b is
        // set), sends the other half to lane ^ b and takes the maximum with
        // what it receives.  After four steps lane l holds row element
        // v = (l >> 1) & 15 reduced over 16 columns; lanes l and l ^ 1 then
        // combine.  16 exchanges instead of the 80 of one butterfly per element.
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int bit = 16 >> k, h = 8 >> k;
            const bool up = (lane & bit) != 0;
#pragma unroll
            for (int i = 0; i < h; ++i) {
                const uint64_t send = up ? rbits[i] : rbits[i + h];
                const uint64_t keep = up ? rbits[i + h] : rbits[i];
                const uint64_t o = static_cast<uint64_t>(__shfl_xor(static_cast<long long>(send), bit, 64));
                rbits[i] = o > keep ? o : keep;
            }
        }
        const uint64_t o = static_cast<uint64_t>(__shfl_xor(static_cast<long long>(rbits[0]), 1, 64));
        const uint64_t mx = o > rbits[0] ? o : rbits[0];
        const int myv = (lane & 31) >> 1;
        const int myrow = row0 + (myv >> 2) * 8 + (myv & 3);
        if ((lane & 1) == 0 && myrow < d.M && mx != 0)
            atomicMax(reinterpret_cast<unsigned long long*>(d.rowmax) + myrow,
                      static_cast<unsigned long long>(mx));
    }
    if (colmax_dst != nullptr) {
        // columns: both halves hold rows of the same column; in the mirrored
        // modes the column's elements are the mirror's row ``col``
        const uint64_t o = static_cast<uint64_t>(__shfl_xor(static_cast<long long>(cmax), 32, 64));
        cmax = o > cmax ? o : cmax;
        if (lane < 32 && col < d.N && cmax != 0)
            atomicMax(reinterpret_cast<unsigned long long*>(colmax_dst) + col,
                      static_cast<unsigned long long>(cmax));
    }
    if (traces) {
        s0 = wave_sum(s0);
        s1 = wave_sum(s1);
        if (lane == 0) {
            red[wave][0] = s0;
            red[wave][1] = s1;
        }
        __syncthreads();
        if (tid == 0) {
            double r0 = 0.0, r1 = 0.0;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) {
                r0 += red[w][0];
                r1 += red[w][1];
            }
            p.partials[int64_t(t) * kPartials + 0] = r0;
            p.partials[int64_t(t) * kPartials + 1] = r1;
        }
    }
    add_clock();
}

static bool purification_mode(int mode) {
    return mode == EPI_SQUARE || mode == EPI_UPDATE || mode == EPI_SQUARE_TRS4;
}

// The parts of a split tail run no epilogue, so one instantiation (the
// purification one) serves every mode.
template <int S, int PHASE>
static void launch_s(bool fp16, const GemmParams& p, int ntiles, int rb, hipStream_t stream) {
    const bool pur = PHASE == kPiece || purification_mode(p.mode);
    if constexpr (S <= kMaxSlices64) {   // the 64-row variant
        if (rb == 2) {
            if (fp16 && pur)
                k_ozgemm<S, true, 0, true, 2, PHASE><<<ntiles, 256, 0, stream>>>(p);
            else if (pur)
                k_ozgemm<S, false, 0, true, 2, PHASE><<<ntiles, 256, 0, stream>>>(p);
            else if constexpr (PHASE != kPiece) {
                if (fp16)
                    k_ozgemm<S, true, 0, false, 2, PHASE><<<ntiles, 256, 0, stream>>>(p);
                else
                    k_ozgemm<S, false, 0, false, 2, PHASE><<<ntiles, 256, 0, stream>>>(p);
            }
            return;
        }
    }
    if (fp16 && pur) {
        k_ozgemm<S, true, 0, true, 4, PHASE><<<ntiles, kGemmThreads, 0, stream>>>(p);
    } else if (pur) {
        k_ozgemm<S, false, 0, true, 4, PHASE><<<ntiles, kGemmThreads, 0, stream>>>(p);
    } else if constexpr (PHASE != kPiece) {
        if (fp16)
            k_ozgemm<S, true, 0, false, 4, PHASE><<<ntiles, kGemmThreads, 0, stream>>>(p);
        else
            k_ozgemm<S, false, 0, false, 4, PHASE><<<ntiles, kGemmThreads, 0, stream>>>(p);
    }
}

// Workgroups of the purification-mode slice GEMM resident per CU.
template <int S>
static int resident_s(bool fp16, int rb, int* per_cu) {
    hipError_t e;
    if constexpr (S <= kMaxSlices64) {
        if (rb == 2) {
            e = fp16 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_ozgemm<S, true, 0, true, 2>, 256, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_ozgemm<S, false, 0, true, 2>, 256, 0);
            return e == hipSuccess ? DMP_OK : DMP_EHIP;
        }
    }
    e = fp16 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_ozgemm<S, true, 0, true>, kGemmThreads, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_ozgemm<S, false, 0, true>, kGemmThreads, 0);
    return e == hipSuccess ? DMP_OK : DMP_EHIP;
}

using GemmFn = void (*)(bool, const GemmParams&, int, int, hipStream_t);
#define DMP_GEMM_TABLE(PH)                                                                    \
    {nullptr,          launch_s<1, PH>,  launch_s<2, PH>,  launch_s<3, PH>,  launch_s<4, PH>,   \
     launch_s<5, PH>,  launch_s<6, PH>,  launch_s<7, PH>,  launch_s<8, PH>,  launch_s<9, PH>,   \
     launch_s<10, PH>, launch_s<11, PH>, launch_s<12, PH>}
static const GemmFn kGemm[3][kMaxSlices + 1] = {DMP_GEMM_TABLE(kWhole), DMP_GEMM_TABLE(kPiece),
                                                DMP_GEMM_TABLE(kFixup)};
#undef DMP_GEMM_TABLE

using ResidentFn = int (*)(bool, int, int*);
static const ResidentFn kResident[kMaxSlices + 1] = {
    nullptr,        resident_s<1>, resident_s<2>,  resident_s<3>,  resident_s<4>,
    resident_s<5>,  resident_s<6>, resident_s<7>,  resident_s<8>,  resident_s<9>,
    resident_s<10>, resident_s<11>, resident_s<12>};

template <int T>
static void launch_terms(const GemmParams& p, int ntiles, hipStream_t stream) {
    if (purification_mode(p.mode))
        k_ozgemm<2, true, T, true><<<ntiles, kGemmThreads, 0, stream>>>(p);
    else
        k_ozgemm<2, true, T, false><<<ntiles, kGemmThreads, 0, stream>>>(p);
}

using TermsFn = void (*)(const GemmParams&, int, hipStream_t);
static const TermsFn kTerms[kMaxTerms + 1] = {nullptr, launch_terms<1>, launch_terms<2>,
                                              launch_terms<3>, launch_terms<4>};

int launch_ozgemm(int S, dmp_kind kind, const GemmParams& p, int ntiles, hipStream_t stream,
                  int rb) {
    if (ntiles <= 0) return DMP_OK;
    if (rb != 4 && (rb != 2 || kind == DMP_MARKIDIS_FP16 || S > kMaxSlices64)) {
        set_error("64-row tiles exist for the Ozaki kinds with S <= %d only", kMaxSlices64);
        return DMP_EINVAL;
    }
    if (p.fix != nullptr) {
        const int tail = ntiles - p.nfull;
        if (kind == DMP_MARKIDIS_FP16 || p.nfull < 0 || tail < 1 ||
            p.nsplit < 2 || int64_t(tail) * p.nsplit > kMaxPieces) {
            set_error("invalid tail split (nfull %d of %d tiles, %d parts)", p.nfull, ntiles, p.nsplit);
            return DMP_EINVAL;
        }
        // whole tiles (full rounds), the parts, then the fixup; each launch
        // starts when the previous one has ended (same stream)
        const bool fp16 = kind == DMP_OZ_FP16;
        if (p.nfull > 0) kGemm[kWhole][S](fp16, p, p.nfull, rb, stream);
        kGemm[kPiece][S](fp16, p, tail * p.nsplit, rb, stream);
        kGemm[kFixup][S](fp16, p, tail, rb, stream);
        DMP_CHECK_HIP(hipGetLastError());
        return DMP_OK;
    }
    if (kind == DMP_MARKIDIS_FP16)
        kTerms[S](p, ntiles, stream);
    else
        kGemm[kWhole][S](kind == DMP_OZ_FP16, p, ntiles, rb, stream);
    DMP_CHECK_HIP(hipGetLastError());
    return DMP_OK;
}

int gemm_slots(int S, dmp_kind kind, int rb, int* slots) {
    *slots = 0;
    if ((kind != DMP_OZ_INT8 && kind != DMP_OZ_FP16) || S < 1 || S > kMaxSlices ||
        (rb == 2 && S > kMaxSlices64) || (rb != 2 && rb != 4)) {
        set_error("no slice GEMM for this kind, S and tile height");
        return DMP_EINVAL;
    }
    int dev = 0, cus = 0, per_cu = 0;
    DMP_CHECK_HIP(hipGetDevice(&dev));
    DMP_CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (kResident[S](kind == DMP_OZ_FP16, rb, &per_cu) != DMP_OK) {
        set_error("occupancy query of the slice GEMM failed");
        return DMP_EHIP;
    }
    *slots = cus * per_cu;
    return DMP_OK;
}

}  // namespace dmp
