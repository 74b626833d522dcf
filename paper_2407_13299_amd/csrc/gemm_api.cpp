// C-ABI entry points of the Ozaki-scheme GEMM (Sec. 2.4).
#include <algorithm>
#include <vector>

#include "host.hpp"

namespace dmp {

namespace {

struct GemmLayout {
    uint8_t* pa;
    uint8_t* pb;
    int* ea;
    int* eb;
    uint64_t* ma;
    uint64_t* mb;
    int* fix;          // part buffer of the split tail (nullable)
    TailSplit tail;
};

// Split tail of the m x n product's 128 x 64 tiles on the current device; the
// workspace query and the launch take the same plan, so the part buffer is
// only as large as the launch needs (none when the tiles fill whole rounds).
TailSplit gemm_tail(int m, int n, int k, int s, dmp_kind kind) {
    const int tiles = m > 0 && n > 0 ? tile_rows(m) * tile_cols(n) : 0;
    TailSplit t{tiles, 1};
    if ((kind != DMP_OZ_INT8 && kind != DMP_OZ_FP16) || k <= 0 || tiles == 0 ||
        !tail_split_enabled())
        return t;
    const int kc = int(chunks_of(k, kind));
    const int cap = tail_split_capacity(tiles, kc, 4);
    int slots = 0;
    if (cap <= 0 || resident_slots(s, kind, 4, &slots) != DMP_OK) {
        clear_error();
        return t;
    }
    return plan_tail_split(tiles, slots, kc, cap);
}

// ``split``: plan a split tail (single products; the grouped launch keeps
// its tiles whole)
GemmLayout carve_gemm(Carver& c, int m, int n, int k, int s, dmp_kind kind, bool split = false) {
    GemmLayout g;
    g.tail = split ? gemm_tail(m, n, k, s, kind) : TailSplit{0, 1};
    g.pa = c.take<uint8_t>(plane_bytes(m, k, s, kind));
    g.pb = c.take<uint8_t>(plane_bytes(n, k, s, kind));
    g.ea = c.take<int>(round_up(m, kPad));
    g.eb = c.take<int>(round_up(n, kPad));
    g.ma = c.take<uint64_t>(round_up(m, kPad));
    g.mb = c.take<uint64_t>(round_up(n, kPad));
    const int tiles = m > 0 && n > 0 ? tile_rows(m) * tile_cols(n) : 0;
    const size_t parts = g.tail.nsplit > 1 ? size_t(tiles - g.tail.nfull) * g.tail.nsplit : 0;
    g.fix = parts > 0 ? c.take<int>(parts * piece_ints(s, 4)) : nullptr;
    return g;
}

__global__ void k_zero_rows(double* c, int m, int n, int ldc) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < int64_t(m) * n) c[(i / n) * ldc + i % n] = 0.0;
}

bool is_trans(char t) { return t == 'T' || t == 't'; }
bool valid_trans(char t) { return t == 'N' || t == 'n' || t == 'T' || t == 't'; }

}  // namespace

}  // namespace dmp

using namespace dmp;

extern "C" {

size_t dmp_gemm_workspace_bytes(int m, int n, int k, int slices, dmp_kind kind) {
    if (kind == DMP_FP64_NATIVE) return 256;
    if (m < 0 || n < 0 || k < 0 || slices < 1 || slices > kMaxSlices) return 0;
    if (kind == DMP_MARKIDIS_FP16 && slices > kMaxTerms) return 0;
    Carver c(nullptr);
    carve_gemm(c, m, n, k, slices, kind, true);
    return c.used();
}

int dmp_ozaki_gemm(char transA, char transB, int m, int n, int k, const double* A, int lda,
                   const double* B, int ldb, double* C, int ldc, int slices, dmp_kind kind,
                   void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    hipStream_t s = static_cast<hipStream_t>(stream);
    DMP_CHECK(check_kind_slices(kind, slices));
    if (!valid_trans(transA) || !valid_trans(transB)) {
        set_error("trans must be 'N' or 'T'");
        return DMP_EINVAL;
    }
    if (m < 0 || n < 0 || k < 0) {
        set_error("negative size");
        return DMP_EINVAL;
    }
    const bool ta = is_trans(transA), tb = is_trans(transB);
    const int a_cols = ta ? m : k, b_cols = tb ? k : n;
    if (lda < std::max(1, a_cols) || ldb < std::max(1, b_cols) || ldc < std::max(1, n)) {
        set_error("leading dimension too small");
        return DMP_EINVAL;
    }
    if (m == 0 || n == 0) return DMP_OK;
    if (C == nullptr || (k > 0 && (A == nullptr || B == nullptr))) {
        set_error("null matrix pointer");
        return DMP_EINVAL;
    }
    if (k == 0) {
        const int64_t tot = int64_t(m) * n;
        k_zero_rows<<<unsigned((tot + 255) / 256), 256, 0, s>>>(C, m, n, ldc);
        DMP_CHECK_HIP(hipGetLastError());
        return DMP_OK;
    }
    if (kind == DMP_FP64_NATIVE) return native_dgemm(s, ta, tb, m, n, k, A, lda, B, ldb, C, ldc);
    if (k > max_k_for(slices, kind)) {
        set_error("k = %d exceeds the exact INT32 range for %d slices (max %lld)", k, slices,
                  (long long)max_k_for(slices, kind));
        return DMP_EINVAL;
    }
    if (m > 65535 * kTileN || n > 65535 * kTileN) {
        set_error("matrix too large");
        return DMP_EINVAL;
    }
    const size_t need = dmp_gemm_workspace_bytes(m, n, k, slices, kind);
    if (ws == nullptr || ws_bytes < need) {
        set_error("workspace of %zu bytes required", need);
        return DMP_ENOMEM;
    }
    DMP_CHECK(check_workspace_alignment(ws));
    Carver c(ws);
    GemmLayout g = carve_gemm(c, m, n, k, slices, kind, true);
    const int KC = int(chunks_of(k, kind));
    const int64_t rb_stride = int64_t(KC) * planes_of(slices, kind) * kFragBytes;

    SplitDesc da{};
    da.A = A;
    da.lda = lda;
    da.R = m;
    da.K = k;
    da.trans = ta ? 1 : 0;
    da.KC = KC;
    da.maxbits = g.ma;
    da.expo = g.ea;
    da.planes = g.pa;
    da.state_index = -1;
    SplitDesc db = da;
    db.A = B;
    db.lda = ldb;
    db.R = n;
    db.trans = tb ? 0 : 1;   // operand row j = column j of op(B)
    db.maxbits = g.mb;
    db.expo = g.eb;
    db.planes = g.pb;
    DMP_CHECK(launch_split(da, slices, kind, nullptr, s));
    DMP_CHECK(launch_split(db, slices, kind, nullptr, s));

    const int tm = tile_rows(m), tn = tile_cols(n);
    const Tile* tiles = nullptr;
    DMP_CHECK(cached_tiles(tm, tn, false, &tiles));
    GemmParams p{};
    p.tiles = tiles;
    p.descs = nullptr;
    p.one.pa = g.pa;
    p.one.pb = g.pb;
    p.one.ea = g.ea;
    p.one.eb = g.eb;
    p.one.out = C;
    p.one.a_rb_stride = rb_stride;
    p.one.b_rb_stride = rb_stride;
    p.one.M = m;
    p.one.N = n;
    p.one.KC = KC;
    p.one.ldc = ldc;
    p.one.state_index = -1;
    p.mode = EPI_STORE;
    if (g.fix != nullptr) {
        p.fix = g.fix;
        p.nfull = g.tail.nfull;
        p.nsplit = g.tail.nsplit;
    }
    return launch_ozgemm(slices, kind, p, tm * tn, s);
}

// ---------------------------------------------------------------------------
// Grouped GEMM: every phase is one launch over all products.

size_t dmp_gemm_batched_workspace_bytes(int count, const int* m, const int* n, const int* k,
                                        int slices, dmp_kind kind) {
    if (count < 0 || slices < 1 || slices > kMaxSlices) return 0;
    if (kind == DMP_MARKIDIS_FP16 && slices > kMaxTerms) return 0;
    if (count > 0 && (!m || !n || !k)) return 0;
    for (int b = 0; b < count; ++b)
        if (m[b] < 1 || n[b] < 1 || k[b] < 1) return 0;
    Carver c(nullptr);
    size_t tiles = 0;
    for (int b = 0; b < count; ++b) {
        if (kind != DMP_FP64_NATIVE) carve_gemm(c, m[b], n[b], k[b], slices, kind);
        tiles += size_t(tile_rows(m[b])) * size_t(tile_cols(n[b]));
    }
    c.take<SplitDesc>(2 * size_t(count));
    c.take<MatDesc>(count);
    c.take<Tile>(std::max<size_t>(1, tiles));
    return c.used();
}

int dmp_ozaki_gemm_batched(int count, const int* m, const int* n, const int* k,
                           const double* const* A, const double* const* B, double* const* C,
                           int slices, dmp_kind kind, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    hipStream_t s = static_cast<hipStream_t>(stream);
    DMP_CHECK(check_kind_slices(kind, slices));
    if (count < 0 || (count > 0 && (!m || !n || !k || !A || !B || !C))) {
        set_error("bad batch arguments");
        return DMP_EINVAL;
    }
    for (int b = 0; b < count; ++b) {
        if (m[b] < 1 || n[b] < 1 || k[b] < 1 || !A[b] || !B[b] || !C[b]) {
            set_error("batch entry %d: sizes must be >= 1 and pointers non-null", b);
            return DMP_EINVAL;
        }
        if (kind != DMP_FP64_NATIVE && k[b] > max_k_for(slices, kind)) {
            set_error("batch entry %d: k too large for %d slices", b, slices);
            return DMP_EINVAL;
        }
    }
    if (count == 0) return DMP_OK;
    if (kind == DMP_FP64_NATIVE) {
        for (int b = 0; b < count; ++b)
            DMP_CHECK(native_dgemm(s, false, false, m[b], n[b], k[b], A[b], k[b], B[b], n[b], C[b], n[b]));
        return DMP_OK;
    }
    const size_t need = dmp_gemm_batched_workspace_bytes(count, m, n, k, slices, kind);
    if (ws == nullptr || ws_bytes < need) {
        set_error("workspace of %zu bytes required", need);
        return DMP_ENOMEM;
    }
    DMP_CHECK(check_workspace_alignment(ws));
    Carver c(ws);
    std::vector<GemmLayout> lay(count);
    for (int b = 0; b < count; ++b) lay[b] = carve_gemm(c, m[b], n[b], k[b], slices, kind);
    SplitDesc* sd_dev = c.take<SplitDesc>(2 * size_t(count));
    MatDesc* md_dev = c.take<MatDesc>(count);
    std::vector<SplitDesc> sa(count), sb(count);
    std::vector<MatDesc> md(count);
    std::vector<Tile> tiles;
    int ur_a = 0, ud_a = 0, ur_b = 0, ud_b = 0;
    for (int b = 0; b < count; ++b) {
        const int KC = int(chunks_of(k[b], kind));
        SplitDesc d{};
        d.A = A[b];
        d.lda = k[b];
        d.R = m[b];
        d.K = k[b];
        d.trans = 0;
        d.KC = KC;
        d.maxbits = lay[b].ma;
        d.expo = lay[b].ea;
        d.planes = lay[b].pa;
        d.state_index = -1;
        d.ub_rowmax = ur_a;
        d.ub_digits = ud_a;
        ur_a += split_units_rowmax(m[b]);
        ud_a += split_units_digits(m[b], KC);
        sa[b] = d;
        // B's operand rows are its columns: transpose the digit read by
        // splitting B^T, i.e. columns of the row-major k x n matrix.
        SplitDesc e = d;
        e.A = B[b];
        e.lda = n[b];
        e.R = n[b];
        e.trans = 1;
        e.maxbits = lay[b].mb;
        e.expo = lay[b].eb;
        e.planes = lay[b].pb;
        e.ub_rowmax = ur_b;
        e.ub_digits = ud_b;
        ur_b += 0;
        ud_b += split_units_digits(n[b], KC);
        sb[b] = e;
        MatDesc q{};
        q.pa = lay[b].pa;
        q.pb = lay[b].pb;
        q.ea = lay[b].ea;
        q.eb = lay[b].eb;
        q.out = C[b];
        q.a_rb_stride = int64_t(KC) * planes_of(slices, kind) * kFragBytes;
        q.b_rb_stride = q.a_rb_stride;
        q.M = m[b];
        q.N = n[b];
        q.KC = KC;
        q.ldc = n[b];
        q.state_index = -1;
        md[b] = q;
    }
    // tiles of the longest reductions first (dispatched in that order)
    std::vector<int> order(count);
    for (int b = 0; b < count; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return k[x] > k[y]; });
    for (int b : order) append_tiles(tiles, tile_rows(m[b]), tile_cols(n[b]), false, uint32_t(b));
    Tile* t_dev = c.take<Tile>(tiles.size());
    // the host vectors must outlive the asynchronous copies (the stream is
    // drained before any error return); the launches below stay asynchronous
    hipError_t e = hipMemcpyAsync(sd_dev, sa.data(), count * sizeof(SplitDesc), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(md_dev, md.data(), count * sizeof(MatDesc), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(t_dev, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice, s);
    const hipError_t e_sync = hipStreamSynchronize(s);
    DMP_CHECK_HIP(e);
    DMP_CHECK_HIP(e_sync);
    // A: one grouped row split; B: column splits (per product, small count)
    DMP_CHECK(launch_split_grouped_rowmax(sd_dev, count, ur_a, nullptr, s));
    DMP_CHECK(launch_split_grouped_digits(sd_dev, count, ud_a, slices, kind, nullptr, s));
    for (int b = 0; b < count; ++b) {
        SplitDesc e = sb[b];
        DMP_CHECK(launch_split(e, slices, kind, nullptr, s));
    }
    GemmParams p{};
    p.tiles = t_dev;
    p.descs = md_dev;
    p.mode = EPI_STORE;
    p.spread = count > 1 ? 1 : 0;
    DMP_CHECK(launch_ozgemm(slices, kind, p, int(tiles.size()), s));
    return DMP_OK;
}

}  // extern "C"
