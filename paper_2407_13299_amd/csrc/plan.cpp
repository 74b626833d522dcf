// Host-side planning of libdmp (pure C++, see plan.hpp).
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "tuned_table.h"
#include "tuned_tiles.h"

namespace dmp {

// ---- error text -------------------------------------------------------------

static thread_local char g_error[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_error, sizeof(g_error), fmt, ap);
    va_end(ap);
}

void clear_error() { g_error[0] = '\0'; }

const char* error_text() { return g_error; }

// ---- argument checks ----------------------------------------------------------

int check_kind_slices(dmp_kind kind, int slices) {
    if (kind != DMP_OZ_INT8 && kind != DMP_OZ_FP16 && kind != DMP_FP64_NATIVE &&
        kind != DMP_MARKIDIS_FP16) {
        set_error("unknown kind %d", int(kind));
        return DMP_EINVAL;
    }
    if (kind == DMP_MARKIDIS_FP16 && (slices < 1 || slices > kMaxTerms)) {
        set_error("terms must lie in [1, %d], got %d", kMaxTerms, slices);
        return DMP_EINVAL;
    }
    if (kind != DMP_FP64_NATIVE && kind != DMP_MARKIDIS_FP16 && (slices < 1 || slices > kMaxSlices)) {
        set_error("slices must lie in [1, %d], got %d", kMaxSlices, slices);
        return DMP_EINVAL;
    }
    return DMP_OK;
}

int check_workspace_alignment(const void* ws) {
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) {
        set_error("workspace %p is not 256-byte aligned", ws);
        return DMP_EINVAL;
    }
    return DMP_OK;
}

int check_method_flags(int method, int flags) {
    if (method != DMP_CANONICAL && method != DMP_TRS4) {
        set_error("unknown method %d", method);
        return DMP_EINVAL;
    }
    if ((flags & ~(DMP_REFINE_MCWEENY | DMP_NATIVE_TRIANGLE)) != 0) {
        set_error("unknown flags 0x%x", flags);
        return DMP_EINVAL;
    }
    return DMP_OK;
}

int validate_purify_args(const double* H, int n, int nocc, double tol, int max_iter, const double* P) {
    if (n < 1 || nocc < 0 || nocc > n) {
        set_error("need n >= 1 and 0 <= nocc <= n (n=%d, nocc=%d)", n, nocc);
        return DMP_EINVAL;
    }
    if (!(tol > 0.0) || max_iter < 1) {
        set_error("need tol > 0 and max_iter >= 1");
        return DMP_EINVAL;
    }
    if (!H || !P || H == P) {
        set_error("H and P must be distinct non-null device pointers");
        return DMP_EINVAL;
    }
    if (n > 65535 * kTileN) {
        set_error("n too large");
        return DMP_EINVAL;
    }
    return DMP_OK;
}

// ---- tile orders ----------------------------------------------------------------

static bool tile_in_upper(int i, int j, int TM) { return kTileN * j + kTileN - 1 >= TM * i; }

void append_tiles(std::vector<Tile>& out, int tm, int tn, bool upper, uint32_t mat, int TM) {
    // super-tiles of GI x GJ tiles = 512 x 512 elements
    const int GI = 512 / TM, GJ = 512 / kTileN;
    const int sm = (tm + GI - 1) / GI, sn = (tn + GJ - 1) / GJ;
    for (int si = 0; si < sm; ++si)
        for (int sj = 0; sj < sn; ++sj)
            for (int i = si * GI; i < std::min(tm, si * GI + GI); ++i)
                for (int j = sj * GJ; j < std::min(tn, sj * GJ + GJ); ++j) {
                    if (upper && !tile_in_upper(i, j, TM)) continue;
                    out.push_back(Tile{uint16_t(i), uint16_t(j), mat});
                }
}

int tile_rows(int m, int TM) { return int(round_up(m, TM) / TM); }
int tile_cols(int n) { return int(round_up(n, kTileN) / kTileN); }

int upper_tile_count(int n, int TM) {
    const int tm = tile_rows(n, TM), tn = tile_cols(n);
    int c = 0;
    for (int i = 0; i < tm; ++i)
        for (int j = 0; j < tn; ++j) c += tile_in_upper(i, j, TM) ? 1 : 0;
    return c;
}

int split_units_rowmax(int R) { return int(round_up(R, kPad)) / 4; }
int split_units_colmax(int R, int K) { return ((R + 63) / 64) * ((K + 255) / 256); }
int split_units_digits(int R, int KC) { return int(round_up(R, kPad)) / kFragRows * ((KC + 3) / 4); }

int64_t chunks_of(int k, dmp_kind kind) { return round_up(k, kKPad) / chunk_k(kind); }

// ---- split tail -------------------------------------------------------------------

static int split_parts_max(int min_kc) { return std::min(kMaxSplit, min_kc / kMinSplitChunks); }

TailSplit plan_tail_split(int ntiles, int slots, int min_kc, int max_pieces) {
    TailSplit t{ntiles, 1};
    // with no full round the fixup launch costs more than the parts save
    if (ntiles <= slots || slots <= 0) return t;
    const int r = ntiles % slots;
    if (r == 0) return t;
    const int parts = std::min({split_parts_max(min_kc), slots / r, max_pieces / r});
    if (parts < 2) return t;
    t.nfull = ntiles - r;
    t.nsplit = parts;
    return t;
}

int tail_split_capacity(int ntiles, int min_kc, int rb) {
    const int parts = split_parts_max(min_kc);
    if (parts < 2 || ntiles <= 0) return 0;
    // 128-row tiles: one workgroup per CU, so half the parts run at once
    const int cap = rb == 4 ? kMaxPieces / 2 : kMaxPieces;
    return int(std::min<int64_t>(cap, int64_t(ntiles) * parts));
}

// ---- tuned choices ------------------------------------------------------------------

int autotune_slices_model(int n, double target, dmp_kind kind) {
    if (kind == DMP_FP64_NATIVE) return 0;
    if (kind == DMP_MARKIDIS_FP16) return kMaxTerms;   // no term count reaches FP64 level
    if (n < 1 || !(target > 0.0)) return kMaxSlices;
    // error model max|dP| ~ C n^a 2^-(8S - 1), with (C, a) measured per kind
    const double c = kind == DMP_OZ_FP16 ? kTunedErrC[1] : kTunedErrC[0];
    const double a = kind == DMP_OZ_FP16 ? kTunedErrA[1] : kTunedErrA[0];
    for (int s = 1; s <= kMaxSlices; ++s) {
        const double err = c * std::pow(double(n), a) * std::ldexp(1.0, -(8 * s - 1));
        if (err <= target && n <= max_k_for_slices(s)) return s;
    }
    return kMaxSlices;
}

// slices > 0: that count for every matrix.  Otherwise the tuned count per
// matrix; matrices that need fewer slices than the batch maximum then run
// with the maximum (a larger S is always at least as accurate) when they
// carry under a quarter of the batch's n^3 work, so that the batch runs as
// one group of launches instead of one group per slice count.
void batch_slices(int count, const int* n, int slices, dmp_kind kind, std::vector<int>& s) {
    s.assign(size_t(std::max(count, 0)), 0);
    if (kind == DMP_FP64_NATIVE) return;
    int smax = 0;
    for (int b = 0; b < count; ++b) {
        s[b] = slices > 0 ? slices : autotune_slices_model(n[b], kTunedTarget, kind);
        smax = std::max(smax, s[b]);
    }
    if (slices > 0 || count < 2) return;
    double low = 0.0, all = 0.0;
    for (int b = 0; b < count; ++b) {
        const double w = double(n[b]) * n[b] * n[b];
        all += w;
        if (s[b] < smax) low += w;
    }
    if (low >= 0.25 * all) return;
    for (int b = 0; b < count; ++b)
        if (n[b] <= max_k_for(smax, kind)) s[b] = smax;
}

TileChoice tile_choice(dmp_kind kind, int S, int n, int forced_rb) {
    // 64-row tiles exist for the Ozaki kinds up to kMaxSlices64 (beyond that
    // two workgroups no longer fit a CU without spills)
    const bool has64 = (kind == DMP_OZ_INT8 || kind == DMP_OZ_FP16) && S >= 1 && S <= kMaxSlices64;
    TileChoice c{4, true};
    for (const TileRule& r : kTileTable) {
        if (r.kind == int(kind) && S >= r.s_lo && S <= r.s_hi && n >= r.n_lo && n <= r.n_hi) {
            c.rb = r.rb;
            c.split_tail = r.split_tail != 0;
            break;
        }
    }
    if (forced_rb == 2 || forced_rb == 4) c.rb = forced_rb;
    if (!has64) c.rb = 4;
    return c;
}

// ---- purification groups ----------------------------------------------------------------

int native_blocks(int n) { return int(std::min<int64_t>(2048, (int64_t(n) * n + 255) / 256)); }
int native_pairs(int n) {
    const int t = (n + 31) / 32;
    return t * (t + 1) / 2;
}
int oz_tiles(int n, int rb) { return upper_tile_count(n, 32 * rb); }

void plan_groups(int count, const int* n, const int* slices, dmp_kind kind, int method,
                 int forced_rb, std::vector<GroupPlan>& groups) {
    groups.clear();
    for (int b = 0; b < count; ++b) {
        const int S = kind == DMP_FP64_NATIVE ? 0 : slices[b];
        const TileChoice tc = kind == DMP_FP64_NATIVE ? TileChoice{4, false}
                                                      : tile_choice(kind, S, n[b], forced_rb);
        GroupPlan* g = nullptr;
        for (auto& x : groups)
            if (x.S == S && x.rb == tc.rb && x.split_tail == tc.split_tail &&
                kind != DMP_FP64_NATIVE)
                g = &x;
        if (!g) {
            groups.emplace_back();
            g = &groups.back();
            g->S = S;
            g->kind = kind;
            g->method = method;
            g->rb = tc.rb;
            g->split_tail = tc.split_tail;
        }
        g->idx.push_back(b);
        g->count++;
    }
}

static MatLayout carve_matrix(Carver& c, int n, int S, dmp_kind kind) {
    MatLayout m{};
    const size_t nn = size_t(n) * n;
    m.X2 = c.take<double>(nn);
    m.Pw = c.take<double>(nn);
    if (kind == DMP_FP64_NATIVE) {
        m.X3 = c.take<double>(nn);
        m.T = c.take<double>(nn);
    } else {
        m.planesP = c.take<uint8_t>(plane_bytes(n, n, S, kind));
        m.planesX = c.take<uint8_t>(plane_bytes(n, n, S, kind));
        m.expP = c.take<int>(round_up(n, kPad));
        m.expX = c.take<int>(round_up(n, kPad));
        m.maxP = c.take<uint64_t>(round_up(n, kPad));
        m.maxX = c.take<uint64_t>(round_up(n, kPad));
    }
    m.rows = c.take<double>(3 * size_t(n));
    m.rowbad = c.take<int>(n);
    m.e0 = c.take<double>(kE0Blocks);
    return m;
}

size_t carve_group(Carver& c, GroupPlan& g, const int* n) {
    size_t parts = 0;
    g.lay.resize(g.count);
    g.max_pairs = 1;
    g.min_kc = g.max_kc = 0;
    for (int b = 0; b < g.count; ++b) {
        const int nb = n[g.idx[b]];
        g.lay[b] = carve_matrix(c, nb, g.S, g.kind);
        if (g.kind == DMP_FP64_NATIVE) {
            parts = std::max<size_t>(parts, std::max(native_blocks(nb), native_pairs(nb)));
        } else {
            parts += size_t(oz_tiles(nb, g.rb));
            const int kc = int(chunks_of(nb, g.kind));
            g.min_kc = b == 0 ? kc : std::min(g.min_kc, kc);
            g.max_kc = std::max(g.max_kc, kc);
        }
        g.max_pairs = std::max(g.max_pairs, native_pairs(nb));
    }
    // part buffer of the tail split (Ozaki kinds), sized for the largest
    // matrix, so that a batch needs no less workspace than any of its members
    g.fix_pieces = (g.kind == DMP_OZ_INT8 || g.kind == DMP_OZ_FP16) && g.split_tail
                       ? tail_split_capacity(int(parts), g.max_kc, g.rb) : 0;
    g.fix = g.fix_pieces > 0 ? c.take<int>(size_t(g.fix_pieces) * piece_ints(g.S, g.rb)) : nullptr;
    // the refinement step reuses the partials of one matrix's tile pairs
    parts = std::max<size_t>(parts, size_t(g.max_pairs));
    g.pd = c.take<PurDesc>(g.count);
    g.st = c.take<DevState>(g.count);
    g.splitP[0] = c.take<SplitDesc>(g.count);
    g.splitP[1] = c.take<SplitDesc>(g.count);
    g.splitX = c.take<SplitDesc>(g.count);
    g.splitT[0] = c.take<SplitDesc>(g.count);
    g.splitT[1] = c.take<SplitDesc>(g.count);
    g.sq[0] = c.take<MatDesc>(g.count);
    g.sq[1] = c.take<MatDesc>(g.count);
    g.up[0] = c.take<MatDesc>(g.count);
    g.up[1] = c.take<MatDesc>(g.count);
    g.tiles = c.take<Tile>(std::max<size_t>(1, g.kind == DMP_FP64_NATIVE ? 1 : parts));
    g.partials = c.take<double>(std::max<size_t>(1, parts) * kPartials);
    g.pairs = c.take<IPair>(g.max_pairs);
    return c.used();
}

void build_group(GroupPlan& g, const double* const* H, double* const* P, const int* n,
                 const int* nocc, int slots, GroupHost& out) {
    const int cnt = g.count;
    out = GroupHost{};
    out.pd.resize(cnt);
    int urow = 0, udig = 0;
    g.max_n = 0;
    // tile list: matrices from the largest to the smallest (each matrix's
    // tiles contiguous, so its partials form one range)
    std::vector<int> order(cnt);
    for (int b = 0; b < cnt; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return n[g.idx[x]] > n[g.idx[y]]; });
    std::vector<int> part_begin(cnt, 0), part_end(cnt, 0);
    if (g.kind != DMP_FP64_NATIVE) {
        out.sp0.resize(cnt);
        out.sp1.resize(cnt);
        out.sx.resize(cnt);
        out.st0.resize(cnt);
        out.st1.resize(cnt);
        out.q0.resize(cnt);
        out.q1.resize(cnt);
        out.u0.resize(cnt);
        out.u1.resize(cnt);
        int pbeg = 0;
        for (int b : order) {
            const int nb = n[g.idx[b]];
            part_begin[b] = pbeg;
            pbeg += oz_tiles(nb, g.rb);
            part_end[b] = pbeg;
            append_tiles(out.tiles, tile_rows(nb, 32 * g.rb), tile_cols(nb), true, uint32_t(b),
                         32 * g.rb);
        }
    }
    for (int b = 0; b < cnt; ++b) {
        const int m = g.idx[b], nb = n[m];
        const MatLayout& L = g.lay[b];
        g.max_n = std::max(g.max_n, nb);
        PurDesc d{};
        d.H = H[m];
        d.Pb[0] = P[m];
        d.Pb[1] = L.Pw;
        d.X2 = L.X2;
        d.X3 = L.X3;
        d.T = L.T;
        d.method = g.method;
        d.rows = L.rows;
        d.rowbad = L.rowbad;
        d.e0 = L.e0;
        d.partials = g.partials;
        d.n = nb;
        d.nocc = nocc[m];
        if (g.kind == DMP_FP64_NATIVE) {
            d.part_begin = 0;
            d.part_end = 0;   // set per phase by the native driver
        } else {
            d.part_begin = part_begin[b];
            d.part_end = part_end[b];
        }
        out.pd[b] = d;
        if (g.kind == DMP_FP64_NATIVE) continue;
        const int KC = int(chunks_of(nb, g.kind));
        const int64_t rbs = int64_t(KC) * planes_of(g.S, g.kind) * kFragBytes;
        SplitDesc sd{};
        sd.lda = nb;
        sd.R = nb;
        sd.K = nb;
        sd.trans = 0;
        sd.KC = KC;
        sd.ub_rowmax = urow;
        sd.ub_digits = udig;
        sd.state_index = b;
        urow += split_units_rowmax(nb);
        udig += split_units_digits(nb, KC);
        // Row maxima: those of P come from the update's epilogue (of P0 from
        // k_rowmax), those of X2 from the square's; each array is zeroed by
        // the split that runs just before its producer.
        // canonical purification keeps its iterates and X2 as upper triangles
        // (upper_only products), so their splits read them as symmetric;
        // TRS4's combined operand needs full rows of both
        const int sym = g.method == DMP_CANONICAL ? 1 : 0;
        sd.A = P[m];
        sd.maxbits = L.maxP;
        sd.expo = L.expP;
        sd.planes = L.planesP;
        sd.clear = L.maxX;
        sd.sym = sym;
        out.sp0[b] = sd;
        sd.A = L.Pw;
        out.sp1[b] = sd;
        sd.sym = 0;
        // TRS4: T = ta P + tb X2 + tc I, split into P's planes (free once the
        // square has run); its row maxima (k_rowmax) go to X2's array, free
        // once X2 is split
        sd.A = P[m];
        sd.A2 = L.X2;
        sd.maxbits = L.maxX;
        sd.clear = nullptr;
        out.st0[b] = sd;
        sd.A = L.Pw;
        out.st1[b] = sd;
        sd.A2 = nullptr;
        sd.A = L.X2;
        sd.maxbits = L.maxX;
        sd.expo = L.expX;
        sd.planes = L.planesX;
        sd.clear = L.maxP;
        sd.sym = sym;
        out.sx[b] = sd;
        MatDesc md{};
        md.a_rb_stride = rbs;
        md.b_rb_stride = rbs;
        md.M = nb;
        md.N = nb;
        md.KC = KC;
        md.ldc = nb;
        md.state_index = b;
        md.H = H[m];
        md.X2 = L.X2;
        // square: A = B = planes of P
        md.pa = L.planesP;
        md.pb = L.planesP;
        md.ea = L.expP;
        md.eb = L.expP;
        md.out = L.X2;
        md.rowmax = L.maxX;
        md.P = P[m];
        out.q0[b] = md;
        md.P = L.Pw;
        out.q1[b] = md;
        // update: A = planes of X2, B = planes of P; P' into the other buffer
        md.pa = L.planesX;
        md.ea = L.expX;
        md.rowmax = L.maxP;
        md.P = P[m];
        md.out = L.Pw;
        out.u0[b] = md;
        md.P = L.Pw;
        md.out = P[m];
        out.u1[b] = md;
    }
    g.ntiles = int(out.tiles.size());
    g.tail = TailSplit{g.ntiles, 1};
    if (g.fix != nullptr && slots > 0)
        g.tail = plan_tail_split(g.ntiles, slots, g.min_kc, g.fix_pieces);
    g.units_rowmax = urow;
    g.units_digits = udig;
    const int t = (g.max_n + 31) / 32;
    for (int i = 0; i < t; ++i)
        for (int j = i; j < t; ++j) out.pairs.push_back(IPair{i, j});
}

std::vector<int64_t> launch_key(const std::vector<GroupPlan>& groups, int m, int device,
                                int extra) {
    std::vector<int64_t> k{int64_t(device), int64_t(m), int64_t(extra), int64_t(groups.size())};
    auto p = [&](const void* x) { k.push_back(int64_t(reinterpret_cast<uintptr_t>(x))); };
    for (const GroupPlan& g : groups) {
        k.insert(k.end(), {int64_t(g.count), int64_t(g.S), int64_t(g.kind), int64_t(g.method),
                           int64_t(g.rb), int64_t(g.ntiles), int64_t(g.units_rowmax),
                           int64_t(g.units_digits), int64_t(g.tail.nfull), int64_t(g.tail.nsplit)});
        p(g.pd);
        p(g.st);
        p(g.splitP[0]);
        p(g.splitP[1]);
        p(g.splitX);
        p(g.splitT[0]);
        p(g.splitT[1]);
        p(g.sq[0]);
        p(g.sq[1]);
        p(g.up[0]);
        p(g.up[1]);
        p(g.tiles);
        p(g.partials);
        p(g.fix);
    }
    return k;
}

std::mutex& purify_mutex() {
    static std::mutex mu;
    return mu;
}

}  // namespace dmp
