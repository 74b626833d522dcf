// Drives the host planning code of libdmp (plan.cpp: tile orders, the split
// tail plan, grouping and carving of batches, the descriptors of every
// launch, the keyed cache and the purification lock) from several threads
// at once.  Built by tests/test_host_sanitizers.py with the address and
// undefined-behaviour sanitizers and, separately, with the thread
// sanitizer; it needs no GPU (device pointers are only stored, never
// dereferenced, except the workspace, which here is host memory of exactly
// the carved size, so a region that overruns it is caught).
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include "plan.hpp"

using namespace dmp;

namespace {

std::atomic<int> g_failures{0};
std::atomic<long> g_live{0};   // values of the keyed cache alive right now

#define EXPECT(cond)                                                                      \
    do {                                                                                  \
        if (!(cond)) {                                                                    \
            std::fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, \
                         #cond);                                                         \
            g_failures++;                                                                 \
        }                                                                                 \
    } while (0)

struct Counted {
    int64_t key;
    explicit Counted(int64_t k) : key(k) { g_live++; }
    ~Counted() { g_live--; }
};

// Regions of one carved workspace, checked for overlap once all are known.
thread_local std::vector<std::pair<const uint8_t*, size_t>> t_regions;

// Write every byte of [p, p + bytes): out of the workspace, the address
// sanitizer stops the run.
void touch(void* p, size_t bytes, const uint8_t* base, size_t size) {
    if (bytes == 0) return;
    EXPECT(p != nullptr);
    const uint8_t* q = static_cast<const uint8_t*>(p);
    EXPECT(q >= base && q + bytes <= base + size);
    std::memset(p, 0x5a, bytes);
    t_regions.emplace_back(q, bytes);
}

// No two regions of the workspace overlap (a region carved too small would
// overlap the next one while staying inside the allocation).
void check_disjoint() {
    auto& r = t_regions;
    std::sort(r.begin(), r.end());
    for (size_t i = 1; i < r.size(); ++i) EXPECT(r[i - 1].first + r[i - 1].second <= r[i].first);
    r.clear();
}

void check_group(const GroupPlan& g, const GroupHost& h, const int* n, const uint8_t* base,
                 size_t size) {
    for (int b = 0; b < g.count; ++b) {
        const MatLayout& L = g.lay[b];
        const int nb = n[g.idx[b]];
        const size_t nn = size_t(nb) * nb;
        touch(L.X2, nn * sizeof(double), base, size);
        touch(L.Pw, nn * sizeof(double), base, size);
        if (g.kind == DMP_FP64_NATIVE) {
            touch(L.X3, nn * sizeof(double), base, size);
            touch(L.T, nn * sizeof(double), base, size);
        } else {
            touch(L.planesP, plane_bytes(nb, nb, g.S, g.kind), base, size);
            touch(L.planesX, plane_bytes(nb, nb, g.S, g.kind), base, size);
            touch(L.expP, size_t(round_up(nb, kPad)) * sizeof(int), base, size);
            touch(L.expX, size_t(round_up(nb, kPad)) * sizeof(int), base, size);
            touch(L.maxP, size_t(round_up(nb, kPad)) * sizeof(uint64_t), base, size);
            touch(L.maxX, size_t(round_up(nb, kPad)) * sizeof(uint64_t), base, size);
        }
        touch(L.rows, 3 * size_t(nb) * sizeof(double), base, size);
        touch(L.rowbad, size_t(nb) * sizeof(int), base, size);
        touch(L.e0, kE0Blocks * sizeof(double), base, size);
    }
    const size_t cnt = size_t(g.count);
    touch(g.pd, cnt * sizeof(PurDesc), base, size);
    touch(g.st, cnt * sizeof(DevState), base, size);
    for (int i = 0; i < 2; ++i) {
        touch(g.splitP[i], cnt * sizeof(SplitDesc), base, size);
        touch(g.splitT[i], cnt * sizeof(SplitDesc), base, size);
        touch(g.sq[i], cnt * sizeof(MatDesc), base, size);
        touch(g.up[i], cnt * sizeof(MatDesc), base, size);
    }
    touch(g.splitX, cnt * sizeof(SplitDesc), base, size);
    touch(g.pairs, h.pairs.size() * sizeof(IPair), base, size);
    if (g.kind != DMP_FP64_NATIVE) {
        // the tile list, its partials and the part buffer of the tail plan
        touch(g.tiles, h.tiles.size() * sizeof(Tile), base, size);
        touch(g.partials, h.tiles.size() * kPartials * sizeof(double), base, size);
        EXPECT(g.ntiles == int(h.tiles.size()));
        int total = 0;
        for (int b = 0; b < g.count; ++b) total += oz_tiles(n[g.idx[b]], g.rb);
        EXPECT(total == g.ntiles);
        // every tile lies inside its matrix, and each matrix's tiles are one
        // contiguous range equal to its partial range
        for (int t = 0; t < g.ntiles; ++t) {
            const Tile& tl = h.tiles[t];
            EXPECT(int(tl.mat) < g.count);
            const PurDesc& d = h.pd[tl.mat];
            EXPECT(t >= d.part_begin && t < d.part_end);
            EXPECT(int(tl.I) * 32 * g.rb < d.n && int(tl.J) * kTileN < d.n);
        }
        if (g.tail.nsplit > 1) {
            EXPECT(g.fix != nullptr);
            const int tail = g.ntiles - g.tail.nfull;
            EXPECT(tail >= 1 && tail * g.tail.nsplit <= g.fix_pieces);
            touch(g.fix, size_t(tail) * g.tail.nsplit * piece_ints(g.S, g.rb) * sizeof(int), base, size);
        } else {
            EXPECT(g.tail.nfull == g.ntiles);
        }
        int ur = 0, ud = 0;
        for (int b = 0; b < g.count; ++b) {
            EXPECT(h.sp0[b].ub_rowmax == ur && h.sp0[b].ub_digits == ud);
            ur += split_units_rowmax(h.sp0[b].R);
            ud += split_units_digits(h.sp0[b].R, h.sp0[b].KC);
        }
        EXPECT(ur == g.units_rowmax && ud == g.units_digits);
    }
}

void plan_once(std::mt19937& rng) {
    std::uniform_int_distribution<int> cnt_d(1, 6), n_d(1, 700), kind_d(0, 2), s_d(1, 12),
        meth_d(0, 1), rb_d(0, 2);
    const int count = cnt_d(rng);
    const int kd = kind_d(rng), rd = rb_d(rng);
    const dmp_kind kind = kd == 0 ? DMP_FP64_NATIVE : kd == 1 ? DMP_OZ_INT8 : DMP_OZ_FP16;
    const int method = meth_d(rng);
    const int forced = rd == 0 ? 0 : rd == 1 ? 2 : 4;
    std::vector<int> n(count), nocc(count), slices(count);
    for (int b = 0; b < count; ++b) {
        n[b] = n_d(rng);
        nocc[b] = n[b] / 2;
        slices[b] = s_d(rng);
        EXPECT(check_kind_slices(kind, slices[b]) == DMP_OK);
    }
    std::vector<int> s_batch;
    batch_slices(count, n.data(), 0, kind, s_batch);
    EXPECT(int(s_batch.size()) == count);
    std::vector<GroupPlan> groups;
    plan_groups(count, n.data(), slices.data(), kind, method, forced, groups);
    int seen = 0;
    for (auto& g : groups) seen += g.count;
    EXPECT(seen == count);
    Carver measure(nullptr);
    for (auto& g : groups) carve_group(measure, g, n.data());
    const size_t size = measure.used();
    uint8_t* base = static_cast<uint8_t*>(std::aligned_alloc(256, size));
    Carver c(base);
    for (auto& g : groups) carve_group(c, g, n.data());
    EXPECT(c.used() == size);
    // fake matrix pointers (stored in descriptors, never dereferenced)
    std::vector<double> dummy(2 * size_t(count));
    std::vector<const double*> H(count);
    std::vector<double*> P(count);
    for (int b = 0; b < count; ++b) {
        H[b] = &dummy[2 * b];
        P[b] = &dummy[2 * b + 1];
    }
    std::uniform_int_distribution<int> slots_d(0, 1024);
    for (auto& g : groups) {
        GroupHost h;
        build_group(g, H.data(), P.data(), n.data(), nocc.data(), slots_d(rng), h);
        check_group(g, h, n.data(), base, size);
    }
    check_disjoint();
    const auto key = launch_key(groups, 4, 0, 0);
    EXPECT(key == launch_key(groups, 4, 0, 0) && key != launch_key(groups, 2, 0, 0));
    std::free(base);
}

void tail_plans(std::mt19937& rng) {
    std::uniform_int_distribution<int> t_d(0, 20000), s_d(0, 1024), kc_d(0, 300), p_d(0, 600);
    for (int i = 0; i < 200; ++i) {
        const int nt = t_d(rng), slots = s_d(rng), kc = kc_d(rng), mp = p_d(rng);
        const TailSplit t = plan_tail_split(nt, slots, kc, mp);
        if (t.nsplit == 1) {
            EXPECT(t.nfull == nt);
        } else {
            const int tail = nt - t.nfull;
            EXPECT(t.nsplit >= 2 && t.nsplit <= kMaxSplit && tail >= 1);
            EXPECT(tail * t.nsplit <= mp && tail * t.nsplit <= slots);
            EXPECT(t.nfull % slots == 0 && kc / t.nsplit >= kMinSplitChunks);
        }
    }
    std::uniform_int_distribution<int> n_d(1, 3000);
    for (int i = 0; i < 20; ++i) {
        const int n = n_d(rng);
        for (int TM : {64, 128}) {
            std::vector<Tile> up, full;
            append_tiles(up, tile_rows(n, TM), tile_cols(n), true, 0, TM);
            append_tiles(full, tile_rows(n, TM), tile_cols(n), false, 0, TM);
            EXPECT(int(up.size()) == upper_tile_count(n, TM));
            EXPECT(int(full.size()) == tile_rows(n, TM) * tile_cols(n));
        }
    }
}

void worker(int id, int rounds, KeyedCache<Counted>* cache, long* guarded) {
    std::mt19937 rng(1234 + id);
    std::uniform_int_distribution<int> key_d(0, 9);
    for (int r = 0; r < rounds; ++r) {
        plan_once(rng);
        tail_plans(rng);
        // the shared cache: values are created once per key while cached and
        // stay alive while held, also when evicted meanwhile
        const int64_t k = key_d(rng);
        auto v = cache->get_or_create({k, 7}, [&]() { return std::make_shared<Counted>(k); });
        EXPECT(v && v->key == k);
        auto w = cache->find({k, 7});
        EXPECT(!w || w->key == k);
        // the purification lock guards this counter
        {
            std::lock_guard<std::mutex> lock(purify_mutex());
            ++*guarded;
        }
        set_error("thread %d round %d", id, r);
        char want[64];
        std::snprintf(want, sizeof(want), "thread %d round %d", id, r);
        EXPECT(std::strcmp(error_text(), want) == 0);
    }
}

}  // namespace

int main(int argc, char** argv) {
    const int threads = argc > 1 ? std::atoi(argv[1]) : 8;
    const int rounds = argc > 2 ? std::atoi(argv[2]) : 40;
    long guarded = 0;
    {
        KeyedCache<Counted> cache(4);
        std::vector<std::thread> th;
        for (int i = 0; i < threads; ++i) th.emplace_back(worker, i, rounds, &cache, &guarded);
        for (auto& t : th) t.join();
        EXPECT(cache.size() <= 4);
        cache.clear();
    }
    EXPECT(g_live.load() == 0);
    EXPECT(guarded == long(threads) * rounds);
    if (g_failures.load() != 0) {
        std::fprintf(stderr, "%d expectation(s) failed\n", g_failures.load());
        return 1;
    }
    std::printf("host planning ok: %d threads x %d rounds\n", threads, rounds);
    return 0;
}
