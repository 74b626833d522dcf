// Host-side planning of libdmp: tile orders, the split-tail plan, workspace
// carving, the grouping of a batch and the descriptors of every launch, and
// the caches the library keeps.  Pure C++17 (no HIP headers), so that this
// part also builds with a plain host compiler under the address, undefined
// behaviour and thread sanitizers (tests/host/).
#pragma once

#include <cstddef>
#include <cstdint>
#include <functional>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <utility>
#include <vector>

#include "layout.hpp"

namespace dmp {

// Carves 256-byte-aligned regions out of a workspace; with base == nullptr it
// only measures.
class Carver {
public:
    explicit Carver(void* base) : base_(static_cast<uint8_t*>(base)) {}
    template <typename T>
    T* take(size_t count) {
        off_ = (off_ + 255) & ~size_t(255);
        T* p = base_ ? reinterpret_cast<T*>(base_ + off_) : nullptr;
        off_ += count * sizeof(T);
        return p;
    }
    size_t used() const { return (off_ + 255) & ~size_t(255); }

private:
    uint8_t* base_;
    size_t off_ = 0;
};

// ---- argument checks ------------------------------------------------------
int check_kind_slices(dmp_kind kind, int slices);
int validate_purify_args(const double* H, int n, int nocc, double tol, int max_iter,
                         const double* P);
int check_method_flags(int method, int flags);
// The caller's workspace starts on a 256-byte boundary (the carved regions
// are 256-byte aligned relative to it, and kernels load 16-byte vectors).
int check_workspace_alignment(const void* ws);

// ---- tile orders ----------------------------------------------------------
// Order of the TM x 64 output tiles of one matrix (TM = 128, or 64 for the
// 64-row variant): 512 x 512 super-tiles, row-major over super-tiles and
// within each; ``upper`` keeps the tiles that reach the upper triangle
// (column >= row somewhere in the tile).
void append_tiles(std::vector<Tile>& out, int tm, int tn, bool upper, uint32_t mat,
                  int TM = kTileM);
int tile_rows(int m, int TM = kTileM);
int tile_cols(int n);
int upper_tile_count(int n, int TM = kTileM);

// Workgroups ("units") of the split kernels for an operand of R rows.
int split_units_rowmax(int R);
int split_units_colmax(int R, int K);
int split_units_digits(int R, int KC);
int64_t chunks_of(int k, dmp_kind kind);

// ---- split tail -----------------------------------------------------------
// Tail split of ``ntiles`` tiles of equal cost: tiles [0, nfull) whole, the
// rest in nsplit parts each (nsplit == 1: no split).
struct TailSplit {
    int nfull, nsplit;
};
// ``slots`` workgroups run at once, so the tiles run in full rounds and a
// last round of r = ntiles mod slots tiles that leaves the rest of the chip
// idle; when there is at least one full round, those r tiles are split into
// as many parts as fill it (at most kMaxSplit, at least kMinSplitChunks of
// the ``min_kc`` chunks each, at most ``max_pieces`` parts in all).
TailSplit plan_tail_split(int ntiles, int slots, int min_kc, int max_pieces);
// Parts of a tail split a group of ``ntiles`` tiles of height 32 rb may need
// (the size of its part buffer in pieces, 0 when no split can arise).
int tail_split_capacity(int ntiles, int min_kc, int rb);

// ---- tuned choices --------------------------------------------------------
// Smallest slice count whose error model (fitted to measurements) meets
// ``target`` for an n x n purification.
int autotune_slices_model(int n, double target, dmp_kind kind);
// Slice count per matrix of a batch (slices > 0: that count for all).
void batch_slices(int count, const int* n, int slices, dmp_kind kind, std::vector<int>& s);
// Tile choice of the products of an n x n Ozaki purification (and of its
// adjoint): 32-row blocks per tile (2: 64-row tiles, 4: 128-row tiles) and
// whether the last, partly filled round of tiles is split along the
// reduction.  A function of (kind, S, n) only, from the measured table;
// ``forced_rb`` (2 or 4, 0 for none) overrides the height where it exists.
struct TileChoice {
    int rb;
    bool split_tail;
};
TileChoice tile_choice(dmp_kind kind, int S, int n, int forced_rb = 0);

// ---- purification groups --------------------------------------------------
struct alignas(8) IPair {   // a 32 x 32 tile pair (I, J), I <= J; same layout as HIP's int2
    int x, y;
};

// Per-matrix regions of the workspace.
struct MatLayout {
    double* X2;
    double* X3;
    double* T;        // native TRS4
    double* Pw;       // workspace iterate (Pb[1])
    uint8_t* planesP;
    uint8_t* planesX;
    int* expP;
    int* expX;
    uint64_t* maxP;
    uint64_t* maxX;
    double* rows;
    int* rowbad;
    double* e0;
};

constexpr int kE0Blocks = 256;   // fixed grid of the P0 / energy pass

// Everything a group of matrices (same S, kind and tile height) needs on the
// device.
struct GroupPlan {
    int count = 0;
    int S = 0;
    dmp_kind kind = DMP_OZ_INT8;
    int method = DMP_CANONICAL;
    std::vector<int> idx;             // positions in the caller's arrays
    std::vector<MatLayout> lay;
    PurDesc* pd = nullptr;            // [count]
    DevState* st = nullptr;           // [count]
    SplitDesc* splitP[2] = {nullptr, nullptr};  // [count] each
    SplitDesc* splitX = nullptr;      // [count]
    SplitDesc* splitT[2] = {nullptr, nullptr};  // TRS4: T from P (parity) and X2
    MatDesc* sq[2] = {nullptr, nullptr};
    MatDesc* up[2] = {nullptr, nullptr};
    Tile* tiles = nullptr;
    double* partials = nullptr;
    int ntiles = 0, units_rowmax = 0, units_digits = 0, max_n = 0;
    IPair* pairs = nullptr;           // 32 x 32 tile pairs I <= J of the largest matrix
    int max_pairs = 0;
    int rb = 4;                       // 32-row blocks per slice-GEMM tile (4 or 2)
    bool split_tail = true;           // the tuned table's choice for this group
    int* fix = nullptr;               // part buffer of the tail split
    int fix_pieces = 0;               // its capacity in parts
    int min_kc = 0, max_kc = 0;       // fewest / most reduction chunks of a matrix
    TailSplit tail{0, 1};             // tail split of the slice GEMMs
};

int native_blocks(int n);
int native_pairs(int n);
int oz_tiles(int n, int rb);

// Partition a batch into groups of equal (S, tile choice); the choice
// follows from each matrix's own (kind, S, n), so a matrix gets the same
// tiles, hence bit-identical fixed-order sums, alone or in a batch.
void plan_groups(int count, const int* n, const int* slices, dmp_kind kind, int method,
                 int forced_rb, std::vector<GroupPlan>& groups);
// Carve the workspace regions of a group (base == nullptr: measure only).
size_t carve_group(Carver& c, GroupPlan& g, const int* n);

// Host copies of a group's descriptors, ready to upload.
struct GroupHost {
    std::vector<PurDesc> pd;
    std::vector<SplitDesc> sp0, sp1, sx, st0, st1;
    std::vector<MatDesc> q0, q1, u0, u1;
    std::vector<Tile> tiles;
    std::vector<IPair> pairs;
};
// Fill the descriptors of a carved group for the caller's matrices; sets
// the group's tile count, unit counts, largest size and tail plan
// (``slots``: workgroups of its slice GEMM resident at once, 0 for no tail
// split).
void build_group(GroupPlan& g, const double* const* H, double* const* P, const int* n,
                 const int* nocc, int slots, GroupHost& out);

// Key of a recorded sequence of launches: every launch argument of m
// iterations of the groups follows from these values (workspace addresses
// and sizes), so equal keys mean an identical launch sequence.
std::vector<int64_t> launch_key(const std::vector<GroupPlan>& groups, int m, int device,
                                int extra);

// ---- caches ---------------------------------------------------------------
// Thread-safe cache keyed by a vector of integers.  Holds at most
// ``capacity`` values (0: no limit); beyond that the least recently used is
// dropped.  Values are shared pointers: dropping one from the cache leaves
// it alive for a caller that still holds it, and its deleter runs when the
// last holder lets go.
template <class V>
class KeyedCache {
public:
    using Key = std::vector<int64_t>;
    using Ptr = std::shared_ptr<V>;

    explicit KeyedCache(size_t capacity = 0) : cap_(capacity) {}

    // The cached value of ``key``, or the one ``create()`` returns (stored
    // unless null).  ``create`` runs under the cache's lock, so a value is
    // created once even when threads ask for it together.
    template <class F>
    Ptr get_or_create(const Key& key, F&& create, bool* created = nullptr) {
        std::lock_guard<std::mutex> lock(mu_);
        if (created) *created = false;
        auto it = index_.find(key);
        if (it != index_.end()) {
            lru_.splice(lru_.begin(), lru_, it->second);
            return it->second->second;
        }
        Ptr v = create();
        if (!v) return v;
        if (created) *created = true;
        lru_.emplace_front(key, v);
        index_[key] = lru_.begin();
        while (cap_ > 0 && lru_.size() > cap_) {
            index_.erase(lru_.back().first);
            lru_.pop_back();
        }
        return v;
    }

    // Value of ``key`` or null; marks it as recently used.
    Ptr find(const Key& key) {
        std::lock_guard<std::mutex> lock(mu_);
        auto it = index_.find(key);
        if (it == index_.end()) return nullptr;
        lru_.splice(lru_.begin(), lru_, it->second);
        return it->second->second;
    }

    size_t size() const {
        std::lock_guard<std::mutex> lock(mu_);
        return lru_.size();
    }

    void clear() {
        std::lock_guard<std::mutex> lock(mu_);
        index_.clear();
        lru_.clear();
    }

private:
    mutable std::mutex mu_;
    size_t cap_;
    std::list<std::pair<Key, Ptr>> lru_;   // most recently used first
    std::map<Key, typename std::list<std::pair<Key, Ptr>>::iterator> index_;
};

// The one lock that serialises the purification entry points of a process
// (dmp_purify*, the batched and the taped variants and the backward pass).
std::mutex& purify_mutex();

}  // namespace dmp
