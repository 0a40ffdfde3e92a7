// Host-side checks of input validation and plan preparation (csrc/host_prep.cpp), built with
// g++ and AddressSanitizer + UndefinedBehaviorSanitizer by test_host_sanitize_cpu.py.  No
// device code runs.  Every product of the preparation is compared with an independent
// computation from the original parent array: counts below every node by walking up from
// each tip (the definition), against the level schedule, the depth-first tip ranges and the
// tail program of the propagation.  Malformed inputs must come back with their status code.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <numeric>
#include <vector>

#include "uf_internal.h"

using namespace ufmi;

namespace {

int g_failures = 0;

void check(bool ok, const char *what, long long a = 0, long long b = 0)
{
    if (!ok) {
        std::fprintf(stderr, "FAIL: %s (%lld, %lld)\n", what, a, b);
        ++g_failures;
    }
}

// splitmix64
struct Rng {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    int32_t below(int32_t n) { return (int32_t)(next() % (uint64_t)n); }
    double unit() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

struct Input {
    std::vector<int32_t> parent;
    std::vector<double> length;
    std::vector<int64_t> indptr;
    std::vector<int32_t> indices, counts, feature_node;
    int32_t n_samples = 0, n_features = 0;
    uf_tree tree() const { return uf_tree{(int32_t)parent.size(), parent.data(), length.data()}; }
    uf_table table() const
    {
        return uf_table{n_samples, n_features, indptr.data(), indices.data(), counts.data(),
                        feature_node.empty() ? nullptr : feature_node.data()};
    }
};

// A random rooted tree on N nodes in shuffled id order (each new node hangs below a random
// earlier one, so degrees vary), a feature on every leaf in shuffled order, and a table of n
// samples with duplicate entries and some zero counts.
Input random_input(Rng &r, int32_t N, int32_t n)
{
    Input in;
    std::vector<int32_t> par(N, -1);
    for (int32_t v = 1; v < N; ++v) par[v] = r.below(v);
    std::vector<int32_t> perm(N);
    std::iota(perm.begin(), perm.end(), 0);
    for (int32_t i = N - 1; i > 0; --i) std::swap(perm[i], perm[r.below(i + 1)]);
    in.parent.assign(N, -1);
    in.length.assign(N, 0.0);
    for (int32_t v = 0; v < N; ++v) {
        in.parent[perm[v]] = par[v] < 0 ? -1 : perm[par[v]];
        in.length[perm[v]] = r.below(4) == 0 ? 0.0 : r.unit();
    }
    std::vector<char> internal(N, 0);
    for (int32_t v = 0; v < N; ++v)
        if (in.parent[v] >= 0) internal[in.parent[v]] = 1;
    for (int32_t v = 0; v < N; ++v)
        if (!internal[v]) in.feature_node.push_back(v);
    for (int32_t i = (int32_t)in.feature_node.size() - 1; i > 0; --i)
        std::swap(in.feature_node[i], in.feature_node[r.below(i + 1)]);
    in.n_features = (int32_t)in.feature_node.size();
    in.n_samples = n;
    in.indptr.push_back(0);
    for (int32_t k = 0; k < n; ++k) {
        const int32_t m = 1 + r.below(12);
        for (int32_t e = 0; e < m; ++e) {
            in.indices.push_back(r.below(in.n_features));
            in.counts.push_back(e == 0 ? 1 + r.below(50) : r.below(50));
        }
        in.indptr.push_back((int64_t)in.indices.size());
    }
    return in;
}

// counts[v][k] by walking up from every entry's tip (the definition)
std::vector<int64_t> walk_up_counts(const Input &in)
{
    const int32_t N = (int32_t)in.parent.size(), n = in.n_samples;
    std::vector<int64_t> C((size_t)N * n, 0);
    for (int32_t k = 0; k < n; ++k)
        for (int64_t e = in.indptr[k]; e < in.indptr[k + 1]; ++e)
            for (int32_t v = in.feature_node[in.indices[e]]; v >= 0; v = in.parent[v])
                C[(size_t)v * n + k] += in.counts[e];
    return C;
}

void check_prepared(const Input &in, const HostPrep &hp)
{
    const int32_t N = (int32_t)in.parent.size(), n = in.n_samples;
    check(hp.n_nodes == N && hp.n_samples == n, "sizes");
    // slots: a permutation, leaves first, root last
    std::vector<int32_t> seen(N, 0);
    for (int32_t v = 0; v < N; ++v) {
        const int32_t s = hp.slot_of_node[v];
        check(s >= 0 && s < N, "slot range", v, s);
        if (s >= 0 && s < N) {
            ++seen[s];
            check(hp.node_of_slot[s] == v, "slot inverse", v, s);
        }
    }
    for (int32_t s = 0; s < N; ++s) check(seen[s] == 1, "slot permutation", s);
    check(hp.slot_of_node[hp.root] == N - 1, "root slot");
    // branch lengths per slot
    for (int32_t v = 0; v < N; ++v) {
        const double want = in.parent[v] < 0 ? 0.0 : in.length[v];
        check(hp.length_slot[hp.slot_of_node[v]] == want, "slot length", v);
    }
    // levels by height: slots of level h in [level_ptr[h], level_ptr[h+1]), the leaves at
    // level 0, children in earlier levels than their parent
    check(hp.level_ptr.size() == (size_t)hp.n_levels + 1, "level_ptr size");
    check(hp.level_ptr[0] == 0 && hp.level_ptr[1] == hp.n_leaf && hp.level_ptr[hp.n_levels] == N,
          "level bounds");
    std::vector<int32_t> level(N, -1);
    for (int32_t h = 0; h < hp.n_levels; ++h)
        for (int32_t s = hp.level_ptr[h]; s < hp.level_ptr[h + 1]; ++s) level[s] = h;
    std::vector<int32_t> n_kids(N, 0);
    for (int32_t v = 0; v < N; ++v)
        if (in.parent[v] >= 0) ++n_kids[in.parent[v]];
    for (int32_t s = hp.n_leaf; s < N; ++s) {
        const int32_t i = s - hp.n_leaf;
        check(hp.child_ptr[i + 1] - hp.child_ptr[i] == n_kids[hp.node_of_slot[s]], "child count", s);
        for (int32_t q = hp.child_ptr[i]; q < hp.child_ptr[i + 1]; ++q) {
            const int32_t c = hp.child_slot[q];
            check(c >= 0 && c < N && in.parent[hp.node_of_slot[c]] == hp.node_of_slot[s], "child link", s, c);
            check(level[c] < level[s], "child level", s, c);
        }
    }
    // counts through the level schedule against the walk-up definition
    const std::vector<int64_t> want = walk_up_counts(in);
    std::vector<int64_t> C((size_t)N * n, 0);
    for (int32_t k = 0; k < n; ++k) {
        int64_t tot = 0;
        for (int64_t e = hp.indptr[k]; e < hp.indptr[k + 1]; ++e) {
            C[(size_t)hp.entry_slot[e] * n + k] += hp.entry_count[e];
            tot += hp.entry_count[e];
        }
        check(tot == hp.totals[k], "sample total", k);
    }
    for (int32_t h = 1; h < hp.n_levels; ++h)
        for (int32_t s = hp.level_ptr[h]; s < hp.level_ptr[h + 1]; ++s)
            for (int32_t q = hp.child_ptr[s - hp.n_leaf]; q < hp.child_ptr[s - hp.n_leaf + 1]; ++q)
                for (int32_t k = 0; k < n; ++k) C[(size_t)s * n + k] += C[(size_t)hp.child_slot[q] * n + k];
    for (int32_t v = 0; v < N; ++v)
        for (int32_t k = 0; k < n; ++k)
            check(C[(size_t)hp.slot_of_node[v] * n + k] == want[(size_t)v * n + k], "level counts", v, k);
    // depth-first ranges: counts from two running sums over the sorted entries
    RangeTables rt;
    range_tables(hp, &rt);
    for (int32_t k = 0; k < n; ++k) {
        const int64_t a = hp.indptr[k], b = hp.indptr[k + 1];
        for (int64_t e = a + 1; e < b; ++e) check(rt.spos[e - 1] <= rt.spos[e], "sorted entries", k, e);
        auto below = [&](int32_t x) {
            int64_t c = 0;
            for (int64_t e = a; e < b && rt.spos[e] < x; ++e) c = rt.scum[e];
            return c;
        };
        for (int32_t s = 0; s < N; ++s)
            check(below(rt.hi[s]) - below(rt.lo[s]) == C[(size_t)s * n + k], "range counts", s, k);
    }
    // the tail program reproduces the top levels from the rows below them
    const int32_t h0 = std::max(narrow_tail_level(hp, 3), 1);
    TailProgramHost tp;
    if (h0 < hp.n_levels && tail_program(hp, h0, &tp)) {
        std::vector<int64_t> X = C;
        for (int32_t s = hp.level_ptr[h0]; s < N; ++s)
            for (int32_t k = 0; k < n; ++k) X[(size_t)s * n + k] = -1;   // must be rewritten
        check(tp.lvl.size() == (size_t)(hp.n_levels - h0) + 1, "tail levels");
        int32_t covered = 0;
        for (size_t c = 0; c + 1 < tp.chunks.size(); c += 2) {
            check(tp.chunks[c] == covered, "tail chunks contiguous", (long long)c);
            covered = tp.chunks[c + 1];
            // one chunk's levels, records and kids must fit the kernel's LDS arrays
            const int32_t r0 = tp.lvl[tp.chunks[c]], r1 = tp.lvl[tp.chunks[c + 1]];
            check(tp.chunks[c + 1] - tp.chunks[c] <= kTailMaxLevels, "tail chunk levels",
                  tp.chunks[c + 1] - tp.chunks[c]);
            check(r1 - r0 <= kTailMaxNodes, "tail chunk nodes", r1 - r0);
            if (r1 > r0)
                check(tp.rec[4 * (r1 - 1) + 2] - tp.rec[4 * r0 + 1] <= kTailMaxKids, "tail chunk kids",
                      tp.rec[4 * (r1 - 1) + 2] - tp.rec[4 * r0 + 1]);
            for (int32_t lv = tp.chunks[c]; lv < tp.chunks[c + 1]; ++lv)
                for (int32_t i = tp.lvl[lv]; i < tp.lvl[lv + 1]; ++i) {
                    const int32_t s = tp.rec[4 * i];
                    for (int32_t k = 0; k < n; ++k) {
                        int64_t acc = 0;
                        for (int32_t q = tp.rec[4 * i + 1]; q < tp.rec[4 * i + 2]; ++q) {
                            const int64_t x = X[(size_t)tp.kid[q] * n + k];
                            check(x >= 0, "tail reads a row before it is written", s, tp.kid[q]);
                            acc += x;
                        }
                        X[(size_t)s * n + k] = acc;
                    }
                }
        }
        check(covered == hp.n_levels - h0, "tail chunks cover the tail", covered);
        for (size_t i = 0; i < X.size(); ++i) check(X[i] == C[i], "tail counts", (long long)i);
    }
}

uf_status prepare(const Input &in)
{
    const uf_tree t = in.tree();
    const uf_table b = in.table();
    HostPrep hp;
    std::string err;
    return validate_and_prepare(&t, &b, &hp, &err);
}

void check_malformed(Rng &r)
{
    const Input base = random_input(r, 40, 5);
    check(prepare(base) == UF_OK, "base input");
    const int32_t N = (int32_t)base.parent.size();
    int32_t root = 0, leaf = base.feature_node[0], inner = -1;
    for (int32_t v = 0; v < N; ++v) {
        if (base.parent[v] < 0) root = v;
        else if (inner < 0 && base.parent[base.parent[v]] >= 0) inner = base.parent[v];
    }
    auto expect = [&](Input in, uf_status code, const char *what) {
        const uf_status s = prepare(in);
        check(s == code, what, s, code);
    };
    { Input in = base; in.parent[leaf] = N; expect(in, UF_E_TREE, "parent out of range"); }
    { Input in = base; in.parent[leaf] = -2; expect(in, UF_E_TREE, "negative parent"); }
    { Input in = base; in.parent[leaf] = leaf; expect(in, UF_E_TREE, "own parent"); }
    { Input in = base; in.parent[leaf] = -1; expect(in, UF_E_TREE, "two roots"); }
    { Input in = base; in.parent[root] = leaf; expect(in, UF_E_TREE, "no root"); }
    if (inner >= 0) {   // inner's parent is not the root: hang that parent below inner
        Input in = base;
        in.parent[in.parent[inner]] = inner;
        const uf_status s = prepare(in);
        check(s == UF_E_TREE, "cycle", s);
    }
    { Input in = base; in.length[leaf] = -1.0; expect(in, UF_E_TREE, "negative length"); }
    { Input in = base; in.length[leaf] = std::nan(""); expect(in, UF_E_TREE, "NaN length"); }
    { Input in = base; in.length[leaf] = std::numeric_limits<double>::infinity(); expect(in, UF_E_TREE, "infinite length"); }
    { Input in = base; in.length[root] = std::nan(""); expect(in, UF_OK, "root length ignored"); }
    { Input in = base; in.indptr[0] = 1; expect(in, UF_E_TABLE, "indptr[0]"); }
    { Input in = base; std::swap(in.indptr[1], in.indptr[2]); if (in.indptr[1] != in.indptr[2]) expect(in, UF_E_TABLE, "indptr order"); }
    { Input in = base; in.indices[0] = in.n_features; expect(in, UF_E_TABLE, "feature id range"); }
    { Input in = base; in.indices[0] = -1; expect(in, UF_E_TABLE, "negative feature id"); }
    { Input in = base; in.counts[0] = -1; expect(in, UF_E_TABLE, "negative count"); }
    { Input in = base; in.feature_node[0] = N; expect(in, UF_E_TABLE, "feature node range"); }
    if (inner >= 0) {
        Input in = base;
        in.feature_node[0] = inner;
        in.indices[0] = 0;
        expect(in, UF_E_TABLE, "feature on an internal node");
    }
    {   // a sample whose entries all count zero
        Input in = base;
        for (int64_t e = in.indptr[1]; e < in.indptr[2]; ++e) in.counts[e] = 0;
        expect(in, UF_E_EMPTY_SAMPLE, "empty sample");
    }
    {   // a sample total beyond int32
        Input in = base;
        in.counts[0] = std::numeric_limits<int32_t>::max();
        in.counts[1] = std::numeric_limits<int32_t>::max();
        if (in.indptr[1] >= 2) expect(in, UF_E_TABLE, "total overflow");
    }
    { Input in = base; in.n_samples = 0; expect(in, UF_E_ARG, "no samples"); }
    { Input in = base; in.n_features = -1; expect(in, UF_E_ARG, "negative feature count"); }
    {
        HostPrep hp;
        std::string err;
        const uf_tree t = base.tree();
        const uf_table b = base.table();
        check(validate_and_prepare(nullptr, &b, &hp, &err) == UF_E_ARG, "NULL tree");
        check(validate_and_prepare(&t, nullptr, &hp, &err) == UF_E_ARG, "NULL table");
        uf_tree t0 = t;
        t0.n_nodes = 0;
        check(validate_and_prepare(&t0, &b, &hp, &err) == UF_E_ARG, "no nodes");
    }
}

}  // namespace

int main(int argc, char **argv)
{
    const int rounds = argc > 1 ? std::atoi(argv[1]) : 200;
    Rng r{20050526};
    for (int i = 0; i < rounds; ++i) {
        const int32_t N = 1 + r.below(i < 20 ? 8 : 300);
        const int32_t n = 1 + r.below(9);
        const Input in = random_input(r, N, n);
        const uf_tree t = in.tree();
        const uf_table b = in.table();
        HostPrep hp;
        std::string err;
        const uf_status s = validate_and_prepare(&t, &b, &hp, &err);
        check(s == UF_OK, "valid input", i, s);
        if (s == UF_OK) check_prepared(in, hp);
        if (i % 10 == 0) check_malformed(r);
    }
    // a deep chain: one tip under many unary nodes (the tail program's chunking)
    {
        Input in;
        const int32_t N = 5000;
        for (int32_t v = 0; v < N; ++v) {
            in.parent.push_back(v == 0 ? -1 : v - 1);
            in.length.push_back(0.5);
        }
        in.feature_node = {N - 1};
        in.n_features = 1;
        in.n_samples = 2;
        in.indptr = {0, 1, 2};
        in.indices = {0, 0};
        in.counts = {3, 4};
        const uf_tree t = in.tree();
        const uf_table b = in.table();
        HostPrep hp;
        std::string err;
        check(validate_and_prepare(&t, &b, &hp, &err) == UF_OK, "chain");
        check_prepared(in, hp);
    }
    // a comb: a chain of internal nodes with four leaves each, so the tail program's chunks
    // are bounded by their kids rather than their nodes
    {
        Input in;
        const int32_t L = 700;
        for (int32_t i = 0; i < L; ++i) {
            in.parent.push_back(i == 0 ? -1 : i - 1);
            in.length.push_back(0.25);
        }
        for (int32_t i = 0; i < L; ++i)
            for (int32_t j = 0; j < 4; ++j) {
                in.feature_node.push_back((int32_t)in.parent.size());
                in.parent.push_back(i);
                in.length.push_back(1.0);
            }
        in.n_features = (int32_t)in.feature_node.size();
        in.n_samples = 3;
        in.indptr = {0};
        for (int32_t k = 0; k < 3; ++k) {
            for (int32_t f = k; f < in.n_features; f += 7) {
                in.indices.push_back(f);
                in.counts.push_back(1 + f % 5);
            }
            in.indptr.push_back((int64_t)in.indices.size());
        }
        const uf_tree t = in.tree();
        const uf_table b = in.table();
        HostPrep hp;
        std::string err;
        check(validate_and_prepare(&t, &b, &hp, &err) == UF_OK, "comb");
        check_prepared(in, hp);
    }
    // three chains under the root: three nodes per level, so the chunks are bounded by their
    // nodes
    {
        Input in;
        const int32_t L = 1500;
        in.parent.push_back(-1);
        in.length.push_back(0.0);
        for (int32_t c = 0; c < 3; ++c)
            for (int32_t i = 0; i < L; ++i) {
                in.parent.push_back(i == 0 ? 0 : (int32_t)in.parent.size() - 1);
                in.length.push_back(0.125 * (c + 1));
            }
        for (int32_t c = 0; c < 3; ++c) in.feature_node.push_back(1 + c * L + L - 1);
        in.n_features = 3;
        in.n_samples = 2;
        in.indptr = {0, 2, 3};
        in.indices = {0, 2, 1};
        in.counts = {5, 1, 2};
        const uf_tree t = in.tree();
        const uf_table b = in.table();
        HostPrep hp;
        std::string err;
        check(validate_and_prepare(&t, &b, &hp, &err) == UF_OK, "three chains");
        check_prepared(in, hp);
    }
    // a table large enough for the threaded table pass: counts against the walk-up definition,
    // and with two planted errors the one of the earlier sample is reported
    {
        Rng rb{7};
        Input in = random_input(rb, 3001, 1);
        in.n_samples = 400;
        in.indices.clear();
        in.counts.clear();
        in.indptr.assign(1, 0);
        for (int32_t k = 0; k < in.n_samples; ++k) {
            for (int32_t e = 0; e < 1500; ++e) {
                in.indices.push_back(rb.below(in.n_features));
                in.counts.push_back(1 + rb.below(9));
            }
            in.indptr.push_back((int64_t)in.indices.size());
        }
        const uf_tree t = in.tree();
        const uf_table b = in.table();
        HostPrep hp;
        std::string err;
        check(validate_and_prepare(&t, &b, &hp, &err) == UF_OK, "large table");
        const std::vector<int64_t> want = walk_up_counts(in);
        std::vector<int64_t> C((size_t)hp.n_nodes * in.n_samples, 0);
        const int32_t n = in.n_samples;
        for (int32_t k = 0; k < n; ++k) {
            int64_t tot = 0;
            for (int64_t e = hp.indptr[k]; e < hp.indptr[k + 1]; ++e) {
                C[(size_t)hp.entry_slot[e] * n + k] += hp.entry_count[e];
                tot += hp.entry_count[e];
            }
            check(tot == hp.totals[k], "large table total", k);
        }
        for (int32_t h = 1; h < hp.n_levels; ++h)
            for (int32_t s = hp.level_ptr[h]; s < hp.level_ptr[h + 1]; ++s)
                for (int32_t q = hp.child_ptr[s - hp.n_leaf]; q < hp.child_ptr[s - hp.n_leaf + 1]; ++q)
                    for (int32_t k = 0; k < n; ++k) C[(size_t)s * n + k] += C[(size_t)hp.child_slot[q] * n + k];
        for (int32_t v = 0; v < hp.n_nodes; ++v)
            for (int32_t k = 0; k < n; ++k)
                check(C[(size_t)hp.slot_of_node[v] * n + k] == want[(size_t)v * n + k], "large table counts", v, k);
        Input bad = in;
        bad.counts[bad.indptr[350] + 3] = -5;                 // late sample
        bad.indices[bad.indptr[120] + 7] = bad.n_features;    // earlier sample
        const uf_table bb = bad.table();
        HostPrep hp2;
        std::string err2;
        check(validate_and_prepare(&t, &bb, &hp2, &err2) == UF_E_TABLE, "large table error code");
        check(err2.find("row 120") != std::string::npos, "first error in sample order");
    }
    std::printf("host checks: %d rounds, %d failures\n", rounds, g_failures);
    return g_failures == 0 ? 0 : 1;
}
