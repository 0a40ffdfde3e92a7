// Host-side validation and preprocessing of the tree and the count table.
//
// Everything here runs before any device work so that a malformed input is rejected with
// a status code and never reaches a kernel.  The products are the level schedule used by
// the level-synchronous embedding propagation (children of a node always sit in an earlier
// level) and the leaf slot of every CSR entry.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <limits>
#include <numeric>
#include <thread>

#include "uf_internal.h"

namespace ufmi {

namespace {
uf_status fail(std::string *err, uf_status code, const char *fmt, long long a = 0,
               long long b = 0)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, fmt, a, b);
    if (err) *err = buf;
    return code;
}
}  // namespace

uf_status validate_and_prepare(const uf_tree *tree, const uf_table *table, HostPrep *hp,
                               std::string *err)
{
    if (!tree || !table) return fail(err, UF_E_ARG, "tree and table must not be NULL");
    const int32_t N = tree->n_nodes;
    if (N < 1) return fail(err, UF_E_ARG, "n_nodes must be >= 1 (got %lld)", N);
    if (!tree->parent || !tree->length)
        return fail(err, UF_E_ARG, "tree parent/length must not be NULL");
    const int32_t n = table->n_samples;
    if (n < 1) return fail(err, UF_E_ARG, "n_samples must be >= 1 (got %lld)", n);
    if (table->n_features < 0) return fail(err, UF_E_ARG, "n_features must be >= 0");
    if (!table->indptr) return fail(err, UF_E_ARG, "table indptr must not be NULL");

    // ---- tree: one root, parents in range, finite non-negative lengths
    const int32_t *par = tree->parent;
    int32_t root = -1;
    for (int32_t v = 0; v < N; ++v) {
        int32_t p = par[v];
        if (p == -1) {
            if (root >= 0) return fail(err, UF_E_TREE, "two roots: nodes %lld and %lld", root, v);
            root = v;
        } else if (p < 0 || p >= N) {
            return fail(err, UF_E_TREE, "parent[%lld] = %lld out of range", v, p);
        } else if (p == v) {
            return fail(err, UF_E_TREE, "node %lld is its own parent", v);
        } else {
            double L = tree->length[v];
            if (!std::isfinite(L) || L < 0.0)
                return fail(err, UF_E_TREE, "length of node %lld is negative or not finite", v);
        }
    }
    if (root < 0) return fail(err, UF_E_TREE, "no root (no parent == -1)");

    // children CSR in node-id order
    std::vector<int32_t> cptr(N + 1, 0), cidx(N > 0 ? N - 1 : 0);
    for (int32_t v = 0; v < N; ++v)
        if (par[v] >= 0) cptr[par[v] + 1]++;
    for (int32_t v = 0; v < N; ++v) cptr[v + 1] += cptr[v];
    {
        std::vector<int32_t> fillp(cptr.begin(), cptr.end() - 1);
        for (int32_t v = 0; v < N; ++v)
            if (par[v] >= 0) cidx[fillp[par[v]]++] = v;
    }
    // breadth-first order from the root; a node not reached sits on a cycle
    std::vector<int32_t> order;
    order.reserve(N);
    order.push_back(root);
    for (size_t h = 0; h < order.size(); ++h) {
        int32_t v = order[h];
        for (int32_t q = cptr[v]; q < cptr[v + 1]; ++q) order.push_back(cidx[q]);
    }
    if ((int32_t)order.size() != N)
        return fail(err, UF_E_TREE, "%lld nodes do not reach the root (cycle)", N - (long long)order.size());

    // heights, children before parents in reverse BFS order
    std::vector<int32_t> height(N, 0);
    for (int32_t h = N - 1; h >= 0; --h) {
        int32_t v = order[h];
        int32_t p = par[v];
        if (p >= 0 && height[p] < height[v] + 1) height[p] = height[v] + 1;
    }
    const int32_t n_levels = height[root] + 1;

    // ---- table: CSR structure, feature ids, leaf mapping, totals
    const int64_t *ip = table->indptr;
    if (ip[0] != 0) return fail(err, UF_E_TABLE, "indptr[0] must be 0 (got %lld)", ip[0]);
    for (int32_t k = 0; k < n; ++k)
        if (ip[k + 1] < ip[k]) return fail(err, UF_E_TABLE, "indptr decreases at row %lld", k);
    const int64_t nnz = ip[n];
    if (nnz > 0 && (!table->indices || !table->counts))
        return fail(err, UF_E_ARG, "table indices/counts must not be NULL");
    if (nnz > (int64_t)std::numeric_limits<int32_t>::max() * 8)
        return fail(err, UF_E_TABLE, "too many entries (%lld)", nnz);
    const int32_t F = table->n_features;
    const int32_t *fnode = table->feature_node;
    if (!fnode && F > N)
        return fail(err, UF_E_TABLE, "feature_node is NULL but n_features %lld > n_nodes %lld", F, N);
    if (fnode)
        for (int32_t f = 0; f < F; ++f)
            if (fnode[f] < 0 || fnode[f] >= N)
                return fail(err, UF_E_TABLE, "feature_node[%lld] = %lld out of range", f, fnode[f]);

    // ---- slots by (height, id)
    hp->n_nodes = N;
    hp->n_samples = n;
    hp->n_features = F;
    hp->root = root;
    hp->n_levels = n_levels;
    hp->nnz = nnz;
    hp->level_ptr.assign(n_levels + 1, 0);
    for (int32_t v = 0; v < N; ++v) hp->level_ptr[height[v] + 1]++;
    for (int32_t h = 0; h < n_levels; ++h) hp->level_ptr[h + 1] += hp->level_ptr[h];
    hp->n_leaf = hp->level_ptr[1];
    hp->slot_of_node.assign(N, 0);
    hp->node_of_slot.assign(N, 0);
    {
        std::vector<int32_t> next(hp->level_ptr.begin(), hp->level_ptr.end() - 1);
        for (int32_t v = 0; v < N; ++v) {
            int32_t s = next[height[v]]++;
            hp->slot_of_node[v] = s;
            hp->node_of_slot[s] = v;
        }
    }
    const int32_t n_int = N - hp->n_leaf;
    hp->child_ptr.assign(n_int + 1, 0);
    hp->child_slot.clear();
    hp->child_slot.reserve(N > 0 ? N - 1 : 0);
    for (int32_t s = hp->n_leaf; s < N; ++s) {
        int32_t v = hp->node_of_slot[s];
        for (int32_t q = cptr[v]; q < cptr[v + 1]; ++q)
            hp->child_slot.push_back(hp->slot_of_node[cidx[q]]);
        hp->child_ptr[s - hp->n_leaf + 1] = (int32_t)hp->child_slot.size();
    }
    hp->length_slot.assign(N, 0.0);
    for (int32_t v = 0; v < N; ++v)
        if (v != root) hp->length_slot[hp->slot_of_node[v]] = tree->length[v];

    hp->indptr.assign(ip, ip + n + 1);
    hp->entry_slot.resize(nnz);
    hp->entry_count.resize(nnz);
    hp->totals.assign(n, 0);
    // The table pass runs on up to 16 host threads over contiguous sample ranges (each writes
    // the entries of its own samples); the error reported is the first one in sample order,
    // the one a single pass would meet.
    const int32_t n_thr = (int32_t)std::max<int64_t>(
        1, std::min<int64_t>({(int64_t)std::max(1u, std::thread::hardware_concurrency()), 16, nnz / 65536 + 1, n}));
    struct Bad {
        uf_status code = UF_OK;
        std::string msg;
    };
    std::vector<Bad> bad(n_thr);
    auto table_pass = [&](int32_t t) {
        const int32_t k0 = (int32_t)((int64_t)n * t / n_thr), k1 = (int32_t)((int64_t)n * (t + 1) / n_thr);
        std::string *msg = &bad[t].msg;
        for (int32_t k = k0; k < k1; ++k) {
            int64_t tot = 0;
            for (int64_t e = ip[k]; e < ip[k + 1]; ++e) {
                int32_t f = table->indices[e];
                if (f < 0 || f >= F) {
                    bad[t].code = fail(msg, UF_E_TABLE, "feature id %lld out of range in row %lld", f, k);
                    return;
                }
                int32_t c = table->counts[e];
                if (c < 0) {
                    bad[t].code = fail(msg, UF_E_TABLE, "negative count in row %lld entry %lld", k, e);
                    return;
                }
                int32_t v = fnode ? fnode[f] : f;
                if (cptr[v + 1] != cptr[v]) {
                    bad[t].code = fail(msg, UF_E_TABLE, "feature %lld sits on internal node %lld", f, v);
                    return;
                }
                hp->entry_slot[e] = hp->slot_of_node[v];
                hp->entry_count[e] = c;
                tot += c;
            }
            if (tot == 0) {
                bad[t].code = fail(msg, UF_E_EMPTY_SAMPLE, "sample %lld has no reads", k);
                return;
            }
            if (tot > std::numeric_limits<int32_t>::max()) {
                bad[t].code = fail(msg, UF_E_TABLE, "sample %lld total %lld exceeds int32", k, tot);
                return;
            }
            hp->totals[k] = (int32_t)tot;
        }
    };
    if (n_thr == 1) {
        table_pass(0);
    } else {
        std::vector<std::thread> pool;
        pool.reserve(n_thr - 1);
        for (int32_t t = 1; t < n_thr; ++t) pool.emplace_back(table_pass, t);
        table_pass(0);
        for (std::thread &th : pool) th.join();
    }
    for (const Bad &b : bad)
        if (b.code != UF_OK) {
            if (err) *err = b.msg;
            return b.code;
        }
    return UF_OK;
}

int32_t narrow_tail_level(const HostPrep &hp, int32_t max_nodes)
{
    int32_t h = hp.n_levels;
    while (h > 1 && hp.level_ptr[h] - hp.level_ptr[h - 1] <= max_nodes) --h;
    return h;
}

bool tail_program(const HostPrep &hp, int32_t h0, TailProgramHost *tp)
{
    tp->lvl.clear();
    tp->kid.clear();
    tp->rec.clear();
    tp->chunks.clear();
    int32_t chunk_first = 0, chunk_recs = 0, chunk_kids = 0;
    for (int32_t h = h0; h < hp.n_levels; ++h) {
        const int32_t nodes = hp.level_ptr[h + 1] - hp.level_ptr[h];
        int32_t kids = 0;
        for (int32_t s = hp.level_ptr[h]; s < hp.level_ptr[h + 1]; ++s)
            kids += hp.child_ptr[s - hp.n_leaf + 1] - hp.child_ptr[s - hp.n_leaf];
        if (nodes > kTailMaxNodes || kids > kTailMaxKids) return false;
        const int32_t lv = h - h0;
        if (chunk_recs + nodes > kTailMaxNodes || chunk_kids + kids > kTailMaxKids ||
            lv - chunk_first >= kTailMaxLevels) {
            tp->chunks.push_back(chunk_first);
            tp->chunks.push_back(lv);
            chunk_first = lv;
            chunk_recs = chunk_kids = 0;
        }
        tp->lvl.push_back((int32_t)(tp->rec.size() / 4));
        for (int32_t s = hp.level_ptr[h]; s < hp.level_ptr[h + 1]; ++s) {
            const int32_t i = s - hp.n_leaf;
            const int32_t k0 = (int32_t)tp->kid.size();
            for (int32_t q = hp.child_ptr[i]; q < hp.child_ptr[i + 1]; ++q) tp->kid.push_back(hp.child_slot[q]);
            tp->rec.insert(tp->rec.end(), {s, k0, (int32_t)tp->kid.size(), 0});
        }
        chunk_recs += nodes;
        chunk_kids += kids;
    }
    const int32_t n_lv = hp.n_levels - h0;
    tp->lvl.push_back((int32_t)(tp->rec.size() / 4));
    if (n_lv > chunk_first) {
        tp->chunks.push_back(chunk_first);
        tp->chunks.push_back(n_lv);
    }
    return true;
}

// Euler-tour tables for generating count rows without the level propagation: tips are
// numbered in depth-first order (children in node-id order), so the tips below any node form
// one contiguous range [lo, hi) of that order, and a sample's reads below the node are the
// difference of two prefix sums over its entries sorted by tip position.
void range_tables(const HostPrep &hp, RangeTables *rt)
{
    const int32_t N = hp.n_nodes, n = hp.n_samples;
    rt->lo.assign(N, 0);
    rt->hi.assign(N, 0);
    std::vector<int32_t> tip_pos(N, -1);
    // iterative depth-first walk over slots from the root (the last slot)
    std::vector<std::pair<int32_t, int32_t>> stack;   // (slot, next child index)
    stack.reserve(64);
    stack.push_back({N - 1, 0});
    int32_t pos = 0;
    while (!stack.empty()) {
        auto &top = stack.back();
        const int32_t s = top.first;
        if (s < hp.n_leaf) {   // a tip
            rt->lo[s] = pos;
            tip_pos[s] = pos++;
            rt->hi[s] = pos;
            stack.pop_back();
            continue;
        }
        const int32_t i = s - hp.n_leaf;
        const int32_t q0 = hp.child_ptr[i], q1 = hp.child_ptr[i + 1];
        if (top.second == 0) rt->lo[s] = pos;
        if (q0 + top.second < q1) {
            const int32_t c = hp.child_slot[q0 + top.second];
            ++top.second;
            stack.push_back({c, 0});
        } else {
            rt->hi[s] = pos;
            stack.pop_back();
        }
    }
    // entries of every sample sorted by tip position, with running sums of their counts
    const int64_t nnz = hp.nnz;
    rt->spos.resize(nnz);
    rt->scum.resize(nnz);
    std::vector<int64_t> idx;
    for (int32_t k = 0; k < n; ++k) {
        const int64_t a = hp.indptr[k], b = hp.indptr[k + 1];
        idx.resize(b - a);
        std::iota(idx.begin(), idx.end(), a);
        std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) {
            return tip_pos[hp.entry_slot[x]] < tip_pos[hp.entry_slot[y]];
        });
        int64_t run = 0;
        for (int64_t t = 0; t < b - a; ++t) {
            rt->spos[a + t] = tip_pos[hp.entry_slot[idx[t]]];
            run += hp.entry_count[idx[t]];
            rt->scum[a + t] = (int32_t)run;   // <= the sample total, which fits in int32
        }
    }
}

}  // namespace ufmi
