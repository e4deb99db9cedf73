// eg_simplify.cpp -- simplification of a finished extremum graph (host).
//
// The paper's two graph operations (Sec. 3.5), both serial there and here:
// the graph has one node per critical point, orders of magnitude fewer than
// the grid has vertices, and the cancellations depend on each other.
//
//   arc bundling      for every pair of maxima that share saddles, the highest
//                     shared saddle represents the pair and the pair's other
//                     saddles are discarded; a saddle survives iff it
//                     represents at least one of its pairs, or has fewer than
//                     two distinct maxima (no pair shares it).
//   cancellation      persistence-directed: saddles in a priority queue keyed
//                     by cost = height of the second-highest of their maxima
//                     - height of the saddle (for a simple saddle the lower of
//                     its two maxima; ties: the lower saddle first), costs
//                     recomputed when a saddle reaches the top: above the
//                     threshold -> discarded; above the cost stored at the
//                     top of the queue -> reinserted; else cancelled: every
//                     maximum of the saddle except the highest merges into
//                     the highest, and the saddle leaves the graph.
//
// Heights follow the graph's order: value, ties by vertex id (Sec. 3.3),
// reversed for a minimum graph.
//
// Cost: bundling is linear in the number of (saddle, pair of maxima) records
// (bucketed by the lower maximum, no comparison sort).  The queue holds the
// initial entries as one sorted run plus a binary heap of reinserted entries;
// a saddle with at most two maxima whose initial cost is above the threshold
// is never queued, since merges only raise such a saddle's maxima and its
// cost cannot fall back (dropping entries above the threshold never changes a
// decision about an entry at or below it).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <queue>
#include <vector>

#include "eg.h"

namespace {

struct Node {
    double h;  // height in the graph's direction
    int32_t id;
};

// a strictly above b in the graph's order
inline bool higher(const Node& a, const Node& b, bool minima)
{
    if (a.h != b.h) return a.h > b.h;
    return minima ? a.id < b.id : a.id > b.id;
}

struct Graph {
    bool minima;
    std::vector<Node> mx, sd;
    const int32_t* off;
    std::vector<int32_t> arc;  // maxima indices
};

bool load(const eg_graph_host* g, Graph* G)
{
    if (!g || g->nmax < 0 || g->nsad < 0 || (g->flags & ~uint32_t(EG_MINIMA))) return false;
    if ((g->nmax > 0 && (!g->maxima || !g->max_values)) || !g->arc_offsets) return false;
    if (g->nsad > 0 && (!g->saddles || !g->sad_values)) return false;
    G->minima = (g->flags & EG_MINIMA) != 0;
    const double sgn = G->minima ? -1.0 : 1.0;
    G->mx.resize((size_t)g->nmax);
    for (int64_t j = 0; j < g->nmax; ++j) {
        if (j > 0 && g->maxima[j] <= g->maxima[j - 1]) return false;  // ascending ids
        G->mx[(size_t)j] = Node{sgn * (double)g->max_values[j], g->maxima[j]};
    }
    G->sd.resize((size_t)g->nsad);
    for (int64_t i = 0; i < g->nsad; ++i) G->sd[(size_t)i] = Node{sgn * (double)g->sad_values[i], g->saddles[i]};
    G->off = g->arc_offsets;
    if (g->arc_offsets[0] != 0) return false;
    for (int64_t i = 0; i < g->nsad; ++i)
        if (g->arc_offsets[i + 1] < g->arc_offsets[i]) return false;
    const int64_t narc = g->arc_offsets[g->nsad];
    if (narc > 0 && !g->arc_maxima) return false;
    G->arc.resize((size_t)narc);
    for (int64_t k = 0; k < narc; ++k) {
        const int32_t* p = std::lower_bound(g->maxima, g->maxima + g->nmax, g->arc_maxima[k]);
        if (p == g->maxima + g->nmax || *p != g->arc_maxima[k]) return false;  // not a maximum
        G->arc[(size_t)k] = (int32_t)(p - g->maxima);
    }
    return true;
}

// Distinct entries of a short row, in place (rows hold at most a few dozen).
int distinct(int32_t* ms, int n)
{
    int k = 0;
    for (int a = 0; a < n; ++a) {
        bool seen = false;
        for (int b = 0; b < k; ++b) seen |= ms[b] == ms[a];
        if (!seen) ms[k++] = ms[a];
    }
    return k;
}

// Saddles that survive bundling (flags per saddle).
std::vector<char> bundle(const Graph& G)
{
    const size_t nsad = G.sd.size(), nmax = G.mx.size();
    std::vector<char> keep(nsad, 0);
    std::vector<int32_t> row;
    // pass 1: pairs per lower maximum index; saddles no pair shares are kept
    std::vector<int64_t> start(nmax + 1, 0);
    for (size_t i = 0; i < nsad; ++i) {
        row.assign(G.arc.begin() + G.off[i], G.arc.begin() + G.off[i + 1]);
        const int k = distinct(row.data(), (int)row.size());
        if (k < 2) keep[i] = 1;
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b)
                if (row[(size_t)a] < row[(size_t)b]) ++start[(size_t)row[(size_t)a] + 1];
    }
    for (size_t j = 0; j < nmax; ++j) start[j + 1] += start[j];
    // pass 2: (higher maximum, saddle) records bucketed by the lower maximum
    std::vector<int32_t> other((size_t)start[nmax]), sad((size_t)start[nmax]);
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (size_t i = 0; i < nsad; ++i) {
        row.assign(G.arc.begin() + G.off[i], G.arc.begin() + G.off[i + 1]);
        const int k = distinct(row.data(), (int)row.size());
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b)
                if (row[(size_t)a] < row[(size_t)b]) {
                    const int64_t at = fill[(size_t)row[(size_t)a]]++;
                    other[(size_t)at] = row[(size_t)b];
                    sad[(size_t)at] = (int32_t)i;
                }
    }
    // pass 3: per lower maximum, the highest saddle of each higher partner
    std::vector<int32_t> best(nmax, -1);
    for (size_t a = 0; a < nmax; ++a) {
        for (int64_t r = start[a]; r < start[a + 1]; ++r) {
            int32_t& b = best[(size_t)other[(size_t)r]];
            const int32_t s = sad[(size_t)r];
            if (b < 0 || higher(G.sd[(size_t)s], G.sd[(size_t)b], G.minima)) b = s;
        }
        for (int64_t r = start[a]; r < start[a + 1]; ++r) {
            int32_t& b = best[(size_t)other[(size_t)r]];
            if (b >= 0) keep[(size_t)b] = 1;
            b = -1;
        }
    }
    return keep;
}

struct UnionFind {
    std::vector<int32_t> parent;  // over maxima indices; a root is a surviving maximum
    explicit UnionFind(size_t n) : parent(n)
    {
        for (size_t j = 0; j < n; ++j) parent[j] = (int32_t)j;
    }
    int32_t root(int32_t m)
    {
        while (parent[(size_t)m] != m) {
            parent[(size_t)m] = parent[(size_t)parent[(size_t)m]];
            m = parent[(size_t)m];
        }
        return m;
    }
};

// Distinct current maxima of saddle i, highest first (into ms); returns how many.
int current_maxima(const Graph& G, UnionFind& U, int32_t i, std::vector<int32_t>& ms)
{
    ms.clear();
    for (int32_t k = G.off[i]; k < G.off[i + 1]; ++k) ms.push_back(U.root(G.arc[(size_t)k]));
    const int n = distinct(ms.data(), (int)ms.size());
    ms.resize((size_t)n);
    std::sort(ms.begin(), ms.end(),
              [&](int32_t a, int32_t b) { return higher(G.mx[(size_t)a], G.mx[(size_t)b], G.minima); });
    return n;
}

struct Entry {
    double cost;
    int32_t sad;
};

}  // namespace

extern "C" eg_status eg_simplify(const eg_graph_host* g, uint32_t ops, double threshold, int32_t* out_offsets,
                                 int32_t* out_arcs, int32_t* max_rep, int32_t* pair_saddle, int32_t* pair_max,
                                 double* pair_cost, int64_t* n_pairs)
{
    Graph G;
    if (!load(g, &G)) return EG_ERR_ARG;
    if (ops & ~uint32_t(EG_SIMPLIFY_BUNDLE | EG_SIMPLIFY_CANCEL)) return EG_ERR_ARG;
    if (std::isnan(threshold)) return EG_ERR_ARG;
    const size_t nsad = G.sd.size(), narc = G.arc.size();
    if (!out_offsets || (narc > 0 && !out_arcs) || (G.mx.size() > 0 && !max_rep) || !n_pairs) return EG_ERR_ARG;
    if ((ops & EG_SIMPLIFY_CANCEL) && narc > 0 && (!pair_saddle || !pair_max || !pair_cost)) return EG_ERR_ARG;

    std::vector<char> live = (ops & EG_SIMPLIFY_BUNDLE) ? bundle(G) : std::vector<char>(nsad, 1);
    UnionFind U(G.mx.size());
    int64_t np = 0;
    if (ops & EG_SIMPLIFY_CANCEL) {
        // (cost, saddle order): lower costs first, lower saddles first among equal costs
        auto before = [&](const Entry& a, const Entry& b) {
            if (a.cost != b.cost) return a.cost < b.cost;
            return higher(G.sd[(size_t)b.sad], G.sd[(size_t)a.sad], G.minima);
        };
        auto after = [&](const Entry& a, const Entry& b) { return before(b, a); };
        std::vector<int32_t> ms;
        // initial entries, one sorted run
        std::vector<Entry> run;
        run.reserve(nsad);
        for (size_t i = 0; i < nsad; ++i) {
            if (!live[i]) continue;
            const int n = current_maxima(G, U, (int32_t)i, ms);
            if (n < 2) continue;
            const double cost = G.mx[(size_t)ms[1]].h - G.sd[i].h;
            if (n == 2 && cost > threshold) continue;  // can never become cheaper
            run.push_back(Entry{cost, (int32_t)i});
        }
        std::sort(run.begin(), run.end(), before);
        std::priority_queue<Entry, std::vector<Entry>, decltype(after)> heap(after);  // reinserted entries
        size_t pos = 0;
        auto empty = [&]() { return pos == run.size() && heap.empty(); };
        auto top = [&]() -> const Entry& {
            if (pos == run.size()) return heap.top();
            if (heap.empty() || before(run[pos], heap.top())) return run[pos];
            return heap.top();
        };
        auto pop = [&]() {
            if (pos < run.size() && (heap.empty() || before(run[pos], heap.top())))
                ++pos;
            else
                heap.pop();
        };
        while (!empty()) {
            const int32_t i = top().sad;
            pop();
            const int n = current_maxima(G, U, i, ms);
            if (n < 2) continue;  // joins a single maximum now: no cost
            const double cost = G.mx[(size_t)ms[1]].h - G.sd[(size_t)i].h;
            if (cost > threshold) continue;  // discarded
            if (!empty() && cost > top().cost) {  // the queue holds cheaper saddles
                heap.push(Entry{cost, i});
                continue;
            }
            for (int k = 1; k < n; ++k) {  // all but the highest merge into it
                U.parent[(size_t)ms[(size_t)k]] = ms[0];
                pair_saddle[np] = i;
                pair_max[np] = ms[(size_t)k];
                pair_cost[np] = cost;
                ++np;
            }
            live[(size_t)i] = 0;  // the cancelled saddle leaves the graph
        }
    }
    *n_pairs = np;
    // rows of the simplified graph: every live saddle, its distinct maxima
    out_offsets[0] = 0;
    int32_t at = 0;
    std::vector<int32_t> ms;
    for (size_t i = 0; i < nsad; ++i) {
        if (live[i]) {
            ms.clear();
            for (int32_t k = G.off[i]; k < G.off[i + 1]; ++k) ms.push_back(G.mx[(size_t)U.root(G.arc[(size_t)k])].id);
            std::sort(ms.begin(), ms.end());
            ms.erase(std::unique(ms.begin(), ms.end()), ms.end());
            for (int32_t m : ms) out_arcs[at++] = m;
        }
        out_offsets[i + 1] = at;
    }
    for (size_t j = 0; j < G.mx.size(); ++j) max_rep[j] = U.root((int32_t)j);
    return EG_OK;
}
