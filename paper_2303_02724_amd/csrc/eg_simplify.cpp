// eg_simplify.cpp -- simplification of a finished extremum graph (host).
//
// The paper's two graph operations (Sec. 3.5), both serial there and here:
// the graph has one node per critical point, orders of magnitude fewer than
// the grid has vertices, and the cancellations depend on each other.
//
//   arc bundling      for every pair of maxima that share saddles, the highest
//                     shared saddle represents the pair; a saddle survives iff
//                     it represents at least one of its pairs (connectivity
//                     between maxima is kept).
//   cancellation      persistence-directed: saddles in a priority queue keyed
//                     by cost = height of the lowest of their maxima - height
//                     of the saddle (ties: the lower saddle first), costs
//                     recomputed lazily when a saddle reaches the top; the
//                     lowest maximum merges into the highest maximum of the
//                     saddle, which stays queued while it still joins two or
//                     more maxima.  Costs above the threshold end a saddle.
//
// Heights follow the graph's order: value, ties by vertex id (Sec. 3.3),
// reversed for a minimum graph.
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

// Saddles that survive bundling (flags per saddle).
std::vector<char> bundle(const Graph& G)
{
    struct PairRec {
        uint64_t key;  // (lower maximum index, higher maximum index)
        int32_t sad;
    };
    std::vector<PairRec> recs;
    std::vector<int32_t> ms;
    for (size_t i = 0; i < G.sd.size(); ++i) {
        ms.assign(G.arc.begin() + G.off[i], G.arc.begin() + G.off[i + 1]);
        std::sort(ms.begin(), ms.end());
        ms.erase(std::unique(ms.begin(), ms.end()), ms.end());
        for (size_t a = 0; a < ms.size(); ++a)
            for (size_t b = a + 1; b < ms.size(); ++b)
                recs.push_back(PairRec{(uint64_t(uint32_t(ms[a])) << 32) | uint32_t(ms[b]), (int32_t)i});
    }
    // group by pair; the highest saddle of each group is its representative
    std::sort(recs.begin(), recs.end(), [&](const PairRec& x, const PairRec& y) {
        if (x.key != y.key) return x.key < y.key;
        return higher(G.sd[(size_t)x.sad], G.sd[(size_t)y.sad], G.minima);
    });
    std::vector<char> keep(G.sd.size(), 0);
    for (size_t r = 0; r < recs.size(); ++r)
        if (r == 0 || recs[r].key != recs[r - 1].key) keep[(size_t)recs[r].sad] = 1;
    return keep;
}

struct Cancel {
    const Graph& G;
    std::vector<int32_t> parent;  // union-find over maxima
    explicit Cancel(const Graph& g) : G(g), parent(g.mx.size())
    {
        for (size_t j = 0; j < parent.size(); ++j) parent[j] = (int32_t)j;
    }
    int32_t root(int32_t m)
    {
        while (parent[(size_t)m] != m) {
            parent[(size_t)m] = parent[(size_t)parent[(size_t)m]];
            m = parent[(size_t)m];
        }
        return m;
    }
    // distinct current maxima of saddle i; lowest and highest among them
    int scan(int32_t i, int32_t* lo, int32_t* hi)
    {
        int n = 0;
        int32_t l = -1, h = -1;
        thread_local std::vector<int32_t> seen;
        seen.clear();
        for (int32_t k = G.off[i]; k < G.off[i + 1]; ++k) {
            const int32_t m = root(G.arc[(size_t)k]);
            if (std::find(seen.begin(), seen.end(), m) != seen.end()) continue;
            seen.push_back(m);
            ++n;
            if (l < 0 || higher(G.mx[(size_t)l], G.mx[(size_t)m], G.minima)) l = m;
            if (h < 0 || higher(G.mx[(size_t)m], G.mx[(size_t)h], G.minima)) h = m;
        }
        *lo = l;
        *hi = h;
        return n;
    }
};

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
    Cancel C(G);
    int64_t np = 0;
    if (ops & EG_SIMPLIFY_CANCEL) {
        // min-queue on (cost, saddle order): lower saddles first among equal costs
        auto after = [&](const Entry& a, const Entry& b) {
            if (a.cost != b.cost) return a.cost > b.cost;
            return higher(G.sd[(size_t)a.sad], G.sd[(size_t)b.sad], G.minima);
        };
        std::priority_queue<Entry, std::vector<Entry>, decltype(after)> q(after);
        auto cost_of = [&](int32_t i, Entry* e) {
            int32_t lo, hi;
            if (C.scan(i, &lo, &hi) < 2) return false;
            *e = Entry{G.mx[(size_t)lo].h - G.sd[(size_t)i].h, i};
            return true;
        };
        for (size_t i = 0; i < nsad; ++i) {
            Entry e;
            if (live[i] && cost_of((int32_t)i, &e)) q.push(e);
        }
        while (!q.empty()) {
            const int32_t i = q.top().sad;
            q.pop();
            Entry e;
            if (!cost_of(i, &e)) continue;         // joins a single maximum now
            if (e.cost > threshold) continue;      // costs only grow: never cancelled
            if (!q.empty() && after(e, q.top())) {  // no longer the cheapest
                q.push(e);
                continue;
            }
            int32_t lo, hi;
            C.scan(i, &lo, &hi);
            C.parent[(size_t)lo] = hi;  // the lower maximum merges into the elder
            pair_saddle[np] = i;
            pair_max[np] = lo;
            pair_cost[np] = e.cost;
            ++np;
            if (cost_of(i, &e)) q.push(e);
        }
    }
    *n_pairs = np;
    // rows of the simplified graph: surviving saddles join >= 2 maxima
    out_offsets[0] = 0;
    int32_t at = 0;
    std::vector<int32_t> ms;
    for (size_t i = 0; i < nsad; ++i) {
        if (live[i]) {
            ms.clear();
            for (int32_t k = G.off[i]; k < G.off[i + 1]; ++k) ms.push_back(G.mx[(size_t)C.root(G.arc[(size_t)k])].id);
            std::sort(ms.begin(), ms.end());
            ms.erase(std::unique(ms.begin(), ms.end()), ms.end());
            if (ms.size() >= 2)
                for (int32_t m : ms) out_arcs[at++] = m;
        }
        out_offsets[i + 1] = at;
    }
    for (size_t j = 0; j < G.mx.size(); ++j) max_rep[j] = C.root((int32_t)j);
    return EG_OK;
}
