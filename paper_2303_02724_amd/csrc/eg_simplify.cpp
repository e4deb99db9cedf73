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
// initial entries as one sorted run (a sample sort over the host's threads)
// plus a binary heap of reinserted entries; a saddle with at most two maxima
// whose initial cost is above the threshold is never queued, since merges
// only raise such a saddle's maxima and its cost cannot fall back (dropping
// entries above the threshold never changes a decision about an entry at or
// below it).  An entry carries the saddle's height and, for a saddle with two
// maxima (the common case), both maxima, so the dependent loop reads neither
// the saddle table nor the arc rows for it: only the union-find roots of its
// two maxima; a saddle with more than two needs only its two highest roots
// unless it is cancelled.  Every phase but that loop (arc look-up, bundling,
// initial costs, the sort of the run, the output rows) splits its items over
// the host's hardware threads; results do not depend on the split.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <queue>
#include <thread>
#include <vector>

#include "eg.h"

namespace {

// f(begin, end) over [0, n), split over up to 16 hardware threads when n is
// large enough to pay for them.
template <class F>
void parallel_for(int64_t n, F&& f)
{
    const unsigned hw = std::thread::hardware_concurrency();
    const int T = n < 32768 ? 1 : (int)std::max(1u, std::min(hw, 16u));
    if (T == 1) {
        f((int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    th.reserve((size_t)T);
    for (int t = 0; t < T; ++t) th.emplace_back([&f, n, t, T] { f(n * t / T, n * (t + 1) / T); });
    for (auto& x : th) x.join();
}

// f(t) for t in [0, T), one thread each.
template <class F>
void parallel_parts(int T, F&& f)
{
    if (T <= 1) {
        f(0);
        return;
    }
    std::vector<std::thread> th;
    th.reserve((size_t)T);
    for (int t = 0; t < T; ++t) th.emplace_back([&f, t] { f(t); });
    for (auto& x : th) x.join();
}

// Large working arrays are allocated without value-initialisation: their
// first touch happens in the parallel loops that fill them, not in one
// thread zeroing pages that are overwritten anyway.
template <class T>
struct NoInit : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = NoInit<U>;
    };
    NoInit() = default;
    template <class U>
    NoInit(const NoInit<U>&) noexcept
    {
    }
    template <class U>
    void construct(U* p) noexcept
    {
        ::new ((void*)p) U;
    }
    template <class U, class... A>
    void construct(U* p, A&&... a)
    {
        ::new ((void*)p) U(std::forward<A>(a)...);
    }
};
template <class T>
using Buf = std::vector<T, NoInit<T>>;

// Sort with the comparator `before`: chunks in parallel, then merged pairwise
// in parallel rounds.
template <class E, class Cmp>
void parallel_sort(std::vector<E>& v, Cmp before)
{
    const int64_t n = (int64_t)v.size();
    const unsigned hw = std::thread::hardware_concurrency();
    const int T = n < 65536 ? 1 : (int)std::max(1u, std::min(hw, 16u));
    if (T == 1) {
        std::sort(v.begin(), v.end(), before);
        return;
    }
    std::vector<int64_t> cut((size_t)T + 1);
    for (int t = 0; t <= T; ++t) cut[(size_t)t] = n * t / T;
    {
        std::vector<std::thread> th;
        for (int t = 0; t < T; ++t)
            th.emplace_back([&, t] { std::sort(v.begin() + cut[(size_t)t], v.begin() + cut[(size_t)t + 1], before); });
        for (auto& x : th) x.join();
    }
    std::vector<E> tmp((size_t)n);
    std::vector<E>* src = &v;
    std::vector<E>* dst = &tmp;
    for (int width = 1; width < T; width *= 2) {
        std::vector<std::thread> th;
        for (int t = 0; t < T; t += 2 * width) {
            const int64_t a = cut[(size_t)t], m = cut[(size_t)std::min(t + width, T)],
                          b = cut[(size_t)std::min(t + 2 * width, T)];
            th.emplace_back([=, &before] {
                std::merge(src->begin() + a, src->begin() + m, src->begin() + m, src->begin() + b, dst->begin() + a,
                           before);
            });
        }
        for (auto& x : th) x.join();
        std::swap(src, dst);
    }
    if (src != &v) v.swap(*src);
}

// The entries of all parts as one run sorted by `before`, a strict total
// order (so the run does not depend on how the parts were cut): a sample
// sort.  Splitters come from regular samples of every part; each part's
// thread finds every entry's bucket and then scatters its entries to their
// bucket's range; each bucket is then sorted by a thread of its own.  The
// parts are released on the way.
template <class E, class Cmp>
Buf<E> sorted_run(std::vector<std::vector<E>>& parts, Cmp before)
{
    const int T = (int)parts.size();
    size_t total = 0;
    for (auto& p : parts) total += p.size();
    Buf<E> run(total);
    if (T == 1 || total < 65536) {
        size_t o = 0;
        for (auto& p : parts) {
            std::copy(p.begin(), p.end(), run.begin() + (int64_t)o);
            o += p.size();
            std::vector<E>().swap(p);
        }
        std::sort(run.begin(), run.end(), before);
        return run;
    }
    constexpr int kSamples = 64;  // per part
    std::vector<E> smp;
    for (auto& p : parts)
        for (int k = 0; k < kSamples && !p.empty(); ++k) smp.push_back(p[p.size() * (size_t)k / kSamples]);
    std::sort(smp.begin(), smp.end(), before);
    const int B = T;  // buckets (at most 16: one byte holds a bucket number)
    std::vector<E> split;
    for (int b = 1; b < B; ++b) split.push_back(smp[smp.size() * (size_t)b / (size_t)B]);
    std::vector<std::vector<uint8_t>> bk((size_t)T);
    std::vector<int64_t> cnt((size_t)T * (size_t)B, 0);
    parallel_parts(T, [&](int t) {
        const std::vector<E>& p = parts[(size_t)t];
        std::vector<uint8_t>& k = bk[(size_t)t];
        k.resize(p.size());
        std::vector<int64_t> c((size_t)B, 0);
        for (size_t r = 0; r < p.size(); ++r) {
            const int b = (int)(std::upper_bound(split.begin(), split.end(), p[r], before) - split.begin());
            k[r] = (uint8_t)b;
            ++c[(size_t)b];
        }
        std::copy(c.begin(), c.end(), cnt.begin() + (int64_t)t * B);
    });
    // bucket b holds the entries of part 0, then part 1, ... that fall in it
    std::vector<int64_t> at((size_t)T * (size_t)B), edge((size_t)B + 1);
    int64_t o = 0;
    for (int b = 0; b < B; ++b) {
        edge[(size_t)b] = o;
        for (int t = 0; t < T; ++t) {
            at[(size_t)t * B + b] = o;
            o += cnt[(size_t)t * B + b];
        }
    }
    edge[(size_t)B] = o;
    parallel_parts(T, [&](int t) {
        std::vector<E>& p = parts[(size_t)t];
        const std::vector<uint8_t>& k = bk[(size_t)t];
        int64_t* a = &at[(size_t)t * B];
        for (size_t r = 0; r < p.size(); ++r) run[(size_t)a[k[r]]++] = p[r];
        std::vector<E>().swap(p);
    });
    parallel_parts(B, [&](int b) {
        std::sort(run.begin() + edge[(size_t)b], run.begin() + edge[(size_t)b + 1], before);
    });
    return run;
}

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

// Inside, maxima are numbered by height (rank 0 the lowest), so comparing two
// maxima is comparing two integers; rank and inv map to and from the caller's
// indices.
struct Graph {
    bool minima;
    std::vector<Node> mx;
    Buf<Node> sd;
    std::vector<int32_t> rank, inv;
    std::vector<double> hr;  // height by rank
    const int32_t* off;
    Buf<int32_t> arc;  // maxima ranks
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
    G->off = g->arc_offsets;
    if (g->arc_offsets[0] != 0) return false;
    std::atomic<bool> bad{false};
    parallel_for(g->nsad, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
            G->sd[(size_t)i] = Node{sgn * (double)g->sad_values[i], g->saddles[i]};
            if (g->arc_offsets[i + 1] < g->arc_offsets[i]) bad.store(true, std::memory_order_relaxed);
        }
    });
    if (bad.load()) return false;
    const int64_t narc = g->arc_offsets[g->nsad];
    if (narc > 0 && !g->arc_maxima) return false;
    const size_t nmax = G->mx.size();
    {
        struct Key {
            Node n;
            int32_t j;
        };
        std::vector<Key> k(nmax);
        for (size_t j = 0; j < nmax; ++j) k[j] = Key{G->mx[j], (int32_t)j};
        const bool minima = G->minima;
        parallel_sort(k, [minima](const Key& a, const Key& b) { return higher(b.n, a.n, minima); });
        G->inv.resize(nmax);
        for (size_t r = 0; r < nmax; ++r) G->inv[r] = k[r].j;
    }
    G->rank.resize(nmax);
    G->hr.resize(nmax);
    for (size_t r = 0; r < nmax; ++r) {
        G->rank[(size_t)G->inv[r]] = (int32_t)r;
        G->hr[r] = G->mx[(size_t)G->inv[r]].h;
    }
    G->arc.resize((size_t)narc);
    // arc endpoints to ranks: a bucket table over the top bits of the ids
    // narrows each binary search to the maxima of one bucket
    const int32_t top = nmax ? g->maxima[nmax - 1] : 0;
    int shift = 0;
    while (shift < 31 && (int64_t(top) >> shift) >= 65536) ++shift;
    const int64_t nb = (int64_t(top) >> shift) + 2;
    std::vector<int32_t> first((size_t)nb, (int32_t)nmax);
    for (int64_t j = (int64_t)nmax - 1; j >= 0; --j) first[(size_t)(g->maxima[j] >> shift)] = (int32_t)j;
    for (int64_t b = nb - 2; b >= 0; --b) first[(size_t)b] = std::min(first[(size_t)b], first[(size_t)b + 1]);
    parallel_for(narc, [&](int64_t k0, int64_t k1) {
        for (int64_t k = k0; k < k1; ++k) {
            const int32_t id = g->arc_maxima[k];
            const int64_t b = id >= 0 && id <= top ? (int64_t(id) >> shift) : -1;
            const int32_t* lo = g->maxima + (b >= 0 ? first[(size_t)b] : 0);
            const int32_t* hi = g->maxima + (b >= 0 ? first[(size_t)b + 1] : 0);
            const int32_t* p = std::lower_bound(lo, hi, id);
            if (b < 0 || p == hi || *p != id) {  // not a maximum
                bad.store(true, std::memory_order_relaxed);
                return;
            }
            G->arc[(size_t)k] = G->rank[(size_t)(p - g->maxima)];
        }
    });
    return !bad.load();
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

// Saddles that survive bundling (flags per saddle).  Every (lower maximum,
// higher maximum, saddle) record goes to the part of the maxima range its
// lower maximum falls in; each part is then grouped by lower maximum (a
// counting sort) and, per lower maximum, the highest saddle of each higher
// partner is kept.  No step shares a counter between threads.
std::vector<char> bundle(const Graph& G)
{
    const int64_t nsad = (int64_t)G.sd.size(), nmax = (int64_t)G.mx.size();
    std::vector<char> keep((size_t)nsad, 0);
    const unsigned hw = std::thread::hardware_concurrency();
    const int T = nsad < 32768 ? 1 : (int)std::max(1u, std::min(hw, 16u));
    struct Rec {
        int32_t a, b, s;  // lower and higher maximum (ranks), saddle
    };
    // part j holds the lower maxima a with j <= a T / nmax < j + 1
    auto part_of = [&](int32_t a) { return (int)((int64_t)a * T / nmax); };
    auto part_lo = [&](int j) { return (int32_t)(((int64_t)j * nmax + T - 1) / T); };
    // records[t][j]: thread t's records of part j, in saddle order
    std::vector<std::vector<std::vector<Rec>>> records((size_t)T, std::vector<std::vector<Rec>>((size_t)T));
    parallel_parts(T, [&](int t) {
        std::vector<int32_t> row;
        std::vector<std::vector<Rec>>& out = records[(size_t)t];
        for (int64_t i = nsad * t / T; i < nsad * (t + 1) / T; ++i) {
            row.assign(G.arc.begin() + G.off[i], G.arc.begin() + G.off[i + 1]);
            const int k = distinct(row.data(), (int)row.size());
            if (k < 2) keep[(size_t)i] = 1;  // no pair shares it
            for (int x = 0; x < k; ++x)
                for (int y = 0; y < k; ++y)
                    if (row[(size_t)x] < row[(size_t)y])
                        out[(size_t)part_of(row[(size_t)x])].push_back(Rec{row[(size_t)x], row[(size_t)y], (int32_t)i});
        }
    });
    parallel_parts(T, [&](int j) {
        const int32_t lo = part_lo(j), hi = part_lo(j + 1);
        // group the part's records by lower maximum
        std::vector<int64_t> start((size_t)(hi - lo) + 1, 0);
        for (int t = 0; t < T; ++t)
            for (const Rec& r : records[(size_t)t][(size_t)j]) ++start[(size_t)(r.a - lo) + 1];
        for (int32_t a = lo; a < hi; ++a) start[(size_t)(a - lo) + 1] += start[(size_t)(a - lo)];
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        std::vector<Rec> g((size_t)start.back());
        for (int t = 0; t < T; ++t) {
            std::vector<Rec>& v = records[(size_t)t][(size_t)j];
            for (const Rec& r : v) g[(size_t)fill[(size_t)(r.a - lo)]++] = r;
            std::vector<Rec>().swap(v);
        }
        // per lower maximum, the highest saddle of each higher partner
        std::vector<int32_t> best((size_t)nmax, -1);
        for (int32_t a = lo; a < hi; ++a) {
            const int64_t r0 = start[(size_t)(a - lo)], r1 = start[(size_t)(a - lo) + 1];
            for (int64_t r = r0; r < r1; ++r) {
                int32_t& b = best[(size_t)g[(size_t)r].b];
                const int32_t s = g[(size_t)r].s;
                if (b < 0 || higher(G.sd[(size_t)s], G.sd[(size_t)b], G.minima)) b = s;
            }
            for (int64_t r = r0; r < r1; ++r) {
                int32_t& b = best[(size_t)g[(size_t)r].b];
                if (b >= 0) __atomic_store_n(&keep[(size_t)b], (char)1, __ATOMIC_RELAXED);
                b = -1;
            }
        }
    });
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
    // the same without path halving, for readers running side by side
    int32_t root_const(int32_t m) const
    {
        while (parent[(size_t)m] != m) m = parent[(size_t)m];
        return m;
    }
};

// A queue entry: the cost when queued, the saddle's height and id (for the
// tie-break), the saddle, and for a saddle with two distinct maxima both of
// them (m1 < 0 marks a saddle whose row must be read again).
struct Entry {
    double cost;
    double sh;
    int32_t sid;
    int32_t sad;
    int32_t m0, m1;
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
        const bool minima = G.minima;
        // saddle a strictly below saddle b, from the heights the entries carry
        auto lower_sad = [minima](const Entry& a, const Entry& b) {
            if (a.sh != b.sh) return a.sh < b.sh;
            return minima ? a.sid > b.sid : a.sid < b.sid;
        };
        // (cost, saddle order): lower costs first, lower saddles first among equal costs
        auto before = [&](const Entry& a, const Entry& b) {
            if (a.cost != b.cost) return a.cost < b.cost;
            return lower_sad(a, b);
        };
        auto after = [&](const Entry& a, const Entry& b) { return before(b, a); };
        // initial entries (no merges yet: every maximum is its own root), one
        // sorted run; each thread fills its own part in saddle order
        const unsigned hw = std::thread::hardware_concurrency();
        const int T = nsad < 32768 ? 1 : (int)std::max(1u, std::min(hw, 16u));
        std::vector<std::vector<Entry>> parts((size_t)T);
        parallel_parts(T, [&](int t) {
            {
                std::vector<int32_t> ms;
                std::vector<Entry>& out = parts[(size_t)t];
                const int64_t i0 = (int64_t)nsad * t / T, i1 = (int64_t)nsad * (t + 1) / T;
                for (int64_t i = i0; i < i1; ++i) {
                    if (!live[(size_t)i]) continue;
                    ms.assign(G.arc.begin() + G.off[i], G.arc.begin() + G.off[i + 1]);
                    const int n = distinct(ms.data(), (int)ms.size());
                    if (n < 2) continue;
                    ms.resize((size_t)n);
                    std::sort(ms.begin(), ms.end(), [](int32_t a, int32_t b) { return a > b; });
                    const double cost = G.hr[(size_t)ms[1]] - G.sd[(size_t)i].h;
                    if (n == 2 && cost > threshold) continue;  // can never become cheaper
                    // two maxima inline; more: -(their count), placed after the sort
                    out.push_back(Entry{cost, G.sd[(size_t)i].h, G.sd[(size_t)i].id, (int32_t)i, ms[0],
                                        n == 2 ? ms[1] : -n});
                }
            }
        });
        Buf<Entry> run = sorted_run(parts, before);
        // maxima of the saddles with more than two, copied in run order: the
        // loop then reads them front to back (m0 becomes the offset)
        Buf<int32_t> many;
        {
            // each thread's chunk of the run: its share of the rows, then
            // the rows at the chunk's offset
            const int64_t nr = (int64_t)run.size();
            const int TR = nr < 32768 ? 1 : T;
            std::vector<int64_t> base((size_t)TR + 1, 0);
            parallel_parts(TR, [&](int t) {
                int64_t c = 0;
                for (int64_t r = nr * t / TR; r < nr * (t + 1) / TR; ++r)
                    c += run[(size_t)r].m1 < 0 ? -run[(size_t)r].m1 : 0;
                base[(size_t)t + 1] = c;
            });
            for (int t = 0; t < TR; ++t) base[(size_t)t + 1] += base[(size_t)t];
            many.resize((size_t)base[(size_t)TR]);
            parallel_parts(TR, [&](int t) {
                std::vector<int32_t> ms;
                int64_t o = base[(size_t)t];
                for (int64_t r = nr * t / TR; r < nr * (t + 1) / TR; ++r) {
                    Entry& e = run[(size_t)r];
                    if (e.m1 >= 0) continue;
                    ms.assign(G.arc.begin() + G.off[e.sad], G.arc.begin() + G.off[e.sad + 1]);
                    const int n = distinct(ms.data(), (int)ms.size());
                    std::copy(ms.begin(), ms.begin() + n, many.begin() + o);
                    e.m0 = (int32_t)o;
                    o += n;
                }
            });
        }
        std::priority_queue<Entry, std::vector<Entry>, decltype(after)> heap(after);  // reinserted entries
        size_t pos = 0;
        auto empty = [&]() { return pos == run.size() && heap.empty(); };
        auto top = [&]() -> const Entry& {
            if (pos == run.size()) return heap.top();
            if (heap.empty() || before(run[pos], heap.top())) return run[pos];
            return heap.top();
        };
        auto pop = [&]() {
            Entry e;
            if (pos < run.size() && (heap.empty() || before(run[pos], heap.top()))) {
                e = run[pos++];
            } else {
                e = heap.top();
                heap.pop();
            }
            return e;
        };
        auto record = [&](int32_t i, int32_t m, double cost) {
            pair_saddle[np] = i;
            pair_max[np] = G.inv[(size_t)m];
            pair_cost[np] = cost;
            ++np;
        };
        std::vector<int32_t> ms;
        constexpr size_t kAhead = 16;  // prefetch distance along the run
        while (!empty()) {
            if (pos + kAhead < run.size()) {
                const Entry& f = run[pos + kAhead];
                if (f.m1 >= 0) {
                    __builtin_prefetch(&U.parent[(size_t)f.m0]);
                    __builtin_prefetch(&U.parent[(size_t)f.m1]);
                } else {
                    for (int k = 0; k < -f.m1; ++k) __builtin_prefetch(&U.parent[(size_t)many[(size_t)f.m0 + k]]);
                }
            }
            Entry e = pop();
            const int32_t i = e.sad;
            if (e.m1 >= 0) {
                // two maxima: their current roots are all the row can give
                int32_t a = U.root(e.m0), b = U.root(e.m1);
                if (a == b) continue;  // joins a single maximum now: no cost
                if (b > a) std::swap(a, b);
                const double cost = G.hr[(size_t)b] - e.sh;
                if (cost > threshold) continue;  // discarded
                if (!empty() && cost > top().cost) {  // the queue holds cheaper saddles
                    e.cost = cost;
                    heap.push(e);
                    continue;
                }
                U.parent[(size_t)b] = a;
                record(i, b, cost);
                live[(size_t)i] = 0;  // the cancelled saddle leaves the graph
                continue;
            }
            // more than two maxima: the cost needs only the two highest of
            // their current roots
            const int32_t* mm = many.data() + e.m0;
            int32_t r0 = -1, r1 = -1;
            for (int k = 0; k < -e.m1; ++k) {
                const int32_t r = U.root(mm[k]);
                if (r > r0) {
                    r1 = r0;
                    r0 = r;
                } else if (r < r0 && r > r1) {
                    r1 = r;
                }
            }
            if (r1 < 0) continue;  // joins a single maximum now: no cost
            const double cost = G.hr[(size_t)r1] - e.sh;
            if (cost > threshold) continue;  // discarded
            if (!empty() && cost > top().cost) {  // the queue holds cheaper saddles
                e.cost = cost;
                heap.push(e);
                continue;
            }
            // cancelled: the distinct roots, highest first
            ms.clear();
            for (int k = 0; k < -e.m1; ++k) ms.push_back(U.root(mm[k]));
            const int n = distinct(ms.data(), (int)ms.size());
            ms.resize((size_t)n);
            std::sort(ms.begin(), ms.end(), [](int32_t a, int32_t b) { return a > b; });
            for (int k = 1; k < n; ++k) {  // all but the highest merge into it
                U.parent[(size_t)ms[(size_t)k]] = ms[0];
                record(i, ms[(size_t)k], cost);
            }
            live[(size_t)i] = 0;  // the cancelled saddle leaves the graph
        }
    }
    *n_pairs = np;
    // rows of the simplified graph: every live saddle, its distinct maxima
    // (sizes first, then the rows, both in parallel)
    std::vector<int32_t> len(nsad, 0);
    auto row_of = [&](size_t i, std::vector<int32_t>& ms) {
        ms.clear();
        for (int32_t k = G.off[i]; k < G.off[i + 1]; ++k)
            ms.push_back(G.mx[(size_t)G.inv[(size_t)U.root_const(G.arc[(size_t)k])]].id);
        std::sort(ms.begin(), ms.end());
        ms.erase(std::unique(ms.begin(), ms.end()), ms.end());
    };
    parallel_for((int64_t)nsad, [&](int64_t i0, int64_t i1) {
        std::vector<int32_t> ms;
        for (int64_t i = i0; i < i1; ++i)
            if (live[(size_t)i]) {
                row_of((size_t)i, ms);
                len[(size_t)i] = (int32_t)ms.size();
            }
    });
    out_offsets[0] = 0;
    for (size_t i = 0; i < nsad; ++i) out_offsets[i + 1] = out_offsets[i] + len[i];
    parallel_for((int64_t)nsad, [&](int64_t i0, int64_t i1) {
        std::vector<int32_t> ms;
        for (int64_t i = i0; i < i1; ++i)
            if (live[(size_t)i]) {
                row_of((size_t)i, ms);
                std::copy(ms.begin(), ms.end(), out_arcs + out_offsets[i]);
            }
    });
    for (size_t j = 0; j < G.mx.size(); ++j) max_rep[j] = G.inv[(size_t)U.root_const(G.rank[j])];
    return EG_OK;
}
