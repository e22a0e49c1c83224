// Host planning: everything that decides shapes, orders and launch
// descriptors.  No amplitude arithmetic happens here; the device kernels do
// all of it.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <functional>
#include <limits>
#include <numeric>
#include <queue>
#include <random>
#include <unordered_set>

#include "internal.h"

namespace tns {

using cd = std::complex<double>;

// ----------------------------------------------------------------------------
// circuit validation and graph

static cd gm(const tns_gate &g, int r, int c, int dim) {
    int i = r * dim + c;
    return cd(g.m[2 * i], g.m[2 * i + 1]);
}

static bool unitary(const tns_gate &g, int dim, double tol) {
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
            cd acc = 0;
            for (int k = 0; k < dim; ++k) acc += std::conj(gm(g, k, i, dim)) * gm(g, k, j, dim);
            if (std::abs(acc - (i == j ? 1.0 : 0.0)) > tol) return false;
        }
    return true;
}

void validate_and_build(const tns_circuit_desc *desc, Circuit &c) {
    if (!desc) fail(TNS_E_INVALID_ARG, "circuit descriptor is NULL");
    const int n = desc->n_qubits;
    if (n < 2 || n > TNS_MAX_QUBITS)
        fail(TNS_E_BAD_CIRCUIT, "n_qubits must be in [2, " + std::to_string(TNS_MAX_QUBITS) + "]");
    if (desc->n_edges < 0 || (desc->n_edges > 0 && !desc->edges))
        fail(TNS_E_INVALID_ARG, "bad edge array");
    if (desc->n_gates < 0 || (desc->n_gates > 0 && !desc->gates))
        fail(TNS_E_INVALID_ARG, "bad gate array");
    c.n = n;
    c.g = Graph{};
    c.g.n = n;
    c.g.legs.assign(n, {});
    for (int e = 0; e < desc->n_edges; ++e) {
        int a = desc->edges[2 * e], b = desc->edges[2 * e + 1];
        if (a < 0 || b < 0 || a >= n || b >= n || a == b)
            fail(TNS_E_BAD_CIRCUIT, "edge " + std::to_string(e) + " has a bad endpoint");
        std::pair<int, int> key{std::min(a, b), std::max(a, b)};
        if (c.g.index.count(key)) fail(TNS_E_BAD_CIRCUIT, "duplicate edge " + std::to_string(e));
        c.g.index[key] = e;
        c.g.edges.push_back(key);
        c.g.legs[a].push_back(e);
        c.g.legs[b].push_back(e);
    }
    for (int q = 0; q < n; ++q) {
        std::sort(c.g.legs[q].begin(), c.g.legs[q].end());
        if ((int)c.g.legs[q].size() > kMaxDeg)
            fail(TNS_E_UNSUPPORTED, "qubit " + std::to_string(q) + " has more than " +
                                        std::to_string(kMaxDeg) + " couplers");
    }
    c.n_real_edges = (int)c.g.edges.size();
    c.n_open = 0;
    c.open_qubits.clear();
    c.gates.assign(desc->gates, desc->gates + desc->n_gates);
    c.max_cycle = 0;
    for (int i = 0; i < desc->n_gates; ++i) {
        const tns_gate &g = c.gates[i];
        if (g.q0 < 0 || g.q0 >= n) fail(TNS_E_BAD_CIRCUIT, "gate " + std::to_string(i) + ": q0 out of range");
        if (g.cycle < 0) fail(TNS_E_BAD_CIRCUIT, "gate " + std::to_string(i) + ": negative cycle");
        c.max_cycle = std::max(c.max_cycle, g.cycle);
        for (int k = 0; k < 32; ++k)
            if (!std::isfinite(g.m[k])) fail(TNS_E_BAD_CIRCUIT, "gate " + std::to_string(i) + ": non-finite entry");
        if (g.q1 < 0) {
            if (!unitary(g, 2, 1e-8)) fail(TNS_E_BAD_CIRCUIT, "gate " + std::to_string(i) + " is not unitary");
        } else {
            if (g.q1 >= n || g.q1 == g.q0) fail(TNS_E_BAD_CIRCUIT, "gate " + std::to_string(i) + ": bad q1");
            if (c.g.edge_id(g.q0, g.q1) < 0)
                fail(TNS_E_BAD_CIRCUIT, "gate " + std::to_string(i) + " acts on a pair that is not an edge");
            if (!unitary(g, 4, 1e-8)) fail(TNS_E_BAD_CIRCUIT, "gate " + std::to_string(i) + " is not unitary");
        }
    }
}

// Operator Schmidt rank of a two-qubit gate, i.e. the number of nonzero
// singular values of O reshaped to [(s0' s0), (s1' s1)] (Eq. (2)).  Local
// single-qubit factors do not change it, so the rank of the base gate is the
// rank of its fused form.  Complete-pivoting elimination with a relative
// threshold well above rounding and well below any physical singular value.
int operator_schmidt_rank(const double *m) {
    cd a[4][4];
    for (int a0p = 0; a0p < 2; ++a0p)
        for (int b0p = 0; b0p < 2; ++b0p)
            for (int a0 = 0; a0 < 2; ++a0)
                for (int b0 = 0; b0 < 2; ++b0) {
                    int r = a0p * 2 + b0p, c = a0 * 2 + b0;   // O[(a' b'), (a b)]
                    int i = r * 4 + c;
                    a[a0p * 2 + a0][b0p * 2 + b0] = cd(m[2 * i], m[2 * i + 1]);
                }
    double scale = 0;
    for (auto &row : a)
        for (auto &x : row) scale = std::max(scale, std::abs(x));
    if (scale == 0) return 0;
    int rank = 0;
    bool rused[4] = {}, cused[4] = {};
    for (int step = 0; step < 4; ++step) {
        int pr = -1, pc = -1;
        double best = 0;
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c)
                if (!rused[r] && !cused[c] && std::abs(a[r][c]) > best) {
                    best = std::abs(a[r][c]);
                    pr = r;
                    pc = c;
                }
        if (pr < 0 || best <= 1e-10 * scale) break;
        ++rank;
        rused[pr] = cused[pc] = true;
        for (int r = 0; r < 4; ++r) {
            if (rused[r]) continue;
            cd f = a[r][pc] / a[pr][pc];
            for (int c = 0; c < 4; ++c) a[r][c] -= f * a[pr][c];
        }
    }
    return rank;
}

// ----------------------------------------------------------------------------
// path search (supplement: score, Cost, Algorithm 1)

namespace {

struct QMask {
    uint64_t w[2] = {0, 0};
    void set(int q) { w[q >> 6] |= 1ULL << (q & 63); }
    bool has(int q) const { return (w[q >> 6] >> (q & 63)) & 1ULL; }
    bool operator==(const QMask &o) const { return w[0] == o.w[0] && w[1] == o.w[1]; }
};
struct QMaskHash {
    size_t operator()(const QMask &m) const {
        uint64_t h = m.w[0] * 0x9E3779B97F4A7C15ULL ^ (m.w[1] + 0x632BE59BD9B4E019ULL + (m.w[0] << 6));
        return (size_t)(h ^ (h >> 29));
    }
};

// Graph restricted to bonds of dimension > 1 (a bond of dimension 1 neither
// costs anything nor connects anything).
struct PG {
    int n = 0;
    std::vector<std::pair<int, int>> edges;
    std::vector<double> d;
    std::vector<std::vector<int>> legs;   // per node: filtered edge ids
    std::vector<std::vector<int>> nbr;    // per node: neighbours
};

// A bond whose second endpoint is n is a dangling (open) leg of its first
// endpoint: it is never contracted and connects nothing.
PG make_pg(int n, const std::vector<std::pair<int, int>> &edges, const std::vector<double> &dims) {
    PG g;
    g.n = n;
    g.legs.assign(n + 1, {});
    g.nbr.assign(n + 1, {});
    for (size_t e = 0; e < edges.size(); ++e) {
        if (!(dims[e] > 1.0)) continue;
        int id = (int)g.edges.size();
        g.edges.push_back(edges[e]);
        g.d.push_back(dims[e]);
        g.legs[edges[e].first].push_back(id);
        if (edges[e].second == n) continue;
        g.legs[edges[e].second].push_back(id);
        g.nbr[edges[e].first].push_back(edges[e].second);
        g.nbr[edges[e].second].push_back(edges[e].first);
    }
    for (auto &v : g.nbr) {
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
    }
    return g;
}

// Score of a fixed order: sum of Cost(C^{set}, C^{j}) with Cost the product
// of the dimensions of every bond carried by either tensor.
double order_score(const PG &g, const std::vector<int> &order, double *peak, int *max_rank) {
    std::vector<char> in(g.n + 1, 0), open(g.edges.size(), 0);
    double size = 1, score = 0, pk = 0;
    int rank = 0, mr = 0;
    for (size_t m = 0; m < order.size(); ++m) {
        int j = order[m];
        double K = 1, N = 1;
        int shared = 0, fresh = 0;
        for (int e : g.legs[j]) {
            int other = g.edges[e].first == j ? g.edges[e].second : g.edges[e].first;
            if (in[other]) { K *= g.d[e]; ++shared; } else { N *= g.d[e]; ++fresh; }
        }
        if (m > 0) score += size * N;
        size = (m == 0) ? N : size / K * N;
        rank = (m == 0) ? fresh : rank - shared + fresh;
        in[j] = 1;
        pk = std::max(pk, size);
        mr = std::max(mr, rank);
    }
    if (peak) *peak = pk;
    if (max_rank) *max_rank = mr;
    return score;
}

// Greedy linear path: from every start, repeatedly absorb the neighbouring
// tensor with the least step cost (criterion 0) or the least resulting size
// (criterion 1); the best full path over both criteria and all starts wins.
PathResult greedy(const PG &g) {
    PathResult best;
    best.score = std::numeric_limits<double>::infinity();
    const int n = g.n;
    for (int crit = 0; crit < 2; ++crit)
    for (int start = 0; start < n; ++start) {
        std::vector<char> in(n + 1, 0);
        std::vector<int> adj(n + 1, 0), order{start};
        in[start] = 1;
        double size = 1, score = 0, peak = 0;
        int rank = 0, mr = 0;
        for (int e : g.legs[start]) { size *= g.d[e]; ++rank; }
        peak = size;
        mr = rank;
        for (int x : g.nbr[start]) adj[x]++;
        for (int m = 1; m < n; ++m) {
            bool any_adj = false;
            for (int j = 0; j < n; ++j)
                if (!in[j] && adj[j]) { any_adj = true; break; }
            int bj = -1, bshared = 0, bfresh = 0;
            double bcost = 0, bsize = 0;
            for (int j = 0; j < n; ++j) {
                if (in[j] || (any_adj && !adj[j])) continue;
                double K = 1, N = 1;
                int shared = 0, fresh = 0;
                for (int e : g.legs[j]) {
                    int other = g.edges[e].first == j ? g.edges[e].second : g.edges[e].first;
                    if (in[other]) { K *= g.d[e]; ++shared; } else { N *= g.d[e]; ++fresh; }
                }
                double cost = size * N, ns = size / K * N;
                bool better = crit == 0 ? (cost < bcost || (cost == bcost && ns < bsize))
                                        : (ns < bsize || (ns == bsize && cost < bcost));
                if (bj < 0 || better) {
                    bj = j; bcost = cost; bsize = ns; bshared = shared; bfresh = fresh;
                }
            }
            in[bj] = 1;
            order.push_back(bj);
            for (int x : g.nbr[bj]) adj[x]++;
            score += bcost;
            size = bsize;
            rank += bfresh - bshared;
            peak = std::max(peak, size);
            mr = std::max(mr, rank);
            if (score > best.score) break;
        }
        if ((int)order.size() == n &&
            (score < best.score || (score == best.score && peak < best.peak))) {
            best.order = order;
            best.score = score;
            best.peak = peak;
            best.max_rank = mr;
        }
    }
    best.states = n;
    best.complete = true;
    return best;
}

struct Node {
    QMask set;
    double score;
    int32_t parent;
    int16_t q, c, m, pad;
};

struct QItem {
    double score;
    int32_t m;
    int64_t seq;
    int32_t node;
};
struct QCmp {
    // std::priority_queue pops the "largest": order so that the least score,
    // then the longest path, then the earliest push comes out first.
    bool operator()(const QItem &a, const QItem &b) const {
        if (a.score != b.score) return a.score > b.score;
        if (a.m != b.m) return a.m < b.m;
        return a.seq > b.seq;
    }
};

// Algorithm 1 of the supplement: best-first search over partial paths, keyed
// by the set of absorbed qubits, with the three assumptions restricting the
// start (boundary qubits), the rank of intermediates (<= M) and connectivity
// (connected, or connected plus one isolated qubit that the next step joins).
PathResult algorithm1(const PG &g, int max_rank, bool assumptions, int64_t max_states,
                      double upper, const PathResult *fallback, double max_size) {
    const int n = g.n;
    std::vector<Node> arena;
    arena.reserve(1 << 16);
    std::priority_queue<QItem, std::vector<QItem>, QCmp> pq;
    std::unordered_set<QMask, QMaskHash> visited;
    int64_t seq = 0;

    int maxdeg = 0;
    for (int v = 0; v < n; ++v) maxdeg = std::max<int>(maxdeg, (int)g.nbr[v].size());
    for (int v = 0; v < n; ++v) {
        bool boundary = !assumptions || (int)g.nbr[v].size() < maxdeg;
        if (!boundary) continue;
        if (max_size > 0) {
            double sz = 1;
            for (int e : g.legs[v]) sz *= g.d[e];
            if (sz > max_size * (1 + 1e-12)) continue;
        }
        Node nd;
        nd.set.set(v);
        nd.score = 0;
        nd.parent = -1;
        nd.q = (int16_t)v;
        nd.c = -1;
        nd.m = 1;
        arena.push_back(nd);
        pq.push({0.0, 1, seq++, (int32_t)arena.size() - 1});
    }
    PathResult res;
    std::vector<char> in(n + 1, 0), open(g.edges.size()), adj(n + 1), near(n + 1);
    while (!pq.empty()) {
        QItem it = pq.top();
        pq.pop();
        const Node cur = arena[it.node];
        if (visited.count(cur.set)) continue;
        visited.insert(cur.set);
        res.states++;
        if (cur.m == n) {
            std::vector<int> order;
            for (int i = it.node; i >= 0; i = arena[i].parent) order.push_back(arena[i].q);
            std::reverse(order.begin(), order.end());
            res.order = order;
            res.score = cur.score;
            order_score(g, order, &res.peak, &res.max_rank);
            res.complete = true;
            return res;
        }
        if (max_states > 0 && res.states >= max_states) break;
        for (int v = 0; v < n; ++v) in[v] = cur.set.has(v);
        double size = 1;
        int rank = 0;
        for (size_t e = 0; e < g.edges.size(); ++e) {
            open[e] = in[g.edges[e].first] != in[g.edges[e].second];
            if (open[e]) { size *= g.d[e]; ++rank; }
        }
        // candidate generation
        std::fill(adj.begin(), adj.end(), 0);
        for (int v = 0; v < n; ++v)
            if (in[v])
                for (int x : g.nbr[v])
                    if (!in[x]) adj[x] = 1;
        auto consider = [&](int j) {
            double K = 1, N = 1;
            int shared = 0, fresh = 0;
            for (int e : g.legs[j]) {
                if (open[e]) { K *= g.d[e]; ++shared; } else { N *= g.d[e]; ++fresh; }
            }
            int nrank = rank - shared + fresh;
            if (assumptions && nrank > max_rank) return;
            // size-aware bound: no intermediate above max_size elements
            if (max_size > 0 && size / K * N > max_size * (1 + 1e-12)) return;
            double ns = cur.score + size * N;
            if (ns > upper) return;
            Node nd;
            nd.set = cur.set;
            nd.set.set(j);
            if (visited.count(nd.set)) return;
            nd.score = ns;
            nd.parent = it.node;
            nd.q = (int16_t)j;
            nd.c = (int16_t)(shared > 0 ? -1 : j);   // conn(): -1 when joined to the set
            nd.m = (int16_t)(cur.m + 1);
            arena.push_back(nd);
            pq.push({ns, nd.m, seq++, (int32_t)arena.size() - 1});
        };
        if (!assumptions) {
            for (int j = 0; j < n; ++j)
                if (!in[j]) consider(j);
        } else if (cur.c < 0) {
            std::fill(near.begin(), near.end(), 0);
            for (int j = 0; j < n; ++j)
                if (adj[j]) {
                    consider(j);
                    for (int x : g.nbr[j])
                        if (!in[x] && !adj[x]) near[x] = 1;
                }
            for (int j = 0; j < n; ++j)
                if (near[j]) consider(j);      // the single isolated qubit (assumption 3)
        } else {
            const int iso = cur.c;
            for (int j = 0; j < n; ++j) {
                if (!adj[j]) continue;
                bool to_iso = false, to_main = false;
                for (int x : g.nbr[j]) {
                    if (x == iso) to_iso = true;
                    else if (in[x]) to_main = true;
                }
                if (to_iso && to_main) consider(j);
            }
        }
    }
    // budget exhausted or no admissible path below the bound: keep the fallback
    if (fallback) {
        PathResult f = *fallback;
        f.states = res.states;
        f.complete = pq.empty();   // empty queue: nothing admissible beats the fallback
        return f;
    }
    fail(TNS_E_BAD_PATH, "path search found no admissible path");
}

}  // namespace

PathResult path_search(int n, const std::vector<std::pair<int, int>> &edges,
                       const std::vector<double> &dims, int mode, int max_rank,
                       bool assumptions, int64_t max_states, double max_size) {
    PG g = make_pg(n, edges, dims);
    PathResult gr = greedy(g);
    if (mode == TNS_PATH_GREEDY) return gr;
    if (mode != TNS_PATH_ALGORITHM1) fail(TNS_E_INVALID_ARG, "unknown path mode");
    int M = max_rank > 0 ? max_rank : gr.max_rank;
    // the greedy path bounds the search only when it is itself admissible
    const bool greedy_fits = !(max_size > 0) || gr.peak <= max_size * (1 + 1e-12);
    double upper = assumptions && greedy_fits ? gr.score : std::numeric_limits<double>::infinity();
    // an exhausted state budget returns the greedy path, marked incomplete
    // (with the assumptions off the search is exact and has no other bound)
    PathResult r = algorithm1(g, M, assumptions, max_states > 0 ? max_states : 4000000, upper, &gr, max_size);
    r.max_rank = std::max(r.max_rank, 0);
    // report the rank bound actually used by the search
    if (assumptions) r.max_rank = M;
    return r;
}

double path_score(int n, const std::vector<std::pair<int, int>> &edges,
                  const std::vector<double> &dims, const std::vector<int> &order, double *peak,
                  int *max_rank) {
    PG g = make_pg(n, edges, dims);
    return order_score(g, order, peak, max_rank);
}

// ----------------------------------------------------------------------------
// fusion of single-qubit gates into two-qubit gates ("Single-qubit gates are
// absorbed", gate-operation paragraph) and the two-sided split

namespace {

int make_chain(Plan &p, std::vector<int> &pending) {
    if (pending.empty()) return -1;
    int id = (int)p.chain_off.size();
    p.chain_off.push_back((int32_t)p.chain_flat.size());
    p.chain_len.push_back((int32_t)pending.size());
    for (int gi : pending) p.chain_flat.push_back(gi);
    pending.clear();
    return id;
}

// Fuse one side's gates (given in time order).  Returns the fused ops in time
// order (indices into p.fuse).  Leftover single-qubit gates go to the
// boundary chains: on the ket side into the last two-qubit gate on that qubit
// (or the initial product state if there is none), on the bra side into the
// final product state <s|.
std::vector<int> fuse_side(Plan &p, const std::vector<int> &gids, bool bra) {
    const Circuit &c = p.circ;
    std::vector<std::vector<int>> pending(c.n);
    std::vector<int> last(c.n, -1), out;
    for (int gi : gids) {
        const tns_gate &g = c.gates[gi];
        if (g.q1 < 0) {
            pending[g.q0].push_back(gi);
            continue;
        }
        FuseDesc f{};
        f.gate = gi;
        f.pre0 = make_chain(p, pending[g.q0]);
        f.pre1 = make_chain(p, pending[g.q1]);
        f.post0 = f.post1 = -1;
        f.transpose = bra ? 1 : 0;
        f.chi = operator_schmidt_rank(g.m);
        out.push_back((int)p.fuse.size());
        p.fuse.push_back(f);
        last[g.q0] = last[g.q1] = out.back();
    }
    for (int q = 0; q < c.n; ++q) {
        if (pending[q].empty()) continue;
        if (!bra && last[q] >= 0) {
            FuseDesc &f = p.fuse[last[q]];
            int ch = make_chain(p, pending[q]);
            if (c.gates[f.gate].q0 == q) f.post0 = ch; else f.post1 = ch;
        } else {
            int ch = make_chain(p, pending[q]);
            (bra ? p.bra_final_chain : p.ket_init_chain)[q] = ch;
        }
    }
    return out;
}

int64_t shape_elems(const SiteShape &s) {
    int64_t v = 1;
    for (int i = 0; i < s.n; ++i) v *= s.d[i];
    return v;
}

// Bond-dimension bookkeeping of one side (Eqs. (3)-(6)).  A gate widens its
// bond by chi; the SVD of Eq. (5) can then keep at most min(rows, cols)
// singular values, rows = 2 * (product of the site's other bonds).  The
// smaller of the two sites' row counts bounds the kept rank; when it is
// below the widened bond the compression is planned on that site.  Exact
// zeros among the kept singular values (non-generic circuits) are kept as
// padding, so every bitstring shares one shape.
SideEvolution evolve_side(const Plan &p, const std::vector<int> &fused_ids, bool reverse) {
    const Circuit &c = p.circ;
    SideEvolution s;
    std::vector<int> dim(c.g.edges.size(), 1);
    // open legs: absent (1) on the ket side, the bra's free output bit (2)
    for (size_t e = c.n_real_edges; e < c.g.edges.size(); ++e) dim[e] = reverse ? 2 : 1;
    auto shape = [&](int q) {
        SiteShape sh{};
        sh.n = 1 + (int)c.g.legs[q].size();
        sh.d[0] = 2;
        for (size_t i = 0; i < c.g.legs[q].size(); ++i) sh.d[1 + i] = dim[c.g.legs[q][i]];
        return sh;
    };
    s.cap.assign(c.n, 2);
    for (int q = 0; q < c.n; ++q) s.cap[q] = shape_elems(shape(q));
    std::vector<int> order = fused_ids;
    if (reverse) std::reverse(order.begin(), order.end());
    for (int fid : order) {
        const FuseDesc &f = p.fuse[fid];
        const tns_gate &g = c.gates[f.gate];
        EvoOp op{};
        op.fused = fid;
        op.q0 = g.q0;
        op.q1 = g.q1;
        op.edge = c.g.edge_id(g.q0, g.q1);
        op.chi = f.chi;
        op.leg0 = c.g.leg_of(g.q0, op.edge);
        op.leg1 = c.g.leg_of(g.q1, op.edge);
        op.s0 = shape(g.q0);
        op.s1 = shape(g.q1);
        op.d_before = dim[op.edge];
        dim[op.edge] *= f.chi;
        op.d_grown = dim[op.edge];
        SiteShape g0 = shape(g.q0), g1 = shape(g.q1);
        s.cap[g.q0] = std::max(s.cap[g.q0], shape_elems(g0));
        s.cap[g.q1] = std::max(s.cap[g.q1], shape_elems(g1));
        int64_t r0 = shape_elems(g0) / op.d_grown, r1 = shape_elems(g1) / op.d_grown;
        int64_t r = std::min(r0, r1);
        if (r < op.d_grown) {
            op.comp = (r0 < r1 || (r0 == r1 && g.q0 < g.q1)) ? 0 : 1;
            dim[op.edge] = (int)r;
        } else {
            op.comp = -1;
        }
        op.d_after = dim[op.edge];
        s.ops.push_back(op);
    }
    s.bond = dim;
    for (int q = 0; q < c.n; ++q) s.final_shape.push_back(shape(q));
    return s;
}

}  // namespace

// ----------------------------------------------------------------------------
// step compilation

namespace {

// Merge adjacent axes that stay adjacent (stride[a] == stride[a+1]*size[a+1])
// and drop unit axes.
Gather compact(const std::vector<int64_t> &size, const std::vector<int64_t> &stride) {
    std::vector<int64_t> sz, st;
    for (size_t a = 0; a < size.size(); ++a) {
        if (size[a] == 1) continue;
        if (!sz.empty() && st.back() == stride[a] * size[a]) {
            sz.back() *= size[a];
            st.back() = stride[a];
        } else {
            sz.push_back(size[a]);
            st.push_back(stride[a]);
        }
    }
    if (sz.empty()) { sz.push_back(1); st.push_back(0); }
    if ((int)sz.size() > kMaxGatherDims)
        fail(TNS_E_UNSUPPORTED, "tensor has more than " + std::to_string(kMaxGatherDims) +
                                    " non-mergeable axes");
    Gather g{};
    g.n = (int)sz.size();
    for (int a = 0; a < g.n; ++a) { g.size[a] = sz[a]; g.stride[a] = st[a]; }
    return g;
}

// Fused-store tables (ScatterStore) of a GEMM step whose product, in its
// natural [M][N] order, the next step permutes with `g` (target axes with
// their natural strides).  Every target axis is a digit field of m or of n (an
// axis straddling the boundary is split in two); with power-of-two sizes the
// digit fields are bit fields, so f(m) = fa[m >> shift] + fb[m & mask] is
// exact.  Returns false where the tables do not apply.
bool build_scatter(const Gather &g, int64_t M, int64_t N, Step &s) {
    auto pow2 = [](int64_t x) { return x > 0 && (x & (x - 1)) == 0; };
    if (!pow2(M) || !pow2(N)) return false;
    std::vector<int64_t> ts(g.n);
    int64_t t = 1;
    for (int a = g.n - 1; a >= 0; --a) { ts[a] = t; t *= g.size[a]; }
    if (t != M * N) return false;
    struct Ax { int64_t stride, size, ts; };
    std::vector<Ax> am, an;   // digit fields of m (strides in rows) and of n
    for (int a = 0; a < g.n; ++a) {
        const int64_t st = g.stride[a], z = g.size[a];
        if (z == 1) continue;
        if (!pow2(z) || !pow2(st)) return false;
        if (st >= N) am.push_back({st / N, z, ts[a]});
        else if (st * z <= N) an.push_back({st, z, ts[a]});
        else {
            const int64_t zl = N / st;
            an.push_back({st, zl, ts[a]});
            am.push_back({1, z / zl, ts[a] * zl});
        }
    }
    auto f = [](const std::vector<Ax> &ax, int64_t x) {
        int64_t y = 0;
        for (const Ax &a : ax) y += ((x / a.stride) % a.size) * a.ts;
        return y;
    };
    int lg = 0;
    while (((int64_t)1 << lg) < M) ++lg;
    const int shift = lg / 2;
    const int64_t na = M >> shift, nb = (int64_t)1 << shift;
    if (na + nb + N > ((int64_t)1 << 23)) return false;
    s.sc_tab.resize(na + nb + N);
    for (int64_t h = 0; h < na; ++h) s.sc_tab[h] = f(am, h << shift);
    for (int64_t l = 0; l < nb; ++l) s.sc_tab[na + l] = f(am, l);
    for (int64_t n = 0; n < N; ++n) s.sc_tab[na + nb + n] = f(an, n);
    // Self-check.  Bounds: the largest entries add up to less than M*N, so
    // no store can leave the unit.  Semantics: decoding f(m) + g(n) over the
    // target axes must lead back to the natural index m*N + n (every pair
    // when M*N <= 2^16, else 4096 pairs and the corners).
    const int64_t *fa = s.sc_tab.data(), *fb = fa + na, *fg = fb + nb;
    const int64_t ma = *std::max_element(fa, fa + na), mb = *std::max_element(fb, fb + nb),
                  mg = *std::max_element(fg, fg + N);
    if (ma + mb + mg >= M * N) fail(TNS_E_BAD_PATH, "internal: fused store leaves the tensor");
    auto back = [&](int64_t m, int64_t n) {
        int64_t r = fa[m >> shift] + fb[m & (nb - 1)] + fg[n], x = 0;
        for (int a = g.n - 1; a >= 0; --a) {
            x += (r % g.size[a]) * g.stride[a];
            r /= g.size[a];
        }
        return x == m * N + n;
    };
    bool ok = back(0, 0) && back(M - 1, N - 1);
    if (M * N <= ((int64_t)1 << 16)) {
        for (int64_t m = 0; m < M && ok; ++m)
            for (int64_t n = 0; n < N && ok; ++n) ok = back(m, n);
    } else {
        uint64_t x = 0x9e3779b97f4a7c15ull;
        for (int i = 0; i < 4096 && ok; ++i) {
            x = x * 6364136223846793005ull + 1442695040888963407ull;
            ok = back((int64_t)((x >> 20) % (uint64_t)M), (int64_t)((x >> 8) % (uint64_t)N));
        }
    }
    if (!ok) fail(TNS_E_BAD_PATH, "internal: fused store tables disagree with the permute");
    s.sc_na = na;
    s.sc_nb = nb;
    s.sc_shift = shift;
    // store order: columns when the new legs stay fastest, else rows when
    // row m+1 follows row m in the target
    const int64_t f1 = M > 1 ? (nb > 1 ? fb[1] : fa[1]) : -1;
    s.sc_mfast = (N > 1 && fg[1] == 1) ? 0 : (f1 == 1 ? 1 : 0);
    return true;
}

}  // namespace

// ----------------------------------------------------------------------------
// Several main paths.  Algorithm 1 keeps one main path (assumption 3 lets a
// single isolated qubit wait to be joined), and the supplement notes that
// nothing guarantees one main path to be the cheaper choice.  Here a linear
// order is relaxed into a main path with side branches: a window [a, b) of
// positions of the order (a >= 1) is contracted by its own linear path, in
// the same order, and the main path absorbs the branch's tensor as one
// operand just before it reaches position b (windows ending at the last
// position are absorbed at the end).  Every step keeps the supplement's
// Cost(A, B): the product of the dimensions of the bonds either operand
// carries.

namespace {

struct LegSet {
    // bonds of a tensor as a bit set over edge ids (at most 256 edges)
    uint64_t w[4] = {0, 0, 0, 0};
    void flip(int e) { w[e >> 6] ^= 1ULL << (e & 63); }
    bool has(int e) const { return (w[e >> 6] >> (e & 63)) & 1; }
    LegSet operator^(const LegSet &o) const { LegSet r; for (int i = 0; i < 4; ++i) r.w[i] = w[i] ^ o.w[i]; return r; }
    LegSet operator|(const LegSet &o) const { LegSet r; for (int i = 0; i < 4; ++i) r.w[i] = w[i] | o.w[i]; return r; }
};

struct TreeCtx {
    std::vector<LegSet> site;   // bonds of each site (dimension > 1)
    std::vector<double> lg;     // log2 dimension per edge
    double size(const LegSet &s) const {
        double x = 0;
        for (int i = 0; i < 4; ++i)
            for (uint64_t m = s.w[i]; m; m &= m - 1) x += lg[64 * i + __builtin_ctzll(m)];
        return x;
    }
};

TreeCtx tree_ctx(const Circuit &c, const std::vector<double> &d) {
    if (c.g.edges.size() > 256) fail(TNS_E_UNSUPPORTED, "more than 256 bonds");
    TreeCtx t;
    t.site.assign(c.n, LegSet{});
    t.lg.assign(256, 0.0);
    for (size_t e = 0; e < c.g.edges.size(); ++e) {
        if (!(d[e] > 1.0)) continue;
        t.lg[e] = std::log2(d[e]);
        t.site[c.g.edges[e].first].flip((int)e);
        if (c.g.edges[e].second < c.n) t.site[c.g.edges[e].second].flip((int)e);
    }
    return t;
}

struct TreeEval {
    double score = 0;        // sum of M K N
    double peak = 0;         // log2 of the largest main-path operand or result
    double branch_peak = 0;  // log2 of the largest branch tensor
};

// windows: disjoint [a, b) ranges of positions, sorted by a, a >= 1
TreeEval tree_eval(const TreeCtx &t, const std::vector<int> &order,
                   const std::vector<std::pair<int, int>> &windows) {
    const int n = (int)order.size();
    std::vector<int> win(n, -1);
    for (size_t w = 0; w < windows.size(); ++w)
        for (int i = windows[w].first; i < windows[w].second; ++i) win[i] = (int)w;
    TreeEval ev;
    auto branch = [&](int w) {
        LegSet B = t.site[order[windows[w].first]];
        ev.branch_peak = std::max(ev.branch_peak, t.size(B));
        for (int i = windows[w].first + 1; i < windows[w].second; ++i) {
            const LegSet &S = t.site[order[i]];
            ev.score += std::exp2(t.size(B | S));
            B = B ^ S;
            ev.branch_peak = std::max(ev.branch_peak, t.size(B));
        }
        return B;
    };
    std::vector<int> by_end(windows.size());
    std::iota(by_end.begin(), by_end.end(), 0);
    std::stable_sort(by_end.begin(), by_end.end(),
                     [&](int x, int y) { return windows[x].second < windows[y].second; });
    size_t next = 0;
    LegSet T;
    bool started = false;
    auto absorb = [&](const LegSet &X) {
        ev.score += std::exp2(t.size(T | X));
        T = T ^ X;
        ev.peak = std::max(ev.peak, t.size(T));
    };
    for (int i = 0; i < n; ++i) {
        if (win[i] >= 0) continue;
        while (started && next < by_end.size() && windows[by_end[next]].second <= i) absorb(branch(by_end[next++]));
        if (!started) {
            T = t.site[order[i]];
            ev.peak = t.size(T);
            started = true;
        } else {
            ev.peak = std::max(ev.peak, t.size(T));
            absorb(t.site[order[i]]);
        }
    }
    while (next < by_end.size()) absorb(branch(by_end[next++]));
    return ev;
}

}  // namespace

// Greedy choice of branch windows for a fixed order: repeatedly add the
// window (length 2..16, disjoint from those chosen) that lowers the summed
// cost most while every main-path tensor stays within log2_limit and every
// branch tensor within log2_branch_limit; stops when no window helps.
std::vector<std::pair<int, int>> choose_branches(const Circuit &c, const std::vector<double> &d,
                                                 const std::vector<int> &order, double log2_limit,
                                                 double log2_branch_limit, double *score_out) {
    const TreeCtx t = tree_ctx(c, d);
    const int n = (int)order.size();
    std::vector<std::pair<int, int>> cur;
    double best = tree_eval(t, order, cur).score;
    for (;;) {
        std::vector<char> used(n, 0);
        for (auto &w : cur)
            for (int i = w.first; i < w.second; ++i) used[i] = 1;
        std::pair<int, int> pick{-1, -1};
        double pick_score = best;
        for (int a = 1; a + 1 < n; ++a) {
            if (used[a]) continue;
            for (int b = a + 2; b <= std::min(n, a + 16); ++b) {
                if (used[b - 1]) break;
                auto trial = cur;
                trial.push_back({a, b});
                std::sort(trial.begin(), trial.end());
                const TreeEval ev = tree_eval(t, order, trial);
                if (ev.peak > log2_limit + 1e-9 || ev.branch_peak > log2_branch_limit + 1e-9) continue;
                if (ev.score < pick_score * (1 - 1e-9)) {
                    pick_score = ev.score;
                    pick = {a, b};
                }
            }
        }
        if (pick.first < 0) break;
        cur.push_back(pick);
        std::sort(cur.begin(), cur.end());
        best = pick_score;
    }
    if (score_out) *score_out = best;
    return cur;
}

static void compile_steps(Plan &p) {
    const Circuit &c = p.circ;
    const int n = c.n;
    const auto &order = p.path.order;
    const int n_edges = (int)c.g.edges.size();
    std::vector<int64_t> d(n_edges);
    std::vector<char> is_cut(n_edges, 0);
    for (int e : p.cuts) is_cut[e] = 1;
    for (int e = 0; e < n_edges; ++e) d[e] = is_cut[e] ? 1 : p.bond_overlap[e];
    auto logical_legs = [&](int q) {
        std::vector<int> v;
        for (int e : c.g.legs[q])
            if (d[e] > 1) v.push_back(e);
        return v;
    };

    // The contraction program in execution order: each chain (0 = the main
    // path, w + 1 = branch w) starts from one site tensor and absorbs sites;
    // the main path absorbs branch w's tensor just before it reaches the end
    // of the branch's window.
    struct Op { int chain, kind, id; };   // kind 0: start at site id, 1: absorb site id, 2: absorb branch id
    std::vector<Op> ops;
    {
        const auto &W = p.branches;
        std::vector<int> win(n, -1), by_end(W.size());
        for (size_t w = 0; w < W.size(); ++w) {
            if (W[w].first < 1 || W[w].second > n || W[w].second - W[w].first < 2)
                fail(TNS_E_BAD_PATH, "internal: bad branch window");
            for (int i = W[w].first; i < W[w].second; ++i) {
                if (win[i] >= 0) fail(TNS_E_BAD_PATH, "internal: overlapping branch windows");
                win[i] = (int)w;
            }
        }
        std::iota(by_end.begin(), by_end.end(), 0);
        std::stable_sort(by_end.begin(), by_end.end(), [&](int x, int y) { return W[x].second < W[y].second; });
        size_t next = 0;
        bool started = false;
        auto branch = [&](int w) {
            ops.push_back({w + 1, 0, order[W[w].first]});
            for (int i = W[w].first + 1; i < W[w].second; ++i) ops.push_back({w + 1, 1, order[i]});
            ops.push_back({0, 2, w});
        };
        for (int i = 0; i < n; ++i) {
            if (win[i] >= 0) continue;
            while (started && next < by_end.size() && W[by_end[next]].second <= i) branch(by_end[next++]);
            ops.push_back({0, started ? 1 : 0, order[i]});
            started = true;
        }
        while (next < by_end.size()) branch(by_end[next++]);
    }
    // the op at which each bond is contracted (open legs: never)
    std::vector<int> cons(n_edges, std::numeric_limits<int>::max());
    {
        std::vector<std::vector<char>> held(p.branches.size() + 1, std::vector<char>(n_edges, 0));
        for (int k = 0; k < (int)ops.size(); ++k) {
            const Op &o = ops[k];
            std::vector<char> x(n_edges, 0);
            if (o.kind == 2) x = held[o.id + 1];
            else for (int e : logical_legs(o.id)) x[e] = 1;
            std::vector<char> &t = held[o.chain];
            if (o.kind == 0) { t = x; continue; }
            for (int e = 0; e < n_edges; ++e) {
                if (t[e] && x[e]) cons[e] = k;
                t[e] ^= x[e];
            }
        }
    }
    auto consumed = [&](int e) { return cons[e]; };
    // physical stride of bond e inside site q's overlap tensor (bonds in edge-id order)
    auto site_stride = [&](int q, int e) {
        int64_t st = 1;
        for (int i = (int)c.g.legs[q].size() - 1; i >= 0; --i) {
            if (c.g.legs[q][i] == e) return st;
            st *= p.site_dims[q][i];
        }
        fail(TNS_E_BAD_PATH, "internal: bond not on site");
    };
    auto by_consumption_desc = [&](std::vector<int> &v) {
        std::stable_sort(v.begin(), v.end(), [&](int a, int b) {
            int ca = consumed(a), cb = consumed(b);
            return ca != cb ? ca > cb : a < b;
        });
    };
    auto prod = [&](const std::vector<int> &v) {
        int64_t x = 1;
        for (int e : v) x *= d[e];
        return x;
    };

    p.steps.clear();
    const int elem = (p.precision == TNS_C128) ? 16 : 8;
    p.peak_elems = 0;
    p.branch_peak_elems = 0;
    p.max_b_elems = 0;
    p.flops_per_amp = p.gemm_bytes_per_amp = p.permute_bytes_per_amp = 0;
    p.path_score = 0;

    std::vector<std::vector<int>> T(p.branches.size() + 1);   // legs of each chain's tensor, storage order
    std::vector<int> last(p.branches.size() + 1, -1);          // step that produced it
    for (int k = 0; k < (int)ops.size(); ++k) {
        const Op &o = ops[k];
        Step s;
        s.chain = o.chain;
        int64_t &peak = o.chain == 0 ? p.peak_elems : p.branch_peak_elems;
        if (o.kind == 0) {
            // the starting tensor of a chain, gathered from its site
            s.start = true;
            s.site = o.id;
            s.n_legs = logical_legs(o.id);
            by_consumption_desc(s.n_legs);
            std::vector<int64_t> sz, st;
            for (int e : s.n_legs) { sz.push_back(d[e]); st.push_back(site_stride(o.id, e)); }
            s.bgather = compact(sz, st);
            s.N = prod(s.n_legs);
            s.out_elems = s.N;
            peak = std::max(peak, s.N);
            T[o.chain] = s.n_legs;
            last[o.chain] = (int)p.steps.size();
            p.steps.push_back(s);
            continue;
        }
        // the absorbed operand: a site tensor, or a branch's tensor (row-major
        // over its legs in storage order)
        std::vector<int> lj;
        std::vector<int64_t> xstride(n_edges, 0);
        if (o.kind == 1) {
            s.site = o.id;
            lj = logical_legs(o.id);
            for (int e : lj) xstride[e] = site_stride(o.id, e);
        } else {
            s.branch = o.id;
            lj = T[o.id + 1];
            int64_t st = 1;
            for (int i = (int)lj.size() - 1; i >= 0; --i) { xstride[lj[i]] = st; st *= d[lj[i]]; }
        }
        s.prev = last[o.chain];
        std::vector<int> &Tc = T[o.chain];
        s.t_legs = Tc;
        std::vector<int> S, Mv;
        for (int e : Tc)
            if (std::find(lj.begin(), lj.end(), e) != lj.end()) S.push_back(e); else Mv.push_back(e);
        // Are the shared legs already the trailing legs of T?
        bool trailing = true;
        for (size_t i = 0; i < S.size(); ++i)
            if (Tc[Tc.size() - S.size() + i] != S[i]) trailing = false;
        if (!trailing) {
            s.permute = true;
            by_consumption_desc(Mv);
            std::vector<int> neworder = Mv;
            neworder.insert(neworder.end(), S.begin(), S.end());
            // source strides of T (row-major over T)
            std::vector<int64_t> tstride(Tc.size());
            int64_t st = 1;
            for (int i = (int)Tc.size() - 1; i >= 0; --i) { tstride[i] = st; st *= d[Tc[i]]; }
            std::vector<int64_t> sz, sst;
            for (int e : neworder) {
                int i = (int)(std::find(Tc.begin(), Tc.end(), e) - Tc.begin());
                sz.push_back(d[e]);
                sst.push_back(tstride[i]);
            }
            s.perm = compact(sz, sst);
            p.permute_bytes_per_amp += 2.0 * elem * (double)prod(Tc);
        }
        s.m_legs = Mv;
        s.k_legs = S;
        for (int e : lj)
            if (std::find(S.begin(), S.end(), e) == S.end()) s.n_legs.push_back(e);
        by_consumption_desc(s.n_legs);
        s.M = prod(Mv);
        s.K = prod(S);
        s.N = prod(s.n_legs);
        {
            // B[n][k]: new legs (slow) then shared legs in T's order (fast)
            std::vector<int64_t> sz, st;
            for (int e : s.n_legs) { sz.push_back(d[e]); st.push_back(xstride[e]); }
            for (int e : S) { sz.push_back(d[e]); st.push_back(xstride[e]); }
            s.bgather = compact(sz, st);
        }
        s.out_elems = s.M * s.N;
        const bool final_op = (k + 1 == (int)ops.size());
        if (final_op && o.chain != 0) fail(TNS_E_BAD_PATH, "internal: the program does not end on the main path");
        if (final_op && c.n_open == 0) {
            if (s.M != 1 || s.N != 1) fail(TNS_E_BAD_PATH, "internal: final step is not a scalar");
            s.kernel = 2;
        } else if (final_op && s.M * s.N != ((int64_t)1 << c.n_open)) {
            fail(TNS_E_BAD_PATH, "internal: final tensor does not hold the open legs");
        } else if (s.K >= 16 && s.N >= 16 && s.M >= 16 && s.K % 2 == 0) {
            // complex64 wide steps: three real products instead of four.  The
            // split-BF16 forms keep the real embedding, except on the
            // small-output long-K steps, which run split over K in FP32: their
            // single long accumulation would otherwise set the amplitude's error
            const bool splitk_shape = s.M <= 64 && s.N <= 64 && s.K >= 4096;
            if (p.precision == TNS_C64) s.kernel = gemm_3m_fits(s.M, s.K, s.N) ? 3 : 0;
            else s.kernel = (p.precision != TNS_C128 && splitk_shape) ? 3 : 0;
        } else {
            s.kernel = 1;
        }
        Tc = Mv;
        Tc.insert(Tc.end(), s.n_legs.begin(), s.n_legs.end());
        peak = std::max(peak, std::max(s.out_elems, s.M * s.K));
        p.max_b_elems = std::max(p.max_b_elems, s.K * s.N);
        const double mkn = (double)s.M * (double)s.K * (double)s.N;
        p.path_score += mkn;
        p.flops_per_amp += 8.0 * mkn;
        p.gemm_bytes_per_amp += elem * ((double)s.M * s.K + (double)s.K * s.N + (double)s.M * s.N);
        last[o.chain] = (int)p.steps.size();
        p.steps.push_back(s);
    }
    const std::vector<int> &Tfinal = T[0];
    // a boundary permute after a GEMM step (either form), or after a small
    // step that the row-tiled kernel takes, goes into that step's store (the
    // step of the same chain that produced the permuted tensor)
    for (size_t m = 0; m < p.steps.size(); ++m) {
        Step &s = p.steps[m];
        if (!s.permute || s.prev < 0) continue;
        Step &prev = p.steps[s.prev];
        if (prev.start) continue;
        if (prev.kernel != 0 && prev.kernel != 3 &&
            !(prev.kernel == 1 && small_rows_fits(prev.M, prev.K, prev.N, elem)))
            continue;
        if (build_scatter(s.perm, prev.M, prev.N, prev)) {
            s.permute_fused = true;
            prev.store_fused = true;
            p.permute_bytes_per_amp -= 2.0 * elem * (double)(prev.M * prev.N);
        }
    }
    // open legs of the last tensor -> output order (first open qubit most significant)
    p.out_per_unit = (int64_t)1 << c.n_open;
    if (c.n_open > 0) {
        std::vector<int64_t> tstride(Tfinal.size());
        int64_t st = 1;
        for (int i = (int)Tfinal.size() - 1; i >= 0; --i) { tstride[i] = st; st *= d[Tfinal[i]]; }
        std::vector<int64_t> sz, sst;
        for (int k = 0; k < c.n_open; ++k) {
            const int e = c.n_real_edges + k;
            const int i = (int)(std::find(Tfinal.begin(), Tfinal.end(), e) - Tfinal.begin());
            if (i >= (int)Tfinal.size()) fail(TNS_E_BAD_PATH, "internal: open leg missing from the last tensor");
            sz.push_back(2);
            sst.push_back(tstride[i]);
        }
        p.final_perm = compact(sz, sst);
    }
    const double ns = (double)p.n_slices;
    p.flops_per_amp *= ns;
    p.gemm_bytes_per_amp *= ns;
    p.permute_bytes_per_amp *= ns;

    // per-site slice maps (slice index = mixed radix over the cuts, last fastest)
    p.slice_map.assign(n, SliceMap{});
    if ((int)p.cuts.size() > kMaxCuts) fail(TNS_E_UNSUPPORTED, "too many cut bonds");
    int64_t div = 1;
    for (int ci = (int)p.cuts.size() - 1; ci >= 0; --ci) {
        const int e = p.cuts[ci];
        for (int q : {c.g.edges[e].first, c.g.edges[e].second}) {
            SliceMap &sm = p.slice_map[q];
            sm.div[sm.n] = div;
            sm.dim[sm.n] = p.bond_overlap[e];
            sm.stride[sm.n] = site_stride(q, e);
            sm.n++;
        }
        div *= p.bond_overlap[e];
    }

    // Slice prefix.  Cutting turns the network into sub-networks that differ
    // only in the indices of the cut bonds, so the pairwise steps before the
    // first tensor that carries a cut bond are the same in every one of them.
    // The leading main-path steps that absorb uncut sites form the prefix,
    // computed once per bitstring; it must end before the last step and hold
    // at least one contraction besides the start.
    p.prefix_steps = 0;
    p.prefix_elems = 0;
    p.prefix_flops = 0;
    if (p.n_slices > 1) {
        int P = 0;
        for (size_t m = 0; m + 1 < p.steps.size(); ++m) {
            const Step &s = p.steps[m];
            if (s.chain != 0 || s.branch >= 0 || p.slice_map[s.site].n > 0) break;
            P = (int)m + 1;
        }
        if (P >= 2) {
            double fl = 0, by = 0;
            for (int m = 0; m < P; ++m) {
                const Step &s = p.steps[m];
                if (s.start) continue;
                fl += 8.0 * (double)s.M * s.K * s.N;
                by += elem * ((double)s.M * s.K + (double)s.K * s.N + (double)s.M * s.N);
            }
            p.prefix_steps = P;
            p.prefix_elems = p.steps[P - 1].out_elems;
            p.prefix_flops = fl;
            p.flops_per_amp -= (ns - 1) * fl;
            p.gemm_bytes_per_amp -= (ns - 1) * by;
        }
    }
}

// ----------------------------------------------------------------------------
// whole host plan

static void split_groups(const Circuit &c, int k, std::vector<int> &ket, std::vector<int> &bra) {
    ket.clear();
    bra.clear();
    for (int i = 0; i < (int)c.gates.size(); ++i) (c.gates[i].cycle < k ? ket : bra).push_back(i);
}

static void evolve_both(Plan &p, int k) {
    p.fuse.clear();
    p.chain_flat.clear();
    p.chain_off.clear();
    p.chain_len.clear();
    p.ket_init_chain.assign(p.circ.n, -1);
    p.bra_final_chain.assign(p.circ.n, -1);
    std::vector<int> kg, bg;
    split_groups(p.circ, k, kg, bg);
    std::vector<int> kf = fuse_side(p, kg, false);
    std::vector<int> bf = fuse_side(p, bg, true);
    p.n_fused_ket = (int)kf.size();
    p.n_fused_bra = (int)bf.size();
    p.ket = evolve_side(p, kf, false);
    p.bra = evolve_side(p, bf, true);
    const auto &E = p.circ.g.edges;
    p.bond_overlap.assign(E.size(), 1);
    for (size_t e = 0; e < E.size(); ++e) p.bond_overlap[e] = p.ket.bond[e] * p.bra.bond[e];
}

static std::vector<double> dims_with_cuts(const Plan &p, const std::vector<int> &cuts) {
    std::vector<double> d(p.bond_overlap.begin(), p.bond_overlap.end());
    for (int e : cuts) d[e] = 1;
    return d;
}

// Sizes of the intermediates along a fixed order; returns the step index of
// the largest one and fills its open bonds.
static double largest_intermediate(const Circuit &c, const std::vector<double> &d,
                                   const std::vector<int> &order, std::vector<int> *open_out) {
    const auto &E = c.g.edges;
    std::vector<char> in(c.n + 1, 0);
    double best = -1;
    for (int j : order) {
        in[j] = 1;
        double sz = 1;
        for (size_t e = 0; e < E.size(); ++e)
            if (d[e] > 1 && in[E[e].first] != in[E[e].second]) sz *= d[e];
        if (sz > best) {
            best = sz;
            if (open_out) {
                open_out->clear();
                for (size_t e = 0; e < E.size(); ++e)
                    if (d[e] > 1 && in[E[e].first] != in[E[e].second]) open_out->push_back((int)e);
            }
        }
    }
    return best;
}

struct Sliced {
    std::vector<int> cuts;
    double total = 0;   // slices x score
    double peak = 0;
    double slices = 1;
};

// Cuts for a fixed contraction order (overlap paragraph: a cut bond of
// dimension D splits the network into D sub-networks with the bond removed).
// For a fixed order the sliced cost is exact: D x score with the bond at
// dimension 1.  While the largest intermediate exceeds the limit, cut the open
// bond of that intermediate that minimises the total.
static Sliced cuts_for_order(const Plan &p, const std::vector<int> &order, std::vector<int> cuts,
                             double limit) {
    const Circuit &c = p.circ;
    Sliced r;
    for (int it = 0; it < 4 * kMaxCuts; ++it) {
        std::vector<double> d = dims_with_cuts(p, cuts);
        std::vector<int> open;
        double pk = largest_intermediate(c, d, order, &open);
        if (pk <= limit) break;
        int be = -1;
        double bt = 0, bp = 0;
        for (int e : open) {
            if (e >= c.n_real_edges) continue;   // open legs are not cut
            std::vector<double> dt = d;
            dt[e] = 1;
            double pke = 0;
            double t = path_score(c.n, c.g.edges, dt, order, &pke, nullptr) * d[e];
            if (be < 0 || t < bt || (t == bt && pke < bp)) { be = e; bt = t; bp = pke; }
        }
        if (be < 0) break;
        cuts.push_back(be);
    }
    std::vector<double> d = dims_with_cuts(p, cuts);
    r.cuts = cuts;
    r.slices = 1;
    for (int e : cuts) r.slices *= p.bond_overlap[e];
    r.total = path_score(c.n, c.g.edges, d, order, &r.peak, nullptr) * r.slices;
    return r;
}

// Cut search by simulated annealing.  The paper cuts first and then plans
// the path of the sliced network; the choice of cut set dominates the cost
// when no single bond stays open across the expensive part of a linear path.
// State: a set of cut bonds.  Evaluation: greedy path of the network with
// those bonds removed, completed by cuts_for_order until every intermediate
// fits the limit; cost = slices x score.  Moves add, remove or replace one
// bond; acceptance is Metropolis on log(cost) with a linearly falling
// temperature.  Deterministic for a given seed.
static Sliced anneal_cuts(const Plan &p, double limit, int iters, uint64_t seed,
                          std::vector<int> *order_out) {
    const Circuit &c = p.circ;
    const auto &E = c.g.edges;
    std::vector<int> cand;
    for (int e = 0; e < c.n_real_edges; ++e)
        if (p.bond_overlap[e] > 1) cand.push_back(e);
    std::mt19937_64 rng(seed);
    auto eval = [&](const std::vector<int> &cuts, std::vector<int> *ord) {
        PathResult r = path_search(c.n, E, dims_with_cuts(p, cuts), TNS_PATH_GREEDY, 0, true, 0);
        Sliced sl = cuts_for_order(p, r.order, cuts, limit);
        if (sl.peak > limit || sl.slices > 1e12 || (int)sl.cuts.size() > kMaxCuts)
            sl.total = std::numeric_limits<double>::infinity();
        if (ord) *ord = r.order;
        return sl;
    };
    std::vector<int> cur, cur_order;
    Sliced cs = eval(cur, &cur_order);
    Sliced best = cs;
    std::vector<int> best_order = cur_order;
    if (cand.empty()) {
        if (order_out) *order_out = best_order;
        return best;
    }
    std::uniform_real_distribution<double> U(0.0, 1.0);
    for (int it = 0; it < iters; ++it) {
        const double temp = 2.0 * (1.0 - (double)it / iters) + 1e-3;
        std::vector<int> prop = cur;
        const double r = U(rng);
        const int pick = cand[rng() % cand.size()];
        if (r < 0.4 || prop.empty()) {
            if (std::find(prop.begin(), prop.end(), pick) == prop.end()) prop.push_back(pick);
        } else if (r < 0.7) {
            prop.erase(prop.begin() + (long)(rng() % prop.size()));
        } else {
            prop[rng() % prop.size()] = pick;
            std::sort(prop.begin(), prop.end());
            prop.erase(std::unique(prop.begin(), prop.end()), prop.end());
        }
        std::vector<int> ord;
        Sliced ps = eval(prop, &ord);
        bool accept = ps.total < cs.total;
        if (!accept && std::isfinite(ps.total) && std::isfinite(cs.total))
            accept = U(rng) < std::exp(-(std::log(ps.total) - std::log(cs.total)) / temp);
        if (!std::isfinite(cs.total) && std::isfinite(ps.total)) accept = true;
        if (accept) {
            cur = prop;
            cs = ps;
            if (ps.total < best.total) {
                best = ps;
                best_order = ord;
            }
        }
    }
    if (order_out) *order_out = best_order;
    return best;
}

// The paper picks its cuts by hand, at narrow parts of the lattice; here the
// choice is automated: plan a path on the whole network, cut against that path, then
// also re-plan the path on the sliced network as the paper does for its
// sub-networks, and keep whichever has the least total cost within the limit.
static void choose_cuts_and_path(Plan &p) {
    const Circuit &c = p.circ;
    const auto &E = c.g.edges;
    const double limit = (double)(p.opts.max_intermediate_elems ? p.opts.max_intermediate_elems
                                                                 : (1ULL << 32));
    p.cuts.clear();
    std::vector<int> given;
    if (p.opts.n_cuts >= 0) {
        for (int i = 0; i < p.opts.n_cuts; ++i) {
            int e = p.opts.cut_edges[i];
            if (e < 0 || e >= c.n_real_edges || std::count(given.begin(), given.end(), e))
                fail(TNS_E_BAD_PATH, "bad cut edge " + std::to_string(e));
            given.push_back(e);
        }
    }
    p.search_complete = true;
    p.search_states = 0;
    // searches on a sliced network also keep every intermediate within the
    // limit (the size-aware bound); the unsliced search, which places the
    // cuts, does not
    auto search = [&](const std::vector<double> &d, int mode, double max_size = 0) {
        PathResult r = path_search(c.n, E, d, mode, p.opts.max_rank, p.opts.path_assumptions != 0,
                                   p.opts.max_search_states, max_size);
        if (mode == TNS_PATH_ALGORITHM1) {
            p.search_complete = p.search_complete && r.complete;
            p.search_states += r.states;
        }
        return r;
    };
    if (p.opts.path) {
        PathResult r;
        r.order.assign(p.opts.path, p.opts.path + c.n);
        Sliced s = p.opts.n_cuts >= 0 ? cuts_for_order(p, r.order, given, 1e300)
                                      : cuts_for_order(p, r.order, {}, limit);
        p.cuts = s.cuts;
        r.score = path_score(c.n, E, dims_with_cuts(p, p.cuts), r.order, &r.peak, &r.max_rank);
        p.path = r;
    } else if (p.opts.n_cuts >= 0) {
        p.cuts = given;
        p.path = search(dims_with_cuts(p, p.cuts), p.opts.path_mode, limit);
    } else {
        std::vector<double> d0 = dims_with_cuts(p, {});
        PathResult best_path;
        Sliced best;
        best.total = std::numeric_limits<double>::infinity();
        // candidates are ranked by the cost they reach once side branches
        // are added (the linear cost when branches are off)
        auto consider = [&](const PathResult &r, const Sliced &s) {
            if (!(s.peak <= limit)) return;
            Sliced t = s;
            if (p.opts.path_branches) {
                double sc = 0;
                choose_branches(c, dims_with_cuts(p, s.cuts), r.order, std::log2(limit),
                                std::min(std::log2(limit), std::log2((double)kBranchPeakElems)), &sc);
                t.total = sc * s.slices;
            }
            if (t.total < best.total) { best = t; best_path = r; }
        };
        std::vector<int> modes{TNS_PATH_GREEDY};
        if (p.opts.path_mode != TNS_PATH_GREEDY) modes.push_back(p.opts.path_mode);
        for (int mode : modes) {
            PathResult r = search(d0, mode);
            Sliced s = cuts_for_order(p, r.order, {}, limit);
            consider(r, s);
            if (s.cuts.empty()) continue;
            // re-plan on the sliced network (the paper's order of operations)
            std::vector<double> ds = dims_with_cuts(p, s.cuts);
            PathResult r2 = search(ds, mode, limit);
            Sliced s2 = cuts_for_order(p, r2.order, s.cuts, limit);
            consider(r2, s2);
        }
        if (!best.cuts.empty() || !std::isfinite(best.total)) {
            // cut search, then the requested path search on the sliced network
            std::vector<int> order;
            Sliced sa = anneal_cuts(p, limit, 2000, 0x5eed5eedULL + p.split, &order);
            if (std::isfinite(sa.total)) {
                PathResult r;
                r.order = order;
                consider(r, sa);
                if (p.opts.path_mode != TNS_PATH_GREEDY) {
                    PathResult r3 = search(dims_with_cuts(p, sa.cuts), p.opts.path_mode, limit);
                    consider(r3, cuts_for_order(p, r3.order, sa.cuts, limit));
                }
            }
        }
        if (!std::isfinite(best.total))
            fail(TNS_E_OUT_OF_MEMORY, "no cut set brings the largest intermediate under the limit");
        p.cuts = best.cuts;
        p.path = best_path;
        p.path.score = path_score(c.n, E, dims_with_cuts(p, p.cuts), p.path.order, &p.path.peak, nullptr);
    }
    if ((int)p.path.order.size() != c.n) fail(TNS_E_BAD_PATH, "path search returned no full path");
    if ((int)p.cuts.size() > kMaxCuts) fail(TNS_E_UNSUPPORTED, "too many cut bonds");
    p.n_slices = 1;
    for (int e : p.cuts) {
        if (p.n_slices > ((int64_t)1 << 40) / p.bond_overlap[e]) fail(TNS_E_OUT_OF_MEMORY, "too many slices");
        p.n_slices *= p.bond_overlap[e];
    }
}

void add_open_legs(Circuit &c, const tns_plan_opts &opts) {
    c.n_real_edges = (int)c.g.edges.size();
    c.n_open = 0;
    c.open_qubits.clear();
    if (opts.n_open < 0 || opts.n_open > 20) fail(TNS_E_INVALID_ARG, "n_open must be in [0, 20]");
    if (opts.n_open > 0 && !opts.open_qubits) fail(TNS_E_INVALID_ARG, "open_qubits is NULL");
    for (int k = 0; k < opts.n_open; ++k) {
        const int q = opts.open_qubits[k];
        if (q < 0 || q >= c.n || std::count(c.open_qubits.begin(), c.open_qubits.end(), q))
            fail(TNS_E_INVALID_ARG, "bad open qubit " + std::to_string(q));
        if ((int)c.g.legs[q].size() + 1 > kMaxDeg) fail(TNS_E_UNSUPPORTED, "open qubit has too many legs");
        c.open_qubits.push_back(q);
        const int e = (int)c.g.edges.size();
        c.g.edges.push_back({q, c.n});   // dangling: second endpoint is the virtual node n
        c.g.legs[q].push_back(e);
    }
    c.n_open = opts.n_open;
}

void plan_host(const Circuit &c, const tns_plan_opts &opts, Plan &p) {
    p.circ = c;
    p.opts = opts;
    p.precision = opts.precision;
    if (opts.precision < TNS_C128 || opts.precision > TNS_C64_SPLIT_BF16_6)
        fail(TNS_E_INVALID_ARG, "unknown precision");
    if (opts.path) {
        std::vector<char> seen(c.n, 0);
        for (int i = 0; i < c.n; ++i) {
            int q = opts.path[i];
            if (q < 0 || q >= c.n || seen[q]) fail(TNS_E_BAD_PATH, "path is not a permutation of 0..N-1");
            seen[q] = 1;
        }
    }
    if (opts.n_cuts > 0 && !opts.cut_edges) fail(TNS_E_INVALID_ARG, "n_cuts > 0 with NULL cut_edges");
    const int depth = c.max_cycle + 1;
    if (opts.split_cycle >= 0) {
        p.split = opts.split_cycle;
    } else {
        // choose the split with the least sliced cost of a greedy path; splits
        // whose network needs cuts get an annealed cut search, but only when
        // their unsliced score could still beat the best total found
        const double limit = (double)(opts.max_intermediate_elems ? opts.max_intermediate_elems
                                                                   : (1ULL << 32));
        const double inf = std::numeric_limits<double>::infinity();
        std::vector<double> total(depth + 1, inf), score0(depth + 1, inf);
        std::vector<char> needs_cuts(depth + 1, 0);
        for (int k = 0; k <= depth; ++k) {
            evolve_both(p, k);
            std::vector<double> d(p.bond_overlap.begin(), p.bond_overlap.end());
            PathResult r = path_search(c.n, c.g.edges, d, TNS_PATH_GREEDY, 0, true, 0);
            Sliced sl = cuts_for_order(p, r.order, {}, limit);
            score0[k] = r.score;
            total[k] = sl.peak <= limit ? sl.total : inf;
            needs_cuts[k] = !sl.cuts.empty();
        }
        double best = *std::min_element(total.begin(), total.end());
        // the greedy score can rank splits differently from the path search
        // that builds the final path: score the cut-free splits near the best
        // (within 1.5x, at most six) with the requested mode as well
        if (opts.path_mode != TNS_PATH_GREEDY) {
            std::vector<int> near;
            for (int k = 0; k <= depth; ++k)
                if (!needs_cuts[k] && total[k] <= 1.5 * best) near.push_back(k);
            std::sort(near.begin(), near.end(), [&](int a2, int b2) { return total[a2] < total[b2]; });
            if (near.size() > 6) near.resize(6);
            for (int k : near) {
                evolve_both(p, k);
                std::vector<double> d(p.bond_overlap.begin(), p.bond_overlap.end());
                PathResult r = path_search(c.n, c.g.edges, d, opts.path_mode, opts.max_rank,
                                           opts.path_assumptions != 0, opts.max_search_states);
                Sliced sl = cuts_for_order(p, r.order, {}, limit);
                if (sl.peak <= limit) total[k] = std::min(total[k], sl.total);
            }
            best = *std::min_element(total.begin(), total.end());
        }
        std::vector<int> byscore(depth + 1);
        std::iota(byscore.begin(), byscore.end(), 0);
        std::sort(byscore.begin(), byscore.end(), [&](int a2, int b2) { return score0[a2] < score0[b2]; });
        for (int k : byscore) {
            if (!needs_cuts[k] || opts.n_cuts >= 0 || !(score0[k] < best)) continue;
            evolve_both(p, k);
            p.split = k;
            Sliced sa = anneal_cuts(p, limit, 600, 0x5eed5eedULL + k, nullptr);
            total[k] = std::min(total[k], sa.total);
            best = std::min(best, total[k]);
        }
        int bk = 0;
        for (int k = 0; k <= depth; ++k)
            if (total[k] < total[bk]) bk = k;
        p.split = bk;
    }
    evolve_both(p, p.split);
    // overlap site tensors (Eq. (8)): bond dims multiply
    p.site_dims.assign(c.n, {});
    p.site_elems.assign(c.n, 1);
    for (int q = 0; q < c.n; ++q)
        for (int e : c.g.legs[q]) {
            p.site_dims[q].push_back(p.bond_overlap[e]);
            p.site_elems[q] *= p.bond_overlap[e];
        }
    choose_cuts_and_path(p);
    // several main paths: side branches of the linear order where they lower
    // the summed cost, within the intermediate limit (or the linear path's
    // own peak, when given cuts leave it above the limit)
    p.branches.clear();
    {
        const std::vector<double> dc = dims_with_cuts(p, p.cuts);
        double lpeak = 0;
        p.linear_score = path_score(c.n, c.g.edges, dc, p.path.order, &lpeak, nullptr);
        if (opts.path_branches) {
            const double limit = (double)(opts.max_intermediate_elems ? opts.max_intermediate_elems
                                                                       : (1ULL << 32));
            const double lim = std::max(std::log2(limit), std::log2(lpeak));
            p.branches = choose_branches(c, dc, p.path.order, lim,
                                         std::min(lim, std::log2((double)kBranchPeakElems)), nullptr);
        }
    }
    compile_steps(p);

    // scratch for the SVD's V' of the bra side (per bitstring)
    p.bra_scratch_elems = 1;
    for (const EvoOp &op : p.bra.ops)
        if (op.comp >= 0) {
            int64_t rows = 1;
            const SiteShape &s = op.comp == 0 ? op.s0 : op.s1;
            for (int i = 0; i < s.n; ++i) rows *= s.d[i];
            rows = rows / op.d_before;   // rows of the widened tensor: 2 * other bonds
            p.bra_scratch_elems = std::max<int64_t>(p.bra_scratch_elems, rows * op.d_grown);
        }
    for (const EvoOp &op : p.ket.ops)
        if (op.comp >= 0) {
            int64_t rows = 1;
            const SiteShape &s = op.comp == 0 ? op.s0 : op.s1;
            for (int i = 0; i < s.n; ++i) rows *= s.d[i];
            rows = rows / op.d_before;
            p.bra_scratch_elems = std::max<int64_t>(p.bra_scratch_elems, rows * op.d_grown);
        }

    // reporting: Eq. (9) with the Sycamore error rates quoted in the paper
    int n1 = 0, n2 = 0;
    for (const auto &g : c.gates) (g.q1 < 0 ? n1 : n2)++;
    double f = std::pow(1 - 0.0016, n1) * std::pow(1 - 0.0062, n2) * std::pow(1 - 0.038, c.n);
    p.fidelity = f;
    p.n_samples = (3.0 / f) * (3.0 / f);

    p.info_path = p.path.order;
    p.info_m.clear(); p.info_k.clear(); p.info_n.clear(); p.info_kernel.clear(); p.info_permute.clear();
    p.info_chain.clear();
    p.info_branch_windows.clear();
    for (auto &w : p.branches) {
        p.info_branch_windows.push_back(w.first);
        p.info_branch_windows.push_back(w.second);
    }
    for (size_t i = 0; i < p.steps.size(); ++i) {
        if (p.steps[i].start) continue;
        p.info_chain.push_back(p.steps[i].chain);
        p.info_m.push_back(p.steps[i].M);
        p.info_k.push_back(p.steps[i].K);
        p.info_n.push_back(p.steps[i].N);
        p.info_kernel.push_back(p.steps[i].kernel);
        p.info_permute.push_back(!p.steps[i].permute ? 0 : (p.steps[i].permute_fused ? 2 : 1));
    }
    const int elem = p.precision == TNS_C128 ? 16 : 8;
    // one unit: two boundary buffers, the B operand (embedded form is 2x) and the partial
    // (a branch's tensors also pass through the main buffer the main path is
    // not using, so it holds the larger of the two peaks)
    p.unit_stride = (std::max(p.peak_elems, p.branch_peak_elems) + 31) / 32 * 32;
    // and, with branches, the branch buffer
    p.branch_stride = p.branches.empty() ? 0 : (p.branch_peak_elems + 31) / 32 * 32;
    p.bytes_per_unit = (2 * p.unit_stride + p.branch_stride) * elem + 2 * p.max_b_elems * elem + 16;
    int64_t sites = 0, bra = 0;
    for (int q = 0; q < c.n; ++q) {
        sites += p.site_elems[q];
        bra += 2 * p.bra.cap[q];
    }
    p.bytes_per_bitstring = sites * elem + bra * 16 + p.bra_scratch_elems * 16 + c.n + 16;
}

}  // namespace tns
