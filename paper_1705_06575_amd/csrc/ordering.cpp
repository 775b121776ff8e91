// ordering.cpp -- graph nested dissection from the pattern alone.
//
// The paper leaves the fill-reducing ordering to the libraries' defaults;
// this is the library's own choice.  Each subgraph is split by a level set
// of a breadth-first search started from a pseudo-peripheral vertex: the
// level where the running vertex count passes one half is the separator,
// separator vertices with no neighbour in the next level move to the lower
// side, the two sides are ordered recursively and the separator last.
// Disconnected subgraphs are split into their components first.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "plan.hpp"

namespace sym {

namespace {

struct Sub {
    std::vector<int32_t> verts;
    int32_t lo;   // first label of this subgraph
};

struct NDState {
    int32_t n;
    const std::vector<int64_t> &xadj;
    const std::vector<int32_t> &adj;
    std::vector<int32_t> region;   // subgraph id of each vertex
    std::vector<int32_t> level;    // BFS level scratch (-1 = unvisited)
    std::vector<int32_t> queue;
    int32_t next_region = 1;
    NDState(int32_t n_, const std::vector<int64_t> &x, const std::vector<int32_t> &a)
        : n(n_), xadj(x), adj(a), region((size_t)n_, 0), level((size_t)n_, -1), queue((size_t)n_) {}

    // BFS inside region `rid` from `root`; returns the number of vertices
    // reached and the last level index.  Leaves `level` set for reached ones.
    int32_t bfs(int32_t rid, int32_t root, int32_t &nlev)
    {
        int32_t head = 0, tail = 0;
        queue[tail++] = root;
        level[root] = 0;
        nlev = 1;
        while (head < tail) {
            int32_t v = queue[head++];
            int32_t lv = level[v];
            for (int64_t p = xadj[v]; p < xadj[v + 1]; ++p) {
                int32_t u = adj[p];
                if (region[u] != rid || level[u] >= 0) continue;
                level[u] = lv + 1;
                if (lv + 2 > nlev) nlev = lv + 2;
                queue[tail++] = u;
            }
        }
        return tail;
    }
    void clear_levels(int32_t count)
    {
        for (int32_t i = 0; i < count; ++i) level[queue[i]] = -1;
    }
    int32_t degree_in(int32_t v, int32_t rid) const
    {
        int32_t d = 0;
        for (int64_t p = xadj[v]; p < xadj[v + 1]; ++p) d += region[adj[p]] == rid;
        return d;
    }
};

}  // namespace

void nested_dissection(int32_t n, const std::vector<int64_t> &xadj,
                       const std::vector<int32_t> &adj, int32_t leaf,
                       std::vector<int32_t> &perm)
{
    perm.assign((size_t)n, -1);
    if (n == 0) return;
    NDState S(n, xadj, adj);
    std::vector<Sub> stack;
    {
        Sub all;
        all.verts.resize((size_t)n);
        for (int32_t v = 0; v < n; ++v) all.verts[v] = v;
        all.lo = 0;
        stack.push_back(std::move(all));
    }
    std::vector<int32_t> tmp;
    while (!stack.empty()) {
        Sub cur = std::move(stack.back());
        stack.pop_back();
        const int32_t m = (int32_t)cur.verts.size();
        if (m == 0) continue;
        if (m <= leaf) {
            std::sort(cur.verts.begin(), cur.verts.end());
            for (int32_t i = 0; i < m; ++i) perm[cur.lo + i] = cur.verts[i];
            continue;
        }
        const int32_t rid = S.next_region++;
        for (int32_t v : cur.verts) S.region[v] = rid;

        // connected component of the first vertex
        int32_t nlev = 0;
        int32_t reached = S.bfs(rid, cur.verts[0], nlev);
        if (reached < m) {
            // split off the component; the rest stays one subgraph
            Sub a, b;
            a.verts.assign(S.queue.begin(), S.queue.begin() + reached);
            S.clear_levels(reached);
            const int32_t rid_a = S.next_region++;
            for (int32_t v : a.verts) S.region[v] = rid_a;
            for (int32_t v : cur.verts)
                if (S.region[v] == rid) b.verts.push_back(v);
            a.lo = cur.lo;
            b.lo = cur.lo + (int32_t)a.verts.size();
            stack.push_back(std::move(a));
            stack.push_back(std::move(b));
            continue;
        }
        // pseudo-peripheral root: restart from a minimum-degree vertex of the
        // last level while the eccentricity grows (at most a few sweeps)
        int32_t root = cur.verts[0];
        for (int it = 0; it < 4; ++it) {
            int32_t best = -1, bestdeg = INT32_MAX;
            for (int32_t i = 0; i < reached; ++i) {
                int32_t v = S.queue[i];
                if (S.level[v] == nlev - 1) {
                    int32_t d = S.degree_in(v, rid);
                    if (d < bestdeg) { bestdeg = d; best = v; }
                }
            }
            S.clear_levels(reached);
            int32_t nlev2 = 0;
            S.bfs(rid, best, nlev2);
            if (nlev2 <= nlev) {
                // no gain: keep the BFS from `best` (same depth) and stop
                root = best;
                nlev = nlev2;
                break;
            }
            root = best;
            nlev = nlev2;
        }
        (void)root;
        // level histogram and the median level
        std::vector<int32_t> cnt((size_t)nlev + 1, 0);
        for (int32_t i = 0; i < m; ++i) cnt[S.level[S.queue[i]]]++;
        int32_t sepl = 0;
        {
            int64_t acc = 0;
            for (int32_t l = 0; l < nlev; ++l) {
                if (acc + cnt[l] > m / 2) { sepl = l; break; }
                acc += cnt[l];
            }
            if (sepl == 0 && nlev > 2) sepl = 1;
            if (sepl >= nlev - 1 && nlev > 2) sepl = nlev - 2;
        }
        if (nlev <= 2) {
            // (nearly) complete graph: no useful separator
            S.clear_levels(m);
            std::sort(cur.verts.begin(), cur.verts.end());
            for (int32_t i = 0; i < m; ++i) perm[cur.lo + i] = cur.verts[i];
            continue;
        }
        Sub lowp, highp;
        std::vector<int32_t> sep;
        for (int32_t i = 0; i < m; ++i) {
            int32_t v = S.queue[i];
            int32_t lv = S.level[v];
            if (lv < sepl) lowp.verts.push_back(v);
            else if (lv > sepl) highp.verts.push_back(v);
            else {
                bool touches_high = false;
                for (int64_t p = xadj[v]; p < xadj[v + 1]; ++p) {
                    int32_t u = adj[p];
                    if (S.region[u] == rid && S.level[u] == sepl + 1) { touches_high = true; break; }
                }
                if (touches_high) sep.push_back(v);
                else lowp.verts.push_back(v);
            }
        }
        S.clear_levels(m);
        std::sort(sep.begin(), sep.end());
        const int32_t sep_lo = cur.lo + m - (int32_t)sep.size();
        for (size_t i = 0; i < sep.size(); ++i) perm[sep_lo + (int32_t)i] = sep[i];
        lowp.lo = cur.lo;
        highp.lo = cur.lo + (int32_t)lowp.verts.size();
        // region ids are reassigned when a subgraph is popped
        stack.push_back(std::move(highp));
        stack.push_back(std::move(lowp));
    }
}

}  // namespace sym
