/*
 * CPU ORACLE -- test infrastructure only.
 *
 * Plain, slow, single-threaded FP64 reference for what one NXgraph iteration
 * computes. Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may load it; the GPU library never does, and the two share no code.
 *
 * Every routine walks the edge list in the order it was given; nothing is
 * blocked, fused or reordered. Where the paper leaves a definition open the
 * reading taken is stated at the routine (the paper is Chi et al., "NXgraph:
 * An Efficient Graph Processing System on a Single Machine", 2015).
 *
 * Conventions: vertex ids are 0-based int32 in [0, n); edge e goes from
 * src[e] to dst[e] (the graph is directed, Sec. II-A; an undirected graph is
 * two opposite edges). Return value 0 = success, nonzero = invalid argument.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_INF INT32_MAX

static int check_edges(int64_t n, int64_t m, const int32_t* src, const int32_t* dst) {
    if (n < 1 || m < 0) return 1;
    for (int64_t e = 0; e < m; ++e)
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return 2;
    return 0;
}

/* Out-degree: number of edges whose source is u (self-loops and repeated
 * edges count). */
int orc_outdeg(int64_t n, int64_t m, const int32_t* src, int64_t* deg) {
    for (int64_t u = 0; u < n; ++u) deg[u] = 0;
    for (int64_t e = 0; e < m; ++e) deg[src[e]] += 1;
    return 0;
}

/*
 * PageRank by synchronous iteration (Alg. 1's update model with ping-pong
 * intervals, Sec. II-B consistency rule and Sec. III-B1 SPU). The paper names
 * PageRank but never writes its formula; the reading used here:
 *
 *   w_e = 1 / outdeg(src_e)   (plain)   or the given weight (weighted);
 *   D   = { u : outdeg(u) = 0 }  (structural dangling set);
 *   x^0 = t;
 *   y_v = sum over edges e with dst_e = v of w_e * x^k[src_e];
 *   delta = sum over u in D of x^k_u, summed in vertex order;
 *   x^{k+1}_v = d * (y_v + delta / n) + (1 - d) * t_v.
 *
 * t == NULL means the uniform teleport 1/n. Runs `iters` iterations, or, when
 * tol > 0, stops after the first iteration whose residual ||x^{k+1}-x^k||_1 is
 * <= tol (at most `iters`). resid (nullable) receives one residual per
 * iteration run; *iters_done (nullable) the number of iterations run.
 * x receives the final vector. x0 (nullable) replaces x^0 = t (warm start).
 */
int orc_pagerank(int64_t n, int64_t m, const int32_t* src, const int32_t* dst, const double* w,
                 const double* t, const double* x0, double d, int64_t iters, double tol,
                 double* x, double* resid, int64_t* iters_done) {
    int rc = check_edges(n, m, src, dst);
    if (rc) return rc;
    int64_t* deg = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    double* cur = (double*)malloc(sizeof(double) * (size_t)n);
    double* y = (double*)malloc(sizeof(double) * (size_t)n);
    if (!deg || !cur || !y) {
        free(deg);
        free(cur);
        free(y);
        return 3;
    }
    orc_outdeg(n, m, src, deg);
    const double un = 1.0 / (double)n;
    for (int64_t v = 0; v < n; ++v) cur[v] = x0 ? x0[v] : (t ? t[v] : un);
    int64_t k = 0;
    for (; k < iters; ++k) {
        for (int64_t v = 0; v < n; ++v) y[v] = 0.0;
        for (int64_t e = 0; e < m; ++e) {
            double we = w ? w[e] : 1.0 / (double)deg[src[e]];
            y[dst[e]] += we * cur[src[e]];
        }
        double delta = 0.0;
        for (int64_t u = 0; u < n; ++u)
            if (deg[u] == 0) delta += cur[u];
        double r = 0.0;
        for (int64_t v = 0; v < n; ++v) {
            double tv = t ? t[v] : un;
            double nv = d * (y[v] + delta / (double)n) + (1.0 - d) * tv;
            r += fabs(nv - cur[v]);
            y[v] = nv;
        }
        double* sw = cur;
        cur = y;
        y = sw;
        if (resid) resid[k] = r;
        if (tol > 0.0 && r <= tol) {
            ++k;
            break;
        }
    }
    memcpy(x, cur, sizeof(double) * (size_t)n);
    if (iters_done) *iters_done = k;
    free(deg);
    free(cur);
    free(y);
    return 0;
}

/*
 * BFS on the directed graph (Alg. 2 Initialize, Alg. 3 Update, Alg. 4 Output),
 * with synchronous rounds (Sec. II-B): every round reads the levels written by
 * the previous round. INT32_MAX stands for the paper's infinity; an edge out of
 * an unreached vertex relaxes nothing (avoids infinity + 1).
 * level[] receives the levels; *rounds the number of rounds that changed a
 * level; *max_level the largest finite level (Alg. 4).
 */
int orc_bfs(int64_t n, int64_t m, const int32_t* src, const int32_t* dst, int32_t root,
            int32_t* level, int64_t* rounds, int32_t* max_level) {
    int rc = check_edges(n, m, src, dst);
    if (rc) return rc;
    if (root < 0 || root >= n) return 4;
    int32_t* nxt = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!nxt) return 3;
    for (int64_t v = 0; v < n; ++v) level[v] = ORC_INF;
    level[root] = 0;
    int64_t r = 0;
    for (;;) {
        memcpy(nxt, level, sizeof(int32_t) * (size_t)n);
        int changed = 0;
        for (int64_t e = 0; e < m; ++e) {
            int32_t ls = level[src[e]];
            if (ls != ORC_INF && ls + 1 < nxt[dst[e]]) {
                nxt[dst[e]] = ls + 1;
                changed = 1;
            }
        }
        if (!changed) break;
        memcpy(level, nxt, sizeof(int32_t) * (size_t)n);
        ++r;
    }
    int32_t mx = 0;
    for (int64_t v = 0; v < n; ++v)
        if (level[v] != ORC_INF && level[v] > mx) mx = level[v];
    *rounds = r;
    *max_level = mx;
    free(nxt);
    return 0;
}

/*
 * Weakly connected components by minimum-label propagation. The paper names
 * WCC only (Sec. IV-D); the reading used: the graph is made undirected by
 * taking every edge in both directions (Sec. II-A), label[v] starts at v, and
 * each synchronous round sets label'[v] = min(label[v], label[u]) over every
 * neighbour u. At the fixed point every vertex holds the smallest id of its
 * component. *rounds = rounds that changed a label.
 */
int orc_wcc(int64_t n, int64_t m, const int32_t* src, const int32_t* dst, int32_t* label,
            int64_t* rounds) {
    int rc = check_edges(n, m, src, dst);
    if (rc) return rc;
    int32_t* nxt = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!nxt) return 3;
    for (int64_t v = 0; v < n; ++v) label[v] = (int32_t)v;
    int64_t r = 0;
    for (;;) {
        memcpy(nxt, label, sizeof(int32_t) * (size_t)n);
        int changed = 0;
        for (int64_t e = 0; e < m; ++e) {
            int32_t a = src[e], b = dst[e];
            if (label[a] < nxt[b]) {
                nxt[b] = label[a];
                changed = 1;
            }
            if (label[b] < nxt[a]) {
                nxt[a] = label[b];
                changed = 1;
            }
        }
        if (!changed) break;
        memcpy(label, nxt, sizeof(int32_t) * (size_t)n);
        ++r;
    }
    *rounds = r;
    free(nxt);
    return 0;
}

/*
 * Adjoint of weighted PageRank at its fixed point x* (not in the paper; the
 * gradient of L = g^T x* with respect to the given edge weights and the
 * teleport vector). With G = d * (W^T + (1/n) 1 1_D^T) the forward fixed point
 * is x = G x + (1 - d) t, so the adjoint vector solves lambda = g + G^T lambda:
 *
 *   lambda_u = g_u + d * sum over edges e with src_e = u of w_e * lambda[dst_e]
 *                  + d * [u in D] * (sum_v lambda_v) / n,
 *
 * iterated from lambda^0 = g until ||lambda^{k+1} - lambda^k||_1 <=
 * tol * ||lambda^{k+1}||_1 (or max_iters). Then
 *   dL/dw_e = d * x*[src_e] * lambda[dst_e]   (input edge order),
 *   dL/dt_v = (1 - d) * lambda_v.
 * gw, gt, lam are outputs (any may be NULL); *iters_done the iterations run.
 */
int orc_pagerank_adjoint(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                         const double* w, const double* xstar, const double* g, double d,
                         double tol, int64_t max_iters, double* lam, double* gw, double* gt,
                         int64_t* iters_done) {
    int rc = check_edges(n, m, src, dst);
    if (rc) return rc;
    int64_t* deg = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    double* cur = (double*)malloc(sizeof(double) * (size_t)n);
    double* nxt = (double*)malloc(sizeof(double) * (size_t)n);
    if (!deg || !cur || !nxt) {
        free(deg);
        free(cur);
        free(nxt);
        return 3;
    }
    orc_outdeg(n, m, src, deg);
    for (int64_t v = 0; v < n; ++v) cur[v] = g[v];
    int64_t k = 0;
    while (k < max_iters) {
        double s = 0.0;
        for (int64_t v = 0; v < n; ++v) s += cur[v];
        for (int64_t u = 0; u < n; ++u) nxt[u] = 0.0;
        for (int64_t e = 0; e < m; ++e) nxt[src[e]] += w[e] * cur[dst[e]];
        double diff = 0.0, norm = 0.0;
        for (int64_t u = 0; u < n; ++u) {
            double v = g[u] + d * nxt[u] + (deg[u] == 0 ? d * s / (double)n : 0.0);
            diff += fabs(v - cur[u]);
            norm += fabs(v);
            nxt[u] = v;
        }
        double* sw = cur;
        cur = nxt;
        nxt = sw;
        ++k;
        if (diff <= tol * norm) break;
    }
    if (lam) memcpy(lam, cur, sizeof(double) * (size_t)n);
    if (gw)
        for (int64_t e = 0; e < m; ++e) gw[e] = d * xstar[src[e]] * cur[dst[e]];
    if (gt)
        for (int64_t v = 0; v < n; ++v) gt[v] = (1.0 - d) * cur[v];
    if (iters_done) *iters_done = k;
    free(deg);
    free(cur);
    free(nxt);
    return 0;
}

/*
 * DSSS order (Sec. II-A, Sec. III-A "Sharding"): P equal intervals of size
 * I = ceil(n / P) (the last may be shorter); sub-shard SS_{i.j} holds the edges
 * with source in interval i and destination in interval j; shard S_j (all
 * sub-shards with destination interval j) is stored contiguously, sub-shards of
 * a shard in increasing i; inside a sub-shard edges are sorted by destination,
 * then by source (Sec. III-A), and edges that compare equal keep input order.
 *
 * `interval` is the interval size I (so P = ceil(n / I)). perm[k] receives the
 * input index of the k-th edge in DSSS order; offsets[s] for s = j * P + i
 * (P*P + 1 entries) the position of the first edge of SS_{i.j}.
 */
typedef struct {
    int64_t shard, sub, d, s, idx;
} orc_key;

static int orc_key_cmp(const void* a, const void* b) {
    const orc_key* x = (const orc_key*)a;
    const orc_key* y = (const orc_key*)b;
    if (x->shard != y->shard) return x->shard < y->shard ? -1 : 1;
    if (x->sub != y->sub) return x->sub < y->sub ? -1 : 1;
    if (x->d != y->d) return x->d < y->d ? -1 : 1;
    if (x->s != y->s) return x->s < y->s ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

int orc_dsss_order(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                   int64_t interval, int64_t* perm, int64_t* offsets) {
    int rc = check_edges(n, m, src, dst);
    if (rc) return rc;
    if (interval < 1) return 4;
    int64_t P = (n + interval - 1) / interval;
    orc_key* keys = (orc_key*)malloc(sizeof(orc_key) * (size_t)(m > 0 ? m : 1));
    if (!keys) return 3;
    for (int64_t e = 0; e < m; ++e) {
        keys[e].shard = dst[e] / interval;
        keys[e].sub = src[e] / interval;
        keys[e].d = dst[e];
        keys[e].s = src[e];
        keys[e].idx = e;
    }
    qsort(keys, (size_t)m, sizeof(orc_key), orc_key_cmp);
    for (int64_t s = 0; s <= P * P; ++s) offsets[s] = 0;
    for (int64_t k = 0; k < m; ++k) {
        perm[k] = keys[k].idx;
        offsets[keys[k].shard * P + keys[k].sub + 1] += 1;
    }
    for (int64_t s = 0; s < P * P; ++s) offsets[s + 1] += offsets[s];
    free(keys);
    return 0;
}

/*
 * Strongly connected components. The paper names SCC among its targeted
 * queries (Sec. IV-D) but gives no algorithm; the reading used is the
 * definition: u and v share a component when each reaches the other (every
 * vertex reaches itself), and label[v] is the smallest vertex id of v's
 * component. Computed with Kosaraju's two depth-first passes: the finishing
 * order of a search over the graph, then searches over the reversed graph
 * started in decreasing finishing time, each of which collects exactly one
 * component. Both searches use explicit stacks. *count = components.
 */
static int orc_csr(int64_t n, int64_t m, const int32_t* from, const int32_t* to, int64_t** off_out,
                   int32_t** adj_out) {
    int64_t* off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t* adj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!off || !adj || !pos) {
        free(off);
        free(adj);
        free(pos);
        return 3;
    }
    for (int64_t e = 0; e < m; ++e) off[from[e] + 1] += 1;
    for (int64_t v = 0; v < n; ++v) off[v + 1] += off[v];
    for (int64_t v = 0; v < n; ++v) pos[v] = off[v];
    for (int64_t e = 0; e < m; ++e) adj[pos[from[e]]++] = to[e];
    free(pos);
    *off_out = off;
    *adj_out = adj;
    return 0;
}

int orc_scc(int64_t n, int64_t m, const int32_t* src, const int32_t* dst, int32_t* label,
            int64_t* count) {
    int rc = check_edges(n, m, src, dst);
    if (rc) return rc;
    int64_t *fo = NULL, *ro = NULL;
    int32_t *fa = NULL, *ra = NULL;
    if (orc_csr(n, m, src, dst, &fo, &fa)) return 3;
    if (orc_csr(n, m, dst, src, &ro, &ra)) {
        free(fo);
        free(fa);
        return 3;
    }
    size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * nn);   /* vertices by finishing time */
    int32_t* stk = (int32_t*)malloc(sizeof(int32_t) * nn);     /* search stack: vertices */
    int64_t* nxt = (int64_t*)malloc(sizeof(int64_t) * nn);     /* next edge to try, per vertex */
    char* seen = (char*)calloc(nn, 1);
    int32_t* members = (int32_t*)malloc(sizeof(int32_t) * nn); /* one component's vertices */
    if (!order || !stk || !nxt || !seen || !members) {
        free(fo); free(fa); free(ro); free(ra);
        free(order); free(stk); free(nxt); free(seen); free(members);
        return 3;
    }
    /* pass 1: depth-first over the graph; a vertex is appended to `order`
       when all its out-neighbours are done */
    int64_t nfin = 0;
    for (int64_t r = 0; r < n; ++r) {
        if (seen[r]) continue;
        int64_t top = 0;
        stk[top++] = (int32_t)r;
        seen[r] = 1;
        nxt[r] = fo[r];
        while (top > 0) {
            int32_t u = stk[top - 1];
            if (nxt[u] < fo[u + 1]) {
                int32_t w = fa[nxt[u]++];
                if (!seen[w]) {
                    seen[w] = 1;
                    nxt[w] = fo[w];
                    stk[top++] = w;
                }
            } else {
                order[nfin++] = u;
                --top;
            }
        }
    }
    /* pass 2: over the reversed graph, roots in decreasing finishing time;
       each search collects one component */
    memset(seen, 0, nn);
    int64_t comps = 0;
    for (int64_t k = n - 1; k >= 0; --k) {
        int32_t r = order[k];
        if (seen[r]) continue;
        int64_t top = 0, cnt = 0;
        stk[top++] = r;
        seen[r] = 1;
        while (top > 0) {
            int32_t u = stk[--top];
            members[cnt++] = u;
            for (int64_t e = ro[u]; e < ro[u + 1]; ++e) {
                int32_t w = ra[e];
                if (!seen[w]) {
                    seen[w] = 1;
                    stk[top++] = w;
                }
            }
        }
        int32_t lo = members[0];
        for (int64_t i = 1; i < cnt; ++i)
            if (members[i] < lo) lo = members[i];
        for (int64_t i = 0; i < cnt; ++i) label[members[i]] = lo;
        ++comps;
    }
    *count = comps;
    free(fo); free(fa); free(ro); free(ra);
    free(order); free(stk); free(nxt); free(seen); free(members);
    return 0;
}
