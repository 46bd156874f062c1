/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, single-threaded, obviously-correct max-flow solvers used to check the
 * HIP solver.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load this library; the product path never does.  It shares no
 * code, header, table or helper with the HIP path.
 *
 * What is computed (section 2.1 of the paper defines the problem: a directed
 * graph with integer capacities c(u,v), source s, sink t, residual graph G_f
 * with residual capacities c_f; the answer is the maximum s-t flow value):
 *
 *   orc_dinic      Dinic's algorithm (section 2.1): BFS level graph from s,
 *                  then a blocking flow by depth-first search with current-arc
 *                  pointers, repeated until t is unreachable.
 *   orc_fifo_pr    Generic push-relabel (section 2.2): preflow saturating the
 *                  source arcs, h(s) = |V|, exact push rule h(u) = h(v) + 1,
 *                  relabel to 1 + the minimum neighbour height, global
 *                  relabelling by backward BFS from the sink, plus the gap
 *                  heuristic; FIFO selection of active vertices.  A second
 *                  phase returns excess that cannot reach t to s, so that a
 *                  flow (not only a preflow) is produced.
 *   orc_check      Independent certificate: capacity bounds, conservation,
 *                  flow value, the canonical sink side (vertices that reach t
 *                  in the residual graph of the flow) and the capacity of the
 *                  cut it defines.  A feasible flow whose value equals the
 *                  capacity of some s-t cut is maximum (weak duality).
 *
 * Representation: every input arc i = (u,v) becomes residual arc 2i (u->v,
 * initial residual c_i) and its mate 2i+1 (v->u, initial residual 0).
 * Self-loops are inert.  This is the textbook arc-pair form, deliberately
 * unlike the merged bidirectional rows of the GPU path.
 *
 * Return codes: 0 ok, -1 bad input or allocation failure, -2 internal
 * inconsistency (must never happen).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n;
    int64_t m;        /* number of input arcs */
    int64_t *first;   /* [n+1] offsets into adj */
    int64_t *adj;     /* residual arc ids grouped by tail */
    int32_t *head;    /* [2m] */
    int32_t *tail;    /* [2m] */
    int64_t *r;       /* [2m] residual capacity */
} rgraph;

static void rg_free(rgraph *g) {
    free(g->first); free(g->adj); free(g->head); free(g->tail); free(g->r);
    memset(g, 0, sizeof(*g));
}

static int validate(int32_t V, int64_t E, const int64_t *rp, const int32_t *col, const int32_t *cap,
                    int32_t s, int32_t t) {
    if (V < 2 || E < 0 || s < 0 || s >= V || t < 0 || t >= V || s == t) return -1;
    if (rp[0] != 0 || rp[V] != E) return -1;
    for (int32_t v = 0; v < V; v++) if (rp[v + 1] < rp[v]) return -1;
    for (int64_t i = 0; i < E; i++) if (col[i] < 0 || col[i] >= V || cap[i] < 0) return -1;
    return 0;
}

static int rg_build(rgraph *g, int32_t V, int64_t E, const int64_t *rp, const int32_t *col,
                    const int32_t *cap) {
    memset(g, 0, sizeof(*g));
    g->n = V; g->m = E;
    size_t m2 = (size_t)(2 * E > 0 ? 2 * E : 1);
    g->first = (int64_t *)calloc((size_t)V + 1, sizeof(int64_t));
    g->adj = (int64_t *)malloc(sizeof(int64_t) * m2);
    g->head = (int32_t *)malloc(sizeof(int32_t) * m2);
    g->tail = (int32_t *)malloc(sizeof(int32_t) * m2);
    g->r = (int64_t *)malloc(sizeof(int64_t) * m2);
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)V + 1));
    if (!g->first || !g->adj || !g->head || !g->tail || !g->r || !fill) { free(fill); rg_free(g); return -1; }
    for (int32_t u = 0; u < V; u++)
        for (int64_t i = rp[u]; i < rp[u + 1]; i++) {
            int32_t v = col[i];
            g->tail[2 * i] = u; g->head[2 * i] = v; g->r[2 * i] = cap[i];
            g->tail[2 * i + 1] = v; g->head[2 * i + 1] = u; g->r[2 * i + 1] = 0;
            if (u != v) { g->first[u + 1]++; g->first[v + 1]++; }
        }
    for (int32_t v = 0; v < V; v++) g->first[v + 1] += g->first[v];
    memcpy(fill, g->first, sizeof(int64_t) * ((size_t)V + 1));
    for (int64_t i = 0; i < E; i++) {
        int32_t u = g->tail[2 * i], v = g->head[2 * i];
        if (u == v) continue;
        g->adj[fill[u]++] = 2 * i;
        g->adj[fill[v]++] = 2 * i + 1;
    }
    free(fill);
    return 0;
}

static void flows_out(const rgraph *g, const int32_t *cap, int32_t *flow) {
    for (int64_t i = 0; i < g->m; i++) {
        if (g->tail[2 * i] == g->head[2 * i]) flow[i] = 0;
        else flow[i] = (int32_t)(cap[i] - g->r[2 * i]);
    }
}

/* ------------------------------------------------------------- Dinic */
int orc_dinic(int32_t V, int64_t E, const int64_t *rp, const int32_t *col, const int32_t *cap,
              int32_t s, int32_t t, int64_t *value, int32_t *flow, int64_t *arc_scans) {
    if (validate(V, E, rp, col, cap, s, t)) return -1;
    rgraph g;
    if (rg_build(&g, V, E, rp, col, cap)) return -1;
    int32_t *level = (int32_t *)malloc(sizeof(int32_t) * (size_t)V);
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)V);
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)V);
    int64_t *stack = (int64_t *)malloc(sizeof(int64_t) * (size_t)V);
    if (!level || !q || !cur || !stack) { free(level); free(q); free(cur); free(stack); rg_free(&g); return -1; }
    int64_t total = 0, scans = 0;
    for (;;) {
        /* level graph: BFS distance from s over arcs with positive residual */
        for (int32_t v = 0; v < V; v++) level[v] = -1;
        int32_t qh = 0, qt = 0;
        level[s] = 0; q[qt++] = s;
        while (qh < qt) {
            int32_t v = q[qh++];
            for (int64_t k = g.first[v]; k < g.first[v + 1]; k++) {
                int64_t a = g.adj[k];
                int32_t w = g.head[a];
                scans++;
                if (g.r[a] > 0 && level[w] < 0) { level[w] = level[v] + 1; q[qt++] = w; }
            }
        }
        if (level[t] < 0) break;
        for (int32_t v = 0; v < V; v++) cur[v] = g.first[v];
        /* blocking flow: advance along level-increasing arcs, retreat from
           dead ends, augment at t by the bottleneck and restart from the
           tail of the first saturated arc */
        int32_t top = 0, v = s;
        for (;;) {
            if (v == t) {
                int64_t f = INT64_MAX;
                for (int32_t i = 0; i < top; i++) if (g.r[stack[i]] < f) f = g.r[stack[i]];
                for (int32_t i = 0; i < top; i++) { g.r[stack[i]] -= f; g.r[stack[i] ^ 1] += f; }
                total += f;
                int32_t k = 0;
                while (k < top && g.r[stack[k]] > 0) k++;
                top = k;
                v = (k == 0) ? s : g.tail[stack[k]];
                continue;
            }
            int advanced = 0;
            while (cur[v] < g.first[v + 1]) {
                int64_t a = g.adj[cur[v]];
                int32_t w = g.head[a];
                scans++;
                if (g.r[a] > 0 && level[w] == level[v] + 1) {
                    stack[top++] = a; v = w; advanced = 1; break;
                }
                cur[v]++;
            }
            if (advanced) continue;
            if (v == s) break;
            level[v] = -1;                 /* dead end: never revisit this phase */
            int64_t a = stack[--top];
            v = g.tail[a];
            cur[v]++;
        }
    }
    if (value) *value = total;
    if (flow) flows_out(&g, cap, flow);
    if (arc_scans) *arc_scans = scans;
    free(level); free(q); free(cur); free(stack);
    rg_free(&g);
    return 0;
}

/* ------------------------------------------------ FIFO push-relabel */
typedef struct {
    int32_t *buf; int64_t cap, head, size;
} fifo;

static int fifo_init(fifo *f, int64_t cap) {
    f->buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
    f->cap = cap > 0 ? cap : 1; f->head = 0; f->size = 0;
    return f->buf ? 0 : -1;
}
static void fifo_push(fifo *f, int32_t v) { f->buf[(f->head + f->size) % f->cap] = v; f->size++; }
static int32_t fifo_pop(fifo *f) { int32_t v = f->buf[f->head]; f->head = (f->head + 1) % f->cap; f->size--; return v; }

/* Exact heights: h(v) = residual distance from v to `root`; vertices that
   cannot reach root get `unreached`.  `skip` is never labelled. */
static void bfs_heights(const rgraph *g, int32_t root, int32_t skip, int32_t unreached, int32_t *h,
                        int32_t *q, int64_t *scans) {
    for (int32_t v = 0; v < g->n; v++) h[v] = unreached;
    int32_t qh = 0, qt = 0;
    h[root] = 0; q[qt++] = root;
    while (qh < qt) {
        int32_t w = q[qh++];
        for (int64_t k = g->first[w]; k < g->first[w + 1]; k++) {
            int64_t a = g->adj[k];          /* arc w -> v; residual v -> w is a^1 */
            int32_t v = g->head[a];
            (*scans)++;
            if (v == skip || h[v] != unreached) continue;
            if (g->r[a ^ 1] > 0) { h[v] = h[w] + 1; q[qt++] = v; }
        }
    }
}

int orc_fifo_pr(int32_t V, int64_t E, const int64_t *rp, const int32_t *col, const int32_t *cap,
                int32_t s, int32_t t, int64_t *value, int32_t *flow, int64_t *arc_scans) {
    if (validate(V, E, rp, col, cap, s, t)) return -1;
    rgraph g;
    if (rg_build(&g, V, E, rp, col, cap)) return -1;
    int32_t n = V;
    int64_t *e = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int32_t *h = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *cnt = (int32_t *)calloc((size_t)2 * n + 2, sizeof(int32_t));
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    char *inq = (char *)calloc((size_t)n, 1);
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    fifo F;
    int rc = 0;
    if (!e || !h || !cnt || !cur || !inq || !q || fifo_init(&F, n)) { rc = -1; goto done; }
    int64_t scans = 0;

    /* ---------------- phase 1: maximum preflow ---------------- */
    for (int64_t k = g.first[s]; k < g.first[s + 1]; k++) {      /* preflow */
        int64_t a = g.adj[k];
        int64_t d = g.r[a];
        if (d <= 0) continue;
        g.r[a] = 0; g.r[a ^ 1] += d;
        e[g.head[a]] += d; e[s] -= d;
    }
    const int64_t gr_period = 6 * (int64_t)n + g.first[n];
    int64_t work = 0;
    int need_gr = 1;
    for (;;) {
        if (need_gr) {
            bfs_heights(&g, t, s, n, h, q, &scans);
            h[s] = n;
            memset(cnt, 0, sizeof(int32_t) * ((size_t)2 * n + 2));
            for (int32_t v = 0; v < n; v++) if (h[v] < n) cnt[h[v]]++;
            F.head = 0; F.size = 0;
            memset(inq, 0, (size_t)n);
            for (int32_t v = 0; v < n; v++) {
                cur[v] = g.first[v];
                if (v != s && v != t && e[v] > 0 && h[v] < n) { fifo_push(&F, v); inq[v] = 1; }
            }
            work = 0; need_gr = 0;
        }
        if (F.size == 0) break;
        int32_t u = fifo_pop(&F);
        inq[u] = 0;
        if (h[u] >= n) continue;
        /* discharge u */
        while (e[u] > 0) {
            if (cur[u] == g.first[u + 1]) {
                /* relabel: 1 + minimum height over residual out-arcs */
                int32_t mh = INT32_MAX;
                for (int64_t k = g.first[u]; k < g.first[u + 1]; k++) {
                    int64_t a = g.adj[k];
                    scans++;
                    if (g.r[a] > 0 && h[g.head[a]] < mh) mh = h[g.head[a]];
                }
                int32_t old = h[u];
                int32_t nh = (mh == INT32_MAX || mh >= n) ? n : mh + 1;
                work += 12 + (g.first[u + 1] - g.first[u]);
                cnt[old]--;
                h[u] = nh;
                if (nh < n) cnt[nh]++;
                cur[u] = g.first[u];
                if (cnt[old] == 0) {
                    /* gap: nothing at height `old` any more, so no vertex
                       above it (and below n) can reach t */
                    for (int32_t v = 0; v < n; v++)
                        if (h[v] > old && h[v] < n && v != s) { cnt[h[v]]--; h[v] = n; }
                    if (h[u] < n) { cnt[h[u]]--; h[u] = n; }
                }
                if (h[u] >= n) break;
                continue;
            }
            int64_t a = g.adj[cur[u]];
            int32_t w = g.head[a];
            scans++;
            if (g.r[a] > 0 && h[u] == h[w] + 1) {
                int64_t d = e[u] < g.r[a] ? e[u] : g.r[a];
                g.r[a] -= d; g.r[a ^ 1] += d;
                e[u] -= d; e[w] += d;
                if (w != s && w != t && !inq[w] && h[w] < n) { fifo_push(&F, w); inq[w] = 1; }
            } else {
                cur[u]++;
            }
        }
        if (work > gr_period) need_gr = 1;
    }
    int64_t val = e[t];

    /* ------------- phase 2: return stranded excess to s ------------- */
    /* Every vertex with excess reaches s in G_f (its excess arrived along a
       path from s).  Heights are distances to s; t is never a target. */
    int any = 0;
    for (int32_t v = 0; v < n; v++) if (v != s && v != t && e[v] > 0) { any = 1; break; }
    if (any) {
        const int32_t BIG = INT32_MAX / 2;
        bfs_heights(&g, s, t, BIG, h, q, &scans);
        h[t] = BIG;
        F.head = 0; F.size = 0;
        memset(inq, 0, (size_t)n);
        for (int32_t v = 0; v < n; v++) {
            cur[v] = g.first[v];
            if (v != s && v != t && e[v] > 0) {
                if (h[v] >= BIG) { rc = -2; goto done; }
                fifo_push(&F, v); inq[v] = 1;
            }
        }
        while (F.size > 0) {
            int32_t u = fifo_pop(&F);
            inq[u] = 0;
            while (e[u] > 0) {
                if (cur[u] == g.first[u + 1]) {
                    int32_t mh = INT32_MAX;
                    for (int64_t k = g.first[u]; k < g.first[u + 1]; k++) {
                        int64_t a = g.adj[k];
                        scans++;
                        if (g.r[a] > 0 && g.head[a] != t && h[g.head[a]] < mh) mh = h[g.head[a]];
                    }
                    if (mh == INT32_MAX || mh >= BIG - 1) { rc = -2; goto done; }
                    h[u] = mh + 1;
                    cur[u] = g.first[u];
                    continue;
                }
                int64_t a = g.adj[cur[u]];
                int32_t w = g.head[a];
                scans++;
                if (w != t && g.r[a] > 0 && h[u] == h[w] + 1) {
                    int64_t d = e[u] < g.r[a] ? e[u] : g.r[a];
                    g.r[a] -= d; g.r[a ^ 1] += d;
                    e[u] -= d; e[w] += d;
                    if (w != s && !inq[w]) { fifo_push(&F, w); inq[w] = 1; }
                } else {
                    cur[u]++;
                }
            }
        }
    }
    if (e[t] != val) { rc = -2; goto done; }
    if (value) *value = val;
    if (flow) flows_out(&g, cap, flow);
    if (arc_scans) *arc_scans = scans;
done:
    free(e); free(h); free(cnt); free(cur); free(inq); free(q); free(F.buf);
    rg_free(&g);
    return rc;
}

/* ----------------------------------------------------- certificate */
/* Returns 0 if `flow` is a feasible s-t flow; then *value is its value,
   side[v] = 1 iff v reaches t in the residual graph of `flow`, and *cutcap
   is the capacity of the cut (side 0 -> side 1).  The flow is maximum iff
   *value == *cutcap (and then side[s] == 0).
   Nonzero returns: 1 capacity bound violated at arc *bad, 2 conservation
   violated at vertex *bad, -1 bad input / allocation. */
int orc_check(int32_t V, int64_t E, const int64_t *rp, const int32_t *col, const int32_t *cap,
              int32_t s, int32_t t, const int32_t *flow, int64_t *value, uint8_t *side,
              int64_t *cutcap, int64_t *bad) {
    if (validate(V, E, rp, col, cap, s, t)) return -1;
    int32_t *src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(E > 0 ? E : 1));
    int64_t *bal = (int64_t *)calloc((size_t)V, sizeof(int64_t));
    int64_t *tfirst = (int64_t *)calloc((size_t)V + 1, sizeof(int64_t));
    int64_t *tarc = (int64_t *)malloc(sizeof(int64_t) * (size_t)(E > 0 ? E : 1));
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)V);
    uint8_t *mark = side ? side : (uint8_t *)malloc((size_t)V);
    int rc = 0;
    if (!src || !bal || !tfirst || !tarc || !q || !mark) { rc = -1; goto out; }
    for (int32_t u = 0; u < V; u++)
        for (int64_t i = rp[u]; i < rp[u + 1]; i++) src[i] = u;
    for (int64_t i = 0; i < E; i++) {
        if (flow[i] < 0 || flow[i] > cap[i]) { if (bad) *bad = i; rc = 1; goto out; }
        bal[col[i]] += flow[i];
        bal[src[i]] -= flow[i];
    }
    for (int32_t v = 0; v < V; v++)
        if (v != s && v != t && bal[v] != 0) { if (bad) *bad = v; rc = 2; goto out; }
    if (value) *value = -bal[s];
    /* transpose: input arcs grouped by head */
    for (int64_t i = 0; i < E; i++) tfirst[col[i] + 1]++;
    for (int32_t v = 0; v < V; v++) tfirst[v + 1] += tfirst[v];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)V + 1));
        if (!fill) { rc = -1; goto out; }
        memcpy(fill, tfirst, sizeof(int64_t) * ((size_t)V + 1));
        for (int64_t i = 0; i < E; i++) tarc[fill[col[i]]++] = i;
        free(fill);
    }
    /* backward reachability of t in the residual graph */
    memset(mark, 0, (size_t)V);
    int32_t qh = 0, qt = 0;
    mark[t] = 1; q[qt++] = t;
    while (qh < qt) {
        int32_t w = q[qh++];
        for (int64_t k = tfirst[w]; k < tfirst[w + 1]; k++) {      /* arc u -> w, residual if f < c */
            int64_t i = tarc[k];
            int32_t u = src[i];
            if (!mark[u] && flow[i] < cap[i]) { mark[u] = 1; q[qt++] = u; }
        }
        for (int64_t i = rp[w]; i < rp[w + 1]; i++) {              /* arc w -> x, residual x -> w if f > 0 */
            int32_t x = col[i];
            if (!mark[x] && flow[i] > 0) { mark[x] = 1; q[qt++] = x; }
        }
    }
    if (cutcap) {
        int64_t cc = 0;
        for (int64_t i = 0; i < E; i++) if (!mark[src[i]] && mark[col[i]]) cc += cap[i];
        *cutcap = cc;
    }
out:
    free(src); free(bal); free(tfirst); free(tarc); free(q);
    if (!side) free(mark);
    return rc;
}
