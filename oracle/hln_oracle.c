/*
 * hln_oracle.c -- CPU oracle for exact closeness centrality on homogeneous
 * multilayer networks (HoMLNs).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file; only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark use it.  It shares no code, header,
 * table or helper with the HIP path.
 *
 * Every function is the plain definition, written for a reader to check
 * against the paper by eye:
 *
 *   - graph normalisation: layers are simple undirected graphs over one
 *     shared vertex set (Sec. 1, Problem Statement; Sec. 4 "undirected");
 *   - one FIFO-queue BFS per source, unweighted distances (Sec. 4: the
 *     closeness routine runs a BFS from every vertex, O(V(V+E)));
 *   - closeness with the Wasserman-Faust normalisation for disconnected
 *     graphs, unreachable vertices contributing 0 to the sum (Sec. 4, Eq. 1
 *     and the text after it);
 *   - the penalised distance sum where an unreachable vertex counts as n
 *     (Sec. 5.1, used by the composition heuristics);
 *   - Boolean AND / OR aggregation of layers (Sec. 3.1);
 *   - CC-node selection: above-average set (Sec. 4) or top-k (Sec. 5.2);
 *   - heuristic CC2: estimated distance sum = max over layers (Sec. 5.2,
 *     Algorithm 1);
 *   - naive composition: intersection of the layers' CC-node sets (Sec. 4).
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - FP64 operation order of the normalised closeness:
 *       q1 = (R-1)/S ; q2 = (R-1)/(n-1) ; cc = q1*q2
 *     with IEEE round-to-nearest division; cc = 0 when R <= 1 or n <= 1.
 *   - "above average" means cc >= mean; the mean is summed in a fixed shape
 *     (sequentially inside id-chunks of 1024, then sequentially over the
 *     chunk sums) and divided by the count.
 *   - ties in every ranking are broken by ascending vertex id.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -shared -fPIC
 *        -pthread (no x87: x86-64 SSE2 doubles are IEEE binary64).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

/* ------------------------------------------------------------------ */
/* Graph normalisation: any edge list -> symmetric CSR, rows sorted,   */
/* no self-loops, no duplicate arcs.                                   */
/* ------------------------------------------------------------------ */

typedef struct { int32_t src, dst; } arc_t;

static int arc_cmp(const void* a, const void* b) {
    const arc_t* x = (const arc_t*)a;
    const arc_t* y = (const arc_t*)b;
    if (x->src != y->src) return x->src < y->src ? -1 : 1;
    if (x->dst != y->dst) return x->dst < y->dst ? -1 : 1;
    return 0;
}

/* Returns the number of arcs written to col_idx (<= 2*m), or -1 on a vertex
 * id out of [0, n), or -2 on allocation failure.  row_ptr has n+1 entries,
 * col_idx room for 2*m. */
int64_t oracle_csr_from_edges(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev,
                              int32_t* row_ptr, int32_t* col_idx) {
    arc_t* arcs = (arc_t*)malloc(sizeof(arc_t) * (size_t)(2 * m + 1));
    if (!arcs) return -2;
    int64_t na = 0;
    for (int64_t i = 0; i < m; ++i) {
        int32_t u = eu[i], v = ev[i];
        if (u < 0 || u >= n || v < 0 || v >= n) { free(arcs); return -1; }
        if (u == v) continue;                 /* simple graph: drop self-loops */
        arcs[na].src = u; arcs[na].dst = v; ++na;
        arcs[na].src = v; arcs[na].dst = u; ++na;   /* undirected: both arcs */
    }
    qsort(arcs, (size_t)na, sizeof(arc_t), arc_cmp);
    int64_t nnz = 0;
    for (int32_t v = 0; v <= n; ++v) row_ptr[v] = 0;
    for (int64_t i = 0; i < na; ++i) {
        if (i > 0 && arcs[i].src == arcs[i - 1].src && arcs[i].dst == arcs[i - 1].dst)
            continue;                         /* simple graph: drop duplicates */
        col_idx[nnz++] = arcs[i].dst;
        row_ptr[arcs[i].src + 1] += 1;
    }
    for (int32_t v = 0; v < n; ++v) row_ptr[v + 1] += row_ptr[v];
    free(arcs);
    return nnz;
}

/* ------------------------------------------------------------------ */
/* All-pairs-from-sources BFS.                                         */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t n;
    const int32_t* row_ptr;
    const int32_t* col_idx;
    int32_t n_src;
    const int32_t* sources;       /* NULL: sources are 0..n-1 */
    int64_t* S;                   /* sum of distances to reachable vertices */
    int32_t* R;                   /* reachable count, the source included */
    int32_t* H2;                  /* vertices at distance exactly 2 (nullable) */
    int32_t* ecc;                 /* largest finite distance (nullable) */
    int64_t* comp_edges;          /* undirected edges of the source's component (nullable) */
    int32_t next;                 /* shared work counter (guarded by lock) */
    pthread_mutex_t lock;
} bfs_job_t;

/* One breadth-first search from s with a FIFO queue; dist = -1 marks
 * "not reached".  Returns nothing; writes the per-source results. */
static void bfs_one(const bfs_job_t* J, int32_t s, int32_t* dist, int32_t* queue,
                    int64_t* S, int32_t* R, int32_t* H2, int32_t* ecc, int64_t* ce) {
    const int32_t n = J->n;
    int32_t head = 0, tail = 0;
    dist[s] = 0;
    queue[tail++] = s;
    int64_t sum = 0, arcs = 0;
    int32_t reached = 0, at2 = 0, far = 0;
    while (head < tail) {
        int32_t u = queue[head++];
        reached += 1;
        sum += dist[u];
        if (dist[u] == 2) at2 += 1;
        if (dist[u] > far) far = dist[u];
        arcs += J->row_ptr[u + 1] - J->row_ptr[u];
        for (int32_t e = J->row_ptr[u]; e < J->row_ptr[u + 1]; ++e) {
            int32_t w = J->col_idx[e];
            if (dist[w] < 0) {
                dist[w] = dist[u] + 1;
                queue[tail++] = w;
            }
        }
    }
    /* reset only what was touched */
    for (int32_t i = 0; i < tail; ++i) dist[queue[i]] = -1;
    (void)n;
    *S = sum; *R = reached; *H2 = at2; *ecc = far; *ce = arcs / 2;
}

static void* bfs_worker(void* arg) {
    bfs_job_t* J = (bfs_job_t*)arg;
    int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(J->n > 0 ? J->n : 1));
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(J->n > 0 ? J->n : 1));
    if (!dist || !queue) { free(dist); free(queue); return (void*)1; }
    for (int32_t i = 0; i < J->n; ++i) dist[i] = -1;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int32_t lo = J->next;
        J->next = lo + 16 < J->n_src ? lo + 16 : J->n_src;
        int32_t hi = J->next;
        pthread_mutex_unlock(&J->lock);
        if (lo >= hi) break;
        for (int32_t i = lo; i < hi; ++i) {
            int32_t s = J->sources ? J->sources[i] : i;
            int64_t S; int32_t R, H2, ecc; int64_t ce;
            bfs_one(J, s, dist, queue, &S, &R, &H2, &ecc, &ce);
            J->S[i] = S; J->R[i] = R;
            if (J->H2) J->H2[i] = H2;
            if (J->ecc) J->ecc[i] = ecc;
            if (J->comp_edges) J->comp_edges[i] = ce;
        }
    }
    free(dist); free(queue);
    return NULL;
}

/* For every source (all vertices when sources == NULL, then n_src must be n)
 * runs one BFS and writes S, R and the optional H2 / ecc / component-edge
 * count at the source's position.  Returns 0, -1 on a bad source id, -2 on
 * allocation or thread failure. */
int oracle_bfs_sums(int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                    int32_t n_src, const int32_t* sources,
                    int64_t* S, int32_t* R, int32_t* H2, int32_t* ecc, int64_t* comp_edges,
                    int32_t nthreads) {
    if (sources)
        for (int32_t i = 0; i < n_src; ++i)
            if (sources[i] < 0 || sources[i] >= n) return -1;
    bfs_job_t J;
    J.n = n; J.row_ptr = row_ptr; J.col_idx = col_idx; J.n_src = n_src; J.sources = sources;
    J.S = S; J.R = R; J.H2 = H2; J.ecc = ecc; J.comp_edges = comp_edges; J.next = 0;
    pthread_mutex_init(&J.lock, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    int started = 0, rc = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (pthread_create(&th[t], NULL, bfs_worker, &J) != 0) { rc = -2; break; }
        ++started;
    }
    for (int t = 0; t < started; ++t) {
        void* ret = NULL;
        pthread_join(th[t], &ret);
        if (ret) rc = -2;
    }
    pthread_mutex_destroy(&J.lock);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Closeness (Sec. 4, Eq. 1 with Wasserman-Faust normalisation) and the */
/* penalised distance sum of Sec. 5.1.                                  */
/* ------------------------------------------------------------------ */

/* cc = ((R-1)/S) * ((R-1)/(n-1)); 0 for an isolated vertex or n <= 1.
 * S sums distances to reachable vertices only (unreachable count 0). */
void oracle_closeness_wf(int32_t n, int32_t count, const int64_t* S, const int32_t* R, double* cc) {
    for (int32_t i = 0; i < count; ++i) {
        if (R[i] > 1 && S[i] > 0 && n > 1) {
            double reach = (double)(R[i] - 1);
            double q1 = reach / (double)S[i];
            double q2 = reach / (double)(n - 1);
            cc[i] = q1 * q2;
        } else {
            cc[i] = 0.0;
        }
    }
}

/* sumDist with every unreachable vertex at distance n: S + n*(n-R). */
void oracle_penalised(int32_t n, int32_t count, const int64_t* S, const int32_t* R, int64_t* P) {
    for (int32_t i = 0; i < count; ++i)
        P[i] = S[i] + (int64_t)n * (int64_t)(n - R[i]);
}

/* ------------------------------------------------------------------ */
/* Boolean AND / OR aggregation of r layers (Sec. 3.1).                 */
/* ------------------------------------------------------------------ */

static int i64_cmp(const void* a, const void* b) {
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* mode 0 = AND (edge kept iff present in every layer), 1 = OR (present in
 * at least one).  Each layer is a normalised symmetric CSR over the same n.
 * The result is written as a normalised symmetric CSR; returns its arc
 * count, -3 if it exceeds cap, -2 on allocation failure. */
int64_t oracle_compose(int32_t mode, int32_t n, int32_t r,
                       const int32_t* const* row_ptrs, const int32_t* const* col_idxs,
                       int32_t* out_row_ptr, int32_t* out_col_idx, int64_t cap) {
    int64_t total = 0;
    for (int32_t l = 0; l < r; ++l) total += row_ptrs[l][n] / 2;
    int64_t* keys = (int64_t*)malloc(sizeof(int64_t) * (size_t)(total + 1));
    if (!keys) return -2;
    int64_t k = 0;
    for (int32_t l = 0; l < r; ++l)
        for (int32_t u = 0; u < n; ++u)
            for (int32_t e = row_ptrs[l][u]; e < row_ptrs[l][u + 1]; ++e) {
                int32_t v = col_idxs[l][e];
                if (u < v) keys[k++] = (int64_t)u * n + v;   /* each edge once, as (min,max) */
            }
    qsort(keys, (size_t)k, sizeof(int64_t), i64_cmp);
    int32_t* eu = (int32_t*)malloc(sizeof(int32_t) * (size_t)(k + 1));
    int32_t* ev = (int32_t*)malloc(sizeof(int32_t) * (size_t)(k + 1));
    if (!eu || !ev) { free(keys); free(eu); free(ev); return -2; }
    int64_t m_out = 0;
    for (int64_t i = 0; i < k;) {
        int64_t j = i;
        while (j < k && keys[j] == keys[i]) ++j;
        int64_t copies = j - i;               /* number of layers holding the edge */
        int keep = (mode == 0) ? (copies == r) : (copies >= 1);
        if (keep) { eu[m_out] = (int32_t)(keys[i] / n); ev[m_out] = (int32_t)(keys[i] % n); ++m_out; }
        i = j;
    }
    free(keys);
    if (2 * m_out > cap) { free(eu); free(ev); return -3; }
    int64_t nnz = oracle_csr_from_edges(n, m_out, eu, ev, out_row_ptr, out_col_idx);
    free(eu); free(ev);
    return nnz;
}

/* ------------------------------------------------------------------ */
/* Selection: mean, above-average set, top-k, CC2, naive.              */
/* ------------------------------------------------------------------ */

/* Mean in the fixed summation shape: sequential sums of id-chunks of 1024,
 * then a sequential sum of the chunk sums, then one division. */
double oracle_mean_fixed_shape(int32_t count, const double* x) {
    if (count <= 0) return 0.0;
    double total = 0.0;
    for (int32_t c = 0; c < count; c += 1024) {
        double part = 0.0;
        int32_t end = c + 1024 < count ? c + 1024 : count;
        for (int32_t i = c; i < end; ++i) part += x[i];
        total += part;
    }
    return total / (double)count;
}

/* ids (ascending) of the entries with x >= mean; returns how many. */
int32_t oracle_above_mean(int32_t count, const double* x, int32_t* ids) {
    double mean = oracle_mean_fixed_shape(count, x);
    int32_t c = 0;
    for (int32_t i = 0; i < count; ++i)
        if (x[i] >= mean) ids[c++] = i;
    return c;
}

typedef struct { double s; int64_t k; int32_t id; } rank_t;

static int rank_desc_cmp(const void* a, const void* b) {
    const rank_t* x = (const rank_t*)a;
    const rank_t* y = (const rank_t*)b;
    if (x->s != y->s) return x->s > y->s ? -1 : 1;   /* larger score first */
    return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}

static int rank_asc_i64_cmp(const void* a, const void* b) {
    const rank_t* x = (const rank_t*)a;
    const rank_t* y = (const rank_t*)b;
    if (x->k != y->k) return x->k < y->k ? -1 : 1;   /* smaller key first */
    return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}

/* The k highest scores, ties by ascending id, in rank order.  Returns k
 * (clamped to count), -2 on allocation failure. */
int32_t oracle_topk_desc(int32_t count, const double* score, int32_t k, int32_t* ids) {
    if (k > count) k = count;
    if (k < 0) k = 0;
    rank_t* t = (rank_t*)malloc(sizeof(rank_t) * (size_t)(count + 1));
    if (!t) return -2;
    for (int32_t i = 0; i < count; ++i) { t[i].s = score[i]; t[i].k = 0; t[i].id = i; }
    qsort(t, (size_t)count, sizeof(rank_t), rank_desc_cmp);
    for (int32_t i = 0; i < k; ++i) ids[i] = t[i].id;
    free(t);
    return k;
}

/* The k smallest integer keys, ties by ascending id, in rank order. */
int32_t oracle_topk_asc_i64(int32_t count, const int64_t* key, int32_t k, int32_t* ids) {
    if (k > count) k = count;
    if (k < 0) k = 0;
    rank_t* t = (rank_t*)malloc(sizeof(rank_t) * (size_t)(count + 1));
    if (!t) return -2;
    for (int32_t i = 0; i < count; ++i) { t[i].s = 0.0; t[i].k = key[i]; t[i].id = i; }
    qsort(t, (size_t)count, sizeof(rank_t), rank_asc_i64_cmp);
    for (int32_t i = 0; i < k; ++i) ids[i] = t[i].id;
    free(t);
    return k;
}

/* CC2 (Sec. 5.2, Algorithm 1): the estimated distance sum of u in the AND
 * graph is the largest of its layers' sums.  The layers' sums are the
 * penalised ones (unreachable = n, Sec. 5.1). */
void oracle_cc2_est(int32_t n, int32_t r, const int64_t* const* S, const int32_t* const* R,
                    int64_t* est) {
    for (int32_t u = 0; u < n; ++u) {
        int64_t best = 0;
        for (int32_t l = 0; l < r; ++l) {
            int64_t p = S[l][u] + (int64_t)n * (int64_t)(n - R[l][u]);
            if (l == 0 || p > best) best = p;
        }
        est[u] = best;
    }
}

/* Eq. 1 applied to the CC2 estimate: (n-1)/est, 0 when est is 0. */
void oracle_cc2_score(int32_t n, const int64_t* est, double* score) {
    for (int32_t u = 0; u < n; ++u)
        score[u] = est[u] > 0 ? (double)(n - 1) / (double)est[u] : 0.0;
}

/* Naive composition (Sec. 4): the intersection of the layers' above-average
 * CC-node sets.  ids ascending; returns how many. */
int32_t oracle_naive(int32_t n, int32_t r, const double* const* cc, int32_t* ids) {
    char* in = (char*)malloc((size_t)n + 1);
    int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
    if (!in || !tmp) { free(in); free(tmp); return -2; }
    for (int32_t u = 0; u < n; ++u) in[u] = 1;
    for (int32_t l = 0; l < r; ++l) {
        char* keep = (char*)calloc((size_t)n + 1, 1);
        if (!keep) { free(in); free(tmp); return -2; }
        int32_t c = oracle_above_mean(n, cc[l], tmp);
        for (int32_t i = 0; i < c; ++i) keep[tmp[i]] = 1;
        for (int32_t u = 0; u < n; ++u) in[u] = in[u] && keep[u];
        free(keep);
    }
    int32_t c = 0;
    for (int32_t u = 0; u < n; ++u) if (in[u]) ids[c++] = u;
    free(in); free(tmp);
    return c;
}

/* Naive composition (Sec. 4) applied to top-k sets: the intersection of
 * the layers' top-k CC-node sets, each by the layer's own closeness (score
 * descending, ties by ascending id).  ids ascending; returns how many (at
 * most k). */
int32_t oracle_naive_topk(int32_t n, int32_t r, const double* const* cc, int32_t k, int32_t* ids) {
    int32_t* hits = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
    int32_t* top = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
    if (!hits || !top) { free(hits); free(top); return -2; }
    for (int32_t l = 0; l < r; ++l) {
        int32_t c = oracle_topk_desc(n, cc[l], k, top);
        if (c < 0) { free(hits); free(top); return c; }
        for (int32_t i = 0; i < c; ++i) hits[top[i]] += 1;
    }
    int32_t c = 0;
    for (int32_t u = 0; u < n; ++u) if (hits[u] == r) ids[c++] = u;
    free(hits); free(top);
    return c;
}

/* ------------------------------------------------------------------ */
/* Closeness of every vertex estimated from a sample of sources (after  */
/* Eppstein and Wang's sampling estimator of closeness, the linear-time */
/* approximation the paper cites among related work, Sec. 2).           */
/* ------------------------------------------------------------------ */

/* Sample sums, source by source: for every vertex v, SQ[v] = sum of d(s, v)
 * over the k listed sources s that reach v, RQ[v] = how many listed sources
 * reach v (v itself when it is listed).  One FIFO BFS per source.  Returns
 * 0, -1 on a bad source id, -2 on allocation failure. */
int oracle_sample_sums(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t k,
                       const int32_t* sources, int64_t* SQ, int32_t* RQ) {
    for (int32_t i = 0; i < k; ++i)
        if (sources[i] < 0 || sources[i] >= n) return -1;
    int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!dist || !queue) { free(dist); free(queue); return -2; }
    for (int32_t v = 0; v < n; ++v) { dist[v] = -1; SQ[v] = 0; RQ[v] = 0; }
    for (int32_t i = 0; i < k; ++i) {
        int32_t s = sources[i], head = 0, tail = 0;
        dist[s] = 0;
        queue[tail++] = s;
        while (head < tail) {
            int32_t u = queue[head++];
            SQ[u] += dist[u];
            RQ[u] += 1;
            for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                int32_t w = col_idx[e];
                if (dist[w] < 0) {
                    dist[w] = 1 + dist[u];
                    queue[tail++] = w;
                }
            }
        }
        for (int32_t j = 0; j < tail; ++j) dist[queue[j]] = -1;
    }
    free(dist); free(queue);
    return 0;
}

/* The same sums for listed vertices only, vertex by vertex: one BFS from v
 * and the distances to the sampled sources added up (the graph is
 * undirected, so d(s, v) = d(v, s)).  in_sample[u] != 0 marks the sample. */
int oracle_sample_sums_at(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const uint8_t* in_sample,
                          int32_t count, const int32_t* verts, int64_t* SQ, int32_t* RQ) {
    int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!dist || !queue) { free(dist); free(queue); return -2; }
    for (int32_t v = 0; v < n; ++v) dist[v] = -1;
    for (int32_t i = 0; i < count; ++i) {
        int32_t v = verts[i], head = 0, tail = 0;
        if (v < 0 || v >= n) { free(dist); free(queue); return -1; }
        int64_t sum = 0;
        int32_t reached = 0;
        dist[v] = 0;
        queue[tail++] = v;
        while (head < tail) {
            int32_t u = queue[head++];
            if (in_sample[u]) { sum += dist[u]; ++reached; }
            for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                int32_t w = col_idx[e];
                if (dist[w] < 0) {
                    dist[w] = dist[u] + (int32_t)1;
                    queue[tail++] = w;
                }
            }
        }
        for (int32_t j = 0; j < tail; ++j) dist[queue[j]] = -1;
        SQ[i] = sum;
        RQ[i] = reached;
    }
    free(dist); free(queue);
    return 0;
}

/* Estimated closeness in the Wasserman-Faust form from sample sums: with
 * q = RQ[v] - [v in sample] (sampled sources other than v reaching v) and
 * k' = k - [v in sample],
 *   mean distance ~ SQ / q, reach fraction ~ q / k',
 *   cc_est = (q / SQ) * (q / k') * ((n_pop - 1) / (n - 1)),
 * where n_pop is the size of the vertex set the sample was drawn from
 * (every vertex outside it reaches nothing).  0 when q == 0 or n <= 1.
 * With the sample equal to all n vertices this is the exact closeness. */
void oracle_sample_estimate(int32_t n, int32_t n_pop, int32_t k, const uint8_t* in_sample, const int64_t* SQ,
                            const int32_t* RQ, double* cc) {
    for (int32_t v = 0; v < n; ++v) {
        int32_t self = in_sample[v] ? 1 : 0;
        int32_t q = RQ[v] - self;
        int32_t kp = k - self;
        if (q > 0 && SQ[v] > 0 && kp > 0 && n > 1) {
            double a = (double)q / (double)SQ[v];
            double b = (double)q / (double)kp;
            double c = (double)(n_pop - 1) / (double)(n - 1);
            cc[v] = (a * b) * c;
        } else {
            cc[v] = 0.0;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Heuristic CC1 (Sec. 5.1, Eq. 2-3).  The paper describes it in words  */
/* and does not print the algorithm; the readings taken here:           */
/*   - sumDist is the penalised sum P = S + n(n - R) (unreachable at    */
/*     distance n, Sec. 5.1);                                           */
/*   - Eq. 2 with r layers: ratio_l(u) = P_l(u) / m(u), m(u) = the      */
/*     smallest degree of u over the layers (the AND graph's degree     */
/*     bound); a vertex with m(u) = 0 has no ratio: it is never central */
/*     and is left out of the average;                                  */
/*   - avg_l = mean of ratio_l over the vertices with m > 0, summed in  */
/*     the fixed shape of oracle_mean_fixed_shape; Eq. 3: the AND       */
/*     graph's average = the largest avg_l;                             */
/*   - central: ratio strictly below that average;                      */
/*   - CH_l = the above-average closeness set of layer l (Sec. 4);      */
/*   - a common CC node c (in every CH_l) is kept when its central      */
/*     neighbour sets C_l(c) overlap significantly: with I = the        */
/*     intersection of the C_l(c) and s = the smallest |C_l(c)|,        */
/*     s > 0 and |I| / s >= tau = tau_num / tau_den (compared as        */
/*     |I| * tau_den >= tau_num * s in integers).                       */
/* ------------------------------------------------------------------ */

/* central: a ratio exists (m > 0) and lies strictly below the average */
static int cc1_central(int32_t m, double ratio, double avg) {
    return m > 0 && ratio < avg;
}

static int in_row(const int32_t* row_ptr, const int32_t* col_idx, int32_t u, int32_t v) {
    for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
        if (col_idx[e] == v) return 1;
    return 0;
}

/* ids ascending of the CC1 nodes; returns how many, -1 on bad arguments,
 * -2 on allocation failure.  avg_out (nullable) receives Eq. 3's value. */
int32_t oracle_cc1(int32_t n, int32_t r, const int32_t* const* row_ptr, const int32_t* const* col_idx,
                   const int64_t* const* S, const int32_t* const* R, int32_t tau_num, int32_t tau_den,
                   int32_t* ids, double* avg_out) {
    if (n < 1 || r < 1 || tau_num < 0 || tau_den < 1) return -1;
    int32_t* m = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    double* ratio = (double*)malloc(sizeof(double) * (size_t)n * (size_t)r);
    double* cc = (double*)malloc(sizeof(double) * (size_t)n);
    int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    char* common = (char*)malloc((size_t)n);
    char* keep = (char*)malloc((size_t)n);
    if (!m || !ratio || !cc || !tmp || !common || !keep) {
        free(m); free(ratio); free(cc); free(tmp); free(common); free(keep);
        return -2;
    }
    /* the AND graph's degree bound */
    for (int32_t u = 0; u < n; ++u) {
        int32_t best = 0;
        for (int32_t l = 0; l < r; ++l) {
            int32_t d = row_ptr[l][u + 1] - row_ptr[l][u];
            if (l == 0 || d < best) best = d;
        }
        m[u] = best;
    }
    /* Eq. 2 per layer, and its average over vertices with a ratio */
    double avg = 0.0;
    for (int32_t l = 0; l < r; ++l) {
        double* x = ratio + (size_t)l * (size_t)n;
        int32_t valid = 0;
        for (int32_t u = 0; u < n; ++u) {
            int64_t P = S[l][u] + (int64_t)n * (int64_t)(n - R[l][u]);
            x[u] = m[u] > 0 ? (double)P / (double)m[u] : 0.0;
            valid += m[u] > 0;
        }
        double total = 0.0;
        for (int32_t c = 0; c < n; c += 1024) {
            double part = 0.0;
            int32_t end = c + 1024 < n ? c + 1024 : n;
            for (int32_t u = c; u < end; ++u)
                if (m[u] > 0) part += x[u];
            total += part;
        }
        double avg_l = valid > 0 ? total / (double)valid : 0.0;
        if (l == 0 || avg_l > avg) avg = avg_l;       /* Eq. 3: the larger average */
    }
    if (avg_out) *avg_out = avg;
    /* common CC nodes */
    for (int32_t u = 0; u < n; ++u) common[u] = 1;
    for (int32_t l = 0; l < r; ++l) {
        oracle_closeness_wf(n, n, S[l], R[l], cc);
        int32_t c = oracle_above_mean(n, cc, tmp);
        for (int32_t u = 0; u < n; ++u) keep[u] = 0;
        for (int32_t i = 0; i < c; ++i) keep[tmp[i]] = 1;
        for (int32_t u = 0; u < n; ++u) common[u] = common[u] && keep[u];
    }
    /* overlap of the central neighbour sets */
    int32_t count = 0;
    for (int32_t c = 0; c < n; ++c) {
        if (!common[c]) continue;
        int64_t smallest = -1;
        for (int32_t l = 0; l < r; ++l) {
            const double* x = ratio + (size_t)l * (size_t)n;
            int64_t size = 0;
            for (int32_t e = row_ptr[l][c]; e < row_ptr[l][c + 1]; ++e) {
                int32_t v = col_idx[l][e];
                size += cc1_central(m[v], x[v], avg);
            }
            if (smallest < 0 || size < smallest) smallest = size;
        }
        int64_t inter = 0;
        for (int32_t e = row_ptr[0][c]; e < row_ptr[0][c + 1]; ++e) {
            int32_t v = col_idx[0][e];
            int all = 1;
            for (int32_t l = 0; l < r && all; ++l)
                all = in_row(row_ptr[l], col_idx[l], c, v) && cc1_central(m[v], ratio[(size_t)l * (size_t)n + v], avg);
            inter += all;
        }
        if (smallest > 0 && inter * (int64_t)tau_den >= (int64_t)tau_num * smallest) ids[count++] = c;
    }
    free(m); free(ratio); free(cc); free(tmp); free(common); free(keep);
    return count;
}
