/*
 * Plain CPU oracle for exact top-k closeness centrality (Borassi, Crescenzi,
 * Marino, "Fast and Simple Computation of Top-k Closeness Centralities").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * GPU library shares no code, header or table with it and never calls it.
 *
 * Everything here is integer arithmetic: distances, reach r(v), farness f(v)
 * and the bounds of Lemma 1 / Lemma 2 are exact integers, and closeness
 * c(v) = (r(v)-1)^2 / ((n-1) f(v)) (Section 1, generalised closeness) is
 * compared through the integer key below instead of a float.
 *
 * Key order (the reading used throughout, since the paper does not discuss
 * ties): every node v gets A(v) = (r(v)-1)^2 and F(v) = f(v), with (A, F) =
 * (0, 1) when r(v) = 1 (closeness 0).  key(v) > key(w) iff
 * A(v) F(w) > A(w) F(v) in unsigned 128-bit arithmetic, or the products are
 * equal and v < w.  The common factor 1/(n-1) never changes the order.
 *
 * Functions:
 *   orc_canonicalize    sort rows, drop self-loops and repeated arcs
 *   orc_bfs             single-source BFS distances
 *   orc_bruteforce      textbook algorithm: one full BFS per node (Section 1)
 *   orc_reach_undirected r(v) = size of the connected component (Section 2.3)
 *   orc_scc             strongly connected components (iterative Tarjan)
 *   orc_alpha_omega     alpha/omega bounds on r(v) over the SCC DAG (Section 2.4)
 *   orc_alpha_omega_ex  the same, optionally with the largest-SCC refinement
 *                       described at the end of Section 2.4
 *   orc_topk            Algorithm 1 with the BFSCut function of Section 2.5
 *   orc_topk_ex         the same, optionally with the tighter bounds the paper
 *                       gives beside the main ones (the undirected footnote of
 *                       Section 2.3 and the largest-SCC refinement)
 *
 * Parity status: pinned (see the oracle tests: closed forms, brute force
 * against SciPy and NetworkX, per-source cut levels re-derived from
 * independent distance matrices, alpha <= r <= omega against brute force).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ CSR */

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* Canonical CSR: each row sorted, self-loops and repeats removed.  Distances
 * and reachability are unchanged by either.  out_col must hold m entries.
 * Returns the new arc count. */
int64_t orc_canonicalize(int32_t n, const int32_t* rp, const int32_t* col,
                         int32_t* out_rp, int32_t* out_col) {
    int64_t w = 0;
    out_rp[0] = 0;
    for (int32_t u = 0; u < n; ++u) {
        int64_t b = rp[u], e = rp[u + 1];
        int64_t start = w;
        for (int64_t i = b; i < e; ++i) out_col[w++] = col[i];
        qsort(out_col + start, (size_t)(w - start), sizeof(int32_t), cmp_i32);
        int64_t k = start;
        for (int64_t i = start; i < w; ++i) {
            int32_t x = out_col[i];
            if (x == u) continue;                      /* self-loop */
            if (k > start && out_col[k - 1] == x) continue; /* repeat */
            out_col[k++] = x;
        }
        w = k;
        out_rp[u + 1] = (int32_t)w;
    }
    return w;
}

/* ------------------------------------------------------------------ BFS */

/* dist[w] = d(src, w) along out-arcs, -1 when w is not reachable. */
void orc_bfs(int32_t n, const int32_t* rp, const int32_t* col, int32_t src, int32_t* dist) {
    int32_t* q = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t i = 0; i < n; ++i) dist[i] = -1;
    int64_t head = 0, tail = 0;
    dist[src] = 0;
    q[tail++] = src;
    while (head < tail) {
        int32_t u = q[head++];
        for (int64_t i = rp[u]; i < rp[u + 1]; ++i) {
            int32_t w = col[i];
            if (dist[w] < 0) {
                dist[w] = dist[u] + 1;
                q[tail++] = w;
            }
        }
    }
    free(q);
}

/* Textbook algorithm: r(v) = |R(v)| (v in R(v)) and f(v) = sum of d(v, w)
 * over w in R(v), by one full BFS per node. */
typedef struct {
    int32_t n;
    const int32_t *rp, *col;
    uint32_t* r;
    uint64_t* f;
    int32_t next;
    pthread_mutex_t mu;
} bf_job;

static void* bf_worker(void* arg) {
    bf_job* J = (bf_job*)arg;
    int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(J->n > 0 ? J->n : 1));
    for (;;) {
        pthread_mutex_lock(&J->mu);
        int32_t v = J->next++;
        pthread_mutex_unlock(&J->mu);
        if (v >= J->n) break;
        orc_bfs(J->n, J->rp, J->col, v, dist);
        uint32_t r = 0;
        uint64_t f = 0;
        for (int32_t w = 0; w < J->n; ++w)
            if (dist[w] >= 0) { r += 1; f += (uint64_t)dist[w]; }
        J->r[v] = r;
        J->f[v] = f;
    }
    free(dist);
    return NULL;
}

void orc_bruteforce(int32_t n, const int32_t* rp, const int32_t* col, uint32_t* r,
                    uint64_t* f, int nthreads) {
    bf_job J = {n, rp, col, r, f, 0, PTHREAD_MUTEX_INITIALIZER};
    if (nthreads < 1) nthreads = 1;
    pthread_t th[256];
    if (nthreads > 256) nthreads = 256;
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, bf_worker, &J);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/* --------------------------------------------------------- reach bounds */

/* Undirected graphs: r(v) is the size of v's connected component, computed
 * once in linear time (Section 2.3). */
void orc_reach_undirected(int32_t n, const int32_t* rp, const int32_t* col, uint32_t* r) {
    int32_t* label = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* q = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t i = 0; i < n; ++i) label[i] = -1;
    for (int32_t s = 0; s < n; ++s) {
        if (label[s] >= 0) continue;
        int64_t head = 0, tail = 0;
        label[s] = s;
        q[tail++] = s;
        while (head < tail) {
            int32_t u = q[head++];
            for (int64_t i = rp[u]; i < rp[u + 1]; ++i)
                if (label[col[i]] < 0) { label[col[i]] = s; q[tail++] = col[i]; }
        }
        for (int64_t i = 0; i < tail; ++i) r[q[i]] = (uint32_t)tail;
    }
    free(label);
    free(q);
}

/* Strongly connected components by Tarjan's algorithm with an explicit
 * stack.  Components are numbered in the order they are completed, which is
 * a reverse topological order of the SCC DAG (a component is completed only
 * after every component it reaches).  Returns the number of components. */
int32_t orc_scc(int32_t n, const int32_t* rp, const int32_t* col, int32_t* comp) {
    size_t N = (size_t)(n > 0 ? n : 1);
    int32_t* index = (int32_t*)malloc(sizeof(int32_t) * N);
    int32_t* low = (int32_t*)malloc(sizeof(int32_t) * N);
    char* on = (char*)calloc(N, 1);
    int32_t* stk = (int32_t*)malloc(sizeof(int32_t) * N);
    int32_t* cs_v = (int32_t*)malloc(sizeof(int32_t) * N);
    int64_t* cs_e = (int64_t*)malloc(sizeof(int64_t) * N);
    int32_t next_index = 0, sp = 0, nc = 0;
    for (int32_t i = 0; i < n; ++i) index[i] = -1;
    for (int32_t s = 0; s < n; ++s) {
        if (index[s] >= 0) continue;
        int32_t top = 0;
        cs_v[0] = s; cs_e[0] = rp[s];
        index[s] = low[s] = next_index++;
        stk[sp++] = s; on[s] = 1;
        while (top >= 0) {
            int32_t v = cs_v[top];
            if (cs_e[top] < rp[v + 1]) {
                int32_t w = col[cs_e[top]++];
                if (index[w] < 0) {
                    index[w] = low[w] = next_index++;
                    stk[sp++] = w; on[w] = 1;
                    ++top;
                    cs_v[top] = w; cs_e[top] = rp[w];
                } else if (on[w] && index[w] < low[v]) {
                    low[v] = index[w];
                }
            } else {
                if (low[v] == index[v]) {
                    int32_t w;
                    do { w = stk[--sp]; on[w] = 0; comp[w] = nc; } while (w != v);
                    ++nc;
                }
                --top;
                if (top >= 0 && low[v] < low[cs_v[top]]) low[cs_v[top]] = low[v];
            }
        }
    }
    free(index); free(low); free(on); free(stk); free(cs_v); free(cs_e);
    return nc;
}

/* Directed graphs: alpha(v) <= r(v) <= omega(v) from the weighted DAG of SCCs
 * (Section 2.4).  With w(C) = |C| and E the set (no repeats) of DAG arcs,
 * processing components in reverse topological order:
 *   alpha(C) = w(C) + max over (C,D) in E of alpha(D)   (0 without successor)
 *   omega(C) = w(C) + sum over (C,D) in E of omega(D),  capped at n
 * The cap keeps the value in range (r(v) <= n always holds).
 *
 * With big_scc != 0 the refinement at the end of Section 2.4 is applied:
 *   - the biggest SCC T (largest w; among equals the one holding the
 *     smallest node id) is not evaluated by the recurrence: a BFS from one
 *     of its nodes gives the exact reach rT = |R(T)|, so alpha(T) = omega(T)
 *     = rT, and the recurrence carries this exact value to every component
 *     that reaches T;
 *   - for a component C that reaches T (C != T), a second upper bound is
 *     rT + omega'(C), where omega' is the same recurrence on the DAG with
 *     every component reachable from T (T included) removed: the nodes that
 *     C reaches outside R(T) are exactly those it reaches in that DAG.
 *     omega(C) is the smaller of the two bounds. */
void orc_alpha_omega_ex(int32_t n, const int32_t* rp, const int32_t* col, int big_scc, uint32_t* alpha,
                        uint32_t* omega) {
    size_t N = (size_t)(n > 0 ? n : 1);
    int32_t* comp = (int32_t*)malloc(sizeof(int32_t) * N);
    int32_t nc = orc_scc(n, rp, col, comp);
    size_t NC = (size_t)(nc > 0 ? nc : 1);
    /* group nodes by component */
    int32_t* cstart = (int32_t*)calloc(NC + 1, sizeof(int32_t));
    int32_t* members = (int32_t*)malloc(sizeof(int32_t) * N);
    for (int32_t v = 0; v < n; ++v) cstart[comp[v] + 1]++;
    for (int32_t c = 0; c < nc; ++c) cstart[c + 1] += cstart[c];
    int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * NC);
    for (int32_t c = 0; c < nc; ++c) fill[c] = cstart[c];
    for (int32_t v = 0; v < n; ++v) members[fill[comp[v]]++] = v;
    uint64_t* a = (uint64_t*)malloc(sizeof(uint64_t) * NC);
    uint64_t* o = (uint64_t*)malloc(sizeof(uint64_t) * NC);
    uint64_t* o2 = (uint64_t*)malloc(sizeof(uint64_t) * NC);   /* omega' (outside R(T)) */
    char* inRT = (char*)calloc(NC, 1);                          /* component in R(T)     */
    char* toT = (char*)calloc(NC, 1);                           /* component reaches T   */
    int32_t* seen = (int32_t*)malloc(sizeof(int32_t) * NC);
    for (int32_t c = 0; c < nc; ++c) seen[c] = -1;
    int32_t T = -1;
    uint64_t rT = 0;
    if (big_scc && n > 0) {
        /* members[] lists each component's nodes in increasing id, so the
         * first member is the component's smallest node */
        for (int32_t c = 0; c < nc; ++c) {
            if (T < 0) { T = c; continue; }
            int32_t wc = cstart[c + 1] - cstart[c], wt = cstart[T + 1] - cstart[T];
            if (wc > wt || (wc == wt && members[cstart[c]] < members[cstart[T]])) T = c;
        }
        int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * N);
        orc_bfs(n, rp, col, members[cstart[T]], dist);
        for (int32_t v = 0; v < n; ++v)
            if (dist[v] >= 0) { rT += 1; inRT[comp[v]] = 1; }
        free(dist);
    }
    for (int32_t c = 0; c < nc; ++c) {   /* completion order = reverse topological */
        uint64_t w = (uint64_t)(cstart[c + 1] - cstart[c]);
        uint64_t amax = 0, osum = 0, osum2 = 0;
        for (int32_t i = cstart[c]; i < cstart[c + 1]; ++i) {
            int32_t v = members[i];
            for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
                int32_t d = comp[col[e]];
                if (d == c || seen[d] == c) continue;  /* each DAG arc once */
                seen[d] = c;
                if (a[d] > amax) amax = a[d];
                osum += o[d];
                if (osum > (uint64_t)n) osum = (uint64_t)n;
                if (d == T || toT[d]) toT[c] = 1;
                if (!inRT[d]) {
                    osum2 += o2[d];
                    if (osum2 > (uint64_t)n) osum2 = (uint64_t)n;
                }
            }
        }
        if (c == T) {
            a[c] = o[c] = rT;   /* exact, from the BFS */
            o2[c] = 0;
            continue;
        }
        a[c] = w + amax;
        o[c] = w + osum;
        if (o[c] > (uint64_t)n) o[c] = (uint64_t)n;
        o2[c] = w + osum2;
        if (o2[c] > (uint64_t)n) o2[c] = (uint64_t)n;
        if (toT[c]) {
            uint64_t b = rT + o2[c];
            if (b > (uint64_t)n) b = (uint64_t)n;
            if (b < o[c]) o[c] = b;
        }
    }
    for (int32_t v = 0; v < n; ++v) {
        alpha[v] = (uint32_t)a[comp[v]];
        omega[v] = (uint32_t)o[comp[v]];
    }
    free(comp); free(cstart); free(members); free(fill); free(a); free(o); free(o2); free(inRT); free(toT);
    free(seen);
}

void orc_alpha_omega(int32_t n, const int32_t* rp, const int32_t* col, uint32_t* alpha, uint32_t* omega) {
    orc_alpha_omega_ex(n, rp, col, 0, alpha, omega);
}

/* ------------------------------------------------------------ top-k list */

typedef struct {
    uint64_t A;   /* (r-1)^2, 0 when r = 1 */
    uint64_t F;   /* f, 1 when r = 1 */
    int32_t id;
    uint32_t r;
    uint64_t f;
} rec_t;

/* key(x) > key(y) */
static int key_gt(const rec_t* x, const rec_t* y) {
    u128 lx = (u128)x->A * (u128)y->F, ly = (u128)y->A * (u128)x->F;
    if (lx != ly) return lx > ly;
    return x->id < y->id;
}

typedef struct {
    rec_t* a;
    int32_t k, cnt;
} topk_t;

/* Keep the k largest keys seen so far, sorted in decreasing key order (the
 * priority queue of Algorithm 1: Kth = a[k-1] once the list is full). */
static void topk_insert(topk_t* T, const rec_t* x) {
    if (T->cnt == T->k && !key_gt(x, &T->a[T->k - 1])) return;
    int32_t i = T->cnt < T->k ? T->cnt++ : T->k - 1;
    while (i > 0 && key_gt(x, &T->a[i - 1])) { T->a[i] = T->a[i - 1]; --i; }
    T->a[i] = *x;
}

/* ------------------------------------------------------------- BFSCut */

typedef struct {
    int32_t n;
    const int32_t *rp, *col;
    int directed;
    const uint32_t *X0, *X1;  /* undirected: X0 = r; directed: X0 = alpha, X1 = omega */
    int footnote;             /* undirected: ~gamma_{d+1} = sum of (deg - 1) over Gamma_d, d >= 1 */
} graph_t;

/* Cut rule of the BFSCut function at level d, right after Gamma_d(v) is
 * known and before it is expanded.  For every candidate reach x (x = r(v)
 * for undirected graphs; x in {alpha(v), omega(v)} for directed ones) the
 * farness lower bound of Lemma 1 is
 *     L_x = f_d - gt + (d+2) (x - n_d),   gt = sum of out-degrees over Gamma_d,
 * and 1/c(v) >= (n-1) min_x L_x / (x-1)^2 (Corollary 1, Lemma 2).  With the
 * current k-th best record th = (A, F, id), v cannot enter the top-k when
 * every x has L_x / (x-1)^2 > F / A, or every x has >= and v > id (ties are
 * broken by id).  Checked by cross-multiplication; L_x <= 0 never cuts. */
static int cut_rule(const graph_t* G, int32_t v, int32_t d, uint64_t nd, uint64_t fd,
                    uint64_t gt, const rec_t* th) {
    uint64_t xs[2];
    int nx = 0;
    xs[nx++] = G->X0[v];
    if (G->directed && G->X1[v] != G->X0[v]) xs[nx++] = G->X1[v];
    int all_gt = 1, all_ge = 1;
    for (int i = 0; i < nx; ++i) {
        uint64_t x = xs[i];
        int64_t L = (int64_t)fd - (int64_t)gt + (int64_t)(d + 2) * ((int64_t)x - (int64_t)nd);
        if (L <= 0) return 0;
        u128 lhs = (u128)(uint64_t)L * (u128)th->A;
        u128 rhs = (u128)th->F * (u128)((x - 1) * (x - 1));
        if (!(lhs > rhs)) all_gt = 0;
        if (!(lhs >= rhs)) all_ge = 0;
    }
    return all_gt || (all_ge && v > th->id);
}

typedef struct {
    uint32_t* mark;   /* mark[w] == stamp  <=>  w visited by the current BFS */
    uint32_t stamp;
    int32_t* queue;   /* BFS queue; Gamma_d occupies queue[qb, qe) */
} scratch_t;

enum { RES_DONE = 0, RES_CUT = 1, RES_TRIVIAL = 2 };

/* The BFSCut function (Section 2.5): BFS from v, tracking
 *   n_d = |N_d(v)|, f_d = sum of distances over N_d(v),
 *   gt  = ~gamma_{d+1}(v) = sum of out-degrees over Gamma_d(v) (Table 1),
 *         or, with G->footnote on an undirected graph and d >= 1, the sum of
 *         (degree - 1): one edge of each node of Gamma_d leads back to
 *         Gamma_{d-1} (the footnote of Section 2.3),
 * testing the cut rule whenever a whole level is known.  Returns RES_CUT with
 * the level of the cut, or RES_DONE with the exact r(v) and f(v).  m_vis
 * counts the arcs scanned. */
static int bfscut(const graph_t* G, scratch_t* S, int32_t v, const rec_t* th, uint32_t* r_out,
                  uint64_t* f_out, int32_t* level_out, uint64_t* mvis_out) {
    const int32_t* rp = G->rp;
    const int32_t* col = G->col;
    *mvis_out = 0;
    if (G->X0[v] <= 1) {  /* r(v) = 1 (undirected) or alpha(v) = 1 (directed) */
        *r_out = 1; *f_out = 0; *level_out = -2;
        return RES_TRIVIAL;
    }
    if (++S->stamp == 0) {
        memset(S->mark, 0, sizeof(uint32_t) * (size_t)G->n);
        S->stamp = 1;
    }
    uint32_t st = S->stamp;
    S->mark[v] = st;
    S->queue[0] = v;
    int64_t qb = 0, qe = 1;
    int32_t d = 0;
    uint64_t nd = 1, fd = 0, gt = (uint64_t)(rp[v + 1] - rp[v]), mvis = 0;
    for (;;) {
        if (th && cut_rule(G, v, d, nd, fd, gt, th)) {
            *level_out = d; *mvis_out = mvis;
            return RES_CUT;
        }
        int64_t ne = qe;
        for (int64_t i = qb; i < qe; ++i) {
            int32_t u = S->queue[i];
            for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
                int32_t w = col[e];
                ++mvis;
                if (S->mark[w] != st) { S->mark[w] = st; S->queue[ne++] = w; }
            }
        }
        if (ne == qe) {  /* Gamma_{d+1} is empty: the visit is complete */
            *r_out = (uint32_t)nd; *f_out = fd; *level_out = -1; *mvis_out = mvis;
            return RES_DONE;
        }
        d += 1;
        uint64_t cnt = (uint64_t)(ne - qe);
        nd += cnt;
        fd += (uint64_t)d * cnt;
        gt = 0;
        for (int64_t i = qe; i < ne; ++i) {
            uint64_t deg = (uint64_t)(rp[S->queue[i] + 1] - rp[S->queue[i]]);
            gt += (G->footnote && !G->directed && deg > 0) ? deg - 1 : deg;
        }
        qb = qe; qe = ne;
    }
}

/* ------------------------------------------------------- Algorithm 1 */

typedef struct {
    uint64_t m_vis;
    uint64_t n_cut, n_done, n_trivial;
} orc_stats;

typedef struct {
    const graph_t* G;
    const int32_t* order;
    topk_t* T;
    int32_t next;
    pthread_mutex_t mu;
    int32_t* cut_level;
    uint64_t* mvis_node;
    orc_stats st;
} run_t;

static void process(run_t* R, scratch_t* S, int32_t v, int locked_updates) {
    rec_t th, *thp = NULL;
    if (locked_updates) pthread_mutex_lock(&R->mu);
    if (R->T->cnt == R->T->k) { th = R->T->a[R->T->k - 1]; thp = &th; }
    if (locked_updates) pthread_mutex_unlock(&R->mu);
    uint32_t r; uint64_t f, mv; int32_t lvl;
    int res = bfscut(R->G, S, v, thp, &r, &f, &lvl, &mv);
    if (locked_updates) pthread_mutex_lock(&R->mu);
    R->st.m_vis += mv;
    if (R->cut_level) R->cut_level[v] = lvl;
    if (R->mvis_node) R->mvis_node[v] = mv;
    if (res == RES_CUT) {
        R->st.n_cut++;
    } else {
        rec_t x;
        x.id = v; x.r = r; x.f = f;
        if (r <= 1) { x.A = 0; x.F = 1; } else { x.A = (uint64_t)(r - 1) * (uint64_t)(r - 1); x.F = f; }
        if (res == RES_TRIVIAL) R->st.n_trivial++; else R->st.n_done++;
        topk_insert(R->T, &x);
    }
    if (locked_updates) pthread_mutex_unlock(&R->mu);
}

static void* topk_worker(void* arg) {
    run_t* R = (run_t*)arg;
    scratch_t S;
    size_t N = (size_t)(R->G->n > 0 ? R->G->n : 1);
    S.mark = (uint32_t*)calloc(N, sizeof(uint32_t));
    S.queue = (int32_t*)malloc(sizeof(int32_t) * N);
    S.stamp = 0;
    for (;;) {
        pthread_mutex_lock(&R->mu);
        int32_t i = R->next++;
        pthread_mutex_unlock(&R->mu);
        if (i >= R->G->n) break;
        process(R, &S, R->order[i], 1);
    }
    free(S.mark); free(S.queue);
    return NULL;
}

static const int32_t* g_deg_for_sort;
static int cmp_degree_order(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    int32_t dx = g_deg_for_sort[x], dy = g_deg_for_sort[y];
    if (dx != dy) return dx > dy ? -1 : 1;  /* decreasing out-degree */
    return (x > y) - (x < y);               /* then increasing id */
}

/* orc_topk_ex flags: the optional tighter bounds (each leaves the result
 * unchanged and can only cut earlier). */
#define ORC_FOOTNOTE 0x1u   /* undirected ~gamma with (degree - 1) for d >= 1 (Section 2.3 footnote) */
#define ORC_BIG_SCC  0x2u   /* directed reach bounds with the largest-SCC refinement (Section 2.4) */

/* Algorithm 1: canonicalise, compute the reach data, then for every node in
 * the given order (decreasing out-degree, ties by increasing id, when
 * order == NULL) run BFSCut against the current k-th best record and keep
 * the top-k list.  With nthreads > 1 the loop is shared by threads that read
 * the k-th best record when they start a node (a stale value only weakens
 * the cut, Section 2.1).  Outputs ids/f/r (min(k, n) entries, decreasing
 * key order); cut_level[v] (-2 trivial, -1 completed, d >= 0 cut at level d)
 * and mvis_node[v] are optional per-node traces.  Returns the entry count,
 * or -1 on an allocation failure. */
int32_t orc_topk_ex(int32_t n, const int32_t* rp_in, const int32_t* col_in, int directed, int32_t k,
                    const int32_t* order_in, int nthreads, uint32_t flags, int32_t* ids, uint64_t* f_out,
                    uint32_t* r_out, int32_t* cut_level, uint64_t* mvis_node, orc_stats* st) {
    if (k <= 0 || n <= 0) {
        if (st) memset(st, 0, sizeof(*st));
        return 0;
    }
    size_t N = (size_t)n;
    int64_t m_in = rp_in[n];
    int32_t* rp = (int32_t*)malloc(sizeof(int32_t) * (N + 1));
    int32_t* col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m_in > 0 ? m_in : 1));
    uint32_t* X0 = (uint32_t*)malloc(sizeof(uint32_t) * N);
    uint32_t* X1 = (uint32_t*)malloc(sizeof(uint32_t) * N);
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * N);
    int32_t kk = k < n ? k : n;
    rec_t* recs = (rec_t*)malloc(sizeof(rec_t) * (size_t)kk);
    if (!rp || !col || !X0 || !X1 || !order || !recs) return -1;
    orc_canonicalize(n, rp_in, col_in, rp, col);
    if (directed) orc_alpha_omega_ex(n, rp, col, (flags & ORC_BIG_SCC) != 0, X0, X1);
    else { orc_reach_undirected(n, rp, col, X0); memcpy(X1, X0, sizeof(uint32_t) * N); }
    if (order_in) {
        memcpy(order, order_in, sizeof(int32_t) * N);
    } else {
        int32_t* deg = (int32_t*)malloc(sizeof(int32_t) * N);
        for (int32_t v = 0; v < n; ++v) { deg[v] = rp[v + 1] - rp[v]; order[v] = v; }
        g_deg_for_sort = deg;
        qsort(order, N, sizeof(int32_t), cmp_degree_order);
        free(deg);
    }
    graph_t G = {n, rp, col, directed, X0, X1, (flags & ORC_FOOTNOTE) != 0};
    topk_t T = {recs, kk, 0};
    run_t R;
    memset(&R, 0, sizeof(R));
    R.G = &G; R.order = order; R.T = &T; R.next = 0;
    pthread_mutex_init(&R.mu, NULL);
    R.cut_level = cut_level; R.mvis_node = mvis_node;
    if (nthreads <= 1) {
        scratch_t S;
        S.mark = (uint32_t*)calloc(N, sizeof(uint32_t));
        S.queue = (int32_t*)malloc(sizeof(int32_t) * N);
        S.stamp = 0;
        for (int32_t i = 0; i < n; ++i) process(&R, &S, order[i], 0);
        free(S.mark); free(S.queue);
    } else {
        if (nthreads > 256) nthreads = 256;
        pthread_t th[256];
        for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, topk_worker, &R);
        for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    }
    for (int32_t i = 0; i < T.cnt; ++i) { ids[i] = recs[i].id; f_out[i] = recs[i].f; r_out[i] = recs[i].r; }
    if (st) *st = R.st;
    int32_t cnt = T.cnt;
    free(rp); free(col); free(X0); free(X1); free(order); free(recs);
    return cnt;
}

int32_t orc_topk(int32_t n, const int32_t* rp_in, const int32_t* col_in, int directed, int32_t k,
                 const int32_t* order_in, int nthreads, int32_t* ids, uint64_t* f_out,
                 uint32_t* r_out, int32_t* cut_level, uint64_t* mvis_node, orc_stats* st) {
    return orc_topk_ex(n, rp_in, col_in, directed, k, order_in, nthreads, 0u, ids, f_out, r_out, cut_level,
                       mvis_node, st);
}
