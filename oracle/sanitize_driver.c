/*
 * Command-line driver of the oracle for sanitizer builds.
 *
 * TEST INFRASTRUCTURE ONLY (built and run by the oracle tests with
 * AddressSanitizer and UndefinedBehaviorSanitizer; never part of the GPU
 * library).  It reads one graph from a binary file, runs every oracle
 * function on it and prints the results as text, so that a test can compare
 * them with the unsanitized oracle loaded in the test process.
 *
 * Input file (little-endian): int32 n, int64 m, int32 directed, int32 k,
 * int32 flags (orc_topk_ex), int32 nthreads, then row_ptr[n + 1] and col[m]
 * as int32.
 *
 * Output lines:
 *   canon <m'>                    arcs after canonicalisation
 *   scc <count>                   strongly connected components
 *   reach <sum lo> <sum hi>       sums of the reach data (alpha/omega or r)
 *   brute <sum r> <sum f>         textbook sums (only when n <= 4000)
 *   topk <count> <m_vis> <n_cut> <n_done> <n_trivial>
 *   <id> <f> <r>                  one line per result
 *   trace <sum cut levels> <sum per-node m_vis>
 */
#include <inttypes.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    uint64_t m_vis, n_cut, n_done, n_trivial;
} orc_stats;

int64_t orc_canonicalize(int32_t n, const int32_t* rp, const int32_t* col, int32_t* out_rp, int32_t* out_col);
void orc_bruteforce(int32_t n, const int32_t* rp, const int32_t* col, uint32_t* r, uint64_t* f, int nthreads);
void orc_reach_undirected(int32_t n, const int32_t* rp, const int32_t* col, uint32_t* r);
int32_t orc_scc(int32_t n, const int32_t* rp, const int32_t* col, int32_t* comp);
void orc_alpha_omega_ex(int32_t n, const int32_t* rp, const int32_t* col, int big_scc, uint32_t* alpha,
                        uint32_t* omega);
int32_t orc_topk_ex(int32_t n, const int32_t* rp, const int32_t* col, int directed, int32_t k,
                    const int32_t* order, int nthreads, uint32_t flags, int32_t* ids, uint64_t* f, uint32_t* r,
                    int32_t* cut_level, uint64_t* mvis, orc_stats* st);

static void* xmalloc(size_t bytes) {
    void* p = malloc(bytes ? bytes : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(3);
    }
    return p;
}

int main(int argc, char** argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s graph.bin\n", argv[0]);
        return 2;
    }
    FILE* fp = fopen(argv[1], "rb");
    if (!fp) return 2;
    int32_t n, directed, k, flags, nthreads;
    int64_t m;
    if (fread(&n, 4, 1, fp) != 1 || fread(&m, 8, 1, fp) != 1 || fread(&directed, 4, 1, fp) != 1 ||
        fread(&k, 4, 1, fp) != 1 || fread(&flags, 4, 1, fp) != 1 || fread(&nthreads, 4, 1, fp) != 1)
        return 2;
    int32_t* rp = xmalloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t* col = xmalloc(sizeof(int32_t) * (size_t)m);
    if (fread(rp, 4, (size_t)n + 1, fp) != (size_t)n + 1 || fread(col, 4, (size_t)m, fp) != (size_t)m) return 2;
    fclose(fp);

    int32_t* crp = xmalloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t* ccol = xmalloc(sizeof(int32_t) * (size_t)m);
    const int64_t mc = orc_canonicalize(n, rp, col, crp, ccol);
    printf("canon %" PRId64 "\n", mc);

    int32_t* comp = xmalloc(sizeof(int32_t) * (size_t)n);
    printf("scc %d\n", orc_scc(n, crp, ccol, comp));

    uint32_t* lo = xmalloc(sizeof(uint32_t) * (size_t)n);
    uint32_t* hi = xmalloc(sizeof(uint32_t) * (size_t)n);
    if (directed) {
        orc_alpha_omega_ex(n, crp, ccol, (flags & 0x2) != 0, lo, hi);
    } else {
        orc_reach_undirected(n, crp, ccol, lo);
        for (int32_t v = 0; v < n; ++v) hi[v] = lo[v];
    }
    uint64_t slo = 0, shi = 0;
    for (int32_t v = 0; v < n; ++v) {
        slo += lo[v];
        shi += hi[v];
    }
    printf("reach %" PRIu64 " %" PRIu64 "\n", slo, shi);

    if (n <= 4000) {
        uint32_t* br = xmalloc(sizeof(uint32_t) * (size_t)n);
        uint64_t* bf = xmalloc(sizeof(uint64_t) * (size_t)n);
        orc_bruteforce(n, crp, ccol, br, bf, nthreads);
        uint64_t sr = 0, sf = 0;
        for (int32_t v = 0; v < n; ++v) {
            sr += br[v];
            sf += bf[v];
        }
        printf("brute %" PRIu64 " %" PRIu64 "\n", sr, sf);
        free(br);
        free(bf);
    }

    const int32_t kk = k < n ? k : n;
    int32_t* ids = xmalloc(sizeof(int32_t) * (size_t)(kk > 0 ? kk : 1));
    uint64_t* f = xmalloc(sizeof(uint64_t) * (size_t)(kk > 0 ? kk : 1));
    uint32_t* r = xmalloc(sizeof(uint32_t) * (size_t)(kk > 0 ? kk : 1));
    int32_t* cl = xmalloc(sizeof(int32_t) * (size_t)n);
    uint64_t* mv = xmalloc(sizeof(uint64_t) * (size_t)n);
    orc_stats st = {0, 0, 0, 0};
    /* the trace (cut levels, per-node arcs) is filled by the sequential loop only */
    const int32_t cnt = orc_topk_ex(n, rp, col, directed, k, NULL, nthreads, (uint32_t)flags, ids, f, r,
                                    nthreads == 1 ? cl : NULL, nthreads == 1 ? mv : NULL, &st);
    printf("topk %d %" PRIu64 " %" PRIu64 " %" PRIu64 " %" PRIu64 "\n", cnt, st.m_vis, st.n_cut, st.n_done,
           st.n_trivial);
    for (int32_t i = 0; i < cnt; ++i) printf("%d %" PRIu64 " %u\n", ids[i], f[i], r[i]);
    if (nthreads == 1) {
        int64_t scl = 0;
        uint64_t smv = 0;
        for (int32_t v = 0; v < n; ++v) {
            scl += cl[v];
            smv += mv[v];
        }
        printf("trace %" PRId64 " %" PRIu64 "\n", scl, smv);
    }
    free(rp);
    free(col);
    free(crp);
    free(ccol);
    free(comp);
    free(lo);
    free(hi);
    free(ids);
    free(f);
    free(r);
    free(cl);
    free(mv);
    return 0;
}
