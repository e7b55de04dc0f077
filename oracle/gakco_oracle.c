/*
 * GaKCo CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of the gapped k-mer
 * string kernel computed by GaKCo (Singh, Sekhon, Lanchantin, Kowsari, Wang,
 * Qi: "GaKCo: a Fast Gapped k-mer string Kernel using Counting",
 * arXiv:1704.07468).  It is the checker the GPU library is compared against;
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header, table or helper with the GPU
 * library, and nothing here is blocked, fused or reordered beyond what the
 * paper's Algorithm 1 states.
 *
 * What it computes (Section 2.1, Eqs. 5-7; Section 2.2, Algorithm 1):
 *   g-mers      every contiguous length-g substring of every sequence
 *               (Section 2.2 step 1; the definition of g_i^x under Eq. 5).
 *   C_m(X,Y)    cumulative mismatch profile: for every one of the C(g,m)
 *               sets of m positions, drop those positions from every g-mer,
 *               sort the reduced strings, and for each run of equal reduced
 *               strings add count_X * count_Y into C_m[X][Y]  (Section 2.2
 *               step 3; Algorithm 1 MISMATCHPROFILE, the loop over masks).
 *   N_m         exact mismatch profile by inclusion-exclusion, Eq. 9:
 *               N_m = C_m - sum_{j<m} C(g-j, m-j) N_j.
 *   K           K = sum_{m=0}^{g-k} h_m N_m with h_m = C(g-m, k)  (Eqs. 6-7;
 *               Algorithm 1 CALCULATEKERNEL).
 *   K-hat       cosine normalisation K_ij / sqrt(K_ii K_jj), 0 when either
 *               diagonal entry is 0.  The paper only says counts are
 *               "normalized" (Eq. 3); this reading is listed with the others
 *               in the design notes.
 *
 * Readings taken where the paper is silent:
 *   - self pairs: Eq. 5 sums over all g-mer pairs, so every group (also a
 *     group of one g-mer) adds count^2 to the diagonal; the "(if > 1)" remark
 *     of Section 2.2 step 2 can only apply to off-diagonal entries.
 *   - a sequence shorter than g has no g-mers: its rows, columns and
 *     normalised diagonal are 0.
 *   - the mask loop of Algorithm 1 runs over the C(g,m) m-subsets of
 *     positions (n_pos of them, upper bound exclusive).
 *
 * Parallel modes (they change no arithmetic: every thread adds exact int64
 * products into a private matrix and the matrices are summed at the end):
 *   per level  Section 2.2 ("Parallelization"): one thread per m, the paper's
 *              own parallel version, offered to time that design;
 *   per mask   Section S:5.3 ("GaKCo-Parallel+"): the position sets of all
 *              levels are dealt to the threads, which is how the tests run
 *              the oracle at full workload sizes.
 *
 * Parity status: every function here is pinned by the CPU tests against
 * brute force on tiny inputs (pairwise Hamming distances, Eq. 4 feature-map
 * enumeration), the Fig. 2 worked example, the k = g spectrum special case
 * and the k = 0 whole-profile invariant.
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2

/* binomial coefficient C(n, r) as an exact 64-bit integer (0 when r<0 or r>n) */
static int64_t orc_binom(int n, int r)
{
    if (r < 0 || n < 0 || r > n) return 0;
    int64_t v = 1;
    for (int i = 1; i <= r; ++i) v = v * (n - r + i) / i;
    return v;
}

int64_t orc_binomial(int n, int r) { return orc_binom(n, r); }

/* number of g-mers of a sequence of length l (Section 2.2 step 1) */
static int64_t orc_ngmers(int32_t l, int32_t g)
{
    return (l >= g) ? (int64_t)(l - g + 1) : 0;
}

int64_t orc_total_gmers(const int32_t *lens, int32_t N, int32_t g)
{
    int64_t T = 0;
    for (int32_t i = 0; i < N; ++i) T += orc_ngmers(lens[i], g);
    return T;
}

/* ---------------------------------------------------------------------- */
/* Step 1: the g-mer array L (Section 2.2 step 1; Algorithm 1 "Require")  */
/* ---------------------------------------------------------------------- */
typedef struct {
    int32_t g;
    int64_t T;
    uint8_t *sym;   /* [T][g] the symbols of each g-mer               */
    int32_t *sid;   /* [T]    the index of the sequence it came from  */
} orc_gmer_list;

static int orc_extract(const int8_t *seqs, const int32_t *lens, int32_t N,
                       int32_t g, orc_gmer_list *L)
{
    L->g = g;
    L->T = orc_total_gmers(lens, N, g);
    L->sym = (uint8_t *)malloc((size_t)(L->T > 0 ? L->T : 1) * (size_t)g);
    L->sid = (int32_t *)malloc((size_t)(L->T > 0 ? L->T : 1) * sizeof(int32_t));
    if (!L->sym || !L->sid) { free(L->sym); free(L->sid); return ORC_ENOMEM; }
    int64_t off = 0, t = 0;
    for (int32_t x = 0; x < N; ++x) {
        for (int64_t p = 0; p < orc_ngmers(lens[x], g); ++p) {
            for (int32_t j = 0; j < g; ++j)
                L->sym[t * g + j] = (uint8_t)seqs[off + p + j];
            L->sid[t] = x;
            ++t;
        }
        off += lens[x];
    }
    return ORC_OK;
}

static void orc_free_list(orc_gmer_list *L)
{
    free(L->sym);
    free(L->sid);
}

int64_t orc_gmers(const int8_t *seqs, const int32_t *lens, int32_t N, int32_t g,
                  uint8_t *sym_out, int32_t *sid_out, int64_t cap)
{
    orc_gmer_list L;
    if (g < 1) return ORC_EINVAL;
    if (orc_extract(seqs, lens, N, g, &L) != ORC_OK) return ORC_ENOMEM;
    if (L.T > cap) { orc_free_list(&L); return ORC_EINVAL; }
    memcpy(sym_out, L.sym, (size_t)L.T * (size_t)g);
    memcpy(sid_out, L.sid, (size_t)L.T * sizeof(int32_t));
    int64_t T = L.T;
    orc_free_list(&L);
    return T;
}

/* ---------------------------------------------------------------------- */
/* removePosition / sort / countAndUpdate for one set of m positions      */
/* (Section 2.2 step 3; Algorithm 1, body of the mask loop)               */
/* ---------------------------------------------------------------------- */

/* A record of the reduced list L^i: the (g-m) kept symbols followed by the
 * sequence index.  Records are compared lexicographically on the symbols,
 * then on the sequence index, so equal reduced strings form one run whose
 * entries are grouped by sequence. */
typedef struct {
    int32_t width; /* g - m */
    size_t stride; /* width + sizeof(int32_t) */
} orc_rec_layout;

static int orc_rec_cmp(const void *a, const void *b, void *ctx)
{
    const orc_rec_layout *lay = (const orc_rec_layout *)ctx;
    int c = memcmp(a, b, (size_t)lay->width);
    if (c != 0) return c;
    int32_t sa, sb;
    memcpy(&sa, (const uint8_t *)a + lay->width, sizeof(int32_t));
    memcpy(&sb, (const uint8_t *)b + lay->width, sizeof(int32_t));
    return (sa > sb) - (sa < sb);
}

/* removePosition(L, P): the reduced list, one record per g-mer */
static uint8_t *orc_remove_positions(const orc_gmer_list *L, const int32_t *removed,
                                     int32_t m, orc_rec_layout *lay)
{
    lay->width = L->g - m;
    lay->stride = (size_t)lay->width + sizeof(int32_t);
    uint8_t *recs = (uint8_t *)malloc((size_t)(L->T > 0 ? L->T : 1) * lay->stride);
    if (!recs) return NULL;
    for (int64_t t = 0; t < L->T; ++t) {
        uint8_t *r = recs + (size_t)t * lay->stride;
        int32_t w = 0;
        for (int32_t j = 0; j < L->g; ++j) {
            int drop = 0;
            for (int32_t q = 0; q < m; ++q)
                if (removed[q] == j) drop = 1;
            if (!drop) r[w++] = L->sym[t * L->g + j];
        }
        memcpy(r + lay->width, &L->sid[t], sizeof(int32_t));
    }
    return recs;
}

/* One group of the sorted reduced list: the sequences holding the reduced
 * string and how many times each holds it. */
typedef struct {
    int32_t n;
    int32_t *sid;
    int64_t *cnt;
} orc_group;

/* Walk the sorted records; call `visit` once per run of equal reduced strings. */
typedef void (*orc_group_visitor)(const orc_group *grp, int64_t first_rec, void *arg);

static void orc_count_groups(const uint8_t *recs, int64_t T, const orc_rec_layout *lay,
                             int32_t *sid_buf, int64_t *cnt_buf,
                             orc_group_visitor visit, void *arg)
{
    int64_t i = 0;
    while (i < T) {
        const uint8_t *ri = recs + (size_t)i * lay->stride;
        int64_t j = i;
        orc_group grp = {0, sid_buf, cnt_buf};
        while (j < T && memcmp(recs + (size_t)j * lay->stride, ri, (size_t)lay->width) == 0) {
            int32_t s;
            memcpy(&s, recs + (size_t)j * lay->stride + lay->width, sizeof(int32_t));
            if (grp.n > 0 && grp.sid[grp.n - 1] == s) {
                grp.cnt[grp.n - 1] += 1;
            } else {
                grp.sid[grp.n] = s;
                grp.cnt[grp.n] = 1;
                grp.n += 1;
            }
            ++j;
        }
        visit(&grp, i, arg);
        i = j;
    }
}

/* countAndUpdate: every ordered pair of sequences in the group gains
 * count_X * count_Y (the diagonal included). */
typedef struct {
    int64_t *C; /* [N][N] */
    int32_t N;
} orc_update_ctx;

static void orc_update_visitor(const orc_group *grp, int64_t first_rec, void *arg)
{
    (void)first_rec;
    orc_update_ctx *u = (orc_update_ctx *)arg;
    for (int32_t a = 0; a < grp->n; ++a)
        for (int32_t b = 0; b < grp->n; ++b)
            u->C[(int64_t)grp->sid[a] * u->N + grp->sid[b]] += grp->cnt[a] * grp->cnt[b];
}

/* C_m^i for one position set, added into C (an N x N int64 matrix). */
static int orc_add_mask(const orc_gmer_list *L, int32_t N, const int32_t *removed,
                        int32_t m, int64_t *C)
{
    orc_rec_layout lay;
    uint8_t *recs = orc_remove_positions(L, removed, m, &lay);
    int32_t *sid_buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
    int64_t *cnt_buf = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    if (!recs || !sid_buf || !cnt_buf) {
        free(recs); free(sid_buf); free(cnt_buf);
        return ORC_ENOMEM;
    }
    qsort_r(recs, (size_t)L->T, lay.stride, orc_rec_cmp, &lay);
    orc_update_ctx u = {C, N};
    orc_count_groups(recs, L->T, &lay, sid_buf, cnt_buf, orc_update_visitor, &u);
    free(recs); free(sid_buf); free(cnt_buf);
    return ORC_OK;
}

/* next m-subset of {0..g-1} in lexicographic order; returns 0 after the last */
static int orc_next_subset(int32_t *P, int32_t m, int32_t g)
{
    int32_t i = m - 1;
    while (i >= 0 && P[i] == g - m + i) --i;
    if (i < 0) return 0;
    P[i] += 1;
    for (int32_t j = i + 1; j < m; ++j) P[j] = P[j - 1] + 1;
    return 1;
}

/* C_m: the sum over all C(g,m) position sets (Algorithm 1, lines 10-17). */
static int orc_cumulative_profile(const orc_gmer_list *L, int32_t N, int32_t m, int64_t *Cm)
{
    memset(Cm, 0, sizeof(int64_t) * (size_t)N * (size_t)N);
    int32_t P[64];
    for (int32_t j = 0; j < m; ++j) P[j] = j;
    do {
        int rc = orc_add_mask(L, N, P, m, Cm);
        if (rc != ORC_OK) return rc;
    } while (m > 0 && orc_next_subset(P, m, L->g));
    return ORC_OK;
}

typedef struct {
    const orc_gmer_list *L;
    int32_t N, m;
    int64_t *Cm;
    int rc;
} orc_level_job;

static void *orc_level_thread(void *arg)
{
    orc_level_job *j = (orc_level_job *)arg;
    j->rc = orc_cumulative_profile(j->L, j->N, j->m, j->Cm);
    return NULL;
}

/* Per-mask parallel mode (Section S:5.3): thread t takes every nthreads-th
 * position set of the list of all levels' position sets and adds its
 * products into a private [M+1][N][N] matrix. */
typedef struct {
    const orc_gmer_list *L;
    int32_t N, M, tid, nthreads;
    int64_t *C;  /* private [M+1][N][N], zeroed */
    int rc;
} orc_mask_job;

static void *orc_mask_thread(void *arg)
{
    orc_mask_job *j = (orc_mask_job *)arg;
    const size_t NN = (size_t)j->N * (size_t)j->N;
    int64_t item = 0;
    for (int32_t m = 0; m <= j->M && j->rc == ORC_OK; ++m) {
        int32_t P[64];
        for (int32_t q = 0; q < m; ++q) P[q] = q;
        do {
            if (item % j->nthreads == j->tid) j->rc = orc_add_mask(j->L, j->N, P, m, j->C + (size_t)m * NN);
            ++item;
        } while (j->rc == ORC_OK && m > 0 && orc_next_subset(P, m, j->L->g));
    }
    return NULL;
}

static int orc_profiles_per_mask(const orc_gmer_list *L, int32_t N, int32_t M, int32_t nthreads, int64_t *C)
{
    const size_t NN = (size_t)N * (size_t)N, tot = NN * (size_t)(M + 1);
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    orc_mask_job jobs[256];
    int rc = ORC_OK;
    int32_t started = 0;
    /* thread 0 adds into C itself, the others into private zeroed copies */
    memset(C, 0, sizeof(int64_t) * tot);
    for (int32_t t = 0; t < nthreads; ++t) {
        int64_t *priv = t ? (int64_t *)calloc(tot ? tot : 1, sizeof(int64_t)) : C;
        if (!priv) { rc = ORC_ENOMEM; break; }
        jobs[t] = (orc_mask_job){L, N, M, t, nthreads, priv, ORC_OK};
        ++started;
    }
    if (rc == ORC_OK) {
        for (int32_t t = 0; t < started; ++t) pthread_create(&th[t], NULL, orc_mask_thread, &jobs[t]);
        for (int32_t t = 0; t < started; ++t) pthread_join(th[t], NULL);
    }
    for (int32_t t = 0; t < started; ++t) {
        if (rc == ORC_OK && jobs[t].rc != ORC_OK) rc = jobs[t].rc;
        if (t == 0) continue;
        if (rc == ORC_OK)
            for (size_t e = 0; e < tot; ++e) C[e] += jobs[t].C[e];
        free(jobs[t].C);
    }
    return rc;
}

/* MISMATCHPROFILE(L, g, M): C_0..C_M, then N_0..N_M by Eq. 9.
 * nthreads <= 1: sequential; otherwise one thread per m (per_mask = 0) or
 * the position sets dealt to nthreads threads (per_mask = 1). */
int orc_mismatch_profile(const int8_t *seqs, const int32_t *lens, int32_t N, int32_t g,
                         int32_t M, int32_t nthreads, int32_t per_mask, int64_t *C_out, int64_t *Nm_out)
{
    if (N < 0 || g < 1 || M < 0 || M > g || !Nm_out) return ORC_EINVAL;
    for (int32_t i = 0; i < N; ++i)
        if (lens[i] < 0) return ORC_EINVAL;
    orc_gmer_list L;
    if (orc_extract(seqs, lens, N, g, &L) != ORC_OK) return ORC_ENOMEM;
    const size_t NN = (size_t)N * (size_t)N;
    int64_t *C = C_out ? C_out : (int64_t *)malloc(sizeof(int64_t) * (NN ? NN : 1) * (size_t)(M + 1));
    if (!C) { orc_free_list(&L); return ORC_ENOMEM; }

    int rc = ORC_OK;
    if (nthreads <= 1) {
        for (int32_t m = 0; m <= M && rc == ORC_OK; ++m)
            rc = orc_cumulative_profile(&L, N, m, C + (size_t)m * NN);
    } else if (per_mask) {
        rc = orc_profiles_per_mask(&L, N, M, nthreads, C);
    } else {
        /* one thread per m, as in the paper's parallel version */
        pthread_t th[65];
        orc_level_job jobs[65];
        for (int32_t m = 0; m <= M; ++m) {
            jobs[m] = (orc_level_job){&L, N, m, C + (size_t)m * NN, ORC_OK};
            pthread_create(&th[m], NULL, orc_level_thread, &jobs[m]);
        }
        for (int32_t m = 0; m <= M; ++m) {
            pthread_join(th[m], NULL);
            if (jobs[m].rc != ORC_OK) rc = jobs[m].rc;
        }
    }
    if (rc == ORC_OK) {
        /* Eq. 9: N_m = C_m - sum_{j<m} C(g-j, m-j) N_j  (Algorithm 1, lines 18-21) */
        for (int32_t m = 0; m <= M; ++m) {
            int64_t *Nm = Nm_out + (size_t)m * NN;
            const int64_t *Cm = C + (size_t)m * NN;
            for (size_t e = 0; e < NN; ++e) Nm[e] = Cm[e];
            for (int32_t j = 0; j < m; ++j) {
                const int64_t coef = orc_binom(g - j, m - j);
                const int64_t *Nj = Nm_out + (size_t)j * NN;
                for (size_t e = 0; e < NN; ++e) Nm[e] -= coef * Nj[e];
            }
        }
    }
    if (!C_out) free(C);
    orc_free_list(&L);
    return rc;
}

/* CALCULATEKERNEL(L, g, k): K = sum_m h_m N_m (Eqs. 6-7), then the cosine
 * normalisation.  Any output pointer may be NULL except that at least one of
 * K_out / Kn_out should be given for the call to be useful. */
int orc_kernel(const int8_t *seqs, const int32_t *lens, int32_t N, int32_t g, int32_t k,
               int32_t nthreads, int32_t per_mask, int64_t *C_out, int64_t *Nm_out, int64_t *K_out,
               double *Kn_out)
{
    if (N < 0 || g < 1 || k < 0 || k > g) return ORC_EINVAL;
    const int32_t M = g - k;
    const size_t NN = (size_t)N * (size_t)N;
    int64_t *Nm = Nm_out ? Nm_out : (int64_t *)malloc(sizeof(int64_t) * (NN ? NN : 1) * (size_t)(M + 1));
    int64_t *K = K_out ? K_out : (int64_t *)malloc(sizeof(int64_t) * (NN ? NN : 1));
    if (!Nm || !K) {
        if (!Nm_out) free(Nm);
        if (!K_out) free(K);
        return ORC_ENOMEM;
    }
    int rc = orc_mismatch_profile(seqs, lens, N, g, M, nthreads, per_mask, C_out, Nm);
    if (rc == ORC_OK) {
        for (size_t e = 0; e < NN; ++e) K[e] = 0;
        for (int32_t m = 0; m <= M; ++m) {
            const int64_t h = orc_binom(g - m, k); /* Eq. 6 */
            for (size_t e = 0; e < NN; ++e) K[e] += h * Nm[(size_t)m * NN + e];
        }
        if (Kn_out) {
            for (int32_t i = 0; i < N; ++i)
                for (int32_t j = 0; j < N; ++j) {
                    const int64_t kii = K[(size_t)i * N + i], kjj = K[(size_t)j * N + j];
                    Kn_out[(size_t)i * N + j] =
                        (kii == 0 || kjj == 0)
                            ? 0.0
                            : (double)K[(size_t)i * N + j] / sqrt((double)kii * (double)kjj);
                }
        }
    }
    if (!Nm_out) free(Nm);
    if (!K_out) free(K);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* One position set on its own (stage parity and per-mask pins)           */
/* ---------------------------------------------------------------------- */
typedef struct {
    int32_t *grp_off, *ent_sid, *ent_cnt, *grp_rep;
    const int32_t *rec_rep; /* original g-mer index of each sorted record */
    int64_t ngrp, nent, cap_grp, cap_ent;
    int overflow;
} orc_dump_ctx;

static void orc_dump_visitor(const orc_group *grp, int64_t first_rec, void *arg)
{
    orc_dump_ctx *d = (orc_dump_ctx *)arg;
    if (d->ngrp + 1 > d->cap_grp || d->nent + grp->n > d->cap_ent) { d->overflow = 1; return; }
    d->grp_off[d->ngrp] = (int32_t)d->nent;
    d->grp_rep[d->ngrp] = d->rec_rep[first_rec];
    for (int32_t a = 0; a < grp->n; ++a) {
        d->ent_sid[d->nent + a] = grp->sid[a];
        d->ent_cnt[d->nent + a] = (int32_t)grp->cnt[a];
    }
    d->nent += grp->n;
    d->ngrp += 1;
    d->grp_off[d->ngrp] = (int32_t)d->nent;
}

/* The groups of the sorted reduced list for one set of removed positions:
 * group q owns entries [grp_off[q], grp_off[q+1]) of (sequence, count), and
 * grp_rep[q] is the index (in extraction order) of one g-mer of the group.
 * Returns the number of groups, or a negative error. */
int64_t orc_mask_groups(const int8_t *seqs, const int32_t *lens, int32_t N, int32_t g,
                        const int32_t *removed, int32_t m, int32_t *grp_off, int32_t *grp_rep,
                        int64_t cap_grp, int32_t *ent_sid, int32_t *ent_cnt, int64_t cap_ent)
{
    if (g < 1 || m < 0 || m > g) return ORC_EINVAL;
    orc_gmer_list L;
    if (orc_extract(seqs, lens, N, g, &L) != ORC_OK) return ORC_ENOMEM;
    orc_rec_layout lay;
    uint8_t *recs = orc_remove_positions(&L, removed, m, &lay);
    /* remember where each record came from: append the extraction index by
     * sorting (record, index) pairs through a parallel array */
    int64_t T = L.T;
    size_t st2 = lay.stride + sizeof(int32_t);
    uint8_t *recs2 = (uint8_t *)malloc((size_t)(T > 0 ? T : 1) * st2);
    int32_t *rep = (int32_t *)malloc(sizeof(int32_t) * (size_t)(T > 0 ? T : 1));
    uint8_t *recs3 = (uint8_t *)malloc((size_t)(T > 0 ? T : 1) * lay.stride);
    int32_t *sid_buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
    int64_t *cnt_buf = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    if (!recs || !recs2 || !rep || !recs3 || !sid_buf || !cnt_buf) {
        free(recs); free(recs2); free(rep); free(recs3); free(sid_buf); free(cnt_buf);
        orc_free_list(&L);
        return ORC_ENOMEM;
    }
    for (int64_t t = 0; t < T; ++t) {
        memcpy(recs2 + (size_t)t * st2, recs + (size_t)t * lay.stride, lay.stride);
        int32_t ti = (int32_t)t;
        memcpy(recs2 + (size_t)t * st2 + lay.stride, &ti, sizeof(int32_t));
    }
    /* the comparator only looks at the reduced string and the sequence index */
    qsort_r(recs2, (size_t)T, st2, orc_rec_cmp, &lay);
    for (int64_t t = 0; t < T; ++t) {
        memcpy(recs3 + (size_t)t * lay.stride, recs2 + (size_t)t * st2, lay.stride);
        memcpy(&rep[t], recs2 + (size_t)t * st2 + lay.stride, sizeof(int32_t));
    }
    orc_dump_ctx d = {grp_off, ent_sid, ent_cnt, grp_rep, rep, 0, 0, cap_grp, cap_ent, 0};
    if (cap_grp > 0) grp_off[0] = 0;
    orc_count_groups(recs3, T, &lay, sid_buf, cnt_buf, orc_dump_visitor, &d);
    free(recs); free(recs2); free(rep); free(recs3); free(sid_buf); free(cnt_buf);
    orc_free_list(&L);
    return d.overflow ? ORC_EINVAL : d.ngrp;
}

/* ---------------------------------------------------------------------- */
/* Kernel rows of queries against a fixed set (Eq. 1 decision values)    */
/* ---------------------------------------------------------------------- */
typedef struct {
    int64_t *Cq;   /* [n_q][n_sv] cross block of C_m */
    int64_t *Cd;   /* [n_sv + n_q] diagonal of C_m    */
    int32_t n_sv, n_q;
} orc_rows_ctx;

/* Sequence ids 0..n_sv-1 are the resident set, n_sv.. are the queries. */
static void orc_rows_visitor(const orc_group *grp, int64_t first_rec, void *arg)
{
    (void)first_rec;
    orc_rows_ctx *r = (orc_rows_ctx *)arg;
    for (int32_t a = 0; a < grp->n; ++a) {
        r->Cd[grp->sid[a]] += grp->cnt[a] * grp->cnt[a];
        if (grp->sid[a] < r->n_sv) continue;
        const int32_t q = grp->sid[a] - r->n_sv;
        for (int32_t b = 0; b < grp->n; ++b)
            if (grp->sid[b] < r->n_sv)
                r->Cq[(int64_t)q * r->n_sv + grp->sid[b]] += grp->cnt[a] * grp->cnt[b];
    }
}

/* The position sets of levels 0..M dealt to nthreads threads (Section S:5.3);
 * thread tid adds the cross block and the diagonal of its sets into its own
 * Cq [M+1][n_q][n_sv] and Cd [M+1][n_sv+n_q]. */
typedef struct {
    const orc_gmer_list *L;
    int32_t n_sv, n_q, M, tid, nthreads;
    int64_t *Cq, *Cd;
    int rc;
} orc_rows_job;

static void *orc_rows_thread(void *arg)
{
    orc_rows_job *j = (orc_rows_job *)arg;
    const int32_t NT = j->n_sv + j->n_q;
    const size_t QS = (size_t)j->n_q * (size_t)j->n_sv;
    int32_t *sid_buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(NT > 0 ? NT : 1));
    int64_t *cnt_buf = (int64_t *)malloc(sizeof(int64_t) * (size_t)(NT > 0 ? NT : 1));
    if (!sid_buf || !cnt_buf) { j->rc = ORC_ENOMEM; free(sid_buf); free(cnt_buf); return NULL; }
    int64_t item = 0;
    for (int32_t m = 0; m <= j->M && j->rc == ORC_OK; ++m) {
        int32_t P[64];
        for (int32_t q = 0; q < m; ++q) P[q] = q;
        orc_rows_ctx r = {j->Cq + (size_t)m * QS, j->Cd + (size_t)m * NT, j->n_sv, j->n_q};
        do {
            if (item % j->nthreads == j->tid) {
                orc_rec_layout lay;
                uint8_t *recs = orc_remove_positions(j->L, P, m, &lay);
                if (!recs) { j->rc = ORC_ENOMEM; break; }
                qsort_r(recs, (size_t)j->L->T, lay.stride, orc_rec_cmp, &lay);
                orc_count_groups(recs, j->L->T, &lay, sid_buf, cnt_buf, orc_rows_visitor, &r);
                free(recs);
            }
            ++item;
        } while (m > 0 && orc_next_subset(P, m, j->L->g));
    }
    free(sid_buf);
    free(cnt_buf);
    return NULL;
}

/* Algorithm 1 on the union of the resident sequences and the queries,
 * keeping only the query-by-resident block and the diagonal; then Eq. 9,
 * Eq. 7, the cosine normalisation, and f(q) = sum_i alpha_i K-hat(sv_i, q) + b
 * (Eq. 1, alpha_i standing for alpha_i * y_i) summed in ascending i.  With
 * nthreads > 1 the position sets are dealt to threads (exact int64 sums). */
int orc_rows(const int8_t *sv_seqs, const int32_t *sv_lens, int32_t n_sv,
             const int8_t *q_seqs, const int32_t *q_lens, int32_t n_q, int32_t g, int32_t k,
             const double *alpha, double bias, int32_t nthreads, double *Krows, int64_t *Nm_rows,
             double *decision)
{
    if (n_sv < 0 || n_q < 0 || g < 1 || k < 0 || k > g) return ORC_EINVAL;
    const int32_t M = g - k, NT = n_sv + n_q;
    int64_t sv_tot = 0, q_tot = 0;
    for (int32_t i = 0; i < n_sv; ++i) sv_tot += sv_lens[i];
    for (int32_t i = 0; i < n_q; ++i) q_tot += q_lens[i];
    int8_t *seqs = (int8_t *)malloc((size_t)(sv_tot + q_tot + 1));
    int32_t *lens = (int32_t *)malloc(sizeof(int32_t) * (size_t)(NT > 0 ? NT : 1));
    const size_t QS = (size_t)n_q * (size_t)n_sv;
    int64_t *Cq = (int64_t *)calloc((QS ? QS : 1) * (size_t)(M + 1), sizeof(int64_t));
    int64_t *Cd = (int64_t *)calloc((size_t)(NT > 0 ? NT : 1) * (size_t)(M + 1), sizeof(int64_t));
    int64_t *Nq = (int64_t *)calloc((QS ? QS : 1) * (size_t)(M + 1), sizeof(int64_t));
    int64_t *Nd = (int64_t *)calloc((size_t)(NT > 0 ? NT : 1) * (size_t)(M + 1), sizeof(int64_t));
    int rc = ORC_OK;
    orc_gmer_list L = {0, 0, NULL, NULL};
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    orc_rows_job jobs[256];
    int32_t started = 0;
    if (!seqs || !lens || !Cq || !Cd || !Nq || !Nd) { rc = ORC_ENOMEM; goto done; }
    memcpy(seqs, sv_seqs, (size_t)sv_tot);
    memcpy(seqs + sv_tot, q_seqs, (size_t)q_tot);
    memcpy(lens, sv_lens, sizeof(int32_t) * (size_t)n_sv);
    memcpy(lens + n_sv, q_lens, sizeof(int32_t) * (size_t)n_q);
    if (orc_extract(seqs, lens, NT, g, &L) != ORC_OK) { rc = ORC_ENOMEM; goto done; }
    /* thread 0 adds into Cq / Cd directly, the others into private copies */
    for (int32_t t = 0; t < nthreads; ++t) {
        int64_t *pq = t ? (int64_t *)calloc((QS ? QS : 1) * (size_t)(M + 1), sizeof(int64_t)) : Cq;
        int64_t *pd = t ? (int64_t *)calloc((size_t)(NT > 0 ? NT : 1) * (size_t)(M + 1), sizeof(int64_t)) : Cd;
        if (!pq || !pd) { if (t) { free(pq); free(pd); } rc = ORC_ENOMEM; break; }
        jobs[t] = (orc_rows_job){&L, n_sv, n_q, M, t, nthreads, pq, pd, ORC_OK};
        ++started;
    }
    if (rc == ORC_OK) {
        for (int32_t t = 0; t < started; ++t) pthread_create(&th[t], NULL, orc_rows_thread, &jobs[t]);
        for (int32_t t = 0; t < started; ++t) pthread_join(th[t], NULL);
    }
    for (int32_t t = 0; t < started; ++t) {
        if (rc == ORC_OK && jobs[t].rc != ORC_OK) rc = jobs[t].rc;
        if (t == 0) continue;
        if (rc == ORC_OK) {
            for (size_t e = 0; e < QS * (size_t)(M + 1); ++e) Cq[e] += jobs[t].Cq[e];
            for (size_t e = 0; e < (size_t)NT * (size_t)(M + 1); ++e) Cd[e] += jobs[t].Cd[e];
        }
        free(jobs[t].Cq);
        free(jobs[t].Cd);
    }
    if (rc != ORC_OK) goto done;
    /* Eq. 9 on the cross block and on the diagonal */
    for (int32_t m = 0; m <= M; ++m) {
        for (size_t e = 0; e < QS; ++e) {
            int64_t v = Cq[(size_t)m * QS + e];
            for (int32_t j = 0; j < m; ++j) v -= orc_binom(g - j, m - j) * Nq[(size_t)j * QS + e];
            Nq[(size_t)m * QS + e] = v;
        }
        for (int32_t e = 0; e < NT; ++e) {
            int64_t v = Cd[(size_t)m * NT + e];
            for (int32_t j = 0; j < m; ++j) v -= orc_binom(g - j, m - j) * Nd[(size_t)j * NT + e];
            Nd[(size_t)m * NT + e] = v;
        }
    }
    for (int32_t q = 0; q < n_q; ++q) {
        int64_t kqq = 0;
        for (int32_t m = 0; m <= M; ++m) kqq += orc_binom(g - m, k) * Nd[(size_t)m * NT + n_sv + q];
        double f = bias;
        for (int32_t i = 0; i < n_sv; ++i) {
            int64_t kq = 0, kss = 0;
            for (int32_t m = 0; m <= M; ++m) {
                kq += orc_binom(g - m, k) * Nq[(size_t)m * QS + (size_t)q * n_sv + i];
                kss += orc_binom(g - m, k) * Nd[(size_t)m * NT + i];
            }
            const double kh = (kqq == 0 || kss == 0) ? 0.0 : (double)kq / sqrt((double)kss * (double)kqq);
            if (Krows) Krows[(size_t)q * n_sv + i] = kh;
            if (alpha) f += alpha[i] * kh;
        }
        if (decision) decision[q] = f;
    }
    if (Nm_rows) memcpy(Nm_rows, Nq, sizeof(int64_t) * QS * (size_t)(M + 1));
done:
    orc_free_list(&L);
    free(seqs); free(lens); free(Cq); free(Cd); free(Nq); free(Nd);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* Training consumer: the support-vector machine of Eq. 1 on the kernel   */
/* ---------------------------------------------------------------------- */
/* The paper trains an SVM on the gapped k-mer kernel (Section 3.1) and
 * classifies with f(x) = sum_i alpha_i y_i K(x_i, x) + b (Eq. 1); it does not
 * fix the solver.  This is the soft-margin dual with the bias absorbed into
 * the kernel (K'(x, x') = K(x, x') + 1, so that b = sum_i alpha_i y_i):
 *     minimise  1/2 alpha^T Q alpha - sum_i alpha_i,  0 <= alpha_i <= C,
 *     Q_ij = y_i y_j K'_ij,
 * solved by dual coordinate descent (Hsieh et al., ICML 2008): coordinates in
 * the order 0..N-1, each set to the clipped minimiser of the objective along
 * it, with the gradient G = Q alpha - 1 kept up to date; an epoch is one pass,
 * and the run stops after the first epoch in which the projected gradients
 * span at most eps, or after max_epochs.
 * K: [N][N] normalised kernel (row-major), y: labels +1 / -1.
 * Outputs: alpha [N], dual_coef [N] = alpha_i y_i, *bias = sum_i alpha_i y_i
 * (ascending i), *epochs = epochs run.  Returns ORC_EINVAL for a bad
 * argument or a label other than +1 / -1. */
int orc_svm_dcd(const double *K, const int8_t *y, int32_t N, double C, double eps, int32_t max_epochs,
                double *alpha, double *dual_coef, double *bias, int32_t *epochs)
{
    if (N < 1 || !(C > 0.0) || eps < 0.0 || max_epochs < 1) return ORC_EINVAL;
    for (int32_t i = 0; i < N; ++i)
        if (y[i] != 1 && y[i] != -1) return ORC_EINVAL;
    double *G = (double *)calloc((size_t)N, sizeof(double)); /* (Q alpha)_j */
    if (!G) return ORC_ENOMEM;
    for (int32_t i = 0; i < N; ++i) alpha[i] = 0.0;
    int32_t ep = 0;
    while (ep < max_epochs) {
        double pgmax = -HUGE_VAL, pgmin = HUGE_VAL;
        for (int32_t i = 0; i < N; ++i) {
            const double qii = K[(size_t)i * N + i] + 1.0;
            const double g = G[i] - 1.0;
            double pg = g;
            if (alpha[i] == 0.0) pg = fmin(g, 0.0);
            else if (alpha[i] == C) pg = fmax(g, 0.0);
            pgmax = fmax(pgmax, pg);
            pgmin = fmin(pgmin, pg);
            if (pg != 0.0) {
                const double a_new = fmin(fmax(alpha[i] - g / qii, 0.0), C);
                const double d = a_new - alpha[i];
                alpha[i] = a_new;
                if (d != 0.0)
                    for (int32_t j = 0; j < N; ++j) {
                        double q = K[(size_t)i * N + j] + 1.0;
                        if (y[i] != y[j]) q = -q;
                        G[j] = G[j] + d * q;
                    }
            }
        }
        ++ep;
        if (pgmax - pgmin <= eps) break;
    }
    double b = 0.0;
    for (int32_t i = 0; i < N; ++i) {
        dual_coef[i] = alpha[i] * (double)y[i];
        b += dual_coef[i];
    }
    *bias = b;
    *epochs = ep;
    free(G);
    return ORC_OK;
}
