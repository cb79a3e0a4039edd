/*
 * Oracle: candidate pairs from shared k-mers (B = A A^T, Section IV-A) and
 * from substitute k-mers (A S A^T, Section IV-C), with the common-k-mer
 * threshold of Section VI.  Test infrastructure only (see oracle.h).
 *
 * Readings of points the paper leaves open:
 *   - seeds: of all shared k-mer position pairs the two with the smallest key
 *     (pos_lo << 16 | pos_hi) are kept, pos_lo taken in the lower-numbered
 *     sequence (Section IV-A keeps "a maximum of two");
 *   - substitute mode: S holds every present k-mer itself at distance 0 plus
 *     its m nearest substitutes; (AS)_{i,s} keeps the k-mer of i closest to s
 *     (smaller position on equal distance, Section IV-C); the directional
 *     product c(r->c) counts the k-mers s of c reached from r, and the output
 *     is made symmetric by keeping the larger direction (lo -> hi on a tie).
 *     With m = 0 both directions are equal and this is exactly B = A A^T.
 *   - the threshold keeps pairs whose count is >= ck_min.
 */
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "oracle.h"

#define NO_SEED 0xFFFFFFFFu

static void seed_insert(uint32_t key, uint32_t *s1, uint32_t *s2) {
    if (key < *s1) {
        *s2 = *s1;
        *s1 = key;
    } else if (key < *s2) {
        *s2 = key;
    }
}

static uint32_t seed_key(uint32_t r, uint32_t c, int32_t pos_r, int32_t pos_c) {
    return (r < c) ? (((uint32_t)pos_r << 16) | (uint32_t)pos_c) : (((uint32_t)pos_c << 16) | (uint32_t)pos_r);
}

typedef struct {
    int64_t *off; /* n+1 */
    int64_t *id;
    int32_t *pos;
} kmer_sets;

static void build_sets(const uint8_t *codes, const int64_t *offsets, int64_t n, int k, kmer_sets *ks) {
    ks->off = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    ks->off[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t len = offsets[i + 1] - offsets[i];
        ks->off[i + 1] = ks->off[i] + (len >= k ? len - k + 1 : 0);
    }
    int64_t cap = ks->off[n] > 0 ? ks->off[n] : 1;
    ks->id = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    ks->pos = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
    int64_t *cnt = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        cnt[i] = orc_kmer_set(codes + offsets[i], offsets[i + 1] - offsets[i], k, ks->id + ks->off[i],
                              ks->pos + ks->off[i]);
    }
    /* compact the per-sequence sets (distinct k-mers only) */
    int64_t w = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t b = ks->off[i];
        for (int64_t t = 0; t < cnt[i]; ++t) {
            ks->id[w + t] = ks->id[b + t];
            ks->pos[w + t] = ks->pos[b + t];
        }
        ks->off[i] = w;
        w += cnt[i];
    }
    ks->off[n] = w;
    free(cnt);
}

static void free_sets(kmer_sets *ks) {
    free(ks->off);
    free(ks->id);
    free(ks->pos);
}

typedef struct {
    uint32_t lo, hi, count, s1, s2;
    uint32_t dir; /* 0: lo -> hi, 1: hi -> lo */
} dentry;

static int cmp_dentry(const void *x, const void *y) {
    const dentry *a = (const dentry *)x, *b = (const dentry *)y;
    if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;
    if (a->hi != b->hi) return a->hi < b->hi ? -1 : 1;
    return (a->dir > b->dir) - (a->dir < b->dir);
}

int64_t orc_candidates_bruteforce(const uint8_t *codes, const int64_t *offsets, int64_t n, int k, int ck_min,
                                  int64_t cap, uint32_t *lo, uint32_t *hi, uint32_t *count, uint32_t *seed1,
                                  uint32_t *seed2) {
    kmer_sets ks;
    build_sets(codes, offsets, n, k, &ks);
    int64_t out = 0;
    /* every pair i < j: |K(i) n K(j)| by merging the two sorted sets */
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            int64_t a = ks.off[i], ae = ks.off[i + 1], b = ks.off[j], be = ks.off[j + 1];
            uint32_t c = 0, s1 = NO_SEED, s2 = NO_SEED;
            while (a < ae && b < be) {
                if (ks.id[a] < ks.id[b]) {
                    ++a;
                } else if (ks.id[a] > ks.id[b]) {
                    ++b;
                } else {
                    ++c;
                    seed_insert(((uint32_t)ks.pos[a] << 16) | (uint32_t)ks.pos[b], &s1, &s2);
                    ++a;
                    ++b;
                }
            }
            if (c >= (uint32_t)ck_min && c > 0) {
                if (out >= cap) {
                    free_sets(&ks);
                    return -1;
                }
                lo[out] = (uint32_t)i;
                hi[out] = (uint32_t)j;
                count[out] = c;
                seed1[out] = s1;
                seed2[out] = s2;
                ++out;
            }
        }
    }
    free_sets(&ks);
    return out;
}

/* postings of every present k-mer: (seq, pos) sorted by seq */
typedef struct {
    int64_t nu;
    int64_t *uid;   /* distinct ids, ascending */
    int64_t *start; /* nu + 1 */
    uint32_t *seq;
    int32_t *pos;
} postings;

typedef struct {
    int64_t id;
    uint32_t seq;
    int32_t pos;
} triple;

static int cmp_triple(const void *x, const void *y) {
    const triple *a = (const triple *)x, *b = (const triple *)y;
    if (a->id != b->id) return a->id < b->id ? -1 : 1;
    return (a->seq > b->seq) - (a->seq < b->seq);
}

static void build_postings(const kmer_sets *ks, int64_t n, postings *P) {
    int64_t nnz = ks->off[n];
    triple *t = (triple *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(triple));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t q = ks->off[i]; q < ks->off[i + 1]; ++q) {
            t[q].id = ks->id[q];
            t[q].seq = (uint32_t)i;
            t[q].pos = ks->pos[q];
        }
    qsort(t, (size_t)nnz, sizeof(triple), cmp_triple);
    P->uid = (int64_t *)malloc((size_t)(nnz + 1) * sizeof(int64_t));
    P->start = (int64_t *)malloc((size_t)(nnz + 2) * sizeof(int64_t));
    P->seq = (uint32_t *)malloc((size_t)(nnz + 1) * sizeof(uint32_t));
    P->pos = (int32_t *)malloc((size_t)(nnz + 1) * sizeof(int32_t));
    int64_t nu = 0;
    for (int64_t q = 0; q < nnz; ++q) {
        if (q == 0 || t[q].id != t[q - 1].id) {
            P->uid[nu] = t[q].id;
            P->start[nu] = q;
            ++nu;
        }
        P->seq[q] = t[q].seq;
        P->pos[q] = t[q].pos;
    }
    P->start[nu] = nnz;
    P->nu = nu;
    free(t);
}

static void free_postings(postings *P) {
    free(P->uid);
    free(P->start);
    free(P->seq);
    free(P->pos);
}

static int64_t find_id(const postings *P, int64_t id) {
    int64_t lo = 0, hi = P->nu;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (P->uid[mid] < id)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < P->nu && P->uid[lo] == id) ? lo : -1;
}

typedef struct {
    int64_t s;
    int32_t dist, pos;
} asent;

static int cmp_asent(const void *x, const void *y) {
    const asent *a = (const asent *)x, *b = (const asent *)y;
    if (a->s != b->s) return a->s < b->s ? -1 : 1;
    if (a->dist != b->dist) return a->dist < b->dist ? -1 : 1;
    return (a->pos > b->pos) - (a->pos < b->pos);
}

typedef struct {
    dentry *v;
    int64_t n, cap;
} dvec;

static void dvec_push(dvec *d, dentry e) {
    if (d->n == d->cap) {
        d->cap = d->cap ? 2 * d->cap : 1024;
        d->v = (dentry *)realloc(d->v, (size_t)d->cap * sizeof(dentry));
    }
    d->v[d->n++] = e;
}

int64_t orc_candidates_index(const uint8_t *codes, const int64_t *offsets, int64_t n, int k, int n_subs,
                             int alpha, int ck_min, const int64_t *rows, int64_t nrows, int64_t cap, uint32_t *lo,
                             uint32_t *hi, uint32_t *count, uint32_t *seed1, uint32_t *seed2) {
    kmer_sets ks;
    build_sets(codes, offsets, n, k, &ks);
    postings P;
    build_postings(&ks, n, &P);
    unsigned char *wanted = NULL;
    if (nrows >= 0) {
        wanted = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
        for (int64_t q = 0; q < nrows; ++q) wanted[rows[q]] = 1;
    }
    const int exact = (n_subs == 0);
    int nthreads = orc_num_threads();
    dvec *found = (dvec *)calloc((size_t)nthreads, sizeof(dvec));

#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        uint32_t *cnt = (uint32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(uint32_t));
        uint32_t *s1 = (uint32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
        uint32_t *s2 = (uint32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
        int64_t *touched = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
        int64_t *nb_id = (int64_t *)malloc((size_t)(n_subs + 1) * sizeof(int64_t));
        int32_t *nb_d = (int32_t *)malloc((size_t)(n_subs + 1) * sizeof(int32_t));
        asent *as = NULL;
        int64_t as_cap = 0;

#pragma omp for schedule(dynamic, 16)
        for (int64_t r = 0; r < n; ++r) {
            int64_t kb = ks.off[r], ke = ks.off[r + 1];
            /* row r of A S: every k-mer p of r expands to S(p) */
            int64_t need = (ke - kb) * (int64_t)(n_subs + 1);
            if (need > as_cap) {
                as_cap = need;
                as = (asent *)realloc(as, (size_t)as_cap * sizeof(asent));
            }
            int64_t na = 0;
            for (int64_t q = kb; q < ke; ++q) {
                as[na].s = ks.id[q];
                as[na].dist = 0;
                as[na].pos = ks.pos[q];
                ++na;
                if (!exact) {
                    int got = orc_subk_bounded(ks.id[q], k, n_subs, alpha, nb_id, nb_d);
                    for (int g = 0; g < got; ++g) {
                        as[na].s = nb_id[g];
                        as[na].dist = nb_d[g];
                        as[na].pos = ks.pos[q];
                        ++na;
                    }
                }
            }
            /* (AS)_{r,s}: the closest k-mer of r, then the smaller position */
            qsort(as, (size_t)na, sizeof(asent), cmp_asent);
            int64_t nt = 0;
            for (int64_t q = 0; q < na; ++q) {
                if (q > 0 && as[q].s == as[q - 1].s) continue;
                int64_t u = find_id(&P, as[q].s);
                if (u < 0) continue;
                for (int64_t z = P.start[u]; z < P.start[u + 1]; ++z) {
                    uint32_t c = P.seq[z];
                    if (c == (uint32_t)r) continue;
                    if (exact && c < (uint32_t)r) continue; /* symmetric: one triangle */
                    if (cnt[c] == 0) {
                        touched[nt++] = c;
                        s1[c] = NO_SEED;
                        s2[c] = NO_SEED;
                    }
                    cnt[c]++;
                    seed_insert(seed_key((uint32_t)r, c, as[q].pos, P.pos[z]), &s1[c], &s2[c]);
                }
            }
            for (int64_t q = 0; q < nt; ++q) {
                uint32_t c = (uint32_t)touched[q];
                if (cnt[c] >= (uint32_t)ck_min && (!wanted || wanted[r] || wanted[c])) {
                    dentry e;
                    e.lo = (uint32_t)r < c ? (uint32_t)r : c;
                    e.hi = (uint32_t)r < c ? c : (uint32_t)r;
                    e.count = cnt[c];
                    e.s1 = s1[c];
                    e.s2 = s2[c];
                    e.dir = (uint32_t)r < c ? 0u : 1u;
                    dvec_push(&found[tid], e);
                }
                cnt[c] = 0;
            }
        }
        free(cnt);
        free(s1);
        free(s2);
        free(touched);
        free(nb_id);
        free(nb_d);
        free(as);
    }

    int64_t total = 0;
    for (int t = 0; t < nthreads; ++t) total += found[t].n;
    dentry *all = (dentry *)malloc((size_t)(total > 0 ? total : 1) * sizeof(dentry));
    int64_t w = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (found[t].n) memcpy(all + w, found[t].v, (size_t)found[t].n * sizeof(dentry));
        w += found[t].n;
        free(found[t].v);
    }
    free(found);
    qsort(all, (size_t)total, sizeof(dentry), cmp_dentry);
    /* symmetrise: one record per (lo, hi), the direction with the larger count */
    int64_t out = 0;
    int64_t status = 0;
    for (int64_t q = 0; q < total;) {
        dentry best = all[q];
        int64_t z = q + 1;
        while (z < total && all[z].lo == best.lo && all[z].hi == best.hi) {
            if (all[z].count > best.count) best = all[z];
            ++z;
        }
        if (out >= cap) {
            status = -1;
            break;
        }
        lo[out] = best.lo;
        hi[out] = best.hi;
        count[out] = best.count;
        seed1[out] = best.s1;
        seed2[out] = best.s2;
        ++out;
        q = z;
    }
    free(all);
    free(wanted);
    free_postings(&P);
    free_sets(&ks);
    return status < 0 ? -1 : out;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops from now on (n <= 0: every available core);
 * a harness setting for timing runs, no effect on any result. */
void orc_set_threads(int n) {
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
    (void)n;
#endif
}

/* Row i of A S as a list sorted by substitute id: for every k-mer s reached
 * from a k-mer of i, the closest such k-mer's position (smaller position on
 * equal distance).  Exact mode (n_subs = 0) gives K(i) itself. */
static int64_t as_row(const kmer_sets *ks, int64_t i, int k, int n_subs, int alpha, asent **buf, int64_t *cap) {
    int64_t kb = ks->off[i], ke = ks->off[i + 1];
    int64_t need = (ke - kb) * (int64_t)(n_subs + 1);
    if (need > *cap) {
        *cap = need;
        *buf = (asent *)realloc(*buf, (size_t)(need > 0 ? need : 1) * sizeof(asent));
    }
    asent *as = *buf;
    int64_t *nb_id = (int64_t *)malloc((size_t)(n_subs + 1) * sizeof(int64_t));
    int32_t *nb_d = (int32_t *)malloc((size_t)(n_subs + 1) * sizeof(int32_t));
    int64_t na = 0;
    for (int64_t q = kb; q < ke; ++q) {
        as[na].s = ks->id[q];
        as[na].dist = 0;
        as[na].pos = ks->pos[q];
        ++na;
        if (n_subs > 0) {
            int got = orc_subk_bounded(ks->id[q], k, n_subs, alpha, nb_id, nb_d);
            for (int g = 0; g < got; ++g) {
                as[na].s = nb_id[g];
                as[na].dist = nb_d[g];
                as[na].pos = ks->pos[q];
                ++na;
            }
        }
    }
    free(nb_id);
    free(nb_d);
    qsort(as, (size_t)na, sizeof(asent), cmp_asent);
    int64_t w = 0;
    for (int64_t q = 0; q < na; ++q)
        if (q == 0 || as[q].s != as[q - 1].s) as[w++] = as[q];
    return w;
}

int64_t orc_pair_counts(const uint8_t *codes, const int64_t *offsets, int64_t n, int k, int n_subs, int alpha,
                        const uint32_t *lo, const uint32_t *hi, int64_t npairs, uint32_t *count, uint32_t *seed1,
                        uint32_t *seed2) {
    /* only the sequences of the listed pairs are needed */
    unsigned char *used = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    for (int64_t q = 0; q < npairs; ++q) {
        if (lo[q] >= hi[q] || hi[q] >= (uint64_t)n) {
            free(used);
            return -1;
        }
        used[lo[q]] = used[hi[q]] = 1;
    }
    int64_t nu = 0;
    int64_t *slot = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) slot[i] = used[i] ? nu++ : -1;
    int64_t *seqs = (int64_t *)malloc((size_t)(nu > 0 ? nu : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i)
        if (used[i]) seqs[slot[i]] = i;
    /* k-mer sets of the used sequences only (others left empty) */
    kmer_sets ks;
    ks.off = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    ks.off[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t len = offsets[i + 1] - offsets[i];
        ks.off[i + 1] = ks.off[i] + ((used[i] && len >= k) ? len - k + 1 : 0);
    }
    int64_t tot = ks.off[n] > 0 ? ks.off[n] : 1;
    ks.id = (int64_t *)malloc((size_t)tot * sizeof(int64_t));
    ks.pos = (int32_t *)malloc((size_t)tot * sizeof(int32_t));
    int64_t *kcount = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t u = 0; u < nu; ++u) {
        int64_t i = seqs[u];
        kcount[i] = orc_kmer_set(codes + offsets[i], offsets[i + 1] - offsets[i], k, ks.id + ks.off[i],
                                 ks.pos + ks.off[i]);
    }
    /* the rows of A S of the used sequences */
    asent **rows = (asent **)calloc((size_t)(nu > 0 ? nu : 1), sizeof(asent *));
    int64_t *rlen = (int64_t *)calloc((size_t)(nu > 0 ? nu : 1), sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t u = 0; u < nu; ++u) {
        int64_t i = seqs[u];
        int64_t off2[2] = {ks.off[i], ks.off[i] + kcount[i]};
        kmer_sets view;
        view.off = off2;
        view.id = ks.id;
        view.pos = ks.pos;
        asent *buf = NULL;
        int64_t cap = 0;
        rlen[u] = as_row(&view, 0, k, n_subs, alpha, &buf, &cap);
        rows[u] = buf;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < npairs; ++q) {
        uint32_t best_c = 0, best_s1 = NO_SEED, best_s2 = NO_SEED;
        for (int dir = 0; dir < 2; ++dir) {
            uint32_t r = dir == 0 ? lo[q] : hi[q], c = dir == 0 ? hi[q] : lo[q];
            const asent *ar = rows[slot[r]];
            int64_t na = rlen[slot[r]];
            int64_t b = ks.off[c], be = ks.off[c] + kcount[c];
            int64_t a = 0;
            uint32_t cnt = 0, s1 = NO_SEED, s2 = NO_SEED;
            /* c(r -> c): the k-mers s of c with (A S)_{r,s} defined */
            while (a < na && b < be) {
                if (ar[a].s < ks.id[b]) {
                    ++a;
                } else if (ar[a].s > ks.id[b]) {
                    ++b;
                } else {
                    ++cnt;
                    seed_insert(seed_key(r, c, ar[a].pos, ks.pos[b]), &s1, &s2);
                    ++a;
                    ++b;
                }
            }
            if (dir == 0 || cnt > best_c) {
                best_c = cnt;
                best_s1 = s1;
                best_s2 = s2;
            }
        }
        count[q] = best_c;
        seed1[q] = best_s1;
        seed2[q] = best_s2;
    }
    for (int64_t u = 0; u < nu; ++u) free(rows[u]);
    free(rows);
    free(rlen);
    free(kcount);
    free(ks.off);
    free(ks.id);
    free(ks.pos);
    free(seqs);
    free(slot);
    free(used);
    return npairs;
}
