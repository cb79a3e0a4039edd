/*
 * Oracle: alphabet, BLOSUM62, k-mer ids and substitute k-mers.
 * Test infrastructure only (see oracle.h).
 */
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* Section V-B: bases are numbered 0..23 in this order. */
static const char ALPHA[25] = "ARNDCQEGHILKMFPSTWYVBZX*";

/* BLOSUM62 (Henikoff & Henikoff 1992), the scoring matrix the paper uses for
 * alignment and for substitute k-mers (Sections IV-B and VI), in the order of
 * ALPHA.  Transcribed from the published matrix. */
static const signed char B62[24][24] = {
    /*        A   R   N   D   C   Q   E   G   H   I   L   K   M   F   P   S   T   W   Y   V   B   Z   X   * */
    /* A */ {4, -1, -2, -2, 0, -1, -1, 0, -2, -1, -1, -1, -1, -2, -1, 1, 0, -3, -2, 0, -2, -1, 0, -4},
    /* R */ {-1, 5, 0, -2, -3, 1, 0, -2, 0, -3, -2, 2, -1, -3, -2, -1, -1, -3, -2, -3, -1, 0, -1, -4},
    /* N */ {-2, 0, 6, 1, -3, 0, 0, 0, 1, -3, -3, 0, -2, -3, -2, 1, 0, -4, -2, -3, 3, 0, -1, -4},
    /* D */ {-2, -2, 1, 6, -3, 0, 2, -1, -1, -3, -4, -1, -3, -3, -1, 0, -1, -4, -3, -3, 4, 1, -1, -4},
    /* C */ {0, -3, -3, -3, 9, -3, -4, -3, -3, -1, -1, -3, -1, -2, -3, -1, -1, -2, -2, -1, -3, -3, -2, -4},
    /* Q */ {-1, 1, 0, 0, -3, 5, 2, -2, 0, -3, -2, 1, 0, -3, -1, 0, -1, -2, -1, -2, 0, 3, -1, -4},
    /* E */ {-1, 0, 0, 2, -4, 2, 5, -2, 0, -3, -3, 1, -2, -3, -1, 0, -1, -3, -2, -2, 1, 4, -1, -4},
    /* G */ {0, -2, 0, -1, -3, -2, -2, 6, -2, -4, -4, -2, -3, -3, -2, 0, -2, -2, -3, -3, -1, -2, -1, -4},
    /* H */ {-2, 0, 1, -1, -3, 0, 0, -2, 8, -3, -3, -1, -2, -1, -2, -1, -2, -2, 2, -3, 0, 0, -1, -4},
    /* I */ {-1, -3, -3, -3, -1, -3, -3, -4, -3, 4, 2, -3, 1, 0, -3, -2, -1, -3, -1, 3, -3, -3, -1, -4},
    /* L */ {-1, -2, -3, -4, -1, -2, -3, -4, -3, 2, 4, -2, 2, 0, -3, -2, -1, -2, -1, 1, -4, -3, -1, -4},
    /* K */ {-1, 2, 0, -1, -3, 1, 1, -2, -1, -3, -2, 5, -1, -3, -1, 0, -1, -3, -2, -2, 0, 1, -1, -4},
    /* M */ {-1, -1, -2, -3, -1, 0, -2, -3, -2, 1, 2, -1, 5, 0, -2, -1, -1, -1, -1, 1, -3, -1, -1, -4},
    /* F */ {-2, -3, -3, -3, -2, -3, -3, -3, -1, 0, 0, -3, 0, 6, -4, -2, -2, 1, 3, -1, -3, -3, -1, -4},
    /* P */ {-1, -2, -2, -1, -3, -1, -1, -2, -2, -3, -3, -1, -2, -4, 7, -1, -1, -4, -3, -2, -2, -1, -2, -4},
    /* S */ {1, -1, 1, 0, -1, 0, 0, 0, -1, -2, -2, 0, -1, -2, -1, 4, 1, -3, -2, -2, 0, 0, 0, -4},
    /* T */ {0, -1, 0, -1, -1, -1, -1, -2, -2, -1, -1, -1, -1, -2, -1, 1, 5, -2, -2, 0, -1, -1, 0, -4},
    /* W */ {-3, -3, -4, -4, -2, -2, -3, -2, -2, -3, -2, -3, -1, 1, -4, -3, -2, 11, 2, -3, -4, -3, -2, -4},
    /* Y */ {-2, -2, -2, -3, -2, -1, -2, -3, 2, -1, -1, -2, -1, 3, -3, -2, -2, 2, 7, -1, -3, -2, -1, -4},
    /* V */ {0, -3, -3, -3, -1, -2, -2, -3, -3, 3, 1, -2, 1, -1, -2, -2, 0, -3, -1, 4, -3, -2, -1, -4},
    /* B */ {-2, -1, 3, 4, -3, 0, 1, -1, 0, -3, -4, 0, -3, -3, -2, 0, -1, -4, -3, -3, 4, 1, -1, -4},
    /* Z */ {-1, 0, 0, 1, -3, 3, 4, -2, 0, -3, -3, 1, -1, -3, -1, 0, -1, -3, -2, -2, 1, 4, -1, -4},
    /* X */ {0, -1, -1, -1, -2, -1, -1, -1, -1, -1, -1, -1, -1, -1, -2, 0, 0, -2, -1, -1, -1, -1, -1, -4},
    /* * */ {-4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, 1},
};

const char *orc_alphabet(void) { return ALPHA; }

int orc_blosum62(int a, int b) { return B62[a][b]; }

int64_t orc_encode(const uint8_t *ascii, int64_t len, uint8_t *codes) {
    for (int64_t t = 0; t < len; ++t) {
        const char *hit = (ascii[t] != 0) ? strchr(ALPHA, (int)ascii[t]) : NULL;
        if (hit == NULL) return t;
        codes[t] = (uint8_t)(hit - ALPHA);
    }
    return -1;
}

/* Section V-B: base b at zero-based position i counted from the right
 * contributes b * 24^i. */
int64_t orc_kmer_id(const uint8_t *codes, int k) {
    int64_t id = 0;
    for (int t = 0; t < k; ++t) id = id * 24 + codes[t];
    return id;
}

typedef struct {
    int64_t id;
    int32_t pos;
} idpos;

static int cmp_idpos(const void *x, const void *y) {
    const idpos *a = (const idpos *)x, *b = (const idpos *)y;
    if (a->id != b->id) return a->id < b->id ? -1 : 1;
    return (a->pos > b->pos) - (a->pos < b->pos);
}

/* A_ij holds the start position of k-mer j in sequence i (Section IV-A).  A
 * sparse matrix keeps one value per entry, so a k-mer that repeats inside a
 * sequence keeps its first start position (the paper is silent here). */
int64_t orc_kmer_set(const uint8_t *codes, int64_t len, int k, int64_t *ids, int32_t *pos) {
    if (len < k) return 0;
    int64_t w = len - k + 1;
    idpos *tmp = (idpos *)malloc((size_t)w * sizeof(idpos));
    for (int64_t t = 0; t < w; ++t) {
        tmp[t].id = orc_kmer_id(codes + t, k);
        tmp[t].pos = (int32_t)t;
    }
    qsort(tmp, (size_t)w, sizeof(idpos), cmp_idpos);
    int64_t m = 0;
    for (int64_t t = 0; t < w; ++t) {
        if (t > 0 && tmp[t].id == tmp[t - 1].id) continue;
        ids[m] = tmp[t].id;
        pos[m] = tmp[t].pos;
        ++m;
    }
    free(tmp);
    return m;
}

/* E = Sort(Diag(C) - C): the expense of replacing base a by b (Section IV-B). */
int orc_expense(int a, int b) { return B62[a][a] - B62[a][b]; }

int orc_expense_row(int a, int alpha, int32_t *base, int32_t *expense) {
    /* insertion sort by (expense, base) */
    int n = 0;
    for (int b = 0; b < alpha; ++b) {
        int ex = orc_expense(a, b);
        int t = n++;
        while (t > 0 && (expense[t - 1] > ex || (expense[t - 1] == ex && base[t - 1] > b))) {
            expense[t] = expense[t - 1];
            base[t] = base[t - 1];
            --t;
        }
        expense[t] = ex;
        base[t] = b;
    }
    return n;
}

static void kmer_decode(int64_t id, int k, int *codes) {
    for (int t = k - 1; t >= 0; --t) {
        codes[t] = (int)(id % 24);
        id /= 24;
    }
}

/* Dist(s, r) = sum over positions of expense(r_t -> s_t). */
static int kmer_dist(const int *r, const int *s, int k) {
    int d = 0;
    for (int t = 0; t < k; ++t) d += orc_expense(r[t], s[t]);
    return d;
}

typedef struct {
    int32_t dist;
    int64_t id;
} distid;

static int cmp_distid(const void *x, const void *y) {
    const distid *a = (const distid *)x, *b = (const distid *)y;
    if (a->dist != b->dist) return a->dist < b->dist ? -1 : 1;
    return (a->id > b->id) - (a->id < b->id);
}

/* The m nearest k-mers (Section IV-B): rank every other k-mer over the
 * substitute alphabet by (Dist, id) and keep the first m.  The paper leaves the
 * order among equal distances open; ascending id is the reading used here. */
int orc_subk_bruteforce(int64_t r, int k, int m, int alpha, int64_t *ids, int32_t *dist) {
    int rc[16], sc[16];
    kmer_decode(r, k, rc);
    int64_t total = 1;
    for (int t = 0; t < k; ++t) total *= alpha;
    /* scan every k-mer; keep the m best seen so far, sorted by (Dist, id) */
    distid *best = (distid *)malloc((size_t)(m > 0 ? m : 1) * sizeof(distid));
    int have = 0;
    for (int64_t x = 0; x < total; ++x) {
        int64_t y = x;
        for (int t = k - 1; t >= 0; --t) {
            sc[t] = (int)(y % alpha);
            y /= alpha;
        }
        int64_t id = 0;
        for (int t = 0; t < k; ++t) id = id * 24 + sc[t];
        if (id == r) continue;
        distid cur = {kmer_dist(rc, sc, k), id};
        if (have == m && cmp_distid(&cur, &best[m - 1]) >= 0) continue;
        int t = (have < m) ? have++ : m - 1;
        while (t > 0 && cmp_distid(&cur, &best[t - 1]) < 0) {
            best[t] = best[t - 1];
            --t;
        }
        best[t] = cur;
    }
    for (int q = 0; q < have; ++q) {
        ids[q] = best[q].id;
        dist[q] = best[q].dist;
    }
    free(best);
    return have;
}

/* All k-mers s != r with Dist(s, r) <= D, visited with partial sums pruned:
 * a prefix whose sum plus the smallest possible rest already exceeds D cannot
 * recover.  (Expenses are not always >= 0: BLOSUM62 scores X-X below X-A.) */
typedef struct {
    const int *rc;
    int k, alpha, D;
    int minrest[17];
    int64_t r;
    int sc[16];
    int64_t count, cap;
    distid *out; /* may be NULL: count only */
} bounded_ctx;

static void bounded_rec(bounded_ctx *c, int t, int partial) {
    if (t == c->k) {
        int64_t id = 0;
        for (int q = 0; q < c->k; ++q) id = id * 24 + c->sc[q];
        if (id == c->r) return;
        if (c->out && c->count < c->cap) {
            c->out[c->count].dist = partial;
            c->out[c->count].id = id;
        }
        c->count++;
        return;
    }
    for (int b = 0; b < c->alpha; ++b) {
        int p = partial + orc_expense(c->rc[t], b);
        if (p + c->minrest[t + 1] > c->D) continue;
        c->sc[t] = b;
        bounded_rec(c, t + 1, p);
    }
}

int orc_subk_bounded(int64_t r, int k, int m, int alpha, int64_t *ids, int32_t *dist) {
    int rc[16];
    kmer_decode(r, k, rc);
    int64_t total = 1;
    for (int t = 0; t < k; ++t) total *= alpha;
    int64_t others = total;
    {
        int in_alpha = 1;
        for (int t = 0; t < k; ++t) in_alpha &= (rc[t] < alpha);
        others -= in_alpha;
    }
    int want = (int)(others < m ? others : m);
    if (want <= 0) return 0;
    bounded_ctx c;
    memset(&c, 0, sizeof(c));
    c.rc = rc;
    c.k = k;
    c.alpha = alpha;
    c.r = r;
    c.minrest[k] = 0;
    for (int t = k - 1; t >= 0; --t) {
        int lo = orc_expense(rc[t], 0);
        for (int b = 1; b < alpha; ++b)
            if (orc_expense(rc[t], b) < lo) lo = orc_expense(rc[t], b);
        c.minrest[t] = c.minrest[t + 1] + lo;
    }
    /* smallest D whose ball holds at least `want` other k-mers */
    for (c.D = c.minrest[0];; ++c.D) {
        c.count = 0;
        c.out = NULL;
        bounded_rec(&c, 0, 0);
        if (c.count >= want) break;
    }
    distid *buf = (distid *)malloc((size_t)c.count * sizeof(distid));
    c.cap = c.count;
    c.count = 0;
    c.out = buf;
    bounded_rec(&c, 0, 0);
    qsort(buf, (size_t)c.count, sizeof(distid), cmp_distid);
    for (int q = 0; q < want; ++q) {
        ids[q] = buf[q].id;
        dist[q] = buf[q].dist;
    }
    free(buf);
    return want;
}
