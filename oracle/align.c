/*
 * Oracle: pairwise alignment (Section IV-E) and the similarity filter
 * (Section IV-F).  Test infrastructure only (see oracle.h).
 *
 * Readings of points the paper leaves open (one canonical answer each):
 *   - a gap of length L costs gap_open + gap_extend * L (11 + L with the
 *     paper's BLOSUM62, 11, 1 setting of Section VI);
 *   - orientation: rows = the shorter sequence, the lower index on equal length;
 *   - SW: among cells holding the maximum score, the end is the smallest row,
 *     then the smallest column; a zero score means no alignment;
 *   - co-optimal paths: traceback prefers the diagonal, then a horizontal gap
 *     (E), then a vertical gap (F); inside a gap, extending is preferred over
 *     opening;
 *   - identity = identical aligned pairs / alignment columns (gap columns
 *     included); coverage = aligned span of the shorter sequence / its length;
 *   - XD: the k seed columns are scored and counted; each side is extended by
 *     an anchored DP (no zero floor) over anti-diagonals d = u + v: a cell with
 *     no live predecessor is not computed; after a whole anti-diagonal is
 *     computed its cells scoring below (best over earlier anti-diagonals) - X
 *     are dead; the extension stops at the first anti-diagonal without a live
 *     cell; its end is the best live cell (earliest anti-diagonal, then the
 *     smallest row, on ties).
 */
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define TB_ZERO 0
#define TB_DIAG 1
#define TB_E 2
#define TB_F 3
#define TB_EEXT 4
#define TB_FEXT 8

static inline int max2(int x, int y) { return x > y ? x : y; }

void orc_sw(const uint8_t *a, int la, const uint8_t *b, int lb, int o, int e, orc_aln *out) {
    memset(out, 0, sizeof(*out));
    out->beg_a = out->end_a = out->beg_b = out->end_b = -1;
    out->seed_used = -1;
    out->cells = (int64_t)la * lb;
    if (la <= 0 || lb <= 0) return;
    const int W = lb + 1;
    uint8_t *tb = (uint8_t *)calloc((size_t)(la + 1) * (size_t)W, 1);
    int *hprev = (int *)calloc((size_t)W, sizeof(int));
    int *hcur = (int *)calloc((size_t)W, sizeof(int));
    int *f = (int *)malloc((size_t)W * sizeof(int));
    for (int j = 0; j <= lb; ++j) f[j] = ORC_NEG_INF;
    int best = 0, bi = 0, bj = 0;
    for (int i = 1; i <= la; ++i) {
        int ecur = ORC_NEG_INF;
        hcur[0] = 0;
        for (int j = 1; j <= lb; ++j) {
            uint8_t t = 0;
            int e_ext = ecur - e, e_open = hcur[j - 1] - o - e;
            if (e_ext >= e_open) t |= TB_EEXT;
            ecur = max2(e_ext, e_open);
            int f_ext = f[j] - e, f_open = hprev[j] - o - e;
            if (f_ext >= f_open) t |= TB_FEXT;
            f[j] = max2(f_ext, f_open);
            int d = hprev[j - 1] + orc_blosum62(a[i - 1], b[j - 1]);
            int h = max2(max2(0, d), max2(ecur, f[j]));
            if (h == 0)
                t |= TB_ZERO;
            else if (h == d)
                t |= TB_DIAG;
            else if (h == ecur)
                t |= TB_E;
            else
                t |= TB_F;
            tb[(size_t)i * W + j] = t;
            hcur[j] = h;
            if (h > best) { /* row-major scan: first maximum = smallest row, then column */
                best = h;
                bi = i;
                bj = j;
            }
        }
        int *sw = hprev;
        hprev = hcur;
        hcur = sw;
    }
    out->score = best;
    if (best > 0) {
        int i = bi, j = bj, state = TB_DIAG; /* TB_DIAG here means "in H" */
        int matches = 0, cols = 0, beg_i = bi, beg_j = bj;
        for (;;) {
            if (state == TB_DIAG) {
                int src = (i > 0 && j > 0) ? (tb[(size_t)i * W + j] & 3) : TB_ZERO;
                if (src == TB_ZERO) break;
                if (src == TB_DIAG) {
                    ++cols;
                    matches += (a[i - 1] == b[j - 1]);
                    beg_i = i;
                    beg_j = j;
                    --i;
                    --j;
                } else if (src == TB_E) {
                    state = TB_E;
                } else {
                    state = TB_F;
                }
            } else if (state == TB_E) {
                ++cols;
                int ext = tb[(size_t)i * W + j] & TB_EEXT;
                --j;
                state = ext ? TB_E : TB_DIAG;
            } else {
                ++cols;
                int ext = tb[(size_t)i * W + j] & TB_FEXT;
                --i;
                state = ext ? TB_F : TB_DIAG;
            }
        }
        out->beg_a = beg_i - 1;
        out->beg_b = beg_j - 1;
        out->end_a = bi - 1;
        out->end_b = bj - 1;
        out->matches = matches;
        out->columns = cols;
    }
    free(tb);
    free(hprev);
    free(hcur);
    free(f);
}

/* ---- x-drop extension over anti-diagonals ---- */

typedef struct {
    int64_t off; /* first cell of this anti-diagonal in the pools */
    int lo, hi;  /* computed u range [lo, hi]; lo > hi when empty */
    int llo, lhi; /* live u range; llo > lhi when none */
} xdiag;

typedef struct {
    xdiag *dg;
    int *H, *E, *F;
    uint8_t *flag; /* bit0 live, bit1 computed, bit2 E-extend, bit3 F-extend */
    int64_t used, cap;
} xstore;

#define XF_LIVE 1
#define XF_COMP 2
#define XF_EEXT 4
#define XF_FEXT 8

static void xs_reserve(xstore *s, int64_t need) {
    if (s->used + need <= s->cap) return;
    int64_t nc = s->cap ? s->cap : 4096;
    while (nc < s->used + need) nc *= 2;
    s->H = (int *)realloc(s->H, (size_t)nc * sizeof(int));
    s->E = (int *)realloc(s->E, (size_t)nc * sizeof(int));
    s->F = (int *)realloc(s->F, (size_t)nc * sizeof(int));
    s->flag = (uint8_t *)realloc(s->flag, (size_t)nc);
    s->cap = nc;
}

/* index of cell u on diagonal d, or -1 when not stored */
static inline int64_t xs_at(const xstore *s, int d, int u) {
    if (d < 0) return -1;
    const xdiag *g = &s->dg[d];
    if (u < g->lo || u > g->hi) return -1;
    return g->off + (u - g->lo);
}

static inline int xs_live(const xstore *s, int64_t c) { return c >= 0 && (s->flag[c] & XF_LIVE); }

int32_t orc_xdrop_extend(const uint8_t *a, int la, const uint8_t *b, int lb, int o, int e, int x, int32_t *u_end,
                         int32_t *v_end, int32_t *matches, int32_t *columns, int64_t *cells) {
    xstore s;
    memset(&s, 0, sizeof(s));
    const int dmax = la + lb;
    s.dg = (xdiag *)malloc((size_t)(dmax + 1) * sizeof(xdiag));
    /* anti-diagonal 0: the anchor */
    xs_reserve(&s, 1);
    s.dg[0].off = 0;
    s.dg[0].lo = s.dg[0].hi = 0;
    s.dg[0].llo = s.dg[0].lhi = 0;
    s.H[0] = 0;
    s.E[0] = s.F[0] = ORC_NEG_INF;
    s.flag[0] = XF_LIVE | XF_COMP;
    s.used = 1;
    int best = 0, bu = 0, bv = 0, last = 0;
    int64_t ncells = 0;
    for (int d = 1; d <= dmax; ++d) {
        const xdiag *p1 = &s.dg[d - 1];
        int lo = 1 << 30, hi = -1;
        if (p1->llo <= p1->lhi) {
            lo = p1->llo;
            hi = p1->lhi + 1;
        }
        if (d >= 2) {
            const xdiag *p2 = &s.dg[d - 2];
            if (p2->llo <= p2->lhi) {
                if (p2->llo + 1 < lo) lo = p2->llo + 1;
                if (p2->lhi + 1 > hi) hi = p2->lhi + 1;
            }
        }
        int umin = d - lb > 0 ? d - lb : 0, umax = d < la ? d : la;
        if (lo < umin) lo = umin;
        if (hi > umax) hi = umax;
        xdiag *g = &s.dg[d];
        g->off = s.used;
        g->lo = lo;
        g->hi = hi;
        g->llo = 1;
        g->lhi = 0;
        if (lo > hi) {
            last = d;
            break;
        }
        xs_reserve(&s, hi - lo + 1);
        for (int u = lo; u <= hi; ++u) {
            int v = d - u;
            int64_t c = g->off + (u - lo);
            int64_t cu = (u >= 1) ? xs_at(&s, d - 1, u - 1) : -1;           /* (u-1, v): vertical */
            int64_t cl = (v >= 1) ? xs_at(&s, d - 1, u) : -1;               /* (u, v-1): horizontal */
            int64_t cd = (u >= 1 && v >= 1) ? xs_at(&s, d - 2, u - 1) : -1; /* (u-1, v-1) */
            int lu = xs_live(&s, cu), ll = xs_live(&s, cl), ld = xs_live(&s, cd);
            uint8_t fl = 0;
            int E = ORC_NEG_INF, F = ORC_NEG_INF, D = ORC_NEG_INF;
            if (ll) {
                int ext = s.E[cl] - e, opn = s.H[cl] - o - e;
                if (ext >= opn) fl |= XF_EEXT;
                E = max2(ext, opn);
            }
            if (lu) {
                int ext = s.F[cu] - e, opn = s.H[cu] - o - e;
                if (ext >= opn) fl |= XF_FEXT;
                F = max2(ext, opn);
            }
            if (ld) D = s.H[cd] + orc_blosum62(a[u - 1], b[v - 1]);
            if (lu || ll || ld) {
                fl |= XF_COMP;
                ++ncells;
            }
            s.H[c] = max2(D, max2(E, F));
            s.E[c] = E;
            s.F[c] = F;
            s.flag[c] = fl;
        }
        s.used += hi - lo + 1;
        /* prune against the best of earlier anti-diagonals, then update it */
        int dbest = best, du = -1;
        for (int u = lo; u <= hi; ++u) {
            int64_t c = g->off + (u - lo);
            if (!(s.flag[c] & XF_COMP)) continue;
            if (s.H[c] < best - x) continue;
            s.flag[c] |= XF_LIVE;
            if (g->llo > g->lhi) g->llo = u;
            g->lhi = u;
            if (s.H[c] > dbest) {
                dbest = s.H[c];
                du = u;
            }
        }
        if (du >= 0) {
            best = dbest;
            bu = du;
            bv = d - du;
        }
        last = d;
        if (g->llo > g->lhi) break;
    }
    (void)last;
    /* canonical path back to the anchor */
    int u = bu, v = bv, state = 0, m = 0, cols = 0; /* 0 = H, 1 = E, 2 = F */
    while (!(u == 0 && v == 0 && state == 0)) {
        int64_t c = xs_at(&s, u + v, u);
        if (state == 0) {
            int64_t cd = (u >= 1 && v >= 1) ? xs_at(&s, u + v - 2, u - 1) : -1;
            if (xs_live(&s, cd) && s.H[c] == s.H[cd] + orc_blosum62(a[u - 1], b[v - 1])) {
                ++cols;
                m += (a[u - 1] == b[v - 1]);
                --u;
                --v;
            } else if (s.H[c] == s.E[c]) {
                state = 1;
            } else {
                state = 2;
            }
        } else if (state == 1) {
            ++cols;
            state = (s.flag[c] & XF_EEXT) ? 1 : 0;
            --v;
        } else {
            ++cols;
            state = (s.flag[c] & XF_FEXT) ? 2 : 0;
            --u;
        }
    }
    *u_end = bu;
    *v_end = bv;
    *matches = m;
    *columns = cols;
    *cells = ncells;
    free(s.dg);
    free(s.H);
    free(s.E);
    free(s.F);
    free(s.flag);
    return best;
}

void orc_xd_seed(const uint8_t *a, int la, const uint8_t *b, int lb, int pos_a, int pos_b, int k, int o, int e,
                 int x, orc_aln *out) {
    memset(out, 0, sizeof(*out));
    out->seed_used = -1;
    int sc = 0, sm = 0;
    for (int t = 0; t < k; ++t) {
        sc += orc_blosum62(a[pos_a + t], b[pos_b + t]);
        sm += (a[pos_a + t] == b[pos_b + t]);
    }
    int32_t ru, rv, rm, rc, lu, lv, lm, lc;
    int64_t rcells, lcells;
    int rs = orc_xdrop_extend(a + pos_a + k, la - pos_a - k, b + pos_b + k, lb - pos_b - k, o, e, x, &ru, &rv, &rm,
                              &rc, &rcells);
    uint8_t *ra = (uint8_t *)malloc((size_t)(pos_a > 0 ? pos_a : 1));
    uint8_t *rb = (uint8_t *)malloc((size_t)(pos_b > 0 ? pos_b : 1));
    for (int t = 0; t < pos_a; ++t) ra[t] = a[pos_a - 1 - t];
    for (int t = 0; t < pos_b; ++t) rb[t] = b[pos_b - 1 - t];
    int ls = orc_xdrop_extend(ra, pos_a, rb, pos_b, o, e, x, &lu, &lv, &lm, &lc, &lcells);
    free(ra);
    free(rb);
    out->score = ls + sc + rs;
    out->beg_a = pos_a - lu;
    out->beg_b = pos_b - lv;
    out->end_a = pos_a + k - 1 + ru;
    out->end_b = pos_b + k - 1 + rv;
    out->matches = lm + sm + rm;
    out->columns = lc + k + rc;
    out->cells = lcells + rcells;
}

int orc_passes(const orc_aln *r, int la, int id_pct, int cov_pct) {
    if (r->score <= 0 || r->columns <= 0) return 0;
    int64_t span = (int64_t)r->end_a - r->beg_a + 1;
    return (100LL * r->matches >= (int64_t)id_pct * r->columns) && (100LL * span >= (int64_t)cov_pct * la);
}

void orc_align_pairs(const uint8_t *codes, const int64_t *offsets, const uint32_t *pi, const uint32_t *pj,
                     const uint32_t *seed1, const uint32_t *seed2, int64_t npairs, int mode, int k, int o, int e,
                     int x, int id_pct, int cov_pct, orc_aln *out) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < npairs; ++q) {
        uint32_t i = pi[q], j = pj[q];
        int li = (int)(offsets[i + 1] - offsets[i]), lj = (int)(offsets[j + 1] - offsets[j]);
        int swapped = !(li < lj || (li == lj && i < j));
        uint32_t ia = swapped ? j : i, ib = swapped ? i : j;
        int la = swapped ? lj : li, lb = swapped ? li : lj;
        const uint8_t *a = codes + offsets[ia], *b = codes + offsets[ib];
        orc_aln r;
        if (mode == 0) {
            orc_sw(a, la, b, lb, o, e, &r);
            r.passed = orc_passes(&r, la, id_pct, cov_pct);
        } else {
            uint32_t seeds[2] = {seed1 ? seed1[q] : 0xFFFFFFFFu, seed2 ? seed2[q] : 0xFFFFFFFFu};
            int have = 0, best_pass = 0;
            int64_t cells = 0;
            memset(&r, 0, sizeof(r));
            r.seed_used = -1;
            r.beg_a = r.end_a = r.beg_b = r.end_b = -1;
            for (int s = 0; s < 2; ++s) {
                if (seeds[s] == 0xFFFFFFFFu) continue;
                /* seed keys hold the position in the lower-numbered sequence first */
                int p_lo = (int)(seeds[s] >> 16), p_hi = (int)(seeds[s] & 0xFFFF);
                int p_i = (i < j) ? p_lo : p_hi, p_j = (i < j) ? p_hi : p_lo;
                int pa = swapped ? p_j : p_i, pb = swapped ? p_i : p_j;
                if (pa < 0 || pb < 0 || pa + k > la || pb + k > lb) continue;
                orc_aln t;
                orc_xd_seed(a, la, b, lb, pa, pb, k, o, e, x, &t);
                cells += t.cells;
                int pass = orc_passes(&t, la, id_pct, cov_pct);
                /* best passing seed; without one, the best seed */
                if (!have || (pass && !best_pass) || (pass == best_pass && t.score > r.score)) {
                    r = t;
                    r.seed_used = s;
                    best_pass = pass;
                    have = 1;
                }
            }
            r.passed = best_pass;
            r.cells = cells;
        }
        r.swapped = swapped;
        out[q] = r;
    }
}
