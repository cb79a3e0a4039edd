/*
 * CPU oracle for many-to-many protein similarity search (PASTIS, SC20).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously-correct C written from the
 * paper's definitions.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it; the GPU library never links, includes
 * or calls anything here, and nothing here comes from the GPU library.
 *
 * Conventions shared by every function (the readings of the paper are listed
 * where they are used):
 *   - residues are codes 0..23 in the order ARNDCQEGHILKMFPSTWYVBZX*
 *     (Section V-B); positions are 0-based;
 *   - integer scores are exact, so every result is compared bit for bit.
 */
#ifndef PASTIS_ORACLE_H
#define PASTIS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NEG_INF (-(1 << 29))

/* ---- alphabet and scoring (Section IV-B figure of BLOSUM62; Section V-B) ---- */
const char *orc_alphabet(void);
int orc_blosum62(int a, int b);
/* ASCII -> code; returns -1 when every byte is valid, else the index of the
 * first byte outside the 24-letter alphabet. */
int64_t orc_encode(const uint8_t *ascii, int64_t len, uint8_t *codes);

/* ---- k-mers (Sections IV-A, V-B) ---- */
/* id = sum_t code[t] * 24^(k-1-t) (leftmost residue most significant). */
int64_t orc_kmer_id(const uint8_t *codes, int k);
/* Distinct k-mers of one sequence with their first start position, sorted by
 * id.  Returns the count (0 when len < k). */
int64_t orc_kmer_set(const uint8_t *codes, int64_t len, int k, int64_t *ids, int32_t *pos);

/* ---- substitute k-mers (Section IV-B, Algorithms 1-3) ---- */
/* expense(a -> b) = C[a][a] - C[a][b]  (E = Sort(Diag(C) - C)). */
int orc_expense(int a, int b);
/* Sorted expense row of base a over the first alpha residues: bases and
 * expenses ascending by (expense, base).  Returns alpha. */
int orc_expense_row(int a, int alpha, int32_t *base, int32_t *expense);
/* m nearest substitutes of k-mer r (distinct from r), ordered by (Dist, id),
 * over all k-mers made of the first `alpha` residues.  Brute force over all
 * alpha^k k-mers.  Returns the number written (min(m, alpha^k - [r in set])). */
int orc_subk_bruteforce(int64_t r, int k, int m, int alpha, int64_t *ids, int32_t *dist);
/* Same set, found by enumerating every k-mer within distance D for the
 * smallest sufficient D (distances are sums of non-negative expenses). */
int orc_subk_bounded(int64_t r, int k, int m, int alpha, int64_t *ids, int32_t *dist);

/* ---- candidate discovery (Sections IV-A, IV-C; CK threshold Section VI) ---- */
/* Sequences are given as codes + offsets[n+1].  Outputs are arrays with one
 * entry per candidate pair lo < hi, sorted by (lo, hi):
 *   count  = shared k-mers (exact) or max-direction substitute count,
 *   seed1/2 = (pos_lo << 16 | pos_hi), the two smallest keys, 0xFFFFFFFF if absent.
 * Returns the number of candidates, or -1 when `cap` is too small. */
int64_t orc_candidates_bruteforce(const uint8_t *codes, const int64_t *offsets, int64_t n, int k, int ck_min,
                                  int64_t cap, uint32_t *lo, uint32_t *hi, uint32_t *count, uint32_t *seed1,
                                  uint32_t *seed2);
/* Row-wise inverted-index form of the same definition; with n_subs > 0 the
 * substitute semiring is used: S(p) = {p} U N_m(p), (AS)_{i,s} keeps the
 * closest k-mer of i (min Dist, then min position), the directional count
 * c(r->c) = |{s in K(c) : (AS)_{r,s} defined}| and the pair keeps the larger
 * direction (tie: lo -> hi).  `rows` (nrows entries) restricts output to
 * pairs with lo or hi in that set when nrows >= 0; pass nrows = -1 for all. */
int64_t orc_candidates_index(const uint8_t *codes, const int64_t *offsets, int64_t n, int k, int n_subs,
                             int alpha, int ck_min, const int64_t *rows, int64_t nrows, int64_t cap, uint32_t *lo,
                             uint32_t *hi, uint32_t *count, uint32_t *seed1, uint32_t *seed2);
/* The same quantities for a given list of pairs lo < hi only (both
 * directions of the substitute product, the larger kept, lo -> hi on a tie):
 * count = 0 when the pair shares nothing.  Needs only the sequences of the
 * pairs, so it runs at any set size.  Returns npairs, or -1 on a bad pair. */
int64_t orc_pair_counts(const uint8_t *codes, const int64_t *offsets, int64_t n, int k, int n_subs, int alpha,
                        const uint32_t *lo, const uint32_t *hi, int64_t npairs, uint32_t *count, uint32_t *seed1,
                        uint32_t *seed2);

/* ---- alignment (Section IV-E) and similarity filter (Section IV-F) ---- */
typedef struct {
    int32_t score;
    int32_t beg_a, end_a, beg_b, end_b; /* 0-based inclusive; -1 when empty */
    int32_t matches, columns;
    int32_t seed_used; /* XD: index of the chosen seed; SW: -1 */
    int32_t passed;    /* 1 when identity and coverage cuts both hold */
    int32_t swapped;   /* 1 when a = second sequence of the pair */
    int64_t cells;     /* DP cells evaluated (SW: La*Lb; XD: live cells) */
} orc_aln;

/* Smith-Waterman with affine gaps (gap of length L costs o + e*L), full
 * traceback.  a has the rows.  Canonical end: smallest row, then column, among
 * maxima; canonical path preference diagonal > E > F, extend > open. */
void orc_sw(const uint8_t *a, int la, const uint8_t *b, int lb, int o, int e, orc_aln *out);
/* One x-drop extension from the anchor (0,0) of a and b (already reversed for
 * a left extension).  Returns score; writes end (u,v), matches, columns, cells. */
int32_t orc_xdrop_extend(const uint8_t *a, int la, const uint8_t *b, int lb, int o, int e, int x, int32_t *u_end,
                         int32_t *v_end, int32_t *matches, int32_t *columns, int64_t *cells);
/* Seed-and-extend for one seed (pos_a, pos_b) of length k. */
void orc_xd_seed(const uint8_t *a, int la, const uint8_t *b, int lb, int pos_a, int pos_b, int k, int o, int e,
                 int x, orc_aln *out);
/* Identity/coverage cut: 100*matches >= id_pct*columns and
 * 100*span_a >= cov_pct*la (a = shorter sequence). */
int orc_passes(const orc_aln *r, int la, int id_pct, int cov_pct);

/* Align candidate pairs (i, j) of a sequence set.  mode 0 = SW, 1 = XD.
 * Orientation: a = shorter sequence, ties -> the lower index.  XD keeps the
 * best-scoring seed among those that pass the cut (tie: first seed); when no
 * seed passes, the best-scoring seed.  Runs pairs in parallel (OpenMP). */
void orc_align_pairs(const uint8_t *codes, const int64_t *offsets, const uint32_t *pi, const uint32_t *pj,
                     const uint32_t *seed1, const uint32_t *seed2, int64_t npairs, int mode, int k, int o, int e,
                     int x, int id_pct, int cov_pct, orc_aln *out);

int orc_num_threads(void);
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
