/*
 * pastis.h -- C ABI of the gfx950 (MI355X) many-to-many protein similarity
 * search library: sequences in, weighted similarity edges out.
 *
 * The operation is the one stated in the paper's problem definition (Selvitopi
 * et al., SC20, Section II): given a set S of n protein sequences and similarity
 * constraints, compute the protein similarity graph G = (V = S, E), where an
 * edge joins two sequences that exceed the similarity threshold and carries a
 * weight.  The pipeline is that of Section IV: candidate pairs from shared
 * (optionally substitute) k-mers through a sparse product A A^T or A S A^T
 * (Sections IV-A to IV-C), pairwise alignment of every candidate by
 * Smith-Waterman or x-drop seed extension (Section IV-E), and the
 * identity/coverage filter (Section IV-F).
 *
 * Conventions for every entry point:
 *   - Every call returns a pastis_status; nothing aborts and no exception
 *     crosses this boundary.  pastis_last_error(ctx) gives a detail string.
 *   - Pointers marked "device" are HIP device pointers; "host" are host
 *     pointers.  Arguments with an `*_on_device` flag accept either.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work of a call is ordered on it.  Inputs are borrowed: the caller
 *     keeps them alive and unmodified until that work completes.  Calls that
 *     return sizes to the host synchronise the stream before returning.
 *   - A pastis_ctx is bound to one device and is not thread-safe; use one per
 *     host thread.  The library owns every buffer it allocates; results are
 *     owned until pastis_result_free.
 *   - Residues are ASCII letters of ARNDCQEGHILKMFPSTWYVBZX* (upper case);
 *     any other byte is rejected with PASTIS_E_BAD_RESIDUE.
 *   - Sequence lengths must be <= 65535 (positions are 16-bit in the kernels);
 *     longer sequences are rejected with PASTIS_E_INVAL.  Sequences shorter
 *     than k are valid and yield no k-mers; n = 0 yields no edges.  A call
 *     that discovers candidates (pastis_discover, pastis_search and the
 *     calls built on them) takes fewer than 2^30 residues in total (k-mer
 *     entries are indexed in 31 bits); more give PASTIS_E_INVAL.
 */
#ifndef PASTIS_H
#define PASTIS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pastis_status {
    PASTIS_OK = 0,
    PASTIS_E_INVAL = 1,       /* bad argument or parameter */
    PASTIS_E_BAD_RESIDUE = 2, /* a byte outside the 24-letter alphabet */
    PASTIS_E_NOMEM = 3,       /* device or host allocation failed */
    PASTIS_E_DEVICE = 4,      /* a HIP runtime error (see pastis_last_error) */
    PASTIS_E_CAPACITY = 5,    /* destination buffer too small; nothing written */
    PASTIS_E_STATE = 6        /* call out of order (e.g. no candidates yet) */
} pastis_status;

typedef enum pastis_align_mode {
    PASTIS_ALIGN_SW = 0, /* Smith-Waterman over whole sequences (Section IV-E) */
    PASTIS_ALIGN_XD = 1  /* seed-and-extend with gapped x-drop from each seed (Section IV-E) */
} pastis_align_mode;

typedef enum pastis_weight_mode {
    PASTIS_WEIGHT_ANI = 0, /* identity weight; identity/coverage cut applies (Section VI-B) */
    PASTIS_WEIGHT_NS = 1   /* score / shorter length; no cut-off (Section VI-B) */
} pastis_weight_mode;

/* Parameters of one search.  Defaults (pastis_default_params) are the paper's
 * settings of Section VI: k = 6, BLOSUM62, gap open 11, gap extend 1,
 * x-drop 49, identity >= 30%, coverage >= 70%. */
typedef struct pastis_params {
    int32_t k;                /* k-mer length, 1..8 (k <= 6 indexes a dense 24^k map of
                                 k-mer ids; longer k-mers, whose id space is too large
                                 for one, are found by binary search over the sorted
                                 distinct ids of the data) */
    int32_t n_subs;           /* m substitute k-mers per k-mer (0 = exact k-mers), 0..64 */
    int32_t sub_alphabet;     /* residues substitutes are drawn from: 20 (standard) or 24 */
    int32_t ck_min;           /* keep candidate pairs sharing >= ck_min k-mers (>= 1) */
    int32_t align_mode;       /* pastis_align_mode */
    int32_t gap_open;         /* a gap of length L costs gap_open + gap_extend * L */
    int32_t gap_extend;
    int32_t xdrop;            /* XD: X */
    int32_t min_identity_pct; /* ANI cut: 100 * matches >= pct * columns */
    int32_t min_coverage_pct; /* ANI cut: 100 * aligned span >= pct * shorter length */
    int32_t weight_mode;      /* pastis_weight_mode */
    int32_t score_width;      /* DP word width of Smith-Waterman pass 1: 16 runs pairs
                                 whose shorter side has at most 2978 rows (scores below
                                 2^15) two per wave in 16-bit lanes (records of pairs without
                                 the statistics pass then carry end_b = -1); 32 runs
                                 every pair in 32-bit lanes; 0 (automatic) takes 16
                                 inside pastis_search with identity weights and 32
                                 elsewhere.  16 needs gap_open + gap_extend >= 4. */
    int32_t full_records;     /* 1: traceback statistics (beg, matches, columns) for every
                                 aligned pair; 0: only for pairs whose coverage cut can
                                 still hold (the others report beg = -1, passed = 0) */
    int32_t filter_mode;      /* 0: align every candidate; 1: align only candidates the
                                 learned filter keeps (pastis_mlp_set first) */
    int32_t graph_mode;       /* 1: run the Smith-Waterman stage as one captured HIP graph
                                 on a stream of the context, replayed while the pair
                                 count, buffers and schedule are unchanged (per-bin
                                 times are then not recorded); 0: direct launches */
    int32_t candidate_room;   /* room, in entries, for the directional candidates of a
                                 discovery (before the two directions merge): 0 sizes it
                                 automatically (products / ck_min when that fits 2^28
                                 entries, else the last call's count plus a quarter); a
                                 discovery that needs more is redone once with room for
                                 all of its entries.  >= 0 */
    int32_t block_entries;    /* pastis_search only: the most directional candidate
                                 entries one row block of the discovery may hold (0: the
                                 2^32 - 16 that 32-bit indices allow).  A block is the set
                                 of pairs whose lower sequence index falls in a range;
                                 the search starts with one block of every sequence and
                                 splits a block whose entries exceed this (into parts
                                 sized from the entries it asked for), then discovers,
                                 aligns and cuts the blocks one after the other, so the
                                 discovery's memory follows one block's entries (24 bytes
                                 each, plus the sort's second buffer) and the edges are
                                 the same as in one block.  A block of one sequence that
                                 still exceeds it fails with PASTIS_E_CAPACITY.  With
                                 several blocks, pastis_candidates_copy has nothing to
                                 copy after the search (PASTIS_E_STATE).  The
                                 substitute product runs every row from a block's first
                                 sequence on, once per block.  >= 0 (the future work of
                                 Section VII: B formed, aligned and freed in parts) */
    int32_t reserved[3];      /* must be zero */
} pastis_params;

/* One similarity edge, 48 bytes.  i < j; edges are sorted by (i, j).
 * Positions are 0-based and inclusive.  identity = matches / columns and
 * ns_weight = score / min(len_i, len_j), both IEEE float32 round-to-nearest.
 * Edges of weight_mode NS carry no traceback results: begins and ends are
 * 0xFFFFFFFF and matches, columns and identity 0 (the weight needs only the
 * score, so the search skips the passes that find them). */
typedef struct pastis_edge {
    uint32_t i, j;
    int32_t score;
    uint32_t matches, columns;
    uint32_t beg_i, end_i, beg_j, end_j;
    uint16_t shared_kmers; /* candidate count (capped at 65535) */
    uint8_t seed_used;     /* XD: 0 or 1; SW: 255 */
    uint8_t flags;         /* bit 0: the alignment's rows were sequence j (j shorter) */
    float identity;
    float ns_weight;
} pastis_edge;

/* Per-pair alignment record returned by pastis_align_pairs, 48 bytes, in the
 * orientation rows = a = the shorter sequence of the pair (the first on equal
 * length), columns = b.  Fields are -1 / 0 when there is no alignment. */
typedef struct pastis_pair_record {
    int32_t score;
    int32_t beg_a, end_a, beg_b, end_b;
    int32_t matches, columns;
    int32_t seed_used; /* XD: index of the chosen seed, -1 if none; SW: -1 */
    int32_t passed;    /* 1 when the identity and coverage cut holds */
    int32_t swapped;   /* 1 when a is the second sequence of the pair */
    int64_t cells;     /* DP cells evaluated for this pair */
} pastis_pair_record;

typedef struct pastis_run_stats {
    int64_t n_sequences;
    int64_t n_residues;
    int64_t n_kmers;          /* nnz(A): distinct (sequence, k-mer) entries */
    int64_t n_candidates;     /* pairs passing the common-k-mer threshold */
    int64_t n_aligned;        /* pairs aligned */
    int64_t n_edges;
    int64_t cells;            /* DP cells evaluated */
    int64_t stats_pass_pairs; /* pairs that needed the statistics pass */
    int64_t int32_pairs;      /* pairs computed with 32-bit DP words */
    double ms_total;    /* host wall time of the call */
    double ms_stage[9]; /* device time (HIP events on the call's stream) of: encode,
                           k-mers, S formation, SpGEMM, schedule, alignment pass 1,
                           alignment pass 2, identity/coverage cut and edges, learned
                           pre-alignment filter */
    /* Smith-Waterman pass 1 per length bin (one kernel launch each): rows per
     * lane R, whether the bin's pairs span several strips of 64 * R rows, and
     * the bin's pairs, DP cells and device time (HIP events around the launch,
     * on the call's stream).  sw_bins = 0 after an x-drop call. */
    int32_t sw_bins;
    int32_t sw_bin_rows[32];
    int32_t sw_bin_multi[32];
    int32_t sw_bin_bits[32]; /* 16: two pairs per wave in 16-bit lanes; 32: one pair */
    int64_t sw_bin_pairs[32];
    int64_t sw_bin_cells[32];
    double sw_bin_ms[32];
    /* Smith-Waterman pairs (and their end-rectangle cells) that took the
     * start-bound pass, and cells of the statistics pass. */
    int64_t bound_pass_pairs;
    int64_t bound_pass_cells;
    int64_t stats_pass_cells;
    int32_t sw_graph;         /* Smith-Waterman stage: 0 direct launches, 1 graph captured
                                 and launched, 2 graph replayed */
    int32_t sw_graph_pad;
    /* candidate discovery: postings visited by the sparse product (one pass
     * over every row's entries; the counting and the seed phase each make
     * one such pass) */
    int64_t spgemm_products;
    /* nnz(S): entries of the substitute matrix's rows over the data's k-mers
     * (each k-mer itself and its substitutes present in some sequence); 0
     * with exact k-mers */
    int64_t n_subs_entries;
    /* row blocks the last pastis_search ran (1 unless block_entries split
     * its discovery); 0 after the other calls */
    int64_t n_row_blocks;
} pastis_run_stats;

typedef struct pastis_ctx pastis_ctx;
typedef struct pastis_result pastis_result;

/* Fill *p with the defaults listed above (n_subs 0, ck_min 1, SW, ANI). */
void pastis_default_params(pastis_params *p);

/* Create a context on HIP device `device` with a validated copy of *p.
 * Errors: PASTIS_E_INVAL (bad parameter), PASTIS_E_DEVICE. */
pastis_status pastis_create(const pastis_params *p, int device, pastis_ctx **out);
void pastis_destroy(pastis_ctx *ctx);

const char *pastis_status_string(pastis_status s);
/* Detail of the last failure on ctx (empty string if none); owned by ctx. */
const char *pastis_last_error(const pastis_ctx *ctx);
/* First offending byte index of the last PASTIS_E_BAD_RESIDUE, else -1. */
int64_t pastis_bad_residue_index(const pastis_ctx *ctx);

/* Stage 1 of Section IV: encode residues (Section V-B numbering) into
 * `codes` (device, n_residues bytes).  residues: device or host per flag.
 * Errors: PASTIS_E_BAD_RESIDUE (index via pastis_bad_residue_index). */
pastis_status pastis_encode(pastis_ctx *ctx, const uint8_t *residues, int64_t n_residues, int input_on_device,
                            uint8_t *codes, void *stream);

/* Align a given list of pairs (Section IV-E) and apply the filter of
 * Section IV-F, with the context's align_mode and scoring parameters.
 *   residues [offsets[n]] ASCII, offsets [n+1] int64: device or host per flag;
 *   pi, pj [npairs] uint32 sequence indices (pi != pj), device;
 *   seed1, seed2 [npairs] uint32 seed keys (pos_in_min(pi,pj) << 16 |
 *     pos_in_max(pi,pj)), 0xFFFFFFFF = absent, device; may be NULL for SW;
 *   out [npairs] pastis_pair_record, device.
 * Errors: PASTIS_E_INVAL (index out of range, length > 65535),
 * PASTIS_E_BAD_RESIDUE, PASTIS_E_DEVICE. */
pastis_status pastis_align_pairs(pastis_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n,
                                 int input_on_device, const uint32_t *pi, const uint32_t *pj, const uint32_t *seed1,
                                 const uint32_t *seed2, int64_t npairs, pastis_pair_record *out, void *stream);

/* pastis_align_pairs for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and records, with every buffer of the call
 * carved from a static workspace of PASTIS_NOALLOC_BYTES per GPU (held
 * until the process ends) instead of the context's allocations.  Inputs and
 * outputs as for pastis_align_pairs with input_on_device = 1: residues,
 * offsets, pi, pj, seeds and out are all device memory, borrowed until the
 * stream reaches the end of the call's work.  Smith-Waterman only
 * (align_mode SW), direct launches (graph_mode is ignored).  The workspace
 * holds the residue codes (one byte each) and about 100 bytes per pair;
 * every sequence of the set must have at most 1,024 residues (longer ones
 * need boundary rows of the long-sequence bins, tens of MiB per residue of
 * length).  A call that needs more than the workspace returns
 * PASTIS_E_CAPACITY without writing out.  Calls that overlap on one GPU (from
 * any context or thread) race on the workspace and must not be issued.
 * Errors otherwise as for pastis_align_pairs. */
#define PASTIS_NOALLOC_BYTES (48u << 20)
pastis_status pastis_align_pairs_noalloc(pastis_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n,
                                         const uint32_t *pi, const uint32_t *pj, const uint32_t *seed1,
                                         const uint32_t *seed2, int64_t npairs, pastis_pair_record *out,
                                         void *stream);

/* Candidate discovery (Sections IV-A to IV-C, threshold of Section VI): k-mers
 * of every sequence (A), the m nearest substitutes of every distinct k-mer
 * when n_subs > 0 (S), the sparse product A A^T or (A S) A^T under the count +
 * seed semiring, the common-k-mer threshold ck_min and, with substitutes,
 * symmetrisation (each pair keeps the direction with the larger count; the
 * lower-numbered sequence's direction on a tie).  Candidates stay in ctx;
 * *n_candidates receives their number.  Inputs as for pastis_align_pairs.
 * Errors: PASTIS_E_INVAL, PASTIS_E_BAD_RESIDUE, PASTIS_E_NOMEM, PASTIS_E_DEVICE. */
pastis_status pastis_discover(pastis_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n,
                              int input_on_device, void *stream, int64_t *n_candidates);

/* Copy the last discovery's candidates, sorted by (lo, hi), lo < hi:
 * count = shared (substitute) k-mers, seed1 / seed2 = the two smallest keys
 * (pos_in_lo << 16 | pos_in_hi), 0xFFFFFFFF when absent.  Any destination may
 * be NULL (skipped).  PASTIS_E_CAPACITY if cap < count (nothing written);
 * PASTIS_E_STATE if there was no discovery. */
pastis_status pastis_candidates_copy(pastis_ctx *ctx, uint32_t *lo, uint32_t *hi, uint32_t *count, uint32_t *seed1,
                                     uint32_t *seed2, int64_t cap, int dst_on_device, void *stream);

/* The ctx's n_subs nearest substitutes (Section IV-B) of n k-mer ids (radix
 * 24 over the context's k, 64-bit: up to 24^8), all device arrays:
 * out_ids / out_dist [n][n_subs], out_count [n] = entries written per k-mer
 * (n_subs unless the k-mer space is smaller).  Within a k-mer the entries
 * are not ordered.
 * Errors: PASTIS_E_INVAL (n_subs == 0 or bad arguments), PASTIS_E_DEVICE. */
pastis_status pastis_subkmers(pastis_ctx *ctx, const uint64_t *kmer_ids, int64_t n, uint64_t *out_ids,
                              int32_t *out_dist, int32_t *out_count, void *stream);

/* Sequences in, weighted similarity edges out (Section II problem, Section IV
 * pipeline): discovery, alignment of every candidate with the context's
 * align_mode, then the Section IV-F cut (weight_mode ANI) or no cut
 * (weight_mode NS, every positive score).  *out owns the edges until
 * pastis_result_free.  Errors as for pastis_discover. */
pastis_status pastis_search(pastis_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n,
                            int input_on_device, void *stream, pastis_result **out);
pastis_status pastis_result_count(const pastis_result *r, int64_t *n_edges);
/* Device pointer to the result's edges (owned by the result). */
const pastis_edge *pastis_result_device_ptr(const pastis_result *r);
/* Copy all edges to dst (host or device); PASTIS_E_CAPACITY if cap is too small. */
pastis_status pastis_result_copy(const pastis_result *r, pastis_edge *dst, int64_t cap, int dst_on_device,
                                 void *stream);
void pastis_result_free(pastis_result *r);

/* ---- learned pre-alignment filter (not part of the paper) ----
 * A 16-128-128-1 MLP (ReLU, sigmoid output) scores each candidate from 16
 * features: shared-k-mer count; seed-1 diagonal (pos_b - pos_a) / Lb;
 * |diag2 - diag1| / Lb; ln La; ln Lb; La / Lb; |composition difference| over
 * the residue groups {AG}{ST}{DE}{NQ}{KRH}{IV}{LM}{FYW}{C}{P} (a = shorter
 * sequence).  Inputs are z-scored and cast to bf16; weights and activations
 * are bf16 copies with fp32 accumulation on matrix cores; biases stay fp32.
 * Parameters: one fp32 vector of PASTIS_MLP_PARAMS values, W1 [128][16],
 * b1 [128], W2 [128][128], b2 [128], w3 [128], b3 [1].  A candidate is kept
 * when its logit >= tau (the logit threshold). */
#define PASTIS_MLP_FEATURES 16
#define PASTIS_MLP_PARAMS 18817

/* Raw features [n_candidates][16] (device, fp32) of the last discovery's
 * candidates over the given sequences (same as that discovery's).
 * PASTIS_E_STATE without a discovery; PASTIS_E_CAPACITY if cap < count. */
pastis_status pastis_mlp_features(pastis_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n,
                                  int input_on_device, float *features, int64_t cap, void *stream);
/* Set the network (host arrays): params [PASTIS_MLP_PARAMS], feature mean and
 * std [16], logit threshold tau.  Resets the optimiser state. */
pastis_status pastis_mlp_set(pastis_ctx *ctx, const float *params, const float *mean, const float *stdv, float tau);
/* Read the network back (host arrays; any may be NULL). */
pastis_status pastis_mlp_get(pastis_ctx *ctx, float *params, float *mean, float *stdv, float *tau);
/* mean / std of each feature column of X [n][16] (device) become the
 * network's normalisation. */
pastis_status pastis_mlp_fit_normalizer(pastis_ctx *ctx, const float *X, int64_t n, void *stream);
/* logits [n] (device) of raw features X [n][16] (device). */
pastis_status pastis_mlp_forward(pastis_ctx *ctx, const float *X, int64_t n, float *logits, void *stream);
/* Gradient (host [PASTIS_MLP_PARAMS]) and value (host) of the mean weighted
 * binary cross-entropy over X [n][16] with labels [n] (device, 0/1):
 * loss = mean(pos_weight * t * softplus(-y) + (1 - t) * softplus(y)). */
pastis_status pastis_mlp_grad(pastis_ctx *ctx, const float *X, const uint8_t *labels, int64_t n, float pos_weight,
                              float *grad, float *loss, void *stream);
/* One pass over the examples order[0..n) (device int32 indices into the
 * n_examples rows of X / labels, checked before any update: PASTIS_E_INVAL if
 * one is out of range) in minibatches of `batch` (multiple of 16, <= 65536):
 * gradient, then an Adam step (beta 0.9 / 0.999, eps 1e-8) on the fp32
 * masters.  *mean_loss (host, may be NULL) gets the mean minibatch loss. */
pastis_status pastis_mlp_train_epoch(pastis_ctx *ctx, const float *X, const uint8_t *labels, int64_t n_examples,
                                     const int32_t *order, int64_t n, int32_t batch, float lr, float pos_weight,
                                     float *mean_loss, void *stream);
/* Logit threshold keeping at least target_recall of the positive examples of
 * X / labels (device); also stored as the network's tau. */
pastis_status pastis_mlp_calibrate(pastis_ctx *ctx, const float *X, const uint8_t *labels, int64_t n,
                                   double target_recall, float *tau, void *stream);

/* ---- filter lifecycle inside the library ----
 * Labelled examples come from the exact pipeline: pastis_mlp_collect runs
 * discovery on a sequence set, computes the 16 features of every candidate
 * and labels it with the pass/fail of its exact alignment (the context's
 * align_mode, the Section IV-F identity/coverage cut), appending both to an
 * example pool the context owns in device memory.  pastis_mlp_train then
 * trains a fresh network on the pool and calibrates its threshold. */

/* Append the labelled candidates of one sequence set to the context's pool.
 * discovery (may be NULL) overrides k, n_subs, sub_alphabet and ck_min for
 * this collection only (so one pool can mix exact and substitute k-mer
 * candidates); the other fields of *discovery are ignored.  *n_added (host,
 * may be NULL) gets the number of examples added.  The discovery's
 * candidates replace the context's current ones.  Errors as for
 * pastis_discover; PASTIS_E_INVAL for discovery fields out of range. */
pastis_status pastis_mlp_collect(pastis_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n,
                                 int input_on_device, const pastis_params *discovery, void *stream,
                                 int64_t *n_added);
/* Empty the example pool (its memory is kept for the next collection). */
pastis_status pastis_mlp_clear(pastis_ctx *ctx);
/* Examples in the pool. */
pastis_status pastis_mlp_pool_size(const pastis_ctx *ctx, int64_t *n);

typedef struct pastis_mlp_train_opts {
    int32_t epochs;       /* passes over the training share, 1..1000 */
    int32_t batch;        /* minibatch: a multiple of 16 in 16..65536 */
    float lr;             /* Adam step size, > 0 */
    float pos_weight;     /* positive-class weight; <= 0: negatives / positives of the training share */
    double target_recall; /* in (0, 1]: share of the calibration positives kept at tau */
    double heldout;       /* in (0, 0.9]: share of the pool held out; one half calibrates
                             tau, the other measures recall and the kept share */
    uint64_t seed;        /* initial weights, the split and every epoch's shuffle */
    int32_t reserved[4];  /* zero */
} pastis_mlp_train_opts;

typedef struct pastis_mlp_train_report {
    int64_t n_examples;    /* pool size */
    int64_t n_train;       /* examples trained on */
    int64_t n_positive;    /* positives among them */
    float pos_weight;      /* positive-class weight used */
    float tau;             /* calibrated logit threshold, also installed in the context */
    double heldout_recall; /* positives of the measuring half with logit >= tau */
    double heldout_kept;   /* share of the measuring half with logit >= tau */
    double seconds;        /* wall time of the call */
    int32_t epochs;        /* epochs run */
    float epoch_loss[32];  /* mean minibatch loss of the first 32 epochs */
} pastis_mlp_train_report;

/* {4, 8192, 2e-3, 0 (auto), 0.995, 0.2, seed 0}. */
void pastis_mlp_default_train_opts(pastis_mlp_train_opts *opts);
/* Train a new network on the pool (opts NULL: the defaults), all on the GPU:
 * a seeded permutation splits the pool into held-out and training shares;
 * the positive-class weight, the z-score normalisation and He-normal initial
 * weights come from the training share; each epoch reshuffles it and runs
 * minibatch gradients and Adam steps (as pastis_mlp_train_epoch); tau is
 * calibrated on half of the held-out share (as pastis_mlp_calibrate) and
 * measured on the other half.  The network replaces the context's.
 * PASTIS_E_STATE if the pool holds fewer than 64 examples or the training
 * share has no positive; PASTIS_E_INVAL for options out of range.  *report
 * (host, may be NULL). */
pastis_status pastis_mlp_train(pastis_ctx *ctx, const pastis_mlp_train_opts *opts, void *stream,
                               pastis_mlp_train_report *report);
/* Write the network (parameters, normalisation, tau) to a file: an 8-byte
 * magic "PASTMLP1", int32 features (16), hidden width (128), parameter count
 * (18817) and 0, then float32 params, mean[16], std[16], tau, little-endian.
 * PASTIS_E_STATE without a network; PASTIS_E_INVAL if the file cannot be
 * written. */
pastis_status pastis_mlp_save(pastis_ctx *ctx, const char *path);
/* Read a network written by pastis_mlp_save and install it (as
 * pastis_mlp_set).  PASTIS_E_INVAL for a missing, short or foreign file or a
 * non-positive std; the context's network is unchanged then. */
pastis_status pastis_mlp_load(pastis_ctx *ctx, const char *path);

/* ---- schedule of the Smith-Waterman stage ----
 * Knobs of the length-binned launches (every setting gives the same results;
 * only the time changes).  A new context starts at {16, 50, 1, 1, 0, 4, 4}.  pastis_autotune times candidate settings on a
 * sample of the given sequences' own candidate pairs and keeps the fastest. */
typedef struct pastis_tuning {
    int32_t sw16_max_rows; /* bins with at most this many rows per lane run two pairs per
                              wave in 16-bit lanes (0: none; at most 16): one-strip bins,
                              and multi-strip bins of sequences of at most 2978 rows;
                              where 16-bit lanes are in use (see score_width) */
    int32_t sw_direct_pct; /* pairs with 100 * score >= this * (shorter length) skip the
                              start-bound pass and go straight to the statistics pass */
    int32_t sw_grid_scale; /* one-strip launches (pass 1, start bound, statistics) of bins
                              with at most 8 rows per lane get this many times the
                              blocks that fit on the device at once (1..64; never more
                              than the call's pairs can fill).  Every launch drains a
                              work queue, so 1 (a resident grid) suffices */
    int32_t sw_grid_scale_wide; /* the same for 9..16 rows per lane (1..64) */
    int32_t sw_intra_pair; /* 1: pass 1 of sequences a longer than 2978 rows (32-bit lanes)
                              runs one workgroup of four waves per pair, strips
                              pipelined across the waves (intra-pair mode); 0: one
                              wave per pair (inter-pair mode) */
    int32_t sw16_narrow_rows; /* pairs per wavefront of the 16-bit bins of at most 4 rows per
                                 lane: bins of at most this many rows per lane (0..4) run
                                 strips of 16 lanes, eight pairs per wave; the others
                                 strips of 32 lanes, four pairs per wave (a wave's pairs
                                 share their shorter sequence, so sets with few candidates
                                 per sequence fill fewer slots of the wider grouping) */
    int32_t sw_long_blocks; /* blocks per CU (1..4) of the multi-strip launches (sequences a
                               over 1024 rows), which run on the context's second stream
                               beside the one-strip bins: fewer leave those more waves */
    int32_t reserved[1];
} pastis_tuning;

pastis_status pastis_get_tuning(const pastis_ctx *ctx, pastis_tuning *out);
/* PASTIS_E_INVAL for values out of range. */
pastis_status pastis_set_tuning(pastis_ctx *ctx, const pastis_tuning *t);
/* Discovery on the given sequences, then for each knob in turn (16-bit rows,
 * start-bound routing, the two grid scales, inter- vs intra-pair mode, pairs
 * per wavefront, the long bins' grid) the alignment of a sample of the candidates under each
 * candidate value, twice, timed with HIP events on the stream; the fastest
 * setting is kept in ctx and written to *out (may be NULL).  The sample is
 * every candidate whose shorter sequence falls in a hashed subset of the
 * sequences sized for about max_pairs candidates (at most max_pairs), so the
 * pairs that share a sequence stay together as in the whole set.  A value
 * replaces the one in force only when it is at least 1% faster on the
 * sample.  When the sample is smaller than the candidate set, the knobs
 * whose effect lies in the tails of the launches, which shrink with the
 * sample (start-bound routing: 25, 50, 75, 100; inter- vs intra-pair mode;
 * the long bins' grid; the two grid scales), are then timed once more per value on all the
 * candidates, where a 0.5% margin applies (skipped for sets of over 2^26
 * candidates, or when one alignment of all of them takes over 2 s).  The
 * discovery's candidates stay in ctx. */
pastis_status pastis_autotune(pastis_ctx *ctx, const uint8_t *residues, const int64_t *offsets, int64_t n,
                              int input_on_device, int64_t max_pairs, void *stream, pastis_tuning *out);

/* ---- the similarity graph as families (Section VI-B, Table II) ---- */

/* Connected components of the undirected graph on n vertices (sequences)
 * with the given edges (device pastis_edge [n_edges], e.g. a search result's
 * device pointer; only i and j are read).  label [n] (device) gets, for
 * every vertex, the smallest vertex of its component.  PASTIS_E_INVAL if an
 * endpoint is >= n (label is then undefined). */
pastis_status pastis_components(pastis_ctx *ctx, const pastis_edge *edges, int64_t n_edges, int64_t n,
                                uint32_t *label, void *stream);
/* Weighted precision and recall (host doubles) of a clustering of n
 * sequences against reference families, both per sequence on the device:
 * cluster [n] uint32 labels < n, family [n] int32 < n, a negative family
 * marking a sequence outside every family (a family of its own).  With n_cf
 * the sequences of cluster c in family f: precision = sum_c max_f n_cf / n
 * (clusters mixing families lose precision), recall = sum_f max_c n_cf / n
 * (families split over clusters lose recall).  PASTIS_E_INVAL for labels or
 * families >= n. */
pastis_status pastis_cluster_scores(pastis_ctx *ctx, const uint32_t *cluster, const int32_t *family, int64_t n,
                                    double *precision, double *recall, void *stream);

/* Counters and per-stage times of the last pastis_search / pastis_align_pairs. */
pastis_status pastis_stats(const pastis_ctx *ctx, pastis_run_stats *out);

#ifdef __cplusplus
}
#endif
#endif
