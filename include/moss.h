/* moss.h - C ABI of the MI355X (gfx950) Moss graphlet sampler.
 *
 * Moss (Wang, Tao, Zhao, Guan, arXiv 1509.08089) estimates n_1..n_6, the numbers
 * of 4-node connected induced subgraphs (CISes) of each motif class of an
 * undirected simple graph, and eta_1..eta_21 for 5 nodes (problem statement,
 * Section 2), by drawing independent samples with degree-based probabilities
 * (MOSS-4, Section 4.1, Algorithm 1; MOSS-4Min, Section 4.2, Algorithm 2; T-5 and
 * Path-5, Section 5.1, Algorithms 3 and 4), classifying each sample and scaling the
 * per-class hit counts by the inverse sampling probability (Theorems 2, 4, 6, 8),
 * with the exact variance formulas of Theorems 3, 5 and 10.
 *
 * Conventions for every call:
 *  - Every call returns a moss_status; outputs are written only on MOSS_OK.
 *    No C++ exception crosses this boundary.
 *  - Device pointers are HIP device addresses on the graph's device; host
 *    pointers are ordinary CPU memory.  Sizes are element counts unless noted.
 *  - A graph and everything built for it live on the device that was current
 *    when it was created; its work is queued on the stream given at creation
 *    (NULL = the default stream).  Calls on one graph must not overlap
 *    (MOSS_E_BUSY otherwise); a server holds a graph registered with it while it
 *    builds or evicts the graph's tables.
 *  - Results are a pure function of (graph, k, n_samples, seed, flags): they do
 *    not depend on grid size, batch membership, tile size or arrival time.
 *
 * Sampling contract (where the paper leaves the choice open):
 *  - random words: B(k, j) = Philox4x64-10(counter (k, j, 0, 0), key (seed, tag))
 *    (Salmon et al., SC 2011), tag = sampler id below, k = sample index;
 *  - a word x picks r = floor(x * N / 2^64) uniformly from [0, N);
 *  - WeightRandomVertex (Section 4.1.3) returns the smallest i with ACC[i] > r over
 *    the inclusive prefix ACC of the weights;
 *  - RandomVertex over a row with excluded slots (Sections 4.1.3, 5.1.1, 5.1.5)
 *    shifts the index past the excluded slots in ascending order.
 */
#ifndef MOSS_H
#define MOSS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MOSS_OK = 0,
  MOSS_E_ARG = -1,         /* bad argument or malformed row_ptr / column id out of range */
  MOSS_E_UNSORTED = -2,    /* a CSR row is not strictly ascending */
  MOSS_E_SELF_LOOP = -3,   /* v in N_v */
  MOSS_E_DUPLICATE = -4,   /* repeated neighbour */
  MOSS_E_ASYMMETRIC = -5,  /* u in N_v but v not in N_u */
  MOSS_E_OVERFLOW = -6,    /* a weight, prefix or Lambda needs more than 64 bits, or a row
                              sum of (d_x - 1) more than 32 bits */
  MOSS_E_NOMEM = -7,       /* device or host allocation failed */
  MOSS_E_DEVICE = -8,      /* HIP runtime error / no usable device */
  MOSS_E_NOT_BUILT = -9,   /* tables for this k were not built */
  MOSS_E_BUSY = -10,       /* another call on the same graph is in flight */
  MOSS_E_TIMEOUT = -11,    /* server wait timed out (the request keeps running) */
  MOSS_E_CANCELLED = -12,  /* server request cancelled or server shut down */
  MOSS_E_ADMISSION = -13,  /* server cannot ever admit the request (memory budget) */
  MOSS_E_TOO_LARGE = -14   /* more samples than moss_sample_range_noalloc's fixed scratch holds */
} moss_status;

/* sampler ids (also the Philox key tag of each sampler) */
#define MOSS_SAMPLER_MOSS4 0x4   /* Algorithm 1 */
#define MOSS_SAMPLER_MOSS4MIN 0x41 /* Algorithm 2 */
#define MOSS_SAMPLER_T5 0x51     /* Algorithm 3 */
#define MOSS_SAMPLER_PATH5 0x52  /* Algorithm 4 */

/* graph creation flags */
#define MOSS_TRUST_CSR 0x1u      /* skip the sortedness/duplicate/symmetry checks
                                    (row_ptr monotonicity and column range are
                                    always checked) */

/* estimate flags: how the two 5-node estimates are mixed (Section 5.1.3) */
#define MOSS_MIX_POOLED 0x0u     /* lambda^(l)_i = K_l p^(l)_i / sum_l K_l p^(l)_i (default) */
#define MOSS_MIX_PAPER 0x1u      /* lambda from the Theorem 7/9 variances evaluated at the
                                    pooled estimate (Eq. mixestimator, Eq. varianceMix) */
/* estimate flag for k = 4: run MOSS-4 and MOSS-4Min on half the budget each and mix
   their estimates of n_3, n_5, n_6 (Section 4.2, Theorem 1), with the pooled or the
   paper's weights as for 5 nodes */
#define MOSS_K4_MIN 0x2u

/* table-build mask bits */
#define MOSS_TABLES_K4 (1u << 4) /* ACC_Gamma, ACC_sigma, node guide */
#define MOSS_TABLES_K5 (1u << 5) /* ACC_Gamma1, ACC_Gamma2, ACC_sigma, ACC_tau, guides */
#define MOSS_TABLES_K4MIN (1u << 6) /* MOSS-4Min: rank tables, rows in descending order,
                                       ACC_check, ACC_check-Gamma, guides */

/* tables that moss_table_read can copy out */
#define MOSS_TAB_ACC_GAMMA 5     /* u64[n]  inclusive prefix of Gamma_v     (Section 4.1.3) */
#define MOSS_TAB_ACC_GAMMA1 6    /* u64[n]  inclusive prefix of Gamma^(1)_v (Section 5.1.1) */
#define MOSS_TAB_ACC_GAMMA2 7    /* u64[n]  inclusive prefix of Gamma^(2)_v (Section 5.1.2) */
#define MOSS_TAB_ACC_SIGMA 8     /* u32[nnz] row-local inclusive prefix of d_x - 1 (ACC_sigma,
                                    Section 4.1.3 = ACC_mu, Section 5.1.5) */
#define MOSS_TAB_ACC_TAU 9       /* u64[nnz] row-local inclusive prefix of the tau weights
                                    (d_u - 1)(S_v - (d_u - 1)) (Section 5.1.2, step 2) */
/* MOSS-4Min (Section 4.2.1) with the order of Section 3.2: a above b when d_a > d_b, or
   d_a = d_b and a > b; N_{v,x} = {y in N_v : y above x}, d_{v,x} = |N_{v,x}| (Table 1) */
#define MOSS_TAB_ACC_GAMMA_MIN 11 /* u64[n]   inclusive prefix of check-Gamma_v =
                                     sum_{x in N_v} d_{v,x} d_{x,v} */
#define MOSS_TAB_ACC_CHECK 12    /* u64[nnz] row-local inclusive prefix of d_{v,x} d_{x,v} */
#define MOSS_TAB_RANK 13         /* u32 pairs, count nnz: per entry (v, x) d_{v,x}, d_{x,v} */
#define MOSS_TAB_COL_RANK 15     /* i32[nnz] each row N_v in descending order */
/* Row guides (an implementation aid, not from the paper): the search windows of the
   weighted picks inside a row.  Rows with d_v >= 64, in node order, each hold 2^g + 1
   u32 entries, g = floor(log2 d_v) - 1; with A the row's prefix, T its last value and
   s = max(0, bitlength(T) - g), entry b is the first i with A[i] > b * 2^s, or d_v - 1
   when there is none.  count = the sum of those lengths over the rows. */
#define MOSS_TAB_SIGMA_GUIDE 16  /* over ACC_sigma (built with K4 or K5) */
#define MOSS_TAB_TAU_GUIDE 17    /* over ACC_tau (K5) */
#define MOSS_TAB_CHECK_GUIDE 18  /* over ACC_check (K4MIN) */

typedef struct moss_graph moss_graph;

typedef struct {
  int32_t n;               /* nodes */
  int32_t max_degree;
  int64_t nnz;             /* CSR entries = 2 |E| */
  uint32_t built_mask;     /* MOSS_TABLES_* bits built so far */
  uint32_t reserved;
  uint64_t gamma;          /* Gamma      (Table 1), valid once K4 tables are built */
  uint64_t gamma1;         /* Gamma^(1)  (Table 1), valid once K5 tables are built */
  uint64_t gamma2;         /* Gamma^(2)  (Table 1) */
  uint64_t lambda3;        /* Lambda_3 = sum_v C(d_v, 3) (Table 1) */
  uint64_t lambda4;        /* Lambda_4 = sum_v C(d_v, 4) (Table 1) */
  uint64_t device_bytes;   /* device memory held by the graph's sampling tables (and CSR
                              copy); the per-graph block made at creation (edge hash
                              set and filter, work items, node records) is not counted */
  uint64_t gamma_min;      /* check-Gamma (Table 1), valid once K4MIN tables are built */
  uint64_t sampling_bytes; /* device bytes the samplers read from: the built tables, the
                              CSR (owned or borrowed) and the edge hash set and filter */
} moss_graph_info;

typedef struct {
  int32_t k;               /* 4 or 5 */
  int32_t n_motifs;        /* 6 or 21 */
  uint32_t flags;          /* estimate flags used */
  int32_t reserved;
  uint64_t n_samples;      /* requested budget */
  uint64_t K[2];           /* k=4: K[0] = n_samples, K[1] = 0; k=5: K[0] = K_1 = ceil(n/2)
                              T-5 samples, K[1] = K_2 = floor(n/2) Path-5 samples (Section
                              5.1.4 sets K_1 = K_2); k=4 with MOSS_K4_MIN: K[0] = ceil(n/2)
                              MOSS-4 and K[1] = floor(n/2) MOSS-4Min samples */
  uint64_t hits[2][22];    /* per sampler: [0] rejected samples, [i] samples of class i
                              (m_i, Sections 4.1.2 and 5.1.1-5.1.2); the class counts sum
                              to K[s], or are all zero when the sampler's Gamma is 0.
                              MOSS-4Min also counts its diamonds (class 5) by the number c
                              of ordered draws that reach them: [7] c = 2, [8] c = 4,
                              [9] c = 6 (not part of that sum) */
  uint64_t gamma[2];       /* k=4: Gamma (and check-Gamma with MOSS_K4_MIN);
                              k=5: Gamma^(1), Gamma^(2) */
  uint64_t lambda;         /* k=4: Lambda_3; k=5: Lambda_4 */
  double estimate[21];     /* estimate[i-1] of n_i (k=4, i <= 6) or eta_i (k=5) */
  double variance[21];     /* Theorem 3 / Theorem 10 evaluated at the estimates */
  double device_ms;        /* device time of the sampling kernels (HIP events) */
} moss_result;

/* ---- errors ---------------------------------------------------------------------- */
const char *moss_status_string(moss_status s);

/* ---- graphs (Section 2: an undirected simple graph; Section 4.1.3: degrees and sorted
 * neighbour lists N_v[1..d_v]) ------------------------------------------------------
 * The graph is given as symmetric CSR: row v = col[row_ptr[v] .. row_ptr[v+1]) lists N_v
 * in strictly ascending order; every edge appears in both rows; no self-loops.
 * n >= 0, 0 <= nnz < 2^31.  The CSR is validated on the device (unless MOSS_TRUST_CSR)
 * and the first defect found is reported as MOSS_E_ARG / _UNSORTED / _SELF_LOOP /
 * _DUPLICATE / _ASYMMETRIC. */

/* Creation also builds the graph's edge hash set and edge filter (the induced-edge
   probes of every sampler read them; the symmetry check uses the hash set) and the
   work items and node records of the O(|E|) kernels.

   Copies host arrays row_ptr[n+1] and col[nnz] to the device.  The caller keeps
   ownership of its arrays, which may be freed when the call returns. */
moss_status moss_graph_create(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col,
                              uint32_t flags, void *hip_stream, moss_graph **out);

/* Borrows device arrays d_row_ptr[n+1], d_col[nnz] (e.g. torch tensors); they must stay
   alive and unchanged until moss_graph_destroy. */
moss_status moss_graph_create_device(int32_t n, int64_t nnz, const int32_t *d_row_ptr,
                                     const int32_t *d_col, uint32_t flags, void *hip_stream,
                                     moss_graph **out);

/* Waits for the graph's work, then releases all its device memory (the library keeps
   released blocks, up to 1 GiB per device, for later graphs of the same size). */
moss_status moss_graph_destroy(moss_graph *g);

/* Initialization of Section 4.1.3 on the device, O(|E|): degrees, the node weights
   Gamma_v (Section 4.1.1), Gamma^(1)_v (Section 5.1.1), Gamma^(2)_v (Section 5.1.2),
   their inclusive prefixes ACC_* over the nodes, the row prefixes ACC_sigma (= ACC_mu) and
   ACC_tau, Lambda_3 and Lambda_4 (Table 1), and guide tables for the node draws.
   k_mask: MOSS_TABLES_K4 and/or MOSS_TABLES_K5.  Tables already built are kept.
   MOSS_E_OVERFLOW if a quantity does not fit (graph left usable for the other k). */
moss_status moss_build_tables(moss_graph *g, uint32_t k_mask);

moss_status moss_graph_get_info(const moss_graph *g, moss_graph_info *info);

/* Copies one table (MOSS_TAB_*) to host memory; count must equal its element count
   (n or nnz).  MOSS_E_NOT_BUILT if the table was not built. */
moss_status moss_table_read(const moss_graph *g, int32_t which, void *host_out, int64_t count);

/* ---- estimation ------------------------------------------------------------------------
 * k = 4: MOSS-4 (Algorithm 1) with K = n_samples >= 1 samples; estimates n_1..n_6 with
 *        n_i = m_i / (K p_i), p_i = 2 phi^(1)_i / Gamma (Theorem 2) for i in {1,3,4,5,6},
 *        n_2 = Lambda_3 - n_4 - 2 n_5 - 4 n_6 (Section 4.1.2) and Theorem 3's variances.
 *        With MOSS_K4_MIN (n_samples >= 2), MOSS-4 on ceil(n/2) and MOSS-4Min (Algorithm 2)
 *        on floor(n/2) samples; n_3, n_5, n_6 mix both (Theorem 1).  MOSS-4Min reaches a
 *        4-cycle by 2 and a 4-clique by 6 ordered draws (Theorem 4), but a diamond by 2,
 *        4 or 6 depending on its nodes' order, so each MOSS-4Min sample is weighted by
 *        its own reach count c: n_i = (check-Gamma / K') sum_c m_{i,c} / c, with the
 *        matching variance (Theorem 5 when c is fixed).  Mix weights: pooled (default)
 *        K p_i / (K p_i + K' q_i), q = 2, 2, 6 / check-Gamma for i = 3, 5, 6; or the
 *        paper's inverse-variance weights (MOSS_MIX_PAPER).
 * k = 5: T-5 (Algorithm 3) with K_1 = ceil(n/2) and Path-5 (Algorithm 4) with
 *        K_2 = floor(n/2) samples (n_samples >= 2), mixed per Section 5.1.3 (flags),
 *        eta_2 = Lambda_4 - sum_{Omega_3*} phi^(3)_i eta_i and Theorem 10's variances.
 * Builds the needed tables first if they are missing.  Synchronous: returns when the
 * result is on the host.  A sampler whose Gamma is 0 draws nothing (its hits are all 0);
 * then the motifs only it can see are estimated as 0, exactly. */
moss_status moss_estimate(moss_graph *g, int32_t k, uint64_t n_samples, uint64_t seed,
                          uint32_t flags, moss_result *out);

/* Raw hit counts of one sampler (MOSS_SAMPLER_*) over sample indices [k0, k1), accumulated
   into hits[22] (host; [0] rejected, [i] class i, MOSS-4Min's diamonds also by reach
   count in [7..9]; overwritten).  If d_class_out is not
   NULL it receives one byte per sample, d_class_out[k - k0] = class of sample k (0 =
   rejected); it must hold k1 - k0 bytes on the device.  Splitting [k0, k1) into pieces
   gives exactly the same total. */
moss_status moss_sample_range(moss_graph *g, int32_t sampler, uint64_t seed, uint64_t k0,
                              uint64_t k1, uint8_t *d_class_out, uint64_t hits[22]);

/* ---- calls that allocate nothing -------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture or in a
 * tight serving loop, and harnesses that forbid hipMalloc.
 *
 * moss_sample_range_noalloc: moss_sample_range (same arguments, same hits and classes,
 * same kernels) with no allocation of any kind.
 *  - The sampler's tables must already be built (moss_build_tables): MOSS_E_NOT_BUILT
 *    otherwise.  Hits go through the graph's own buffers, made at its creation.
 *  - k1 - k0 <= MOSS_NOALLOC_MAX_SAMPLES (2^22), else MOSS_E_TOO_LARGE.  Larger ranges
 *    go as several calls; their hits add up to those of the whole range.
 *  - When the samples run XCD-grouped (moss_tuning.schedule), their sorting scratch
 *    (each sample's group and sorted place, per-block group counts, window cursors) is a
 *    fixed device array of MOSS_NOALLOC_SCRATCH_BYTES (32 MiB) inside the library.  Each
 *    device holds its own copy from the library's load until the process ends, and the
 *    array keeps the last call's contents, which no call reads before writing.  Calls on
 *    one device share that array: the library lets one of them use it at a time (a call
 *    waits while another, on any graph of the device, runs), so calls that would overlap
 *    on one device run one after the other.
 *  - Synchronous: returns when the hits are on the host. */
#define MOSS_NOALLOC_MAX_SAMPLES (1ull << 22)
#define MOSS_NOALLOC_SCRATCH_BYTES (32ull << 20)
moss_status moss_sample_range_noalloc(moss_graph *g, int32_t sampler, uint64_t seed, uint64_t k0, uint64_t k1,
                                      uint8_t *d_class_out, uint64_t hits[22]);

/* Node tuples of chosen samples: for each of the count sample indices d_index[i] (device
   u64), d_nodes_out[5 i .. 5 i + 4] (device i32) receives v, u, w, r, t (t = -1 for
   MOSS-4) and d_class_out[i] (device u8, may be NULL) the class (0 = rejected). */
moss_status moss_sample_nodes(moss_graph *g, int32_t sampler, uint64_t seed, const uint64_t *d_index,
                              int64_t count, int32_t *d_nodes_out, uint8_t *d_class_out);

/* The classification table a sampler's kernel uses (host only, no device needed): entry m
   is the motif id of a sample whose probed pairs are the set bits of m.  MOSS-4 and
   MOSS-4Min (len 8): bit 0 = u~w, 1 = v~r, 2 = w~r.  T-5 (len 64): u~w, u~r, w~r, v~t, w~t, r~t.  Path-5
   (len 64): v~r, v~t, u~w, u~t, w~r, r~t.  Ids follow the paper's motif numbering, which
   its printed constants fix (Section 4.1.2 for 4 nodes, Table 2 for 5 nodes). */
moss_status moss_class_lut(int32_t sampler, uint8_t *out, int32_t len);

/* Host-only finals: fills out->estimate / variance from out->k, K, hits, gamma, lambda and
   flags (Theorems 2, 3, 6-10).  Used by the estimate calls; exposed for re-scaling. */
moss_status moss_finals(moss_result *out);

/* ---- sampling budget and concentrations ------------------------------------------------
 * The budget that keeps each motif's relative error below eps with probability about
 * 1 - delta (the closing remark of Section 4.1.2, with Theorem 1's normal limit).  Every
 * variance of Theorems 3, 5 and 10 scales as 1/K, so from a pilot result
 *   K_i = max(1, ceil(z^2 variance[i] K_p / (eps estimate[i])^2)),  K_p = K[0] + K[1],
 * with z the two-sided normal quantile: erfc(z / sqrt 2) = delta, found by 200 halvings
 * of [0, 40] (the midpoint of the last interval).  budget[i] = K_i for the motifs with a
 * positive estimate, 0 for the others; *max_budget = the largest K_i over motif_mask
 * (bit i - 1 = motif i; 0 = every motif), 0 if none.  Needs eps > 0 and 0 < delta < 1.
 * Host only. */
moss_status moss_plan_budget(const moss_result *pilot, double eps, double delta, uint32_t motif_mask,
                             uint64_t budget[21], uint64_t *max_budget);

/* A pilot estimate (pilot_samples, pilot_seed), the planned budget (the pilot's size when
   no motif of the mask can be planned) clamped to [the least valid budget, max_samples],
   then the estimate with that budget and `seed` into *out (out->n_samples is the budget
   used).  Both runs are moss_estimate calls with `flags`. */
moss_status moss_estimate_to_precision(moss_graph *g, int32_t k, double eps, double delta, uint32_t motif_mask,
                                       uint64_t pilot_samples, uint64_t pilot_seed, uint64_t max_samples,
                                       uint64_t seed, uint32_t flags, moss_result *out);

/* Motif concentrations omega_i = estimate_i / sum_j estimate_j (Section 6.2) into
   omega[0 .. n_motifs - 1] (the rest 0); all 0 when the sum is 0.  Host only. */
moss_status moss_concentrations(const moss_result *r, double omega[21]);

/* ---- batching: many requests in one persistent launch --------------------------------
 * One persistent kernel (replayed from a captured hipGraph) takes the requests' sample
 * ranges as a list of items in graph-major order, cuts them into tiles of consecutive
 * sample indices as its workgroups ask for work, draws each tile's samples in the order
 * of their first random word, and keeps per-request hit counts; items with many samples
 * on graphs with large tables run instead as XCD-grouped launches of their own after it
 * (moss_tuning's grouping thresholds).  out[i] equals moss_estimate(reqs[i]...) exactly.
 * Requests may name different graphs (all on the current device). */
typedef struct {
  moss_graph *g;
  int32_t k;               /* 4 or 5 */
  uint32_t flags;          /* MOSS_MIX_*, MOSS_K4_MIN */
  uint64_t n_samples;
  uint64_t seed;
} moss_request;

moss_status moss_estimate_batch(const moss_request *reqs, int32_t n, moss_result *out, void *hip_stream);

/* Launch shape knobs (0 = automatic).  tile_samples: samples per tile in the batched
   kernel (a tile's samples are shared by the block's waves: tile_samples / (threads
   per block / 64) per wavefront); blocks_per_cu: resident workgroups per compute unit for
   the sampling kernels; schedule: how a plain estimate spreads its samples
   (MOSS_SCHEDULE_*); group_min_samples_log2 / group_min_footprint_mb: a batched or
   served item runs as an XCD-grouped launch of its own (instead of in the persistent
   kernel) when it has at least 2^group_min_samples_log2 samples (default 2^20) on a
   graph whose sampled bytes reach group_min_footprint_mb MB (default 32).  No knob
   changes any result. */
enum {
  MOSS_SCHEDULE_AUTO = 0,   /* by the graph's footprint */
  MOSS_SCHEDULE_PLAIN = 1,  /* grid-stride over the sample indices */
  MOSS_SCHEDULE_XCD = 2     /* samples grouped by the top bits of their first random word,
                               one group per XCD (see moss_estimate) */
};

typedef struct {
  uint32_t tile_samples;
  uint32_t blocks_per_cu;
  uint32_t threads_per_block;
  uint32_t schedule;
  uint32_t group_min_samples_log2;  /* <= 40 */
  uint32_t group_min_footprint_mb;  /* <= 2^20 */
  uint32_t sort_window;             /* samples a block of the sorted sampling kernel takes at
                                       a time (a multiple of 64, <= 512; 0 = 256 on graphs
                                       past 256 MB of sampled bytes, else 512) */
} moss_tuning;

moss_status moss_set_tuning(const moss_tuning *t);
moss_status moss_get_tuning(moss_tuning *t);

/* Autotuner: times moss_estimate_batch over the given requests (host tile list and
   staging included; best of two calls) first for each tile size {2048, 4096, 16384,
   65536} and occupancy {2, 3, 4, 5, 6, 8} blocks per CU, then, with the best of those,
   for each grouping threshold (items of at least 2^{17..22} samples on graphs of at
   least {4, 8, 16, 32, 64} MB of sampled bytes), then for each sorted window {128, 256,
   512} of the grouped launches; results are identical for every candidate (checked).  Keeps the fastest as the process-wide tuning (the schedule knob
   is left as it was); best_ms receives its wall time. */
moss_status moss_autotune(const moss_request *reqs, int32_t n, moss_tuning *best, double *best_ms);

/* ---- serving: continuous batching over resident graphs --------------------------------
 * A server owns a worker thread that repeatedly gathers the next chunk of samples of
 * every admitted request into one tile list and runs it with the batched kernel, so
 * requests that arrive while others run join at the next iteration.  A request is
 * admitted when a slot is free and its graph's tables fit the memory budget (tables of
 * idle graphs are evicted, the largest first, least recently used among equal sizes);
 * small requests (express_samples) take an express path beside the iterations.
 * Missing tables of a graph with no running request are built by a second server
 * thread while launches go on; the request joins the iteration after they are in. */
typedef struct moss_server moss_server;

typedef struct {
  uint64_t mem_budget_bytes;   /* device bytes for sampling tables (0 = unlimited) */
  uint32_t max_slots;          /* requests in the iterations at once, and in one express
                                  launch (0 = 256) */
  uint32_t express_off;        /* non-zero: every request goes through the iterations */
  uint64_t chunk_samples;      /* at most this many samples per request per iteration (0 = 2^25) */
  uint64_t iteration_samples;  /* samples per iteration in all (0 = 2^25): the requests with
                                  the fewest samples left go first, each still gets at least
                                  iteration_samples / 16 (within chunk_samples), so short
                                  requests finish in the next launch and long ones take the
                                  rest; no setting changes any result */
  uint64_t express_samples;    /* requests of at most this many samples (0 = 2^22) are
                                  launched whole by an express thread with a runner of its
                                  own as soon as their tables are in, beside the iteration
                                  under way, instead of waiting for it to end */
} moss_server_config;

typedef struct {
  uint64_t completed;
  uint64_t samples;            /* samples drawn by completed requests */
  uint64_t iterations;         /* scheduler iterations (batched launches) */
  uint64_t queued;             /* requests waiting for admission now */
  uint64_t active;             /* requests admitted and running now (express path included) */
  double p50_ms, p99_ms;       /* submit-to-result latency over completed requests */
  double samples_per_s;        /* samples of completed requests / wall time since first submit */
  uint64_t table_bytes;        /* device bytes of resident tables now */
  uint64_t evictions;
  uint64_t express_launches;   /* launches of the express thread */
} moss_server_stats;

moss_status moss_server_create(const moss_server_config *cfg, void *hip_stream, moss_server **out);
/* Registers a graph (the server does not own it; keep it alive until destroy). */
moss_status moss_server_add_graph(moss_server *s, moss_graph *g, int32_t *graph_id);
moss_status moss_server_submit(moss_server *s, int32_t graph_id, int32_t k, uint64_t n_samples,
                               uint64_t seed, uint32_t flags, uint64_t *ticket);
/* Waits up to timeout_ms (< 0: forever) for a ticket's result; MOSS_E_TIMEOUT if not done. */
moss_status moss_server_wait(moss_server *s, uint64_t ticket, int64_t timeout_ms, moss_result *out);
moss_status moss_server_cancel(moss_server *s, uint64_t ticket);
moss_status moss_server_stats_get(moss_server *s, moss_server_stats *out);
/* Stops the worker (pending requests end with MOSS_E_CANCELLED) and frees the server. */
moss_status moss_server_destroy(moss_server *s);

#ifdef __cplusplus
}
#endif
#endif /* MOSS_H */
