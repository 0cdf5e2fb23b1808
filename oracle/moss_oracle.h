/* Moss oracle: plain, slow, single-purpose CPU reference of the Moss estimators
 * (Wang, Tao, Zhao, Guan: "Moss: A Scalable Tool for Efficiently Sampling and
 * Counting 4- and 5-Node Graphlets", arXiv 1509.08089).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no source,
 * header, table or generator with the GPU library.
 *
 * Every function cites the passage of the paper it follows.  Where the paper
 * leaves a choice open (the random number generator, how a random number is
 * mapped to an outcome, how an excluded element is skipped), the oracle follows
 * one fixed sampling contract:
 *   words    B(k, j) = Philox4x64-10(counter = (k, j, 0, 0), key = (seed, tag)),
 *            tag 0x4 for MOSS-4, 0x41 for MOSS-4Min, 0x51 for T-5, 0x52 for Path-5,
 *            k the sample index
 *   bounded  U(x, N) = floor(x * N / 2^64)
 *   pick     pick(A, x) = min{ i : A[i] > U(x, A[L-1]) } over an inclusive prefix A
 *   skips    an index draw that must avoid positions a < b is shifted past them in
 *            ascending order; "a neighbour of u other than v" reads the sorted row
 *            and steps over v.
 */
#ifndef MOSS_ORACLE_H
#define MOSS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0, ORC_E_ARG = -1, ORC_E_UNSORTED = -2, ORC_E_SELF_LOOP = -3,
  ORC_E_DUPLICATE = -4, ORC_E_ASYMMETRIC = -5, ORC_E_OVERFLOW = -6, ORC_E_NOMEM = -7
};

/* sampler ids */
enum { ORC_MOSS4 = 4, ORC_MOSS4MIN = 0x41, ORC_T5 = 0x51, ORC_PATH5 = 0x52 };

/* mix modes for 5-node finals */
enum { ORC_MIX_POOLED = 0, ORC_MIX_PAPER = 1 };

typedef struct orc_graph orc_graph;

/* tables that can be copied out (orc_table) */
enum {
  ORC_TAB_S = 0,        /* u64[n]  sum_{x in N_v} (d_x - 1)                      */
  ORC_TAB_Q = 1,        /* u64[n]  sum_{x in N_v} (d_x - 1)^2                    */
  ORC_TAB_GAMMA = 2,    /* u64[n]  Gamma_v                                       */
  ORC_TAB_GAMMA1 = 3,   /* u64[n]  Gamma^(1)_v                                   */
  ORC_TAB_GAMMA2 = 4,   /* u64[n]  Gamma^(2)_v                                   */
  ORC_TAB_ACC_GAMMA = 5,  /* u64[n] inclusive prefix of Gamma_v                   */
  ORC_TAB_ACC_GAMMA1 = 6, /* u64[n]                                               */
  ORC_TAB_ACC_GAMMA2 = 7, /* u64[n]                                               */
  ORC_TAB_ACC_SIGMA = 8,  /* u32[nnz] row-local inclusive prefix of (d_x - 1)     */
  ORC_TAB_ACC_TAU = 9,    /* u64[nnz] row-local inclusive prefix of the tau weights */
  /* MOSS-4Min (Section 4.2.1), with the order a > b when d_a > d_b, or d_a = d_b and a > b */
  ORC_TAB_GAMMA_MIN = 10,     /* u64[n]   check-Gamma_v = sum_{x in N_v} d_{v,x} d_{x,v}    */
  ORC_TAB_ACC_GAMMA_MIN = 11, /* u64[n]   inclusive prefix of check-Gamma_v                  */
  ORC_TAB_ACC_CHECK = 12,     /* u64[nnz] row-local inclusive prefix of d_{v,x} d_{x,v}      */
  ORC_TAB_RANK = 13,          /* u32[nnz] d_{v,x} for the entry (v, x)                       */
  ORC_TAB_RANK_MIRROR = 14,   /* u32[nnz] d_{x,v} for the entry (v, x)                       */
  ORC_TAB_COL_RANK = 15       /* i32[nnz] each row N_v in descending order                   */
};

typedef struct {
  uint64_t gamma, gamma1, gamma2, lambda3, lambda4;
  uint64_t gamma_min;        /* check-Gamma (Table 1), valid when min_status == ORC_OK */
  int32_t min_status;        /* ORC_OK, or ORC_E_OVERFLOW when a MOSS-4Min prefix needs > 64 bits */
  int32_t pad;
} orc_totals;

typedef struct {
  int32_t k;                 /* 4 or 5 */
  int32_t n_motifs;          /* 6 or 21 */
  uint64_t K[2];             /* k=4: K[0]; k=5: K1 (T-5), K2 (Path-5) */
  uint64_t hits[2][22];      /* [sampler][0] rejected, [sampler][i] class i */
  double estimate[21];       /* estimate[i-1] for motif i */
  double variance[21];
} orc_result;

int orc_build(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col,
              int validate, orc_graph **out);
void orc_free(orc_graph *g);
int orc_totals_get(const orc_graph *g, orc_totals *t);
int orc_table(const orc_graph *g, int which, void *out);

/* primitives, exposed for the contract's own checks */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
uint64_t orc_bounded(uint64_t x, uint64_t n);
int64_t orc_pick_u64(const uint64_t *acc, int64_t len, uint64_t x);
int orc_classify(int k, const uint8_t *adj /* k*k row-major 0/1 */);

/* one sample by index; nodes[] gets v,u,w,r(,t); returns class (0 = rejected),
   or a negative status.  MOSS-4Min hits: [0] rejected, [1..6] per class, and the
   diamonds (class 5) once more by the number of ways c(s) in {2, 4, 6} that the
   sampler can reach them: [7] c = 2, [8] c = 4, [9] c = 6. */
int orc_sample(const orc_graph *g, int sampler, uint64_t seed, uint64_t k, int32_t nodes[5]);

/* hits over sample indices [k0, k1) of one sampler, split over nthreads threads */
int orc_run(const orc_graph *g, int sampler, uint64_t seed, uint64_t k0, uint64_t k1,
            int nthreads, uint64_t hits[22]);

/* estimator finals from hits (Thm 3 and Thm 10 with the readings above) */
int orc_finals4(uint64_t K, const uint64_t hits[7], uint64_t gamma, uint64_t lambda3,
                double est[6], double var[6]);
int orc_finals5(uint64_t K1, uint64_t K2, const uint64_t hits1[22], const uint64_t hits2[22],
                uint64_t gamma1, uint64_t gamma2, uint64_t lambda4, int mix,
                double est[21], double var[21], double *cov /* 21*21 or NULL */);

/* MOSS-4 with K samples and MOSS-4Min with Kc samples, mixed for n_3, n_5, n_6
   (Section 4.2 with Theorem 1).  MOSS-4Min's estimate weights each sample by the
   inverse of its own CIS's probability c(s) / check-Gamma (c(s) the number of
   ordered draws that reach s; Theorem 4's constants hold for c = 2 of the 4-cycle and
   c = 6 of the 4-clique, but a diamond has c in {2, 4, 6}).  K = 0 or Kc = 0 leaves
   that sampler out (not both). */
int orc_finals4min(uint64_t K, const uint64_t hits[7], uint64_t gamma, uint64_t lambda3, uint64_t Kc,
                   const uint64_t hits_min[10], uint64_t gamma_min, int mix, double est[6], double var[6]);

/* Number of ordered node tuples (w, v, u, r) of the 4-node set whose pairwise
   adjacency is adj (4x4, 0/1) and whose order keys are key[] (a > b iff key[a] >
   key[b]) with edges w-v, v-u, u-r, w > u and r > v: the draws of MOSS-4Min that
   give this set. */
int orc_ways_of(const uint8_t adj[16], const uint64_t key[4]);

/* the whole estimate: k=4 -> MOSS-4 with K samples; k=5 -> T-5 with ceil(K/2) and
   Path-5 with floor(K/2) samples, then the mix */
int orc_estimate(const orc_graph *g, int k, uint64_t n_samples, uint64_t seed, int mix,
                 int nthreads, orc_result *res);
/* k = 4 with MOSS-4 on ceil(n/2) and MOSS-4Min on floor(n/2) samples (n >= 2), mixed */
int orc_estimate4min(const orc_graph *g, uint64_t n_samples, uint64_t seed, int mix, int nthreads,
                     orc_result *res);

/* Sampling budget (the closing remark of Section 4.1.2 with Theorem 1's normal limit).
   z: the two-sided normal quantile, erfc(z / sqrt 2) = delta, found by 200 halvings of
   [0, 40] (the midpoint of the last interval).  Every variance of Theorems 3, 5 and 10
   scales as 1/K, so the budget that makes z sqrt(Var_i) <= eps est_i is
     K_i = max(1, ceil(z^2 var_i K_p / (eps est_i)^2)),   K_p = K[0] + K[1] of the pilot,
   for each motif with a positive pilot estimate (0 for the others); *max_budget is the
   largest K_i over the motifs in motif_mask (bit i-1 = motif i; 0 = every motif). */
double orc_normal_two_sided(double delta);
int orc_plan_budget(const orc_result *pilot, double eps, double delta, uint32_t motif_mask, uint64_t budget[21],
                    uint64_t *max_budget);

/* Concentrations omega_i = est_i / sum_j est_j (Section 6.2), 0 when the sum is 0. */
int orc_concentrations(const orc_result *r, double omega[21]);

/* A pilot estimate (pilot_samples, pilot_seed), the planned budget clamped to
   [smallest valid, max_samples] (the pilot's size when no motif can be planned), then
   the estimate with that budget and `seed`.  with_min: k = 4 with MOSS-4Min. */
int orc_estimate_to_precision(const orc_graph *g, int k, int with_min, double eps, double delta, uint32_t motif_mask,
                              uint64_t pilot_samples, uint64_t pilot_seed, uint64_t max_samples, uint64_t seed,
                              int mix, int nthreads, orc_result *res, uint64_t *final_samples);

/* exact counts of k-node connected induced subgraphs per class (ESU enumeration) */
int orc_count_cis(const orc_graph *g, int k, int nthreads, uint64_t counts[22]);

/* exact counts n_1..n_6 (counts[1..6]) from non-induced pattern counts: 3-paths, 3-stars,
   4-cycles, triangles with a pendant, diamonds and 4-cliques, converted with the matrix of
   how many copies of each pattern every motif contains.  Same result as orc_count_cis(4)
   but feasible on graphs with millions of edges. */
int orc_count4_exact(const orc_graph *g, uint64_t counts[7]);

/* mean number of distinct 64-byte lines one sample reads when every search is a
   plain binary search and nothing is reused between samples; arrays are taken to
   start on 64-byte boundaries with the widths of the sampling tables */
int orc_line_count(const orc_graph *g, int sampler, uint64_t seed, uint64_t k0, uint64_t k1,
                   double *mean_lines);

#ifdef __cplusplus
}
#endif
#endif
