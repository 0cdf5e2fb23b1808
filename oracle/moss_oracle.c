/* Moss oracle: plain, slow CPU reference (test infrastructure only).
 *
 * Paper: Wang, Tao, Zhao, Guan, "Moss: A Scalable Tool for Efficiently Sampling
 * and Counting 4- and 5-Node Graphlets", arXiv 1509.08089.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg load
 * this file's library; the GPU library neither includes nor links it and it
 * includes nothing of the GPU library.  Counts are exact integers; floating
 * point appears only in the estimator finals, in double precision.
 *
 * Pinning: the functions here are checked against (a) numpy's Philox, (b) the
 * motif constants of Table 2 and of Section 4.1.2 through an independent
 * isomorphism enumeration, (c) brute-force enumeration of all k-subsets on tiny
 * graphs, (d) exact rational enumeration of every sampler outcome (Theorems 2,
 * 6, 8 and the variance theorems), (e) closed forms on paths, cycles, stars,
 * complete and complete bipartite graphs, and (f) per-run invariants.
 */
#include "moss_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

struct orc_graph {
  int32_t n;
  int64_t nnz;
  int32_t *rp;           /* row_ptr[n+1] (own copy) */
  int32_t *col;          /* col[nnz] (own copy) */
  uint64_t *S, *Q, *gam, *gam1, *gam2;
  uint64_t *acc_gam, *acc_gam1, *acc_gam2;
  uint32_t *acc_sigma;
  uint64_t *acc_tau;
  /* MOSS-4Min (Section 4.2.1) */
  uint32_t *rank, *rank_mirror;  /* per entry (v, x): d_{v,x} and d_{x,v} */
  int32_t *col_rank;             /* rows in descending order */
  uint64_t *acc_check;           /* per entry: row prefix of d_{v,x} d_{x,v} */
  uint64_t *gmin, *acc_gmin;     /* check-Gamma_v and its prefix */
  orc_totals tot;
};

/* ------------------------------------------------------------------------ */
/* Random words.  The paper only asks for "a number selected at random"       */
/* (Section 4.1.3, steps 1 of WeightRandomVertex and RandomVertex).  The      */
/* oracle uses the counter-based generator Philox4x64 with 10 rounds from      */
/* Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2,   */
/* 3" (SC 2011): each round multiplies words 0 and 2 by fixed odd constants,   */
/* and the new words are (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^ k1, */
/* lo(M0*x0)); the key is bumped by two Weyl constants between rounds.         */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL
#define PHILOX_W1 0xBB67AE8584CAA73BULL

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    u128 p0 = (u128)PHILOX_M0 * x0;
    u128 p1 = (u128)PHILOX_M1 * x2;
    uint64_t y0 = (uint64_t)(p1 >> 64) ^ x1 ^ k0;
    uint64_t y1 = (uint64_t)p1;
    uint64_t y2 = (uint64_t)(p0 >> 64) ^ x3 ^ k1;
    uint64_t y3 = (uint64_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void words(uint64_t seed, uint64_t tag, uint64_t k, uint64_t block, uint64_t w[4]) {
  uint64_t ctr[4] = {k, block, 0, 0};
  uint64_t key[2] = {seed, tag};
  orc_philox4x64_10(ctr, key, w);
}

/* "Select rnd from {1, ..., N} at random": the word x in [0, 2^64) is mapped to
   floor(x * N / 2^64), a monotone map whose preimages differ in size by at most 1. */
uint64_t orc_bounded(uint64_t x, uint64_t n) { return (uint64_t)(((u128)x * n) >> 64); }

/* WeightRandomVertex (Section 4.1.3): with rnd = r + 1 drawn uniformly from
   {1..ACC[L]}, return the i with ACC[i-1] < rnd <= ACC[i]; in 0-based terms the
   smallest i with acc[i] > r.  Binary search, as the paper says. */
static int64_t pick_search_u64(const uint64_t *acc, int64_t len, uint64_t r) {
  int64_t lo = 0, hi = len - 1; /* answer in [lo, hi] since acc[len-1] > r */
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (acc[mid] > r) hi = mid; else lo = mid + 1;
  }
  return lo;
}

int64_t orc_pick_u64(const uint64_t *acc, int64_t len, uint64_t x) {
  if (len <= 0 || acc[len - 1] == 0) return -1;
  return pick_search_u64(acc, len, orc_bounded(x, acc[len - 1]));
}

/* ------------------------------------------------------------------------ */
/* Motif classes.  The drawings of the motifs are not available, so a class   */
/* id is identified by the constants the paper prints for it: for 4 nodes the */
/* number of spanning subgraphs isomorphic to the 3-path M1 (phi^(1), Section */
/* 4.1.2) and to the 3-star M2 (phi^(2), Section 4.1.2, the estimate of n_2); */
/* for 5 nodes the numbers of spanning subgraphs isomorphic to M3 (the fork), */
/* M1 (the 4-path) and M2 (the 4-star), phi^(1..3) of Table 2.  Each class    */
/* has a distinct tuple.  The classifier counts those spanning trees of the   */
/* sample by trying every (k-1)-edge subset and looks the tuple up.           */
/* ------------------------------------------------------------------------ */
static const int PHI4_PATH[7] = {0, 1, 0, 4, 2, 6, 12};  /* phi^(1)_i, Sec 4.1.2 */
static const int PHI4_STAR[7] = {0, 0, 1, 0, 1, 2, 4};   /* phi^(2)_i, Sec 4.1.2 */
static const int PHI5_FORK[22] = {0, 0, 0, 1, 1, 2, 0, 2, 2, 4, 4, 5, 4, 6, 10, 9, 12, 10, 20, 20, 36, 60};
static const int PHI5_PATH[22] = {0, 1, 0, 0, 2, 2, 5, 1, 0, 4, 7, 2, 4, 6, 10, 6, 6, 14, 24, 18, 36, 60};
static const int PHI5_STAR[22] = {0, 0, 1, 0, 0, 0, 0, 0, 1, 0, 0, 1, 1, 0, 1, 1, 2, 0, 1, 2, 3, 5};

int orc_classify(int k, const uint8_t *adj) {
  if (k != 4 && k != 5) return -1;
  int ea[10], eb[10], ne = 0;
  for (int i = 0; i < k; ++i)
    for (int j = i + 1; j < k; ++j)
      if (adj[i * k + j]) { ea[ne] = i; eb[ne] = j; ++ne; }
  int trees_by_maxdeg[5] = {0, 0, 0, 0, 0};
  for (int mask = 0; mask < (1 << ne); ++mask) {
    if (__builtin_popcount(mask) != k - 1) continue;
    int parent[5], deg[5];
    for (int i = 0; i < k; ++i) { parent[i] = i; deg[i] = 0; }
    int comps = k;
    for (int e = 0; e < ne; ++e) {
      if (!(mask >> e & 1)) continue;
      int a = ea[e], b = eb[e];
      ++deg[a]; ++deg[b];
      while (parent[a] != a) a = parent[a];
      while (parent[b] != b) b = parent[b];
      if (a != b) { parent[a] = b; --comps; }
    }
    if (comps != 1) continue; /* k-1 edges, connected: a spanning tree */
    int maxdeg = 0;
    for (int i = 0; i < k; ++i) if (deg[i] > maxdeg) maxdeg = deg[i];
    ++trees_by_maxdeg[maxdeg];
  }
  if (k == 4) {
    /* trees on 4 nodes: the path (max degree 2) and the star (max degree 3) */
    for (int i = 1; i <= 6; ++i)
      if (trees_by_maxdeg[2] == PHI4_PATH[i] && trees_by_maxdeg[3] == PHI4_STAR[i]) return i;
    return -1;
  }
  /* trees on 5 nodes: path (max degree 2), fork (3), star (4) */
  for (int i = 1; i <= 21; ++i)
    if (trees_by_maxdeg[3] == PHI5_FORK[i] && trees_by_maxdeg[2] == PHI5_PATH[i] &&
        trees_by_maxdeg[4] == PHI5_STAR[i])
      return i;
  return -1;
}

/* The classifier is a pure function of the sample's adjacency; the samplers
   and the enumerator call it through a table indexed by the pair bits
   (bit p set when the p-th pair (i<j, in row-major order) is an edge). */
static int8_t class4_of_mask[64], class5_of_mask[1024];
static pthread_once_t class_once = PTHREAD_ONCE_INIT;

static void adj_from_mask(int k, int mask, uint8_t *adj) {
  memset(adj, 0, (size_t)k * k);
  int p = 0;
  for (int i = 0; i < k; ++i)
    for (int j = i + 1; j < k; ++j, ++p)
      if (mask >> p & 1) adj[i * k + j] = adj[j * k + i] = 1;
}

static void init_class_tables(void) {
  uint8_t adj[25];
  for (int m = 0; m < 64; ++m) { adj_from_mask(4, m, adj); class4_of_mask[m] = (int8_t)orc_classify(4, adj); }
  for (int m = 0; m < 1024; ++m) { adj_from_mask(5, m, adj); class5_of_mask[m] = (int8_t)orc_classify(5, adj); }
}

/* ------------------------------------------------------------------------ */
/* Graph store and initialization (Section 4.1.3 "Initialization"; weights    */
/* Gamma_v (Sec 4.1.1), Gamma^(1)_v (Sec 5.1.1), Gamma^(2)_v (Sec 5.1.2), the */
/* per-row arrays ACC_sigma (Sec 4.1.3) = ACC_mu (Sec 5.1.5) and the per-row  */
/* prefix of the tau weights of Sec 5.1.2; Lambda_3, Lambda_4 of Table 1).     */
/* ------------------------------------------------------------------------ */
static int32_t degree(const orc_graph *g, int32_t v) { return g->rp[v + 1] - g->rp[v]; }

static int validate_csr(int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col) {
  if (rp[0] != 0 || rp[n] != nnz) return ORC_E_ARG;
  for (int32_t v = 0; v < n; ++v) {
    if (rp[v + 1] < rp[v]) return ORC_E_ARG;
    for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
      if (col[e] < 0 || col[e] >= n) return ORC_E_ARG;
      if (col[e] == v) return ORC_E_SELF_LOOP;
      if (e > rp[v]) {
        if (col[e] == col[e - 1]) return ORC_E_DUPLICATE;
        if (col[e] < col[e - 1]) return ORC_E_UNSORTED;
      }
    }
  }
  for (int32_t v = 0; v < n; ++v)
    for (int64_t e = rp[v]; e < rp[v + 1]; ++e) {
      int32_t x = col[e];
      int64_t lo = rp[x], hi = rp[x + 1];
      int found = 0;
      while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] == v) { found = 1; break; }
        if (col[mid] < v) lo = mid + 1; else hi = mid;
      }
      if (!found) return ORC_E_ASYMMETRIC;
    }
  return ORC_OK;
}

static int fits(u128 x) { return (x >> 64) == 0; }

static u128 choose(uint64_t d, int r) {
  if (d < (uint64_t)r) return 0;
  u128 c = 1;
  for (int i = 0; i < r; ++i) c = c * (d - (uint64_t)i) / (u128)(i + 1);
  return c;
}

/* ------------------------------------------------------------------------ */
/* MOSS-4Min tables (Section 4.2.1).  The total order is the example of      */
/* Section 3.2: a > b when d_a > d_b, or d_a = d_b and the id of a is larger. */
/* As a number, key(a) = d_a * 2^32 + a, and a > b exactly when key(a) >     */
/* key(b).  From Table 1: N_{u,v} = {x in N_u : x > v}, d_{u,v} = |N_{u,v}|. */
/* MOSS-4Min weighs node v by check-Gamma_v = sum_{x in N_v} d_{v,x} d_{x,v}, */
/* and u in N_v by d_{u,v} d_{v,u}.  Each row is also kept sorted by the      */
/* order, largest first: there N_{v,x} is the first d_{v,x} entries of row v. */
/* ------------------------------------------------------------------------ */
static uint64_t order_key(const orc_graph *g, int32_t a) {
  return ((uint64_t)(uint32_t)degree(g, a) << 32) | (uint64_t)(uint32_t)a;
}

static int key_descending(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return x < y ? 1 : (x > y ? -1 : 0);
}

static int build_min_tables(orc_graph *g) {
  size_t nn = (size_t)g->n + 1, ne = (size_t)g->nnz + 1;
  int32_t dmax = 0;
  for (int32_t v = 0; v < g->n; ++v) if (degree(g, v) > dmax) dmax = degree(g, v);
  g->rank = (uint32_t *)calloc(ne, 4);
  g->rank_mirror = (uint32_t *)calloc(ne, 4);
  g->col_rank = (int32_t *)calloc(ne, 4);
  g->acc_check = (uint64_t *)calloc(ne, 8);
  g->gmin = (uint64_t *)calloc(nn, 8);
  g->acc_gmin = (uint64_t *)calloc(nn, 8);
  uint64_t *sorted = (uint64_t *)malloc((size_t)(dmax + 1) * 8);
  if (!g->rank || !g->rank_mirror || !g->col_rank || !g->acc_check || !g->gmin || !g->acc_gmin || !sorted) {
    free(sorted);
    return ORC_E_NOMEM;
  }
  /* d_{v,x}: the number of keys of row v above key(x), i.e. x's place in the row
     sorted largest first */
  for (int32_t v = 0; v < g->n; ++v) {
    int64_t base = g->rp[v], d = degree(g, v);
    for (int64_t j = 0; j < d; ++j) sorted[j] = order_key(g, g->col[base + j]);
    qsort(sorted, (size_t)d, sizeof(uint64_t), key_descending);
    for (int64_t j = 0; j < d; ++j) g->col_rank[base + j] = (int32_t)(uint32_t)(sorted[j] & 0xFFFFFFFFu);
    for (int64_t j = 0; j < d; ++j) {
      uint64_t key = order_key(g, g->col[base + j]);
      int64_t lo = 0, hi = d; /* first place whose key is not above `key` */
      while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (sorted[mid] > key) lo = mid + 1; else hi = mid;
      }
      g->rank[base + j] = (uint32_t)lo;
    }
  }
  free(sorted);
  /* d_{x,v} from the entry (x, v) of row x; weights, row prefixes and node weights */
  u128 tot = 0;
  g->tot.min_status = ORC_OK;
  for (int32_t v = 0; v < g->n; ++v) {
    u128 s = 0;
    for (int64_t e = g->rp[v]; e < g->rp[v + 1]; ++e) {
      int32_t x = g->col[e];
      int64_t lo = g->rp[x], hi = g->rp[x + 1], m = -1;
      while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (g->col[mid] == v) { m = mid; break; }
        if (g->col[mid] < v) lo = mid + 1; else hi = mid;
      }
      if (m < 0) return ORC_E_ASYMMETRIC; /* only without validation */
      g->rank_mirror[e] = g->rank[m];
      s += (u128)g->rank[e] * g->rank_mirror[e];
      if (!fits(s)) g->tot.min_status = ORC_E_OVERFLOW;
      g->acc_check[e] = (uint64_t)s;
    }
    g->gmin[v] = (uint64_t)s;
    tot += s;
    if (!fits(tot)) g->tot.min_status = ORC_E_OVERFLOW;
    g->acc_gmin[v] = (uint64_t)tot;
  }
  g->tot.gamma_min = g->tot.min_status == ORC_OK ? (uint64_t)tot : 0;
  return ORC_OK;
}

void orc_free(orc_graph *g) {
  if (!g) return;
  free(g->rp); free(g->col); free(g->S); free(g->Q); free(g->gam); free(g->gam1); free(g->gam2);
  free(g->acc_gam); free(g->acc_gam1); free(g->acc_gam2); free(g->acc_sigma); free(g->acc_tau);
  free(g->rank); free(g->rank_mirror); free(g->col_rank); free(g->acc_check); free(g->gmin); free(g->acc_gmin);
  free(g);
}

int orc_build(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col, int validate,
              orc_graph **out) {
  if (!out || n < 0 || nnz < 0 || (n > 0 && !row_ptr) || (nnz > 0 && !col)) return ORC_E_ARG;
  pthread_once(&class_once, init_class_tables);
  if (n == 0 && nnz != 0) return ORC_E_ARG;
  if (validate && n > 0) {
    int st = validate_csr(n, nnz, row_ptr, col);
    if (st != ORC_OK) return st;
  }
  orc_graph *g = (orc_graph *)calloc(1, sizeof(orc_graph));
  if (!g) return ORC_E_NOMEM;
  g->n = n;
  g->nnz = nnz;
  size_t nn = (size_t)n + 1, ne = (size_t)nnz + 1;
  g->rp = (int32_t *)malloc(nn * sizeof(int32_t));
  g->col = (int32_t *)malloc(ne * sizeof(int32_t));
  g->S = (uint64_t *)calloc(nn, 8); g->Q = (uint64_t *)calloc(nn, 8);
  g->gam = (uint64_t *)calloc(nn, 8); g->gam1 = (uint64_t *)calloc(nn, 8); g->gam2 = (uint64_t *)calloc(nn, 8);
  g->acc_gam = (uint64_t *)calloc(nn, 8); g->acc_gam1 = (uint64_t *)calloc(nn, 8); g->acc_gam2 = (uint64_t *)calloc(nn, 8);
  g->acc_sigma = (uint32_t *)calloc(ne, 4);
  g->acc_tau = (uint64_t *)calloc(ne, 8);
  if (!g->rp || !g->col || !g->S || !g->Q || !g->gam || !g->gam1 || !g->gam2 || !g->acc_gam ||
      !g->acc_gam1 || !g->acc_gam2 || !g->acc_sigma || !g->acc_tau) {
    orc_free(g);
    return ORC_E_NOMEM;
  }
  if (n > 0) memcpy(g->rp, row_ptr, (size_t)(n + 1) * sizeof(int32_t));
  else g->rp[0] = 0;
  if (nnz > 0) memcpy(g->col, col, (size_t)nnz * sizeof(int32_t));

  u128 tot_gam = 0, tot_gam1 = 0, tot_gam2 = 0, lam3 = 0, lam4 = 0;
  for (int32_t v = 0; v < n; ++v) {
    int64_t dv = degree(g, v);
    /* S_v = sum_{x in N_v} (d_x - 1), Q_v = sum (d_x - 1)^2 and the row prefix ACC_sigma */
    u128 s = 0, q = 0;
    for (int64_t e = g->rp[v]; e < g->rp[v + 1]; ++e) {
      uint64_t dx1 = (uint64_t)(degree(g, g->col[e]) - 1);
      s += dx1;
      q += (u128)dx1 * dx1;
      if (s > 0xFFFFFFFFu) { orc_free(g); return ORC_E_OVERFLOW; }
      g->acc_sigma[e] = (uint32_t)s;
    }
    if (!fits(q)) { orc_free(g); return ORC_E_OVERFLOW; }
    g->S[v] = (uint64_t)s;
    g->Q[v] = (uint64_t)q;
    /* Gamma_v = (d_v - 1) S_v ;  Gamma^(1)_v = (d_v - 1)(d_v - 2) S_v ;
       Gamma^(2)_v = S_v^2 - Q_v  (zero when d_v < 2: then S_v = 0 or the factors vanish) */
    u128 g0 = dv >= 1 ? (u128)(uint64_t)(dv - 1) * s : 0;
    u128 g1 = dv >= 2 ? (u128)(uint64_t)(dv - 1) * (uint64_t)(dv - 2) * s : 0;
    u128 g2 = s * s - q;
    if (!fits(g0) || !fits(g1) || !fits(g2)) { orc_free(g); return ORC_E_OVERFLOW; }
    g->gam[v] = (uint64_t)g0;
    g->gam1[v] = (uint64_t)g1;
    g->gam2[v] = (uint64_t)g2;
    /* per-row prefix of tau weights (d_u - 1) * (S_v - (d_u - 1))  (Sec 5.1.2, step 2) */
    u128 t = 0;
    for (int64_t e = g->rp[v]; e < g->rp[v + 1]; ++e) {
      uint64_t du1 = (uint64_t)(degree(g, g->col[e]) - 1);
      t += (u128)du1 * ((uint64_t)s - du1);
      if (!fits(t)) { orc_free(g); return ORC_E_OVERFLOW; }
      g->acc_tau[e] = (uint64_t)t;
    }
    tot_gam += g0; tot_gam1 += g1; tot_gam2 += g2;
    if (!fits(tot_gam) || !fits(tot_gam1) || !fits(tot_gam2)) { orc_free(g); return ORC_E_OVERFLOW; }
    g->acc_gam[v] = (uint64_t)tot_gam;
    g->acc_gam1[v] = (uint64_t)tot_gam1;
    g->acc_gam2[v] = (uint64_t)tot_gam2;
    lam3 += choose((uint64_t)dv, 3);
    lam4 += choose((uint64_t)dv, 4);
    if (!fits(lam3) || !fits(lam4)) { orc_free(g); return ORC_E_OVERFLOW; }
  }
  g->tot.gamma = (uint64_t)tot_gam;
  g->tot.gamma1 = (uint64_t)tot_gam1;
  g->tot.gamma2 = (uint64_t)tot_gam2;
  g->tot.lambda3 = (uint64_t)lam3;
  g->tot.lambda4 = (uint64_t)lam4;
  int st = build_min_tables(g);
  if (st != ORC_OK) { orc_free(g); return st; }
  *out = g;
  return ORC_OK;
}

int orc_totals_get(const orc_graph *g, orc_totals *t) {
  if (!g || !t) return ORC_E_ARG;
  *t = g->tot;
  return ORC_OK;
}

int orc_table(const orc_graph *g, int which, void *out) {
  if (!g || !out) return ORC_E_ARG;
  size_t n8 = (size_t)g->n * 8;
  switch (which) {
    case ORC_TAB_S: memcpy(out, g->S, n8); break;
    case ORC_TAB_Q: memcpy(out, g->Q, n8); break;
    case ORC_TAB_GAMMA: memcpy(out, g->gam, n8); break;
    case ORC_TAB_GAMMA1: memcpy(out, g->gam1, n8); break;
    case ORC_TAB_GAMMA2: memcpy(out, g->gam2, n8); break;
    case ORC_TAB_ACC_GAMMA: memcpy(out, g->acc_gam, n8); break;
    case ORC_TAB_ACC_GAMMA1: memcpy(out, g->acc_gam1, n8); break;
    case ORC_TAB_ACC_GAMMA2: memcpy(out, g->acc_gam2, n8); break;
    case ORC_TAB_ACC_SIGMA: memcpy(out, g->acc_sigma, (size_t)g->nnz * 4); break;
    case ORC_TAB_ACC_TAU: memcpy(out, g->acc_tau, (size_t)g->nnz * 8); break;
    case ORC_TAB_GAMMA_MIN: memcpy(out, g->gmin, n8); break;
    case ORC_TAB_ACC_GAMMA_MIN: memcpy(out, g->acc_gmin, n8); break;
    case ORC_TAB_ACC_CHECK: memcpy(out, g->acc_check, (size_t)g->nnz * 8); break;
    case ORC_TAB_RANK: memcpy(out, g->rank, (size_t)g->nnz * 4); break;
    case ORC_TAB_RANK_MIRROR: memcpy(out, g->rank_mirror, (size_t)g->nnz * 4); break;
    case ORC_TAB_COL_RANK: memcpy(out, g->col_rank, (size_t)g->nnz * 4); break;
    default: return ORC_E_ARG;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Memory-read recorder for the line-count mode (inactive when rec == NULL).  */
/* ------------------------------------------------------------------------ */
enum { ARR_RP = 0, ARR_COL, ARR_ACC_NODE, ARR_ACC_SIGMA, ARR_ACC_TAU, ARR_ACC_CHECK, ARR_RANK, ARR_RANK_MIRROR,
       ARR_COL_RANK };
typedef struct { int n; uint64_t key[512]; } reads;

static void note(reads *rec, int arr, int64_t idx, int width) {
  if (!rec) return;
  uint64_t key = ((uint64_t)arr << 56) | (uint64_t)((idx * width) / 64);
  for (int i = 0; i < rec->n; ++i) if (rec->key[i] == key) return;
  if (rec->n < 512) rec->key[rec->n++] = key;
}

static int32_t rp_at(const orc_graph *g, int32_t i, reads *rec) { note(rec, ARR_RP, i, 4); return g->rp[i]; }
static int32_t col_at(const orc_graph *g, int64_t e, reads *rec) { note(rec, ARR_COL, e, 4); return g->col[e]; }

static int64_t pick_node(const uint64_t *acc, int32_t n, uint64_t r, reads *rec) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    note(rec, ARR_ACC_NODE, mid, 8);
    if (acc[mid] > r) hi = mid; else lo = mid + 1;
  }
  return lo;
}

static int64_t pick_sigma(const orc_graph *g, int64_t base, int64_t len, uint64_t r, reads *rec) {
  int64_t lo = 0, hi = len - 1;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    note(rec, ARR_ACC_SIGMA, base + mid, 4);
    if ((uint64_t)g->acc_sigma[base + mid] > r) hi = mid; else lo = mid + 1;
  }
  return lo;
}

static int64_t pick_tau(const orc_graph *g, int64_t base, int64_t len, uint64_t r, reads *rec) {
  int64_t lo = 0, hi = len - 1;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    note(rec, ARR_ACC_TAU, base + mid, 8);
    if (g->acc_tau[base + mid] > r) hi = mid; else lo = mid + 1;
  }
  return lo;
}

static int64_t pick_check(const orc_graph *g, int64_t base, int64_t len, uint64_t r, reads *rec) {
  int64_t lo = 0, hi = len - 1;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    note(rec, ARR_ACC_CHECK, base + mid, 8);
    if (g->acc_check[base + mid] > r) hi = mid; else lo = mid + 1;
  }
  return lo;
}

/* Is b a neighbour of a?  Binary search of the shorter of the two sorted rows. */
static int is_adj(const orc_graph *g, int32_t a, int32_t b, reads *rec) {
  int64_t ra = rp_at(g, a, rec), ra1 = rp_at(g, a + 1, rec);
  int64_t rb = rp_at(g, b, rec), rb1 = rp_at(g, b + 1, rec);
  int64_t lo, hi;
  int32_t key;
  if (ra1 - ra <= rb1 - rb) { lo = ra; hi = ra1; key = b; }
  else { lo = rb; hi = rb1; key = a; }
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    int32_t c = col_at(g, mid, rec);
    if (c == key) return 1;
    if (c < key) lo = mid + 1; else hi = mid;
  }
  return 0;
}

/* RandomVertex(N_a - {b}) for b in N_a (Section 4.1.3): an index j uniform in
   [0, d_a - 1) addresses the sorted row with b's slot removed, so the entry at
   j is used unless it is >= b, in which case the next one is. */
static int32_t neighbour_skipping(const orc_graph *g, int32_t a, int32_t b, uint64_t word, reads *rec) {
  int64_t base = rp_at(g, a, rec), end = rp_at(g, a + 1, rec);
  uint64_t j = orc_bounded(word, (uint64_t)(end - base - 1));
  int32_t x = col_at(g, base + (int64_t)j, rec);
  if (x >= b) x = col_at(g, base + (int64_t)j + 1, rec);
  return x;
}

static int class_of(int k, const int32_t *nodes, const orc_graph *g, reads *rec) {
  int mask = 0, p = 0;
  for (int i = 0; i < k; ++i)
    for (int j = i + 1; j < k; ++j, ++p)
      if (is_adj(g, nodes[i], nodes[j], rec)) mask |= 1 << p;
  return k == 4 ? class4_of_mask[mask] : class5_of_mask[mask];
}

/* Which pairs must be probed: the sampled structure already fixes some edges.
   For classification the oracle simply probes all pairs; the line-count mode
   counts only the unknown pairs (the known ones need no read). */
static int class_of_counting(int k, const int32_t *nodes, const orc_graph *g, reads *rec,
                             const int *known_pairs) {
  int mask = 0, p = 0;
  for (int i = 0; i < k; ++i)
    for (int j = i + 1; j < k; ++j, ++p) {
      int e = known_pairs[p] ? 1 : is_adj(g, nodes[i], nodes[j], rec);
      if (e) mask |= 1 << p;
    }
  return k == 4 ? class4_of_mask[mask] : class5_of_mask[mask];
}

/* ------------------------------------------------------------------------ */
/* MOSS-4 (Section 4.1.1, Algorithm 1): v ~ pi (weights Gamma_v), u ~ sigma^(v)*/
/* (weights d_u - 1), w uniform in N_v - {u}, r uniform in N_u - {v}; the     */
/* sample is dropped when r = w (the test r != u can never fail in a simple    */
/* graph).  Pair order for the class mask: (v,u),(v,w),(v,r),(u,w),(u,r),(w,r).*/
/* ------------------------------------------------------------------------ */
static const int KNOWN4[6] = {1, 1, 0, 0, 1, 0};
/* T-5 (Section 5.1.1, Algorithm 3): v ~ rho^(1) (weights Gamma^(1)_v), u ~     */
/* sigma^(v), w and r two different nodes of N_v - {u}, t uniform in           */
/* N_u - {v}; dropped when t is w or r.  Known edges vu, vw, vr, ut.           */
static const int KNOWN5_T[10] = {1, 1, 1, 0, 0, 0, 1, 0, 0, 0};
/* Path-5 (Section 5.1.2, Algorithm 4): v ~ rho^(2) (weights Gamma^(2)_v), u ~  */
/* tau^(v), w ~ mu^(v,u) over N_v - {u}, r uniform in N_u - {v}, t uniform in  */
/* N_w - {v}; dropped when t = u, r = w or t = r.  Known edges vu, vw, ur, wt. */
static const int KNOWN5_P[10] = {1, 1, 0, 0, 0, 1, 0, 0, 1, 0};
/* MOSS-4Min (Section 4.2.1, Algorithm 2): v ~ check-pi (weights check-Gamma_v), u ~  */
/* check-sigma^(v) (weights d_{u,v} d_{v,u} over N_v), w uniform in N_{v,u}, r       */
/* uniform in N_{u,v}; dropped when r = w (r = u cannot happen).  Known edges vu,   */
/* vw, ur, as for MOSS-4.                                                           */
/* pair order for 5 nodes (v,u,w,r,t):
   (v,u),(v,w),(v,r),(v,t),(u,w),(u,r),(u,t),(w,r),(w,t),(r,t) */

static int sample_one(const orc_graph *g, int sampler, uint64_t seed, uint64_t k, int32_t nodes[5],
                      reads *rec) {
  uint64_t W[4], W2[4];
  words(seed, (uint64_t)sampler, k, 0, W);
  if (sampler == ORC_MOSS4) {
    if (g->tot.gamma == 0) return ORC_E_ARG;
    int32_t v = (int32_t)pick_node(g->acc_gam, g->n, orc_bounded(W[0], g->tot.gamma), rec);
    int64_t base = rp_at(g, v, rec), dv = rp_at(g, v + 1, rec) - base;
    int64_t iu = pick_sigma(g, base, dv, orc_bounded(W[1], g->acc_sigma[base + dv - 1]), rec);
    note(rec, ARR_ACC_SIGMA, base + dv - 1, 4);
    int32_t u = col_at(g, base + iu, rec);
    int64_t j = (int64_t)orc_bounded(W[2], (uint64_t)(dv - 1));
    if (j >= iu) ++j;
    int32_t w = col_at(g, base + j, rec);
    int32_t r = neighbour_skipping(g, u, v, W[3], rec);
    nodes[0] = v; nodes[1] = u; nodes[2] = w; nodes[3] = r; nodes[4] = -1;
    if (r == w) return 0;
    return rec ? class_of_counting(4, nodes, g, rec, KNOWN4) : class_of(4, nodes, g, NULL);
  }
  if (sampler == ORC_MOSS4MIN) {
    if (g->tot.min_status != ORC_OK) return g->tot.min_status;
    if (g->tot.gamma_min == 0) return ORC_E_ARG;
    int32_t v = (int32_t)pick_node(g->acc_gmin, g->n, orc_bounded(W[0], g->tot.gamma_min), rec);
    int64_t base = rp_at(g, v, rec), dv = rp_at(g, v + 1, rec) - base;
    note(rec, ARR_ACC_CHECK, base + dv - 1, 8);
    int64_t iu = pick_check(g, base, dv, orc_bounded(W[1], g->acc_check[base + dv - 1]), rec);
    int32_t u = col_at(g, base + iu, rec);
    note(rec, ARR_RANK, base + iu, 4);
    note(rec, ARR_RANK_MIRROR, base + iu, 4);
    uint64_t dvu = g->rank[base + iu], duv = g->rank_mirror[base + iu];
    /* N_{v,u} is the first d_{v,u} entries of row v taken largest first */
    int64_t jw = base + (int64_t)orc_bounded(W[2], dvu);
    note(rec, ARR_COL_RANK, jw, 4);
    int32_t w = g->col_rank[jw];
    int64_t jr = rp_at(g, u, rec) + (int64_t)orc_bounded(W[3], duv);
    note(rec, ARR_COL_RANK, jr, 4);
    int32_t r = g->col_rank[jr];
    nodes[0] = v; nodes[1] = u; nodes[2] = w; nodes[3] = r; nodes[4] = -1;
    if (r == w) return 0;
    return rec ? class_of_counting(4, nodes, g, rec, KNOWN4) : class_of(4, nodes, g, NULL);
  }
  if (sampler == ORC_T5) {
    if (g->tot.gamma1 == 0) return ORC_E_ARG;
    words(seed, (uint64_t)sampler, k, 1, W2);
    int32_t v = (int32_t)pick_node(g->acc_gam1, g->n, orc_bounded(W[0], g->tot.gamma1), rec);
    int64_t base = rp_at(g, v, rec), dv = rp_at(g, v + 1, rec) - base;
    int64_t iu = pick_sigma(g, base, dv, orc_bounded(W[1], g->acc_sigma[base + dv - 1]), rec);
    note(rec, ARR_ACC_SIGMA, base + dv - 1, 4);
    int32_t u = col_at(g, base + iu, rec);
    int64_t iw = (int64_t)orc_bounded(W[2], (uint64_t)(dv - 1));
    if (iw >= iu) ++iw;
    int32_t w = col_at(g, base + iw, rec);
    /* RandomVertex(N_v - {u, w}): skip the two excluded slots in ascending order */
    int64_t a = iu < iw ? iu : iw, b = iu < iw ? iw : iu;
    int64_t ir = (int64_t)orc_bounded(W[3], (uint64_t)(dv - 2));
    if (ir >= a) ++ir;
    if (ir >= b) ++ir;
    int32_t r = col_at(g, base + ir, rec);
    int32_t t = neighbour_skipping(g, u, v, W2[0], rec);
    nodes[0] = v; nodes[1] = u; nodes[2] = w; nodes[3] = r; nodes[4] = t;
    if (t == w || t == r) return 0;
    return rec ? class_of_counting(5, nodes, g, rec, KNOWN5_T) : class_of(5, nodes, g, NULL);
  }
  if (sampler == ORC_PATH5) {
    if (g->tot.gamma2 == 0) return ORC_E_ARG;
    words(seed, (uint64_t)sampler, k, 1, W2);
    int32_t v = (int32_t)pick_node(g->acc_gam2, g->n, orc_bounded(W[0], g->tot.gamma2), rec);
    int64_t base = rp_at(g, v, rec), dv = rp_at(g, v + 1, rec) - base;
    int64_t iu = pick_tau(g, base, dv, orc_bounded(W[1], g->acc_tau[base + dv - 1]), rec);
    note(rec, ARR_ACC_TAU, base + dv - 1, 8);
    int32_t u = col_at(g, base + iu, rec);
    /* WeightRandomVertex(N_v - {u}, mu^(v,u)) (Section 5.1.5): rnd ranges over
       {1..ACC_mu[d_v]} minus u's block {ACC_mu[POS-1]+1 .. ACC_mu[POS]}; the
       0-based draw x over the shortened range is moved past that block. */
    uint64_t sv = g->acc_sigma[base + dv - 1];
    uint64_t lo = iu > 0 ? g->acc_sigma[base + iu - 1] : 0;
    uint64_t du1 = (uint64_t)g->acc_sigma[base + iu] - lo;
    note(rec, ARR_ACC_SIGMA, base + dv - 1, 4);
    note(rec, ARR_ACC_SIGMA, base + iu, 4);
    if (iu > 0) note(rec, ARR_ACC_SIGMA, base + iu - 1, 4);
    uint64_t x = orc_bounded(W[2], sv - du1);
    if (x >= lo) x += du1;
    int64_t iw = pick_sigma(g, base, dv, x, rec);
    int32_t w = col_at(g, base + iw, rec);
    int32_t r = neighbour_skipping(g, u, v, W[3], rec);
    int32_t t = neighbour_skipping(g, w, v, W2[0], rec);
    nodes[0] = v; nodes[1] = u; nodes[2] = w; nodes[3] = r; nodes[4] = t;
    if (t == u || r == w || t == r) return 0;
    return rec ? class_of_counting(5, nodes, g, rec, KNOWN5_P) : class_of(5, nodes, g, NULL);
  }
  return ORC_E_ARG;
}

int orc_sample(const orc_graph *g, int sampler, uint64_t seed, uint64_t k, int32_t nodes[5]) {
  if (!g || !nodes) return ORC_E_ARG;
  return sample_one(g, sampler, seed, k, nodes, NULL);
}

/* The draws of MOSS-4Min that give a node set s: ordered tuples (w, v, u, r) of its
   nodes with edges w-v, v-u, u-r, w > u (w in N_{v,u}) and r > v (r in N_{u,v}).  Each
   such tuple has probability 1/check-Gamma (the node, edge and two uniform draws of
   Section 4.2.1 multiply to it), so s is drawn with probability c(s)/check-Gamma. */
int orc_ways_of(const uint8_t adj[16], const uint64_t key[4]) {
  int c = 0;
  for (int w = 0; w < 4; ++w)
    for (int v = 0; v < 4; ++v)
      for (int u = 0; u < 4; ++u)
        for (int r = 0; r < 4; ++r) {
          if (w == v || w == u || w == r || v == u || v == r || u == r) continue;
          if (adj[w * 4 + v] && adj[v * 4 + u] && adj[u * 4 + r] && key[w] > key[u] && key[r] > key[v]) ++c;
        }
  return c;
}

static int ways_of_nodes(const orc_graph *g, const int32_t nodes[4]) {
  uint8_t adj[16];
  uint64_t key[4];
  for (int i = 0; i < 4; ++i) {
    key[i] = order_key(g, nodes[i]);
    for (int j = 0; j < 4; ++j) adj[i * 4 + j] = i != j && is_adj(g, nodes[i], nodes[j], NULL);
  }
  return orc_ways_of(adj, key);
}

typedef struct {
  const orc_graph *g;
  int sampler;
  uint64_t seed, k0, k1;
  uint64_t hits[22];
  int status;
} run_job;

static void *run_range(void *arg) {
  run_job *job = (run_job *)arg;
  int32_t nodes[5];
  for (uint64_t k = job->k0; k < job->k1; ++k) {
    int c = sample_one(job->g, job->sampler, job->seed, k, nodes, NULL);
    if (c < 0) { job->status = c; return NULL; }
    ++job->hits[c];
    if (job->sampler == ORC_MOSS4MIN && c == 5) ++job->hits[6 + ways_of_nodes(job->g, nodes) / 2];
  }
  return NULL;
}

int orc_run(const orc_graph *g, int sampler, uint64_t seed, uint64_t k0, uint64_t k1, int nthreads,
            uint64_t hits[22]) {
  if (!g || !hits || k1 < k0) return ORC_E_ARG;
  if (sampler != ORC_MOSS4 && sampler != ORC_MOSS4MIN && sampler != ORC_T5 && sampler != ORC_PATH5)
    return ORC_E_ARG;
  if (sampler == ORC_MOSS4MIN && g->tot.min_status != ORC_OK) return g->tot.min_status;
  memset(hits, 0, 22 * sizeof(uint64_t));
  uint64_t total = sampler == ORC_MOSS4      ? g->tot.gamma
                   : sampler == ORC_MOSS4MIN ? g->tot.gamma_min
                   : sampler == ORC_T5       ? g->tot.gamma1
                                             : g->tot.gamma2;
  if (total == 0 || k1 == k0) return ORC_OK; /* nothing can be drawn */
  if (nthreads < 1) nthreads = 1;
  if ((uint64_t)nthreads > k1 - k0) nthreads = (int)(k1 - k0);
  run_job *jobs = (run_job *)calloc((size_t)nthreads, sizeof(run_job));
  pthread_t *tids = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
  if (!jobs || !tids) { free(jobs); free(tids); return ORC_E_NOMEM; }
  uint64_t span = k1 - k0;
  for (int t = 0; t < nthreads; ++t) {
    jobs[t].g = g; jobs[t].sampler = sampler; jobs[t].seed = seed;
    jobs[t].k0 = k0 + span * (uint64_t)t / (uint64_t)nthreads;
    jobs[t].k1 = k0 + span * (uint64_t)(t + 1) / (uint64_t)nthreads;
  }
  for (int t = 1; t < nthreads; ++t) pthread_create(&tids[t], NULL, run_range, &jobs[t]);
  run_range(&jobs[0]);
  for (int t = 1; t < nthreads; ++t) pthread_join(tids[t], NULL);
  int status = ORC_OK;
  for (int t = 0; t < nthreads; ++t) {
    if (jobs[t].status) status = jobs[t].status;
    for (int c = 0; c < 22; ++c) hits[c] += jobs[t].hits[c];
  }
  free(jobs); free(tids);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Estimator finals, double precision.                                         */
/* ------------------------------------------------------------------------ */

/* MOSS-4 (Section 4.1.2, Theorems 2 and 3): p_i = 2 phi^(1)_i / Gamma,
   n_i = m_i / (K p_i) for i in {1,3,4,5,6};  n_2 = Lambda_3 - n_4 - 2 n_5 - 4 n_6;
   Var(n_i) = (n_i / K)(1/p_i - n_i);
   Var(n_2) = (n_4/p_4 + 4 n_5/p_5 + 16 n_6/p_6 - (n_4 + 2 n_5 + 4 n_6)^2) / K,
   with the unknown n_i replaced by their estimates. */
int orc_finals4(uint64_t K, const uint64_t hits[7], uint64_t gamma, uint64_t lambda3, double est[6],
                double var[6]) {
  if (!hits || !est || !var || K == 0) return ORC_E_ARG;
  double Kd = (double)K;
  double p[7] = {0};
  for (int i = 0; i < 6; ++i) { est[i] = 0.0; var[i] = 0.0; }
  if (gamma > 0) {
    for (int i = 1; i <= 6; ++i) {
      if (PHI4_PATH[i] == 0) continue;
      p[i] = 2.0 * (double)PHI4_PATH[i] / (double)gamma;
      est[i - 1] = (double)hits[i] / (Kd * p[i]);
      double v = est[i - 1] / Kd * (1.0 / p[i] - est[i - 1]);
      var[i - 1] = v > 0.0 ? v : 0.0;
    }
  }
  double n4 = est[3], n5 = est[4], n6 = est[5];
  est[1] = (double)lambda3 - n4 - 2.0 * n5 - 4.0 * n6;
  if (gamma > 0) {
    double s = n4 + 2.0 * n5 + 4.0 * n6;
    double v = (n4 / p[4] + 4.0 * n5 / p[5] + 16.0 * n6 / p[6] - s * s) / Kd;
    var[1] = v > 0.0 ? v : 0.0;
  }
  return ORC_OK;
}

/* MOSS-5 (Section 5.1.3 and Theorem 10).  Per sampler l: p^(l)_i = 2 phi^(l)_i / Gamma^(l),
   defined when phi^(l)_i > 0 and Gamma^(l) > 0.  The paper's weights lambda depend on the
   unknown eta_i.  Pooled reading (default): lambda^(l)_i = K_l p^(l)_i / sum_l K_l p^(l)_i,
   which gives eta_i = (m^(1)_i + m^(2)_i) / (K_1 p^(1)_i + K_2 p^(2)_i), unbiased, and
   the paper's lambda in the limit eta_i p_i -> 0.  Paper reading: lambda from the Theorem 7/9
   variances evaluated at the pooled estimate.  With coefficients a^(l)_i (= lambda^(l)_i, 1 or 0):
   Var(eta_i) = sum_l (a^(l)_i)^2 (eta_i / K_l)(1/p^(l)_i - eta_i)  (pooled);
   V1 V2 / (V1 + V2) (paper, Eq. varianceMix);
   Cov(eta_i, eta_j) = -eta_i eta_j sum_l a^(l)_i a^(l)_j / K_l;
   eta_2 = Lambda_4 - sum_{i in Omega3*} phi^(3)_i eta_i and
   Var(eta_2) = sum_{i,j in Omega3*} phi^(3)_i phi^(3)_j Cov(eta_i, eta_j). */
int orc_finals5(uint64_t K1, uint64_t K2, const uint64_t hits1[22], const uint64_t hits2[22],
                uint64_t gamma1, uint64_t gamma2, uint64_t lambda4, int mix, double est[21],
                double var[21], double *cov) {
  if (!hits1 || !hits2 || !est || !var || K1 == 0 || K2 == 0) return ORC_E_ARG;
  if (mix != ORC_MIX_POOLED && mix != ORC_MIX_PAPER) return ORC_E_ARG;
  double K[2] = {(double)K1, (double)K2};
  double a[2][22];
  memset(a, 0, sizeof(a));
  for (int i = 0; i < 21; ++i) { est[i] = 0.0; var[i] = 0.0; }
  for (int i = 1; i <= 21; ++i) {
    if (i == 2) continue;
    double p1 = (PHI5_FORK[i] > 0 && gamma1 > 0) ? 2.0 * PHI5_FORK[i] / (double)gamma1 : 0.0;
    double p2 = (PHI5_PATH[i] > 0 && gamma2 > 0) ? 2.0 * PHI5_PATH[i] / (double)gamma2 : 0.0;
    double denom = K[0] * p1 + K[1] * p2;
    if (denom == 0.0) continue;
    double pooled = ((double)hits1[i] + (double)hits2[i]) / denom;
    double l1 = K[0] * p1 / denom, l2 = K[1] * p2 / denom;
    double e = pooled, v;
    double v1 = p1 > 0.0 ? pooled / K[0] * (1.0 / p1 - pooled) : 0.0;
    double v2 = p2 > 0.0 ? pooled / K[1] * (1.0 / p2 - pooled) : 0.0;
    if (v1 < 0.0) v1 = 0.0;
    if (v2 < 0.0) v2 = 0.0;
    if (mix == ORC_MIX_PAPER && p1 > 0.0 && p2 > 0.0 && v1 + v2 > 0.0) {
      l1 = v2 / (v1 + v2);
      l2 = v1 / (v1 + v2);
      double e1 = (double)hits1[i] / (K[0] * p1);
      double e2 = (double)hits2[i] / (K[1] * p2);
      e = l1 * e1 + l2 * e2;
      v = v1 * v2 / (v1 + v2);
    } else {
      v = l1 * l1 * v1 + l2 * l2 * v2;
    }
    a[0][i] = l1;
    a[1][i] = l2;
    est[i - 1] = e;
    var[i - 1] = v > 0.0 ? v : 0.0;
  }
  /* eta_2 by subtraction over Omega3* = {i != 2 : phi^(3)_i > 0} */
  double sub = 0.0;
  for (int i = 1; i <= 21; ++i)
    if (i != 2 && PHI5_STAR[i] > 0) sub += PHI5_STAR[i] * est[i - 1];
  est[1] = (double)lambda4 - sub;
  double v2sum = 0.0;
  for (int i = 1; i <= 21; ++i) {
    if (i == 2 || PHI5_STAR[i] == 0) continue;
    for (int j = 1; j <= 21; ++j) {
      if (j == 2 || PHI5_STAR[j] == 0) continue;
      double c;
      if (i == j) c = var[i - 1];
      else c = -est[i - 1] * est[j - 1] * (a[0][i] * a[0][j] / K[0] + a[1][i] * a[1][j] / K[1]);
      v2sum += (double)PHI5_STAR[i] * PHI5_STAR[j] * c;
    }
  }
  var[1] = v2sum > 0.0 ? v2sum : 0.0;
  if (cov) {
    for (int i = 1; i <= 21; ++i)
      for (int j = 1; j <= 21; ++j) {
        double c;
        if (i == j) c = var[i - 1];
        else if (i == 2 || j == 2) c = 0.0; /* not reported */
        else c = -est[i - 1] * est[j - 1] * (a[0][i] * a[0][j] / K[0] + a[1][i] * a[1][j] / K[1]);
        cov[(i - 1) * 21 + (j - 1)] = c;
      }
  }
  return ORC_OK;
}

/* MOSS-4 together with MOSS-4Min (Section 4.2: Algorithm 2, Theorems 4 and 5, and
   Theorem 1's mix for n_3, n_5, n_6).
   MOSS-4Min reaches a CIS s with probability c(s)/check-Gamma (orc_ways_of).  For
   the 4-cycle c = 2 and for the 4-clique c = 6, as Theorem 4 states; a diamond has
   c = 2, 4 or 6 depending on how its nodes are ordered, so Theorem 4's constant is
   replaced by each sample's own c (a Horvitz-Thompson weight):
     check-n_i = (check-Gamma / Kc) sum_c m_{i,c} / c,
     Var = (A_i - n_i^2) / Kc with A_i = sum_{s in C_i} check-Gamma / c(s),
   A_i estimated by (check-Gamma^2 / Kc) sum_c m_{i,c} / c^2 (unbiased); for c fixed
   this is Theorem 5.  Mix weights lambda_i (on MOSS-4), as for 5 nodes:
     pooled: lambda_i = K p_i / (K p_i + Kc q_i), q_3 = 2/check-Gamma, q_6 = 6/check-Gamma,
             q_5 = 2/check-Gamma (the least reach; a fixed weight keeps the mix
             unbiased), Var = lambda^2 V_1 + (1 - lambda)^2 V_2 with both variances at
             the mixed estimate (A_3 = n_3 / q_3, A_6 = n_6 / q_6, A_5 from the samples);
     paper:  lambda_i = V_2 / (V_1 + V_2) with V_1, V_2 at the pooled estimate,
             Var = V_1 V_2 / (V_1 + V_2).
   n_1, n_4 as MOSS-4 alone; n_2 = Lambda_3 - n_4 - 2 n_5 - 4 n_6 with variance
     (n_4/p_4 + 4 l_5^2 n_5/p_5 + 16 l_6^2 n_6/p_6 - (n_4 + 2 l_5 n_5 + 4 l_6 n_6)^2) / K
   + (4 (1-l_5)^2 A_5 + 16 (1-l_6)^2 A_6 - (2 (1-l_5) n_5 + 4 (1-l_6) n_6)^2) / Kc,
   each part taken as 0 when negative (the samplers are independent). */
int orc_finals4min(uint64_t K, const uint64_t hits[7], uint64_t gamma, uint64_t lambda3, uint64_t Kc,
                   const uint64_t hits_min[10], uint64_t gamma_min, int mix, double est[6], double var[6]) {
  if (!hits || !hits_min || !est || !var || (K == 0 && Kc == 0)) return ORC_E_ARG;
  if (mix != ORC_MIX_POOLED && mix != ORC_MIX_PAPER) return ORC_E_ARG;
  const double Kd = (double)K, Kcd = (double)Kc, G = (double)gamma, Gc = (double)gamma_min;
  double p[7] = {0}, q[7] = {0}, nhat[7] = {0}, ncheck[7] = {0}, lam[7], A5 = 0.0;
  for (int i = 0; i < 6; ++i) { est[i] = 0.0; var[i] = 0.0; }
  for (int i = 0; i < 7; ++i) lam[i] = 1.0;
  if (K > 0 && gamma > 0)
    for (int i = 1; i <= 6; ++i) {
      if (PHI4_PATH[i] == 0) continue;
      p[i] = 2.0 * (double)PHI4_PATH[i] / G;
      nhat[i] = (double)hits[i] / (Kd * p[i]);
    }
  if (Kc > 0 && gamma_min > 0) {
    q[3] = 2.0 / Gc; q[5] = 2.0 / Gc; q[6] = 6.0 / Gc;
    ncheck[3] = (double)hits_min[3] * Gc / (2.0 * Kcd);
    ncheck[6] = (double)hits_min[6] * Gc / (6.0 * Kcd);
    ncheck[5] = Gc / Kcd * ((double)hits_min[7] / 2.0 + (double)hits_min[8] / 4.0 + (double)hits_min[9] / 6.0);
    A5 = Gc * Gc / Kcd * ((double)hits_min[7] / 4.0 + (double)hits_min[8] / 16.0 + (double)hits_min[9] / 36.0);
  }
  /* n_1, n_4: MOSS-4 alone (Theorems 2 and 3) */
  for (int i = 1; i <= 4; i += 3) {
    if (p[i] == 0.0) continue;
    est[i - 1] = nhat[i];
    double v = nhat[i] / Kd * (1.0 / p[i] - nhat[i]);
    var[i - 1] = v > 0.0 ? v : 0.0;
  }
  for (int i = 3; i <= 6; ++i) {
    if (i == 4) continue;
    double a = Kd * p[i], b = Kcd * q[i], D = a + b;
    if (D == 0.0) continue;
    double l = a / D;
    double e = l * nhat[i] + (1.0 - l) * ncheck[i];
    double v1 = p[i] > 0.0 ? e / Kd * (1.0 / p[i] - e) : 0.0;
    double Ai = i == 5 ? A5 : (q[i] > 0.0 ? e / q[i] : 0.0);
    double v2 = q[i] > 0.0 ? (Ai - e * e) / Kcd : 0.0;
    if (v1 < 0.0) v1 = 0.0;
    if (v2 < 0.0) v2 = 0.0;
    double v;
    if (mix == ORC_MIX_PAPER && p[i] > 0.0 && q[i] > 0.0 && v1 + v2 > 0.0) {
      l = v2 / (v1 + v2);
      e = l * nhat[i] + (1.0 - l) * ncheck[i];
      v = v1 * v2 / (v1 + v2);
    } else {
      v = l * l * v1 + (1.0 - l) * (1.0 - l) * v2;
    }
    lam[i] = l;
    est[i - 1] = e;
    var[i - 1] = v > 0.0 ? v : 0.0;
  }
  double n4 = est[3], n5 = est[4], n6 = est[5];
  est[1] = (double)lambda3 - n4 - 2.0 * n5 - 4.0 * n6;
  double X = 0.0, Y = 0.0;
  if (p[4] > 0.0) {
    double s = n4 + 2.0 * lam[5] * n5 + 4.0 * lam[6] * n6;
    X = (n4 / p[4] + 4.0 * lam[5] * lam[5] * n5 / p[5] + 16.0 * lam[6] * lam[6] * n6 / p[6] - s * s) / Kd;
    if (X < 0.0) X = 0.0;
  }
  if (q[6] > 0.0) {
    double m5 = 1.0 - lam[5], m6 = 1.0 - lam[6];
    double t = 2.0 * m5 * n5 + 4.0 * m6 * n6;
    Y = (4.0 * m5 * m5 * A5 + 16.0 * m6 * m6 * (n6 / q[6]) - t * t) / Kcd;
    if (Y < 0.0) Y = 0.0;
  }
  var[1] = X + Y;
  return ORC_OK;
}

int orc_estimate4min(const orc_graph *g, uint64_t n_samples, uint64_t seed, int mix, int nthreads,
                     orc_result *res) {
  if (!g || !res || n_samples < 2) return ORC_E_ARG;
  memset(res, 0, sizeof(*res));
  uint64_t K = (n_samples + 1) / 2, Kc = n_samples / 2;
  res->k = 4; res->n_motifs = 6; res->K[0] = K; res->K[1] = Kc;
  int st = orc_run(g, ORC_MOSS4, seed, 0, K, nthreads, res->hits[0]);
  if (st) return st;
  st = orc_run(g, ORC_MOSS4MIN, seed, 0, Kc, nthreads, res->hits[1]);
  if (st) return st;
  return orc_finals4min(K, res->hits[0], g->tot.gamma, g->tot.lambda3, Kc, res->hits[1], g->tot.gamma_min, mix,
                        res->estimate, res->variance);
}

/* Theorem 1: an estimate is asymptotically normal around the count, so
   P(|est - n| >= z sqrt(Var)) -> P(|Z| >= z) = erfc(z / sqrt 2).  (The theorem prints
   the one-sided tail; the two-sided event needs both.) */
double orc_normal_two_sided(double delta) {
  double lo = 0.0, hi = 40.0;
  for (int it = 0; it < 200; ++it) {
    double mid = lo + (hi - lo) / 2.0;
    if (erfc(mid / sqrt(2.0)) > delta) lo = mid; else hi = mid;
  }
  return (lo + hi) / 2.0;
}

int orc_plan_budget(const orc_result *pilot, double eps, double delta, uint32_t motif_mask, uint64_t budget[21],
                    uint64_t *max_budget) {
  if (!pilot || !budget || !max_budget || !(eps > 0.0) || !(delta > 0.0) || !(delta < 1.0)) return ORC_E_ARG;
  if (pilot->n_motifs != 6 && pilot->n_motifs != 21) return ORC_E_ARG;
  double z = orc_normal_two_sided(delta);
  double Kp = (double)(pilot->K[0] + pilot->K[1]);
  *max_budget = 0;
  for (int i = 0; i < 21; ++i) {
    budget[i] = 0;
    if (i >= pilot->n_motifs) continue;
    double e = pilot->estimate[i];
    if (!(e > 0.0)) continue;
    double num = z * z * pilot->variance[i] * Kp;
    double den = eps * eps * e * e;
    double kk = num / den;
    uint64_t Ki;
    if (!(kk > 1.0)) Ki = 1;
    else if (kk >= 18446744073709549568.0) Ki = UINT64_MAX;
    else Ki = (uint64_t)ceil(kk);
    budget[i] = Ki;
    if ((motif_mask == 0 || (motif_mask >> i & 1)) && Ki > *max_budget) *max_budget = Ki;
  }
  return ORC_OK;
}

int orc_concentrations(const orc_result *r, double omega[21]) {
  if (!r || !omega || (r->n_motifs != 6 && r->n_motifs != 21)) return ORC_E_ARG;
  double sum = 0.0;
  for (int i = 0; i < r->n_motifs; ++i) sum += r->estimate[i];
  for (int i = 0; i < 21; ++i) omega[i] = (i < r->n_motifs && sum != 0.0) ? r->estimate[i] / sum : 0.0;
  return ORC_OK;
}

int orc_estimate_to_precision(const orc_graph *g, int k, int with_min, double eps, double delta, uint32_t motif_mask,
                              uint64_t pilot_samples, uint64_t pilot_seed, uint64_t max_samples, uint64_t seed,
                              int mix, int nthreads, orc_result *res, uint64_t *final_samples) {
  if (!g || !res || !final_samples || (k != 4 && k != 5) || (with_min && k != 4)) return ORC_E_ARG;
  uint64_t least = (k == 4 && !with_min) ? 1 : 2;
  if (pilot_samples < least || max_samples < least) return ORC_E_ARG;
  orc_result pilot;
  int st = with_min ? orc_estimate4min(g, pilot_samples, pilot_seed, mix, nthreads, &pilot)
                    : orc_estimate(g, k, pilot_samples, pilot_seed, mix, nthreads, &pilot);
  if (st) return st;
  uint64_t budget[21], K;
  st = orc_plan_budget(&pilot, eps, delta, motif_mask, budget, &K);
  if (st) return st;
  if (K == 0) K = pilot_samples;
  if (K < least) K = least;
  if (K > max_samples) K = max_samples;
  *final_samples = K;
  return with_min ? orc_estimate4min(g, K, seed, mix, nthreads, res) : orc_estimate(g, k, K, seed, mix, nthreads, res);
}

int orc_estimate(const orc_graph *g, int k, uint64_t n_samples, uint64_t seed, int mix, int nthreads,
                 orc_result *res) {
  if (!g || !res) return ORC_E_ARG;
  memset(res, 0, sizeof(*res));
  if (k == 4) {
    if (n_samples == 0) return ORC_E_ARG;
    res->k = 4; res->n_motifs = 6; res->K[0] = n_samples;
    int st = orc_run(g, ORC_MOSS4, seed, 0, n_samples, nthreads, res->hits[0]);
    if (st) return st;
    return orc_finals4(n_samples, res->hits[0], g->tot.gamma, g->tot.lambda3, res->estimate, res->variance);
  }
  if (k == 5) {
    if (n_samples < 2) return ORC_E_ARG;
    uint64_t K1 = (n_samples + 1) / 2, K2 = n_samples / 2; /* K1 = K2 up to one sample (Sec 5.1.4) */
    res->k = 5; res->n_motifs = 21; res->K[0] = K1; res->K[1] = K2;
    int st = orc_run(g, ORC_T5, seed, 0, K1, nthreads, res->hits[0]);
    if (st) return st;
    st = orc_run(g, ORC_PATH5, seed, 0, K2, nthreads, res->hits[1]);
    if (st) return st;
    return orc_finals5(K1, K2, res->hits[0], res->hits[1], g->tot.gamma1, g->tot.gamma2, g->tot.lambda4,
                       mix, res->estimate, res->variance, NULL);
  }
  return ORC_E_ARG;
}

/* ------------------------------------------------------------------------ */
/* Exact counts by enumerating every connected induced k-node subgraph once  */
/* (the ESU procedure of Wernicke, "Efficient detection of network motifs",   */
/* 2006): from each start vertex s, grow the node set only with vertices      */
/* larger than s that are exclusive neighbours of the newly added vertex.     */
/* This is the plain definition n_i = |C_i| of Section 2.                      */
/* ------------------------------------------------------------------------ */
typedef struct {
  const orc_graph *g;
  int k;
  int32_t sub[5];
  int32_t *ext[6];   /* ext[sz]: extension set while the subgraph has sz nodes */
  uint64_t *counts;
} esu_state;

static int in_closed_nbhd(const esu_state *st, int sz, int32_t x) {
  for (int i = 0; i < sz; ++i)
    if (st->sub[i] == x || is_adj(st->g, st->sub[i], x, NULL)) return 1;
  return 0;
}

static void esu_extend(esu_state *st, int sz, int level, int ext_len, int32_t start) {
  if (sz == st->k) {
    int mask = 0, p = 0;
    for (int i = 0; i < st->k; ++i)
      for (int j = i + 1; j < st->k; ++j, ++p)
        if (is_adj(st->g, st->sub[i], st->sub[j], NULL)) mask |= 1 << p;
    int c = st->k == 4 ? class4_of_mask[mask] : class5_of_mask[mask];
    if (c > 0) ++st->counts[c];
    return;
  }
  int32_t *ext = st->ext[level];
  while (ext_len > 0) {
    int32_t w = ext[--ext_len];
    int32_t *next = st->ext[level + 1];
    int nl = 0;
    for (int i = 0; i < ext_len; ++i) next[nl++] = ext[i];
    for (int64_t e = st->g->rp[w]; e < st->g->rp[w + 1]; ++e) {
      int32_t x = st->g->col[e];
      if (x <= start) continue;
      if (in_closed_nbhd(st, sz, x)) continue;
      next[nl++] = x;
    }
    st->sub[sz] = w;
    esu_extend(st, sz + 1, level + 1, nl, start);
  }
}

/* One worker of the enumeration: the start vertices s = first, first + step, ... */
typedef struct {
  const orc_graph *g;
  int k, first, step, status;
  uint64_t counts[22];
} esu_job;

static void *esu_run(void *arg) {
  esu_job *job = (esu_job *)arg;
  const orc_graph *g = job->g;
  int32_t dmax = 0;
  for (int32_t v = 0; v < g->n; ++v) if (degree(g, v) > dmax) dmax = degree(g, v);
  size_t cap = (size_t)job->k * (size_t)(dmax + 1) + 1;
  esu_state st;
  memset(&st, 0, sizeof(st));
  st.g = g; st.k = job->k; st.counts = job->counts;
  for (int i = 0; i < 6; ++i) {
    st.ext[i] = (int32_t *)malloc(cap * sizeof(int32_t));
    if (!st.ext[i]) {
      for (int j = 0; j < i; ++j) free(st.ext[j]);
      job->status = ORC_E_NOMEM;
      return NULL;
    }
  }
  for (int32_t s = job->first; s < g->n; s += job->step) {
    int len = 0;
    for (int64_t e = g->rp[s]; e < g->rp[s + 1]; ++e)
      if (g->col[e] > s) st.ext[1][len++] = g->col[e];
    st.sub[0] = s;
    esu_extend(&st, 1, 1, len, s);
  }
  for (int i = 0; i < 6; ++i) free(st.ext[i]);
  job->status = ORC_OK;
  return NULL;
}

/* Every CIS is enumerated exactly once, from its smallest vertex; the start vertices
   are dealt to `nthreads` workers in turn and their counts added. */
int orc_count_cis(const orc_graph *g, int k, int nthreads, uint64_t counts[22]) {
  if (!g || !counts || (k != 4 && k != 5)) return ORC_E_ARG;
  if (nthreads < 1) nthreads = 1;
  esu_job *jobs = (esu_job *)calloc((size_t)nthreads, sizeof(esu_job));
  pthread_t *tids = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
  if (!jobs || !tids) { free(jobs); free(tids); return ORC_E_NOMEM; }
  for (int t = 0; t < nthreads; ++t) {
    jobs[t].g = g; jobs[t].k = k; jobs[t].first = t; jobs[t].step = nthreads;
  }
  for (int t = 1; t < nthreads; ++t) pthread_create(&tids[t], NULL, esu_run, &jobs[t]);
  esu_run(&jobs[0]);
  for (int t = 1; t < nthreads; ++t) pthread_join(tids[t], NULL);
  int status = ORC_OK;
  memset(counts, 0, 22 * sizeof(uint64_t));
  for (int t = 0; t < nthreads; ++t) {
    if (jobs[t].status != ORC_OK) status = jobs[t].status;
    for (int c = 0; c < 22; ++c) counts[c] += jobs[t].counts[c];
  }
  free(jobs); free(tids);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Exact 4-node counts through non-induced patterns.  With N_P4, N_star, N_C4, */
/* N_paw, N_diamond, N_K4 the numbers of (not necessarily induced) copies, and */
/* c[j][i] the number of copies of pattern j inside motif M_i^(4):             */
/*   N_P4 = n1 + 4n3 + 2n4 + 6n5 + 12n6   (the phi^(1) row of Section 4.1.2)   */
/*   N_star = n2 + n4 + 2n5 + 4n6         (the phi^(2) row, Eq. n2)            */
/*   N_C4 = n3 + n5 + 3n6,  N_paw = n4 + 4n5 + 12n6,  N_diamond = n5 + 6n6,     */
/*   N_K4 = n6;                                                                */
/* the system is triangular and solved from n6 up.  The pattern counts use    */
/* t_e (triangles on edge e): T = sum t_e / 3, N_P4 = Gamma/2 - 3T,           */
/* N_paw = sum_v T_v (d_v - 2), N_diamond = sum_e C(t_e, 2), N_C4 = half of    */
/* sum over node pairs of C(common neighbours, 2), N_K4 by listing the common */
/* neighbours of each edge.                                                   */
/* ------------------------------------------------------------------------ */
static int64_t row_find(const orc_graph *g, int32_t a, int32_t b) {
  int64_t lo = g->rp[a], hi = g->rp[a + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (g->col[mid] == b) return mid;
    if (g->col[mid] < b) lo = mid + 1; else hi = mid;
  }
  return -1;
}

int orc_count4_exact(const orc_graph *g, uint64_t counts[7]) {
  if (!g || !counts) return ORC_E_ARG;
  memset(counts, 0, 7 * sizeof(uint64_t));
  int32_t n = g->n;
  uint64_t *te = (uint64_t *)calloc((size_t)g->nnz + 1, sizeof(uint64_t)); /* per CSR entry */
  uint32_t *cnt = (uint32_t *)calloc((size_t)n + 1, sizeof(uint32_t));
  int32_t *touched = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
  int32_t *common = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
  if (!te || !cnt || !touched || !common) { free(te); free(cnt); free(touched); free(common); return ORC_E_NOMEM; }
  u128 tri3 = 0, diamonds = 0, paws = 0, c4 = 0, k4 = 0;
  /* triangles per edge: common neighbours of v and u (v < u) by merging the sorted rows */
  for (int32_t v = 0; v < n; ++v) {
    for (int64_t e = g->rp[v]; e < g->rp[v + 1]; ++e) {
      int32_t u = g->col[e];
      if (u <= v) continue;
      int64_t i = g->rp[v], j = g->rp[u];
      int nc = 0;
      while (i < g->rp[v + 1] && j < g->rp[u + 1]) {
        if (g->col[i] == g->col[j]) { common[nc++] = g->col[i]; ++i; ++j; }
        else if (g->col[i] < g->col[j]) ++i; else ++j;
      }
      te[e] = (uint64_t)nc;
      te[row_find(g, u, v)] = (uint64_t)nc;
      tri3 += (u128)nc;
      diamonds += (u128)nc * (u128)(nc > 0 ? nc - 1 : 0) / 2;
      /* 4-cliques {v, u, x, y} with u < x < y counted once at their two smallest members */
      for (int a = 0; a < nc; ++a) {
        if (common[a] <= u) continue;
        for (int b = a + 1; b < nc; ++b)
          if (row_find(g, common[a], common[b]) >= 0) ++k4;
      }
    }
  }
  /* paws: triangles at v times the d_v - 2 other neighbours */
  for (int32_t v = 0; v < n; ++v) {
    u128 tv2 = 0; /* 2 T_v = sum over v's edges of t_e */
    for (int64_t e = g->rp[v]; e < g->rp[v + 1]; ++e) tv2 += te[e];
    int64_t dv = g->rp[v + 1] - g->rp[v];
    if (dv >= 2) paws += (tv2 / 2) * (u128)(dv - 2);
  }
  /* 4-cycles: for each a, count 2-paths a - x - b to every b > a */
  for (int32_t a = 0; a < n; ++a) {
    int nt = 0;
    for (int64_t e = g->rp[a]; e < g->rp[a + 1]; ++e) {
      int32_t x = g->col[e];
      for (int64_t f = g->rp[x]; f < g->rp[x + 1]; ++f) {
        int32_t b = g->col[f];
        if (b <= a) continue;
        if (cnt[b]++ == 0) touched[nt++] = b;
      }
    }
    for (int i = 0; i < nt; ++i) {
      uint64_t c = cnt[touched[i]];
      c4 += (u128)c * (c - 1) / 2;
      cnt[touched[i]] = 0;
    }
  }
  c4 /= 2; /* each 4-cycle has two diagonals */
  free(te); free(cnt); free(touched); free(common);
  u128 T = tri3 / 3;
  u128 p4 = (u128)g->tot.gamma / 2 - 3 * T;
  u128 star = g->tot.lambda3;
  /* triangular solve; every count is non-negative in exact arithmetic */
  u128 n6 = k4;
  u128 n5 = diamonds - 6 * n6;
  u128 n4 = paws - 4 * n5 - 12 * n6;
  u128 n3 = c4 - n5 - 3 * n6;
  u128 n2 = star - n4 - 2 * n5 - 4 * n6;
  u128 n1 = p4 - 4 * n3 - 2 * n4 - 6 * n5 - 12 * n6;
  u128 res[7] = {0, n1, n2, n3, n4, n5, n6};
  for (int i = 1; i <= 6; ++i) {
    if (!fits(res[i])) return ORC_E_OVERFLOW;
    counts[i] = (uint64_t)res[i];
  }
  return ORC_OK;
}

int orc_line_count(const orc_graph *g, int sampler, uint64_t seed, uint64_t k0, uint64_t k1,
                   double *mean_lines) {
  if (!g || !mean_lines || k1 <= k0) return ORC_E_ARG;
  reads *rec = (reads *)malloc(sizeof(reads));
  if (!rec) return ORC_E_NOMEM;
  double total = 0.0;
  int32_t nodes[5];
  for (uint64_t k = k0; k < k1; ++k) {
    rec->n = 0;
    int c = sample_one(g, sampler, seed, k, nodes, rec);
    if (c < 0) { free(rec); return c; }
    total += rec->n;
  }
  free(rec);
  *mean_lines = total / (double)(k1 - k0);
  return ORC_OK;
}
