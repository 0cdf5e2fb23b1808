// Estimator finals in double precision (host).
//
// MOSS-4, Section 4.1.2 / Theorems 2-3:
//   p_i = 2 phi^(1)_i / Gamma, phi^(1) = (1, 0, 4, 2, 6, 12)
//   n_i = m_i / (K p_i), i in {1,3,4,5,6};   n_2 = Lambda_3 - n_4 - 2 n_5 - 4 n_6
//   Var(n_i) = n_i / K (1/p_i - n_i)
//   Var(n_2) = (n_4/p_4 + 4 n_5/p_5 + 16 n_6/p_6 - (n_4 + 2 n_5 + 4 n_6)^2) / K
// MOSS-5, Sections 5.1.1-5.1.3 / Theorems 6-10, for sampler l (1 = T-5, 2 = Path-5):
//   p^(l)_i = 2 phi^(l)_i / Gamma^(l)   (Table 2)
//   mix weights lambda^(l)_i: pooled (default) K_l p^(l)_i / sum_l K_l p^(l)_i, which
//   turns the mix into (m^(1)_i + m^(2)_i) / (K_1 p^(1)_i + K_2 p^(2)_i); or the paper's
//   inverse-variance weights with Var(eta^(l)_i) = eta_i / K_l (1/p^(l)_i - eta_i) taken at
//   the pooled estimate.  Classes seen by one sampler only get weight 1 on it.
//   Cov(eta_i, eta_j) = -eta_i eta_j sum_l lambda^(l)_i lambda^(l)_j / K_l (i != j)
//   eta_2 = Lambda_4 - sum_{i in Omega_3*} phi^(3)_i eta_i,
//   Var(eta_2) = sum_{i,j in Omega_3*} phi^(3)_i phi^(3)_j Cov(eta_i, eta_j)
// MOSS-4 with MOSS-4Min (k = 4, MOSS_K4_MIN; Section 4.2, Theorems 1, 4, 5):
//   MOSS-4Min draws each ordered (w, v, u, r) with w above u and r above v with
//   probability 1/check-Gamma, so a CIS s is drawn with probability c(s)/check-Gamma
//   (c = 2 for the 4-cycle, 6 for the 4-clique, 2, 4 or 6 for a diamond, counted per
//   sample in hits[1][7..9]).  Per-sample weights give
//     n'_i = (check-Gamma / K') sum_c m_{i,c} / c,  Var = (A_i - n_i^2) / K',
//     A_i = sum_{s in C_i} check-Gamma / c(s), for the diamond estimated by
//     (check-Gamma^2 / K') sum_c m_{5,c} / c^2, for the others n_i / q_i,
//   q_3 = 2 / check-Gamma, q_5 = 2 / check-Gamma (fixed weight only), q_6 = 6 / check-Gamma.
//   n_3, n_5, n_6 mix MOSS-4 and MOSS-4Min with lambda_i = K p_i / (K p_i + K' q_i)
//   (pooled; variances at the mixed value) or V'_i / (V_i + V'_i) (paper, variances
//   at the pooled value); n_1, n_4 are MOSS-4's; n_2 = Lambda_3 - n_4 - 2 n_5 - 4 n_6
//   with Var = MOSS-4's share (n_4/p_4 + 4 l5^2 n_5/p_5 + 16 l6^2 n_6/p_6
//   - (n_4 + 2 l5 n_5 + 4 l6 n_6)^2) / K plus MOSS-4Min's share (4 (1-l5)^2 A_5
//   + 16 (1-l6)^2 A_6 - (2 (1-l5) n_5 + 4 (1-l6) n_6)^2) / K', each at least 0.
// The unknown counts inside the variance formulas are replaced by the estimates;
// reported variances are clamped at zero.
#include <cmath>
#include <cstdint>
#include <cstring>

#include "internal.h"

namespace {

constexpr int kPhi4[7] = {0, 1, 0, 4, 2, 6, 12};
// Table 2, rows phi^(1) (forks), phi^(2) (4-paths), phi^(3) (4-stars); index 0 unused
constexpr int kPhi5[3][22] = {
    {0, 0, 0, 1, 1, 2, 0, 2, 2, 4, 4, 5, 4, 6, 10, 9, 12, 10, 20, 20, 36, 60},
    {0, 1, 0, 0, 2, 2, 5, 1, 0, 4, 7, 2, 4, 6, 10, 6, 6, 14, 24, 18, 36, 60},
    {0, 0, 1, 0, 0, 0, 0, 0, 1, 0, 0, 1, 1, 0, 1, 1, 2, 0, 1, 2, 3, 5},
};

double nonneg(double x) { return x > 0.0 ? x : 0.0; }

void finals4(moss_result* r) {
  const double K = (double)r->K[0];
  const uint64_t G = r->gamma[0];
  double p[7] = {};
  double n[7] = {};
  for (int i = 1; i <= 6; ++i) {
    if (kPhi4[i] == 0 || G == 0) continue;
    p[i] = 2.0 * kPhi4[i] / (double)G;
    n[i] = (double)r->hits[0][i] / (K * p[i]);
    r->estimate[i - 1] = n[i];
    r->variance[i - 1] = nonneg(n[i] / K * (1.0 / p[i] - n[i]));
  }
  r->estimate[1] = (double)r->lambda - n[4] - 2.0 * n[5] - 4.0 * n[6];
  if (G != 0) {
    const double s = n[4] + 2.0 * n[5] + 4.0 * n[6];
    r->variance[1] = nonneg((n[4] / p[4] + 4.0 * n[5] / p[5] + 16.0 * n[6] / p[6] - s * s) / K);
  }
}

void finals4_min(moss_result* r) {
  const double K = (double)r->K[0], Kc = (double)r->K[1];
  const uint64_t G = r->gamma[0], Gc = r->gamma[1];
  const uint64_t* h = r->hits[0];
  const uint64_t* hm = r->hits[1];
  double p[7] = {}, q[7] = {}, a4[7] = {}, amin[7] = {}, lam[7] = {1, 1, 1, 1, 1, 1, 1};
  if (G != 0)
    for (int i = 1; i <= 6; ++i)
      if (kPhi4[i] != 0) {
        p[i] = 2.0 * kPhi4[i] / (double)G;
        a4[i] = (double)h[i] / (K * p[i]);
      }
  double A5 = 0.0;
  if (Gc != 0) {
    const double gc = (double)Gc;
    q[3] = 2.0 / gc;
    q[5] = 2.0 / gc;
    q[6] = 6.0 / gc;
    amin[3] = (double)hm[3] * gc / (2.0 * Kc);
    amin[6] = (double)hm[6] * gc / (6.0 * Kc);
    amin[5] = gc / Kc * ((double)hm[7] / 2.0 + (double)hm[8] / 4.0 + (double)hm[9] / 6.0);
    A5 = gc * gc / Kc * ((double)hm[7] / 4.0 + (double)hm[8] / 16.0 + (double)hm[9] / 36.0);
  }
  double n[7] = {};
  for (int i : {1, 4}) {
    if (p[i] == 0.0) continue;
    n[i] = a4[i];
    r->variance[i - 1] = nonneg(n[i] / K * (1.0 / p[i] - n[i]));
  }
  for (int i : {3, 5, 6}) {
    const double w4 = K * p[i], wmin = Kc * q[i];
    if (w4 + wmin == 0.0) continue;
    double l = w4 / (w4 + wmin);
    double est = l * a4[i] + (1.0 - l) * amin[i];
    const double v1 = p[i] > 0.0 ? nonneg(est / K * (1.0 / p[i] - est)) : 0.0;
    const double Ai = i == 5 ? A5 : (q[i] > 0.0 ? est / q[i] : 0.0);
    const double v2 = q[i] > 0.0 ? nonneg((Ai - est * est) / Kc) : 0.0;
    double var;
    if ((r->flags & MOSS_MIX_PAPER) && p[i] > 0.0 && q[i] > 0.0 && v1 + v2 > 0.0) {
      l = v2 / (v1 + v2);
      est = l * a4[i] + (1.0 - l) * amin[i];
      var = v1 * v2 / (v1 + v2);
    } else {
      var = l * l * v1 + (1.0 - l) * (1.0 - l) * v2;
    }
    lam[i] = l;
    n[i] = est;
    r->variance[i - 1] = nonneg(var);
  }
  for (int i = 1; i <= 6; ++i) r->estimate[i - 1] = n[i];
  r->estimate[1] = (double)r->lambda - n[4] - 2.0 * n[5] - 4.0 * n[6];
  double v4 = 0.0, vmin = 0.0;
  if (p[4] > 0.0) {
    const double s = n[4] + 2.0 * lam[5] * n[5] + 4.0 * lam[6] * n[6];
    v4 = nonneg((n[4] / p[4] + 4.0 * lam[5] * lam[5] * n[5] / p[5] + 16.0 * lam[6] * lam[6] * n[6] / p[6] - s * s) / K);
  }
  if (q[6] > 0.0) {
    const double m5 = 1.0 - lam[5], m6 = 1.0 - lam[6];
    const double t = 2.0 * m5 * n[5] + 4.0 * m6 * n[6];
    vmin = nonneg((4.0 * m5 * m5 * A5 + 16.0 * m6 * m6 * (n[6] / q[6]) - t * t) / Kc);
  }
  r->variance[1] = v4 + vmin;
}

void finals5(moss_result* r) {
  const double K[2] = {(double)r->K[0], (double)r->K[1]};
  double lam[2][22] = {};
  double eta[22] = {};
  for (int i = 1; i <= 21; ++i) {
    if (i == 2) continue;
    double p[2];
    for (int l = 0; l < 2; ++l)
      p[l] = (kPhi5[l][i] > 0 && r->gamma[l] > 0) ? 2.0 * kPhi5[l][i] / (double)r->gamma[l] : 0.0;
    const double denom = K[0] * p[0] + K[1] * p[1];
    if (denom == 0.0) continue;
    const double pooled = ((double)r->hits[0][i] + (double)r->hits[1][i]) / denom;
    double l1 = K[0] * p[0] / denom, l2 = K[1] * p[1] / denom;
    const double v1 = p[0] > 0.0 ? nonneg(pooled / K[0] * (1.0 / p[0] - pooled)) : 0.0;
    const double v2 = p[1] > 0.0 ? nonneg(pooled / K[1] * (1.0 / p[1] - pooled)) : 0.0;
    double est = pooled, var;
    if ((r->flags & MOSS_MIX_PAPER) && p[0] > 0.0 && p[1] > 0.0 && v1 + v2 > 0.0) {
      l1 = v2 / (v1 + v2);
      l2 = v1 / (v1 + v2);
      est = l1 * ((double)r->hits[0][i] / (K[0] * p[0])) + l2 * ((double)r->hits[1][i] / (K[1] * p[1]));
      var = v1 * v2 / (v1 + v2);
    } else {
      var = l1 * l1 * v1 + l2 * l2 * v2;
    }
    lam[0][i] = l1;
    lam[1][i] = l2;
    eta[i] = est;
    r->estimate[i - 1] = est;
    r->variance[i - 1] = nonneg(var);
  }
  double sub = 0.0;
  for (int i = 1; i <= 21; ++i)
    if (i != 2 && kPhi5[2][i] > 0) sub += kPhi5[2][i] * eta[i];
  r->estimate[1] = (double)r->lambda - sub;
  double v = 0.0;
  for (int i = 1; i <= 21; ++i) {
    if (i == 2 || kPhi5[2][i] == 0) continue;
    for (int j = 1; j <= 21; ++j) {
      if (j == 2 || kPhi5[2][j] == 0) continue;
      const double c = i == j ? r->variance[i - 1]
                              : -eta[i] * eta[j] * (lam[0][i] * lam[0][j] / K[0] + lam[1][i] * lam[1][j] / K[1]);
      v += (double)kPhi5[2][i] * kPhi5[2][j] * c;
    }
  }
  r->variance[1] = nonneg(v);
}

}  // namespace

extern "C" moss_status moss_finals(moss_result* r) {
  if (!r) return MOSS_E_ARG;
  std::memset(r->estimate, 0, sizeof(r->estimate));
  std::memset(r->variance, 0, sizeof(r->variance));
  if (r->flags & ~(MOSS_MIX_PAPER | MOSS_K4_MIN)) return MOSS_E_ARG;
  if (r->k == 4) {
    if (r->K[0] == 0) return MOSS_E_ARG;
    r->n_motifs = 6;
    if (r->flags & MOSS_K4_MIN) {
      if (r->K[1] == 0) return MOSS_E_ARG;
      finals4_min(r);
    } else {
      finals4(r);
    }
    return MOSS_OK;
  }
  if (r->k == 5) {
    if (r->K[0] == 0 || r->K[1] == 0 || (r->flags & MOSS_K4_MIN)) return MOSS_E_ARG;
    r->n_motifs = 21;
    finals5(r);
    return MOSS_OK;
  }
  return MOSS_E_ARG;
}

namespace {

// Two-sided normal quantile (Theorem 1's limit): the z with erfc(z / sqrt 2) = delta,
// by halving [0, 40] 200 times; erfc falls monotonically, so the root stays inside.
double two_sided_quantile(double delta) {
  double lo = 0.0, hi = 40.0;
  const double r2 = std::sqrt(2.0);
  for (int it = 0; it < 200; ++it) {
    const double mid = lo + (hi - lo) / 2.0;
    if (std::erfc(mid / r2) > delta) lo = mid;
    else hi = mid;
  }
  return (lo + hi) / 2.0;
}

}  // namespace

extern "C" moss_status moss_plan_budget(const moss_result* pilot, double eps, double delta, uint32_t motif_mask,
                                        uint64_t budget[21], uint64_t* max_budget) {
  if (!pilot || !budget || !max_budget || !(eps > 0.0) || !(delta > 0.0) || !(delta < 1.0)) return MOSS_E_ARG;
  if (pilot->n_motifs != 6 && pilot->n_motifs != 21) return MOSS_E_ARG;
  const double z = two_sided_quantile(delta);
  const double Kp = (double)(pilot->K[0] + pilot->K[1]);
  uint64_t best = 0;
  for (int i = 0; i < 21; ++i) {
    budget[i] = 0;
    const double e = pilot->estimate[i];
    if (i >= pilot->n_motifs || !(e > 0.0)) continue;
    // K_i from Var_i(K) = Var_i(K_p) K_p / K and z sqrt(Var_i(K)) <= eps e
    const double num = z * z * pilot->variance[i] * Kp;
    const double den = eps * eps * e * e;
    const double x = num / den;
    uint64_t Ki = 1;
    if (x >= 18446744073709549568.0) Ki = UINT64_MAX;  // largest double below 2^64
    else if (x > 1.0) Ki = (uint64_t)std::ceil(x);
    budget[i] = Ki;
    if ((motif_mask == 0 || ((motif_mask >> i) & 1u)) && Ki > best) best = Ki;
  }
  *max_budget = best;
  return MOSS_OK;
}

extern "C" moss_status moss_concentrations(const moss_result* r, double omega[21]) {
  if (!r || !omega || (r->n_motifs != 6 && r->n_motifs != 21)) return MOSS_E_ARG;
  double sum = 0.0;
  for (int i = 0; i < r->n_motifs; ++i) sum += r->estimate[i];
  for (int i = 0; i < 21; ++i) omega[i] = (i < r->n_motifs && sum != 0.0) ? r->estimate[i] / sum : 0.0;
  return MOSS_OK;
}
