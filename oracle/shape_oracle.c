/*
 * shape_oracle.c -- plain, slow, FP64 CPU reference for the importance-sampling
 * (IS) estimator of Gaussian molecular shape overlap (Tuzharov, Bochenkova,
 * Maximov, "Importance-Sampling Estimation of Gaussian Molecular Shape Overlap:
 * Exact Union Volumes and Confidence-Bounded Virtual Screening").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with the
 * HIP path.
 *
 * Every function computes its quantity straight from the definition in the
 * paper (section / equation named at each function), in double precision, with
 * no blocking, fusion or reordering beyond the definition.  Inputs arrive as
 * float32 (the canonical input representation) and are promoted to double.
 *
 * Readings of points the paper leaves open (stated where used):
 *   R1 Gaussian widths: unit-height atom Gaussians (Eq. occ) with
 *      alpha = kappa / (lambda R^2), kappa = pi (3/(4 pi))^(2/3).
 *   R2 Random numbers: one Philox4x32-10 block per sample point, counter
 *      (k mod 2^32, k div 2^32, mol_id, 0), key (seed mod 2^32, seed div 2^32).
 *      Words 1..3 give uniforms u = ((x >> 8) + 0.5) / 2^24 turned into standard
 *      normals by the inverse normal CDF; word 0 picks the mixture component
 *      through integer thresholds floor(2^32 * cumsum(v)/Z).
 *   R3 Symmetrised estimate = plain average of the A-sided and B-sided
 *      estimates (section "Importance-sampling estimator").
 *   R4 Sample variances use the n-1 denominator, two-pass.
 *   R5 Tanimoto standard error: the paper's delta-method expression (section
 *      "Confidence-bounded screening"); a full delta-method value that also
 *      propagates the self-overlap errors is reported beside it.
 *   R6 Adaptive screening: rounds of 256 samples per side (512 per pair); after
 *      each round stop when SE(T) <= tau or the pair total reaches the cap.
 *   R7 Pose: unnormalised quaternion q (rotation R(q/|q|)) and translation t
 *      acting on every centre of B about B's own origin.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as    */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with the  */
/* Weyl-sequence key schedule.                                               */
/* ------------------------------------------------------------------------- */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                      uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------- */
/* Inverse of the standard normal CDF, Phi(z) = erfc(-z/sqrt 2)/2, solved by  */
/* bracketed Newton iteration on the C library's erfc.  The lower half is     */
/* solved directly; the upper half by symmetry from 1-u (exact for the        */
/* uniforms used here).                                                       */
/* ------------------------------------------------------------------------- */
static double or_phi_cdf(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

double or_norm_inv(double u) {
  if (!(u > 0.0 && u < 1.0)) return NAN;
  if (u > 0.5) return -or_norm_inv(1.0 - u);
  if (u == 0.5) return 0.0;
  /* solve Phi(z) = u for z < 0 */
  double lo = -40.0, hi = 0.0;
  double z = -sqrt(-2.0 * log(u)); /* |z| over-estimate: Phi(z) < u here */
  if (z < lo) z = lo;
  for (int it = 0; it < 200; ++it) {
    double f = or_phi_cdf(z) - u;
    if (f > 0) hi = z; else lo = z;
    double dens = exp(-0.5 * z * z) / sqrt(2.0 * OR_PI);
    double zn = z - f / dens;
    if (!(zn > lo && zn < hi)) zn = 0.5 * (lo + hi); /* fall back to bisection */
    if (fabs(zn - z) <= 1e-16 * fabs(z) || hi - lo <= 1e-16 * fabs(z)) {
      z = zn;
      break;
    }
    z = zn;
  }
  return z;
}

/* ------------------------------------------------------------------------- */
/* Atom widths (Eq. occ): alpha = kappa/(lambda R^2), kappa = pi(3/4pi)^(2/3). */
/* ------------------------------------------------------------------------- */
void or_alpha_from_radius(const float* radius, int64_t n, double lambda,
                          float* alpha_out) {
  const double kappa = OR_PI * pow(3.0 / (4.0 * OR_PI), 2.0 / 3.0);
  for (int64_t i = 0; i < n; ++i) {
    double R = (double)radius[i];
    alpha_out[i] = (float)(kappa / (lambda * R * R));
  }
}

/* ------------------------------------------------------------------------- */
/* Molecule: centres and widths promoted to double, mixture weights           */
/* v_i = (pi/alpha_i)^(3/2), Z = sum v_i (section "Importance-sampling         */
/* estimator"), and the component-selection thresholds of reading R2.          */
/* ------------------------------------------------------------------------- */
typedef struct {
  int n;
  double* c;       /* [n][3] */
  double* alpha;   /* [n] */
  double* v;       /* [n] */
  uint32_t* thr;   /* [n-1] */
  double Z;
} or_mol;

static int or_mol_init(or_mol* M, int n, const float* xyz, const float* alpha) {
  M->n = n;
  M->c = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  M->alpha = (double*)malloc(sizeof(double) * (size_t)n);
  M->v = (double*)malloc(sizeof(double) * (size_t)n);
  M->thr = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 1 ? n - 1 : 1));
  if (!M->c || !M->alpha || !M->v || !M->thr) return -1;
  double Z = 0.0;
  for (int i = 0; i < n; ++i) {
    for (int d = 0; d < 3; ++d) M->c[3 * i + d] = (double)xyz[3 * i + d];
    M->alpha[i] = (double)alpha[i];
    double t = OR_PI / M->alpha[i];
    M->v[i] = t * sqrt(t);
    Z += M->v[i];
  }
  M->Z = Z;
  double cum = 0.0;
  for (int i = 0; i + 1 < n; ++i) {
    cum += M->v[i];
    double f = floor(4294967296.0 * (cum / Z));
    if (f > 4294967295.0) f = 4294967295.0;
    M->thr[i] = (uint32_t)f;
  }
  return 0;
}

static void or_mol_free(or_mol* M) {
  free(M->c); free(M->alpha); free(M->v); free(M->thr);
}

/* exported: weights, Z and thresholds of one molecule (for host-prep checks) */
int or_mol_prep(int n, const float* xyz, const float* alpha, double* v_out,
                double* Z_out, uint32_t* thr_out) {
  or_mol M;
  if (or_mol_init(&M, n, xyz, alpha)) return -1;
  for (int i = 0; i < n; ++i) v_out[i] = M.v[i];
  for (int i = 0; i + 1 < n; ++i) thr_out[i] = M.thr[i];
  *Z_out = M.Z;
  or_mol_free(&M);
  return 0;
}

/* Sample k of molecule M (reading R2): exact draw from q_M = m_M / Z_M: pick
 * component j with probability v_j/Z, then r ~ N(c_j, I/(2 alpha_j)). */
static int or_sample(const or_mol* M, uint32_t mol_id, uint64_t k, uint64_t seed,
                     double r[3]) {
  uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(k >> 32), mol_id, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t x[4];
  or_philox4x32_10(ctr, key, x);
  int j = 0;
  for (int i = 0; i + 1 < M->n; ++i)
    if (x[0] >= M->thr[i]) j++;
  double sd = 1.0 / sqrt(2.0 * M->alpha[j]);
  for (int d = 0; d < 3; ++d) {
    double u = ((double)(x[d + 1] >> 8) + 0.5) / 16777216.0;
    r[d] = M->c[3 * j + d] + or_norm_inv(u) * sd;
  }
  return j;
}

/* Antithetic sample k (section "Importance-sampling estimator": each Gaussian
 * draw c_j + L eps is paired with its reflection c_j - L eps): samples 2p and
 * 2p+1 share the component and normal draws of Philox block p and take the
 * signs + and -. */
static int or_sample_anti(const or_mol* M, uint32_t mol_id, uint64_t k, uint64_t seed,
                          double r[3]) {
  double c[3];
  int j = or_sample(M, mol_id, k >> 1, seed, r);
  if (k & 1) {
    for (int d = 0; d < 3; ++d) c[d] = M->c[3 * j + d];
    for (int d = 0; d < 3; ++d) r[d] = c[d] - (r[d] - c[d]);
  }
  return j;
}

/* exported: sample points of one molecule for counters k0..k0+n-1 */
int or_sample_points(int n_atoms, const float* xyz, const float* alpha,
                     uint32_t mol_id, uint64_t seed, uint64_t k0, int64_t n, int anti,
                     double* r_out, int32_t* comp_out) {
  or_mol M;
  if (or_mol_init(&M, n_atoms, xyz, alpha)) return -1;
  for (int64_t k = 0; k < n; ++k) {
    int j = anti ? or_sample_anti(&M, mol_id, k0 + (uint64_t)k, seed, r_out + 3 * k)
                 : or_sample(&M, mol_id, k0 + (uint64_t)k, seed, r_out + 3 * k);
    if (comp_out) comp_out[k] = j;
  }
  or_mol_free(&M);
  return 0;
}

/* Densities at r (Eqs. occ, union and the first-order sum):
 * o_i = exp(-alpha_i |r-c_i|^2), m = sum o_i, u = 1 - prod (1 - o_i). */
static void or_density(const or_mol* M, const double r[3], double* m, double* u) {
  double sm = 0.0, prod = 1.0;
  for (int i = 0; i < M->n; ++i) {
    double dx = r[0] - M->c[3 * i], dy = r[1] - M->c[3 * i + 1],
           dz = r[2] - M->c[3 * i + 2];
    double o = exp(-M->alpha[i] * (dx * dx + dy * dy + dz * dz));
    sm += o;
    prod *= (1.0 - o);
  }
  *m = sm;
  *u = 1.0 - prod;
}

/* exported: m and u of a molecule at given points */
int or_densities(int n_atoms, const float* xyz, const float* alpha, int64_t n_pts,
                 const double* r, double* m_out, double* u_out) {
  or_mol M;
  if (or_mol_init(&M, n_atoms, xyz, alpha)) return -1;
  for (int64_t k = 0; k < n_pts; ++k) or_density(&M, r + 3 * k, m_out + k, u_out + k);
  or_mol_free(&M);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* One side of the estimator: samples from P, integrands for the pair (P, Q). */
/* Eq. union-is (bounded weight) and Eq. expectation / Eq. var (FO channel).   */
/* ------------------------------------------------------------------------- */
enum { F_PQ = 0, F_PP = 1, F_V = 2, F_FOPQ = 3, F_FOPP = 4, NF = 5 };

/* per-sample integrands for counters [k0, k1) into f[NF][k1-k0] */
static void or_side_integrands(const or_mol* P, const or_mol* Q, uint32_t id_p,
                               uint64_t seed, int64_t k0, int64_t k1, int anti, double* f) {
  int64_t n = k1 - k0;
  for (int64_t k = k0; k < k1; ++k) {
    double r[3], mP, uP, mQ, uQ;
    if (anti)
      or_sample_anti(P, id_p, (uint64_t)k, seed, r);
    else
      or_sample(P, id_p, (uint64_t)k, seed, r);
    or_density(P, r, &mP, &uP);
    or_density(Q, r, &mQ, &uQ);
    double w = (mP > 0.0) ? uP / mP : 0.0;
    int64_t i = k - k0;
    f[F_PQ * n + i] = w * uQ;
    f[F_PP * n + i] = w * uP;
    f[F_V * n + i] = w;
    f[F_FOPQ * n + i] = mQ;
    f[F_FOPP * n + i] = mP;
  }
}

typedef struct {
  double mean[NF];
  double var[NF];   /* sample variance, n-1 */
  double cov12;     /* sample covariance of f_PQ and f_PP, n-1 */
  int64_t n;
} or_side_stats;

/* Means over the n samples; variances (n-1) and the covariance of f_PQ and
 * f_PP over the independent terms: the samples themselves, or for
 * antithetic sampling the n/2 pair means g = (f(r_2p) + f(r_2p+1))/2,
 * stored as 2 var(g) so that SE = Z sqrt(var / n) = Z sqrt(var(g) / (n/2)). */
static void or_stats(const double* f, int64_t n, int anti, or_side_stats* s) {
  s->n = n;
  int64_t c = anti ? n / 2 : n;
  double* g = (double*)malloc(sizeof(double) * NF * (size_t)(c > 0 ? c : 1));
  for (int a = 0; a < NF; ++a)
    for (int64_t i = 0; i < c; ++i)
      g[a * c + i] = anti ? 0.5 * (f[a * n + 2 * i] + f[a * n + 2 * i + 1]) : f[a * n + i];
  for (int a = 0; a < NF; ++a) {
    double sum = 0.0;
    for (int64_t i = 0; i < c; ++i) sum += g[a * c + i];
    s->mean[a] = sum / (double)c;
    double ss = 0.0;
    for (int64_t i = 0; i < c; ++i) {
      double d = g[a * c + i] - s->mean[a];
      ss += d * d;
    }
    s->var[a] = (c > 1) ? ss / (double)(c - 1) * (double)n / (double)c : 0.0;
  }
  double cs = 0.0;
  for (int64_t i = 0; i < c; ++i)
    cs += (g[F_PQ * c + i] - s->mean[F_PQ]) * (g[F_PP * c + i] - s->mean[F_PP]);
  s->cov12 = (c > 1) ? cs / (double)(c - 1) * (double)n / (double)c : 0.0;
  free(g);
}

/* Result of one pair (all FP64). */
typedef struct {
  double O_ab, O_aa, O_bb, V_a, V_b, T;
  double se_O_ab, se_O_aa, se_O_bb, se_V_a, se_V_b, se_T, se_T_full;
  double O_ab_from_a, O_ab_from_b, Ofo_ab_is, Ofo_aa_is, Ofo_bb_is;
  int64_t n_a, n_b;
} or_result;

/* Pair combination: symmetrised overlap (R3), Tanimoto and its delta-method
 * standard errors (section "Confidence-bounded screening"; R5). */
static void or_combine(double Za, double Zb, const or_side_stats* A,
                       const or_side_stats* B, or_result* out) {
  double na = (double)A->n, nb = (double)B->n;
  double Xa = Za * A->mean[F_PQ], Xb = Zb * B->mean[F_PQ];
  double se_Xa = Za * sqrt(A->var[F_PQ] / na), se_Xb = Zb * sqrt(B->var[F_PQ] / nb);
  out->O_ab_from_a = Xa;
  out->O_ab_from_b = Xb;
  out->O_ab = 0.5 * (Xa + Xb);
  out->se_O_ab = 0.5 * sqrt(se_Xa * se_Xa + se_Xb * se_Xb);
  out->O_aa = Za * A->mean[F_PP];
  out->O_bb = Zb * B->mean[F_PP];
  out->se_O_aa = Za * sqrt(A->var[F_PP] / na);
  out->se_O_bb = Zb * sqrt(B->var[F_PP] / nb);
  out->V_a = Za * A->mean[F_V];
  out->V_b = Zb * B->mean[F_V];
  out->se_V_a = Za * sqrt(A->var[F_V] / na);
  out->se_V_b = Zb * sqrt(B->var[F_V] / nb);
  out->Ofo_ab_is = 0.5 * (Za * A->mean[F_FOPQ] + Zb * B->mean[F_FOPQ]);
  out->Ofo_aa_is = Za * A->mean[F_FOPP];
  out->Ofo_bb_is = Zb * B->mean[F_FOPP];
  double S = out->O_aa + out->O_bb;
  double D = S - out->O_ab;
  out->T = out->O_ab / D;
  out->se_T = fabs(S / (D * D)) * out->se_O_ab;
  double g_ab = S / (D * D), g_s = -out->O_ab / (D * D);
  double var_ab = out->se_O_ab * out->se_O_ab;
  double var_s = out->se_O_aa * out->se_O_aa + out->se_O_bb * out->se_O_bb;
  double cov = 0.5 * Za * Za * A->cov12 / na + 0.5 * Zb * Zb * B->cov12 / nb;
  double vt = g_ab * g_ab * var_ab + g_s * g_s * var_s + 2.0 * g_ab * g_s * cov;
  out->se_T_full = sqrt(vt > 0 ? vt : 0.0);
  out->n_a = A->n;
  out->n_b = B->n;
}

static int or_pair_estimate(const or_mol* A, const or_mol* B, uint32_t id_a,
                            uint32_t id_b, int64_t n_a, int64_t n_b, uint64_t seed, int anti,
                            or_result* out) {
  double* fa = (double*)malloc(sizeof(double) * NF * (size_t)n_a);
  double* fb = (double*)malloc(sizeof(double) * NF * (size_t)n_b);
  if (!fa || !fb) { free(fa); free(fb); return -1; }
  or_side_integrands(A, B, id_a, seed, 0, n_a, anti, fa);
  or_side_integrands(B, A, id_b, seed, 0, n_b, anti, fb);
  or_side_stats sa, sb;
  or_stats(fa, n_a, anti, &sa);
  or_stats(fb, n_b, anti, &sb);
  or_combine(A->Z, B->Z, &sa, &sb, out);
  free(fa); free(fb);
  return 0;
}

/* exported: single pair estimate */
int or_estimate(int na_atoms, const float* xyz_a, const float* alpha_a, uint32_t id_a,
                int nb_atoms, const float* xyz_b, const float* alpha_b, uint32_t id_b,
                int64_t n_a, int64_t n_b, uint64_t seed, int anti, double* out20) {
  if (na_atoms < 1 || nb_atoms < 1 || n_a < 2 || n_b < 2) return -2;
  if (anti && ((n_a & 1) || (n_b & 1) || n_a < 4 || n_b < 4)) return -2;
  or_mol A, B;
  if (or_mol_init(&A, na_atoms, xyz_a, alpha_a)) return -1;
  if (or_mol_init(&B, nb_atoms, xyz_b, alpha_b)) { or_mol_free(&A); return -1; }
  or_result r;
  int rc = or_pair_estimate(&A, &B, id_a, id_b, n_a, n_b, seed, anti, &r);
  memcpy(out20, &r, sizeof(double) * 18);
  out20[18] = (double)r.n_a;
  out20[19] = (double)r.n_b;
  or_mol_free(&A); or_mol_free(&B);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Screening: one query against listed library molecules (CSR layout).       */
/* mode 0: fixed n per side.  mode 1: adaptive rounds (R6).                    */
/* Outputs per pair (double): T, se_T, O_ab, O_aa, O_bb, n_used (pair total). */
/* ------------------------------------------------------------------------- */
int or_screen(int nq, const float* xyz_q, const float* alpha_q, uint32_t id_q,
              int32_t n_lib, const int32_t* lib_off, const float* lib_xyz,
              const float* lib_alpha, const uint32_t* lib_id, const int32_t* pairs,
              int32_t n_pairs, int mode, int64_t n_fixed, int64_t round_per_pair,
              int64_t cap_per_pair, double tau, uint64_t seed, int n_threads,
              const int32_t* n_start, int anti, double* out6) {
  /* the rules the rounds rely on: whole rounds of equal halves per side (of
   * even length for antithetic pairs), and a cap of whole rounds */
  if (nq < 1 || n_pairs < 0 || n_lib < 0) return -2;
  if (mode == 0) {
    if (n_fixed < 2 || (anti && (n_fixed < 4 || (n_fixed & 1)))) return -2;
  } else if (mode == 1) {
    if (round_per_pair < 2 || (round_per_pair & 1) || (anti && (round_per_pair & 3))) return -2;
    if (cap_per_pair < round_per_pair || cap_per_pair % round_per_pair) return -2;
    if (!(tau > 0.0) || !isfinite(tau)) return -2;
  } else {
    return -2;
  }
  or_mol Q;
  if (or_mol_init(&Q, nq, xyz_q, alpha_q)) return -1;
  int err = 0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
#endif
  for (int32_t p = 0; p < n_pairs; ++p) {
    int32_t m = pairs ? pairs[p] : p;
    if (m < 0 || m >= n_lib) {
      /* a pair index outside the library scores nothing */
      for (int j = 0; j < 5; ++j) out6[6 * (size_t)p + j] = NAN;
      out6[6 * (size_t)p + 5] = 0.0;
      continue;
    }
    int32_t a0 = lib_off[m], a1 = lib_off[m + 1];
    uint32_t idm = lib_id ? lib_id[m] : (uint32_t)m;
    or_mol B;
    if (or_mol_init(&B, a1 - a0, lib_xyz + 3 * (size_t)a0, lib_alpha + a0)) { err |= 1; continue; }
    or_result r;
    if (mode == 0) {
      if (or_pair_estimate(&Q, &B, id_q, idm, n_fixed, n_fixed, seed, anti, &r)) err |= 1;
    } else {
      int64_t side_round = round_per_pair / 2;
      int64_t max_side = cap_per_pair / 2;
      double* fa = (double*)malloc(sizeof(double) * NF * (size_t)max_side);
      double* fb = (double*)malloc(sizeof(double) * NF * (size_t)max_side);
      double* ta = (double*)malloc(sizeof(double) * NF * (size_t)max_side);
      double* tb = (double*)malloc(sizeof(double) * NF * (size_t)max_side);
      if (!fa || !fb || !ta || !tb) { err |= 1; free(fa); free(fb); free(ta); free(tb); or_mol_free(&B); continue; }
      int64_t n = 0;
      for (;;) {
        /* round: samples [n, n + side_round) on each side */
        double* ra = (double*)malloc(sizeof(double) * NF * (size_t)side_round);
        double* rb = (double*)malloc(sizeof(double) * NF * (size_t)side_round);
        if (!ra || !rb) { free(ra); free(rb); err |= 1; break; }
        or_side_integrands(&Q, &B, id_q, seed, n, n + side_round, anti, ra);
        or_side_integrands(&B, &Q, idm, seed, n, n + side_round, anti, rb);
        int64_t nn = n + side_round;
        /* re-pack [NF][nn] */
        for (int a = 0; a < NF; ++a) {
          for (int64_t i = 0; i < n; ++i) { ta[a * nn + i] = fa[a * n + i]; tb[a * nn + i] = fb[a * n + i]; }
          for (int64_t i = 0; i < side_round; ++i) {
            ta[a * nn + n + i] = ra[a * side_round + i];
            tb[a * nn + n + i] = rb[a * side_round + i];
          }
        }
        free(ra); free(rb);
        memcpy(fa, ta, sizeof(double) * NF * (size_t)nn);
        memcpy(fb, tb, sizeof(double) * NF * (size_t)nn);
        n = nn;
        or_side_stats sa, sb;
        or_stats(fa, n, anti, &sa);
        or_stats(fb, n, anti, &sb);
        or_combine(Q.Z, B.Z, &sa, &sb, &r);
        /* a seeded budget defers the first stop test until it is spent */
        if (n_start && 2 * n < (int64_t)n_start[p] && 2 * n < cap_per_pair) continue;
        if (r.se_T <= tau || 2 * n >= cap_per_pair) break;
      }
      free(fa); free(fb); free(ta); free(tb);
      if (n == 0) { or_mol_free(&B); continue; }
    }
    out6[6 * (size_t)p + 0] = r.T;
    out6[6 * (size_t)p + 1] = r.se_T;
    out6[6 * (size_t)p + 2] = r.O_ab;
    out6[6 * (size_t)p + 3] = r.O_aa;
    out6[6 * (size_t)p + 4] = r.O_bb;
    out6[6 * (size_t)p + 5] = (double)(r.n_a + r.n_b);
    or_mol_free(&B);
  }
  or_mol_free(&Q);
  return err ? -1 : 0;
}

/* ------------------------------------------------------------------------- */
/* Closed forms.                                                              */
/* ------------------------------------------------------------------------- */

/* Integral of a product of unit-height Gaussians exp(-a_i |r-c_i|^2) over R^3
 * (Gaussian product theorem, the building block of Eq. fo):
 * (pi/A)^(3/2) exp(-sum_{i<j} a_i a_j |c_i-c_j|^2 / A), A = sum a_i. */
static double or_gauss_product_integral(int k, const double* c, const double* a) {
  double A = 0.0;
  for (int i = 0; i < k; ++i) A += a[i];
  double e = 0.0;
  for (int i = 0; i < k; ++i)
    for (int j = i + 1; j < k; ++j) {
      double dx = c[3 * i] - c[3 * j], dy = c[3 * i + 1] - c[3 * j + 1],
             dz = c[3 * i + 2] - c[3 * j + 2];
      e += a[i] * a[j] * (dx * dx + dy * dy + dz * dz);
    }
  double t = OR_PI / A;
  return t * sqrt(t) * exp(-e / A);
}

/* Eq. fo: first-order overlap int m_A m_B. */
double or_fo_overlap(int na, const float* xyz_a, const float* alpha_a, int nb,
                     const float* xyz_b, const float* alpha_b) {
  double s = 0.0;
  for (int i = 0; i < na; ++i)
    for (int j = 0; j < nb; ++j) {
      double c[6], a[2];
      for (int d = 0; d < 3; ++d) { c[d] = xyz_a[3 * i + d]; c[3 + d] = xyz_b[3 * j + d]; }
      a[0] = alpha_a[i]; a[1] = alpha_b[j];
      s += or_gauss_product_integral(2, c, a);
    }
  return s;
}

/* int m_A m_B^2 = Z_A E_qA[m_B^2]: the second moment behind Eq. var. */
double or_fo_second_moment(int na, const float* xyz_a, const float* alpha_a, int nb,
                           const float* xyz_b, const float* alpha_b) {
  double s = 0.0;
  for (int i = 0; i < na; ++i)
    for (int j = 0; j < nb; ++j)
      for (int l = 0; l < nb; ++l) {
        double c[9], a[3];
        for (int d = 0; d < 3; ++d) {
          c[d] = xyz_a[3 * i + d]; c[3 + d] = xyz_b[3 * j + d]; c[6 + d] = xyz_b[3 * l + d];
        }
        a[0] = alpha_a[i]; a[1] = alpha_b[j]; a[2] = alpha_b[l];
        s += or_gauss_product_integral(3, c, a);
      }
  return s;
}

/* Eq. incexc summed in full: int u_A u_B, int u_A^2 (pass B = A) and int u_A
 * (pass nb = 0) for small molecules: every non-empty subset S of A and T of B
 * contributes (-1)^(|S|+|T|) int prod_S o prod_T o. */
double or_incexc(int na, const float* xyz_a, const float* alpha_a, int nb,
                 const float* xyz_b, const float* alpha_b) {
  if (na > 16 || nb > 16) return NAN;
  double c[3 * 32], a[32];
  double total = 0.0;
  uint32_t nsa = 1u << na, nsb = 1u << nb;
  for (uint32_t S = 1; S < nsa; ++S) {
    uint32_t Tlo = (nb == 0) ? 0 : 1;
    uint32_t Thi = (nb == 0) ? 1 : nsb;
    for (uint32_t T = Tlo; T < Thi; ++T) {
      int k = 0, sz = 0;
      for (int i = 0; i < na; ++i)
        if (S >> i & 1u) {
          for (int d = 0; d < 3; ++d) c[3 * k + d] = xyz_a[3 * i + d];
          a[k++] = alpha_a[i];
          sz++;
        }
      for (int j = 0; j < nb; ++j)
        if (T >> j & 1u) {
          for (int d = 0; d < 3; ++d) c[3 * k + d] = xyz_b[3 * j + d];
          a[k++] = alpha_b[j];
          sz++;
        }
      /* u_A u_B: sign (-1)^(|S|+|T|); u_A alone: (-1)^(|S|+1) */
      int sgn_exp = (nb == 0) ? sz + 1 : sz;
      double term = or_gauss_product_integral(k, c, a);
      total += (sgn_exp & 1) ? -term : term;
    }
  }
  return total;
}

/* Pointwise union by the expanded series (Eq. incexc) at one point. */
double or_union_series_at(int n, const float* xyz, const float* alpha, const double r[3]) {
  if (n > 20) return NAN;
  double o[20];
  for (int i = 0; i < n; ++i) {
    double dx = r[0] - xyz[3 * i], dy = r[1] - xyz[3 * i + 1], dz = r[2] - xyz[3 * i + 2];
    o[i] = exp(-(double)alpha[i] * (dx * dx + dy * dy + dz * dz));
  }
  double s = 0.0;
  for (uint32_t S = 1; S < (1u << n); ++S) {
    double p = 1.0;
    int sz = 0;
    for (int i = 0; i < n; ++i)
      if (S >> i & 1u) { p *= o[i]; sz++; }
    s += (sz & 1) ? p : -p;
  }
  return s;
}

/* Dense-grid quadrature (section "Exact union overlap by bounded reweighting"
 * names it as ground truth): trapezoid rule with spacing h over the box of
 * both molecules' atom extents padded by pad on every side, Neumaier-summed.
 * out8 = int u_A u_B, int u_A^2, int u_B^2, int u_A, int u_B, int m_A m_B,
 *        int m_A^2, int m_B^2. */
int or_grid_integrals(int na, const float* xyz_a, const float* alpha_a, int nb,
                      const float* xyz_b, const float* alpha_b, double h, double pad,
                      int n_threads, double* out8) {
  or_mol A, B;
  if (or_mol_init(&A, na, xyz_a, alpha_a)) return -1;
  if (or_mol_init(&B, nb, xyz_b, alpha_b)) { or_mol_free(&A); return -1; }
  double lo[3], hi[3];
  for (int d = 0; d < 3; ++d) { lo[d] = 1e300; hi[d] = -1e300; }
  for (int i = 0; i < na; ++i)
    for (int d = 0; d < 3; ++d) { lo[d] = fmin(lo[d], A.c[3 * i + d]); hi[d] = fmax(hi[d], A.c[3 * i + d]); }
  for (int i = 0; i < nb; ++i)
    for (int d = 0; d < 3; ++d) { lo[d] = fmin(lo[d], B.c[3 * i + d]); hi[d] = fmax(hi[d], B.c[3 * i + d]); }
  int ng[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] -= pad; hi[d] += pad;
    ng[d] = (int)ceil((hi[d] - lo[d]) / h) + 1;
  }
  double acc[8] = {0}, comp[8] = {0};
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
  int nx = ng[0];
  double* part = (double*)calloc((size_t)nx * 16, sizeof(double));
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int ix = 0; ix < nx; ++ix) {
    double s[8] = {0}, cc[8] = {0};
    double wx = (ix == 0 || ix == ng[0] - 1) ? 0.5 : 1.0;
    for (int iy = 0; iy < ng[1]; ++iy) {
      double wy = (iy == 0 || iy == ng[1] - 1) ? 0.5 : 1.0;
      for (int iz = 0; iz < ng[2]; ++iz) {
        double wz = (iz == 0 || iz == ng[2] - 1) ? 0.5 : 1.0;
        double r[3] = {lo[0] + ix * h, lo[1] + iy * h, lo[2] + iz * h};
        double mA, uA, mB, uB;
        or_density(&A, r, &mA, &uA);
        or_density(&B, r, &mB, &uB);
        double w = wx * wy * wz;
        double v[8] = {uA * uB, uA * uA, uB * uB, uA, uB, mA * mB, mA * mA, mB * mB};
        for (int q = 0; q < 8; ++q) {
          /* Neumaier compensated summation */
          double x = w * v[q];
          double t = s[q] + x;
          if (fabs(s[q]) >= fabs(x)) cc[q] += (s[q] - t) + x; else cc[q] += (x - t) + s[q];
          s[q] = t;
        }
      }
    }
    for (int q = 0; q < 8; ++q) { part[16 * ix + q] = s[q]; part[16 * ix + 8 + q] = cc[q]; }
  }
  for (int ix = 0; ix < nx; ++ix)
    for (int q = 0; q < 8; ++q) {
      double x = part[16 * ix + q] + part[16 * ix + 8 + q];
      double t = acc[q] + x;
      if (fabs(acc[q]) >= fabs(x)) comp[q] += (acc[q] - t) + x; else comp[q] += (x - t) + acc[q];
      acc[q] = t;
    }
  free(part);
  double h3 = h * h * h;
  for (int q = 0; q < 8; ++q) out8[q] = (acc[q] + comp[q]) * h3;
  or_mol_free(&A); or_mol_free(&B);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Alignment (section "Differentiable alignment and the hybrid pipeline").    */
/* ------------------------------------------------------------------------- */

/* Rotation matrix of the unit quaternion (w, x, y, z), row-major. */
static void or_quat_matrix(const double q[4], double R[9]) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* dR/dq_hat_i for the matrix above (i = w, x, y, z), each row-major 3x3. */
static void or_quat_matrix_grad(const double q[4], double dR[4][9]) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  /* d/dw */
  double Dw[9] = {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0};
  /* d/dx */
  double Dx[9] = {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
  /* d/dy */
  double Dy[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y};
  /* d/dz */
  double Dz[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0};
  memcpy(dR[0], Dw, sizeof Dw); memcpy(dR[1], Dx, sizeof Dx);
  memcpy(dR[2], Dy, sizeof Dy); memcpy(dR[3], Dz, sizeof Dz);
}

/* Self terms of the aligned Tanimoto: O_PP = Z_P * mean(u_P^2/m_P) over the
 * first n samples of P (pose invariant). */
static double or_self_overlap(const or_mol* P, uint32_t id, int64_t n, uint64_t seed) {
  double s = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    double r[3], m, u;
    or_sample(P, id, (uint64_t)k, seed, r);
    or_density(P, r, &m, &u);
    s += (m > 0 ? u / m : 0.0) * u;
  }
  return P->Z * s / (double)n;
}

/* Value and gradient of T(xi) = O(xi)/(O_aa + O_bb - O(xi)) with
 * O(xi) = Z_A/n sum_k w_A(r_k) u_B(r_k; xi), r_k the first n samples of A held
 * fixed (Eq. grad, common random numbers).  Gradient with respect to the seven
 * pose parameters (qw, qx, qy, qz, tx, ty, tz), q unnormalised (R7); the
 * derivative of u_B with respect to o_j is prod_{l != j} (1 - o_l), formed
 * directly. */
static void or_align_eval(const or_mol* A, const or_mol* B, uint32_t id_a,
                          const double* ra, const double* wa, int64_t n,
                          double O_aa, double O_bb, const double pose[7],
                          double* T_out, double* O_out, double grad[7]) {
  double qn = sqrt(pose[0] * pose[0] + pose[1] * pose[1] + pose[2] * pose[2] + pose[3] * pose[3]);
  double qh[4] = {pose[0] / qn, pose[1] / qn, pose[2] / qn, pose[3] / qn};
  double R[9], dR[4][9];
  or_quat_matrix(qh, R);
  or_quat_matrix_grad(qh, dR);
  int nb = B->n;
  double* cp = (double*)malloc(sizeof(double) * 3 * (size_t)nb);
  double* o = (double*)malloc(sizeof(double) * (size_t)nb);
  for (int j = 0; j < nb; ++j)
    for (int a = 0; a < 3; ++a)
      cp[3 * j + a] = R[3 * a] * B->c[3 * j] + R[3 * a + 1] * B->c[3 * j + 1] +
                      R[3 * a + 2] * B->c[3 * j + 2] + pose[4 + a];
  double sumO = 0.0;
  double gc[4] = {0}, gt[3] = {0};  /* d O / d q_hat, d O / d t (before Z/n) */
  (void)id_a;
  for (int64_t k = 0; k < n; ++k) {
    const double* r = ra + 3 * k;
    double prod = 1.0;
    for (int j = 0; j < nb; ++j) {
      double dx = r[0] - cp[3 * j], dy = r[1] - cp[3 * j + 1], dz = r[2] - cp[3 * j + 2];
      o[j] = exp(-B->alpha[j] * (dx * dx + dy * dy + dz * dz));
      prod *= (1.0 - o[j]);
    }
    double uB = 1.0 - prod;
    sumO += wa[k] * uB;
    for (int j = 0; j < nb; ++j) {
      double others = 1.0;
      for (int l = 0; l < nb; ++l)
        if (l != j) others *= (1.0 - o[l]);
      /* d u_B / d c'_j = others * 2 alpha_j o_j (r - c'_j) */
      double coef = wa[k] * others * 2.0 * B->alpha[j] * o[j];
      double g[3] = {coef * (r[0] - cp[3 * j]), coef * (r[1] - cp[3 * j + 1]),
                     coef * (r[2] - cp[3 * j + 2])};
      for (int a = 0; a < 3; ++a) gt[a] += g[a];
      for (int i = 0; i < 4; ++i) {
        /* d c'_j / d q_hat_i = dR_i c_j */
        for (int a = 0; a < 3; ++a) {
          double dc = dR[i][3 * a] * B->c[3 * j] + dR[i][3 * a + 1] * B->c[3 * j + 1] +
                      dR[i][3 * a + 2] * B->c[3 * j + 2];
          gc[i] += g[a] * dc;
        }
      }
    }
  }
  double scale = A->Z / (double)n;
  double O = scale * sumO;
  double S = O_aa + O_bb;
  double D = S - O;
  double T = O / D;
  double dT_dO = S / (D * D);
  /* chain q_hat = q/|q|: d q_hat_i / d q_k = (delta_ik - qh_i qh_k)/|q| */
  for (int kk = 0; kk < 4; ++kk) {
    double s = 0.0;
    for (int i = 0; i < 4; ++i) s += gc[i] * (((i == kk) ? 1.0 : 0.0) - qh[i] * qh[kk]) / qn;
    grad[kk] = dT_dO * scale * s;
  }
  for (int a = 0; a < 3; ++a) grad[4 + a] = dT_dO * scale * gt[a];
  *T_out = T;
  if (O_out) *O_out = O;
  free(cp); free(o);
}

typedef struct {
  double* ra;
  double* wa;
  double O_aa, O_bb;
} or_align_fixed;

static int or_align_setup(const or_mol* A, const or_mol* B, uint32_t id_a, uint32_t id_b,
                          int64_t n, uint64_t seed, or_align_fixed* F) {
  F->ra = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  F->wa = (double*)malloc(sizeof(double) * (size_t)n);
  if (!F->ra || !F->wa) { free(F->ra); free(F->wa); return -1; }
  for (int64_t k = 0; k < n; ++k) {
    double m, u;
    or_sample(A, id_a, (uint64_t)k, seed, F->ra + 3 * k);
    or_density(A, F->ra + 3 * k, &m, &u);
    F->wa[k] = m > 0 ? u / m : 0.0;
  }
  F->O_aa = or_self_overlap(A, id_a, n, seed);
  F->O_bb = or_self_overlap(B, id_b, n, seed);
  return 0;
}

/* exported: T and dT/dpose for poses [n_poses][7] of one pair; also returns the
 * self-overlaps used (2 doubles). */
int or_align_grad(int na, const float* xyz_a, const float* alpha_a, uint32_t id_a,
                  int nb, const float* xyz_b, const float* alpha_b, uint32_t id_b,
                  int64_t n_samples, uint64_t seed, int32_t n_poses, const double* poses,
                  double* T_out, double* grad_out, double* self_out) {
  or_mol A, B;
  if (or_mol_init(&A, na, xyz_a, alpha_a)) return -1;
  if (or_mol_init(&B, nb, xyz_b, alpha_b)) { or_mol_free(&A); return -1; }
  or_align_fixed F;
  if (or_align_setup(&A, &B, id_a, id_b, n_samples, seed, &F)) {
    or_mol_free(&A); or_mol_free(&B);
    return -1;
  }
  for (int32_t p = 0; p < n_poses; ++p)
    or_align_eval(&A, &B, id_a, F.ra, F.wa, n_samples, F.O_aa, F.O_bb, poses + 7 * p,
                  T_out + p, NULL, grad_out + 7 * p);
  if (self_out) { self_out[0] = F.O_aa; self_out[1] = F.O_bb; }
  free(F.ra); free(F.wa);
  or_mol_free(&A); or_mol_free(&B);
  return 0;
}

/* Adam (Kingma and Ba) on a flat parameter vector, step t >= 1, descending. */
void or_adam(int64_t n, double* p, const double* g, double* m, double* v, int32_t t, double lr,
             double b1, double b2, double eps) {
  for (int64_t i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1 - b1) * g[i];
    v[i] = b2 * v[i] + (1 - b2) * g[i] * g[i];
    double mh = m[i] / (1 - pow(b1, t)), vh = v[i] / (1 - pow(b2, t));
    p[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* One ascent step on T for a pose: Adam descends on -dT/dpose, then the
 * quaternion part is renormalised. */
static void or_pose_adam_step(double x[7], const double dT[7], double m[7], double v[7],
                              int32_t t, double lr) {
  double g[7];
  for (int i = 0; i < 7; ++i) g[i] = -dT[i];
  or_adam(7, x, g, m, v, t, lr, 0.9, 0.999, 1e-8);
  double qn = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2] + x[3] * x[3]);
  for (int i = 0; i < 4; ++i) x[i] /= qn;
}

/* Adam (Kingma and Ba) on -T over the seven pose parameters, renormalising q
 * after each step; returns the final pose and T evaluated at it for each start.
 * betas (0.9, 0.999), eps 1e-8. */
int or_align_adam(int na, const float* xyz_a, const float* alpha_a, uint32_t id_a,
                  int nb, const float* xyz_b, const float* alpha_b, uint32_t id_b,
                  int64_t n_samples, uint64_t seed, int32_t n_starts, const double* pose0,
                  int32_t n_steps, double lr, double* pose_out, double* T_out) {
  or_mol A, B;
  if (or_mol_init(&A, na, xyz_a, alpha_a)) return -1;
  if (or_mol_init(&B, nb, xyz_b, alpha_b)) { or_mol_free(&A); return -1; }
  or_align_fixed F;
  if (or_align_setup(&A, &B, id_a, id_b, n_samples, seed, &F)) {
    or_mol_free(&A); or_mol_free(&B);
    return -1;
  }
  for (int32_t s = 0; s < n_starts; ++s) {
    double x[7], m[7] = {0}, v[7] = {0}, g[7], T;
    memcpy(x, pose0 + 7 * s, sizeof x);
    for (int32_t it = 1; it <= n_steps; ++it) {
      or_align_eval(&A, &B, id_a, F.ra, F.wa, n_samples, F.O_aa, F.O_bb, x, &T, NULL, g);
      or_pose_adam_step(x, g, m, v, it, lr);
    }
    or_align_eval(&A, &B, id_a, F.ra, F.wa, n_samples, F.O_aa, F.O_bb, x, &T, NULL, g);
    memcpy(pose_out + 7 * s, x, sizeof x);
    T_out[s] = T;
  }
  free(F.ra); free(F.wa);
  or_mol_free(&A); or_mol_free(&B);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Hybrid pipeline (section "Differentiable alignment and the hybrid          */
/* pipeline"): align on the first-order overlap, then score with the union    */
/* estimator.                                                                 */
/* ------------------------------------------------------------------------- */

/* T_FO(xi) = O(xi) / (O_AA + O_BB - O(xi)) with O(xi) = sum_ij K_ij,
 * K_ij = (pi/(a_i+a_j))^(3/2) exp(-a_i a_j/(a_i+a_j) |c_i - c''_j|^2) (Eq. fo)
 * and c''_j = R(q/|q|) c_j + t (Eq. pose, quaternion form).  Gradient with
 * respect to the seven pose parameters through dR/dq_hat and the
 * normalisation of q (the same parameterisation as the IS alignment). */
static void or_fo_align_eval(const or_mol* A, const or_mol* B, double O_aa, double O_bb,
                             const double pose[7], double* T_out, double grad[7]) {
  double qn = sqrt(pose[0] * pose[0] + pose[1] * pose[1] + pose[2] * pose[2] + pose[3] * pose[3]);
  double qh[4] = {pose[0] / qn, pose[1] / qn, pose[2] / qn, pose[3] / qn};
  double R[9], dR[4][9];
  or_quat_matrix(qh, R);
  or_quat_matrix_grad(qh, dR);
  double O = 0.0, gc[4] = {0}, gt[3] = {0};
  for (int j = 0; j < B->n; ++j) {
    const double* cb = B->c + 3 * j;
    double cp[3];
    for (int a = 0; a < 3; ++a)
      cp[a] = R[3 * a] * cb[0] + R[3 * a + 1] * cb[1] + R[3 * a + 2] * cb[2] + pose[4 + a];
    double g[3] = {0, 0, 0};  /* d O / d c''_j */
    for (int i = 0; i < A->n; ++i) {
      const double* ca = A->c + 3 * i;
      double ai = A->alpha[i], aj = B->alpha[j];
      double s = ai + aj, kap = ai * aj / s;
      double d[3] = {ca[0] - cp[0], ca[1] - cp[1], ca[2] - cp[2]};
      double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      double K = pow(OR_PI / s, 1.5) * exp(-kap * d2);
      O += K;
      for (int a = 0; a < 3; ++a) g[a] += 2.0 * kap * K * d[a];
    }
    for (int a = 0; a < 3; ++a) gt[a] += g[a];
    for (int i = 0; i < 4; ++i)
      for (int a = 0; a < 3; ++a)
        gc[i] += g[a] * (dR[i][3 * a] * cb[0] + dR[i][3 * a + 1] * cb[1] +
                         dR[i][3 * a + 2] * cb[2]);
  }
  double S = O_aa + O_bb, D = S - O;
  *T_out = O / D;
  if (grad) {
    double dT_dO = S / (D * D);
    for (int kk = 0; kk < 4; ++kk) {
      double acc = 0.0;
      for (int i = 0; i < 4; ++i) acc += gc[i] * (((i == kk) ? 1.0 : 0.0) - qh[i] * qh[kk]) / qn;
      grad[kk] = dT_dO * acc;
    }
    for (int a = 0; a < 3; ++a) grad[4 + a] = dT_dO * gt[a];
  }
}

/* exported: T_FO and dT_FO/dpose for poses [n_poses][7] of one pair */
int or_fo_align_grad(int na, const float* xyz_a, const float* alpha_a, int nb,
                     const float* xyz_b, const float* alpha_b, int32_t n_poses,
                     const double* poses, double* T_out, double* grad_out) {
  or_mol A, B;
  if (or_mol_init(&A, na, xyz_a, alpha_a)) return -1;
  if (or_mol_init(&B, nb, xyz_b, alpha_b)) { or_mol_free(&A); return -1; }
  double O_aa = or_fo_overlap(na, xyz_a, alpha_a, na, xyz_a, alpha_a);
  double O_bb = or_fo_overlap(nb, xyz_b, alpha_b, nb, xyz_b, alpha_b);
  for (int32_t p = 0; p < n_poses; ++p)
    or_fo_align_eval(&A, &B, O_aa, O_bb, poses + 7 * p, T_out + p,
                     grad_out ? grad_out + 7 * p : NULL);
  or_mol_free(&A); or_mol_free(&B);
  return 0;
}

/* exported: Adam on -T_FO from each start (the update of or_align_adam:
 * betas 0.9, 0.999, eps 1e-8, q renormalised after each step); final poses
 * and T_FO at them. */
int or_fo_align_adam(int na, const float* xyz_a, const float* alpha_a, int nb,
                     const float* xyz_b, const float* alpha_b, int32_t n_starts,
                     const double* pose0, int32_t n_steps, double lr, double* pose_out,
                     double* T_out) {
  or_mol A, B;
  if (or_mol_init(&A, na, xyz_a, alpha_a)) return -1;
  if (or_mol_init(&B, nb, xyz_b, alpha_b)) { or_mol_free(&A); return -1; }
  double O_aa = or_fo_overlap(na, xyz_a, alpha_a, na, xyz_a, alpha_a);
  double O_bb = or_fo_overlap(nb, xyz_b, alpha_b, nb, xyz_b, alpha_b);
  for (int32_t s = 0; s < n_starts; ++s) {
    double x[7], m[7] = {0}, v[7] = {0}, g[7], T;
    memcpy(x, pose0 + 7 * s, sizeof x);
    for (int32_t it = 1; it <= n_steps; ++it) {
      or_fo_align_eval(&A, &B, O_aa, O_bb, x, &T, g);
      or_pose_adam_step(x, g, m, v, it, lr);
    }
    or_fo_align_eval(&A, &B, O_aa, O_bb, x, &T, NULL);
    memcpy(pose_out + 7 * s, x, sizeof x);
    T_out[s] = T;
  }
  or_mol_free(&A); or_mol_free(&B);
  return 0;
}

/* Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations: eigenvalues
 * descending in ev, unit eigenvectors in the columns of V (row-major). */
static void or_sym3_eigvec(double a[3][3], double ev[3], double V[9]) {
  double U[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]);
    if (off < 1e-300) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (a[p][q] == 0.0) continue;
        double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < 3; ++k) {
          double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - sn * akq;
          a[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {
          double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - sn * aqk;
          a[q][k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          double ukp = U[k][p], ukq = U[k][q];
          U[k][p] = c * ukp - sn * ukq;
          U[k][q] = sn * ukp + c * ukq;
        }
      }
  }
  int idx[3] = {0, 1, 2};
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j)
      if (a[idx[j]][idx[j]] > a[idx[i]][idx[i]]) { int t = idx[i]; idx[i] = idx[j]; idx[j] = t; }
  for (int c = 0; c < 3; ++c) {
    ev[c] = a[idx[c]][idx[c]];
    for (int r = 0; r < 3; ++r) V[3 * r + c] = U[r][idx[c]];
  }
}

/* Principal frame of a molecule's mixture: mean mu = sum pi_i c_i and the
 * eigenvectors of sum pi_i (c_i - mu)(c_i - mu)^T (pi_i = v_i / Z), as the
 * columns of U: descending eigenvalues, the largest-magnitude component of
 * the first two made positive, the third their cross product (right-handed). */
static void or_principal_frame(const or_mol* M, double mu[3], double U[9]) {
  mu[0] = mu[1] = mu[2] = 0.0;
  for (int i = 0; i < M->n; ++i)
    for (int d = 0; d < 3; ++d) mu[d] += M->v[i] / M->Z * M->c[3 * i + d];
  double C[3][3] = {{0}};
  for (int i = 0; i < M->n; ++i) {
    double w = M->v[i] / M->Z;
    double x[3] = {M->c[3 * i] - mu[0], M->c[3 * i + 1] - mu[1], M->c[3 * i + 2] - mu[2]};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) C[r][c] += w * x[r] * x[c];
  }
  double ev[3];
  or_sym3_eigvec(C, ev, U);
  for (int c = 0; c < 2; ++c) {
    int big = 0;
    for (int r = 1; r < 3; ++r)
      if (fabs(U[3 * r + c]) > fabs(U[3 * big + c])) big = r;
    if (U[3 * big + c] < 0)
      for (int r = 0; r < 3; ++r) U[3 * r + c] = -U[3 * r + c];
  }
  U[2] = U[3] * U[7] - U[6] * U[4];
  U[5] = U[6] * U[1] - U[0] * U[7];
  U[8] = U[0] * U[4] - U[3] * U[1];
}

/* Unit quaternion (w, x, y, z), w >= 0, of a rotation matrix (Shepperd). */
static void or_matrix_quat(const double R[9], double q[4]) {
  double tr = R[0] + R[4] + R[8];
  double w, x, y, z;
  if (tr >= R[0] && tr >= R[4] && tr >= R[8]) {
    double s = sqrt(1.0 + tr) * 2.0;
    w = 0.25 * s; x = (R[7] - R[5]) / s; y = (R[2] - R[6]) / s; z = (R[3] - R[1]) / s;
  } else if (R[0] >= R[4] && R[0] >= R[8]) {
    double s = sqrt(1.0 + R[0] - R[4] - R[8]) * 2.0;
    w = (R[7] - R[5]) / s; x = 0.25 * s; y = (R[1] + R[3]) / s; z = (R[2] + R[6]) / s;
  } else if (R[4] >= R[8]) {
    double s = sqrt(1.0 + R[4] - R[0] - R[8]) * 2.0;
    w = (R[2] - R[6]) / s; x = (R[1] + R[3]) / s; y = 0.25 * s; z = (R[5] + R[7]) / s;
  } else {
    double s = sqrt(1.0 + R[8] - R[0] - R[4]) * 2.0;
    w = (R[3] - R[1]) / s; x = (R[2] + R[6]) / s; y = (R[5] + R[7]) / s; z = 0.25 * s;
  }
  double sg = w < 0 ? -1.0 : 1.0;
  q[0] = sg * w; q[1] = sg * x; q[2] = sg * y; q[3] = sg * z;
}

/* exported: the alignment starts of one pair, [5 + n_random][7]: the given
 * pose (identity), the four proper principal-axis alignments
 * R = U_A D U_B^T with D = diag(1,1,1), diag(1,-1,-1), diag(-1,1,-1),
 * diag(-1,-1,1) and t = mu_A - R mu_B, then n_random uniformly random
 * rotations about B's mean (Shoemake's construction from the three 24-bit
 * uniforms of Philox block (s, pair_id, 0x5157A27, 0) under the key seed)
 * with the same centring translation. */
int or_fo_starts(int na, const float* xyz_a, const float* alpha_a, int nb,
                 const float* xyz_b, const float* alpha_b, uint32_t pair_id, int32_t n_random,
                 uint64_t seed, double* poses) {
  or_mol A, B;
  if (or_mol_init(&A, na, xyz_a, alpha_a)) return -1;
  if (or_mol_init(&B, nb, xyz_b, alpha_b)) { or_mol_free(&A); return -1; }
  double muA[3], UA[9], muB[3], UB[9];
  or_principal_frame(&A, muA, UA);
  or_principal_frame(&B, muB, UB);
  double* p0 = poses;
  p0[0] = 1.0; p0[1] = p0[2] = p0[3] = 0.0; p0[4] = p0[5] = p0[6] = 0.0;
  static const double Ds[4][3] = {{1, 1, 1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};
  for (int s = 0; s < 4 + n_random; ++s) {
    double R[9];
    if (s < 4) {
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          double acc = 0.0;
          for (int k = 0; k < 3; ++k) acc += UA[3 * r + k] * Ds[s][k] * UB[3 * c + k];
          R[3 * r + c] = acc;
        }
    } else {
      uint32_t ctr[4] = {(uint32_t)(s - 4), pair_id, 0x5157A27u, 0u};
      uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
      uint32_t x[4];
      or_philox4x32_10(ctr, key, x);
      double u1 = ((double)(x[0] >> 8) + 0.5) / 16777216.0;
      double u2 = ((double)(x[1] >> 8) + 0.5) / 16777216.0;
      double u3 = ((double)(x[2] >> 8) + 0.5) / 16777216.0;
      double q[4] = {sqrt(u1) * cos(2 * OR_PI * u3), sqrt(1 - u1) * sin(2 * OR_PI * u2),
                     sqrt(1 - u1) * cos(2 * OR_PI * u2), sqrt(u1) * sin(2 * OR_PI * u3)};
      or_quat_matrix(q, R);
    }
    double q[4];
    or_matrix_quat(R, q);
    double* out = poses + 7 * (1 + s);
    for (int i = 0; i < 4; ++i) out[i] = q[i];
    for (int a = 0; a < 3; ++a)
      out[4 + a] = muA[a] - (R[3 * a] * muB[0] + R[3 * a + 1] * muB[1] + R[3 * a + 2] * muB[2]);
  }
  or_mol_free(&A); or_mol_free(&B);
  return 0;
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Surrogate features (no counterpart in the paper: the learned triage model  */
/* that seeds confidence-bounded screening).  Per molecule, 24 numbers:       */
/*   [0..15]  histogram of |c_i - mu| in 0.5 A bins over [0, 8), last bin     */
/*            open, mu = sum pi_i c_i the mixture mean (pi_i = v_i / Z)       */
/*   [16..18] square roots of the eigenvalues (descending) of the mixture    */
/*            covariance sum pi_i (c_i c_i^T + I/(2 alpha_i)) - mu mu^T       */
/*   [19..22] counts of atoms in four width classes, alpha < 0.767,          */
/*            [0.767, 0.893), [0.893, 0.995), >= 0.995 A^-2                   */
/*   [23]     first-order self-overlap (Eq. fo with B = A)                    */
/* Eigenvalues by Jacobi rotations (plain, converged to machine precision).   */
/* ------------------------------------------------------------------------- */
static void or_sym3_eig(double a[3][3], double ev[3]) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]);
    if (off < 1e-300) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (a[p][q] == 0.0) continue;
        double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; ++k) {  /* columns p, q */
          double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - s * akq;
          a[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {  /* rows p, q */
          double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - s * aqk;
          a[q][k] = s * apk + c * aqk;
        }
      }
  }
  ev[0] = a[0][0]; ev[1] = a[1][1]; ev[2] = a[2][2];
  /* descending */
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j)
      if (ev[j] > ev[i]) { double t = ev[i]; ev[i] = ev[j]; ev[j] = t; }
}

int or_features(int32_t n_mols, const int32_t* off, const float* xyz, const float* alpha,
                double* out24) {
  for (int32_t m = 0; m < n_mols; ++m) {
    int a0 = off[m], n = off[m + 1] - off[m];
    double* f = out24 + 24 * (size_t)m;
    for (int k = 0; k < 24; ++k) f[k] = 0.0;
    or_mol M;
    if (or_mol_init(&M, n, xyz + 3 * (size_t)a0, alpha + a0)) return -1;
    double mu[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i)
      for (int d = 0; d < 3; ++d) mu[d] += (M.v[i] / M.Z) * M.c[3 * i + d];
    for (int i = 0; i < n; ++i) {
      double dx = M.c[3 * i] - mu[0], dy = M.c[3 * i + 1] - mu[1], dz = M.c[3 * i + 2] - mu[2];
      double r = sqrt(dx * dx + dy * dy + dz * dz);
      int b = (int)floor(r / 0.5);
      if (b > 15) b = 15;
      f[b] += 1.0;
    }
    double cov[3][3] = {{0}};
    for (int i = 0; i < n; ++i) {
      double pi = M.v[i] / M.Z;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          cov[a][b] += pi * (M.c[3 * i + a] * M.c[3 * i + b] + (a == b ? 0.5 / M.alpha[i] : 0.0));
    }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) cov[a][b] -= mu[a] * mu[b];
    double ev[3];
    or_sym3_eig(cov, ev);
    for (int k = 0; k < 3; ++k) f[16 + k] = sqrt(ev[k] > 0 ? ev[k] : 0.0);
    for (int i = 0; i < n; ++i) {
      double al = M.alpha[i];
      int cls = al < 0.767 ? 0 : (al < 0.893 ? 1 : (al < 0.995 ? 2 : 3));
      f[19 + cls] += 1.0;
    }
    f[23] = or_fo_overlap(n, xyz + 3 * (size_t)a0, alpha + a0, n, xyz + 3 * (size_t)a0, alpha + a0);
    or_mol_free(&M);
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Surrogate MLP in FP64: L dense layers, ReLU between them, linear output.   */
/* Layer l maps width[l] -> width[l+1]: h_{l+1} = act(h_l W_l + b_l), W_l     */
/* row-major [width[l]][width[l+1]].  Parameters are packed W_0, b_0, W_1,    */
/* b_1, ...  Loss: sum over outputs j of lw_j * mean_b (y_bj - t_bj)^2.       */
/* or_mlp_loss_grad returns the loss and d loss / d params (same packing).    */
/* ------------------------------------------------------------------------- */
int64_t or_mlp_nparams(int L, const int32_t* width) {
  int64_t n = 0;
  for (int l = 0; l < L; ++l) n += (int64_t)width[l] * width[l + 1] + width[l + 1];
  return n;
}

int or_mlp_forward(int L, const int32_t* width, const double* params, int32_t batch,
                   const double* x, double* y) {
  int maxw = 0;
  for (int l = 0; l <= L; ++l) if (width[l] > maxw) maxw = width[l];
  double* h = (double*)malloc(sizeof(double) * (size_t)batch * maxw);
  double* g = (double*)malloc(sizeof(double) * (size_t)batch * maxw);
  if (!h || !g) { free(h); free(g); return -1; }
  memcpy(h, x, sizeof(double) * (size_t)batch * width[0]);
  const double* p = params;
  for (int l = 0; l < L; ++l) {
    int ni = width[l], no = width[l + 1];
    const double* W = p;
    const double* b = p + (size_t)ni * no;
    for (int32_t s = 0; s < batch; ++s)
      for (int j = 0; j < no; ++j) {
        double acc = b[j];
        for (int i = 0; i < ni; ++i) acc += h[(size_t)s * ni + i] * W[(size_t)i * no + j];
        g[(size_t)s * no + j] = (l + 1 < L && acc < 0.0) ? 0.0 : acc;
      }
    double* t = h; h = g; g = t;
    p += (size_t)ni * no + no;
  }
  memcpy(y, h, sizeof(double) * (size_t)batch * width[L]);
  free(h); free(g);
  return 0;
}

int or_mlp_loss_grad(int L, const int32_t* width, const double* params, int32_t batch,
                     const double* x, const double* target, const double* lw,
                     double* loss_out, double* grad) {
  /* keep every layer's output */
  int64_t offs[17];
  if (L > 16) return -2;
  int64_t tot = 0;
  for (int l = 0; l <= L; ++l) { offs[l] = tot; tot += (int64_t)batch * width[l]; }
  double* H = (double*)malloc(sizeof(double) * (size_t)tot);
  if (!H) return -1;
  memcpy(H, x, sizeof(double) * (size_t)batch * width[0]);
  const double* p = params;
  for (int l = 0; l < L; ++l) {
    int ni = width[l], no = width[l + 1];
    const double* W = p;
    const double* b = p + (size_t)ni * no;
    for (int32_t s = 0; s < batch; ++s)
      for (int j = 0; j < no; ++j) {
        double acc = b[j];
        for (int i = 0; i < ni; ++i) acc += H[offs[l] + (size_t)s * ni + i] * W[(size_t)i * no + j];
        H[offs[l + 1] + (size_t)s * no + j] = (l + 1 < L && acc < 0.0) ? 0.0 : acc;
      }
    p += (size_t)ni * no + no;
  }
  int nout = width[L];
  double loss = 0.0;
  int maxw = 0;
  for (int l = 0; l <= L; ++l) if (width[l] > maxw) maxw = width[l];
  double* d = (double*)malloc(sizeof(double) * (size_t)batch * maxw);
  double* dn = (double*)malloc(sizeof(double) * (size_t)batch * maxw);
  if (!d || !dn) { free(H); free(d); free(dn); return -1; }
  for (int32_t s = 0; s < batch; ++s)
    for (int j = 0; j < nout; ++j) {
      double e = H[offs[L] + (size_t)s * nout + j] - target[(size_t)s * nout + j];
      loss += lw[j] * e * e / batch;
      d[(size_t)s * nout + j] = 2.0 * lw[j] * e / batch;
    }
  *loss_out = loss;
  /* walk layers backwards; parameter offsets */
  int64_t poff[17];
  int64_t acc = 0;
  for (int l = 0; l < L; ++l) { poff[l] = acc; acc += (int64_t)width[l] * width[l + 1] + width[l + 1]; }
  for (int l = L - 1; l >= 0; --l) {
    int ni = width[l], no = width[l + 1];
    const double* W = params + poff[l];
    double* gW = grad + poff[l];
    double* gb = gW + (size_t)ni * no;
    for (int i = 0; i < ni; ++i)
      for (int j = 0; j < no; ++j) {
        double s2 = 0.0;
        for (int32_t s = 0; s < batch; ++s) s2 += H[offs[l] + (size_t)s * ni + i] * d[(size_t)s * no + j];
        gW[(size_t)i * no + j] = s2;
      }
    for (int j = 0; j < no; ++j) {
      double s2 = 0.0;
      for (int32_t s = 0; s < batch; ++s) s2 += d[(size_t)s * no + j];
      gb[j] = s2;
    }
    if (l > 0) {
      for (int32_t s = 0; s < batch; ++s)
        for (int i = 0; i < ni; ++i) {
          double s2 = 0.0;
          for (int j = 0; j < no; ++j) s2 += d[(size_t)s * no + j] * W[(size_t)i * no + j];
          /* ReLU of layer l's output: derivative 1 where the output is > 0 */
          dn[(size_t)s * ni + i] = H[offs[l] + (size_t)s * ni + i] > 0.0 ? s2 : 0.0;
        }
      double* t = d; d = dn; dn = t;
    }
  }
  free(H); free(d); free(dn);
  return 0;
}

