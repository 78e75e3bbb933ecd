/*
 * Plain FP64 CPU oracle for the DMC hot path (Slater-Jastrow, LCAO orbitals).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no code
 * with the HIP library.  Build: gcc -O2 -ffp-contract=off -fopenmp -shared.
 *
 * Paper passages followed (arXiv 2504.07948, QMC section):
 *   Eq. 1   imaginary-time projection; fixed-node constraint (text after Eq. 1)
 *   Eq. 2   Psi_T = exp(sum J) sum_k C_k D_k^up D_k^dn, phi_i = sum_l C_l^i Phi_l
 *   Eq. 3   d ln D / d lambda = tr(A^{-1} B), B = dA/d lambda, A_ij = phi_j(r_i)
 *   DMC parameters: time step 0.01 a.u., walkers evaluated as a crowd.
 * Readings of what the paper leaves open (Pade Jastrow form, Cartesian
 * Gaussians, no drift limiter, fixed population with log-weights, Philox
 * stream layout) are listed with the project documentation.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ basis */
/* Cartesian exponent triples, canonical component order. */
static const int CART[3][6][3] = {
    {{0, 0, 0}},
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
    {{2, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}},
};
static const int NCART[3] = {1, 3, 6};

/* c * x^n with the convention x^n = 0 for n < 0 (derivative of a monomial). */
static double mono(double x, int n) {
  if (n < 0) return 0.0;
  double v = 1.0;
  for (int k = 0; k < n; ++k) v *= x;
  return v;
}

/* Phi(r) = x^a y^b z^c * R(s^2), R(s^2) = sum_p d_p exp(-alpha_p s^2),
 * with (x,y,z) = r - R_atom.  Derivatives from the product rule:
 *   dPhi/dx = (dP/dx) R + P * 2x R'      (R' = dR/d(s^2))
 *   lap Phi = R lap P + 2 grad P . grad R + P lap R,
 *   grad R = 2 r R',  lap R = 6 R' + 4 s^2 R''. */
int orc_basis_vgl(const orc_system *s, const double r[3], double *out) {
  int prim = 0, fn = 0;
  for (int sh = 0; sh < s->n_shell; ++sh) {
    const int l = s->shell_l[sh];
    if (l < 0 || l > 2) return 1;
    const double *c = s->ion_xyz + 3 * s->shell_atom[sh];
    const double d[3] = {r[0] - c[0], r[1] - c[1], r[2] - c[2]};
    const double s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double R0 = 0.0, R1 = 0.0, R2 = 0.0;
    for (int p = 0; p < s->shell_nprim[sh]; ++p, ++prim) {
      const double a = s->prim_alpha[prim];
      const double e = s->prim_coef[prim] * exp(-a * s2);
      R0 += e;
      R1 += -a * e;
      R2 += a * a * e;
    }
    const double gradR[3] = {2.0 * d[0] * R1, 2.0 * d[1] * R1, 2.0 * d[2] * R1};
    const double lapR = 6.0 * R1 + 4.0 * s2 * R2;
    for (int k = 0; k < NCART[l]; ++k, ++fn) {
      const int *e = CART[l][k];
      const double px = mono(d[0], e[0]), py = mono(d[1], e[1]), pz = mono(d[2], e[2]);
      const double P = px * py * pz;
      const double dP[3] = {e[0] * mono(d[0], e[0] - 1) * py * pz,
                            e[1] * px * mono(d[1], e[1] - 1) * pz,
                            e[2] * px * py * mono(d[2], e[2] - 1)};
      const double lapP = e[0] * (e[0] - 1) * mono(d[0], e[0] - 2) * py * pz +
                          e[1] * (e[1] - 1) * px * mono(d[1], e[1] - 2) * pz +
                          e[2] * (e[2] - 1) * px * py * mono(d[2], e[2] - 2);
      double *o = out + 5 * fn;
      o[0] = P * R0;
      for (int x = 0; x < 3; ++x) o[1 + x] = dP[x] * R0 + P * gradR[x];
      o[4] = lapP * R0 + 2.0 * (dP[0] * gradR[0] + dP[1] * gradR[1] + dP[2] * gradR[2]) +
             P * lapR;
    }
  }
  return fn == s->n_basis ? 0 : 1;
}

/* phi_j = sum_l C_lj Phi_l, for value, gradient and Laplacian rows. */
int orc_orbitals_vgl(const orc_system *s, const double r[3], int32_t n_orb, double *out) {
  double *b = (double *)malloc(sizeof(double) * 5 * (size_t)s->n_basis);
  if (!b) return 2;
  int rc = orc_basis_vgl(s, r, b);
  for (int c = 0; c < 5; ++c)
    for (int j = 0; j < n_orb; ++j) {
      double acc = 0.0;
      for (int l = 0; l < s->n_basis; ++l) acc += s->mo_coef[(size_t)l * s->n_mo + j] * b[5 * l + c];
      out[c * n_orb + j] = acc;
    }
  free(b);
  return rc;
}

/* ------------------------------------------------------------ dense LU --- */
int orc_lu_slogdet_inv(int32_t n, const double *A, double *logdet, int32_t *sign, double *inv) {
  double *lu = (double *)malloc(sizeof(double) * (size_t)n * n + 1);
  int *piv = (int *)malloc(sizeof(int) * (size_t)n + 1);
  memcpy(lu, A, sizeof(double) * (size_t)n * n);
  int sgn = 1, singular = 0;
  double ld = 0.0;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = fabs(lu[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i)
      if (fabs(lu[(size_t)i * n + k]) > best) { best = fabs(lu[(size_t)i * n + k]); p = i; }
    piv[k] = p;
    if (p != k) {
      for (int j = 0; j < n; ++j) {
        double t = lu[(size_t)k * n + j];
        lu[(size_t)k * n + j] = lu[(size_t)p * n + j];
        lu[(size_t)p * n + j] = t;
      }
      sgn = -sgn;
    }
    const double pv = lu[(size_t)k * n + k];
    if (pv == 0.0) { singular = 1; break; }
    if (pv < 0) sgn = -sgn;
    ld += log(fabs(pv));
    for (int i = k + 1; i < n; ++i) {
      const double m = lu[(size_t)i * n + k] / pv;
      lu[(size_t)i * n + k] = m;
      for (int j = k + 1; j < n; ++j) lu[(size_t)i * n + j] -= m * lu[(size_t)k * n + j];
    }
  }
  if (logdet) *logdet = singular ? -INFINITY : ld;
  if (sign) *sign = singular ? 0 : sgn;
  if (inv && !singular) {
    /* solve A X = I column by column: P A = L U */
    double *col = (double *)malloc(sizeof(double) * (size_t)n + 1);
    for (int c = 0; c < n; ++c) {
      for (int i = 0; i < n; ++i) col[i] = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < n; ++k)
        if (piv[k] != k) { double t = col[k]; col[k] = col[piv[k]]; col[piv[k]] = t; }
      for (int i = 0; i < n; ++i)
        for (int k = 0; k < i; ++k) col[i] -= lu[(size_t)i * n + k] * col[k];
      for (int i = n - 1; i >= 0; --i) {
        for (int k = i + 1; k < n; ++k) col[i] -= lu[(size_t)i * n + k] * col[k];
        col[i] /= lu[(size_t)i * n + i];
      }
      for (int i = 0; i < n; ++i) inv[(size_t)i * n + c] = col[i];
    }
    free(col);
  }
  free(lu);
  free(piv);
  return singular;
}

/* ------------------------------------------------------------- Jastrow --- */
/* Pade u(r) = a r / (1 + b r), u' = a/(1+br)^2, u'' = -2ab/(1+br)^3. */
static double pade(double a, double b, double r) { return a * r / (1.0 + b * r); }
static double pade_d1(double a, double b, double r) {
  const double t = 1.0 + b * r;
  return a / (t * t);
}
static double pade_d2(double a, double b, double r) {
  const double t = 1.0 + b * r;
  return -2.0 * a * b / (t * t * t);
}

static int spin_of(const orc_system *s, int i) { return i < s->n_up ? 0 : 1; }

static double ee_a(const orc_system *s, int i, int j) {
  return spin_of(s, i) == spin_of(s, j) ? s->jee_a_para : s->jee_a_anti;
}

/* J = sum_{i<j} u_ee(r_ij) + sum_{i,A} u_A(r_iA) */
int orc_jastrow(const orc_system *s, const double *R, double *J, double *grad, double *lap) {
  const int ne = s->n_up + s->n_dn;
  double jv = 0.0;
  if (grad) memset(grad, 0, sizeof(double) * 3 * ne);
  if (lap) memset(lap, 0, sizeof(double) * ne);
  for (int i = 0; i < ne; ++i) {
    for (int j = 0; j < ne; ++j) {
      if (j == i) continue;
      const double d[3] = {R[3 * i] - R[3 * j], R[3 * i + 1] - R[3 * j + 1], R[3 * i + 2] - R[3 * j + 2]};
      const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const double a = ee_a(s, i, j), b = s->jee_b;
      if (j > i) jv += pade(a, b, r);
      const double u1 = pade_d1(a, b, r), u2 = pade_d2(a, b, r);
      if (grad)
        for (int x = 0; x < 3; ++x) grad[3 * i + x] += u1 * d[x] / r;
      if (lap) lap[i] += u2 + 2.0 * u1 / r;
    }
    for (int A = 0; A < s->n_atom; ++A) {
      const double *c = s->ion_xyz + 3 * A;
      const double d[3] = {R[3 * i] - c[0], R[3 * i + 1] - c[1], R[3 * i + 2] - c[2]};
      const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const double a = s->jen_a[A], b = s->jen_b;
      jv += pade(a, b, r);
      const double u1 = pade_d1(a, b, r), u2 = pade_d2(a, b, r);
      if (grad)
        for (int x = 0; x < 3; ++x) grad[3 * i + x] += u1 * d[x] / r;
      if (lap) lap[i] += u2 + 2.0 * u1 / r;
    }
  }
  if (J) *J = jv;
  return 0;
}

/* J and grad_i J of electron i placed at ri, the rest at R (one-electron sums). */
static void jastrow_one(const orc_system *s, const double *R, int i, const double ri[3], double *u,
                        double g[3]) {
  const int ne = s->n_up + s->n_dn;
  double acc = 0.0, gg[3] = {0, 0, 0};
  for (int j = 0; j < ne; ++j) {
    if (j == i) continue;
    const double d[3] = {ri[0] - R[3 * j], ri[1] - R[3 * j + 1], ri[2] - R[3 * j + 2]};
    const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double a = ee_a(s, i, j), b = s->jee_b;
    acc += pade(a, b, r);
    const double u1 = pade_d1(a, b, r);
    for (int x = 0; x < 3; ++x) gg[x] += u1 * d[x] / r;
  }
  for (int A = 0; A < s->n_atom; ++A) {
    const double *c = s->ion_xyz + 3 * A;
    const double d[3] = {ri[0] - c[0], ri[1] - c[1], ri[2] - c[2]};
    const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double a = s->jen_a[A], b = s->jen_b;
    acc += pade(a, b, r);
    const double u1 = pade_d1(a, b, r);
    for (int x = 0; x < 3; ++x) gg[x] += u1 * d[x] / r;
  }
  *u = acc;
  for (int x = 0; x < 3; ++x) g[x] = gg[x];
}

/* ----------------------------------------------------------- potential --- */
double orc_potential(const orc_system *s, const double *R) {
  const int ne = s->n_up + s->n_dn;
  double v = 0.0;
  for (int i = 0; i < ne; ++i)
    for (int j = i + 1; j < ne; ++j) {
      const double d[3] = {R[3 * i] - R[3 * j], R[3 * i + 1] - R[3 * j + 1], R[3 * i + 2] - R[3 * j + 2]};
      v += 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    }
  for (int i = 0; i < ne; ++i)
    for (int A = 0; A < s->n_atom; ++A) {
      const double *c = s->ion_xyz + 3 * A;
      const double d[3] = {R[3 * i] - c[0], R[3 * i + 1] - c[1], R[3 * i + 2] - c[2]};
      v -= s->ion_charge[A] / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    }
  for (int A = 0; A < s->n_atom; ++A)
    for (int B = A + 1; B < s->n_atom; ++B) {
      const double *a = s->ion_xyz + 3 * A, *b = s->ion_xyz + 3 * B;
      const double d[3] = {a[0] - b[0], a[1] - b[1], a[2] - b[2]};
      v += s->ion_charge[A] * s->ion_charge[B] / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    }
  /* local pseudopotential terms */
  for (int t = 0; t < s->pp_n_term; ++t) {
    if (s->pp_l[t] != -1) continue;
    const double *c = s->ion_xyz + 3 * s->pp_atom[t];
    for (int i = 0; i < ne; ++i) {
      const double d[3] = {R[3 * i] - c[0], R[3 * i + 1] - c[1], R[3 * i + 2] - c[2]};
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      v += s->pp_beta[t] * pow(sqrt(r2), s->pp_n[t] - 2) * exp(-s->pp_alpha[t] * r2);
    }
  }
  return v;
}

/* ---------------------------------------------------- walker state ------ */
typedef struct {
  int ne, nsig[2];
  double *rows;      /* [ne][5][nmax]: orbital VGL of each electron */
  double *A[2];      /* [n][n] value matrices */
  double *G[2];      /* [n][n] inverses (orbital x electron) */
  double logdet[2];
  int sign[2];
  int nmax;
} wstate;

static int ws_init(const orc_system *s, wstate *w, const double *R) {
  w->ne = s->n_up + s->n_dn;
  w->nsig[0] = s->n_up;
  w->nsig[1] = s->n_dn;
  w->nmax = s->n_up > s->n_dn ? s->n_up : s->n_dn;
  w->rows = (double *)calloc((size_t)w->ne * 5 * w->nmax + 1, sizeof(double));
  int rc = 0;
  for (int sp = 0; sp < 2; ++sp) {
    const int n = w->nsig[sp];
    w->A[sp] = (double *)calloc((size_t)n * n + 1, sizeof(double));
    w->G[sp] = (double *)calloc((size_t)n * n + 1, sizeof(double));
  }
  for (int i = 0; i < w->ne; ++i) {
    const int sp = spin_of(s, i), ii = i - sp * s->n_up, n = w->nsig[sp];
    double *row = w->rows + (size_t)i * 5 * w->nmax;
    rc |= orc_orbitals_vgl(s, R + 3 * i, n, row);
    /* orbitals_vgl packs [5][n]; re-stride to [5][nmax] */
    if (n != w->nmax)
      for (int c = 4; c >= 0; --c)
        for (int j = n - 1; j >= 0; --j) row[c * w->nmax + j] = row[c * n + j];
    for (int j = 0; j < n; ++j) w->A[sp][(size_t)ii * n + j] = row[j];
  }
  for (int sp = 0; sp < 2; ++sp) {
    if (w->nsig[sp] == 0) { w->logdet[sp] = 0.0; w->sign[sp] = 1; continue; }
    rc |= orc_lu_slogdet_inv(w->nsig[sp], w->A[sp], &w->logdet[sp], &w->sign[sp], w->G[sp]);
  }
  return rc;
}

static void ws_free(wstate *w) {
  free(w->rows);
  for (int sp = 0; sp < 2; ++sp) { free(w->A[sp]); free(w->G[sp]); }
}

/* (grad D / D) and (lap D / D) for electron i: Eq. 3 with B = grad A, lap A. */
static void det_derivs(const orc_system *s, const wstate *w, int i, double g[3], double *l) {
  const int sp = spin_of(s, i), ii = i - sp * s->n_up, n = w->nsig[sp];
  const double *row = w->rows + (size_t)i * 5 * w->nmax;
  double acc[4] = {0, 0, 0, 0};
  for (int j = 0; j < n; ++j) {
    const double gji = w->G[sp][(size_t)j * n + ii];
    for (int c = 0; c < 4; ++c) acc[c] += row[(c + 1) * w->nmax + j] * gji;
  }
  g[0] = acc[0];
  g[1] = acc[1];
  g[2] = acc[2];
  *l = acc[3];
}

/* E_L = -1/2 sum_i [lap_i J + |grad_i J|^2 + 2 grad_i J . g_i + l_i] + V */
static double ws_local_energy(const orc_system *s, const wstate *w, const double *R, double *Jout,
                              double *drift) {
  const int ne = w->ne;
  double *gj = (double *)malloc(sizeof(double) * 3 * ne);
  double *lj = (double *)malloc(sizeof(double) * ne);
  double J;
  orc_jastrow(s, R, &J, gj, lj);
  double kin = 0.0;
  for (int i = 0; i < ne; ++i) {
    double g[3], l;
    det_derivs(s, w, i, g, &l);
    const double *q = gj + 3 * i;
    kin += lj[i] + q[0] * q[0] + q[1] * q[1] + q[2] * q[2] +
           2.0 * (q[0] * g[0] + q[1] * g[1] + q[2] * g[2]) + l;
    if (drift)
      for (int x = 0; x < 3; ++x) drift[3 * i + x] = q[x] + g[x];
  }
  if (Jout) *Jout = J;
  free(gj);
  free(lj);
  return -0.5 * kin + orc_potential(s, R);
}

int orc_msd_evaluate(const orc_system *s, const double *R, double *log_psi, int32_t *sign,
                     double *e_local, double *drift);

int orc_evaluate(const orc_system *s, const double *R, double *log_psi, int32_t *sign,
                 double *e_local, double *drift) {
  if (s->n_det > 1) return orc_msd_evaluate(s, R, log_psi, sign, e_local, drift);
  wstate w;
  int rc = ws_init(s, &w, R);
  double J = 0.0;
  const double el = ws_local_energy(s, &w, R, &J, drift);
  if (log_psi) *log_psi = J + w.logdet[0] + w.logdet[1];
  if (sign) *sign = w.sign[0] * w.sign[1];
  if (e_local) *e_local = el;
  ws_free(&w);
  return rc;
}

int orc_evaluate_batch(const orc_system *s, int32_t W, const double *R, double *log_psi,
                       int32_t *sign, double *e_local, int32_t n_threads) {
  const int ne = s->n_up + s->n_dn;
  int rc = 0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(static) reduction(| : rc)
  for (int w = 0; w < W; ++w)
    rc |= orc_evaluate(s, R + (size_t)w * ne * 3, log_psi ? log_psi + w : NULL,
                       sign ? sign + w : NULL, e_local ? e_local + w : NULL, NULL);
  return rc;
}

/* --------------------------------------------------------------- Philox --- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
 * 32x32->64 multiplies with a Weyl-sequence key schedule. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Counter = (electron, walker, step low 32 bits, draw), key = seed. */
static void draw_uniform2(uint64_t seed, int64_t step, int32_t walker, int32_t elec, uint32_t draw,
                          double u[2]) {
  const uint32_t ctr[4] = {(uint32_t)elec, (uint32_t)walker, (uint32_t)(uint64_t)step, draw};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t x[4];
  orc_philox4x32_10(ctr, key, x);
  const uint64_t a = ((uint64_t)x[0] << 32) | x[1], b = ((uint64_t)x[2] << 32) | x[3];
  u[0] = (double)(a >> 11) * 0x1.0p-53;
  u[1] = (double)(b >> 11) * 0x1.0p-53;
}

/* Box-Muller: (sqrt(-2 ln(1-u1)) cos(2 pi u2), ... sin(2 pi u2)). */
void orc_move_draws(uint64_t seed, int64_t step, int32_t walker, int32_t elec, double chi[3],
                    double *u_acc) {
  const double twopi = 6.283185307179586476925286766559;
  double u[2];
  draw_uniform2(seed, step, walker, elec, 0u, u);
  double rad = sqrt(-2.0 * log(1.0 - u[0]));
  chi[0] = rad * cos(twopi * u[1]);
  chi[1] = rad * sin(twopi * u[1]);
  draw_uniform2(seed, step, walker, elec, 1u, u);
  rad = sqrt(-2.0 * log(1.0 - u[0]));
  chi[2] = rad * cos(twopi * u[1]);
  draw_uniform2(seed, step, walker, elec, 2u, u);
  *u_acc = u[0];
}

/* ------------------------------------------- non-local pseudopotential --- */
/* The paper's QMC runs use ccECP pseudopotentials (QMC section), whose
 * semilocal form is V = V_loc(r) + sum_l v_l(r) sum_m |lm><lm| per atom with
 * Gaussian radial terms.  The non-local part acts on Psi through the angular
 * integral over the sphere of radius r_iA about the atom,
 *   V_NL Psi / Psi = sum_l v_l(r_iA) (2l+1)/(4 pi) int dOmega P_l(cos) Psi(r')/Psi(r),
 * here by the 12-point icosahedral rule (weights 1/12, exact for the
 * polynomials of degree <= 5 on the sphere) whose directions are turned by a
 * uniformly random rotation per electron and evaluation (Shoemake's
 * quaternion from three uniforms).  Psi(r')/Psi(R) is taken from a fresh LU
 * of the Slater matrix with the electron's row replaced and the Jastrow
 * factor at both positions: the plain definition. */
static const double ICO_PHI = 1.6180339887498948482;

/* direction q of the icosahedral rule: cyclic permutations of (0, +-1, +-phi) */
static void ico_dir(int q, double d[3]) {
  const double a = (q & 1) ? -ICO_PHI : ICO_PHI; /* sign of the phi entry */
  const double b = (q & 2) ? -1.0 : 1.0;         /* sign of the 1 entry */
  const double nrm = 1.0 / sqrt(1.0 + ICO_PHI * ICO_PHI);
  double v[3];
  switch (q >> 2) {
    case 0: v[0] = 0.0; v[1] = b; v[2] = a; break;  /* (0, +-1, +-phi) */
    case 1: v[0] = b; v[1] = a; v[2] = 0.0; break;  /* (+-1, +-phi, 0) */
    default: v[0] = a; v[1] = 0.0; v[2] = b; break; /* (+-phi, 0, +-1) */
  }
  for (int x = 0; x < 3; ++x) d[x] = v[x] * nrm;
}

void orc_nlpp_rotation(uint64_t seed, int64_t step, int32_t walker, int32_t elec, double rot[9]) {
  const double twopi = 6.283185307179586476925286766559;
  double u[2], u3[2];
  draw_uniform2(seed, step, walker, elec, 3u, u);
  draw_uniform2(seed, step, walker, elec, 4u, u3);
  const double s1 = sqrt(1.0 - u[0]), s2 = sqrt(u[0]);
  const double x = s1 * sin(twopi * u[1]), y = s1 * cos(twopi * u[1]);
  const double z = s2 * sin(twopi * u3[0]), w = s2 * cos(twopi * u3[0]);
  rot[0] = 1.0 - 2.0 * (y * y + z * z); rot[1] = 2.0 * (x * y - z * w); rot[2] = 2.0 * (x * z + y * w);
  rot[3] = 2.0 * (x * y + z * w); rot[4] = 1.0 - 2.0 * (x * x + z * z); rot[5] = 2.0 * (y * z - x * w);
  rot[6] = 2.0 * (x * z - y * w); rot[7] = 2.0 * (y * z + x * w); rot[8] = 1.0 - 2.0 * (x * x + y * y);
}

static double legendre(int l, double x) {
  switch (l) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return 0.5 * (3.0 * x * x - 1.0);
    default: return 0.5 * (5.0 * x * x * x - 3.0 * x);
  }
}

int orc_nlpp(const orc_system *s, const double *R, uint64_t seed, int64_t step, int32_t walker,
             double *v_nl) {
  *v_nl = 0.0;
  if (s->pp_n_term == 0) return 0;
  if (s->n_det > 1) return 4;
  const int ne = s->n_up + s->n_dn;
  int rc = 0;
  /* Slater matrices, their log|det| and sign, and J at R */
  const int nmax = s->n_up > s->n_dn ? s->n_up : s->n_dn;
  double *A[2], ld[2];
  int32_t sg[2];
  double *orb = (double *)malloc(sizeof(double) * 5 * (nmax > 0 ? nmax : 1));
  double *Ak = (double *)malloc(sizeof(double) * (nmax * nmax > 0 ? nmax * nmax : 1));
  double *Rq = (double *)malloc(sizeof(double) * 3 * ne);
  for (int sp = 0; sp < 2; ++sp) {
    const int n = sp == 0 ? s->n_up : s->n_dn, e0 = sp == 0 ? 0 : s->n_up;
    A[sp] = (double *)malloc(sizeof(double) * (n * n > 0 ? n * n : 1));
    for (int i = 0; i < n; ++i) {
      rc |= orc_orbitals_vgl(s, R + 3 * (e0 + i), n, orb);
      for (int j = 0; j < n; ++j) A[sp][i * n + j] = orb[j];
    }
    ld[sp] = 0.0;
    sg[sp] = 1;
    if (n > 0) rc |= orc_lu_slogdet_inv(n, A[sp], &ld[sp], &sg[sp], NULL);
  }
  double J0;
  orc_jastrow(s, R, &J0, NULL, NULL);
  double acc = 0.0;
  for (int i = 0; i < ne; ++i) {
    const int sp = spin_of(s, i), n = sp == 0 ? s->n_up : s->n_dn, ii = i - sp * s->n_up;
    double rot[9];
    int have_rot = 0;
    for (int At = 0; At < s->n_atom; ++At) {
      /* the atom's non-local channels */
      int lmax = -1;
      for (int t = 0; t < s->pp_n_term; ++t)
        if (s->pp_atom[t] == At && s->pp_l[t] > lmax) lmax = s->pp_l[t];
      if (lmax < 0) continue;
      const double *c = s->ion_xyz + 3 * At;
      const double d[3] = {R[3 * i] - c[0], R[3 * i + 1] - c[1], R[3 * i + 2] - c[2]};
      const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      if (!(r < s->pp_rcut[At])) continue;
      if (!have_rot) {
        orc_nlpp_rotation(seed, step, walker, i, rot);
        have_rot = 1;
      }
      double vl[4] = {0.0, 0.0, 0.0, 0.0};
      for (int t = 0; t < s->pp_n_term; ++t)
        if (s->pp_atom[t] == At && s->pp_l[t] >= 0)
          vl[s->pp_l[t]] += s->pp_beta[t] * pow(r, s->pp_n[t] - 2) * exp(-s->pp_alpha[t] * r * r);
      for (int q = 0; q < 12; ++q) {
        double o[3], od[3];
        ico_dir(q, o);
        for (int x = 0; x < 3; ++x) od[x] = rot[3 * x] * o[0] + rot[3 * x + 1] * o[1] + rot[3 * x + 2] * o[2];
        const double cth = (od[0] * d[0] + od[1] * d[1] + od[2] * d[2]) / r;
        /* Psi with electron i at c + r od, over Psi(R) */
        for (int k = 0; k < 3 * ne; ++k) Rq[k] = R[k];
        for (int x = 0; x < 3; ++x) Rq[3 * i + x] = c[x] + r * od[x];
        rc |= orc_orbitals_vgl(s, Rq + 3 * i, n, orb);
        for (int k = 0; k < n * n; ++k) Ak[k] = A[sp][k];
        for (int j = 0; j < n; ++j) Ak[ii * n + j] = orb[j];
        double ldq;
        int32_t sgq;
        orc_lu_slogdet_inv(n, Ak, &ldq, &sgq, NULL);
        double Jq;
        orc_jastrow(s, Rq, &Jq, NULL, NULL);
        const double ratio = (double)(sgq * sg[sp]) * exp(ldq - ld[sp] + Jq - J0);
        double f = 0.0;
        for (int l = 0; l <= lmax; ++l) f += vl[l] * (2 * l + 1) * legendre(l, cth);
        acc += f * ratio / 12.0;
      }
    }
  }
  *v_nl = acc;
  for (int sp = 0; sp < 2; ++sp) free(A[sp]);
  free(orb);
  free(Ak);
  free(Rq);
  return rc;
}

/* Derivative of the pseudopotential operator with respect to its centres
 * (the Hellmann-Feynman part of the Eq. 3 force; Psi, with its basis and
 * Jastrow centres, held fixed): dvpp[A][3] = d(V_loc + V_NL)/dR_A at fixed
 * electrons and rotations.  With d = r_i - R_A, r = |d|, n = d / r,
 * o_q = Q Omega_q, c_q = o_q . n, r_q = R_A + r o_q, rho_q = Psi(r_q)/Psi(R):
 *   dr/dR_A = -n,  dc_q/dR_A = -(o_q - c_q n) / r,
 *   drho_q/dR_A = (I - o_q n^T)^T grad rho_q = g - n (o_q . g),
 *   g = rho_q grad_{r_q} ln Psi (the drift of electron i at the moved
 *   configuration, from a plain evaluation there). */
int orc_pp_ion_grads(const orc_system *s, const double *R, uint64_t seed, int64_t step,
                     int32_t walker, double *dvpp) {
  const int ne = s->n_up + s->n_dn;
  for (int k = 0; k < 3 * s->n_atom; ++k) dvpp[k] = 0.0;
  if (s->pp_n_term == 0) return 0;
  if (s->n_det > 1) return 4;
  int rc = 0;
  /* local terms: d/dR_A beta r^(n-2) exp(-alpha r^2) = -f'(r) n */
  for (int t = 0; t < s->pp_n_term; ++t) {
    if (s->pp_l[t] != -1) continue;
    const int A = s->pp_atom[t];
    const double *c = s->ion_xyz + 3 * A;
    for (int i = 0; i < ne; ++i) {
      const double d[3] = {R[3 * i] - c[0], R[3 * i + 1] - c[1], R[3 * i + 2] - c[2]};
      const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const int n = s->pp_n[t];
      const double f = s->pp_beta[t] * pow(r, n - 2) * exp(-s->pp_alpha[t] * r * r);
      const double fp = f * ((n - 2) / r - 2.0 * s->pp_alpha[t] * r);
      for (int x = 0; x < 3; ++x) dvpp[3 * A + x] -= fp * d[x] / r;
    }
  }
  double lp0, e0;
  int32_t sg0;
  rc |= orc_evaluate(s, R, &lp0, &sg0, &e0, NULL);
  double *Rq = (double *)malloc(sizeof(double) * 3 * ne);
  double *drq = (double *)malloc(sizeof(double) * 3 * ne);
  for (int i = 0; i < ne; ++i) {
    double rot[9];
    int have_rot = 0;
    for (int At = 0; At < s->n_atom; ++At) {
      int lmax = -1;
      for (int t = 0; t < s->pp_n_term; ++t)
        if (s->pp_atom[t] == At && s->pp_l[t] > lmax) lmax = s->pp_l[t];
      if (lmax < 0) continue;
      const double *c = s->ion_xyz + 3 * At;
      const double d[3] = {R[3 * i] - c[0], R[3 * i + 1] - c[1], R[3 * i + 2] - c[2]};
      const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      if (!(r < s->pp_rcut[At])) continue;
      if (!have_rot) {
        orc_nlpp_rotation(seed, step, walker, i, rot);
        have_rot = 1;
      }
      const double nv[3] = {d[0] / r, d[1] / r, d[2] / r};
      double vl[4] = {0, 0, 0, 0}, vlp[4] = {0, 0, 0, 0};
      for (int t = 0; t < s->pp_n_term; ++t)
        if (s->pp_atom[t] == At && s->pp_l[t] >= 0) {
          const int n = s->pp_n[t];
          const double f = s->pp_beta[t] * pow(r, n - 2) * exp(-s->pp_alpha[t] * r * r);
          vl[s->pp_l[t]] += f;
          vlp[s->pp_l[t]] += f * ((n - 2) / r - 2.0 * s->pp_alpha[t] * r);
        }
      for (int q = 0; q < 12; ++q) {
        double o[3], od[3];
        ico_dir(q, o);
        for (int x = 0; x < 3; ++x) od[x] = rot[3 * x] * o[0] + rot[3 * x + 1] * o[1] + rot[3 * x + 2] * o[2];
        const double cq = od[0] * nv[0] + od[1] * nv[1] + od[2] * nv[2];
        for (int k = 0; k < 3 * ne; ++k) Rq[k] = R[k];
        for (int x = 0; x < 3; ++x) Rq[3 * i + x] = c[x] + r * od[x];
        double lpq, eq;
        int32_t sgq;
        rc |= orc_evaluate(s, Rq, &lpq, &sgq, &eq, drq);
        const double rho = (double)(sgq * sg0) * exp(lpq - lp0);
        const double g[3] = {rho * drq[3 * i], rho * drq[3 * i + 1], rho * drq[3 * i + 2]};
        const double og = od[0] * g[0] + od[1] * g[1] + od[2] * g[2];
        double f = 0.0, fp = 0.0, fc = 0.0; /* sum_l (2l+1)/12 x (v_l P_l, v_l' P_l, v_l P_l') */
        for (int l = 0; l <= lmax; ++l) {
          const double P = legendre(l, cq);
          const double dP = l == 0 ? 0.0 : (l == 1 ? 1.0 : (l == 2 ? 3.0 * cq : 0.5 * (15.0 * cq * cq - 3.0)));
          f += (2 * l + 1) / 12.0 * vl[l] * P;
          fp += (2 * l + 1) / 12.0 * vlp[l] * P;
          fc += (2 * l + 1) / 12.0 * vl[l] * dP;
        }
        for (int x = 0; x < 3; ++x)
          dvpp[3 * At + x] += -fp * nv[x] * rho - fc * (od[x] - cq * nv[x]) / r * rho +
                              f * (g[x] - nv[x] * og);
      }
    }
  }
  free(Rq);
  free(drq);
  return rc;
}

int orc_nlpp_batch(const orc_system *s, int32_t W, const double *R, uint64_t seed, int64_t step,
                   int32_t walker_offset, double *v_nl, int32_t n_threads) {
  const int ne = s->n_up + s->n_dn;
  int rc = 0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic) reduction(| : rc)
  for (int w = 0; w < W; ++w)
    rc |= orc_nlpp(s, R + (size_t)w * ne * 3, seed, step, walker_offset + w, v_nl + w);
  return rc;
}

/* ---------------------------------------------------------------- DMC --- */
static int msd_walker_run(const orc_system *s, double *R, double *log_w, double *e_local,
                          int64_t step0, int32_t n_steps, int32_t mode, double tau, uint64_t seed,
                          double e_trial, int32_t walker_index, uint8_t *acc_row, size_t acc_stride,
                          double *e_row, size_t e_stride);

static int walker_run(const orc_system *s, int wi, double *R, double *log_w, double *e_local,
                      int64_t step0, int32_t n_steps, int32_t mode, double tau, uint64_t seed,
                      double e_trial, int32_t walker_index, uint8_t *acc_row, size_t acc_stride,
                      double *e_row, size_t e_stride) {
  if (s->n_det > 1) {
    if (s->pp_n_term > 0) return 4;  /* pseudopotentials: single determinant only */
    return msd_walker_run(s, R, log_w, e_local, step0, n_steps, mode, tau, seed, e_trial,
                          walker_index, acc_row, acc_stride, e_row, e_stride);
  }
  wstate w;
  int rc = ws_init(s, &w, R);
  const int ne = w.ne, nmax = w.nmax;
  double *trial = (double *)malloc(sizeof(double) * 5 * nmax);
  double e_old = ws_local_energy(s, &w, R, NULL, NULL);
  if (s->pp_n_term > 0) {
    double vnl;
    rc |= orc_nlpp(s, R, seed, step0, walker_index, &vnl);
    e_old += vnl;
  }
  const double sqt = sqrt(tau);
  for (int st = 0; st < n_steps; ++st) {
    const int64_t step = step0 + st;
    for (int i = 0; i < ne; ++i) {
      const int sp = spin_of(s, i), ii = i - sp * s->n_up, n = w.nsig[sp];
      double *ri = R + 3 * i;
      double *G = w.G[sp];
      /* drift at the current position */
      double uo, gjo[3], gd[3], l_unused;
      jastrow_one(s, R, i, ri, &uo, gjo);
      det_derivs(s, &w, i, gd, &l_unused);
      const double v[3] = {gjo[0] + gd[0], gjo[1] + gd[1], gjo[2] + gd[2]};
      double chi[3], uacc;
      orc_move_draws(seed, step, walker_index, i, chi, &uacc);
      double rn[3];
      for (int x = 0; x < 3; ++x) rn[x] = ri[x] + tau * v[x] + sqt * chi[x];
      rc |= orc_orbitals_vgl(s, rn, n, trial);
      /* determinant ratio: det(A')/det(A) = sum_j phi_j(r') (A^{-1})_{j i} */
      double rho = 0.0;
      for (int j = 0; j < n; ++j) rho += trial[j] * G[(size_t)j * n + ii];
      int accepted = 0;
      if (!(mode == 1 && !(rho > 0.0))) {
        double un, gjn[3];
        jastrow_one(s, R, i, rn, &un, gjn);
        /* grad ln D' at r': column i of the new inverse is G[:, i] / rho */
        double gdn[3] = {0, 0, 0};
        for (int j = 0; j < n; ++j)
          for (int x = 0; x < 3; ++x) gdn[x] += trial[(1 + x) * n + j] * G[(size_t)j * n + ii];
        double vn[3];
        for (int x = 0; x < 3; ++x) vn[x] = gjn[x] + gdn[x] / rho;
        double fwd = 0.0, bwd = 0.0;
        for (int x = 0; x < 3; ++x) {
          const double a = rn[x] - ri[x] - tau * v[x];
          const double b = ri[x] - rn[x] - tau * vn[x];
          fwd += a * a;
          bwd += b * b;
        }
        const double lnq = 2.0 * (log(fabs(rho)) + (un - uo)) + (fwd - bwd) / (2.0 * tau);
        const double p = lnq >= 0.0 ? 1.0 : exp(lnq);
        accepted = uacc < p;
      }
      if (accepted) {
        for (int x = 0; x < 3; ++x) ri[x] = rn[x];
        double *row = w.rows + (size_t)i * 5 * nmax;
        for (int c = 0; c < 5; ++c)
          for (int j = 0; j < n; ++j) row[c * nmax + j] = trial[c * n + j];
        for (int j = 0; j < n; ++j) w.A[sp][(size_t)ii * n + j] = trial[j];
        /* the inverse is always recomputed from scratch (plain definition) */
        rc |= orc_lu_slogdet_inv(n, w.A[sp], &w.logdet[sp], &w.sign[sp], G);
      }
      if (acc_row) acc_row[(size_t)st * acc_stride + i] = (uint8_t)accepted;
    }
    double e_new = ws_local_energy(s, &w, R, NULL, NULL);
    if (s->pp_n_term > 0) {
      double vnl;
      rc |= orc_nlpp(s, R, seed, step, walker_index, &vnl);
      e_new += vnl;
    }
    if (mode == 1) *log_w += -tau * (0.5 * (e_old + e_new) - e_trial);
    if (e_row) e_row[(size_t)st * e_stride] = e_new;
    e_old = e_new;
  }
  *e_local = e_old;
  (void)wi;
  free(trial);
  ws_free(&w);
  return rc;
}

int orc_run(const orc_system *s, int32_t W, double *R, double *log_w, double *e_local,
            int64_t step0, int32_t n_steps, int32_t mode, double tau, uint64_t seed,
            double e_trial, int32_t walker_offset, uint8_t *accept_log, double *e_log,
            int32_t n_threads) {
  const int ne = s->n_up + s->n_dn;
  int rc = 0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(static) reduction(| : rc)
  for (int w = 0; w < W; ++w) {
    rc |= walker_run(s, w, R + (size_t)w * ne * 3, log_w + w, e_local + w, step0, n_steps, mode,
                     tau, seed, e_trial, walker_offset + w,
                     accept_log ? accept_log + (size_t)w * ne : NULL, (size_t)W * ne,
                     e_log ? e_log + w : NULL, (size_t)W);
  }
  return rc;
}

/* ------------------------------------------------------- branching --- */
/* Birth/death branching of the DMC population (the weights of Eq. 1 turned
 * into walker counts; the paper leaves the control scheme open).  Walker j
 * has weight w_j = exp(log_w_j) (a non-finite log w or a non-zero flag: 0)
 * and M_j = floor(w_j + u_j) copies, u_j the first uniform of the Philox
 * draw 5 of (electron 0, walker j, step) under the key.  The new population
 * has W' = sum M_j walkers; its layout (the slot rule):
 *   - a walker with M_j >= 1 keeps its slot;
 *   - its M_j - 1 extra copies, walkers in order, fill the slots of the
 *     walkers without a copy, lowest first, and then the slots W, W + 1, ...;
 *   - when the extras do not fill every empty slot below W', the walkers in
 *     slots >= W' move, in slot order, into the empty slots below W', lowest
 *     first.
 * Every destination is an empty or new slot and every source a surviving
 * walker's own slot, so all copies read the population before the branch.
 * pairs[2p] = destination, pairs[2p + 1] = source, p < *n_pairs (W' + W at
 * most); copies[W] = M_j.  Returns 5 (nothing selected) when W' < 1 or
 * W' > cap. */
int orc_branch(int32_t W, const double *log_w, const uint8_t *flags, uint64_t seed, int64_t step,
               int32_t cap, int32_t *copies, int32_t *pairs, int32_t *n_pairs, int32_t *w_new) {
  double tot = 0.0;
  for (int j = 0; j < W; ++j) {
    double u[2];
    draw_uniform2(seed, step, j, 0, 5u, u);
    const int ok = isfinite(log_w[j]) && (!flags || flags[j] == 0);
    const double m = ok ? floor(exp(log_w[j]) + u[0]) : 0.0;
    tot += m;
    copies[j] = m > (double)cap ? cap + 1 : (int32_t)m;
  }
  *n_pairs = 0;
  *w_new = tot > (double)cap ? cap + 1 : (int32_t)tot;
  if (tot < 1.0 || tot > (double)cap) return 5;
  const int Wn = (int)tot;
  int np = 0;
  /* empty slots below W, in order; extras in walker order */
  int *empty = (int *)malloc(sizeof(int) * (W > 0 ? W : 1));
  int ne = 0;
  for (int j = 0; j < W; ++j)
    if (copies[j] == 0) empty[ne++] = j;
  int fill = 0, next_new = W;
  for (int j = 0; j < W; ++j)
    for (int k = 1; k < copies[j]; ++k) {
      const int dst = fill < ne ? empty[fill++] : next_new++;
      pairs[2 * np] = dst;
      pairs[2 * np + 1] = j;
      ++np;
    }
  /* remaining empty slots below W': filled by the walkers in slots >= W' */
  int mv = Wn; /* next slot >= W' to inspect */
  for (int e = fill; e < ne && empty[e] < Wn; ++e) {
    while (mv < W && copies[mv] == 0) ++mv;
    pairs[2 * np] = empty[e];
    pairs[2 * np + 1] = mv;
    ++np;
    ++mv;
  }
  free(empty);
  *n_pairs = np;
  *w_new = Wn;
  return 0;
}

/* ---------------------------------------------------- E_T feedback --- */
/* DMC steps with the trial energy of the projection (Eq. 1) fed back from
 * the population after every step (population control; the paper leaves E_T
 * open):  E_T <- <E_L>_w - (gain / tau) ln(W_tot / W_T),
 * <E_L>_w = sum_w omega_w E_w / sum_w omega_w, W_tot = sum_w exp(log w_w),
 * omega_w = exp(log w_w - m), m the largest log w, over the walkers whose
 * log w and E_L are finite (E_T unchanged if there is none).  Each step is
 * one orc_run step of every walker; et_log[s] (may be NULL) receives the E_T
 * that step s used, *e_trial_out the one the next step would use.  W_T is
 * the target population: w_target, or W when w_target is 0 (a population
 * that branching has moved away from its target feeds back through it). */
int orc_run_feedback(const orc_system *s, int32_t W, double *R, double *log_w, double *e_local,
                     int64_t step0, int32_t n_steps, double tau, uint64_t seed, double e_trial,
                     double gain, int32_t w_target, int32_t walker_offset, uint8_t *accept_log, double *e_log,
                     double *et_log, double *e_trial_out, int32_t n_threads) {
  const int ne = s->n_up + s->n_dn;
  int rc = 0;
  double et = e_trial;
  for (int st = 0; st < n_steps; ++st) {
    if (et_log) et_log[st] = et;
    rc |= orc_run(s, W, R, log_w, e_local, step0 + st, 1, 1, tau, seed, et, walker_offset,
                  accept_log ? accept_log + (size_t)st * W * ne : NULL,
                  e_log ? e_log + (size_t)st * W : NULL, n_threads);
    double m = -INFINITY;
    int any = 0;
    for (int w = 0; w < W; ++w)
      if (isfinite(log_w[w]) && isfinite(e_local[w])) {
        if (log_w[w] > m) m = log_w[w];
        any = 1;
      }
    if (!any) continue;
    double s0 = 0.0, s1 = 0.0;
    for (int w = 0; w < W; ++w)
      if (isfinite(log_w[w]) && isfinite(e_local[w])) {
        const double om = exp(log_w[w] - m);
        s0 += om;
        s1 += om * e_local[w];
      }
    const double ln_wtot = m + log(s0);
    et = s1 / s0 - gain / tau * (ln_wtot - log((double)(w_target > 0 ? w_target : W)));
  }
  if (e_trial_out) *e_trial_out = et;
  return rc;
}

/* ------------------------------------------- Jastrow parameter derivatives --- */
/* Derivatives of ln Psi and of E_L with respect to the Jastrow parameters
 * (QMC section: the Jastrow factor of Eq. 2; its parameters are what the
 * VMC linear-method optimisation varies).  Parameters, in order:
 *   0  b of the electron-electron Pade terms u = a r / (1 + b r),
 *   1  b of the electron-nucleus Pade terms,
 *   2..7  coefficients c_k of a three-body electron-electron-nucleus term
 *      J3 = sum_k c_k sum_A sum_{i<j} (s_iA^l s_jA^m + s_iA^m s_jA^l) s_ij^n,
 *      s(r) = r / (1 + r), (l, m, n) = (1,1,0), (1,0,1), (1,1,1), (2,1,0),
 *      (2,0,1), (1,0,2), entering at c = 0 (the trial function is unchanged;
 *      these are the derivatives of a first optimisation step).
 * With O_p = d ln Psi / dp = dJ / dp and v_i = grad_i ln|Psi|,
 *   dE_L / dp = -1/2 sum_i [lap_i O_p + 2 v_i . grad_i O_p].
 * dlogpsi[8] = O_p, dEL[8].  Single determinant only (4 otherwise). */
static const int J3_LMN[6][3] = {{1, 1, 0}, {1, 0, 1}, {1, 1, 1}, {2, 1, 0}, {2, 0, 1}, {1, 0, 2}};

static double ipow(double x, int k) {
  double r = 1.0;
  for (int q = 0; q < k; ++q) r *= x;
  return r;
}

/* d/db of a r / (1 + b r) and its first two r-derivatives */
static void pade_db(double a, double b, double r, double *h, double *h1, double *h2) {
  const double q = 1.0 / (1.0 + b * r);
  *h = -a * r * r * q * q;
  *h1 = -2.0 * a * r * q * q * q;
  *h2 = -2.0 * a * (1.0 - 2.0 * b * r) * q * q * q * q;
}

int orc_jastrow_param_grads(const orc_system *s, const double *R, double *dlogpsi, double *dEL) {
  if (s->n_det > 1) return 4;
  const int ne = s->n_up + s->n_dn, na = s->n_atom, NP8 = 8;
  double lp, el;
  int32_t sg;
  double *v = (double *)malloc(sizeof(double) * 3 * ne);
  double *go = (double *)calloc((size_t)NP8 * ne * 3, sizeof(double));  /* grad_i O_p */
  double *lo = (double *)calloc((size_t)NP8 * ne, sizeof(double));      /* lap_i O_p */
  int rc = orc_evaluate(s, R, &lp, &sg, &el, v);
  for (int p = 0; p < NP8; ++p) dlogpsi[p] = 0.0;
  for (int i = 0; i < ne; ++i) {
    const double *ri = R + 3 * i;
    /* electron-electron Pade b */
    for (int j = 0; j < ne; ++j) {
      if (j == i) continue;
      const double d[3] = {ri[0] - R[3 * j], ri[1] - R[3 * j + 1], ri[2] - R[3 * j + 2]};
      const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      double h, h1, h2;
      pade_db(ee_a(s, i, j), s->jee_b, r, &h, &h1, &h2);
      if (j > i) dlogpsi[0] += h;
      for (int x = 0; x < 3; ++x) go[(0 * ne + i) * 3 + x] += h1 * d[x] / r;
      lo[0 * ne + i] += h2 + 2.0 * h1 / r;
    }
    /* electron-nucleus Pade b */
    for (int A = 0; A < na; ++A) {
      const double *c = s->ion_xyz + 3 * A;
      const double d[3] = {ri[0] - c[0], ri[1] - c[1], ri[2] - c[2]};
      const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      double h, h1, h2;
      pade_db(s->jen_a[A], s->jen_b, r, &h, &h1, &h2);
      dlogpsi[1] += h;
      for (int x = 0; x < 3; ++x) go[(1 * ne + i) * 3 + x] += h1 * d[x] / r;
      lo[1 * ne + i] += h2 + 2.0 * h1 / r;
    }
    /* three-body terms: f(x, y, z) with x = |r_i - R_A|, y = |r_j - R_A|,
     * z = |r_i - r_j|; electron i sees df/dx along (r_i - R_A)/x and df/dz
     * along (r_i - r_j)/z */
    for (int j = 0; j < ne; ++j) {
      if (j == i) continue;
      const double dz[3] = {ri[0] - R[3 * j], ri[1] - R[3 * j + 1], ri[2] - R[3 * j + 2]};
      const double z = sqrt(dz[0] * dz[0] + dz[1] * dz[1] + dz[2] * dz[2]);
      for (int A = 0; A < na; ++A) {
        const double *c = s->ion_xyz + 3 * A;
        const double dx[3] = {ri[0] - c[0], ri[1] - c[1], ri[2] - c[2]};
        const double x = sqrt(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
        const double y = sqrt((R[3 * j] - c[0]) * (R[3 * j] - c[0]) +
                              (R[3 * j + 1] - c[1]) * (R[3 * j + 1] - c[1]) +
                              (R[3 * j + 2] - c[2]) * (R[3 * j + 2] - c[2]));
        const double sx = x / (1.0 + x), sy = y / (1.0 + y), sz = z / (1.0 + z);
        const double sx1 = 1.0 / ((1.0 + x) * (1.0 + x)), sz1 = 1.0 / ((1.0 + z) * (1.0 + z));
        const double sx2 = -2.0 / ((1.0 + x) * (1.0 + x) * (1.0 + x));
        const double sz2 = -2.0 / ((1.0 + z) * (1.0 + z) * (1.0 + z));
        double cosxz = 0.0;
        for (int q = 0; q < 3; ++q) cosxz += dx[q] * dz[q];
        cosxz /= x * z;
        for (int k = 0; k < 6; ++k) {
          const int l = J3_LMN[k][0], m = J3_LMN[k][1], n = J3_LMN[k][2];
          /* P(sx) = sx^l sy^m + sx^m sy^l and its sx-derivatives; Q(sz) = sz^n */
          const double P = ipow(sx, l) * ipow(sy, m) + ipow(sx, m) * ipow(sy, l);
          const double P1 = (l ? l * ipow(sx, l - 1) * ipow(sy, m) : 0.0) +
                            (m ? m * ipow(sx, m - 1) * ipow(sy, l) : 0.0);
          const double P2 = (l > 1 ? l * (l - 1) * ipow(sx, l - 2) * ipow(sy, m) : 0.0) +
                            (m > 1 ? m * (m - 1) * ipow(sx, m - 2) * ipow(sy, l) : 0.0);
          const double Q = ipow(sz, n);
          const double Q1 = n ? n * ipow(sz, n - 1) : 0.0;
          const double Q2 = n > 1 ? n * (n - 1) * ipow(sz, n - 2) : 0.0;
          if (j > i) dlogpsi[2 + k] += P * Q;
          const double fx = P1 * sx1 * Q, fz = P * Q1 * sz1;
          const double fxx = (P2 * sx1 * sx1 + P1 * sx2) * Q;
          const double fzz = P * (Q2 * sz1 * sz1 + Q1 * sz2);
          const double fxz = P1 * sx1 * Q1 * sz1;
          for (int q = 0; q < 3; ++q) go[((2 + k) * ne + i) * 3 + q] += fx * dx[q] / x + fz * dz[q] / z;
          lo[(2 + k) * ne + i] += fxx + fzz + 2.0 * fxz * cosxz + 2.0 * fx / x + 2.0 * fz / z;
        }
      }
    }
  }
  for (int p = 0; p < NP8; ++p) {
    double acc = 0.0;
    for (int i = 0; i < ne; ++i) {
      double vg = 0.0;
      for (int x = 0; x < 3; ++x) vg += v[3 * i + x] * go[(p * ne + i) * 3 + x];
      acc += lo[p * ne + i] + 2.0 * vg;
    }
    dEL[p] = -0.5 * acc;
  }
  free(v);
  free(go);
  free(lo);
  return rc;
}

int orc_j3_values(const orc_system *s, const double *R, double *F) {
  const int ne = s->n_up + s->n_dn;
  for (int k = 0; k < 6; ++k) F[k] = 0.0;
  for (int A = 0; A < s->n_atom; ++A)
    for (int i = 0; i < ne; ++i)
      for (int j = i + 1; j < ne; ++j) {
        double x2 = 0.0, y2 = 0.0, z2 = 0.0;
        for (int q = 0; q < 3; ++q) {
          const double a = R[3 * i + q] - s->ion_xyz[3 * A + q];
          const double b = R[3 * j + q] - s->ion_xyz[3 * A + q];
          const double c = R[3 * i + q] - R[3 * j + q];
          x2 += a * a;
          y2 += b * b;
          z2 += c * c;
        }
        const double x = sqrt(x2), y = sqrt(y2), z = sqrt(z2);
        const double sx = x / (1.0 + x), sy = y / (1.0 + y), sz = z / (1.0 + z);
        for (int k = 0; k < 6; ++k) {
          const int l = J3_LMN[k][0], m = J3_LMN[k][1], n = J3_LMN[k][2];
          F[k] += (ipow(sx, l) * ipow(sy, m) + ipow(sx, m) * ipow(sy, l)) * ipow(sz, n);
        }
      }
  return 0;
}

/* The eight Jastrow-parameter directions of a configuration, from their
 * definitions: O_0 = sum_{i<j} dU_ee/db, O_1 = sum_{i,A} dU_en/db,
 * O_{2+k} = F_k(R) (the three-body sums). */
static void jastrow_param_values(const orc_system *s, const double *R, double O[8]) {
  const int ne = s->n_up + s->n_dn;
  double h, h1, h2;
  O[0] = O[1] = 0.0;
  for (int i = 0; i < ne; ++i) {
    for (int j = i + 1; j < ne; ++j) {
      double r2 = 0.0;
      for (int x = 0; x < 3; ++x) r2 += (R[3 * i + x] - R[3 * j + x]) * (R[3 * i + x] - R[3 * j + x]);
      pade_db(ee_a(s, i, j), s->jee_b, sqrt(r2), &h, &h1, &h2);
      O[0] += h;
    }
    for (int A = 0; A < s->n_atom; ++A) {
      double r2 = 0.0;
      for (int x = 0; x < 3; ++x)
        r2 += (R[3 * i + x] - s->ion_xyz[3 * A + x]) * (R[3 * i + x] - s->ion_xyz[3 * A + x]);
      pade_db(s->jen_a[A], s->jen_b, sqrt(r2), &h, &h1, &h2);
      O[1] += h;
    }
  }
  orc_j3_values(s, R, O + 2);
}

/* Derivatives of the non-local pseudopotential energy with respect to the
 * eight Jastrow parameters (the same directions as orc_jastrow_param_grads,
 * whose dEL covers the kinetic part): each quadrature ratio Psi(R_q)/Psi(R)
 * carries exp(J(R_q) - J(R)), so at fixed rotations
 *   dV_NL/dp = sum_{i,A,q} (1/12) f_q rho_q (O_p(R_q) - O_p(R)),
 * f_q = sum_l v_l(r) (2l+1) P_l(cos theta_q), O_p as above.  Straight from
 * that sum: every moved configuration is evaluated in full.  dv[8]. */
int orc_nlpp_param_grads(const orc_system *s, const double *R, uint64_t seed, int64_t step,
                         int32_t walker, double *dv) {
  for (int p = 0; p < 8; ++p) dv[p] = 0.0;
  if (s->pp_n_term == 0) return 0;
  if (s->n_det > 1) return 4;
  const int ne = s->n_up + s->n_dn;
  double *Rq = (double *)malloc(sizeof(double) * 3 * ne);
  double lp0, lpq, O0[8], Oq[8];
  int32_t sg0, sgq;
  int rc = orc_evaluate(s, R, &lp0, &sg0, NULL, NULL);
  jastrow_param_values(s, R, O0);
  for (int i = 0; i < ne; ++i) {
    double rot[9];
    int have_rot = 0;
    for (int At = 0; At < s->n_atom; ++At) {
      int lmax = -1;
      for (int t = 0; t < s->pp_n_term; ++t)
        if (s->pp_atom[t] == At && s->pp_l[t] > lmax) lmax = s->pp_l[t];
      if (lmax < 0) continue;
      const double *c = s->ion_xyz + 3 * At;
      const double d[3] = {R[3 * i] - c[0], R[3 * i + 1] - c[1], R[3 * i + 2] - c[2]};
      const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      if (!(r < s->pp_rcut[At])) continue;
      if (!have_rot) {
        orc_nlpp_rotation(seed, step, walker, i, rot);
        have_rot = 1;
      }
      double vl[4] = {0.0, 0.0, 0.0, 0.0};
      for (int t = 0; t < s->pp_n_term; ++t)
        if (s->pp_atom[t] == At && s->pp_l[t] >= 0)
          vl[s->pp_l[t]] += s->pp_beta[t] * pow(r, s->pp_n[t] - 2) * exp(-s->pp_alpha[t] * r * r);
      for (int q = 0; q < 12; ++q) {
        double o[3], od[3];
        ico_dir(q, o);
        for (int x = 0; x < 3; ++x) od[x] = rot[3 * x] * o[0] + rot[3 * x + 1] * o[1] + rot[3 * x + 2] * o[2];
        const double cth = (od[0] * d[0] + od[1] * d[1] + od[2] * d[2]) / r;
        for (int k = 0; k < 3 * ne; ++k) Rq[k] = R[k];
        for (int x = 0; x < 3; ++x) Rq[3 * i + x] = c[x] + r * od[x];
        rc |= orc_evaluate(s, Rq, &lpq, &sgq, NULL, NULL);
        jastrow_param_values(s, Rq, Oq);
        const double ratio = (double)(sgq * sg0) * exp(lpq - lp0);
        double f = 0.0;
        for (int l = 0; l <= lmax; ++l) f += vl[l] * (2 * l + 1) * legendre(l, cth);
        for (int p = 0; p < 8; ++p) dv[p] += f * ratio * (Oq[p] - O0[p]) / 12.0;
      }
    }
  }
  free(Rq);
  return rc;
}

int orc_jastrow_param_grads_batch(const orc_system *s, int32_t W, const double *R,
                                  double *dlogpsi, double *dEL, int32_t n_threads) {
  const int ne = s->n_up + s->n_dn;
  int rc = 0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic) reduction(| : rc)
  for (int w = 0; w < W; ++w)
    rc |= orc_jastrow_param_grads(s, R + (size_t)w * ne * 3, dlogpsi + 8 * w, dEL + 8 * w);
  return rc;
}

/* ---------------------------------------------------------- ion grads --- */
/* d ln|D_sigma| / dR_{a,x} = tr(G B), B_ij = dA_ij/dR_{a,x}
 *                          = -sum_{l on atom a} C_lj dPhi_l/dx (r_i)   (Eq. 3)
 * dJ/dR_a = -sum_i u_a'(r_ia) (r_i - R_a)/r_ia
 * dV/dR_a = -Z_a sum_i (r_i - R_a)/r_ia^3 - sum_{b != a} Z_a Z_b (R_a - R_b)/R_ab^3 */
static int msd_ion_det_grads(const orc_system *s, const double *R, double *dlogpsi);

int orc_ion_grads(const orc_system *s, const double *R, double *dlogpsi, double *dV) {
  wstate w;
  int rc = ws_init(s, &w, R);
  const int ne = w.ne, na = s->n_atom, nb = s->n_basis;
  int *fn_atom = (int *)malloc(sizeof(int) * nb);
  for (int sh = 0, f = 0; sh < s->n_shell; ++sh)
    for (int k = 0; k < NCART[s->shell_l[sh]]; ++k) fn_atom[f++] = s->shell_atom[sh];
  memset(dlogpsi, 0, sizeof(double) * 3 * na);
  memset(dV, 0, sizeof(double) * 3 * na);
  double *bvgl = (double *)malloc(sizeof(double) * 5 * nb);
  if (s->n_det > 1) rc |= msd_ion_det_grads(s, R, dlogpsi);
  for (int sp = 0; sp < 2 && s->n_det <= 1; ++sp) {
    const int n = w.nsig[sp];
    if (n == 0) continue;
    /* B[a][x][i][j] */
    double *B = (double *)calloc((size_t)na * 3 * n * n + 1, sizeof(double));
    for (int ii = 0; ii < n; ++ii) {
      const int i = ii + sp * s->n_up;
      rc |= orc_basis_vgl(s, R + 3 * i, bvgl);
      for (int l = 0; l < nb; ++l) {
        const int a = fn_atom[l];
        for (int x = 0; x < 3; ++x) {
          const double dphi = bvgl[5 * l + 1 + x];
          double *Bax = B + ((size_t)(a * 3 + x) * n + ii) * n;
          for (int j = 0; j < n; ++j) Bax[j] -= s->mo_coef[(size_t)l * s->n_mo + j] * dphi;
        }
      }
    }
    for (int a = 0; a < na; ++a)
      for (int x = 0; x < 3; ++x) {
        const double *Bax = B + (size_t)(a * 3 + x) * n * n;
        double tr = 0.0;
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j) tr += w.G[sp][(size_t)j * n + i] * Bax[(size_t)i * n + j];
        dlogpsi[3 * a + x] += tr;
      }
    free(B);
  }
  for (int a = 0; a < na; ++a) {
    const double *c = s->ion_xyz + 3 * a;
    for (int i = 0; i < ne; ++i) {
      const double d[3] = {R[3 * i] - c[0], R[3 * i + 1] - c[1], R[3 * i + 2] - c[2]};
      const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const double u1 = pade_d1(s->jen_a[a], s->jen_b, r);
      for (int x = 0; x < 3; ++x) {
        dlogpsi[3 * a + x] -= u1 * d[x] / r;
        dV[3 * a + x] -= s->ion_charge[a] * d[x] / (r * r * r);
      }
    }
    for (int b = 0; b < na; ++b) {
      if (b == a) continue;
      const double *e = s->ion_xyz + 3 * b;
      const double d[3] = {c[0] - e[0], c[1] - e[1], c[2] - e[2]};
      const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      for (int x = 0; x < 3; ++x)
        dV[3 * a + x] -= s->ion_charge[a] * s->ion_charge[b] * d[x] / (r * r * r);
    }
  }
  free(bvgl);
  free(fn_atom);
  ws_free(&w);
  return rc;
}

int orc_ion_grads_batch(const orc_system *s, int32_t W, const double *R, double *dlogpsi,
                        double *dV, int32_t n_threads) {
  const int ne = s->n_up + s->n_dn, na = s->n_atom;
  int rc = 0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(static) reduction(| : rc)
  for (int w = 0; w < W; ++w)
    rc |= orc_ion_grads(s, R + (size_t)w * ne * 3, dlogpsi + (size_t)w * na * 3,
                        dV + (size_t)w * na * 3);
  return rc;
}

/* ------------------------------------------------------------------ MSD --- */
/* Psi_MSD / Psi_0 = sum_d c_d (D_d^up / D_0^up)(D_d^dn / D_0^dn), each
 * excited determinant from its own LU (Eq. 2 with M > 1).  det_exc rows:
 * [nu, nd, hu0, hu1, pu0, pu1, hd0, hd1, pd0, pd1]; a hole is an occupied
 * orbital index, a particle the MO index that replaces it. */
static double det_with_columns(const orc_system *s, const double *R, int sp, const int *cols,
                               int n, int32_t *sgn) {
  double *A = (double *)malloc(sizeof(double) * (size_t)n * n + 1);
  double *ob = (double *)malloc(sizeof(double) * 5 * (size_t)s->n_mo + 1);
  for (int ii = 0; ii < n; ++ii) {
    const int i = ii + sp * s->n_up;
    orc_orbitals_vgl(s, R + 3 * i, s->n_mo, ob);
    for (int j = 0; j < n; ++j) A[(size_t)ii * n + j] = ob[cols[j]];
  }
  double ld;
  orc_lu_slogdet_inv(n, A, &ld, sgn, NULL);
  free(A);
  free(ob);
  return ld;
}

int orc_msd_ratio_direct(const orc_system *s, const double *R, double *psi_over_psi0) {
  const int nsig[2] = {s->n_up, s->n_dn};
  double ld0[2];
  int32_t sg0[2];
  int *cols = (int *)malloc(sizeof(int) * (size_t)(nsig[0] > nsig[1] ? nsig[0] : nsig[1]) + 1);
  for (int sp = 0; sp < 2; ++sp) {
    for (int j = 0; j < nsig[sp]; ++j) cols[j] = j;
    ld0[sp] = det_with_columns(s, R, sp, cols, nsig[sp], &sg0[sp]);
  }
  double acc = 0.0;
  for (int d = 0; d < s->n_det; ++d) {
    const int32_t *e = s->det_exc + 10 * d;
    double term = s->ci_coef[d];
    for (int sp = 0; sp < 2; ++sp) {
      const int ne = e[sp];
      if (ne == 0) continue;
      const int *h = e + (sp == 0 ? 2 : 6), *p = e + (sp == 0 ? 4 : 8);
      for (int j = 0; j < nsig[sp]; ++j) cols[j] = j;
      for (int k = 0; k < ne; ++k) cols[h[k]] = p[k];
      int32_t sg;
      const double ld = det_with_columns(s, R, sp, cols, nsig[sp], &sg);
      term *= (double)(sg * sg0[sp]) * exp(ld - ld0[sp]);
    }
    acc += term;
  }
  free(cols);
  *psi_over_psi0 = acc;
  return 0;
}

/* ----------------------------------------- multideterminant value, E_L --- */
/* Psi = exp(J) Phi, Phi = sum_d c_d D_d^up D_d^dn (Eq. 2 with M > 1).  Every
 * determinant is built from its own columns and gets its own LU inverse; its
 * per-electron log-derivatives follow from Eq. 3 with that inverse:
 *   grad_i D_d / D_d = sum_j grad phi_{c_j}(r_i) (A_d^{-1})_{j i}, same for lap.
 * With R_d^s = D_d^s / D_0^s and S = sum_d c_d R_d^up R_d^dn:
 *   grad_i Phi / Phi = sum_d c_d R_d^up R_d^dn grad_i D_d / D_d / S,
 *   lap_i Phi / Phi  = sum_d c_d R_d^up R_d^dn lap_i D_d / D_d / S,
 *   E_L = -1/2 sum_i [lap_i J + |grad_i J|^2 + 2 grad_i J . grad_i Phi/Phi
 *                     + lap_i Phi/Phi] + V. */

/* highest MO index the expansion refers to, plus one */
static int msd_n_mo(const orc_system *s) {
  int nmo = s->n_up > s->n_dn ? s->n_up : s->n_dn;
  for (int d = 0; d < s->n_det; ++d)
    for (int k = 0; k < 4; ++k) {
      const int p = s->det_exc[10 * d + (k < 2 ? 4 + k : 6 + k)];
      if (p + 1 > nmo) nmo = p + 1;
    }
  return nmo;
}

/* one spin of every determinant at the orbital table orb[ne][5][nmo] */
typedef struct {
  int n;            /* electrons of this spin */
  double ld0;       /* log|D_0| */
  int sg0;          /* sign D_0 */
  double *ratio;    /* [n_det] D_d / D_0 */
  double *g;        /* [n_det][n][3] grad_i D_d / D_d */
  double *l;        /* [n_det][n] lap_i D_d / D_d */
} msd_spin;

static void msd_spin_alloc(const orc_system *s, msd_spin *m, int sp) {
  m->n = sp == 0 ? s->n_up : s->n_dn;
  m->ratio = (double *)calloc((size_t)s->n_det + 1, sizeof(double));
  m->g = (double *)calloc((size_t)s->n_det * m->n * 3 + 1, sizeof(double));
  m->l = (double *)calloc((size_t)s->n_det * m->n + 1, sizeof(double));
}

static void msd_spin_free(msd_spin *m) {
  free(m->ratio);
  free(m->g);
  free(m->l);
}

static void msd_spin_copy(const orc_system *s, msd_spin *dst, const msd_spin *src) {
  dst->ld0 = src->ld0;
  dst->sg0 = src->sg0;
  memcpy(dst->ratio, src->ratio, sizeof(double) * s->n_det);
  memcpy(dst->g, src->g, sizeof(double) * s->n_det * src->n * 3);
  memcpy(dst->l, src->l, sizeof(double) * s->n_det * src->n);
}

static int msd_spin_eval(const orc_system *s, const double *orb, int nmo, int sp, msd_spin *m) {
  const int n = m->n, e0 = sp == 0 ? 0 : s->n_up;
  int rc = 0;
  if (n == 0) {
    m->ld0 = 0.0;
    m->sg0 = 1;
    for (int d = 0; d < s->n_det; ++d) m->ratio[d] = 1.0;
    return 0;
  }
  double *A = (double *)malloc(sizeof(double) * (size_t)n * n);
  double *G = (double *)malloc(sizeof(double) * (size_t)n * n);
  int *cols = (int *)malloc(sizeof(int) * (size_t)n);
  for (int d = 0; d < s->n_det; ++d) {
    const int32_t *e = s->det_exc + 10 * d;
    const int nx = e[sp];
    if (d > 0 && nx == 0) {  /* same columns as the reference */
      m->ratio[d] = 1.0;
      memcpy(m->g + (size_t)d * n * 3, m->g, sizeof(double) * n * 3);
      memcpy(m->l + (size_t)d * n, m->l, sizeof(double) * n);
      continue;
    }
    for (int j = 0; j < n; ++j) cols[j] = j;
    const int *h = e + (sp == 0 ? 2 : 6), *p = e + (sp == 0 ? 4 : 8);
    for (int k = 0; k < nx; ++k) cols[h[k]] = p[k];
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = orb[((size_t)(e0 + i) * 5) * nmo + cols[j]];
    double ld;
    int32_t sg;
    const int sing = orc_lu_slogdet_inv(n, A, &ld, &sg, G);
    if (d == 0) {
      rc |= sing;
      m->ld0 = ld;
      m->sg0 = sg;
    }
    if (sing) {  /* a vanishing excited determinant drops out of the sum */
      m->ratio[d] = 0.0;
      continue;
    }
    m->ratio[d] = d == 0 ? 1.0 : (double)(sg * m->sg0) * exp(ld - m->ld0);
    for (int i = 0; i < n; ++i) {
      const double *row = orb + (size_t)(e0 + i) * 5 * nmo;
      double acc[4] = {0, 0, 0, 0};
      for (int j = 0; j < n; ++j) {
        const double gji = G[(size_t)j * n + i];
        for (int c = 0; c < 4; ++c) acc[c] += row[(size_t)(c + 1) * nmo + cols[j]] * gji;
      }
      for (int x = 0; x < 3; ++x) m->g[((size_t)d * n + i) * 3 + x] = acc[x];
      m->l[(size_t)d * n + i] = acc[3];
    }
  }
  free(A);
  free(G);
  free(cols);
  return rc;
}

/* log|Phi|, sign(Phi), and (if dphi/lphi) grad_i Phi / Phi, lap_i Phi / Phi */
static void msd_combine(const orc_system *s, const msd_spin m[2], double *logabs, int *sign,
                        double *dphi, double *lphi) {
  double S = 0.0;
  for (int d = 0; d < s->n_det; ++d) S += s->ci_coef[d] * m[0].ratio[d] * m[1].ratio[d];
  *logabs = m[0].ld0 + m[1].ld0 + log(fabs(S));
  *sign = m[0].sg0 * m[1].sg0 * (S > 0.0 ? 1 : (S < 0.0 ? -1 : 0));
  if (!dphi && !lphi) return;
  for (int sp = 0; sp < 2; ++sp) {
    const int n = m[sp].n, e0 = sp == 0 ? 0 : s->n_up;
    for (int i = 0; i < n; ++i) {
      double g[3] = {0, 0, 0}, l = 0.0;
      for (int d = 0; d < s->n_det; ++d) {
        const double w = s->ci_coef[d] * m[0].ratio[d] * m[1].ratio[d];
        for (int x = 0; x < 3; ++x) g[x] += w * m[sp].g[((size_t)d * n + i) * 3 + x];
        l += w * m[sp].l[(size_t)d * n + i];
      }
      if (dphi)
        for (int x = 0; x < 3; ++x) dphi[3 * (e0 + i) + x] = g[x] / S;
      if (lphi) lphi[e0 + i] = l / S;
    }
  }
}

static int msd_orbital_table(const orc_system *s, const double *R, int nmo, double *orb) {
  const int ne = s->n_up + s->n_dn;
  int rc = 0;
  for (int i = 0; i < ne; ++i) rc |= orc_orbitals_vgl(s, R + 3 * i, nmo, orb + (size_t)i * 5 * nmo);
  return rc;
}

static double msd_local_energy(const orc_system *s, const double *R, const msd_spin m[2],
                               double *J, double *logabs, int *sign, double *drift) {
  const int ne = s->n_up + s->n_dn;
  double *dphi = (double *)malloc(sizeof(double) * 3 * ne);
  double *lphi = (double *)malloc(sizeof(double) * ne);
  double *gj = (double *)malloc(sizeof(double) * 3 * ne);
  double *lj = (double *)malloc(sizeof(double) * ne);
  msd_combine(s, m, logabs, sign, dphi, lphi);
  orc_jastrow(s, R, J, gj, lj);
  double kin = 0.0;
  for (int i = 0; i < ne; ++i) {
    const double *q = gj + 3 * i, *g = dphi + 3 * i;
    kin += lj[i] + q[0] * q[0] + q[1] * q[1] + q[2] * q[2] +
           2.0 * (q[0] * g[0] + q[1] * g[1] + q[2] * g[2]) + lphi[i];
    if (drift)
      for (int x = 0; x < 3; ++x) drift[3 * i + x] = q[x] + g[x];
  }
  free(dphi);
  free(lphi);
  free(gj);
  free(lj);
  return -0.5 * kin + orc_potential(s, R);
}

int orc_msd_evaluate(const orc_system *s, const double *R, double *log_psi, int32_t *sign,
                     double *e_local, double *drift) {
  const int ne = s->n_up + s->n_dn, nmo = msd_n_mo(s);
  double *orb = (double *)malloc(sizeof(double) * (size_t)ne * 5 * nmo);
  int rc = msd_orbital_table(s, R, nmo, orb);
  msd_spin m[2];
  for (int sp = 0; sp < 2; ++sp) {
    msd_spin_alloc(s, &m[sp], sp);
    rc |= msd_spin_eval(s, orb, nmo, sp, &m[sp]);
  }
  double J, la;
  int sg;
  const double el = msd_local_energy(s, R, m, &J, &la, &sg, drift);
  if (log_psi) *log_psi = J + la;
  if (sign) *sign = sg;
  if (e_local) *e_local = el;
  for (int sp = 0; sp < 2; ++sp) msd_spin_free(&m[sp]);
  free(orb);
  return rc;
}

/* The DMC step of walker_run with the multideterminant Psi: every proposal
 * re-evaluates all determinants of the mover's spin at R' from scratch, the
 * ratio is Phi(R')/Phi(R) exp(J(R') - J(R)), and the drift at R' comes from
 * the same evaluation. */
static int msd_walker_run(const orc_system *s, double *R, double *log_w, double *e_local,
                          int64_t step0, int32_t n_steps, int32_t mode, double tau, uint64_t seed,
                          double e_trial, int32_t walker_index, uint8_t *acc_row, size_t acc_stride,
                          double *e_row, size_t e_stride) {
  const int ne = s->n_up + s->n_dn, nmo = msd_n_mo(s);
  double *orb = (double *)malloc(sizeof(double) * (size_t)ne * 5 * nmo);
  double *orb_t = (double *)malloc(sizeof(double) * (size_t)ne * 5 * nmo);
  double *dphi = (double *)malloc(sizeof(double) * 3 * ne);
  double *dphi_t = (double *)malloc(sizeof(double) * 3 * ne);
  int rc = msd_orbital_table(s, R, nmo, orb);
  msd_spin m[2], t[2];
  for (int sp = 0; sp < 2; ++sp) {
    msd_spin_alloc(s, &m[sp], sp);
    msd_spin_alloc(s, &t[sp], sp);
    rc |= msd_spin_eval(s, orb, nmo, sp, &m[sp]);
  }
  double J, la;
  int sg;
  double e_old = msd_local_energy(s, R, m, &J, &la, &sg, NULL);
  const double sqt = sqrt(tau);
  for (int st = 0; st < n_steps; ++st) {
    const int64_t step = step0 + st;
    for (int i = 0; i < ne; ++i) {
      const int sp = spin_of(s, i);
      double *ri = R + 3 * i;
      double logabs, uo, gjo[3];
      int sgn;
      msd_combine(s, m, &logabs, &sgn, dphi, NULL);
      jastrow_one(s, R, i, ri, &uo, gjo);
      const double v[3] = {gjo[0] + dphi[3 * i], gjo[1] + dphi[3 * i + 1], gjo[2] + dphi[3 * i + 2]};
      double chi[3], uacc;
      orc_move_draws(seed, step, walker_index, i, chi, &uacc);
      double rn[3];
      for (int x = 0; x < 3; ++x) rn[x] = ri[x] + tau * v[x] + sqt * chi[x];
      /* trial state: electron i at r', the other spin's determinants unchanged */
      memcpy(orb_t, orb, sizeof(double) * (size_t)ne * 5 * nmo);
      rc |= orc_orbitals_vgl(s, rn, nmo, orb_t + (size_t)i * 5 * nmo);
      msd_spin_copy(s, &t[1 - sp], &m[1 - sp]);
      msd_spin_eval(s, orb_t, nmo, sp, &t[sp]);
      double logabs_t;
      int sgn_t;
      msd_combine(s, t, &logabs_t, &sgn_t, dphi_t, NULL);
      const double rho_sign = (double)(sgn_t * sgn);
      int accepted = 0;
      if (!(mode == 1 && !(rho_sign > 0.0)) && sgn_t != 0) {
        double un, gjn[3];
        jastrow_one(s, R, i, rn, &un, gjn);
        double vn[3];
        for (int x = 0; x < 3; ++x) vn[x] = gjn[x] + dphi_t[3 * i + x];
        double fwd = 0.0, bwd = 0.0;
        for (int x = 0; x < 3; ++x) {
          const double a = rn[x] - ri[x] - tau * v[x];
          const double b = ri[x] - rn[x] - tau * vn[x];
          fwd += a * a;
          bwd += b * b;
        }
        const double lnq = 2.0 * ((logabs_t - logabs) + (un - uo)) + (fwd - bwd) / (2.0 * tau);
        const double p = lnq >= 0.0 ? 1.0 : exp(lnq);
        accepted = uacc < p;
      }
      if (accepted) {
        for (int x = 0; x < 3; ++x) ri[x] = rn[x];
        memcpy(orb, orb_t, sizeof(double) * (size_t)ne * 5 * nmo);
        msd_spin_copy(s, &m[sp], &t[sp]);
      }
      if (acc_row) acc_row[(size_t)st * acc_stride + i] = (uint8_t)accepted;
    }
    const double e_new = msd_local_energy(s, R, m, &J, &la, &sg, NULL);
    if (mode == 1) *log_w += -tau * (0.5 * (e_old + e_new) - e_trial);
    if (e_row) e_row[(size_t)st * e_stride] = e_new;
    e_old = e_new;
  }
  *e_local = e_old;
  for (int sp = 0; sp < 2; ++sp) {
    msd_spin_free(&m[sp]);
    msd_spin_free(&t[sp]);
  }
  free(orb);
  free(orb_t);
  free(dphi);
  free(dphi_t);
  return rc;
}

/* Ion gradient of ln|Phi|, Phi = sum_d c_d D_d^up D_d^dn, forward mode per
 * determinant (Eq. 3 with lambda = R_{a,x} for each determinant's own
 * matrix):  d ln|D_d| = tr(A_d^{-1} dA_d),
 *   dA_d[i][j] = -sum_{l on a} C_{l, c_j} dPhi_l/dx (r_i),
 *   d ln|Phi| = sum_d c_d R_d^up R_d^dn (d ln|D_d^up| + d ln|D_d^dn|) / S. */
static int msd_ion_det_grads(const orc_system *s, const double *R, double *dlogpsi) {
  const int na = s->n_atom, nb = s->n_basis, nmo = msd_n_mo(s), nd = s->n_det;
  int rc = 0;
  int *fn_atom = (int *)malloc(sizeof(int) * nb);
  for (int sh = 0, f = 0; sh < s->n_shell; ++sh)
    for (int k = 0; k < NCART[s->shell_l[sh]]; ++k) fn_atom[f++] = s->shell_atom[sh];
  double *bvgl = (double *)malloc(sizeof(double) * 5 * nb);
  double *ratio = (double *)malloc(sizeof(double) * 2 * nd);     /* [2][nd] */
  double *dl = (double *)calloc((size_t)2 * nd * na * 3, sizeof(double)); /* [2][nd][na*3] */
  for (int sp = 0; sp < 2; ++sp) {
    const int n = sp == 0 ? s->n_up : s->n_dn, e0 = sp == 0 ? 0 : s->n_up;
    if (n == 0) {
      for (int d = 0; d < nd; ++d) ratio[sp * nd + d] = 1.0;
      continue;
    }
    /* values phi_p(r_i) and derivatives dphi[i][a*3+x][p] of every MO used */
    double *val = (double *)calloc((size_t)n * nmo, sizeof(double));
    double *dphi = (double *)calloc((size_t)n * na * 3 * nmo, sizeof(double));
    for (int ii = 0; ii < n; ++ii) {
      rc |= orc_basis_vgl(s, R + 3 * (e0 + ii), bvgl);
      for (int l = 0; l < nb; ++l) {
        const int a = fn_atom[l];
        for (int p = 0; p < nmo; ++p) {
          const double c = s->mo_coef[(size_t)l * s->n_mo + p];
          val[(size_t)ii * nmo + p] += c * bvgl[5 * l];
          for (int x = 0; x < 3; ++x)
            dphi[((size_t)ii * na * 3 + a * 3 + x) * nmo + p] -= c * bvgl[5 * l + 1 + x];
        }
      }
    }
    double *A = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *G = (double *)malloc(sizeof(double) * (size_t)n * n);
    int *cols = (int *)malloc(sizeof(int) * (size_t)n);
    double ld0 = 0.0;
    int32_t sg0 = 1;
    for (int d = 0; d < nd; ++d) {
      const int32_t *e = s->det_exc + 10 * d;
      const int nx = e[sp];
      for (int j = 0; j < n; ++j) cols[j] = j;
      const int *h = e + (sp == 0 ? 2 : 6), *p = e + (sp == 0 ? 4 : 8);
      for (int k = 0; k < nx; ++k) cols[h[k]] = p[k];
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = val[(size_t)i * nmo + cols[j]];
      double ld;
      int32_t sg;
      const int sing = orc_lu_slogdet_inv(n, A, &ld, &sg, G);
      if (d == 0) {
        rc |= sing;
        ld0 = ld;
        sg0 = sg;
      }
      if (sing) {
        ratio[sp * nd + d] = 0.0;
        continue;
      }
      ratio[sp * nd + d] = d == 0 ? 1.0 : (double)(sg * sg0) * exp(ld - ld0);
      for (int k = 0; k < na * 3; ++k) {
        double tr = 0.0;
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j)
            tr += G[(size_t)j * n + i] * dphi[((size_t)i * na * 3 + k) * nmo + cols[j]];
        dl[((size_t)sp * nd + d) * na * 3 + k] = tr;
      }
    }
    free(A);
    free(G);
    free(cols);
    free(val);
    free(dphi);
  }
  double S = 0.0;
  for (int d = 0; d < nd; ++d) S += s->ci_coef[d] * ratio[d] * ratio[nd + d];
  for (int d = 0; d < nd; ++d) {
    const double wgt = s->ci_coef[d] * ratio[d] * ratio[nd + d] / S;
    for (int k = 0; k < na * 3; ++k)
      dlogpsi[k] += wgt * (dl[(size_t)d * na * 3 + k] + dl[((size_t)nd + d) * na * 3 + k]);
  }
  free(ratio);
  free(dl);
  free(bvgl);
  free(fn_atom);
  return rc;
}

/* ------------------------------------------------------ population control */
/* Comb reconfiguration at fixed population (see oracle.h): the DMC weights of
 * Eq. 1 decide how many copies of each walker the next population holds. */
int orc_reconfigure(int32_t W, const double *log_w, double u, int32_t *copies, int32_t *pairs,
                    int32_t *n_pairs, double *log_wbar) {
  if (W < 1 || !(u >= 0.0 && u < 1.0)) return -1;
  double m = -INFINITY;
  for (int32_t j = 0; j < W; ++j)
    if (isfinite(log_w[j]) && log_w[j] > m) m = log_w[j];
  *n_pairs = 0;
  if (!isfinite(m)) {
    for (int32_t j = 0; j < W; ++j) copies[j] = 1;
    *log_wbar = NAN;
    return 0;
  }
  double *C = (double *)malloc(sizeof(double) * (size_t)W);
  double acc = 0.0;
  int32_t last = 0;
  for (int32_t j = 0; j < W; ++j) {
    const double w = isfinite(log_w[j]) ? exp(log_w[j] - m) : 0.0;
    if (w > 0.0) last = j;
    acc += w;
    C[j] = acc;
    copies[j] = 0;
  }
  const double S = acc;
  const double step = S / (double)W;
  /* each tooth: the first walker whose cumulative weight exceeds it */
  for (int32_t k = 0; k < W; ++k) {
    const double t = ((double)k + u) * step;
    int32_t sel = last;
    for (int32_t j = 0; j < W; ++j) {
      if (t < C[j]) { sel = j; break; }
    }
    copies[sel] += 1;
  }
  free(C);
  /* extra copies, walkers in order, into the free slots, lowest first */
  int32_t p = 0, f = 0;
  for (int32_t j = 0; j < W; ++j) {
    for (int32_t e = 1; e < copies[j]; ++e) {
      while (copies[f] != 0) ++f;
      pairs[2 * p] = f;
      pairs[2 * p + 1] = j;
      ++p;
      ++f;
    }
  }
  *n_pairs = p;
  *log_wbar = m + log(S / (double)W);
  return 0;
}

/* ======================================================================
 * Derivative of the local energy with respect to the ions (Single
 * Determinant QMC Forces, Eq. 4) and the space-warp transformation.
 *
 * E_L = -1/2 sum_sigma tr(A^{-1} B) - 1/2 sum_i [lap_i J + |grad_i J|^2] + V
 * with the one-body operator matrix of each spin
 *   B_ij = lap phi_j(r_i) + 2 sum_y (d_y J)(r_i) d_y phi_j(r_i)
 * (so that tr(A^{-1} B) = sum_i [l_i + 2 grad_i J . g_i]).  Along any
 * direction lambda of the ions and electrons, Eq. 4 gives
 *   d tr(A^{-1} B) = tr(A^{-1} dB - X dA),  X = A^{-1} B A^{-1},
 * and Eq. 3 gives d ln|D| = tr(A^{-1} dA).  The Jastrow, its derivatives and
 * V are differentiated pair by pair.  Single determinant only.
 *
 * Space warp (Filippi and Umrigar, PRB 61 R16291): when ion a moves by dR,
 * every electron moves by omega_a(r_i) dR with
 *   omega_a(r) = F(|r - R_a|) / sum_b F(|r - R_b|),  F(d) = d^-4,
 * which changes the sampled density by the Jacobian of r -> r + omega dR;
 * d ln(Jacobian) = sum_i d omega_a(r_i) / d r_i,x for component x.
 * ==================================================================== */

/* d^k/dx^k of x^n. */
static double mono_d(double x, int n, int k) {
  if (k > n) return 0.0;
  double c = 1.0;
  for (int q = 0; q < k; ++q) c *= (double)(n - q);
  return c * mono(x, n - k);
}

/* Basis derivatives of function Phi = P(d) R(s^2) by the Leibniz rule over
 * the derivative axes ax[0..n-1] (n <= 3): sum over subsets S of the axes of
 * (d_S P)(d_{rest} R), with
 *   R_a = 2 d_a R',  R_ab = 2 delta_ab R' + 4 d_a d_b R'',
 *   R_abc = 4 (delta_ab d_c + delta_ac d_b + delta_bc d_a) R'' + 8 d_a d_b d_c R'''. */
static double radial_d(const double d[3], const double Rk[4], const int *ax, int n) {
  if (n == 0) return Rk[0];
  if (n == 1) return 2.0 * d[ax[0]] * Rk[1];
  if (n == 2) return 2.0 * (ax[0] == ax[1]) * Rk[1] + 4.0 * d[ax[0]] * d[ax[1]] * Rk[2];
  const int a = ax[0], b = ax[1], c = ax[2];
  return 4.0 * ((a == b) * d[c] + (a == c) * d[b] + (b == c) * d[a]) * Rk[2] +
         8.0 * d[a] * d[b] * d[c] * Rk[3];
}
static double poly_d(const double d[3], const int *e, const int *ax, int n) {
  int k[3] = {0, 0, 0};
  for (int q = 0; q < n; ++q) k[ax[q]]++;
  return mono_d(d[0], e[0], k[0]) * mono_d(d[1], e[1], k[1]) * mono_d(d[2], e[2], k[2]);
}
static double leibniz(const double d[3], const int *e, const double Rk[4], const int *ax, int n) {
  double acc = 0.0;
  for (int m = 0; m < (1 << n); ++m) {
    int sa[3], ra[3], ns = 0, nr = 0;
    for (int q = 0; q < n; ++q) {
      if (m & (1 << q)) sa[ns++] = ax[q];
      else ra[nr++] = ax[q];
    }
    acc += poly_d(d, e, sa, ns) * radial_d(d, Rk, ra, nr);
  }
  return acc;
}

/* Hessian component order (xx, xy, xz, yy, yz, zz). */
static const int HESS[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
static int hidx(int a, int b) {
  for (int q = 0; q < 6; ++q)
    if ((HESS[q][0] == a && HESS[q][1] == b) || (HESS[q][0] == b && HESS[q][1] == a)) return q;
  return -1;
}

/* out[n_basis][14]: value, gradient (3), Hessian (6), Laplacian, gradient of
 * the Laplacian (3), at r. */
int orc_basis_d3(const orc_system *s, const double r[3], double *out) {
  int prim = 0, fn = 0;
  for (int sh = 0; sh < s->n_shell; ++sh) {
    const int l = s->shell_l[sh];
    if (l < 0 || l > 2) return 1;
    const double *c = s->ion_xyz + 3 * s->shell_atom[sh];
    const double d[3] = {r[0] - c[0], r[1] - c[1], r[2] - c[2]};
    const double s2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double Rk[4] = {0, 0, 0, 0};
    for (int p = 0; p < s->shell_nprim[sh]; ++p, ++prim) {
      const double a = s->prim_alpha[prim];
      const double e = s->prim_coef[prim] * exp(-a * s2);
      Rk[0] += e;
      Rk[1] += -a * e;
      Rk[2] += a * a * e;
      Rk[3] += -a * a * a * e;
    }
    for (int k = 0; k < NCART[l]; ++k, ++fn) {
      const int *e = CART[l][k];
      double *o = out + 14 * fn;
      o[0] = leibniz(d, e, Rk, NULL, 0);
      for (int a = 0; a < 3; ++a) o[1 + a] = leibniz(d, e, Rk, &a, 1);
      for (int q = 0; q < 6; ++q) o[4 + q] = leibniz(d, e, Rk, HESS[q], 2);
      o[10] = o[4] + o[7] + o[9];
      for (int cc = 0; cc < 3; ++cc) {
        double g = 0.0;
        for (int a = 0; a < 3; ++a) {
          const int ax[3] = {a, a, cc};
          g += leibniz(d, e, Rk, ax, 3);
        }
        o[11 + cc] = g;
      }
    }
  }
  return fn == s->n_basis ? 0 : 1;
}

/* Pade u(r) = a r/(1 + b r) as a function of the vector d (r = |d|):
 * gradient u' d/r, Hessian u'' dd^T/r^2 + (u'/r)(I - dd^T/r^2), Laplacian
 * u'' + 2u'/r, gradient of the Laplacian (u''' + 2u''/r - 2u'/r^2) d/r,
 * with u''' = 6 a b^2 / (1 + b r)^4. */
typedef struct { double u, g[3], H[3][3], lap, glap[3]; } pair_d;
static pair_d pade_vec(double a, double b, const double d[3]) {
  pair_d p;
  const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const double t = 1.0 + b * r;
  const double u1 = a / (t * t), u2 = -2.0 * a * b / (t * t * t), u3 = 6.0 * a * b * b / (t * t * t * t);
  p.u = a * r / t;
  for (int x = 0; x < 3; ++x) {
    p.g[x] = u1 * d[x] / r;
    for (int y = 0; y < 3; ++y)
      p.H[x][y] = u2 * d[x] * d[y] / (r * r) + (u1 / r) * ((x == y) - d[x] * d[y] / (r * r));
    p.glap[x] = (u3 + 2.0 * u2 / r - 2.0 * u1 / (r * r)) * d[x] / r;
  }
  p.lap = u2 + 2.0 * u1 / r;
  return p;
}

/* Space-warp weight omega_a(r) of every atom and its gradient in r. */
static void warp_weights(const orc_system *s, const double r[3], double *om, double *dom) {
  const int na = s->n_atom;
  double S = 0.0, dS[3] = {0, 0, 0};
  for (int a = 0; a < na; ++a) {
    const double *c = s->ion_xyz + 3 * a;
    const double d[3] = {r[0] - c[0], r[1] - c[1], r[2] - c[2]};
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const double F = 1.0 / (r2 * r2);
    om[a] = F;
    for (int x = 0; x < 3; ++x) {
      dom[3 * a + x] = -4.0 * F / r2 * d[x]; /* dF/dr_x = -4 d_x / |d|^6 */
      dS[x] += dom[3 * a + x];
    }
    S += F;
  }
  for (int a = 0; a < na; ++a) {
    for (int x = 0; x < 3; ++x) dom[3 * a + x] = (dom[3 * a + x] * S - om[a] * dS[x]) / (S * S);
    om[a] /= S;
  }
}

int orc_warp_weights(const orc_system *s, const double r[3], double *omega, double *domega) {
  warp_weights(s, r, omega, domega);
  return 0;
}

/* Everything the directional derivatives need at one configuration. */
typedef struct {
  int ne, nb, na, nmax, nsig[2];
  double *bd;   /* [ne][n_basis][14] basis derivatives */
  double *od;   /* [ne][14][nmax] orbital derivatives (MOs 0..n_sigma-1) */
  double *G[2]; /* [n][n] inverses, G[j][i] = (A^{-1})_{ji} */
  double *X[2]; /* X = G B G */
  double *Bm[2];/* B (one-body operator matrix, electron row i, orbital j) */
  double *cj;   /* [ne][3] grad_i J */
  double logdet[2];
  int sign[2];
  int *fn_atom;
} zvstate;

static void zv_free(zvstate *z) {
  free(z->bd); free(z->od); free(z->cj); free(z->fn_atom);
  for (int sp = 0; sp < 2; ++sp) { free(z->G[sp]); free(z->X[sp]); free(z->Bm[sp]); }
}

static int zv_init(const orc_system *s, const double *R, zvstate *z) {
  int rc = 0;
  z->ne = s->n_up + s->n_dn;
  z->nb = s->n_basis;
  z->na = s->n_atom;
  z->nsig[0] = s->n_up;
  z->nsig[1] = s->n_dn;
  z->nmax = s->n_up > s->n_dn ? s->n_up : s->n_dn;
  const int ne = z->ne, nb = z->nb, nm = z->nmax;
  z->bd = (double *)malloc(sizeof(double) * (size_t)ne * nb * 14 + 1);
  z->od = (double *)calloc((size_t)ne * 14 * nm + 1, sizeof(double));
  z->cj = (double *)malloc(sizeof(double) * 3 * ne + 1);
  z->fn_atom = (int *)malloc(sizeof(int) * nb + 1);
  for (int sh = 0, f = 0; sh < s->n_shell; ++sh)
    for (int k = 0; k < NCART[s->shell_l[sh]]; ++k) z->fn_atom[f++] = s->shell_atom[sh];
  for (int i = 0; i < ne; ++i) {
    double *b = z->bd + (size_t)i * nb * 14;
    rc |= orc_basis_d3(s, R + 3 * i, b);
    const int n = z->nsig[spin_of(s, i)];
    double *o = z->od + (size_t)i * 14 * nm;
    for (int q = 0; q < 14; ++q)
      for (int j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int l = 0; l < nb; ++l) acc += s->mo_coef[(size_t)l * s->n_mo + j] * b[14 * l + q];
        o[q * nm + j] = acc;
      }
  }
  orc_jastrow(s, R, NULL, z->cj, NULL);
  for (int sp = 0; sp < 2; ++sp) {
    const int n = z->nsig[sp];
    z->G[sp] = (double *)calloc((size_t)n * n + 1, sizeof(double));
    z->X[sp] = (double *)calloc((size_t)n * n + 1, sizeof(double));
    z->Bm[sp] = (double *)calloc((size_t)n * n + 1, sizeof(double));
    if (n == 0) { z->logdet[sp] = 0.0; z->sign[sp] = 1; continue; }
    double *A = (double *)malloc(sizeof(double) * (size_t)n * n);
    for (int ii = 0; ii < n; ++ii) {
      const int i = ii + sp * s->n_up;
      const double *o = z->od + (size_t)i * 14 * nm;
      for (int j = 0; j < n; ++j) {
        A[(size_t)ii * n + j] = o[j];
        /* B_ij = lap phi_j + 2 grad J . grad phi_j */
        z->Bm[sp][(size_t)ii * n + j] =
            o[10 * nm + j] + 2.0 * (z->cj[3 * i] * o[1 * nm + j] + z->cj[3 * i + 1] * o[2 * nm + j] +
                                    z->cj[3 * i + 2] * o[3 * nm + j]);
      }
    }
    rc |= orc_lu_slogdet_inv(n, A, &z->logdet[sp], &z->sign[sp], z->G[sp]);
    /* X = G B G (orbital x electron, like G) */
    double *T = (double *)calloc((size_t)n * n, sizeof(double));
    for (int i = 0; i < n; ++i)      /* T = B G : electron x electron */
      for (int k = 0; k < n; ++k) {
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += z->Bm[sp][(size_t)i * n + j] * z->G[sp][(size_t)j * n + k];
        T[(size_t)i * n + k] = acc;
      }
    for (int j = 0; j < n; ++j)      /* X = G T : orbital x electron */
      for (int k = 0; k < n; ++k) {
        double acc = 0.0;
        for (int i = 0; i < n; ++i) acc += z->G[sp][(size_t)j * n + i] * T[(size_t)i * n + k];
        z->X[sp][(size_t)j * n + k] = acc;
      }
    free(T);
    free(A);
  }
  return rc;
}

/* Directional derivative of E_L and ln|Psi| when the ions move by dion
 * [n_atom][3] and the electrons by del [ne][3] (both per unit lambda). */
static void zv_direction(const orc_system *s, const double *R, const zvstate *z,
                         const double *dion, const double *del, double *dEL, double *dlogpsi) {
  const int ne = z->ne, nb = z->nb, na = z->na, nm = z->nmax;
  /* ---- determinant part: Eq. 3 and Eq. 4 per spin */
  double det_e = 0.0, det_l = 0.0;
  double *dA = (double *)malloc(sizeof(double) * (size_t)nm + 1);
  double *dBl = (double *)malloc(sizeof(double) * (size_t)nm + 1);
  double *dBg = (double *)malloc(sizeof(double) * 3 * (size_t)nm + 1);
  double *dcj = (double *)calloc((size_t)3 * ne + 1, sizeof(double));
  /* d(grad_i J) along the direction (needed inside dB) */
  for (int i = 0; i < ne; ++i) {
    for (int j = 0; j < ne; ++j) {
      if (j == i) continue;
      const double d[3] = {R[3 * i] - R[3 * j], R[3 * i + 1] - R[3 * j + 1], R[3 * i + 2] - R[3 * j + 2]};
      const pair_d p = pade_vec(ee_a(s, i, j), s->jee_b, d);
      for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y) dcj[3 * i + x] += p.H[x][y] * (del[3 * i + y] - del[3 * j + y]);
    }
    for (int A = 0; A < na; ++A) {
      const double *c = s->ion_xyz + 3 * A;
      const double d[3] = {R[3 * i] - c[0], R[3 * i + 1] - c[1], R[3 * i + 2] - c[2]};
      const pair_d p = pade_vec(s->jen_a[A], s->jen_b, d);
      for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y) dcj[3 * i + x] += p.H[x][y] * (del[3 * i + y] - dion[3 * A + y]);
    }
  }
  for (int i = 0; i < ne; ++i) {
    const int sp = spin_of(s, i), ii = i - sp * s->n_up, n = z->nsig[sp];
    const double *o = z->od + (size_t)i * 14 * nm;
    const double *b = z->bd + (size_t)i * nb * 14;
    const double *dr = del + 3 * i;
    /* row i of dA, d(grad A) and d(lap A): electron part through the orbital
     * derivatives, ion part through the basis functions of each moving atom */
    for (int j = 0; j < n; ++j) {
      double a = 0.0, lp = 0.0, g[3] = {0, 0, 0};
      for (int x = 0; x < 3; ++x) {
        a += o[(1 + x) * nm + j] * dr[x];
        lp += o[(11 + x) * nm + j] * dr[x];
        for (int y = 0; y < 3; ++y) g[y] += o[(4 + hidx(x, y)) * nm + j] * dr[x];
      }
      dA[j] = a;
      dBl[j] = lp;
      for (int y = 0; y < 3; ++y) dBg[y * nm + j] = g[y];
    }
    for (int l = 0; l < nb; ++l) {
      const double *dR = dion + 3 * z->fn_atom[l];
      if (dR[0] == 0.0 && dR[1] == 0.0 && dR[2] == 0.0) continue;
      const double *bl = b + 14 * l;
      double a = 0.0, lp = 0.0, g[3] = {0, 0, 0};
      for (int x = 0; x < 3; ++x) {
        a -= bl[1 + x] * dR[x];
        lp -= bl[11 + x] * dR[x];
        for (int y = 0; y < 3; ++y) g[y] -= bl[4 + hidx(x, y)] * dR[x];
      }
      for (int j = 0; j < n; ++j) {
        const double C = s->mo_coef[(size_t)l * s->n_mo + j];
        dA[j] += C * a;
        dBl[j] += C * lp;
        for (int y = 0; y < 3; ++y) dBg[y * nm + j] += C * g[y];
      }
    }
    /* tr(G dA), tr(G dB) and tr(X dA) restricted to row i */
    const double *ci = z->cj + 3 * i, *dci = dcj + 3 * i;
    for (int j = 0; j < n; ++j) {
      const double gji = z->G[sp][(size_t)j * n + ii], xji = z->X[sp][(size_t)j * n + ii];
      double dB = dBl[j];
      for (int y = 0; y < 3; ++y) dB += 2.0 * (dci[y] * o[(1 + y) * nm + j] + ci[y] * dBg[y * nm + j]);
      det_l += gji * dA[j];
      det_e += gji * dB - xji * dA[j];
    }
  }
  /* ---- Jastrow and potential, pair by pair */
  double jl = 0.0, jq = 0.0, dJ = 0.0, dV = 0.0;
  for (int i = 0; i < ne; ++i) {
    const double *ci = z->cj + 3 * i, *dci = dcj + 3 * i;
    jq += 2.0 * (ci[0] * dci[0] + ci[1] * dci[1] + ci[2] * dci[2]); /* d |grad_i J|^2 */
    for (int j = 0; j < ne; ++j) {
      if (j == i) continue;
      const double d[3] = {R[3 * i] - R[3 * j], R[3 * i + 1] - R[3 * j + 1], R[3 * i + 2] - R[3 * j + 2]};
      const double dd[3] = {del[3 * i] - del[3 * j], del[3 * i + 1] - del[3 * j + 1],
                            del[3 * i + 2] - del[3 * j + 2]};
      const pair_d p = pade_vec(ee_a(s, i, j), s->jee_b, d);
      const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      for (int x = 0; x < 3; ++x) {
        jl += p.glap[x] * dd[x];
        if (j > i) {
          dJ += p.g[x] * dd[x];
          dV -= d[x] / (r * r * r) * dd[x];
        }
      }
    }
    for (int A = 0; A < na; ++A) {
      const double *c = s->ion_xyz + 3 * A;
      const double d[3] = {R[3 * i] - c[0], R[3 * i + 1] - c[1], R[3 * i + 2] - c[2]};
      const double dd[3] = {del[3 * i] - dion[3 * A], del[3 * i + 1] - dion[3 * A + 1],
                            del[3 * i + 2] - dion[3 * A + 2]};
      const pair_d p = pade_vec(s->jen_a[A], s->jen_b, d);
      const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      for (int x = 0; x < 3; ++x) {
        jl += p.glap[x] * dd[x];
        dJ += p.g[x] * dd[x];
        dV += s->ion_charge[A] * d[x] / (r * r * r) * dd[x];
      }
    }
  }
  for (int A = 0; A < na; ++A)
    for (int B = A + 1; B < na; ++B) {
      const double *a = s->ion_xyz + 3 * A, *b = s->ion_xyz + 3 * B;
      const double d[3] = {a[0] - b[0], a[1] - b[1], a[2] - b[2]};
      const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      for (int x = 0; x < 3; ++x)
        dV -= s->ion_charge[A] * s->ion_charge[B] * d[x] / (r * r * r) * (dion[3 * A + x] - dion[3 * B + x]);
    }
  *dEL = -0.5 * (det_e + jl + jq) + dV;
  *dlogpsi = det_l + dJ;
  free(dA); free(dBl); free(dBg); free(dcj);
}

int orc_local_energy_dir(const orc_system *s, const double *R, const double *dion,
                         const double *del, double *dEL, double *dlogpsi) {
  if (s->n_det > 1) return 4;
  zvstate z;
  int rc = zv_init(s, R, &z);
  zv_direction(s, R, &z, dion, del, dEL, dlogpsi);
  zv_free(&z);
  return rc;
}

/* Per ion coordinate (a, x): dE_L, d ln|Psi| and d ln(Jacobian) along the
 * ion displacement alone (warp = 0) or with the space warp (warp = 1).
 * Outputs [n_atom][3] each. */
int orc_zv_grads(const orc_system *s, const double *R, int32_t warp, double *dEL,
                 double *dlogpsi, double *dlogjac) {
  if (s->n_det > 1) return 4;
  const int ne = s->n_up + s->n_dn, na = s->n_atom;
  zvstate z;
  int rc = zv_init(s, R, &z);
  double *om = (double *)calloc((size_t)ne * na + 1, sizeof(double));
  double *dom = (double *)calloc((size_t)ne * na * 3 + 1, sizeof(double));
  if (warp)
    for (int i = 0; i < ne; ++i) warp_weights(s, R + 3 * i, om + (size_t)i * na, dom + (size_t)i * na * 3);
  double *dion = (double *)calloc((size_t)na * 3 + 1, sizeof(double));
  double *del = (double *)calloc((size_t)ne * 3 + 1, sizeof(double));
  for (int a = 0; a < na; ++a)
    for (int x = 0; x < 3; ++x) {
      memset(dion, 0, sizeof(double) * na * 3);
      memset(del, 0, sizeof(double) * ne * 3);
      dion[3 * a + x] = 1.0;
      double jac = 0.0;
      for (int i = 0; i < ne; ++i) {
        del[3 * i + x] = om[(size_t)i * na + a];
        jac += dom[((size_t)i * na + a) * 3 + x];
      }
      zv_direction(s, R, &z, dion, del, dEL + 3 * a + x, dlogpsi + 3 * a + x);
      dlogjac[3 * a + x] = jac;
    }
  free(om); free(dom); free(dion); free(del);
  zv_free(&z);
  return rc;
}

int orc_zv_grads_batch(const orc_system *s, int32_t W, const double *R, int32_t warp, double *dEL,
                       double *dlogpsi, double *dlogjac, int32_t n_threads) {
  const int ne = s->n_up + s->n_dn, na = s->n_atom;
  int rc = 0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic) reduction(| : rc)
  for (int w = 0; w < W; ++w)
    rc |= orc_zv_grads(s, R + (size_t)w * ne * 3, warp, dEL + (size_t)w * na * 3,
                       dlogpsi + (size_t)w * na * 3, dlogjac + (size_t)w * na * 3);
  return rc;
}
