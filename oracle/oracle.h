/*
 * Plain FP64 CPU oracle for the batched-walker DMC step of a Slater-Jastrow
 * wavefunction with contracted-Gaussian LCAO orbitals.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the HIP library; both read the same seeded inputs.
 *
 * Everything is computed from its plain definition, in double precision,
 * with no blocking, fusion or delayed update:
 *   - trial function Psi = exp(J) D_up D_dn (Eq. 2, one determinant; the
 *     multideterminant sum of Eq. 2 by one direct LU per determinant);
 *   - orbitals phi_j(r) = sum_l C_lj Phi_l(r) (the LCAO form below Eq. 2);
 *   - determinant ratios and log-derivatives through A^{-1} of a fresh LU
 *     (Eq. 3: d ln D / d lambda = tr(A^{-1} dA/d lambda));
 *   - the DMC step of Eq. 1 under the fixed-node constraint, drift-diffusion
 *     proposal with Metropolis acceptance, time step tau;
 *   - ion gradients in forward mode, one tr(A^{-1} dA/dR_{a,x}) per ion
 *     coordinate (Eq. 3 with lambda = R_{a,x}).
 */
#ifndef DMC_ORACLE_H
#define DMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_atom;
  const double *ion_xyz;      /* [n_atom][3] */
  const double *ion_charge;   /* [n_atom]    */
  int32_t n_shell;
  const int32_t *shell_atom;  /* [n_shell] */
  const int32_t *shell_l;     /* [n_shell], 0..2 */
  const int32_t *shell_nprim; /* [n_shell] */
  const double *prim_alpha;   /* [sum nprim] */
  const double *prim_coef;    /* [sum nprim], normalisation folded in */
  int32_t n_basis, n_mo;
  const double *mo_coef;      /* [n_basis][n_mo] */
  int32_t n_up, n_dn;
  double jee_a_anti, jee_a_para, jee_b;
  const double *jen_a;        /* [n_atom] */
  double jen_b;
  /* multideterminant expansion; n_det == 0 means a single determinant */
  int32_t n_det;
  const int32_t *det_exc;     /* [n_det][10] */
  const double *ci_coef;      /* [n_det] */
  /* semilocal pseudopotential terms beta r^(n-2) exp(-alpha r^2) of atom
   * pp_atom[t] in channel pp_l[t] (-1: local, added to V; l >= 0: projected
   * on angular momentum l); pp_rcut[A]: radius beyond which atom A's
   * non-local channels are taken as zero.  pp_n_term == 0: none. */
  int32_t pp_n_term;
  const int32_t *pp_atom, *pp_l, *pp_n;
  const double *pp_beta, *pp_alpha;
  const double *pp_rcut;      /* [n_atom] */
} orc_system;

/* Basis values, gradients and Laplacians at r: out[n_basis][5] =
 * (Phi, dPhi/dx, dPhi/dy, dPhi/dz, lap Phi), canonical order. */
int orc_basis_vgl(const orc_system *s, const double r[3], double *out);

/* First n_orb orbitals at r: out[5][n_orb]. */
int orc_orbitals_vgl(const orc_system *s, const double r[3], int32_t n_orb, double *out);

/* LU with partial pivoting: log|det A|, sign, and A^{-1} (if inv != NULL).
 * A is [n][n] row-major.  Returns 0, or 1 when a pivot is exactly zero. */
int orc_lu_slogdet_inv(int32_t n, const double *A, double *logdet, int32_t *sign, double *inv);

/* Jastrow J(R), per-electron gradient grad[n_elec][3] and Laplacian lap[n_elec]. */
int orc_jastrow(const orc_system *s, const double *R, double *J, double *grad, double *lap);

/* Coulomb potential V(R) (e-e, e-ion, ion-ion). */
double orc_potential(const orc_system *s, const double *R);

/* Everything at one configuration R[n_elec][3]:
 * log|Psi|, sign(Psi), E_L and the drift v[n_elec][3] (may be NULL). */
int orc_evaluate(const orc_system *s, const double *R, double *log_psi, int32_t *sign,
                 double *e_local, double *drift);

/* Philox4x32-10 block: out = philox(ctr, key). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The three per-move draws: chi[3] ~ N(0,1), u_acc ~ U[0,1). */
void orc_move_draws(uint64_t seed, int64_t step, int32_t walker, int32_t elec,
                    double chi[3], double *u_acc);

/* mode: 0 = VMC, 1 = DMC (fixed node, log-weights). Walkers are updated in
 * place; log_w[W] accumulates the DMC weight; e_local[W] is written with the
 * local energy after the last step.  accept_log[n_steps][W][n_elec] and
 * e_log[n_steps][W] may be NULL.  Walker w uses Philox walker index
 * walker_offset + w.  n_threads <= 0 lets OpenMP decide. */
int orc_run(const orc_system *s, int32_t W, double *R, double *log_w, double *e_local,
            int64_t step0, int32_t n_steps, int32_t mode, double tau, uint64_t seed,
            double e_trial, int32_t walker_offset, uint8_t *accept_log, double *e_log,
            int32_t n_threads);

/* Ion gradients of log|Psi| and of V at R, forward mode (Eq. 3):
 * dlogpsi[n_atom][3], dV[n_atom][3]. */
int orc_ion_grads(const orc_system *s, const double *R, double *dlogpsi, double *dV);

/* Same for a crowd: R[W][n_elec][3] -> [W][n_atom][3] each. */
int orc_ion_grads_batch(const orc_system *s, int32_t W, const double *R, double *dlogpsi,
                        double *dV, int32_t n_threads);

/* Evaluate a crowd without moving it: log|Psi|, sign, E_L per walker. */
int orc_evaluate_batch(const orc_system *s, int32_t W, const double *R, double *log_psi,
                       int32_t *sign, double *e_local, int32_t n_threads);

/* Multideterminant value: Psi_MSD / Psi_0 (ratio to the reference product
 * of determinants), from one direct LU per excited determinant. */
int orc_msd_ratio_direct(const orc_system *s, const double *R, double *psi_over_psi0);

/* log|Psi|, sign, E_L and drift of the multideterminant trial function, every
 * determinant with its own LU inverse.  orc_evaluate and orc_run take this
 * path by themselves when n_det > 1 (each proposal then re-evaluates all
 * determinants of the mover's spin from scratch). */
int orc_msd_evaluate(const orc_system *s, const double *R, double *log_psi, int32_t *sign,
                     double *e_local, double *drift);

/* Population control at fixed population by comb reconfiguration (the
 * published systematic-resampling scheme; the paper fixes the DMC weights of
 * Eq. 1, not how the population is controlled).  Walker j has weight
 * w_j = exp(log_w[j] - m), m the largest finite log_w (a non-finite log_w
 * counts as weight 0); C_j = w_0 + ... + w_j summed in walker order,
 * S = C_{W-1}.  Tooth k = 0..W-1 sits at t_k = (k + u) * (S / W) and selects
 * the first j with t_k < C_j (the last positive-weight walker if rounding
 * leaves none).  copies[j] = teeth selecting j.  The slots of walkers with no
 * copy are filled, lowest slot first, by the extra copies of the walkers in
 * walker order: pairs[2p] = destination, pairs[2p + 1] = source, p < *n_pairs.
 * *log_wbar = m + log(S / W), the log of the mean weight, which every walker
 * carries afterwards.  With no positive weight nothing is selected: copies
 * are all 1, *n_pairs = 0 and *log_wbar = NaN.  Returns -1 for u outside
 * [0, 1) or W < 1. */
int orc_reconfigure(int32_t W, const double *log_w, double u, int32_t *copies, int32_t *pairs,
                    int32_t *n_pairs, double *log_wbar);


/* Birth/death branching: copies[W] = floor(w_j + u_j), the new population's
 * (destination, source) pairs and size W' (see oracle.c); 5 when W' < 1 or
 * W' > cap (nothing selected). */
int orc_branch(int32_t W, const double *log_w, const uint8_t *flags, uint64_t seed, int64_t step,
               int32_t cap, int32_t *copies, int32_t *pairs, int32_t *n_pairs, int32_t *w_new);

/* DMC steps with E_T fed back from the population after every step:
 * E_T <- <E_L>_w - (gain / tau) ln(sum_w exp(log w) / W_T), W_T = w_target
 * or, when it is 0, W (see oracle.c). */
int orc_run_feedback(const orc_system *s, int32_t W, double *R, double *log_w, double *e_local,
                     int64_t step0, int32_t n_steps, double tau, uint64_t seed, double e_trial,
                     double gain, int32_t w_target, int32_t walker_offset, uint8_t *accept_log, double *e_log,
                     double *et_log, double *e_trial_out, int32_t n_threads);

/* Derivatives of ln Psi and E_L with respect to the 8 Jastrow parameters
 * (e-e Pade b, e-n Pade b, six three-body coefficients at zero; see
 * oracle.c): dlogpsi[8], dEL[8]; the batch form [W][8] each. */
int orc_jastrow_param_grads(const orc_system *s, const double *R, double *dlogpsi, double *dEL);
int orc_jastrow_param_grads_batch(const orc_system *s, int32_t W, const double *R,
                                  double *dlogpsi, double *dEL, int32_t n_threads);
/* d V_NL / dp for the same eight directions at fixed quadrature rotations
 * (the non-local part of dE_L/dp; see oracle.c); 4 with a multideterminant
 * expansion. */
int orc_nlpp_param_grads(const orc_system *s, const double *R, uint64_t seed, int64_t step,
                         int32_t walker, double *dv);
/* The six three-body basis sums F_k(R) themselves (c = 0 derivatives of J). */
int orc_j3_values(const orc_system *s, const double *R, double *F);

/* Non-local pseudopotential energy of the walker at R (see oracle.c):
 * sum over electrons i and atoms A within A's cutoff of
 * sum_l v_l(r_iA) (2l + 1) sum_q (1/12) P_l(cos theta_q) Psi(.., r_q, ..)/Psi(R),
 * r_q on the sphere of radius r_iA about A in the 12 icosahedral directions
 * rotated by the electron's random rotation (Philox draws 3 and 4 of
 * (electron, walker, step)).  Single determinant only (4 otherwise). */
int orc_nlpp(const orc_system *s, const double *R, uint64_t seed, int64_t step, int32_t walker,
             double *v_nl);
int orc_nlpp_batch(const orc_system *s, int32_t W, const double *R, uint64_t seed, int64_t step,
                   int32_t walker_offset, double *v_nl, int32_t n_threads);
/* d(V_loc + V_NL)/dR_A at fixed electrons, rotations and Psi (the
 * pseudopotential's Hellmann-Feynman force term): dvpp[n_atom][3]. */
int orc_pp_ion_grads(const orc_system *s, const double *R, uint64_t seed, int64_t step,
                     int32_t walker, double *dvpp);
/* The rotation of electron elec of walker walker at step: rot[3][3]. */
void orc_nlpp_rotation(uint64_t seed, int64_t step, int32_t walker, int32_t elec, double rot[9]);

/* Derivative of the local energy (Single Determinant QMC Forces, Eq. 4) and
 * of ln|Psi| (Eq. 3) along a direction of the ions (dion [n_atom][3]) and
 * electrons (del [ne][3]); single determinant only (4 otherwise). */
int orc_local_energy_dir(const orc_system *s, const double *R, const double *dion,
                         const double *del, double *dEL, double *dlogpsi);
/* Per ion coordinate: dE_L, d ln|Psi|, d ln(Jacobian) [n_atom][3], with
 * (warp = 1) or without the space warp. */
int orc_zv_grads(const orc_system *s, const double *R, int32_t warp, double *dEL,
                 double *dlogpsi, double *dlogjac);
int orc_zv_grads_batch(const orc_system *s, int32_t W, const double *R, int32_t warp, double *dEL,
                       double *dlogpsi, double *dlogjac, int32_t n_threads);
/* Basis value, gradient, Hessian (xx,xy,xz,yy,yz,zz), Laplacian and
 * gradient of the Laplacian: out[n_basis][14]. */
int orc_basis_d3(const orc_system *s, const double r[3], double *out);
/* Space-warp weights omega_a(r) [n_atom] and their gradients [n_atom][3]. */
int orc_warp_weights(const orc_system *s, const double r[3], double *omega, double *domega);

#ifdef __cplusplus
}
#endif
#endif
