/*
 * dmcx -- batched-walker diffusion Monte Carlo hot path for MI355X (gfx950).
 *
 * The library moves a crowd of walkers through the DMC step of a
 * Slater-Jastrow trial function built from contracted-Gaussian LCAO orbitals
 * and returns local energies and ion-coordinate derivatives (arXiv
 * 2504.07948, QMC section):
 *   Eq. 1  imaginary-time projection, run under the fixed-node constraint;
 *   Eq. 2  Psi_T(R) = exp(sum J) sum_k C_k D_k^up D_k^dn with
 *          phi_i = sum_l C_l^i Phi_l (single determinant or, with n_det > 1,
 *          an excitation-based multideterminant expansion);
 *   Eq. 3  d ln D / d lambda = tr(A^{-1} dA/d lambda), A_ij = phi_j(r_i), used
 *          for drift, local energy and ion forces.
 * Every step runs in hand-written HIP kernels on the device; the host side of
 * this library only validates, uploads and launches.
 *
 * Conventions (all calls):
 *   - Units are Hartree atomic units (bohr, Hartree).
 *   - Electrons 0..n_up-1 are spin up, n_up..n_up+n_dn-1 spin down.
 *   - Orbital VGL order is (value, d/dx, d/dy, d/dz, Laplacian).
 *   - Basis order is atom -> shell -> Cartesian component,
 *     p = (x, y, z), d = (xx, xy, xz, yy, yz, zz).
 *   - Every call returns a dmcx_status; DMCX_OK == 0.  Nothing throws across
 *     this interface and nothing aborts.  dmcx_last_error() gives text.
 *   - Buffers tagged DMCX_HOST are read or written before the call returns.
 *     Buffers tagged DMCX_DEVICE (e.g. a torch tensor's data_ptr()) are used
 *     in stream order on the context's stream and must stay valid until that
 *     work completes (dmcx_sync).  The library never frees caller memory.
 *   - A context is bound to one HIP stream and is not thread-safe.
 *   - Walkers of several systems are concatenated in creation order; every
 *     per-walker array below has W = sum(walkers_per_sys) leading entries and
 *     uses the largest electron count N_e (atom count n_atom_max) of all
 *     systems as its stride.  Entries beyond a system's own count are not
 *     read on input and not written on output (host accept logs: zero).
 */
#ifndef DMCX_H
#define DMCX_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dmcx_ctx dmcx_ctx; /* opaque; owns all device state */

typedef enum {
  DMCX_OK = 0,
  DMCX_E_INVALID = 1,     /* bad argument, shape or state for this call */
  DMCX_E_NOMEM = 2,       /* device allocation failed */
  DMCX_E_HIP = 3,         /* a HIP runtime call failed */
  DMCX_E_SINGULAR = 4,    /* a Slater matrix had a zero pivot in the LU recompute */
  DMCX_E_NONFINITE = 5,   /* some walker produced NaN/Inf; see dmcx_walker_flags */
  DMCX_E_STATE = 6,       /* call out of order (e.g. accept without ratio_grad) */
  DMCX_E_UNSUPPORTED = 7  /* valid request this build does not implement */
} dmcx_status;

/* DMCX_FP64: every step in FP64.
 * DMCX_MIXED: the sweep (basis, orbital GEMM, ratios, delayed updates) runs
 * in FP32 on MFMA with FP32 accumulation; at the end of every step the value
 * rows of A are evaluated again in FP64 (FP64 basis and MFMA GEMM), inverted
 * in FP64 (which also resets the FP32 inverse and log|D|), and E_L is taken
 * from that FP64 inverse with the FP32 derivative rows, so the energy error
 * does not grow with cond(A); the recompute period then has no effect.  With
 * DMCX_FLAG_FP32_ENERGY, or with a multideterminant expansion, E_L comes from
 * the FP32 rows and inverse, and the FP64 recompute runs every
 * recompute_period steps. */
typedef enum { DMCX_FP64 = 0, DMCX_MIXED = 1 } dmcx_precision;
typedef enum { DMCX_VMC = 0, DMCX_DMC = 1 } dmcx_mode;
typedef enum { DMCX_HOST = 0, DMCX_DEVICE = 1 } dmcx_mem;

/* One molecule.  dmcx_create deep-copies it; the caller may free it after. */
typedef struct {
  int32_t n_atom;
  const double *ion_xyz;     /* [n_atom][3] */
  const double *ion_charge;  /* [n_atom], effective charge Z_A (V_en, V_nn) */
  int32_t n_shell;
  const int32_t *shell_atom; /* [n_shell] atom index of each shell */
  const int32_t *shell_l;    /* [n_shell] angular momentum, 0..2 */
  const int32_t *shell_nprim;/* [n_shell] primitives per shell, 1..8 */
  const double *prim_alpha;  /* [sum nprim] exponents, shell order */
  const double *prim_coef;   /* [sum nprim] coefficients, normalisation folded in */
  int32_t n_basis, n_mo;     /* n_basis must equal the Cartesian function count */
  const double *mo_coef;     /* [n_basis][n_mo] row-major LCAO coefficients C_l^i */
  int32_t n_up, n_dn;        /* electrons per spin; determinants use MOs 0..n_sigma-1 */
  /* Pade Jastrow u(r) = a r / (1 + b r): e-e with a = jee_a_anti (opposite
   * spins) or jee_a_para (same spin), e-n with a = jen_a[A]; exponent +J. */
  double jee_a_anti, jee_a_para, jee_b;
  const double *jen_a;       /* [n_atom] */
  double jen_b;
  /* Multideterminant expansion (Eq. 2 with M > 1).  n_det == 0 or 1 with
   * only the reference selects the single-determinant path. */
  int32_t n_det;
  const int32_t *det_exc;    /* [n_det][10]: nu, nd, hu0, hu1, pu0, pu1, hd0, hd1, pd0, pd1
                                holes = occupied column index, particles = MO index */
  const double *ci_coef;     /* [n_det] */
  /* Semilocal pseudopotential (the ccECP form of the paper's QMC runs):
   * pp_n_term terms beta r^(n-2) exp(-alpha r^2), term t of atom pp_atom[t]
   * in channel pp_l[t] (-1: local, added to V; 0..3: non-local, projected on
   * angular momentum l and evaluated by quadrature, see dmcx_run);
   * pp_rcut[A] (bohr): beyond it atom A's non-local channels are taken as
   * zero.  pp_n_term == 0 (all pointers may be NULL): no pseudopotential. */
  int32_t pp_n_term;
  const int32_t *pp_atom;    /* [pp_n_term] */
  const int32_t *pp_l;       /* [pp_n_term] */
  const int32_t *pp_n;       /* [pp_n_term] */
  const double *pp_beta;     /* [pp_n_term] */
  const double *pp_alpha;    /* [pp_n_term] */
  const double *pp_rcut;     /* [n_atom] */
} dmcx_system;

/* dmcx_options.flags */
#define DMCX_FLAG_GRAPH 1u  /* dmcx_run replays one captured step graph per step */
/* Mixed form only: take E_L, log|Psi| and the weights from the FP32 orbital
 * rows and the FP32 inverse, with the FP64 recompute every recompute_period
 * steps (faster; its energy error grows with cond(A), see DMCX_MIXED). */
#define DMCX_FLAG_FP32_ENERGY 2u

typedef struct {
  int32_t precision;         /* dmcx_precision */
  int32_t delay_rank;        /* k of the delayed rank-k inverse update, 1..64 (capped at
                                n_sigma); 0 = chosen by the autotuner at the first run */
  int32_t recompute_period;  /* P: full FP64 inverse recompute every P steps (>= 1) */
  double tau;                /* DMC time step (a.u.), > 0 */
  uint64_t seed;             /* Philox4x32-10 key */
  uint32_t flags;            /* DMCX_FLAG_*; other bits must be 0 */
} dmcx_options;

/* Create a context for n_sys systems (n_sys >= 1) with walkers_per_sys[s]
 * walkers each, bound to hip_stream (a hipStream_t; NULL = default stream).
 * Allocates all device memory the context will ever use (the delay-rank
 * autotuner and the first graph capture allocate small temporaries once).
 * Walkers start undefined: call dmcx_set_walkers before anything that reads
 * them.  Every system runs with the same options; walker w of system s uses
 * the Philox counter (electron, w, step) under the shared key, so a system
 * in a group moves exactly as it would in a context of its own.
 * With n_sys > 1 the systems may differ in electron, atom and basis counts;
 * dmcx_run forks them onto streams of their own (default priority) and
 * joins them back into hip_stream.  The move-by-move calls
 * (dmcx_eval_orbitals, dmcx_ratio_grad, dmcx_accept) need n_sys == 1 and
 * return DMCX_E_UNSUPPORTED otherwise. */
dmcx_status dmcx_create(const dmcx_system *sys, int32_t n_sys, const int32_t *walkers_per_sys,
                        const dmcx_options *opt, void *hip_stream, dmcx_ctx **out);
void dmcx_destroy(dmcx_ctx *ctx);

/* Passage: QMC section, Eq. 2 (the trial function evaluated at each walker's
 * configuration) and Eq. 1 (each walker carries the weight of the projection).
 * R: [W][N_e][3] positions; log_w: [W] log-weights or NULL (= all zero).
 * Evaluates all orbitals, recomputes every inverse in FP64 (LU) and the
 * local energy of each walker.  Resets the step counter to 0. */
dmcx_status dmcx_set_walkers(dmcx_ctx *ctx, const double *R, const double *log_w, dmcx_mem mem);
dmcx_status dmcx_get_walkers(dmcx_ctx *ctx, double *R, double *log_w, dmcx_mem mem);

/* Step counter used as the Philox counter's step field (checkpoint/resume: a
 * run resumed with dmcx_set_walkers + dmcx_set_step at the saved step draws
 * the same random numbers as an uninterrupted one).  dmcx_set_step also sets
 * the counter later evaluations outside a run take their pseudopotential
 * quadrature rotations from (measure, ion and parameter derivatives).  The
 * paper does not fix the random stream; these calls carry no physics. */
dmcx_status dmcx_set_step(dmcx_ctx *ctx, int64_t step);
dmcx_status dmcx_get_step(const dmcx_ctx *ctx, int64_t *step);

/* Passage: Single Determinant QMC Forces (the ion coordinates R_a that Eq. 3
 * and Eq. 4 differentiate).
 * Replace the ion coordinates of system sys_index ([n_atom][3]) and
 * re-evaluate orbitals, inverses and local energies at the current walkers. */
dmcx_status dmcx_set_ions(dmcx_ctx *ctx, int32_t sys_index, const double *ion_xyz, dmcx_mem mem);

/* Passage: Single Determinant QMC Forces (A_ij = phi_j(r_i) and its inverse,
 * Eq. 3); ln|D| and its sign enter Eq. 2.
 * Apply pending delayed updates, then rebuild every inverse from the cached
 * orbital rows with an FP64 LU (partial pivoting); resets log|D| and sign.
 * DMCX_E_SINGULAR if any walker's matrix had a zero pivot. */
dmcx_status dmcx_recompute(dmcx_ctx *ctx);

/* Passage: QMC section, Eq. 2 (phi_i = sum_l C_l^i Phi_l, with the value,
 * gradient and Laplacian of every orbital).
 * Orbitals of the given spin at one point per walker: r [W][3] ->
 * vgl [W][5][n_sigma_max] (n_sigma_max = largest n_up/n_dn over systems). */
dmcx_status dmcx_eval_orbitals(dmcx_ctx *ctx, int32_t spin, const double *r, double *vgl,
                               dmcx_mem mem);

/* Passage: Single Determinant QMC Forces, Eq. 3 with lambda = the moved
 * electron's coordinate (the ratio det(A')/det(A) is the row of A' dotted
 * with a column of A^{-1}; the drift is tr(A^{-1} dA/dr)), times the Jastrow
 * factor of Eq. 2.
 * Ratio Psi(R')/Psi(R) for moving electron iel of every walker to r_new
 * [W][3] (Jastrow included) and grad_{iel} ln|Psi(R')| [W][3].  The proposal
 * is kept for the next dmcx_accept.  Uses the delayed-updated inverse:
 * consecutive electrons of one spin form blocks of delay_rank moves. */
dmcx_status dmcx_ratio_grad(dmcx_ctx *ctx, int32_t iel, const double *r_new, double *ratio,
                            double *grad, dmcx_mem mem);

/* Passage: QMC section, Eq. 1 under the fixed-node constraint (the accepted
 * move changes one row of A of Eq. 3, so A^{-1} changes by rank one).
 * accept [W] (0/1) for the proposal of the last dmcx_ratio_grad(iel).
 * Accepted walkers move electron iel; inverses are updated (delayed). */
dmcx_status dmcx_accept(dmcx_ctx *ctx, int32_t iel, const uint8_t *accept, dmcx_mem mem);

/* Passage: Single Determinant QMC Forces (the inverse A^{-1} of Eq. 3 after
 * the accepted moves; the rank-k form is the published Woodbury identity).
 * Apply all pending delayed updates now (rank-k GEMM flush). */
dmcx_status dmcx_flush(dmcx_ctx *ctx);

/* Passage: QMC section, Eq. 1 (imaginary-time projection as drift-diffusion
 * moves with fixed-node rejection and weights), trial function of Eq. 2,
 * walker-level batching of QMC Energy and Wavefunction Evaluation.
 * Run n_steps full sweeps (every electron proposes one drift-diffusion move
 * per step, up electrons then down).  DMCX_DMC rejects node crossings and
 * updates log-weights with E_T = e_trial; DMCX_VMC leaves weights alone.
 * accept_log [n_steps][W][N_e] (uint8) and e_log [n_steps][W] may be NULL;
 * both are device pointers if mem == DMCX_DEVICE.  Each step is: FP64
 * inverse recompute when step = 0 (mod P), the sweep, local energies and
 * weights.  With DMCX_FLAG_GRAPH the step (of every system) is captured once
 * into a hipGraph and replayed n_steps times; the capture is redone when
 * the log pointers, the delay rank or the ions change.  Results are the same
 * bits as without the flag.  With delay_rank == 0 the first run first
 * times 2 sweeps per candidate (tile shape, rank) (dmcx_autotune) and
 * restores the walkers (inverses are then freshly recomputed). */
dmcx_status dmcx_run(dmcx_ctx *ctx, dmcx_mode mode, int32_t n_steps, double e_trial,
                     uint8_t *accept_log, double *e_log, dmcx_mem mem);

/* Tile shapes of the single-determinant sweep (8 walkers per workgroup of 8
 * waves in both): DMCX_TILE_DEEP stages 4 x stage depth basis functions per
 * LDS stage of the orbital GEMM (one workgroup per CU at the FP64 register
 * count); DMCX_TILE_SHALLOW stages half as many with four waves per SIMD (two
 * workgroups per CU).  The FP32 (mixed) single-determinant sweep offers both
 * (default shallow); the FP64 and multideterminant sweeps are deep only. */
#define DMCX_TILE_DEEP 0
#define DMCX_TILE_SHALLOW 1

/* Passage: QMC Energy and Wavefunction Evaluation (batching chosen to keep
 * the GPU busy); tile shapes and the delay rank are not in the paper.
 * Autotuner of the sweep: for every system, time `steps` sweeps (after one
 * untimed sweep) for each candidate pair (tile shape, rank): the shapes the
 * system's sweep offers, and the ranks k in {8, 16, 24, 32, 48, 64} below
 * n_sigma plus n_sigma itself, limited to the rank the buffers were sized
 * for at create (min(64, n_sigma) with delay_rank == 0, else delay_rank);
 * keep the fastest pair, restore the walkers and recompute the inverses.
 * chosen_k [n_sys] may be NULL.  The walker configurations and weights are
 * unchanged; the step counter is unchanged. */
dmcx_status dmcx_autotune(dmcx_ctx *ctx, int32_t steps, int32_t *chosen_k);

/* The autotuner's last measurements for system sys_index: up to max_n
 * candidates, each a rank, a tile shape (DMCX_TILE_*) and its average sweep
 * time (ms); *n_cand = number of candidates (0 if the tuner has not run).
 * ranks / shapes / ms may be NULL. */
dmcx_status dmcx_autotune_report(const dmcx_ctx *ctx, int32_t sys_index, int32_t max_n,
                                 int32_t *ranks, int32_t *shapes, float *ms_per_sweep,
                                 int32_t *n_cand);

/* Set the tile shape of system sys_index's sweep (DMCX_TILE_*), in place of
 * the autotuner's choice.  DMCX_E_UNSUPPORTED for a shape the system's sweep
 * does not offer (see DMCX_TILE_DEEP), DMCX_E_INVALID for a bad index or
 * shape.  Results differ between shapes only by the order of the FP32 (or
 * FP64) sums of the orbital GEMM. */
dmcx_status dmcx_set_tile_shape(dmcx_ctx *ctx, int32_t sys_index, int32_t shape);
/* Tile shape currently used by system sys_index's sweep. */
dmcx_status dmcx_get_tile_shape(const dmcx_ctx *ctx, int32_t sys_index, int32_t *shape);

/* Delay rank currently used by system sys_index. */
dmcx_status dmcx_get_delay_rank(const dmcx_ctx *ctx, int32_t sys_index, int32_t *k);

/* Passage: QMC section, Eq. 2 (log|Psi_T| and sign) and Single Determinant
 * QMC Forces (E_L through tr(A^{-1} B) with B the Laplacian rows, Eq. 3).
 * Current local energy, log|Psi| and sign of every walker ([W] each;
 * any pointer may be NULL).  With a pseudopotential, E_L carries its local
 * terms and its non-local energy: per electron and atom within the cutoff
 * the 12-point icosahedral rule, turned by a random rotation (Philox draws 3
 * and 4 of (electron, walker, step) under the seed, step = the step counter
 * when the energy was formed: the step's own index inside a run). */
dmcx_status dmcx_measure(dmcx_ctx *ctx, double *e_local, double *log_psi, int8_t *sign,
                         dmcx_mem mem);

/* Passage: QMC section (the many-body Hamiltonian's potential; its ion
 * derivative is the Hellmann-Feynman term of Single Determinant QMC Forces).
 * Coulomb potential V(R) of each walker's current configuration, [W]
 * (electron-electron + electron-ion + ion-ion), plus the pseudopotential's
 * local and non-local energies when the system has one. */
dmcx_status dmcx_potential(dmcx_ctx *ctx, double *v, dmcx_mem mem);

/* Passage: Single Determinant QMC Forces, Eq. 3 with lambda = an ion
 * coordinate R_a (Pulay term) and dV/dR_a (Hellmann-Feynman term);
 * Multideterminant QMC Forces for n_det > 1.
 * Per-walker ion derivatives: dlogpsi_dR and dV_dR, [W][n_atom_max][3]
 * (either may be NULL).  Reverse-mode adjoint of basis, MO contraction,
 * log-determinant and Jastrow (Eq. 3 with lambda = an ion coordinate).
 * With a pseudopotential dV_dR includes its Hellmann-Feynman term, the
 * derivative of the local terms and of the non-local quadrature with respect
 * to the pseudopotential's centre at fixed electrons and Psi (rotations of
 * the current step counter). */
dmcx_status dmcx_ion_grads(dmcx_ctx *ctx, double *dlogpsi_dR, double *dV_dR, dmcx_mem mem);

/* Passage: Single Determinant QMC Forces, Eq. 3 (the same derivatives as
 * dmcx_ion_grads, contracted with a caller's cotangent per walker).
 * Vector-Jacobian products over walkers: grad_R[n_atom_max][3] (per system
 * when n_sys > 1: [n_sys][n_atom_max][3]) = sum_w gbar[w] d(.)_w/dR. */
dmcx_status dmcx_logpsi_vjp(dmcx_ctx *ctx, const double *gbar, double *grad_R, dmcx_mem mem);
dmcx_status dmcx_potential_vjp(dmcx_ctx *ctx, const double *gbar, double *grad_R, dmcx_mem mem);

/* Passage: Single Determinant QMC Forces (force estimator built from Eq. 3)
 * with the walker weights of Eq. 1.
 * Hellmann-Feynman + Pulay force estimate from the current walkers,
 * weighted by exp(log_w): F = -<dV/dR> - 2(<E_L dlnPsi/dR> - <E_L><dlnPsi/dR>).
 * F: [n_sys][n_atom_max][3]. */
dmcx_status dmcx_forces(dmcx_ctx *ctx, double *F, dmcx_mem mem);

/* Passage: Single Determinant QMC Forces, Eq. 4 (d E_L / d R_a =
 * tr(A^{-1} dB/dR_a - X dA/dR_a), X = A^{-1} B A^{-1}, with B read as the
 * one-body operator matrix B_ij = lap phi_j(r_i) + 2 grad_i J . grad phi_j(r_i)
 * so that tr(A^{-1} B) carries the determinant part of the kinetic energy)
 * and the space-warp transformation of the same section (Filippi-Umrigar
 * warp: electrons follow ion a with weight omega_a(r) = F_a / sum_b F_b,
 * F_b = |r - R_b|^-4).
 * Per-walker derivatives along every ion coordinate, [W][n_atom_max][3] each
 * (any pointer may be NULL): dEL = dE_L/dR (zero-variance term, kinetic and
 * potential parts), dlogpsi = d ln|Psi|/dR, dlogjac = d ln(Jacobian)/dR of
 * the warp.  warp = 0: the ion coordinate alone (dlogjac = 0); warp = 1:
 * ion plus warped electrons.  Reverse-mode adjoint through the inverse, the
 * MO contraction (two MFMA products per electron) and third derivatives of
 * the basis.  Single-determinant systems without a pseudopotential only
 * (DMCX_E_UNSUPPORTED otherwise); DMCX_E_INVALID for warp outside {0, 1}. */
dmcx_status dmcx_zv_grads(dmcx_ctx *ctx, int32_t warp, double *dEL, double *dlogpsi,
                          double *dlogjac, dmcx_mem mem);

/* Passage: Single Determinant QMC Forces (zero-variance force estimator of
 * Eq. 4 with the Pulay covariance and the space warp), walker weights of Eq. 1.
 * F[n_sys][n_atom_max][3] = -<dE_L/dR> - (<E_L q> - <E_L><q>),
 * q = 2 d ln|Psi|/dR + d ln(Jacobian)/dR, weights exp(log w); walkers with a
 * status flag or a non-finite log w or E_L have weight zero.  Errors as
 * dmcx_zv_grads. */
dmcx_status dmcx_forces_zv(dmcx_ctx *ctx, int32_t warp, double *F, dmcx_mem mem);

/* Passage: QMC section, Eq. 1 (the walker weights of the projection) and the
 * fixed-node DMC estimators built on them.
 * Weighted estimators of each system's walkers, in FP64: out[n_sys][11] with
 *   [0]  walkers counted (finite log w and E_L, no status flag),
 *   [1]  m = largest log w of those walkers (the log-sum-exp shift),
 *   [2]  S0 = sum omega,  omega = exp(log w - m),
 *   [3]  S1 = sum omega E_L,  [4] S2 = sum omega E_L^2,  [5] Q = sum omega^2,
 *   [6]  <E_L> = S1 / S0 (the weighted mixed energy estimate),
 *   [7]  weighted variance of E_L, from centred moments merged block by block
 *        (never S2/S0 - <E_L>^2),
 *   [8]  smallest log w of the counted walkers,
 *   [9]  acceptance ratio: accepted / proposed moves since the previous
 *        dmcx_estimators call (or dmcx_set_walkers); NaN if none,
 *   [10] moves proposed in that span (dmcx_run sweeps and dmcx_accept calls).
 * log of the total weight is m + log S0; the effective walker count is
 * S0^2 / Q.  With no walker counted, [1]..[8] are NaN.  The call clears the
 * move counters.  It enqueues two kernels on the context's stream and
 * allocates nothing; with DMCX_DEVICE it does not synchronise (out is
 * written in stream order).  Errors: DMCX_E_STATE (walkers not set). */
#define DMCX_N_ESTIMATORS 11
dmcx_status dmcx_estimators(dmcx_ctx *ctx, double *out, dmcx_mem mem);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * estimators of dmcx_estimators over plain per-walker device arrays, with no
 * context and no allocation.  The block records of the first pass live in a
 * scratch array of the library's own, one per GPU for the life of the
 * process, sized for at most DMCX_NOALLOC_MAX_WALKERS walkers (4096 records
 * of 80 bytes, 320 KiB); its device address is looked up once per device,
 * on the first call with that device current.
 *   n_walkers   0..DMCX_NOALLOC_MAX_WALKERS; more is DMCX_E_INVALID.
 *   log_w       [n_walkers] FP64 log-weights, device memory.
 *   e_local     [n_walkers] FP64 local energies, device memory.
 *   flags       [n_walkers] status bytes as written by dmcx_walker_flags, or
 *               NULL; a walker with a nonzero byte is not counted.
 *   n_accepted, n_proposed
 *               [n_walkers] move counters (uint32), both or neither (NULL:
 *               out[9] is NaN and out[10] is 0); read and cleared.
 *   out         [11] doubles in device memory, laid out as one system's
 *               record of dmcx_estimators.
 *   hip_stream  the stream (of the current device) the two kernels are
 *               enqueued on; nothing synchronises.
 * Inputs and outputs are borrowed until that work completes.  Every call on
 * one GPU shares the one scratch array, so calls that overlap on a GPU (on
 * different streams or host threads) race and must be ordered by the caller.
 * Every record the second pass reads is written by the first pass of the
 * same call, so nothing needs clearing between calls.  Errors:
 * DMCX_E_INVALID (sizes, null pointers), DMCX_E_HIP (launch or symbol
 * lookup); dmcx_last_error(NULL) gives the text. */
#define DMCX_NOALLOC_MAX_WALKERS 1048576
dmcx_status dmcx_estimators_noalloc(int32_t n_walkers, const double *log_w, const double *e_local,
                                    const uint8_t *flags, uint32_t *n_accepted,
                                    uint32_t *n_proposed, double *out, void *hip_stream);

/* Mixed form (DMCX_MIXED without DMCX_FLAG_FP32_ENERGY): the number of
 * walkers whose E_L the last energy evaluation (step end, measure or
 * recompute) recomputed from FP64 derivative rows because their first-order
 * error bound from the FP32 rows, (u / 2) sum_ij (|lap phi_j(r_i)| +
 * 2 |grad_i J|_1 |grad phi_j(r_i)|_1) |(A^{-1})_ji| with u = 2^-24, exceeded
 * 1e-4 Ha per electron (Eq. 2 trial function, E_L of Eq. 3 form).  0 for the
 * other forms.  Synchronises the context's stream. */
dmcx_status dmcx_energy_escalations(dmcx_ctx *ctx, int32_t *n);
/* The bound of those re-evaluations, in Ha per electron (default 1e-4; 0
 * re-evaluates every walker with a finite E_L, which makes every E_L the
 * FP64 rows' and inverse's).  Applies to later energy evaluations of the
 * mixed form with its FP64 energy; no effect on the other forms.  Errors:
 * DMCX_E_INVALID (negative or non-finite cap). */
dmcx_status dmcx_set_energy_escalation_cap(dmcx_ctx *ctx, double cap);

/* Passage: QMC section, Eq. 1 (the trial energy E_T of the projection) and
 * the population control its weights need (not fixed by the paper).
 * E_T feedback for the DMC steps of later dmcx_run calls: after every step
 * each system's E_T becomes <E_L>_w - (gain / tau) ln(W_tot / W), with
 * <E_L>_w the weighted mean local energy, W_tot = sum_w exp(log w_w) over the
 * walkers counted by dmcx_estimators and W the system's walker count when
 * this call was made (the target population once dmcx_branch varies it; FP64,
 * log-sum-exp; unchanged when no walker counts).  dmcx_run's e_trial is the
 * E_T of the first step.  gain < 0 switches it off (E_T held fixed, the
 * default).  Errors: DMCX_E_INVALID (non-finite gain). */
dmcx_status dmcx_set_et_feedback(dmcx_ctx *ctx, double gain);
/* E_T the next step would use, per system: e_trial[n_sys] (host).
 * Synchronises the context's stream. */
dmcx_status dmcx_get_trial_energy(dmcx_ctx *ctx, double *e_trial);

/* Passage: QMC section, Eq. 2 (the Jastrow factor of the trial function,
 * whose parameters the VMC optimisation varies before the DMC projection of
 * Eq. 1; the paper does not fix the optimiser, the linear method is the
 * published one).
 * Derivatives with respect to DMCX_N_JASTROW_PARAMS = 8 Jastrow parameters,
 * in order: 0 the b of the e-e Pade terms, 1 the b of the e-n Pade terms,
 * 2..7 the coefficients c_k of six three-body e-e-n terms
 * sum_A sum_{i<j} (s_iA^l s_jA^m + s_iA^m s_jA^l) s_ij^n, s(r) = r / (1 + r),
 * (l, m, n) = (1,1,0), (1,0,1), (1,1,1), (2,1,0), (2,0,1), (1,0,2), taken at
 * c = 0 (the trial function itself has no three-body term).
 * Per walker at the current configuration: dlogpsi[W][8] = O_p = d ln Psi/dp
 * and dEL[W][8] = dE_L/dp = -1/2 sum_i [lap_i O_p + 2 grad_i ln|Psi| . grad_i O_p]
 * (either may be NULL); with a pseudopotential dEL also holds the non-local
 * energy's part, sum over the quadrature points of (1/12) f rho
 * (O_p(R_q) - O_p(R)) with the rotations of the current step counter (each
 * quadrature ratio carries the Jastrow factor's change).  FP64 arithmetic;
 * grad_i ln|Psi| and the quadrature ratios come from the context's inverse
 * and orbital rows (FP32 in the mixed form).  Single-determinant systems only
 * (DMCX_E_UNSUPPORTED otherwise). */
#define DMCX_N_JASTROW_PARAMS 8
dmcx_status dmcx_jastrow_param_grads(dmcx_ctx *ctx, double *dlogpsi, double *dEL, dmcx_mem mem);

/* Passage: as dmcx_jastrow_param_grads.
 * Linear-method matrices of each system's walkers in the basis
 * {Psi, (O_k - <O_k>) Psi}: S[n_sys][9][9], H[n_sys][9][9] with
 *   S[0][0] = 1, S[0][k] = S[k][0] = 0, S[k][l] = <dO_k dO_l>,
 *   H[0][0] = <E_L>, H[k][0] = <dO_k E_L>, H[0][l] = <E_L dO_l> + <dE_L/dp_l>,
 *   H[k][l] = <dO_k (dO_l E_L + dE_L/dp_l)>,
 * dO_k = O_k - <O_k>, <x> = sum_w omega_w x_w / sum_w omega_w in walker
 * order, omega = exp(log w - max log w) over the walkers with finite log w
 * and E_L and no status flag (every entry NaN if none counts).  Solving
 * H c = E S c for the lowest E gives the parameter update c_k / c_0.
 * Errors as dmcx_jastrow_param_grads. */
dmcx_status dmcx_linear_method(dmcx_ctx *ctx, double *S, double *H, dmcx_mem mem);

/* Per-walker status bits [W]: 1 = non-finite value, 2 = singular matrix
 * (a zero pivot of A of Eq. 3 in the FP64 recompute).  Bits stay set until
 * the next dmcx_set_walkers. */
dmcx_status dmcx_walker_flags(dmcx_ctx *ctx, uint8_t *flags, dmcx_mem mem);

/* Passage: QMC section, Eq. 1 (walker weights of the projection).
 * Population control at fixed population: comb reconfiguration of each
 * system's walkers by their DMC weights (the weights of Eq. 1; the paper does
 * not fix the control scheme, this is the published systematic resampling).
 * For system s with W_s walkers: w_j = exp(log_w_j - m), m the largest finite
 * log_w (a non-finite log_w is weight 0); C_j = w_0 + ... + w_j in walker
 * order; S = C_{W_s - 1}.  Tooth k = 0..W_s-1 at t_k = (k + u[s]) * (S / W_s)
 * selects the first walker with t_k < C_j.  Walkers without a copy are
 * replaced, lowest slot first, by the extra copies of the others in walker
 * order; a copy takes every state the walker carries between steps
 * (positions, inverses, cached orbital rows, log|D| and sign, E_L, log|Psi|,
 * V, flags, multideterminant table).  Every walker of system s then has
 * log_w = log(S / W_s) + m, so the total weight is kept.  With no positive
 * weight the population is left as it is and log_wbar[s] is NaN.
 * u: [n_sys] comb offsets in [0, 1) (host memory; the caller draws them).
 * copies: [W] int32 copies of each walker, or NULL.  log_wbar: [n_sys] log
 * of the mean weight before the call, or NULL.  mem applies to copies and
 * log_wbar; host outputs are complete on return.  The walker step counter is
 * unchanged, so copies draw different Philox streams from their next step on
 * (the walker index is part of the counter).  Errors: DMCX_E_INVALID (u
 * outside [0, 1)), DMCX_E_STATE (walkers not set, or an electron block of the
 * move-by-move calls pending). */
dmcx_status dmcx_reconfigure(dmcx_ctx *ctx, const double *u, int32_t *copies, double *log_wbar,
                             dmcx_mem mem);

/* Passage: Eq. 3 (the determinant ratios through the inverse A^{-1} that the
 * delayed updates keep and the periodic LU recompute rebuilds).
 * Residual of the stored inverses, a diagnostic: res[W][2], for walker w and
 * spin s, max_ij |sum_k A_ik (A^{-1})_kj - delta_ij| over the spin's Slater
 * matrix A_ik = phi_k(r_i) of the current positions (the cached orbital
 * value rows) and the stored inverse, in the working precision of the
 * context (FP32 for the mixed forms), products and sums in FP64.  NaN when
 * any entry is NaN, 0 for an empty spin.  Right after an FP64 recompute it
 * is at round-off; between recomputes it shows the drift of the delayed
 * updates.  A pending electron block of the move-by-move calls is flushed
 * first.  mem applies to res; host output is complete on return.  Errors:
 * DMCX_E_STATE (walkers not set). */
dmcx_status dmcx_inverse_residual(dmcx_ctx *ctx, double *res, dmcx_mem mem);

/* Passage: QMC section, Eq. 1 (walker weights of the projection).
 * Birth/death branching of a one-system context: the weights become walker
 * counts, so the population size varies (the paper does not fix the control
 * scheme; this is the published integer branching with a uniform offset).
 * Walker j of W gets M_j = floor(w_j + u_j) copies, w_j = exp(log_w_j) (0
 * for a non-finite log_w or a flagged walker), u_j the first uniform of the
 * Philox block of counter (electron 0, walker j, step, draw 5) under the
 * context's seed; so E[M_j] = w_j.  The new population has W' = sum M_j
 * walkers, each with log_w = 0, laid out as follows:
 *   - a walker with a copy keeps its slot;
 *   - its extra copies, walkers in order, fill the slots of the walkers
 *     without a copy, lowest first, and then the slots W, W + 1, ...;
 *   - walkers left in slots >= W' move into the empty slots below W', both
 *     in slot order.
 * A copy takes every state the walker carries between steps (as in
 * dmcx_reconfigure).  step: the Philox step counter of the draws (the
 * caller's choice, e.g. the step after the last one run).
 * copies: [W] int32 (the count before the call), or NULL; mem applies to it.
 * n_walkers: W' (host), or NULL; read also on DMCX_E_INVALID, where it holds
 * 0 (nothing survives) or the capacity + 1 (too many).  Walker counts of
 * later calls (dmcx_run, dmcx_get_walkers, the estimators, ...) are W'.
 * Synchronises the context's stream (the new count sizes later launches).
 * Errors: DMCX_E_INVALID (W' < 1 or W' > capacity: nothing changed),
 * DMCX_E_STATE (walkers not set, electron block pending),
 * DMCX_E_UNSUPPORTED (a context of several systems). */
dmcx_status dmcx_branch(dmcx_ctx *ctx, int64_t step, int32_t *copies, int32_t *n_walkers,
                        dmcx_mem mem);

/* Passage: QMC section, Eq. 1 (the walker population).
 * Sets the walker count of a one-system context to n_walkers, 1 ..
 * capacity (the n_walkers it was created with, which sizes its buffers);
 * dmcx_set_walkers must follow (the walkers are unset).  Errors:
 * DMCX_E_INVALID (count out of range), DMCX_E_STATE (electron block
 * pending), DMCX_E_UNSUPPORTED (a context of several systems). */
dmcx_status dmcx_set_walker_count(dmcx_ctx *ctx, int32_t n_walkers);

/* Current walker count and capacity (host, either may be NULL); for a
 * context of several systems both are the total over its systems. */
dmcx_status dmcx_walker_count(const dmcx_ctx *ctx, int32_t *n_walkers, int32_t *capacity);

/* Wait for all work queued on the context's stream. */
dmcx_status dmcx_sync(dmcx_ctx *ctx);

/* Average duration (ms) of the most expensive kernel (the sweep) per launch
 * over the last dmcx_run, measured with HIP events on the stream it ran on,
 * and the number of such launches (all systems of a group); for roofline
 * reporting.  Graph runs (DMCX_FLAG_GRAPH) are not timed: 0 launches. */
dmcx_status dmcx_last_run_timing(const dmcx_ctx *ctx, double *sweep_ms_avg, int32_t *n_launches,
                                 double *total_ms);

/* Device self-checks (Philox known answers, MFMA operand layouts).  Runs a
 * few tiny kernels; DMCX_OK when all match. */
dmcx_status dmcx_selftest(void *hip_stream);

/* Raw Philox4x32-10 outputs for n counters ctr [n][4] under key [2] -> out [n][4]
 * (host buffers); lets tests compare the device stream with other
 * implementations bit for bit. */
dmcx_status dmcx_philox(const uint32_t *ctr, const uint32_t *key, int32_t n, uint32_t *out);

const char *dmcx_strerror(dmcx_status s);
/* Text of the context's last error; with ctx == NULL, of this thread's last
 * context-free call. */
const char *dmcx_last_error(const dmcx_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* DMCX_H */
