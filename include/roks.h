/*
 * roks.h -- C ABI of the MI355X (gfx950) restricted open-shell Kohn-Sham
 * (ROKS) plane-wave hot path.
 *
 * The method is the one of Sahre, Romanelli, Marsman, Gonzalez and Kresse,
 * "Excited States from Restricted Open Shell Plane-Wave DFT" (equations are
 * cited by their LaTeX labels, sections by number):
 *
 *   E = sum_L c_L E_L - sum_mn gamma_mn (<m|S|n> - delta_mn)    Sec. II A
 *   with the mixed-spin (c = 2) and triplet (c = -1) configurations of the
 *   Ziegler sum rule E_S = 2 E_M - E_T (Eq. ziegler_sum), minimised over one
 *   set of real Gamma-point orbitals by preconditioned Fletcher-Reeves CG
 *   (Eqs. orbital_update, cg_search, gradient, prec_grad_I, prec_k) with the
 *   in-subspace rotation of Eqs. r_matrix_singlet and prec_grad_IIa-c, and
 *   Hellmann-Feynman forces (Eq. force_hf).
 *
 * Units: Hartree atomic units (bohr, Ha).  Overlap operator S = 1 (the
 * projectors carry no augmentation charge, q_kl = 0).
 *
 * Plane-wave storage ("half sphere"): the library owns the list of stored
 * reciprocal vectors G = h b1 + k b2 + l b3 with |G|^2/2 <= ecut; of each
 * pair {G, -G} one is stored, c(-G) = conj(c(G)) is implied, and G = 0 is
 * entry 0.  roks_gvectors() returns the Miller triples in storage order.
 * A band is npw complex numbers stored as [npw][2] doubles (re, im); band
 * arrays are [nbands][npw][2].  psi(r) = Omega^-1/2 sum_G c(G) e^{iG.r} over
 * the full sphere, so <a|b> = a(0) b(0) + 2 Re sum_{G != 0, stored} a* b.
 *
 * Ownership: the caller owns every array it passes; the library copies what
 * it keeps during the call.  The context owns all device state (orbitals,
 * potentials, projector tables, CG state).  All device work is ordered on
 * the context's HIP stream; calls taking host pointers synchronise that
 * stream before returning, calls whose name ends in _d take device pointers
 * and only enqueue work: the caller's work producing their inputs must be
 * complete (or ordered on the context's stream, by passing that stream to
 * roks_create).  A host process that also uses a framework carrying its own
 * HIP runtime (PyTorch's wheels do) must initialise that framework's GPU
 * context before the first roks_create.
 *
 * Errors: every call returns a roks_status; argument and shape checks come
 * before any device work.  roks_last_error() gives a message for the last
 * failing call on that context (or the last failing roks_create when ctx is
 * NULL).  On ROKS_ERR_NOT_PD, ROKS_ERR_LINESEARCH or ROKS_ERR_NAN inside
 * roks_pcg_step the orbitals and CG state are those of the last accepted
 * iterate.
 */
#ifndef ROKS_H
#define ROKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct roks_ctx_s* roks_ctx;

typedef enum {
  ROKS_OK = 0,
  ROKS_ERR_ARG = 1,        /* invalid argument value                     */
  ROKS_ERR_SHAPE = 2,      /* inconsistent sizes (grid too small, ...)   */
  ROKS_ERR_HIP = 3,        /* HIP runtime error or no usable GPU         */
  ROKS_ERR_OOM = 4,        /* device allocation failed                   */
  ROKS_ERR_NOT_PD = 5,     /* Gram matrix not positive definite          */
  ROKS_ERR_LINESEARCH = 6, /* no energy decrease found along the search  */
  ROKS_ERR_NAN = 7,        /* non-finite energy or gradient              */
  ROKS_ERR_STATE = 8       /* call out of order (e.g. no orbitals set)   */
} roks_status;

/* Arithmetic tier of the FFT, pointwise and projector work.  Gram, Cholesky,
 * rotation, energy sums and the line search are FP64 in every tier, and so
 * are the band overlaps (Theta, <S|S>, the preconditioner's projections).
 *   ROKS_FP64         everything FP64.
 *   ROKS_FP32         FFTs, potentials and the pointwise work in FP32; the
 *                     products with the projector table FP64.
 *   ROKS_FP32_BF16X3  as ROKS_FP32, and the products with the projector
 *                     table (<beta|psi>, <d beta|psi>, sum_p (D P) beta_p;
 *                     Sec. II A and Eq. force_hf) on the BF16 matrix cores:
 *                     both operands split as x = hi + lo with hi = bf16(x),
 *                     lo = bf16(x - hi), the three terms lo.hi + hi.lo +
 *                     hi.hi accumulated in FP32 over K chunks of at most
 *                     4096 that are added in FP64, an error of at most
 *                     (3 2^-16 + 4096 2^-24) sum_k |a_k b_k| per inner
 *                     product.  The first use splits the projector table
 *                     (4 bytes per entry in each of two orientations) and
 *                     allocates a band-sized BF16 buffer. */
typedef enum { ROKS_FP64 = 0, ROKS_FP32 = 1, ROKS_FP32_BF16X3 = 2 } roks_precision;

enum {
  ROKS_XC_PW92 = 0, /* spin LDA: Slater exchange + Perdew-Wang 1992 correlation */
  ROKS_XC_X = 1,    /* spin LDA exchange only                                   */
  ROKS_XC_PBE = 2   /* spin GGA: Perdew-Burke-Ernzerhof 1996 exchange and
                       correlation (the functional of the paper's Sec. III);
                       density gradients and the divergence of the gradient
                       terms spectral on the FFT grid, Nyquist components
                       zeroed on even grids                                    */
};

enum {
  /* Sec. II A (collapse to a triplet-like state): set the F^a - F^b block of
   * R (Eq. r_matrix_singlet) to zero, i.e. do not rotate open shell a into b. */
  ROKS_FLAG_SUPPRESS_OPEN_COUPLING = 1u,
  /* also rotate within occupied shells with the Jacobi angle that diagonalises
   * the shell's own block of R (energy neutral) */
  ROKS_FLAG_CANONICALIZE = 2u,
  /* divide the Teter preconditioner of band n by its weight sum c_L f_n */
  ROKS_FLAG_WEIGHT_PRECOND = 4u,
  /* choose the split count of the band-space GEMMs by timing candidates on
   * the first use of each (M, N, K) shape; the choice is shared by all the
   * process's contexts.  It changes the order of the FP64 sums, so results
   * agree to rounding, not bit for bit, between processes.  With the
   * environment variable ROKS_TUNE_CACHE naming a file, the choices are read
   * from it on the first use (entries of the same GPU architecture and
   * compute-unit count only) and the file is rewritten (JSON, through a
   * temporary file and a rename) after every newly timed shape, so processes
   * that share the file make the same choices and agree bit for bit; an
   * unreadable or unwritable file only means timing again. */
  ROKS_FLAG_AUTOTUNE = 8u,
  /* roks_solve (and so roks_batch_solve) runs its iterations in graph mode
   * (roks_graph_steps, 8 at a time) while the context is within that mode's
   * scope and at least 8 iterations remain, and a host step after a rejected
   * one; the convergence test reads the records in order (iterations run
   * past the point of convergence within a replay are counted). */
  ROKS_FLAG_GRAPH = 16u
};

/* Separable Gaussian projector of one radial channel (Sec. II A, projector
 * functions beta): unit-normalised exp(-r^2/(2 rp^2)) times a real solid
 * harmonic of degree l in {0, 1} (l = 1 expands to x, y, z). */
typedef struct {
  int32_t l;
  double rp; /* bohr, > 0 */
} roks_proj;

/* Species: local Gaussian well v(r) = -A exp(-r^2/(2 sigma^2)) and nproj
 * radial channels with the symmetric coupling D[nproj][nproj] (Ha) of
 * V_NL = sum_ij |beta_i> D_ij <beta_j|; D_ij must vanish when l_i != l_j.
 * q[nproj][nproj] (NULL: zeros) are the overlap coefficients of Sec. II A's
 * PAW overlap S = 1 + sum_kl q_kl |beta_l><beta_k| over each atom's
 * projectors: symmetric, zero when l_k != l_l, S positive definite.  S
 * enters the orthonormality constraint <m|S|n> = delta_mn and with it the
 * gradient (Eq. gradient: g_I = (1 - sum_m S|m><m|) F^n|n>), the projection
 * of the preconditioned gradient (Eq. prec_grad_I), the orthonormalisation
 * and the overlap term of the forces (Eq. force_hf); the density carries no
 * augmentation charge (sum_n f_n |psi_n|^2), so the energy depends on q only
 * through the constraint.  With q != 0 the orbitals move with the atoms:
 * roks_set_positions S-orthonormalises them for the new S. */
typedef struct {
  double A;
  double sigma;
  int32_t nproj;
  const roks_proj* proj;
  const double* D;
  const double* q;
} roks_species;

/* The problem statement (Sec. II A / III): cell, cutoff, atoms, projectors,
 * bands and the occupations f_n^{sigma L} of each configuration L with
 * weight c_L.  occ is [nconfig][2 spins (up, down)][nbands] with entries in
 * {0, 1}; bands must be ordered closed shell, open shells, virtual (the
 * shells are the groups of identical occupation patterns, Sec. II A). */
typedef struct {
  double cell[3][3];  /* rows a1, a2, a3 (bohr); non-singular               */
  double ecut;        /* Ha, sphere |G|^2/2 <= ecut                        */
  int32_t grid[3];    /* FFT grid; every size of the form 2^a 3^b 5^c <= 128;
                         {0, 0, 0}: the grid rule G_cut = pi N_d / (2 |a_d|),
                         N_d the next such size >= 2 sqrt(2 ecut) |a_d| / pi  */
  int32_t natoms;
  const int32_t* species; /* [natoms] index into spec                     */
  const double* pos;      /* [natoms][3] Cartesian bohr                   */
  int32_t nspecies;
  const roks_species* spec;
  int32_t nbands;
  int32_t nconfig;        /* 1 (ground state, triplet) or 2 (singlet ROKS) */
  const uint8_t* occ;
  const double* cL;       /* [nconfig], e.g. {2, -1}                       */
  int32_t xc;             /* ROKS_XC_*                                     */
  int32_t precision;      /* roks_precision                                */
  uint32_t flags;         /* ROKS_FLAG_*                                   */
  double exx;             /* fraction a of exact (Fock) exchange mixed into
                             PBE (xc = ROKS_XC_PBE; 0: none; 0.25 is PBE0,
                             1/eps_inf a dielectric-dependent hybrid, Sec.
                             III): E_xc = a E_x^HF + (1 - a) E_x^PBE + E_c^PBE
                             per configuration, E_x^HF[L] = -1/2 sum_sigma
                             sum_mn f_m f_n int psi_m psi_n V[psi_m psi_n]
                             with the Coulomb kernel without G = 0, and
                             H^{sigma L} += a K^{sigma L}, K|v> = -sum_m
                             f_m^{sigma L} psi_m V[psi_m v].  Costs one
                             Poisson transform per (band pair, occupied
                             orbital) in every apply and energy
                             evaluation.  In [0, 1].                       */
} roks_system;

/* Energies of the current orbitals (Sec. II A, constrained functional). */
typedef struct {
  double E;             /* sum_L c_L E_L (E_S for the singlet)            */
  double E_L[2];        /* configuration energies                         */
  double kinetic[2];    /* sum_sigma,n f <n|T|n> per configuration        */
  double nonlocal[2];   /* sum_sigma,n f <n|V_NL|n>                       */
  double external[2];   /* int V_ext rho_L                                */
  double hartree[2];    /* 1/2 int V_H[rho_L] rho_L                       */
  double xc[2];         /* E_xc[rho_L^up, rho_L^down]                     */
} roks_energies;

/* Outcome of one CG iteration. */
typedef struct {
  double E0;       /* energy at the start of the step                     */
  double E1;       /* energy after the step                               */
  double delta;    /* accepted step length                                */
  double beta;     /* Fletcher-Reeves ratio used (0 after a restart)      */
  double dE0;      /* directional derivative dE/d delta at 0              */
  double norm_gI;  /* || g_I ||, out-of-subspace gradient (Eq. gradient)  */
  double max_Rab;  /* max |<a|F^a - F^b|b>| over the open shells (Eq. stat2) */
  int32_t restarted;   /* CG direction reset to the preconditioned gradient */
  int32_t stalled;     /* no decrease found at rounding level: no move      */
  int32_t evaluations; /* trial-energy evaluations in the line search       */
  int32_t iteration;
  int32_t learned;     /* the step used the attached network's rescaling    */
  int32_t fallback;    /* the learned direction failed; the step was redone
                          with the plain Teter preconditioner, beta = 0     */
} roks_step_info;

/* Build a context: validate the system, build the plane-wave sphere and FFT
 * maps, upload V_ext and the projector tables.  hip_stream may be NULL (the
 * null stream) or a hipStream_t owned by the caller that outlives ctx. */
roks_status roks_create(const roks_system* sys, void* hip_stream, roks_ctx* out);
roks_status roks_destroy(roks_ctx ctx);
const char* roks_last_error(roks_ctx ctx);
const char* roks_version(void);

/* The FFT grid of the grid rule (Sec. III's cells: the density-exact grid
 * of the cutoff sphere), what roks_create takes for grid = {0, 0, 0}:
 * N_d = the smallest 2^a 3^b 5^c >= 2 sqrt(2 ecut) |a_d| / pi.  Host only,
 * no device needed.  ROKS_ERR_ARG for ecut <= 0 or NULL pointers. */
roks_status roks_grid_rule(const double cell[3][3], double ecut, int32_t grid[3]);

/* Sizes: stored plane waves, FFT grid, projectors (l = 1 counts 3), bands. */
roks_status roks_sizes(roks_ctx ctx, int32_t* npw, int32_t grid[3], int32_t* nproj,
                       int32_t* nbands);
/* Miller triples of the stored plane waves, [npw][3] int32, storage order. */
roks_status roks_gvectors(roks_ctx ctx, int32_t* miller);

/* Set the orbitals from c [nbands][npw][2]; orthonormalize != 0 applies the
 * Cholesky orthonormalisation in band order (Gram-Schmidt; of <m|S|n> with
 * overlap coefficients q, so that the orbitals are S-orthonormal).  Resets the CG
 * state.  The G = 0 coefficient of a real orbital is real: roks_set_coeffs
 * rejects a nonzero Im c_n(0) with ROKS_ERR_ARG; roks_set_coeffs_d (which
 * does not read the data on the host) sets Im c_n(0) to zero.  Linearly
 * dependent bands (a Cholesky pivot below 1e-12 of its Gram diagonal) give
 * ROKS_ERR_NOT_PD.  roks_pcg_step / roks_solve take the orbitals to be orthonormal
 * (every step keeps them so): pass orthonormalize = 0 only for orthonormal
 * input.  roks_get_coeffs copies the current orbitals out. */
roks_status roks_set_coeffs(roks_ctx ctx, const double* c, int32_t orthonormalize);
roks_status roks_get_coeffs(roks_ctx ctx, double* c);
roks_status roks_set_coeffs_d(roks_ctx ctx, const void* c_dev, int32_t orthonormalize);
roks_status roks_get_coeffs_d(roks_ctx ctx, void* c_dev);

/* Move the atoms ([natoms][3] bohr): rebuilds V_ext and the projector tables
 * and resets the CG state; orbitals are kept (with overlap coefficients q
 * they are S-orthonormalised for the new S, ROKS_ERR_NOT_PD as in
 * roks_set_coeffs). */
roks_status roks_set_positions(roks_ctx ctx, const double* pos);

/* Apply the Kohn-Sham operators of the current orbitals' density to the
 * vectors c_in [nbands][npw][2] (NULL: the current orbitals).
 *   channel_mask == 0 ("shell mode"): h_out[n] = F^{X(n)} c_in[n] with F^X
 *     the shell operator of band n (Eq. shell_operator; zero for virtual
 *     bands); h_out is [nbands][npw][2].
 *   channel_mask != 0: bit (2 L + s) selects H^{sigma L} (Eq. for H^{sigma L}:
 *     T + V_NL + V_ext + V_H[rho_L] + v_xc^sigma[rho_L]); h_out is
 *     [popcount(mask)][nbands][npw][2] in increasing bit order.
 * Input bands are real orbitals: roks_apply_h rejects a nonzero Im c_n(0)
 * (ROKS_ERR_ARG); roks_apply_h_d does not read it (takes it as zero). */
roks_status roks_apply_h(roks_ctx ctx, const double* c_in, uint32_t channel_mask,
                         double* h_out);
roks_status roks_apply_h_d(roks_ctx ctx, const void* c_in_dev, uint32_t channel_mask,
                           void* h_out_dev);

/* For callers that cannot allocate device memory while they run (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * roks_apply_h_d with every scratch buffer of its kernels -- the FFT column
 * buffer, the projections <beta|c_in> and D<beta|c_in>, the split-K partials
 * of the projection product -- taken from one static device array of
 * ROKS_NOALLOC_SCRATCH_BYTES per GPU (held from the first context on that GPU
 * until the process ends) instead of the context's buffers; the bands go
 * through the column buffer in as many chunks of band pairs as needed.  It
 * calls no allocator (the split autotuner is bypassed).  Same arguments,
 * layouts and results as roks_apply_h_d (c_in_dev NULL: the orbitals).
 * Requires the potentials of the current orbitals (after roks_energy_gradient,
 * roks_apply_h or a CG step; else ROKS_ERR_STATE) and the FP64 or FP32
 * tier (ROKS_ERR_STATE in ROKS_FP32_BF16X3); ROKS_ERR_SHAPE when the
 * system's projections (two nproj x nbands arrays, one with c_in_dev NULL)
 * and one band pair's column buffer do not fit the array.  Every call on one
 * GPU uses that GPU's array and leaves its contents behind (nothing in it
 * has to start at zero): calls that overlap on one GPU, from any contexts or
 * streams, race and must be serialised by the caller. */
#define ROKS_NOALLOC_SCRATCH_BYTES (64u << 20)
roks_status roks_apply_h_noalloc_d(roks_ctx ctx, const void* c_in_dev, uint32_t channel_mask,
                                   void* h_out_dev);

/* Energies of the current orbitals and, if grad != NULL, the out-of-subspace
 * gradient g_I,n = (1 - sum_m S|m><m|) F^n|n> (Eq. gradient), [nbands][npw][2];
 * if theta != NULL the matrix theta_mn = <m|F^n|n> (Sec. II A, theta form of
 * the gradient), [nbands][nbands] row-major (row m). */
roks_status roks_energy_gradient(roks_ctx ctx, roks_energies* e, double* grad,
                                 double* theta);

/* Subspace matrices of the current orbitals, each [nbands][nbands]
 * row-major: R_mn (Eq. r_matrix_singlet, with <m|F^c|n> in the block of the
 * virtual bands, zero there without a closed shell), the pair curvature
 * kappa_mn and the rotation generator A_mn (Eqs. prec_grad_IIb/c).  Any
 * pointer may be NULL. */
roks_status roks_subspace(roks_ctx ctx, double* R, double* kappa, double* A);

/* One preconditioned CG iteration with line search (Eqs. orbital_update,
 * cg_search, prec_grad_I, prec_k and the conjugated rotation
 * U = exp(Delta (A^i + gamma A^{i-1}))).  info is complete on return; the
 * update of the carried directions (S_old, D_old) may still run on the
 * context's stream, ordered before the work of every later call (an
 * exception to the synchronisation rule above: nothing the caller can read
 * depends on it). */
roks_status roks_pcg_step(roks_ctx ctx, roks_step_info* info);
/* Graph mode: k CG iterations with every decision taken on the device, so
 * that they form one fixed launch sequence, captured once as a HIP graph
 * (kept with the context, captured again when k, the tier or the flags
 * change) and replayed by each call.  Each iteration is roks_pcg_step's
 * (the same equations, the same first line-search attempt: trial at the
 * kept step length, the parabola's step, the lower of the two taken if it
 * lies below E(0) with dE0 < 0, the Fletcher-Reeves ratio dropped when the
 * direction does not descend), with the energy sums, the ratio, the trial
 * steps and the choice formed by small kernels from device scalars, and
 * the new orbitals and carried directions copied in only when the step is
 * accepted.  The first rejected iteration halts the rest (they change
 * nothing): *accepted receives the number of leading accepted iterations,
 * and a caller continues with roks_pcg_step, whose halvings of the trial
 * step and steepest-descent retry graph mode does not take.  info (nullable)
 * receives k records (stalled = 1 from the first rejected one; evaluations
 * 2 for each iteration run before the halt).  Within rounding the results
 * are those of roks_pcg_step (the first trial's potentials are formed too
 * and kept when it is taken, the energy of the orbitals a replay starts
 * from is evaluated again, and past 78 bands the trial rotation exp(delta
 * D) takes a Taylor polynomial of degree 18 and the squarings (at most 12,
 * else the trial fails) chosen on the device).  Scope (else
 * ROKS_ERR_STATE): the FP64 or FP32 tier, no exact exchange, overlap
 * coefficients, recording, canonicalisation or autotuning (periodic
 * restarts and an attached network's rescaling are taken on the device; a
 * learned search that fails halts the replay, and the host step then
 * retries with the plain preconditioner); ROKS_ERR_ARG for k outside
 * 1 .. 1024.  The call synchronizes the context's stream; the first call
 * for a k (or after a change of tier or flags) also runs one iteration that
 * commits nothing (first-use set-up outside the capture). */
roks_status roks_graph_steps(roks_ctx ctx, int32_t k, roks_step_info* info, int32_t* accepted);

/* Forget the carried search directions (next step is steepest descent). */
roks_status roks_reset_cg(roks_ctx ctx);
/* Restart the CG recursion every `period` steps (0, the default: never, the
 * plain Fletcher-Reeves recursion).  A restart drops the carried directions
 * and resets the trial step length; the step reports restarted = 1.  The
 * count starts at roks_set_coeffs / roks_reset_cg. */
roks_status roks_set_restart(roks_ctx ctx, int32_t period);
/* Switch the arithmetic tier (roks_precision) for the following calls,
 * keeping the orbitals and the CG state: a precision ladder runs FP32 (or
 * FP32_BF16X3) iterations first and polishes in FP64.  With overlap
 * coefficients q, leaving FP32_BF16X3 S-orthonormalises the orbitals again
 * in the new tier and resets the CG state (that tier forms the q part of
 * the S-Gram matrix from split-precision projections, so its orbitals are
 * S-orthonormal only to that rounding); ROKS_ERR_NOT_PD as in
 * roks_set_coeffs. */
roks_status roks_set_precision(roks_ctx ctx, int32_t precision);
/* Iterate roks_pcg_step until |E_{i+1} - E_i| < tol on two consecutive
 * iterations or maxiter; *iterations receives the count, *last the final
 * step's info (either may be NULL).  A stalled step (no decrease found) does
 * not count toward the two: the carried directions are dropped and the step
 * is retried from the preconditioned gradient.  If that stalls too, the solve
 * ends with ROKS_OK when the first-order decrease the line search could reach,
 * |dE0| times its smallest trial step, is below max(tol, r |E|) (r = 1e-12 in
 * FP64, 2e-6 in the FP32 tier: the energy's resolution), and otherwise with
 * ROKS_ERR_LINESEARCH (orbitals of the last accepted step). */
roks_status roks_solve(roks_ctx ctx, double tol, int32_t maxiter, roks_step_info* last,
                       int32_t* iterations);

/* DIIS on the residual of Eq. residual_frank (Sec. II A; the DIIS method of
 * Hutter, Luthi and Parrinello that the paper names), an alternative to the
 * CG step that can also converge onto saddle points of the functional.
 * Each step, from the current orbitals:
 *   r_n = F^n|n> - sum_m |m> Lambda_mn, Lambda_mn = theta_mn -
 *         lambda_mn (theta_mn - theta_nm), theta_mn = <m|F^n|n>, with
 *         lambda_mn = 1/2 (r is then the full gradient of Eq. gradient) or,
 *         with `asymmetric`, lambda_ab = 1/2 and lambda_ba = -1/2 for the two
 *         open bands a < b (the coupling the paper uses to steer away from
 *         the triplet-like collapse; lambda_mn multiplies the coefficient of
 *         |m> in the residual of band n);
 *   e_n = K_n r_n, the Teter preconditioner of Eq. prec_k with E_ref =
 *         1.5 <r_n|T|r_n> / <r_n|r_n> and no projection;
 *   the orbitals and e of the last `history` steps are kept; c minimises
 *         c^T B c subject to sum c = 1, B_ij = sum_n <e^i_n|e^j_n> (the
 *         oldest iterates are dropped while that system is singular);
 *   psi = sum_i c_i (psi^i + step e^i), orthonormalised by the Cholesky
 *         factor of its Gram matrix in band order.
 * The kept iterates stay with the context until roks_diis_reset,
 * roks_set_coeffs, roks_set_positions, a CG step, or a call with another
 * history or coupling; a DIIS step drops the carried CG directions.  The
 * first step allocates 2 ROKS_DIIS_MAX_HISTORY band arrays.  If the new
 * orbitals are linearly dependent (ROKS_ERR_NOT_PD) the step's input
 * orbitals are kept and the history is dropped. */
#define ROKS_DIIS_MAX_HISTORY 8
typedef struct {
  int32_t history;    /* iterates combined, 1 .. ROKS_DIIS_MAX_HISTORY    */
  double step;        /* length of the preconditioned residual step, > 0  */
  int32_t asymmetric; /* 1: lambda_ab = 1/2, lambda_ba = -1/2             */
} roks_diis_params;
typedef struct {
  double E;             /* energy of the step's input orbitals            */
  double rnorm2;        /* sum_n <r_n|r_n>                                */
  double open_coupling; /* theta_ab - theta_ba of the open pair (0 without) */
  int32_t used;         /* iterates combined                              */
  double coeffs[ROKS_DIIS_MAX_HISTORY]; /* their coefficients, oldest first */
} roks_diis_info;
roks_status roks_diis_step(roks_ctx ctx, const roks_diis_params* params, roks_diis_info* info);
/* roks_diis_step until |E_{i+1} - E_i| < tol on two consecutive steps or
 * maxiter (the CG solve's rule); *last and *iterations as in roks_solve. */
roks_status roks_diis_solve(roks_ctx ctx, const roks_diis_params* params, double tol,
                            int32_t maxiter, roks_diis_info* last, int32_t* iterations);
roks_status roks_diis_reset(roks_ctx ctx);

/* Hellmann-Feynman forces F_I = -dE/dR_I (Eq. force_hf) at the current
 * orbitals, [natoms][3] Ha/bohr.  With overlap coefficients q the overlap
 * term -sum_{m,n occupied} gamma_mn <m|dS/dR_I|n>, gamma_mn = (theta_mn +
 * theta_nm) / 2 (Eq. gamma_def), is included; it costs one more application
 * of the shell operators.  The term is contracted as Tr(gamma S'), equal to
 * the gamma-diagonalised form of SI section S2. */
roks_status roks_forces(roks_ctx ctx, double* f);

/* Geometry relaxation and the Franck-Condon cycle (Sec. IV B).  The total
 * energy of a geometry is the electronic E at its minimum (roks_solve from
 * the current orbitals with the CG restarted every scf_restart iterations:
 * without restarts an excited state's solve from ground-state orbitals can
 * stall far above its minimum; the context's own restart period is restored
 * afterwards) plus an ion-ion pair repulsion
 *   sum_{I<J} sum_t pair_B exp(-|R_I - R_J - t| / pair_rho)
 * over the 27 nearest cell translations t (the synthetic Gaussian-well
 * atoms carry no ionic charge, and the paper's total energies include the
 * ions' repulsion; pair_B = 0 drops it); the forces are Eq. force_hf's plus
 * that term's.  Positions move by BFGS on the Cartesian coordinates (fixed
 * cell): inverse Hessian h0 I to start, step s = H F scaled so that no atom
 * moves more than max_step, the BFGS update of H when s.(F_old - F_new) > 0
 * (else h0 I again); a step that raises the energy is halved, at most four
 * times, from the accepted geometry's orbitals, with H reset.  Stops when
 * max_I |F_I| < fmax or after maxsteps steps.  Units: Ha, bohr. */
typedef struct {
  double fmax;          /* force threshold, Ha/bohr                       */
  int32_t maxsteps;     /* BFGS steps                                     */
  double scf_tol;       /* roks_solve tolerance at every geometry, Ha     */
  int32_t scf_maxiter;  /* roks_solve iteration limit                     */
  int32_t scf_restart;  /* CG restart period of those solves (0: none)    */
  double max_step;      /* largest atomic displacement of a step, bohr    */
  double h0;            /* initial inverse Hessian, bohr^2 / Ha           */
  double pair_B;        /* pair repulsion amplitude, Ha (>= 0)            */
  double pair_rho;      /* pair repulsion range, bohr (> 0)               */
} roks_relax_params;
typedef struct {
  double E;             /* total energy at the last geometry              */
  double fmax;          /* its largest atomic force                       */
  int32_t steps;        /* BFGS steps taken                               */
  int32_t scf_iterations; /* CG iterations over all geometries            */
  int32_t converged;    /* fmax reached                                   */
} roks_relax_info;
/* Relax the context's positions (and orbitals); needs orbitals. */
roks_status roks_relax(roks_ctx ctx, const roks_relax_params* params, roks_relax_info* info);
/* The current positions [natoms][3]. */
roks_status roks_get_positions(roks_ctx ctx, double* pos);
typedef struct {
  double E_gs_at_gs, E_ex_at_gs, E_ex_at_ex, E_gs_at_ex; /* total energies  */
  double E_abs;   /* E^ex(R_gs) - E^gs(R_gs), vertical absorption          */
  double E_FC_ex; /* E^ex(R_gs) - E^ex(R_ex)                               */
  double E_FC_gs; /* E^gs(R_ex) - E^gs(R_gs)                               */
  double E_emi;   /* E_abs - E_FC_ex - E_FC_gs                             */
  double dQ;      /* [sum_I M_I |R^ex_I - R^gs_I|^2]^1/2, amu^1/2 bohr      */
  int32_t gs_steps, ex_steps, converged;
} roks_fc_result;
/* The cycle of Sec. IV B on two contexts of one system, `gs` with the
 * ground-state occupations (its orbitals the start) and `ex` with the
 * excited ones: relax gs (R_gs); solve ex at R_gs from the relaxed
 * ground-state orbitals; relax ex from there (R_ex); solve gs at R_ex from
 * its relaxed orbitals.  masses [natoms] in amu.  Both contexts end at R_ex
 * with their last orbitals. */
roks_status roks_franck_condon(roks_ctx gs, roks_ctx ex, const roks_relax_params* params,
                               const double* masses, roks_fc_result* out);

/* Wait for all work enqueued on the context's stream. */
roks_status roks_synchronize(roks_ctx ctx);

/* Diagnostics (no paper counterpart): GPU time of the library's kernels,
 * measured with HIP events recorded on the context's stream around each
 * launch.  roks_timing_enable(ctx, 1) clears the totals and starts
 * recording, 0 stops.  roks_timing_read() synchronises the stream and
 * returns, for one kernel family ("zpass_bwd", "plane_apply",
 * "plane_density", "zpass_fwd", "fft3d", "gemm_wdot", "gemm_expand", "xc",
 * "proj_bf3": the split and product launches of a BF16x3 projector product,
 * its flops those of the three BF16 products),
 * the summed milliseconds, the launch count and the summed algorithmic HBM
 * bytes and flops of those launches (the minimum traffic and arithmetic the
 * launches' inputs and outputs imply); unknown names give zero.  Any output
 * pointer may be NULL. */
roks_status roks_timing_enable(roks_ctx ctx, int32_t enable);
/* Record only the launches of one kernel family (NULL or "": all).  Every
 * recorded launch adds two events to the stream; restricting the recording
 * to the family being measured keeps the others' timing undisturbed. */
roks_status roks_timing_only(roks_ctx ctx, const char* kernel);
roks_status roks_timing_read(roks_ctx ctx, const char* kernel, double* total_ms,
                             int32_t* launches, double* bytes, double* flops);

/* ------------------------------------------------------------------------
 * Learned rescaling of the Teter preconditioner.  Not part of the paper: it
 * modifies K of Eq. prec_k to s K, p_I = (1 - P)(s K g_I), with
 * s = exp(2 tanh(o)) in [e^-2, e^2] (K stays negative definite) and o the
 * output of a 3-64-64-1 network with GELU activations (erf form).  The
 * network sees, for band n and one distinct |G|^2 ("G shell"), the features
 *   x = (log(1 + (|G|^2/2)/E_ref,n), log <n|T|n>, log ||g_I,n||),
 * E_ref,n = 1.5 <g_n|T|g_n>/<g_n|g_n>, and its factor is shared by every G
 * of the shell.  Parameters (ROKS_MLP_PARAMS floats, flat, row-major):
 *   W1[64][3], b1[64], W2[64][64], b2[64], w3[64], b3.
 * The library keeps FP32 master parameters and evaluates with their BF16
 * rounding (nearest, ties to even); activations and sums are FP32.
 *
 * Training pairs: roks_record() makes the following roks_pcg_step calls keep
 * the iterate psi_i, the plain Teter K g_I and the features.  Once converged,
 * roks_mlp_collect() takes the context's orbitals as psi_inf, aligns them to
 * each recorded psi_i within every occupation shell by the orthogonal polar
 * factor Q of O_mn = <psi_inf_m|psi_i,n> (psi_inf'_n = sum_m Q_mn psi_inf_m),
 * forms the correction delta_n = (1 - P_i) psi_inf'_n and stores, for each
 * occupied band n with a usable gradient and each G shell k, the features
 * and the moments alpha = <Kg_n|delta_n>_k, beta = <Kg_n|Kg_n>_k,
 * gamma = <delta_n|delta_n>_k (full-sphere sums restricted to the shell).
 * The samples of one recorded iterate form a segment; its loss is
 * 1 - A^2/(B C) with A = sum s alpha, B = sum s^2 beta, C = sum gamma over
 * the segment: one minus the squared cosine between the rescaled
 * preconditioned gradient of all bands and the correction of all bands.  It
 * fixes the shape and the relative weights of the bands, not the overall
 * length (the line search sets it).  The training loss is the mean over
 * segments with B, C > 0, minimised with Adam (beta1 = 0.9, beta2 = 0.999,
 * eps = 1e-8, bias-corrected).
 *
 * Inside a CG step the factor is renormalised by one constant for all bands
 * so that sum_n <s K g_n|g_n> equals the plain sum_n <K g_n|g_n>: the
 * first-order energy change along the out-of-subspace direction, and its
 * balance with the rotation that shares the line search, stay those of the
 * plain preconditioner.
 *
 * A network's calls are ordered on its stream and synchronise it before
 * returning; a network attached to contexts must not be trained while their
 * steps run.  Errors as for contexts; roks_mlp_last_error gives the message.
 * ------------------------------------------------------------------------ */
#define ROKS_MLP_PARAMS 4481
typedef struct roks_mlp_s* roks_mlp;

/* theta: initial parameters [ROKS_MLP_PARAMS] (copied), or NULL for the
 * library's seeded initialisation (uniform +-1/sqrt(fan_in), the output
 * layer scaled by 1e-2, b3 = 0; splitmix64 stream from seed).  hip_stream
 * NULL: the network creates its own. */
roks_status roks_mlp_create(const float* theta, uint64_t seed, void* hip_stream, roks_mlp* out);
roks_status roks_mlp_destroy(roks_mlp mlp);
const char* roks_mlp_last_error(roks_mlp mlp);
/* Replace the parameters (and reset the Adam moments); read the FP32 master copy. */
roks_status roks_mlp_set_params(roks_mlp mlp, const float* theta);
roks_status roks_mlp_get_params(roks_mlp mlp, float* theta);
/* o for nsamples feature rows x [nsamples][3] (host arrays). */
roks_status roks_mlp_forward(roks_mlp mlp, const float* x, int64_t nsamples, float* o);
/* Size of the training set: samples and segments (recorded iterates). */
roks_status roks_mlp_num_samples(roks_mlp mlp, int64_t* nsamples, int32_t* nsegments);
/* Copy the training set out: x [nsamples][3], moments [3][nsamples] (alpha,
 * beta, gamma), segment_offsets [nsegments + 1] (segment j is samples
 * segment_offsets[j] .. segment_offsets[j+1]-1, band-major, shells in
 * ascending |G|^2).  Any pointer may be NULL. */
roks_status roks_mlp_get_samples(roks_mlp mlp, float* x, double* moments,
                                 int32_t* segment_offsets);
roks_status roks_mlp_clear_samples(roks_mlp mlp);
/* Loss over the training set at the current parameters and, if grad is not
 * NULL, its gradient [ROKS_MLP_PARAMS].  ROKS_ERR_STATE without samples. */
roks_status roks_mlp_loss_grad(roks_mlp mlp, double* loss, float* grad);
/* steps Adam iterations with learning rate lr > 0; loss_history [steps]
 * (nullable) receives the loss before each update. */
roks_status roks_mlp_train(roks_mlp mlp, int32_t steps, double lr, double* loss_history);

/* Record every stride-th iterate (iteration count modulo stride == 0) of the
 * following roks_pcg_step calls, at most max_records (device memory:
 * max_records x (2 nbands npw_half 16 B + nbands n_shells 12 B)); 0 stops
 * recording and drops what is kept. */
roks_status roks_record(roks_ctx ctx, int32_t max_records, int32_t stride);
/* Turn the context's records into training samples of mlp with the current
 * orbitals as psi_inf, then drop the records.  *used counts the records
 * taken, *skipped those whose polar iteration did not converge (an exactly
 * singular overlap block). */
roks_status roks_mlp_collect(roks_mlp mlp, roks_ctx ctx, int32_t* used, int32_t* skipped);
/* Attach a network to the context (NULL: plain Teter).  Its steps then use
 * s K and fall back to the plain preconditioner when the learned direction
 * finds no decrease. */
roks_status roks_set_mlp(roks_ctx ctx, roks_mlp mlp);

/* ------------------------------------------------------------------------
 * Batches of independent systems (many structures and both configurations
 * of uneven sizes).  A batch holds existing contexts (not owned; no context
 * may appear twice).  Up to `workers` host threads take the contexts from a
 * queue ordered by decreasing estimated cost (nb N^3 log N + nproj nb npw:
 * longest first), so the kernels of different systems overlap on the GPU.
 * roks_batch_create makes one stream per worker on the device of ctxs[0]
 * (ROKS_ERR_HIP if it cannot); while a worker runs a context of that device,
 * the context's launches go to the worker's stream, with the context's own
 * stream synchronized before and the worker's after, so results do not
 * depend on the stream; contexts of other devices run on their own streams.
 * No other call may use a context of a running batch.  Per-context outcomes
 * are returned in arrays indexed like `ctxs`; the call returns ROKS_OK when
 * the batch ran (check the per-context statuses).
 * ------------------------------------------------------------------------ */
typedef struct roks_batch_s* roks_batch;
roks_status roks_batch_create(const roks_ctx* ctxs, int32_t n, int32_t workers, roks_batch* out);
roks_status roks_batch_destroy(roks_batch batch);
/* roks_solve(tol, maxiter) on every context; with switch_tol > 0 a context in
 * the FP32 tier first solves to switch_tol, then switches to FP64 (the
 * precision ladder).  status [n] (nullable), iterations [n] (nullable, the
 * total over both tiers), last [n] (nullable, the final step's info). */
roks_status roks_batch_solve(roks_batch batch, double tol, int32_t maxiter, double switch_tol,
                             roks_status* status, int32_t* iterations, roks_step_info* last);
/* `steps` CG steps on every context (a fixed amount of work). */
roks_status roks_batch_steps(roks_batch batch, int32_t steps, roks_status* status);
/* roks_graph_steps(k) on every context, each graph replayed on its
 * worker's stream: status [n] and accepted [n] (both nullable). */
roks_status roks_batch_graph_steps(roks_batch batch, int32_t k, roks_status* status,
                                   int32_t* accepted);

#ifdef __cplusplus
}
#endif

#endif /* ROKS_H */
