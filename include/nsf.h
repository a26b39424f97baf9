/*
 * nsf.h -- C ABI of the MI355X null-space-free Maxwell eigensolver.
 *
 * The library solves the discrete Maxwell GEP on a Yee grid,
 *     diag(C, C^*) [E; H] = omega * i [[zeta_d, mu_d], [-eps_d, -xi_d]] [E; H]
 * (Sec. 3), through the null-space-free HHPD pencil of Thm 4.2,
 *     B_r y = omega^{-1} A_r y,
 *     A_r = diag(P_r^*, Q_r^*) L diag(Phi^{-1}, mu_d^{-1}) L^* diag(P_r, Q_r),
 *     B_r = i [[0, Sigma_r^{-1}], [-Sigma_r^{-1}, 0]],
 * where C = P_r Sigma_r Q_r^* is the SVD of the single-curl operator
 * (Thm 2.5).  P_r and Q_r are applied with twisted 3-D FFTs (Sec. 4.2), the
 * linear systems with A_r are solved by conjugate gradients (Sec. 4.2) and the
 * pencil by invert Lanczos with thick restarts (Sec. 4.2, Algorithm 1).
 *
 * Conventions (all calls):
 *  - Every function returns an int status (NSF_OK = 0).  Nothing throws or
 *    aborts across this boundary.  nsf_last_error() gives a message.
 *  - Complex numbers are nsf_c128 {re, im} (layout of hipDoubleComplex).
 *  - Grid index g = i1 + n1*i2 + n1*n2*i3 (x fastest), the Kronecker order of
 *    C_1 = delta_x^{-1} (I (x) I (x) K) (Sec. 2).  Frequency index f uses the
 *    same order over (i1, i2, i3), i_l in [0, n_l).
 *  - A 3n field vector is [x-component; y-component; z-component], n each.
 *  - A 4n pencil vector is y = [y_a; y_b; y_c; y_d], n each, frequency order;
 *    [y_a; y_b] multiplies P_r = [P_2, P_1] and [y_c; y_d] multiplies
 *    Q_r = [Q_1, Q_2] (Thm 2.5).
 *  - Pointers marked "device" are HIP device pointers; the call enqueues its
 *    work on the plan's stream and returns without waiting unless it returns
 *    host results.  Pointers marked "host" are ordinary host memory.
 *  - The caller owns every buffer it passes.  The plan owns its tables and its
 *    workspace (hipMalloc'd lazily, freed by nsf_plan_destroy).
 *  - A plan is not thread-safe; distinct plans are independent.
 */
#ifndef NSF_H
#define NSF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nsf_plan_s* nsf_plan;
typedef struct { double re, im; } nsf_c128;

/* Solver counters returned by nsf_eigs / nsf_cg_solve. */
typedef struct {
  long long matvecs;         /* A_r applies (CG iterations + exact applies)     */
  long long cg_iters_total;  /* CG iterations over all solves                   */
  int cg_solves;             /* number of CG solves                             */
  int lanczos_steps;         /* basis expansions                                */
  int restarts;              /* thick restarts                                  */
  int converged;             /* wanted pairs with residual <= res_tol           */
  int ortho_passes;          /* Gram-Schmidt passes over the basis              */
  double cg_iters_avg;       /* cg_iters_total / cg_solves                      */
  double ms_total;           /* wall time of the call (host clock)              */
  double bytes_alg;          /* algorithmic HBM bytes of the A_r applies        */
  double ms_cg;              /* eigensolver phases (host clock, for a batch the */
  double ms_orth;            /*   whole batch's time in each phase): CG solves   */
  double ms_restart;         /*   and exact applies; Gram-Schmidt and basis      */
                             /*   admission; restarts and the final refinement   */
} nsf_stats;

enum {
  NSF_OK = 0,
  NSF_NOT_CONVERGED = 1,  /* results filled; residuals tell which pairs        */
  NSF_E_ARG = -1,         /* bad size, pointer or parameter                    */
  NSF_E_KPOINT = -2,      /* Lambda_q singular: every k_l * a is an integer    */
  NSF_E_BASIS = -3,       /* alpha, beta make Lambda_p rank deficient          */
  NSF_E_NOT_HHPD = -4,    /* mu_d or Phi not HPD, or xi^* != zeta (Sec. 4.1)   */
  NSF_E_BREAKDOWN = -5,   /* CG: p^* A_r p <= 0 or not finite                  */
  NSF_E_NOMEM = -6,       /* device allocation failed                          */
  NSF_E_HIP = -7,         /* HIP runtime error                                 */
  NSF_E_STATE = -8        /* call needs state the plan does not have yet       */
};

/* Medium kinds reported by nsf_plan_query. */
enum { NSF_MEDIUM_NONE = 0, NSF_MEDIUM_CHIRAL = 1, NSF_MEDIUM_PSEUDOCHIRAL = 2, NSF_MEDIUM_GENERAL = 3,
       NSF_MEDIUM_NFSEP = 4 };

/*
 * Create a plan for one Bloch vector on an n1 x n2 x n3 Yee grid of the simple
 * cubic lattice a_l = a e_l (Sec. 1), mesh delta_l = a / n_l.
 *   k[3]        Bloch vector in reciprocal units (2 pi k is the wave vector);
 *               the twist e^{i 2 pi k_l a} closes K_{a,m} (Sec. 2).
 *   alpha, beta the free entries of a = (alpha, beta, 1) in Lambda_p
 *               (Lemma 2.2); the spectrum does not depend on them.
 *   hip_stream  hipStream_t to enqueue on (NULL: the null stream).
 * Host-only: validates and builds the per-axis tables; no device call is made
 * until device work is requested.  Errors: NSF_E_ARG (n_l < 2 or > 512 or with
 * a prime factor other than 2, 3, 5; a <= 0; out == NULL), NSF_E_KPOINT
 * (sigma_f = 0 for some f, i.e. all k_l a integer, Lemma 2.2 (a)),
 * NSF_E_BASIS (Lambda_p has a zero column, Lemma 2.2 (b)).
 */
int nsf_plan_create(nsf_plan* out, int n1, int n2, int n3, double a,
                    const double k[3], double alpha, double beta,
                    void* hip_stream);

/* Tuning options of a plan (nsf_plan_set_option). */
enum {
  NSF_OPT_FFT_PATH = 1,  /* 0: two-level register passes where the axis length
                            allows them, else generic (default),
                            1: generic LDS-staged passes only,
                            2: single-wave passes (E'/H' lane halves) for the
                               x and fused z passes where possible          */
  NSF_OPT_MID_COLS = 2,  /* pencils per workgroup of the fused z pass: 1..16,
                            power of two (default 16)                         */
  NSF_OPT_CG_GRAPH = 3,  /* 1: the eigensolver captures 1, 2, 4 and 8 CG
                            iterations of all unfinished instances as HIP
                            graphs and replays them (default); 0: launches
                            every kernel each iteration                      */
  NSF_OPT_X_ROWS = 4,    /* grid rows per workgroup of the two-level x passes:
                            1, 2 or 4 (default 4; lowered where it does not fit) */
  NSF_OPT_YZ_COLS = 5,   /* pencils per workgroup of the two-level y / z passes:
                            1..16, power of two (default 16; lowered to fit)    */
  NSF_OPT_MID_PAIRS = 6, /* fused z pass of the two-level path: 1 one coupled
                            (E', H') field pair per workgroup (default), 0 all
                            six fields per workgroup                           */
  NSF_OPT_CG_START = 7,  /* eigensolver inner CG: 1 starts from the A_r-Galerkin
                            solution in the span of the Lanczos basis (default),
                            0 from zero; the Lanczos direction is the same     */
  NSF_OPT_VERIFY = 8,    /* nsf_eigs multiplicity checks, 0..16 (default 0): a
                            single start vector finds one direction of a
                            multiple eigenvalue only; each check restarts from a
                            fresh random vector A_r-orthogonal to the converged
                            pairs, keeps the best nev of the union, and stops
                            when nothing changed.  Needed for spectra with
                            multiple eigenvalues (symmetric media at symmetric
                            k-points; air): without it a multiple eigenvalue
                            may be returned fewer times than it occurs.
                            nsf_batch_eigs applies each instance's setting
                            after that instance has converged               */
  NSF_OPT_ORTHO_GATE = 9, /* eigensolver Gram-Schmidt: 1 removes from a new
                            Lanczos direction only its components whose
                            A_r-cosine with a basis vector exceeds 1e-2
                            res_tol, capped at 1e-10, reading just those
                            basis columns (default); 0 always runs the full
                            classical pass; converged pairs meet the
                            residual tolerance either way                    */
  NSF_OPT_GMRES_RESTART = 10, /* restart length of the GMRES inner solves of
                            nsf_eigs_nfsep, 4..500 (default 12: at 128^3 the
                            classical Gram-Schmidt over a long basis costs
                            more than the extra iterations of restarting)  */
  NSF_OPT_MEDIUM_PALETTE = 11, /* general and NFSEP media, read by the next
                            nsf_set_medium_tensor / nsf_set_medium_nfsep: 1
                            stores the distinct voxel factors once plus a
                            16-bit index per voxel when there are at most
                            4096 of them (default; piecewise-constant media),
                            0 always stores one factor per voxel           */
  NSF_OPT_CG_RELAX = 12,  /* eigensolver inner CG tolerance (nsf_eigs,
                            nsf_batch_eigs): 0 (default) solves every system
                            to cg_rtol; 1 relaxes the solves as the Ritz
                            residuals fall (relaxation of inexact Krylov
                            methods): after each restart
                            max(cg_rtol, s min(0.3, 0.1 / eta) res_tol), eta
                            the largest residual of the wanted pairs and
                            s = theta_nev / theta_1 their spread, back to
                            cg_rtol for good once two restarts in a row fail
                            to halve eta.  Measured at 128^3: 3-7% fewer
                            applies at generic k; without s the k-points next
                            to Gamma stalled.  The projected matrix is exact
                            and the returned pairs are checked with exact
                            applies either way                               */
  NSF_OPT_WARM_CHAIN = 13,/* nsf_batch_eigs, set on instance i (default 0):
                            when instance i - 1 has the same grid and was
                            solved in an earlier wave (every instance of
                            2^21 voxels or more is a wave of its own), the
                            Lanczos start of instance i combines the Ritz
                            vectors of instance i - 1 (as nsf_eigs_set_start),
                            which saves steps along a path of nearby k-points;
                            results are checked by their own residuals as
                            for any start                                    */
  NSF_OPT_CG_RING = 14,   /* 1 (default): the q-free fused CG (chiral and
                            pseudochiral media on the fast passes, plan
                            memory) keeps its last 16 directions p_j on the
                            device and adds x += sum alpha_j p_j once every
                            16 iterations and at the end of the solve,
                            instead of reading and writing x in every
                            iteration (128 n bytes less per iteration,
                            16 x 64 n bytes of device memory more); the
                            residual recurrence is unchanged, and a fold
                            performs the same multiply-adds in the same
                            order, so iterations, residuals and x are the
                            same.  0: x updated every iteration           */
  NSF_OPT_VACUUM = 15     /* 1 (default): with a chiral or pseudochiral medium
                            on the two-level passes, the field-pair z pass
                            transforms only the tiles (P pencil columns of
                            one y) holding a voxel other than vacuum (eps 1,
                            gamma 0), and both y passes only the groups of
                            consecutive x holding one: where the middle
                            factor is the identity the transforms around it
                            cancel, once the 1/n normalisation is split as
                            1/n3 (z pass), 1/n2 (forward y) and 1/n1
                            (projection).  p^* A_r p is then |p|^2 plus the
                            listed tiles' share.  The lists are built when
                            the medium is set.  Same operator up to
                            rounding; 0 transforms everything              */
};

/*
 * Environment switches (read at each call):
 *   NSF_TRACE=1|stderr|<file>  one JSON line per finished nsf_eigs, per instance
 *                              of nsf_batch_eigs and per nsf_eigs_nfsep (status,
 *                              counters, phase times, largest residual);
 *   NSF_SYNC_CHECK=1           synchronise the device after every HIP call the
 *                              library checks and report the first failing call
 *                              (debugging; graph capture of CG iterations off);
 *   NSF_TUNE_CACHE=<file>      autotune results kept per grid shape and medium.
 */

/*
 * Device bytes per voxel that an A_r / Kern apply reads for the medium: 16
 * for chiral and pseudochiral media ((eps, gamma)), 336 (general) or 576
 * (NFSEP) for factors stored per voxel, 2 with a palette; palette (nullable)
 * receives the number of distinct voxel factors, 0 when stored per voxel or
 * for chiral / pseudochiral media.  Host-only.
 */
int nsf_plan_medium_info(nsf_plan plan, int* palette, long long* voxel_bytes);

/*
 * Set a tuning option.  Options change speed: the tilings change results by
 * rounding only, the eigensolver options within the requested tolerances.
 * Host-only.  NSF_E_ARG for an unknown option or value.
 */
int nsf_plan_set_option(nsf_plan plan, int option, int value);

/*
 * Autotuner of the FFT pass family and workgroup tiles.  Times reps A_r
 * applies (after two untimed ones) per candidate, by coordinate descent from
 * the defaults (two sweeps): NSF_OPT_FFT_PATH over the families the grid
 * allows, then for the two-level family NSF_OPT_MID_PAIRS {1, 0},
 * NSF_OPT_MID_COLS {4, 8, 16}, NSF_OPT_X_ROWS {1, 2, 4} and NSF_OPT_YZ_COLS
 * {4, 8, 16}.  Keeps the fastest as the plan's
 * options.  Needs a medium (NSF_E_STATE); allocates two 4n scratch vectors
 * for the call (NSF_E_NOMEM).  Results of later calls agree with the defaults
 * to rounding.  Synchronises the stream.
 *   reps    1..1000 timed applies per candidate
 *   result  nullable; the chosen options, the average apply time with them and
 *           with the defaults (microseconds), and the candidates timed
 */
typedef struct {
  int fft_path, mid_cols, x_rows, yz_cols, mid_pairs;
  double us_best, us_default;
  int tried;
} nsf_tune;
int nsf_plan_autotune(nsf_plan plan, int reps, nsf_tune* result);
/* With NSF_TUNE_CACHE naming a text file, nsf_plan_autotune first looks up the
 * grid shape and medium kind there (a hit applies the stored tiling, reports
 * tried = 0 and times nothing) and appends each new result.  With vacuum
 * skipping (NSF_OPT_VACUUM) the kind column also holds 16 x (1 + the share of
 * z-pass tiles that are not all vacuum, in tenths): sparse media tune apart. */

/*
 * Caller-provided workspace (for example from PyTorch's caching allocator).
 * nsf_plan_workspace_size: the device bytes an nsf_eigs call with this nev and
 *   max_basis (as nsf_eigs; 0 for the default) needs for the six field arrays
 *   (96 n B), the CG and Lanczos-step vectors (384 n B), the basis V and A_r V
 *   (2 (m+1) 64 n B) and the projected-matrix scratch, alignment included.
 * nsf_plan_set_workspace: the plan carves those buffers from dev_ptr (any
 *   alignment; the caller keeps ownership and must keep it alive and unused
 *   elsewhere until the plan is destroyed or given another workspace), frees
 *   its own copies of them, and never allocates them again.  An eigensolve that
 *   needs a larger basis than fits returns NSF_E_NOMEM.  dev_ptr = NULL returns
 *   to library-allocated buffers.  NSF_E_ARG if bytes cannot hold the fields,
 *   the CG vectors and a 2-vector basis.  Synchronises the plan's stream; the
 *   contents of the old buffers are not carried over.  Tables, reduction
 *   scratch and the medium stay library-allocated (small, or set once).
 */
int nsf_plan_workspace_size(nsf_plan plan, int nev, int max_basis, size_t* bytes);
int nsf_plan_set_workspace(nsf_plan plan, void* dev_ptr, size_t bytes);

/* Free the plan and all device memory it owns.  NULL is accepted. */
void nsf_plan_destroy(nsf_plan plan);

/*
 * Query plan facts (host).  Any output pointer may be NULL.
 *   n              n1*n2*n3
 *   medium_kind    NSF_MEDIUM_*
 *   sigma_min/max  extreme singular values sigma_f = Lambda_q^{1/2} (Thm 2.5)
 */
int nsf_plan_query(nsf_plan plan, long long* n, int* medium_kind,
                   double* sigma_min, double* sigma_max);

/*
 * Chiral medium (Sec. 4.3): eps_d = diag(eps), mu_d = I, xi_d = i diag(gamma),
 * zeta_d = -i diag(gamma), per voxel g (length n each, float64).  host or
 * device pointers (on_device = 0 / 1); the library keeps its own copy.  The
 * values are validated on the host (device data is copied there first) against
 * the Sec. 4.1 assumption: Phi = eps - gamma^2 > 0 and all finite, else
 * NSF_E_NOT_HHPD or NSF_E_ARG naming the voxel.  Synchronises the stream.
 */
int nsf_set_medium_chiral(nsf_plan plan, const double* eps, const double* gamma,
                          int on_device);

/*
 * Pseudochiral medium (Sec. 4.3): xi_d = i gamma (e_a e_b^T + e_b e_a^T),
 * zeta_d = xi_d^*, mu_d = I, eps_d = diag(eps); axis_a != axis_b in {0,1,2}
 * (0 = x).  Phi = diag(eps - gamma^2 on axes a and b, eps on the third) must
 * be positive.  Errors as nsf_set_medium_chiral.
 */
int nsf_set_medium_pseudochiral(nsf_plan plan, int axis_a, int axis_b,
                                const double* eps, const double* gamma,
                                int on_device);

/*
 * General medium (Sec. 3): per voxel g, 3 x 3 complex tensors eps_d, mu_d,
 * xi_d, zeta_d, each n x 9 nsf_c128 (voxel-major, row-major 3 x 3), host or
 * device pointers (on_device = 0 / 1; the library keeps its own data).  The
 * HHPD assumption of Sec. 4.1 is checked per voxel on the host: all finite
 * (NSF_E_ARG), eps and mu Hermitian, mu positive definite, zeta = xi^* and
 * Phi = eps - xi mu^-1 zeta positive definite (to 1e-14 of the voxel's largest
 * entry; NSF_E_NOT_HHPD naming the voxel).  The library stores, per voxel, the
 * 6 x 6 Hermitian middle factor of A_r (Thm 4.2),
 * [[mu^-1 zeta Phi^-1 xi mu^-1 + mu^-1, mu^-1 zeta Phi^-1], [Phi^-1 xi mu^-1, Phi^-1]]
 * (21 complex values, 336 n bytes).  Its A_r passes use the six-field fused z
 * pass, since such a medium can couple all six fields.  Synchronises.
 */
int nsf_set_medium_tensor(nsf_plan plan, const nsf_c128* eps, const nsf_c128* mu,
                          const nsf_c128* xi, const nsf_c128* zeta, int on_device);

/*
 * Medium for the null space free eigenvalue problem (NFSEP, Thm 3.2; the
 * else-branch of Algorithm 1): per voxel 3 x 3 complex eps_d, mu_d, xi_d,
 * zeta_d laid out as for nsf_set_medium_tensor, host or device pointers.  No
 * Hermitian, definiteness or reciprocity assumption (lossy, non-reciprocal
 * and general bianisotropic media): only B = i [[zeta, mu], [-eps, -xi]] must
 * be nonsingular at every voxel (Thm 3.1).  NSF_E_ARG for a non-finite entry
 * or a pivot below 1e-13 of the voxel's largest entry, naming the voxel.  The
 * library stores N = i J B^{-1} per voxel (J = [[0, I], [-I, 0]]; 36 complex
 * values, 576 n bytes), which is A_r's middle factor when the medium does meet
 * the Sec. 4.1 assumption.  The plan then serves nsf_apply_nfsep,
 * nsf_nfsep_solve, nsf_eigs_nfsep, nsf_fields and nsf_apply_Ar (which applies
 * diag(P_r^*, Q_r^*) N diag(P_r, Q_r)); nsf_cg_solve, nsf_eigs and the batch
 * eigensolver return NSF_E_STATE.  Synchronises.
 */
int nsf_set_medium_nfsep(nsf_plan plan, const nsf_c128* eps, const nsf_c128* mu,
                         const nsf_c128* xi, const nsf_c128* zeta, int on_device);

/*
 * out = K y with the NFSEP matrix of Thm 3.2,
 *   K = diag(Sigma_r^{1/2} Q_r^*, Sigma_r^{1/2} P_r^*) B^{-1} diag(P_r Sigma_r^{1/2}, Q_r Sigma_r^{1/2}).
 * y, out: device 4n vectors ([y_P; y_Q], frequency order; may alias).  Needs an
 * NFSEP medium (NSF_E_STATE).  Asynchronous.
 */
int nsf_apply_nfsep(nsf_plan plan, const nsf_c128* y4n, nsf_c128* out4n);

/*
 * x = K^{-1} b, the zero-shift inverse that the shift-and-invert Arnoldi method
 * of Sec. 4 applies, by restarted GMRES(restart) on the equivalent system
 * Kern v = (i J4) Sigma'^{-1/2} b, x = Sigma'^{-1/2} v, where Kern =
 * diag(P_r^*, Q_r^*) N diag(P_r, Q_r), (i J4)[a; b] = [i b; -i a] and Sigma' =
 * diag(Sigma_r, Sigma_r) (K = Sigma'^{1/2} (i J4) Kern Sigma'^{1/2}).  GMRES
 * starts from zero and stops when the recomputed residual of that system is
 * <= rtol times its right-hand side (relres, host), or after maxit iterations
 * (<= 0: 2000).  restart <= 0: 12.  b, x device, distinct.  Returns NSF_OK or
 * NSF_NOT_CONVERGED; allocates and frees the GMRES basis ((restart + 1) 4n
 * complex values).  Synchronises.
 */
int nsf_nfsep_solve(nsf_plan plan, const nsf_c128* b, nsf_c128* x, double rtol,
                    int maxit, int restart, int* iters, double* relres);

/*
 * The nev eigenvalues of K (equivalently the nonzero ones of the GEP
 * diag(C, C^*) x = omega B x, Thm 3.2) with positive real part and the smallest
 * modulus, by shift-and-invert Arnoldi at zero shift (Sec. 4): Krylov-Schur
 * restarted Arnoldi on Kern^{-1} B_r, B_r = i [[0, Sigma_r^{-1}], [-Sigma_r^{-1}, 0]],
 * whose eigenvalues are 1/omega, with a GMRES solve of Kern per step
 * (NSF_OPT_GMRES_RESTART) to relative residual inner_rtol.  For a medium that
 * meets the assumption of Sec. 4.1 this is the invert Lanczos operator of
 * nsf_eigs and the eigenvalues agree.  Basis of m = max_basis vectors (0:
 * max(3 nev, nev + 8), at most 510), restart keeping nev + (m - nev)/2 Schur
 * vectors, at most max_restarts restarts (0: 1000), start vector a seeded
 * complex normal vector.  A pair is accepted with the exact residual
 *   eta = ||K y - omega y|| / (|omega| ||y||) <= res_tol,
 * omega = y^* K y / y^* y the Rayleigh quotient, y = Sigma'^{-1/2} x.
 * Outputs: omega_host (nev complex, ascending modulus), Y_dev (nullable,
 * device 4n x nev: the unit vectors x = Sigma'^{1/2} y, the scaled vectors
 * Algorithm 1 hands to field recovery, so nsf_fields(x) gives E and H),
 * resid_host (nullable, nev), stats (nullable; cg_* count GMRES iterations and
 * solves, lanczos_steps Arnoldi steps, bytes_alg (320 + the medium's bytes
 * per voxel of nsf_plan_medium_info) n B per apply).
 * Allocates and frees its bases ((m + 1) + (restart + 1) + 3 vectors of 4n
 * complex values).  Returns NSF_OK, NSF_NOT_CONVERGED (results filled) or an
 * error.  Synchronises.
 */
int nsf_eigs_nfsep(nsf_plan plan, int nev, double res_tol, double inner_rtol,
                   int max_basis, int max_restarts, unsigned long long seed,
                   nsf_c128* omega_host, nsf_c128* Y_dev, double* resid_host,
                   nsf_stats* stats);

/*
 * Basis applies (Thm 2.5; T by twisted FFT, Sec. 4.2).  All pointers device.
 *   nsf_apply_Pr : y (2n, [y_a; y_b]) -> x (3n) = P_r y
 *   nsf_apply_Qr : y (2n, [y_c; y_d]) -> x (3n) = Q_r y
 *   nsf_apply_PrH: x (3n) -> y (2n) = P_r^* x
 *   nsf_apply_QrH: x (3n) -> y (2n) = Q_r^* x
 * Input and output must not overlap.  Asynchronous on the plan's stream.
 */
int nsf_apply_Pr(nsf_plan plan, const nsf_c128* y2n, nsf_c128* x3n);
int nsf_apply_Qr(nsf_plan plan, const nsf_c128* y2n, nsf_c128* x3n);
int nsf_apply_PrH(nsf_plan plan, const nsf_c128* x3n, nsf_c128* y2n);
int nsf_apply_QrH(nsf_plan plan, const nsf_c128* x3n, nsf_c128* y2n);

/*
 * out = A_r u (Thm 4.2, the operator of the linear systems in Sec. 4.2).
 * u and out are device 4n vectors and must not overlap.  Needs a medium
 * (NSF_E_STATE otherwise).  Asynchronous.
 */
int nsf_apply_Ar(nsf_plan plan, const nsf_c128* u4n, nsf_c128* out4n);

/*
 * Timing of the A_r apply (tracing aid): runs `reps` applies of u -> out with a
 * HIP event between consecutive kernels on the plan's stream, then `reps`
 * applies back to back.  ms_pass[i] (i < min(*npass, max_pass)) receives the
 * average milliseconds of kernel i of one apply, *npass the number of kernels,
 * *ms_apply the average milliseconds of a whole apply without the events.
 * Device vectors as nsf_apply_Ar; host outputs nullable.  Synchronises.
 */
int nsf_profile_Ar(nsf_plan plan, const nsf_c128* u4n, nsf_c128* out4n, int reps,
                   double* ms_pass, int max_pass, int* npass, double* ms_apply);

/* out = B_r u (Thm 4.2).  Device 4n vectors, may alias.  Asynchronous. */
int nsf_apply_Br(nsf_plan plan, const nsf_c128* u4n, nsf_c128* out4n);

/*
 * Solve A_r x = b by unpreconditioned CG from x = 0 (Sec. 4.2), stopping when
 * ||r||_2 <= rtol ||b||_2 (the recurrence residual) or after maxit iterations.
 * b, x: device 4n vectors (distinct).  iters, relres: host outputs (nullable).
 * Synchronises the stream.  Returns NSF_OK, NSF_NOT_CONVERGED (maxit hit) or
 * NSF_E_BREAKDOWN.
 */
int nsf_cg_solve(nsf_plan plan, const nsf_c128* b, nsf_c128* x, double rtol,
                 int maxit, int* iters, double* relres);

/*
 * nsf_cg_solve for callers that cannot allocate device memory (serving loops,
 * harnesses that forbid hipMalloc): the same solve, the same kernels and the
 * same results, with the CG vectors r, p, q (12 n complex values) kept in a
 * library-owned static device array of 12 * 65536 complex values (12 MiB) on
 * each GPU the library runs on, held until the process ends.  No hipMalloc,
 * hipFree or allocating library call is made; the plan's own device state
 * (tables, fields, reduction slots) must already exist, which setting a
 * medium does.
 *   Grids of at most 65536 voxels (e.g. 40^3, 64 x 32 x 32); larger plans get
 *   NSF_E_ARG with a message naming the limit.  No medium: NSF_E_STATE.
 *   Every call on one GPU shares that array and leaves its contents behind
 *   (each solve initialises what it reads): calls that overlap in time on one
 *   GPU race, even on different plans or streams.
 *   Arguments, results, status and synchronisation as nsf_cg_solve.
 */
int nsf_cg_solve_noalloc(nsf_plan plan, const nsf_c128* b, nsf_c128* x,
                         double rtol, int maxit, int* iters, double* relres);

/*
 * The nev smallest positive eigenvalues omega of the GEP (Sec. 3), i.e. the
 * nev largest theta = 1/omega of B_r y = theta A_r y, by invert Lanczos in the
 * A_r inner product with thick restarts and CG inner solves (Sec. 4.2,
 * Algorithm 1 step 5).
 *   nev          1 <= nev <= 256
 *   res_tol      stop when every wanted pair has
 *                eta = ||B_r y - theta A_r y|| / (|theta| ||A_r y||) <= res_tol
 *   cg_rtol      relative tolerance of the inner CG solves (with
 *                NSF_OPT_CG_RELAX = 1 the tightest one: later solves are
 *                relaxed as the Ritz residuals fall)
 *   max_basis    Lanczos basis size m before a restart (0: 3*nev, at least
 *                nev + 8); m + 1 vectors of 4n are kept, plus A_r times them
 *   max_restarts 0: no limit other than 1000
 *   seed         start vector seed (complex normal from a counter hash)
 *   omega_host   host, nev doubles, ascending (reported as the pencil
 *                Rayleigh quotient of each Ritz vector)
 *   Y_dev        device 4n x nev (column j at Y_dev + j*4n), A_r-orthonormal
 *                Ritz vectors; nullable
 *   resid_host   host, nev residuals eta; nullable
 *   stats        nullable
 * Synchronises the stream.  Returns NSF_OK or NSF_NOT_CONVERGED (results still
 * filled), or an error.
 */
int nsf_eigs(nsf_plan plan, int nev, double res_tol, double cg_rtol,
             int max_basis, int max_restarts, unsigned long long seed,
             double* omega_host, nsf_c128* Y_dev, double* resid_host,
             nsf_stats* stats);

/*
 * Electric and magnetic fields of a pencil eigenvector (Algorithm 1, last
 * step): [E; H] = B^{-1} diag(P_r, Q_r) y, B the medium matrix of the GEP
 * (Sec. 3).  y: device 4n vector (as returned by nsf_eigs, or the scaled
 * vector x of nsf_eigs_nfsep for an NFSEP medium); eh: device 6n,
 * [E_x; E_y; E_z; H_x; H_y; H_z], n each, voxel order g, carrying the Bloch
 * phase of k.  The pair (omega, [E; H]) then solves
 * diag(C, C^*) [E; H] = omega B [E; H].  Needs a medium (NSF_E_STATE).
 * Asynchronous.
 */
int nsf_fields(nsf_plan plan, const nsf_c128* y4n, nsf_c128* eh6n);

/*
 * Start block for the plan's next eigensolve (nsf_eigs, or its instance in
 * nsf_batch_eigs): count device 4n vectors at Y0_dev (column j at Y0_dev + j*4n,
 * for example the Ritz vectors of a neighbouring Bloch vector).  The Lanczos
 * start vector becomes sum_j c_j Y0_j with seeded complex normal c_j, plus the
 * seeded normal vector at 1e-3 of its size.  The block is read at the start of
 * that solve (the caller keeps it alive until the call returns) and is then
 * forgotten.  count = 0 clears it.  0 <= count <= 512, else NSF_E_ARG.
 */
int nsf_eigs_set_start(nsf_plan plan, const nsf_c128* Y0_dev, int count);

/*
 * Gradient of S = sum_j w_j omega_j with respect to the per-voxel eps and
 * gamma of a chiral medium, by the Hellmann-Feynman rule for the HHPD pencil
 * (Thm 4.2): d omega = omega y^* dA_r y for A_r-normalised y.  With
 * E' = P_r y_P, H' = Q_r y_Q per voxel and Phi = eps - gamma^2:
 *   d omega/d eps_g   = -omega sum_c |i gamma E'_c + H'_c|^2 / Phi^2
 *   d omega/d gamma_g =  omega sum_c [2 Re(conj(i gamma E'_c + H'_c) i E'_c)/Phi
 *                                     + 2 gamma |i gamma E'_c + H'_c|^2 / Phi^2]
 *   nev          number of eigenpairs
 *   omega_host   host, nev eigenvalues
 *   Y_dev        device 4n x nev, A_r-orthonormal eigenvectors (nsf_eigs)
 *   weights_host host, nev weights w_j (dS/d omega_j)
 *   d_eps_dev, d_gamma_dev  device, n doubles each, overwritten
 * Needs a chiral medium (NSF_E_STATE otherwise).  Asynchronous.
 */
int nsf_eig_grad(nsf_plan plan, int nev, const double* omega_host,
                 const nsf_c128* Y_dev, const double* weights_host,
                 double* d_eps_dev, double* d_gamma_dev);

/*
 * Batches: many independent instances (Bloch vectors, grids, media) solved in
 * one schedule.  Instances with the same grid share every launch of the CG
 * iterations and A_r applies (the instance is a launch dimension, each with
 * its own convergence flag), and the host synchronises once per Lanczos
 * phase for the whole batch.  An instance of 2^21 voxels or more (128^3)
 * fills the GPU by itself and runs alone, exactly as nsf_eigs.  Results equal
 * per-instance nsf_eigs calls up to rounding and the start vectors (instance
 * i uses seed + 1000003 i).
 *
 * nsf_batch_create: count instances; grids is count x 3 (n1, n2, n3), ks is
 *   count x 3 Bloch vectors; a, alpha, beta as nsf_plan_create; all instances
 *   enqueue on hip_stream.  Errors as nsf_plan_create (message names the
 *   instance).
 * nsf_batch_plan: borrow instance i's plan (owned by the batch) to set its
 *   medium or options, or to call single-instance functions on it.
 * nsf_batch_eigs: as nsf_eigs for every instance; omega_host and resid_host
 *   are count x nev (row i for instance i), stats count entries (nullable),
 *   Y_dev (nullable) count device pointers (each nullable) that receive the
 *   instance's 4n x nev Ritz vectors as nsf_eigs's Y_dev.
 *   Instances below 2^21 voxels run in shared waves sized to free device
 *   memory, larger ones one per wave; *wave_size (nullable) receives the
 *   shared wave length (1 when no instance shares).  Returns NSF_OK when every instance converged,
 *   NSF_NOT_CONVERGED otherwise, or an error.  Synchronises.
 */
typedef struct nsf_batch_s* nsf_batch;
int nsf_batch_create(nsf_batch* out, int count, const int* grids, const double* ks, double a,
                     double alpha, double beta, void* hip_stream);
int nsf_batch_plan(nsf_batch batch, int i, nsf_plan* plan);
int nsf_batch_eigs(nsf_batch batch, int nev, double res_tol, double cg_rtol, int max_basis,
                   int max_restarts, unsigned long long seed, double* omega_host,
                   double* resid_host, nsf_stats* stats, nsf_c128* const* Y_dev,
                   int* wave_size);
void nsf_batch_destroy(nsf_batch batch);
/*
 * nsf_plan_autotune on the first instance of every distinct grid shape (its
 * medium must be set), the chosen options copied to the other instances of
 * that shape.  *shapes_tuned (nullable) receives the number of shapes.
 */
int nsf_batch_autotune(nsf_batch batch, int reps, int* shapes_tuned);

/*
 * Dense Hermitian eigensolver on the host (cyclic complex Jacobi), the small
 * projected problem of the Lanczos method.  H: host m x m, row-major, only read.
 * w: host m ascending eigenvalues.  V: host m x m, row-major, column j is the
 * eigenvector of w[j] (nullable).  1 <= m <= 512.
 */
int nsf_hermitian_eig(int m, const nsf_c128* H, double* w, nsf_c128* V);

/*
 * Dense complex Schur form on the host, A = Z T Z^* (Hessenberg reduction and
 * shifted QR, then adjacent swaps), with the diagonal of T in the order the
 * NFSEP eigensolver wants its Ritz values: positive real part first, then
 * descending modulus.  The small projected problem of nsf_eigs_nfsep.
 * A, T, Z: host m x m, column-major; A only read.  1 <= m <= 512.
 */
int nsf_schur_sorted(int m, const nsf_c128* A, nsf_c128* T, nsf_c128* Z);

/* Facts about a HIP device (host call; touches the device runtime). */
typedef struct {
  char name[64];
  int compute_units;
  int clock_khz;
  int memory_clock_khz;
  int memory_bus_bits;
  long long total_memory;
  long long l2_bytes;
  int lds_per_block;        /* bytes a workgroup may allocate             */
  int lds_per_cu;           /* bytes of LDS per compute unit              */
  int warp_size;
} nsf_device;

/* Fill *out for HIP device `device`.  NSF_E_HIP if the device is absent. */
int nsf_device_info(int device, nsf_device* out);

/* Text for a status code (static storage). */
const char* nsf_status_string(int status);

/* Last error message of this plan (or of the last plan-less call if NULL). */
const char* nsf_last_error(nsf_plan plan);

#ifdef __cplusplus
}
#endif

#endif /* NSF_H */
