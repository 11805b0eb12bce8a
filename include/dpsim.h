/*
 * dpsim.h -- C ABI of the MI355X dual-porosity oil-water simulator hot path.
 *
 * The library computes, on one gfx950 GPU, the fully implicit backward-Euler /
 * two-point-flux discretisation of the dual-porosity two-phase system (paper
 * Sec. 2, Eqs. (3)-(5); Sec. 3, first paragraph), its inexact Newton iteration
 * (Algorithm 1), and the linear solve of every Newton step: the decoupled
 * system D^-1 A x = D^-1 b (Eq. (14)) by GMRES with the CPR-FPF preconditioner
 * (Sec. 3.2): block ILU(0) smoothing of the full system, an algebraic
 * multigrid V-cycle on the pressure system, block ILU(0) smoothing again.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns dp_status: DP_OK (0) or a negative error code.  No
 *   C++ exception crosses this boundary.  After an error, sim_last_error()
 *   returns a message; the handle stays usable unless DP_E_DEVICE is returned.
 * - Node order ("canonical order") of all host arrays: cell c = i + nx*(j +
 *   ny*k); node 2c is the fracture node and node 2c+1 the matrix node of cell
 *   c; well w follows as block 2n+w.  A node carries (p_o [Pa], S_w); its two
 *   equations are the oil and the water mass balance [kg/s].  A well carries
 *   (p_b [Pa], dummy); its equations are the control equation and dummy = 0.
 * - Units are SI.  Permeabilities in m^2, porosities as fractions of the cell
 *   bulk volume, viscosities in Pa s, compressibilities in 1/Pa, rates in m^3/s
 *   at the reference water density.
 * - Memory: the caller owns every host array (the library copies what it needs
 *   during the call) and the device workspace (sim_footprint bytes, device
 *   pointer, 256-byte aligned, alive until sim_destroy).  The library makes no
 *   device allocation of its own.  All device work is enqueued on the caller's
 *   HIP stream; functions that return host values synchronise that stream.
 * - One handle must not be used from two threads at once.  Distinct handles on
 *   distinct streams may run concurrently.
 */
#ifndef DPSIM_H
#define DPSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dp_status;

enum {
    DP_OK = 0,
    DP_E_INVALID = -1, /* bad argument or descriptor */
    DP_E_NOMEM = -2,   /* workspace too small (message gives the bytes needed) */
    DP_E_DEVICE = -3,  /* a HIP call failed */
    DP_E_NOCONV = -4,  /* Newton or GMRES did not converge */
    DP_E_STATE = -5,   /* call out of order (e.g. solve before setup) */
    DP_E_NUMERIC = -6  /* NaN / Inf or a zero pivot */
};

enum { DP_WELL_INJ = 0, DP_WELL_PROD = 1 };   /* water injector | producer */
enum { DP_CTRL_RATE = 0, DP_CTRL_BHP = 1, DP_CTRL_ORATE = 2 };   /* control equation of a well */
enum { DP_FP64 = 0, DP_FP32 = 1 };            /* preconditioner precision */
/* Decoupling D^-1 of Eq. (14), per node row (Sec. 3.2): DP_DEC_GJ one
 * Gauss-Jordan step on the diagonal block (row0 -= a01/a11 row1; for 2x2 blocks
 * this is also the Quasi-IMPES operator); DP_DEC_ABF alternate block
 * factorisation, the inverse of the diagonal block; DP_DEC_TI true-IMPES
 * (row0 -= c01/c11 row1, c_i the sum of block column i, where the fluxes
 * cancel).  Well rows are not changed. */
enum { DP_DEC_GJ = 0, DP_DEC_ABF = 1, DP_DEC_TI = 2 };
/* CPR composition with F = block ILU(0), P = pressure stage: FPF z1 = F^-1 r,
 * z2 = z1 + R^T Mp^-1 R (r - A z1), z = z2 + F^-1 (r - A z2); FP (two-stage,
 * pressure first) z1 = R^T Mp^-1 R r, z = z1 + F^-1 (r - A z1). */
enum { DP_CPR_FPF = 0, DP_CPR_FP = 1 };

typedef struct dp_sim dp_sim;

/* A vertical well perforating the fracture nodes of cells (i, j, k0..k1).
 * Eq. (6): perforation rate q = rho W lambda (p_b - p); Eq. (7): well rate is
 * the sum over perforations; Eq. (8) with Eq. (10): W = 2 pi sqrt(kx ky) dz /
 * (ln(r_e/r_w) + skin), r_e Peaceman's, unless wi > 0 gives W directly (the
 * examples of Sec. 4 state an injector's index).  Mobility is taken upstream: an
 * injector's perforation with p_b >= p injects water only, with the block's
 * total mobility; a perforation in back-flow produces each phase with the
 * block's phase mobility.  Rate control (injectors) fixes the well's net mass
 * rate (both phases) at rho_w_ref * target; oil-rate control (producers) fixes
 * the produced oil mass rate at rho_o_ref * target.  A rate-controlled injector
 * whose converged p_b exceeds bhp_limit (its maximum), or an oil-rate producer
 * whose converged p_b falls below bhp_limit (its minimum), switches to BHP
 * control at bhp_limit (once per step). */
typedef struct {
    int32_t i, j, k0, k1;
    int32_t kind;     /* DP_WELL_INJ | DP_WELL_PROD */
    int32_t control;  /* DP_CTRL_RATE (injectors) | DP_CTRL_ORATE (producers) | DP_CTRL_BHP */
    double target;    /* rate: m^3/s at rho_w_ref; oil rate: m^3/s at rho_o_ref, > 0
                         for production; BHP: Pa */
    double bhp_limit; /* Pa: an injector's maximum, a producer's minimum */
    double rw, skin;  /* m, - */
    double wi;        /* well index W, m^3, used for every perforation when > 0;
                         0 computes Peaceman's */
} dp_well;

typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz;        /* m */
    double top_depth;         /* depth of the top layer's cell centres, m (z down) */
    double gravity;           /* m/s^2 */
    const double *kx, *ky, *kz; /* [n] fracture permeability, m^2 */
    const double *km;         /* [n] matrix permeability, m^2 */
    const double *phi_f, *phi_m; /* [n] */
    double sigma;             /* shape factor, 1/m^2: omega = sigma km V */
    double rho_w_ref, rho_o_ref, p_ref, c_w, c_o; /* rho = rho_ref exp(c (p - p_ref)) */
    double c_r;               /* rock compressibility, 1/Pa: the pore volume of a node is
                                 V phi (1 + c_r (p - p_ref)) (Sec. 4 examples); 0 for none */
    double mu_w, mu_o;        /* Pa s */
    double swc, sor, n_w, n_o, krw_max, kro_max; /* Corey curves */
    int32_t nwells;
    const dp_well *wells;     /* [nwells]; at most one perforation per cell */
    /* solver options (0 selects the default given in brackets) */
    int32_t precond_precision; /* DP_FP64 | DP_FP32 [DP_FP64] */
    int32_t gmres_restart;    /* [30], at most 30 */
    int32_t lin_maxit;        /* [300] */
    double lin_rtol;          /* GMRES relative tolerance in newton_step/timestep [1e-6] */
    int32_t amg_coarse_max;   /* [2000], at most 4096 */
    int32_t amg_max_levels;   /* [25] */
    double amg_theta;         /* [0.25] */
    int32_t amg_trunc;        /* interpolation entries kept per row [3], at most 8 */
    double newton_tol;        /* CNV: max over rows of |R| dt/(rho_ref phi V) (well rows scaled by
                                 their target) [1e-3] */
    int32_t max_newton;       /* [20] */
    int32_t max_cuts;         /* [8] */
    double mb_tol;            /* MB: per phase |sum_nodes R| dt / sum_nodes(rho_ref phi V) [1e-7];
                                 Newton has converged when CNV <= newton_tol and MB <= mb_tol */
    /* Linear tolerance eta_l of timestep's Newton iterations (Algorithm 1, Eq. (12)):
     * forcing 0 keeps lin_rtol; 1, 2, 3 select the adaptive choices of Eq. (13):
     * eta_l = ||b_l - r_{l-1}|| / ||b_{l-1}||, | ||b_l|| - ||r_{l-1}|| | / ||b_{l-1}||, or
     * gamma (||b_l|| / ||b_{l-1}||)^beta, with b = -R and r_{l-1} = b_{l-1} - J_{l-1} y_{l-1}
     * (2-norms of the undecoupled system); the first iteration uses forcing_eta0;
     * safeguards: choices 1-2 max(eta, eta_{l-1}^phi) if eta_{l-1}^phi > 0.1 (phi the
     * golden ratio), choice 3 max(eta, gamma eta_{l-1}^beta) if that exceeds 0.1; then
     * eta is clamped to [forcing_eta_min, forcing_eta_max]. */
    int32_t forcing;          /* [0] */
    double forcing_eta0;      /* [0.1] */
    double forcing_gamma;     /* [0.9] */
    double forcing_beta;      /* [2], in (1, 2] */
    double forcing_eta_min;   /* [1e-8] */
    double forcing_eta_max;   /* [0.9] */
    int32_t precond_eager;    /* preconditioner apply: 1 launches its kernels one by one; 2 captures
                                 them into a HIP graph after each setup and replays it on every
                                 apply; 0 (auto) replays below 1M unknowns, where launches
                                 dominate, and launches one by one above (the phase timers always
                                 use the one-by-one path) [0] */
    int32_t decoupling;       /* DP_DEC_GJ | DP_DEC_ABF | DP_DEC_TI [DP_DEC_GJ] */
    int32_t cpr_variant;      /* DP_CPR_FPF | DP_CPR_FP [DP_CPR_FPF] */
    int32_t newton_stall;     /* stagnation exit of a sub-step's Newton loop, when > 0: the
                                 sub-step fails (and is cut) once this many iterations in a row
                                 have not lowered the smallest CNV of its updated iterates
                                 (iterations 1, 2, ...; iteration 0 is the start state); 0 or
                                 less leaves max_newton as the only limit [off] */
    int32_t fail_setup;       /* test hook for the error paths: when > 0, the fail_setup-th AMG
                                 setup of the handle (counted from 1 over its lifetime) fails
                                 with DP_E_NOMEM right after its first level's launches are
                                 queued, as a workspace overflow in the middle of a setup
                                 would; 0 or less never [off] */
} dp_sim_desc;

typedef struct {
    int32_t converged;   /* 1 if the residual met both tolerances before the update */
    int32_t lin_iters;   /* GMRES iterations of this step */
    double res_scaled;   /* CNV of the residual at the start */
    double lin_rel_res;  /* final relative decoupled residual of GMRES */
    double mb_scaled;    /* MB of the residual at the start (larger of the two phases) */
} dp_newton_info;

typedef struct {
    double dt;           /* time advanced (the requested dt on success) */
    int32_t substeps;    /* accepted sub-steps */
    int32_t cuts;        /* timestep cuts */
    int32_t newton_iters;
    int32_t lin_iters;
    double mb_oil, mb_water; /* max over sub-steps of |M^{n+1}-M^n-dt Q|/M^{n+1} */
    double res_scaled;   /* final scaled residual */
} dp_step_info;

/* Device bytes that sim_create needs for this descriptor (an upper bound that
 * includes the AMG hierarchy and its setup scratch). */
dp_status sim_footprint(const dp_sim_desc *desc, size_t *device_bytes);

/* Create a handle.  p0, sw0: [2n] initial node states in canonical order
 * (host).  Rate and oil-rate wells start with p_b at the mean of p0; BHP wells at their
 * target.  d_workspace: device memory of at least sim_footprint bytes.
 * hip_stream: a hipStream_t (NULL = default stream). */
dp_status sim_create(const dp_sim_desc *desc, const double *p0, const double *sw0,
                     void *d_workspace, size_t workspace_bytes, void *hip_stream,
                     dp_sim **out);
dp_status sim_destroy(dp_sim *sim);
const char *sim_last_error(const dp_sim *sim);

/* Record the current state as the start of a timestep (old accumulation M^n).
 * timestep() does this itself; direct callers of newton_step or
 * assemble_residual_jacobian call it once per step. */
dp_status sim_mark_old(dp_sim *sim);

/* Residual R and Jacobian J at the current iterate for step length dt (Eq. (5)
 * discretised; Algorithm 1, "assemble b" and "compute A").  Writes the CNV of R
 * to *res_scaled if not NULL (synchronises). */
dp_status assemble_residual_jacobian(dp_sim *sim, double dt, double *res_scaled);

/* Decouple (Eq. (14), Gauss-Jordan reading), factor block ILU(0), extract the
 * pressure system and build its AMG hierarchy.  Requires a prior assembly. */
dp_status cpr_fpf_setup(dp_sim *sim);

/* GMRES(restart) on the decoupled system D^-1 J y = -D^-1 R with CPR-FPF (right
 * preconditioning) from y = 0, to ||b - A y|| <= rtol ||b|| (Sec. 3.2).  The
 * Arnoldi columns are those of classical Gram-Schmidt with one
 * re-orthogonalisation pass; the correction and normalisation of each new
 * basis vector are applied in the next iteration's first pass over the basis,
 * two passes per iteration.  One host synchronisation per iteration (the
 * Givens rotations run on the host).  The correction stays on the device for
 * newton_update.  Returns DP_E_NOCONV (keeping the best iterate) if maxit is
 * reached. */
dp_status krylov_solve(dp_sim *sim, double rtol, int32_t maxit, int32_t *iters,
                       double *rel_res);

/* x <- x + y with the saturation chop (|dS| <= 0.2), a stop at the
 * relative-permeability end point the change would cross from inside the
 * mobile range, and the clamp to [0,1]; BHP wells keep p_b at their target. */
dp_status newton_update(dp_sim *sim);

/* One inexact-Newton iteration of Algorithm 1 with forcing term eta: assemble,
 * and if not yet converged, setup + solve + update. */
dp_status newton_step(dp_sim *sim, double dt, double eta, dp_newton_info *info);

/* Advance the state by dt: Newton to convergence, halving the sub-step on
 * failure (at most max_cuts times in all) and doubling it again after each
 * accepted sub-step (never beyond what remains of dt), well-control switching,
 * material balance.  On
 * DP_E_NOCONV the state is rolled back to the start of the step. */
dp_status timestep(dp_sim *sim, double dt, dp_step_info *info);

/* Served form: advance every handle in sims[0..n) by its dt[i], overlapping
 * their work on the device (each handle on its own stream).  info[i] and the
 * per-handle status in status[i] (may be NULL). */
dp_status batch_timestep(dp_sim **sims, int32_t n, const double *dt,
                         dp_step_info *info, dp_status *status);

/* Host copies of the state in canonical order: p, sw [2n], bhp [nwells]. */
dp_status sim_get_state(dp_sim *sim, double *p, double *sw, double *bhp);
dp_status sim_set_state(dp_sim *sim, const double *p, const double *sw, const double *bhp);

/* ---- inspection (tests and diagnostics) -------------------------------- */

/* Sizes: n_dof = 4n + 2*nwells; nnz = point nonzeros of the block pattern. */
dp_status sim_system_size(const dp_sim *sim, int32_t *n_dof, int64_t *nnz);

/* Point CSR in canonical order of the current system.  which = 0: J and R as
 * assembled; which = 1: the decoupled matrix D^-1 J and D^-1 (-R) (after
 * cpr_fpf_setup).  rowptr [n_dof+1], colind/vals [nnz], rhs [n_dof]. */
dp_status sim_export_system(dp_sim *sim, int32_t which, int32_t *rowptr, int32_t *colind,
                            double *vals, double *rhs);

/* Block ILU(0) factors in canonical block indices.  perm [nb]: elimination
 * position -> canonical block.  For every pattern block (brow[e], bcol[e]):
 * vals[4e..4e+3] row-major = L block (strictly lower in the elimination
 * order), U block (strictly upper) or the inverse of U's diagonal block.  Sizes
 * [nnzb] with nnzb = nnz / 4. */
dp_status sim_export_ilu(dp_sim *sim, int32_t *perm, int32_t *brow, int32_t *bcol, double *vals);

/* AMG hierarchy sizes: levels, rows[l], nnz[l] (arrays of amg_max_levels). */
dp_status sim_amg_info(dp_sim *sim, int32_t *levels, int32_t *rows, int64_t *nnz);

/* Linear tolerances of the Newton iterations of the last timestep call, in
 * order, across its sub-steps and retries: five doubles per iteration, rec[5i..]
 * = (eta_l, ||b_l||, ||r_l||, ||b_l - r_{l-1}||, l) with the norms of the
 * forcing terms (zero when forcing = 0, where eta_l = lin_rtol) and l the
 * iteration's index within its Newton solve.  Copies at most cap records into
 * rec (host) and stores the full count. */
dp_status sim_eta_history(dp_sim *sim, double *rec, int32_t cap, int32_t *count);

/* Setup statistics since sim_create: the number of AMG sort-and-sum steps
 * (interpolation rows, R = P^T, A P and R (A P), per level and setup) that had
 * rows too long for the row-wise LDS tiles (more than 4096 terms).  Those rows
 * are sorted by the global radix sort, to the same result; the other rows stay
 * in the tiles. */
dp_status sim_amg_stats(dp_sim *sim, int64_t *global_sort_products);

/* Level l: splitting cf[rows[l]] (1 = C, -1 = F; not for the coarsest), the
 * operator A_l in CSR, and for l < levels-1 the interpolation P_l in CSR.
 * Level 0 is the pressure system with the matrix-node pressures eliminated
 * exactly: its rows are the fracture nodes in elimination order (even cells,
 * then odd cells, each by cell index), then the wells.  Pass NULL to skip an
 * output.  p_nnz returns nnz(P_l). */
dp_status sim_export_amg_level(dp_sim *sim, int32_t level, int32_t *cf, int32_t *a_rowptr,
                               int32_t *a_col, double *a_val, int32_t *p_rowptr, int32_t *p_col,
                               double *p_val, int64_t *p_nnz);

/* The correction y of the last krylov_solve (solution of J y = -R through the
 * decoupled system), host vector [n_dof] in canonical order.  Synchronises. */
dp_status sim_get_correction(dp_sim *sim, double *dx);

/* z = M^-1 r (CPR-FPF) and y = A x (decoupled matrix), host vectors in
 * canonical order [n_dof].  After cpr_fpf_setup. */
dp_status sim_apply_precond(dp_sim *sim, const double *r, double *z);
dp_status sim_apply_matrix(dp_sim *sim, const double *x, double *y);

/* One stage of the preconditioner on host vectors.  stage 0: z = (LU)^-1 r,
 * block ILU(0) [n_dof, canonical order].  stage 1: z = V-cycle(r) on the
 * level-0 pressure system [rows[0], the order of sim_export_amg_level]. */
dp_status sim_apply_stage(dp_sim *sim, int32_t stage, const double *r, double *z);

/* Self-test of the dense coarse-level inverse (blocked Gauss-Jordan with MFMA
 * updates): ainv = a^-1 for a row-major n x n host matrix, n <= 4096.  Uses
 * the caller's device workspace (at least 16 n'^2 + 65536 bytes, n' = n
 * rounded up to 32) and stream. */
dp_status dp_selftest_dense_inverse(const double *a, int32_t n, double *ainv, void *d_workspace,
                                    size_t workspace_bytes, void *hip_stream);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc or take a workspace from an allocator, such as tight serving loops
 * or harnesses that forbid it): dp_selftest_dense_inverse with its device
 * scratch (the padded matrix, the pivot blocks, a column panel and the pivot
 * flag) in a static device array of the library, 8.7 MB on every GPU it runs
 * on, held until the process ends, instead of a caller workspace.  Same
 * kernels and results.  n <= 1024; larger n returns DP_E_INVALID.  The array
 * keeps the previous call's contents; every call writes what it reads and
 * clears the flag first.  All calls of the process share one array per GPU and
 * are serialised by a lock inside the library (the call synchronises
 * hip_stream before it returns), so they never overlap; do not call it while
 * capturing a HIP graph (it synchronises). */
dp_status dp_selftest_dense_inverse_noalloc(const double *a, int32_t n, double *ainv,
                                            void *hip_stream);

/* Time one kernel group on the handle's stream with HIP events, reps launches
 * after one untimed launch; returns the average ms per launch and the
 * algorithmic bytes one launch must move (values and indices read once, vectors
 * read and written once).  kernel 0: FP64 block SpMV of the decoupled matrix;
 * 1: block ILU(0) solve (preconditioner precision); 2: AMG V-cycle; 3:
 * residual/Jacobian assembly; 4: whole CPR-FPF apply; 5: plain copy of one
 * vector of 2 nb doubles (the reference for HBM traffic counters).  After
 * cpr_fpf_setup. */
dp_status sim_bench_kernel(dp_sim *sim, int32_t kernel, int32_t reps, double *avg_ms,
                           double *bytes);

/* Live kernel timing inside the normal calls.  While a timer is on, every
 * launch of its kernel records a pair of HIP events on the handle's stream (up
 * to 2048 launches) and adds the launch's algorithmic bytes.  kernel: 0 FP64
 * block SpMV of the decoupled matrix in GMRES; 1 block ILU(0) solve (its four
 * kernels as one launch); 2 row-wise AMG products A P and R (A P) (wavefront
 * tiles and the two workgroup tiers as one launch); 3 AMG V-cycle of the
 * pressure stage (all its levels as one launch; not timed while the
 * preconditioner replays from its graph); 4 the two classical Gram-Schmidt
 * passes over the Krylov basis of one GMRES iteration, with their reductions
 * (as one launch).  on != 0 resets and
 * starts, 0 stops.  sim_kernel_time synchronises the stream and returns the
 * summed device time (ms), the number of timed launches and the summed bytes. */
dp_status sim_kernel_timer(dp_sim *sim, int32_t kernel, int32_t on);
dp_status sim_kernel_time(dp_sim *sim, int32_t kernel, double *ms_total, int64_t *launches,
                          double *bytes);

/* Average device time (ms) of the named phase over the calls since the last
 * reset: 0 assembly, 1 setup, 2 solve, 3 SpMV, 4 preconditioner apply.
 * Timed with HIP events on the handle's stream when timing is enabled. */
dp_status sim_enable_timing(dp_sim *sim, int32_t on);
dp_status sim_phase_time(dp_sim *sim, int32_t phase, double *ms_total, int64_t *count);

#ifdef __cplusplus
}
#endif
#endif /* DPSIM_H */
