/*
 * pp.h -- C ABI of libpp, the MI355X (gfx950) particle step of the Photon-Plasma
 * relativistic particle-in-cell method (Haugboelle, Frederiksen & Nordlund,
 * arXiv:1211.4575).
 *
 * One time step, in the paper's order (Sec. III, numbered list of the five updates;
 * the sort sits between the particle and field updates):
 *
 *     pp_gather_push_deposit(run);   steps 1-3: E^n,B^n,x^n,u^{n-1/2} -> x^{n+1},u^{n+1/2},J^{n+1}
 *     pp_sort_particles(run, -1);    particles re-ordered by cell
 *     pp_field_step(run);            steps 4-5: B^{n+1} (implicit), E^{n+1} (explicit)
 *     pp_diagnostics(run, ...);      optional, FP64 sums and residuals
 *
 * Conventions (all calls):
 *   - Periodic box of n[0] x n[1] x n[2] cells of size d[0..2].  Positions are in
 *     cell units.  Mesh arrays are FP64 device arrays, x fastest:
 *     idx = i + n0*(j + n1*k).  A vector field is three consecutive blocks of
 *     ncell = n0*n1*n2 values (x, y, z components).
 *   - Yee staggering (Sec. III): rho at (i,j,k); E_x and J_x at (i+1/2,j,k);
 *     B_x at (i,j+1/2,k+1/2); other components cyclic.  Element [i] of a
 *     staggered array holds the value at i+1/2 along its staggered axes.
 *   - Units: mu0 = 1/(eps0 c^2).  u is the proper velocity gamma*v.
 *   - Memory: every pointer passed in is a device pointer owned by the caller
 *     (in practice torch tensors).  The library keeps non-owning views and
 *     never frees caller memory; it owns only internal scratch allocated in
 *     pp_create and released in pp_destroy.
 *   - Streams: all work is enqueued asynchronously on the HIP stream given to
 *     pp_create; a call returns once its kernels are enqueued, except
 *     pp_diagnostics, which synchronises the stream before it returns.
 *   - Errors: calls return a pp_status; host-side validation happens before
 *     anything is enqueued, and a failing call enqueues nothing.  Device-side
 *     faults of the data (a particle moving a cell or more in a step, non-finite
 *     state, a particle outside the tile it was sorted into) set bits in a
 *     device flag word reported by pp_diagnostics; the offending particle is
 *     left unchanged and deposits nothing.  No call aborts, throws or exits.
 *   - Threads: one host thread per pp_run handle at a time.
 */
#ifndef PP_H
#define PP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pp_status;
enum {
    PP_OK = 0,
    PP_E_ARG = -1,       /* invalid argument or parameter                         */
    PP_E_CFL = -2,       /* c dt >= min cell size: a particle could cross a cell  */
    PP_E_NONFINITE = -3, /* non-finite parameter                                  */
    PP_E_NOCONV = -4,    /* field relaxation did not reach its tolerance          */
    PP_E_CAPACITY = -5,  /* too many species / size limits                        */
    PP_E_HIP = -6,       /* a HIP runtime call failed (see pp_last_hip_error)     */
    PP_E_STATE = -7      /* call order violated (e.g. push of unsorted particles) */
};

enum { PP_PREC_FP64 = 0, PP_PREC_FP32_SPLIT = 1 };
enum { PP_PUSH_VAY = 0, PP_PUSH_BORIS = 1 };
/* Current schemes: charge-conserving (Esirkepov form, Sec. III.C, with the high-order line
 * solve for field orders 4 and 6) or direct (eq. "jj2": q w v W at the staggered J nodes, at the
 * time-centred position; no line solve; does not satisfy eq. "cc1"). */
enum { PP_CURRENT_CC = 0, PP_CURRENT_DIRECT = 1 };
enum { PP_MAX_GAUSS_PASSES = 64 };
enum { PP_MAX_SPECIES = 8 };

/* device flag bits reported in pp_diag.flags */
enum { PP_FLAG_CFL = 1, PP_FLAG_NONFINITE = 2, PP_FLAG_OUT_OF_TILE = 4 };

/* diagnostics selection bits for pp_diagnostics */
enum {
    PP_DIAG_MOMENTS = 1,  /* kinetic energy and momentum per species            */
    PP_DIAG_FIELDS = 2,   /* field energies                                      */
    PP_DIAG_RHO = 4,      /* deposit rho^{n}; Gauss residual; CC residual        */
    PP_DIAG_DIVB = 8,     /* max |div B|                                         */
    PP_DIAG_RELAX = 16,   /* measured residual of the last B relaxation          */
    PP_DIAG_ALL = 31
};

/* Run parameters (Sec. II weight order, Sec. III.A pusher, Sec. III.B alpha and
 * difference order, Sec. III.C current scheme).  Host validation rejects:
 * shape_order not in {2,3} (TSC, PCS), field_order not in {2,4,6}, alpha outside
 * [1/2, 1), any n < 1, d <= 0, dt <= 0, c <= 0, eps0 <= 0, non-finite values, and
 * c*dt >= min(d) (PP_E_CFL: the fixed O+2 node current stencil needs every
 * displacement under one cell). */
typedef struct pp_params {
    int32_t n[3];          /* cells per dimension (1 allowed)                        */
    double d[3];           /* cell sizes                                              */
    double dt, c, eps0;    /* time step, speed of light, vacuum permittivity          */
    int32_t shape_order;   /* 2 = TSC, 3 = PCS (cubic)                                */
    int32_t field_order;   /* 2, 4 or 6 (staggered differences and current order)     */
    double alpha;          /* implicit de-centering, 1/2 <= alpha < 1                 */
    int32_t pusher;        /* PP_PUSH_VAY (default) or PP_PUSH_BORIS                  */
    int32_t precision;     /* PP_PREC_FP64 or PP_PREC_FP32_SPLIT                      */
    double relax_tol;      /* target relative residual of the B relaxation, e.g. 1e-14 */
    int32_t relax_max_iter;/* upper bound on relaxation sweeps                        */
    double rho_background; /* fixed neutralising charge density (0 if none)          */
    double rad_tau;        /* radiative cooling (Sec. "Radiative cooling", eqs. "prad",
                            * "udot"): mu0 q^2 / (6 pi m c) for unit charge and mass in
                            * the run's units, scaled by q^2/m per species; after the
                            * electromagnetic push each particle loses
                            * k (gamma0/u0^2)(|du/dt|^2 + |du/dt x u0|^2/c^2) u0 dt with
                            * u0 the mean of the old and new proper velocities and du/dt
                            * their difference over dt (explicit, no iteration).  0 (the
                            * default) turns it off; must be finite and >= 0.          */
    int32_t current_scheme;  /* PP_CURRENT_CC (default) or PP_CURRENT_DIRECT              */
    int32_t gauss_filter_passes; /* 0..PP_MAX_GAUSS_PASSES passes of the Gauss-law filter
                            * at the end of pp_field_step (Sec. "Charge conservation":
                            * the paper corrects E after a non-conserving current): each
                            * pass computes r = div- E - (rho + rho_bg)/eps0 with rho of
                            * the current positions and adds kappa d+ r to E, kappa =
                            * 1 / max |K|^2 over the grid's wave numbers (K the symbol of
                            * the field-order first derivative).  Runs with passes > 0 are
                            * not accepted by pp_batch_add.                           */
    int32_t time_order;    /* 2 (leapfrog, default) or 4: pp_step composes three
                            * leapfrog substeps (Sec. III.A, symmetric fourth-order
                            * integrator; the Forest-Ruth position form with theta =
                            * 1/(2 - 2^(1/3)): (kick, drift) = (theta, (1-theta)/2),
                            * (1-2 theta, (1-theta)/2), (theta, theta) times dt, fields
                            * advanced with the drifts).  The state's positions and fields
                            * are then a drift of theta dt/2 ahead of the momenta (load
                            * x + theta dt/2 v for synchronised x, u).  Order 4 needs
                            * theta c dt < min(d) and is not accepted by pp_batch_add.   */
    int32_t gauss_filter_every; /* cadence of the Gauss-law filter passes: 0 or 1 = after
                            * every field step; k > 1 = only after the field step that
                            * completes a step whose number (pp_diag.step) is a multiple
                            * of k (Sec. "Charge conservation": in single precision the
                            * paper filters about every fifth step).  0..2^20; values
                            * above 1 need time_order 2.                                */
} pp_params;

/* Caller-owned FP64 mesh (device pointers, 3*ncell doubles each). */
typedef struct pp_mesh {
    double* E;
    double* B;
    double* J;
} pp_mesh;

/* Caller-owned particle storage of one species, structure of arrays (device).
 *  PP_PREC_FP64:       pos[d] -> double X_d in cell units, [0, n_d);  cell unused.
 *  PP_PREC_FP32_SPLIT: cell   -> int32 linear index i + n0*(j + n1*k) of the particle's
 *                                 cell, pos[d] -> float offset X_d - i in [lo, lo + 2):
 *                      lo = -1/2 for shape_order 2, 0 for shape_order 3.  A loader
 *                      gives i = floor(X - lo) mod n0 (offset in [lo, lo + 1): the
 *                      nearest node for quadratic, the node below for cubic weights).
 *                      The push keeps a particle whose last displacement, repeated (times
 *                      the ratio of the next drift to this one in a composed step), would
 *                      cross the lower face of its cell in the cell below (offset in
 *                      [lo + 1, lo + 2)), so that the stencils of the next step line up.
 *  u[d]: proper velocity (double for FP64, float for FP32_SPLIT).
 *  id:   optional int64 tag per particle carried along by the sort (NULL = none).
 *  *_alt: a second buffer of the same types and length (the sort writes there and
 *         the two buffers swap roles; pp_get_particles returns the current one). */
typedef struct pp_particles {
    int64_t n;
    int32_t* cell;
    void* pos[3];
    void* u[3];
    int64_t* id;
    int32_t* cell_alt;
    void* pos_alt[3];
    void* u_alt[3];
    int64_t* id_alt;
} pp_particles;

typedef struct pp_diag {
    double kinetic[PP_MAX_SPECIES];     /* sum w V m c^2 (gamma - 1), u at n+1/2     */
    double momentum[PP_MAX_SPECIES][3]; /* sum w V m u                              */
    double field_E, field_B, field_Ex;  /* sum eps0 E^2 V/2, B^2 V/(2 mu0), x part   */
    double gauss_max;  /* max |div E - (rho + rho_bg)/eps0|, field-order divergence   */
    double cc_max;     /* max |rho^{n} - rho^{n-1} + dt div J^{n}| (NaN if no rho^{n-1}) */
    double rho_ref;    /* max_s |q_s| n_s (mean number density): normalisation       */
    double divB_max;   /* max |div B| (up-shifted divergence)                         */
    double relax_resid;/* a-priori bound of the residual reduction of the last B
                        * relaxation (Chebyshev error bound times the condition number)  */
    int32_t relax_iters;
    int32_t flags;     /* PP_FLAG_* bits accumulated since the last pp_diagnostics    */
    int64_t step;      /* number of completed pp_gather_push_deposit calls          */
    double relax_resid_meas; /* PP_DIAG_RELAX: max |rhs - A B| / max |rhs| of the last
                        * field step's relaxation (Sec. III.B, eq. "EllipticB": A = 1 -
                        * alpha^2 c^2 dt^2 lap, rhs its right-hand side, B the field after
                        * the step), computed on the device from the stored right-hand side
                        * and the current B; NaN when not requested, before the first field
                        * step, or after Gauss-law filter passes (they reuse its storage) */
} pp_diag;

typedef struct pp_run pp_run;

/* Device memory a run with these parameters allocates inside the library (its
 * scratch: relaxation buffers, the fixed-point current, sort buckets and
 * scratch, per-species offsets), for nspecies species of at most
 * max_particles particles each; the caller-owned mesh and particle arrays are
 * not included.  For admission by memory footprint (several runs sharing one
 * GPU).  Validates params like pp_create; no device call. */
pp_status pp_workspace_size(const pp_params* params, int64_t max_particles, int32_t nspecies, size_t* bytes);

/* Create a run: validates params, records the mesh views and the stream
 * (a hipStream_t; NULL = default stream) and allocates internal scratch of
 * O(ncell) doubles.  *out receives the handle. */
pp_status pp_create(const pp_params* params, const pp_mesh* mesh, void* hip_stream, pp_run** out);

/* Register species s (0 <= s < PP_MAX_SPECIES) with charge q, mass m and weight w
 * (number density contributed per macro-particle, so rho = sum q w W, eq. "rho2")
 * and its particle storage (Sec. II macro-particles).  Host-side checks: m > 0,
 * w >= 0, finite q, non-null arrays for the run's precision.  For
 * PP_PREC_FP32_SPLIT the particles are sorted by cell immediately (enqueued). */
pp_status pp_init_species(pp_run* run, int32_t s, double q, double m, double w, const pp_particles* parts);

/* Steps 1-3 of Sec. III for every registered species: gather E^n and B^n to each
 * particle with the B-spline weights of the run's order (eq. "pfields"), push
 * u^{n-1/2} -> u^{n+1/2} (Vay or Boris, Sec. III.A), move x^{n+1} = x^n +
 * dt u/gamma, and deposit the charge-conserving current (Sec. III.C: Esirkepov's
 * split with per-particle prefix sums, then for field order 4/6 the line solve of
 * eqs. "jj6d"/"penta").  J is overwritten with J^{n+1}.  FP32_SPLIT requires the
 * particles to be sorted since their last push (PP_E_STATE otherwise). */
pp_status pp_gather_push_deposit(pp_run* run);

/* Steps 4-5 of Sec. III: B^{n+1} from the elliptic equation "EllipticB" (with
 * the J term's sign derived from "bnplus1"/"enplus1") by Jacobi relaxation from
 * B^n, then E^{n+1} from "enplus1".  E and B are updated in place.  The number of
 * sweeps is the smallest whose bound on the residual reduction (Chebyshev error
 * bound times the condition number of the operator) reaches relax_tol, at most
 * relax_max_iter; when the cap is reached first the step is still completed with
 * relax_max_iter sweeps and PP_E_NOCONV is returned (pp_diag.relax_resid gives the
 * bound reached; PP_DIAG_RELAX measures the residual itself). */
pp_status pp_field_step(pp_run* run);

/* Counting sort of species s (-1 = all) by tile-major cell key (Sec. III: the
 * particle arrays are sorted by cell between steps 3 and 4).  The order inside a
 * cell is unspecified.  The current and alternate buffers swap roles.  FP32_SPLIT:
 * after a push the sort computes the new order only; the particles are moved into it
 * by the next pp_gather_push_deposit (together with their update) or by
 * pp_get_particles, whichever comes first. */
pp_status pp_sort_particles(pp_run* run, int32_t s);

/* One whole time step in the run's time order (Sec. III step list): for time_order 2,
 * pp_gather_push_deposit, pp_sort_particles(run, -1) and pp_field_step; for time_order 4,
 * the three substeps of the composition (pp_params.time_order), each a particle update
 * with its own kick and drift, a sort and a field step over its drift.  The three calls
 * above, used one by one, always take one leapfrog step of dt.  After a composed step
 * the continuity residual of pp_diagnostics is not defined (NaN): J is that of the last
 * substep.  Errors as the three calls (PP_E_NOCONV once the whole step is done). */
pp_status pp_step(pp_run* run);

/* FP64 diagnostics selected by `what` (PP_DIAG_* bits) written to *out (host
 * memory).  Also reports and clears the device flag word.  Synchronises the
 * run's stream. */
pp_status pp_diagnostics(pp_run* run, uint32_t what, pp_diag* out);

/* Current buffer assignment of species s after sorts (host struct), with the particles
 * in sorted order: a new order left pending by pp_sort_particles is applied first
 * (enqueued on the run's stream). */
pp_status pp_get_particles(pp_run* run, int32_t s, pp_particles* out);

/* Time of the gather/push/deposit kernels: when enabled, HIP events bracket every
 * launch of the main particle kernel on the run's stream; pp_timing_read returns
 * the accumulated milliseconds and the number of launches timed, then resets. */
pp_status pp_timing_enable(pp_run* run, int32_t enable);
pp_status pp_timing_read(pp_run* run, double* ms_total, int64_t* launches);

/* Release internal scratch.  Caller memory is untouched. */
pp_status pp_destroy(pp_run* run);

/* ---- continuous batching of many runs ------------------------------------------------
 * A batch steps a changing set of runs together: every phase of a time step (the particle
 * kernel, the line solve, the sort of each species slot, the field step) is one launch over
 * all member runs.  Runs are created, loaded and destroyed with the calls above and join or
 * leave the batch between steps; their memory stays theirs.  Members must use
 * PP_PREC_FP32_SPLIT, grids with at least 4 cells per axis (4x4x4 tiles), the batch's
 * stream and one common shape order.  A member's results equal those of stepping it alone
 * (the current is an exact integer sum; every other reduction has a fixed order).
 * Calls that overlap on one batch race; one host thread per batch. */
typedef struct pp_batch pp_batch;

/* Create an empty batch for at most max_runs members on a HIP stream.  Also allocates two
 * pinned host staging buffers of PP_BATCH_NOALLOC_TABLE_BYTES and, the first time on a GPU,
 * looks up the device address of that GPU's static table array (pp_batch_step_noalloc). */
pp_status pp_batch_create(int32_t max_runs, void* hip_stream, pp_batch** out);

/* Add a run (PP_E_ARG if it cannot be batched, PP_E_CAPACITY if full, PP_E_STATE if it is
 * already a member or has unsorted species). */
pp_status pp_batch_add(pp_batch* batch, pp_run* run);

/* Remove a run (PP_E_STATE if it is not a member).  The run itself stays valid. */
pp_status pp_batch_remove(pp_batch* batch, pp_run* run);

/* Number of member runs. */
pp_status pp_batch_size(const pp_batch* batch, int32_t* n);

/* One whole time step of every member (Sec. III order: particles, sort, fields), enqueued
 * on the batch's stream.  Each member's step counter advances by one.  PP_E_NOCONV (the
 * step done) when a member's relaxation is capped by its relax_max_iter. */
pp_status pp_batch_step(pp_batch* batch);

/* Release the batch's own buffers (members are untouched). */
pp_status pp_batch_destroy(pp_batch* batch);

/* ---- the batch step without allocation ------------------------------------------------
 * For callers that cannot allocate memory inside their stepping loop (tight serving loops,
 * harnesses that forbid hipMalloc while they run): the same step as pp_batch_step (same
 * kernels, bitwise the same results), but the step's descriptor tables (per member: kernel
 * arguments, block prefixes, sort and field descriptors) go to a fixed array of
 * PP_BATCH_NOALLOC_TABLE_BYTES in device memory instead of the batch's own growable buffer,
 * staged through the pinned host buffers that pp_batch_create allocates.  The call itself
 * allocates nothing, on the device or the host.
 *  - The array is static: each GPU the library runs on holds one copy, from the first
 *    pp_batch_create on it until the process ends.  It is shared by every batch on that GPU
 *    and keeps the last call's tables; every call writes the whole part it reads, so nothing
 *    has to start at zero.  Calls that overlap on one GPU (batches stepped from two threads,
 *    or on two streams whose work overlaps) race on it and must be serialised by the caller.
 *  - PP_E_CAPACITY, with nothing enqueued and a message in pp_last_hip_error, when the
 *    members' tables need more than PP_BATCH_NOALLOC_TABLE_BYTES (about 5 KiB per member run
 *    with two species); PP_E_STATE if the batch's GPU has no static array; otherwise the
 *    statuses of pp_batch_step.
 *  - The batch must be stepped on the GPU that was current at pp_batch_create. */
enum { PP_BATCH_NOALLOC_TABLE_BYTES = 2 * 1024 * 1024 };
pp_status pp_batch_step_noalloc(pp_batch* batch);

/* Static description of a status code. */
const char* pp_status_str(pp_status st);

/* Last HIP error string recorded by the library in this process ("" if none). */
const char* pp_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PP_H */
