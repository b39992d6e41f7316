/*
 * eu.h -- C-ABI of the MI355X (gfx950) adaptive finite-volume library for the
 * compressible Euler equations (ideal gas, Cartesian 2D/3D), after
 * Deiterding, Domingues, Gomes, Schneider, "Comparison of adaptive
 * multiresolution and adaptive mesh refinement applied to simulations of the
 * compressible Euler equations" (arXiv:1603.05211).
 *
 * Method (Sec. 2): cell averages Q of (rho, rho v, rho e) on nested Cartesian
 * levels, dQ/dt = -F(Q) with a second-order MUSCL reconstruction in primitive
 * variables, van Albada limiter, AUSM+ flux (Liou 1996) and the explicit
 * midpoint rule (RK2).  Adaptivity (Sec. 2.1, 2.2): cell-average
 * multiresolution analysis (projection = mean of children, third-order
 * quadratic prediction), hard thresholding of the density details, one level
 * of preventive refinement, a one-cell buffer, proper nesting, and block
 * patches generated with the efficiency rule eta_tol.
 *
 * Conventions
 *  - Every function returns an int status (EU_OK = 0); no exception and no
 *    exit() crosses this boundary.  The text of the last error of a context
 *    is available from eu_last_error().
 *  - Device memory is owned by the caller.  eu_query_sizes() reports the
 *    bytes of the two buffers the caller allocates (state, scratch); the
 *    library carves everything it needs out of them and never allocates or
 *    frees device memory itself.  The context owns only host metadata and
 *    the HIP graphs it creates.  The one exception is a static 4 MiB array
 *    per GPU, part of the library's loaded code, used only by
 *    eu_conserved_totals_static.
 *  - Pointers are device pointers unless the name ends in _host.  A _host
 *    output makes the call synchronise the context's stream.
 *  - All work is enqueued on the stream given in eu_config.stream (a
 *    hipStream_t; NULL = the legacy default stream).  A context is not
 *    thread-safe; one context per stream.
 *  - State layout (per level or instance): the d+2 conserved fields rho,
 *    m_1..m_d, E stored one after another, each a dense n^d array with x
 *    fastest; the element type is double (EU_FP64) or float (EU_FP32).
 */
#ifndef EU_H
#define EU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
enum {
    EU_OK = 0,
    EU_EINVAL = 1,    /* invalid argument or configuration                  */
    EU_ENOMEM = 2,    /* a caller buffer is too small                        */
    EU_EHIP = 3,      /* a HIP runtime call failed (text in eu_last_error)   */
    EU_ENONPHYS = 4,  /* rho <= 0, p <= 0 or NaN met; sticky until cleared   */
    EU_ESTATE = 5     /* call out of order (e.g. stepping before init)       */
};

enum { EU_FP64 = 0, EU_FP32 = 1 };               /* state / flux precision   */
enum { EU_BC_TRANSMISSIVE = 0, EU_BC_PERIODIC = 1 };
enum { EU_DT_GLOBAL = 0, EU_DT_LTS = 1 };        /* time stepping           */
enum { EU_RESTRICT = 0, EU_PROLONG = 1, EU_GHOST = 2 }; /* eu_project modes */
enum { EU_IC_QUADRANT = 0, EU_IC_ELLIPSOID = 1, EU_IC_RIEMANN1D = 2, EU_IC_UNIFORM = 3 };
enum { EU_SCHEME_MR = 0, EU_SCHEME_AMR = 1 };      /* finite-volume scheme     */
enum { EU_CRIT_MR = 0, EU_CRIT_GRADIENT = 1 };     /* refinement criterion     */
enum { EU_RK_MIDPOINT = 0, EU_RK_HEUN = 1 };       /* MR scheme time stepping  */
enum { EU_AUSM_MEAN = 0, EU_AUSM_CRITICAL = 1 };   /* AUSM+ sound speed        */
enum { EU_TILER_BLOCKS = 0, EU_TILER_BR = 1 };     /* patch generation        */
enum { EU_CFL_SUM = 0, EU_CFL_MAX = 1 };           /* CFL signal speed        */
enum { EU_STAGE_SCHEDULES = 10, EU_STRIP_SCHEDULE0 = 6 }; /* see eu_autotune  */

/* Problem size and method parameters (Sec. 2; Sec. 4 for the values used
 * there).  All fields are read by eu_query_sizes / eu_create. */
typedef struct {
    int dim;             /* 2 or 3                                            */
    int precision;       /* EU_FP64 | EU_FP32 (FP32 state and flux; the CFL
                            reduction, conserved totals and detail threshold
                            stay FP64)                                        */
    double gamma;        /* ratio of specific heats (1.4)                     */
    double lo, hi;       /* cubic domain [lo, hi]^d                           */
    int n0;              /* cells per side of level 0 (power of two)          */
    int levels;          /* number of levels L >= 1; level l has n0 2^l cells
                            per side; 1 = uniform grid                        */
    int bc;              /* EU_BC_TRANSMISSIVE (outflow) | EU_BC_PERIODIC      */
    double cfl;          /* CFL number of eu_cfl_dt                           */
    double t_end;        /* end time: the last step is clipped to reach it
                            (INFINITY: never clipped)                         */
    double eps;          /* MR threshold on density details (same on all
                            levels)                                           */
    double eta;          /* patch efficiency eta_tol (flagged / all cells)    */
    int patch_min;       /* smallest patch side (must be 8)                   */
    int patch_max;       /* largest patch side (8, 16, 32 or 64)              */
    int time_mode;       /* EU_DT_GLOBAL | EU_DT_LTS                          */
    int n_instances;     /* > 1: batch of independent uniform grids            */
    const int32_t *inst_side_host; /* per-instance cells per side (multiples
                            of 8), n_instances entries; NULL when 1 instance  */
    void *stream;        /* hipStream_t                                       */
    int scheme;          /* EU_SCHEME_MR (0): MUSCL, van Albada, AUSM+,
                            midpoint RK2 (the paper's MR runs); EU_SCHEME_AMR:
                            unsplit MUSCL-Hancock with Minmod in primitive
                            variables and AUSMDV (Wada and Liou 1997), the
                            paper's AMR runs (Sec. 2); one launch per step:
                            the Hancock tile kernel (hierarchies and uniform
                            grids; schedules 0-2: 128, 192, 256 threads per
                            tile in 2D, 0-1: 256, 512 in 3D), a face next to
                            a covered cell taking the mean of the finer
                            level's fluxes, or the Hancock strips (2D
                            schedules 6 and 7; uniform grids and batches); with EU_DT_LTS (AMRLT) one
                            Hancock step per level step in the recursive
                            cycle, flux correction from the recorded fluxes;
                            with a global step the state alternates
                            between the two state arrays (tracked by the
                            library)                                          */
    int criterion;       /* EU_CRIT_MR (0): MR details against eps with one
                            level of preventive refinement (Sec. 2.1);
                            EU_CRIT_GRADIENT: the AMR method's scaled-gradient
                            indicators (Sec. 2.2): a cell of a level, in a
                            patch of it, is flagged when |w(Q_{i+a}) -
                            w(Q_i)| > eps_w for a neighbour i+a, a in {0,1}^d,
                            w = rho (eps_w = eps) and w = p (eps_p);
                            hierarchies (levels >= 2) only                    */
    double eps_p;        /* EU_CRIT_GRADIENT: pressure threshold (<= 0: the
                            density alone)                                    */
    int eps_levels;      /* EU_CRIT_MR: 0 (the paper's runs) eps on every
                            level; 1 level-dependent thresholds eps_l =
                            2^(d (l + 2 - L)) eps for the details of level
                            l = 0 .. L-2 (eps on the finest details, halved
                            d times per coarser level, as in Harten's MR
                            analysis)                                         */
    int rk;              /* MR scheme: EU_RK_MIDPOINT (0, the paper's MR
                            scheme) Q* = Q - dt/2 F(Q), Q <- Q - dt F(Q*);
                            EU_RK_HEUN: Q* = Q - dt F(Q), Q <- (Q + Q*)/2 -
                            dt/2 F(Q*) (global time step; tile schedules)     */
    int ausm_speed;      /* MR scheme: AUSM+ interface sound speed,
                            EU_AUSM_MEAN (0) the mean of the two sound
                            speeds; EU_AUSM_CRITICAL Liou's min(c*_L^2 /
                            max(c*_L, u_L), c*_R^2 / max(c*_R, -u_R)), c*^2
                            = 2 (gamma-1)/(gamma+1) H (tile schedules)       */
    int tiler;           /* patch generation inside each patch_max block from
                            the flags of the next coarser level (Sec. 2.2):
                            EU_TILER_BLOCKS (0) aligned square blocks, split
                            in 2^d halves until the flagged fraction of a
                            block reaches eta (or the block is a smallest
                            patch); EU_TILER_BR Berger-Rigoutsos clustering
                            (Berger and Rigoutsos 1991) into rectangular
                            unions of 8^d blocks: shrink to the flagged
                            blocks, emit when the flagged fraction reaches
                            eta or one block is left, else cut at the zero of
                            the flag signature nearest the middle (longest
                            axis first), else at its strongest inflection,
                            else halve the longest axis; the lower part
                            first.  EU_TILER_BR needs (patch_max / 8)^d <= 64
                            (3D: patch_max <= 32)                           */
    int cfl_mode;        /* CFL signal speed of a cell: EU_CFL_SUM (0) the sum
                            over axes of |v_d| + c, the stable choice for the
                            unsplit schemes; EU_CFL_MAX the largest |v_d| + c
                            (for runs with paper-style step sizes)          */
    int regrid_every;    /* eu_advance rebuilds the hierarchy after step n
                            (counted from initialisation; level-0 steps with
                            local time stepping) when n is a multiple of
                            regrid_every; 0 or 1: after every step (the
                            paper's AMR runs, Sec. 4)                       */
} eu_config;

/* Initial data (Sec. 4.1 four-quadrant Riemann problem, Sec. 4.2 ellipsoid,
 * a 1D Riemann problem along one axis, or a uniform state).  Cell-centre
 * sampling on the finest level. */
typedef struct {
    int kind;                /* EU_IC_*                                       */
    double quad[4][4];       /* quadrants I..IV: rho, v1, v2, p               */
    double x0, y0;           /* quadrant split point                          */
    double ell[8];           /* a, b, c, cos th, sin th, cos ph, sin ph, r_c  */
    double ell_states[4];    /* rho_in, p_in, rho_out, p_out                  */
    double lr[6];            /* 1D Riemann: rho_L, u_L, p_L, rho_R, u_R, p_R  */
    int axis;                /* 1D Riemann: axis of the velocity / split      */
    double split;            /* 1D Riemann: split coordinate                  */
    double uniform[5];       /* uniform primitive state rho, v..., p          */
    const double *inst_quad_host; /* batch: n_instances x 16 quadrant states
                                 (rows I..IV of rho, v1, v2, p), or NULL to use
                                 quad for every instance                      */
} eu_problem;

typedef struct eu_ctx eu_ctx;

/* Bytes of the state buffer and the scratch buffer for a configuration.
 * Returns EU_EINVAL for an invalid configuration. */
int eu_query_sizes(const eu_config *cfg, size_t *state_bytes, size_t *scratch_bytes);

/* Create a context on caller buffers of at least the queried sizes (device
 * memory, 256-byte aligned).  *out receives the context.  The work lists of
 * a regrid are built in one launch, or in two for ranges of more than 1024
 * blocks; the environment variable EU_LIST_BUILD=2, read here, selects the
 * two-launch build for every hierarchy (same lists; for tests).  Where the
 * patch masks of a pmax block fit one word (2D with patch_max <= 32, 3D
 * with patch_max <= 16) and there are three levels or more, every level is
 * flagged in one launch, which also builds the lists when they take one
 * launch; EU_FLAG_BUILD=levels, read here, selects one flagging launch per
 * level instead (same flags and lists; for tests).  The waits between the
 * workgroups of these launches are bounded: a wait past its bound makes
 * the next synchronising call return EU_EHIP.  EU_WAIT_TEST=stale, read
 * here, makes the list build wait for an epoch no workgroup publishes, with
 * a short bound (a test of that path: the lists are then left incomplete,
 * every kernel ends, and the context is only fit to be destroyed). */
int eu_create(const eu_config *cfg, void *state_dev, size_t state_bytes,
              void *scratch_dev, size_t scratch_bytes, eu_ctx **out);

/* Destroy a context (host metadata and graphs only; caller buffers stay). */
int eu_destroy(eu_ctx *ctx);

/* Initial data (Sec. 4): write the finest level (every instance), project it
 * down through all levels, analyse every level, flag, close and tile (the
 * patches keep the projected data), fill ghost cells; t = 0. */
int eu_init_state(eu_ctx *ctx, const eu_problem *p);

/* Same as eu_init_state with arbitrary finest-level data of instance inst
 * given as FP64 host values in the state layout (converted to the state
 * precision).  For a batch, call once per instance. */
int eu_set_finest(eu_ctx *ctx, int inst, const double *q_host);

/* MR decomposition (Sec. 2.1): project every level onto the cells it covers
 * (finest first) and compute, in FP64, the detail norm
 * D = max over the 2^d children |rho - predicted rho| of every refined cell. */
int eu_mr_decompose(eu_ctx *ctx);

/* MR thresholding and new mesh (Sec. 2.1 refinement/coarsening, Sec. 2.2
 * Remesh): significant details (D >= eps) keep their children; their
 * children are refined one more level (preventive refinement); flags get a
 * one-cell buffer and the nesting closure, finest level first, and are tiled
 * into aligned patches with the efficiency rule.  Old cells keep their data;
 * new cells are predicted from the next coarser level; ghost cells are
 * filled.  eps >= 0 replaces the threshold of the configuration (the
 * details of the last eu_mr_decompose are taken against it, and later steps
 * keep it); eps < 0 keeps the current one; NaN is EU_EINVAL.  nflag_host
 * (nullable, levels entries) receives the number of flagged cells per level
 * (synchronises). */
int eu_mr_flag(eu_ctx *ctx, double eps, int64_t *nflag_host);

/* Inter-level transfer (Sec. 2.1 projection / prediction, Sec. 2.2 ghost
 * cells): EU_RESTRICT projects every covered cell (finest first);
 * EU_PROLONG predicts cells created by the last eu_mr_flag; EU_GHOST fills
 * every ghost cell by prediction from the next coarser level. */
int eu_project(eu_ctx *ctx, int mode);

/* CFL time step (FP64; the paper's runs use CFL about 0.4, Sec. 4.2):
 * dt = min over levels cfl dx_l / max over leaves of the signal speed
 * (cfl_mode: sum_d (|v_d| + c), or max_d (|v_d| + c)) (with
 * local time stepping the level-0 step min over levels of that times 2^l),
 * clipped to reach t_end and to t_remaining, per instance for a batch.
 * cfl > 0 replaces the configuration's CFL number for this call (else it is
 * used); t_remaining >= 0 clips this step (a step with t_remaining = 0 is
 * marked done), t_remaining < 0 or INFINITY does not.  NaN arguments are
 * EU_EINVAL.  The result stays on the device for eu_fv_step; dt_dev
 * (nullable, device memory, 1 double, or n_instances for a batch) receives
 * a copy on the stream, dt_host (nullable) receives it for instance 0
 * (synchronises).  Computing dt commits the step it sizes: the context time
 * advances to t + dt here (a step starting at t >= t_end is marked done and
 * every later kernel of that step does nothing).  Detects non-physical
 * leaves (EU_ENONPHYS at the next synchronising call). */
int eu_cfl_dt(eu_ctx *ctx, double cfl, double t_remaining, double *dt_dev, double *dt_host);

/* One explicit midpoint (RK2) step of every leaf (Sec. 2, dQ/dt = -F(Q)):
 * Q* = Q - dt/2 F(Q), Q <- Q - dt F(Q*), each stage followed by projection
 * onto covered cells and ghost fill; faces between a leaf and a covered cell
 * take the mean of the fine fluxes.  dt_dev NULL: the dt of the last
 * eu_cfl_dt; else device memory holding the step's dt (1 double, or
 * n_instances for a batch; e.g. a minimum over several subdomains): the
 * step committed by the last eu_cfl_dt takes it, and the context time
 * becomes that step's start time plus it (negative values count as 0).
 * level -1: every level; with EU_DT_LTS one level-0 step of the recursive
 * level cycle (Sec. 2.2, Fig. 2).  level l >= 0 (EU_DT_LTS only): the
 * cycle from level l (its step of dt_l = dt_0 / 2^l, then its finer levels'
 * substeps, projection and flux correction) as the first substep of its
 * parent's step, whose start and end states level l-1 must hold.  A level
 * out of range, or level >= 0 with a global time step, is EU_EINVAL. */
int eu_fv_step(eu_ctx *ctx, const double *dt_dev, int level);

/* One full time step: eu_cfl_dt, eu_fv_step and, if regrid != 0,
 * eu_mr_decompose + eu_mr_flag (configuration CFL number and threshold). */
int eu_step(eu_ctx *ctx, int regrid);

/* nsteps calls of eu_step(ctx, regrid) (or until t_end), regrid as
 * regrid_every says, replayed from captured HIP graphs when use_graph != 0
 * (runs of sixteen steps, or of regrid_every steps from a regrid to the next,
 * in one graph; other steps one at a time).  steps_done_host (nullable)
 * receives the number of steps taken. */
int eu_advance(eu_ctx *ctx, int nsteps, int use_graph, int *steps_done_host);

/* Conserved totals sum over leaves of Q_f |cell| in FP64 (fixed summation
 * order), per instance: the quantities the flux correction at refinement
 * boundaries keeps constant up to boundary fluxes (Sec. 2.2).  totals_dev
 * (nullable, device memory) receives n_instances x (d+2) values on the
 * stream without synchronising (graph-capturable); totals_host (nullable)
 * receives them after a synchronisation. */
int eu_conserved_totals(eu_ctx *ctx, double *totals_dev, double *totals_host);

/* For callers that cannot allocate device memory or hand the library a
 * workspace at the call (code under HIP graph capture, tight serving
 * loops): eu_conserved_totals with its scratch -- the per-tile partial sums
 * and the per-instance totals -- in a static array of the library's own
 * device memory (4 MiB, one copy per GPU, held until the process ends)
 * instead of the context's scratch buffer.  Same kernels, same summation
 * order: the results equal eu_conserved_totals bit for bit.  totals_dev
 * (device memory, n_instances x (d+2) doubles, required) receives them on
 * the stream without synchronising.  EU_ENOMEM when the context's leaf-tile
 * capacity times d+2, plus n_instances times d+2, exceeds 2^19 doubles
 * (e.g. a batch of more than about 1.5e5 tiles of 8^2 cells); no device
 * memory is allocated or freed.  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (several streams or host threads)
 * race and must be serialised by the caller. */
int eu_conserved_totals_static(eu_ctx *ctx, double *totals_dev);

/* Copy one level (instance inst for a batch, level ignored) of the current
 * state (which = 0) or the RK2 stage state (which = 1) to FP64 host memory
 * in the state layout: (d+2) n^d values. */
int eu_copy_level(eu_ctx *ctx, int inst, int level, int which, double *dst_host);

/* The adaptive solution projected onto the finest uniform grid (the error
 * assessment of Sec. 3): level 0, then on each finer level every cell in a
 * patch keeps its value and every other cell is predicted (Sec. 2.1) from
 * the level below.  dst_host receives nv fields of n_finest^d values (SoA,
 * x fastest, converted to double).  The composite is built in the stage
 * array, which the next step recomputes.  Hierarchy only (EU_EINVAL for a
 * batch); synchronises the stream. */
int eu_copy_uniform(eu_ctx *ctx, double *dst_host);

/* Per-cell masks of a level (n^d bytes): patch membership (eu_get_active),
 * final refinement flags (eu_get_flags, levels 0..L-2), FP64 details
 * (eu_get_details, levels 0..L-2). */
int eu_get_active(eu_ctx *ctx, int level, uint8_t *dst_host);
int eu_get_flags(eu_ctx *ctx, int level, uint8_t *dst_host);
int eu_get_details(eu_ctx *ctx, int level, double *dst_host);

/* Patch table of the new mesh (the rectangular submeshes G_{l,m} of
 * Sec. 2.2, generated with the efficiency rule eta_tol): rows of 7 ints
 * {level, ox, oy, oz, sx, sy, sz} (origin and extents in cells of the
 * level; 2D: oz = 0, sz = 1) ordered by level, then Morton order of the
 * enclosing patch_max block, then the order the tiler emitted them (the
 * recursive split order, or the depth-first order of the clustering).  At
 * most cap rows are written to dst_host; *npatch_host receives the total
 * (synchronises). */
int eu_patch_table(eu_ctx *ctx, int32_t *dst_host, int cap, int *npatch_host);

/* Leaf and active (patch) cell counts per level (levels entries each). */
int eu_counters(eu_ctx *ctx, int64_t *leaves_host, int64_t *active_host);

/* Leaf cells advanced and steps taken since initialisation (a leaf advanced
 * one step of its level counts once; a batch counts every cell). */
int eu_leaf_updates(eu_ctx *ctx, int64_t *updates_host, int *steps_host);

/* Simulation time and last dt (instance 0). */
int eu_time(eu_ctx *ctx, double *t_host, double *dt_host);

/* Kernel timing with HIP events on the context's stream: when enabled,
 * every finite-volume stage launch is bracketed by events; eu_kernel_time
 * returns the summed milliseconds and the launch count since enabling. */
int eu_profile(eu_ctx *ctx, int enable);
int eu_kernel_time(eu_ctx *ctx, double *ms_host, int64_t *launches_host);

/* Schedule of the finite-volume update (Sec. 2: both stages of the
 * midpoint rule on every leaf).  Schedules 0 .. 5 apply everywhere: the
 * tile kernel (one 8^d block with its halo in LDS per workgroup) with 64,
 * 128 or 192 threads per tile in 2D (256 or 512 in 3D), faces axis by axis,
 * axis by axis from per-cell face states, or all axes in one pass.
 * Schedules EU_STRIP_SCHEDULE0 .. EU_STAGE_SCHEDULES-1 apply to grids of
 * one level (a uniform grid or a batch): the strip kernels (64 columns per
 * wave, slopes once per cell, x neighbours by lane exchange).  2D: one wave
 * per strip marching up the rows; 6 and 7 one stage per launch, 8 and 9 both
 * stages fused in one launch that keeps the stage state in registers
 * (outflow boundaries only; the state then alternates between the two
 * state arrays, which the library tracks); 6 and 8 with strips of 32 rows,
 * 7 and 9 of 128.  3D: one workgroup per strip of 8 output rows (6, 8) or
 * 16 (7, 9), one wave per row, marching through 32 (6, 7) or 64 (8, 9)
 * planes, y neighbours through LDS; one stage per launch.  The AMR scheme
 * takes the schedules its scheme field names; the MR-scheme variants (rk,
 * ausm_speed) run on schedules 0 .. 5.  In FP64 every schedule gives bit-identical results; in
 * FP32 they agree to rounding (the compiler contracts each differently).
 * eu_autotune times each schedule that applies (reps passes of one step's
 * finite-volume work on the current state -- both stages, the second in
 * its form reading the current state, or the fused launch; with local time
 * stepping the first stage of every level -- replayed from one HIP graph,
 * HIP events on the context's stream; the state is left unchanged) and
 * keeps the fastest: *variant_host receives it, ms_host (nullable,
 * EU_STAGE_SCHEDULES entries) the mean time of a pass of each (INFINITY
 * where a schedule does not apply).  eu_set_variant forces one
 * (EU_EINVAL where it does not apply).  Both drop captured graphs. */
int eu_autotune(eu_ctx *ctx, int reps, int *variant_host, float *ms_host);

/* Duration of the finite-volume update on the current state with the
 * current schedule: reps passes as eu_autotune times them, captured in one
 * HIP graph, replayed once untimed and once between two HIP events on the
 * context's stream (eager launches on the default stream); the state is
 * left unchanged.  *ms_host: mean milliseconds per pass; *cells_host:
 * cell-stages one pass computes (twice the leaves, or every cell of a
 * uniform grid or batch, for a global step; every cell once with the AMR
 * scheme; the patch cells of every level with local time stepping);
 * *launches_host: launches per pass.  Outputs
 * are nullable.  EU_ESTATE before initialisation or after t_end. */
int eu_stage_time(eu_ctx *ctx, int reps, float *ms_host, int64_t *cells_host, int *launches_host);
int eu_set_variant(eu_ctx *ctx, int variant);

/* Non-physical status: EU_OK or EU_ENONPHYS (synchronises). */
int eu_status(eu_ctx *ctx);
int eu_clear_status(eu_ctx *ctx);
const char *eu_last_error(const eu_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* EU_H */
