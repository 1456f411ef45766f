/*
 * janc.h -- C ABI of the MI355X (gfx950) library for the per-time-step core
 * update of the compressible reacting-flow solver of arXiv 2504.13750 (JANC).
 *
 * The library advances the 2-D multi-species reactive Euler equations
 * (paper Sec. 4.1, Eq. 4.1-4.9) with the numerics of Sec. 4.2: Lax-Friedrichs
 * flux-vector splitting with a global wave speed (Eq. 4.11), WENO5
 * reconstruction with 3 ghost layers, the conservative difference (Eq. 4.10),
 * third-order TVD Runge-Kutta, Newton for T from the internal energy, and the
 * first-order point-implicit chemistry step (Eq. 4.12-4.13). Block tables carry
 * the block-structured AMR of Sec. 3 (synchronous advance, Fig. 2b, or the
 * crossover advance, Fig. 2a) and ensembles of independent problems.
 *
 * Conventions for every call:
 *   - Arrays marked (device) are FP64 device memory owned by the caller; arrays
 *     marked (host) are read during the call only.
 *   - Layout is structure-of-arrays, field-major, x fastest: U[f][j][i] for a
 *     grid, U[f][cell] for a pool. Conserved fields are
 *     [rho, rho u, rho v, E, rho Y_1 .. rho Y_{Ns-1}] (Ns-1 = 1 for the
 *     one-step model, none for the perfect gas); T[cell] is the temperature.
 *   - Calls only enqueue work on the given stream (a hipStream_t passed as
 *     void*, NULL = default stream) and return without synchronizing, except
 *     where stated. A context is used by one host thread at a time.
 *   - Argument, table and launch errors return a negative janc_status at once,
 *     with a message in janc_last_error(). Numerical failures inside kernels
 *     (rho <= 0, p <= 0, non-finite values, Newton not converged) set a sticky
 *     device status word that janc_sync_status() reads and clears.
 *   - No exceptions cross this interface.
 */
#ifndef JANC_H
#define JANC_H

#ifdef __cplusplus
extern "C" {
#endif

typedef int janc_status;
enum {
    JANC_OK = 0,
    JANC_EINVAL = -1,      /* bad argument, table or unsupported size */
    JANC_ENOMEM = -2,      /* device allocation failed */
    JANC_EHIP = -3,        /* HIP runtime error */
    JANC_ENONFINITE = -4,  /* device: NaN/Inf produced */
    JANC_ENEWTON = -5,     /* device: T Newton did not converge in 50 iterations */
    JANC_ENEGATIVE = -6    /* device: rho, p or T not positive */
};

/* Boundary kinds (paper Sec. 4.3: user boundary functions), sides W, E, S, N. */
enum { JANC_BC_PERIODIC = 0, JANC_BC_ZEROGRAD = 1, JANC_BC_SLIPWALL = 2, JANC_BC_DIRICHLET = 3 };

/* Thermodynamic / chemistry models. */
enum {
    JANC_MODEL_CPG = 0,      /* calorically perfect gas, 4 fields */
    JANC_MODEL_ONESTEP = 1,  /* one-step Arrhenius source advanced inside RK3 (Sec. 4.3 item 3), 5 fields */
    JANC_MODEL_DETAILED = 2  /* NASA-7 + mass-action mechanism, point-implicit (Eq. 4.2-4.9, 4.12) */
};

enum { JANC_MAX_FIELDS = 16, JANC_MAX_LEVELS = 8, JANC_MAX_PROBES = 8 };

/* Detailed mechanism (host arrays, copied at janc_create), SI units:
 * M [ns] kg/mol; nasa [ns][7] NASA-7 coefficients a0..a6 (Eq. 4.3-4.5): the
 * only set, or with nasa_high / t_mid the low-temperature set (T < t_mid);
 * A [nr] in (m^3/mol)^(order-1)/s; b [nr]; Ea [nr] J/mol (Eq. 4.8); nu_f, nu_b
 * [nr][ns] integer stoichiometry (Eq. 4.6), at most 3 molecules per side;
 * tb [nr][ns] third-body efficiencies, used when has_tb[i] (Eq. 4.7);
 * reversible [nr]: k_b = k_f / K_eq (Eq. 4.9) when set, else 0. The last
 * species is the complement 1 - sum(Y). Kernels are compiled for every ns from 2 to
 * 12 (other sizes: JANC_EINVAL); nr <= 64. */
typedef struct {
    int ns, nr;
    const double *M, *nasa, *A, *b, *Ea;
    const int *nu_f, *nu_b;
    const double *tb;
    const int *has_tb, *reversible;
    const double *nasa_high;   /* [ns][7] high-temperature NASA-7 set, or NULL (one range) */
    const double *t_mid;       /* [ns] K: nasa_high applies for T >= t_mid (one value for all
                                  species, else JANC_EINVAL); NULL with nasa_high */
} janc_mech;

/* Per-problem physics: gamma and R for CPG/ONESTEP (R only scales T = p/(rho R));
 * Q, Ea, k of the one-step model rate -k rho Y exp(-Ea/T). Ignored for DETAILED. */
typedef struct {
    double gamma, R, Q, Ea, k;
} janc_physics;

/* A uniform grid (or the level-0 grid of a block-table domain). ny = 1 means
 * one-dimensional: no y sweep and no y term in the CFL bound. bc_prim[s] is
 * the primitive state of a Dirichlet side s (layout of janc_init_state). */
typedef struct {
    int nx, ny;
    double dx, dy;
    int bc[4];
    double bc_prim[4][JANC_MAX_FIELDS];
} janc_grid;

/* Time step: dt = cfl / max((|u|+c)/dx + (|v|+c)/dy) over solved cells, or
 * dt_fixed when > 0; clipped so that t does not pass t_end when t_end > 0
 * (steps after t_end leave the state unchanged). dt is formed from the state at
 * the start of the step.
 *
 * split selects how the chemistry (JANC_MODEL_DETAILED only) is combined with
 * the flux update (Sec. 4.2):
 *   JANC_SPLIT_LIE    three RK stages over dt, then the point-implicit step over
 *                     dt (the order of the paper's advance_one_step listing);
 *   JANC_SPLIT_STRANG point-implicit step over dt/2, three RK stages over dt,
 *                     point-implicit step over dt/2 (Strang splitting, Sec. 4.2).
 * jac selects the Jacobian of the point-implicit step (Eq. 4.12):
 *   JANC_JAC_FROZEN_T derivatives with respect to rho Y_1 .. rho Y_{Ns-1} with T,
 *                     rho, E and momentum held constant (as Sec. 4.2 states);
 *   JANC_JAC_FULL     the same variables, with T following the composition at
 *                     fixed rho and internal energy: J + (dS/dT)(dT/d rho Y)^T,
 *                     dT/d rho Y_m = -(e_m - e_Ns) / (rho c_v).
 * Any other value of split or jac, and JANC_SPLIT_STRANG or JANC_JAC_FULL with a
 * model without chemistry, is JANC_EINVAL. */
enum { JANC_SPLIT_LIE = 0, JANC_SPLIT_STRANG = 1 };
enum { JANC_JAC_FROZEN_T = 0, JANC_JAC_FULL = 1 };

typedef struct {
    double cfl, dt_fixed, t_end;
    int split;
    int jac;
} janc_time;

typedef struct janc_ctx janc_ctx;

/* Create a context on HIP device `device` for one model. mech is required for
 * JANC_MODEL_DETAILED and ignored otherwise. For the detailed model the context also
 * compiles (hipRTC, once per distinct mechanism in the process) the point-implicit
 * chemistry kernel specialised to the mechanism; see janc_set_chem_kernel. */
janc_status janc_create(janc_ctx **out, int model, const janc_mech *mech, int device);
void janc_destroy(janc_ctx *ctx);
const char *janc_last_error(const janc_ctx *ctx);
int janc_num_fields(const janc_ctx *ctx);

/* The point-implicit chemistry kernel of a detailed-model context (Eq. 4.12-4.13; the
 * specialisation is a systems pattern, not in the paper). JANC_CHEM_GENERIC: one kernel
 * per species count that reads each reaction's reactants and products from the mechanism
 * table (per-thread LDS columns indexed by those species numbers). JANC_CHEM_SPECIALIZED
 * (the default once it is built): the same arithmetic, operation for operation, with the
 * mechanism's structure -- participants of every reaction, reversibility, third-body
 * reactions, non-zero stoichiometric changes -- and its rate, stoichiometric, third-body
 * and molar-mass numbers compiled in as constants (exact literals), so that the cell's
 * state lives in registers; the results equal the generic kernel's bitwise. The adjoint's
 * reversed chemistry step (janc_adjoint) follows the same selection. The species + T Jacobian
 * (JANC_JAC_FULL) always uses the generic kernel. Selecting JANC_CHEM_SPECIALIZED where it
 * could not be built is JANC_EINVAL (janc_last_error gives the compiler's reason). */
enum { JANC_CHEM_GENERIC = 0, JANC_CHEM_SPECIALIZED = 1 };
janc_status janc_set_chem_kernel(janc_ctx *ctx, int mode);
janc_status janc_get_chem_kernel(const janc_ctx *ctx, int *mode);

/* Generates and compiles (hipRTC, no device needed) the specialised chemistry kernels of
 * a mechanism (the forward step, as janc_create does, and the adjoint's reversed step, as
 * the first janc_adjoint does): JANC_OK, or JANC_EINVAL for a mechanism janc_create
 * rejects, or JANC_EHIP with the compiler log in log (host, log_cap bytes incl. the
 * terminating zero; may be NULL). */
janc_status janc_chem_kernel_check(const janc_mech *mech, char *log, int log_cap);

/* Synchronizes the stream, returns and clears the sticky device status
 * (JANC_OK or one of JANC_ENONFINITE, JANC_ENEWTON, JANC_ENEGATIVE). */
janc_status janc_sync_status(janc_ctx *ctx, void *stream);

/* Conserved state from primitives (paper Eq. 4.2): W (device) [nfields][n] is
 *   CPG:      [rho, u, v, p]
 *   ONESTEP:  [rho, u, v, p, Y]
 *   DETAILED: [p, u, v, T, Y_1 .. Y_{Ns-1}]
 * and U (device) [nfields][n], T (device) [n] receive the conserved state and
 * the temperature. */
janc_status janc_init_state(janc_ctx *ctx, const janc_physics *phys, long long n,
                            const double *W, double *U, double *T, void *stream);

/* nsteps steps of the full update on a uniform grid (Sec. 4.3 advance_one_step:
 * CFL, RK3 flux stages, then chemistry for DETAILED; with JANC_SPLIT_STRANG the
 * chemistry takes half steps before and after the stages). U (device) [nfields][ny][nx]
 * and T (device) [ny][nx] are updated in place; T is re-solved from U at entry
 * with the given T as the Newton warm start. t (device) [1] is advanced by each
 * dt. dt_log (device) [nsteps] receives each dt, or may be NULL. */
janc_status janc_step(janc_ctx *ctx, const janc_grid *grid, const janc_physics *phys,
                      const janc_time *time, double *U, double *T, int nsteps, double *t,
                      double *dt_log, void *stream);

/* Bytes of the static device array that holds every workspace of janc_step_noalloc
 * (one per device, resident from the library's first janc_create on that device until
 * the process ends). */
#define JANC_NOALLOC_SCRATCH_BYTES (64ll << 20)

/* For callers that cannot allocate device memory (code under stream capture, serving
 * loops, harnesses that forbid hipMalloc): janc_step with the same arguments, results
 * and errors, that calls no hipMalloc, hipFree or allocating library routine. Its stage
 * states, reductions and plan tables live in the static array above: a grid needs about
 * 16 (nfields + 1) bytes per cell plus small tables (9 species: about 320 k cells; the
 * one-step model: about 690 k cells); larger grids are rejected with JANC_EINVAL and a
 * message, before any device work. The steps are launched directly (no graph); the tables
 * are copied into the array on `stream` at every call. Every call on a device shares that
 * device's array, which keeps the last call's contents: calls that overlap on one device
 * (other streams, other threads, other contexts) race and must be serialized by the
 * caller. */
janc_status janc_step_noalloc(janc_ctx *ctx, const janc_grid *grid, const janc_physics *phys,
                              const janc_time *time, double *U, double *T, int nsteps,
                              double *t, double *dt_log, void *stream);

/* ------------------------------------------------------------------ block tables */
/* A domain is one independent problem: a level-0 grid, its boundaries, its
 * physics and the number of refinement levels (ratio 2, Sec. 3.1). Each domain
 * has its own dt: in the synchronous advance (Fig. 2b) all its levels share it;
 * in the crossover advance (Fig. 2a) level l uses dt_0 / 2^l. */
typedef struct {
    janc_grid grid;
    janc_physics phys;
    int nlevels;
} janc_domain;

/* A block (Sec. 3.1.3 "data" + "info"): nx x ny cells at (i0, j0) of its level's
 * index space, stored at pool cell `offset` (x fastest). Invalid blocks are
 * reserved space that is neither solved nor read. Levels >= 1 need origins and
 * sizes that are multiples of 8 and sizes <= 256; level 0 must tile its domain. */
typedef struct {
    int domain, level, i0, j0, nx, ny;
    long long offset;
    int valid, pad;
} janc_block;

typedef struct janc_plan janc_plan;

enum {
    JANC_PLAN_DEFAULT = 0,
    JANC_PLAN_PER_BLOCK = 1,   /* one launch per block and stage (comparison form) */
    JANC_PLAN_NO_GRAPH = 2,    /* launch kernels directly instead of a captured hipGraph */
    JANC_PLAN_CROSSOVER = 4,   /* crossover advance (Fig. 2a, Alg. 2) instead of the synchronous one */
    JANC_PLAN_PER_LEVEL = 8,   /* one stage launch per refinement level (comparison form: the
                                  paper's per-level batching of equal-shape blocks, Alg. 2) */
    JANC_PLAN_AUTOTUNE = 16,   /* the first janc_step_blocks call runs janc_plan_autotune on its
                                  input state (5 timed launches per candidate) before stepping */
    JANC_PLAN_RESOLVE_HALOS = 32  /* no halo source table: the stage kernel looks up every
                                  off-block or coarse-fine ring source itself (comparison form;
                                  also the form of plans whose pool has 2^28 cells or more) */
};

/* Validate a block table and build its device work lists (blocks, level maps,
 * coarse-fine ring masks, tiles, restriction lists). Blocks and domains are
 * host arrays; pool_cells is the pool length. Synchronous. */
janc_status janc_plan_create(janc_ctx *ctx, int ndomains, const janc_domain *domains,
                             int nblocks, const janc_block *blocks, long long pool_cells,
                             int flags, janc_plan **out);
void janc_plan_destroy(janc_plan *plan);

/* Plan statistics (host) out[4]: cells of valid blocks, coarse-fine ring cells
 * among them (not solved; they hold the coarser level's value), valid blocks,
 * and tiles of one stage launch. */
janc_status janc_plan_stats(const janc_plan *plan, long long *out);

/* Per-plan tile shape (autotuner hook): 0 = automatic, else tile width in cells
 * for 2-D blocks (16 or 32 or 64; height = 256 / width). Synchronous. */
janc_status janc_plan_set_tile(janc_plan *plan, int tile_width);

/* Tile width (as janc_plan_set_tile) and the order in which workgroups take tiles:
 * linear = 1: workgroup b takes tile b; linear = 0 (default): the workgroups dealt to
 * each of the 8 XCDs take one contiguous run of tiles, so that neighbouring tiles,
 * whose halos overlap, are read through the same L2. Results do not depend on either. */
janc_status janc_plan_set_schedule(janc_plan *plan, int tile_width, int linear);

/* Autotuner of the batched stage launch (systems pattern, not in the paper). Candidates:
 * 2-D tile width 16, 32, 64 (16x16, 32x8, 64x4 cells) times the two workgroup orders of
 * janc_plan_set_schedule; 1-D-only plans: the two orders. A measurement is one RK stage
 * triple on the state U, T (device, read only; only the plan's workspaces are written),
 * timed with HIP events on `stream`; the candidates are measured in `reps` (1..1000)
 * interleaved rounds after one warm-up round and compared by their median. The plan keeps
 * its current shape unless a candidate is faster by more than 2 %; a linear-order
 * candidate's time is charged 3 % extra, since that order reads 2-3x the HBM bytes.
 * Synchronous on the host. choice (host [2], may be NULL) receives the tile width and the
 * order kept; ms (host [6], may be NULL) the median triple time of each candidate in the
 * order (16, XCD), (16, linear), (32, XCD), (32, linear), (64, XCD), (64, linear), -1
 * where not timed. Every candidate gives bitwise the same results. */
janc_status janc_plan_autotune(janc_ctx *ctx, janc_plan *plan, const janc_time *time,
                               const double *U, const double *T, int reps, int *choice,
                               double *ms, void *stream);

/* nsteps steps over a block table (Alg. 2 and Alg. 3 per stage): per domain dt;
 * per (domain, level) alpha; after each step coarse cells under finer blocks
 * become the mean of their four children (finest level first) and ring cells
 * are refilled. Synchronous advance (default): every level takes each RK stage
 * together with dt = CFL / max over all levels of (|u|+c)/dx_l + (|v|+c)/dy_l;
 * ring cells of levels >= 1 take the coarser level's value at the same stage.
 * Crossover advance (JANC_PLAN_CROSSOVER): a step is one step of level 0 with
 * dt_0 = CFL / max over all levels of (|u|+c)/dx_0 + (|v|+c)/dy_0; before each
 * step of level l, level l + 1 takes two steps of dt_0 / 2^(l+1) (deepest level
 * first), reading its ring and uncovered halo cells from the coarser level's
 * current state. U_pool (device) [nfields][pool], T_pool (device) [pool],
 * t (device) [ndomains]. */
janc_status janc_step_blocks(janc_ctx *ctx, janc_plan *plan, const janc_time *time,
                             double *U_pool, double *T_pool, int nsteps, double *t,
                             void *stream);

/* ------------------------------------------------------------------ layer update */
/* Parameters of the layer update (regridding, Sec. 3.1.2 and 3.1.4, Alg. 2).
 * A layer-l cell is masked when, on the effective layer-l density field (the
 * covering layer-l block, else the coarser layer's value, with the boundary
 * rules outside the domain),
 *     max(|rho(I+1,J) - rho(I-1,J)|, |rho(I,J+1) - rho(I,J-1)|) > 2 threshold rho(I,J)
 * (a central-difference density-gradient criterion normalized by the cell's
 * density and spacing). Each block of the new layer l is cut into fixed
 * subregions of sub x sub layer-l cells (the last row and column may be
 * narrower); a subregion becomes a layer-(l+1) block when a masked cell of layer
 * l lies in it or within `buffer` cells of it (the buffer cells), unless it
 * contains coarse-fine ring cells of layer l. sub: multiple of 4 in 4..128;
 * buffer >= 0; threshold >= 0. */
typedef struct {
    double threshold;
    int buffer;
    int sub;
} janc_regrid_params;

/* New block table of a plan's domains from the state U_pool (device, the plan's
 * pool layout; only rho is read). The level-0 blocks are kept in plan order;
 * layers 1, 2, ... follow, each ordered by parent block and subregion (row by
 * row); offsets are packed from 0. out (host) [cap] receives the table and
 * *nout its length; *pool_out the new pool length. When the table needs more
 * than cap entries the call returns JANC_EINVAL with *nout set to the length
 * needed. Level-0 blocks of refined domains need sizes that are multiples of 4.
 * Synchronizes the stream. */
janc_status janc_regrid(janc_ctx *ctx, janc_plan *plan, const janc_regrid_params *params,
                        const double *U_pool, janc_block *out, int cap, int *nout,
                        long long *pool_out, void *stream);

/* Pools of a new plan (same domains) from the state of an old plan: each block
 * of the new plan with the same domain, level, origin and size as a valid block
 * of the old plan takes that block's data (U and T, unaltered blocks keep their
 * data); every other block takes the one-to-four injection of the new plan's
 * coarser level, which is filled first (refinement operation, Sec. 3.1.4).
 * Level-0 blocks must all be unaltered. U_old, T_old (device) on the old plan's
 * pool; U_new, T_new (device) on the new plan's pool. */
janc_status janc_regrid_fill(janc_ctx *ctx, janc_plan *old_plan, const double *U_old,
                             const double *T_old, janc_plan *new_plan, double *U_new,
                             double *T_new, void *stream);

/* Profiling aid: one step of a plan (as in janc_step_blocks, after the call-entry
 * temperature solve) launched without graph capture, with HIP events recorded on
 * `stream` around each launch group. ms (host) [6] receives the durations in
 * milliseconds of RK stage 1, stage 2, stage 3, the chemistry step, the
 * restriction (all levels) and the ring refill. U_pool, T_pool and t advance by
 * the step. Synchronizes the stream. Crossover plans and Strang splitting return
 * JANC_EINVAL. */
janc_status janc_profile_step(janc_ctx *ctx, janc_plan *plan, const janc_time *time,
                              double *U_pool, double *T_pool, double *t, double *ms,
                              void *stream);

/* ------------------------------------------------------------------ adjoint */
/* Discrete adjoint (the exact gradient of the discrete map) of nsteps steps of
 * janc_step with a fixed dt (time->dt_fixed > 0), in the sense of the adjoint method
 * of Sec. 6.1 (Eq. 6.1-6.5) applied to the discrete trajectory, for the one-step model
 * and for the detailed model (Lie splitting and the frozen-T Jacobian: the temperature
 * Newton of Eq. 4.2-4.5 is differentiated by the implicit-function theorem, the
 * point-implicit step of Eq. 4.12-4.13 through its transposed solve and the rate
 * derivatives along its increment). Loss = sum_{n=1..N} dt * sum_q w_q *
 * p(U^n at cell probe_cell[q]). W0 (device) [nfields][ny][nx] are the initial
 * primitives in janc_init_state's layout; the state is checkpointed every ckpt_every
 * steps and recomputed inside each segment. Outputs (device): loss[1], dL_dW0
 * [nfields][ny][nx], dL_dtheta[2] = {dL/dQ, dL/dEa} of the one-step model (Q enters
 * through the equation of state and the initial energy), zeros for the detailed model.
 * probe_cell and probe_w are host arrays of nprobes (0 .. JANC_MAX_PROBES) entries; a
 * probe cell out of range, a count out of range, dt_fixed <= 0, t_end > 0, the CPG
 * model, Strang splitting or the species + T Jacobian return JANC_EINVAL. */
janc_status janc_adjoint(janc_ctx *ctx, const janc_grid *grid, const janc_physics *phys,
                         const janc_time *time, const double *W0, int nsteps, int ckpt_every,
                         int nprobes, const int *probe_cell, const double *probe_w,
                         double *loss, double *dL_dW0, double *dL_dtheta, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* JANC_H */
