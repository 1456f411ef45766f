// janc_internal.h -- device data layouts shared by the kernels and the host
// runtime of the JANC step library (gfx950). Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace janc {

constexpr int MAXF = 16;        // conserved fields (4 + species - 1)
constexpr int MAXL = 8;         // refinement levels per domain
constexpr int MAXS = 12;        // species
constexpr int MAXR = 64;        // reactions
constexpr int MAXP = 8;         // adjoint probes (JANC_MAX_PROBES)
constexpr int MAXLIST = 3;      // reactant / product molecules per reaction
constexpr int WG = 256;         // threads per workgroup of the tile and cell kernels
constexpr int AWG = 256;        // threads per workgroup of the adjoint kernels
constexpr double RU = 8.314472;     // J/(mol K), paper Sec. 4.1
constexpr double PATM = 101325.0;   // Pa, Eq. 4.9

enum Model { CPG = 0, ONESTEP = 1, DETAILED = 2 };
enum { BC_PERIODIC = 0, BC_ZEROGRAD = 1, BC_SLIPWALL = 2, BC_DIRICHLET = 3 };

// Sticky status bits written by kernels.
enum : unsigned { STB_NONFINITE = 1u, STB_NEWTON = 2u, STB_NEGATIVE = 4u };

// A domain: level-0 grid + boundaries + physics + per-level block maps.
struct DevDomain {
    int nx0, ny0, nlevels, twod;
    int bc[4];
    int dir[4];               // row of the Dirichlet table per side (-1 = none)
    int map_off[MAXL];        // offset of each level's block map (8x8-cell granularity)
    int map_w[MAXL];
    int slot0;                // alpha slot of level 0 (slot0 + level)
    int cfl_slot;             // index of this domain's CFL slot
    double dx0, dy0;
    double gamma, R, Q, Ea, k;
};

// A valid block. ring[s]: bit g set when the 8-cell segment g of side s
// (W, E, S, N) faces in-domain cells not covered at this level; the 3 cell
// layers along such a segment are coarse-fine ring cells.
struct DevBlock {
    int domain, level, i0, j0, nx, ny;
    long long offset;
    unsigned ring[4];
    int fine_child;           // 1 if a finer level exists in this domain
    int pad;
};

// One tile of a block: origin (x0, y0) in block-local cells.
struct Tile {
    int block, x0, y0, kind;  // kind 0 = 2-D tile shape, 1 = 1-D row tile
};

// Detailed mechanism in the layout the kernels read (uniform loads).
struct DevMech {
    int ns, nr;
    int two_range;                     // a high-temperature NASA-7 set is present
    int pad;
    double invM[MAXS];
    double Rk[MAXS];                   // R_u / M_k
    double nasa[MAXS][7];              // the one set, or the low-temperature set
    double nasa_hi[MAXS][7];           // high-temperature set (T >= tmid)
    double tmid[MAXS];
    double lnA[MAXR], b[MAXR], EaR[MAXR];
    int rev[MAXR], has_tb[MAXR], dnsum[MAXR], pad2[MAXR];
    int lf[MAXR][4], lb[MAXR][4];      // reactant / product species lists, padded with ns (= 1.0)
    int dnu[MAXR][MAXS];
    double Mdnu[MAXR][MAXS];           // M_k (nu_b - nu_f), production weights
    double tb[MAXR][MAXS];
};

// Reduction slots (buffers of `stride` slots): per (domain, level) unit the maxima
// of |u|+c and |v|+c (Eq. 4.11), per domain the CFL bound max((|u|+c)/dx +
// (|v|+c)/dy). Non-negative doubles are stored by bit pattern, so an unsigned
// integer max is the floating-point max. Buffers 0-2 rotate through the RK stages
// (stage s reads s - 1, writes s mod 3, clears s + 1 mod 3); buffer 3 carries the
// maxima of the first half chemistry step to stage 1 under Strang splitting.
// Each slot is one 64-bit word alone in a 128-byte line (SLOT_WORDS words apart):
// every workgroup of a launch takes an atomic max on its slots while others read
// the slots of the previous stage, and slots sharing a line serialise on it (packed
// slots made a launch whose slots shared a line with the slots it read 0.25 ms
// slower on 7,750 workgroups).
constexpr int RED_BUFS = 4;
constexpr int SLOT_WORDS = 16;

struct Reduce {
    unsigned long long* buf;
    int stride;
    int nunits;
    int ndom;
    int pad;
};

struct TimeArgs {
    double cfl, dt_fixed, t_end;
};

struct StageArgs {
    const DevDomain* dom;
    const DevBlock* blk;
    const int* maps;
    const Tile* tiles;
    int ntiles;
    int stage;                // 1..3
    const double* dirU;       // Dirichlet rows: MAXF conserved values then T
    const DevMech* mech;
    const double* U0;         // step start state U^n
    const double* Uin;        // stage input U^(s-1)
    double* Uout;             // stage output U^(s)
    const double* Tin;
    double* Tout;
    long long pool;           // field stride of the pools
    Reduce red;
    int reduce_out;           // accumulate maxima of the output state
    int ndom;
    double* dt;               // [ndom] this step's dt
    double* t;                // [ndom] time
    double* dt_log;           // [capacity][ndom] or null
    int* step;                // device step counter (for dt_log)
    int dt_log_cap;
    TimeArgs tm;
    unsigned* status;
    int strang;               // Strang splitting: chemistry over dt/2 before and after the stages
    int chem_phase;           // chemistry launch: 0 whole dt, 1 first half, 2 second half
    int full_jac;             // point-implicit Jacobian with T following the composition
    // crossover advance (per-level launches, dt_l = dt_0 / 2^l); all zero otherwise
    int cross;
    int xfirst;               // first launch of the step: computes dt_0
    int xlast;                // last launch of the step: advances t and the step counter
    int xskip_cov;            // last step of this level in the step: covered cells leave the maxima
    int xlevels;              // levels with reduction slot triples
    unsigned long long* xred; // all levels' slot sets (level l at l * RED_BUFS * red.stride)
    const double* Tbase;      // T of the pool (coarser levels' current state)
    int linear_sched;         // stage launches: workgroup b takes tile b (else XCD-contiguous runs)
    // halo source table of the plan (or null: the stage kernel resolves every source):
    // entry [tile * hstride + point] = 8 * source + flags for each point whose source is
    // not its own block's cell at that position
    const int* hsrc;
    int hstride;
};

// Layer update: a candidate subregion (layer-`lev` cells) and a fill job.
struct RegridCand {
    int domain, i0, j0, w, h, pad;
};
struct RegridFill {
    int block, pad;           // block of the new plan
    long long src;            // its cells in the old pool, or -1: inject from the coarser layer
};

// Launchers implemented in janc_kernels.hip (regrid: janc_regrid.hip).
hipError_t launch_clear_reduce(const Reduce& r, int which, hipStream_t s);
hipError_t launch_zero_int(int* p, hipStream_t s);
hipError_t launch_stage(int model, int ns, int kind_mask, int tile_w, const StageArgs& a,
                        int first_tile, int ntiles, hipStream_t s);
hipError_t launch_init(int model, int ns, int tile_w, const StageArgs& a, hipStream_t s);
// Halo source table (row stride: the largest point count of the tile kinds in kind_mask)
int halo_table_stride(int tile_w, int kind_mask);
hipError_t launch_halo_table(int tile_w, const StageArgs& a, int* out, int stride, hipStream_t s);
hipError_t launch_chem(int model, int ns, int tile_w, const StageArgs& a, hipStream_t s);
hipError_t launch_restrict(int model, int ns, const StageArgs& a, const int* fine_blocks,
                           int nfine, hipStream_t s);
hipError_t launch_ring_fill(int model, int ns, const StageArgs& a, const int* ring_blocks,
                            int nring, hipStream_t s);
hipError_t launch_regrid_flag(const StageArgs& a, const RegridCand* cand, int n, int lev,
                              int buffer, double thr, int* flags, hipStream_t s);
hipError_t launch_regrid_fill(const StageArgs& a, const RegridFill* job, int n, long long old_pool,
                              int nu, hipStream_t s);
hipError_t launch_prim_to_cons(int model, int ns, const DevMech* mech, double gamma, double R,
                               double Q, long long n, const double* W, double* U, double* T,
                               long long stride_in, long long stride_out, hipStream_t s);
bool model_supported(int model, int ns);


// Discrete adjoint (uniform grid; one-step and detailed models): grid constants and
// the arguments of one stage's reverse sweep. A stored state of the detailed model
// is [NU][n] conserved fields followed by [n] temperatures (the Newton solution the
// forward stored with it); one-step states are [NU][n].
struct AdjGrid {
    int nx, ny, twod, pad;
    int bc[4];
    int dir[4];
    double idx, idy;
    double gamma, R, Q, Ea, k;
    const double* dirU;
};

struct AdjArgs {
    AdjGrid g;
    long long n;              // cells
    const double* V;          // stage input [NU][n]
    const double* VT;         // its temperatures [n] (detailed model)
    const DevMech* mech;      // detailed model: the mechanism
    const double* lamW;       // adjoint of the stage output [NU][n]
    double* lamOut;           // adjoint of the stage input [NU][n]
    double* acc;              // adjoint of the step start U^n [NU][n]
    double b, a, dt;
    int init_acc, add_out;
    double *cx, *cy;          // reverse WENO5 weights per interface [NU][10][interfaces]
    const double* alpha;      // [2] alpha_x, alpha_y of the stage input
    const int* argm;          // [2] lowest cell attaining them
    double* part;             // [nbd][4] block partials
    int nbd;                  // cell blocks
    double* theta;            // [2]: dL/dQ, dL/dEa
    const double* seedU;      // state whose probe loss seeds acc after this stage (or null)
    const double* seedT;      // its temperatures (detailed model)
    const int* pc;
    const double* pw;
    int np;
};

// Alpha maxima and argmax of every stage input of a run of steps (one launch):
// slice z = 3 m + (stage - 1) reads base[stage - 1] + m * step_stride.
struct AlphaArgs {
    AdjGrid g;
    long long n;
    const DevMech* mech;
    const double* base[3];    // (detailed model: temperatures at base + NU n)
    long long step_stride;
    int nsteps;
    int nbd;
    double* part;             // [slices][nbd][4]
    double* alpha;            // [slices][2]
    int* argm;                // [slices][2]
};

// Chemistry step of the detailed model in reverse (one launch, one cell per thread):
// lam (adjoint of the step's output U^{n+1}) becomes the adjoint of its input U*
// (the third stage's output, at temperature Tstar).
struct AdjChemArgs {
    long long n;
    const DevMech* mech;
    const double* Ustar;      // [NU][n]
    const double* Tstar;      // [n]
    const double* lamIn;      // adjoint of U^{n+1} [NU][n]
    double* lamOut;           // adjoint of U* [NU][n]
    double dt;
    unsigned* status;
};

// model: ONESTEP or DETAILED; ns: species of the detailed model (2 or 9)
hipError_t adj_alpha_launch(int model, int ns, const AlphaArgs& P, hipStream_t s);
hipError_t adj_stage(int model, int ns, const AdjArgs& A, hipStream_t s);
hipError_t adj_chem_launch(int ns, const AdjChemArgs& A, hipStream_t s);
hipError_t adj_loss_launch(int model, int ns, const AdjGrid& g, const DevMech* mech,
                           const double* base, long long stride, int count, const double* last,
                           int n0, long long n, const int* pc, const double* pw, int np, double dt,
                           double* term, hipStream_t s);
hipError_t adj_loss_sum_launch(const double* term, int nsteps, double* loss, hipStream_t s);
hipError_t adj_seed_launch(int model, int ns, const AdjGrid& g, const DevMech* mech,
                           const double* U, long long n, const int* pc, const double* pw, int np,
                           double dt, double* lam, double* theta, hipStream_t s);
hipError_t adj_chain_launch(int model, int ns, const AdjGrid& g, const DevMech* mech,
                            const double* W, const double* lam, long long n, double* gW,
                            double* part, double* theta, hipStream_t s);

// Launches of the detailed model for one species count NS (janc_species.hip, one
// translation unit per count): the step's kernels and the adjoint's.
struct SpeciesOps {
    int ns;
    hipError_t (*stage)(int kind_mask, int tile_w, const StageArgs& a, int first_tile, int ntiles,
                        int owner, hipStream_t s);
    hipError_t (*init)(const StageArgs& a, hipStream_t s);
    hipError_t (*chem)(const StageArgs& a, hipStream_t s);
    hipError_t (*restrict_fine)(const StageArgs& a, const int* fine_blocks, int nfine, hipStream_t s);
    hipError_t (*ring_fill)(const StageArgs& a, const int* ring_blocks, int nring, hipStream_t s);
    hipError_t (*prim_to_cons)(const DevMech* mech, long long n, const double* W, double* U, double* T,
                               long long stride_in, long long stride_out, hipStream_t s);
    hipError_t (*adj_alpha)(const AlphaArgs& P, hipStream_t s);     // before adj_alpha_reduce
    hipError_t (*adj_stage)(const AdjArgs& A, hipStream_t s);
    hipError_t (*adj_chem)(const AdjChemArgs& A, hipStream_t s);
    hipError_t (*adj_loss)(const AdjGrid& g, const DevMech* mech, const double* base, long long stride,
                           int count, const double* last, int n0, long long n, const int* pc,
                           const double* pw, int np, double dt, double* term, hipStream_t s);
    hipError_t (*adj_seed)(const AdjGrid& g, const DevMech* mech, const double* U, long long n,
                           const int* pc, const double* pw, int np, double dt, double* lam,
                           double* theta, hipStream_t s);
    hipError_t (*adj_chain)(const AdjGrid& g, const DevMech* mech, const double* W, const double* lam,
                            long long n, double* gW, double* part, hipStream_t s);   // before adj_chain_sum
};

// Species counts with compiled kernels: JANC_NS_FIRST .. JANC_NS_LAST (all of them).
constexpr int JANC_NS_FIRST = 2, JANC_NS_LAST = MAXS;
const SpeciesOps* species_ops(int ns);   // null: no kernels for this count

}  // namespace janc
