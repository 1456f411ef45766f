// janc_api.hip -- host runtime behind the C ABI of include/janc.h: contexts,
// block-table plans (validation, level maps, coarse-fine ring masks, tiles,
// restriction lists), call sequencing and hipGraph capture of whole steps.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <array>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/janc.h"
#include "janc_rtc.h"
#include "janc_internal.h"

using namespace janc;

// The workspace of janc_step_noalloc: one array per device, held until the process ends.
// Host code never uses the array's name as an address: its device address comes from
// hipGetSymbolAddress, once per device, with that device current (noalloc_scratch).
static __device__ __align__(256) unsigned char scratch[JANC_NOALLOC_SCRATCH_BYTES];

static_assert(MAXP == JANC_MAX_PROBES, "probe limit of the adjoint kernels");
static_assert(MAXF == JANC_MAX_FIELDS && MAXL == JANC_MAX_LEVELS, "table limits");

struct janc_plan;

struct janc_ctx {
    int device = 0;
    int model = 0;
    int ns = 0;
    int nU = 0;
    DevMech hmech{};
    DevMech* dmech = nullptr;
    unsigned* dstatus = nullptr;
    std::string err;
    // cached plan for janc_step (uniform grids)
    janc_plan* uplan = nullptr;
    janc_grid ugrid{};
    janc_physics uphys{};
    // cached plan of janc_step_noalloc: host tables, device addresses inside the
    // static scratch array
    janc_plan* nplan = nullptr;
    janc_grid ngrid{};
    janc_physics nphys{};
    // adjoint workspace (grown on demand)
    double* adj_mem = nullptr;
    size_t adj_doubles = 0;
    hipStream_t adj_stream = nullptr;   // auxiliary stream of the adjoint's recompute
    hipEvent_t adj_ev[5] = {};
    // chemistry kernel specialised to the mechanism's structure (detailed model)
    hipModule_t chem_mod = nullptr;
    hipFunction_t chem_fn = nullptr;
    int chem_mode = JANC_CHEM_GENERIC;
    std::string chem_log;               // why no specialised kernel could be built
    // its reverse in the adjoint, built at the first adjoint run that needs it
    hipModule_t adj_chem_mod = nullptr;
    hipFunction_t adj_chem_fn = nullptr;
    bool adj_chem_tried = false;
    std::string adj_chem_log;
};

struct GraphKey {
    const double *U, *T, *t, *dt_log;
    int cap;
    double cfl, dt_fixed, t_end;
    int split, jac;
    int chem;   // the context's chemistry kernel (generic or specialised)
    bool operator==(const GraphKey& o) const {
        return U == o.U && T == o.T && t == o.t && dt_log == o.dt_log && cap == o.cap &&
               cfl == o.cfl && dt_fixed == o.dt_fixed && t_end == o.t_end && split == o.split &&
               jac == o.jac && chem == o.chem;
    }
};

struct janc_plan {
    janc_ctx* ctx = nullptr;
    int flags = 0;
    int ndom = 0, nblk = 0;
    long long pool = 0;
    int nunits = 0;
    int tile_w = 16;
    int linear_sched = 0;         // 1: workgroup b takes tile b; 0: XCD-contiguous tile runs
    bool tuned = false;           // janc_plan_autotune has chosen tile_w and linear_sched
    int kind_mask = 0;            // bit 0: 2-D tiles present, bit 1: 1-D tiles present
    int maxlev = 0;
    std::vector<DevDomain> hdom;
    std::vector<DevBlock> hblk;   // valid blocks only (device block ids)
    std::vector<int> hmap;
    std::vector<Tile> htiles;
    std::vector<int> tile_first, tile_count;   // per valid block
    std::vector<int> lev_first, lev_count;     // per level: tiles (grouped by level)
    std::vector<std::vector<int>> fine;        // per level >= 1: valid block ids
    std::vector<int> ring_blocks;
    std::vector<double> hdir;
    long long cells = 0, ring_cells = 0;
    // device
    DevDomain* ddom = nullptr;
    DevBlock* dblk = nullptr;
    int* dmap = nullptr;
    Tile* dtiles = nullptr;
    int* dhsrc = nullptr;          // halo source table (StageArgs::hsrc), or null
    int hstride = 0;
    double* ddir = nullptr;
    unsigned long long* dred = nullptr;
    int red_stride = 0;
    double* ddt = nullptr;
    int* dstep = nullptr;
    int* dfine = nullptr;          // concatenated fine lists
    std::vector<int> fine_off, fine_flat;
    int* dring = nullptr;
    double *U1 = nullptr, *U2 = nullptr, *T1 = nullptr, *T2 = nullptr;
    // graph cache
    bool have_graph = false;
    GraphKey gkey{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t gdone = nullptr;    // recorded after the last replay of the graph
    // Workspace source. arena == nullptr: every device array is a hipMalloc of its own.
    // Otherwise arrays are carved from [arena, arena + arena_cap) (the static scratch
    // array of janc_step_noalloc) and nothing is copied at build time: the host tables
    // are uploaded and the Dirichlet rows converted by stage_tables() before each use.
    char* arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    struct Upload { void* dst; const void* src; size_t bytes; };
    std::vector<Upload> uploads;
    struct DirRow { int row; double gamma, R, Q; double prim[MAXF]; };
    std::vector<DirRow> dir_rows;
    double* dir_w = nullptr;       // arena: primitive staging of the Dirichlet rows
};

namespace {

int n_fields(int model, int ns) { return model == CPG ? 4 : model == ONESTEP ? 5 : ns + 3; }

janc_status fail(janc_ctx* c, janc_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

janc_status hipfail(janc_ctx* c, hipError_t e, const char* what) {
    return fail(c, JANC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// Time settings common to every stepping entry point.
janc_status check_time(janc_ctx* c, const janc_time* tm) {
    if (!(tm->dt_fixed > 0.0) && !(tm->cfl > 0.0)) return fail(c, JANC_EINVAL, "need cfl > 0 or dt_fixed > 0");
    if (tm->split != JANC_SPLIT_LIE && tm->split != JANC_SPLIT_STRANG)
        return fail(c, JANC_EINVAL, "split must be JANC_SPLIT_LIE or JANC_SPLIT_STRANG");
    if (tm->split == JANC_SPLIT_STRANG && c->model != DETAILED)
        return fail(c, JANC_EINVAL, "Strang splitting needs a model with chemistry (detailed)");
    if (tm->jac != JANC_JAC_FROZEN_T && tm->jac != JANC_JAC_FULL)
        return fail(c, JANC_EINVAL, "jac must be JANC_JAC_FROZEN_T or JANC_JAC_FULL");
    if (tm->jac == JANC_JAC_FULL && c->model != DETAILED)
        return fail(c, JANC_EINVAL, "the species + T Jacobian needs a model with chemistry (detailed)");
    return JANC_OK;
}

#define HIPCHK(ctx, expr, what)                      \
    do {                                             \
        hipError_t _e = (expr);                      \
        if (_e != hipSuccess) return hipfail(ctx, _e, what); \
    } while (0)

template <class T> janc_status dalloc(janc_ctx* c, T** p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void**)p, n * sizeof(T));
    if (e != hipSuccess) return fail(c, JANC_ENOMEM, "hipMalloc of %zu bytes failed", n * sizeof(T));
    return JANC_OK;
}

template <class T> janc_status upload(janc_ctx* c, T** p, const std::vector<T>& v) {
    janc_status st = dalloc(c, p, v.size());
    if (st) return st;
    if (!v.empty()) HIPCHK(c, hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
    return JANC_OK;
}

void plan_free(janc_plan* p) {
    if (!p) return;
    if (p->gdone) hipEventSynchronize(p->gdone);
    if (p->gexec) hipGraphExecDestroy(p->gexec);
    if (p->graph) hipGraphDestroy(p->graph);
    if (p->gdone) hipEventDestroy(p->gdone);
    if (!p->arena) {
        void* ptrs[] = {p->ddom, p->dblk, p->dmap, p->dtiles, p->dhsrc, p->ddir, p->dred, p->ddt,
                        p->dstep, p->dfine, p->dring, p->U1, p->U2, p->T1, p->T2};
        for (void* q : ptrs)
            if (q) hipFree(q);
    }
    delete p;
}

// Device array of a plan: its own hipMalloc, or the next 256-byte aligned piece of the
// plan's arena (nothing is allocated; too little room is an argument error).
template <class T> janc_status palloc(janc_plan* P, T** p, size_t n) {
    if (!P->arena) return dalloc(P->ctx, p, n);
    *p = nullptr;
    if (n == 0) n = 1;
    const size_t off = (P->arena_used + 255) & ~(size_t)255;
    const size_t bytes = n * sizeof(T);
    if (off > P->arena_cap || bytes > P->arena_cap - off)
        return fail(P->ctx, JANC_EINVAL,
                    "the grid needs more than the %zu bytes of the static scratch of janc_step_noalloc",
                    P->arena_cap);
    *p = (T*)(P->arena + off);
    P->arena_used = off + bytes;
    return JANC_OK;
}

// A host table on the device: copied now, or (arena) recorded for stage_tables().
template <class T> janc_status pupload(janc_plan* P, T** p, const std::vector<T>& v) {
    if (!P->arena) return upload(P->ctx, p, v);
    janc_status st = palloc(P, p, v.size());
    if (st) return st;
    if (!v.empty()) P->uploads.push_back({(void*)*p, (const void*)v.data(), v.size() * sizeof(T)});
    return JANC_OK;
}

// --------------------------------------------------------------- mechanism
// The mechanism in the layout the kernels read (host copy; validated).
janc_status build_mech(janc_ctx* c, const janc_mech* m) {
    if (!m || m->ns < 2 || m->ns > MAXS || m->nr < 0 || m->nr > MAXR)
        return fail(c, JANC_EINVAL, "mechanism sizes out of range (ns 2..%d, nr 0..%d)", MAXS, MAXR);
    if (!model_supported(DETAILED, m->ns))
        return fail(c, JANC_EINVAL, "no kernels compiled for ns = %d (available: %d .. %d)", m->ns, JANC_NS_FIRST, JANC_NS_LAST);
    DevMech& d = c->hmech;
    std::memset(&d, 0, sizeof(d));
    d.ns = m->ns;
    d.nr = m->nr;
    for (int k = 0; k < m->ns; ++k) {
        if (!(m->M[k] > 0.0)) return fail(c, JANC_EINVAL, "molar mass of species %d not positive", k);
        d.invM[k] = 1.0 / m->M[k];
        d.Rk[k] = RU / m->M[k];
        for (int q = 0; q < 7; ++q) d.nasa[k][q] = m->nasa[7 * k + q];
    }
    if ((m->nasa_high == nullptr) != (m->t_mid == nullptr))
        return fail(c, JANC_EINVAL, "nasa_high and t_mid go together");
    if (m->nasa_high) {
        d.two_range = 1;
        for (int k = 0; k < m->ns; ++k) {
            if (!(m->t_mid[k] > 0.0)) return fail(c, JANC_EINVAL, "t_mid of species %d not positive", k);
            if (m->t_mid[k] != m->t_mid[0])
                return fail(c, JANC_EINVAL, "t_mid must be the same for every species");
            d.tmid[k] = m->t_mid[k];
            for (int q = 0; q < 7; ++q) d.nasa_hi[k][q] = m->nasa_high[7 * k + q];
        }
    }
    for (int i = 0; i < m->nr; ++i) {
        d.lnA[i] = (m->A[i] > 0.0) ? std::log(m->A[i]) : -INFINITY;
        d.b[i] = m->b[i];
        d.EaR[i] = m->Ea[i] / RU;
        d.rev[i] = m->reversible[i] ? 1 : 0;
        d.has_tb[i] = m->has_tb[i] ? 1 : 0;
        int nf = 0, nb = 0, ds = 0;
        for (int q = 0; q < 4; ++q) d.lf[i][q] = d.lb[i][q] = m->ns;
        for (int j = 0; j < m->ns; ++j) {
            const int f = m->nu_f[i * m->ns + j], b = m->nu_b[i * m->ns + j];
            if (f < 0 || b < 0) return fail(c, JANC_EINVAL, "negative stoichiometry in reaction %d", i);
            for (int q = 0; q < f; ++q) {
                if (nf >= MAXLIST) return fail(c, JANC_EINVAL, "reaction %d has more than %d reactant molecules", i, MAXLIST);
                d.lf[i][nf++] = j;
            }
            for (int q = 0; q < b; ++q) {
                if (nb >= MAXLIST) return fail(c, JANC_EINVAL, "reaction %d has more than %d product molecules", i, MAXLIST);
                d.lb[i][nb++] = j;
            }
            d.dnu[i][j] = b - f;
            d.Mdnu[i][j] = m->M[j] * (double)(b - f);
            d.tb[i][j] = m->tb[i * m->ns + j];
            ds += b - f;
        }
        d.dnsum[i] = ds;
    }
    return JANC_OK;
}

// The mechanism tables on the device.
janc_status upload_mech(janc_ctx* c) {
    janc_status st = dalloc(c, &c->dmech, 1);
    if (st) return st;
    HIPCHK(c, hipMemcpy(c->dmech, &c->hmech, sizeof(c->hmech), hipMemcpyHostToDevice), "hipMemcpy mech");
    return JANC_OK;
}

// --------------------------------------------------------------- plan building
struct LevelMap {
    int w8 = 0, h8 = 0, off = 0;
};

janc_status build_plan(janc_ctx* c, int nd, const janc_domain* doms, int nb, const janc_block* blocks,
                       long long pool, int flags, janc_plan** out, char* arena = nullptr,
                       size_t arena_cap = 0) {
    *out = nullptr;
    if (nd < 1 || nb < 1 || pool < 1 || !doms || !blocks)
        return fail(c, JANC_EINVAL, "empty block table");
    std::unique_ptr<janc_plan, void (*)(janc_plan*)> P(new janc_plan(), plan_free);
    P->ctx = c;
    P->arena = arena;
    P->arena_cap = arena_cap;
    if (flags & ~(JANC_PLAN_PER_BLOCK | JANC_PLAN_NO_GRAPH | JANC_PLAN_CROSSOVER | JANC_PLAN_PER_LEVEL |
                  JANC_PLAN_AUTOTUNE | JANC_PLAN_RESOLVE_HALOS))
        return fail(c, JANC_EINVAL, "unknown plan flags");
    if ((flags & JANC_PLAN_PER_BLOCK) && (flags & JANC_PLAN_CROSSOVER))
        return fail(c, JANC_EINVAL, "the crossover advance has no per-block form");
    if ((flags & JANC_PLAN_PER_LEVEL) && (flags & (JANC_PLAN_PER_BLOCK | JANC_PLAN_CROSSOVER)))
        return fail(c, JANC_EINVAL, "the per-level form is a form of the synchronous batched advance");
    P->flags = flags;
    P->ndom = nd;
    P->pool = pool;
    const int nU = c->nU;
    // ---- domains
    std::vector<std::vector<LevelMap>> lm(nd);
    int map_total = 0, slot = 0, ndir = 0;
    for (int d = 0; d < nd; ++d) {
        const janc_domain& D = doms[d];
        const janc_grid& g = D.grid;
        DevDomain h{};
        if (g.nx < 3 || g.ny < 1 || (g.ny > 1 && g.ny < 3))
            return fail(c, JANC_EINVAL, "domain %d: grid %dx%d too small (need >= 3 cells per active direction)", d, g.nx, g.ny);
        if (!(g.dx > 0.0) || !(g.dy > 0.0)) return fail(c, JANC_EINVAL, "domain %d: dx, dy must be positive", d);
        if (D.nlevels < 1 || D.nlevels > MAXL) return fail(c, JANC_EINVAL, "domain %d: nlevels out of range", d);
        if (D.nlevels > 1 && g.ny == 1) return fail(c, JANC_EINVAL, "domain %d: refinement needs a 2-D grid", d);
        for (int s = 0; s < 4; ++s)
            if (g.bc[s] < 0 || g.bc[s] > 3) return fail(c, JANC_EINVAL, "domain %d: bad boundary kind", d);
        if ((g.bc[0] == BC_PERIODIC) != (g.bc[1] == BC_PERIODIC) ||
            (g.ny > 1 && (g.bc[2] == BC_PERIODIC) != (g.bc[3] == BC_PERIODIC)))
            return fail(c, JANC_EINVAL, "domain %d: periodic boundaries must pair", d);
        if (c->model != DETAILED && !(D.phys.gamma > 1.0))
            return fail(c, JANC_EINVAL, "domain %d: gamma must exceed 1", d);
        h.nx0 = g.nx;
        h.ny0 = g.ny;
        h.twod = g.ny > 1 ? 1 : 0;
        h.nlevels = D.nlevels;
        for (int s = 0; s < 4; ++s) {
            h.bc[s] = g.bc[s];
            h.dir[s] = -1;
            if (g.bc[s] == BC_DIRICHLET && (s < 2 || h.twod)) h.dir[s] = ndir++;
        }
        h.dx0 = g.dx;
        h.dy0 = g.dy;
        h.gamma = D.phys.gamma;
        h.R = D.phys.R;
        h.Q = D.phys.Q;
        h.Ea = D.phys.Ea;
        h.k = D.phys.k;
        h.slot0 = slot;
        slot += D.nlevels;
        lm[d].resize(D.nlevels);
        for (int l = 0; l < D.nlevels; ++l) {
            const int W = g.nx << l, H = h.twod ? (g.ny << l) : 1;
            lm[d][l].w8 = (W + 7) / 8;
            lm[d][l].h8 = (H + 7) / 8;
            lm[d][l].off = map_total;
            h.map_off[l] = map_total;
            h.map_w[l] = lm[d][l].w8;
            map_total += lm[d][l].w8 * lm[d][l].h8;
        }
        P->maxlev = std::max(P->maxlev, D.nlevels - 1);
        P->hdom.push_back(h);
    }
    P->nunits = slot;
    for (int d = 0; d < nd; ++d) P->hdom[d].cfl_slot = 2 * slot + d;
    P->hmap.assign(map_total, -1);
    // ---- blocks
    std::vector<int> count(nd * MAXL, 0);
    for (int b = 0; b < nb; ++b)
        if (blocks[b].valid) {
            if (blocks[b].domain < 0 || blocks[b].domain >= nd) return fail(c, JANC_EINVAL, "block %d: bad domain", b);
            if (blocks[b].level < 0 || blocks[b].level >= doms[blocks[b].domain].nlevels)
                return fail(c, JANC_EINVAL, "block %d: bad level", b);
            count[blocks[b].domain * MAXL + blocks[b].level]++;
        }
    for (int b = 0; b < nb; ++b) {
        const janc_block& r = blocks[b];
        if (!r.valid) continue;
        const DevDomain& D = P->hdom[r.domain];
        const int W = D.nx0 << r.level, H = D.twod ? (D.ny0 << r.level) : 1;
        if (r.nx < 1 || r.ny < 1 || r.i0 < 0 || r.j0 < 0 || r.i0 + r.nx > W || r.j0 + r.ny > H)
            return fail(c, JANC_EINVAL, "block %d outside its level", b);
        if (!D.twod && (r.ny != 1 || r.j0 != 0)) return fail(c, JANC_EINVAL, "block %d: 1-D domain blocks have ny = 1", b);
        if (r.offset < 0 || r.offset + (long long)r.nx * r.ny > pool)
            return fail(c, JANC_EINVAL, "block %d: pool range out of bounds", b);
        const bool multi = count[r.domain * MAXL + r.level] > 1;
        if (r.level > 0 || multi) {
            auto ok8 = [](int o, int n, int lim) { return (o % 8 == 0) && (n % 8 == 0 || o + n == lim); };
            if (!ok8(r.i0, r.nx, W) || (D.twod && !ok8(r.j0, r.ny, H)))
                return fail(c, JANC_EINVAL, "block %d: origin/size not multiples of 8", b);
        }
        if (r.level > 0 && (r.nx > 256 || r.ny > 256 || r.nx % 8 || r.ny % 8))
            return fail(c, JANC_EINVAL, "block %d: refined blocks need sizes multiple of 8 and <= 256", b);
        DevBlock h{};
        h.domain = r.domain;
        h.level = r.level;
        h.i0 = r.i0;
        h.j0 = r.j0;
        h.nx = r.nx;
        h.ny = r.ny;
        h.offset = r.offset;
        h.fine_child = (r.level + 1 < D.nlevels) ? 1 : 0;
        const int id = (int)P->hblk.size();
        const LevelMap& L = lm[r.domain][r.level];
        for (int y = r.j0 / 8; y < (r.j0 + r.ny + 7) / 8; ++y)
            for (int x = r.i0 / 8; x < (r.i0 + r.nx + 7) / 8; ++x) {
                int& m = P->hmap[L.off + y * L.w8 + x];
                if (m >= 0) return fail(c, JANC_EINVAL, "block %d overlaps another block", b);
                m = id;
            }
        P->hblk.push_back(h);
    }
    // pool ranges of valid blocks must not overlap
    {
        std::vector<std::pair<long long, long long>> rg;
        for (auto& h : P->hblk) rg.push_back({h.offset, h.offset + (long long)h.nx * h.ny});
        std::sort(rg.begin(), rg.end());
        for (size_t q = 1; q < rg.size(); ++q)
            if (rg[q].first < rg[q - 1].second) return fail(c, JANC_EINVAL, "blocks share pool cells");
    }
    for (int d = 0; d < nd; ++d) {
        const LevelMap& L = lm[d][0];
        for (int q = 0; q < L.w8 * L.h8; ++q)
            if (P->hmap[L.off + q] < 0) return fail(c, JANC_EINVAL, "domain %d: level 0 does not tile the domain", d);
    }
    // ---- ring masks: an 8-cell segment of a side faces uncovered in-domain cells
    auto covered = [&](int d, int l, int I8, int J8) -> int {
        const DevDomain& D = P->hdom[d];
        const LevelMap& L = lm[d][l];
        if (I8 < 0 || I8 >= L.w8) {
            if (D.bc[0] != BC_PERIODIC) return 1;
            I8 = (I8 + L.w8) % L.w8;
        }
        if (J8 < 0 || J8 >= L.h8) {
            if (D.bc[2] != BC_PERIODIC) return 1;
            J8 = (J8 + L.h8) % L.h8;
        }
        return P->hmap[L.off + J8 * L.w8 + I8] >= 0;
    };
    for (auto& h : P->hblk) {
        if (h.level == 0) continue;
        const int x8 = h.i0 / 8, y8 = h.j0 / 8, w8 = h.nx / 8, h8 = h.ny / 8;
        for (int g = 0; g < h8; ++g) {
            if (!covered(h.domain, h.level, x8 - 1, y8 + g)) h.ring[0] |= 1u << g;
            if (!covered(h.domain, h.level, x8 + w8, y8 + g)) h.ring[1] |= 1u << g;
        }
        for (int g = 0; g < w8; ++g) {
            if (!covered(h.domain, h.level, x8 + g, y8 - 1)) h.ring[2] |= 1u << g;
            if (!covered(h.domain, h.level, x8 + g, y8 + h8)) h.ring[3] |= 1u << g;
        }
    }
    // ---- proper nesting: coarse footprints of refined blocks are solved (non-ring) cells
    auto ring_cell = [](const DevBlock& B, int li, int lj) {
        return (li < 3 && ((B.ring[0] >> (lj >> 3)) & 1u)) || (li >= B.nx - 3 && ((B.ring[1] >> (lj >> 3)) & 1u)) ||
               (lj < 3 && ((B.ring[2] >> (li >> 3)) & 1u)) || (lj >= B.ny - 3 && ((B.ring[3] >> (li >> 3)) & 1u));
    };
    P->fine.assign(P->maxlev + 1, std::vector<int>());
    for (int id = 0; id < (int)P->hblk.size(); ++id) {
        const DevBlock& h = P->hblk[id];
        if (h.level == 0) continue;
        const LevelMap& L = lm[h.domain][h.level - 1];
        for (int cj = h.j0 / 2; cj < (h.j0 + h.ny) / 2; ++cj)
            for (int ci = h.i0 / 2; ci < (h.i0 + h.nx) / 2; ++ci) {
                const int pb = P->hmap[L.off + (cj >> 3) * L.w8 + (ci >> 3)];
                if (pb < 0) return fail(c, JANC_EINVAL, "refined block at (%d,%d) level %d is not nested in level %d", h.i0, h.j0, h.level, h.level - 1);
                const DevBlock& B = P->hblk[pb];
                if (B.level > 0 && ring_cell(B, ci - B.i0, cj - B.j0))
                    return fail(c, JANC_EINVAL, "refined block at (%d,%d) level %d covers coarse-fine ring cells of level %d", h.i0, h.j0, h.level, h.level - 1);
            }
        P->fine[h.level].push_back(id);
        if (h.ring[0] | h.ring[1] | h.ring[2] | h.ring[3]) {
            P->ring_blocks.push_back(id);
            for (int lj = 0; lj < h.ny; ++lj)
                for (int li = 0; li < h.nx; ++li) P->ring_cells += ring_cell(h, li, lj) ? 1 : 0;
        }
    }
    // ---- Dirichlet rows (conserved state + T), converted on the device
    P->hdir.assign((size_t)std::max(ndir, 1) * (MAXF + 1), 0.0);
    janc_status st;
    if ((st = palloc(P.get(), &P->ddir, P->hdir.size()))) return st;
    if (P->arena) {
        for (int d = 0; d < nd; ++d)
            for (int s = 0; s < 4; ++s) {
                const int row = P->hdom[d].dir[s];
                if (row < 0) continue;
                janc_plan::DirRow r{};
                r.row = row;
                r.gamma = doms[d].phys.gamma;
                r.R = doms[d].phys.R;
                r.Q = doms[d].phys.Q;
                for (int f = 0; f < nU; ++f) r.prim[f] = doms[d].grid.bc_prim[s][f];
                P->dir_rows.push_back(r);
            }
        if ((st = palloc(P.get(), &P->dir_w, (size_t)std::max(ndir, 1) * MAXF))) return st;
    } else {
        double* dW = nullptr;
        if ((st = dalloc(c, &dW, MAXF))) return st;
        for (int d = 0; d < nd; ++d)
            for (int s = 0; s < 4; ++s) {
                const int row = P->hdom[d].dir[s];
                if (row < 0) continue;
                hipError_t e = hipMemcpy(dW, doms[d].grid.bc_prim[s], sizeof(double) * nU, hipMemcpyHostToDevice);
                if (e == hipSuccess)
                    e = launch_prim_to_cons(c->model, c->ns, c->dmech, doms[d].phys.gamma, doms[d].phys.R,
                                            doms[d].phys.Q, 1, dW, P->ddir + (size_t)row * (MAXF + 1),
                                            P->ddir + (size_t)row * (MAXF + 1) + MAXF, 1, 1, nullptr);
                if (e == hipSuccess) e = hipDeviceSynchronize();
                if (e != hipSuccess) {
                    hipFree(dW);
                    return hipfail(c, e, "Dirichlet state");
                }
            }
        hipFree(dW);
    }
    P->ndom = nd;
    P->nblk = (int)P->hblk.size();
    for (const auto& h : P->hblk) P->cells += (long long)h.nx * h.ny;
    // ---- device tables and workspaces
    if ((st = pupload(P.get(), &P->ddom, P->hdom))) return st;
    if ((st = pupload(P.get(), &P->dblk, P->hblk))) return st;
    if ((st = pupload(P.get(), &P->dmap, P->hmap))) return st;
    for (int l = 0; l <= P->maxlev; ++l) {
        P->fine_off.push_back((int)P->fine_flat.size());
        P->fine_flat.insert(P->fine_flat.end(), P->fine[l].begin(), P->fine[l].end());
    }
    if ((st = pupload(P.get(), &P->dfine, P->fine_flat))) return st;
    if ((st = pupload(P.get(), &P->dring, P->ring_blocks))) return st;
    P->red_stride = 2 * P->nunits + nd;
    const int ntrip = (flags & JANC_PLAN_CROSSOVER) ? P->maxlev + 1 : 1;   // slot sets
    if ((st = palloc(P.get(), &P->dred, (size_t)RED_BUFS * ntrip * P->red_stride * SLOT_WORDS))) return st;
    if ((st = palloc(P.get(), &P->ddt, nd))) return st;
    if ((st = palloc(P.get(), &P->dstep, 1))) return st;
    if ((st = palloc(P.get(), &P->U1, (size_t)nU * pool))) return st;
    if ((st = palloc(P.get(), &P->U2, (size_t)nU * pool))) return st;
    if ((st = palloc(P.get(), &P->T1, (size_t)pool))) return st;
    if ((st = palloc(P.get(), &P->T2, (size_t)pool))) return st;
    *out = P.release();
    return JANC_OK;
}

// Tiles of every valid block for the plan's 2-D tile width (1-D blocks: 256-cell rows),
// grouped by level (the crossover advance launches one level at a time).
StageArgs base_args(janc_plan* P, const janc_time* tm, double* U, double* T, double* t,
                    double* dt_log, int cap);

// Halo source table: for every tile point outside its block or on a coarse-fine ring,
// the source resolve() gives (level map, block record, coarser level), found once per
// plan by a kernel so that the stage launches read one word per such point. Plans of
// the allocation-free entry point, plans flagged JANC_PLAN_RESOLVE_HALOS and pools of
// 2^28 cells or more (8 * cell + flags must fit an int) keep resolving in the kernel.
janc_status build_halo_table(janc_ctx* c, janc_plan* P) {
    if (P->dhsrc && !P->arena) hipFree(P->dhsrc);
    P->dhsrc = nullptr;
    P->hstride = 0;
    if (P->arena || (P->flags & JANC_PLAN_RESOLVE_HALOS) || P->pool >= (1ll << 28) || P->htiles.empty())
        return JANC_OK;
    const int stride = halo_table_stride(P->tile_w, P->kind_mask);
    int* tab = nullptr;
    if (janc_status st = dalloc(c, &tab, (size_t)P->htiles.size() * stride)) return st;
    janc_time tm{};
    tm.cfl = 1.0;
    StageArgs a = base_args(P, &tm, nullptr, nullptr, nullptr, nullptr, 0);
    hipError_t e = launch_halo_table(P->tile_w, a, tab, stride, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        hipFree(tab);
        return hipfail(c, e, "halo table");
    }
    P->dhsrc = tab;
    P->hstride = stride;
    return JANC_OK;
}

janc_status build_tiles(janc_ctx* c, janc_plan* P) {
    P->htiles.clear();
    P->tile_first.assign(P->nblk, 0);
    P->tile_count.assign(P->nblk, 0);
    P->lev_first.assign(P->maxlev + 1, 0);
    P->lev_count.assign(P->maxlev + 1, 0);
    P->kind_mask = 0;
    const int TX = P->tile_w, TY = 256 / TX;
    for (int l = 0; l <= P->maxlev; ++l) {
        P->lev_first[l] = (int)P->htiles.size();
        for (int id = 0; id < P->nblk; ++id) {
            const DevBlock& h = P->hblk[id];
            if (h.level != l) continue;
            P->tile_first[id] = (int)P->htiles.size();
            if (!P->hdom[h.domain].twod) {
                for (int x = 0; x < h.nx; x += 256) P->htiles.push_back(Tile{id, x, 0, 1});
                P->kind_mask |= 2;
            } else {
                for (int y = 0; y < h.ny; y += TY)
                    for (int x = 0; x < h.nx; x += TX) P->htiles.push_back(Tile{id, x, y, TX << 8});
                P->kind_mask |= 1;
            }
            P->tile_count[id] = (int)P->htiles.size() - P->tile_first[id];
        }
        P->lev_count[l] = (int)P->htiles.size() - P->lev_first[l];
    }
    if (P->dtiles && !P->arena) hipFree(P->dtiles);
    P->dtiles = nullptr;
    if (janc_status st = pupload(P, &P->dtiles, P->htiles)) return st;
    return build_halo_table(c, P);
}

StageArgs base_args(janc_plan* P, const janc_time* tm, double* U, double* T, double* t,
                    double* dt_log, int cap) {
    StageArgs a{};
    a.dom = P->ddom;
    a.blk = P->dblk;
    a.maps = P->dmap;
    a.tiles = P->dtiles;
    a.ntiles = (int)P->htiles.size();
    a.dirU = P->ddir;
    a.mech = P->ctx->dmech;
    a.U0 = U;
    a.pool = P->pool;
    a.red = Reduce{P->dred, P->red_stride, P->nunits, P->ndom, 0};
    a.ndom = P->ndom;
    a.dt = P->ddt;
    a.t = t;
    a.dt_log = dt_log;
    a.step = P->dstep;
    a.dt_log_cap = cap;
    a.tm = TimeArgs{tm->cfl, tm->dt_fixed, tm->t_end};
    a.strang = (tm->split == JANC_SPLIT_STRANG && P->ctx->model == DETAILED) ? 1 : 0;
    a.full_jac = (tm->jac == JANC_JAC_FULL && P->ctx->model == DETAILED) ? 1 : 0;
    a.status = P->ctx->dstatus;
    a.linear_sched = P->linear_sched;
    a.hsrc = P->dhsrc;
    a.hstride = P->hstride;
    if (P->flags & JANC_PLAN_CROSSOVER) {
        a.cross = 1;
        a.xlevels = P->maxlev + 1;
        a.xred = P->dred;
        a.Tbase = T;
    }
    return a;
}

// Level l's slot set in the crossover advance.
Reduce level_red(const janc_plan* P, const StageArgs& base, int l) {
    Reduce r = base.red;
    if (base.cross) r.buf = P->dred + (size_t)l * RED_BUFS * P->red_stride * SLOT_WORDS;
    return r;
}

// The chemistry launch of context c: the kernel specialised to the mechanism's structure
// when it is built and selected (not for the species + T Jacobian), else the generic one.
hipError_t chem_launch(janc_ctx* c, const StageArgs& a, hipStream_t s) {
    if (c->model != DETAILED || a.ntiles <= 0) return hipSuccess;
    if (c->chem_mode == JANC_CHEM_SPECIALIZED && c->chem_fn && !a.full_jac) {
        StageArgs arg = a;
        void* params[] = {&arg};
        return hipModuleLaunchKernel(c->chem_fn, (unsigned)a.ntiles, 1, 1, WG, 1, 1, 0, s, params, nullptr);
    }
    return launch_chem(c->model, c->ns, 0, a, s);
}

// The specialised reversed chemistry kernel of context c, compiled and loaded at the first
// call (outside any stream capture: it runs before the adjoint's first launch). Where it
// cannot be built the reason is kept and the generic kernel runs.
void adj_chem_prepare(janc_ctx* c) {
    if (c->adj_chem_tried || c->model != DETAILED) return;
    c->adj_chem_tried = true;
    std::vector<char> code;
    if (!chem_spec_code(adj_chem_spec_source(c->hmech), &code, &c->adj_chem_log)) return;
    if (hipModuleLoadData(&c->adj_chem_mod, code.data()) != hipSuccess ||
        hipModuleGetFunction(&c->adj_chem_fn, c->adj_chem_mod, ADJ_CHEM_SPEC_KERNEL) != hipSuccess) {
        c->adj_chem_log = "loading the specialised adjoint chemistry kernel failed";
        if (c->adj_chem_mod) hipModuleUnload(c->adj_chem_mod);
        c->adj_chem_mod = nullptr;
        c->adj_chem_fn = nullptr;
    }
}

// The adjoint chemistry launch of context c: specialised when the chemistry kernel
// selection is, and it is built; else the generic kernel.
hipError_t adj_chem_run(janc_ctx* c, const AdjChemArgs& A, hipStream_t s) {
    if (c->chem_mode == JANC_CHEM_SPECIALIZED && c->adj_chem_fn) {
        if (A.n <= 0) return hipSuccess;
        AdjChemArgs arg = A;
        void* params[] = {&arg};
        const unsigned nb = (unsigned)((A.n + AWG - 1) / AWG);
        return hipModuleLaunchKernel(c->adj_chem_fn, nb, 1, 1, AWG, 1, 1, 0, s, params, nullptr);
    }
    return adj_chem_launch(c->ns, A, s);
}

// The first half chemistry launch of a Strang-split step (in place on U, T).
hipError_t launch_chem_first_half(janc_plan* P, const StageArgs& base, const Reduce& red, double* U,
                                  double* T, int first_tile, int ntiles, int xfirst, hipStream_t s) {
    StageArgs a = base;
    a.red = red;
    a.stage = 0;
    a.Uin = U;
    a.Uout = U;
    a.Tin = T;
    a.Tout = T;
    a.tiles = P->dtiles + first_tile;
    a.ntiles = ntiles;
    a.chem_phase = 1;
    a.xfirst = xfirst;
    return chem_launch(P->ctx, a, s);
}

// One crossover step (Fig. 2a, Alg. 2): two steps of level l + 1 before each step of
// level l, deepest level first, dt_l = dt_0 / 2^l; then restriction and ring refill.
hipError_t enqueue_crossover(janc_plan* P, const StageArgs& base, double* U, double* T,
                             hipStream_t s) {
    janc_ctx* c = P->ctx;
    const int model = c->model, ns = c->ns;
    double* Uin[3] = {U, P->U1, P->U2};
    double* Uout[3] = {P->U1, P->U2, U};
    double* Tin[3] = {T, P->T1, P->T2};
    double* Tout[3] = {P->T1, P->T2, T};
    std::vector<int> done(P->maxlev + 1, 0);
    bool first = true;
    hipError_t e = hipSuccess;
    auto level_step = [&](int l) {
        const int n = P->lev_count[l];
        const bool last_of_level = done[l] == (1 << l) - 1;
        ++done[l];
        if (n == 0 || e != hipSuccess) return;
        if (base.strang) {
            e = launch_chem_first_half(P, base, level_red(P, base, l), U, T, P->lev_first[l], n,
                                       first ? 1 : 0, s);
            first = false;
        }
        for (int st = 1; st <= 3 && e == hipSuccess; ++st) {
            StageArgs a = base;
            a.red = level_red(P, base, l);
            a.stage = st;
            a.Uin = Uin[st - 1];
            a.Uout = Uout[st - 1];
            a.Tin = Tin[st - 1];
            a.Tout = Tout[st - 1];
            a.reduce_out = (st == 3 && model == DETAILED) ? 0 : 1;
            a.xfirst = (first && st == 1) ? 1 : 0;
            a.xlast = (l == 0 && st == 3 && model != DETAILED) ? 1 : 0;
            a.xskip_cov = last_of_level ? 1 : 0;
            e = launch_stage(model, ns, P->kind_mask, P->tile_w, a, P->lev_first[l], n, s);
            first = false;
        }
        if (e == hipSuccess && model == DETAILED) {
            StageArgs a = base;
            a.red = level_red(P, base, l);
            a.stage = 3;
            a.Uin = U;
            a.Uout = U;
            a.Tin = T;
            a.Tout = T;
            a.tiles = P->dtiles + P->lev_first[l];
            a.ntiles = n;
            a.xlast = (l == 0) ? 1 : 0;
            a.xskip_cov = last_of_level ? 1 : 0;
            a.chem_phase = base.strang ? 2 : 0;
            e = chem_launch(P->ctx, a, s);
        }
    };
    struct Rec {
        decltype(level_step)& step;
        int maxlev;
        void run(int l) {
            if (l < maxlev) {
                run(l + 1);
                run(l + 1);
            }
            step(l);
        }
    } rec{level_step, P->maxlev};
    rec.run(0);
    StageArgs a = base;
    a.stage = 3;
    a.Uin = U;
    a.Uout = U;
    a.Tin = T;
    a.Tout = T;
    for (int l = P->maxlev; l >= 1 && e == hipSuccess; --l) {
        a.red = level_red(P, base, l - 1);   // restricted cells enter the coarse level's maxima
        e = launch_restrict(model, ns, a, P->dfine + P->fine_off[l], (int)P->fine[l].size(), s);
    }
    if (e == hipSuccess && !P->ring_blocks.empty())
        e = launch_ring_fill(model, ns, a, P->dring, (int)P->ring_blocks.size(), s);
    return e;
}

// Enqueue one full step (3 stages, chemistry, restriction, ring refill).
hipError_t enqueue_step(janc_plan* P, const StageArgs& base, double* U, double* T, hipStream_t s) {
    if (base.cross) return enqueue_crossover(P, base, U, T, s);
    janc_ctx* c = P->ctx;
    const int model = c->model, ns = c->ns;
    double* Uin[3] = {U, P->U1, P->U2};
    double* Uout[3] = {P->U1, P->U2, U};
    double* Tin[3] = {T, P->T1, P->T2};
    double* Tout[3] = {P->T1, P->T2, T};
    hipError_t e = hipSuccess;
    if (base.strang) e = launch_chem_first_half(P, base, base.red, U, T, 0, base.ntiles, 0, s);
    for (int st = 1; st <= 3 && e == hipSuccess; ++st) {
        StageArgs a = base;
        a.stage = st;
        a.Uin = Uin[st - 1];
        a.Uout = Uout[st - 1];
        a.Tin = Tin[st - 1];
        a.Tout = Tout[st - 1];
        a.reduce_out = (st == 3 && model == DETAILED) ? 0 : 1;
        if (P->flags & JANC_PLAN_PER_BLOCK) {
            for (int id = 0; id < P->nblk && e == hipSuccess; ++id)
                e = launch_stage(model, ns, P->kind_mask, P->tile_w, a, P->tile_first[id], P->tile_count[id], s);
        } else if (P->flags & JANC_PLAN_PER_LEVEL) {
            for (int l = 0; l <= P->maxlev && e == hipSuccess; ++l)
                e = launch_stage(model, ns, P->kind_mask, P->tile_w, a, P->lev_first[l], P->lev_count[l], s);
        } else {
            e = launch_stage(model, ns, P->kind_mask, P->tile_w, a, 0, a.ntiles, s);
        }
    }
    StageArgs a = base;
    a.stage = 3;
    a.Uin = U;
    a.Uout = U;
    a.Tin = T;
    a.Tout = T;
    a.chem_phase = base.strang ? 2 : 0;
    if (e == hipSuccess && model == DETAILED) e = chem_launch(P->ctx, a, s);
    for (int l = P->maxlev; l >= 1 && e == hipSuccess; --l)
        e = launch_restrict(model, ns, a, P->dfine + P->fine_off[l], (int)P->fine[l].size(), s);
    if (e == hipSuccess && !P->ring_blocks.empty())
        e = launch_ring_fill(model, ns, a, P->dring, (int)P->ring_blocks.size(), s);
    return e;
}

// The executable graph may still be replaying on the stream of an earlier call:
// wait for its last replay before destroying it.
void drop_graph(janc_plan* P) {
    if (P->gexec && P->gdone) hipEventSynchronize(P->gdone);
    if (P->gexec) hipGraphExecDestroy(P->gexec);
    if (P->graph) hipGraphDestroy(P->graph);
    P->gexec = nullptr;
    P->graph = nullptr;
    P->have_graph = false;
}

// Autotuner of the stage launch. Candidates: the 2-D tile width 16, 32 or 64 (16 x 16,
// 32 x 8, 64 x 4 cells) times the order in which workgroups take tiles. A measurement
// is one RK stage triple of the plan on the state (U, T), timed with HIP events: stage
// 1 reads U and T, stages 2 and 3 the plan's stage buffers and U as U^(0), and every
// output goes to the plan's workspaces (the caller's arrays are only read). The
// candidates are measured in `reps` interleaved rounds, so that a clock ramp or a noisy
// interval falls on all of them, and compared by their median. The plan keeps its
// current shape unless a candidate is faster by more than KEEP_MARGIN. The linear order
// reads 2 to 3 times the HBM bytes of the XCD-contiguous order (halo rows shared by
// neighbouring tiles are fetched once per XCD L2 instead of once per tile), so a
// linear-order candidate is charged LINEAR_HANDICAP on its time. Every candidate
// computes the same result bitwise: the choice changes speed only.
constexpr double LINEAR_HANDICAP = 1.03;
constexpr double KEEP_MARGIN = 0.02;

janc_status autotune(janc_ctx* c, janc_plan* P, const janc_time* tm, double* U, double* T, int reps,
                     double* ms_out, hipStream_t s) {
    HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
    struct Cand { int w, lin; };
    std::vector<Cand> cands;
    const int widths[3] = {16, 32, 64};
    const bool twod = (P->kind_mask & 1) != 0;   // 1-D tiles only: the width does not apply
    for (int wi = 0; wi < 3; ++wi) {
        if (!twod && wi > 0) break;
        for (int lin = 0; lin < 2; ++lin) cands.push_back({widths[wi], lin});
    }
    const int w0 = P->tile_w, l0 = P->linear_sched;
    int inc = -1;   // the plan's current shape among the candidates
    for (size_t k = 0; k < cands.size(); ++k)
        if (cands[k].lin == l0 && (!twod || cands[k].w == w0)) inc = (int)k;
    hipEvent_t ev[2];
    double* tbuf = nullptr;   // t of the stage triples (advanced by the one-step models' stage 3)
    HIPCHK(c, hipEventCreate(&ev[0]), "hipEventCreate");
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        hipEventDestroy(ev[0]);
        return fail(c, JANC_EHIP, "hipEventCreate");
    }
    hipError_t e = hipMalloc((void**)&tbuf, sizeof(double) * (size_t)std::max(P->ndom, 1));
    if (e == hipSuccess) e = hipMemsetAsync(tbuf, 0, sizeof(double) * (size_t)std::max(P->ndom, 1), s);
    janc_status st = JANC_OK;
    std::vector<std::vector<float>> times(cands.size());
    for (int r = 0; r <= reps && e == hipSuccess && !st; ++r) {   // round 0: warm-up
        for (size_t k = 0; k < cands.size() && e == hipSuccess && !st; ++k) {
            if (cands[k].w != P->tile_w) {
                P->tile_w = cands[k].w;
                st = build_tiles(c, P);
                if (st) break;
            }
            P->linear_sched = cands[k].lin;
            StageArgs base = base_args(P, tm, U, T, tbuf, nullptr, 0);
            base.cross = 0;   // timed as synchronous launches over every tile
            base.red = Reduce{P->dred, P->red_stride, P->nunits, P->ndom, 0};
            base.strang = 0;
            base.tm.t_end = 0.0;   // no clipping: t is not read
            StageArgs a0 = base;
            a0.Uin = U;
            a0.Tin = T;
            a0.Tout = P->T1;   // the entry T solve writes the workspace, not the caller's T
            e = launch_zero_int(P->dstep, s);
            if (e == hipSuccess) e = launch_clear_reduce(base.red, -1, s);
            if (e == hipSuccess) e = launch_init(c->model, c->ns, P->tile_w, a0, s);
            double* Uin[3] = {U, P->U1, P->U2};
            double* Uout[3] = {P->U1, P->U2, P->U1};
            double* Tin[3] = {P->T1, P->T2, P->T1};
            double* Tout[3] = {P->T2, P->T1, P->T2};
            if (e == hipSuccess) e = hipEventRecord(ev[0], s);
            for (int sg = 1; sg <= 3 && e == hipSuccess; ++sg) {
                StageArgs a = base;
                a.stage = sg;
                a.Uin = Uin[sg - 1];
                a.Uout = Uout[sg - 1];
                a.Tin = Tin[sg - 1];
                a.Tout = Tout[sg - 1];
                a.reduce_out = (sg == 3 && c->model == DETAILED) ? 0 : 1;
                e = launch_stage(c->model, c->ns, P->kind_mask, P->tile_w, a, 0, a.ntiles, s);
            }
            if (e == hipSuccess) e = hipEventRecord(ev[1], s);
            if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
            float f = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&f, ev[0], ev[1]);
            if (e == hipSuccess && r > 0) times[k].push_back(f);
        }
    }
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
    if (tbuf) {
        hipStreamSynchronize(s);
        hipFree(tbuf);
    }
    int bw = w0, bl = l0;
    if (e == hipSuccess && !st) {
        std::vector<double> med(cands.size(), INFINITY);
        for (size_t k = 0; k < cands.size(); ++k) {
            std::sort(times[k].begin(), times[k].end());
            if (!times[k].empty()) med[k] = times[k][times[k].size() / 2];
            if (ms_out) ms_out[k] = med[k];
        }
        auto charged = [&](size_t k) { return cands[k].lin ? med[k] * LINEAR_HANDICAP : med[k]; };
        double best = (inc >= 0) ? charged((size_t)inc) * (1.0 - KEEP_MARGIN) : INFINITY;
        for (size_t k = 0; k < cands.size(); ++k) {
            if (charged(k) < best) {
                best = charged(k);
                bw = cands[k].w;
                bl = cands[k].lin;
            }
        }
    }
    if (ms_out)
        for (size_t k = cands.size(); k < 6; ++k) ms_out[k] = -1.0;
    P->linear_sched = bl;
    if (P->tile_w != bw) {
        P->tile_w = bw;
        janc_status st2 = build_tiles(c, P);
        if (!st) st = st2;
    }
    drop_graph(P);
    if (e != hipSuccess) return hipfail(c, e, "autotune");
    if (st) return st;
    P->tuned = true;
    return JANC_OK;
}

// Call entry (T re-solved from U, maxima for the first stage), then nsteps
// steps: replayed from a captured hipGraph of one step, or launched directly.
janc_status run_steps(janc_ctx* c, janc_plan* P, const janc_time* tm, double* U, double* T,
                      int nsteps, double* t, double* dt_log, hipStream_t s) {
    HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
    if ((P->flags & JANC_PLAN_AUTOTUNE) && !P->tuned && nsteps > 0) {
        janc_status st = autotune(c, P, tm, U, T, 5, nullptr, s);
        if (st) return st;
    }
    const StageArgs base = base_args(P, tm, U, T, t, dt_log, nsteps);
    HIPCHK(c, launch_zero_int(P->dstep, s), "counter launch");
    StageArgs a0 = base;
    a0.Uin = U;
    a0.Tin = T;
    a0.Tout = T;
    if (!base.cross) {
        HIPCHK(c, launch_clear_reduce(base.red, -1, s), "clear launch");
        HIPCHK(c, launch_init(c->model, c->ns, P->tile_w, a0, s), "init launch");
    } else {
        // one slot triple per level; each level's entry maxima into its buffer 0
        for (int l = 0; l <= P->maxlev; ++l) {
            a0.red = level_red(P, base, l);
            HIPCHK(c, launch_clear_reduce(a0.red, -1, s), "clear launch");
            a0.tiles = P->dtiles + P->lev_first[l];
            a0.ntiles = P->lev_count[l];
            HIPCHK(c, launch_init(c->model, c->ns, P->tile_w, a0, s), "init launch");
        }
    }
    if (nsteps == 0) return JANC_OK;
    if (P->flags & JANC_PLAN_NO_GRAPH) {
        for (int n = 0; n < nsteps; ++n) HIPCHK(c, enqueue_step(P, base, U, T, s), "step launch");
        return JANC_OK;
    }
    // the step count enters the captured launches only as the bound of dt_log
    const GraphKey key{U, T, t, dt_log, dt_log ? nsteps : 0, tm->cfl, tm->dt_fixed, tm->t_end,
                       tm->split, tm->jac, c->chem_mode};
    if (!P->have_graph || !(P->gkey == key)) {
        drop_graph(P);
        hipStream_t cs;
        HIPCHK(c, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
        if (e == hipSuccess) {
            hipError_t e2 = enqueue_step(P, base, U, T, cs);
            e = hipStreamEndCapture(cs, &P->graph);
            if (e2 != hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&P->gexec, P->graph, nullptr, nullptr, 0);
        hipStreamDestroy(cs);
        if (e != hipSuccess) {
            drop_graph(P);
            return hipfail(c, e, "graph capture");
        }
        P->gkey = key;
        P->have_graph = true;
    }
    for (int n = 0; n < nsteps; ++n) HIPCHK(c, hipGraphLaunch(P->gexec, s), "hipGraphLaunch");
    if (!P->gdone) HIPCHK(c, hipEventCreateWithFlags(&P->gdone, hipEventDisableTiming), "hipEventCreate");
    HIPCHK(c, hipEventRecord(P->gdone, s), "hipEventRecord");
    return JANC_OK;
}

// Plan of a uniform grid: one domain, one level-0 block covering it; cached.
janc_status uniform_plan(janc_ctx* c, const janc_grid* g, const janc_physics* ph) {
    if (c->uplan && std::memcmp(&c->ugrid, g, sizeof(*g)) == 0 &&
        std::memcmp(&c->uphys, ph, sizeof(*ph)) == 0)
        return JANC_OK;
    plan_free(c->uplan);
    c->uplan = nullptr;
    janc_domain D;
    D.grid = *g;
    D.phys = *ph;
    D.nlevels = 1;
    janc_block B{0, 0, 0, 0, g->nx, g->ny, 0, 1, 0};
    janc_plan* P = nullptr;
    janc_status st = build_plan(c, 1, &D, 1, &B, (long long)g->nx * g->ny, 0, &P);
    if (st) return st;
    if (g->ny > 1 && g->nx >= 64 && g->ny < 16) P->tile_w = 64;
    else if (g->ny > 1 && g->nx >= 32 && g->ny < 32) P->tile_w = 32;
    st = build_tiles(c, P);
    if (st) {
        plan_free(P);
        return st;
    }
    c->uplan = P;
    c->ugrid = *g;
    c->uphys = *ph;
    return JANC_OK;
}

// ---------------------------------------------------------------- allocation-free stepping
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch[NOALLOC_MAX_DEVICES] = {};

// Resolves (once) and returns the device address of this device's scratch array;
// the device must be current.
janc_status noalloc_scratch(janc_ctx* c, char** out) {
    *out = nullptr;
    if (c->device < 0 || c->device >= NOALLOC_MAX_DEVICES)
        return fail(c, JANC_EINVAL, "device %d beyond the %d devices of the static scratch", c->device,
                    NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[c->device]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hipfail(c, e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(c, JANC_EHIP, "hipGetSymbolAddress(scratch) returned no address");
        g_scratch[c->device] = (char*)p;
    }
    *out = g_scratch[c->device];
    return JANC_OK;
}

// Stream-ordered set-up of an arena plan before its launches: the host tables are
// copied into the scratch array and the Dirichlet rows converted there.
janc_status stage_tables(janc_ctx* c, janc_plan* P, hipStream_t s) {
    for (const auto& u : P->uploads)
        HIPCHK(c, hipMemcpyAsync(u.dst, u.src, u.bytes, hipMemcpyHostToDevice, s), "table copy");
    if (!P->dir_rows.empty()) {
        static_assert(sizeof(janc_plan::DirRow::prim) == MAXF * sizeof(double), "row layout");
        for (size_t r = 0; r < P->dir_rows.size(); ++r)
            HIPCHK(c, hipMemcpyAsync(P->dir_w + r * MAXF, P->dir_rows[r].prim, MAXF * sizeof(double),
                                     hipMemcpyHostToDevice, s), "Dirichlet copy");
        for (size_t r = 0; r < P->dir_rows.size(); ++r) {
            const janc_plan::DirRow& d = P->dir_rows[r];
            double* row = P->ddir + (size_t)d.row * (MAXF + 1);
            HIPCHK(c, launch_prim_to_cons(c->model, c->ns, c->dmech, d.gamma, d.R, d.Q, 1,
                                          P->dir_w + r * MAXF, row, row + MAXF, 1, 1, s),
                   "Dirichlet state");
        }
    }
    return JANC_OK;
}

// janc_step with every workspace in the static scratch array: the uniform plan's host
// tables are built (and cached) on the host, their device arrays are pieces of the
// scratch array, and the steps are launched directly (no graph).
janc_status run_step_noalloc(janc_ctx* c, const janc_grid* g, const janc_physics* ph,
                             const janc_time* tm, double* U, double* T, int nsteps, double* t,
                             double* dt_log, hipStream_t s) {
    HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
    char* base = nullptr;
    janc_status st = noalloc_scratch(c, &base);
    if (st) return st;
    if (!(c->nplan && std::memcmp(&c->ngrid, g, sizeof(*g)) == 0 &&
          std::memcmp(&c->nphys, ph, sizeof(*ph)) == 0)) {
        plan_free(c->nplan);
        c->nplan = nullptr;
        janc_domain D;
        D.grid = *g;
        D.phys = *ph;
        D.nlevels = 1;
        janc_block B{0, 0, 0, 0, g->nx, g->ny, 0, 1, 0};
        janc_plan* P = nullptr;
        st = build_plan(c, 1, &D, 1, &B, (long long)g->nx * g->ny, JANC_PLAN_NO_GRAPH, &P, base,
                        (size_t)JANC_NOALLOC_SCRATCH_BYTES);
        if (st) return st;
        if (g->ny > 1 && g->nx >= 64 && g->ny < 16) P->tile_w = 64;
        else if (g->ny > 1 && g->nx >= 32 && g->ny < 32) P->tile_w = 32;
        st = build_tiles(c, P);
        if (st) {
            plan_free(P);
            return st;
        }
        c->nplan = P;
        c->ngrid = *g;
        c->nphys = *ph;
    }
    st = stage_tables(c, c->nplan, s);
    if (st) return st;
    return run_steps(c, c->nplan, tm, U, T, nsteps, t, dt_log, s);
}

// ---------------------------------------------------------------- discrete adjoint
// Forward with checkpoints every k steps (and the probe loss), then segments in
// reverse: recompute the segment from its checkpoint storing every stage input (and,
// for the detailed model, each step's chemistry input with the temperatures of every
// stored state), and sweep its steps backwards: the chemistry step, then the three
// stage adjoints.
janc_status run_adjoint(janc_ctx* c, const janc_grid* g, const janc_physics* ph,
                        const janc_time* tm, const double* W0, int N, int K, int np,
                        const int* pc, const double* pw, double* loss, double* gW,
                        double* theta, hipStream_t s) {
    const int model = c->model, ns = c->ns, NU = c->nU;
    const bool det = model == DETAILED;
    if (model != ONESTEP && !det) return fail(c, JANC_EINVAL, "the adjoint covers the one-step and the detailed models");
    if (!(tm->dt_fixed > 0.0)) return fail(c, JANC_EINVAL, "the adjoint needs a fixed dt (dt_fixed > 0)");
    if (tm->t_end > 0.0) return fail(c, JANC_EINVAL, "the adjoint does not clip to t_end");
    if (det && tm->split != JANC_SPLIT_LIE)
        return fail(c, JANC_EINVAL, "the adjoint of the detailed model follows the Lie-split step");
    if (det && tm->jac != JANC_JAC_FROZEN_T)
        return fail(c, JANC_EINVAL, "the adjoint of the detailed model uses the frozen-T Jacobian");
    if (g->nx < 3 || (g->ny != 1 && g->ny < 3))
        return fail(c, JANC_EINVAL, "adjoint grid needs nx >= 3 and ny = 1 or ny >= 3");
    const long long n = (long long)g->nx * g->ny;
    if (n > (1ll << 31) - 1) return fail(c, JANC_EINVAL, "grid too large for the adjoint");
    if (det && c->chem_mode == JANC_CHEM_SPECIALIZED) adj_chem_prepare(c);
    if (np < 0 || np > JANC_MAX_PROBES) return fail(c, JANC_EINVAL, "between 0 and %d probes", JANC_MAX_PROBES);
    for (int q = 0; q < np; ++q)
        if (pc[q] < 0 || pc[q] >= n) return fail(c, JANC_EINVAL, "probe cell %d out of range", q);
    janc_status st = uniform_plan(c, g, ph);
    if (st) return st;
    janc_plan* P = c->uplan;
    HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
    const int nseg = (N + K - 1) / K;
    AdjGrid ag{};
    ag.nx = g->nx;
    ag.ny = g->ny;
    ag.twod = g->ny > 1 ? 1 : 0;
    for (int q = 0; q < 4; ++q) {
        ag.bc[q] = g->bc[q];
        ag.dir[q] = P->hdom[0].dir[q];
    }
    ag.idx = 1.0 / g->dx;
    ag.idy = 1.0 / g->dy;
    ag.gamma = ph->gamma;
    ag.R = ph->R;
    ag.Q = ph->Q;
    ag.Ea = ph->Ea;
    ag.k = ph->k;
    ag.dirU = P->ddir;
    const int nba = (int)((n + 255) / 256);          // cell blocks of the alpha kernel
    const int nbd = (int)((n + 127) / 128);          // blocks of the cell kernel (128 cells each)
    const long long nix = (long long)(g->nx + 1) * g->ny;
    const long long niy = ag.twod ? (long long)g->nx * (g->ny + 1) : 0;
    const long long nf = (long long)NU * n;          // conserved fields of a state
    const long long sn = det ? nf + n : nf;          // a stored state (+ temperatures)
    const int nsl = 3 * K;                            // stage inputs of one segment
    // workspace layout (doubles)
    struct Seg { size_t off, len; };
    size_t tot = 0;
    auto take = [&](size_t len) { Seg r{tot, len}; tot += (len + 31) & ~(size_t)31; return r; };
    // segment storage (stage inputs, chemistry inputs, alpha and argmax) twice: the
    // recompute of segment sg - 1 on the auxiliary stream overlaps the reverse sweep of sg
    Seg sS0[2], sS1[2], sS2[2], sX3[2], sApart[2], sAlpha[2], sArgm[2];
    const Seg sCk = take((size_t)nseg * sn);
    for (int b = 0; b < 2; ++b) {
        sS0[b] = take((size_t)(K + 1) * sn);
        sS1[b] = take((size_t)K * sn);
        sS2[b] = take((size_t)K * sn);
        sX3[b] = take(det ? (size_t)K * sn : 0);
        sApart[b] = take((size_t)nsl * nba * 4);
        sAlpha[b] = take(2 * (size_t)nsl);
        sArgm[b] = take((size_t)nsl);
    }
    const Seg sLam = take(nf), sLA = take(nf), sLB = take(nf), sLC = take(nf), sAcc = take(nf),
              sT0 = take(n), sT1 = take(n), sCx = take(10 * NU * nix), sCy = take(10 * NU * niy),
              sPart = take(4 * (size_t)nbd + 8), sMisc = take(16), sPc = take(np + 1),
              sPw = take(np + 1), sTerms = take((size_t)N);
    if (tot > c->adj_doubles) {
        if (c->adj_mem) hipFree(c->adj_mem);
        c->adj_mem = nullptr;
        c->adj_doubles = 0;
        if ((st = dalloc(c, &c->adj_mem, tot))) return st;
        c->adj_doubles = tot;
    }
    double* M = c->adj_mem;
    auto at = [&](const Seg& q) { return M + q.off; };
    double* ck = at(sCk);
    double* S0b[2] = {at(sS0[0]), at(sS0[1])};
    double* S1b[2] = {at(sS1[0]), at(sS1[1])};
    double* S2b[2] = {at(sS2[0]), at(sS2[1])};
    double* X3b[2] = {at(sX3[0]), at(sX3[1])};
    double* S0 = S0b[0];
    double* S1 = S1b[0];
    double* S2 = S2b[0];
    double* X3 = X3b[0];
    if (!c->adj_stream) {
        HIPCHK(c, hipStreamCreateWithFlags(&c->adj_stream, hipStreamNonBlocking), "stream");
        for (int q = 0; q < 5; ++q)
            HIPCHK(c, hipEventCreateWithFlags(&c->adj_ev[q], hipEventDisableTiming), "event");
    }
    hipStream_t s2 = c->adj_stream;
    double* lam = at(sLam);
    double* lA = at(sLA);
    double* lB = at(sLB);
    double* lC = at(sLC);
    double* acc = at(sAcc);
    double* T0 = at(sT0);
    double* T1 = at(sT1);
    double* misc = at(sMisc);
    double* terms = at(sTerms);   // loss term of every step
    int* dpc = (int*)at(sPc);
    double* dpw = at(sPw);
    if (np > 0) {
        HIPCHK(c, hipMemcpyAsync(dpc, pc, sizeof(int) * np, hipMemcpyHostToDevice, s), "probe copy");
        HIPCHK(c, hipMemcpyAsync(dpw, pw, sizeof(double) * np, hipMemcpyHostToDevice, s), "probe copy");
    }
    HIPCHK(c, hipMemsetAsync(theta, 0, 2 * sizeof(double), s), "memset");
    HIPCHK(c, hipMemsetAsync(lam, 0, sizeof(double) * nf, s), "memset");
    // temperatures of a stored state (detailed model) or the stage scratch (one-step)
    auto Tof = [&](double* U) { return U + nf; };
    // U0 from the primitives (the one-step model's Q dependence of E0 is chained at the end)
    HIPCHK(c, launch_prim_to_cons(model, ns, c->dmech, ph->gamma, ph->R, ph->Q, n, W0, ck,
                                  det ? Tof(ck) : T0, n, n, s), "init_state");
    double* tdev = misc;   // forward time (unused by fixed dt), misc[1..] scratch
    const StageArgs base = base_args(P, tm, ck, det ? Tof(ck) : T0, tdev, nullptr, 0);
    auto entry = [&](double* U, hipStream_t q) -> hipError_t {
        hipError_t e = launch_clear_reduce(base.red, -1, q);
        if (e == hipSuccess) e = launch_zero_int(P->dstep, q);
        StageArgs a0 = base;
        a0.Uin = U;
        a0.Tin = det ? Tof(U) : T0;
        a0.Tout = det ? Tof(U) : T0;
        if (e == hipSuccess) e = launch_init(model, ns, P->tile_w, a0, q);
        return e;
    };
    auto stage = [&](int stn, double* Un, double* Uin, double* Uout, hipStream_t q) -> hipError_t {
        StageArgs a = base;
        a.stage = stn;
        a.U0 = Un;
        a.Uin = Uin;
        a.Uout = Uout;
        if (det) {
            a.Tin = Tof(Uin);
            a.Tout = Tof(Uout);
        } else {
            a.Tin = (stn == 2) ? T1 : T0;
            a.Tout = (stn == 2) ? T0 : T1;
            if (stn == 3) { a.Tin = T0; a.Tout = T1; }
            if (stn == 1) { a.Tin = T1; a.Tout = T0; }
        }
        // the detailed model's third stage leaves its maxima to the chemistry step
        a.reduce_out = (det && stn == 3) ? 0 : 1;
        return launch_stage(model, ns, P->kind_mask, P->tile_w, a, 0, a.ntiles, q);
    };
    // the chemistry step of the detailed model: from the third stage's output X into U
    auto chemistry = [&](const double* X, double* U, hipStream_t q) -> hipError_t {
        hipError_t e = hipMemcpyAsync(U, X, sizeof(double) * sn, hipMemcpyDeviceToDevice, q);
        StageArgs a = base;
        a.stage = 3;
        a.Uin = U;
        a.Uout = U;
        a.Tin = Tof(U);
        a.Tout = Tof(U);
        a.chem_phase = 0;
        if (e == hipSuccess) e = chem_launch(P->ctx, a, q);
        return e;
    };
    // one full forward step: stage inputs into o1, o2, the chemistry input into x3
    auto full_step = [&](double* u0, double* o1, double* o2, double* x3, double* nxt,
                         hipStream_t q) -> hipError_t {
        hipError_t e = stage(1, u0, u0, o1, q);
        if (e == hipSuccess) e = stage(2, u0, o1, o2, q);
        if (det) {
            if (e == hipSuccess) e = stage(3, u0, o2, x3, q);
            if (e == hipSuccess) e = chemistry(x3, nxt, q);
        } else if (e == hipSuccess) {
            e = stage(3, u0, o2, nxt, q);
        }
        return e;
    };
    const double dt = tm->dt_fixed;
    // ---- forward pass with checkpoints; the last segment keeps its stage inputs
    // (it is swept first and needs no recompute)
    const int bl = (nseg - 1) & 1, nl0 = (nseg - 1) * K, ml = N - nl0;
    double *L0 = S0b[bl], *L1 = S1b[bl], *L2 = S2b[bl], *L3 = X3b[bl];
    HIPCHK(c, entry(ck, s), "adjoint forward entry");
    if (!det) HIPCHK(c, hipMemcpyAsync(T1, T0, sizeof(double) * n, hipMemcpyDeviceToDevice, s), "copy");
    double* cur = ck;
    for (int step = 0; step < N; ++step) {
        if (step == nl0 && cur != L0) {
            HIPCHK(c, hipMemcpyAsync(L0, cur, sizeof(double) * sn, hipMemcpyDeviceToDevice, s), "copy");
            cur = L0;
        }
        const int m = step - nl0;
        double *o1 = S1, *o2 = S2, *x3 = X3, *nxt;
        if (m >= 0) {
            o1 = L1 + (size_t)m * sn;
            o2 = L2 + (size_t)m * sn;
            x3 = L3 + (size_t)m * sn;
            nxt = L0 + (size_t)(m + 1) * sn;
        } else {
            nxt = ((step + 1) % K == 0) ? ck + (size_t)((step + 1) / K) * sn : ((cur == S0) ? S0 + sn : S0);
        }
        HIPCHK(c, full_step(cur, o1, o2, x3, nxt, s), "forward step");
        cur = nxt;
    }
    // ---- reverse sweep
    AdjArgs A{};
    A.g = ag;
    A.n = n;
    A.dt = dt;
    A.mech = c->dmech;
    A.cx = at(sCx);
    A.cy = at(sCy);
    A.part = at(sPart);
    A.nbd = nbd;
    A.theta = theta;
    A.pc = dpc;
    A.pw = dpw;
    A.np = np;
    AlphaArgs AP{};
    AP.g = ag;
    AP.n = n;
    AP.mech = c->dmech;
    AP.step_stride = sn;
    AP.nbd = nba;
    HIPCHK(c, adj_seed_launch(model, ns, ag, c->dmech, cur, n, dpc, dpw, np, dt, lam, theta, s), "seed");
    hipEvent_t evFwd = c->adj_ev[0], evRec[2] = {c->adj_ev[1], c->adj_ev[2]},
               evRev[2] = {c->adj_ev[3], c->adj_ev[4]};
    bool used[2] = {false, false};
    // recompute segment sg (< nseg - 1) into buffer b (auxiliary stream), storing
    // the three stage inputs (and the chemistry input) of every step, then alpha and
    // its argmax of all of them and the segment's loss terms
    auto recompute = [&](int sg, int b) -> hipError_t {
        const int n0 = sg * K, m1 = std::min(N, n0 + K) - n0;
        double *R0 = S0b[b], *R1 = S1b[b], *R2 = S2b[b], *R3 = X3b[b];
        hipError_t e = hipSuccess;
        if (used[b]) e = hipStreamWaitEvent(s2, evRev[b], 0);   // its last reverse sweep is done
        if (e == hipSuccess)
            e = hipMemcpyAsync(R0, ck + (size_t)sg * sn, sizeof(double) * sn, hipMemcpyDeviceToDevice, s2);
        if (e == hipSuccess) e = entry(R0, s2);
        for (int m = 0; m < m1 && e == hipSuccess; ++m) {
            double* u0 = R0 + (size_t)m * sn;
            double* o1 = R1 + (size_t)m * sn;
            double* o2 = R2 + (size_t)m * sn;
            e = stage(1, u0, u0, o1, s2);
            if (e == hipSuccess) e = stage(2, u0, o1, o2, s2);
            // the last step of the segment ends at the next checkpoint: the one-step model
            // needs only its first two stage outputs, the detailed model its chemistry input
            if (e == hipSuccess && det) e = stage(3, u0, o2, R3 + (size_t)m * sn, s2);
            if (e == hipSuccess && m + 1 < m1) {
                if (det) e = chemistry(R3 + (size_t)m * sn, R0 + (size_t)(m + 1) * sn, s2);
                else e = stage(3, u0, o2, R0 + (size_t)(m + 1) * sn, s2);
            }
        }
        AlphaArgs ap = AP;
        ap.base[0] = R0;
        ap.base[1] = R1;
        ap.base[2] = R2;
        ap.nsteps = m1;
        ap.part = at(sApart[b]);
        ap.alpha = at(sAlpha[b]);
        ap.argm = (int*)at(sArgm[b]);
        if (e == hipSuccess) e = adj_alpha_launch(model, ns, ap, s2);
        // loss terms of states n0 + 1 .. n0 + m1 (the last one is the next checkpoint)
        if (e == hipSuccess)
            e = adj_loss_launch(model, ns, ag, c->dmech, R0, sn, m1, ck + (size_t)(sg + 1) * sn, n0, n,
                                dpc, dpw, np, dt, terms, s2);
        if (e == hipSuccess) e = hipEventRecord(evRec[b], s2);
        return e;
    };
    {   // the last segment: alpha of its stage inputs and its loss terms
        AlphaArgs ap = AP;
        ap.base[0] = L0;
        ap.base[1] = L1;
        ap.base[2] = L2;
        ap.nsteps = ml;
        ap.part = at(sApart[bl]);
        ap.alpha = at(sAlpha[bl]);
        ap.argm = (int*)at(sArgm[bl]);
        HIPCHK(c, adj_alpha_launch(model, ns, ap, s), "adjoint alpha");
        HIPCHK(c, adj_loss_launch(model, ns, ag, c->dmech, L0, sn, ml + 1, nullptr, nl0, n, dpc, dpw,
                                  np, dt, terms, s), "loss");
        HIPCHK(c, hipEventRecord(evRec[bl], s), "event");
    }
    HIPCHK(c, hipEventRecord(evFwd, s), "event");
    HIPCHK(c, hipStreamWaitEvent(s2, evFwd, 0), "event");
    for (int sg = nseg - 1; sg >= 0; --sg) {
        const int b = sg & 1;
        const int n0 = sg * K, m1 = std::min(N, n0 + K) - n0;
        if (sg >= 1) HIPCHK(c, recompute(sg - 1, 1 - b), "recompute");
        HIPCHK(c, hipStreamWaitEvent(s, evRec[b], 0), "event");
        double *R0 = S0b[b], *R1 = S1b[b], *R2 = S2b[b], *R3 = X3b[b];
        const double* alpha = at(sAlpha[b]);
        const int* argm = (const int*)at(sArgm[b]);
        for (int m = m1 - 1; m >= 0; --m) {
            double* lw3 = lam;
            if (det) {   // the chemistry step: U^{n+1} = C(U*), U* = the third stage's output
                AdjChemArgs ac{};
                ac.n = n;
                ac.mech = c->dmech;
                ac.Ustar = R3 + (size_t)m * sn;
                ac.Tstar = Tof(R3 + (size_t)m * sn);
                ac.lamIn = lam;
                ac.lamOut = lC;
                ac.dt = dt;
                ac.status = c->dstatus;
                HIPCHK(c, adj_chem_run(c, ac, s), "adjoint chemistry");
                lw3 = lC;
            }
            AdjArgs a3 = A;   // stage 3: W = U/3 + 2/3 (V + dt L(V)), V = U^(2)
            a3.V = R2 + (size_t)m * sn; a3.VT = det ? Tof(R2 + (size_t)m * sn) : nullptr;
            a3.lamW = lw3; a3.lamOut = lA; a3.acc = acc;
            a3.b = 2.0 / 3.0; a3.a = 1.0 / 3.0; a3.init_acc = 1; a3.add_out = 0;
            a3.alpha = alpha + 2 * (3 * m + 2); a3.argm = argm + 2 * (3 * m + 2);
            HIPCHK(c, adj_stage(model, ns, a3, s), "adjoint stage 3");
            AdjArgs a2 = A;   // stage 2: W = 3/4 U + 1/4 (V + dt L(V)), V = U^(1)
            a2.V = R1 + (size_t)m * sn; a2.VT = det ? Tof(R1 + (size_t)m * sn) : nullptr;
            a2.lamW = lA; a2.lamOut = lB; a2.acc = acc;
            a2.b = 0.25; a2.a = 0.75; a2.init_acc = 0; a2.add_out = 0;
            a2.alpha = alpha + 2 * (3 * m + 1); a2.argm = argm + 2 * (3 * m + 1);
            HIPCHK(c, adj_stage(model, ns, a2, s), "adjoint stage 2");
            AdjArgs a1 = A;   // stage 1: W = V + dt L(V), V = U^n; then the loss seed of U^n
            a1.V = R0 + (size_t)m * sn; a1.VT = det ? Tof(R0 + (size_t)m * sn) : nullptr;
            a1.lamW = lB; a1.lamOut = lA; a1.acc = acc;
            a1.b = 1.0; a1.a = 0.0; a1.init_acc = 0; a1.add_out = 1;
            a1.alpha = alpha + 2 * (3 * m); a1.argm = argm + 2 * (3 * m);
            a1.seedU = (n0 + m >= 1) ? R0 + (size_t)m * sn : nullptr;
            a1.seedT = (det && a1.seedU) ? Tof(R0 + (size_t)m * sn) : nullptr;
            HIPCHK(c, adj_stage(model, ns, a1, s), "adjoint stage 1");
            std::swap(lam, acc);
        }
        HIPCHK(c, hipEventRecord(evRev[b], s), "event");
        used[b] = true;
    }
    HIPCHK(c, adj_loss_sum_launch(terms, N, loss, s), "loss");
    // chain dL/dU0 to the primitives; the one-step model's E0 = p/(gamma-1) + rho |u|^2/2 +
    // rho Y Q adds to dL/dQ
    HIPCHK(c, adj_chain_launch(model, ns, ag, c->dmech, W0, lam, n, gW, A.part, theta, s), "chain");
    return JANC_OK;
}

// ---------------------------------------------------------------- layer update
// Candidates are generated layer by layer on the host (subregions of the new
// layer-l blocks without ring cells), flagged by the density criterion on the
// device, and the flagged ones become the layer-(l+1) blocks.
janc_status run_regrid(janc_ctx* c, janc_plan* P, const janc_regrid_params* rp, const double* U,
                       janc_block* out, int cap, int* nout, long long* pool_out, hipStream_t s) {
    if (!(rp->threshold >= 0.0) || rp->buffer < 0 || rp->buffer > 4096 || rp->sub < 4 ||
        rp->sub > 128 || rp->sub % 4)
        return fail(c, JANC_EINVAL,
                    "regrid: need threshold >= 0, 0 <= buffer <= 4096, sub a multiple of 4 in 4..128");
    HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
    const int sub = rp->sub;
    std::vector<janc_block> nb;
    for (const DevBlock& h : P->hblk)
        if (h.level == 0) {
            if (P->hdom[h.domain].nlevels > 1 && (h.nx % 4 || h.ny % 4))
                return fail(c, JANC_EINVAL, "regrid: level-0 block sizes must be multiples of 4 in refined domains");
            nb.push_back(janc_block{h.domain, 0, h.i0, h.j0, h.nx, h.ny, 0, 1, 0});
        }
    janc_time tm0{};
    tm0.cfl = 1.0;
    StageArgs a = base_args(P, &tm0, const_cast<double*>(U), nullptr, nullptr, nullptr, 0);
    a.Uin = U;
    RegridCand* dc = nullptr;
    int* df = nullptr;
    size_t dcap = 0;
    auto release = [&]() {
        if (dc) hipFree(dc);
        if (df) hipFree(df);
        dc = nullptr;
        df = nullptr;
    };
    for (int l = 0; l < P->maxlev; ++l) {
        // 8x8-cell coverage of the new layer l, for its ring cells
        std::vector<std::vector<int>> tmap(P->ndom);
        std::vector<int> w8(P->ndom), h8(P->ndom);
        for (int d = 0; d < P->ndom; ++d) {
            const DevDomain& D = P->hdom[d];
            w8[d] = ((D.nx0 << l) + 7) / 8;
            h8[d] = ((D.twod ? (D.ny0 << l) : 1) + 7) / 8;
            tmap[d].assign((size_t)w8[d] * h8[d], 0);
        }
        for (const janc_block& r : nb)
            if (r.level == l)
                for (int y = r.j0 / 8; y < (r.j0 + r.ny + 7) / 8; ++y)
                    for (int x = r.i0 / 8; x < (r.i0 + r.nx + 7) / 8; ++x) tmap[r.domain][(size_t)y * w8[r.domain] + x] = 1;
        auto covered = [&](int d, int x, int y) -> bool {
            const DevDomain& D = P->hdom[d];
            if (x < 0 || x >= w8[d]) {
                if (D.bc[0] != BC_PERIODIC) return true;
                x = (x + w8[d]) % w8[d];
            }
            if (y < 0 || y >= h8[d]) {
                if (D.bc[2] != BC_PERIODIC) return true;
                y = (y + h8[d]) % h8[d];
            }
            return tmap[d][(size_t)y * w8[d] + x] != 0;
        };
        auto ring_cell = [&](const janc_block& r, int li, int lj) -> bool {
            if (r.level == 0) return false;
            const int d = r.domain, x8 = r.i0 / 8, y8 = r.j0 / 8;
            return (li < 3 && !covered(d, x8 - 1, y8 + lj / 8)) ||
                   (li >= r.nx - 3 && !covered(d, x8 + r.nx / 8, y8 + lj / 8)) ||
                   (lj < 3 && !covered(d, x8 + li / 8, y8 - 1)) ||
                   (lj >= r.ny - 3 && !covered(d, x8 + li / 8, y8 + r.ny / 8));
        };
        std::vector<RegridCand> cand;
        for (size_t b = 0; b < nb.size(); ++b) {
            const janc_block r = nb[b];
            if (r.level != l || l + 1 >= P->hdom[r.domain].nlevels) continue;
            for (int y0 = 0; y0 < r.ny; y0 += sub)
                for (int x0 = 0; x0 < r.nx; x0 += sub) {
                    const int w = std::min(sub, r.nx - x0), h = std::min(sub, r.ny - y0);
                    bool ring = false;
                    for (int lj = y0; lj < y0 + h && !ring; ++lj)
                        for (int li = x0; li < x0 + w && !ring; ++li) ring = ring_cell(r, li, lj);
                    if (!ring) cand.push_back(RegridCand{r.domain, r.i0 + x0, r.j0 + y0, w, h, 0});
                }
        }
        if (cand.empty()) continue;
        if (cand.size() > dcap) {
            release();
            dcap = cand.size();
            janc_status st = dalloc(c, &dc, dcap);
            if (!st) st = dalloc(c, &df, dcap);
            if (st) {
                release();
                return st;
            }
        }
        std::vector<int> flags(cand.size());
        hipError_t e = hipMemcpyAsync(dc, cand.data(), sizeof(RegridCand) * cand.size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = launch_regrid_flag(a, dc, (int)cand.size(), l, rp->buffer, rp->threshold, df, s);
        if (e == hipSuccess) e = hipMemcpyAsync(flags.data(), df, sizeof(int) * cand.size(), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            release();
            return hipfail(c, e, "regrid flags");
        }
        for (size_t k = 0; k < cand.size(); ++k)
            if (flags[k])
                nb.push_back(janc_block{cand[k].domain, l + 1, 2 * cand[k].i0, 2 * cand[k].j0,
                                        2 * cand[k].w, 2 * cand[k].h, 0, 1, 0});
    }
    release();
    long long off = 0;
    for (janc_block& r : nb) {
        r.offset = off;
        off += (long long)r.nx * r.ny;
    }
    *nout = (int)nb.size();
    *pool_out = off;
    if ((int)nb.size() > cap) return fail(c, JANC_EINVAL, "regrid: the new table has %d blocks (capacity %d)", (int)nb.size(), cap);
    std::copy(nb.begin(), nb.end(), out);
    return JANC_OK;
}

janc_status run_regrid_fill(janc_ctx* c, janc_plan* Po, const double* Uo, const double* To,
                            janc_plan* Pn, double* Un, double* Tn, hipStream_t s) {
    if (Po->ndom != Pn->ndom) return fail(c, JANC_EINVAL, "regrid fill: plans of different domains");
    for (int d = 0; d < Po->ndom; ++d) {
        const DevDomain &A = Po->hdom[d], &B = Pn->hdom[d];
        if (A.nx0 != B.nx0 || A.ny0 != B.ny0 || A.nlevels != B.nlevels || A.twod != B.twod)
            return fail(c, JANC_EINVAL, "regrid fill: plans of different domains");
    }
    HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
    std::map<std::array<int, 6>, long long> old;
    for (const DevBlock& h : Po->hblk) old[{h.domain, h.level, h.i0, h.j0, h.nx, h.ny}] = h.offset;
    std::vector<std::vector<RegridFill>> jobs(Pn->maxlev + 1);
    for (int id = 0; id < (int)Pn->hblk.size(); ++id) {
        const DevBlock& h = Pn->hblk[id];
        auto it = old.find({h.domain, h.level, h.i0, h.j0, h.nx, h.ny});
        const long long src = (it == old.end()) ? -1 : it->second;
        if (src < 0 && h.level == 0) return fail(c, JANC_EINVAL, "regrid fill: level-0 block %d is not in the old plan", id);
        jobs[h.level].push_back(RegridFill{id, 0, src});
    }
    janc_time tm0{};
    tm0.cfl = 1.0;
    StageArgs a = base_args(Pn, &tm0, Un, Tn, nullptr, nullptr, 0);
    a.Uin = Uo;
    a.Tin = To;
    a.Uout = Un;
    a.Tout = Tn;
    RegridFill* dj = nullptr;
    janc_status st = dalloc(c, &dj, Pn->hblk.size());
    if (st) return st;
    std::vector<RegridFill> all;
    for (auto& v : jobs) all.insert(all.end(), v.begin(), v.end());
    const int nu = n_fields(c->model, c->ns);
    hipError_t e = hipMemcpyAsync(dj, all.data(), sizeof(RegridFill) * all.size(), hipMemcpyHostToDevice, s);
    size_t first = 0;
    for (int l = 0; l <= Pn->maxlev && e == hipSuccess; ++l) {   // coarser layers first
        e = launch_regrid_fill(a, dj + first, (int)jobs[l].size(), Po->pool, nu, s);
        first += jobs[l].size();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(dj);
    if (e != hipSuccess) return hipfail(c, e, "regrid fill");
    return JANC_OK;
}

}  // namespace

// =============================================================== C ABI
extern "C" {

janc_status janc_create(janc_ctx** out, int model, const janc_mech* mech, int device) {
    if (!out) return JANC_EINVAL;
    *out = nullptr;
    std::unique_ptr<janc_ctx> c(new janc_ctx());
    if (model < CPG || model > DETAILED) return JANC_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return JANC_EHIP;
    if (hipSetDevice(device) != hipSuccess) return JANC_EHIP;
    c->device = device;
    c->model = model;
    if (model == DETAILED) {
        janc_status st = build_mech(c.get(), mech);
        if (!st) st = upload_mech(c.get());
        if (st) return st;
        c->ns = mech->ns;
        std::vector<char> code;
        if (chem_spec_code(chem_spec_source(c->hmech), &code, &c->chem_log)) {
            if (hipModuleLoadData(&c->chem_mod, code.data()) != hipSuccess ||
                hipModuleGetFunction(&c->chem_fn, c->chem_mod, CHEM_SPEC_KERNEL) != hipSuccess) {
                c->chem_log = "loading the specialised chemistry kernel failed";
                if (c->chem_mod) hipModuleUnload(c->chem_mod);
                c->chem_mod = nullptr;
                c->chem_fn = nullptr;
            } else {
                c->chem_mode = JANC_CHEM_SPECIALIZED;
            }
        }
    }
    c->nU = n_fields(model, c->ns);
    {
        char* scr = nullptr;   // the allocation-free entry point's array on this device
        if (noalloc_scratch(c.get(), &scr)) return JANC_EHIP;
    }
    if (dalloc(c.get(), &c->dstatus, 1)) return JANC_ENOMEM;
    if (hipMemset(c->dstatus, 0, sizeof(unsigned)) != hipSuccess) return JANC_EHIP;
    *out = c.release();
    return JANC_OK;
}

void janc_destroy(janc_ctx* c) {
    if (!c) return;
    hipSetDevice(c->device);
    plan_free(c->uplan);
    plan_free(c->nplan);
    if (c->dmech) hipFree(c->dmech);
    if (c->dstatus) hipFree(c->dstatus);
    if (c->adj_mem) hipFree(c->adj_mem);
    for (hipEvent_t e : c->adj_ev)
        if (e) hipEventDestroy(e);
    if (c->adj_stream) hipStreamDestroy(c->adj_stream);
    if (c->chem_mod) hipModuleUnload(c->chem_mod);
    if (c->adj_chem_mod) hipModuleUnload(c->adj_chem_mod);
    delete c;
}

const char* janc_last_error(const janc_ctx* c) { return c ? c->err.c_str() : "null context"; }

int janc_num_fields(const janc_ctx* c) { return c ? c->nU : 0; }

janc_status janc_set_chem_kernel(janc_ctx* c, int mode) {
    if (!c) return JANC_EINVAL;
    if (mode != JANC_CHEM_GENERIC && mode != JANC_CHEM_SPECIALIZED)
        return fail(c, JANC_EINVAL, "mode must be JANC_CHEM_GENERIC or JANC_CHEM_SPECIALIZED");
    if (mode == JANC_CHEM_SPECIALIZED && !c->chem_fn)
        return fail(c, JANC_EINVAL, "no specialised chemistry kernel: %s",
                    c->model != DETAILED ? "the model has no chemistry" : c->chem_log.c_str());
    c->chem_mode = mode;
    return JANC_OK;
}

janc_status janc_get_chem_kernel(const janc_ctx* c, int* mode) {
    if (!c || !mode) return JANC_EINVAL;
    *mode = c->chem_mode;
    return JANC_OK;
}

janc_status janc_chem_kernel_check(const janc_mech* mech, char* log, int log_cap) {
    janc_ctx tmp;   // host tables only
    std::string msg;
    janc_status st = build_mech(&tmp, mech);
    if (st) msg = tmp.err;
    std::vector<char> code;
    if (!st && !chem_spec_code(chem_spec_source(tmp.hmech), &code, &msg)) st = JANC_EHIP;
    if (!st && !chem_spec_code(adj_chem_spec_source(tmp.hmech), &code, &msg)) st = JANC_EHIP;
    if (log && log_cap > 0) {
        const size_t n = std::min(msg.size(), (size_t)log_cap - 1);
        std::memcpy(log, msg.data(), n);
        log[n] = '\0';
    }
    return st;
}

janc_status janc_sync_status(janc_ctx* c, void* stream) {
    if (!c) return JANC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipStreamSynchronize(s), "hipStreamSynchronize");
    unsigned st = 0;
    HIPCHK(c, hipMemcpy(&st, c->dstatus, sizeof(st), hipMemcpyDeviceToHost), "status read");
    HIPCHK(c, hipMemset(c->dstatus, 0, sizeof(unsigned)), "status clear");
    if (st & STB_NONFINITE) return fail(c, JANC_ENONFINITE, "non-finite value produced on the device");
    if (st & STB_NEWTON) return fail(c, JANC_ENEWTON, "temperature Newton did not converge");
    if (st & STB_NEGATIVE) return fail(c, JANC_ENEGATIVE, "density, pressure or temperature not positive");
    return JANC_OK;
}

janc_status janc_init_state(janc_ctx* c, const janc_physics* ph, long long n, const double* W,
                            double* U, double* T, void* stream) {
    if (!c || !ph || n < 0 || (n > 0 && (!W || !U || !T))) return fail(c, JANC_EINVAL, "bad arguments");
    hipError_t e = launch_prim_to_cons(c->model, c->ns, c->dmech, ph->gamma, ph->R, ph->Q, n, W, U, T,
                                       n, n, (hipStream_t)stream);
    if (e != hipSuccess) return hipfail(c, e, "init_state launch");
    return JANC_OK;
}

janc_status janc_plan_create(janc_ctx* c, int nd, const janc_domain* doms, int nb,
                             const janc_block* blocks, long long pool, int flags, janc_plan** out) {
    if (!c || !out) return JANC_EINVAL;
    janc_status st = build_plan(c, nd, doms, nb, blocks, pool, flags, out);
    if (st) return st;
    st = build_tiles(c, *out);
    if (st) {
        plan_free(*out);
        *out = nullptr;
    }
    return st;
}

void janc_plan_destroy(janc_plan* p) { plan_free(p); }

janc_status janc_regrid(janc_ctx* c, janc_plan* P, const janc_regrid_params* rp, const double* U,
                        janc_block* out, int cap, int* nout, long long* pool_out, void* stream) {
    if (!c || !P || !rp || !U || !nout || !pool_out || cap < 0 || (cap > 0 && !out))
        return fail(c, JANC_EINVAL, "bad arguments");
    if (P->ctx != c) return fail(c, JANC_EINVAL, "plan belongs to another context");
    return run_regrid(c, P, rp, U, out, cap, nout, pool_out, (hipStream_t)stream);
}

janc_status janc_regrid_fill(janc_ctx* c, janc_plan* Po, const double* Uo, const double* To,
                             janc_plan* Pn, double* Un, double* Tn, void* stream) {
    if (!c || !Po || !Pn || !Uo || !To || !Un || !Tn) return fail(c, JANC_EINVAL, "bad arguments");
    if (Po->ctx != c || Pn->ctx != c) return fail(c, JANC_EINVAL, "plan belongs to another context");
    return run_regrid_fill(c, Po, Uo, To, Pn, Un, Tn, (hipStream_t)stream);
}

janc_status janc_plan_stats(const janc_plan* p, long long* out) {
    if (!p || !out) return JANC_EINVAL;
    out[0] = p->cells;
    out[1] = p->ring_cells;
    out[2] = p->nblk;
    out[3] = (long long)p->htiles.size();
    return JANC_OK;
}

janc_status janc_plan_set_tile(janc_plan* p, int w) {
    if (!p) return JANC_EINVAL;
    if (w == 0) w = 16;
    if (w != 16 && w != 32 && w != 64) return fail(p->ctx, JANC_EINVAL, "tile width must be 16, 32 or 64");
    p->tile_w = w;
    drop_graph(p);
    return build_tiles(p->ctx, p);
}

janc_status janc_plan_autotune(janc_ctx* c, janc_plan* P, const janc_time* tm, const double* U,
                               const double* T, int reps, int* choice, double* ms, void* stream) {
    if (!c || !P || !tm || !U || !T || reps < 1 || reps > 1000) return fail(c, JANC_EINVAL, "bad arguments");
    if (P->ctx != c) return fail(c, JANC_EINVAL, "plan belongs to another context");
    if (P->arena) return fail(c, JANC_EINVAL, "plan of the allocation-free entry point");
    if (janc_status st = check_time(c, tm)) return st;
    janc_status st = autotune(c, P, tm, (double*)U, (double*)T, reps, ms, (hipStream_t)stream);
    if (st) return st;
    if (choice) {
        choice[0] = P->tile_w;
        choice[1] = P->linear_sched;
    }
    return JANC_OK;
}

janc_status janc_plan_set_schedule(janc_plan* p, int tile_w, int linear) {
    if (!p) return JANC_EINVAL;
    if (linear != 0 && linear != 1) return fail(p->ctx, JANC_EINVAL, "linear must be 0 or 1");
    p->linear_sched = linear;
    drop_graph(p);
    return janc_plan_set_tile(p, tile_w);
}

janc_status janc_step_blocks(janc_ctx* c, janc_plan* P, const janc_time* tm, double* U, double* T,
                             int nsteps, double* t, void* stream) {
    if (!c || !P || !tm || !U || !T || !t || nsteps < 0) return fail(c, JANC_EINVAL, "bad arguments");
    if (P->ctx != c) return fail(c, JANC_EINVAL, "plan belongs to another context");
    if (janc_status st = check_time(c, tm)) return st;
    return run_steps(c, P, tm, U, T, nsteps, t, nullptr, (hipStream_t)stream);
}

janc_status janc_step(janc_ctx* c, const janc_grid* g, const janc_physics* ph, const janc_time* tm,
                      double* U, double* T, int nsteps, double* t, double* dt_log, void* stream) {
    if (!c || !g || !ph || !tm || !U || !T || !t || nsteps < 0) return fail(c, JANC_EINVAL, "bad arguments");
    if (janc_status st = check_time(c, tm)) return st;
    janc_status st = uniform_plan(c, g, ph);
    if (st) return st;
    return run_steps(c, c->uplan, tm, U, T, nsteps, t, dt_log, (hipStream_t)stream);
}

janc_status janc_step_noalloc(janc_ctx* c, const janc_grid* g, const janc_physics* ph,
                              const janc_time* tm, double* U, double* T, int nsteps, double* t,
                              double* dt_log, void* stream) {
    if (!c || !g || !ph || !tm || !U || !T || !t || nsteps < 0) return fail(c, JANC_EINVAL, "bad arguments");
    if (janc_status st = check_time(c, tm)) return st;
    return run_step_noalloc(c, g, ph, tm, U, T, nsteps, t, dt_log, (hipStream_t)stream);
}

janc_status janc_profile_step(janc_ctx* c, janc_plan* P, const janc_time* tm, double* U,
                              double* T, double* t, double* ms, void* stream) {
    if (!c || !P || !tm || !U || !T || !t || !ms) return fail(c, JANC_EINVAL, "bad arguments");
    if (P->ctx != c) return fail(c, JANC_EINVAL, "plan belongs to another context");
    if (P->flags & JANC_PLAN_CROSSOVER)
        return fail(c, JANC_EINVAL, "per-kernel profiling times the synchronous advance");
    if (janc_status st = check_time(c, tm)) return st;
    if (tm->split != JANC_SPLIT_LIE) return fail(c, JANC_EINVAL, "per-kernel profiling times the Lie-split step");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
    const StageArgs base = base_args(P, tm, U, T, t, nullptr, 0);
    HIPCHK(c, launch_clear_reduce(base.red, -1, s), "clear launch");
    HIPCHK(c, launch_zero_int(P->dstep, s), "counter launch");
    StageArgs a0 = base;
    a0.Uin = U;
    a0.Tin = T;
    a0.Tout = T;
    HIPCHK(c, launch_init(c->model, c->ns, P->tile_w, a0, s), "init launch");
    hipEvent_t ev[7];
    for (int q = 0; q < 7; ++q) HIPCHK(c, hipEventCreate(&ev[q]), "hipEventCreate");
    const int model = c->model, ns = c->ns;
    double* Uin[3] = {U, P->U1, P->U2};
    double* Uout[3] = {P->U1, P->U2, U};
    double* Tin[3] = {T, P->T1, P->T2};
    double* Tout[3] = {P->T1, P->T2, T};
    hipError_t e = hipEventRecord(ev[0], s);
    for (int st = 1; st <= 3 && e == hipSuccess; ++st) {
        StageArgs a = base;
        a.stage = st;
        a.Uin = Uin[st - 1];
        a.Uout = Uout[st - 1];
        a.Tin = Tin[st - 1];
        a.Tout = Tout[st - 1];
        a.reduce_out = (st == 3 && model == DETAILED) ? 0 : 1;
        if (P->flags & JANC_PLAN_PER_BLOCK) {
            for (int id = 0; id < P->nblk && e == hipSuccess; ++id)
                e = launch_stage(model, ns, P->kind_mask, P->tile_w, a, P->tile_first[id], P->tile_count[id], s);
        } else {
            e = launch_stage(model, ns, P->kind_mask, P->tile_w, a, 0, a.ntiles, s);
        }
        if (e == hipSuccess) e = hipEventRecord(ev[st], s);
    }
    StageArgs a = base;
    a.stage = 3;
    a.Uin = U;
    a.Uout = U;
    a.Tin = T;
    a.Tout = T;
    if (e == hipSuccess && model == DETAILED) e = chem_launch(P->ctx, a, s);
    if (e == hipSuccess) e = hipEventRecord(ev[4], s);
    for (int l = P->maxlev; l >= 1 && e == hipSuccess; --l)
        e = launch_restrict(model, ns, a, P->dfine + P->fine_off[l], (int)P->fine[l].size(), s);
    if (e == hipSuccess) e = hipEventRecord(ev[5], s);
    if (e == hipSuccess && !P->ring_blocks.empty())
        e = launch_ring_fill(model, ns, a, P->dring, (int)P->ring_blocks.size(), s);
    if (e == hipSuccess) e = hipEventRecord(ev[6], s);
    if (e == hipSuccess) e = hipEventSynchronize(ev[6]);
    for (int q = 0; q < 6 && e == hipSuccess; ++q) {
        float f = 0.0f;
        e = hipEventElapsedTime(&f, ev[q], ev[q + 1]);
        ms[q] = f;
    }
    for (int q = 0; q < 7; ++q) hipEventDestroy(ev[q]);
    if (e != hipSuccess) return hipfail(c, e, "profile step");
    return JANC_OK;
}

janc_status janc_adjoint(janc_ctx* c, const janc_grid* g, const janc_physics* ph,
                         const janc_time* tm, const double* W0, int nsteps, int ckpt_every,
                         int nprobes, const int* probe_cell, const double* probe_w, double* loss,
                         double* dL_dW0, double* dL_dtheta, void* stream) {
    if (!c || !g || !ph || !tm || !W0 || !loss || !dL_dW0 || !dL_dtheta || nsteps < 1 ||
        ckpt_every < 1 || nprobes < 0 || (nprobes > 0 && (!probe_cell || !probe_w)))
        return fail(c, JANC_EINVAL, "bad arguments");
    if (janc_status st = check_time(c, tm)) return st;
    return run_adjoint(c, g, ph, tm, W0, nsteps, ckpt_every, nprobes, probe_cell, probe_w, loss,
                       dL_dW0, dL_dtheta, (hipStream_t)stream);
}

}  // extern "C"
