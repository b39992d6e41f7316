// eu_api.cpp -- host side of the C-ABI (include/eu.h): configuration
// checks, carving of the caller's device buffers, the launch sequences of
// the method's steps, HIP graph capture and replay, host copies.
#include "../../include/eu.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "eu_internal.hpp"
#include "eu_kset.hpp"

using namespace eu;

// state of the CFL slots (host view)
enum { CFL_ZERO = 0, CFL_READY = 1, CFL_STALE = 2 };

// Scratch of eu_conserved_totals_static, in the library's own device memory:
// the per-tile partial sums, then the per-group totals.  Every GPU the
// library runs on holds one copy until the process ends; every call on that
// GPU shares it (overlapping calls race).  In host code the name is only a
// host-side handle: kernels take the device address that
// hipGetSymbolAddress returns for the current device (scratch_addr).
constexpr int64_t STATIC_SCRATCH_DOUBLES = int64_t(1) << 19;   // 4 MiB
static __device__ __align__(256) double scratch[STATIC_SCRATCH_DOUBLES];
constexpr int STATIC_MAX_DEV = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_dev[STATIC_MAX_DEV];   // device address of scratch per device

struct eu_ctx {
    eu_config cfg;
    std::vector<int32_t> sides;
    const KSet *ks = nullptr;
    View v{};
    std::vector<Grid> grids;
    hipStream_t stream = nullptr;
    int L = 1, ngrid = 1, dim = 2, nv = 4, mode = MODE_HIER;
    int64_t nbt = 0;            // blocks of all grids
    int max_tiles = 0;
    int ngroups = 1;
    int64_t state_elems = 0;    // elements of one state array
    std::vector<int64_t> pbase; // per level: first pmax-block slot (levels 1 .. L-1)
    bool initialized = false;
    int device = 0;             // device of the caller's buffers
    double *static_scratch = nullptr;   // that device's address of scratch (nullptr: unresolved)
    int variant = 0;            // stage-kernel schedule (eu_autotune)
    int cfl_state = 0;          // CFL slots: CFL_ZERO, CFL_READY (of the current state) or CFL_STALE
    std::string err;
    // graphs of one step and of GRAPH_RUN steps, by qswap (the fused strip
    // schedules and the AMR scheme's global step alternate the state between
    // the two arrays)
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipGraphExec_t grun[2] = {nullptr, nullptr};
    hipGraphExec_t gcycle[2] = {nullptr, nullptr};   // regrid_every steps, the last regrids
    int qswap = 0;              // the current state is in the second array
    // strip lists (2D, one level)
    Strip *strips = nullptr;
    int64_t max_strips = 0;
    int nstrips = 0;
    int strip_var = -1;         // schedule whose list is on the device
    // profiling
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
    double prof_ms = 0.0;
    int64_t prof_n = 0;
};

namespace {

int set_err(eu_ctx *c, int code, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIPCHK(ctx, call)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return set_err((ctx), EU_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));     \
    } while (0)

int64_t ipow(int64_t b, int e)
{
    int64_t r = 1;
    while (e--) r *= b;
    return r;
}

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Layout of the two caller buffers.
struct Layout {
    int L, ngrid, dim, nv, mode;
    std::vector<Grid> grids;
    int64_t state_elems = 0;
    int narrays = 2;
    int64_t nbt = 0, ncoarse = 0, nslot = 0, max_tiles = 0, reg_elems = 0;
    int ncls = 1;
    int ngroups = 1;
    std::vector<int64_t> pbase;
    // scratch offsets
    size_t o_grids, o_act, o_nact, o_code, o_gmask, o_sig, o_flag, o_D, o_leaf, o_cov, o_ghost, o_fresh, o_pslot,
        o_pcnt, o_fcnt, o_cpart, o_wcnt, o_lword, o_fword, o_pbase, o_actv, o_reg, o_meta, o_smax, o_dt, o_t, o_t0, o_partial, o_cfls, o_totals, o_goff, o_gcnt, o_strips;
    int64_t max_strips = 0;
    size_t scratch = 0, state = 0;
};

int validate(const eu_config *c, std::string &why)
{
    if (!c) { why = "null config"; return EU_EINVAL; }
    if (c->dim != 2 && c->dim != 3) { why = "dim must be 2 or 3"; return EU_EINVAL; }
    if (c->precision != EU_FP64 && c->precision != EU_FP32) { why = "bad precision"; return EU_EINVAL; }
    if (!(c->gamma > 1.0)) { why = "gamma must exceed 1"; return EU_EINVAL; }
    if (!(c->hi > c->lo)) { why = "hi must exceed lo"; return EU_EINVAL; }
    if (c->bc != EU_BC_TRANSMISSIVE && c->bc != EU_BC_PERIODIC) { why = "bad bc"; return EU_EINVAL; }
    if (!(c->cfl > 0.0)) { why = "cfl must be positive"; return EU_EINVAL; }
    if (c->time_mode != EU_DT_GLOBAL && c->time_mode != EU_DT_LTS) { why = "bad time_mode"; return EU_EINVAL; }
    if (c->scheme != EU_SCHEME_MR && c->scheme != EU_SCHEME_AMR) { why = "bad scheme"; return EU_EINVAL; }
    if (c->criterion != EU_CRIT_MR && c->criterion != EU_CRIT_GRADIENT) { why = "bad criterion"; return EU_EINVAL; }
    if (c->criterion == EU_CRIT_GRADIENT && (c->n_instances > 1 || c->levels < 2)) {
        why = "the gradient criterion refines a hierarchy (levels >= 2)";
        return EU_EINVAL;
    }
    if (std::isnan(c->eps_p)) { why = "eps_p is NaN"; return EU_EINVAL; }
    if (c->eps_levels != 0 && c->eps_levels != 1) { why = "eps_levels must be 0 or 1"; return EU_EINVAL; }
    if (c->rk != EU_RK_MIDPOINT && c->rk != EU_RK_HEUN) { why = "bad rk"; return EU_EINVAL; }
    if (c->ausm_speed != EU_AUSM_MEAN && c->ausm_speed != EU_AUSM_CRITICAL) { why = "bad ausm_speed"; return EU_EINVAL; }
    if ((c->rk || c->ausm_speed) && c->scheme != EU_SCHEME_MR) {
        why = "rk and ausm_speed are variants of the MR scheme";
        return EU_EINVAL;
    }
    if (c->rk == EU_RK_HEUN && c->time_mode == EU_DT_LTS) {
        why = "local time steps use the midpoint rule";
        return EU_EINVAL;
    }
    if (c->eps_levels && c->criterion != EU_CRIT_MR) {
        why = "level-dependent thresholds apply to the MR criterion";
        return EU_EINVAL;
    }
    if (c->cfl_mode != EU_CFL_SUM && c->cfl_mode != EU_CFL_MAX) { why = "bad cfl_mode"; return EU_EINVAL; }
    if (c->regrid_every < 0) { why = "regrid_every must be >= 0"; return EU_EINVAL; }

    if (c->time_mode == EU_DT_LTS && c->n_instances > 1) { why = "a batch has no levels to step locally"; return EU_EINVAL; }
    if (c->n_instances > 1) {
        if (!c->inst_side_host) { why = "inst_side_host required for a batch"; return EU_EINVAL; }
        if (c->levels != 1) { why = "a batch holds uniform grids (levels = 1)"; return EU_EINVAL; }
        for (int i = 0; i < c->n_instances; ++i)
            if (c->inst_side_host[i] < eu::BS || c->inst_side_host[i] % eu::BS) {
                why = "instance sides must be positive multiples of 8";
                return EU_EINVAL;
            }
        for (int i = 0; i < c->n_instances; ++i)
            if (std::pow((double)c->inst_side_host[i], c->dim) >= 2147483648.0) {
                why = "every instance must have fewer than 2^31 cells";
                return EU_EINVAL;
            }
        return EU_OK;
    }
    if (c->n_instances < 0) { why = "bad n_instances"; return EU_EINVAL; }
    if (c->levels < 1 || c->levels > eu::MAXLEV) { why = "levels out of range"; return EU_EINVAL; }
    if (!is_pow2(c->n0) || c->n0 < eu::BS) { why = "n0 must be a power of two >= 8"; return EU_EINVAL; }
    if (c->levels > 1) {
        if (c->patch_min != eu::BS) { why = "patch_min must be 8"; return EU_EINVAL; }
        if (!is_pow2(c->patch_max) || c->patch_max < 8 || c->patch_max > 64) {
            why = "patch_max must be 8, 16, 32 or 64";
            return EU_EINVAL;
        }
        if ((2 * c->n0) % c->patch_max) { why = "2 n0 must be a multiple of patch_max"; return EU_EINVAL; }
        if (!(c->eta > 0.0 && c->eta <= 1.0)) { why = "eta must lie in (0, 1]"; return EU_EINVAL; }
        if (!(c->eps >= 0.0)) { why = "eps must be >= 0"; return EU_EINVAL; }
    }
    if (c->tiler != EU_TILER_BLOCKS && c->tiler != EU_TILER_BR) { why = "bad tiler"; return EU_EINVAL; }
    // the clustering runs on one wave: one lane per 8^d block of a patch_max block
    if (c->tiler == EU_TILER_BR && c->levels > 1 && ipow(c->patch_max / eu::BS, c->dim) > 64) {
        why = "the Berger-Rigoutsos tiler needs (patch_max / 8)^dim <= 64";
        return EU_EINVAL;
    }
    if (c->bc == EU_BC_PERIODIC && c->n0 < 4) { why = "periodic grids need n0 >= 4"; return EU_EINVAL; }
    // every grid must have fewer than 2^31 cells (32-bit cell indices)
    if (c->levels >= 1 && c->n0 > 0) {
        const double nf = (double)c->n0 * (double)(1LL << (c->levels - 1));
        if (std::pow(nf, c->dim) >= 2147483648.0) { why = "the finest grid must have fewer than 2^31 cells"; return EU_EINVAL; }
    }
    return EU_OK;
}

void make_layout(const eu_config *c, Layout &lay)
{
    const int D = c->dim;
    lay.dim = D;
    lay.nv = D + 2;
    const bool batch = c->n_instances > 1;
    lay.mode = batch ? MODE_BATCH : MODE_HIER;
    lay.L = batch ? 1 : c->levels;
    lay.ngrid = batch ? c->n_instances : c->levels;
    lay.grids.resize(lay.ngrid);
    int64_t off = 0, boff = 0, coff = 0;
    for (int g = 0; g < lay.ngrid; ++g) {
        Grid &G = lay.grids[g];
        G.n = batch ? c->inst_side_host[g] : (c->n0 << g);
        G.nb = G.n / eu::BS;
        G.ncell = ipow(G.n, D);
        G.off = off;
        off += lay.nv * G.ncell;
        G.boff = boff;
        boff += ipow(G.nb, D);
        G.lvl = batch ? 0 : g;
        G.fine = (!batch && g + 1 < lay.L) ? g + 1 : -1;
        G.coarse = (!batch && g >= 1) ? g - 1 : -1;
        if (!batch && g < lay.L - 1) {
            G.coff = coff;
            coff += G.ncell;
        } else {
            G.coff = -1;
        }
        G.pad = 0;
        G.dx = (c->hi - c->lo) / (double)G.n;
    }
    lay.state_elems = off;
    lay.nbt = boff;
    lay.ncoarse = coff;
    lay.max_tiles = boff;
    lay.pbase.assign(eu::MAXLEV + 1, 0);
    int64_t ns = 0;
    if (!batch && lay.L > 1) {
        for (int l = 1; l < lay.L; ++l) {
            lay.pbase[l] = ns;
            ns += ipow(lay.grids[l].n / c->patch_max, D);
        }
    }
    lay.nslot = ns;
    const int64_t R = (!batch && lay.L > 1) ? c->patch_max / eu::BS : 1;
    const int64_t nsub = ipow(R, D);
    lay.ngroups = batch ? lay.ngrid : 1;

    const size_t es = c->precision == EU_FP64 ? 8 : 4;
    const bool lts = !batch && c->time_mode == EU_DT_LTS;
    lay.narrays = lts ? 3 : 2;
    lay.state = lay.narrays * align256((size_t)lay.state_elems * es);
    // local time stepping flux registers: coarse side on levels 0 .. L-2
    // (d fields of faces per cell), fine side on levels 1 .. L-1 (two substeps)
    int64_t roff = 0;
    for (int g = 0; g < lay.ngrid; ++g) {
        Grid &G = lay.grids[g];
        G.rcoff = -1;
        G.rfoff = -1;
        if (!lts) continue;
        if (g < lay.L - 1) { G.rcoff = roff; roff += (int64_t)D * lay.nv * G.ncell; }
        if (g >= 1) { G.rfoff = roff; roff += 2 * (int64_t)D * lay.nv * G.ncell; }
    }
    lay.reg_elems = roff;

    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += align256(bytes ? bytes : 1); return r; };
    lay.o_grids = take(sizeof(Grid) * lay.ngrid);
    lay.o_act = take(lay.nbt);
    lay.o_nact = take(lay.nbt);
    lay.o_code = take(lay.nbt);
    lay.o_gmask = take(sizeof(uint32_t) * lay.nbt);
    lay.o_sig = take(lay.ncoarse);
    lay.o_flag = take(lay.ncoarse);
    lay.o_D = take(8 * lay.ncoarse);
    lay.o_leaf = take(sizeof(Tile) * lay.max_tiles);
    lay.o_cov = take(sizeof(Tile) * lay.nbt);
    lay.o_ghost = take(sizeof(Tile) * lay.nbt);
    lay.o_fresh = take(sizeof(Tile) * lay.nbt);
    lay.o_actv = take(sizeof(Tile) * lay.nbt);
    lay.o_reg = take(es * lay.reg_elems);
    lay.o_pslot = take(sizeof(int) * 7 * lay.nslot * nsub);
    lay.o_pcnt = take(sizeof(int) * lay.nslot);
    lay.o_fcnt = take(sizeof(int) * lay.nslot);
    lay.ncls = (int)std::min<int64_t>(std::max<int64_t>((lay.nbt + 255) / 256, 1), 256);
    lay.o_cpart = take(sizeof(long long) * eu::NPART * eu::MAXLEV * lay.ncls);
    lay.o_wcnt = take(sizeof(int) * 5 * lay.ncls);
    lay.o_lword = take(sizeof(unsigned long long) * 2 * lay.ncls);
    lay.o_fword = take(sizeof(unsigned long long) * std::max<int64_t>(lay.nslot, 1));
    lay.o_pbase = take(sizeof(int64_t) * (eu::MAXLEV + 1));
    lay.o_meta = take(sizeof(Meta));
    lay.o_smax = take(8 * lay.ngrid);
    lay.o_dt = take(8 * lay.ngrid);
    lay.o_t = take(8 * lay.ngrid);
    lay.o_t0 = take(8 * lay.ngrid);
    // per-tile partial totals
    lay.o_partial = take(8 * std::max<int64_t>(lay.nv * lay.max_tiles, 1));
    lay.o_cfls = take(8 * (int64_t)eu::cfl_slot(eu::CFL_STRIDE, 0));
    lay.o_totals = take(8 * lay.nv * lay.ngroups);
    lay.o_goff = take(sizeof(int) * lay.ngroups);
    lay.o_gcnt = take(sizeof(int) * lay.ngroups);
    // strip lists of the strip schedules (2D, one level): at most the count
    // of the narrowest strips with the fewest rows
    if (D == 2 && lay.L == 1) {
        const int w = eu::strip_width(true), ty = eu::strip_rows(eu::FV_STRIP0);
        for (const Grid &G : lay.grids) lay.max_strips += (int64_t)((G.n + w - 1) / w) * ((G.n + ty - 1) / ty);
    } else if (D == 3 && lay.L == 1) {
        const int w = eu::strip_width(false), ny = eu::strip3_waves(eu::FV_STRIP0);
        const int nz = eu::strip3_planes(eu::FV_STRIP0);
        for (const Grid &G : lay.grids)
            lay.max_strips += (int64_t)((G.n + w - 1) / w) * ((G.n + ny - 1) / ny) * ((G.n + nz - 1) / nz);
    }
    lay.o_strips = take(sizeof(eu::Strip) * lay.max_strips);
    lay.scratch = o;
}

template <typename P> P *at(void *base, size_t off) { return (P *)((char *)base + off); }

int sync_status(eu_ctx *c)
{
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int st = 0;
    HIPCHK(c, hipMemcpy(&st, &c->v.meta->status, sizeof(int), hipMemcpyDeviceToHost));
    if (st & 1) return set_err(c, EU_ENONPHYS, "non-physical state (rho <= 0, p <= 0 or NaN)");
    if (st & 2) return set_err(c, EU_EHIP, "flagging or work-list build: a workgroup's wait for another timed out");
    return EU_OK;
}

int check_launch(eu_ctx *c)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_err(c, EU_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    return EU_OK;
}

int64_t nblocks_grid(const eu_ctx *c, int g) { return ipow(c->grids[g].nb, c->dim); }

// Device address of scratch on device dev, resolved once per device with
// that device current (the current device is restored).
hipError_t scratch_addr(int dev, double **out)
{
    *out = nullptr;
    if (dev < 0 || dev >= STATIC_MAX_DEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = (double *)p;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

// Leaf and patch cells per level of the current hierarchy: host sums of the
// classification partials (one pair per workgroup and level).
int level_cells(eu_ctx *c, int64_t *leaf, int64_t *act)
{
    std::vector<long long> p((size_t)c->v.ncls * MAXLEV * NPART);
    HIPCHK(c, hipMemcpy(p.data(), c->v.cpart, sizeof(long long) * p.size(), hipMemcpyDeviceToHost));
    for (int l = 0; l < c->L; ++l) {
        int64_t a = 0, b = 0;
        for (int w = 0; w < c->v.ncls; ++w) {
            a += p[((size_t)w * MAXLEV + l) * NPART + 0];
            b += p[((size_t)w * MAXLEV + l) * NPART + 1];
        }
        if (leaf) leaf[l] = a;
        if (act) act[l] = b;
    }
    return EU_OK;
}

// Flagged cells per level (levels 0 .. L-2) from the per pmax-block counts
// of the last flagging.
int level_flags(eu_ctx *c, int64_t *nflag)
{
    std::vector<int> f((size_t)c->v.nslot);
    if (!f.empty()) HIPCHK(c, hipMemcpy(f.data(), c->v.fcnt, sizeof(int) * f.size(), hipMemcpyDeviceToHost));
    for (int l = 0; l < c->L; ++l) nflag[l] = 0;
    for (int l = 1; l < c->L; ++l)
        for (int64_t s = c->pbase[l]; s < (l + 1 < c->L ? c->pbase[l + 1] : c->v.nslot); ++s) nflag[l - 1] += f[(size_t)s];
    return EU_OK;
}

// ---- launch sequences ------------------------------------------------------

// Projection of every covered cell, finest level first: in 2D two levels
// per launch (three make the coarsest items of a launch its long pole), in
// 3D one.  fine_done: the stage kernel has projected
// level L-2 (2D).  In 2D the last launch can also fill the ghost cells of
// every level (ghosts) or compute the MR details (details), projecting the
// values of the levels it projects itself where they are read (not both:
// the details read ghost cells the fill writes).  Returns whether it did the
// extra work.
bool seq_restrict(eu_ctx *c, int arr, bool ghosts = false, bool details = false, bool fine_done = false)
{
    if (ghosts && details) ghosts = details = false;
    if (c->dim == 2) {
        const int top = c->L - 2 - (fine_done ? 1 : 0);   // levels 0 .. top left to project
        if (top < 0) return false;
        int64_t ndet = 0;
        if (details)
            for (int l = 0; l < c->L - 1; ++l) ndet += c->grids[l].ncell;
        constexpr int GROUP = 2;   // levels per launch
        for (int hi = top; hi >= 0; hi -= GROUP) {
            const int lo = std::max(0, hi - GROUP + 1), nlev = hi - lo + 1;
            const bool last = lo == 0;
            int64_t nbl = 0;
            for (int k = lo; k <= hi; ++k) nbl += nblocks_grid(c, k);
            // a block two levels deep is four work items (one per field)
            int64_t nb = nbl + (nlev == 2 ? 3 * nblocks_grid(c, lo) : 0);
            if (last && ghosts) nb += c->nbt;
            if (last && details) {
                // 8x8 blocks of the levels projected here, 64-cell chunks of the rest
                int64_t fine = ndet;
                for (int k = 0; k <= hi; ++k) fine -= c->grids[k].ncell;
                nb += nbl + (fine + 63) / 64;
            }
            c->ks->restrict2(c->v, arr, lo, nlev, last && ghosts ? 1 : 0, last ? ndet : 0,
                             (int)std::min<int64_t>(nb, INT32_MAX), c->stream);
        }
        return ghosts || details;
    }
    for (int l = c->L - 2; l >= 0; --l)
        c->ks->restrict_cov(c->v, arr, l, (int)nblocks_grid(c, l), c->stream);
    return false;
}

void seq_ghost(eu_ctx *c, int arr)
{
    if (c->L > 1) c->ks->predict(c->v, arr, 0, 1, 1, 0.0, 0, (int)(c->nbt), c->stream);
}

// CFL slots cleared (a fill kernel: graph-safe)
void cfl_zero(eu_ctx *c)
{
    launch_fill_u8((uint8_t *)c->v.cfls, 8 * (int64_t)cfl_slot(CFL_STRIDE, 0), 0, c->stream);
    if (c->mode == MODE_BATCH) launch_fill_u8((uint8_t *)c->v.smax, 8 * (int64_t)c->ngrid, 0, c->stream);
    c->cfl_state = CFL_ZERO;
}
// CFL slots of the current state: left by the last regrid when the state
// has not changed since, else a reduction over the leaves into zero slots
// (the reduction kernel clears them after reading)
void cfl_ready(eu_ctx *c)
{
    if (c->cfl_state == CFL_READY) return;
    if (c->cfl_state == CFL_STALE) cfl_zero(c);
    c->ks->cfl_slots(c->v, c->max_tiles, c->stream);
    c->cfl_state = CFL_READY;
}
// The state changed: slots that held its partials are stale.
void cfl_stale(eu_ctx *c)
{
    if (c->cfl_state == CFL_READY) c->cfl_state = CFL_STALE;
}

// dt of the step from the CFL slots (one-wave reduction kernel, which clears
// them), or per instance from the batch's maxima (also cleared)
void seq_cfl(eu_ctx *c)
{
    cfl_ready(c);
    launch_cfl_final(c->v, c->stream);
    c->cfl_state = CFL_ZERO;
}

void prof_begin(eu_ctx *c, hipEvent_t *a)
{
    *a = nullptr;
    if (!c->prof) return;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return; }
    (void)hipEventRecord(e0, c->stream);
    c->ev_pending.push_back({e0, e1});
    *a = e1;
}

void prof_end(eu_ctx *c, hipEvent_t e1)
{
    if (e1) (void)hipEventRecord(e1, c->stream);
}

// One step of the FV scheme on every leaf (two stages), each stage followed
// by the projection; after the second, the ghost fill (ghost_after) or the MR
// details (details), folded into the last projection launch where it can.
void seq_details(eu_ctx *c);
void seq_fv_step(eu_ctx *c, bool ghost_after, bool details = false)
{
    if (c->cfg.scheme == EU_SCHEME_AMR && !strip_variant(c->variant)) {
        // the AMR scheme on the tile kernel (2D hierarchy or uniform grid):
        // one Hancock launch (Q -> Qs; the finest tiles also project onto
        // level L-2), the state moves to the other array, the projection
        // and the ghost fill (the refinement analysis reads ghost cells),
        // then the details
        hipEvent_t e;
        const bool fine = c->dim == 2 && c->L >= 2;
        prof_begin(c, &e);
        c->ks->hancock_tile(c->v, c->variant, fine ? 1 : 0, c->state_elems, c->max_tiles, -1, 0, 0, c->stream);
        prof_end(c, e);
        std::swap(c->v.Q, c->v.Qs);
        c->qswap ^= 1;
        if (c->L >= 2 && !seq_restrict(c, ARR_Q, true, false, fine)) seq_ghost(c, ARR_Q);
        if (details) seq_details(c);
        return;
    }
    if (strip_variant(c->variant)) {
        // one 2D level (uniform grid or batch): no projection, ghost fill or
        // details; the fused form and the AMR scheme leave the new state in
        // the other array; the launch that writes the new state leaves its
        // CFL partials
        hipEvent_t e;
        if (c->cfl_state != CFL_ZERO) cfl_zero(c);
        if (c->dim == 3) {
            const int wv = strip3_waves(c->variant);
            prof_begin(c, &e);
            c->ks->fv_strip3(c->v, wv, 1, 0, c->strips, c->nstrips, c->v.Q, c->v.Q, c->v.Qs, 0.5, c->stream);
            prof_end(c, e);
            prof_begin(c, &e);
            c->ks->fv_strip3(c->v, wv, 0, 1, c->strips, c->nstrips, c->v.Qs, c->v.Q, c->v.Q, 1.0, c->stream);
            prof_end(c, e);
        } else if (c->cfg.scheme == EU_SCHEME_AMR) {
            prof_begin(c, &e);
            c->ks->hancock_strip(c->v, 1, c->strips, c->nstrips, c->v.Q, c->v.Qs, c->stream);
            prof_end(c, e);
            std::swap(c->v.Q, c->v.Qs);
            c->qswap ^= 1;
        } else if (strip_fused(c->variant)) {
            prof_begin(c, &e);
            c->ks->fv_strip(c->v, 1, 0, 1, c->strips, c->nstrips, c->v.Q, c->v.Q, c->v.Qs, 1.0, c->stream);
            prof_end(c, e);
            std::swap(c->v.Q, c->v.Qs);
            c->qswap ^= 1;
        } else {
            prof_begin(c, &e);
            c->ks->fv_strip(c->v, 0, 1, 0, c->strips, c->nstrips, c->v.Q, c->v.Q, c->v.Qs, 0.5, c->stream);
            prof_end(c, e);
            prof_begin(c, &e);
            c->ks->fv_strip(c->v, 0, 0, 1, c->strips, c->nstrips, c->v.Qs, c->v.Q, c->v.Q, 1.0, c->stream);
            prof_end(c, e);
        }
        c->cfl_state = CFL_READY;
        return;
    }
    // 2D hierarchy: the stage kernel also projects its finest tiles onto
    // level L-2
    const bool fine = c->dim == 2 && c->mode == MODE_HIER && c->L >= 2;
    hipEvent_t e;
    prof_begin(c, &e);
    c->ks->fv_stage(c->v, 1, -1, 0, 0, c->max_tiles, c->variant, fine ? 1 : 0, c->stream);
    prof_end(c, e);
    if (!seq_restrict(c, ARR_QS, true, false, fine)) seq_ghost(c, ARR_QS);
    prof_begin(c, &e);
    c->ks->fv_stage(c->v, 2, -1, 0, 0, c->max_tiles, c->variant, fine ? 1 : 0, c->stream);
    prof_end(c, e);
    if (!seq_restrict(c, ARR_Q, ghost_after, details, fine)) {
        if (ghost_after) seq_ghost(c, ARR_Q);
        if (details) seq_details(c);
    }
}

// The refinement analysis of levels 0 .. L-2: MR details, or the gradient
// indicators (which read ghost cells: the caller fills them first).
void seq_details(eu_ctx *c)
{
    if (c->L < 2) return;
    int64_t n = 0;
    for (int l = 0; l < c->L - 1; ++l) n += c->grids[l].ncell;
    if (c->v.crit == EU_CRIT_GRADIENT) c->ks->gradient(c->v, n, c->stream);
    else c->ks->details(c->v, n, c->stream);
}

// Prediction launches of a regrid, coarse to fine, two levels per launch:
// the first level and the level count of launch i, and its block bound.
int predict_launches(const eu_ctx *c, int *lvl, int *nlev, int64_t *maxb)
{
    int n = 0;
    for (int l = 1; l < c->L; l += 2, ++n) {
        lvl[n] = l;
        nlev[n] = l + 1 < c->L ? 2 : 1;
        maxb[n] = nblocks_grid(c, l) + (nlev[n] == 2 ? nblocks_grid(c, l + 1) : 0);
    }
    return n;
}

// Whether a step (with regrid) leaves the CFL slots of the next one: the
// last prediction launch of the regrid of a hierarchy of two levels or more.
bool step_leaves_slots(const eu_ctx *c)
{
    return (c->mode == MODE_HIER && c->L >= 2) || strip_variant(c->variant);
}

// flags, closure and tiling (finest first), lists, then either the
// prediction of new cells and ghost cells (coarse to fine, two levels per
// launch; the last launch also leaves the CFL partials of the new state) or
// the ghost fill alone.
void seq_flag_tile(eu_ctx *c, bool prolong)
{
    if (flag_chain_ok(c->v)) {
        int wg0[MAXLEV], total = 0, nseg = 0;
        for (int l = c->L - 2; l >= 0; --l) {
            wg0[nseg++] = total;
            total += (int)ipow(c->grids[l + 1].n / c->cfg.patch_max, c->dim);
        }
        // the list build joins the launch when one launch can build them
        const bool lists = flag_chain_lists(c->v, c->nbt);
        launch_flag_chain(c->v, wg0, nseg, total, c->nbt, lists, c->stream);
        if (!lists) launch_build_lists(c->v, c->nbt, c->stream);
    } else {
        for (int l = c->L - 2; l >= 0; --l) {
            const int nbp = c->grids[l + 1].n / c->cfg.patch_max;
            launch_flag_tile(c->v, l, (int)ipow(nbp, c->dim), c->stream);
        }
        launch_build_lists(c->v, c->nbt, c->stream);
    }
    cfl_stale(c);
    if (prolong) {
        int lvl[MAXLEV], nlev[MAXLEV];
        int64_t maxb[MAXLEV];
        const int n = predict_launches(c, lvl, nlev, maxb);
        for (int i = 0; i < n; ++i) {
            const int fuse = i == n - 1 && c->mode == MODE_HIER ? 1 : 0;
            // the last launch adds into the CFL slots: they must be zero
            if (fuse && c->cfl_state != CFL_ZERO) cfl_zero(c);
            c->ks->predict(c->v, ARR_Q, lvl[i], nlev[i], 3, 0.0, fuse,
                           (int)std::min<int64_t>(maxb[i], INT32_MAX), c->stream);
            if (fuse) c->cfl_state = CFL_READY;
        }
    } else {
        seq_ghost(c, ARR_Q);
    }
}

// Local time stepping: advance level l by one of its steps (substep k of
// its parent's step): keep its start state, two stages on its patches (the
// second-stage ghost cells interpolated in time at the stage time), then two
// substeps of level l+1 with time-interpolated ghost cells, projection of
// level l+1 onto level l, and the flux correction.
void lts_advance(eu_ctx *c, int l, int k)
{
    const int nbl = (int)nblocks_grid(c, l);
    hipEvent_t e;
    c->ks->copy_level(c->v, l, nbl, 0, c->stream);
    if (c->cfg.scheme == EU_SCHEME_AMR) {
        // the AMR scheme: one Hancock step of the level's patches into the
        // stage array (fluxes recorded), copied back
        prof_begin(c, &e);
        c->ks->hancock_tile(c->v, c->variant, 0, c->state_elems, nbl, l, k, 1, c->stream);
        prof_end(c, e);
        c->ks->copy_level(c->v, l, nbl, 1, c->stream);
    } else {
        prof_begin(c, &e);
        c->ks->fv_stage(c->v, 1, l, k, 0, nbl, c->variant, 0, c->stream);
        prof_end(c, e);
        if (l >= 1) c->ks->predict(c->v, ARR_QS, l, 1, 2, (double)(2 * k + 1) * 0.25, 0, nbl, c->stream);
        prof_begin(c, &e);
        c->ks->fv_stage(c->v, 2, l, k, 1, nbl, c->variant, 0, c->stream);
        prof_end(c, e);
    }
    if (l + 1 < c->L) {
        const int nbf = (int)nblocks_grid(c, l + 1);
        for (int kk = 0; kk < 2; ++kk) {
            c->ks->predict(c->v, ARR_Q, l + 1, 1, 2, (double)kk * 0.5, 0, nbf, c->stream);
            lts_advance(c, l + 1, kk);
        }
        c->ks->restrict_cov(c->v, ARR_Q, l, nbl, c->stream);
        c->ks->reflux(c->v, l, nbl, c->stream);
    }
}

void seq_step(eu_ctx *c, bool regrid)
{
    const bool rg = regrid && c->L > 1;
    seq_cfl(c);
    const bool grad = c->v.crit == EU_CRIT_GRADIENT;
    if (c->v.lts) {
        lts_advance(c, 0, 0);
        if (rg) {
            if (grad) seq_ghost(c, ARR_Q);
            seq_details(c);
            seq_flag_tile(c, true);
        } else {
            seq_ghost(c, ARR_Q);
        }
        return;
    }
    if (grad && rg) {
        // the indicators read ghost cells: the last projection fills them
        seq_fv_step(c, true, false);
        seq_details(c);
    } else {
        seq_fv_step(c, !rg, rg);
    }
    if (rg) seq_flag_tile(c, true);
}

int upload(eu_ctx *c, void *dst, const void *src, size_t bytes)
{
    HIPCHK(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return EU_OK;
}

void drop_graphs(eu_ctx *c)
{
    for (auto &g : c->gexec)
        if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
    for (auto &g : c->grun)
        if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
    for (auto &g : c->gcycle)
        if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
}

// Whether schedule var applies to this context: the strip schedules need a
// 2D grid of one level (a uniform grid or a batch), the fused ones outflow
// boundaries; the AMR scheme runs the Hancock tile kernel (schedules 0-2)
// on hierarchies and uniform grids, the Hancock strips (6, 7) on uniform
// grids and batches.
bool variant_ok(const eu_ctx *c, int var)
{
    if (var < 0 || var >= FV_VARIANTS) return false;
    if (c->cfg.scheme == EU_SCHEME_AMR) {
        const bool tile = var < hancock_tile_variants(c->dim);
        const bool strip = c->dim == 2 && strip_variant(var) && !strip_fused(var);
        return c->mode == MODE_BATCH ? strip : c->L > 1 || c->v.lts ? tile : tile || strip;
    }
    if (!strip_variant(var)) return true;
    if (c->L != 1) return false;
    if (c->v.rk || c->v.ausm_cs) return false;   // the variants run on the tile kernel
    if (c->dim == 3) return true;
    return !strip_fused(var) || c->cfg.bc == EU_BC_TRANSMISSIVE;
}

// The strip list of schedule var on the device (a synchronous upload; not
// during capture).  Strips of one grid in column-major order, so list
// neighbours share their halo rows.
int strips_for(eu_ctx *c, int var)
{
    if (!strip_variant(var) || c->strip_var == var) return EU_OK;
    const bool fused = c->dim == 2 && strip_fused(var);
    const int w = strip_width(fused), h = strip_halo(fused), ty = strip_rows(var);
    std::vector<Strip> st;
    for (int g = 0; g < c->ngrid; ++g) {
        const int n = c->grids[g].n;
        if (c->dim == 3) {
            // planes outermost, then columns, rows innermost: list neighbours
            // share their halo rows
            const int ny = strip3_waves(var), tz = strip3_planes(var);
            for (int z0 = 0; z0 < n; z0 += tz)
                for (int x0 = 0; x0 < n; x0 += w)
                    for (int y0 = 0; y0 < n; y0 += ny)
                        st.push_back(Strip{g, x0 - h, y0, std::min(ny, n - y0), z0, std::min(tz, n - z0)});
            continue;
        }
        for (int x0 = 0; x0 < n; x0 += w)
            for (int y0 = 0; y0 < n; y0 += ty) st.push_back(Strip{g, x0 - h, y0, std::min(ty, n - y0), 0, 1});
    }
    if ((int64_t)st.size() > c->max_strips) return set_err(c, EU_EHIP, "strip list exceeds its capacity");
    int r = upload(c, c->strips, st.data(), sizeof(Strip) * st.size());
    if (r) return r;
    c->nstrips = (int)st.size();
    c->strip_var = var;
    return EU_OK;
}

// The finite-volume work of one step over the current state, without
// changing it (the state Q is read; the stage array receives the results,
// and every step recomputes it): a global step's two stages (the second in
// its form reading Q: the same loads, arithmetic and stores), or both fused;
// with local time stepping the first stage of every level.  The strip list
// of var must be on the device.  Sets the cell-stages and launches of a pass.
void fv_pass(eu_ctx *c, int var, int *launches)
{
    if (c->v.lts) {
        for (int l = 0; l < c->L; ++l) {
            if (c->cfg.scheme == EU_SCHEME_AMR)
                c->ks->hancock_tile(c->v, var, 0, c->state_elems, (int)nblocks_grid(c, l), l, 0, 0, c->stream);
            else
                c->ks->fv_stage(c->v, 1, l, 0, 0, (int)nblocks_grid(c, l), var, 0, c->stream);
        }
        *launches = c->L;
    } else if (strip_variant(var) && c->dim == 3) {
        const int wv = strip3_waves(var);
        c->ks->fv_strip3(c->v, wv, 1, 0, c->strips, c->nstrips, c->v.Q, c->v.Q, c->v.Qs, 0.5, c->stream);
        c->ks->fv_strip3(c->v, wv, 0, 2, c->strips, c->nstrips, c->v.Q, c->v.Q, c->v.Qs, 1.0, c->stream);
        *launches = 2;
    } else if (c->cfg.scheme == EU_SCHEME_AMR && !strip_variant(var)) {
        c->ks->hancock_tile(c->v, var, c->dim == 2 && c->L >= 2 ? 1 : 0, c->state_elems, c->max_tiles, -1, 0, 0,
                            c->stream);
        *launches = 1;
    } else if (c->cfg.scheme == EU_SCHEME_AMR) {
        c->ks->hancock_strip(c->v, 2, c->strips, c->nstrips, c->v.Q, c->v.Qs, c->stream);
        *launches = 1;
    } else if (strip_variant(var)) {
        if (strip_fused(var)) {
            c->ks->fv_strip(c->v, 1, 0, 2, c->strips, c->nstrips, c->v.Q, c->v.Q, c->v.Qs, 1.0, c->stream);
            *launches = 1;
        } else {
            c->ks->fv_strip(c->v, 0, 1, 0, c->strips, c->nstrips, c->v.Q, c->v.Q, c->v.Qs, 0.5, c->stream);
            c->ks->fv_strip(c->v, 0, 0, 2, c->strips, c->nstrips, c->v.Q, c->v.Q, c->v.Qs, 1.0, c->stream);
            *launches = 2;
        }
    } else {
        const bool fine = c->dim == 2 && c->mode == MODE_HIER && c->L >= 2;
        c->ks->fv_stage(c->v, 1, -1, 0, 0, c->max_tiles, var, fine ? 1 : 0, c->stream);
        c->ks->fv_stage(c->v, 3, -1, 0, 0, c->max_tiles, var, fine ? 1 : 0, c->stream);
        *launches = 2;
    }
}

int stage_ready(eu_ctx *c)
{
    if (!c->initialized) return set_err(c, EU_ESTATE, "not initialised");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    Meta m;
    HIPCHK(c, hipMemcpy(&m, c->v.meta, sizeof(Meta), hipMemcpyDeviceToHost));
    if (m.done) return set_err(c, EU_ESTATE, "the run has reached t_end");
    return EU_OK;
}

// Mean time of one pass (fv_pass) of schedule var: one untimed pass, then
// reps passes back to back between two events on the context's stream.
int time_pass(eu_ctx *c, int var, int reps, float *ms_out, int *launches)
{
    int r0 = strips_for(c, var);
    if (r0) return r0;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_err(c, EU_EHIP, "hipEventCreate failed");
    }
    // the passes replayed from one graph (as a step is), so that the host's
    // launch rate does not pace them; eager launches on the default stream
    hipGraphExec_t ge = nullptr;
    if (c->stream) {
        hipGraph_t g;
        hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            for (int r = 0; r < reps; ++r) fv_pass(c, var, launches);
            e = hipStreamEndCapture(c->stream, &g);
            if (e == hipSuccess) {
                e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) ge = nullptr;
            }
        }
        if (!ge) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return set_err(c, EU_EHIP, "stage timing: graph capture failed: %s", hipGetErrorString(e));
        }
        (void)hipGraphLaunch(ge, c->stream);   // untimed replay
    } else {
        fv_pass(c, var, launches);
    }
    (void)hipEventRecord(e0, c->stream);
    if (ge) (void)hipGraphLaunch(ge, c->stream);
    else
        for (int r = 0; r < reps; ++r) fv_pass(c, var, launches);
    (void)hipEventRecord(e1, c->stream);
    hipError_t err = hipEventSynchronize(e1);
    if (ge) (void)hipGraphExecDestroy(ge);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return set_err(c, EU_EHIP, "stage timing failed: %s", hipGetErrorString(err));
    int r = check_launch(c);
    if (r) return r;
    *ms_out = ms / (float)reps;
    return EU_OK;
}

int harvest_profile(eu_ctx *c)
{
    for (auto &p : c->ev_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.second) == hipSuccess && hipEventElapsedTime(&ms, p.first, p.second) == hipSuccess) {
            c->prof_ms += ms;
            c->prof_n += 1;
        }
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    c->ev_pending.clear();
    return EU_OK;
}

InitArgs make_init(const eu_ctx *c, const eu_problem *p, int inst)
{
    InitArgs a{};
    a.kind = p->kind;
    a.axis = p->axis;
    a.lo = c->cfg.lo;
    a.hi = c->cfg.hi;
    a.x0 = p->x0;
    a.y0 = p->y0;
    const double *q = (p->inst_quad_host && inst >= 0) ? p->inst_quad_host + 16 * inst : &p->quad[0][0];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) a.quad[i][j] = q[4 * i + j];
    for (int i = 0; i < 8; ++i) a.ell[i] = p->ell[i];
    for (int i = 0; i < 4; ++i) a.es[i] = p->ell_states[i];
    for (int i = 0; i < 6; ++i) a.lr[i] = p->lr[i];
    a.split = p->split;
    for (int i = 0; i < 5; ++i) a.uni[i] = p->uniform[i];
    return a;
}

// After the finest level holds initial data: project down, analyse every
// level with all cells present, flag, tile; the patches keep the projected
// data; ghost fill.  t = 0.
int finish_init(eu_ctx *c)
{
    HIPCHK(c, hipMemsetAsync(c->v.cfls, 0, 8 * (size_t)cfl_slot(CFL_STRIDE, 0), c->stream));
    c->cfl_state = CFL_ZERO;
    HIPCHK(c, hipMemsetAsync(c->v.meta, 0, sizeof(Meta), c->stream));
    HIPCHK(c, hipMemsetAsync(c->v.t, 0, 8 * c->ngrid, c->stream));
    HIPCHK(c, hipMemsetAsync(c->v.t0, 0, 8 * c->ngrid, c->stream));
    HIPCHK(c, hipMemsetAsync(c->v.dt, 0, 8 * c->ngrid, c->stream));
    HIPCHK(c, hipMemsetAsync(c->v.smax, 0, 8 * c->ngrid, c->stream));
    // the list build's words start with one epoch
    HIPCHK(c, hipMemsetAsync(c->v.lword, 0, 2 * sizeof(unsigned long long) * c->v.ncls, c->stream));
    // and so do the flagging words
    HIPCHK(c, hipMemsetAsync(c->v.fword, 0, sizeof(unsigned long long) * std::max<int64_t>(c->v.nslot, 1),
                             c->stream));
    if (c->mode == MODE_HIER) {
        for (int l = c->L - 2; l >= 0; --l)
            c->ks->restrict_full(c->v, ARR_Q, l, c->grids[l].ncell, c->stream);
        launch_fill_u8(c->v.act, c->nbt, 1, c->stream);
        launch_fill_u8(c->v.nact, c->nbt, 1, c->stream);
        seq_details(c);
        seq_flag_tile(c, false);
    } else {
        // batch: every block of every instance is a leaf; the lists are static
        std::vector<Tile> leaf;
        std::vector<int> goff(c->ngrid), gcnt(c->ngrid);
        leaf.reserve(c->nbt);
        for (int g = 0; g < c->ngrid; ++g) {
            goff[g] = (int)leaf.size();
            const int64_t nb = nblocks_grid(c, g);
            for (int64_t b = 0; b < nb; ++b) leaf.push_back(Tile{g, (int)b});
            gcnt[g] = (int)nb;
        }
        launch_fill_u8(c->v.act, c->nbt, 1, c->stream);
        Meta m{};
        m.nleaf = (int)leaf.size();
        int r;
        if ((r = upload(c, c->v.leaf, leaf.data(), sizeof(Tile) * leaf.size()))) return r;
        if ((r = upload(c, (void *)c->v.grp_off, goff.data(), sizeof(int) * c->ngrid))) return r;
        if ((r = upload(c, (void *)c->v.grp_cnt, gcnt.data(), sizeof(int) * c->ngrid))) return r;
        if ((r = upload(c, c->v.meta, &m, sizeof(Meta)))) return r;
    }
    int r = check_launch(c);
    if (r) return r;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // captured step graphs stay valid: they depend on the buffers and the
    // schedule, not on the data, and a replay starts from CFL slots that
    // eu_advance prepares for the current state
    c->initialized = true;
    return EU_OK;
}

}  // namespace

// ============================================================================
// C-ABI
// ============================================================================
extern "C" {

// Thresholds of the details of levels 0 .. L-2: eps, or with eps_levels set
// eps_l = 2^(d (l + 2 - L)) eps (exact powers of two).
static void set_eps_levels(View &v, int L, int dim, double eps, int mode)
{
    for (int l = 0; l < MAXLEV; ++l) v.eps_lv[l] = mode ? std::ldexp(eps, dim * (l + 2 - L)) : eps;
}

int eu_query_sizes(const eu_config *cfg, size_t *state_bytes, size_t *scratch_bytes)
{
    std::string why;
    if (validate(cfg, why)) return EU_EINVAL;
    Layout lay;
    make_layout(cfg, lay);
    if (state_bytes) *state_bytes = lay.state;
    if (scratch_bytes) *scratch_bytes = lay.scratch;
    return EU_OK;
}

int eu_create(const eu_config *cfg, void *state_dev, size_t state_bytes, void *scratch_dev,
              size_t scratch_bytes, eu_ctx **out)
{
    if (!out) return EU_EINVAL;
    *out = nullptr;
    std::string why;
    if (validate(cfg, why)) return EU_EINVAL;
    if (!state_dev || !scratch_dev) return EU_EINVAL;
    if (((uintptr_t)state_dev & 255) || ((uintptr_t)scratch_dev & 255)) return EU_EINVAL;
    Layout lay;
    make_layout(cfg, lay);
    if (state_bytes < lay.state || scratch_bytes < lay.scratch) return EU_ENOMEM;

    eu_ctx *c = new (std::nothrow) eu_ctx();
    if (!c) return EU_ENOMEM;
    c->cfg = *cfg;
    if (cfg->n_instances > 1) c->sides.assign(cfg->inst_side_host, cfg->inst_side_host + cfg->n_instances);
    c->cfg.inst_side_host = c->sides.empty() ? nullptr : c->sides.data();
    c->ks = cfg->precision == EU_FP64 ? &kset_f64 : &kset_f32;
    c->stream = (hipStream_t)cfg->stream;
    c->L = lay.L;
    c->ngrid = lay.ngrid;
    c->dim = lay.dim;
    c->nv = lay.nv;
    c->mode = lay.mode;
    c->nbt = lay.nbt;
    c->max_tiles = (int)lay.max_tiles;
    c->ngroups = lay.ngroups;
    c->grids = lay.grids;
    c->state_elems = lay.state_elems;
    c->pbase = lay.pbase;

    View &v = c->v;
    v.dim = lay.dim;
    v.nv = lay.nv;
    v.L = lay.L;
    v.ngrid = lay.ngrid;
    v.bc = cfg->bc;
    v.mode = lay.mode;
    v.pmin = cfg->patch_min;
    v.pmax = cfg->patch_max > 0 ? cfg->patch_max : eu::BS;
    v.gamma = cfg->gamma;
    v.cfl = cfg->cfl;
    v.t_end = cfg->t_end;
    v.eps = cfg->eps;
    set_eps_levels(v, lay.L, cfg->dim, cfg->eps, cfg->eps_levels);
    v.rk = cfg->rk;
    v.ausm_cs = cfg->ausm_speed;
    v.tiler = cfg->tiler;
    v.cfl_max = cfg->cfl_mode;
    v.crit = cfg->criterion;
    v.eps_p = cfg->eps_p;
    v.eta = cfg->eta;
    const size_t es = cfg->precision == EU_FP64 ? 8 : 4;
    v.Q = state_dev;
    v.Qs = (char *)state_dev + align256((size_t)lay.state_elems * es);
    v.Qo = lay.narrays == 3 ? (char *)state_dev + 2 * align256((size_t)lay.state_elems * es) : nullptr;
    v.lts = lay.narrays == 3 ? 1 : 0;
    v.actv = at<Tile>(scratch_dev, lay.o_actv);
    v.reg = at<char>(scratch_dev, lay.o_reg);
    v.grids = at<Grid>(scratch_dev, lay.o_grids);
    for (int g = 0; g < lay.ngrid && g < eu::MAXLEV; ++g) v.gt[g] = lay.grids[(size_t)g];
    for (int l = 0; l <= eu::MAXLEV; ++l) v.pb[l] = lay.pbase[(size_t)l];
    v.act = at<uint8_t>(scratch_dev, lay.o_act);
    v.nact = at<uint8_t>(scratch_dev, lay.o_nact);
    v.code = at<uint8_t>(scratch_dev, lay.o_code);
    v.gmask = at<uint32_t>(scratch_dev, lay.o_gmask);
    v.nslot = lay.nslot;
    v.sig = at<uint8_t>(scratch_dev, lay.o_sig);
    v.flag = at<uint8_t>(scratch_dev, lay.o_flag);
    v.D = at<double>(scratch_dev, lay.o_D);
    v.leaf = at<Tile>(scratch_dev, lay.o_leaf);
    v.cov = at<Tile>(scratch_dev, lay.o_cov);
    v.ghost = at<Tile>(scratch_dev, lay.o_ghost);
    v.fresh = at<Tile>(scratch_dev, lay.o_fresh);
    v.pslot = at<int>(scratch_dev, lay.o_pslot);
    v.pcnt = at<int>(scratch_dev, lay.o_pcnt);
    v.fcnt = at<int>(scratch_dev, lay.o_fcnt);
    v.cpart = at<long long>(scratch_dev, lay.o_cpart);
    v.ncls = lay.ncls;
    {
        // EU_LIST_BUILD=2: the two-kernel list build also where one launch
        // would do (it is otherwise reached only by very large hierarchies)
        const char *lb = std::getenv("EU_LIST_BUILD");
        v.lists2 = lb && lb[0] == '2' ? 1 : 0;
        // EU_FLAG_BUILD=levels: one flagging launch per level also where one
        // launch for all of them would do
        const char *fb = std::getenv("EU_FLAG_BUILD");
        v.flags1 = fb && std::strcmp(fb, "levels") == 0 ? 1 : 0;
        // EU_WAIT_TEST=stale: the list build waits for an epoch that is never
        // published, with a short bound, so its waits give up (tests of the
        // give-up path; every kernel still ends)
        const char *wt = std::getenv("EU_WAIT_TEST");
        v.wait_stale = wt && std::strcmp(wt, "stale") == 0 ? 1 : 0;
        if (v.wait_stale) v.wait_spin = 64;
    }
    v.nbt = (int)lay.nbt;
    v.wcnt = at<int>(scratch_dev, lay.o_wcnt);
    v.lword = at<unsigned long long>(scratch_dev, lay.o_lword);
    v.fword = at<unsigned long long>(scratch_dev, lay.o_fword);
    v.pbase = at<int64_t>(scratch_dev, lay.o_pbase);
    v.meta = at<Meta>(scratch_dev, lay.o_meta);
    v.smax = at<unsigned long long>(scratch_dev, lay.o_smax);
    v.dt = at<double>(scratch_dev, lay.o_dt);
    v.t = at<double>(scratch_dev, lay.o_t);
    v.t0 = at<double>(scratch_dev, lay.o_t0);
    v.t_rem = INFINITY;
    v.wait_spin = 1 << 20;
    v.partial = at<double>(scratch_dev, lay.o_partial);
    v.cfls = at<unsigned long long>(scratch_dev, lay.o_cfls);
    v.totals = at<double>(scratch_dev, lay.o_totals);
    v.grp_off = at<int>(scratch_dev, lay.o_goff);
    v.grp_cnt = at<int>(scratch_dev, lay.o_gcnt);
    v.max_tiles = (int)lay.max_tiles;
    c->strips = at<Strip>(scratch_dev, lay.o_strips);
    c->max_strips = lay.max_strips;

    int r;
    if ((r = upload(c, (void *)v.grids, lay.grids.data(), sizeof(Grid) * lay.ngrid)) ||
        (r = upload(c, v.pbase, lay.pbase.data(), sizeof(int64_t) * (eu::MAXLEV + 1)))) {
        delete c;
        return r;
    }
    hipError_t e = hipMemsetAsync(v.meta, 0, sizeof(Meta), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(v.act, 0, c->nbt, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(v.nact, 0, c->nbt, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        delete c;
        return EU_EHIP;
    }
    // the device of the caller's buffers, and its copy of the static scratch
    hipPointerAttribute_t pa;
    e = hipPointerGetAttributes(&pa, state_dev);
    if (e == hipSuccess) {
        c->device = pa.device;
        e = scratch_addr(c->device, &c->static_scratch);
    }
    if (e != hipSuccess) {
        delete c;
        return EU_EHIP;
    }
    // the AMR scheme runs on the Hancock strip kernel (grids of one level)
    // or the Hancock tile kernel (hierarchies)
    if (cfg->scheme == EU_SCHEME_AMR) {
        c->variant = c->L > 1 || c->v.lts || c->dim == 3 ? 0 : FV_STRIP0;
        if ((r = strips_for(c, c->variant))) {
            delete c;
            return r;
        }
    }
    *out = c;
    return EU_OK;
}

int eu_destroy(eu_ctx *c)
{
    if (!c) return EU_EINVAL;
    (void)hipStreamSynchronize(c->stream);
    harvest_profile(c);
    drop_graphs(c);
    delete c;
    return EU_OK;
}

int eu_init_state(eu_ctx *c, const eu_problem *p)
{
    if (!c || !p) return EU_EINVAL;
    if (p->kind < EU_IC_QUADRANT || p->kind > EU_IC_UNIFORM) return set_err(c, EU_EINVAL, "bad problem kind");
    if (p->kind == EU_IC_QUADRANT && c->dim != 2) return set_err(c, EU_EINVAL, "quadrant data is 2D");
    if (p->kind == EU_IC_ELLIPSOID && c->dim != 3) return set_err(c, EU_EINVAL, "ellipsoid data is 3D");
    if (p->kind == EU_IC_RIEMANN1D && (p->axis < 0 || p->axis >= c->dim))
        return set_err(c, EU_EINVAL, "bad axis");
    if (c->mode == MODE_HIER) {
        const int g = c->L - 1;
        c->ks->init(c->v, make_init(c, p, -1), g, c->grids[g].ncell, c->stream);
    } else {
        for (int g = 0; g < c->ngrid; ++g)
            c->ks->init(c->v, make_init(c, p, g), g, c->grids[g].ncell, c->stream);
    }
    int r = check_launch(c);
    if (r) return r;
    return finish_init(c);
}

int eu_set_finest(eu_ctx *c, int inst, const double *q_host)
{
    if (!c || !q_host) return EU_EINVAL;
    const int g = c->mode == MODE_BATCH ? inst : c->L - 1;
    if (g < 0 || g >= c->ngrid) return set_err(c, EU_EINVAL, "bad instance");
    cfl_stale(c);
    const Grid &G = c->grids[g];
    const int64_t n = c->nv * G.ncell;
    if (c->cfg.precision == EU_FP64) {
        HIPCHK(c, hipMemcpy((double *)c->v.Q + G.off, q_host, 8 * n, hipMemcpyHostToDevice));
    } else {
        std::vector<float> tmp(n);
        for (int64_t i = 0; i < n; ++i) tmp[i] = (float)q_host[i];
        HIPCHK(c, hipMemcpy((float *)c->v.Q + G.off, tmp.data(), 4 * n, hipMemcpyHostToDevice));
    }
    if (c->mode == MODE_BATCH && c->initialized) return EU_OK;
    return finish_init(c);
}

int eu_mr_decompose(eu_ctx *c)
{
    if (!c) return EU_EINVAL;
    if (!c->initialized) return set_err(c, EU_ESTATE, "not initialised");
    if (c->mode != MODE_HIER) return set_err(c, EU_EINVAL, "a batch has no hierarchy");
    cfl_stale(c);
    if (c->v.crit == EU_CRIT_GRADIENT) {
        if (!seq_restrict(c, ARR_Q, true, false)) seq_ghost(c, ARR_Q);
        seq_details(c);
    } else if (!seq_restrict(c, ARR_Q, false, true)) {
        seq_details(c);
    }
    return check_launch(c);
}

int eu_mr_flag(eu_ctx *c, double eps, int64_t *nflag_host)
{
    if (!c) return EU_EINVAL;
    if (!c->initialized) return set_err(c, EU_ESTATE, "not initialised");
    if (c->mode != MODE_HIER) return set_err(c, EU_EINVAL, "a batch has no hierarchy");
    if (std::isnan(eps)) return set_err(c, EU_EINVAL, "eps is NaN");
    if (eps >= 0.0 && eps != c->v.eps) {
        // a new threshold: the significance of the details of the last
        // decomposition is taken again against it, and kept for later steps
        c->v.eps = eps;
        c->cfg.eps = eps;
        set_eps_levels(c->v, c->L, c->dim, eps, c->cfg.eps_levels);
        drop_graphs(c);
        int64_t n = 0;
        for (int l = 0; l < c->L - 1; ++l) n += c->grids[l].ncell;
        // the gradient indicators are evaluated again on the current state
        if (c->v.crit == EU_CRIT_GRADIENT) seq_details(c);
        else if (n > 0) launch_threshold(c->v, n, c->stream);
    }
    if (c->L > 1) seq_flag_tile(c, true);
    int r = check_launch(c);
    if (r) return r;
    if (nflag_host) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        r = level_flags(c, nflag_host);
        if (r) return r;
    }
    return EU_OK;
}

int eu_project(eu_ctx *c, int mode)
{
    if (!c) return EU_EINVAL;
    if (!c->initialized) return set_err(c, EU_ESTATE, "not initialised");
    cfl_stale(c);
    if (mode == EU_RESTRICT) seq_restrict(c, ARR_Q);
    else if (mode == EU_PROLONG) {
        for (int l = 1; l < c->L; ++l)
            c->ks->predict(c->v, ARR_Q, l, 1, 0, 0.0, 0, (int)nblocks_grid(c, l), c->stream);
    } else if (mode == EU_GHOST) seq_ghost(c, ARR_Q);
    else return set_err(c, EU_EINVAL, "bad projection mode");
    return check_launch(c);
}

int eu_cfl_dt(eu_ctx *c, double cfl, double t_remaining, double *dt_dev, double *dt_host)
{
    if (!c) return EU_EINVAL;
    if (!c->initialized) return set_err(c, EU_ESTATE, "not initialised");
    if (std::isnan(cfl) || std::isnan(t_remaining)) return set_err(c, EU_EINVAL, "cfl or t_remaining is NaN");
    // this call's CFL number and clip, by value in the kernel arguments
    View v = c->v;
    if (cfl > 0.0) v.cfl = cfl;
    if (t_remaining >= 0.0) v.t_rem = t_remaining;
    std::swap(v, c->v);
    seq_cfl(c);
    std::swap(v, c->v);
    int r = check_launch(c);
    if (r) return r;
    if (dt_dev) {
        const int n = c->mode == MODE_HIER ? 1 : c->ngrid;
        launch_copy_f64(dt_dev, c->v.dt, n, c->stream);
        if ((r = check_launch(c))) return r;
    }
    if (dt_host) {
        if ((r = sync_status(c))) return r;
        HIPCHK(c, hipMemcpy(dt_host, c->v.dt, 8, hipMemcpyDeviceToHost));
    }
    return EU_OK;
}

int eu_fv_step(eu_ctx *c, const double *dt_dev, int level)
{
    if (!c) return EU_EINVAL;
    if (!c->initialized) return set_err(c, EU_ESTATE, "not initialised");
    if (level < -1 || level >= c->L) return set_err(c, EU_EINVAL, "bad level");
    if (level >= 0 && !c->v.lts)
        return set_err(c, EU_EINVAL, "a global time step advances every level together (level -1)");
    cfl_stale(c);
    if (dt_dev) launch_set_dt(c->v, dt_dev, c->stream);
    if (c->v.lts) {
        lts_advance(c, level < 0 ? 0 : level, 0);
        seq_ghost(c, ARR_Q);
    } else {
        seq_fv_step(c, true);
    }
    return check_launch(c);
}

int eu_step(eu_ctx *c, int regrid)
{
    if (!c) return EU_EINVAL;
    if (!c->initialized) return set_err(c, EU_ESTATE, "not initialised");
    seq_step(c, regrid != 0);
    return check_launch(c);
}

// steps per graph of a run (even)
constexpr int GRAPH_RUN = 16;

int eu_advance(eu_ctx *c, int nsteps, int use_graph, int *steps_done)
{
    if (!c || nsteps < 0) return EU_EINVAL;
    if (!c->initialized) return set_err(c, EU_ESTATE, "not initialised");
    int s0 = 0;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(&s0, &c->v.meta->steps, sizeof(int), hipMemcpyDeviceToHost));
    // regrid after step n (counted from initialisation) when n is a
    // multiple of regrid_every (every step with 0 or 1)
    const int every = c->cfg.regrid_every > 1 && c->L > 1 ? c->cfg.regrid_every : 1;
    auto regrid_after = [&](int i) { return (s0 + i + 1) % every == 0; };
    if (use_graph && !c->prof) {
        if (!c->stream) return set_err(c, EU_EINVAL, "graph capture needs a non-default stream");
        // a step that leaves the CFL slots of the next starts from them:
        // the first replay needs them of the current state; otherwise the
        // step computes them itself, and the capture must record that
        if (step_leaves_slots(c)) cfl_ready(c);
        else if (c->cfl_state != CFL_ZERO) cfl_zero(c);
        // one graph per array holding the state (the fused strip schedules
        // move it to the other array every step); recording a step changes
        // only host bookkeeping, which is restored after each capture (the
        // CFL slots are left by a step as the lines above prepare them)
        const bool alt = (c->cfg.scheme == EU_SCHEME_AMR && !c->v.lts) ||
                         (strip_variant(c->variant) && c->dim == 2 && strip_fused(c->variant));
        // capture n consecutive steps from the state in array q (steps
        // after the end time are skipped by the kernels themselves); a
        // cycle regrids after its last step only
        auto capture = [&](int q, int n, bool cycle, hipGraphExec_t *out) -> int {
            const View saved = c->v;
            const int sq = c->qswap, scfl = c->cfl_state;
            if (q != c->qswap) {
                std::swap(c->v.Q, c->v.Qs);
                c->qswap ^= 1;
            }
            hipGraph_t g;
            HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            // (a step that moves the state to the other array says so in
            // the host bookkeeping, so the next recorded step starts there)
            for (int k = 0; k < n; ++k) seq_step(c, !cycle || k == n - 1);
            hipError_t e = hipStreamEndCapture(c->stream, &g);
            c->v = saved;
            c->qswap = sq;
            c->cfl_state = scfl;
            if (e != hipSuccess) return set_err(c, EU_EHIP, "graph capture failed: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                *out = nullptr;
                return set_err(c, EU_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
            }
            return EU_OK;
        };
        // a replayed graph of n steps leaves the state in the other array
        // after an odd number of alternating steps
        auto moved = [&](int n) {
            if (alt && (n & 1)) {
                std::swap(c->v.Q, c->v.Qs);
                c->qswap ^= 1;
            }
        };
        int i = 0;
        if (every > 1) {
            // steps up to the next regrid eagerly, then whole cycles from a
            // regrid to the next from one graph each, then the rest eagerly
            for (; i < nsteps && (s0 + i) % every != 0; ++i) {
                seq_step(c, regrid_after(i));
                int r = check_launch(c);
                if (r) return r;
            }
            for (; i + every <= nsteps; i += every) {
                const int q = c->qswap;
                if (!c->gcycle[q]) {
                    int r = capture(q, every, true, &c->gcycle[q]);
                    if (r) return r;
                }
                HIPCHK(c, hipGraphLaunch(c->gcycle[q], c->stream));
                moved(every);
            }
            for (; i < nsteps; ++i) {
                seq_step(c, regrid_after(i));
                int r = check_launch(c);
                if (r) return r;
            }
        }
        // one graph per array holding the state; recording steps changes
        // only host bookkeeping, which is restored after each capture (the
        // CFL slots are left by a step as the lines above prepare them).
        // Runs of GRAPH_RUN steps replay one graph (an even count: a run
        // ends in the array it started from), which saves the gap between
        // graph launches; the rest replays the graphs of one step.
        if (nsteps - i >= GRAPH_RUN) {
            const int q = c->qswap;
            if (!c->grun[q]) {
                int r = capture(q, GRAPH_RUN, false, &c->grun[q]);
                if (r) return r;
            }
            for (; i + GRAPH_RUN <= nsteps; i += GRAPH_RUN) HIPCHK(c, hipGraphLaunch(c->grun[q], c->stream));
        }
        for (int p = 0; p < (alt ? 2 : 1) && i < nsteps; ++p) {
            const int q = c->qswap ^ p;
            if (c->gexec[q]) continue;
            int r = capture(q, 1, false, &c->gexec[q]);
            if (r) return r;
        }
        for (; i < nsteps; ++i) {
            HIPCHK(c, hipGraphLaunch(c->gexec[c->qswap], c->stream));
            moved(1);
        }
    } else {
        for (int i = 0; i < nsteps; ++i) {
            seq_step(c, regrid_after(i));
            int r = check_launch(c);
            if (r) return r;
        }
    }
    int r = sync_status(c);
    if (c->prof) harvest_profile(c);
    int s1 = 0;
    HIPCHK(c, hipMemcpy(&s1, &c->v.meta->steps, sizeof(int), hipMemcpyDeviceToHost));
    if (steps_done) *steps_done = s1 - s0;
    return r;
}

int eu_conserved_totals(eu_ctx *c, double *totals_dev, double *totals_host)
{
    if (!c) return EU_EINVAL;
    if (!c->initialized) return set_err(c, EU_ESTATE, "not initialised");
    c->ks->totals(c->v, c->max_tiles, c->stream);
    launch_totals_final(c->v, c->ngroups, c->stream);
    if (totals_dev) launch_copy_f64(totals_dev, c->v.totals, c->nv * c->ngroups, c->stream);
    int r = check_launch(c);
    if (r) return r;
    if (totals_host) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        HIPCHK(c, hipMemcpy(totals_host, c->v.totals, 8 * c->nv * c->ngroups, hipMemcpyDeviceToHost));
    }
    return EU_OK;
}

int eu_conserved_totals_static(eu_ctx *c, double *totals_dev)
{
    if (!c || !totals_dev) return EU_EINVAL;
    if (!c->initialized) return set_err(c, EU_ESTATE, "not initialised");
    if (!c->static_scratch) return set_err(c, EU_EHIP, "no device address of the static scratch");
    // partial sums of every tile the leaf list can hold, then the totals
    const int64_t npart = ((int64_t)c->max_tiles * c->nv + 31) / 32 * 32;
    const int64_t need = npart + (int64_t)c->ngroups * c->nv;
    if (need > STATIC_SCRATCH_DOUBLES)
        return set_err(c, EU_ENOMEM,
                       "eu_conserved_totals_static: %lld tiles x %d fields and %d groups need %lld doubles of "
                       "scratch; the static scratch holds %lld",
                       (long long)c->max_tiles, c->nv, c->ngroups, (long long)need,
                       (long long)STATIC_SCRATCH_DOUBLES);
    View v = c->v;
    v.partial = c->static_scratch;
    v.totals = c->static_scratch + npart;
    c->ks->totals(v, c->max_tiles, c->stream);
    launch_totals_final(v, c->ngroups, c->stream);
    launch_copy_f64(totals_dev, v.totals, c->nv * c->ngroups, c->stream);
    return check_launch(c);
}

int eu_copy_level(eu_ctx *c, int inst, int level, int which, double *dst)
{
    if (!c || !dst) return EU_EINVAL;
    const int g = c->mode == MODE_BATCH ? inst : level;
    if (g < 0 || g >= c->ngrid) return set_err(c, EU_EINVAL, "bad level / instance");
    if (which != 0 && which != 1) return set_err(c, EU_EINVAL, "bad array");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const Grid &G = c->grids[g];
    const int64_t n = c->nv * G.ncell;
    const void *base = which == 0 ? c->v.Q : c->v.Qs;
    if (c->cfg.precision == EU_FP64) {
        HIPCHK(c, hipMemcpy(dst, (const double *)base + G.off, 8 * n, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(n);
        HIPCHK(c, hipMemcpy(tmp.data(), (const float *)base + G.off, 4 * n, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i) dst[i] = tmp[i];
    }
    return EU_OK;
}

int eu_copy_uniform(eu_ctx *c, double *dst)
{
    if (!c || !dst) return EU_EINVAL;
    if (!c->initialized) return set_err(c, EU_ESTATE, "not initialised");
    if (c->mode != MODE_HIER) return set_err(c, EU_EINVAL, "a batch has no hierarchy");
    for (int l = 0; l < c->L; ++l) c->ks->composite(c->v, l, c->grids[l].ncell, c->stream);
    int r = check_launch(c);
    if (r) return r;
    return eu_copy_level(c, 0, c->L - 1, 1, dst);
}

int eu_get_active(eu_ctx *c, int level, uint8_t *dst)
{
    if (!c || !dst) return EU_EINVAL;
    if (level < 0 || level >= c->ngrid) return set_err(c, EU_EINVAL, "bad level");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const Grid &G = c->grids[level];
    const int64_t nbk = nblocks_grid(c, level);
    std::vector<uint8_t> m(nbk);
    HIPCHK(c, hipMemcpy(m.data(), c->v.act + G.boff, nbk, hipMemcpyDeviceToHost));
    const int n = G.n, nb = G.nb;
    for (int64_t i = 0; i < G.ncell; ++i) {
        const int x = (int)(i % n), y = (int)((i / n) % n), z = c->dim == 3 ? (int)(i / ((int64_t)n * n)) : 0;
        dst[i] = m[(x >> 3) + (int64_t)nb * ((y >> 3) + (int64_t)nb * (z >> 3))];
    }
    return EU_OK;
}

int eu_get_flags(eu_ctx *c, int level, uint8_t *dst)
{
    if (!c || !dst) return EU_EINVAL;
    if (c->mode != MODE_HIER || level < 0 || level >= c->L - 1) return set_err(c, EU_EINVAL, "bad level");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const Grid &G = c->grids[level];
    HIPCHK(c, hipMemcpy(dst, c->v.flag + G.coff, G.ncell, hipMemcpyDeviceToHost));
    return EU_OK;
}

int eu_get_details(eu_ctx *c, int level, double *dst)
{
    if (!c || !dst) return EU_EINVAL;
    if (c->mode != MODE_HIER || level < 0 || level >= c->L - 1) return set_err(c, EU_EINVAL, "bad level");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const Grid &G = c->grids[level];
    HIPCHK(c, hipMemcpy(dst, c->v.D + G.coff, 8 * G.ncell, hipMemcpyDeviceToHost));
    return EU_OK;
}

// The rows come from the per pmax-block slots of the last flagging, read in
// slot order (levels in order, pmax blocks in Morton order) and, within a
// slot, in the order the split emitted them.
int eu_patch_table(eu_ctx *c, int32_t *dst, int cap, int *npatch)
{
    if (!c || !npatch || cap < 0 || (cap > 0 && !dst)) return EU_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *npatch = 0;
    if (c->mode != MODE_HIER || c->v.nslot == 0) return EU_OK;
    const int R = c->cfg.patch_max / BS;
    const int64_t nsub = c->dim == 2 ? R * R : R * R * R;
    std::vector<int> cnt((size_t)c->v.nslot), rows((size_t)(c->v.nslot * nsub * 7));
    HIPCHK(c, hipMemcpy(cnt.data(), c->v.pcnt, sizeof(int) * cnt.size(), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(rows.data(), c->v.pslot, sizeof(int) * rows.size(), hipMemcpyDeviceToHost));
    int n = 0;
    for (int64_t sl = 0; sl < c->v.nslot; ++sl)
        for (int j = 0; j < cnt[(size_t)sl]; ++j, ++n)
            if (n < cap)
                for (int e = 0; e < 7; ++e) dst[7 * (int64_t)n + e] = rows[(size_t)((sl * nsub + j) * 7 + e)];
    *npatch = n;
    return EU_OK;
}

int eu_counters(eu_ctx *c, int64_t *leaves, int64_t *active)
{
    if (!c) return EU_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->mode == MODE_HIER) return level_cells(c, leaves, active);
    int64_t s = 0;
    for (int g = 0; g < c->ngrid; ++g) s += c->grids[g].ncell;
    for (int l = 0; l < c->L; ++l) {
        if (leaves) leaves[l] = s;
        if (active) active[l] = s;
    }
    return EU_OK;
}

int eu_leaf_updates(eu_ctx *c, int64_t *updates_host, int *steps_host)
{
    if (!c) return EU_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    Meta m;
    HIPCHK(c, hipMemcpy(&m, c->v.meta, sizeof(Meta), hipMemcpyDeviceToHost));
    if (steps_host) *steps_host = m.steps;
    if (updates_host) {
        if (c->mode == MODE_HIER) *updates_host = m.leaf_updates;
        else {
            int64_t s = 0;
            for (int g = 0; g < c->ngrid; ++g) s += c->grids[g].ncell;
            *updates_host = s * (int64_t)m.steps;
        }
    }
    return EU_OK;
}

int eu_time(eu_ctx *c, double *t_host, double *dt_host)
{
    if (!c) return EU_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (t_host) HIPCHK(c, hipMemcpy(t_host, c->v.t, 8, hipMemcpyDeviceToHost));
    if (dt_host) HIPCHK(c, hipMemcpy(dt_host, c->v.dt, 8, hipMemcpyDeviceToHost));
    return EU_OK;
}

int eu_profile(eu_ctx *c, int enable)
{
    if (!c) return EU_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    harvest_profile(c);
    c->prof = enable != 0;
    c->prof_ms = 0.0;
    c->prof_n = 0;
    return EU_OK;
}

int eu_kernel_time(eu_ctx *c, double *ms, int64_t *launches)
{
    if (!c) return EU_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    harvest_profile(c);
    if (ms) *ms = c->prof_ms;
    if (launches) *launches = c->prof_n;
    return EU_OK;
}

int eu_set_variant(eu_ctx *c, int variant)
{
    if (!c) return EU_EINVAL;
    if (!variant_ok(c, variant))
        return set_err(c, EU_EINVAL, "schedule %d does not apply to this configuration", variant);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int r = strips_for(c, variant);
    if (r) return r;
    c->variant = variant;
    drop_graphs(c);
    return EU_OK;
}

int eu_autotune(eu_ctx *c, int reps, int *variant_host, float *ms_host)
{
    if (!c || reps < 1) return EU_EINVAL;
    int r = stage_ready(c);
    if (r) return r;
    int best = -1;
    float best_ms = 0.f;
    for (int var = 0; var < FV_VARIANTS; ++var) {
        float ms = INFINITY;
        if (variant_ok(c, var)) {
            int launches = 0;
            r = time_pass(c, var, reps, &ms, &launches);
            if (r) return r;
            if (best < 0 || ms < best_ms) { best = var; best_ms = ms; }
        }
        if (ms_host) ms_host[var] = ms;
    }
    if ((r = strips_for(c, best))) return r;
    c->variant = best;
    drop_graphs(c);
    if (variant_host) *variant_host = best;
    return EU_OK;
}

int eu_stage_time(eu_ctx *c, int reps, float *ms_host, int64_t *cells_host, int *launches_host)
{
    if (!c || reps < 1) return EU_EINVAL;
    int r = stage_ready(c);
    if (r) return r;
    float ms = 0.f;
    int launches = 0;
    r = time_pass(c, c->variant, reps, &ms, &launches);
    if (r) return r;
    int64_t cells = 0;
    if (c->mode != MODE_HIER) {
        for (int g = 0; g < c->ngrid; ++g) cells += c->grids[g].ncell;
    } else {
        int64_t lc[MAXLEV], ac[MAXLEV];
        r = level_cells(c, lc, ac);
        if (r) return r;
        for (int l = 0; l < c->L; ++l) cells += c->v.lts ? ac[l] : lc[l];
    }
    // cell-stages of a pass: both stages of every leaf, or the first stage
    // of every patch cell with local time stepping
    if (ms_host) *ms_host = ms;
    if (cells_host) *cells_host = c->v.lts || c->cfg.scheme == EU_SCHEME_AMR ? cells : 2 * cells;
    if (launches_host) *launches_host = launches;
    return EU_OK;
}

int eu_status(eu_ctx *c)
{
    if (!c) return EU_EINVAL;
    return sync_status(c);
}

int eu_clear_status(eu_ctx *c)
{
    if (!c) return EU_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int z = 0;
    HIPCHK(c, hipMemcpy(&c->v.meta->status, &z, sizeof(int), hipMemcpyHostToDevice));
    return EU_OK;
}

const char *eu_last_error(const eu_ctx *c)
{
    if (!c) return "null context";
    return c->err.c_str();
}

}  // extern "C"
