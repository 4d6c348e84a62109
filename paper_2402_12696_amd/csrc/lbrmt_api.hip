// Host side of the gfx950 LBRMT library: the C ABI of include/lbrmt.h.
//
// One step (Alg. 1) is a fixed launch sequence.  The reference-map chain
// (advect, 11 extrapolation layers, relabel, force) runs on an internal side
// stream while the lattice Boltzmann update of every tile outside the band
// region runs on the caller's stream; the band tiles are updated after the
// chain has produced this step's force.  Buffer parities repeat every 6 steps
// (lattice / xi / force double buffers, 3-slot window ring), so 6 steps are
// captured once into a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/lbrmt.h"
#include "lbrmt_internal.h"

using namespace lbrmt;

// Static scratch of lbrmt_diag_noalloc (see there): the diagnostic's partial
// records (1024 blocks x 11 doubles), its reduced record (16 doubles) and one
// record of 7 doubles per solid, for up to LBRMT_DIAG_NOALLOC_MAX_SOLIDS.
namespace {
constexpr size_t NOALLOC_PART_BYTES = 1024 * 11 * 8;
constexpr size_t NOALLOC_PART_OFF = 0;
constexpr size_t NOALLOC_OUT_OFF = NOALLOC_PART_BYTES;
constexpr size_t NOALLOC_SOLID_OFF = NOALLOC_OUT_OFF + 256;
constexpr size_t NOALLOC_BYTES =
    NOALLOC_SOLID_OFF + (size_t)LBRMT_DIAG_NOALLOC_MAX_SOLIDS * 7 * 8;
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
}  // namespace
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

constexpr int GRAPH_STEPS = 6;
constexpr size_t ALIGN = 256;
constexpr uint32_t STATE_MAGIC = 0x4c42524d;  // "LBRM"
constexpr uint32_t STATE_VERSION = 1;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Window of each solid of a several-solid context (the same for all solids).
struct MbGeom {
    int nx, ny;        // window extents
    int wx, wy;        // sub-window axes
    int pp;
    size_t pplane;
    long long lcap;
};

MbGeom mb_geom(const lbrmt_grid_desc* d)
{
    const int W = d->body_window > 0 ? d->body_window : 128;
    MbGeom m;
    m.wx = d->periodic_x && d->nx % FB == 0 && d->nx >= W + 2 * PAD + 32;
    m.wy = d->periodic_y && d->ny % FB == 0 && d->ny >= W + 2 * PAD + 32;
    m.nx = m.wx ? W : d->nx;
    m.ny = m.wy ? W : d->ny;
    m.pp = (int)round_up((size_t)m.nx + 2 * PAD, 32);
    m.pplane = (size_t)m.pp * (m.ny + 2 * PAD);
    m.lcap = sub_cap_tiles(m.nx, m.ny);
    return m;
}

// Per-solid block of a several-solid workspace.
struct BodyLayout {
    size_t off_X[2], off_Y[2], off_phi[2], off_tag, off_gcol, off_lists, off_lcount,
        off_boxpart, off_ticket, off_win, total;
};

BodyLayout body_layout(const lbrmt_grid_desc* d, const MbGeom& m)
{
    BodyLayout B;
    const size_t es = d->precision == LBRMT_FP64 ? 8 : 4;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = round_up(o + bytes, ALIGN);
        return r;
    };
    for (int k = 0; k < 2; k++) {
        B.off_X[k] = take(m.pplane * es);
        B.off_Y[k] = take(m.pplane * es);
        B.off_phi[k] = take(m.pplane * es);
    }
    B.off_tag = take(m.pplane);
    B.off_gcol = take(m.pplane);
    B.off_lists = take((size_t)m.lcap * NSUB * 4 * (size_t)(d->layers + 1));
    B.off_lcount = take((size_t)(MAX_LAYERS + 1) * NSUB * LCOUNT_PAD * 4);
    B.off_boxpart = take((size_t)std::max(BOX_BLOCKS, MB_BAND_BLOCKS) * 4 * 4);
    B.off_ticket = take(4);
    B.off_win = take(3 * sizeof(Win));
    B.total = o;
    return B;
}

struct Layout {
    int pitch, pp;
    size_t plane, pplane;
    size_t rm_es;  // bytes per reference-map value: 8 (FP64 xi) or 4 (FP32 displacement)
    size_t off_lat[2], off_fx[2], off_fy[2], off_drho, off_X[2], off_Y[2], off_phi[2], off_tag,
        off_win, off_health, off_dpart, off_dout, off_gcol, off_lists, off_lcount, off_boxpart,
        off_ticket, off_cut_layer, off_cut_tiles, off_ncut, off_ff_flag, off_ff_list, off_ff_n,
        total;
    size_t lat_bytes;
    // several solids
    int nbx, nby;
    size_t off_stamp[2], off_mlist[2], off_mcount, off_dstep, off_mbtab, off_tabs, off_bsum,
        off_mord, off_bodies, body_bytes;
};

Layout make_layout(const lbrmt_grid_desc* d, int max_solids = 1)
{
    const bool multi = max_solids > 1;
    Layout L;
    L.pitch = (int)round_up((size_t)d->nx, 64);
    L.pp = (int)round_up((size_t)d->nx + 2 * PAD, 32);
    L.plane = (size_t)L.pitch * d->ny;
    L.pplane = (size_t)L.pp * (d->ny + 2 * PAD);
    L.rm_es = d->precision == LBRMT_FP64 ? 8 : 4;
    const size_t s = d->precision == LBRMT_FP32 ? 4 : 8;
    L.lat_bytes = NQ * L.plane * s;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = round_up(o + bytes, ALIGN);
        return r;
    };
    for (int k = 0; k < 2; k++) L.off_lat[k] = take(L.lat_bytes);
    for (int k = 0; k < 2; k++) {
        L.off_fx[k] = take(L.plane * 8);
        L.off_fy[k] = take(L.plane * 8);
    }
    L.off_drho = take(L.plane * 8);
    // the single solid's reference map (several solids: per-solid blocks)
    const size_t rp = multi ? 0 : L.pplane;
    for (int k = 0; k < 2; k++) {
        L.off_X[k] = take(rp * L.rm_es);
        L.off_Y[k] = take(rp * L.rm_es);
        L.off_phi[k] = take(rp * L.rm_es);
    }
    L.off_tag = take(rp);
    L.off_gcol = take(rp);
    L.off_lists = take(multi ? 0 : (size_t)sub_cap((long long)L.pplane) * NSUB * 4 *
                                        (size_t)(d->layers + 1));
    L.off_lcount = take((size_t)(MAX_LAYERS + 1) * NSUB * LCOUNT_PAD * 4);
    L.off_boxpart = take((size_t)std::max(RELABEL_BLOCKS, BOX_BLOCKS) * 4 * 4);
    L.off_ticket = take(4);
    const size_t ntile = multi ? 0 : (size_t)fused_tiles(d->nx, d->ny);
    L.off_cut_layer = take(ntile);
    L.off_cut_tiles = take(ntile * 4);
    L.off_ncut = take(4);
    L.off_ff_flag = take(ntile * 4);
    L.off_ff_list = take(ntile * 4);
    L.off_ff_n = take(4);
    L.off_win = take(3 * sizeof(Win));
    L.off_health = take(LBRMT_H_COUNT * sizeof(unsigned));
    L.off_dpart = take(diag_partial_doubles() * 8);
    L.off_dout = take(16 * 8);
    L.nbx = (d->nx + FB - 1) / FB;
    L.nby = (d->ny + FB - 1) / FB;
    L.body_bytes = 0;
    if (multi) {
        const size_t nblk = (size_t)L.nbx * L.nby;
        for (int k = 0; k < 2; k++) {
            L.off_stamp[k] = take(nblk * 4);
            L.off_mlist[k] = take(nblk * 4);
        }
        L.off_mcount = take(2 * 4);
        L.off_dstep = take(8);
        L.off_mbtab = take((size_t)max_solids * sizeof(MbBody));
        L.off_tabs = take(7 * ((size_t)max_solids * (sizeof(AdvectArgs) + sizeof(LayersArgs) +
                                                     sizeof(FitArgs) + sizeof(EdgesArgs)) +
                               4 * ALIGN));
        L.off_bsum = take((size_t)max_solids * 7 * 8);
        L.off_mord = take((size_t)max_solids * 4);
        L.body_bytes = body_layout(d, mb_geom(d)).total;
        L.off_bodies = take((size_t)max_solids * L.body_bytes);
    }
    L.total = o;
    return L;
}

const char* kernel_names[] = {"advect", "extrap", "relabel", "force", "lb_bulk", "lb_band"};
constexpr int NKERN = 6;

}  // namespace

struct lbrmt_ctx {
    lbrmt_grid_desc d;
    Layout L;
    GridP g;
    BodyP body;
    int max_solids = 0, nsolid = 0;
    lbrmt_solid_desc solid{};
    hipStream_t st = nullptr;
    hipStream_t side = nullptr;
    hipStream_t cap = nullptr;
    // the cross-stream events of step n are those of slot n mod 6: inside a
    // captured sequence no event is recorded twice, and a wait on the
    // previous step's record names that step's event
    hipEvent_t ev_fork[GRAPH_STEPS] = {}, ev_join[GRAPH_STEPS] = {}, ev_adv[GRAPH_STEPS] = {},
               ev_bulk[GRAPH_STEPS] = {};
    char* ws = nullptr;
    void* lat[2];
    double *Fx[2], *Fy[2], *drho;
    BandBufs bb;
    double *dpart, *dout;
    long long step = 0;
    bool inited = false;
    bool overlap = true;  // the chain on an internal stream beside the bulk lattice update
    int lb_variant = 3;    // set per precision by lbrmt_create
    hipGraphExec_t gexec = nullptr;
    // steps 6 + p .. 6 + p + r - 1 (r < 6): replayed for step runs that do not
    // start or end on a six-step boundary, captured on first use
    hipGraphExec_t pexec[GRAPH_STEPS][GRAPH_STEPS] = {};
    // the captured graphs of gexec and pexec, kept until their executable
    // graphs are destroyed
    hipGraph_t gsrc = nullptr;
    hipGraph_t psrc[GRAPH_STEPS][GRAPH_STEPS] = {};
    bool graph = true;  // replay captured six-step graphs
    bool member = false;  // member of a batch (stepped by the batch only)
    int bulk_blocks = 0;  // cap on the blocks of the overlapped bulk update (0: one per tile)
    int fused_fit = -1;  // block size of the one-launch extrapolation (0: one launch per layer, -1: by size)
    // hold the bulk update until the advection pass ends: -1 when it is
    // uncapped (default), 1 always (refused with a cap), 0 never
    int hold_bulk = -1;
    // thousandths of a held bulk update's tiles launched early, when the
    // previous step's chain ends (-1: by grid size)
    int bulk_early = -1;
    bool timing = false;
    struct Pending {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    double t_ms[NKERN] = {0};
    long long t_n[NKERN] = {0};
    std::string err;
    // several solids (max_solids > 1): one window per solid
    bool multi = false;
    MbGeom mg{};
    BodyLayout BL{};
    std::vector<MbBody> mbh;   // host copy of the solid table
    MbBody* mbd = nullptr;     // device table
    BatchTables mtab[7];       // chain argument tables, phases as for batches
    int* mord = nullptr;       // solids by decreasing size (rows of the chain's block grids)
    int* stamp[2] = {nullptr, nullptr};
    int* mlist[2] = {nullptr, nullptr};
    int* mcount = nullptr;
    long long* dstep = nullptr;
    double* bsum = nullptr;
    int adj_flip = 0;  // which half of an adjoint buffer holds state n + 1
};

static int fail(lbrmt_ctx* c, const char* what, hipError_t e)
{
    if (c) {
        char buf[512];
        snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
        c->err = buf;
    }
    return LBRMT_EHIP;
}

#define HIPCHK(c, expr)                                   \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return fail((c), #expr, e_); \
    } while (0)

static hipEvent_t pool_get(lbrmt_ctx* c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// timing brackets (eager launches only)
struct Bracket {
    lbrmt_ctx* c;
    int kind;
    hipStream_t s;
    hipEvent_t a = nullptr;
    Bracket(lbrmt_ctx* c_, int k, hipStream_t s_) : c(c_), kind(k), s(s_)
    {
        if (c->timing) {
            a = pool_get(c);
            if (a) (void)hipEventRecord(a, s);
        }
    }
    void done()
    {
        if (c->timing && a) {
            hipEvent_t b = pool_get(c);
            if (b) {
                (void)hipEventRecord(b, s);
                c->pending.push_back({kind, a, b});
            }
        }
    }
};

static int collect_timing(lbrmt_ctx* c)
{
    if (c->pending.empty()) return LBRMT_OK;
    for (auto& p : c->pending) {
        HIPCHK(c, hipEventSynchronize(p.b));
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, p.a, p.b));
        c->t_ms[p.kind] += ms;
        c->t_n[p.kind] += 1;
        c->pool.push_back(p.a);
        c->pool.push_back(p.b);
    }
    c->pending.clear();
    return LBRMT_OK;
}

static double fpo_x(const lbrmt_ctx* c, long long n) { return n == 0 ? 0.0 : c->d.fext_x; }
static double fpo_y(const lbrmt_ctx* c, long long n) { return n == 0 ? 0.0 : c->d.fext_y; }

// the per-phase argument tables of the several-solid chain
static MbTabs mb_tabs(const lbrmt_ctx* c)
{
    MbTabs t{};
    for (int p = 0; p < 7; p++) {
        t.adv[p] = c->mtab[p].adv;
        t.lay[p] = c->mtab[p].lay;
        t.fit[p] = c->mtab[p].fit;
        t.edg[p] = c->mtab[p].edg;
    }
    return t;
}

// several solids, step n on stream st: the chain of every solid (relabel
// only), the force blocks and the combined forces, the sub-windows that need
// to follow their solids, the lattice update
static int enqueue_step_mb(lbrmt_ctx* c, long long n, hipStream_t st)
{
    const StepSlots s = slots_for(n);
    const int p = n == 0 ? 6 : (int)(n % 6);
    const int nb = c->nsolid;
    const int prec = c->d.precision;
    if (nb > 0) {
        HIPCHK(c, launch_batch_band(prec, c->mtab[p], nb, c->d.layers, st, true, MB_DT_BLOCKS,
                                    0, MB_BAND_BLOCKS));
        HIPCHK(c, launch_mb_mark(c->g, c->mbd, nb, s.wcur, s.wnext, MB_BAND_BLOCKS,
                                 c->stamp[s.cur], 0, c->mlist[s.cur], &c->mcount[s.cur],
                                 c->L.nbx, c->bb.health, st, c->dstep));
        HIPCHK(c, launch_mb_combine(c->g, prec, c->mbd, nb, s.nxt, s.wcur, c->mlist[s.cur],
                                    &c->mcount[s.cur], &c->mcount[s.nxt], c->L.nbx,
                                    c->Fx[s.cur], c->Fy[s.cur], c->drho, false, c->bb.health,
                                    st));
        // the maps of step n + 1 are in buffer s.nxt, their boxes in slots
        // s.wcur (validity) and s.wnext (solid set)
        if (c->mg.wx || c->mg.wy)
            HIPCHK(c, launch_mb_recentre(prec, c->mbd, nb, mb_tabs(c), s.nxt, s.wcur, s.wnext,
                                         st));
    }
    HIPCHK(c, launch_lb_mb(c->g, prec, c->lb_variant, c->lat[s.cur], c->lat[s.nxt],
                           c->Fx[s.nxt], c->Fy[s.nxt], c->Fx[s.cur], c->Fy[s.cur], c->drho,
                           StampValid{c->stamp[s.nxt], 0, c->L.nbx},
                           StampValid{c->stamp[s.cur], 0, c->L.nbx}, fpo_x(c, n), fpo_y(c, n),
                           c->bb.health, st, c->dstep));
    HIPCHK(c, launch_mb_tick(c->dstep, st));
    return LBRMT_OK;
}

// where F^{n-1} is held for reads of state n (several solids: the stamps)
static StampValid prev_valid(const lbrmt_ctx* c)
{
    if (!c->multi) return StampValid{nullptr, 0, 0};
    return StampValid{c->stamp[slots_for(c->step).nxt], (int)c->step, c->L.nbx};
}

// Block size of the one-launch extrapolation (default 1024; one launch per
// layer, 0, by default when the bulk update's workgroups are capped), 0 for
// one launch per layer.
// The early part of a held bulk update: -1 (default) takes the far tiles of
// the first 30 % on grids of 2048^2 nodes or more, where the bulk update
// outlasts the chain's latency-bound head (MI355X, cavity with a disc,
// ms/step without -> with: 2048^2 FP64 0.1732 -> 0.1624, FP32 0.1124 ->
// 0.1072), and none on smaller ones, where it only slows the advection pass
// beside it (1024^2 FP64 0.0796 -> 0.0854 with half the tiles)
static int bulk_early(const lbrmt_ctx* c)
{
    if (c->bulk_early >= 0) return c->bulk_early;
    return (long long)c->d.nx * c->d.ny >= 2048ll * 2048 ? 300 : 0;
}

static int fused_threads(const lbrmt_ctx* c)
{
    if (c->fused_fit >= 0) return c->fused_fit;
    if (c->bulk_blocks > 0) return 0;
    // FP64: blocks of 512 (198 registers, none spilled, two waves per SIMD)
    // beside the bulk update, 0.1613 -> 0.1595 ms per 2048^2 step against
    // 1024; FP32 keeps 1024 (0.1070 against 0.1091 at 512)
    return c->d.precision == 0 ? 512 : 1024;
}

// Step n on stream main_s.  With overlap the reference-map chain runs on the
// internal stream beside the bulk lattice update; `first` and `last` bracket
// a sequence of steps enqueued together (a captured graph): the chain stream
// is forked from main_s before the first and joined back after the last.
// Inside a sequence each step needs only these cross-stream orders:
//   bulk update of step n  after the advection pass of step n (held) or the
//                          chain of step n - 1 (not held), which follows the
//                          force pass of step n - 1 (lattice and window ring);
//   force pass of step n   after the bulk update of step n - 1 (the halo of
//                          the window, and the planes both write next);
// the advection pass reads the lattice only inside the previous step's
// window, which that step's force pass updated (checked per node), so the
// chain of step n does not wait for the bulk update of step n - 1.
static int enqueue_step(lbrmt_ctx* c, long long n, hipStream_t main_s, bool first = true,
                        bool last = true)
{
    if (c->multi) return enqueue_step_mb(c, n, main_s);
    const StepSlots s = slots_for(n);
    const GridP& g = c->g;
    const int prec = c->d.precision;
    const double ox = fpo_x(c, n), oy = fpo_y(c, n);
    const int ek = (int)(n % GRAPH_STEPS), ep = (int)((n + GRAPH_STEPS - 1) % GRAPH_STEPS);
    hipEvent_t ev_fork = c->ev_fork[ek], ev_adv = c->ev_adv[ek], ev_join = c->ev_join[ek];
    hipEvent_t ev_bulk = c->ev_bulk[ek];
    hipEvent_t prev_join = c->ev_join[ep], prev_bulk = c->ev_bulk[ep];
    if (c->nsolid > 0) {
        hipStream_t band = main_s;
        if (c->overlap) {
            if (first) {
                HIPCHK(c, hipEventRecord(ev_fork, main_s));
                HIPCHK(c, hipStreamWaitEvent(c->side, ev_fork, 0));
            }
            band = c->side;
        }
        // the extrapolation in one launch (its tile list comes from the
        // distance transform)
        const int ff = fused_threads(c);
        const bool fused = ff > 0 && fused_fit_ok(g);
        {
            // advection and the layers of the extrapolation zone (one pass)
            Bracket b(c, 0, band);
            HIPCHK(c, launch_advect_layers(g, prec, c->bb, s, c->lat[s.cur], c->Fx[s.nxt],
                                           c->Fy[s.nxt], band, fused));
            b.done();
        }
        // with the one-launch extrapolation the bulk update starts when the
        // advection pass ends: the extrapolation's few large blocks are then
        // resident before the bulk update's many fill the compute units (not
        // with a capped bulk update: held and capped at 512 workgroups, steps
        // stalled for about 0.1 s on MI355X)
        const bool hold_bulk = c->overlap && fused && c->bulk_blocks == 0 && c->hold_bulk != 0;
        if (hold_bulk) HIPCHK(c, hipEventRecord(ev_adv, band));
        {
            Bracket b(c, 1, band);
            HIPCHK(c, launch_extrapolate(g, c->bb, s, band, fused ? ff : 0));
            b.done();
        }
        // the bulk update of the previous step in this sequence (the first
        // step's is ordered by the fork).  Not before the extrapolation: the
        // wait delays its launch until the bulk update has filled the
        // compute units (FP64 step 0.179 -> 0.213 ms)
        if (c->overlap && !first) HIPCHK(c, hipStreamWaitEvent(band, prev_bulk, 0));
        {
            // relabel and the stress divergence (one pass); with overlap also
            // the lattice update of the window's nodes
            Bracket b(c, 3, band);
            const LbFuse lf{c->lat[s.cur], c->lat[s.nxt], c->Fx[s.nxt], c->Fy[s.nxt], s.wprev,
                            ox, oy};
            HIPCHK(c, launch_force(g, c->body, c->bb, s, c->Fx[s.cur], c->Fy[s.cur], c->drho,
                                   band, c->overlap ? &lf : nullptr));
            // the new solid box into the next ring slot (the band lattice
            // launch does this when the force pass leaves the lattice to it)
            if (c->overlap) HIPCHK(c, launch_reduce_window(g, c->bb, s.wcur, s.wnext, band));
            b.done();
        }
        if (c->overlap) {
            // prev_join and prev_bulk are the previous step's events
            // the early tiles of a held bulk update: the tile rows of its
            // range that lie wholly below the previous step's window (by more
            // than BULK_EARLY_GAP rows), launched after the previous step's
            // bulk update alone.  The chain of the previous step writes the
            // lattice and the forces only inside that window, and reads the
            // lattice only there and one node around it; this step's window
            // lies above those rows (its box moves down by BULK_EARLY_GAP rows
            // at most, else health[6] counts it), and the launch reads
            // neither this step's window nor a force plane
            const int early = hold_bulk && !c->timing ? bulk_early(c) : 0;
            if (early > 0)
                HIPCHK(c, launch_lb(g, prec, c->lb_variant, c->lat[s.cur], c->lat[s.nxt],
                                    c->Fx[s.nxt], c->Fy[s.nxt], c->Fx[s.cur], c->Fy[s.cur],
                                    c->drho, c->bb.win, s.wprev, s.wcur, ox, oy, 3,
                                    c->bb.health, main_s, 0, nullptr, 0, nullptr, 0, 0, early,
                                    1));
            if (hold_bulk) HIPCHK(c, hipStreamWaitEvent(main_s, ev_adv, 0));
            else if (!first) HIPCHK(c, hipStreamWaitEvent(main_s, prev_join, 0));
            HIPCHK(c, hipEventRecord(ev_join, c->side));
            {
                // every node outside the window (but the early tiles): its
                // update needs no force of this step's chain
                Bracket b(c, 4, main_s);
                HIPCHK(c, launch_lb(g, prec, c->lb_variant, c->lat[s.cur], c->lat[s.nxt], c->Fx[s.nxt],
                                    c->Fy[s.nxt], c->Fx[s.cur], c->Fy[s.cur], c->drho, c->bb.win,
                                    s.wprev, s.wcur, ox, oy, 3, c->bb.health, main_s,
                                    c->bulk_blocks, nullptr, 0, nullptr, 0, early, 1000,
                                    early > 0 ? 2 : 0));
                b.done();
            }
            if (last) HIPCHK(c, hipStreamWaitEvent(main_s, ev_join, 0));
            else HIPCHK(c, hipEventRecord(ev_bulk, main_s));
            return LBRMT_OK;
        }
    }
    Bracket b(c, 4, main_s);
    HIPCHK(c, launch_lb(g, prec, c->lb_variant, c->lat[s.cur], c->lat[s.nxt], c->Fx[s.nxt],
                        c->Fy[s.nxt], c->Fx[s.cur], c->Fy[s.cur], c->drho, c->bb.win, s.wprev,
                        s.wcur, ox, oy, 0, c->bb.health, main_s, 0, c->bb.boxpart,
                        c->nsolid > 0 ? RELABEL_BLOCKS : 0, c->bb.win, s.wnext));
    b.done();
    return LBRMT_OK;
}

// Capture steps 6 + p .. 6 + p + r - 1 into *out.  Steps n and n + 6 (n >= 6)
// enqueue identical launches (every buffer parity and ring slot repeats with
// period six), so such a graph replays any run of r steps that starts at a
// step count = p mod 6, p + r <= 6.
// The captured graph goes to *src, kept (as the executable graph needs
// nothing of it) until the executable graph is destroyed.
static int capture_steps(lbrmt_ctx* c, int p, int r, hipGraphExec_t* out, hipGraph_t* src)
{
    hipGraph_t graph = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    int rc = LBRMT_OK;
    for (int k = 0; k < r && rc == LBRMT_OK; k++)
        rc = enqueue_step(c, GRAPH_STEPS + p + k, c->cap, k == 0, k == r - 1);
    hipError_t e = hipStreamEndCapture(c->cap, &graph);
    if (rc != LBRMT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(c, "hipStreamEndCapture", e);
    e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        *out = nullptr;
        return fail(c, "hipGraphInstantiate", e);
    }
    *src = graph;
    return LBRMT_OK;
}

static int build_graph(lbrmt_ctx* c)
{
    return capture_steps(c, 0, GRAPH_STEPS, &c->gexec, &c->gsrc);
}

// every executable graph, then the graph it was made from
static void destroy_graphs(lbrmt_ctx* c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->gsrc) (void)hipGraphDestroy(c->gsrc);
    c->gexec = nullptr;
    c->gsrc = nullptr;
    for (int p = 0; p < GRAPH_STEPS; p++)
        for (int r = 0; r < GRAPH_STEPS; r++) {
            if (c->pexec[p][r]) (void)hipGraphExecDestroy(c->pexec[p][r]);
            if (c->psrc[p][r]) (void)hipGraphDestroy(c->psrc[p][r]);
            c->pexec[p][r] = nullptr;
            c->psrc[p][r] = nullptr;
        }
}

// Destroy every captured graph (after synchronising the stream that replays
// them): they bake the launch configuration and the solids in.
static int drop_graphs(lbrmt_ctx* c)
{
    bool any = c->gexec != nullptr;
    for (int p = 0; p < GRAPH_STEPS; p++)
        for (int r = 0; r < GRAPH_STEPS; r++) any = any || c->pexec[p][r];
    if (!any) return LBRMT_OK;
    HIPCHK(c, hipStreamSynchronize(c->st));
    destroy_graphs(c);
    return LBRMT_OK;
}

static bool desc_ok(const lbrmt_grid_desc* d)
{
    return d && d->nx >= 8 && d->ny >= 8 && d->tau > 0.5 && d->layers >= 1 &&
           d->layers <= MAX_LAYERS && (long long)(d->nx + 4) * (d->ny + 4) < (1ll << 26) &&
           d->r_max >= 2 && d->r_max <= 32 && d->eps > 0.0 && d->rho_f > 0.0 &&
           (d->lid_rho_mode == 0 || d->lid_rho_mode == 1) && !std::isnan(d->kappa_J) &&
           (d->precision == LBRMT_FP64 || d->precision == LBRMT_FP32);
}

extern "C" {

const char* lbrmt_status_string(int s)
{
    switch (s) {
    case LBRMT_OK: return "ok";
    case LBRMT_EINVAL: return "invalid argument";
    case LBRMT_EWORKSPACE: return "workspace too small or misaligned";
    case LBRMT_EHIP: return "HIP error";
    case LBRMT_EUNSTABLE: return "device health counters report a failure";
    case LBRMT_ECAPACITY: return "capacity exceeded";
    case LBRMT_ESTATE: return "call out of order";
    default: return "unknown status";
    }
}

const char* lbrmt_last_error(const lbrmt_ctx* c) { return c ? c->err.c_str() : ""; }

int lbrmt_workspace_bytes(const lbrmt_grid_desc* d, int32_t max_solids, size_t* bytes)
{
    if (!desc_ok(d) || !bytes || max_solids < 0 || max_solids > LBRMT_MAX_SOLIDS)
        return LBRMT_EINVAL;
    *bytes = make_layout(d, max_solids).total;
    return LBRMT_OK;
}

// Lattice tile variants chosen by lbrmt_autotune / lbrmt_batch_autotune,
// remembered for the process: per (nx, ny, precision) for a context, per
// (member count, node total, precision) for a batch.  Contexts and batches
// created later with the same key start with the remembered variant.
static std::mutex g_tune_mu;
static std::map<std::tuple<int, long long, long long, int>, int> g_tuned;

static int tuned_variant(int kind, long long a, long long b, int precision, int fallback)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(std::make_tuple(kind, a, b, precision));
    return it == g_tuned.end() ? fallback : it->second;
}

static void remember_variant(int kind, long long a, long long b, int precision, int v)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[std::make_tuple(kind, a, b, precision)] = v;
}

static int create_impl(const lbrmt_grid_desc* d, int32_t max_solids, void* ws, size_t bytes,
                       void* stream, lbrmt_ctx** out, bool member)
{
    if (!desc_ok(d) || !out || !ws || max_solids < 0) return LBRMT_EINVAL;
    if (max_solids > LBRMT_MAX_SOLIDS || (member && max_solids > 1)) return LBRMT_ECAPACITY;
    if ((uintptr_t)ws % ALIGN) return LBRMT_EWORKSPACE;
    Layout L = make_layout(d, max_solids);
    if (bytes < L.total) return LBRMT_EWORKSPACE;
    lbrmt_ctx* c = new lbrmt_ctx();
    c->d = *d;
    // measured fastest tile shapes: 64 x 4 (FP64), 256 x 1 (FP32), nontemporal
    // stores; or the variant an earlier lbrmt_autotune chose for this shape
    c->lb_variant = d->precision == LBRMT_FP64 ? 3 : 5;
    if (!member) c->lb_variant = tuned_variant(0, d->nx, d->ny, d->precision, c->lb_variant);
    c->L = L;
    c->max_solids = max_solids;
    c->st = (hipStream_t)stream;
    c->ws = (char*)ws;
    GridP& g = c->g;
    g.nx = d->nx;
    g.ny = d->ny;
    g.pitch = L.pitch;
    g.pp = L.pp;
    g.plane = (long long)L.plane;
    g.pplane = (long long)L.pplane;
    g.px = d->periodic_x ? 1 : 0;
    g.py = d->periodic_y ? 1 : 0;
    g.layers = d->layers;
    g.r_max = d->r_max;
    g.omega = 1.0 / d->tau;
    g.cforce = 1.0 - 1.0 / (2.0 * d->tau);
    g.lid_ux = d->periodic_y ? 0.0 : d->lid_ux;
    g.gx = d->gx;
    g.gy = d->gy;
    g.fext_x = d->fext_x;
    g.fext_y = d->fext_y;
    g.rho_f = d->rho_f;
    g.eps = d->eps;
    g.det_rel = d->det_rel;
    g.detJ_min = d->detJ_min;
    g.rm32 = d->precision == LBRMT_FP64 ? 0 : 1;
    g.ox = g.oy = 0;
    g.wx = g.wy = 0;
    g.lnx = g.nx;
    g.lny = g.ny;
    g.lpx = g.px;
    g.lpy = g.py;
    g.eta = d->eta;
    g.lcap = sub_cap(g.pplane);
    g.kappa_J = d->kappa_J > 0.0 ? d->kappa_J : 0.25;
    g.lid_rho_mode = d->lid_rho_mode;
    c->body.present = 0;
    for (int k = 0; k < 2; k++) {
        c->lat[k] = c->ws + L.off_lat[k];
        c->Fx[k] = (double*)(c->ws + L.off_fx[k]);
        c->Fy[k] = (double*)(c->ws + L.off_fy[k]);
        c->bb.X[k] = (void*)(c->ws + L.off_X[k]);
        c->bb.Y[k] = (void*)(c->ws + L.off_Y[k]);
        c->bb.phi[k] = (void*)(c->ws + L.off_phi[k]);
    }
    c->drho = (double*)(c->ws + L.off_drho);
    c->bb.tag = (int8_t*)(c->ws + L.off_tag);
    c->bb.gcol = (int8_t*)(c->ws + L.off_gcol);
    c->bb.lists = (int*)(c->ws + L.off_lists);
    c->bb.lcount = (int*)(c->ws + L.off_lcount);
    c->bb.boxpart = (int*)(c->ws + L.off_boxpart);
    c->bb.ticket = (unsigned*)(c->ws + L.off_ticket);
    c->bb.cut_layer = (int8_t*)(c->ws + L.off_cut_layer);
    c->bb.cut_tiles = (int*)(c->ws + L.off_cut_tiles);
    c->bb.ncut = (int*)(c->ws + L.off_ncut);
    c->bb.ff_flag = (int*)(c->ws + L.off_ff_flag);
    c->bb.ff_list = (int*)(c->ws + L.off_ff_list);
    c->bb.ff_n = (int*)(c->ws + L.off_ff_n);
    c->bb.win = (Win*)(c->ws + L.off_win);
    c->bb.health = (unsigned*)(c->ws + L.off_health);
    c->dpart = (double*)(c->ws + L.off_dpart);
    c->dout = (double*)(c->ws + L.off_dout);
    c->member = member;
    if (max_solids > 1) {
        c->multi = true;
        c->mg = mb_geom(d);
        c->BL = body_layout(d, c->mg);
        for (int k = 0; k < 2; k++) {
            c->stamp[k] = (int*)(c->ws + L.off_stamp[k]);
            c->mlist[k] = (int*)(c->ws + L.off_mlist[k]);
        }
        c->mcount = (int*)(c->ws + L.off_mcount);
        c->dstep = (long long*)(c->ws + L.off_dstep);
        c->mbd = (MbBody*)(c->ws + L.off_mbtab);
        c->bsum = (double*)(c->ws + L.off_bsum);
        c->mord = (int*)(c->ws + L.off_mord);
        char* t = c->ws + L.off_tabs;
        auto carve = [&](size_t bytes_) {
            char* p_ = t;
            t += round_up(bytes_, ALIGN);
            return p_;
        };
        for (int p = 0; p < 7; p++) {
            c->mtab[p].adv = (AdvectArgs*)carve(max_solids * sizeof(AdvectArgs));
            c->mtab[p].lay = (LayersArgs*)carve(max_solids * sizeof(LayersArgs));
            c->mtab[p].fit = (FitArgs*)carve(max_solids * sizeof(FitArgs));
            c->mtab[p].edg = (EdgesArgs*)carve(max_solids * sizeof(EdgesArgs));
            c->mtab[p].lb = nullptr;
            c->mtab[p].ord = c->mord;
        }
    }
    if (member) {
        // a batch member is stepped by its batch, on the batch's stream
        c->graph = false;
        *out = c;
        return LBRMT_OK;
    }
    hipError_t e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
    for (int k = 0; k < GRAPH_STEPS; k++) {
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork[k], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join[k], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_adv[k], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_bulk[k], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        int rc = fail(c, "stream/event creation", e);
        lbrmt_destroy(c);
        return rc;
    }
    *out = c;
    return LBRMT_OK;
}

int lbrmt_create(const lbrmt_grid_desc* d, int32_t max_solids, void* ws, size_t bytes,
                 void* stream, lbrmt_ctx** out)
{
    return create_impl(d, max_solids, ws, bytes, stream, out, false);
}

void lbrmt_destroy(lbrmt_ctx* c)
{
    if (!c) return;
    // (st may be the null stream: it is synchronised too)
    (void)hipStreamSynchronize(c->st);
    if (c->side) (void)hipStreamSynchronize(c->side);
    for (auto& p : c->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    destroy_graphs(c);
    for (int k = 0; k < GRAPH_STEPS; k++) {
        if (c->ev_fork[k]) (void)hipEventDestroy(c->ev_fork[k]);
        if (c->ev_join[k]) (void)hipEventDestroy(c->ev_join[k]);
        if (c->ev_adv[k]) (void)hipEventDestroy(c->ev_adv[k]);
        if (c->ev_bulk[k]) (void)hipEventDestroy(c->ev_bulk[k]);
    }
    if (c->cap) (void)hipStreamDestroy(c->cap);
    if (c->side) (void)hipStreamDestroy(c->side);
    delete c;
}

// disc of radius a > 0, or ellipse of semi-axes a, b > 0
static bool solid_shape_ok(const lbrmt_solid_desc& s)
{
    return (s.shape == 0 && s.a > 0.0) || (s.shape == 1 && s.a > 0.0 && s.b > 0.0);
}

// largest distance from the centre to the reference shape's boundary
static double solid_extent(const lbrmt_solid_desc& s)
{
    return s.shape == 1 ? std::max(s.a, s.b) : s.a;
}

static BodyP body_of(const lbrmt_solid_desc& s)
{
    BodyP b{};
    b.present = 1;
    b.shape = s.shape;
    b.cx = s.cx;
    b.cy = s.cy;
    b.R = s.a;
    b.Rb = s.shape == 1 ? s.b : s.a;
    b.ct = s.shape == 1 ? std::cos(s.theta) : 1.0;
    b.st = s.shape == 1 ? std::sin(s.theta) : 0.0;
    b.G = s.G;
    b.rho_s = s.rho_s;
    return b;
}

// solid k of a several-solid context: its window grid and buffers
static MbBody mb_body(lbrmt_ctx* c, int k, const lbrmt_solid_desc& s)
{
    MbBody m{};
    const MbGeom& G = c->mg;
    GridP g = c->g;
    g.nx = G.nx;
    g.ny = G.ny;
    g.pp = G.pp;
    g.pplane = (long long)G.pplane;
    g.px = G.wx ? 0 : c->g.px;
    g.py = G.wy ? 0 : c->g.py;
    g.wx = G.wx;
    g.wy = G.wy;
    g.ox = G.wx ? (int)std::floor(s.cx) - G.nx / 2 : 0;
    g.oy = G.wy ? (int)std::floor(s.cy) - G.ny / 2 : 0;
    g.lcap = G.lcap;
    m.g = g;
    m.b = body_of(s);
    char* base = c->ws + c->L.off_bodies + (size_t)k * c->L.body_bytes;
    for (int q = 0; q < 2; q++) {
        m.X[q] = base + c->BL.off_X[q];
        m.Y[q] = base + c->BL.off_Y[q];
        m.phi[q] = base + c->BL.off_phi[q];
    }
    m.win = (Win*)(base + c->BL.off_win);
    m.boxpart = (int*)(base + c->BL.off_boxpart);
    m.reg = make_int4(0, -1, 0, -1);
    return m;
}

// the chain buffers of solid k (health counters shared by the context)
static BandBufs mb_bufs(const lbrmt_ctx* c, int k)
{
    BandBufs b{};
    const MbBody& m = c->mbh[k];
    char* base = c->ws + c->L.off_bodies + (size_t)k * c->L.body_bytes;
    for (int q = 0; q < 2; q++) {
        b.X[q] = m.X[q];
        b.Y[q] = m.Y[q];
        b.phi[q] = m.phi[q];
    }
    b.tag = (int8_t*)(base + c->BL.off_tag);
    b.gcol = (int8_t*)(base + c->BL.off_gcol);
    b.lists = (int*)(base + c->BL.off_lists);
    b.lcount = (int*)(base + c->BL.off_lcount);
    b.boxpart = m.boxpart;
    b.ticket = (unsigned*)(base + c->BL.off_ticket);
    b.win = m.win;
    b.health = c->bb.health;
    b.cut_layer = nullptr;  // one launch per layer for several solids
    b.cut_tiles = nullptr;
    b.ncut = nullptr;
    b.ff_flag = nullptr;
    b.ff_list = nullptr;
    b.ff_n = nullptr;
    return b;
}

int lbrmt_add_solids(lbrmt_ctx* c, const lbrmt_solid_desc* s, int32_t n)
{
    if (!c || (n > 0 && !s) || n < 0) return LBRMT_EINVAL;
    if (c->inited) return LBRMT_ESTATE;
    if (c->nsolid + n > c->max_solids) return LBRMT_ECAPACITY;
    for (int k = 0; k < n; k++) {
        if (!solid_shape_ok(s[k]) || !(s[k].rho_s > 0.0) || !(s[k].G >= 0.0))
            return LBRMT_EINVAL;
        // a solid and its zone must fit its window with a margin
        if (c->multi && (c->mg.wx || c->mg.wy)) {
            const double need = 2.0 * (std::ceil(solid_extent(s[k])) + c->d.layers + 4);
            if ((c->mg.wx && need > c->mg.nx) || (c->mg.wy && need > c->mg.ny))
                return LBRMT_ECAPACITY;
        }
    }
    if (c->multi) {
        for (int k = 0; k < n; k++) c->mbh.push_back(mb_body(c, c->nsolid + k, s[k]));
        c->nsolid += n;
        return LBRMT_OK;
    }
    if (n > 0) {
        c->solid = s[0];
        c->nsolid = 1;
        c->body = body_of(s[0]);
    }
    return LBRMT_OK;
}

// argument tables of the chain kernels of every solid for the seven phases
// (n mod 6 for n >= 1, and n = 0), and the device solid table
static int mb_tables(lbrmt_ctx* c)
{
    const int nb = c->nsolid;
    if (nb == 0) return LBRMT_OK;
    std::vector<AdvectArgs> adv(nb);
    std::vector<LayersArgs> lay(nb);
    std::vector<FitArgs> fit(nb);
    std::vector<EdgesArgs> edg(nb);
    // the advection and extrapolation passes (a group of blocks, or one
    // block, per solid; more than the GPU holds at once) start the largest
    // solids first, so that the last blocks to start are the shortest: their
    // block rows take the solids by decreasing semi-axis sum (each solid's
    // work is its own, so the order changes no result)
    std::vector<int> ord(nb);
    for (int k = 0; k < nb; k++) ord[k] = k;
    auto size_of = [&](int k) {
        const BodyP& b = c->mbh[k].b;
        return b.R + (b.shape == 1 ? b.Rb : b.R);
    };
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int x, int y) { return size_of(x) > size_of(y); });
    HIPCHK(c, hipMemcpyAsync(c->mord, ord.data(), nb * sizeof(int), hipMemcpyHostToDevice, c->st));
    for (int p = 0; p < 7; p++) {
        const long long nstep = p == 6 ? 0 : (p == 0 ? 6 : p);
        const StepSlots s = slots_for(nstep);
        for (int k = 0; k < nb; k++) {
            const BandBufs b = mb_bufs(c, k);
            const GridP& g = c->mbh[k].g;
            adv[k] = AdvectArgs{g, c->lat[s.cur], c->Fx[s.nxt], c->Fy[s.nxt], b.X[s.cur],
                                b.Y[s.cur], b.phi[s.cur], b.X[s.nxt], b.Y[s.nxt], b.tag, b.win,
                                s.wprev, s.wcur, b.lists, b.lcount, b.health};
            lay[k] = LayersArgs{g, b.win, s.wcur, b.tag, b.gcol, b.lists, b.lcount, b.health};
            fit[k] = FitArgs{g, b.win, s.wcur, s.wprev, b.tag, b.lists, b.lcount, b.phi[s.cur],
                             b.X[s.nxt], b.Y[s.nxt], b.health};
            edg[k] = EdgesArgs{g, c->mbh[k].b, b.win, s.wcur, b.boxpart, b.X[s.nxt], b.Y[s.nxt],
                               b.tag, b.phi[s.nxt], nullptr, nullptr, nullptr, b.lcount,
                               b.health};
        }
        const BatchTables& T = c->mtab[p];
        HIPCHK(c, hipMemcpyAsync(T.adv, adv.data(), nb * sizeof(AdvectArgs), hipMemcpyHostToDevice, c->st));
        HIPCHK(c, hipMemcpyAsync(T.lay, lay.data(), nb * sizeof(LayersArgs), hipMemcpyHostToDevice, c->st));
        HIPCHK(c, hipMemcpyAsync(T.fit, fit.data(), nb * sizeof(FitArgs), hipMemcpyHostToDevice, c->st));
        HIPCHK(c, hipMemcpyAsync(T.edg, edg.data(), nb * sizeof(EdgesArgs), hipMemcpyHostToDevice, c->st));
        // the host vectors are reused for the next phase: wait for the copies
        HIPCHK(c, hipStreamSynchronize(c->st));
    }
    HIPCHK(c, hipMemcpyAsync(c->mbd, c->mbh.data(), nb * sizeof(MbBody), hipMemcpyHostToDevice,
                             c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    return LBRMT_OK;
}

// several solids: every solid's initial map on its window (as for one solid),
// then the density excess of the mixture, then f = f^eq
static int init_mb(lbrmt_ctx* c, const double* d_u0)
{
    hipStream_t st = c->st;
    const size_t nblk = (size_t)c->L.nbx * c->L.nby;
    for (int k = 0; k < 2; k++) HIPCHK(c, hipMemsetAsync(c->stamp[k], 0, nblk * 4, st));
    HIPCHK(c, hipMemsetAsync(c->mcount, 0, 2 * 4, st));
    HIPCHK(c, hipMemsetAsync(c->dstep, 0, 8, st));
    const int nb = c->nsolid;
    for (int k = 0; k < nb; k++) {
        const BandBufs b = mb_bufs(c, k);
        const GridP& g = c->mbh[k].g;
        const BodyP& bp = c->mbh[k].b;
        HIPCHK(c, hipMemsetAsync(b.ticket, 0, 4, st));
        HIPCHK(c, hipMemsetAsync(b.lcount, 0, (size_t)(MAX_LAYERS + 1) * NSUB * LCOUNT_PAD * 4, st));
        for (int q = 0; q < 3; q++) HIPCHK(c, launch_win_reset(b.win, q, st));
        HIPCHK(c, launch_init_solid_box(g, bp, b, 0, 2, st));
        HIPCHK(c, launch_init_tags(g, bp, b, 0, st));
        HIPCHK(c, launch_layers(g, b, 0, st));
        HIPCHK(c, launch_init_fill(g, bp, b, 0, st));
    }
    int rc = mb_tables(c);
    if (rc != LBRMT_OK) return rc;
    if (nb > 0) {
        // the blocks of the initial regions (stamp -1, which no step uses)
        HIPCHK(c, launch_mb_mark(c->g, c->mbd, nb, 0, 0, 0, c->stamp[1], -1, c->mlist[1],
                                 &c->mcount[1], c->L.nbx, c->bb.health, st));
        HIPCHK(c, launch_mb_combine(c->g, c->d.precision, c->mbd, nb, 0, 0, c->mlist[1],
                                    &c->mcount[1], &c->mcount[0], c->L.nbx, c->Fx[0], c->Fy[0],
                                    c->drho, true, c->bb.health, st));
    }
    BodyP none{};
    HIPCHK(c, launch_init_populations(c->g, c->d.precision, none, nullptr, c->bb.win, 0, d_u0,
                                      c->lat[1], c->lat[0], st, c->drho));
    c->step = 0;
    c->inited = true;
    return LBRMT_OK;
}

// the fused extrapolation's tile lists start empty (k_fit_rest leaves them so)
static hipError_t clear_cut_tiles(lbrmt_ctx* c, hipStream_t st)
{
    if (c->multi) return hipSuccess;  // several solids: no fused extrapolation
    const size_t nt = (size_t)fused_tiles(c->d.nx, c->d.ny);
    hipError_t e = hipMemsetAsync(c->bb.cut_layer, FF_NO_CUT, nt, st);
    if (e == hipSuccess) e = hipMemsetAsync(c->bb.ncut, 0, 4, st);
    if (e == hipSuccess) e = hipMemsetAsync(c->bb.ff_flag, 0, nt * 4, st);
    if (e == hipSuccess) e = hipMemsetAsync(c->bb.ff_n, 0, 4, st);
    return e;
}

int lbrmt_init(lbrmt_ctx* c, const double* d_u0)
{
    if (!c) return LBRMT_EINVAL;
    const GridP& g = c->g;
    hipStream_t st = c->st;
    HIPCHK(c, hipMemsetAsync(c->bb.health, 0, LBRMT_H_COUNT * sizeof(unsigned), st));
    for (int k = 0; k < 2; k++) {
        HIPCHK(c, hipMemsetAsync(c->Fx[k], 0, c->L.plane * 8, st));
        HIPCHK(c, hipMemsetAsync(c->Fy[k], 0, c->L.plane * 8, st));
    }
    HIPCHK(c, hipMemsetAsync(c->drho, 0, c->L.plane * 8, st));
    HIPCHK(c, hipMemsetAsync(c->bb.ticket, 0, 4, st));
    HIPCHK(c, clear_cut_tiles(c, st));
    for (int k = 0; k < 3; k++) HIPCHK(c, launch_win_reset(c->bb.win, k, st));
    {
        // graphs captured for an earlier initialisation bake the old solids in
        int rc = drop_graphs(c);
        if (rc != LBRMT_OK) return rc;
    }
    if (c->multi) return init_mb(c, d_u0);
    if (c->nsolid > 0) {
        // box of S^0 into the slots of "current" (0) and "previous" (2)
        HIPCHK(c, launch_init_solid_box(g, c->body, c->bb, 0, 2, st));
        HIPCHK(c, launch_init_tags(g, c->body, c->bb, 0, st));
        HIPCHK(c, launch_layers(g, c->bb, 0, st));
        HIPCHK(c, launch_init_fill(g, c->body, c->bb, 0, st));
    }
    HIPCHK(c, launch_init_populations(g, c->d.precision, c->body, c->bb.phi[0], c->bb.win, 0,
                                      d_u0, c->lat[1], c->lat[0], st));
    c->step = 0;
    c->inited = true;
    return LBRMT_OK;
}

int lbrmt_step(lbrmt_ctx* c, int64_t nsteps)
{
    if (!c || nsteps < 0) return LBRMT_EINVAL;
    if (!c->inited || c->member) return LBRMT_ESTATE;
    int64_t left = nsteps;
    while (left > 0) {
        const bool use_graph = c->graph && !c->timing && c->step >= GRAPH_STEPS;
        const int p = (int)(c->step % GRAPH_STEPS);
        if (use_graph && p == 0 && left >= GRAPH_STEPS) {
            if (!c->gexec) {
                int rc = build_graph(c);
                if (rc != LBRMT_OK) return rc;
            }
            HIPCHK(c, hipGraphLaunch(c->gexec, c->st));
            c->step += GRAPH_STEPS;
            left -= GRAPH_STEPS;
        } else if (use_graph) {
            // up to the next six-step boundary, or the end of the run
            const int r = (int)std::min<int64_t>(left, GRAPH_STEPS - p);
            if (!c->pexec[p][r]) {
                int rc = capture_steps(c, p, r, &c->pexec[p][r], &c->psrc[p][r]);
                if (rc != LBRMT_OK) return rc;
            }
            HIPCHK(c, hipGraphLaunch(c->pexec[p][r], c->st));
            c->step += r;
            left -= r;
        } else {
            int rc = enqueue_step(c, c->step, c->st);
            if (rc != LBRMT_OK) return rc;
            c->step += 1;
            left -= 1;
        }
    }
    return LBRMT_OK;
}

int64_t lbrmt_step_count(const lbrmt_ctx* c) { return c ? c->step : -1; }

int lbrmt_read_macro(lbrmt_ctx* c, double* rho, double* ux, double* uy)
{
    if (!c) return LBRMT_EINVAL;
    if (!c->inited) return LBRMT_ESTATE;
    const StepSlots s = slots_for(c->step);
    HIPCHK(c, launch_gather_macro(c->g, c->d.precision, c->lat[s.cur], c->Fx[s.nxt], c->Fy[s.nxt],
                                  c->bb.win, s.wprev, fpo_x(c, c->step), fpo_y(c, c->step), rho,
                                  ux, uy, nullptr, c->st, prev_valid(c)));
    return LBRMT_OK;
}

int lbrmt_read_populations(lbrmt_ctx* c, double* f9)
{
    if (!c || !f9) return LBRMT_EINVAL;
    if (!c->inited) return LBRMT_ESTATE;
    const StepSlots s = slots_for(c->step);
    HIPCHK(c, launch_gather_macro(c->g, c->d.precision, c->lat[s.cur], c->Fx[s.nxt], c->Fy[s.nxt],
                                  c->bb.win, s.wprev, fpo_x(c, c->step), fpo_y(c, c->step),
                                  nullptr, nullptr, nullptr, f9, c->st, prev_valid(c)));
    return LBRMT_OK;
}

int lbrmt_read_force(lbrmt_ctx* c, double* fx, double* fy)
{
    if (!c || !fx || !fy) return LBRMT_EINVAL;
    if (!c->inited) return LBRMT_ESTATE;
    const StepSlots s = slots_for(c->step);
    HIPCHK(c, launch_read_force(c->g, c->Fx[s.nxt], c->Fy[s.nxt], c->bb.win, s.wprev,
                                fpo_x(c, c->step), fpo_y(c, c->step), fx, fy, c->st,
                                prev_valid(c)));
    return LBRMT_OK;
}

int lbrmt_read_refmap(lbrmt_ctx* c, int32_t solid, double* X, double* Y, double* phi)
{
    if (!c || solid < 0 || solid >= c->nsolid) return LBRMT_EINVAL;
    if (!c->inited) return LBRMT_ESTATE;
    const StepSlots s = slots_for(c->step);
    if (c->multi) {
        HIPCHK(c, launch_mb_read_refmap(c->g, c->d.precision, c->mbd, solid, s.cur, s.wprev, X, Y,
                                        phi, c->st));
        return LBRMT_OK;
    }
    HIPCHK(c, launch_read_refmap(c->g, c->body, c->bb, s.cur, s.wprev, X, Y, phi, c->st));
    return LBRMT_OK;
}

int lbrmt_read_stress(lbrmt_ctx* c, double* sxx, double* sxy, double* syy)
{
    if (!c || !sxx || !sxy || !syy) return LBRMT_EINVAL;
    if (!c->inited) return LBRMT_ESTATE;
    const StepSlots s = slots_for(c->step);
    if (c->multi) {
        HIPCHK(c, launch_mb_read_stress(c->g, c->d.precision, c->mbd, c->nsolid, s.cur, s.wprev,
                                        c->L.nbx, c->L.nby, sxx, sxy, syy, c->bb.health, c->st));
        return LBRMT_OK;
    }
    HIPCHK(c, launch_read_stress(c->g, c->body, c->bb, s.cur, s.wprev, sxx, sxy, syy, c->st));
    return LBRMT_OK;
}

// The reductions of lbrmt_diag with their scratch (per-block partial records,
// the reduced record, the per-solid sums) at the given device pointers.
static int diag_into(lbrmt_ctx* c, lbrmt_diag_t* out, double* dpart, double* dout, double* bsum)
{
    const StepSlots s = slots_for(c->step);
    BodyP none{};
    HIPCHK(c, launch_diag(c->g, c->d.precision, c->multi ? none : c->body, c->lat[s.cur],
                          c->Fx[s.nxt], c->Fy[s.nxt], c->bb.win, s.wprev, fpo_x(c, c->step),
                          fpo_y(c, c->step), c->bb, s.cur, dpart, dout, c->st,
                          prev_valid(c)));
    double h[16];
    unsigned hc[LBRMT_H_COUNT];
    std::vector<double> bs;
    HIPCHK(c, hipMemcpyAsync(h, dout, 11 * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipMemcpyAsync(hc, c->bb.health, sizeof hc, hipMemcpyDeviceToHost, c->st));
    if (c->multi && c->nsolid > 0) {
        bs.resize((size_t)c->nsolid * 7);
        HIPCHK(c, launch_mb_diag(c->d.precision, c->mbd, c->nsolid, s.cur, s.wprev, bsum,
                                 c->st));
        HIPCHK(c, hipMemcpyAsync(bs.data(), bsum, bs.size() * sizeof(double),
                                 hipMemcpyDeviceToHost, c->st));
    }
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (c->multi) {
        // the solid terms summed over the solids, in index order
        double t[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int k = 0; k < c->nsolid; k++)
            for (int q = 0; q < 7; q++) t[q] += bs[(size_t)k * 7 + q];
        h[3] = t[0];
        h[4] = t[1];
        h[5] = t[2];
        h[6] = t[3];
        h[7] = t[4];
        h[8] = t[5];
        h[9] = t[6];
    }
    out->step = c->step;
    out->mass = h[0];
    out->mom_x = h[1];
    out->mom_y = h[2];
    out->centroid_x = h[3] > 0 ? h[4] / h[3] : NAN;
    out->centroid_y = h[3] > 0 ? h[5] / h[3] : NAN;
    out->disp_x = h[3] > 0 ? h[6] / h[3] : NAN;
    out->disp_y = h[3] > 0 ? h[7] / h[3] : NAN;
    out->n_solid = h[8];
    out->n_band = h[9];
    out->lambda_sum = h[3];
    out->max_u = h[10];
    for (int k = 0; k < LBRMT_H_COUNT; k++) out->health[k] = hc[k];
    if (hc[LBRMT_H_NONFINITE] || hc[LBRMT_H_DETJ_SOLID] || hc[LBRMT_H_EXTRAP_FAIL] ||
        hc[LBRMT_H_LIST_OVERFLOW] || hc[LBRMT_H_WINDOW_CLIP] || !std::isfinite(h[0]))
        return LBRMT_EUNSTABLE;
    return LBRMT_OK;
}

int lbrmt_diag(lbrmt_ctx* c, lbrmt_diag_t* out)
{
    if (!c || !out) return LBRMT_EINVAL;
    if (!c->inited) return LBRMT_ESTATE;
    return diag_into(c, out, c->dpart, c->dout, c->bsum);
}

int lbrmt_diag_sums(lbrmt_ctx* c, double* d_out)
{
    if (!c || !d_out) return LBRMT_EINVAL;
    if (!c->inited) return LBRMT_ESTATE;
    if (c->multi) {
        c->err = "lbrmt_diag_sums: one solid at most (use lbrmt_diag)";
        return LBRMT_ESTATE;
    }
    const StepSlots s = slots_for(c->step);
    HIPCHK(c, launch_diag(c->g, c->d.precision, c->body, c->lat[s.cur], c->Fx[s.nxt],
                          c->Fy[s.nxt], c->bb.win, s.wprev, fpo_x(c, c->step),
                          fpo_y(c, c->step), c->bb, s.cur, c->dpart, d_out, c->st,
                          prev_valid(c)));
    return LBRMT_OK;
}

// lbrmt_diag_noalloc: the same reductions with their scratch in a file-scope
// device array instead of the context's workspace.  Each GPU holds its own
// copy of the array (until the process ends); its address on a device is
// looked up once, with that device current, on the first call there.  In
// host code `scratch` names a host-side stand-in, never the device memory:
// only the looked-up address is passed to kernels and copies.
int lbrmt_diag_noalloc(lbrmt_ctx* c, lbrmt_diag_t* out)
{
    if (!c || !out) return LBRMT_EINVAL;
    if (!c->inited) return LBRMT_ESTATE;
    if (c->multi && c->nsolid > LBRMT_DIAG_NOALLOC_MAX_SOLIDS) {
        char buf[160];
        snprintf(buf, sizeof buf,
                 "lbrmt_diag_noalloc: %d solids exceed the %d its static scratch holds",
                 c->nsolid, (int)LBRMT_DIAG_NOALLOC_MAX_SOLIDS);
        c->err = buf;
        return LBRMT_EINVAL;
    }
    if (diag_partial_doubles() * 8 > NOALLOC_PART_BYTES) {
        c->err = "lbrmt_diag_noalloc: partial records exceed the static scratch";
        return LBRMT_EINVAL;
    }
    char* base = nullptr;
    {
        int dev = -1;
        HIPCHK(c, hipGetDevice(&dev));
        if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
            c->err = "lbrmt_diag_noalloc: device index beyond the supported range";
            return LBRMT_EINVAL;
        }
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void* p = nullptr;
            HIPCHK(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
            if (!p) {
                c->err = "lbrmt_diag_noalloc: no device address for the static scratch";
                return LBRMT_EHIP;
            }
            g_scratch_ptr[dev] = (char*)p;
        }
        base = g_scratch_ptr[dev];
    }
    // every kernel of the diagnostic writes its whole slice of the scratch
    // (one record per reduction block, the reduced record, one record per
    // solid), so nothing is cleared first
    return diag_into(c, out, (double*)(base + NOALLOC_PART_OFF), (double*)(base + NOALLOC_OUT_OFF),
                     (double*)(base + NOALLOC_SOLID_OFF));
}

int lbrmt_diag_solid(lbrmt_ctx* c, int32_t solid, double* out)
{
    if (!c || !out || solid < 0 || solid >= c->nsolid) return LBRMT_EINVAL;
    if (!c->inited) return LBRMT_ESTATE;
    if (!c->multi) {
        lbrmt_diag_t d;
        const int rc = lbrmt_diag(c, &d);
        if (rc != LBRMT_OK && rc != LBRMT_EUNSTABLE) return rc;
        out[0] = d.centroid_x;
        out[1] = d.centroid_y;
        out[2] = d.disp_x;
        out[3] = d.disp_y;
        out[4] = d.n_solid;
        out[5] = d.n_band;
        return LBRMT_OK;
    }
    const StepSlots s = slots_for(c->step);
    std::vector<double> bs((size_t)c->nsolid * 7);
    HIPCHK(c, launch_mb_diag(c->d.precision, c->mbd, c->nsolid, s.cur, s.wprev, c->bsum, c->st));
    HIPCHK(c, hipMemcpyAsync(bs.data(), c->bsum, bs.size() * sizeof(double),
                             hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    const double* a = &bs[(size_t)solid * 7];
    out[0] = a[0] > 0 ? a[1] / a[0] : NAN;
    out[1] = a[0] > 0 ? a[2] / a[0] : NAN;
    out[2] = a[0] > 0 ? a[3] / a[0] : NAN;
    out[3] = a[0] > 0 ? a[4] / a[0] : NAN;
    out[4] = a[5];
    out[5] = a[6];
    return LBRMT_OK;
}

// ---------------------------------------------------------------- adjoint

namespace {

struct SnapLayout {
    size_t A, fpx, fpy, fcx, fcy, X0, Y0, P0, X1, Y1, P1, tag, win, fpo, total;
};

SnapLayout snap_layout(const lbrmt_ctx* c)
{
    SnapLayout S;
    size_t o = 0;
    auto take = [&](size_t b) {
        size_t r = o;
        o = round_up(o + b, ALIGN);
        return r;
    };
    const size_t pl = c->L.plane * 8, rp = c->L.pplane * 8;
    S.A = take(c->L.lat_bytes);
    S.fpx = take(pl);
    S.fpy = take(pl);
    S.fcx = take(pl);
    S.fcy = take(pl);
    S.X0 = take(rp);
    S.Y0 = take(rp);
    S.P0 = take(rp);
    S.X1 = take(rp);
    S.Y1 = take(rp);
    S.P1 = take(rp);
    S.tag = take(c->L.pplane);
    S.win = take(2 * sizeof(Win));
    S.fpo = take(2 * 8);
    S.total = o;
    return S;
}

AdjSnap adj_snap(const lbrmt_ctx* c, const void* snap)
{
    const SnapLayout S = snap_layout(c);
    const char* b = (const char*)snap;
    AdjSnap a;
    a.A = (const double*)(b + S.A);
    a.fpx = (const double*)(b + S.fpx);
    a.fpy = (const double*)(b + S.fpy);
    a.fcx = (const double*)(b + S.fcx);
    a.fcy = (const double*)(b + S.fcy);
    a.X0 = (const double*)(b + S.X0);
    a.Y0 = (const double*)(b + S.Y0);
    a.P0 = (const double*)(b + S.P0);
    a.X1 = (const double*)(b + S.X1);
    a.Y1 = (const double*)(b + S.Y1);
    a.P1 = (const double*)(b + S.P1);
    a.tag = (const int8_t*)(b + S.tag);
    a.win = (const Win*)(b + S.win);
    a.fpo = (const double*)(b + S.fpo);
    return a;
}

struct AdjLayout {
    size_t fb[2], x[2], y[2], p[2], Fx[2], Fy[2], acc, total;
};

AdjLayout adj_layout(const lbrmt_ctx* c)
{
    AdjLayout A;
    size_t o = 0;
    auto take = [&](size_t b) {
        size_t r = o;
        o = round_up(o + b, ALIGN);
        return r;
    };
    const size_t N = (size_t)c->d.nx * c->d.ny, rp = c->L.pplane * 8;
    for (int k = 0; k < 2; k++) {
        A.fb[k] = take(NQ * N * 8);
        A.x[k] = take(rp);
        A.y[k] = take(rp);
        A.p[k] = take(rp);
        A.Fx[k] = take(N * 8);
        A.Fy[k] = take(N * 8);
    }
    A.acc = take(2 * 8);
    A.total = o;
    return A;
}

AdjBufs adj_bufs(const lbrmt_ctx* c, void* adj)
{
    const AdjLayout L = adj_layout(c);
    char* b = (char*)adj;
    const int f = c->adj_flip, h = 1 - f;
    AdjBufs a;
    a.fb_in = (const double*)(b + L.fb[f]);
    a.fb_out = (double*)(b + L.fb[h]);
    a.xbar1 = (double*)(b + L.x[f]);
    a.ybar1 = (double*)(b + L.y[f]);
    a.pbar1 = (double*)(b + L.p[f]);
    a.xbar0 = (double*)(b + L.x[h]);
    a.ybar0 = (double*)(b + L.y[h]);
    a.pbar0 = (double*)(b + L.p[h]);
    a.Fcbar_x = (double*)(b + L.Fx[f]);
    a.Fcbar_y = (double*)(b + L.Fy[f]);
    a.Fpbar_x = (double*)(b + L.Fx[h]);
    a.Fpbar_y = (double*)(b + L.Fy[h]);
    a.acc = (double*)(b + L.acc);
    return a;
}

bool adj_ok(const lbrmt_ctx* c)
{
    return c && !c->multi && !c->member && c->d.precision == LBRMT_FP64 && c->nsolid <= 1;
}

}  // namespace

int lbrmt_snapshot_bytes(const lbrmt_ctx* c, size_t* bytes)
{
    if (!c || !bytes) return LBRMT_EINVAL;
    if (!adj_ok(c)) return LBRMT_ESTATE;
    *bytes = snap_layout(c).total;
    return LBRMT_OK;
}

int lbrmt_step_snapshot(lbrmt_ctx* c, void* snap)
{
    if (!c || !snap) return LBRMT_EINVAL;
    if (!c->inited || !adj_ok(c)) return LBRMT_ESTATE;
    const long long n = c->step;
    const StepSlots s = slots_for(n);
    // eager launches; with the chain on the internal stream the step ends
    // joined into the context stream, so the copies below follow all of it
    int rc = enqueue_step(c, n, c->st);
    if (rc != LBRMT_OK) return rc;
    c->step = n + 1;
    const SnapLayout S = snap_layout(c);
    char* b = (char*)snap;
    const hipMemcpyKind D2D = hipMemcpyDeviceToDevice;
    const size_t pl = c->L.plane * 8, rp = c->L.pplane * 8;
    hipStream_t st = c->st;
    HIPCHK(c, hipMemcpyAsync(b + S.A, c->lat[s.cur], c->L.lat_bytes, D2D, st));
    HIPCHK(c, hipMemcpyAsync(b + S.fpx, c->Fx[s.nxt], pl, D2D, st));
    HIPCHK(c, hipMemcpyAsync(b + S.fpy, c->Fy[s.nxt], pl, D2D, st));
    HIPCHK(c, hipMemcpyAsync(b + S.fcx, c->Fx[s.cur], pl, D2D, st));
    HIPCHK(c, hipMemcpyAsync(b + S.fcy, c->Fy[s.cur], pl, D2D, st));
    if (c->nsolid > 0) {
        HIPCHK(c, hipMemcpyAsync(b + S.X0, c->bb.X[s.cur], rp, D2D, st));
        HIPCHK(c, hipMemcpyAsync(b + S.Y0, c->bb.Y[s.cur], rp, D2D, st));
        HIPCHK(c, hipMemcpyAsync(b + S.P0, c->bb.phi[s.cur], rp, D2D, st));
        HIPCHK(c, hipMemcpyAsync(b + S.X1, c->bb.X[s.nxt], rp, D2D, st));
        HIPCHK(c, hipMemcpyAsync(b + S.Y1, c->bb.Y[s.nxt], rp, D2D, st));
        HIPCHK(c, hipMemcpyAsync(b + S.P1, c->bb.phi[s.nxt], rp, D2D, st));
        HIPCHK(c, hipMemcpyAsync(b + S.tag, c->bb.tag, c->L.pplane, D2D, st));
    }
    HIPCHK(c, hipMemcpyAsync(b + S.win, c->bb.win + s.wprev, sizeof(Win), D2D, st));
    HIPCHK(c, hipMemcpyAsync(b + S.win + sizeof(Win), c->bb.win + s.wcur, sizeof(Win), D2D, st));
    HIPCHK(c, launch_set2((double*)(b + S.fpo), fpo_x(c, n), fpo_y(c, n), st));
    return LBRMT_OK;
}

int lbrmt_adjoint_bytes(const lbrmt_ctx* c, size_t* bytes)
{
    if (!c || !bytes) return LBRMT_EINVAL;
    if (!adj_ok(c)) return LBRMT_ESTATE;
    *bytes = adj_layout(c).total;
    return LBRMT_OK;
}

int lbrmt_adjoint_zero(lbrmt_ctx* c, void* adj)
{
    if (!c || !adj) return LBRMT_EINVAL;
    if (!adj_ok(c)) return LBRMT_ESTATE;
    HIPCHK(c, hipMemsetAsync(adj, 0, adj_layout(c).total, c->st));
    c->adj_flip = 0;
    return LBRMT_OK;
}

int lbrmt_adjoint_loss(lbrmt_ctx* c, void* adj, const void* snap, int32_t which,
                       const double* coef)
{
    if (!c || !adj || !snap || !coef || (which != 0 && which != 1)) return LBRMT_EINVAL;
    if (!adj_ok(c)) return LBRMT_ESTATE;
    LossCoef lc;
    lc.c[0] = coef[0];
    lc.c[1] = coef[1];
    lc.d[0] = coef[2];
    lc.d[1] = coef[3];
    lc.gc[0] = coef[4];
    lc.gc[1] = coef[5];
    lc.gd[0] = coef[6];
    lc.gd[1] = coef[7];
    HIPCHK(c, launch_adjoint_loss(c->g, c->body, adj_snap(c, snap), adj_bufs(c, adj), which, lc,
                                  c->st));
    return LBRMT_OK;
}

int lbrmt_adjoint_step(lbrmt_ctx* c, void* adj, const void* snap)
{
    if (!c || !adj || !snap) return LBRMT_EINVAL;
    if (!adj_ok(c)) return LBRMT_ESTATE;
    HIPCHK(c, launch_adjoint_step(c->g, c->body, adj_snap(c, snap), adj_bufs(c, adj), c->st));
    // state n becomes the next step's state n + 1; the spent half is cleared
    c->adj_flip = 1 - c->adj_flip;
    const AdjLayout L = adj_layout(c);
    const int h = 1 - c->adj_flip;
    char* b = (char*)adj;
    const size_t rp = c->L.pplane * 8;
    HIPCHK(c, hipMemsetAsync(b + L.x[h], 0, rp, c->st));
    HIPCHK(c, hipMemsetAsync(b + L.y[h], 0, rp, c->st));
    HIPCHK(c, hipMemsetAsync(b + L.p[h], 0, rp, c->st));
    return LBRMT_OK;
}

int lbrmt_adjoint_init(lbrmt_ctx* c, void* adj, const void* snap0, double* u0bar,
                       double* host_GU)
{
    if (!c || !adj || !snap0) return LBRMT_EINVAL;
    if (!adj_ok(c)) return LBRMT_ESTATE;
    const AdjBufs a = adj_bufs(c, adj);
    if (u0bar) HIPCHK(c, launch_adjoint_init(c->g, c->body, adj_snap(c, snap0), a, u0bar, c->st));
    if (host_GU) {
        HIPCHK(c, hipMemcpyAsync(host_GU, a.acc, 2 * sizeof(double), hipMemcpyDeviceToHost,
                                 c->st));
        HIPCHK(c, hipStreamSynchronize(c->st));
    }
    return LBRMT_OK;
}

// ---------------------------------------------------------------- checkpoint

struct StateHeader {
    uint32_t magic, version;
    int64_t step;
    int32_t nx, ny, precision, nsolid;
    uint64_t lat_bytes, plane_bytes, pplane_bytes;
};

// Blob layout.  One solid: header, lattice, F^{n-1}, xi, phi, window ring and
// health.  Several solids (off[4..7] differ): the two force-block stamp
// arrays with the block-list counters and the device step counter, the
// solid table (only its region boxes and window origins are restored: the
// rest is fixed by the context), and every solid's block (its maps of both
// steps, tags, lists and window ring), then the health counters.
static size_t state_layout(const lbrmt_ctx* c, size_t off[8])
{
    size_t o = 0;
    auto take = [&](size_t b) {
        size_t r = o;
        o = round_up(o + b, ALIGN);
        return r;
    };
    off[0] = take(sizeof(StateHeader));
    off[1] = take(c->L.lat_bytes);     // lattice A
    off[2] = take(c->L.plane * 8);     // F^{n-1} x
    off[3] = take(c->L.plane * 8);     // F^{n-1} y
    if (c->multi) {
        const size_t nblk = (size_t)c->L.nbx * c->L.nby;
        off[4] = take(2 * nblk * 4);                        // stamps
        off[5] = take(2 * 4 + 8);                           // list counters, step counter
        off[6] = take((size_t)c->nsolid * sizeof(MbBody));  // solid table
        off[7] = take((size_t)c->nsolid * c->L.body_bytes + LBRMT_H_COUNT * sizeof(unsigned));
        return o;
    }
    off[4] = take(c->L.pplane * c->L.rm_es);    // X
    off[5] = take(c->L.pplane * c->L.rm_es);    // Y
    off[6] = take(c->L.pplane * c->L.rm_es);    // phi
    off[7] = take(3 * sizeof(Win) + LBRMT_H_COUNT * sizeof(unsigned));
    return o;
}

// the several-solid parts of a blob (off from state_layout); load: blob -> ctx
static int state_copy_mb(lbrmt_ctx* c, char* b, const size_t off[8], bool load)
{
    const hipMemcpyKind D2D = hipMemcpyDeviceToDevice;
    const size_t nblk = (size_t)c->L.nbx * c->L.nby;
    const size_t bodies = (size_t)c->nsolid * c->L.body_bytes;
    char* bod = c->ws + c->L.off_bodies;
    auto cp = [&](void* ctxp, size_t boff, size_t n) {
        return load ? hipMemcpyAsync(ctxp, b + boff, n, D2D, c->st)
                    : hipMemcpyAsync(b + boff, ctxp, n, D2D, c->st);
    };
    for (int k = 0; k < 2; k++) HIPCHK(c, cp(c->stamp[k], off[4] + k * nblk * 4, nblk * 4));
    HIPCHK(c, cp(c->mcount, off[5], 2 * 4));
    HIPCHK(c, cp(c->dstep, off[5] + 8, 8));
    if (load) {
        HIPCHK(c, launch_mb_copy_reg((const MbBody*)(b + off[6]), c->mbd, c->nsolid, mb_tabs(c),
                                     c->st));
    } else {
        HIPCHK(c, hipMemcpyAsync(b + off[6], c->mbd, (size_t)c->nsolid * sizeof(MbBody), D2D,
                                 c->st));
    }
    HIPCHK(c, cp(bod, off[7], bodies));
    HIPCHK(c, cp(c->bb.health, off[7] + bodies, LBRMT_H_COUNT * sizeof(unsigned)));
    return LBRMT_OK;
}

int lbrmt_state_bytes(const lbrmt_ctx* c, size_t* bytes)
{
    if (!c || !bytes) return LBRMT_EINVAL;
    size_t off[8];
    *bytes = state_layout(c, off);
    return LBRMT_OK;
}

int lbrmt_save_state(lbrmt_ctx* c, void* buf)
{
    if (!c || !buf) return LBRMT_EINVAL;
    if (!c->inited) return LBRMT_ESTATE;
    size_t off[8];
    state_layout(c, off);
    char* b = (char*)buf;
    const StepSlots s = slots_for(c->step);
    StateHeader h{STATE_MAGIC, STATE_VERSION, c->step, c->d.nx, c->d.ny, c->d.precision,
                  c->nsolid, c->L.lat_bytes, c->L.plane * 8, c->L.pplane * c->L.rm_es};
    const hipMemcpyKind D2D = hipMemcpyDeviceToDevice;
    HIPCHK(c, hipMemcpyAsync(b + off[1], c->lat[s.cur], c->L.lat_bytes, D2D, c->st));
    HIPCHK(c, hipMemcpyAsync(b + off[2], c->Fx[s.nxt], c->L.plane * 8, D2D, c->st));
    HIPCHK(c, hipMemcpyAsync(b + off[3], c->Fy[s.nxt], c->L.plane * 8, D2D, c->st));
    if (c->multi) {
        h.pplane_bytes = c->L.body_bytes;
        int rc = state_copy_mb(c, b, off, false);
        if (rc != LBRMT_OK) return rc;
        HIPCHK(c, hipMemcpyAsync(b + off[0], &h, sizeof h, hipMemcpyHostToDevice, c->st));
        HIPCHK(c, hipStreamSynchronize(c->st));  // h lives on this stack frame
        return LBRMT_OK;
    }
    HIPCHK(c, hipMemcpyAsync(b + off[4], c->bb.X[s.cur], c->L.pplane * c->L.rm_es, D2D, c->st));
    HIPCHK(c, hipMemcpyAsync(b + off[5], c->bb.Y[s.cur], c->L.pplane * c->L.rm_es, D2D, c->st));
    HIPCHK(c, hipMemcpyAsync(b + off[6], c->bb.phi[s.cur], c->L.pplane * c->L.rm_es, D2D, c->st));
    HIPCHK(c, hipMemcpyAsync(b + off[7], c->bb.win, 3 * sizeof(Win), D2D, c->st));
    HIPCHK(c, hipMemcpyAsync(b + off[7] + 3 * sizeof(Win), c->bb.health,
                             LBRMT_H_COUNT * sizeof(unsigned), D2D, c->st));
    HIPCHK(c, hipMemcpyAsync(b + off[0], &h, sizeof h, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));  // h lives on this stack frame
    return LBRMT_OK;
}

int lbrmt_load_state(lbrmt_ctx* c, const void* buf)
{
    if (c && c->member) return LBRMT_ESTATE;
    if (!c || !buf) return LBRMT_EINVAL;
    size_t off[8];
    state_layout(c, off);
    const char* b = (const char*)buf;
    StateHeader h;
    HIPCHK(c, hipMemcpyAsync(&h, b + off[0], sizeof h, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    const uint64_t shape_bytes = c->multi ? c->L.body_bytes : c->L.pplane * c->L.rm_es;
    if (h.magic != STATE_MAGIC || h.version != STATE_VERSION || h.nx != c->d.nx ||
        h.ny != c->d.ny || h.precision != c->d.precision || h.nsolid != c->nsolid ||
        h.lat_bytes != c->L.lat_bytes || h.pplane_bytes != shape_bytes || h.step < 0) {
        c->err = "state blob does not match this context";
        return LBRMT_EINVAL;
    }
    c->step = h.step;
    const StepSlots s = slots_for(c->step);
    const hipMemcpyKind D2D = hipMemcpyDeviceToDevice;
    HIPCHK(c, hipMemcpyAsync(c->lat[s.cur], b + off[1], c->L.lat_bytes, D2D, c->st));
    HIPCHK(c, hipMemcpyAsync(c->Fx[s.nxt], b + off[2], c->L.plane * 8, D2D, c->st));
    HIPCHK(c, hipMemcpyAsync(c->Fy[s.nxt], b + off[3], c->L.plane * 8, D2D, c->st));
    if (c->multi) {
        int rc = state_copy_mb(c, (char*)b, off, true);
        if (rc != LBRMT_OK) return rc;
        c->inited = true;
        return LBRMT_OK;
    }
    HIPCHK(c, hipMemcpyAsync(c->bb.X[s.cur], b + off[4], c->L.pplane * c->L.rm_es, D2D, c->st));
    HIPCHK(c, hipMemcpyAsync(c->bb.Y[s.cur], b + off[5], c->L.pplane * c->L.rm_es, D2D, c->st));
    HIPCHK(c, hipMemcpyAsync(c->bb.phi[s.cur], b + off[6], c->L.pplane * c->L.rm_es, D2D, c->st));
    HIPCHK(c, hipMemcpyAsync(c->bb.win, b + off[7], 3 * sizeof(Win), D2D, c->st));
    HIPCHK(c, hipMemcpyAsync(c->bb.health, b + off[7] + 3 * sizeof(Win),
                             LBRMT_H_COUNT * sizeof(unsigned), D2D, c->st));
    HIPCHK(c, hipMemsetAsync(c->bb.lcount, 0, (size_t)(MAX_LAYERS + 1) * NSUB * LCOUNT_PAD * 4,
                             c->st));
    HIPCHK(c, hipMemsetAsync(c->bb.ticket, 0, 4, c->st));
    HIPCHK(c, clear_cut_tiles(c, c->st));
    c->inited = true;
    return LBRMT_OK;
}

int lbrmt_debug_poke(lbrmt_ctx* c, int32_t field, int64_t index, double value)
{
    if (!c || field != 0 || index < 0 || index >= (int64_t)c->d.nx * c->d.ny) return LBRMT_EINVAL;
    if (!c->inited) return LBRMT_ESTATE;
    const StepSlots s = slots_for(c->step);
    HIPCHK(c, launch_poke(c->g, c->d.precision, c->lat[s.cur], index, value, c->st));
    return LBRMT_OK;
}

int lbrmt_validate(const lbrmt_grid_desc* d, const lbrmt_solid_desc* s, int32_t n,
                   lbrmt_validation_t* out)
{
    if (!d || !out || n < 0 || (n > 0 && !s)) return LBRMT_EINVAL;
    if (!(d->tau > 0.5) || d->nx < 8 || d->ny < 8) return LBRMT_EINVAL;
    memset(out, 0, sizeof *out);
    // App. A: nu = c_s^2 (tau - 1/2), Ma* = U* / c_s*
    out->nu = (d->tau - 0.5) / 3.0;
    const double U = std::fabs(d->periodic_y ? 0.0 : d->lid_ux);
    out->mach_lb = U / std::sqrt(1.0 / 3.0);
    out->reynolds = out->nu > 0 ? U * d->nx / out->nu : 0.0;
    out->tau_ok = d->tau > 0.5 && d->tau <= 1.0;
    out->mach_ok = out->mach_lb <= 0.3;
    out->solids_inside = 1;
    for (int k = 0; k < n; k++) {
        if (!solid_shape_ok(s[k])) return LBRMT_EINVAL;
        const double m = solid_extent(s[k]) + d->layers;
        if (!d->periodic_x && (s[k].cx - m < -2 || s[k].cx + m > d->nx + 2)) out->solids_inside = 0;
        if (!d->periodic_y && (s[k].cy - m < -2 || s[k].cy + m > d->ny + 2)) out->solids_inside = 0;
        if (d->periodic_x && (s[k].cx - m < 0 || s[k].cx + m > d->nx)) out->solids_inside = 0;
        if (d->periodic_y && (s[k].cy - m < 0 || s[k].cy + m > d->ny)) out->solids_inside = 0;
    }
    return LBRMT_OK;
}

int lbrmt_set_timing(lbrmt_ctx* c, int32_t enable)
{
    if (!c) return LBRMT_EINVAL;
    int rc = collect_timing(c);
    if (rc != LBRMT_OK) return rc;
    c->timing = enable != 0;
    for (int k = 0; k < NKERN; k++) {
        c->t_ms[k] = 0.0;
        c->t_n[k] = 0;
    }
    return LBRMT_OK;
}

int lbrmt_kernel_time(lbrmt_ctx* c, const char* name, double* avg_ms, int64_t* launches)
{
    if (!c || !name || !avg_ms || !launches) return LBRMT_EINVAL;
    int rc = collect_timing(c);
    if (rc != LBRMT_OK) return rc;
    for (int k = 0; k < NKERN; k++)
        if (!strcmp(name, kernel_names[k])) {
            *launches = c->t_n[k];
            *avg_ms = c->t_n[k] ? c->t_ms[k] / c->t_n[k] : 0.0;
            return LBRMT_OK;
        }
    return LBRMT_EINVAL;
}

int lbrmt_set_option(lbrmt_ctx* c, int32_t option, int64_t value)
{
    if (!c) return LBRMT_EINVAL;
    if (c->member) return LBRMT_ESTATE;
    int64_t cur = 0;
    if (option != LBRMT_OPT_LB_VARIANT_COUNT && lbrmt_get_option(c, option, &cur) == LBRMT_OK &&
        cur == value)
        return LBRMT_OK;  // unchanged: the captured graphs stay valid
    switch (option) {
    case LBRMT_OPT_OVERLAP:
        if (value != 0 && value != 1) return LBRMT_EINVAL;
        c->overlap = value != 0;
        break;
    case LBRMT_OPT_LB_VARIANT:
        if (value < 0 || value >= lb_variant_count()) return LBRMT_EINVAL;
        c->lb_variant = (int)value;
        break;
    case LBRMT_OPT_GRAPH:
        if (value != 0 && value != 1) return LBRMT_EINVAL;
        c->graph = value != 0;
        break;
    case LBRMT_OPT_BULK_BLOCKS:
        if (value < 0 || value > (1 << 24)) return LBRMT_EINVAL;
        if (value > 0 && c->hold_bulk == 1) {
            c->err = "a capped bulk update cannot be held (LBRMT_OPT_HOLD_BULK is 1)";
            return LBRMT_EINVAL;
        }
        c->bulk_blocks = (int)value;
        break;
    case LBRMT_OPT_FUSED_FIT:
        if (value != -1 && value != 0 && value != 1 && value != 256 && value != 512 &&
            value != 1024)
            return LBRMT_EINVAL;
        c->fused_fit = (int)value;
        break;
    case LBRMT_OPT_HOLD_BULK:
        if (value < -1 || value > 1) return LBRMT_EINVAL;
        if (value == 1 && c->bulk_blocks > 0) {
            // the held and capped combination stalled the stream for about
            // 0.1 s per step once; it is not offered
            c->err = "a capped bulk update cannot be held (LBRMT_OPT_BULK_BLOCKS > 0)";
            return LBRMT_EINVAL;
        }
        c->hold_bulk = (int)value;
        break;
    case LBRMT_OPT_BULK_EARLY:
        if (value < -1 || value > 1000) return LBRMT_EINVAL;
        c->bulk_early = (int)value;
        break;
    default:
        return LBRMT_EINVAL;
    }
    // the captured step graphs bake the launch configuration in
    return drop_graphs(c);
}

int lbrmt_get_option(const lbrmt_ctx* c, int32_t option, int64_t* value)
{
    if (!c || !value) return LBRMT_EINVAL;
    switch (option) {
    case LBRMT_OPT_OVERLAP: *value = c->overlap ? 1 : 0; return LBRMT_OK;
    case LBRMT_OPT_LB_VARIANT: *value = c->lb_variant; return LBRMT_OK;
    case LBRMT_OPT_LB_VARIANT_COUNT: *value = lb_variant_count(); return LBRMT_OK;
    case LBRMT_OPT_GRAPH: *value = c->graph ? 1 : 0; return LBRMT_OK;
    case LBRMT_OPT_BULK_BLOCKS: *value = c->bulk_blocks; return LBRMT_OK;
    case LBRMT_OPT_FUSED_FIT: *value = c->fused_fit; return LBRMT_OK;
    case LBRMT_OPT_HOLD_BULK: *value = c->hold_bulk; return LBRMT_OK;
    case LBRMT_OPT_BULK_EARLY: *value = c->bulk_early; return LBRMT_OK;
    default: return LBRMT_EINVAL;
    }
}

int lbrmt_band_nodes(lbrmt_ctx* c, int64_t* band_nodes, int64_t* window_nodes)
{
    if (!c || !band_nodes || !window_nodes) return LBRMT_EINVAL;
    if (!c->inited || c->multi) return LBRMT_ESTATE;
    Win w[3];
    HIPCHK(c, hipMemcpyAsync(w, c->bb.win, sizeof w, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    const StepSlots s = slots_for(c->step);
    auto dil = [&](const Win& b, int& i0, int& i1, int& j0, int& j1) {
        if (b.i0 > b.i1) return false;
        const int L = c->g.layers;
        i0 = std::max(b.i0 - L, 0);
        i1 = std::min(b.i1 + L, c->g.nx - 1);
        j0 = std::max(b.j0 - L, 0);
        j1 = std::min(b.j1 + L, c->g.ny - 1);
        return i0 <= i1 && j0 <= j1;
    };
    int a0, a1, a2, a3, b0, b1, b2, b3;
    const bool pa = dil(w[s.wprev], a0, a1, a2, a3), pb = dil(w[s.wcur], b0, b1, b2, b3);
    *window_nodes = pb ? (int64_t)(b1 - b0 + 1) * (b3 - b2 + 1) : 0;
    if (c->overlap && c->nsolid > 0) {
        // the force pass updates the window's nodes, the bulk launch the rest
        *band_nodes = *window_nodes;
        return LBRMT_OK;
    }
    if (!pa && !pb) {
        *band_nodes = 0;
        return LBRMT_OK;
    }
    int u0 = pa ? a0 : b0, u1 = pa ? a1 : b1, u2 = pa ? a2 : b2, u3 = pa ? a3 : b3;
    if (pb) {
        u0 = std::min(u0, b0);
        u1 = std::max(u1, b1);
        u2 = std::min(u2, b2);
        u3 = std::max(u3, b3);
    }
    // nodes of the lattice tiles the band update covers (whole tiles, clipped)
    int LB_TX, LB_TY;
    lb_variant_tile(c->lb_variant, &LB_TX, &LB_TY);
    const int x0 = u0 / LB_TX * LB_TX, x1 = std::min((u1 / LB_TX + 1) * LB_TX, c->g.nx) - 1;
    const int y0 = u2 / LB_TY * LB_TY, y1 = std::min((u3 / LB_TY + 1) * LB_TY, c->g.ny) - 1;
    *band_nodes = (int64_t)(x1 - x0 + 1) * (y1 - y0 + 1);
    return LBRMT_OK;
}



// ---------------------------------------------------------------- tile-shape autotuner

// Times every lattice tile variant on the context's current state: the update
// reads lattice A (the state) and writes lattice B, which the next step
// overwrites anyway, so the state is not changed.  Picks the fastest.
int lbrmt_autotune(lbrmt_ctx* c, int32_t reps, int32_t* best_variant, double* best_ms)
{
    if (!c || reps < 1) return LBRMT_EINVAL;
    if (!c->inited || c->member || c->multi) return LBRMT_ESTATE;
    const StepSlots s = slots_for(c->step);
    const double ox = fpo_x(c, c->step), oy = fpo_y(c, c->step);
    hipEvent_t a = nullptr, b = nullptr;
    HIPCHK(c, hipEventCreate(&a));
    HIPCHK(c, hipEventCreate(&b));
    int best = c->lb_variant;
    float best_t = 1e30f;
    for (int v = 0; v < lb_variant_count(); v++) {
        auto launch = [&]() {
            return launch_lb(c->g, c->d.precision, v, c->lat[s.cur], c->lat[s.nxt], c->Fx[s.nxt],
                             c->Fy[s.nxt], c->Fx[s.cur], c->Fy[s.cur], c->drho, c->bb.win,
                             s.wprev, s.wcur, ox, oy, 0, c->bb.health, c->st);
        };
        HIPCHK(c, launch());  // warm-up
        HIPCHK(c, hipEventRecord(a, c->st));
        for (int r = 0; r < reps; r++) HIPCHK(c, launch());
        HIPCHK(c, hipEventRecord(b, c->st));
        HIPCHK(c, hipEventSynchronize(b));
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, a, b));
        if (ms < best_t) {
            best_t = ms;
            best = v;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    int rc = lbrmt_set_option(c, LBRMT_OPT_LB_VARIANT, best);
    if (rc != LBRMT_OK) return rc;
    remember_variant(0, c->d.nx, c->d.ny, c->d.precision, best);
    if (best_variant) *best_variant = best;
    if (best_ms) *best_ms = best_t / reps;
    return LBRMT_OK;
}

int lbrmt_autotune_steps(lbrmt_ctx* c, int32_t steps, int32_t* best_fused, double* best_ms)
{
    if (!c || steps < 1) return LBRMT_EINVAL;
    if (!c->inited || c->member || c->multi) return LBRMT_ESTATE;
    if (c->nsolid == 0 || !fused_fit_ok(c->g)) {
        if (best_fused) *best_fused = c->fused_fit;
        if (best_ms) *best_ms = 0.0;
        return LBRMT_OK;
    }
    hipEvent_t a = nullptr, b = nullptr;
    HIPCHK(c, hipEventCreate(&a));
    HIPCHK(c, hipEventCreate(&b));
    const int modes[2] = {1024, 0};
    const long long timed = ((long long)steps + GRAPH_STEPS - 1) / GRAPH_STEPS * GRAPH_STEPS;
    int best = modes[0];
    float best_t = 1e30f;
    int rc = LBRMT_OK;
    for (int m = 0; m < 2 && rc == LBRMT_OK; m++) {
        rc = lbrmt_set_option(c, LBRMT_OPT_FUSED_FIT, modes[m]);
        // warm-up (and graph capture), ending on a six-step boundary so that
        // the timed steps are whole graph replays
        long long warm = steps / 4 + GRAPH_STEPS;
        warm += (GRAPH_STEPS - (c->step + warm) % GRAPH_STEPS) % GRAPH_STEPS;
        if (rc == LBRMT_OK) rc = lbrmt_step(c, warm);
        if (rc != LBRMT_OK) break;
        HIPCHK(c, hipEventRecord(a, c->st));
        rc = lbrmt_step(c, timed);
        if (rc != LBRMT_OK) break;
        HIPCHK(c, hipEventRecord(b, c->st));
        HIPCHK(c, hipEventSynchronize(b));
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, a, b));
        if (ms < best_t) {
            best_t = ms;
            best = modes[m];
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc != LBRMT_OK) return rc;
    rc = lbrmt_set_option(c, LBRMT_OPT_FUSED_FIT, best);
    if (rc != LBRMT_OK) return rc;
    // capture the chosen mode's six-step graph now, so that the first steps
    // after the choice do not pay for it
    if (c->graph && !c->gexec) {
        rc = build_graph(c);
        if (rc != LBRMT_OK) return rc;
    }
    if (best_fused) *best_fused = best;
    if (best_ms) *best_ms = best_t / (double)timed;
    return LBRMT_OK;
}

// ---------------------------------------------------------------- batches

// Independent members of different sizes stepped together: every kernel of
// the step is one launch over all members (the reference-map kernels take the
// member from blockIdx.y, the lattice update runs over the concatenated tile
// lists), so one step costs 17 launches whatever the member count.  Members
// are ordinary contexts on slices of the batch workspace; their argument
// tables for the six phases n mod 6 (and n = 0) live in the workspace too.
struct lbrmt_batch {
    int n = 0;
    int precision = 0, layers = 0;
    std::vector<lbrmt_ctx*> m;
    hipStream_t st = nullptr, cap = nullptr;
    char* ws = nullptr;
    BatchTables tab[7];
    int* tile_sim = nullptr;
    size_t tile_cap = 0;
    int total_tiles = 0;
    int lb_variant = 3;
    long long nodes = 0;  // interior nodes of all members (the autotune key)
    bool graph = true;
    int fused_fit = 0;  // 1024: one extrapolation launch if every member can; 0 (-1): per layer
    hipGraphExec_t gexec = nullptr;
    hipGraph_t gsrc = nullptr;  // the captured graph of gexec
    long long step = 0;
    bool inited = false;
    std::string err;
};

namespace {

struct BatchLayout {
    size_t tables, tiles, total;
    std::vector<size_t> member_off, member_bytes;
    size_t tile_cap;
};

size_t batch_tile_count(const lbrmt_grid_desc& d, int v)
{
    int tx, ty;
    lb_variant_tile(v, &tx, &ty);
    return (size_t)((d.nx + tx - 1) / tx) * (size_t)((d.ny + ty - 1) / ty);
}

bool batch_layout(const lbrmt_grid_desc* d, int32_t n, BatchLayout& B)
{
    size_t o = 0;
    auto take = [&](size_t b) {
        size_t r = o;
        o = round_up(o + b, ALIGN);
        return r;
    };
    const size_t per = sizeof(AdvectArgs) + sizeof(LayersArgs) + sizeof(FitArgs) +
                       sizeof(EdgesArgs) + sizeof(LbArgs);
    B.tables = take(7 * (size_t)n * per + 6 * 7 * ALIGN);
    B.tile_cap = 0;
    for (int v = 0; v < lb_variant_count(); v++) {
        size_t t = 0;
        for (int k = 0; k < n; k++) t += batch_tile_count(d[k], v);
        B.tile_cap = std::max(B.tile_cap, t);
    }
    if (B.tile_cap > (size_t)0x7fffffff) return false;
    B.tiles = take(B.tile_cap * sizeof(int));
    B.member_off.resize(n);
    B.member_bytes.resize(n);
    for (int k = 0; k < n; k++) {
        const Layout L = make_layout(&d[k]);
        B.member_bytes[k] = L.total;
        B.member_off[k] = take(L.total);
    }
    B.total = o;
    return true;
}

int bfail(lbrmt_batch* b, const char* what, hipError_t e)
{
    char buf[512];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    b->err = buf;
    return LBRMT_EHIP;
}

#define BCHK(b, expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return bfail(b, #expr, e_); \
    } while (0)

// argument tables of phase p (p = n mod 6 for n >= 1; p = 6 for n = 0)
// with LBRMT_OPT_FUSED_FIT = 1024 the batch fits every member's layers in one
// launch when every member can (one solid on walled axes, at most FF_LAYERS
// layers).  Not the default: with many members the one launch holds thousands
// of long 1024-thread blocks for a few hundred slots, where eleven launches
// over all members keep the GPU fuller (96-member ensemble, FP32: 1.077
// against 0.844 ms per step).
bool batch_fused(const lbrmt_batch* b)
{
    if (b->fused_fit != 1024) return false;
    for (const lbrmt_ctx* c : b->m)
        if (c->nsolid == 0 || !fused_fit_ok(c->g)) return false;
    return true;
}

int batch_tables(lbrmt_batch* b)
{
    const int n = b->n;
    std::vector<AdvectArgs> adv(n);
    std::vector<LayersArgs> lay(n);
    std::vector<FitArgs> fit(n);
    std::vector<EdgesArgs> edg(n);
    std::vector<LbArgs> lb(n);
    int base = 0;
    std::vector<int> tile_sim;
    for (int k = 0; k < n; k++) {
        const size_t t = batch_tile_count(b->m[k]->d, b->lb_variant);
        tile_sim.insert(tile_sim.end(), t, k);
    }
    if (tile_sim.size() > b->tile_cap) return LBRMT_EWORKSPACE;
    b->total_tiles = (int)tile_sim.size();
    for (int p = 0; p < 7; p++) {
        const long long nstep = p == 6 ? 0 : (p == 0 ? 6 : p);
        const StepSlots s = slots_for(nstep);
        base = 0;
        for (int k = 0; k < n; k++) {
            lbrmt_ctx* c = b->m[k];
            const GridP& g = c->g;
            const bool ff = batch_fused(b);
            adv[k] = AdvectArgs{g, c->lat[s.cur], c->Fx[s.nxt], c->Fy[s.nxt], c->bb.X[s.cur],
                                c->bb.Y[s.cur], c->bb.phi[s.cur], c->bb.X[s.nxt], c->bb.Y[s.nxt],
                                c->bb.tag, c->bb.win, s.wprev, s.wcur, c->bb.lists,
                                c->bb.lcount, c->bb.health, ff ? c->bb.ff_flag : nullptr,
                                ff ? c->bb.ff_list : nullptr, ff ? c->bb.ff_n : nullptr};
            lay[k] = LayersArgs{g, c->bb.win, s.wcur, c->bb.tag, c->bb.gcol, c->bb.lists,
                                c->bb.lcount, c->bb.health};
            fit[k] = FitArgs{g, c->bb.win, s.wcur, s.wprev, c->bb.tag, c->bb.lists, c->bb.lcount,
                             c->bb.phi[s.cur], c->bb.X[s.nxt], c->bb.Y[s.nxt], c->bb.health,
                             c->bb.cut_layer, c->bb.cut_tiles, c->bb.ncut, c->bb.ff_flag,
                             c->bb.ff_list, c->bb.ff_n};
            edg[k] = EdgesArgs{g, c->body, c->bb.win, s.wcur, c->bb.boxpart, c->bb.X[s.nxt],
                               c->bb.Y[s.nxt], c->bb.tag, c->bb.phi[s.nxt], c->Fx[s.cur],
                               c->Fy[s.cur], c->drho, c->bb.lcount, c->bb.health};
            lb[k] = LbArgs{g, c->lat[s.cur], c->lat[s.nxt], c->Fx[s.nxt], c->Fy[s.nxt],
                           c->Fx[s.cur], c->Fy[s.cur], c->drho, c->bb.win, s.wprev, s.wcur,
                           fpo_x(c, nstep), fpo_y(c, nstep), c->bb.health, base, c->bb.win,
                           c->bb.boxpart, c->nsolid > 0 ? BATCH_BAND_BLOCKS : 0, s.wnext};
            base += (int)batch_tile_count(c->d, b->lb_variant);
        }
        const BatchTables& T = b->tab[p];
        BCHK(b, hipMemcpyAsync(T.adv, adv.data(), n * sizeof(AdvectArgs), hipMemcpyHostToDevice, b->st));
        BCHK(b, hipMemcpyAsync(T.lay, lay.data(), n * sizeof(LayersArgs), hipMemcpyHostToDevice, b->st));
        BCHK(b, hipMemcpyAsync(T.fit, fit.data(), n * sizeof(FitArgs), hipMemcpyHostToDevice, b->st));
        BCHK(b, hipMemcpyAsync(T.edg, edg.data(), n * sizeof(EdgesArgs), hipMemcpyHostToDevice, b->st));
        BCHK(b, hipMemcpyAsync(T.lb, lb.data(), n * sizeof(LbArgs), hipMemcpyHostToDevice, b->st));
        // the host vectors are reused for the next phase: wait for the copies
        BCHK(b, hipStreamSynchronize(b->st));
    }
    if (!tile_sim.empty()) {
        BCHK(b, hipMemcpyAsync(b->tile_sim, tile_sim.data(), tile_sim.size() * sizeof(int),
                               hipMemcpyHostToDevice, b->st));
        BCHK(b, hipStreamSynchronize(b->st));
    }
    return LBRMT_OK;
}

int batch_enqueue(lbrmt_batch* b, long long n, hipStream_t st)
{
    const int p = n == 0 ? 6 : (int)(n % 6);
    const BatchTables& T = b->tab[p];
    BCHK(b, launch_batch_band(b->precision, T, b->n, b->layers, st, false, BATCH_DT_BLOCKS,
                              BATCH_FIT_BLOCKS, BATCH_BAND_BLOCKS, batch_fused(b)));
    BCHK(b, launch_lb_batch(b->precision, b->lb_variant, T.lb, b->tile_sim, b->total_tiles, st));
    return LBRMT_OK;
}

int batch_graph(lbrmt_batch* b)
{
    hipGraph_t graph = nullptr;
    BCHK(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    int rc = LBRMT_OK;
    for (int k = 0; k < GRAPH_STEPS && rc == LBRMT_OK; k++) rc = batch_enqueue(b, 6 + k, b->cap);
    hipError_t e = hipStreamEndCapture(b->cap, &graph);
    if (rc != LBRMT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return bfail(b, "hipStreamEndCapture", e);
    e = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        b->gexec = nullptr;
        return bfail(b, "hipGraphInstantiate", e);
    }
    b->gsrc = graph;  // kept until the executable graph is destroyed
    return LBRMT_OK;
}

void batch_drop_graph(lbrmt_batch* b)
{
    if (b->gexec) {
        (void)hipStreamSynchronize(b->st);
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    if (b->gsrc) (void)hipGraphDestroy(b->gsrc);
    b->gsrc = nullptr;
}

}  // namespace

int lbrmt_batch_workspace_bytes(const lbrmt_grid_desc* descs, int32_t n, size_t* bytes)
{
    if (!descs || n < 1 || !bytes) return LBRMT_EINVAL;
    for (int k = 0; k < n; k++)
        if (!desc_ok(&descs[k]) || descs[k].precision != descs[0].precision ||
            descs[k].layers != descs[0].layers)
            return LBRMT_EINVAL;
    BatchLayout B;
    if (!batch_layout(descs, n, B)) return LBRMT_EINVAL;
    *bytes = B.total;
    return LBRMT_OK;
}

int lbrmt_batch_create(const lbrmt_grid_desc* descs, const lbrmt_solid_desc* solids,
                       const int32_t* has_solid, int32_t n, void* ws, size_t bytes, void* stream,
                       lbrmt_batch** out)
{
    if (!descs || n < 1 || !ws || !out) return LBRMT_EINVAL;
    size_t need = 0;
    int rc = lbrmt_batch_workspace_bytes(descs, n, &need);
    if (rc != LBRMT_OK) return rc;
    if ((uintptr_t)ws % ALIGN || bytes < need) return LBRMT_EWORKSPACE;
    BatchLayout B;
    batch_layout(descs, n, B);
    lbrmt_batch* b = new lbrmt_batch();
    b->n = n;
    b->precision = descs[0].precision;
    b->layers = descs[0].layers;
    b->lb_variant = b->precision == LBRMT_FP64 ? 3 : 5;
    for (int k = 0; k < n; k++) b->nodes += (long long)descs[k].nx * descs[k].ny;
    b->lb_variant = tuned_variant(1, n, b->nodes, b->precision, b->lb_variant);
    b->st = (hipStream_t)stream;
    b->ws = (char*)ws;
    size_t o = B.tables;
    auto carve = [&](size_t bytes_) {
        char* p_ = b->ws + o;
        o = round_up(o + bytes_, ALIGN);
        return p_;
    };
    for (int p = 0; p < 7; p++) {
        b->tab[p].adv = (AdvectArgs*)carve(n * sizeof(AdvectArgs));
        b->tab[p].lay = (LayersArgs*)carve(n * sizeof(LayersArgs));
        b->tab[p].fit = (FitArgs*)carve(n * sizeof(FitArgs));
        b->tab[p].edg = (EdgesArgs*)carve(n * sizeof(EdgesArgs));
        b->tab[p].lb = (LbArgs*)carve(n * sizeof(LbArgs));
    }
    b->tile_sim = (int*)(b->ws + B.tiles);
    b->tile_cap = B.tile_cap;
    b->m.assign(n, nullptr);
    for (int k = 0; k < n && rc == LBRMT_OK; k++) {
        rc = create_impl(&descs[k], 1, b->ws + B.member_off[k], B.member_bytes[k], stream,
                         &b->m[k], true);
        if (rc == LBRMT_OK && solids && (!has_solid || has_solid[k]))
            rc = lbrmt_add_solids(b->m[k], &solids[k], 1);
    }
    if (rc == LBRMT_OK) {
        hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
        if (e != hipSuccess) rc = bfail(b, "stream creation", e);
    }
    if (rc != LBRMT_OK) {
        lbrmt_batch_destroy(b);
        return rc;
    }
    *out = b;
    return LBRMT_OK;
}

void lbrmt_batch_destroy(lbrmt_batch* b)
{
    if (!b) return;
    // (st may be the null stream: it is synchronised too)
    (void)hipStreamSynchronize(b->st);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->gsrc) (void)hipGraphDestroy(b->gsrc);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (auto c : b->m) lbrmt_destroy(c);
    delete b;
}

int lbrmt_batch_init(lbrmt_batch* b)
{
    if (!b) return LBRMT_EINVAL;
    for (auto c : b->m) {
        int rc = lbrmt_init(c, nullptr);
        if (rc != LBRMT_OK) {
            b->err = c->err;
            return rc;
        }
    }
    batch_drop_graph(b);
    int rc = batch_tables(b);
    if (rc != LBRMT_OK) return rc;
    b->step = 0;
    b->inited = true;
    return LBRMT_OK;
}

int lbrmt_batch_step(lbrmt_batch* b, int64_t nsteps)
{
    if (!b || nsteps < 0) return LBRMT_EINVAL;
    if (!b->inited) return LBRMT_ESTATE;
    int64_t left = nsteps;
    while (left > 0) {
        const bool use_graph = b->graph && b->step >= GRAPH_STEPS &&
                               b->step % GRAPH_STEPS == 0 && left >= GRAPH_STEPS;
        int adv = 1;
        if (use_graph) {
            if (!b->gexec) {
                int rc = batch_graph(b);
                if (rc != LBRMT_OK) return rc;
            }
            BCHK(b, hipGraphLaunch(b->gexec, b->st));
            adv = GRAPH_STEPS;
        } else {
            int rc = batch_enqueue(b, b->step, b->st);
            if (rc != LBRMT_OK) return rc;
        }
        b->step += adv;
        left -= adv;
        for (auto c : b->m) c->step += adv;
    }
    return LBRMT_OK;
}

int32_t lbrmt_batch_size(const lbrmt_batch* b) { return b ? b->n : -1; }

lbrmt_ctx* lbrmt_batch_member(lbrmt_batch* b, int32_t k)
{
    if (!b || k < 0 || k >= b->n) return nullptr;
    return b->m[k];
}

int lbrmt_batch_set_option(lbrmt_batch* b, int32_t option, int64_t value)
{
    if (!b) return LBRMT_EINVAL;
    switch (option) {
    case LBRMT_OPT_LB_VARIANT:
        if (value < 0 || value >= lb_variant_count()) return LBRMT_EINVAL;
        b->lb_variant = (int)value;
        break;
    case LBRMT_OPT_GRAPH:
        if (value != 0 && value != 1) return LBRMT_EINVAL;
        b->graph = value != 0;
        break;
    case LBRMT_OPT_FUSED_FIT:
        if (value != -1 && value != 0 && value != 1024) return LBRMT_EINVAL;
        b->fused_fit = (int)value;
        break;
    default:
        return LBRMT_EINVAL;
    }
    batch_drop_graph(b);
    if (b->inited) return batch_tables(b);
    return LBRMT_OK;
}

int lbrmt_batch_get_option(const lbrmt_batch* b, int32_t option, int64_t* value)
{
    if (!b || !value) return LBRMT_EINVAL;
    switch (option) {
    case LBRMT_OPT_LB_VARIANT: *value = b->lb_variant; return LBRMT_OK;
    case LBRMT_OPT_LB_VARIANT_COUNT: *value = lb_variant_count(); return LBRMT_OK;
    case LBRMT_OPT_GRAPH: *value = b->graph ? 1 : 0; return LBRMT_OK;
    case LBRMT_OPT_FUSED_FIT: *value = b->fused_fit; return LBRMT_OK;
    default: return LBRMT_EINVAL;
    }
}

int lbrmt_batch_autotune(lbrmt_batch* b, int32_t reps, int32_t* best_variant, double* best_ms)
{
    if (!b || reps < 1) return LBRMT_EINVAL;
    if (!b->inited) return LBRMT_ESTATE;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BCHK(b, hipEventCreate(&e0));
    BCHK(b, hipEventCreate(&e1));
    const int keep = b->lb_variant;
    int best = keep;
    float best_t = 1e30f;
    const int p = b->step == 0 ? 6 : (int)(b->step % 6);
    for (int v = 0; v < lb_variant_count(); v++) {
        b->lb_variant = v;
        int rc = batch_tables(b);  // tile list of this shape
        if (rc != LBRMT_OK) return rc;
        BCHK(b, launch_lb_batch(b->precision, v, b->tab[p].lb, b->tile_sim, b->total_tiles, b->st));
        BCHK(b, hipEventRecord(e0, b->st));
        for (int r = 0; r < reps; r++)
            BCHK(b, launch_lb_batch(b->precision, v, b->tab[p].lb, b->tile_sim, b->total_tiles,
                                    b->st));
        BCHK(b, hipEventRecord(e1, b->st));
        BCHK(b, hipEventSynchronize(e1));
        float ms = 0.f;
        BCHK(b, hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_t) {
            best_t = ms;
            best = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)keep;
    int rc = lbrmt_batch_set_option(b, LBRMT_OPT_LB_VARIANT, best);
    if (rc != LBRMT_OK) return rc;
    remember_variant(1, b->n, b->nodes, b->precision, best);
    if (best_variant) *best_variant = best;
    if (best_ms) *best_ms = best_t / reps;
    return LBRMT_OK;
}

const char* lbrmt_batch_last_error(const lbrmt_batch* b) { return b ? b->err.c_str() : ""; }

}  // extern "C"
