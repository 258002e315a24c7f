// Host runtime of libtete: descriptor validation (stability bound (25)),
// workspace layout, grid state and the C-ABI entry points of include/tete.h.
// All device work is enqueued on the grid's stream; the library never
// allocates device memory.

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "tete_impl.h"

using namespace tete;

namespace {

constexpr double kEps0 = 8.8541878128e-12;   // vacuum permittivity [F/m] (CODATA 2018)
constexpr size_t kAlign = 256;

size_t up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t lam, wacc, wit, wmid, partial, epart, scal, pidx, eser, pser, code, field[12], mat[6], imp[4], imp_le, imp_lh,
        imp_cnt, skip[2], skip_act[2], cls, ctab, craw, total;
};

int64_t series_cap(const tete_grid_desc* d) { return d->max_series > 0 ? d->max_series : 4096; }

// Workgroups whose energy partial sums a two-step launch can keep (energy
// samples taken inside two-step launches; larger launches sample apart).
enum { EN_PARTS = 65536 };

// Tiles of the finest tiling of the two-step kernel and of the materials step.
int64_t skip_cap(Geo g) { return std::max(fused2_tile_cap(g), fused_tile_cap(g)); }

bool make_layout(const tete_grid_desc* d, Layout* L)
{
    const int64_t np = (int64_t)(d->nx + 1) * (d->ny + 1) * (d->nz + 1);
    const size_t rb = d->precision == TETE_FP32 ? 4 : 8;
    size_t o = 0;
    L->lam = o;     o = up(o + sizeof(double) * TETE_MAX_BUNCH_CELLS);
    L->wacc = o;    o = up(o + sizeof(double) * TETE_MAX_WAKE);
    L->wit = o;     o = up(o + sizeof(double) * TETE_WITNESS_LINES * TETE_MAX_WAKE);
    L->wmid = o;    o = up(o + rb * TETE_WITNESS_LINES * (size_t)d->nz);
    L->partial = o; o = up(o + sizeof(double) * 2 * RED_BLOCKS);
    L->epart = o;   o = up(o + sizeof(double) * 2 * EN_PARTS);
    L->scal = o;    o = up(o + sizeof(double) * 64);
    L->pidx = o;    o = up(o + sizeof(int64_t) * TETE_MAX_PROBES);
    L->eser = o;    o = up(o + sizeof(double) * (size_t)series_cap(d));
    L->pser = o;    o = up(o + sizeof(double) * (size_t)series_cap(d) * TETE_MAX_PROBES);
    L->code = o;    o = up(o + (size_t)np);
    for (int c = 0; c < 12; ++c) { L->field[c] = o; o = up(o + rb * (size_t)np); }
    for (int c = 0; c < 6; ++c) {
        if (d->flags & TETE_F_MATERIALS) { L->mat[c] = o; o = up(o + rb * (size_t)np); }
        else L->mat[c] = 0;
    }
    L->cls = L->ctab = L->craw = 0;
    if (d->flags & TETE_F_MATERIALS) {     // materials by class: class bytes, step table, table as given
        L->cls = o;  o = up(o + (size_t)np);
        L->ctab = o; o = up(o + rb * TETE_MAX_CLASSES * CLS_STRIDE);
        L->craw = o; o = up(o + sizeof(double) * TETE_MAX_CLASSES * 6);
    }
    for (int c = 0; c < 4; ++c) {          // plane-solve work arrays of the implicit scheme
        if (d->flags & TETE_F_IMPLICIT) { L->imp[c] = o; o = up(o + rb * (size_t)np); }
        else L->imp[c] = 0;
    }
    L->imp_le = L->imp_lh = L->imp_cnt = 0;
    if (d->flags & TETE_F_IMPLICIT) {      // row lists of the plane systems and their chunk counts
        L->imp_le = o;  o = up(o + sizeof(int) * (size_t)np);
        L->imp_lh = o;  o = up(o + sizeof(int) * (size_t)np);
        L->imp_cnt = o; o = up(o + sizeof(int) * 2 * (size_t)implicit_list_chunks(np));
    }
    L->skip[0] = L->skip[1] = L->skip_act[0] = L->skip_act[1] = 0;
    if (d->flags & TETE_F_SKIP_STATIC) {   // static-tile table and active-tile list of each tiling kind
        Geo g = {d->nx, d->ny, d->nz, d->nz + 1, (d->ny + 1) * (d->nz + 1), (int)np};
        const int64_t cap = skip_cap(g);
        for (int kind = 0; kind < 2; ++kind) {
            L->skip[kind] = o;     o = up(o + (size_t)cap);
            L->skip_act[kind] = o; o = up(o + sizeof(int) * (size_t)cap);
        }
    }
    L->total = o;
    return true;
}

// Runs f() with dev current, restoring the previous device afterwards.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard()
    {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

struct tete_grid {
    tete_grid_desc d;
    hipStream_t stream;
    int device;
    char* ws;
    Layout L;
    Geo geo;
    int fp32;
    int yee;           // Yee's scheme (7) instead of (23)
    int implicit;      // the implicit scheme (16) instead of (23)
    int imp_lists;     // row lists built for the current geometry
    int imp_ne, imp_nh;
    void* f[2][6];
    int cur;           // f[cur] holds y^n
    uint8_t* code;
    void* mat[6];
    int mat_set;
    // materials by class (tete_set_material_classes): the class bytes, the
    // step kernels' table and the table as given; mat_cls is set while the
    // material arrays hold the classes' expansion
    int mat_cls;
    uint8_t* cls;
    void* ctab;
    double* craw;
    // static-tile skip (TETE_F_SKIP_STATIC): per tiling kind (0: two-step
    // kernel, 1: fused single step) the table and the list of the
    // skip_nact[kind] active tiles for the tiling (skip_rows, skip_xc,
    // skip_order)[kind], skip_rows[kind] = -1 while none is built for the
    // current codes or materials; skip_live is set once a launch has written
    // the other field set since the fields or codes were last set, so that
    // both sets agree on every static tile
    int skip;
    uint8_t* skip_tab[2];
    int* skip_act[2];
    int skip_rows[2], skip_xc[2], skip_order[2], skip_nact[2];
    int64_t skip_nt[2];
    int skip_live;
    // sticky error state: TETE_ERR_NONFINITE once a read-out found NaN or
    // Inf, until tete_set_fields; tete_step refuses to run meanwhile
    tete_status err;
    double *lam, *wacc, *partial, *epart, *scal, *eser, *pser;
    double* wit;       // witness accumulators, TETE_WITNESS_LINES x TETE_MAX_WAKE
    void* wmid;        // e_z^{n+1/2} of the witness lines in a two-step launch (TETE_WITNESS_LINES x nz)
    int witness;       // witness lines armed (tete_set_witness)
    int32_t iw, jw;
    int64_t* pidx;
    int64_t n;         // step index of y^n: 0 after create / set_fields, the start step of an open-pipe run
    int has_bunch;
    tete_bunch b;
    int32_t kend;      // open-pipe run: the wake quadrature ends before edge kend (0: all nz edges)
    int diag_every;
    int64_t ecount, pcount, cap;
    int nprobe;
    double kv[3], mv[3], alpha;
    tete_tuning tune;
    // live kernel timing (tete_set_timing): 3 events per timed launch and the
    // steps each launch took (1, or 2 for the two-step kernel)
    int timing;
    hipEvent_t* ev;
    unsigned char* ev_nst;
    int64_t ev_cap, ev_steps;
};

#define HIPCHK(x)                                      \
    do {                                               \
        if ((x) != hipSuccess) return TETE_ERR_DEVICE; \
    } while (0)

namespace {

template <typename R>
Fields<R> fields(tete_grid* g, int set)
{
    Fields<R> F;
    for (int c = 0; c < 6; ++c) F.c[c] = (R*)g->f[set][c];
    return F;
}

template <typename R>
Mat<R> mats(tete_grid* g)
{
    Mat<R> M;
    M.code = g->code;
    for (int c = 0; c < 6; ++c) M.arr[c] = g->mat_set ? (const R*)g->mat[c] : nullptr;
    for (int c = 0; c < 3; ++c) { M.k[c] = (R)g->kv[c]; M.m[c] = (R)g->mv[c]; }
    M.cls = g->mat_cls ? g->cls : nullptr;
    M.ctab = g->mat_cls ? (const R*)g->ctab : nullptr;
    return M;
}

// Edges k < wake_end(g) enter the wake quadrature: all nz, or those before
// the end that an open-pipe run set.
int wake_end(const tete_grid* g) { return g->kend > 0 ? g->kend : g->d.nz; }

Src source(tete_grid* g, int64_t n)
{
    Src s;
    s.on = g->has_bunch;
    s.i0 = g->b.i0;
    s.j0 = g->b.j0;
    s.M = g->b.half_cells;
    s.n = n;
    s.lam = g->lam;
    s.wacc = g->wacc;
    s.jmin = g->b.jmin;
    s.nw = g->b.nw;
    s.kend = wake_end(g);
    return s;
}

// Witness node and its neighbours -x, +x, -y, +y (the order of tete_witness_wake)
constexpr int kWdi[TETE_WITNESS_LINES] = {0, -1, 1, 0, 0};
constexpr int kWdj[TETE_WITNESS_LINES] = {0, 0, 0, -1, 1};

// Array offsets of (i, j, 0) of the witness node line and its four neighbours,
// in the order of tete_witness_wake
Witness witness_lines(const tete_grid* g)
{
    Witness w;
    for (int l = 0; l < TETE_WITNESS_LINES; ++l)
        w.base[l] = ((int64_t)(g->iw + kWdi[l]) * g->geo.sp + (int64_t)(g->jw + kWdj[l]) * g->geo.sz);
    return w;
}

template <typename R>
WitMid<R> witness_mid(const tete_grid* g)
{
    WitMid<R> w;
    w.mid = (R*)g->wmid;
    w.iw = g->iw;
    w.jw = g->jw;
    return w;
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

// Read-out values of a grid: a NaN or Inf puts the grid into the sticky
// TETE_ERR_NONFINITE state (cleared by tete_set_fields).
tete_status check_finite(tete_grid* g, const double* v, int64_t n)
{
    for (int64_t e = 0; e < n; ++e)
        if (!isfinite(v[e])) {
            g->err = TETE_ERR_NONFINITE;
            break;
        }
    return g->err;
}

// weight of the alpha^2 terms in the energy and the charges: none for the
// implicit scheme (16), whose transverse operators are time-centred
double rweight(const tete_grid* g) { return g->implicit ? 0.0 : 1.0; }

template <typename R>
ImpWork<R> imp_work(tete_grid* g)
{
    ImpWork<R> w;
    w.b = (R*)(g->ws + g->L.imp[0]);
    w.r = (R*)(g->ws + g->L.imp[1]);
    w.d[0] = (R*)(g->ws + g->L.imp[2]);
    w.d[1] = (R*)(g->ws + g->L.imp[3]);
    w.le = (const int*)(g->ws + g->L.imp_le);
    w.lh = (const int*)(g->ws + g->L.imp_lh);
    w.ne = g->imp_ne;
    w.nh = g->imp_nh;
    return w;
}

// The fused kernel covers vacuum cells with staircase PEC codes and, in its
// materials instance, per-entry materials.
bool use_fused(const tete_grid* g)
{
    if (g->yee || g->implicit || !fused_fits(g->geo, g->fp32 ? 4 : 8)) return false;
    return g->tune.kernel != TETE_KERNEL_SPLIT;
}

// The two-step kernel (automatic choice, or asked for) when the grid
// qualifies; do_steps still takes single steps where a diagnostic needs the
// state in between.
// Rows of the two-step kernel: the class instance's for materials by class
// (FP32 24, FP64 the default), else the tuning's rows when it asks for 16, 24
// or 32 (24, 32: FP32 only), else the default.
int fused2_rows(const tete_grid* g)
{
    if (g->mat_cls) return g->fp32 ? 24 : 0;
    const int r = g->tune.rows;
    return r == 16 || ((r == 24 || r == 32) && g->fp32) ? r : 0;
}

// X-chunk of the two-step kernel: the tuning's, else for grids that skip
// static tiles chunks of 32 planes (short chunks find more tiles wholly in
// the metal, at seven halo planes per chunk), else the library's choice (0).
int fused2_xchunk(const tete_grid* g)
{
    return g->tune.xchunk != 0 ? g->tune.xchunk : g->skip ? 32 : 0;
}

// FP32 per-entry arrays: the two-step kernel's arrays instance, without
// witness lines or a static-tile list.
bool arrays_fused2(const tete_grid* g) { return g->fp32 && !g->skip; }

// Per-entry materials step as single steps, except materials by class, which
// the two-step kernel's class instance takes, and FP32 arrays, which its
// arrays instance takes (both without witness lines).
bool use_fused2(const tete_grid* g)
{
    const bool want = g->tune.kernel == TETE_KERNEL_FUSED2 || g->tune.kernel == TETE_KERNEL_AUTO;
    const bool wit = g->witness && g->has_bunch;
    const bool mat_ok = !g->mat_set || (g->mat_cls && !wit) || (!g->mat_cls && arrays_fused2(g) && !wit);
    return want && mat_ok && use_fused(g) && fused2_fits(g->geo, g->fp32 ? 4 : 8);
}

// Builds the static-tile table for the current tiling of the two-step
// kernel unless it is already there.
// Builds the static-tile table and active list of one tiling kind (0: the
// two-step kernel, 1: the fused single step) for the current tiling unless it
// is already there.  Each kind keeps its own, so alternating two-step and
// single launches do not rebuild them.
template <typename R>
tete_status static_table(tete_grid* g, bool wit, bool single)
{
    const int kind = single ? 1 : 0;
    int rows, xc, order = g->tune.order;
    if (single) {   // the fused single step's tiling; kappa marks the PEC edges of materials
        rows = g->mat_set || g->tune.rows == 24 || g->tune.rows == 32 ? 0 : g->tune.rows;
        xc = g->tune.xchunk;
    } else {        // the instance that keeps witness lines has the default rows only
        rows = wit ? 0 : fused2_rows(g);
        xc = fused2_xchunk(g);
    }
    if (g->skip_rows[kind] == rows && g->skip_xc[kind] == xc && g->skip_order[kind] == order) return TETE_OK;
    if (single) {
        const R* kap[3] = {(const R*)g->mat[0], (const R*)g->mat[1], (const R*)g->mat[2]};
        HIPCHK(fused_static_tiles<R>(g->mat_set ? kap : nullptr, g->code, g->geo, rows, xc, order, g->skip_tab[1],
                                     g->skip_act[1], skip_cap(g->geo), &g->skip_nt[1], &g->skip_nact[1], g->stream));
    } else {
        HIPCHK(fused2_static_tiles<R>(g->code, g->geo, rows, xc, order, g->skip_tab[0], g->skip_act[0],
                                      skip_cap(g->geo), &g->skip_nt[0], &g->skip_nact[0], g->stream));
    }
    g->skip_rows[kind] = rows;
    g->skip_xc[kind] = xc;
    g->skip_order[kind] = order;
    return TETE_OK;
}

// The static-tile tables no longer match the codes or materials.
void skip_invalidate(tete_grid* g)
{
    g->skip_rows[0] = g->skip_rows[1] = -1;
    g->skip_live = 0;
}

template <typename R>
tete_status do_steps(tete_grid* g, int64_t nsteps)
{
    Mat<R> M = mats<R>(g);
    const bool two = use_fused2(g);
    // Yee grids: two steps per launch unless the tuning asks for single steps
    const bool two_yee = g->yee && g->tune.kernel != TETE_KERNEL_FUSED && yee2_fits(g->geo, g->fp32 ? 4 : 8);
    // energy samples inside two-step launches: vacuum grids (with or without
    // witness lines) and materials by class, without static-tile lists,
    // launches of at most EN_PARTS workgroups
    int64_t en_blocks = 0;
    const bool en_fuse = two && g->diag_every > 0 && (!g->mat_set || g->mat_cls) && !g->skip &&
                         (en_blocks = fused2_blocks<R>(g->geo, fused2_xchunk(g), g->tune.order)) > 0 &&
                         en_blocks <= EN_PARTS;
    for (int64_t s = 0; s < nsteps; ++s) {
        const bool at_n = g->diag_every > 0 && g->n % g->diag_every == 0;
        const bool at_n1 = g->diag_every > 0 && (g->n + 1) % g->diag_every == 0;
        // two steps at once unless the state after the first is observed
        // (an energy sample of it is taken inside the launch where it can be;
        // the probes' values of it are recomputed from the launch's input)
        const bool wit = g->witness && g->has_bunch;
        const bool pair = (two || two_yee) && s + 1 < nsteps && (g->nprobe == 0 || two) && (!at_n1 || en_fuse);
        const bool en_pair = pair && en_fuse && (at_n || at_n1);
        if (at_n && !en_pair) {
            HIPCHK(launch_energy<R>(fields<R>(g, g->cur), M, g->geo, g->alpha, rweight(g), g->partial, g->eser + g->ecount,
                                    g->stream));
            g->ecount++;
        }
        hipEvent_t* ev = nullptr;
        if (g->timing) {
            if (g->ev_steps >= g->ev_cap) return TETE_ERR_STATE;
            ev = g->ev + 3 * g->ev_steps;
            g->ev_nst[g->ev_steps] = pair ? 2 : 1;
            g->ev_steps++;
        }
        if (pair && g->yee) {
            HIPCHK(launch_step_yee2<R>(fields<R>(g, g->cur), fields<R>(g, 1 - g->cur), M, g->geo, (R)g->alpha,
                                       g->tune.xchunk, g->tune.order, g->stream, ev));
            g->cur = 1 - g->cur;
            g->n += 2;
            ++s;
            continue;
        }
        if (pair) {
            WitMid<R> wm;
            if (wit) wm = witness_mid<R>(g);
            const int* act = nullptr;
            if (g->skip && g->skip_live) {
                if (static_table<R>(g, wit, false) != TETE_OK) return TETE_ERR_DEVICE;
                act = g->skip_act[0];
                // static tiles store no witness values: their e_z is zero
                if (wit) HIPCHK(launch_zero_bytes(g->wmid, (g->fp32 ? 4 : 8) * (size_t)TETE_WITNESS_LINES * g->d.nz,
                                                  g->stream));
            }
            if (g->nprobe > 0)   // the probes after step n+1, from y^n before the launch replaces it
                HIPCHK(launch_probes_next<R>(fields<R>(g, g->cur), M, g->geo, (R)g->alpha, source(g, g->n), g->pidx,
                                             g->nprobe, g->pser + g->pcount * g->nprobe, g->stream));
            EnergyPair en = {(at_n ? 1 : 0) | (at_n1 ? 2 : 0), g->alpha, g->epart, EN_PARTS, g->eser + g->ecount,
                             g->mat_cls ? g->craw : nullptr};
            HIPCHK(launch_step_fused2<R>(fields<R>(g, g->cur), fields<R>(g, 1 - g->cur), M, g->geo, (R)g->alpha,
                                         source(g, g->n), wit ? &wm : nullptr, fused2_rows(g), g->tune.depth,
                                         fused2_xchunk(g), g->tune.order, g->stream, ev, act, g->skip_nact[0],
                                         en_pair ? &en : nullptr));
            if (en_pair) g->ecount += (at_n ? 1 : 0) + (at_n1 ? 1 : 0);
            g->skip_live = 1;
            if (wit)   // e_z^{n-1/2} in the old set, e_z^{n+1/2} in wm.mid, e_z^{n+3/2} in the new set
                HIPCHK(launch_witness2<R>((const R*)g->f[g->cur][2], wm.mid, (const R*)g->f[1 - g->cur][2],
                                          witness_lines(g), g->geo, g->n, g->b.half_cells, g->b.jmin, g->b.nw,
                                          wake_end(g), g->wit, g->stream));
            g->cur = 1 - g->cur;
            g->n += 2;
            ++s;
            if (g->nprobe > 0) {   // the probes after step n+2
                HIPCHK(launch_probes<R>((const R*)g->f[g->cur][2], g->pidx, g->nprobe,
                                        g->pser + (g->pcount + 1) * g->nprobe, g->stream));
                g->pcount += 2;
            }
            continue;
        }
        if (g->implicit && !g->imp_lists) {   // once per geometry
            HIPCHK(implicit_build_lists<R>(M, g->geo, (int*)(g->ws + g->L.imp_cnt), (int*)(g->ws + g->L.imp_le),
                                           (int*)(g->ws + g->L.imp_lh), &g->imp_ne, &g->imp_nh, g->stream));
            g->imp_lists = 1;
        }
        if (g->implicit)
            HIPCHK(launch_step_implicit<R>(fields<R>(g, g->cur), fields<R>(g, 1 - g->cur), M, g->geo, g->d.dx,
                                           g->d.dy, (R)g->alpha, source(g, g->n), imp_work<R>(g), g->stream, ev));
        else if (g->yee)
            HIPCHK(launch_step_yee<R>(fields<R>(g, g->cur), fields<R>(g, 1 - g->cur), M, g->geo, (R)g->alpha,
                                      g->tune.xchunk, g->tune.order, g->stream, ev));
        else if (use_fused(g)) {
            const int* act = nullptr;
            if (g->skip && g->skip_live) {
                if (static_table<R>(g, false, true) != TETE_OK) return TETE_ERR_DEVICE;
                act = g->skip_act[1];
            }
            HIPCHK(launch_step_fused<R>(fields<R>(g, g->cur), fields<R>(g, 1 - g->cur), M, g->geo, (R)g->alpha,
                                        source(g, g->n), g->tune.rows == 24 || g->tune.rows == 32 ? 0 : g->tune.rows,
                                        g->tune.xchunk,
                                        g->tune.depth, g->tune.order, g->stream, ev, act, g->skip_nact[1]));
        }
        else
            HIPCHK(launch_step<R>(fields<R>(g, g->cur), fields<R>(g, 1 - g->cur), M, g->geo, (R)g->alpha,
                                  source(g, g->n), g->stream, ev));
        if (wit)   // the step leaves e_z^{n-1/2} in the old set and e_z^{n+1/2} in the new one
            HIPCHK(launch_witness<R>((const R*)g->f[g->cur][2], (const R*)g->f[1 - g->cur][2], witness_lines(g),
                                     g->geo, g->n, g->b.half_cells, g->b.jmin, g->b.nw, wake_end(g), g->wit,
                                     g->stream));
        g->cur = 1 - g->cur;
        g->n++;
        g->skip_live = 1;
        if (g->nprobe > 0) {
            HIPCHK(launch_probes<R>((const R*)g->f[g->cur][2], g->pidx, g->nprobe, g->pser + g->pcount * g->nprobe,
                                    g->stream));
            g->pcount++;
        }
    }
    return TETE_OK;
}

tete_status reset_series(tete_grid* g)
{
    g->n = 0;
    g->ecount = 0;
    g->pcount = 0;
    HIPCHK(launch_fill_f64(g->wacc, TETE_MAX_WAKE, 0.0, g->stream));
    HIPCHK(launch_fill_f64(g->wit, (int64_t)TETE_WITNESS_LINES * TETE_MAX_WAKE, 0.0, g->stream));
    return TETE_OK;
}

}  // namespace

// Reduction scratch of tete_energy_noalloc: the partial sums of the energy
// reduction and its result, in a file-scope device array (each GPU holds its
// own copy until the process ends).  In host code the name stands for a
// host-side shadow, never a device address: kernels get the address that
// hipGetSymbolAddress returns for the current device.
constexpr int kScratchDoubles = RED_BLOCKS + 8;
static_assert(RED_BLOCKS + 1 <= kScratchDoubles, "the energy reduction's partials and result fit the scratch");
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices];   // device address of scratch, per device

// Device address of the scratch array on device dev (which must be current),
// looked up once per device.
tete_status scratch_on(int dev, double** out)
{
    if (dev < 0 || dev >= kMaxDevices) return TETE_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TETE_ERR_DEVICE;
        g_scratch_dev[dev] = (double*)p;
    }
    *out = g_scratch_dev[dev];
    return TETE_OK;
}

}  // namespace

extern "C" {

const char* tete_status_str(tete_status s)
{
    switch (s) {
    case TETE_OK: return "TETE_OK";
    case TETE_ERR_ARG: return "TETE_ERR_ARG";
    case TETE_ERR_UNSTABLE: return "TETE_ERR_UNSTABLE";
    case TETE_ERR_NOMEM: return "TETE_ERR_NOMEM";
    case TETE_ERR_DEVICE: return "TETE_ERR_DEVICE";
    case TETE_ERR_STATE: return "TETE_ERR_STATE";
    case TETE_ERR_NONFINITE: return "TETE_ERR_NONFINITE";
    }
    return "TETE_ERR_UNKNOWN";
}

tete_status tete_check_desc(const tete_grid_desc* d)
{
    if (!d) return TETE_ERR_ARG;
    if (d->nx < 2 || d->ny < 2 || d->nz < 2) return TETE_ERR_ARG;
    const int64_t np = (int64_t)(d->nx + 1) * (d->ny + 1) * (d->nz + 1);
    // entries fit int indices with room for the grid-stride loops' last step
    if (np > ((int64_t)1 << 31) - ((int64_t)1 << 24)) return TETE_ERR_ARG;
    if (!finite_pos(d->dx) || !finite_pos(d->dy) || !finite_pos(d->dz) || !finite_pos(d->cdt)) return TETE_ERR_ARG;
    if (d->precision != TETE_FP64 && d->precision != TETE_FP32) return TETE_ERR_ARG;
    if (d->flags & ~(uint32_t)(TETE_F_MATERIALS | TETE_F_YEE | TETE_F_IMPLICIT | TETE_F_SKIP_STATIC))
        return TETE_ERR_ARG;
    if ((d->flags & TETE_F_SKIP_STATIC) && (d->flags & (TETE_F_YEE | TETE_F_IMPLICIT))) return TETE_ERR_ARG;
    if ((d->flags & TETE_F_YEE) && (d->flags & TETE_F_MATERIALS)) return TETE_ERR_ARG;
    if ((d->flags & TETE_F_IMPLICIT) && (d->flags & (TETE_F_MATERIALS | TETE_F_YEE))) return TETE_ERR_ARG;
    if (d->max_series < 0 || d->max_series > (1 << 24)) return TETE_ERR_ARG;
    const double tol = 1.0 + 1e-12;
    if (d->flags & TETE_F_YEE) {
        // (8): dtau <= (dx^-2 + dy^-2 + dz^-2)^(-1/2)
        const double b8 = 1.0 / sqrt(1.0 / (d->dx * d->dx) + 1.0 / (d->dy * d->dy) + 1.0 / (d->dz * d->dz));
        if (d->cdt > b8 * tol) return TETE_ERR_UNSTABLE;
        return TETE_OK;
    }
    if (d->flags & TETE_F_IMPLICIT) {
        // (22): dtau <= dz; the transverse operators are implicit (no transverse bound)
        if (d->cdt > d->dz * tol) return TETE_ERR_UNSTABLE;
        return TETE_OK;
    }
    // (25): dtau <= dz and dtau <= (dx^-2 + dy^-2)^(-1/2), equality allowed
    const double bt = 1.0 / sqrt(1.0 / (d->dx * d->dx) + 1.0 / (d->dy * d->dy));
    if (d->cdt > d->dz * tol || d->cdt > bt * tol) return TETE_ERR_UNSTABLE;
    return TETE_OK;
}

size_t tete_workspace_bytes(const tete_grid_desc* d)
{
    if (tete_check_desc(d) == TETE_ERR_ARG) return 0;
    Layout L;
    make_layout(d, &L);
    return L.total;
}

tete_status tete_grid_create(const tete_grid_desc* d, void* dev_ws, size_t ws_bytes, void* hip_stream,
                             tete_grid** out)
{
    if (!out) return TETE_ERR_ARG;
    *out = nullptr;
    tete_status st = tete_check_desc(d);
    if (st != TETE_OK) return st;
    if (!dev_ws || ((uintptr_t)dev_ws % kAlign) != 0) return TETE_ERR_ARG;
    Layout L;
    make_layout(d, &L);
    if (ws_bytes < L.total) return TETE_ERR_NOMEM;

    tete_grid* g = (tete_grid*)calloc(1, sizeof(tete_grid));
    if (!g) return TETE_ERR_NOMEM;
    g->d = *d;
    g->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&g->device) != hipSuccess) { free(g); return TETE_ERR_DEVICE; }
    g->ws = (char*)dev_ws;
    g->L = L;
    g->geo.nx = d->nx;
    g->geo.ny = d->ny;
    g->geo.nz = d->nz;
    g->geo.sz = d->nz + 1;
    g->geo.sp = (d->ny + 1) * (d->nz + 1);
    g->geo.np = (d->nx + 1) * g->geo.sp;
    g->fp32 = d->precision == TETE_FP32;
    g->yee = (d->flags & TETE_F_YEE) != 0;
    g->implicit = (d->flags & TETE_F_IMPLICIT) != 0;
    if (g->yee && !yee_fits(g->geo, g->fp32 ? 4 : 8)) {   // planes too large for the Yee kernel's buffers
        free(g);
        return TETE_ERR_ARG;
    }
    for (int s = 0; s < 2; ++s)
        for (int c = 0; c < 6; ++c) g->f[s][c] = g->ws + L.field[6 * s + c];
    g->cur = 0;
    g->code = (uint8_t*)(g->ws + L.code);
    g->skip = (d->flags & TETE_F_SKIP_STATIC) != 0;
    for (int kind = 0; kind < 2; ++kind) {
        g->skip_tab[kind] = g->skip ? (uint8_t*)(g->ws + L.skip[kind]) : nullptr;
        g->skip_act[kind] = g->skip ? (int*)(g->ws + L.skip_act[kind]) : nullptr;
        g->skip_xc[kind] = g->skip_order[kind] = g->skip_nact[kind] = 0;
        g->skip_nt[kind] = 0;
    }
    skip_invalidate(g);
    g->err = TETE_OK;
    for (int c = 0; c < 6; ++c) g->mat[c] = (d->flags & TETE_F_MATERIALS) ? g->ws + L.mat[c] : nullptr;
    g->mat_cls = 0;
    g->cls = (d->flags & TETE_F_MATERIALS) ? (uint8_t*)(g->ws + L.cls) : nullptr;
    g->ctab = (d->flags & TETE_F_MATERIALS) ? (void*)(g->ws + L.ctab) : nullptr;
    g->craw = (d->flags & TETE_F_MATERIALS) ? (double*)(g->ws + L.craw) : nullptr;
    g->lam = (double*)(g->ws + L.lam);
    g->wacc = (double*)(g->ws + L.wacc);
    g->wit = (double*)(g->ws + L.wit);
    g->wmid = g->ws + L.wmid;
    g->partial = (double*)(g->ws + L.partial);
    g->epart = (double*)(g->ws + L.epart);
    g->scal = (double*)(g->ws + L.scal);
    g->pidx = (int64_t*)(g->ws + L.pidx);
    g->eser = (double*)(g->ws + L.eser);
    g->pser = (double*)(g->ws + L.pser);
    g->cap = series_cap(d);
    // vacuum M_eps^-1 and M_mu^-1 (c = eps0 = mu0 = 1): edge length / dual facet area
    g->kv[0] = g->mv[0] = d->dx / (d->dy * d->dz);
    g->kv[1] = g->mv[1] = d->dy / (d->dz * d->dx);
    g->kv[2] = g->mv[2] = d->dz / (d->dx * d->dy);
    g->alpha = 0.5 * d->cdt;   // alpha = dtau / 2, eq. (17)
    g->tune.kernel = TETE_KERNEL_AUTO;
    g->tune.rows = 0;
    g->tune.xchunk = 0;
    g->tune.depth = 0;
    g->tune.order = 0;

    // zero the whole workspace, then mark the box walls
    if (launch_zero_bytes(g->ws, L.total, g->stream) != hipSuccess ||
        launch_build_codes(g->code, nullptr, g->geo, g->stream) != hipSuccess) {
        free(g);
        return TETE_ERR_DEVICE;
    }
    *out = g;
    return TETE_OK;
}

tete_status tete_grid_destroy(tete_grid* g)
{
    if (!g) return TETE_ERR_ARG;
    for (int64_t e = 0; e < 3 * g->ev_cap; ++e) (void)hipEventDestroy(g->ev[e]);
    free(g->ev);
    free(g->ev_nst);
    free(g);
    return TETE_OK;
}

tete_status tete_set_tuning(tete_grid* g, const tete_tuning* t)
{
    if (!g || !t) return TETE_ERR_ARG;
    if (t->kernel < TETE_KERNEL_AUTO || t->kernel > TETE_KERNEL_FUSED2) return TETE_ERR_ARG;
    if (t->rows != 0 && t->rows != 12 && t->rows != 16 && t->rows != 24 && t->rows != 32) return TETE_ERR_ARG;
    if (t->xchunk < 0) return TETE_ERR_ARG;
    if (t->depth < 0 || t->depth > 3) return TETE_ERR_ARG;
    if (t->order < 0 || t->order > 6) return TETE_ERR_ARG;
    if (t->kernel == TETE_KERNEL_FUSED2 && g->mat_set && !g->mat_cls && !arrays_fused2(g)) return TETE_ERR_STATE;
    g->tune = *t;
    return TETE_OK;
}

tete_status tete_get_tuning(tete_grid* g, tete_tuning* t)
{
    if (!g || !t) return TETE_ERR_ARG;
    *t = g->tune;
    t->kernel = g->implicit ? TETE_KERNEL_IMPLICIT : g->yee ? TETE_KERNEL_YEE
              : use_fused2(g) ? TETE_KERNEL_FUSED2 : use_fused(g) ? TETE_KERNEL_FUSED : TETE_KERNEL_SPLIT;
    return TETE_OK;
}

tete_status tete_set_timing(tete_grid* g, int64_t max_steps)
{
    if (!g || max_steps < 0 || max_steps > (1 << 20)) return TETE_ERR_ARG;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    HIPCHK(hipStreamSynchronize(g->stream));
    if (max_steps > g->ev_cap) {
        hipEvent_t* ev = (hipEvent_t*)realloc(g->ev, sizeof(hipEvent_t) * 3 * max_steps);
        if (!ev) return TETE_ERR_NOMEM;
        g->ev = ev;
        unsigned char* nst = (unsigned char*)realloc(g->ev_nst, (size_t)max_steps);
        if (!nst) return TETE_ERR_NOMEM;
        g->ev_nst = nst;
        for (int64_t e = 3 * g->ev_cap; e < 3 * max_steps; ++e) {
            if (hipEventCreate(&g->ev[e]) != hipSuccess) {
                g->ev_cap = e / 3;
                return TETE_ERR_DEVICE;
            }
        }
        g->ev_cap = max_steps;
    }
    g->timing = max_steps > 0;
    g->ev_steps = 0;
    return TETE_OK;
}

tete_status tete_timing(tete_grid* g, double* ms, int32_t nphase, int64_t* steps)
{
    if (!g || !ms || !steps || nphase < 1) return TETE_ERR_ARG;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    HIPCHK(hipStreamSynchronize(g->stream));
    for (int p = 0; p < nphase; ++p) ms[p] = 0.0;
    int64_t nst = 0;
    for (int64_t s = 0; s < g->ev_steps; ++s) {
        float t0 = 0.f, t1 = 0.f;
        HIPCHK(hipEventElapsedTime(&t0, g->ev[3 * s], g->ev[3 * s + 1]));
        HIPCHK(hipEventElapsedTime(&t1, g->ev[3 * s + 1], g->ev[3 * s + 2]));
        ms[0] += t0;
        if (nphase > 1) ms[1] += t1;
        nst += g->ev_nst[s];
    }
    *steps = nst;
    g->ev_steps = 0;
    return TETE_OK;
}

tete_status tete_set_pec_cells(tete_grid* g, const uint8_t* cells)
{
    if (!g) return TETE_ERR_ARG;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    HIPCHK(launch_build_codes(g->code, cells, g->geo, g->stream));
    g->mat_set = 0;
    g->mat_cls = 0;
    g->imp_lists = 0;
    g->kend = 0;
    skip_invalidate(g);
    if (g->fp32) HIPCHK(launch_zero_pec<float>(fields<float>(g, g->cur), mats<float>(g), g->geo, g->stream));
    else HIPCHK(launch_zero_pec<double>(fields<double>(g, g->cur), mats<double>(g), g->geo, g->stream));
    return TETE_OK;
}

extern "C++" {
namespace {

// Materials by class recognised in imported per-entry arrays: if the arrays
// hold at most TETE_MAX_CLASSES distinct coefficient tuples and kappa is 0 on
// every edge the PEC codes mark, the grid gets their class bytes and table,
// so that paired steps run the two-step kernel's class instance; the arrays
// stay as they are (the class expansion would give them bitwise).  Otherwise
// nothing changes.  Work space: the reduction partials (hash keys, tuples,
// slot classes) and scalars (flags).
template <typename R>
tete_status find_classes(tete_grid* g)
{
    unsigned long long* keys = (unsigned long long*)g->partial;
    double* vals = g->partial + CLS_SLOTS;
    int* slot_class = (int*)(g->partial + 7 * CLS_SLOTS);
    static_assert(7 * CLS_SLOTS + CLS_SLOTS / 2 <= 2 * RED_BLOCKS, "the class search fits the partials");
    int* flags = (int*)(g->scal + 16);
    R* arr[6];
    for (int c = 0; c < 6; ++c) arr[c] = (R*)g->mat[c];
    HIPCHK(launch_zero_bytes(keys, sizeof(unsigned long long) * CLS_SLOTS, g->stream));
    HIPCHK(launch_zero_bytes(flags, 4 * sizeof(int), g->stream));
    HIPCHK(launch_classify<R>(arr, g->code, g->geo, keys, vals, nullptr, nullptr, flags, 0, g->stream));
    std::vector<unsigned long long> hk(CLS_SLOTS);
    int hf[4];
    HIPCHK(hipMemcpyAsync(hk.data(), keys, sizeof(unsigned long long) * CLS_SLOTS, hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    if (hf[0] || hf[1]) return TETE_OK;
    // classes numbered in the order of their keys (the same numbering every run)
    std::vector<std::pair<unsigned long long, int>> used;
    for (int t = 0; t < CLS_SLOTS; ++t)
        if (hk[t]) used.emplace_back(hk[t], t);
    if (used.empty() || used.size() > (size_t)TETE_MAX_CLASSES) return TETE_OK;
    std::sort(used.begin(), used.end());
    std::vector<int> sc(CLS_SLOTS, -1);
    for (size_t c = 0; c < used.size(); ++c) sc[used[c].second] = (int)c;
    HIPCHK(hipMemcpyAsync(slot_class, sc.data(), sizeof(int) * CLS_SLOTS, hipMemcpyHostToDevice, g->stream));
    HIPCHK(launch_classify<R>(arr, g->code, g->geo, keys, vals, slot_class, g->cls, flags, 1, g->stream));
    std::vector<double> hv((size_t)6 * CLS_SLOTS);
    HIPCHK(hipMemcpyAsync(hv.data(), vals, sizeof(double) * hv.size(), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));   // sc and hv are host temporaries
    if (hf[2]) return TETE_OK;                 // two tuples shared a key: keep the arrays alone
    std::vector<double> t((size_t)6 * TETE_MAX_CLASSES, 0.0);
    for (size_t c = 0; c < used.size(); ++c)
        for (int e = 0; e < 6; ++e) t[6 * c + e] = hv[(size_t)6 * used[c].second + e];
    HIPCHK(hipMemcpyAsync(g->craw, t.data(), sizeof(double) * t.size(), hipMemcpyHostToDevice, g->stream));
    HIPCHK(launch_class_table<R>((R*)g->ctab, g->craw, (R)g->alpha, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));   // t is a host temporary
    g->mat_cls = 1;
    return TETE_OK;
}

}  // namespace
}  // extern "C++"

tete_status tete_set_materials(tete_grid* g, const void* const inv_eps[3], const void* const inv_mu[3], int32_t dtype)
{
    if (!g || !inv_eps || !inv_mu) return TETE_ERR_ARG;
    if (dtype != TETE_FP64 && dtype != TETE_FP32) return TETE_ERR_ARG;
    for (int c = 0; c < 3; ++c)
        if (!inv_eps[c] || !inv_mu[c]) return TETE_ERR_ARG;
    if (!(g->d.flags & TETE_F_MATERIALS)) return TETE_ERR_STATE;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    const void* src[6] = {inv_eps[0], inv_eps[1], inv_eps[2], inv_mu[0], inv_mu[1], inv_mu[2]};
    {
        // Q^e >= 0 (Sec. 4.4) by the Gershgorin row sums of its three blocks,
        // before anything is imported: an unstable set leaves the grid as it was
        double bound;
        HIPCHK(launch_mat_bound(src, dtype == TETE_FP32, g->geo, g->alpha, g->partial, g->scal + 4, g->stream));
        HIPCHK(hipMemcpyAsync(&bound, g->scal + 4, sizeof(double), hipMemcpyDeviceToHost, g->stream));
        HIPCHK(hipStreamSynchronize(g->stream));
        if (!(bound == bound)) return TETE_ERR_ARG;           // a negative or non-finite value
        if (bound > 1.0 + 1e-12) return TETE_ERR_UNSTABLE;
    }
    if (g->tune.kernel == TETE_KERNEL_FUSED || g->tune.kernel == TETE_KERNEL_FUSED2) g->tune.kernel = TETE_KERNEL_AUTO;
    if (g->fp32) {
        float* dst[6];
        for (int c = 0; c < 6; ++c) dst[c] = (float*)g->mat[c];
        HIPCHK(launch_import_materials<float>(dst, src, dtype == TETE_FP32, g->geo, g->stream));
        g->mat_set = 1;
        g->mat_cls = 0;
        skip_invalidate(g);
        HIPCHK(launch_zero_pec<float>(fields<float>(g, g->cur), mats<float>(g), g->geo, g->stream));
    } else {
        double* dst[6];
        for (int c = 0; c < 6; ++c) dst[c] = (double*)g->mat[c];
        HIPCHK(launch_import_materials<double>(dst, src, dtype == TETE_FP32, g->geo, g->stream));
        g->mat_set = 1;
        g->mat_cls = 0;
        skip_invalidate(g);
        HIPCHK(launch_zero_pec<double>(fields<double>(g, g->cur), mats<double>(g), g->geo, g->stream));
    }
    return g->fp32 ? find_classes<float>(g) : find_classes<double>(g);
}

tete_status tete_set_material_classes(tete_grid* g, const uint8_t* cls, const double* table, int32_t ncls)
{
    if (!g || !cls || !table || ncls < 1 || ncls > TETE_MAX_CLASSES) return TETE_ERR_ARG;
    for (int64_t e = 0; e < 6 * (int64_t)ncls; ++e)
        if (!(table[e] >= 0.0) || !isfinite(table[e])) return TETE_ERR_ARG;
    if (!(g->d.flags & TETE_F_MATERIALS)) return TETE_ERR_STATE;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    // the table as given, padded with zero classes, into the staging area
    // (used only here and by the expansion below)
    std::vector<double> t((size_t)6 * TETE_MAX_CLASSES, 0.0);
    std::copy(table, table + 6 * (int64_t)ncls, t.begin());
    HIPCHK(hipMemcpyAsync(g->craw, t.data(), sizeof(double) * t.size(), hipMemcpyHostToDevice, g->stream));
    {
        // Q^e >= 0 (Sec. 4.4) for the per-entry values the classes give, and
        // every class byte below ncls, before anything changes
        double bound;
        HIPCHK(launch_mat_bound_cls(g->code, cls, g->craw, ncls, g->geo, g->alpha, g->partial, g->scal + 4,
                                    g->stream));
        HIPCHK(hipMemcpyAsync(&bound, g->scal + 4, sizeof(double), hipMemcpyDeviceToHost, g->stream));
        HIPCHK(hipStreamSynchronize(g->stream));
        if (!(bound == bound)) return TETE_ERR_ARG;
        if (bound > 1.0 + 1e-12) return TETE_ERR_UNSTABLE;
    }
    HIPCHK(hipMemcpyAsync(g->cls, cls, (size_t)g->geo.np, hipMemcpyDeviceToDevice, g->stream));
    if (g->tune.kernel == TETE_KERNEL_FUSED) g->tune.kernel = TETE_KERNEL_AUTO;
    if (g->fp32) {
        float* dst[6];
        for (int c = 0; c < 6; ++c) dst[c] = (float*)g->mat[c];
        HIPCHK(launch_expand_classes<float>(dst, (float*)g->ctab, g->code, g->cls, g->craw, (float)g->alpha, g->geo,
                                            g->stream));
    } else {
        double* dst[6];
        for (int c = 0; c < 6; ++c) dst[c] = (double*)g->mat[c];
        HIPCHK(launch_expand_classes<double>(dst, (double*)g->ctab, g->code, g->cls, g->craw, g->alpha, g->geo,
                                             g->stream));
    }
    g->mat_set = 1;
    g->mat_cls = 1;
    skip_invalidate(g);
    if (g->fp32) HIPCHK(launch_zero_pec<float>(fields<float>(g, g->cur), mats<float>(g), g->geo, g->stream));
    else HIPCHK(launch_zero_pec<double>(fields<double>(g, g->cur), mats<double>(g), g->geo, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));   // the staging vector is a host temporary
    return TETE_OK;
}

tete_status tete_set_fields(tete_grid* g, const void* const f[6], int32_t dtype)
{
    if (!g || !f) return TETE_ERR_ARG;
    if (dtype != TETE_FP64 && dtype != TETE_FP32) return TETE_ERR_ARG;
    for (int c = 0; c < 6; ++c)
        if (!f[c]) return TETE_ERR_ARG;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    if (g->fp32) HIPCHK(launch_import<float>(fields<float>(g, g->cur), f, dtype == TETE_FP32, mats<float>(g), g->geo, g->stream));
    else HIPCHK(launch_import<double>(fields<double>(g, g->cur), f, dtype == TETE_FP32, mats<double>(g), g->geo, g->stream));
    g->skip_live = 0;
    g->err = TETE_OK;
    g->kend = 0;
    return reset_series(g);
}

tete_status tete_static_tiles(tete_grid* g, int64_t* skipped, int64_t* total)
{
    if (!g || !skipped || !total) return TETE_ERR_ARG;
    if (!g->skip) return TETE_ERR_STATE;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    const bool wit = g->witness && g->has_bunch;
    // the tiling of paired steps (the two-step kernel), or of the single step
    // where tete_step pairs no steps: no two-step kernel, or an energy sample
    // before every step (skip grids take samples apart from the launches)
    const bool single = !use_fused2(g) || g->diag_every == 1;
    tete_status st = g->fp32 ? static_table<float>(g, wit, single) : static_table<double>(g, wit, single);
    if (st != TETE_OK) return st;
    const int kind = single ? 1 : 0;
    *skipped = g->skip_nt[kind] - g->skip_nact[kind];
    *total = g->skip_nt[kind];
    return TETE_OK;
}

tete_status tete_get_fields(tete_grid* g, void* const f[6], int32_t dtype)
{
    if (!g || !f) return TETE_ERR_ARG;
    if (dtype != TETE_FP64 && dtype != TETE_FP32) return TETE_ERR_ARG;
    for (int c = 0; c < 6; ++c)
        if (!f[c]) return TETE_ERR_ARG;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    if (g->fp32) HIPCHK(launch_export<float>(f, dtype == TETE_FP32, fields<float>(g, g->cur), g->geo, g->stream));
    else HIPCHK(launch_export<double>(f, dtype == TETE_FP32, fields<double>(g, g->cur), g->geo, g->stream));
    return TETE_OK;
}

tete_status tete_set_bunch(tete_grid* g, const tete_bunch* b)
{
    if (!g || !b) return TETE_ERR_ARG;
    if (!isfinite(b->charge_C) || b->charge_C == 0.0 || !finite_pos(b->sigma_z)) return TETE_ERR_ARG;
    if (b->i0 <= 0 || b->i0 >= g->d.nx || b->j0 <= 0 || b->j0 >= g->d.ny) return TETE_ERR_ARG;
    if (b->half_cells < 0 || 2 * (int64_t)b->half_cells + 1 > TETE_MAX_BUNCH_CELLS) return TETE_ERR_ARG;
    if (b->nw < 1 || b->nw > TETE_MAX_WAKE) return TETE_ERR_ARG;
    if (g->d.cdt != g->d.dz) return TETE_ERR_STATE;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    HIPCHK(launch_lambda(g->lam, b->charge_C, b->sigma_z, g->d.dz, b->half_cells, g->stream));
    HIPCHK(launch_fill_f64(g->wacc, TETE_MAX_WAKE, 0.0, g->stream));
    HIPCHK(launch_fill_f64(g->wit, (int64_t)TETE_WITNESS_LINES * TETE_MAX_WAKE, 0.0, g->stream));
    g->b = *b;
    g->has_bunch = 1;
    g->kend = 0;
    return TETE_OK;
}

namespace {

// Zero the six arrays of field set o (after their use as scratch they must
// hold zeros again: entries outside a component's range are read as 0).
tete_status zero_set(tete_grid* g, int o)
{
    const size_t bytes = (size_t)(g->fp32 ? 4 : 8) * (size_t)g->geo.np;
    for (int c = 0; c < 6; ++c) HIPCHK(launch_zero_bytes(g->f[o][c], bytes, g->stream));
    return TETE_OK;
}

}  // namespace

tete_status tete_set_open_pipes(tete_grid* g, int64_t start_step, int32_t kend, int32_t* iterations)
{
    if (!g) return TETE_ERR_ARG;
    if (!g->has_bunch || g->yee || g->implicit || (g->d.flags & TETE_F_MATERIALS)) return TETE_ERR_STATE;
    const int nz = g->d.nz;
    if (start_step < 0 || start_step >= nz || kend < 0 || kend > nz) return TETE_ERR_ARG;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    const int64_t n2 = (int64_t)(g->d.nx + 1) * (g->d.ny + 1);
    // scratch: the other field set, whose arrays (np entries, np >= 2 n2) each
    // hold n2 doubles; the next step rewrites it, and it is zeroed below
    if ((size_t)(g->fp32 ? 4 : 8) * (size_t)g->geo.np < sizeof(double) * (size_t)n2 + 256) return TETE_ERR_ARG;
    const int o = 1 - g->cur;
    double* a[6];
    for (int c = 0; c < 6; ++c) a[c] = (double*)g->f[o][c];
    const CgPlane P = {g->d.nx, g->d.ny, n2, g->d.dy / g->d.dx, g->d.dx / g->d.dy};
    const CgWork W = {a[0], a[1], a[2], a[3], a[4], g->partial, g->scal + 8};
    int* bad = (int*)a[5];
    const int64_t src = (int64_t)g->b.i0 * (g->d.ny + 1) + g->b.j0;
    HIPCHK(launch_zero_bytes(bad, 256, g->stream));
    HIPCHK(launch_pipe_check(W.w, g->code, g->geo, P, (int)start_step + 1, bad, g->stream));
    int hbad = 0;
    double wsrc = 0.0;
    HIPCHK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipMemcpyAsync(&wsrc, W.w + src, sizeof(double), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    if (hbad || wsrc == 0.0) {
        // a non-uniform entrance pipe, or the bunch line on PEC
        tete_status st = zero_set(g, o);
        HIPCHK(hipStreamSynchronize(g->stream));
        return st == TETE_OK ? TETE_ERR_ARG : st;
    }
    // |r|^2 <= 1e-32 |b|^2 (b = delta): the residual at the rounding level
    HIPCHK(launch_cg_init(W, P, src, 1e-32, g->stream));
    const int cap = 20 * (g->d.nx + g->d.ny) + 1000, chunk = 32;
    double hs[8] = {0};
    int done = 0;
    for (int it = 0; it < cap && !done; it += chunk) {
        HIPCHK(launch_cg_iterations(W, P, chunk, g->stream));
        HIPCHK(hipMemcpyAsync(hs, W.sc, sizeof(hs), hipMemcpyDeviceToHost, g->stream));
        HIPCHK(hipStreamSynchronize(g->stream));
        done = hs[3] != 0.0;
        if (!(hs[0] == hs[0])) break;                // NaN: cannot converge
    }
    if (!done) {
        tete_status st = zero_set(g, o);
        HIPCHK(hipStreamSynchronize(g->stream));
        return st == TETE_OK ? TETE_ERR_STATE : st;
    }
    // the profile table in the witness accumulators (reset below)
    HIPCHK(launch_pipe_profile(g->wit, g->lam, g->b.half_cells, g->d.cdt, g->stream));
    if (g->fp32)
        HIPCHK(launch_pipe_field<float>(fields<float>(g, g->cur), g->code, W.x, g->wit, g->b.half_cells, start_step,
                                        g->d.dx / g->d.dy, g->d.dy / g->d.dx, g->geo, g->stream));
    else
        HIPCHK(launch_pipe_field<double>(fields<double>(g, g->cur), g->code, W.x, g->wit, g->b.half_cells, start_step,
                                         g->d.dx / g->d.dy, g->d.dy / g->d.dx, g->geo, g->stream));
    tete_status st = zero_set(g, o);
    if (st != TETE_OK) return st;
    g->skip_live = 0;
    g->err = TETE_OK;
    st = reset_series(g);
    if (st != TETE_OK) return st;
    g->n = start_step;
    g->kend = kend;
    HIPCHK(hipStreamSynchronize(g->stream));
    if (iterations) *iterations = (int32_t)hs[5];
    return TETE_OK;
}

tete_status tete_clear_bunch(tete_grid* g)
{
    if (!g) return TETE_ERR_ARG;
    g->has_bunch = 0;
    g->kend = 0;
    return TETE_OK;
}

tete_status tete_set_diagnostics(tete_grid* g, int32_t every)
{
    if (!g || every < 0) return TETE_ERR_ARG;
    if (g->yee && every > 0) return TETE_ERR_STATE;
    g->diag_every = every;
    return TETE_OK;
}

tete_status tete_set_probes(tete_grid* g, const int64_t* idx, int32_t np_)
{
    if (!g || np_ < 0 || np_ > TETE_MAX_PROBES || (np_ > 0 && !idx)) return TETE_ERR_ARG;
    for (int p = 0; p < np_; ++p)
        if (idx[p] < 0 || idx[p] >= g->geo.np) return TETE_ERR_ARG;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    if (np_ > 0) {
        HIPCHK(hipMemcpyAsync(g->pidx, idx, sizeof(int64_t) * np_, hipMemcpyHostToDevice, g->stream));
        HIPCHK(hipStreamSynchronize(g->stream));
    }
    g->nprobe = np_;
    g->pcount = 0;
    return TETE_OK;
}

tete_status tete_step(tete_grid* g, int64_t nsteps)
{
    if (!g || nsteps < 0) return TETE_ERR_ARG;
    if (g->err != TETE_OK) return g->err;
    if (nsteps == 0) return TETE_OK;
    // capacity of the series for the steps requested
    int64_t need_e = 0;
    if (g->diag_every > 0) {
        int64_t e = g->diag_every;
        int64_t first = (g->n + e - 1) / e * e;
        need_e = first < g->n + nsteps ? (g->n + nsteps - 1 - first) / e + 1 : 0;
    }
    if (g->ecount + need_e > g->cap) return TETE_ERR_STATE;
    if (g->nprobe > 0 && g->pcount + nsteps > g->cap) return TETE_ERR_STATE;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    return g->fp32 ? do_steps<float>(g, nsteps) : do_steps<double>(g, nsteps);
}

tete_status tete_grid_status(tete_grid* g)
{
    if (!g) return TETE_ERR_ARG;
    return g->err;
}

tete_status tete_stream_probe(void* const in[6], void* const out[6], const uint8_t* code, int64_t n, int32_t dtype,
                              void* hip_stream)
{
    if (!in || !out || !code || n < 0) return TETE_ERR_ARG;
    if (dtype != TETE_FP64 && dtype != TETE_FP32) return TETE_ERR_ARG;
    for (int c = 0; c < 6; ++c) {
        if (!in[c] || !out[c] || ((uintptr_t)in[c] % 16) != 0 || ((uintptr_t)out[c] % 16) != 0) return TETE_ERR_ARG;
    }
    if (((uintptr_t)code % 4) != 0) return TETE_ERR_ARG;
    HIPCHK(launch_stream(in, out, code, n, dtype == TETE_FP32, (hipStream_t)hip_stream));
    return TETE_OK;
}

tete_status tete_steps_done(tete_grid* g, int64_t* n)
{
    if (!g || !n) return TETE_ERR_ARG;
    *n = g->n;
    return TETE_OK;
}

tete_status tete_wake(tete_grid* g, double* W, int32_t nw)
{
    if (!g || !W) return TETE_ERR_ARG;
    if (!g->has_bunch) return TETE_ERR_STATE;
    if (nw < 1 || nw > g->b.nw) return TETE_ERR_ARG;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    HIPCHK(hipMemcpyAsync(W, g->wacc, sizeof(double) * nw, hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    const double s = 1.0 / (g->b.charge_C * kEps0);
    for (int j = 0; j < nw; ++j) W[j] *= s;
    return check_finite(g, W, nw);
}

tete_status tete_set_witness(tete_grid* g, int32_t iw, int32_t jw)
{
    if (!g) return TETE_ERR_ARG;
    if (!g->has_bunch) return TETE_ERR_STATE;
    if (iw < 1 || iw > g->d.nx - 1 || jw < 1 || jw > g->d.ny - 1) return TETE_ERR_ARG;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    HIPCHK(launch_fill_f64(g->wit, (int64_t)TETE_WITNESS_LINES * TETE_MAX_WAKE, 0.0, g->stream));
    g->iw = iw;
    g->jw = jw;
    g->witness = 1;
    return TETE_OK;
}

tete_status tete_clear_witness(tete_grid* g)
{
    if (!g) return TETE_ERR_ARG;
    g->witness = 0;
    return TETE_OK;
}

tete_status tete_witness_wake(tete_grid* g, double* W, double* Wx, double* Wy, int32_t nw)
{
    if (!g || !W) return TETE_ERR_ARG;
    if (!g->has_bunch || !g->witness) return TETE_ERR_STATE;
    if (nw < 1 || nw > g->b.nw) return TETE_ERR_ARG;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    for (int l = 0; l < TETE_WITNESS_LINES; ++l)
        HIPCHK(hipMemcpyAsync(W + (size_t)l * nw, g->wit + (size_t)l * TETE_MAX_WAKE, sizeof(double) * nw,
                              hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    const double q = 1.0 / (g->b.charge_C * kEps0);
    for (size_t e = 0; e < (size_t)TETE_WITNESS_LINES * nw; ++e) W[e] *= q;
    if (check_finite(g, W, (int64_t)TETE_WITNESS_LINES * nw) != TETE_OK) return g->err;
    // Panofsky-Wenzel: dW_perp/ds = grad_perp W_par, centred differences across
    // the witness node, trapezoid rule in s from the first sample
    const double ds = g->d.dz;
    const double* Wm[2] = {W + 1 * (size_t)nw, W + 3 * (size_t)nw};
    const double* Wp[2] = {W + 2 * (size_t)nw, W + 4 * (size_t)nw};
    const double h2[2] = {2.0 * g->d.dx, 2.0 * g->d.dy};
    double* out[2] = {Wx, Wy};
    for (int c = 0; c < 2; ++c) {
        if (!out[c]) continue;
        double prev = (Wp[c][0] - Wm[c][0]) / h2[c], sum = 0.0;
        out[c][0] = 0.0;
        for (int j = 1; j < nw; ++j) {
            const double d = (Wp[c][j] - Wm[c][j]) / h2[c];
            sum += 0.5 * (d + prev) * ds;
            out[c][j] = sum;
            prev = d;
        }
    }
    return TETE_OK;
}

tete_status tete_energy(tete_grid* g, double* W, int64_t* n)
{
    if (!g || !W) return TETE_ERR_ARG;
    if (g->yee) return TETE_ERR_STATE;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    if (g->fp32) HIPCHK(launch_energy<float>(fields<float>(g, g->cur), mats<float>(g), g->geo, g->alpha, rweight(g), g->partial, g->scal, g->stream));
    else HIPCHK(launch_energy<double>(fields<double>(g, g->cur), mats<double>(g), g->geo, g->alpha, rweight(g), g->partial, g->scal, g->stream));
    double v;
    HIPCHK(hipMemcpyAsync(&v, g->scal, sizeof(double), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    *W = v;
    if (n) *n = g->n;
    return check_finite(g, &v, 1);
}

tete_status tete_energy_noalloc(tete_grid* g, double* W, int64_t* n)
{
    if (!g || !W) return TETE_ERR_ARG;
    if (g->yee) return TETE_ERR_STATE;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    double* sc;
    tete_status st = scratch_on(g->device, &sc);
    if (st != TETE_OK) return st;
    // the same kernels as tete_energy; every partial sum and the result are
    // written before they are read, so nothing is cleared first
    double* partial = sc;
    double* result = sc + RED_BLOCKS;
    if (g->fp32) HIPCHK(launch_energy<float>(fields<float>(g, g->cur), mats<float>(g), g->geo, g->alpha, rweight(g), partial, result, g->stream));
    else HIPCHK(launch_energy<double>(fields<double>(g, g->cur), mats<double>(g), g->geo, g->alpha, rweight(g), partial, result, g->stream));
    double v;
    HIPCHK(hipMemcpyAsync(&v, result, sizeof(double), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    *W = v;
    if (n) *n = g->n;
    return check_finite(g, &v, 1);
}

tete_status tete_energy_series(tete_grid* g, double* out, int64_t max, int64_t* count)
{
    if (!g || !count || max < 0 || (max > 0 && !out)) return TETE_ERR_ARG;
    if (g->yee) return TETE_ERR_STATE;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    int64_t c = std::min(max, g->ecount);
    if (c > 0) HIPCHK(hipMemcpyAsync(out, g->eser, sizeof(double) * c, hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    *count = g->ecount;
    return check_finite(g, out, c);
}

tete_status tete_probes(tete_grid* g, double* out, int64_t max, int64_t* count)
{
    if (!g || !count || max < 0 || (max > 0 && !out)) return TETE_ERR_ARG;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    int64_t c = std::min(max, g->pcount * g->nprobe);
    if (c > 0) HIPCHK(hipMemcpyAsync(out, g->pser, sizeof(double) * c, hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    *count = g->pcount;
    return check_finite(g, out, c);
}

tete_status tete_charges(tete_grid* g, double* max_res_e, double* max_abs_h)
{
    if (!g || !max_res_e || !max_abs_h) return TETE_ERR_ARG;
    if (g->n < 1 || g->yee) return TETE_ERR_STATE;
    DeviceGuard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    Src s = source(g, g->n - 1);
    if (g->fp32)
        HIPCHK(launch_charges<float>(fields<float>(g, 1 - g->cur), fields<float>(g, g->cur), mats<float>(g), g->geo,
                                     g->alpha * rweight(g), s, g->partial, g->scal + 2, g->stream));
    else
        HIPCHK(launch_charges<double>(fields<double>(g, 1 - g->cur), fields<double>(g, g->cur), mats<double>(g),
                                      g->geo, g->alpha * rweight(g), s, g->partial, g->scal + 2, g->stream));
    double v[2];
    HIPCHK(hipMemcpyAsync(v, g->scal + 2, sizeof(double) * 2, hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    *max_res_e = v[0];
    *max_abs_h = v[1];
    return check_finite(g, v, 2);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches: many grids stepped together by one persistent launch per step.
// ---------------------------------------------------------------------------

struct tete_batch {
    int fp32;
    hipStream_t stream;       // caller's stream
    hipStream_t gstream;      // private stream the steps run on (graphs cannot be captured on the null stream)
    hipEvent_t ev_in, ev_out; // order gstream after / before the caller's stream
    int device;
    void* table;              // device BatchTable<R>
    void* host;               // host staging copy
    size_t bytes;
    tete_grid* slot[TETE_MAX_BATCH];
    int64_t seen_n[TETE_MAX_BATCH];   // (n, cur) of each member when the table was built
    int seen_cur[TETE_MAX_BATCH];
    int kernel;               // TETE_KERNEL_AUTO, _FUSED or _FUSED2
    int two;                  // the table holds two-step arguments and blocks use them
    int rows, depth, graph_steps;
    int dirty;
    int phase;
    int grid;                 // persistent workgroups
    hipGraph_t graph;
    hipGraphExec_t exec;
    int graph_ok;
};

namespace {

void batch_drop_graph(tete_batch* b)
{
    if (b->graph_ok) {
        (void)hipGraphExecDestroy(b->exec);
        (void)hipGraphDestroy(b->graph);
        b->graph_ok = 0;
    }
}

template <typename R>
size_t batch_table_bytes() { return up(sizeof(BatchTable<R>)); }

// Tile order of a batch member: its own, or k-tiles first (the blocked
// orders, which match a single grid's tiles to the XCDs, do not apply when
// the items of many grids share the persistent workgroups).
int batch_order(const tete_grid* g) { return g->tune.order != 0 ? g->tune.order : 2; }

// Two-step arguments of one member for both parities.
template <typename R>
bool batch_two_args(tete_grid* g, BatchItem<R>& it, int phase, int& total2)
{
    FArgs<R> f2 = fused_args<R>(fields<R>(g, g->cur), fields<R>(g, 1 - g->cur), mats<R>(g), g->geo, (R)g->alpha,
                                source(g, g->n));
    FArgs<R> b2 = fused_args<R>(fields<R>(g, 1 - g->cur), fields<R>(g, g->cur), mats<R>(g), g->geo, (R)g->alpha,
                                source(g, g->n));
    const int xc = g->tune.kernel == TETE_KERNEL_FUSED2 ? g->tune.xchunk : 0;
    if (!fused2_setup<R>(f2, 0, xc, batch_order(g)) || !fused2_setup<R>(b2, 0, xc, batch_order(g))) return false;
    it.a2[phase] = f2;
    it.a2[1 - phase] = b2;
    total2 += f2.nblk;
    return true;
}

template <typename R>
tete_status batch_build(tete_batch* b)
{
    BatchTable<R>* H = (BatchTable<R>*)b->host;
    memset(H, 0, sizeof(BatchTable<R>));
    H->phase = b->phase;
    // two steps per launch unless the single step was asked for, and only if
    // every member's planes fit the two-step kernel
    bool two = b->kernel != TETE_KERNEL_FUSED;
    for (int s = 0; s < TETE_MAX_BATCH && two; ++s)
        if (b->slot[s] && !fused2_fits(b->slot[s]->geo, b->fp32 ? 4 : 8)) two = false;
    if ((int)two != b->two) {
        batch_drop_graph(b);   // the captured block launches the other kernel
        b->two = two;
    }
    int total = 0, total2 = 0;
    for (int s = 0; s < TETE_MAX_BATCH; ++s) {
        tete_grid* g = b->slot[s];
        if (!g) continue;
        const int i = H->ninst++;
        Mat<R> M = mats<R>(g);
        Src src = source(g, g->n);
        FArgs<R> fwd = fused_args<R>(fields<R>(g, g->cur), fields<R>(g, 1 - g->cur), M, g->geo, (R)g->alpha, src);
        FArgs<R> bwd = fused_args<R>(fields<R>(g, 1 - g->cur), fields<R>(g, g->cur), M, g->geo, (R)g->alpha, src);
        if (!fused_setup<R>(fwd, b->rows, g->tune.xchunk, batch_order(g)) ||
            !fused_setup<R>(bwd, b->rows, g->tune.xchunk, batch_order(g)))
            return TETE_ERR_ARG;
        // at the current phase the grid reads its current set
        H->item[i].a[b->phase] = fwd;
        H->item[i].a[1 - b->phase] = bwd;
        H->offset[i] = total;
        H->offset2[i] = total2;
        if (two && !batch_two_args<R>(g, H->item[i], b->phase, total2)) return TETE_ERR_ARG;
        H->step[i] = g->n;
        total += fwd.nblk;
        b->seen_n[s] = g->n;
        b->seen_cur[s] = g->cur;
    }
    H->offset[H->ninst] = total;
    H->offset2[H->ninst] = total2;
    H->total = total;
    H->total2 = total2;
    HIPCHK(hipMemcpyAsync(b->table, H, sizeof(BatchTable<R>), hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    b->dirty = 0;
    return TETE_OK;
}

// Launches of a block of `steps` steps (two per launch where the batch uses
// the two-step kernel, a single step for an odd last one); the number of
// launches, each of which swaps the ping-pong sets once.
int batch_block_launches(const tete_batch* b, int steps) { return b->two ? (steps + 1) / 2 : steps; }

template <typename R>
tete_status batch_launch_block(tete_batch* b, int steps)
{
    BatchTable<R>* T = (BatchTable<R>*)b->table;
    int done = 0, flips = 0;
    if (b->two)
        for (; done + 2 <= steps; done += 2, ++flips)
            HIPCHK(launch_batch_step2<R>(T, b->grid, flips, done, b->gstream));
    for (; done < steps; ++done, ++flips)
        HIPCHK(launch_batch_step<R>(T, b->rows, b->depth, b->grid, flips, done, b->gstream));
    HIPCHK(launch_batch_advance<R>(T, steps, flips, b->gstream));
    return TETE_OK;
}

template <typename R>
tete_status batch_step(tete_batch* b, int64_t nsteps)
{
    for (int s = 0; s < TETE_MAX_BATCH; ++s)
        if (b->slot[s] && (b->slot[s]->n != b->seen_n[s] || b->slot[s]->cur != b->seen_cur[s])) b->dirty = 1;
    if (b->dirty) {
        tete_status st = batch_build<R>(b);
        if (st != TETE_OK) return st;
    }
    if (((BatchTable<R>*)b->host)->ninst == 0) return TETE_OK;
    const int K = b->graph_steps;
    const int64_t full = K > 0 ? nsteps / K : 0;
    const int rem = (int)(nsteps - full * K);
    HIPCHK(hipEventRecord(b->ev_in, b->stream));
    HIPCHK(hipStreamWaitEvent(b->gstream, b->ev_in, 0));
    if (full > 0 && !b->graph_ok) {
        HIPCHK(hipStreamBeginCapture(b->gstream, hipStreamCaptureModeThreadLocal));
        tete_status st = batch_launch_block<R>(b, K);
        hipGraph_t graph;
        hipError_t e = hipStreamEndCapture(b->gstream, &graph);
        if (st != TETE_OK || e != hipSuccess) return TETE_ERR_DEVICE;
        if (hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return TETE_ERR_DEVICE;
        }
        b->graph = graph;
        b->graph_ok = 1;
    }
    for (int64_t f = 0; f < full; ++f) HIPCHK(hipGraphLaunch(b->exec, b->gstream));
    if (rem > 0) {
        tete_status st = batch_launch_block<R>(b, rem);
        if (st != TETE_OK) return st;
    }
    HIPCHK(hipEventRecord(b->ev_out, b->gstream));
    HIPCHK(hipStreamWaitEvent(b->stream, b->ev_out, 0));
    const int flip = (int)((full * batch_block_launches(b, K) + batch_block_launches(b, rem)) & 1);
    for (int s = 0; s < TETE_MAX_BATCH; ++s) {
        tete_grid* g = b->slot[s];
        if (!g) continue;
        g->n += nsteps;
        g->cur ^= flip;
        b->seen_n[s] = g->n;
        b->seen_cur[s] = g->cur;
    }
    b->phase ^= flip;
    return TETE_OK;
}

}  // namespace

extern "C" {

size_t tete_batch_bytes(int32_t precision)
{
    if (precision == TETE_FP32) return batch_table_bytes<float>();
    if (precision == TETE_FP64) return batch_table_bytes<double>();
    return 0;
}

tete_status tete_batch_create(int32_t precision, void* dev_table, size_t bytes, void* hip_stream, tete_batch** out)
{
    if (!out) return TETE_ERR_ARG;
    *out = nullptr;
    const size_t need = tete_batch_bytes(precision);
    if (need == 0 || !dev_table || ((uintptr_t)dev_table % kAlign) != 0) return TETE_ERR_ARG;
    if (bytes < need) return TETE_ERR_NOMEM;
    tete_batch* b = (tete_batch*)calloc(1, sizeof(tete_batch));
    if (!b) return TETE_ERR_NOMEM;
    b->host = calloc(1, need);
    if (!b->host) { free(b); return TETE_ERR_NOMEM; }
    b->fp32 = precision == TETE_FP32;
    b->stream = (hipStream_t)hip_stream;
    b->table = dev_table;
    b->bytes = bytes;
    b->rows = 0;
    b->depth = 1;   // the persistent kernel at depth 2 or 3 exceeds the register file
    b->graph_steps = 8;
    b->dirty = 1;
    int cus = 0;
    if (hipGetDevice(&b->device) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess) {
        free(b->host);
        free(b);
        return TETE_ERR_DEVICE;
    }
    b->grid = cus > 0 ? cus : 256;
    if (hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking) != hipSuccess) {
        free(b->host);
        free(b);
        return TETE_ERR_DEVICE;
    }
    if (hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess) {
        (void)hipStreamDestroy(b->gstream);
        free(b->host);
        free(b);
        return TETE_ERR_DEVICE;
    }
    *out = b;
    return TETE_OK;
}

tete_status tete_batch_destroy(tete_batch* b)
{
    if (!b) return TETE_ERR_ARG;
    (void)hipStreamSynchronize(b->gstream);
    batch_drop_graph(b);
    (void)hipEventDestroy(b->ev_in);
    (void)hipEventDestroy(b->ev_out);
    (void)hipStreamDestroy(b->gstream);
    free(b->host);
    free(b);
    return TETE_OK;
}

tete_status tete_batch_set(tete_batch* b, int32_t slot, tete_grid* g)
{
    if (!b || slot < 0 || slot >= TETE_MAX_BATCH) return TETE_ERR_ARG;
    if (g) {
        if (g->fp32 != b->fp32 || g->device != b->device) return TETE_ERR_ARG;
        if (g->yee || g->implicit || g->mat_set || g->witness || !fused_fits(g->geo, g->fp32 ? 4 : 8))
            return TETE_ERR_STATE;
        if (g->err != TETE_OK) return g->err;
        for (int s = 0; s < TETE_MAX_BATCH; ++s)
            if (s != slot && b->slot[s] == g) return TETE_ERR_ARG;
    }
    b->slot[slot] = g;
    b->dirty = 1;
    return TETE_OK;
}

tete_status tete_batch_set_launch(tete_batch* b, int32_t kernel, int32_t rows, int32_t depth, int32_t graph_steps)
{
    if (!b || (rows != 0 && rows != 12 && rows != 16) || depth < 0 || depth > 3 || graph_steps < 0 ||
        graph_steps > 1024)
        return TETE_ERR_ARG;
    if (kernel != TETE_KERNEL_AUTO && kernel != TETE_KERNEL_FUSED && kernel != TETE_KERNEL_FUSED2) return TETE_ERR_ARG;
    b->kernel = kernel;
    b->rows = rows;
    b->depth = depth == 0 ? 1 : depth;
    b->graph_steps = graph_steps;
    batch_drop_graph(b);
    b->dirty = 1;
    return TETE_OK;
}

tete_status tete_batch_step(tete_batch* b, int64_t nsteps)
{
    if (!b || nsteps < 0) return TETE_ERR_ARG;
    if (nsteps == 0) return TETE_OK;
    for (int s = 0; s < TETE_MAX_BATCH; ++s) {   // a witness set after joining: batched steps would skip it
        if (b->slot[s] && b->slot[s]->witness) return TETE_ERR_STATE;
        if (b->slot[s] && b->slot[s]->err != TETE_OK) return b->slot[s]->err;
    }
    DeviceGuard dg(b->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    return b->fp32 ? batch_step<float>(b, nsteps) : batch_step<double>(b, nsteps);
}

tete_status tete_batch_count(tete_batch* b, int32_t* active)
{
    if (!b || !active) return TETE_ERR_ARG;
    int c = 0;
    for (int s = 0; s < TETE_MAX_BATCH; ++s) c += b->slot[s] != nullptr;
    *active = c;
    return TETE_OK;
}

}  // extern "C"
