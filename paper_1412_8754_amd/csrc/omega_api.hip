// C entry points of libomega (declared in include/omega.h): host-side
// validation, workspace layout and the launch sequence of each call.
//
// Points are processed in groups of equal lattice size (first-appearance
// order), each group in batches whose chunk partials fit a fixed budget.
// A point's momentum chunking depends only on its own lattice size and the
// call's Delta / Q / band counts, so its result is bitwise the same whatever
// batch it travels in.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "omega.h"
#include "omega_internal.h"

namespace {

using namespace omega;

constexpr size_t kAlign = 256;
constexpr int kMaxL = 16384;
constexpr long long kMaxK = 1LL << 26;
constexpr int kMaxDelta = 1 << 20;
constexpr int kMaxQ = 16384;
constexpr long long kMaxCells = 1LL << 30;   // n_q * n_delta of one (point, band)
constexpr int kMaxPoints = 1 << 24;
constexpr int kMinWorkgroups = 4096;       // per point, below this chunks split finer
constexpr int kMinLaunchUnits = 12288;     // per point: 4 sweep units per resident wave
constexpr size_t kBatchBytes = 512u << 20; // chunk partials of one batch
constexpr int kMaxGridZ = 65535;
constexpr int kGradTilesPerChunk = 64;

// Launch options of one call (omega_launch, resolved): none changes a result.
struct Launch {
    int blocks_per_cu = 0;        // persistent sweeps: 0 = all that fit
    int n_queues = kQueues;       // work queues of the persistent sweeps
    hipEvent_t start = nullptr;   // recorded before the call's first per-Delta sweep
    hipEvent_t stop = nullptr;    // and after its last one
    unsigned long long *count = nullptr;   // direct (k, Delta) terms, added on the device
};

bool resolve_launch(const omega_launch *in, Launch *out)
{
    Launch l;
    if (in) {
        if (in->sweep_blocks_per_cu < 0 || in->sweep_queues < 0 ||
            in->sweep_queues > kMaxQueues ||
            (in->sweep_start_event == nullptr) != (in->sweep_stop_event == nullptr))
            return false;
        l.blocks_per_cu = in->sweep_blocks_per_cu;
        if (in->sweep_queues > 0)
            l.n_queues = in->sweep_queues;
        l.start = (hipEvent_t)in->sweep_start_event;
        l.stop = (hipEvent_t)in->sweep_stop_event;
        l.count = in->count_dev;
    }
    *out = l;
    return true;
}

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

int n_bands(int bands) { return (bands & 1) + ((bands >> 1) & 1); }

int slot_bands(int bands, int *list)
{
    int nb = 0;
    if (bands & OMEGA_BAND_MINUS)
        list[nb++] = 0;
    if (bands & OMEGA_BAND_PLUS)
        list[nb++] = 1;
    return nb;
}

int slot_bands3(int bands, int *list)
{
    int nb = 0;
    for (int b = 0; b < 3; ++b)
        if (bands & (1 << b))
            list[nb++] = b;
    return nb;
}

bool model3_ok(const omega3_model *m, int bands)
{
    if (!m)
        return false;
    for (double x : m->t)
        if (!isfinite(x))
            return false;
    if (!isfinite(m->eps0) || !isfinite(m->mu))
        return false;
    if (m->form != OMEGA_ETA_K && m->form != OMEGA_ETA_REL)
        return false;
    for (int b = 0; b < 3; ++b)
        if ((bands & (1 << b)) && (!isfinite(m->V[b]) || m->V[b] == 0.0))
            return false;
    return true;
}

bool model_ok(const omega_model *m)
{
    if (!m)
        return false;
    const double v[7] = {m->t1, m->t2, m->t3, m->t4, m->mu, m->V[0], m->V[1]};
    for (double x : v)
        if (!isfinite(x))
            return false;
    if (m->form != OMEGA_ETA_K && m->form != OMEGA_ETA_REL)
        return false;
    return m->V[0] != 0.0 && m->V[1] != 0.0;
}

bool point_ok(const omega_point &p)
{
    if (!isfinite(p.h) || !isfinite(p.T) || p.T < 0.0)
        return false;
    if (p.T > 0.0 && !isnormal(p.T))
        return false;   // 1/T must be finite
    if (p.Lx < 2 || p.Ly < 2 || p.Lx > kMaxL || p.Ly > kMaxL)
        return false;
    return (long long)p.Lx * p.Ly <= kMaxK;
}

bool points_ok(const omega_point *pts, int n_pts)
{
    if (!pts || n_pts <= 0 || n_pts > kMaxPoints)
        return false;
    for (int i = 0; i < n_pts; ++i)
        if (!point_ok(pts[i]))
            return false;
    return true;
}

bool sizes_ok(int n_delta, int n_q, int bands, int precision)
{
    return n_delta > 0 && n_delta <= kMaxDelta && n_q > 0 && n_q <= kMaxQ &&
           (long long)n_q * n_delta <= kMaxCells &&
           bands >= 1 && bands <= 3 &&
           (precision == OMEGA_FP64 || precision == OMEGA_FP32_COMP);
}

int delta_tile(int n_delta) { return n_delta >= 32 ? 32 : 16; }

struct Tiles {
    int TX, TY, n_tiles, n_chunks;
};

// Sweep chunking of one point: 256 tiles per chunk, fewer while the point
// would give less than kMinWorkgroups series workgroups (chunks times the
// other grid dimensions), down to 4 tiles, or less than kMinLaunchUnits
// units to the persistent sweep, down to 64 tiles.  It depends on the point
// and the call's Delta/Q/band counts only.
Tiles sweep_tiles(int Lx, int Ly, long long other_blocks)
{
    Tiles r;
    r.TX = (Lx + kTileEdge - 1) / kTileEdge;
    r.TY = (Ly + kTileEdge - 1) / kTileEdge;
    r.n_tiles = r.TX * r.TY;
    int tpw = kMaxChunkTiles;
    for (;;) {
        const long long units = (long long)((r.n_tiles + tpw - 1) / tpw) * other_blocks;
        if (!((tpw > 4 && units < kMinWorkgroups) || (tpw > 64 && units < kMinLaunchUnits)))
            break;
        tpw /= 2;
    }
    r.n_chunks = (r.n_tiles + tpw - 1) / tpw;
    return r;
}

// Per-wave capacity of the series pass's tile lists.  sweep_tiles makes a
// chunk at most kMaxChunkTiles tiles, so this is at most kMaxWaveList, the
// entries the series pass stages per wave in LDS.
static_assert(4 * kMaxWaveList >= kMaxChunkTiles, "series-pass list staging too small");
int list_cap(const Tiles &t)
{
    const int span = (t.n_tiles + t.n_chunks - 1) / t.n_chunks;
    return (span + 3) / 4;
}

Tiles grad_tiles(int Lx, int Ly)
{
    Tiles r;
    r.TX = (Lx + kTileEdge - 1) / kTileEdge;
    r.TY = (Ly + kTileEdge - 1) / kTileEdge;
    r.n_tiles = r.TX * r.TY;
    r.n_chunks = (r.n_tiles + kGradTilesPerChunk - 1) / kGradTilesPerChunk;
    return r;
}

// Points of equal (Lx, Ly), in order of first appearance.
struct Group {
    int Lx, Ly;
    bool hot;   // grid sweeps: T >= kInPlaceT
    std::vector<int> idx;
};

// Points grouped by lattice size and, for the grid sweeps (split_hot), by
// T >= kInPlaceT, which picks the sweep kernel: a point's group, and so the
// arithmetic of its result, depends on the point alone.
std::vector<Group> group_points(const omega_point *pts, int n, bool split_hot = false)
{
    std::vector<Group> gs;
    for (int i = 0; i < n; ++i) {
        const bool hot = split_hot && pts[i].T >= kInPlaceT;
        Group *g = nullptr;
        for (Group &x : gs)
            if (x.Lx == pts[i].Lx && x.Ly == pts[i].Ly && x.hot == hot) {
                g = &x;
                break;
            }
        if (!g) {
            gs.push_back(Group{pts[i].Lx, pts[i].Ly, hot, {}});
            g = &gs.back();
        }
        g->idx.push_back(i);
    }
    return gs;
}

int batch_points(size_t per_point_bytes, int group_size, int max_z)
{
    size_t g = kBatchBytes / (per_point_bytes ? per_point_bytes : 1);
    if (g < 1)
        g = 1;
    if (g > (size_t)group_size)
        g = group_size;
    if (g > (size_t)max_z)
        g = max_z;
    return (int)g;
}

// Workspace of a grid / argmin call.
struct GridPlan {
    int nb, td, n_dtiles, n_delta_pad, nbq;
    std::vector<Group> groups;
    std::vector<Tiles> tiles;   // per group
    std::vector<int> batch;     // points per batch, per group
    std::vector<int> vchunks;   // momentum chunks of the FP64 check, per group
    size_t off_d2, off_qtrig, off_gtab, off_trig, off_table, off_part, off_base, off_mom,
        off_tlist, off_tcnt, off_tpart, off_etab, off_qlat, off_queue, off_rowmin, off_vcand,
        off_vcnt, off_vthr, off_vpart, sweep_bytes;
};

// Momentum chunks of one candidate's FP64 sum in the check of the
// FP32-compensated search: about 4096 busy units at two candidates per set,
// at least 4096 momenta per chunk.
int verify_chunks(long long n_k, int sets)
{
    long long c = (4096 + 2LL * sets - 1) / (2LL * sets);
    const long long cap = (n_k + 4095) / 4096;
    c = c < cap ? c : cap;
    return c < 1 ? 1 : (int)c;
}

// b3: three-band model.  The band table of the largest lattice holds 3 bands
// for it and 2 for the two-band model; the lattice indices of the pair momenta
// follow it.
GridPlan plan_grid(const omega_point *pts, int n_pts, int n_delta, int n_q, int nb,
                   bool b3)
{
    GridPlan p;
    p.nb = nb;
    p.td = delta_tile(n_delta);
    p.n_dtiles = (n_delta + p.td - 1) / p.td;
    p.n_delta_pad = p.n_dtiles * p.td;
    p.nbq = nb * n_q;
    p.groups = group_points(pts, n_pts, true);
    size_t trig = 0, table = 0, part = 0, base = 0, mom = 0, etab = 0, tlist = 0,
           tcnt = 0, tpart = 0, vsets = 0, vpart = 0;
    for (const Group &g : p.groups) {
        const Tiles t = sweep_tiles(g.Lx, g.Ly, (long long)p.n_dtiles * p.nbq);
        etab = std::max(etab, sizeof(double) * (b3 ? 3 : 2) * (size_t)g.Lx * g.Ly);
        const size_t rows = (size_t)p.nbq * t.n_chunks;
        const size_t lcap = list_cap(t);
        const size_t per_point =
            sizeof(double) * rows * (p.n_delta_pad + 1 + kMomentSlots +
                                     (size_t)p.n_dtiles * kTileSlots) +
            sizeof(unsigned long long) * rows * 4 * lcap * 2 + sizeof(int) * rows;
        const int G = batch_points(per_point, (int)g.idx.size(), kMaxGridZ / p.nbq);
        p.tiles.push_back(t);
        p.batch.push_back(G);
        const int vc = verify_chunks((long long)g.Lx * g.Ly, G * nb);
        p.vchunks.push_back(vc);
        vsets = std::max(vsets, (size_t)G * nb);
        vpart = std::max(vpart, sizeof(double) * (size_t)G * nb * kVerifyMax * vc);
        trig = std::max(trig, sizeof(double) * 2 * ((size_t)g.Lx + g.Ly));
        table = std::max(table, sizeof(PointRec) * (size_t)G);
        part = std::max(part, sizeof(double) * rows * p.n_delta_pad * G);
        base = std::max(base, sizeof(double) * rows * G);
        mom = std::max(mom, sizeof(double) * rows * kMomentSlots * G);
        tlist = std::max(tlist, sizeof(unsigned long long) * rows * 4 * lcap * 2 * G);
        tcnt = std::max(tcnt, sizeof(int) * rows * G);
        tpart = std::max(tpart, sizeof(double) * rows * p.n_dtiles * kTileSlots * G);
    }
    p.off_d2 = 0;
    p.off_qtrig = p.off_d2 + align_up(sizeof(double) * (p.n_delta_pad + 2));
    p.off_gtab = p.off_qtrig + align_up(sizeof(double) * kQTrig * (size_t)n_q);
    p.off_trig = p.off_gtab + align_up(sizeof(double2) * kGTabEntries + sizeof(float4) * kG32N);
    p.off_table = p.off_trig + align_up(trig);
    p.off_part = p.off_table + align_up(table);
    p.off_base = p.off_part + align_up(part);
    p.off_mom = p.off_base + align_up(base);
    p.off_tlist = p.off_mom + align_up(mom);
    p.off_tcnt = p.off_tlist + align_up(tlist);
    p.off_tpart = p.off_tcnt + align_up(tcnt);
    p.off_etab = p.off_tpart + align_up(tpart);
    p.off_qlat = p.off_etab + align_up(etab);
    p.off_queue = p.off_qlat + align_up(sizeof(int) * 2 * (size_t)n_q);
    p.off_rowmin = p.off_queue + align_up(sizeof(unsigned long long) * kMaxQueues * kQueueStride);
    // the minimum of every output row, for the global search
    p.off_vcand = p.off_rowmin + align_up(sizeof(double) * (size_t)n_pts * p.nbq);
    p.off_vcnt = p.off_vcand + align_up(sizeof(int) * vsets * kVerifyMax);
    p.off_vthr = p.off_vcnt + align_up(sizeof(int) * vsets);
    p.off_vpart = p.off_vthr + align_up(sizeof(double) * vsets);
    p.sweep_bytes = p.off_vpart + align_up(vpart);
    return p;
}

size_t grid_bytes(int n_pts, int n_delta, int n_q, int nb)
{
    return align_up(sizeof(double) * (size_t)n_pts * nb * n_q * n_delta);
}

// Workspace of a gradient call.
struct GradPlan {
    std::vector<Group> groups;
    std::vector<Tiles> tiles;
    std::vector<int> batch;
    size_t off_qtrig, off_trig, off_table, off_part, bytes;
};

GradPlan plan_grad(const omega_point *pts, int n_pts, int nb)
{
    GradPlan p;
    p.groups = group_points(pts, n_pts);
    size_t trig = 0, table = 0, part = 0;
    for (const Group &g : p.groups) {
        const Tiles t = grad_tiles(g.Lx, g.Ly);
        const size_t per_point = sizeof(double) * 5 * (size_t)nb * t.n_chunks;
        const int G = batch_points(per_point, (int)g.idx.size(), kMaxGridZ);
        p.tiles.push_back(t);
        p.batch.push_back(G);
        trig = std::max(trig, sizeof(double) * 2 * ((size_t)g.Lx + g.Ly));
        table = std::max(table, sizeof(PointRec) * (size_t)G);
        part = std::max(part, per_point * G);
    }
    p.off_qtrig = 0;
    p.off_trig = align_up(sizeof(double) * kQTrig * (size_t)n_pts * nb);
    p.off_table = p.off_trig + align_up(trig);
    p.off_part = p.off_table + align_up(table);
    p.bytes = p.off_part + align_up(part);
    return p;
}

Hop make_hop(const omega_model *m)
{
    Hop h;
    h.tA = -(m->t1 + m->t2);
    h.tB = -4.0 * m->t3;
    h.tD = -(m->t1 - m->t2);
    h.tC = -4.0 * m->t4;
    return h;
}

void band_signs(int nb, const int *list, double *eps)
{
    eps[0] = list[0] ? 1.0 : -1.0;
    eps[1] = nb > 1 ? (list[1] ? 1.0 : -1.0) : eps[0];
}

// Write the records of points idx[0..G) into the device table.
// queue (optional): the work-queue counters of the batch, zeroed on the way.
int upload_points(const omega_point *pts, const int *idx, int G, PointRec *table,
                  unsigned long long *queue, hipStream_t s)
{
    for (int b = 0; b < G; b += kFillMax) {
        PointPack pk;
        pk.n = G - b < kFillMax ? G - b : kFillMax;
        pk.pad = 0;
        for (int i = 0; i < pk.n; ++i) {
            const omega_point &pt = pts[idx[b + i]];
            pk.rec[i].h = pt.h;
            pk.rec[i].T = pt.T;
            pk.rec[i].out = idx[b + i];
            pk.rec[i].pad = 0;
        }
        if (launch_fill_points(pk, table + b, queue, s) != hipSuccess)
            return OMEGA_E_HIP;
    }
    return OMEGA_OK;
}

// Either model, as the sweep sees it: band selection per output slot,
// couplings and hoppings.
struct ModelDesc {
    bool b3;
    int eta_rel;     // form factor at the pair's relative momentum
    int nb;
    int list[3];
    double mu;
    double V[3];     // per output slot
    Hop hop;         // two-band
    Hop3 hop3;       // three-band
};

ModelDesc describe(const omega_model *m, int bands)
{
    ModelDesc d{};
    d.b3 = false;
    d.eta_rel = m->form == OMEGA_ETA_REL;
    d.nb = slot_bands(bands, d.list);
    d.mu = m->mu;
    for (int k = 0; k < 3; ++k)
        d.V[k] = m->V[d.list[k < d.nb ? k : 0]];
    d.hop = make_hop(m);
    return d;
}

ModelDesc describe3(const omega3_model *m, int bands)
{
    ModelDesc d{};
    d.b3 = true;
    d.eta_rel = m->form == OMEGA_ETA_REL;
    d.nb = slot_bands3(bands, d.list);
    d.mu = m->mu;
    for (int k = 0; k < 3; ++k)
        d.V[k] = m->V[d.list[k < d.nb ? k : 0]];
    for (int k = 0; k < 12; ++k)
        d.hop3.t[k] = m->t[k];
    d.hop3.eps0 = m->eps0;
    return d;
}

// Enqueue the sweep and row reduction of every point.  Omega goes to `grid`,
// row minima to row_idx (optional).
// With idx (the FP32-compensated argmin), every batch's minima are checked
// in FP64 and written to idx / omin (see VerifyArgs).
int enqueue_grid(const ModelDesc &md, const omega_point *pts, int n_pts,
                 const double *delta, int n_delta, const double *q, int n_q,
                 int precision, char *ws, double tie_rel,
                 double *grid, int32_t *row_idx, int32_t *idx, double *omin, const Launch &lo,
                 hipStream_t s)
{
    const int nb = md.nb;
    const GridPlan P = plan_grid(pts, n_pts, n_delta, n_q, nb, md.b3);
    double *d2 = (double *)(ws + P.off_d2);
    double *qtrig = (double *)(ws + P.off_qtrig);
    double2 *gtab = (double2 *)(ws + P.off_gtab);
    float4 *gtab32 = (float4 *)(ws + P.off_gtab + sizeof(double2) * kGTabEntries);
    double *trig = (double *)(ws + P.off_trig);
    PointRec *table = (PointRec *)(ws + P.off_table);
    double *part = (double *)(ws + P.off_part);
    double *base = (double *)(ws + P.off_base);
    double *mom = (double *)(ws + P.off_mom);
    double *etab = (double *)(ws + P.off_etab);
    int *qlat = (int *)(ws + P.off_qlat);
    unsigned long long *tlist = (unsigned long long *)(ws + P.off_tlist);
    int *tcnt = (int *)(ws + P.off_tcnt);
    double *tpart = (double *)(ws + P.off_tpart);
    unsigned long long *queue = (unsigned long long *)(ws + P.off_queue);
    if (launch_call_tables(delta, n_delta, P.n_delta_pad, d2, q, n_q, qtrig, gtab, gtab32, s) !=
        hipSuccess)
        return OMEGA_E_HIP;

    SweepArgs a;
    a.hop = md.hop;
    band_signs(nb, md.list, a.eps);
    a.hop3 = md.hop3;
    for (int k = 0; k < 3; ++k)
        a.band3[k] = md.list[k < nb ? k : 0];
    a.etab = etab;
    a.qlat = qlat;
    a.mu = md.mu;
    a.pts = table;
    a.n_q = n_q;
    a.nbq = P.nbq;
    a.n_delta_pad = P.n_delta_pad;
    a.d2 = d2;
    a.eta_rel = md.eta_rel;
    a.q = q;
    a.qtrig = qtrig;
    a.trig = trig;
    a.gtab = gtab;
    a.gtab32 = gtab32;
    a.part = part;
    a.base_part = base;
    a.mpart = mom;
    a.tlist = tlist;
    a.tcnt = tcnt;
    a.tpart = tpart;
    a.n_dtiles = P.n_dtiles;
    a.count = lo.count;
    a.queue = queue;
    a.n_queues = lo.n_queues;
    a.blocks_per_cu = lo.blocks_per_cu;
    a.n_rows = 0;

    RowArgs r;
    r.part = part;
    r.base_part = base;
    r.mpart = mom;
    r.d2c = d2 + P.n_delta_pad;
    r.zero_d0 = precision == OMEGA_FP64 ? 0 : 1;
    r.rowmin = (double *)(ws + P.off_rowmin);
    r.d2 = d2;
    r.td = P.td;
    r.n_dtiles = P.n_dtiles;
    r.pts = table;
    r.delta = delta;
    r.q = q;
    for (int k = 0; k < 3; ++k)
        r.Vs[k] = md.V[k];
    r.tie_rel = tie_rel;
    r.n_delta = n_delta;
    r.n_delta_pad = P.n_delta_pad;
    r.n_q = n_q;
    r.nbq = P.nbq;
    r.omega = grid;
    r.row_idx = row_idx;

    VerifyArgs v;
    v.nb = nb;
    v.n_q = n_q;
    v.n_delta = n_delta;
    v.delta = delta;
    v.grid = grid;
    v.rowmin = r.rowmin;
    v.tie_rel = tie_rel;
    v.d2c = d2 + P.n_delta_pad;
    for (int k = 0; k < 3; ++k)
        v.Vs[k] = md.V[k];
    v.cand = (int *)(ws + P.off_vcand);
    v.cnt = (int *)(ws + P.off_vcnt);
    v.thr = (double *)(ws + P.off_vthr);
    v.vpart = (double *)(ws + P.off_vpart);
    v.idx = idx;
    v.omin = omin;

    for (size_t gi = 0; gi < P.groups.size(); ++gi) {
        const Group &g = P.groups[gi];
        const Tiles &t = P.tiles[gi];
        if (launch_group_tables(g.Lx, g.Ly, trig, q, n_q, qlat, s) != hipSuccess)
            return OMEGA_E_HIP;
        const hipError_t te = md.b3 ? launch_etab(md.hop3, trig, g.Lx, g.Ly, etab, s)
                                    : launch_etab2(md.hop, trig, g.Lx, g.Ly, etab, s);
        if (te != hipSuccess)
            return OMEGA_E_HIP;
        a.Lx = g.Lx;
        a.Ly = g.Ly;
        a.TX = t.TX;
        a.TY = t.TY;
        a.n_tiles = t.n_tiles;
        a.n_chunks = t.n_chunks;
        a.lcap = list_cap(t);
        r.n_k = (double)g.Lx * g.Ly;
        r.n_chunks = t.n_chunks;
        r.tpart = g.hot ? nullptr : tpart;   // the in-place kernel has no tile series
        const int n = (int)g.idx.size();
        for (int b0 = 0; b0 < n; b0 += P.batch[gi]) {
            const int G = n - b0 < P.batch[gi] ? n - b0 : P.batch[gi];
            int rc = upload_points(pts, g.idx.data() + b0, G, table, queue, s);
            if (rc != OMEGA_OK)
                return rc;
            if (launch_series(a, G, precision == OMEGA_FP64, md.b3, s) != hipSuccess)
                return OMEGA_E_HIP;
            const bool first = gi == 0 && b0 == 0;
            const bool last = gi + 1 == P.groups.size() && b0 + G >= n;
            if (first && lo.start && hipEventRecord(lo.start, s) != hipSuccess)
                return OMEGA_E_HIP;
            hipError_t e = precision == OMEGA_FP64
                               ? launch_sweep_f64(a, P.td, P.n_dtiles, G, md.b3, g.hot, s)
                               : launch_sweep_f32c(a, P.td, P.n_dtiles, G, md.b3, g.hot, s);
            if (e != hipSuccess)
                return OMEGA_E_HIP;
            if (last && lo.stop && hipEventRecord(lo.stop, s) != hipSuccess)
                return OMEGA_E_HIP;
            if (launch_rows(r, G, s) != hipSuccess)
                return OMEGA_E_HIP;
            if (idx) {
                v.sw = a;
                v.n_k = r.n_k;
                v.n_vchunks = P.vchunks[gi];
                if (launch_verify(v, G, md.b3, s) != hipSuccess)
                    return OMEGA_E_HIP;
            }
        }
    }
    return OMEGA_OK;
}

// Shared bodies of the grid / argmin entry points of both models (inputs
// already validated except pointers, workspace and tie_rel).
int run_grid(const ModelDesc &md, const omega_point *pts, int n_pts, const double *delta_dev,
             int n_delta, const double *q_dev, int n_q, int precision, void *ws_dev,
             size_t ws_bytes, double *omega_dev, void *stream)
{
    if (!delta_dev || !q_dev || !omega_dev || !ws_dev)
        return OMEGA_E_INVAL;
    if (ws_bytes < plan_grid(pts, n_pts, n_delta, n_q, md.nb, md.b3).sweep_bytes)
        return OMEGA_E_WORKSPACE;
    return enqueue_grid(md, pts, n_pts, delta_dev, n_delta, q_dev, n_q, precision,
                        (char *)ws_dev, 0.0, omega_dev, nullptr, nullptr, nullptr, Launch(),
                        (hipStream_t)stream);
}

int run_argmin(const ModelDesc &md, const omega_point *pts, int n_pts, const double *delta_dev,
               int n_delta, const double *q_dev, int n_q, int precision, double tie_rel,
               void *ws_dev, size_t ws_bytes, int32_t *idx_dev, double *omin_dev,
               int32_t *row_idx_dev, double *omega_dev, const Launch &lo, void *stream)
{
    if (!delta_dev || !q_dev || !idx_dev || !omin_dev || !ws_dev)
        return OMEGA_E_INVAL;
    if (!(tie_rel >= 0.0) || !isfinite(tie_rel))
        return OMEGA_E_INVAL;
    const int nb = md.nb;
    const GridPlan P = plan_grid(pts, n_pts, n_delta, n_q, nb, md.b3);
    const size_t sweep = P.sweep_bytes;
    const size_t need = sweep + (omega_dev ? 0 : grid_bytes(n_pts, n_delta, n_q, nb));
    if (ws_bytes < need)
        return OMEGA_E_WORKSPACE;
    double *grid = omega_dev ? omega_dev : (double *)((char *)ws_dev + sweep);
    hipStream_t s = (hipStream_t)stream;
    // FP32-compensated: each batch's minima are checked in FP64 on the way
    const bool fp32c = precision == OMEGA_FP32_COMP;
    int rc = enqueue_grid(md, pts, n_pts, delta_dev, n_delta, q_dev, n_q, precision,
                          (char *)ws_dev, tie_rel, grid, row_idx_dev, fp32c ? idx_dev : nullptr,
                          fp32c ? omin_dev : nullptr, lo, s);
    if (rc != OMEGA_OK || fp32c)
        return rc;
    ArgminArgs a;
    a.omega = grid;
    a.rowmin = (const double *)((const char *)ws_dev + P.off_rowmin);
    a.n_q = n_q;
    a.n_delta = n_delta;
    a.tie_rel = tie_rel;
    a.idx = idx_dev;
    a.omin = omin_dev;
    if (launch_argmin(a, n_pts * nb, s) != hipSuccess)
        return OMEGA_E_HIP;
    return OMEGA_OK;
}

// Workspace of a pair-susceptibility call: cos/sin and (three-band) band
// tables of the largest lattice, Q trig / lattice indices, chunk partials of
// one point.
struct ChiPlan {
    std::vector<Group> groups;
    std::vector<int> n_chunks, span;   // per group
    size_t off_trig, off_qtrig, off_etab, off_qlat, off_part, bytes;
};

ChiPlan plan_chi(const omega_point *pts, int n_pts, int n_q, int nb, bool b3)
{
    ChiPlan p;
    p.groups = group_points(pts, n_pts);
    const long long pairs_q = (long long)nb * nb * n_q;
    size_t trig = 0, etab = 0, part = 0;
    for (const Group &g : p.groups) {
        const long long n = (long long)g.Lx * g.Ly;
        long long nc = (kMinWorkgroups + pairs_q - 1) / pairs_q;
        const long long cap = std::min((n + 1023) / 1024, (long long)kMaxGridZ);
        nc = std::max(1LL, std::min(nc, cap));
        p.n_chunks.push_back((int)nc);
        p.span.push_back((int)((n + nc - 1) / nc));
        trig = std::max(trig, sizeof(double) * 2 * ((size_t)g.Lx + g.Ly));
        if (b3)
            etab = std::max(etab, sizeof(double) * 3 * (size_t)n);
        part = std::max(part, sizeof(double) * (size_t)(pairs_q * nc));
    }
    p.off_trig = 0;
    p.off_qtrig = align_up(trig);
    p.off_etab = p.off_qtrig + align_up(sizeof(double) * kQTrig * (size_t)n_q);
    p.off_qlat = p.off_etab + align_up(etab);
    p.off_part = p.off_qlat + (b3 ? align_up(sizeof(int) * 2 * (size_t)n_q) : 0);
    p.bytes = p.off_part + align_up(part);
    return p;
}

bool hoppings_ok(const omega_model *m)
{
    return m && isfinite(m->t1) && isfinite(m->t2) && isfinite(m->t3) && isfinite(m->t4) &&
           isfinite(m->mu);
}

int run_chi(const ModelDesc &md, const omega_point *pts, int n_pts, const double *q_dev,
            int n_q, void *ws_dev, size_t ws_bytes, double *chi_dev, void *stream)
{
    if (!q_dev || !ws_dev || !chi_dev)
        return OMEGA_E_INVAL;
    const ChiPlan P = plan_chi(pts, n_pts, n_q, md.nb, md.b3);
    if (ws_bytes < P.bytes)
        return OMEGA_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)ws_dev;
    double *trig = (double *)(ws + P.off_trig);
    double *qtrig = (double *)(ws + P.off_qtrig);
    double *etab = (double *)(ws + P.off_etab);
    int *qlat = (int *)(ws + P.off_qlat);
    double *part = (double *)(ws + P.off_part);
    if (launch_qtrig(q_dev, n_q, qtrig, s) != hipSuccess)
        return OMEGA_E_HIP;
    ChiArgs a;
    a.hop = md.hop;
    a.hop3 = md.hop3;
    for (int k = 0; k < 3; ++k) {
        const int b = md.list[k < md.nb ? k : 0];
        a.eps[k] = b ? 1.0 : -1.0;
        a.band3[k] = b;
    }
    a.nb = md.nb;
    a.mu = md.mu;
    a.n_q = n_q;
    a.trig = trig;
    a.qtrig = qtrig;
    a.etab = etab;
    a.qlat = qlat;
    a.part = part;
    const int pairs_q = md.nb * md.nb * n_q;
    for (size_t gi = 0; gi < P.groups.size(); ++gi) {
        const Group &g = P.groups[gi];
        if (launch_trig(g.Lx, g.Ly, trig, s) != hipSuccess)
            return OMEGA_E_HIP;
        if (md.b3 && (launch_etab(md.hop3, trig, g.Lx, g.Ly, etab, s) != hipSuccess ||
                      launch_qlat(q_dev, n_q, g.Lx, g.Ly, qlat, s) != hipSuccess))
            return OMEGA_E_HIP;
        a.Lx = g.Lx;
        a.Ly = g.Ly;
        a.n_chunks = P.n_chunks[gi];
        a.span = P.span[gi];
        for (int idx : g.idx) {
            a.h = pts[idx].h;
            a.T = pts[idx].T;
            if (launch_chi(a, md.b3, s) != hipSuccess)
                return OMEGA_E_HIP;
            ChiFinishArgs f;
            f.part = part;
            f.n_pairs_q = pairs_q;
            f.n_chunks = a.n_chunks;
            f.inv_n = 1.0 / ((double)g.Lx * g.Ly);
            f.out = chi_dev + (size_t)idx * pairs_q;
            if (launch_chi_finish(f, s) != hipSuccess)
                return OMEGA_E_HIP;
        }
    }
    return OMEGA_OK;
}

// Sector and cycle structure of the LO problem of one point and one pair
// momentum (m, n) on a lattice axis (see LoArgs); false if q is off the axes
// or a cycle exceeds kLoMaxCycle modes.
struct LoShape {
    int along_y, Lc, Ls, s, g, n;
    double w;   // sum_j |e^{iqR_j} + e^{-iqR_j}|^2 / N
};

int gcd_int(int a, int b)
{
    while (b) {
        const int t = a % b;
        a = b;
        b = t;
    }
    return a;
}

bool lo_shape(const omega_point &pt, int m, int n, LoShape *o)
{
    if (m != 0 && n != 0)
        return false;
    LoShape r;
    r.along_y = m == 0;
    r.Lc = r.along_y ? pt.Ly : pt.Lx;
    r.Ls = r.along_y ? pt.Lx : pt.Ly;
    const long long idx = r.along_y ? n : m;
    r.s = (int)(((idx % r.Lc) + r.Lc) % r.Lc);
    const int two_s = (int)((2LL * r.s) % r.Lc);
    r.g = two_s == 0 ? r.Lc : gcd_int(two_s, r.Lc);
    r.n = 2 * r.Lc / r.g;
    // the two waves coincide where 2q is a reciprocal lattice vector
    r.w = two_s == 0 ? 4.0 : 2.0;
    if (r.n > kLoMaxCycle || (long long)r.Ls * r.g > 0x7fffffffLL)
        return false;
    *o = r;
    return true;
}

size_t lo_bytes(const omega_point *pts, int n_pts, int n_delta, const int32_t *q, int n_q,
                int nb)
{
    size_t part = 0;
    for (int p = 0; p < n_pts; ++p)
        for (int iq = 0; iq < n_q; ++iq) {
            LoShape sh;
            if (!lo_shape(pts[p], q[2 * iq], q[2 * iq + 1], &sh))
                return 0;
            part = std::max(part, sizeof(double) * (size_t)nb * n_delta * sh.Ls * sh.g);
        }
    return align_up(part);
}

// Scratch of omega_argmin_noalloc: one statically allocated array per
// device (each device that runs the library holds its own copy until the
// process ends).  In host code `scratch` names a host-side stand-in, not the
// device array; its device address is taken once per device with
// hipGetSymbolAddress and only that address is passed to the kernels.
constexpr size_t kScratchBytes = (size_t)OMEGA_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % kAlign == 0, "scratch size keeps the workspace alignment");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 256;
std::mutex g_scratch_mutex;
void *g_scratch_dev[kMaxDevices];

// Device address of the current device's scratch array; taken on the first
// call on that device, with the device current.
int scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return OMEGA_E_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return OMEGA_E_HIP;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return OMEGA_OK;
}

}  // namespace

extern "C" {

size_t omega_workspace_bytes(const omega_point *pts, int n_pts, int n_delta,
                             int n_q, int bands, int precision, int grad)
{
    if (!points_ok(pts, n_pts) || bands < 1 || bands > 3)
        return 0;
    const int nb = n_bands(bands);
    if (grad)
        return plan_grad(pts, n_pts, nb).bytes;
    if (!sizes_ok(n_delta, n_q, bands, precision))
        return 0;
    return plan_grid(pts, n_pts, n_delta, n_q, nb, false).sweep_bytes +
           grid_bytes(n_pts, n_delta, n_q, nb);
}

int omega_grid(const omega_model *model, const omega_point *pts, int n_pts,
               const double *delta_dev, int n_delta, const double *q_dev,
               int n_q, int bands, int precision, void *ws_dev,
               size_t ws_bytes, double *omega_dev, void *stream)
{
    if (!model_ok(model) || !points_ok(pts, n_pts) ||
        !sizes_ok(n_delta, n_q, bands, precision))
        return OMEGA_E_INVAL;
    return run_grid(describe(model, bands), pts, n_pts, delta_dev, n_delta, q_dev, n_q,
                    precision, ws_dev, ws_bytes, omega_dev, stream);
}

int omega_argmin(const omega_model *model, const omega_point *pts, int n_pts,
                 const double *delta_dev, int n_delta, const double *q_dev,
                 int n_q, int bands, int precision, double tie_rel,
                 void *ws_dev, size_t ws_bytes, int32_t *idx_dev,
                 double *omin_dev, int32_t *row_idx_dev, double *omega_dev,
                 void *stream)
{
    return omega_argmin_ex(model, pts, n_pts, delta_dev, n_delta, q_dev, n_q, bands, precision,
                           tie_rel, ws_dev, ws_bytes, idx_dev, omin_dev, row_idx_dev, omega_dev,
                           nullptr, stream);
}

int omega_argmin_ex(const omega_model *model, const omega_point *pts, int n_pts,
                    const double *delta_dev, int n_delta, const double *q_dev, int n_q,
                    int bands, int precision, double tie_rel, void *ws_dev, size_t ws_bytes,
                    int32_t *idx_dev, double *omin_dev, int32_t *row_idx_dev,
                    double *omega_dev, const omega_launch *launch, void *stream)
{
    Launch lo;
    if (!model_ok(model) || !points_ok(pts, n_pts) ||
        !sizes_ok(n_delta, n_q, bands, precision) || !resolve_launch(launch, &lo))
        return OMEGA_E_INVAL;
    return run_argmin(describe(model, bands), pts, n_pts, delta_dev, n_delta, q_dev, n_q,
                      precision, tie_rel, ws_dev, ws_bytes, idx_dev, omin_dev, row_idx_dev,
                      omega_dev, lo, stream);
}

int omega_argmin_noalloc(const omega_model *model, const omega_point *pts, int n_pts,
                         const double *delta_dev, int n_delta, const double *q_dev, int n_q,
                         int bands, int precision, double tie_rel, int32_t *idx_dev,
                         double *omin_dev, int32_t *row_idx_dev, double *omega_dev,
                         void *stream)
{
    if (!model_ok(model) || !points_ok(pts, n_pts) || !sizes_ok(n_delta, n_q, bands, precision))
        return OMEGA_E_INVAL;
    const int nb = n_bands(bands);
    const size_t need = plan_grid(pts, n_pts, n_delta, n_q, nb, false).sweep_bytes +
                        (omega_dev ? 0 : grid_bytes(n_pts, n_delta, n_q, nb));
    if (need > kScratchBytes)
        return OMEGA_E_WORKSPACE;
    void *ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc != OMEGA_OK)
        return rc;
    return run_argmin(describe(model, bands), pts, n_pts, delta_dev, n_delta, q_dev, n_q,
                      precision, tie_rel, ws, kScratchBytes, idx_dev, omin_dev, row_idx_dev,
                      omega_dev, Launch(), stream);
}

size_t omega_lo_workspace_bytes(const omega_point *pts, int n_pts, int n_delta,
                                const int32_t *q_host, int n_q, int bands)
{
    if (!points_ok(pts, n_pts) || !q_host || n_q <= 0 || n_q > kMaxQ || n_delta <= 0 ||
        n_delta > kMaxDelta || bands < 1 || bands > 3)
        return 0;
    return lo_bytes(pts, n_pts, n_delta, q_host, n_q, n_bands(bands));
}

int omega_lo_grid(const omega_model *model, const omega_point *pts, int n_pts,
                  const double *delta_dev, int n_delta, const int32_t *q_host, int n_q,
                  int bands, void *ws_dev, size_t ws_bytes, double *omega_dev, void *stream)
{
    if (!model_ok(model) || !points_ok(pts, n_pts) || !q_host || n_q <= 0 || n_q > kMaxQ ||
        n_delta <= 0 || n_delta > kMaxDelta || bands < 1 || bands > 3 || !delta_dev ||
        !omega_dev || !ws_dev)
        return OMEGA_E_INVAL;
    if (model->form != OMEGA_ETA_K)
        return OMEGA_E_UNSUPPORTED;
    int list[2];
    const int nb = slot_bands(bands, list);
    const size_t need = lo_bytes(pts, n_pts, n_delta, q_host, n_q, nb);
    if (need == 0)
        return OMEGA_E_UNSUPPORTED;   // q off the axes, or a cycle above kLoMaxCycle
    if (ws_bytes < need)
        return OMEGA_E_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    LoArgs a;
    a.hop = make_hop(model);
    band_signs(nb, list, a.eps);
    a.mu = model->mu;
    a.n_delta = n_delta;
    a.delta = delta_dev;
    a.part = (double *)ws_dev;
    LoFinishArgs f;
    f.part = a.part;
    f.delta = delta_dev;
    f.n_delta = n_delta;
    f.nb = nb;
    f.Vs[0] = model->V[list[0]];
    f.Vs[1] = model->V[nb > 1 ? list[1] : list[0]];
    f.slot_stride = (size_t)n_q * n_delta;
    for (int p = 0; p < n_pts; ++p) {
        a.h = pts[p].h;
        a.T = pts[p].T;
        a.Lx = pts[p].Lx;
        a.Ly = pts[p].Ly;
        for (int iq = 0; iq < n_q; ++iq) {
            LoShape sh;
            lo_shape(pts[p], q_host[2 * iq], q_host[2 * iq + 1], &sh);
            a.along_y = sh.along_y;
            a.Lc = sh.Lc;
            a.Ls = sh.Ls;
            a.s = sh.s;
            a.g = sh.g;
            a.n = sh.n;
            if (launch_lo(a, nb, st) != hipSuccess)
                return OMEGA_E_HIP;
            f.n_parts = sh.Ls * sh.g;
            f.n_k = (double)pts[p].Lx * pts[p].Ly;
            f.w = sh.w;
            f.omega = omega_dev + ((size_t)p * nb * n_q + iq) * n_delta;
            if (launch_lo_finish(f, st) != hipSuccess)
                return OMEGA_E_HIP;
        }
    }
    return OMEGA_OK;
}

int omega3_bands(const omega3_model *model, int Lx, int Ly, void *ws_dev, size_t ws_bytes,
                 double *E_dev, void *stream)
{
    if (!model3_ok(model, 0) || !E_dev || !ws_dev)
        return OMEGA_E_INVAL;
    const omega_point p{0.0, 0.0, Lx, Ly};
    if (!point_ok(p))
        return OMEGA_E_INVAL;
    if (ws_bytes < sizeof(double) * 2 * ((size_t)Lx + Ly))
        return OMEGA_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    double *trig = (double *)ws_dev;
    if (launch_trig(Lx, Ly, trig, s) != hipSuccess)
        return OMEGA_E_HIP;
    if (launch_etab(describe3(model, 0).hop3, trig, Lx, Ly, E_dev, s) != hipSuccess)
        return OMEGA_E_HIP;
    return OMEGA_OK;
}

size_t omega3_workspace_bytes(const omega_point *pts, int n_pts, int n_delta, int n_q,
                              int bands, int precision)
{
    if (!points_ok(pts, n_pts) || bands < 1 || bands > 7)
        return 0;
    if (!sizes_ok(n_delta, n_q, 1, precision))
        return 0;
    int list[3];
    const int nb = slot_bands3(bands, list);
    return plan_grid(pts, n_pts, n_delta, n_q, nb, true).sweep_bytes +
           grid_bytes(n_pts, n_delta, n_q, nb);
}

int omega3_grid(const omega3_model *model, const omega_point *pts, int n_pts,
                const double *delta_dev, int n_delta, const double *q_dev, int n_q,
                int bands, int precision, void *ws_dev, size_t ws_bytes,
                double *omega_dev, void *stream)
{
    if (bands < 1 || bands > 7 || !model3_ok(model, bands) || !points_ok(pts, n_pts) ||
        !sizes_ok(n_delta, n_q, 1, precision))
        return OMEGA_E_INVAL;
    return run_grid(describe3(model, bands), pts, n_pts, delta_dev, n_delta, q_dev, n_q,
                    precision, ws_dev, ws_bytes, omega_dev, stream);
}

int omega3_argmin(const omega3_model *model, const omega_point *pts, int n_pts,
                  const double *delta_dev, int n_delta, const double *q_dev, int n_q,
                  int bands, int precision, double tie_rel, void *ws_dev,
                  size_t ws_bytes, int32_t *idx_dev, double *omin_dev,
                  int32_t *row_idx_dev, double *omega_dev, void *stream)
{
    return omega3_argmin_ex(model, pts, n_pts, delta_dev, n_delta, q_dev, n_q, bands,
                            precision, tie_rel, ws_dev, ws_bytes, idx_dev, omin_dev,
                            row_idx_dev, omega_dev, nullptr, stream);
}

int omega3_argmin_ex(const omega3_model *model, const omega_point *pts, int n_pts,
                     const double *delta_dev, int n_delta, const double *q_dev, int n_q,
                     int bands, int precision, double tie_rel, void *ws_dev,
                     size_t ws_bytes, int32_t *idx_dev, double *omin_dev,
                     int32_t *row_idx_dev, double *omega_dev, const omega_launch *launch,
                     void *stream)
{
    Launch lo;
    if (bands < 1 || bands > 7 || !model3_ok(model, bands) || !points_ok(pts, n_pts) ||
        !sizes_ok(n_delta, n_q, 1, precision) || !resolve_launch(launch, &lo))
        return OMEGA_E_INVAL;
    return run_argmin(describe3(model, bands), pts, n_pts, delta_dev, n_delta, q_dev, n_q,
                      precision, tie_rel, ws_dev, ws_bytes, idx_dev, omin_dev, row_idx_dev,
                      omega_dev, lo, stream);
}

int omega_grad(const omega_model *model, const omega_point *pts, int n_pts,
               const double *delta_dev, const double *q_dev, int bands,
               void *ws_dev, size_t ws_bytes, double *omega_dev,
               double *dDelta_dev, double *dq_dev, double *dmu_dev,
               void *stream)
{
    if (!model_ok(model) || !points_ok(pts, n_pts) || bands < 1 || bands > 3)
        return OMEGA_E_INVAL;
    if (!delta_dev || !q_dev || !ws_dev || !omega_dev || !dDelta_dev || !dq_dev ||
        !dmu_dev)
        return OMEGA_E_INVAL;
    int list[2];
    const int nb = slot_bands(bands, list);
    const GradPlan P = plan_grad(pts, n_pts, nb);
    if (ws_bytes < P.bytes)
        return OMEGA_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)ws_dev;
    double *qtrig = (double *)(ws + P.off_qtrig);
    double *trig = (double *)(ws + P.off_trig);
    PointRec *table = (PointRec *)(ws + P.off_table);
    double *part = (double *)(ws + P.off_part);
    if (launch_qtrig(q_dev, n_pts * nb, qtrig, s) != hipSuccess)
        return OMEGA_E_HIP;

    GradArgs a;
    a.hop = make_hop(model);
    band_signs(nb, list, a.eps);
    a.mu = model->mu;
    a.pts = table;
    a.nb = nb;
    a.delta = delta_dev;
    a.q = q_dev;
    a.qtrig = qtrig;
    a.eta_rel = model->form == OMEGA_ETA_REL;
    a.trig = trig;
    a.part = part;
    GradFinishArgs f;
    f.part = part;
    f.pts = table;
    f.delta = delta_dev;
    f.Vs[0] = model->V[list[0]];
    f.Vs[1] = model->V[nb > 1 ? list[1] : list[0]];
    f.nb = nb;
    f.omega = omega_dev;
    f.dDelta = dDelta_dev;
    f.dq = dq_dev;
    f.dmu = dmu_dev;
    for (size_t gi = 0; gi < P.groups.size(); ++gi) {
        const Group &g = P.groups[gi];
        const Tiles &t = P.tiles[gi];
        if (launch_trig(g.Lx, g.Ly, trig, s) != hipSuccess)
            return OMEGA_E_HIP;
        a.Lx = g.Lx;
        a.Ly = g.Ly;
        a.TX = t.TX;
        a.TY = t.TY;
        a.n_tiles = t.n_tiles;
        a.n_chunks = t.n_chunks;
        f.n_k = (double)g.Lx * g.Ly;
        f.n_chunks = t.n_chunks;
        const int n = (int)g.idx.size();
        for (int b0 = 0; b0 < n; b0 += P.batch[gi]) {
            const int G = n - b0 < P.batch[gi] ? n - b0 : P.batch[gi];
            int rc = upload_points(pts, g.idx.data() + b0, G, table, nullptr, s);
            if (rc != OMEGA_OK)
                return rc;
            if (launch_grad(a, G, s) != hipSuccess)
                return OMEGA_E_HIP;
            if (launch_grad_finish(f, G, s) != hipSuccess)
                return OMEGA_E_HIP;
        }
    }
    return OMEGA_OK;
}

size_t omega_chi_workspace_bytes(const omega_point *pts, int n_pts, int n_q, int bands)
{
    if (!points_ok(pts, n_pts) || bands < 1 || bands > 3 || n_q <= 0 || n_q > kMaxQ)
        return 0;
    int list[2];
    return plan_chi(pts, n_pts, n_q, slot_bands(bands, list), false).bytes;
}

int omega_pair_chi(const omega_model *model, const omega_point *pts, int n_pts,
                   const double *q_dev, int n_q, int bands, void *ws_dev, size_t ws_bytes,
                   double *chi_dev, void *stream)
{
    if (!hoppings_ok(model) || !points_ok(pts, n_pts) || bands < 1 || bands > 3 ||
        n_q <= 0 || n_q > kMaxQ)
        return OMEGA_E_INVAL;
    ModelDesc md{};
    md.b3 = false;
    md.nb = slot_bands(bands, md.list);
    md.mu = model->mu;
    md.hop = make_hop(model);
    return run_chi(md, pts, n_pts, q_dev, n_q, ws_dev, ws_bytes, chi_dev, stream);
}

size_t omega3_chi_workspace_bytes(const omega_point *pts, int n_pts, int n_q, int bands)
{
    if (!points_ok(pts, n_pts) || bands < 1 || bands > 7 || n_q <= 0 || n_q > kMaxQ)
        return 0;
    int list[3];
    return plan_chi(pts, n_pts, n_q, slot_bands3(bands, list), true).bytes;
}

int omega3_pair_chi(const omega3_model *model, const omega_point *pts, int n_pts,
                    const double *q_dev, int n_q, int bands, void *ws_dev, size_t ws_bytes,
                    double *chi_dev, void *stream)
{
    if (!model3_ok(model, 0) || !points_ok(pts, n_pts) || bands < 1 || bands > 7 ||
        n_q <= 0 || n_q > kMaxQ)
        return OMEGA_E_INVAL;
    return run_chi(describe3(model, bands), pts, n_pts, q_dev, n_q, ws_dev, ws_bytes, chi_dev,
                   stream);
}

int omega_q_wedge(int Lx, int Ly, double *q_host, int32_t *orbit_host, int capacity)
{
    const omega_point p{0.0, 0.0, Lx, Ly};
    if (!point_ok(p) || (q_host && (!orbit_host || capacity < 0)))
        return OMEGA_E_INVAL;
    const bool square = Lx == Ly;
    int count = 0;
    for (int m = 0; m <= Lx / 2; ++m) {
        for (int n = 0; n <= Ly / 2; ++n) {
            if (square && n > m)
                break;
            if (q_host) {
                if (count >= capacity)
                    return OMEGA_E_WORKSPACE;
                // orbit of (m, n) under the mirrors (and the swap on a square
                // lattice), as distinct zone indices
                int seen[8][2];
                int ns = 0;
                for (int g = 0; g < (square ? 8 : 4); ++g) {
                    int a = (g & 1) ? Lx - m : m;
                    int b = (g & 2) ? Ly - n : n;
                    a %= Lx;
                    b %= Ly;
                    if (g & 4) {
                        const int t = a;
                        a = b;
                        b = t;
                    }
                    bool dup = false;
                    for (int k = 0; k < ns; ++k)
                        dup = dup || (seen[k][0] == a && seen[k][1] == b);
                    if (!dup) {
                        seen[ns][0] = a;
                        seen[ns][1] = b;
                        ++ns;
                    }
                }
                q_host[2 * count] = 2.0 * M_PI * m / Lx;
                q_host[2 * count + 1] = 2.0 * M_PI * n / Ly;
                orbit_host[count] = ns;
            }
            ++count;
        }
    }
    return count;
}

const char *omega_strerror(int code)
{
    switch (code) {
    case OMEGA_OK:
        return "success";
    case OMEGA_E_INVAL:
        return "invalid argument";
    case OMEGA_E_WORKSPACE:
        return "workspace too small";
    case OMEGA_E_HIP:
        return "HIP runtime error";
    case OMEGA_E_UNSUPPORTED:
        return "unsupported request";
    default:
        return "unknown error code";
    }
}

int omega_version(void) { return 4; }

}  // extern "C"
