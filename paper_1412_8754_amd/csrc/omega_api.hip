// C entry points of libomega (declared in include/omega.h): host-side
// validation, workspace layout and the launch sequence of each call.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include "omega.h"
#include "omega_internal.h"

namespace {

using namespace omega;

constexpr size_t kAlign = 256;
constexpr int kMaxL = 16384;
constexpr long long kMaxK = 1LL << 26;
constexpr int kMaxDelta = 1 << 20;
constexpr int kMaxQ = 16384;
constexpr int kMinWorkgroups = 4096;   // below this the chunks are split finer

hipEvent_t g_sweep_start = nullptr;   // benchmark hook, see omega_set_sweep_events
hipEvent_t g_sweep_stop = nullptr;

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

bool model_ok(const omega_model *m)
{
    if (!m)
        return false;
    const double v[7] = {m->t1, m->t2, m->t3, m->t4, m->mu, m->V[0], m->V[1]};
    for (double x : v)
        if (!isfinite(x))
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
    if (!pts || n_pts <= 0)
        return false;
    for (int i = 0; i < n_pts; ++i)
        if (!point_ok(pts[i]))
            return false;
    return true;
}

int delta_tile(int n_delta) { return n_delta >= 32 ? 32 : 16; }

struct Plan {
    int TX, TY, n_tiles, tiles_per_wg, n_chunks;
};

Plan plan_tiles(int Lx, int Ly, long long other_blocks)
{
    Plan r;
    r.TX = (Lx + kTileEdge - 1) / kTileEdge;
    r.TY = (Ly + kTileEdge - 1) / kTileEdge;
    r.n_tiles = r.TX * r.TY;
    int tpw = 64;
    while (tpw > 4 &&
           (long long)((r.n_tiles + tpw - 1) / tpw) * other_blocks < kMinWorkgroups)
        tpw /= 2;
    r.tiles_per_wg = tpw;
    r.n_chunks = (r.n_tiles + tpw - 1) / tpw;
    return r;
}

// Per-point scratch of the sweep: trig tables, Delta^2, chunk partials.
struct SweepLayout {
    size_t trig, d2, part, base, total;
};

SweepLayout sweep_layout(const omega_point &p, int n_delta, int n_q, int nb)
{
    const int td = delta_tile(n_delta);
    const int n_dtiles = (n_delta + td - 1) / td;
    const int n_delta_pad = n_dtiles * td;
    const Plan pl = plan_tiles(p.Lx, p.Ly, (long long)n_dtiles * nb * n_q);
    SweepLayout l;
    l.trig = 0;
    l.d2 = l.trig + align_up(sizeof(double) * 2 * ((size_t)p.Lx + p.Ly));
    l.part = l.d2 + align_up(sizeof(double) * n_delta_pad);
    l.base = l.part +
             align_up(sizeof(double) * (size_t)nb * n_q * pl.n_chunks * n_delta_pad);
    l.total = l.base + align_up(sizeof(double) * (size_t)nb * n_q * pl.n_chunks);
    return l;
}

size_t sweep_bytes(const omega_point *pts, int n_pts, int n_delta, int n_q, int nb)
{
    size_t mx = 0;
    for (int i = 0; i < n_pts; ++i) {
        size_t b = sweep_layout(pts[i], n_delta, n_q, nb).total;
        mx = b > mx ? b : mx;
    }
    return mx;
}

size_t grid_bytes(int n_pts, int n_delta, int n_q, int nb)
{
    return align_up(sizeof(double) * (size_t)n_pts * nb * n_q * n_delta);
}

Plan grad_plan(const omega_point &p, int nb)
{
    return plan_tiles(p.Lx, p.Ly, nb);
}

size_t grad_bytes(const omega_point *pts, int n_pts, int nb)
{
    size_t mx = 0;
    for (int i = 0; i < n_pts; ++i) {
        const Plan pl = grad_plan(pts[i], nb);
        size_t b = align_up(sizeof(double) * 2 * ((size_t)pts[i].Lx + pts[i].Ly)) +
                   align_up(sizeof(double) * 5 * (size_t)nb * pl.n_chunks);
        mx = b > mx ? b : mx;
    }
    return mx;
}

bool sizes_ok(int n_delta, int n_q, int bands, int precision)
{
    return n_delta > 0 && n_delta <= kMaxDelta && n_q > 0 && n_q <= kMaxQ &&
           bands >= 1 && bands <= 3 &&
           (precision == OMEGA_FP64 || precision == OMEGA_FP32_COMP);
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

// Enqueue the sweep and row reduction of every point.  Omega goes to `grid`,
// row minima to row_idx (optional).
int enqueue_grid(const omega_model *m, const omega_point *pts, int n_pts,
                 const double *delta, int n_delta, const double *q, int n_q,
                 int bands, int precision, char *ws, double tie_rel,
                 double *grid, int32_t *row_idx, hipStream_t s)
{
    int list[2];
    const int nb = slot_bands(bands, list);
    const int td = delta_tile(n_delta);
    const int n_dtiles = (n_delta + td - 1) / td;
    const int n_delta_pad = n_dtiles * td;
    const int nbq = nb * n_q;
    for (int p = 0; p < n_pts; ++p) {
        const omega_point &pt = pts[p];
        const SweepLayout l = sweep_layout(pt, n_delta, n_q, nb);
        const Plan pl = plan_tiles(pt.Lx, pt.Ly, (long long)n_dtiles * nbq);
        double *trig = (double *)(ws + l.trig);
        double *d2 = (double *)(ws + l.d2);
        double *part = (double *)(ws + l.part);
        double *base = (double *)(ws + l.base);
        if (launch_prep(pt.Lx, pt.Ly, trig, delta, n_delta, n_delta_pad, d2, s) !=
            hipSuccess)
            return OMEGA_E_HIP;

        SweepArgs a;
        a.hop = make_hop(m);
        a.eps[0] = list[0] ? 1.0 : -1.0;
        a.eps[1] = nb > 1 ? (list[1] ? 1.0 : -1.0) : a.eps[0];
        a.mu_up = m->mu + pt.h;
        a.mu_dn = m->mu - pt.h;
        a.T = pt.T;
        a.invT = pt.T > 0.0 ? 1.0 / pt.T : 0.0;
        a.cutT = kCutFp64 * pt.T;
        a.Tf = (float)pt.T;
        a.invTf = pt.T > 0.0 ? (float)(1.0 / pt.T) : 0.0f;
        a.cutTf = kCutFp32 * (float)pt.T;
        a.Lx = pt.Lx;
        a.Ly = pt.Ly;
        a.TX = pl.TX;
        a.TY = pl.TY;
        a.n_tiles = pl.n_tiles;
        a.n_chunks = pl.n_chunks;
        a.n_q = n_q;
        a.n_delta_pad = n_delta_pad;
        a.d2 = d2;
        a.q = q;
        a.trig = trig;
        a.part = part;
        a.base_part = base;
        if (g_sweep_start && hipEventRecord(g_sweep_start, s) != hipSuccess)
            return OMEGA_E_HIP;
        hipError_t e = precision == OMEGA_FP64
                           ? launch_sweep_f64(a, td, n_dtiles, nbq, s)
                           : launch_sweep_f32c(a, td, n_dtiles, nbq, s);
        if (e != hipSuccess)
            return OMEGA_E_HIP;
        if (g_sweep_stop && hipEventRecord(g_sweep_stop, s) != hipSuccess)
            return OMEGA_E_HIP;

        RowArgs r;
        r.part = part;
        r.base_part = base;
        r.delta = delta;
        r.q = q;
        r.Vs[0] = m->V[list[0]];
        r.Vs[1] = m->V[nb > 1 ? list[1] : list[0]];
        r.n_k = (double)pt.Lx * pt.Ly;
        r.tie_rel = tie_rel;
        r.n_chunks = pl.n_chunks;
        r.n_delta = n_delta;
        r.n_delta_pad = n_delta_pad;
        r.n_q = n_q;
        r.omega = grid + (size_t)p * nbq * n_delta;
        r.row_idx = row_idx ? row_idx + (size_t)p * nbq : nullptr;
        if (launch_rows(r, nbq, s) != hipSuccess)
            return OMEGA_E_HIP;
    }
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
        return grad_bytes(pts, n_pts, nb);
    if (!sizes_ok(n_delta, n_q, bands, precision))
        return 0;
    return sweep_bytes(pts, n_pts, n_delta, n_q, nb) +
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
    if (!delta_dev || !q_dev || !omega_dev || !ws_dev)
        return OMEGA_E_INVAL;
    const int nb = n_bands(bands);
    if (ws_bytes < sweep_bytes(pts, n_pts, n_delta, n_q, nb))
        return OMEGA_E_WORKSPACE;
    return enqueue_grid(model, pts, n_pts, delta_dev, n_delta, q_dev, n_q, bands,
                        precision, (char *)ws_dev, 0.0, omega_dev, nullptr,
                        (hipStream_t)stream);
}

int omega_argmin(const omega_model *model, const omega_point *pts, int n_pts,
                 const double *delta_dev, int n_delta, const double *q_dev,
                 int n_q, int bands, int precision, double tie_rel,
                 void *ws_dev, size_t ws_bytes, int32_t *idx_dev,
                 double *omin_dev, int32_t *row_idx_dev, double *omega_dev,
                 void *stream)
{
    if (!model_ok(model) || !points_ok(pts, n_pts) ||
        !sizes_ok(n_delta, n_q, bands, precision))
        return OMEGA_E_INVAL;
    if (!delta_dev || !q_dev || !idx_dev || !omin_dev || !ws_dev)
        return OMEGA_E_INVAL;
    if (!(tie_rel >= 0.0) || !isfinite(tie_rel))
        return OMEGA_E_INVAL;
    const int nb = n_bands(bands);
    const size_t sweep = sweep_bytes(pts, n_pts, n_delta, n_q, nb);
    const size_t need = sweep + (omega_dev ? 0 : grid_bytes(n_pts, n_delta, n_q, nb));
    if (ws_bytes < need)
        return OMEGA_E_WORKSPACE;
    double *grid = omega_dev ? omega_dev : (double *)((char *)ws_dev + sweep);
    hipStream_t s = (hipStream_t)stream;
    int rc = enqueue_grid(model, pts, n_pts, delta_dev, n_delta, q_dev, n_q, bands,
                          precision, (char *)ws_dev, tie_rel, grid, row_idx_dev, s);
    if (rc != OMEGA_OK)
        return rc;
    ArgminArgs a;
    a.omega = grid;
    a.n_q = n_q;
    a.n_delta = n_delta;
    a.tie_rel = tie_rel;
    a.idx = idx_dev;
    a.omin = omin_dev;
    if (launch_argmin(a, n_pts * nb, s) != hipSuccess)
        return OMEGA_E_HIP;
    return OMEGA_OK;
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
    if (ws_bytes < grad_bytes(pts, n_pts, nb))
        return OMEGA_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)ws_dev;
    for (int p = 0; p < n_pts; ++p) {
        const omega_point &pt = pts[p];
        const Plan pl = grad_plan(pt, nb);
        double *trig = (double *)ws;
        double *part =
            (double *)(ws + align_up(sizeof(double) * 2 * ((size_t)pt.Lx + pt.Ly)));
        if (launch_prep(pt.Lx, pt.Ly, trig, delta_dev, 1, 0, nullptr, s) != hipSuccess)
            return OMEGA_E_HIP;
        GradArgs a;
        a.hop = make_hop(model);
        a.eps[0] = list[0] ? 1.0 : -1.0;
        a.eps[1] = nb > 1 ? (list[1] ? 1.0 : -1.0) : a.eps[0];
        a.mu_up = model->mu + pt.h;
        a.mu_dn = model->mu - pt.h;
        a.T = pt.T;
        a.invT = pt.T > 0.0 ? 1.0 / pt.T : 0.0;
        a.Lx = pt.Lx;
        a.Ly = pt.Ly;
        a.TY = pl.TY;
        a.n_tiles = pl.n_tiles;
        a.tiles_per_wg = pl.tiles_per_wg;
        a.n_chunks = pl.n_chunks;
        a.delta = delta_dev + (size_t)p * nb;
        a.q = q_dev + (size_t)p * nb * 2;
        a.trig = trig;
        a.part = part;
        if (launch_grad(a, nb, s) != hipSuccess)
            return OMEGA_E_HIP;
        GradFinishArgs f;
        f.part = part;
        f.delta = a.delta;
        f.Vs[0] = model->V[list[0]];
        f.Vs[1] = model->V[nb > 1 ? list[1] : list[0]];
        f.n_k = (double)pt.Lx * pt.Ly;
        f.n_chunks = pl.n_chunks;
        f.omega = omega_dev + (size_t)p * nb;
        f.dDelta = dDelta_dev + (size_t)p * nb;
        f.dq = dq_dev + (size_t)p * nb * 2;
        f.dmu = dmu_dev + (size_t)p * nb;
        if (launch_grad_finish(f, nb, s) != hipSuccess)
            return OMEGA_E_HIP;
    }
    return OMEGA_OK;
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

int omega_version(void) { return 1; }

int omega_set_sweep_events(void *start_event, void *stop_event)
{
    if ((start_event == nullptr) != (stop_event == nullptr))
        return OMEGA_E_INVAL;
    g_sweep_start = (hipEvent_t)start_event;
    g_sweep_stop = (hipEvent_t)stop_event;
    return OMEGA_OK;
}

}  // extern "C"
