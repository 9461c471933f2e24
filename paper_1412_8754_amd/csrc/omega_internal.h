// Internal declarations shared by the kernels and the C entry points of
// libomega.  Not installed; the public interface is include/omega.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace omega {

// Two-band energies of App. A, Eqs. (A.1)-(A.4), regrouped as
//   (T11 + T22)/2 = tA (cx + cy) + tB cx cy,  tA = -(t1 + t2), tB = -4 t3
//   (T11 - T22)/2 = tD (cx - cy),             tD = -(t1 - t2)
//   T12           = tC sx sy,                 tC = -4 t4
// and E_eps = (T11 + T22)/2 + eps sqrt(((T11 - T22)/2)^2 + T12^2).
struct Hop {
    double tA, tB, tD, tC;
};

// Three-band model of App. B: hoppings t1..t12 (t[0] = t1) and the d_xy
// on-site energy; bands are the eigenvalues of the 3x3 orbital matrix in
// ascending order, tabulated per lattice (Sec. 3.2: precomputed and stored).
struct Hop3 {
    double t[12];
    double eps0;
};

// Skip threshold of the thermal term of the grid sweeps: where |E|/T exceeds
// this, T ln(1 + exp(-|E|/T)) < T e^-30 = 9.4e-14 T and the term is dropped.
// Both branches of a momentum together move Omega by less than 1.9e-13 T
// per momentum, i.e. by 1.9e-13 T N at most, one-signed: below 3e-13 of the
// scale |Omega| >= 0.03 N of the E_+ band's rows (the smaller band) up to
// T = 0.05, inside the 1e-12 parity bar.
constexpr double kCutFp64 = 30.0;
// The gradient sweep keeps the Fermi function to 2.3e-16: it drops the
// thermal parts beyond 36 T.
constexpr double kCutGrad = 36.0;
// The FP32 loop of the FP32-compensated path drops T ln(1 + exp(-|E|/T))
// beyond 20 T: each branch then moves by less than T e^-20 = 2.1e-9 T,
// one-signed, so Omega by less than 4.2e-9 T N: below 7e-9 of
// |Omega| >= 0.03 N up to T = 0.05, well inside the stated 1e-7.  Its
// classification of terms (exactly zero / cold over a Delta tile or the
// whole Delta range / per-Delta loop) and its FP64 base term keep the FP64
// cut, so that Omega at Delta = 0 stays the FP64 value.
constexpr float kCutFp32 = 20.0f;
// From this temperature on, a point's marked terms run the per-Delta loop in
// place rather than being classified per Delta tile and queued (at higher T
// almost none is zero or on a tile series), in both precisions.
constexpr double kInPlaceT = 0.005;

// Table of the FP64 thermal term G(a) = ln(1 + e^-a), 0 <= a <= 30, at
// a0 = N / kGStep: the Taylor coefficients of G at a0 in the scaled variable
// r = kGStep (a - a0), |r| <= 1/2, c_n = G^(n)(a0) / (n! kGStep^n).  Two
// arrays of kGTabN double2 one behind the other: (c0, c1), then (c2, c3);
// c4 follows from c2 (see log1p_exp_tab).
constexpr int kGStep = 64;
constexpr int kGTabN = 30 * kGStep + 1;
constexpr int kGTabEntries = 2 * kGTabN;   // double2 entries of the table
static_assert(kCutFp64 == 30.0, "the thermal table ends at the FP64 cut");

// FP32 table of the same G for the FP32-compensated loop, 0 <= a <= 20 at
// a0 = N / kG32Step: float4 (c0, c1, c2, c3), c_n = G^(n)(a0) / (n! kG32Step^n)
// (rounded from FP64); degree 3 in r = kG32Step (a - a0), |r| <= 1/2, leaves
// at most |G''''| (1/64)^4 / 24 <= 2.5e-9 G (|G''''| <= p <= G).
constexpr int kG32Step = 32;
constexpr int kG32N = 20 * kG32Step + 1;
static_assert(kCutFp32 == 20.0f, "the FP32 thermal table ends at the FP32 cut");

// Series path of the sweep.  With x = Delta^2, the centre x0 and half-width
// hw of the call's Delta^2 range, R0 = sqrt(s^2 + x0 eta^2) and
// z = (x - x0) eta^2 / R0^2, the Delta-dependent term is
//   R - |d| = (R0 - |d|) + R0 sum_{n>=1} c_n z^n,  c_n = binomial(1/2, n).
// Where A0 = |s| - |d| >= 30 T (R - |d| >= 30 T for every Delta: cold,
// positive, no thermal part) and hw eta^2 <= kSeriesRho R0^2 (so |z| <= 1/3),
// it is summed over k through the moments C0 = sum (R0 - |d|) and
// M_n = sum R0 (eta^2/R0^2)^n, n = 1..kSeriesTerms.  Since |c_n| decreases,
// the truncation is below |c_32| 3^-32 / (1 - 1/3) = 1.3e-18 of R0 per term.
constexpr double kSeriesRho = 1.0 / 3.0;
constexpr int kSeriesTerms = 31;
constexpr int kMomentSlots = 32;   // C0, M_1..M_31

// A wave whose series terms all have a smaller ratio rho = hw eta^2 / R0^2
// needs fewer terms for the same bound: N terms suffice while
// |c_{N+1}| rho^{N+1} / (1 - rho) stays below the bound above.  The wave
// takes the smallest of the levels kSeriesLevel[] that covers all its lanes;
// series_level_rho(N) is the largest rho that N terms cover (by bisection).
// With the paper-scale workload a wave needs 7 terms on average.
constexpr int kSeriesLevels = 4;
constexpr int kSeriesLevel[kSeriesLevels] = {6, 10, 16, kSeriesTerms};

constexpr double abs_half_binomial(int n)
{
    double c = 1.0;
    for (int k = 1; k <= n; ++k)
        c *= (k - 1.5 < 0.0 ? 1.5 - k : k - 1.5) / k;
    return c;
}

constexpr double series_tail(int N, double rho)
{
    double p = 1.0;
    for (int k = 0; k <= N; ++k)
        p *= rho;
    return abs_half_binomial(N + 1) * p / (1.0 - rho);
}

constexpr double series_level_rho(int N)
{
    const double bound = series_tail(kSeriesTerms, kSeriesRho);
    double lo = 0.0, hi = kSeriesRho;
    for (int it = 0; it < 80; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (series_tail(N, mid) <= bound)
            lo = mid;
        else
            hi = mid;
    }
    return N >= kSeriesTerms ? kSeriesRho : lo;
}

struct SeriesLevelRho {
    double v[kSeriesLevels];
    constexpr SeriesLevelRho() : v()
    {
        for (int k = 0; k < kSeriesLevels; ++k)
            v[k] = series_level_rho(kSeriesLevel[k]);
    }
};

// Tile series of the queued sweep (both precisions; in the FP32-compensated
// one the moments are of (R - |d|) - P(0), C0 taking P(0) off).  Within one
// Delta tile (the TD Delta of a sweep unit; x = Delta^2 in [x_lo, x_hi],
// centre xc, half-width ht), a
// direct term that is cold and positive over the whole tile
// (R(x_lo) >= |d| + 30 T: R - |d| >= 30 T for every Delta of the tile, no
// thermal part) has R - |d| = (Rc - |d|) + Rc sum_{n>=1} c_n z^n with
// Rc^2 = s^2 + xc eta^2 and z = (x - xc) eta^2 / Rc^2.  Where
// u = ht eta^2 / Rc^2 <= kTileRho it is summed through kTileSlots moments per
// tile (C0 = sum w (Rc - |d|), M_n = sum w Rc (eta^2/Rc^2)^n, n <=
// kTileTerms); the truncation is below |c_16| u^16 / (1 - u) Rc, at most
// 6.7e-15 Rc.  With Rc = (ht eta^2 / u)^(1/2) that is at most
// (ht)^(1/2) |c_16| 0.18^15.5 / 0.82 = 3.2e-15 per term for Delta^2 tiles of
// half-width ht <= 0.042 (Delta up to 0.6 in 8 tiles), 1.1e-13 of the scale
// |Omega| >= 0.03 N.  Terms with R(x_hi) <= |d| - 30 T are exactly zero over
// the tile.
constexpr double kTileRho = 0.18;
constexpr int kTileTerms = 15;
constexpr int kTileSlots = 16;
constexpr int kTileBatch = 64;   // Delta tiles per LDS batch of the rows kernel

constexpr int kBlock = 256;      // threads per workgroup (4 wave64)

// Work queues of the persistent sweeps: kQueues counters by default (at most
// kMaxQueues, a launch option), each on its own 256-byte line (one counter
// sustains about 80 device-scope atomics per microsecond, eight on separate
// lines about 500).
constexpr int kQueues = 8;
constexpr int kMaxQueues = 16;
constexpr int kQueueStride = 32;   // unsigned long long
constexpr int kTileEdge = 8;     // k tile of one wavefront: 8 x 8 momenta
constexpr int kMaxChunkTiles = 256;   // k tiles of one sweep chunk, at most
// entries of one wave's list in the series pass (it visits every 4th tile)
constexpr int kMaxWaveList = kMaxChunkTiles / 4;

// Per-point record of a batch, written into the workspace by fill_points.
struct PointRec {
    double h, T;       // Zeeman field, temperature
    int32_t out;       // index of the point in the caller's arrays
    int32_t pad;
};

// Records travel to the device inside kernel arguments (no host copy, so a
// call stays capturable in a graph); kFillMax of them per fill launch.
constexpr int kFillMax = 128;
struct PointPack {
    int32_t n, pad;
    PointRec rec[kFillMax];
};

// Arguments of one Delta-sweep launch: a batch of G points of one lattice
// size.  series_kernel runs on the grid (chunk, band*Q + nbq*g); the sweeps
// take (chunk, Delta tile, band*Q + nbq*g) units from a work queue.
// Doubles per pair momentum in the Q trig table (see qtrig_at).
constexpr int kQTrig = 8;

struct SweepArgs {
    Hop hop;
    double eps[2];       // two-band: band sign per output slot (-1: E_-, +1: E_+)
    Hop3 hop3;           // three-band: model, for momenta off the lattice
    int band3[3];        // band index per output slot (0, 1 two-band; 0..2 three-band)
    const double *etab;  // E_b(k) over the lattice, [2 or 3][Lx][Ly]
    const int *qlat;     // [n_q][2] lattice index of Q, or -1 if off it
    double mu;           // chemical potential
    const PointRec *pts; // [G] this batch
    int Lx, Ly;
    int TX, TY;          // tiles along x and y (ceil(L / 8))
    int n_tiles;         // TX * TY
    int n_chunks;        // workgroups along the momentum axis per point
    int n_q;
    int nbq;             // bands * n_q
    int n_delta_pad;     // n_delta rounded up to the Delta tile
    const double *d2;    // [n_delta_pad + 2] Delta^2 (padding repeats the last),
                         // then centre and half-width of the Delta^2 range
    int eta_rel;         // 1: form factor at the pair's relative momentum, eta(k - Q/2)
    const double *q;     // [n_q][2]
    const double *qtrig; // [n_q][kQTrig] cos/sin of qx, qy, qx/2, qy/2
    const double *trig;  // cos kx [Lx], sin kx [Lx], cos ky [Ly], sin ky [Ly]
    const double2 *gtab; // [kGTabEntries] thermal table (FP64 sweeps; P(0) of the FP32-compensated series pass)
    const float4 *gtab32; // [kG32N] FP32 thermal table (FP32-compensated sweeps)
    double *part;        // [G*nbq][n_chunks][n_delta_pad] sums of Delta parts
    double *base_part;   // [G*nbq][n_chunks] sums of Delta-independent parts
    double *mpart;       // [G*nbq][n_chunks][kMomentSlots] series moments
    unsigned long long *tlist;   // [G*nbq][n_chunks][4 lcap][2] ((ti << 32) | tj, lane
                                 // mask) of the tiles with lanes evaluated per Delta,
                                 // listed by the series pass, first entries used
    int *tcnt;           // [G*nbq][n_chunks] list lengths
    double *tpart;       // [G*nbq][n_chunks][n_dtiles][kTileSlots] tile-series moments
    int n_dtiles;
    int lcap;            // list capacity per wave: ceil(ceil(n_tiles/n_chunks)/4)
    unsigned long long *count;   // optional: per-Delta terms evaluated directly
    unsigned long long *queue;   // work-queue counters of the persistent sweeps,
                                 // kMaxQueues of them kQueueStride apart
    int n_queues;        // queues in use (1 for a grid of fewer workgroups)
    int n_rows;          // G * nbq rows of this launch
    int blocks_per_cu;   // persistent grid: workgroups per CU (0: all that fit)
};

// Arguments of the per-row reduction / epilogue / row search: grid
// (band*Q, g) over a batch of G points.
struct RowArgs {
    const double *part;
    const double *base_part;
    const double *mpart;   // [G*nbq][n_chunks][kMomentSlots] series moments
    const double *d2c;     // centre of the Delta^2 range (series variable x - x0)
    const double *tpart;   // tile-series moments of the sweep
    int zero_d0;           // 1: the FP32-compensated sweep, whose Delta-dependent
                           // part vanishes at Delta = 0: the tile series is not
                           // added there
    const double *d2;      // [n_delta_pad] Delta^2 (tile centres)
    int td, n_dtiles;
    const PointRec *pts;   // [G]
    const double *delta;   // [n_delta]
    const double *q;       // [n_q][2]
    double Vs[3];          // V per output slot
    double n_k;            // Lx * Ly
    double tie_rel;
    int n_chunks, n_delta, n_delta_pad, n_q, nbq;
    double *omega;         // [n_pts][nbq][n_delta] (all points of the call)
    int32_t *row_idx;      // [n_pts][nbq], or nullptr
    double *rowmin;        // [n_pts][nbq] minimum of each row (NaN ignored)
};

struct ArgminArgs {
    const double *omega;   // [n_set][n_q][n_delta]
    const double *rowmin;  // [n_set][n_q] minimum of each row (rows_kernel)
    int n_q, n_delta;
    double tie_rel;
    int32_t *idx;          // [n_set][2]
    double *omin;          // [n_set]
};

// FP64 check of the FP32-compensated search ("scan in low precision, verify
// in double precision", Sec. 3.3).  Per (point, band) set of a batch, the
// cells whose FP32-compensated Omega lies within twice the stated FP32 error
// bound plus the tie band of the set's FP32 minimum are candidates for the
// FP64 minimum: kVerifyMax of them with Delta != 0 (the lowest-valued ones
// when there are more) are evaluated again in FP64, Delta = 0 cells are FP64
// in both sweeps already, and the tie rule picks among the checked cells by
// their FP64 values.  Grid pointers are indexed by output set.
constexpr int kVerifyMax = 32;
constexpr double kFp32RelBound = 1e-7;           // stated |dOmega| / |Omega| of the FP32 sweep
constexpr int kFp32FloorSites = 64 * 64;        // below this, plus 2^-20 N |Delta|

struct VerifyArgs {
    SweepArgs sw;          // model, lattice tables and points of the batch
    int nb, n_q, n_delta;
    const double *delta;   // [n_delta]
    const double *grid;    // [n_pts][nb][n_q][n_delta] FP32-compensated Omega
    const double *rowmin;  // [n_pts][nb][n_q]
    double tie_rel;
    const double *d2c;     // centre and half-width of the Delta^2 range (max Delta^2 =
                           // their sum), for the small-lattice floor 2^-20 N max|Delta|
    double Vs[3];
    double n_k;
    int n_vchunks;         // momentum chunks of one candidate's FP64 sum
    int *cand;             // [G*nb][kVerifyMax] cell index iq * n_delta + id
    int *cnt;              // [G*nb] candidates (Delta != 0)
    double *thr;           // [G*nb] candidate threshold
    double *vpart;         // [G*nb][kVerifyMax][n_vchunks] chunk sums
    int32_t *idx;          // [n_pts][nb][2]
    double *omin;          // [n_pts][nb]
};

hipError_t launch_verify(const VerifyArgs &v, int G, bool b3, hipStream_t s);

// Gradient sweep over a batch of G points of one lattice size: grid
// (chunk, band slot, g); one (Delta, Q) per point and slot.
struct GradArgs {
    Hop hop;
    double eps[2];
    double mu;
    const PointRec *pts;   // [G]
    int Lx, Ly, TX, TY, n_tiles, n_chunks, nb;
    const double *delta;   // [n_pts][nb] (all points of the call)
    const double *q;       // [n_pts][nb][2]
    const double *qtrig;   // [n_pts][nb][kQTrig] cos/sin of q and q/2
    int eta_rel;           // form factor eta(k - q/2)
    const double *trig;
    double *part;          // [G][nb][n_chunks][5]
};

struct GradFinishArgs {
    const double *part;
    const PointRec *pts;
    const double *delta;
    double Vs[2];
    double n_k;
    int n_chunks, nb;
    double *omega, *dDelta, *dq, *dmu;   // [n_pts][nb] ([n_pts][nb][2])
};

// Static Cooper-pair susceptibility (App. C) of one point: grid
// (band pair * n_q, chunk); part[(pair * n_q + iq) * n_chunks + chunk].
struct ChiArgs {
    Hop hop;
    Hop3 hop3;
    double eps[3];        // two-band: band sign per selected band
    int band3[3];         // three-band: band index per selected band
    int nb;
    double mu, h, T;
    int Lx, Ly;
    int n_q, n_chunks, span;   // span: momenta per chunk
    const double *trig;
    const double *qtrig;  // [n_q][kQTrig]
    const double *etab;   // three-band table [3][Lx][Ly]
    const int *qlat;      // three-band: lattice index of q, or -1
    double *part;
};

struct ChiFinishArgs {
    const double *part;
    int n_pairs_q, n_chunks;
    double inv_n;
    double *out;          // [nb * nb * n_q] of this point
};

hipError_t launch_chi(const ChiArgs &a, bool b3, hipStream_t s);
hipError_t launch_chi_finish(const ChiFinishArgs &a, hipStream_t s);
hipError_t launch_fill_points(const PointPack &pk, PointRec *dst, unsigned long long *queue,
                              hipStream_t s);
hipError_t launch_trig(int Lx, int Ly, double *trig, hipStream_t s);
hipError_t launch_qtrig(const double *q, int n, double *out, hipStream_t s);
hipError_t launch_gtable(double2 *gtab, hipStream_t s);
// delta2 + qtrig + both thermal tables in one launch
hipError_t launch_call_tables(const double *delta, int n_delta, int n_delta_pad, double *d2,
                              const double *q, int n_q, double *qtrig, double2 *gt,
                              float4 *gt32, hipStream_t s);
// trig + qlat in one launch
hipError_t launch_group_tables(int Lx, int Ly, double *trig, const double *q, int n_q,
                               int *qlat, hipStream_t s);
hipError_t launch_delta2(const double *delta, int n_delta, int n_delta_pad,
                         double *d2, hipStream_t s);
hipError_t launch_etab2(const Hop &h, const double *trig, int Lx, int Ly, double *etab,
                        hipStream_t s);
hipError_t launch_etab(const Hop3 &h, const double *trig, int Lx, int Ly, double *etab,
                       hipStream_t s);
hipError_t launch_qlat(const double *q, int n_q, int Lx, int Ly, int *qlat, hipStream_t s);
hipError_t launch_series(const SweepArgs &a, int G, bool fp64, bool b3, hipStream_t s);
// hot: the batch's points all have T >= kInPlaceT (the in-place kernels,
// which write no tile-series moments)
hipError_t launch_sweep_f64(const SweepArgs &a, int td, int n_dtiles, int G, bool b3,
                            bool hot, hipStream_t s);
hipError_t launch_sweep_f32c(const SweepArgs &a, int td, int n_dtiles, int G, bool b3,
                             bool hot, hipStream_t s);
hipError_t launch_rows(const RowArgs &a, int G, hipStream_t s);
hipError_t launch_argmin(const ArgminArgs &a, int n_set, hipStream_t s);
hipError_t launch_grad(const GradArgs &a, int G, hipStream_t s);
hipError_t launch_grad_finish(const GradFinishArgs &a, int G, hipStream_t s);

// LO pairing (two plane waves, q and -q, of equal amplitude) of one point and
// one pair momentum q on a lattice axis.  The momentum across q labels Ls
// independent sectors; in each, c_{k up} of the chain index j couples to the
// holes d_{j -+ s} (d_p = c^+_{-p down}, s the lattice index of q along the
// chain), so the 2 Lc Nambu modes of a sector fall into g = gcd(2s, Lc)
// cycles of n = 2 Lc / g modes, each a periodic tridiagonal matrix.  Grid
// (sector * g + cycle, Delta, band slot); one workgroup diagonalises one
// cycle (cyclic Jacobi in LDS) and writes the sum of -T ln(1 + e^{-E/T})
// over its eigenvalues plus xi_down of its spin-up momenta.
constexpr int kLoMaxCycle = 128;   // largest cycle the LO kernel takes
struct LoArgs {
    Hop hop;
    double eps[2];        // band sign per output slot
    double mu, h, T;
    int Lx, Ly;
    int along_y;          // 1: q = (0, qy), chains along ky, sectors kx
    int Lc, Ls;           // chain length, sectors
    int s;                // lattice index of q along the chain, in [0, Lc)
    int g, n;             // cycles per sector, modes per cycle
    int n_delta;
    const double *delta;
    double *part;         // [nb][n_delta][Ls * g]
};
struct LoFinishArgs {
    const double *part;
    const double *delta;
    int n_delta, nb, n_parts;
    double n_k;           // Lx * Ly
    double w;             // sum_j |e^{iqR_j} + e^{-iqR_j}|^2 / N: 2, or 4 where 2q = 0
    double Vs[2];
    double *omega;        // output row of (point, slot 0, q); slot b at + b * slot_stride
    size_t slot_stride;
};
hipError_t launch_lo(const LoArgs &a, int nb, hipStream_t s);
hipError_t launch_lo_finish(const LoFinishArgs &a, hipStream_t s);

}  // namespace omega
