// Device code of libomega: the Delta sweep of Eq. (4)-(5), the fixed-order
// reductions, the searches of Algorithm 1 and the hand-derived gradient sweep.
//
// Work decomposition of the sweep (one point per launch):
//   blockIdx.z  = (band slot, Q) pair
//   blockIdx.y  = tile of TD consecutive Delta values (held in registers)
//   blockIdx.x  = chunk of 8x8 momentum tiles (one tile per wavefront pass)
// Every thread owns one momentum k at a time; it evaluates the band energies
// for (k, Q) once and reuses them for its TD Delta values.  Per Delta only
// the Delta-dependent remainder of the term is evaluated; the remainder is a
// sum of non-negative pieces, so plain FP64 accumulation is well conditioned.
// The Delta-independent piece carries the cancellation of Eq. (5) and is
// summed once per (k, Q) with Neumaier compensation.
//
// Symmetry: for Q = (qx, 0) the term at (kx, ky) equals the term at
// (kx, -ky) (E_k is even in ky, eta is even, and Q - k maps to its mirror),
// so a workgroup whose Q has qy == 0 sums ky indices 0..Ly/2 only, with
// weight 2 on every row that has a distinct mirror.  The Lx*Ly grid is still
// the one summed; half of it is reached through the mirror.
#include <hip/hip_runtime.h>
#include <math.h>
#include <type_traits>

#include "omega_internal.h"

namespace omega {

// ------------------------------------------------------------------ math

// sqrt(x) for x >= 0 from the hardware reciprocal square root (relative
// error ~5e-8 on gfx950), one Goldschmidt step and one residual correction;
// x = 0 is handled by clamping the reciprocal.  Correctly rounded on every
// input we have measured.
__device__ __forceinline__ double sqrt_rn(double x)
{
    double r = fmin(__builtin_amdgcn_rsq(x), 1e300);
    double s = x * r, h = 0.5 * r;
    double e = fma(-h, s, 0.5);
    s = fma(s, e, s);
    h = fma(h, e, h);
    double d = fma(-s, s, x);
    return fma(d, h, s);
}

// sqrt(x) for x > 0 with one Goldschmidt step only: relative error below
// 5e-15 (the Delta sweep, where it is far inside the required accuracy).
__device__ __forceinline__ double sqrt_1s(double x)
{
    double r = __builtin_amdgcn_rsq(x);
    double s = x * r;
    double t = fma(-r, s, 1.0);
    return fma(0.5 * s, t, s);
}

// 1/x for x > 0 (normal): hardware reciprocal and two Newton steps.
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// exp(z) for -745 < z <= 0: z = n ln2 + r, |r| <= ln2/2, Taylor series of
// degree 11 (truncation < 7e-15 relative), scaled by 2^n.
__device__ __forceinline__ double exp_nonpos(double z)
{
    const double kLog2e = 1.4426950408889634;
    const double kLn2Hi = 6.93147180369123816490e-01;
    const double kLn2Lo = 1.90821492927058770002e-10;
    double n = rint(z * kLog2e);
    double r = fma(-n, kLn2Hi, z);
    r = fma(-n, kLn2Lo, r);
    double p = 1.0 / 39916800.0;
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return __builtin_amdgcn_ldexp(p, (int)n);
}

// ln(1 + z) for 0 <= z <= 3: 1 + z = 2^e f with f in [1/sqrt2, sqrt2),
// ln f = 2 atanh(u), u = (f - 1)/(f + 1), |u| < 0.172, odd series to u^19
// (truncation < 1e-16).  The rounding of 1 + z costs at most 1.2e-16 absolute.
__device__ __forceinline__ double log1p_small(double z)
{
    const double kLn2Hi = 6.93147180369123816490e-01;
    const double kLn2Lo = 1.90821492927058770002e-10;
    double w = 1.0 + z;
    double f = __builtin_amdgcn_frexp_mant(w);
    int e = __builtin_amdgcn_frexp_exp(w);
    bool low = f < 0.70710678118654752440;
    f = low ? f + f : f;
    e = low ? e - 1 : e;
    double num = f - 1.0, den = f + 1.0;
    double rc = __builtin_amdgcn_rcp(den);
    rc = fma(rc, fma(-den, rc, 1.0), rc);
    double u = num * rc;
    u = fma(fma(-den, u, num), rc, u);
    double u2 = u * u;
    double p = 2.0 / 19.0;
    p = fma(p, u2, 2.0 / 17.0);
    p = fma(p, u2, 2.0 / 15.0);
    p = fma(p, u2, 2.0 / 13.0);
    p = fma(p, u2, 2.0 / 11.0);
    p = fma(p, u2, 2.0 / 9.0);
    p = fma(p, u2, 2.0 / 7.0);
    p = fma(p, u2, 2.0 / 5.0);
    p = fma(p, u2, 2.0 / 3.0);
    double lf = fma(p * u2, u, 2.0 * u);
    double de = (double)e;
    return fma(de, kLn2Hi, fma(de, kLn2Lo, lf));
}

// G(a) = ln(1 + e^-a) for 0 <= a <= 30 (the thermal term over T) from the
// table, given as = kGStep a.  With a0 = N / kGStep the nearest table point,
// r = as - N (|r| <= 1/2, exact) and sigma = 1/(1 + e^a0), p = sigma (1 -
// sigma), b = 1 - 2 sigma, the derivatives of G at a0 are
//   G' = -sigma, G'' = p, G''' = -p b, G'''' = p (1 - 6p),
//   G^(5) = -p b (1 - 12p)
// (from sigma' = -p, p' = -p b, b' = 2p).  The table holds the scaled Taylor
// coefficients c_n = G^(n)(a0) / (n! kGStep^n), n = 0..3; c4 = p (1 - 6p) /
// (24 kGStep^4) = c2 (1/49152 - c2) for kGStep = 64, since p = 8192 c2.  The
// polynomial of degree 4 leaves at most |G^(5)| (1/128)^5 / 120 <= 4.9e-13 G,
// as |G^(5)| <= 2p and p <= sigma <= G; checked against a long-double
// reference over [0, 30]: 2.4e-13 relative and 3.1e-14 absolute at most,
// without bias.  With the factor T and at most two such terms per momentum,
// Omega moves by less than 1e-13 T per momentum.  The caller guarantees
// a < 30 (1 + 4 eps) (|E| < 30 T with T zero or normal), so N <= kGTabN - 1
// and the table reads stay in range.
static_assert(kGStep == 64, "c4 from c2 below assumes kGStep = 64");
__device__ __forceinline__ double log1p_exp_tab(double as, const double2 *gt)
{
    const double N = rint(as);
    const double r = as - N;
    const int n = (int)N;
    const double2 c01 = gt[n];
    const double2 c23 = gt[kGTabN + n];
    const double c4 = c23.x * (1.0 / 49152.0 - c23.x);
    double g = fma(c4, r, c23.y);
    g = fma(g, r, c23.x);
    g = fma(g, r, c01.y);
    return fma(g, r, c01.x);
}

// Thermal part of the two quasiparticle branches, ln((1 + u1)(1 + u2)) =
// G(ax/T) + G(y/T) with u1 = exp(-ax/T), u2 = exp(-y/T), from the thermal
// table gt (the second term dropped beyond the cut; the caller has
// ax < cutT); invTs = kGStep / T.  Kept out of line: series_kernel needs it
// for few momenta and would otherwise hold its registers across the tile
// loop.
__device__ __attribute__((noinline)) double thermal_tab(double ax, double y, double invTs,
                                                        double cutT, const double2 *gt)
{
    double L = log1p_exp_tab(ax * invTs, gt);
    if (y < cutT)
        L += log1p_exp_tab(y * invTs, gt);
    return L;
}

// Band energy of App. A, (A.4), from cos/sin of the two momentum components.
__device__ __forceinline__ double band_energy(const Hop &t, double eps,
                                              double cx, double sx, double cy,
                                              double sy)
{
    double A = fma(t.tB * cx, cy, t.tA * (cx + cy));
    double D = t.tD * (cx - cy);
    double C = t.tC * sx * sy;
    return fma(eps, sqrt_rn(fma(D, D, C * C)), A);
}

// Neumaier (improved Kahan) accumulation step.
__device__ __forceinline__ void neumaier(double &s, double &c, double x)
{
    double t = s + x;
    double e = (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
    c += e;
    s = t;
}

// Neumaier sum of p[0], p[stride], ..., p[(n-1) stride] in that order.  The
// loads run kAhead elements ahead of the additions, so a sum of chunk
// partials waits for memory once per kAhead elements, not once per element.
constexpr int kAhead = 8;
__device__ __forceinline__ double ordered_sum(const double *p, size_t stride, int n)
{
    double s = 0.0, c = 0.0;
    int k = 0;
    for (; k + kAhead <= n; k += kAhead) {
        double v[kAhead];
#pragma unroll
        for (int u = 0; u < kAhead; ++u)
            v[u] = p[(size_t)(k + u) * stride];
#pragma unroll
        for (int u = 0; u < kAhead; ++u)
            neumaier(s, c, v[u]);
    }
    for (; k < n; ++k)
        neumaier(s, c, p[(size_t)k * stride]);
    return s + c;
}

// Two chains of ordered_sum in one loop, each with exactly its arithmetic,
// so that the loads of both are in flight together; a null p1 or p2 leaves
// its sum at 0.
__device__ __forceinline__ void ordered_sum2(const double *p1, size_t stride1,
                                             const double *p2, size_t stride2, int n,
                                             double &sum1, double &sum2)
{
    double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0;
    int k = 0;
    for (; k + kAhead <= n; k += kAhead) {
        double v1[kAhead], v2[kAhead];
#pragma unroll
        for (int u = 0; u < kAhead; ++u) {
            v1[u] = p1 ? p1[(size_t)(k + u) * stride1] : 0.0;
            v2[u] = p2 ? p2[(size_t)(k + u) * stride2] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kAhead; ++u) {
            neumaier(s1, c1, v1[u]);
            neumaier(s2, c2, v2[u]);
        }
    }
    for (; k < n; ++k) {
        neumaier(s1, c1, p1 ? p1[(size_t)k * stride1] : 0.0);
        neumaier(s2, c2, p2 ? p2[(size_t)k * stride2] : 0.0);
    }
    sum1 = s1 + c1;
    sum2 = s2 + c2;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

template <int N>
struct Log2 {
    static constexpr int value = 1 + Log2<N / 2>::value;
};
template <>
struct Log2<1> {
    static constexpr int value = 0;
};

// Sum TD per-lane accumulators over the 64 lanes of a wavefront by recursive
// halving: at each exchange a lane keeps one half of its values and receives
// the partner's copy of that half.  Afterwards acc[0] of lane l holds the
// wave-wide sum for Delta index (l >> (6 - log2 TD)) & (TD - 1).  The order
// of additions is fixed, so the result is bitwise reproducible.
template <int TD>
__device__ __forceinline__ void wave_reduce_halving(double (&acc)[TD], int lane)
{
    constexpr int LOG = Log2<TD>::value;
    static_assert(LOG <= 6, "Delta tile larger than a wavefront");
#pragma unroll
    for (int s = 0; s < LOG; ++s) {
        const int off = 32 >> s;
        const int half = TD >> (s + 1);
        const bool upper = (lane & off) != 0;
#pragma unroll
        for (int t = 0; t < half; ++t) {
            double lo = acc[t], hi = acc[t + half];
            double send = upper ? lo : hi;
            double keep = upper ? hi : lo;
            acc[t] = keep + __shfl_xor(send, off, 64);
        }
    }
#pragma unroll
    for (int off = 32 >> LOG; off >= 1; off >>= 1)
        acc[0] += __shfl_xor(acc[0], off, 64);
}

// ------------------------------------------------------------------ prep

// Point records of a batch, from kernel arguments into the workspace.
// Also zeroes the work-queue counters of the persistent sweep (queue may be
// null), which runs after it on the stream.
static_assert(kMaxQueues <= kFillMax, "fill_points_kernel zeroes the queues");
__global__ void fill_points_kernel(const PointPack pk, PointRec *dst,
                                   unsigned long long *queue)
{
    const int t = threadIdx.x;
    if (t < pk.n)
        dst[t] = pk.rec[t];
    if (queue && t < kMaxQueues)
        queue[(size_t)t * kQueueStride] = 0ull;
}

hipError_t launch_fill_points(const PointPack &pk, PointRec *dst, unsigned long long *queue,
                              hipStream_t s)
{
    hipLaunchKernelGGL(fill_points_kernel, dim3(1), dim3(kFillMax), 0, s, pk, dst, queue);
    return hipGetLastError();
}

// cos/sin of the lattice momenta 2 pi i / L.
__device__ __forceinline__ void trig_at(int t, int Lx, int Ly, double *trig)
{
    double s, c;
    if (t < Lx) {
        sincospi(2.0 * t / Lx, &s, &c);
        trig[t] = c;
        trig[Lx + t] = s;
    }
    if (t < Ly) {
        sincospi(2.0 * t / Ly, &s, &c);
        trig[2 * Lx + t] = c;
        trig[2 * Lx + Ly + t] = s;
    }
}

__global__ void trig_kernel(int Lx, int Ly, double *trig)
{
    trig_at(blockIdx.x * blockDim.x + threadIdx.x, Lx, Ly, trig);
}

hipError_t launch_trig(int Lx, int Ly, double *trig, hipStream_t s)
{
    const int n = Lx > Ly ? Lx : Ly;
    hipLaunchKernelGGL(trig_kernel, dim3((n + 255) / 256), dim3(256), 0, s, Lx, Ly,
                       trig);
    return hipGetLastError();
}

// Squared Delta values, padded to a whole Delta tile with the last value;
// workgroup 0 also writes max Delta^2 (NaN ignored) into d2[n_delta_pad].
__device__ __forceinline__ void delta2_block(int blk, const double *delta, int n_delta,
                                             int n_delta_pad, double *d2)
{
    const int t = blk * kBlock + threadIdx.x;
    if (t < n_delta_pad) {
        const double D = delta[t < n_delta ? t : n_delta - 1];
        d2[t] = D * D;
    }
    if (blk == 0) {
        // centre and half-width of [min Delta^2, max Delta^2] (NaN ignored;
        // a NaN Delta still poisons its own output through Delta^2)
        __shared__ double sh[2][kBlock];
        double mx = 0.0, mn = __builtin_inf();
        for (int i = threadIdx.x; i < n_delta; i += kBlock) {
            const double x = delta[i] * delta[i];
            mx = fmax(mx, x);
            mn = fmin(mn, x);
        }
        sh[0][threadIdx.x] = mx;
        sh[1][threadIdx.x] = mn;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                sh[0][threadIdx.x] = fmax(sh[0][threadIdx.x], sh[0][threadIdx.x + w]);
                sh[1][threadIdx.x] = fmin(sh[1][threadIdx.x], sh[1][threadIdx.x + w]);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const double hi = sh[0][0];
            const double lo = fmin(sh[1][0], hi);
            d2[n_delta_pad] = 0.5 * (lo + hi);
            d2[n_delta_pad + 1] = 0.5 * (hi - lo);
        }
    }
}

__global__ __launch_bounds__(kBlock) void delta2_kernel(const double *delta, int n_delta,
                                                        int n_delta_pad, double *d2)
{
    delta2_block(blockIdx.x, delta, n_delta, n_delta_pad, d2);
}

hipError_t launch_delta2(const double *delta, int n_delta, int n_delta_pad,
                         double *d2, hipStream_t s)
{
    hipLaunchKernelGGL(delta2_kernel, dim3((n_delta_pad + kBlock - 1) / kBlock),
                       dim3(kBlock), 0, s, delta, n_delta, n_delta_pad, d2);
    return hipGetLastError();
}

// cos and sin of both components of n pair momenta and of their halves,
// [n][kQTrig] = (cos qx, sin qx, cos qy, sin qy, cos qx/2, sin qx/2,
// cos qy/2, sin qy/2), once per call.
__device__ __forceinline__ void qtrig_at(int t, const double *q, int n, double *out)
{
    if (t < n) {
        double s, c;
        double *o = out + (size_t)kQTrig * t;
        sincos(q[2 * t], &s, &c);
        o[0] = c;
        o[1] = s;
        sincos(q[2 * t + 1], &s, &c);
        o[2] = c;
        o[3] = s;
        sincos(0.5 * q[2 * t], &s, &c);
        o[4] = c;
        o[5] = s;
        sincos(0.5 * q[2 * t + 1], &s, &c);
        o[6] = c;
        o[7] = s;
    }
}

__global__ void qtrig_kernel(const double *q, int n, double *out)
{
    qtrig_at(blockIdx.x * blockDim.x + threadIdx.x, q, n, out);
}

hipError_t launch_qtrig(const double *q, int n, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(qtrig_kernel, dim3((n + 255) / 256), dim3(256), 0, s, q, n, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ sweep

// Per (k, Q) invariants of one band.
// Thermal table at a0 = n / kGStep: (c0, c1) at gt[n] and (c2, c3) at
// gt[kGTabN + n], c_k = G^(k)(a0) / (k! kGStep^k) (see log1p_exp_tab).
__device__ __forceinline__ void gtable_at(int n, double2 *gt)
{
    if (n < kGTabN) {
        const double e = exp(-n * (1.0 / kGStep));
        const double sg = e / (1.0 + e);              // sigma = 1/(1 + e^a0)
        const double p = sg * (1.0 - sg);
        const double b = 1.0 - 2.0 * sg;
        const double s1 = 1.0 / kGStep;
        gt[n] = make_double2(log1p(e), -sg * s1);
        gt[kGTabN + n] = make_double2(p * (0.5 * s1 * s1), -(p * b) * (s1 * s1 * s1 / 6.0));
    }
}

// FP32 thermal table at a0 = n / kG32Step: (c0, c1, c2, c3), c_k =
// G^(k)(a0) / (k! kG32Step^k), computed in FP64 and rounded.
__device__ __forceinline__ void gtable32_at(int n, float4 *gt)
{
    if (n < kG32N) {
        const double e = exp(-n * (1.0 / kG32Step));
        const double sg = e / (1.0 + e);
        const double p = sg * (1.0 - sg);
        const double b = 1.0 - 2.0 * sg;
        const double s1 = 1.0 / kG32Step;
        gt[n] = make_float4((float)log1p(e), (float)(-sg * s1), (float)(p * (0.5 * s1 * s1)),
                            (float)(-(p * b) * (s1 * s1 * s1 / 6.0)));
    }
}

__global__ void gtable_kernel(double2 *gt)
{
    gtable_at(blockIdx.x * blockDim.x + threadIdx.x, gt);
}

// The per-call tables of a grid call in one launch: Delta^2 (with its
// range), cos/sin of Q and the FP64 and FP32 thermal tables, in consecutive
// workgroup ranges.
__global__ __launch_bounds__(kBlock) void call_tables_kernel(const double *delta, int n_delta,
                                                             int n_delta_pad, double *d2,
                                                             const double *q, int n_q,
                                                             double *qtrig, double2 *gt,
                                                             float4 *gt32)
{
    const int nd = (n_delta_pad + kBlock - 1) / kBlock;
    const int nqb = (n_q + kBlock - 1) / kBlock;
    const int ngb = (kGTabN + kBlock - 1) / kBlock;
    const int b = blockIdx.x;
    if (b < nd)
        delta2_block(b, delta, n_delta, n_delta_pad, d2);
    else if (b < nd + nqb)
        qtrig_at((b - nd) * kBlock + threadIdx.x, q, n_q, qtrig);
    else if (b < nd + nqb + ngb)
        gtable_at((b - nd - nqb) * kBlock + threadIdx.x, gt);
    else
        gtable32_at((b - nd - nqb - ngb) * kBlock + threadIdx.x, gt32);
}

hipError_t launch_call_tables(const double *delta, int n_delta, int n_delta_pad, double *d2,
                              const double *q, int n_q, double *qtrig, double2 *gt,
                              float4 *gt32, hipStream_t s)
{
    const int blocks = (n_delta_pad + kBlock - 1) / kBlock + (n_q + kBlock - 1) / kBlock +
                       (kGTabN + kBlock - 1) / kBlock + (kG32N + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(call_tables_kernel, dim3(blocks), dim3(kBlock), 0, s, delta, n_delta,
                       n_delta_pad, d2, q, n_q, qtrig, gt, gt32);
    return hipGetLastError();
}

hipError_t launch_gtable(double2 *gtab, hipStream_t s)
{
    hipLaunchKernelGGL(gtable_kernel, dim3((kGTabN + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                       gtab);
    return hipGetLastError();
}

struct KQ {
    double s2;     // ((a + b)/2)^2
    double as;     // |s|
    double m;      // |(a - b)/2|
    double eta2;   // (cos kx cos ky)^2
    double base;   // Delta-independent part of the term
};

// a = E(k) - mu - h (k up), b = E(Q - k) - mu + h (-k+Q down); Eq. (4) reads
// E^+- = d +- R with s = (a+b)/2, d = (a-b)/2, R = sqrt(s^2 + Delta^2 eta^2).
// Using min(E,0) - T ln(1 + exp(-|E|/T)) for each branch and
// {|d+R|, |d-R|} = {|R - |d||, R + |d|}, the term of Eq. (5) is
//   2 min(d, 0) + E_{k down}                     (Delta-independent)
//   - max(R - |d|, 0) - T ln[(1 + u1)(1 + u2)]   (Delta-dependent)
// with u1 = exp(-|R - |d||/T), u2 = exp(-(R + |d|)/T).
__device__ __forceinline__ KQ kq_from(double Ek, double Eq, double mu_up, double mu_dn,
                                      double cx, double cy)
{
    double up = Ek - mu_up;
    double dn = Eq - mu_dn;
    double s = 0.5 * (up + dn);
    double d = 0.5 * (up - dn);
    double eta = cx * cy;
    KQ r;
    r.s2 = s * s;
    r.as = fabs(s);
    r.m = fabs(d);
    r.eta2 = eta * eta;
    r.base = 2.0 * fmin(d, 0.0) + (Ek - mu_dn);
    return r;
}

// Real symmetric 3x3 matrix [[a00, a01, a02], [a01, a11, a12], [a02, a12, a22]].
struct Sym3 {
    double a00, a11, a22, a01, a02, a12;
};

// One Jacobi rotation in the (p, q) plane annihilating apq; r is the third
// index.  t = tan of the rotation angle, the smaller root of
// t^2 + 2 theta t - 1 = 0 with theta = (aqq - app) / (2 apq); tau = s/(1 + c).
__device__ __forceinline__ void jacobi_rotate(double &app, double &aqq, double &apq,
                                              double &arp, double &arq)
{
    if (fabs(apq) <= 1e-18 * (fabs(app) + fabs(aqq)) + 1e-300) {
        apq = 0.0;
        return;
    }
    const double theta = (aqq - app) / (2.0 * apq);
    const double t = copysign(1.0, theta) / (fabs(theta) + sqrt(fma(theta, theta, 1.0)));
    const double c = 1.0 / sqrt(fma(t, t, 1.0));
    const double sn = t * c;
    const double tau = sn / (1.0 + c);
    app = fma(-t, apq, app);
    aqq = fma(t, apq, aqq);
    apq = 0.0;
    const double rp = arp, rq = arq;
    arp = rp - sn * fma(tau, rp, rq);
    arq = rq + sn * fma(-tau, rq, rp);
}

// Eigenvalues of App. B's orbital matrix at one momentum, ascending.  With
// T13 = i alpha and T23 = i beta (alpha, beta real) the unitary
// diag(1, 1, i) maps the Hermitian matrix onto the real symmetric one with
// off-diagonals (T12, alpha, beta) up to a common sign of the last two,
// which leaves the spectrum unchanged; it is diagonalised by cyclic Jacobi
// sweeps (backward stable: eigenvalue errors of order 1e-16 of the norm).
__device__ __forceinline__ void eig3(const Hop3 &h, double cx, double sx, double cy,
                                     double sy, double c2x, double c2y, double *E)
{
    const double *t = h.t;   // t[0] = t1
    Sym3 A;
    const double cxy = cx * cy, c2xy = c2x * c2y, dc2 = c2x - c2y;
    A.a00 = 2.0 * t[1] * cx + 2.0 * t[0] * cy + 4.0 * t[2] * cxy + 2.0 * t[10] * dc2 +
            4.0 * t[11] * c2xy;
    A.a11 = 2.0 * t[0] * cx + 2.0 * t[1] * cy + 4.0 * t[2] * cxy - 2.0 * t[10] * dc2 +
            4.0 * t[11] * c2xy;
    A.a22 = h.eps0 + 2.0 * t[4] * (cx + cy) + 4.0 * t[5] * cxy + 2.0 * t[8] * (c2x + c2y) +
            4.0 * t[9] * (c2x * cy + cx * c2y);
    A.a01 = 4.0 * t[3] * sx * sy;
    A.a02 = 2.0 * t[6] * sx + 4.0 * t[7] * sx * cy;
    A.a12 = 2.0 * t[6] * sy + 4.0 * t[7] * sy * cx;
#pragma unroll 1
    for (int sweep = 0; sweep < 12; ++sweep) {
        if (A.a01 == 0.0 && A.a02 == 0.0 && A.a12 == 0.0)
            break;
        jacobi_rotate(A.a00, A.a11, A.a01, A.a02, A.a12);
        jacobi_rotate(A.a00, A.a22, A.a02, A.a01, A.a12);
        jacobi_rotate(A.a11, A.a22, A.a12, A.a01, A.a02);
    }
    double e0 = A.a00, e1 = A.a11, e2 = A.a22, tmp;
    if (e0 > e1) { tmp = e0; e0 = e1; e1 = tmp; }
    if (e1 > e2) { tmp = e1; e1 = e2; e2 = tmp; }
    if (e0 > e1) { tmp = e0; e0 = e1; e1 = tmp; }
    E[0] = e0;
    E[1] = e1;
    E[2] = e2;
}

// One band of eig3 at Q - k, for pair momenta off the lattice.
__device__ __forceinline__ double eig3_band(const Hop3 &h, double c, double sn, double cy,
                                            double sy, int b)
{
    double ev[3];
    eig3(h, c, sn, cy, sy, (c - sn) * (c + sn), (cy - sy) * (cy + sy), ev);
    return b == 0 ? ev[0] : (b == 1 ? ev[1] : ev[2]);
}

// Load of base[idx] with a 32-bit unsigned offset from a wave-uniform base
// (every table here holds fewer than 2^29 doubles), so that the address is
// a scalar base plus a 32-bit vector offset rather than 64-bit arithmetic.
__device__ __forceinline__ double ldg(const double *base, unsigned idx)
{
    return *(const double *)((const char *)base + (idx << 3));
}

// E(k) and E(Q - k) of momentum (i, j) for output slot `slot` and pair
// momentum iq, whose lattice index (mx, my) (-1 off the lattice) the caller
// reads once; rowk = i * Ly.  E(k) comes from the lattice table of either
// model, and so does E(Q - k) when Q lies on the lattice.  Otherwise E(Q - k)
// is computed at Q - k, with cos/sin of Q - k by angle subtraction: (A.4) in
// closed form for the two-band model, by diagonalising for the three-band
// model.
// The form factor is eta(k) = cos kx cos ky, or with a.eta_rel eta(k - Q/2)
// = cos(kx - qx/2) cos(ky - qy/2) from cos/sin of Q/2 (angle subtraction).
template <bool B3>
__device__ __forceinline__ KQ kq_setup(const SweepArgs &a, int slot, int iq, int mx, int my,
                                       int i, int j, unsigned rowk, double eps, double mu_up,
                                       double mu_dn, double cqx, double sqx, double cqy,
                                       double sqy)
{
    const int b = a.band3[slot];
    const unsigned n = (unsigned)a.Lx * (unsigned)a.Ly;
    const double *E = a.etab + (size_t)b * n;
    const double Ek = ldg(E, rowk + (unsigned)j);
    const double cx = ldg(a.trig, (unsigned)i), sx = ldg(a.trig + a.Lx, (unsigned)i);
    const double cy = ldg(a.trig + 2 * a.Lx, (unsigned)j);
    const double sy = ldg(a.trig + 2 * a.Lx + a.Ly, (unsigned)j);
    double Eq;
    if (mx >= 0 && my >= 0) {
        // ((mx - i) mod Lx) Ly + (my - j) mod Ly, from mx Ly - i Ly
        const int di = mx - i, dj = my - j;
        unsigned idx = (unsigned)mx * (unsigned)a.Ly - rowk + (unsigned)dj;
        idx += di < 0 ? n : 0u;
        idx += dj < 0 ? (unsigned)a.Ly : 0u;
        Eq = ldg(E, idx);
    } else {
        const double cpx = fma(cqx, cx, sqx * sx);
        const double spx = fma(sqx, cx, -(cqx * sx));
        const double cpy = fma(cqy, cy, sqy * sy);
        const double spy = fma(sqy, cy, -(cqy * sy));
        if constexpr (!B3)
            Eq = band_energy(a.hop, eps, cpx, spx, cpy, spy);
        else
            Eq = eig3_band(a.hop3, cpx, spx, cpy, spy, b);
    }
    if (a.eta_rel) {
        const double *qh = a.qtrig + kQTrig * iq + 4;   // cos, sin of qx/2 and qy/2
        return kq_from(Ek, Eq, mu_up, mu_dn, fma(cx, qh[0], sx * qh[1]),
                       fma(cy, qh[2], sy * qh[3]));
    }
    return kq_from(Ek, Eq, mu_up, mu_dn, cx, cy);
}

// Band table of the two-band model over the lattice, [2][Lx][Ly]: E_- then
// E_+ of (A.4), from the cos/sin table.
__global__ void etab2_kernel(const Hop h, const double *trig, int Lx, int Ly, double *E)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)Lx * Ly;
    if (t >= n)
        return;
    const int i = (int)(t / Ly);
    const int j = (int)(t - (long long)i * Ly);
    const double *cxt = trig, *sxt = trig + Lx, *cyt = trig + 2 * Lx, *syt = cyt + Ly;
    E[t] = band_energy(h, -1.0, cxt[i], sxt[i], cyt[j], syt[j]);
    E[n + t] = band_energy(h, 1.0, cxt[i], sxt[i], cyt[j], syt[j]);
}

hipError_t launch_etab2(const Hop &h, const double *trig, int Lx, int Ly, double *etab,
                        hipStream_t s)
{
    const long long n = (long long)Lx * Ly;
    hipLaunchKernelGGL(etab2_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, h, trig, Lx, Ly, etab);
    return hipGetLastError();
}

// Band table of the three-band model over the lattice, [3][Lx][Ly], from the
// cos/sin table (cos 2k at the lattice index 2i mod L).
__global__ void etab_kernel(const Hop3 h, const double *trig, int Lx, int Ly, double *E)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)Lx * Ly;
    if (t >= n)
        return;
    const int i = (int)(t / Ly);
    const int j = (int)(t - (long long)i * Ly);
    const double *cxt = trig, *sxt = trig + Lx, *cyt = trig + 2 * Lx, *syt = cyt + Ly;
    const int i2 = (int)((2LL * i) % Lx), j2 = (int)((2LL * j) % Ly);
    double ev[3];
    eig3(h, cxt[i], sxt[i], cyt[j], syt[j], cxt[i2], cyt[j2], ev);
    E[t] = ev[0];
    E[n + t] = ev[1];
    E[2 * n + t] = ev[2];
}

hipError_t launch_etab(const Hop3 &h, const double *trig, int Lx, int Ly, double *etab,
                       hipStream_t s)
{
    const long long n = (long long)Lx * Ly;
    hipLaunchKernelGGL(etab_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, h, trig, Lx, Ly, etab);
    return hipGetLastError();
}

// Lattice index of each pair momentum: (m, n) with Q = (2 pi m/Lx, 2 pi n/Ly)
// to within 1e-13 (m, n reduced into [0, L)), else (-1, -1).
__device__ __forceinline__ void qlat_at(int t, const double *q, int n_q, int Lx, int Ly,
                                        int *qlat)
{
    if (t >= n_q)
        return;
    int idx[2] = {-1, -1};
    const int L[2] = {Lx, Ly};
    bool ok = true;
    for (int c = 0; c < 2; ++c) {
        const double v = q[2 * t + c];
        const double step = 2.0 * M_PI / L[c];
        const double m = rint(v / step);
        if (!(fabs(v - m * step) <= 1e-13 * fmax(1.0, fabs(v))) || fabs(m) > 1e9) {
            ok = false;
            break;
        }
        long long mi = (long long)m % L[c];
        idx[c] = (int)(mi < 0 ? mi + L[c] : mi);
    }
    qlat[2 * t] = ok ? idx[0] : -1;
    qlat[2 * t + 1] = ok ? idx[1] : -1;
}

__global__ void qlat_kernel(const double *q, int n_q, int Lx, int Ly, int *qlat)
{
    qlat_at(blockIdx.x * blockDim.x + threadIdx.x, q, n_q, Lx, Ly, qlat);
}

// The per-lattice tables of a grid call in one launch: cos/sin of the
// lattice momenta and the lattice index of each Q.
__global__ __launch_bounds__(kBlock) void group_tables_kernel(int Lx, int Ly, double *trig,
                                                              const double *q, int n_q,
                                                              int *qlat)
{
    const int nl = Lx > Ly ? Lx : Ly;
    const int nt = (nl + kBlock - 1) / kBlock;
    if ((int)blockIdx.x < nt)
        trig_at(blockIdx.x * kBlock + threadIdx.x, Lx, Ly, trig);
    else
        qlat_at((blockIdx.x - nt) * kBlock + threadIdx.x, q, n_q, Lx, Ly, qlat);
}

hipError_t launch_group_tables(int Lx, int Ly, double *trig, const double *q, int n_q,
                               int *qlat, hipStream_t s)
{
    const int nl = Lx > Ly ? Lx : Ly;
    const int blocks = (nl + kBlock - 1) / kBlock + (n_q + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(group_tables_kernel, dim3(blocks), dim3(kBlock), 0, s, Lx, Ly, trig, q,
                       n_q, qlat);
    return hipGetLastError();
}

hipError_t launch_qlat(const double *q, int n_q, int Lx, int Ly, int *qlat, hipStream_t s)
{
    hipLaunchKernelGGL(qlat_kernel, dim3((n_q + kBlock - 1) / kBlock), dim3(kBlock), 0, s, q,
                       n_q, Lx, Ly, qlat);
    return hipGetLastError();
}

// Whether the (k, Q) term's Delta dependence goes through the Delta^2 series
// (see kSeriesRho) rather than the per-Delta loop; R02 = s^2 + x0 eta^2.
// Decided once, in series_kernel, and handed to the sweeps as a per-tile lane
// mask.
__device__ __forceinline__ bool series_term(const KQ &r, double R02, double hw, double cutT)
{
    return (r.as - r.m) >= cutT && hw * r.eta2 <= kSeriesRho * R02;
}

// Momentum range of one workgroup.  Both models have E(-kx, ky) =
// E(kx, -ky) = E(kx, ky), and eta^2 is even in each component, so with
// qy == 0 the term at ky equals the term at -ky and only ky indices 0..Ly/2
// are visited; likewise kx with qx == 0 (Q = 0: a quarter of the zone).  On a
// square lattice both models are also symmetric under kx <-> ky (it swaps
// the two orbitals of App. A, and d_xz with d_yz in App. B), and so is
// eta^2; with Q = 0, E(Q - k) = E(k) keeps the term symmetric too, so only
// the triangle j <= i of that quarter is visited (an eighth of the zone).
// The tiles of the layout, the rectangle TXw x TYw or the triangle tj <= ti,
// row after row, are spread evenly over the same n_chunks workgroups.
struct KRange {
    bool fx, fy, fd;
    int TYw;        // tiles along ky in this layout (rectangle)
    int ilim, jlim; // kx / ky index bounds
    int begin, end; // tile range of this workgroup
};

__device__ __forceinline__ KRange k_range(const SweepArgs &a, double qx, double qy, int chunk)
{
    KRange k;
    k.fx = (qx == 0.0);
    k.fy = (qy == 0.0);
    k.fd = k.fx && k.fy && a.Lx == a.Ly;
    k.ilim = k.fx ? a.Lx / 2 + 1 : a.Lx;
    k.jlim = k.fy ? a.Ly / 2 + 1 : a.Ly;
    const int TXw = (k.ilim + kTileEdge - 1) / kTileEdge;
    k.TYw = (k.jlim + kTileEdge - 1) / kTileEdge;
    const int nt = k.fd ? TXw * (TXw + 1) / 2 : TXw * k.TYw;
    const int span = (nt + a.n_chunks - 1) / a.n_chunks;
    k.begin = chunk * span;
    k.end = min(k.begin + span, nt);
    return k;
}

// Tiles in row ti of the layout (FD: the triangle).
template <bool FD>
__device__ __forceinline__ int tile_row_len(const KRange &k, int ti)
{
    return FD ? ti + 1 : k.TYw;
}

// Position (ti, tj) of tile t of the layout (wave-uniform).
__device__ __forceinline__ void tile_pos(const KRange &k, int t, int &ti, int &tj)
{
    if (!k.fd) {
        ti = t / k.TYw;
        tj = t - ti * k.TYw;
        return;
    }
    // row ti holds tiles ti (ti + 1) / 2 .. ti (ti + 1) / 2 + ti
    int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while (r > 0 && r * (r + 1) / 2 > t)
        --r;
    while ((r + 1) * (r + 2) / 2 <= t)
        ++r;
    ti = r;
    tj = t - r * (r + 1) / 2;
}

// Whether momentum (i, j) belongs to the layout (FD: the triangle).
template <bool FD>
__device__ __forceinline__ bool in_layout(const KRange &k, int i, int j)
{
    return i < k.ilim && j < k.jlim && (!FD || j <= i);
}

// weight of momentum (i, j): 2 per folded axis whose mirror index L - i is
// a different momentum, and 2 more off the diagonal when kx <-> ky is folded
// (FD, known at compile time, or k.fd)
template <bool FD>
__device__ __forceinline__ double mirror_weight_t(const KRange &k, int i, int j, int Lx, int Ly)
{
    const double wx = (k.fx && i != 0 && 2 * i != Lx) ? 2.0 : 1.0;
    const double wy = (k.fy && j != 0 && 2 * j != Ly) ? 2.0 : 1.0;
    if constexpr (FD)
        return (i != j ? 2.0 : 1.0) * (wx * wy);
    else
        return wx * wy;
}

__device__ __forceinline__ double mirror_weight(const KRange &k, int i, int j, int Lx, int Ly)
{
    const double wx = (k.fx && i != 0 && 2 * i != Lx) ? 2.0 : 1.0;
    const double wy = (k.fy && j != 0 && 2 * j != Ly) ? 2.0 : 1.0;
    const double wd = (k.fd && i != j) ? 2.0 : 1.0;
    return wx * wy * wd;
}

// The listed tiles of one (batch point, band, Q) and chunk, as the series
// pass wrote them: the four wave lists one behind the other, each entry the
// tile's position (ti << 32) | tj and its lane mask.  The lists are written
// by an earlier kernel and only read here, so they are read through the
// constant address space (scalar loads of wave-uniform entries).
typedef const __attribute__((address_space(4))) unsigned long long *ConstU64Ptr;

struct TileList {
    ConstU64Ptr base;
    int total;
};

__device__ __forceinline__ TileList tile_list(const SweepArgs &a, int bz, int chunk)
{
    TileList t;
    const size_t row = (size_t)bz * a.n_chunks + chunk;
    t.base = (ConstU64Ptr)(a.tlist + row * 4 * a.lcap * 2);
    t.total = *(const __attribute__((address_space(4))) int *)(a.tcnt + row);
    return t;
}

// Entry e (wave-uniform) of the list: tile (ti, tj) and lane mask.
__device__ __forceinline__ void listed_tile(const TileList &t, int e, int &ti, int &tj,
                                            unsigned long long &mask)
{
    const unsigned long long pos = t.base[2 * e];
    ti = (int)(pos >> 32);
    tj = (int)(unsigned)pos;
    mask = t.base[2 * e + 1];
}

// The argument block of a kernel whose only parameter is a SweepArgs: the
// kernarg segment starts with it.  Reading the fields through this pointer,
// made opaque once per unit of a persistent kernel, reloads them with scalar
// loads instead of holding them in registers across the whole unit.
typedef const __attribute__((address_space(4))) SweepArgs *ConstArgs;

// Per-unit constants of the queued sweep (sweep_kernel), in LDS: the tile's
// Delta^2 range [x_lo, x_hi] with centre and half-width, mu +- h, T, 1/T,
// the cut 30 T and kGStep / T (the thermal table's argument scale).
enum {
    kUcXlo, kUcXhi, kUcXc, kUcHt, kUcMuUp, kUcMuDn, kUcT, kUcInvT, kUcCutT, kUcInvTs,
    kUnitConsts
};

// Work queues of the persistent sweeps: nq = a.n_queues 64-bit counters in
// the workspace (kMaxQueues of them zeroed by fill_points_kernel before every
// batch).  Units are (chunk, Delta tile, row).  The groups g = (row, chunk)
// are dealt out to the queues, g = q mod nq going to queue q (1 queue for a
// grid of fewer workgroups than queues), and a queue hands out the Delta tiles of one group
// one after the other: the waves that take them run on one XCD at about the
// same time and share that chunk's tile list and band-table entries in its
// L2.  Queue q is served by the workgroups with blockIdx.x = q mod nq, so
// every unit has a taker whatever the placement of the workgroups.  The
// chunk index is rotated by the row, so that each queue sees chunks from
// the whole zone.  take_unit returns the next unit of queue q as {chunk,
// Delta tile, row}, with row -1 once the queue is empty; a wave stops at the
// first -1, so every wave ends.
__device__ __forceinline__ int sweep_queues(const SweepArgs &a)
{
    return gridDim.x < (unsigned)a.n_queues ? 1 : a.n_queues;
}

__device__ __forceinline__ int3 take_unit(const SweepArgs &a, int q, int nq)
{
    const unsigned long long k = atomicAdd(a.queue + (size_t)q * kQueueStride, 1ull);
    const unsigned long long nd = (unsigned long long)a.n_dtiles;
    const unsigned long long nc = (unsigned long long)a.n_chunks;
    const unsigned long long m = k / nd;
    const unsigned long long g = (unsigned long long)q + (unsigned long long)nq * m;
    if (g >= nc * (unsigned long long)a.n_rows)
        return make_int3(0, 0, -1);
    const unsigned long long dtile = k - m * nd;
    const unsigned long long row = g / nc;
    const unsigned long long chunk = (g - row * nc + row) % nc;
    return make_int3((int)chunk, (int)dtile, (int)row);
}

// Largest ratio of each series level (see kSeriesLevel).
__constant__ constexpr SeriesLevelRho kLevelRho{};

// Whether m terms is one of the series levels short of the full count.
__device__ constexpr bool is_series_level(int m)
{
    for (int k = 0; k + 1 < kSeriesLevels; ++k)
        if (kSeriesLevel[k] == m)
            return true;
    return false;
}

// Per-(k, Q) pass over one (band, Q, point) and momentum chunk, shared by
// both precisions:
//   - the Delta-independent part of the term, Neumaier-summed (for the FP32
//     sweep minus P(0), the full Delta-dependent part at Delta = 0);
//   - the Delta^2 series moments C0 = sum w (R0 - |d|) (for the FP32 sweep
//     sum w (R0 - |s|), as |s| - |d| is part of P(0)) and
//     M_n = sum w R0 (eta^2/R0^2)^n;
//   - per wave, the list of 8 x 8 tiles with lanes the per-Delta sweep must
//     evaluate directly, with the ballot of those lanes (the sweeps walk
//     these lists).
// Grid (chunk, band*Q + nbq*g).
// Two-band: 4 waves/SIMD (a few spills outside the moment loop beat the
// 3-wave occupancy its registers would otherwise give); three-band: 3.
template <bool B3, bool F64>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(B3 ? 3 : 4)))
void series_kernel(const SweepArgs a)
{
    const int chunk = blockIdx.x;
    const int g = blockIdx.y / a.nbq;
    const int bq = blockIdx.y - g * a.nbq;
    const int slot = bq / a.n_q;
    const int iq = bq - slot * a.n_q;
    const double eps = slot ? a.eps[1] : a.eps[0];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const double qy = a.q[2 * iq + 1];
    const KRange kr = k_range(a, a.q[2 * iq], qy, chunk);
    const PointRec pt = a.pts[g];
    const double mu_up = a.mu + pt.h, mu_dn = a.mu - pt.h;
    const double T = pt.T;
    const double invT = T > 0.0 ? 1.0 / T : 0.0;
    // the FP32-compensated path classifies with its own (FP32) cut
    constexpr bool fp64 = F64;
    const double cutT = kCutFp64 * T;
    const double x0 = a.d2[a.n_delta_pad];
    const double hw = a.d2[a.n_delta_pad + 1];
    const double cqx = a.qtrig[kQTrig * iq], sqx = a.qtrig[kQTrig * iq + 1];
    const double cqy = a.qtrig[kQTrig * iq + 2], sqy = a.qtrig[kQTrig * iq + 3];
    const int qmx = __builtin_amdgcn_readfirstlane(a.qlat[2 * iq]);
    const int qmy = __builtin_amdgcn_readfirstlane(a.qlat[2 * iq + 1]);
    // the wave's list, staged here and written out behind the lists of the
    // lower waves once all four are known
    __shared__ unsigned long long lst[4][2 * kMaxWaveList];
    __shared__ int lcnt[4];
    int n_listed = 0;
    double mom[kMomentSlots];
#pragma unroll
    for (int n = 0; n < kMomentSlots; ++n)
        mom[n] = 0.0;
    double bs = 0.0, bc = 0.0;
    const int li = lane >> 3, lj = lane & 7;
    const unsigned liLy = (unsigned)li * (unsigned)a.Ly;
    // the walk, compiled once per layout: the rectangle, and the triangle
    // of Q = 0 on a square lattice
    auto walk = [&](auto fd_tag) __attribute__((always_inline)) {
        constexpr bool FD = decltype(fd_tag)::value;
        // tile (ti, tj), advanced by 4 without a division per tile
        int ti = 0, tj = 0;
        tile_pos(kr, kr.begin + wave, ti, tj);
        for (int tile = kr.begin + wave; tile < kr.end; tile += 4) {
            const int i = ti * kTileEdge + li;
            const int j = tj * kTileEdge + lj;
            bool direct = false;
            if (in_layout<FD>(kr, i, j)) {
                const KQ r = kq_setup<B3>(a, slot, iq, qmx, qmy, i, j,
                                          (unsigned)(ti * kTileEdge) * (unsigned)a.Ly + liLy, eps,
                                          mu_up, mu_dn, cqx, sqx, cqy, sqy);
                const double w = mirror_weight_t<FD>(kr, i, j, a.Lx, a.Ly);
                const double A0 = r.as - r.m;
                double base = r.base;
                if constexpr (!fp64) {
                    // P(0) for the FP32-compensated sweep, its thermal part
                    // from the thermal table (read through the cache)
                    double P0 = fmax(A0, 0.0);
                    if (fabs(A0) < cutT)
                        P0 = fma(T, thermal_tab(fabs(A0), r.as + r.m, kGStep * invT, cutT, a.gtab), P0);
                    base -= P0;
                }
                neumaier(bs, bc, w * base);
                const double R02 = fma(x0, r.eta2, r.s2);
                if (series_term(r, R02, hw, cutT)) {
                    const double R0 = sqrt_rn(R02);
                    // R0 - |s| = x0 eta^2 / (R0 + |s|) without cancellation
                    const double c0 = fp64 ? R0 - r.m
                                           : (R02 > 0.0 ? x0 * r.eta2 * rcp_nr(R0 + r.as) : 0.0);
                    mom[0] = fma(w, c0, mom[0]);
                    // R0 = 0 only with s = 0 and eta^2 x0 = 0: then the powers vanish
                    const double ratio = R02 > 0.0 ? r.eta2 * rcp_nr(R02) : 0.0;
                    // terms this wave needs: the smallest level that covers the
                    // ratio of every series lane (the active lanes here)
                    const double rho = hw * ratio;
                    int nt = kSeriesTerms;
    #pragma unroll
                    for (int k = kSeriesLevels - 2; k >= 0; --k)
                        if (__ballot(rho > kLevelRho.v[k]) == 0ull)
                            nt = kSeriesLevel[k];
                    double t = w * R0;
    #pragma unroll
                    for (int n = 1; n <= kSeriesTerms; ++n) {
                        if (is_series_level(n - 1) && n > nt)
                            break;
                        t *= ratio;
                        mom[n] += t;
                    }
                } else {
                    direct = true;
                }
            }
            const unsigned long long ballot = __ballot(direct);
            if (ballot != 0ull) {
                if (lane == 0) {
                    lst[wave][2 * n_listed] =
                        ((unsigned long long)(unsigned)ti << 32) | (unsigned)tj;
                    lst[wave][2 * n_listed + 1] = ballot;
                }
                ++n_listed;
            }
            tj += 4;
            while (tj >= tile_row_len<FD>(kr, ti)) {
                tj -= tile_row_len<FD>(kr, ti);
                ++ti;
            }
        }
    };
    if (kr.fd)
        walk(std::true_type{});
    else
        walk(std::false_type{});
    if (lane == 0)
        lcnt[wave] = n_listed;
    __shared__ double red[4][64];
    __shared__ double bred[4];
    const double bv = wave_sum(bs + bc);
    if (lane == 0)
        bred[wave] = bv;
    wave_reduce_halving<kMomentSlots>(mom, lane);
    red[wave][lane] = mom[0];
    __syncthreads();
    {
        const size_t row = (size_t)blockIdx.y * a.n_chunks + chunk;
        const int pre = (wave > 0 ? lcnt[0] : 0) + (wave > 1 ? lcnt[1] : 0) +
                        (wave > 2 ? lcnt[2] : 0);
        unsigned long long *tl = a.tlist + row * 4 * a.lcap * 2 + 2 * (size_t)pre;
        for (int x = lane; x < 2 * n_listed; x += 64)
            tl[x] = lst[wave][x];
        if (threadIdx.x == 0)
            a.tcnt[row] = ((lcnt[0] + lcnt[1]) + lcnt[2]) + lcnt[3];
    }
    constexpr int SHIFT = 6 - Log2<kMomentSlots>::value;
    if (threadIdx.x < kMomentSlots) {
        const int src = threadIdx.x << SHIFT;
        a.mpart[((size_t)blockIdx.y * a.n_chunks + chunk) * kMomentSlots + threadIdx.x] =
            ((red[0][src] + red[1][src]) + red[2][src]) + red[3][src];
    }
    if (threadIdx.x == 0)
        a.base_part[(size_t)blockIdx.y * a.n_chunks + chunk] =
            ((bred[0] + bred[1]) + bred[2]) + bred[3];
}

hipError_t launch_series(const SweepArgs &a, int G, bool fp64, bool b3, hipStream_t s)
{
    const dim3 grid(a.n_chunks, a.nbq * G);
    if (b3 && fp64)
        hipLaunchKernelGGL((series_kernel<true, true>), grid, dim3(kBlock), 0, s, a);
    else if (b3)
        hipLaunchKernelGGL((series_kernel<true, false>), grid, dim3(kBlock), 0, s, a);
    else if (fp64)
        hipLaunchKernelGGL((series_kernel<false, true>), grid, dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((series_kernel<false, false>), grid, dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// Workgroups of a persistent launch: as many as stay resident at once on the
// current device (or blocks_per_cu of them per CU, if fewer), but no more
// than there are units.
template <typename K>
static int persistent_blocks(K kernel, int threads, unsigned long long units, int blocks_per_cu)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess)
        return -1;
    if (per_cu < 1)
        per_cu = 1;
    if (blocks_per_cu > 0 && blocks_per_cu < per_cu)
        per_cu = blocks_per_cu;
    const unsigned long long n = (unsigned long long)cus * per_cu;
    return (int)(n < units ? n : units);
}

// FP32-compensated sweep.  With P(Delta) = max(R - |d|, 0) + T ln((1+u1)(1+u2))
// the term of Eq. (5) is [2 min(d,0) + E_{k down}] - P(Delta), split as
//   [2 min(d,0) + E_{k down} - P(0)]          FP64, in series_kernel
//   - [P(Delta) - P(0)]                       FP32, per Delta
// With A0 = |s| - |d| and delta = R - |s| = Delta^2 eta^2 / (R + |s|) (no
// cancellation), the cold part of the difference is delta when A0 >= 0 and
// max(A0 + delta, 0) otherwise.  The thermal part is T (L(Delta) - L(0)) with
// both logarithms in FP32.  The difference vanishes at Delta = 0, where the
// result is exactly the FP64 value (Delta = 0 slots are zeroed), so the
// Q-degenerate normal-state row keeps its FP64 degeneracy; elsewhere it is
// small where the term is large.  Terms on the series path contribute
// delta through the FP64 moments instead, and terms on a Delta tile's series
// (R - |d|) - P(0) through FP64 tile moments.  Each lane sums the few queued
// terms it evaluates per unit in FP32 before the FP64 reduction tree.
struct KQf {
    float s2, as, m, eta2, A0;
    float P0;      // T * L(0) in FP32, through the Delta loop's own arithmetic
};

// G(a) = ln(1 + e^-a) in FP32 from the FP32 table, given as = kG32Step a
// with 0 <= a < 20 (1 + 2^-22): r = as - N is exact and |r| <= 1/2, and
// N <= kG32N - 1.
__device__ __forceinline__ float log1p_exp_tab32(float as, const float4 *gt)
{
    const float N = __builtin_rintf(as);
    const float r = as - N;
    const float4 c = gt[(int)N];
    return fmaf(fmaf(fmaf(c.w, r, c.z), r, c.y), r, c.x);
}

// FP32 thermal logarithm of the Delta loop, ln((1 + u1)(1 + u2)) =
// G(ax/T) + G(y/T), u1 = e^-ax/T, u2 = e^-y/T, the second dropped beyond the
// cut (the caller has ax < cutT); invTs = kG32Step / T.
__device__ __forceinline__ float thermal_log_f32(float ax, float y, float invTs, float cutT,
                                                 const float4 *gt)
{
    float L = log1p_exp_tab32(ax * invTs, gt);
    if (y < cutT)
        L += log1p_exp_tab32(y * invTs, gt);
    return L;
}

// invT = 1/T; gt the FP32 thermal table.
__device__ __forceinline__ KQf kq_setup_f32(const KQ &q, double T, double invT,
                                            const float4 *gt)
{
    KQf r;
    r.s2 = (float)q.s2;
    // |s| >= 1e-30 keeps R + |s| > 0 at s = Delta = 0 (delta stays 0 there)
    r.as = (float)fmax(q.as, 1e-30);
    r.m = (float)q.m;
    r.eta2 = (float)q.eta2;
    r.A0 = (float)(q.as - q.m);
    const float Tf = (float)T, cutTf = kCutFp32 * Tf;
    const float ax0 = fabsf(r.A0);
    r.P0 = ax0 < cutTf
               ? Tf * thermal_log_f32(ax0, __builtin_amdgcn_sqrtf(r.s2) + r.m,
                                      (float)(kG32Step * invT), cutTf, gt)
               : 0.0f;
    return r;
}

// The per-Delta FP32 loop of one term: acc[t] += w (P(Delta_t) - P(0)),
// Delta^2 from the hi/lo pairs dp[0..TD] (dp[TD] only read ahead); invTs =
// kG32Step / T, gt the FP32 thermal table.
template <int TD>
__device__ __forceinline__ void f32_steps(float (&acc)[TD], const KQf &f, float wf,
                                          const float2 *dp, float Tf, float invTs,
                                          float cutTf, const float4 *gt)
{
    const bool pos = f.A0 >= 0.0f;
    float2 dcur = dp[0];
#pragma unroll
    for (int t = 0; t < TD; ++t) {
        const float2 dnext = dp[t + 1];
        const float g2 = fmaf(dcur.x, f.eta2, dcur.y * f.eta2);
        const float R = __builtin_amdgcn_sqrtf(f.s2 + g2);
        const float del = g2 * __builtin_amdgcn_rcpf(R + f.as);
        const float x = f.A0 + del;
        float piece = pos ? del : fmaxf(x, 0.0f);
        const float ax = fabsf(x);
        // beyond the cut only -P(0) is left of the thermal part
        if (ax < cutTf)
            piece += fmaf(Tf, thermal_log_f32(ax, R + f.m, invTs, cutTf, gt), -f.P0);
        else
            piece -= f.P0;
        acc[t] = fmaf(wf, piece, acc[t]);
        dcur = dnext;
    }
}

// The per-Delta FP64 loop of one term: acc[t] += w P(Delta_t), with
// P = max(x, 0) + T ln((1 + u1)(1 + u2)), x = R - |d|, u1 = e^-|x|/T,
// u2 = e^-(R + |d|)/T (each thermal part skipped beyond the cut 30 T);
// s2p = s^2 (floored), Delta^2 from dp[0..TD] (dp[TD] only read ahead),
// invTs = kGStep / T (the thermal table's scaled argument).
template <int TD>
__device__ __forceinline__ void f64_steps(double (&acc)[TD], double s2p, double m,
                                          double eta2, double w, double T, double invTs,
                                          double cutT, const double *dp, const double2 *gt)
{
    const double wT = w * T;
    double dcur = dp[0];
#pragma unroll
    for (int t = 0; t < TD; ++t) {
        const double dnext = dp[t + 1];
        const double R = sqrt_1s(fma(dcur, eta2, s2p));
        const double x = R - m;
        acc[t] = fma(w, fmax(x, 0.0), acc[t]);
        const double ax = fabs(x);
        if (ax < cutT) {
            double L = log1p_exp_tab(ax * invTs, gt);
            const double y = R + m;
            if (y < cutT)
                L += log1p_exp_tab(y * invTs, gt);
            acc[t] = fma(wT, L, acc[t]);
        }
        dcur = dnext;
    }
}

// Per-Delta sweep over the lanes series_kernel marked for direct
// evaluation; tiles without such lanes are skipped whole.  The kernel is
// persistent and each wave works on its own: it takes (chunk, Delta tile,
// row) units from the work queue until it runs dry (see take_unit), walks
// all listed tiles of the unit's chunk and writes the unit's sums itself, so
// no wave waits for another.  Per Delta tile a marked term is exactly zero,
// summed through the tile series, or queued for the per-Delta loop.
// F32 = false: everything in FP64; the workgroup shares the thermal table,
// loaded into LDS once.  F32 = true (the FP32-compensated sweep): the
// classification and the tile series stay FP64, and the loop evaluates
// P(Delta) - P(0) in FP32 (see KQf).
// Waves per workgroup of the queued sweep: the FP64 sweep shares one LDS
// copy of the thermal table among 12 waves (3 per SIMD, one workgroup per
// CU); the FP32 sweep has no table and runs 4-wave workgroups.
template <bool F32>
constexpr int sweep_waves() { return F32 ? 4 : 12; }

template <int TD, bool B3, bool F32>
__global__ __launch_bounds__(64 * sweep_waves<F32>()) __attribute__((amdgpu_waves_per_eu(3)))
void sweep_kernel(const SweepArgs args)
{
    constexpr int NW = sweep_waves<F32>();
    const SweepArgs &a0 = args;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // per wave: Delta^2 of the unit's tile, read from LDS inside the loop
    // (one extra slot for the look-ahead read of the last iteration), and
    // the unit's constants (kept in LDS rather than in registers across the
    // tile loop); per workgroup: the thermal table
    __shared__ double d2s[NW][TD + 1];
    // FP32 sweep: the same Delta^2 as an unevaluated FP32 pair hi + lo
    // (rounding Delta^2 to one float would shift every momentum's term at
    // that Delta the same way, a systematic 6e-8 that the sum would not
    // average out)
    __shared__ float2 d2f[NW][F32 ? TD + 1 : 1];
    __shared__ double uc[NW][kUnitConsts];
    __shared__ double2 gt[F32 ? 1 : kGTabEntries];
    __shared__ float4 gt32[F32 ? kG32N : 1];
    // per wave: queue of the (k, Q) terms that need the per-Delta loop and
    // their mirror weights; the loop runs on 64 of them at a time, so that
    // every lane of the wave has a term.  FP64: s^2 (floored), |d|, eta^2;
    // FP32: the six floats of KQf.  Each instance uses its own member only.
    union Queue {
        double d[3][2 * 64];
        float f[6][2 * 64];
    };
    __shared__ Queue lq[NW];
    __shared__ float lqw[NW][2 * 64];
    if constexpr (!F32) {
        for (int n = threadIdx.x; n < kGTabEntries; n += 64 * NW)
            gt[n] = a0.gtab[n];
    } else {
        for (int n = threadIdx.x; n < kG32N; n += 64 * NW)
            gt32[n] = a0.gtab32[n];
    }
    __syncthreads();
    int n_direct = 0;
    const int nq = sweep_queues(args);
    const int q = (int)(blockIdx.x % (unsigned)nq);
    for (;;) {
        ConstArgs ap = (ConstArgs)__builtin_amdgcn_kernarg_segment_ptr();
        asm volatile("" : "+s"(ap));
        const SweepArgs &a = *(const SweepArgs *)ap;   // the argument, reloaded per unit
        int3 un = make_int3(0, 0, -1);
        if (lane == 0)
            un = take_unit(a, q, nq);
        const int bz = __builtin_amdgcn_readfirstlane(un.z);
        if (bz < 0)
            break;
        const int chunk = __builtin_amdgcn_readfirstlane(un.x);
        const int dtile = __builtin_amdgcn_readfirstlane(un.y);
        const int g = bz / a.nbq;                  // point within the batch
        const int bq = bz - g * a.nbq;
        const int slot = bq / a.n_q;
        const int iq = bq - slot * a.n_q;
        const double eps = slot ? a.eps[1] : a.eps[0];
        const double qy = a.q[2 * iq + 1];
        const KRange kr = k_range(a, a.q[2 * iq], qy, chunk);
        const double cqx = a.qtrig[kQTrig * iq], sqx = a.qtrig[kQTrig * iq + 1];
        const double cqy = a.qtrig[kQTrig * iq + 2], sqy = a.qtrig[kQTrig * iq + 3];
        int qmx = __builtin_amdgcn_readfirstlane(a.qlat[2 * iq]);
        int qmy = __builtin_amdgcn_readfirstlane(a.qlat[2 * iq + 1]);
        // held in scalar registers for the unit, so that the tile walk does
        // not load them again ahead of the E(Q - k) read that needs them
        asm volatile("" : "+s"(qmx), "+s"(qmy));

        // the tile's Delta^2 (the padding repeats the last value) and range
        const double dl = a.d2[dtile * TD + (lane < TD ? lane : TD - 1)];
        double lo = dl, hi = dl;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            lo = fmin(lo, __shfl_xor(lo, off, 64));
            hi = fmax(hi, __shfl_xor(hi, off, 64));
        }
        if (lane <= TD) {
            d2s[wave][lane] = dl;
            if constexpr (F32) {
                const float dhi = (float)dl;
                d2f[wave][lane] = make_float2(dhi, (float)(dl - (double)dhi));
            }
        }
        if (lane == 0) {
            // centre and half-width of the tile series
            double *u = uc[wave];
            u[kUcXlo] = lo;
            u[kUcXhi] = hi;
            u[kUcXc] = 0.5 * (lo + hi);
            u[kUcHt] = 0.5 * (hi - lo);
            const PointRec pt = a.pts[g];
            u[kUcMuUp] = a.mu + pt.h;   // spin up: E - mu - h
            u[kUcMuDn] = a.mu - pt.h;   // spin down: E - mu + h
            u[kUcT] = pt.T;
            u[kUcInvT] = pt.T > 0.0 ? 1.0 / pt.T : 0.0;
            u[kUcCutT] = kCutFp64 * pt.T;
            u[kUcInvTs] = pt.T > 0.0 ? kGStep / pt.T : 0.0;
        }
        // the wave's LDS writes above are visible to all of its lanes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        using Acc = std::conditional_t<F32, float, double>;
        Acc acc[TD];
#pragma unroll
        for (int t = 0; t < TD; ++t)
            acc[t] = Acc(0);
        double tm[kTileSlots];
#pragma unroll
        for (int n = 0; n < kTileSlots; ++n)
            tm[n] = 0.0;

        const TileList tl = tile_list(a, bz, chunk);
        int pending = 0;   // queued terms of this wave
        // the next entry of the walk is fetched one tile ahead
        int e = 0;
        int nt_ti = 0, nt_tj = 0;
        unsigned long long nt_mask = 0ull;
        if (e < tl.total)
            listed_tile(tl, e, nt_ti, nt_tj, nt_mask);
        for (; e < tl.total; ++e) {
            const int ti = nt_ti, tj = nt_tj;
            const unsigned long long mk = nt_mask;
            if (e + 1 < tl.total)
                listed_tile(tl, e + 1, nt_ti, nt_tj, nt_mask);
            // the lane's place in the tile, from its lane id (cheaper than
            // keeping it in a register across the unit)
            const int ln = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
            const int i = ti * kTileEdge + (ln >> 3);
            const int j = tj * kTileEdge + (ln & 7);
            // an opaque zero offset keeps the Delta^2 and unit-constant reads
            // in LDS, read per tile, instead of hoisting them out of the loop
            // into (scarce) registers
            int zoff = 0;
            asm volatile("" : "+v"(zoff));
            const double *dp = d2s[wave] + zoff;
            const double *cp = uc[wave] + zoff;
            const double cutT = cp[kUcCutT];
            bool loop = false, tser = false;
            KQ r;
            double w = 0.0, Rc2 = 0.0;
            if ((mk >> lane) & 1ull) {
                r = kq_setup<B3>(a, slot, iq, qmx, qmy, i, j,
                                 (unsigned)i * (unsigned)a.Ly,
                                 eps, cp[kUcMuUp], cp[kUcMuDn], cqx, sqx, cqy, sqy);
                w = mirror_weight(kr, i, j, a.Lx, a.Ly);
                const double up = r.m + cutT, dn = r.m - cutT;
                const double x_lo = cp[kUcXlo], x_hi = cp[kUcXhi], ht = cp[kUcHt];
                Rc2 = fma(cp[kUcXc], r.eta2, r.s2);
                // cold and positive over the tile, and the tile series converges
                tser = fma(x_lo, r.eta2, r.s2) >= up * up && ht * r.eta2 <= kTileRho * Rc2;
                // exactly zero over the tile where R(x_hi) <= |d| - 30 T
                loop = !tser && !(dn > 0.0 && fma(x_hi, r.eta2, r.s2) <= dn * dn);
            }
            if (tser) {
                // moments of the tile series, accumulated per lane
                const double Rc = sqrt_rn(Rc2);
                // Rc = 0 only with s = 0 and xc eta^2 = 0: the powers vanish
                const double ratio = Rc2 > 0.0 ? r.eta2 * rcp_nr(Rc2) : 0.0;
                double c0 = Rc - r.m;
                if constexpr (F32) {
                    // minus P(0): its cold part in FP64, its thermal part in
                    // FP32 as the loop terms take it (kq_setup_f32)
                    const double A0 = r.as - r.m;
                    const float Tf = (float)cp[kUcT], cutTf = kCutFp32 * Tf;
                    const float ax0 = (float)fabs(A0);
                    const float P0f =
                        ax0 < cutTf ? Tf * thermal_log_f32(ax0, (float)(r.as + r.m),
                                                           (float)(kG32Step * cp[kUcInvT]),
                                                           cutTf, gt32)
                                    : 0.0f;
                    c0 -= fmax(A0, 0.0) + (double)P0f;
                }
                tm[0] = fma(w, c0, tm[0]);
                double tp = w * Rc;
#pragma unroll
                for (int n = 1; n < kTileSlots; ++n) {
                    tp *= ratio;
                    tm[n] += tp;
                }
            }
            // queue this tile's loop terms behind the pending ones
            const unsigned long long lb = __ballot(loop);
            n_direct += __popcll(lb);
            if (loop) {
                // R^2 >= 1e-300 keeps the reciprocal square root finite; the
                // floor is absorbed unless s^2 and Delta^2 eta^2 are both < 1e-284
                const int at = pending + (int)__builtin_amdgcn_mbcnt_hi(
                                             (unsigned)(lb >> 32),
                                             __builtin_amdgcn_mbcnt_lo((unsigned)lb, 0u));
                if constexpr (F32) {
                    const KQf f = kq_setup_f32(r, cp[kUcT], cp[kUcInvT], gt32);
                    float(*lf)[2 * 64] = lq[wave].f;
                    lf[0][at] = f.s2;
                    lf[1][at] = f.as;
                    lf[2][at] = f.m;
                    lf[3][at] = f.eta2;
                    lf[4][at] = f.A0;
                    lf[5][at] = f.P0;
                } else {
                    lq[wave].d[0][at] = r.s2 + 1e-300;
                    lq[wave].d[1][at] = r.m;
                    lq[wave].d[2][at] = r.eta2;
                }
                lqw[wave][at] = (float)w;
            }
            pending += __popcll(lb);
            // run the loop on full waves of queued terms; after the last tile
            // also on what is left
            const bool last = e + 1 >= tl.total;
            while (pending >= 64 || (last && pending > 0)) {
                // the wave's queue writes above are visible to all its lanes
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const int nb = pending < 64 ? pending : 64;
                if (F32 && lane < nb) {
                    // P(Delta) - P(0) in FP32 (see KQf)
                    const float(*lf)[2 * 64] = lq[wave].f;
                    KQf f;
                    f.s2 = lf[0][lane];
                    f.as = lf[1][lane];
                    f.m = lf[2][lane];
                    f.eta2 = lf[3][lane];
                    f.A0 = lf[4][lane];
                    f.P0 = lf[5][lane];
                    const float Tf = (float)cp[kUcT];
                    if constexpr (F32)
                        f32_steps<TD>(acc, f, lqw[wave][lane], d2f[wave] + zoff, Tf,
                                      (float)(kG32Step * cp[kUcInvT]), kCutFp32 * Tf, gt32);
                } else if (!F32 && lane < nb) {
                    if constexpr (!F32)
                        f64_steps<TD>(acc, lq[wave].d[0][lane], lq[wave].d[1][lane],
                                      lq[wave].d[2][lane], (double)lqw[wave][lane], cp[kUcT],
                                      cp[kUcInvTs], cutT, dp, gt);
                }
                // terms beyond the first 64 move to the front of the queue
                pending -= nb;
                if (lane < pending) {
                    if constexpr (F32) {
#pragma unroll
                        for (int c = 0; c < 6; ++c)
                            lq[wave].f[c][lane] = lq[wave].f[c][64 + lane];
                    } else {
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            lq[wave].d[c][lane] = lq[wave].d[c][64 + lane];
                    }
                    lqw[wave][lane] = lqw[wave][64 + lane];
                }
            }
        }

        // the unit's sums: lane t << SHIFT holds Delta t, lane n << TSHIFT
        // moment n
        double accd[TD];
#pragma unroll
        for (int t = 0; t < TD; ++t) {
            if constexpr (F32)   // the FP32 difference is zero at Delta = 0
                accd[t] = d2s[wave][t] == 0.0 ? 0.0 : (double)acc[t];
            else
                accd[t] = acc[t];
        }
        wave_reduce_halving<TD>(accd, lane);
        constexpr int SHIFT = 6 - Log2<TD>::value;
        if ((lane & ((1 << SHIFT) - 1)) == 0)
            a.part[((size_t)bz * a.n_chunks + chunk) * a.n_delta_pad + dtile * TD +
                   (lane >> SHIFT)] = accd[0];
        wave_reduce_halving<kTileSlots>(tm, lane);
        constexpr int TSHIFT = 6 - Log2<kTileSlots>::value;
        if ((lane & ((1 << TSHIFT) - 1)) == 0)
            a.tpart[(((size_t)bz * a.n_chunks + chunk) * a.n_dtiles + dtile) * kTileSlots +
                    (lane >> TSHIFT)] = tm[0];
    }
    if (a0.count && lane == 0 && n_direct)
        atomicAdd(a0.count, (unsigned long long)n_direct * TD);
}

template <int TD, bool B3, bool F32>
static hipError_t launch_persistent(const SweepArgs &a, hipStream_t s)
{
    const unsigned long long units =
        (unsigned long long)a.n_chunks * a.n_dtiles * (unsigned long long)a.n_rows;
    constexpr int threads = 64 * sweep_waves<F32>();
    const int blocks =
        persistent_blocks(sweep_kernel<TD, B3, F32>, threads, units, a.blocks_per_cu);
    if (blocks <= 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((sweep_kernel<TD, B3, F32>), dim3(blocks), dim3(threads), 0, s, a);
    return hipGetLastError();
}

// The FP64 sweep for points at T >= kInPlaceT, where almost no marked term
// is zero or on a tile series over a Delta tile: every marked lane runs the
// FP64 loop in place, without classification or queue, and without the
// tile-series registers the queued kernel holds (two-band: 4 waves/SIMD
// instead of 3; three-band: 3).
// Persistent like sweep_kernel, with the same work queues and units, one
// unit per wave at a time.
// Waves per workgroup of the in-place FP64 sweep: one workgroup per CU
// shares the LDS thermal table (two-band: 4 waves per SIMD; three-band: 3).
template <bool B3>
constexpr int hot_waves() { return B3 ? 12 : 16; }

template <int TD, bool B3>
__global__ __launch_bounds__(64 * hot_waves<B3>()) __attribute__((amdgpu_waves_per_eu(B3 ? 3 : 4)))
void sweep_f64_hot_kernel(const SweepArgs args)
{
    constexpr int NW = hot_waves<B3>();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    __shared__ double d2s[NW][TD + 1];
    __shared__ double2 gt[kGTabEntries];
    for (int n = threadIdx.x; n < kGTabEntries; n += 64 * NW)
        gt[n] = args.gtab[n];
    __syncthreads();
    int n_direct = 0;
    const int li = lane >> 3, lj = lane & 7;
    const int nq = sweep_queues(args);
    const int q = (int)(blockIdx.x % (unsigned)nq);
    for (;;) {
        ConstArgs ap = (ConstArgs)__builtin_amdgcn_kernarg_segment_ptr();
        asm volatile("" : "+s"(ap));
        const SweepArgs &a = *(const SweepArgs *)ap;   // the argument, reloaded per unit
        int3 un = make_int3(0, 0, -1);
        if (lane == 0)
            un = take_unit(a, q, nq);
        const int bz = __builtin_amdgcn_readfirstlane(un.z);
        if (bz < 0)
            break;
        const int chunk = __builtin_amdgcn_readfirstlane(un.x);
        const int dtile = __builtin_amdgcn_readfirstlane(un.y);
        const int g = bz / a.nbq;                  // point within the batch
        const int bq = bz - g * a.nbq;
        const int slot = bq / a.n_q;
        const int iq = bq - slot * a.n_q;
        const double eps = slot ? a.eps[1] : a.eps[0];
        const double qy = a.q[2 * iq + 1];
        const KRange kr = k_range(a, a.q[2 * iq], qy, chunk);
        const PointRec pt = a.pts[g];
        const double mu_up = a.mu + pt.h;
        const double mu_dn = a.mu - pt.h;
        const double T = pt.T;
        const double invT = T > 0.0 ? 1.0 / T : 0.0;
        const double cutT = kCutFp64 * T;
        const double cqx = a.qtrig[kQTrig * iq], sqx = a.qtrig[kQTrig * iq + 1];
        const double cqy = a.qtrig[kQTrig * iq + 2], sqy = a.qtrig[kQTrig * iq + 3];
        const int qmx = __builtin_amdgcn_readfirstlane(a.qlat[2 * iq]);
        const int qmy = __builtin_amdgcn_readfirstlane(a.qlat[2 * iq + 1]);

        if (lane <= TD)
            d2s[wave][lane] = a.d2[dtile * TD + (lane < TD ? lane : TD - 1)];
        // the wave's LDS writes above are visible to all of its lanes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        double acc[TD];
#pragma unroll
        for (int t = 0; t < TD; ++t)
            acc[t] = 0.0;
        const TileList tl = tile_list(a, bz, chunk);
        // the next entry of the walk is fetched one tile ahead
        int e = 0;
        int nt_ti = 0, nt_tj = 0;
        unsigned long long nt_mask = 0ull;
        if (e < tl.total)
            listed_tile(tl, e, nt_ti, nt_tj, nt_mask);
        for (; e < tl.total; ++e) {
            const int ti = nt_ti, tj = nt_tj;
            const unsigned long long mk = nt_mask;
            if (e + 1 < tl.total)
                listed_tile(tl, e + 1, nt_ti, nt_tj, nt_mask);
            const int i = ti * kTileEdge + li;
            const int j = tj * kTileEdge + lj;
            int zoff = 0;
            asm volatile("" : "+v"(zoff));
            n_direct += __popcll(mk);
            if ((mk >> lane) & 1ull) {
                const KQ r = kq_setup<B3>(a, slot, iq, qmx, qmy, i, j, (unsigned)i * (unsigned)a.Ly,
                                          eps, mu_up, mu_dn, cqx, sqx, cqy, sqy);
                // R^2 >= 1e-300 keeps the reciprocal square root finite
                f64_steps<TD>(acc, r.s2 + 1e-300, r.m, r.eta2,
                              mirror_weight(kr, i, j, a.Lx, a.Ly), T, kGStep * invT, cutT,
                              d2s[wave] + zoff, gt);
            }
        }
        // lane t << SHIFT holds Delta t
        wave_reduce_halving<TD>(acc, lane);
        constexpr int SHIFT = 6 - Log2<TD>::value;
        if ((lane & ((1 << SHIFT) - 1)) == 0)
            a.part[((size_t)bz * a.n_chunks + chunk) * a.n_delta_pad + dtile * TD +
                   (lane >> SHIFT)] = acc[0];
    }
    if (args.count && lane == 0 && n_direct)
        atomicAdd(args.count, (unsigned long long)n_direct * TD);
}

template <int TD, bool B3>
static hipError_t launch_persistent_f64_hot(const SweepArgs &a, hipStream_t s)
{
    const unsigned long long units =
        (unsigned long long)a.n_chunks * a.n_dtiles * (unsigned long long)a.n_rows;
    constexpr int threads = 64 * hot_waves<B3>();
    const int blocks =
        persistent_blocks(sweep_f64_hot_kernel<TD, B3>, threads, units, a.blocks_per_cu);
    if (blocks <= 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((sweep_f64_hot_kernel<TD, B3>), dim3(blocks), dim3(threads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sweep_f64(const SweepArgs &a, int td, int n_dtiles, int G, bool b3,
                            bool hot, hipStream_t s)
{
    SweepArgs p = a;
    p.n_dtiles = n_dtiles;
    p.n_rows = a.nbq * G;
    if (hot) {
        if (td == 16 && !b3)
            return launch_persistent_f64_hot<16, false>(p, s);
        if (td == 32 && !b3)
            return launch_persistent_f64_hot<32, false>(p, s);
        if (td == 16)
            return launch_persistent_f64_hot<16, true>(p, s);
        if (td == 32)
            return launch_persistent_f64_hot<32, true>(p, s);
        return hipErrorInvalidValue;
    }
    if (td == 16 && !b3)
        return launch_persistent<16, false, false>(p, s);
    if (td == 32 && !b3)
        return launch_persistent<32, false, false>(p, s);
    if (td == 16)
        return launch_persistent<16, true, false>(p, s);
    if (td == 32)
        return launch_persistent<32, true, false>(p, s);
    return hipErrorInvalidValue;
}

// The FP32-compensated per-Delta sweep for points at T >= kInPlaceT, where
// almost no marked term is zero or on a tile series over a Delta tile: every
// marked lane runs the FP32 loop in place, without classification or queue.
// Persistent like sweep_kernel, with the same work queues and units, one
// unit per wave at a time.  Two-band: 5
// waves/SIMD (a few spills outside the Delta loop beat the 4 waves its
// registers would otherwise give); three-band: 4.
template <int TD, bool B3>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(B3 ? 4 : 5)))
void sweep_f32c_hot_kernel(const SweepArgs args)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // per wave: Delta^2 of the unit's tile as an unevaluated FP32 pair
    // hi + lo (rounding Delta^2 to one float would shift every momentum's
    // term at that Delta the same way, a systematic 6e-8 that the sum would
    // not average out)
    __shared__ float2 d2s[4][TD + 1];
    __shared__ float4 gt32[kG32N];
    for (int n = threadIdx.x; n < kG32N; n += kBlock)
        gt32[n] = args.gtab32[n];
    __syncthreads();
    int n_direct = 0;
    const int li = lane >> 3, lj = lane & 7;
    const int nq = sweep_queues(args);
    const int q = (int)(blockIdx.x % (unsigned)nq);
    for (;;) {
        ConstArgs ap = (ConstArgs)__builtin_amdgcn_kernarg_segment_ptr();
        asm volatile("" : "+s"(ap));
        const SweepArgs &a = *(const SweepArgs *)ap;   // the argument, reloaded per unit
        int3 un = make_int3(0, 0, -1);
        if (lane == 0)
            un = take_unit(a, q, nq);
        const int bz = __builtin_amdgcn_readfirstlane(un.z);
        if (bz < 0)
            break;
        const int chunk = __builtin_amdgcn_readfirstlane(un.x);
        const int dtile = __builtin_amdgcn_readfirstlane(un.y);
        const int g = bz / a.nbq;                  // point within the batch
        const int bq = bz - g * a.nbq;
        const int slot = bq / a.n_q;
        const int iq = bq - slot * a.n_q;
        const double eps = slot ? a.eps[1] : a.eps[0];
        const double qy = a.q[2 * iq + 1];
        const KRange kr = k_range(a, a.q[2 * iq], qy, chunk);
        const PointRec pt = a.pts[g];
        const double mu_up = a.mu + pt.h;
        const double mu_dn = a.mu - pt.h;
        const double T = pt.T;
        const double invT = T > 0.0 ? 1.0 / T : 0.0;

        const double cqx = a.qtrig[kQTrig * iq], sqx = a.qtrig[kQTrig * iq + 1];
        const double cqy = a.qtrig[kQTrig * iq + 2], sqy = a.qtrig[kQTrig * iq + 3];
        const int qmx = __builtin_amdgcn_readfirstlane(a.qlat[2 * iq]);
        const int qmy = __builtin_amdgcn_readfirstlane(a.qlat[2 * iq + 1]);

        if (lane <= TD) {
            const double v = a.d2[dtile * TD + (lane < TD ? lane : TD - 1)];
            const float hi = (float)v;
            d2s[wave][lane] = make_float2(hi, (float)(v - (double)hi));
        }
        // the wave's LDS writes above are visible to all of its lanes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        float acc[TD];
#pragma unroll
        for (int t = 0; t < TD; ++t)
            acc[t] = 0.0f;
        const float Tf = (float)T, invTs = (float)(kG32Step * invT), cutTf = kCutFp32 * Tf;

        const TileList tl = tile_list(a, bz, chunk);
        // the next entry of the walk is fetched one tile ahead
        int e = 0;
        int nt_ti = 0, nt_tj = 0;
        unsigned long long nt_mask = 0ull;
        if (e < tl.total)
            listed_tile(tl, e, nt_ti, nt_tj, nt_mask);
        for (; e < tl.total; ++e) {
            const int ti = nt_ti, tj = nt_tj;
            const unsigned long long mk = nt_mask;
            if (e + 1 < tl.total)
                listed_tile(tl, e + 1, nt_ti, nt_tj, nt_mask);
            const int i = ti * kTileEdge + li;
            const int j = tj * kTileEdge + lj;
            int zoff = 0;
            asm volatile("" : "+v"(zoff));
            const float2 *dp = d2s[wave] + zoff;
            n_direct += __popcll(mk);
            if ((mk >> lane) & 1ull) {
                const KQ q64 = kq_setup<B3>(a, slot, iq, qmx, qmy, i, j,
                                            (unsigned)(ti * kTileEdge) * (unsigned)a.Ly +
                                                (unsigned)li * (unsigned)a.Ly,
                                            eps, mu_up, mu_dn, cqx, sqx, cqy, sqy);
                const KQf r = kq_setup_f32(q64, T, invT, gt32);
                const float wf = (float)mirror_weight(kr, i, j, a.Lx, a.Ly);
                const bool pos = r.A0 >= 0.0f;
                float2 dcur = dp[0];
#pragma unroll
                for (int t = 0; t < TD; ++t) {
                    const float2 dnext = dp[t + 1];
                    float g2 = fmaf(dcur.x, r.eta2, dcur.y * r.eta2);
                    float R = __builtin_amdgcn_sqrtf(r.s2 + g2);
                    float del = g2 * __builtin_amdgcn_rcpf(R + r.as);
                    float x = r.A0 + del;
                    float piece = pos ? del : fmaxf(x, 0.0f);
                    float ax = fabsf(x);
                    if (ax < cutTf)
                        piece += fmaf(Tf, thermal_log_f32(ax, R + r.m, invTs, cutTf, gt32), -r.P0);
                    else
                        piece -= r.P0;
                    acc[t] = fmaf(wf, piece, acc[t]);
                    dcur = dnext;
                }
            }
        }

        // Delta = 0 slots: the FP32 difference is zero by construction
        double accd[TD];
#pragma unroll
        for (int t = 0; t < TD; ++t)
            accd[t] = (d2s[wave][t].x == 0.0f && d2s[wave][t].y == 0.0f) ? 0.0
                                                                         : (double)acc[t];
        // lane t << SHIFT holds Delta t
        wave_reduce_halving<TD>(accd, lane);
        constexpr int SHIFT = 6 - Log2<TD>::value;
        if ((lane & ((1 << SHIFT) - 1)) == 0)
            a.part[((size_t)bz * a.n_chunks + chunk) * a.n_delta_pad + dtile * TD +
                   (lane >> SHIFT)] = accd[0];
    }
    if (args.count && lane == 0 && n_direct)
        atomicAdd(args.count, (unsigned long long)n_direct * TD);
}

template <int TD, bool B3>
static hipError_t launch_persistent_f32c_hot(const SweepArgs &a, hipStream_t s)
{
    const unsigned long long units =
        (unsigned long long)a.n_chunks * a.n_dtiles * (unsigned long long)a.n_rows;
    const int blocks =
        persistent_blocks(sweep_f32c_hot_kernel<TD, B3>, kBlock, units, a.blocks_per_cu);
    if (blocks <= 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((sweep_f32c_hot_kernel<TD, B3>), dim3(blocks), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sweep_f32c(const SweepArgs &a, int td, int n_dtiles, int G, bool b3,
                             bool hot, hipStream_t s)
{
    SweepArgs p = a;
    p.n_dtiles = n_dtiles;
    p.n_rows = a.nbq * G;
    if (hot) {
        if (td == 16 && !b3)
            return launch_persistent_f32c_hot<16, false>(p, s);
        if (td == 32 && !b3)
            return launch_persistent_f32c_hot<32, false>(p, s);
        if (td == 16)
            return launch_persistent_f32c_hot<16, true>(p, s);
        if (td == 32)
            return launch_persistent_f32c_hot<32, true>(p, s);
        return hipErrorInvalidValue;
    }
    if (td == 16 && !b3)
        return launch_persistent<16, false, true>(p, s);
    if (td == 32 && !b3)
        return launch_persistent<32, false, true>(p, s);
    if (td == 16)
        return launch_persistent<16, true, true>(p, s);
    if (td == 32)
        return launch_persistent<32, true, true>(p, s);
    return hipErrorInvalidValue;
}

// ------------------------------------------------- pair susceptibility

// Summand of the static Cooper-pair susceptibility of App. C,
// F = (1 - f(E1) - f(E2)) / (E1 + E2), f the Fermi function.  With
// a = |E1|/2T, b = |E2|/2T and u = (E1 + E2)/2T, |u| <= a + b, and
// tanh x1 + tanh x2 = sinh(u) sech x1 sech x2,
//   F = (e^{|u|-a-b} - e^{-|u|-a-b}) / (2|u|) / (T (1 + e^{-2a}) (1 + e^{-2b})),
// every exponent <= 0; for |u| < 1/2 the difference is e^{-|u|-a-b}
// expm1(2|u|) (the limit |u| -> 0 is e^{-a-b}).  T = 0: the step function,
// (sgn E1 + sgn E2) / (2 (E1 + E2)), 0 where E1 + E2 = 0.
__device__ __forceinline__ double pair_summand(double E1, double E2, double T, double invT)
{
    if (T == 0.0) {
        const double S = E1 + E2;
        if (S == 0.0)
            return 0.0;
        const double sg = (double)((E1 > 0.0) - (E1 < 0.0)) + (double)((E2 > 0.0) - (E2 < 0.0));
        return sg / (2.0 * S);
    }
    const double a = 0.5 * fabs(E1) * invT;
    const double b = 0.5 * fabs(E2) * invT;
    const double au = fabs(0.5 * (E1 + E2) * invT);
    double num;
    if (au < 0.5)
        num = au == 0.0 ? exp(-a - b) : exp(-au - a - b) * (expm1(2.0 * au) / (2.0 * au));
    else
        num = (exp(au - a - b) - exp(-au - a - b)) / (2.0 * au);
    return num / (T * (1.0 + exp(-2.0 * a)) * (1.0 + exp(-2.0 * b)));
}

// chi_{eps eps'}(q) partial sums over one chunk of momenta:
//   sum_k eta(-k-q)^2 F(E_eps(k) - mu - h, E_eps'(-k-q) - mu + h),
// eta = 4 cos kx cos ky (App. C).  E(-p) = E(p) for both models, so the
// partner energy is taken at p = k + q (angle addition; three-band: table
// index of k + q on the lattice, else diagonalised).
template <bool B3>
__global__ __launch_bounds__(kBlock) void chi_kernel(const ChiArgs a)
{
    const int pq = blockIdx.x;                 // (pair, q)
    const int chunk = blockIdx.y;
    const int pair = pq / a.n_q;
    const int iq = pq - pair * a.n_q;
    const int ia = pair / a.nb, ib = pair - (pair / a.nb) * a.nb;
    const double cqx = a.qtrig[kQTrig * iq], sqx = a.qtrig[kQTrig * iq + 1];
    const double cqy = a.qtrig[kQTrig * iq + 2], sqy = a.qtrig[kQTrig * iq + 3];
    // three-band: lattice index of q, read once (-1 off the lattice)
    int qmx = -1, qmy = -1;
    if constexpr (B3) {
        qmx = __builtin_amdgcn_readfirstlane(a.qlat[2 * iq]);
        qmy = __builtin_amdgcn_readfirstlane(a.qlat[2 * iq + 1]);
    }
    const double invT = a.T > 0.0 ? 1.0 / a.T : 0.0;
    const double mu_up = a.mu + a.h, mu_dn = a.mu - a.h;
    const double *cxt = a.trig, *sxt = a.trig + a.Lx;
    const double *cyt = a.trig + 2 * a.Lx, *syt = cyt + a.Ly;
    const long long n = (long long)a.Lx * a.Ly;
    const long long k0 = (long long)chunk * a.span;
    const long long k1 = k0 + a.span < n ? k0 + a.span : n;
    double s = 0.0, c = 0.0;
    for (long long k = k0 + threadIdx.x; k < k1; k += kBlock) {
        const int i = (int)(k / a.Ly);
        const int j = (int)(k - (long long)i * a.Ly);
        const double cx = cxt[i], sx = sxt[i], cy = cyt[j], sy = syt[j];
        // p = k + q
        const double cpx = fma(cx, cqx, -(sx * sqx));
        const double spx = fma(sx, cqx, cx * sqx);
        const double cpy = fma(cy, cqy, -(sy * sqy));
        const double spy = fma(sy, cqy, cy * sqy);
        double E1, E2;
        if constexpr (!B3) {
            E1 = band_energy(a.hop, a.eps[ia], cx, sx, cy, sy);
            E2 = band_energy(a.hop, a.eps[ib], cpx, spx, cpy, spy);
        } else {
            const double *Ea = a.etab + (size_t)a.band3[ia] * n;
            const double *Eb = a.etab + (size_t)a.band3[ib] * n;
            E1 = Ea[k];
            if (qmx >= 0 && qmy >= 0) {
                int ii = i + qmx;
                ii -= ii >= a.Lx ? a.Lx : 0;
                int jj = j + qmy;
                jj -= jj >= a.Ly ? a.Ly : 0;
                E2 = Eb[(size_t)ii * a.Ly + jj];
            } else {
                double ev[3];
                eig3(a.hop3, cpx, spx, cpy, spy, (cpx - spx) * (cpx + spx),
                     (cpy - spy) * (cpy + spy), ev);
                const int bb = a.band3[ib];
                E2 = bb == 0 ? ev[0] : (bb == 1 ? ev[1] : ev[2]);
            }
        }
        const double eta = 4.0 * cpx * cpy;
        neumaier(s, c, eta * eta * pair_summand(E1 - mu_up, E2 - mu_dn, a.T, invT));
    }
    __shared__ double red[4];
    const double v = wave_sum(s + c);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        a.part[(size_t)pq * a.n_chunks + chunk] = ((red[0] + red[1]) + red[2]) + red[3];
}

hipError_t launch_chi(const ChiArgs &a, bool b3, hipStream_t s)
{
    const dim3 grid(a.nb * a.nb * a.n_q, a.n_chunks);
    if (b3)
        hipLaunchKernelGGL(chi_kernel<true>, grid, dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(chi_kernel<false>, grid, dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// Fixed-order Neumaier sum of the chunk partials of every (pair, q), / N.
__global__ void chi_finish_kernel(const ChiFinishArgs a)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.n_pairs_q)
        return;
    a.out[t] = ordered_sum(a.part + (size_t)t * a.n_chunks, 1, a.n_chunks) * a.inv_n;
}

hipError_t launch_chi_finish(const ChiFinishArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(chi_finish_kernel, dim3((a.n_pairs_q + kBlock - 1) / kBlock),
                       dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ rows

__device__ __forceinline__ double nan_min(double x, double y)
{
    if (x != x)
        return y;
    if (y != y)
        return x;
    return y < x ? y : x;
}

// Block-wide min over 256 threads (NaN ignored unless all are NaN).
__device__ double block_nan_min(double v, double *sh)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v = nan_min(v, __shfl_xor(v, off, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
        sh[wave] = v;
    __syncthreads();
    return nan_min(nan_min(sh[0], sh[1]), nan_min(sh[2], sh[3]));
}

__device__ int block_int_min(int v, int *sh)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        int o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
        sh[wave] = v;
    __syncthreads();
    int r = sh[0];
    for (int w = 1; w < 4; ++w)
        r = sh[w] < r ? sh[w] : r;
    return r;
}

// tie threshold, rounded exactly as written (no fused multiply-add)
__device__ __forceinline__ double tie_threshold(double best, double tie_rel)
{
    return __dadd_rn(best, __dmul_rn(tie_rel, fabs(best)));
}

// One workgroup per (band slot, Q) row of one point: fixed-order chunk sums,
// the epilogue of Eq. (5) (+ N (-2 Delta^2 / V)), and the row search of
// Algorithm 1 ("find and save Delta for this q").
// binomial(1/2, n), n = 0..kMomentSlots-1, by the recurrence
// c_{n+1} = c_n (1/2 - n) / (n + 1), evaluated at compile time
struct HalfBinomial {
    double c[kMomentSlots];
    constexpr HalfBinomial() : c()
    {
        double v = 1.0;
        for (int n = 0; n < kMomentSlots; ++n) {
            c[n] = v;
            v = v * (0.5 - n) / (n + 1);
        }
    }
};
__constant__ constexpr HalfBinomial kHalfBinomial{};
static_assert(kTileSlots <= kMomentSlots, "tile series uses the same coefficients");

__global__ __launch_bounds__(kBlock) void rows_kernel(const RowArgs r)
{
    const int bq = blockIdx.x;
    const int g = blockIdx.y;
    const int slot = bq / r.n_q;
    const int iq = bq - slot * r.n_q;
    const size_t row = (size_t)g * r.nbq + bq;       // partial row of the batch
    const size_t orow = (size_t)r.pts[g].out * r.nbq + bq;  // output row
    const int t = threadIdx.x;
    __shared__ double sh_base;
    __shared__ double shd[4];
    __shared__ int shi[4];
    __shared__ double sh_mom[kMomentSlots];   // C0, c_n M_n
    // tile series of the queued sweep, per Delta tile: c_n times the
    // fixed-order chunk sums of its moments, and the tile centre, a batch of
    // kTileBatch tiles at a time
    __shared__ double sh_tm[kTileBatch][kTileSlots];
    __shared__ double sh_tc[kTileBatch];
    const double x0 = *r.d2c;
    // 0 * q is 0 for finite q and NaN for NaN q: a NaN momentum poisons the row
    const double qpoison = 0.0 * r.q[2 * iq] + 0.0 * r.q[2 * iq + 1];
    const double V = r.Vs[slot];
    double *out = r.omega + orow * r.n_delta;
    const double *pp = r.part + row * r.n_chunks * r.n_delta_pad;
    const double *mp = r.mpart + row * r.n_chunks * kMomentSlots;
    double best = __longlong_as_double(0x7ff8000000000000LL);
    for (int b0 = 0; b0 < r.n_dtiles; b0 += kTileBatch) {
        const int nbt = min(kTileBatch, r.n_dtiles - b0);
        const int id_end = min(r.n_delta, (b0 + nbt) * r.td);
        const int id0 = b0 * r.td + t;   // this thread's first Delta of the batch
        // Every thread sums the chunks of its first Delta together with one
        // other fixed-order chunk sum: in the first batch the series moments
        // and the base term, then the tile moments of the batch.
        const int nfix = b0 == 0 ? kMomentSlots + 1 : 0;
        const int ntm = r.tpart ? nbt * kTileSlots : 0;
        const double *p2 = nullptr;
        size_t s2 = 0;
        if (t < nfix) {
            p2 = t < kMomentSlots ? mp + t : r.base_part + row * r.n_chunks;
            s2 = t < kMomentSlots ? kMomentSlots : 1;
        } else if (t - nfix < ntm) {
            const int u = t - nfix;
            p2 = r.tpart + (row * r.n_chunks * r.n_dtiles + b0 + u / kTileSlots) * kTileSlots +
                 u % kTileSlots;
            s2 = (size_t)r.n_dtiles * kTileSlots;
        }
        double sp0 = 0.0, v2 = 0.0;
        ordered_sum2(id0 < id_end ? pp + id0 : nullptr, r.n_delta_pad, p2, s2, r.n_chunks, sp0,
                     v2);
        if (t < nfix) {
            // moments are positive terms; times binomial(1/2, n) (c_0 = 1: C0 as it is)
            if (t < kMomentSlots)
                sh_mom[t] = t == 0 ? v2 : kHalfBinomial.c[t] * v2;
            else
                sh_base = v2;
        } else if (t - nfix < ntm) {
            const int u = t - nfix;
            sh_tm[u / kTileSlots][u % kTileSlots] = kHalfBinomial.c[u % kTileSlots] * v2;
        }
        // tile moments beyond one per thread
        for (int u = kBlock - nfix + t; u < ntm; u += kBlock) {
            const double m =
                ordered_sum(r.tpart + (row * r.n_chunks * r.n_dtiles + b0 + u / kTileSlots) *
                                          kTileSlots + u % kTileSlots,
                            (size_t)r.n_dtiles * kTileSlots, r.n_chunks);
            sh_tm[u / kTileSlots][u % kTileSlots] = kHalfBinomial.c[u % kTileSlots] * m;
        }
        if (r.tpart) {
            for (int u = t; u < nbt; u += kBlock) {
                // same arithmetic as the sweep's tile range
                const double *dt2 = r.d2 + (size_t)(b0 + u) * r.td;
                double lo = dt2[0], hi = dt2[0];
                for (int k = 1; k < r.td; ++k) {
                    lo = fmin(lo, dt2[k]);
                    hi = fmax(hi, dt2[k]);
                }
                sh_tc[u] = 0.5 * (lo + hi);
            }
        }
        __syncthreads();
        const double base = sh_base;
        for (int id = id0; id < id_end; id += kBlock) {
            const double sp = id == id0 ? sp0 : ordered_sum(pp + id, r.n_delta_pad, r.n_chunks);
            const double D = r.delta[id];
            // series part: C0 + sum_n c_n M_n (Delta^2 - x0)^n by Horner
            const double x = D * D - x0;
            double ser = sh_mom[kSeriesTerms];
            for (int n = kSeriesTerms - 1; n >= 1; --n)
                ser = fma(ser, x, sh_mom[n]);
            ser = fma(ser, x, sh_mom[0]);
            double sp_t = 0.0;
            if (r.tpart && !(r.zero_d0 && D * D == 0.0)) {
                const int u = id / r.td - b0;
                const double z = D * D - sh_tc[u];
                double ts = sh_tm[u][kTileSlots - 1];
                for (int n = kTileSlots - 2; n >= 0; --n)
                    ts = fma(ts, z, sh_tm[u][n]);
                sp_t = ts;
            }
            const double om = (base - ((sp + sp_t) + ser)) + r.n_k * (-2.0 * D * D / V) + qpoison;
            out[id] = om;
            best = nan_min(best, om);
        }
        // the next batch rewrites the shared tables
        __syncthreads();
    }
    best = block_nan_min(best, shd);
    if (t == 0)
        r.rowmin[orow] = best;
    if (!r.row_idx)
        return;
    int pick = 0x7fffffff;
    if (best == best) {
        const double thr = tie_threshold(best, r.tie_rel);
        for (int id = threadIdx.x; id < r.n_delta; id += kBlock) {
            const double v = out[id];
            if (v <= thr) {
                pick = id;
                break;
            }
        }
    }
    pick = block_int_min(pick, shi);
    if (threadIdx.x == 0)
        r.row_idx[orow] = pick == 0x7fffffff ? -1 : pick;
}

hipError_t launch_rows(const RowArgs &a, int G, hipStream_t s)
{
    hipLaunchKernelGGL(rows_kernel, dim3(a.nbq, G), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ argmin

// One workgroup per (point, band) set: global search of Algorithm 1 with the
// tie rule (lexicographically smallest (iDelta, iq) within the tie band).
// The global minimum is the minimum of the row minima rows_kernel stored;
// only rows whose minimum lies within the tie band can hold the pick.  The
// first 256 keys (key = iDelta n_q + iq) are checked at once, which settles
// the common tie of the Delta = 0 row over lattice Q; otherwise each wave
// scans its rows within the tie band 64 Delta at a time from the start, the
// first Delta at or below the threshold giving the row's smallest key.
__global__ __launch_bounds__(kBlock) void argmin_kernel(const ArgminArgs a)
{
    const size_t set = blockIdx.x;
    const int n = a.n_q * a.n_delta;
    const double *g = a.omega + set * (size_t)n;
    const double *rm = a.rowmin + set * (size_t)a.n_q;
    __shared__ double shd[4];
    __shared__ int shi[4];
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    double best = nan;
    for (int iq = threadIdx.x; iq < a.n_q; iq += kBlock)
        best = nan_min(best, rm[iq]);
    best = block_nan_min(best, shd);
    int key = 0x7fffffff;
    if (best == best) {
        const double thr = tie_threshold(best, a.tie_rel);
        const int k = (int)threadIdx.x;
        bool hit = false;
        if (k < n) {
            const int id = k / a.n_q;
            const int iq = k - id * a.n_q;
            hit = rm[iq] <= thr && g[(size_t)iq * a.n_delta + id] <= thr;
        }
        key = block_int_min(hit ? k : 0x7fffffff, shi);
        if (key == 0x7fffffff) {
            const int lane = threadIdx.x & 63;
            const int wave = threadIdx.x >> 6;
            for (int iq = wave; iq < a.n_q; iq += kBlock / 64) {
                if (!(rm[iq] <= thr))
                    continue;
                for (int d0 = 0; d0 < a.n_delta; d0 += 64) {
                    const int id = d0 + lane;
                    const bool h = id < a.n_delta && g[(size_t)iq * a.n_delta + id] <= thr;
                    const unsigned long long b = __ballot(h);
                    if (b != 0ull) {
                        const int kk = (d0 + __builtin_ctzll(b)) * a.n_q + iq;
                        key = kk < key ? kk : key;
                        break;
                    }
                }
            }
            key = block_int_min(key, shi);
        }
    }
    if (threadIdx.x == 0) {
        if (key == 0x7fffffff) {
            a.idx[2 * set] = -1;
            a.idx[2 * set + 1] = -1;
            a.omin[set] = nan;
        } else {
            const int id = key / a.n_q;
            const int iq = key - id * a.n_q;
            a.idx[2 * set] = id;
            a.idx[2 * set + 1] = iq;
            a.omin[set] = g[(size_t)iq * a.n_delta + id];
        }
    }
}

hipError_t launch_argmin(const ArgminArgs &a, int n_set, hipStream_t s)
{
    hipLaunchKernelGGL(argmin_kernel, dim3(n_set), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------ FP64 check of the FP32 search

__device__ int block_int_sum(int v, int *sh)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
        sh[wave] = v;
    __syncthreads();
    return ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// One workgroup per (point, band) set of the batch: the candidate threshold
// and the candidate cells with Delta != 0 (see VerifyArgs).  Where more than
// kVerifyMax cells lie under the threshold, the threshold is lowered by
// bisection until at most kVerifyMax do (the lowest-valued cells stay), and
// cells are taken in key order (iDelta, iq) up to the capacity.
// The cells under the threshold are gathered into LDS in one pass over the
// rows whose minimum lies under it (no other row holds such a cell), and the
// bisection counts there; only if more than kCandCap cells qualify does it
// count over the whole grid.  Both give the same threshold and cells.
constexpr int kCandCap = 2048;
__global__ __launch_bounds__(kBlock) void verify_cand_kernel(const VerifyArgs v)
{
    const int sl = blockIdx.x;
    const int g = sl / v.nb;
    const int slot = sl - g * v.nb;
    const size_t oset = (size_t)v.sw.pts[g].out * v.nb + slot;
    const int ncell = v.n_q * v.n_delta;
    const double *G = v.grid + oset * (size_t)ncell;
    const double *rm = v.rowmin + oset * (size_t)v.n_q;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ double shd[4];
    __shared__ int shi[4];
    __shared__ double cv[kCandCap];   // values of the gathered cells
    __shared__ int ck[kCandCap];      // their keys iDelta n_q + iq
    __shared__ int n_gath;
    __shared__ int sel[kVerifyMax];   // keys of the chosen cells
    __shared__ int n_sel;
    double best = __longlong_as_double(0x7ff8000000000000LL);
    for (int iq = threadIdx.x; iq < v.n_q; iq += kBlock)
        best = nan_min(best, rm[iq]);
    best = block_nan_min(best, shd);
    if (!(best == best)) {
        if (threadIdx.x == 0) {
            v.cnt[sl] = 0;
            v.thr[sl] = best;
        }
        return;
    }
    const double ab = fabs(best);
    const double floor_abs =
        v.n_k < (double)kFp32FloorSites ? ldexp(v.n_k * sqrt(v.d2c[0] + v.d2c[1]), -20) : 0.0;
    const double e = kFp32RelBound * ab + floor_abs;
    // Delta = 0 cells hold FP64 values (the FP32 difference vanishes there):
    // the lowest of them, from up to 8 such columns
    __shared__ int zc[8];
    __shared__ int nzc;
    if (threadIdx.x == 0)
        nzc = 0;
    __syncthreads();
    for (int id = threadIdx.x; id < v.n_delta; id += kBlock) {
        const double D = v.delta[id];
        if (D * D == 0.0) {
            const int at = atomicAdd(&nzc, 1);
            if (at < 8)
                zc[at] = id;
        }
    }
    __syncthreads();
    const int nz = nzc;
    double zb = __longlong_as_double(0x7ff8000000000000LL);
    if (nz <= 8)
        for (int k = 0; k < nz; ++k)
            for (int iq = threadIdx.x; iq < v.n_q; iq += kBlock)
                zb = nan_min(zb, G[(size_t)iq * v.n_delta + zc[k]]);
    zb = block_nan_min(zb, shd);
    // a cell in the FP64 tie band has an FP32 value at most best + 2e +
    // tie_rel |best| (to first order; the factor covers the second); e
    // instead of 2e where the lowest value is an FP64 one (at Delta = 0)
    const double we = (nz <= 8 && zb <= best) ? 1.0 : 2.0;
    const double thr = best + (we * e + v.tie_rel * ab) * (1.0 + 1e-6);

    // gather: one wave per row whose minimum is under the threshold
    if (threadIdx.x == 0)
        n_gath = 0;
    __syncthreads();
    for (int iq = wave; iq < v.n_q; iq += kBlock / 64) {
        if (!(rm[iq] <= thr))
            continue;
        for (int id = lane; id - lane < v.n_delta; id += 64) {
            bool take = false;
            double x = 0.0;
            if (id < v.n_delta) {
                const double D = v.delta[id];
                x = G[(size_t)iq * v.n_delta + id];
                take = D * D != 0.0 && x <= thr;
            }
            const unsigned long long b = __ballot(take);
            if (b) {
                int base = 0;
                if (lane == 0)
                    base = atomicAdd(&n_gath, __popcll(b));
                base = __shfl(base, 0, 64);
                const int at = base + (int)__popcll(b & ((1ull << lane) - 1ull));
                if (take && at < kCandCap) {
                    cv[at] = x;
                    ck[at] = id * v.n_q + iq;
                }
            }
        }
    }
    __syncthreads();
    const int ng = n_gath;
    const bool in_lds = ng <= kCandCap;
    auto count_le = [&](double t) {
        int c = 0;
        if (in_lds) {
            for (int k = threadIdx.x; k < ng; k += kBlock)
                c += cv[k] <= t ? 1 : 0;
        } else {
            for (int cell = threadIdx.x; cell < ncell; cell += kBlock) {
                const int iq = cell / v.n_delta;
                const double D = v.delta[cell - iq * v.n_delta];
                c += (D * D != 0.0 && G[cell] <= t) ? 1 : 0;
            }
        }
        return block_int_sum(c, shi);
    };
    double t = thr;
    if (ng > kVerifyMax) {
        double lo = best, hi = thr;
        for (int it = 0; it < 64 && lo < hi; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi)
                break;
            if (count_le(mid) <= kVerifyMax)
                lo = mid;
            else
                hi = mid;
        }
        t = lo;
    }
    int total = 0;
    // more than kVerifyMax cells at t itself (exact ties) take the scan of
    // the whole grid in key order below
    if (in_lds && count_le(t) <= kVerifyMax) {
        // at most kVerifyMax gathered cells lie under t: their keys, then
        // each one's place in key order
        if (threadIdx.x == 0)
            n_sel = 0;
        __syncthreads();
        for (int k = threadIdx.x; k < ng; k += kBlock) {
            if (cv[k] <= t) {
                const int at = atomicAdd(&n_sel, 1);
                if (at < kVerifyMax)
                    sel[at] = ck[k];
            }
        }
        __syncthreads();
        total = n_sel < kVerifyMax ? n_sel : kVerifyMax;
        if (threadIdx.x < total) {
            const int key = sel[threadIdx.x];
            int pos = 0;
            for (int k = 0; k < total; ++k)
                pos += sel[k] < key ? 1 : 0;
            const int iq = key % v.n_q;
            v.cand[(size_t)sl * kVerifyMax + pos] = iq * v.n_delta + key / v.n_q;
        }
    } else {
        // cells under t in key order (iDelta n_q + iq), up to the capacity
        __shared__ int wcnt[4];
        for (int k0 = 0; k0 < ncell && total < kVerifyMax; k0 += kBlock) {
            const int key = k0 + threadIdx.x;
            int cell = 0;
            bool take = false;
            if (key < ncell) {
                const int id = key / v.n_q;
                const int iq = key - id * v.n_q;
                const double D = v.delta[id];
                cell = iq * v.n_delta + id;
                take = D * D != 0.0 && G[cell] <= t;
            }
            const unsigned long long b = __ballot(take);
            __syncthreads();
            if (lane == 0)
                wcnt[wave] = __popcll(b);
            __syncthreads();
            int at = total;
            for (int w = 0; w < wave; ++w)
                at += wcnt[w];
            at += __popcll(b & ((1ull << lane) - 1ull));
            if (take && at < kVerifyMax)
                v.cand[(size_t)sl * kVerifyMax + at] = cell;
            total += ((wcnt[0] + wcnt[1]) + wcnt[2]) + wcnt[3];
        }
        total = total < kVerifyMax ? total : kVerifyMax;
    }
    if (threadIdx.x == 0) {
        v.cnt[sl] = total;
        v.thr[sl] = thr;
    }
}

// FP64 sum over one momentum chunk of the Eq. (5) terms of one candidate:
// units (set, candidate, chunk), grid-stride over all of them; units of
// empty candidate slots are skipped.  Each term is evaluated in full (no
// series), with the FP64 sweep's arithmetic for its Delta-dependent part:
// the Delta-independent part minus max(R - |d|, 0) + T [G(|R - |d||/T) +
// G((R + |d|)/T)], G(a) = ln(1 + e^-a) from the thermal table and dropped
// beyond the cut 30 T.  Pair momenta on an axis sum the mirror-folded zone
// (qy = 0: ky indices 0..Ly/2, weight 2 where the mirror is another index;
// likewise qx = 0), as the sweep does: E and eta^2 are even in each
// component for both models and both form factors.
template <bool B3>
__global__ __launch_bounds__(kBlock) void verify_eval_kernel(const VerifyArgs v, int n_units)
{
    const SweepArgs &a = v.sw;
    __shared__ double red[4];
    for (int u = blockIdx.x; u < n_units; u += gridDim.x) {
        const int chunk = u % v.n_vchunks;
        const int ks = u / v.n_vchunks;
        const int sl = ks / kVerifyMax;
        const int kc = ks - sl * kVerifyMax;
        if (kc >= v.cnt[sl])
            continue;
        const int cell = v.cand[(size_t)sl * kVerifyMax + kc];
        const int iq = cell / v.n_delta;
        const int id = cell - iq * v.n_delta;
        const int g = sl / v.nb;
        const int slot = sl - g * v.nb;
        const double eps = slot ? a.eps[1] : a.eps[0];
        const PointRec pt = a.pts[g];
        const double mu_up = a.mu + pt.h, mu_dn = a.mu - pt.h;
        const double T = pt.T;
        const double invTs = T > 0.0 ? kGStep / T : 0.0;
        const double cutT = kCutFp64 * T;
        const double D = v.delta[id];
        const double D2 = D * D;
        const double cqx = a.qtrig[kQTrig * iq], sqx = a.qtrig[kQTrig * iq + 1];
        const double cqy = a.qtrig[kQTrig * iq + 2], sqy = a.qtrig[kQTrig * iq + 3];
        const int qmx = __builtin_amdgcn_readfirstlane(a.qlat[2 * iq]);
        const int qmy = __builtin_amdgcn_readfirstlane(a.qlat[2 * iq + 1]);
        const bool fx = a.q[2 * iq] == 0.0, fy = a.q[2 * iq + 1] == 0.0;
        const int nx = fx ? a.Lx / 2 + 1 : a.Lx;
        const int ny = fy ? a.Ly / 2 + 1 : a.Ly;
        const long long n = (long long)nx * ny;
        const long long span = (n + v.n_vchunks - 1) / v.n_vchunks;
        const long long k0 = (long long)chunk * span;
        const long long k1 = k0 + span < n ? k0 + span : n;
        double s = 0.0, c = 0.0;
        for (long long kk = k0 + threadIdx.x; kk < k1; kk += kBlock) {
            const int i = (int)(kk / ny);
            const int j = (int)(kk - (long long)i * ny);
            const double w = ((fx && i != 0 && 2 * i != a.Lx) ? 2.0 : 1.0) *
                             ((fy && j != 0 && 2 * j != a.Ly) ? 2.0 : 1.0);
            const KQ r = kq_setup<B3>(a, slot, iq, qmx, qmy, i, j, (unsigned)i * (unsigned)a.Ly,
                                      eps, mu_up, mu_dn, cqx, sqx, cqy, sqy);
            const double R = sqrt_rn(fma(D2, r.eta2, r.s2));
            const double x = R - r.m;
            double P = fmax(x, 0.0);
            const double ax = fabs(x);
            if (ax < cutT) {
                double L = log1p_exp_tab(ax * invTs, a.gtab);
                const double y = R + r.m;
                if (y < cutT)
                    L += log1p_exp_tab(y * invTs, a.gtab);
                P = fma(T, L, P);
            }
            neumaier(s, c, w * (r.base - P));
        }
        const double w = wave_sum(s + c);
        __syncthreads();
        if ((threadIdx.x & 63) == 0)
            red[threadIdx.x >> 6] = w;
        __syncthreads();
        if (threadIdx.x == 0)
            v.vpart[(size_t)ks * v.n_vchunks + chunk] = ((red[0] + red[1]) + red[2]) + red[3];
    }
}

// One wave per set: FP64 Omega of the candidates (fixed-order chunk sums
// plus N (-2 Delta^2 / V)), with the Delta = 0 cells under the threshold at
// their grid values, then the tie rule over these checked cells.
__global__ __launch_bounds__(64) void verify_pick_kernel(const VerifyArgs v)
{
    const int sl = blockIdx.x;
    const int g = sl / v.nb;
    const int slot = sl - g * v.nb;
    const size_t oset = (size_t)v.sw.pts[g].out * v.nb + slot;
    const double *G = v.grid + oset * (size_t)v.n_q * v.n_delta;
    const int lane = threadIdx.x;
    const int cnt = v.cnt[sl];
    const double thr = v.thr[sl];
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    double val = nan;
    int key = 0x7fffffff;
    if (lane < cnt) {
        const int cell = v.cand[(size_t)sl * kVerifyMax + lane];
        const int iq = cell / v.n_delta;
        const int id = cell - iq * v.n_delta;
        const double D = v.delta[id];
        val = ordered_sum(v.vpart + ((size_t)sl * kVerifyMax + lane) * v.n_vchunks, 1,
                          v.n_vchunks) +
              v.n_k * (-2.0 * D * D / v.Vs[slot]);
        key = id * v.n_q + iq;
    }
    // calls f(id) for every Delta = 0 column in increasing id (found 64
    // columns at a time)
    auto zero_columns = [&](auto f) {
        for (int id0 = 0; id0 < v.n_delta; id0 += 64) {
            bool z = false;
            if (id0 + lane < v.n_delta) {
                const double D = v.delta[id0 + lane];
                z = D * D == 0.0;
            }
            unsigned long long b = __ballot(z);
            while (b) {
                const int k = __ffsll((unsigned long long)b) - 1;
                b &= b - 1ull;
                f(id0 + k);
            }
        }
    };
    // the lowest checked value: candidates, then the Delta = 0 cells
    double best = val;
    zero_columns([&](int id) {
        for (int iq = lane; iq < v.n_q; iq += 64) {
            const double x = G[(size_t)iq * v.n_delta + id];
            if (x <= thr)
                best = nan_min(best, x);
        }
    });
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        best = nan_min(best, __shfl_xor(best, off, 64));
    int pick = 0x7fffffff;
    double pv = nan;
    if (best == best) {
        const double t64 = tie_threshold(best, v.tie_rel);
        if (key != 0x7fffffff && val <= t64) {
            pick = key;
            pv = val;
        }
        zero_columns([&](int id) {
            for (int iq = lane; iq < v.n_q; iq += 64) {
                const double x = G[(size_t)iq * v.n_delta + id];
                const int k = id * v.n_q + iq;
                if (x <= thr && x <= t64 && k < pick) {
                    pick = k;
                    pv = x;
                }
            }
        });
    }
    int m = pick;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int o = __shfl_xor(m, off, 64);
        m = o < m ? o : m;
    }
    if (m == 0x7fffffff) {
        if (lane == 0) {
            v.idx[2 * oset] = -1;
            v.idx[2 * oset + 1] = -1;
            v.omin[oset] = nan;
        }
    } else if (pick == m) {
        // one lane holds the smallest key (keys of different cells differ)
        v.idx[2 * oset] = m / v.n_q;
        v.idx[2 * oset + 1] = m % v.n_q;
        v.omin[oset] = pv;
    }
}

hipError_t launch_verify(const VerifyArgs &v, int G, bool b3, hipStream_t s)
{
    const int sets = G * v.nb;
    hipLaunchKernelGGL(verify_cand_kernel, dim3(sets), dim3(kBlock), 0, s, v);
    if (hipGetLastError() != hipSuccess)
        return hipErrorLaunchFailure;
    const long long units = (long long)sets * kVerifyMax * v.n_vchunks;
    if (units > 0x7fffffffLL)
        return hipErrorInvalidValue;
    const int blocks = (int)(units < 4096 ? units : 4096);
    if (b3)
        hipLaunchKernelGGL(verify_eval_kernel<true>, dim3(blocks), dim3(kBlock), 0, s, v,
                           (int)units);
    else
        hipLaunchKernelGGL(verify_eval_kernel<false>, dim3(blocks), dim3(kBlock), 0, s, v,
                           (int)units);
    if (hipGetLastError() != hipSuccess)
        return hipErrorLaunchFailure;
    hipLaunchKernelGGL(verify_pick_kernel, dim3(sets), dim3(64), 0, s, v);
    return hipGetLastError();
}

// ------------------------------------------------------------------ gradient

// Gradient of (A.4) at p from cos/sin of its components; the non-smooth part
// is 0 where the two bands touch.
__device__ __forceinline__ void band_grad(const Hop &t, double eps, double cx,
                                          double sx, double cy, double sy,
                                          double &E, double &gx, double &gy)
{
    double A = fma(t.tB * cx, cy, t.tA * (cx + cy));
    double D = t.tD * (cx - cy);
    double C = t.tC * sx * sy;
    double rho = sqrt(fma(D, D, C * C));
    E = fma(eps, rho, A);
    double Ax = -sx * fma(t.tB, cy, t.tA);
    double Ay = -sy * fma(t.tB, cx, t.tA);
    double Dx = -t.tD * sx, Dy = t.tD * sy;
    double Cx = t.tC * cx * sy, Cy = t.tC * sx * cy;
    if (rho > 0.0) {
        double er = eps / rho;
        gx = fma(er, fma(D, Dx, C * Cx), Ax);
        gy = fma(er, fma(D, Dy, C * Cy), Ay);
    } else {
        gx = Ax;
        gy = Ay;
    }
}

// Fermi function f(E) = 1/(1 + exp(E/T)) and -T ln(1 + exp(-E/T)) of one
// quasiparticle branch.  Beyond |E| >= 36 T both take their T -> 0 values
// (changes below 2.4e-16 relative); T = 0 gives the step (1/2 at E = 0).
struct Thermal {
    double f, sp;
};

__device__ __forceinline__ Thermal thermal_branch(double E, double T, double invT,
                                                  double cutT)
{
    const double aE = fabs(E);
    Thermal r;
    const double lo = fmin(E, 0.0);
    if (aE < cutT) {
        const double e = exp_nonpos(-aE * invT);
        r.f = (E > 0.0 ? e : 1.0) * rcp_nr(1.0 + e);
        r.sp = lo - T * log1p_small(e);
    } else {
        r.f = E < 0.0 ? 1.0 : (E > 0.0 ? 0.0 : 0.5);
        r.sp = lo;
    }
    return r;
}

// Per k: the term of Eq. (5) and its derivatives with respect to Delta,
// qx, qy and mu; 5 compensated sums per thread, fixed-order block reduction.
// Grid (chunk, band slot, point of the batch).
__global__ __launch_bounds__(kBlock) void grad_kernel(const GradArgs a)
{
    const int chunk = blockIdx.x;
    const int slot = blockIdx.y;
    const int g = blockIdx.z;
    const PointRec pt = a.pts[g];
    const size_t io = (size_t)pt.out * a.nb + slot;   // input/output slot
    const double eps = slot ? a.eps[1] : a.eps[0];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double mu_up = a.mu + pt.h, mu_dn = a.mu - pt.h;
    const double T = pt.T;
    const double invT = T > 0.0 ? 1.0 / T : 0.0;
    const double cutT = kCutGrad * T;
    const double D = a.delta[io];
    const double cqx = a.qtrig[kQTrig * io], sqx = a.qtrig[kQTrig * io + 1];
    const double cqy = a.qtrig[kQTrig * io + 2], sqy = a.qtrig[kQTrig * io + 3];
    const double *cxt = a.trig, *sxt = a.trig + a.Lx;
    const double *cyt = a.trig + 2 * a.Lx, *syt = cyt + a.Ly;
    double s_[5] = {0, 0, 0, 0, 0}, c_[5] = {0, 0, 0, 0, 0};
    const int li = lane >> 3, lj = lane & 7;
    const int span = (a.n_tiles + a.n_chunks - 1) / a.n_chunks;
    const int tile_begin = chunk * span;
    const int tile_end = min(tile_begin + span, a.n_tiles);
    for (int tile = tile_begin + wave; tile < tile_end; tile += 4) {
        const int ti = tile / a.TY;
        const int tj = tile - ti * a.TY;
        const int i = ti * kTileEdge + li;
        const int j = tj * kTileEdge + lj;
        if (i < a.Lx && j < a.Ly) {
            const double cx = cxt[i], sx = sxt[i], cy = cyt[j], sy = syt[j];
            double Ek = band_energy(a.hop, eps, cx, sx, cy, sy);
            double cpx = fma(cqx, cx, sqx * sx), spx = fma(sqx, cx, -(cqx * sx));
            double cpy = fma(cqy, cy, sqy * sy), spy = fma(sqy, cy, -(cqy * sy));
            double Eq, bx, by;
            band_grad(a.hop, eps, cpx, spx, cpy, spy, Eq, bx, by);
            double up = Ek - mu_up, dn = Eq - mu_dn;
            double s = 0.5 * (up + dn), d = 0.5 * (up - dn);
            // form factor and, at the relative momentum, its q derivatives
            double ex = cx, ey = cy, dex = 0.0, dey = 0.0;
            if (a.eta_rel) {
                const double *qh = a.qtrig + kQTrig * io + 4;
                ex = fma(cx, qh[0], sx * qh[1]);    // cos(kx - qx/2)
                ey = fma(cy, qh[2], sy * qh[3]);
                dex = 0.5 * fma(sx, qh[0], -(cx * qh[1])) * ey;   // sin(kx - qx/2) ey / 2
                dey = 0.5 * ex * fma(sy, qh[2], -(cy * qh[3]));
            }
            double eta = ex * ey;
            double gap = D * eta;
            double R = sqrt_rn(fma(s, s, gap * gap));
            double Ep = d + R, Em = d - R;
            const Thermal tp = thermal_branch(Ep, T, invT, cutT);
            const Thermal tm = thermal_branch(Em, T, invT, cutT);
            const double fp = tp.f, fm = tm.f;
            const double rR = R > 0.0 ? rcp_nr(R) : 0.0;
            double sr = s * rR;
            double dr = gap * eta * rR;
            double w = 0.5 * fp * (sr - 1.0) - 0.5 * fm * (sr + 1.0);
            neumaier(s_[0], c_[0], (tp.sp + tm.sp) + (Ek - mu_dn));
            neumaier(s_[1], c_[1], dr * (fp - fm));
            // dOmega_k / d eta = Delta (gap / R) (f+ - f-), through deta/dq
            const double ge = D * gap * rR * (fp - fm);
            neumaier(s_[2], c_[2], fma(ge, dex, bx * w));
            neumaier(s_[3], c_[3], fma(ge, dey, by * w));
            neumaier(s_[4], c_[4], sr * (fm - fp));
        }
    }
    __shared__ double red[5][4];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        double v = wave_sum(s_[c] + c_[c]);
        if (lane == 0)
            red[c][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        const int c = threadIdx.x;
        a.part[(((size_t)g * a.nb + slot) * a.n_chunks + chunk) * 5 + c] =
            ((red[c][0] + red[c][1]) + red[c][2]) + red[c][3];
    }
}

hipError_t launch_grad(const GradArgs &a, int G, hipStream_t s)
{
    hipLaunchKernelGGL(grad_kernel, dim3(a.n_chunks, a.nb, G), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// Fixed-order chunk sums of the gradient sweep plus the Delta terms of
// Eq. (5): grid (band slot, point of the batch), one lane per quantity.
__global__ void grad_finish_kernel(const GradFinishArgs a)
{
    const int slot = blockIdx.x;
    const int g = blockIdx.y;
    const int c = threadIdx.x;
    if (c >= 5)
        return;
    const size_t io = (size_t)a.pts[g].out * a.nb + slot;
    const double *pp = a.part + ((size_t)g * a.nb + slot) * a.n_chunks * 5;
    double v = ordered_sum(pp + c, 5, a.n_chunks);
    const double D = a.delta[io];
    const double V = slot ? a.Vs[1] : a.Vs[0];
    switch (c) {
    case 0:
        a.omega[io] = v + a.n_k * (-2.0 * D * D / V);
        break;
    case 1:
        a.dDelta[io] = v - 4.0 * a.n_k * D / V;
        break;
    case 2:
        a.dq[2 * io] = v;
        break;
    case 3:
        a.dq[2 * io + 1] = v;
        break;
    default:
        a.dmu[io] = v - a.n_k;
        break;
    }
}

hipError_t launch_grad_finish(const GradFinishArgs &a, int G, hipStream_t s)
{
    hipLaunchKernelGGL(grad_finish_kernel, dim3(a.nb, G), dim3(64), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ LO pairing

// One cycle of an LO sector (see LoArgs): the n x n matrix in LDS (row
// stride n + 1), cyclic Jacobi with the round-robin ordering (n/2 disjoint
// rotations per step, n - 1 steps per sweep; backward stable, eigenvalue
// errors of order 1e-16 of the matrix norm) until the off-diagonal part
// falls below 1e-32 of the whole (squared Frobenius norms), then the thermal
// sum over the diagonal.  Nodes along the cycle: 2t is c_{(r - 2ts) mod Lc}
// (diagonal E - mu - h), 2t + 1 is d_{(r - (2t+1)s) mod Lc} (diagonal
// -(E - mu + h)); node 2t couples to its two neighbours with Delta eta of
// its own momentum, node 2t + 1 to node 2t + 2 with Delta eta of that one's.
template <int NMAX>
__global__ __launch_bounds__(kBlock) void lo_cycle_kernel(const LoArgs a)
{
    constexpr int LD = NMAX + 1;
    __shared__ double A[NMAX * LD];
    __shared__ double cs[NMAX / 2][2];
    __shared__ int pq[NMAX / 2][2];
    __shared__ double red[4];
    const int n = a.n;
    const int sector = blockIdx.x / a.g;
    const int r = blockIdx.x - sector * a.g;
    const int id = blockIdx.y;
    const int slot = blockIdx.z;
    const double eps = slot ? a.eps[1] : a.eps[0];
    const double D = a.delta[id];
    const int tid = threadIdx.x;
    double ssec, csec;
    sincospi(2.0 * sector / a.Ls, &ssec, &csec);
    for (int x = tid; x < n * LD; x += kBlock)
        A[x] = 0.0;
    __syncthreads();
    // diagonal, couplings, and xi_down of the cycle's spin-up momenta
    double cdn = 0.0;
    for (int t = tid; t < n / 2; t += kBlock) {
        const int jc = (int)(((long long)r - 2LL * t * a.s) % a.Lc + a.Lc) % a.Lc;
        const int jd = (int)(((long long)r - (2LL * t + 1) * a.s) % a.Lc + a.Lc) % a.Lc;
        const int jn = (int)(((long long)r - (2LL * t + 2) * a.s) % a.Lc + a.Lc) % a.Lc;
        double sc, cc, sd, cd, sn, cn;
        sincospi(2.0 * jc / a.Lc, &sc, &cc);
        sincospi(2.0 * jd / a.Lc, &sd, &cd);
        sincospi(2.0 * jn / a.Lc, &sn, &cn);
        // (kx, ky) of a chain index: the chain runs along ky when along_y
        const double Ec = a.along_y ? band_energy(a.hop, eps, csec, ssec, cc, sc)
                                    : band_energy(a.hop, eps, cc, sc, csec, ssec);
        const double Ed = a.along_y ? band_energy(a.hop, eps, csec, ssec, cd, sd)
                                    : band_energy(a.hop, eps, cd, sd, csec, ssec);
        const double eta_c = csec * cc, eta_n = csec * cn;
        A[(2 * t) * LD + 2 * t] = Ec - (a.mu + a.h);
        A[(2 * t + 1) * LD + 2 * t + 1] = -(Ed - (a.mu - a.h));
        cdn += Ec - (a.mu - a.h);
        if (n > 2) {
            const int u = (2 * t + 2) % n;
            A[(2 * t) * LD + 2 * t + 1] = D * eta_c;
            A[(2 * t + 1) * LD + 2 * t] = D * eta_c;
            A[(2 * t + 1) * LD + u] = D * eta_n;
            A[u * LD + 2 * t + 1] = D * eta_n;
        } else {
            // both waves join the same two modes (2q = 0)
            A[1] = 2.0 * D * eta_c;
            A[LD] = 2.0 * D * eta_c;
        }
    }
    __syncthreads();
    for (int sweep = 0; sweep < 30; ++sweep) {
        // off-diagonal against total squared Frobenius norm
        double off = 0.0, tot = 0.0;
        for (int x = tid; x < n * n; x += kBlock) {
            const int i = x / n, j = x - (x / n) * n;
            const double v = A[i * LD + j];
            tot += v * v;
            off += i != j ? v * v : 0.0;
        }
        off = wave_sum(off);
        tot = wave_sum(tot);
        __shared__ double nrm[4][2];
        if ((tid & 63) == 0) {
            nrm[tid >> 6][0] = off;
            nrm[tid >> 6][1] = tot;
        }
        __syncthreads();
        const double offs = ((nrm[0][0] + nrm[1][0]) + nrm[2][0]) + nrm[3][0];
        const double tots = ((nrm[0][1] + nrm[1][1]) + nrm[2][1]) + nrm[3][1];
        __syncthreads();
        if (!(offs > 1e-32 * tots))
            break;
        for (int step = 0; step < n - 1; ++step) {
            // round robin: mode n - 1 meets mode step, (step + i, step - i) mod n - 1
            for (int i = tid; i < n / 2; i += kBlock) {
                int p, q;
                if (i == 0) {
                    p = step;
                    q = n - 1;
                } else {
                    p = (step + i) % (n - 1);
                    q = (step - i + (n - 1)) % (n - 1);
                }
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                const double app = A[p * LD + p], aqq = A[q * LD + q], apq = A[p * LD + q];
                double c = 1.0, sn = 0.0;
                if (apq != 0.0) {
                    const double th = (aqq - app) / (2.0 * apq);
                    const double t = copysign(1.0, th) / (fabs(th) + sqrt(fma(th, th, 1.0)));
                    c = 1.0 / sqrt(fma(t, t, 1.0));
                    sn = t * c;
                }
                cs[i][0] = c;
                cs[i][1] = sn;
                pq[i][0] = p;
                pq[i][1] = q;
            }
            __syncthreads();
            // rows p, q: (J^T A)
            for (int x = tid; x < (n / 2) * n; x += kBlock) {
                const int i = x / n, j = x - (x / n) * n;
                const int p = pq[i][0], q = pq[i][1];
                const double c = cs[i][0], sn = cs[i][1];
                const double ap = A[p * LD + j], aq = A[q * LD + j];
                A[p * LD + j] = c * ap - sn * aq;
                A[q * LD + j] = sn * ap + c * aq;
            }
            __syncthreads();
            // columns p, q: (J^T A) J
            for (int x = tid; x < (n / 2) * n; x += kBlock) {
                const int i = x / n, j = x - (x / n) * n;
                const int p = pq[i][0], q = pq[i][1];
                const double c = cs[i][0], sn = cs[i][1];
                const double ap = A[j * LD + p], aq = A[j * LD + q];
                A[j * LD + p] = c * ap - sn * aq;
                A[j * LD + q] = sn * ap + c * aq;
            }
            __syncthreads();
            for (int i = tid; i < n / 2; i += kBlock) {
                const int p = pq[i][0], q = pq[i][1];
                A[p * LD + q] = 0.0;
                A[q * LD + p] = 0.0;
            }
            __syncthreads();
        }
    }
    // -T ln(1 + e^{-E/T}) over the eigenvalues, as min(E, 0) - T log1p(e^{-|E|/T})
    double sum = cdn, cmp = 0.0;
    const double invT = a.T > 0.0 ? 1.0 / a.T : 0.0;
    for (int i = tid; i < n; i += kBlock) {
        const double E = A[i * LD + i];
        double v = fmin(E, 0.0);
        if (a.T > 0.0)
            v -= a.T * log1p_small(exp_nonpos(-fmin(fabs(E) * invT, 700.0)));
        neumaier(sum, cmp, v);
    }
    const double w = wave_sum(sum + cmp);
    if ((tid & 63) == 0)
        red[tid >> 6] = w;
    __syncthreads();
    if (tid == 0)
        a.part[((size_t)slot * a.n_delta + id) * ((size_t)a.Ls * a.g) + blockIdx.x] =
            ((red[0] + red[1]) + red[2]) + red[3];
}

// Cycles of at most 64 modes: one wave per cycle, kLoWaves cycles per
// workgroup, no workgroup barrier.  The symmetric matrix is kept once, as
// its upper triangle packed by rows in LDS.  Each step applies the n/2
// disjoint rotations of the round-robin ordering (the same pairs and the
// same c, s as lo_cycle_kernel) as 2 x 2 block updates: the block of rows
// (p_a, q_a) and columns (p_b, q_b) of each pair of pairs a <= b becomes
// R_a^T B R_b (rows first, then columns, as in lo_cycle_kernel), and the
// pivot element of a diagonal block is set to zero.  Every matrix element
// is read and written once per step.
constexpr int kLoWaves = 4;

__device__ __forceinline__ int lo_tri(int i, int j, int n)
{
    // (i, j) with i <= j in the packed upper triangle
    return i * n - ((i * (i - 1)) >> 1) + (j - i);
}

__device__ __forceinline__ int lo_sym(int i, int j, int n)
{
    return i <= j ? lo_tri(i, j, n) : lo_tri(j, i, n);
}

template <int NMAX>
__global__ __launch_bounds__(64 * kLoWaves) void lo_wave_kernel(const LoArgs a)
{
    constexpr int PACK = NMAX * (NMAX + 1) / 2;
    __shared__ double Aw[kLoWaves][PACK];
    __shared__ double csw[kLoWaves][NMAX / 2][2];
    __shared__ int pqw[kLoWaves][NMAX / 2][2];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int n = a.n;
    const int h = n / 2;
    const int n_cyc = a.Ls * a.g;
    const int cyc = blockIdx.x * kLoWaves + wave;
    if (cyc >= n_cyc)
        return;
    double *A = Aw[wave];
    double(*cs)[2] = csw[wave];
    int(*pq)[2] = pqw[wave];
    const int sector = cyc / a.g;
    const int r = cyc - sector * a.g;
    const int id = blockIdx.y;
    const int slot = blockIdx.z;
    const double eps = slot ? a.eps[1] : a.eps[0];
    const double D = a.delta[id];
    double ssec, csec;
    sincospi(2.0 * sector / a.Ls, &ssec, &csec);
    const int npack = n * (n + 1) / 2;
    for (int x = lane; x < npack; x += 64)
        A[x] = 0.0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // diagonal, couplings, and xi_down of the cycle's spin-up momenta (the
    // node layout of lo_cycle_kernel)
    double cdn = 0.0;
    for (int t = lane; t < h; t += 64) {
        const int jc = (int)(((long long)r - 2LL * t * a.s) % a.Lc + a.Lc) % a.Lc;
        const int jd = (int)(((long long)r - (2LL * t + 1) * a.s) % a.Lc + a.Lc) % a.Lc;
        const int jn = (int)(((long long)r - (2LL * t + 2) * a.s) % a.Lc + a.Lc) % a.Lc;
        double sc, cc, sd, cd, sn, cn;
        sincospi(2.0 * jc / a.Lc, &sc, &cc);
        sincospi(2.0 * jd / a.Lc, &sd, &cd);
        sincospi(2.0 * jn / a.Lc, &sn, &cn);
        const double Ec = a.along_y ? band_energy(a.hop, eps, csec, ssec, cc, sc)
                                    : band_energy(a.hop, eps, cc, sc, csec, ssec);
        const double Ed = a.along_y ? band_energy(a.hop, eps, csec, ssec, cd, sd)
                                    : band_energy(a.hop, eps, cd, sd, csec, ssec);
        const double eta_c = csec * cc, eta_n = csec * cn;
        A[lo_tri(2 * t, 2 * t, n)] = Ec - (a.mu + a.h);
        A[lo_tri(2 * t + 1, 2 * t + 1, n)] = -(Ed - (a.mu - a.h));
        cdn += Ec - (a.mu - a.h);
        if (n > 2) {
            A[lo_tri(2 * t, 2 * t + 1, n)] = D * eta_c;
            A[lo_sym(2 * t + 1, (2 * t + 2) % n, n)] = D * eta_n;
        } else {
            // both waves join the same two modes (2q = 0)
            A[lo_tri(0, 1, n)] = 2.0 * D * eta_c;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // pairs of pairs a <= b, folded so that consecutive indices fill rows
    // r and H - 1 - r (H = h rounded up to even; pair index h, if any, is a
    // placeholder and skipped); at most (NMAX/2 + 1) NMAX/4 of them
    // this lane's blocks, (a | b << 8) or -1, fixed for the whole cycle
    constexpr int NB = ((NMAX / 2 + 1) * (NMAX / 4) + 63) / 64;
    int blk[NB];
    {
        const int H = h + (h & 1);
        const int nblk = (H / 2) * (H + 1);
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            const int k = lane + 64 * m;
            int code = -1;
            if (k < nblk) {
                const int rr = k / (H + 1);
                const int e = k - rr * (H + 1);
                int ia, ib;
                if (e < H - rr) {
                    ia = rr;
                    ib = rr + e;
                } else {
                    ia = H - 1 - rr;
                    ib = ia + (e - (H - rr));
                }
                if (ib < h)
                    code = ia | (ib << 8);
            }
            blk[m] = code;
        }
    }
    for (int sweep = 0; sweep < 30; ++sweep) {
        // off-diagonal against total squared Frobenius norm
        double off = 0.0, dia = 0.0;
        for (int i = 0; i < n; ++i) {
            const int row = lo_tri(i, i, n);
            for (int j = i + 1 + lane; j < n; j += 64) {
                const double v = A[row + (j - i)];
                off += v * v;
            }
        }
        for (int i = lane; i < n; i += 64) {
            const double v = A[lo_tri(i, i, n)];
            dia += v * v;
        }
        // both triangles off the diagonal, and the whole matrix
        const double offs = 2.0 * wave_sum(off);
        const double tots = offs + wave_sum(dia);
        if (!(offs > 1e-32 * tots))
            break;
        for (int step = 0; step < n - 1; ++step) {
            // round robin: mode n - 1 meets mode step, (step + i, step - i) mod n - 1
            for (int i = lane; i < h; i += 64) {
                int p, q;
                if (i == 0) {
                    p = step;
                    q = n - 1;
                } else {
                    p = (step + i) % (n - 1);
                    q = (step - i + (n - 1)) % (n - 1);
                }
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                const double app = A[lo_tri(p, p, n)], aqq = A[lo_tri(q, q, n)],
                             apq = A[lo_tri(p, q, n)];
                double c = 1.0, sn = 0.0;
                if (apq != 0.0) {
                    const double th = (aqq - app) / (2.0 * apq);
                    const double t = copysign(1.0, th) / (fabs(th) + sqrt(fma(th, th, 1.0)));
                    c = 1.0 / sqrt(fma(t, t, 1.0));
                    sn = t * c;
                }
                cs[i][0] = c;
                cs[i][1] = sn;
                pq[i][0] = p;
                pq[i][1] = q;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int m = 0; m < NB; ++m) {
                if (blk[m] < 0)
                    continue;
                const int ia = blk[m] & 255, ib = blk[m] >> 8;
                const int pa = pq[ia][0], qa = pq[ia][1];
                const double ca = cs[ia][0], sa = cs[ia][1];
                if (ia == ib) {
                    const int ip = lo_tri(pa, pa, n), iq = lo_tri(qa, qa, n),
                              ipq = lo_tri(pa, qa, n);
                    const double app = A[ip], aqq = A[iq], apq = A[ipq];
                    // rows p, q, then columns p, q; the pivot becomes 0
                    const double xpp = ca * app - sa * apq, xqp = sa * app + ca * apq;
                    const double xpq = ca * apq - sa * aqq, xqq = sa * apq + ca * aqq;
                    A[ip] = ca * xpp - sa * xpq;
                    A[iq] = sa * xqp + ca * xqq;
                    A[ipq] = 0.0;
                } else {
                    const int pb = pq[ib][0], qb = pq[ib][1];
                    const double cb = cs[ib][0], sb = cs[ib][1];
                    const int i00 = lo_sym(pa, pb, n), i01 = lo_sym(pa, qb, n),
                              i10 = lo_sym(qa, pb, n), i11 = lo_sym(qa, qb, n);
                    const double b00 = A[i00], b01 = A[i01], b10 = A[i10], b11 = A[i11];
                    // rows (p_a, q_a) by R_a
                    const double x00 = ca * b00 - sa * b10, x10 = sa * b00 + ca * b10;
                    const double x01 = ca * b01 - sa * b11, x11 = sa * b01 + ca * b11;
                    // columns (p_b, q_b) by R_b
                    A[i00] = cb * x00 - sb * x01;
                    A[i01] = sb * x00 + cb * x01;
                    A[i10] = cb * x10 - sb * x11;
                    A[i11] = sb * x10 + cb * x11;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    // -T ln(1 + e^{-E/T}) over the eigenvalues, as min(E, 0) - T log1p(e^{-|E|/T})
    double sum = cdn, cmp = 0.0;
    const double invT = a.T > 0.0 ? 1.0 / a.T : 0.0;
    for (int i = lane; i < n; i += 64) {
        const double E = A[lo_tri(i, i, n)];
        double v = fmin(E, 0.0);
        if (a.T > 0.0)
            v -= a.T * log1p_small(exp_nonpos(-fmin(fabs(E) * invT, 700.0)));
        neumaier(sum, cmp, v);
    }
    const double w = wave_sum(sum + cmp);
    if (lane == 0)
        a.part[((size_t)slot * a.n_delta + id) * (size_t)n_cyc + cyc] = w;
}

hipError_t launch_lo(const LoArgs &a, int nb, hipStream_t s)
{
    const dim3 grid(a.Ls * a.g, a.n_delta, nb);
    const dim3 wgrid((a.Ls * a.g + kLoWaves - 1) / kLoWaves, a.n_delta, nb);
    if (a.n <= 32)
        hipLaunchKernelGGL(lo_wave_kernel<32>, wgrid, dim3(64 * kLoWaves), 0, s, a);
    else if (a.n <= 64)
        hipLaunchKernelGGL(lo_wave_kernel<64>, wgrid, dim3(64 * kLoWaves), 0, s, a);
    else if (a.n <= kLoMaxCycle)
        hipLaunchKernelGGL(lo_cycle_kernel<kLoMaxCycle>, grid, dim3(kBlock), 0, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Fixed-order sum of the cycle partials plus -(2/V) sum_j |Delta(R_j)|^2 =
// -2 N w Delta^2 / V: one thread per (band slot, Delta).
__global__ void lo_finish_kernel(const LoFinishArgs a)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.nb * a.n_delta)
        return;
    const int slot = t / a.n_delta, id = t - (t / a.n_delta) * a.n_delta;
    const double D = a.delta[id];
    const double v = ordered_sum(a.part + (size_t)t * a.n_parts, 1, a.n_parts);
    a.omega[slot * a.slot_stride + id] = v + a.n_k * (-2.0 * a.w * D * D / a.Vs[slot]);
}

hipError_t launch_lo_finish(const LoFinishArgs &a, hipStream_t s)
{
    const int n = a.nb * a.n_delta;
    hipLaunchKernelGGL(lo_finish_kernel, dim3((n + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace omega
