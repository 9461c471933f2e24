/*
 * omega.h -- C interface of libomega, the gfx950 (MI355X) implementation of
 * the free-energy search of Januszewski, Ptok, Crivelli & Gardas, "GPU-based
 * acceleration of free energy calculations in solid state physics".
 *
 * What is computed (all in the paper's notation, k_B = 1):
 *   band energies    E_{eps,k}: App. A, Eqs. (A.1)-(A.4) (two-band model,
 *                    eps = - hole-like, eps = + electron-like);
 *   spin shift       E_{eps,k,sigma} = E_{eps,k} - (mu + sigma h), sigma = +1
 *                    for spin up (Sec. 2, Eq. (1) and the text below it);
 *   quasiparticles   Sec. 2, Eq. (4), pairs (k up, -k+Q down), gap
 *                    Delta_{eps,k} = Delta cos kx cos ky (s+- form factor);
 *   free energy      Sec. 2, Eq. (5):
 *                    Omega_eps = -T sum_{+-,k} ln(1 + exp(-E^{+-}_{eps,k}/T))
 *                                + sum_k (E_{eps,k,down} - 2 Delta^2 / V_eps)
 *                    over the Lx x Ly momenta kx = 2 pi i/Lx, ky = 2 pi j/Ly;
 *   search           Sec. 3.2, Algorithm 1 (Delta minimum per Q row, then the
 *                    global minimum; bands are minimised separately).
 *
 * Conventions shared by every entry point
 *   - Units: energies in |t1|.  T >= 0; T = 0 is the zero-temperature limit
 *     (-T ln(1 + exp(-E/T)) -> min(E, 0)).  V_eps < 0 is attractive.
 *   - Ownership: the caller owns every buffer.  "_dev" pointers are device
 *     memory on the current HIP device; "_host" / plain struct pointers are
 *     host memory read during the call only.  The library allocates no device
 *     memory; scratch comes from the caller's workspace (ws_dev, ws_bytes),
 *     sized by omega_workspace_bytes().
 *   - Asynchrony: work is enqueued on `stream` (a hipStream_t; NULL = the null
 *     stream) and the call returns without synchronising.  Outputs are valid
 *     once the stream has reached the enqueued work.  Host arguments are
 *     consumed before the call returns.  Calls sharing one workspace must be
 *     ordered (same stream or explicit events).
 *   - Errors: arguments are validated on the host before anything is
 *     enqueued; an invalid call returns a negative OMEGA_E_* code and enqueues
 *     nothing.  A HIP launch failure returns OMEGA_E_HIP.  Device arrays are
 *     not validated: NaN in delta_dev or q_dev propagates into Omega.
 *   - Determinism: for fixed inputs the results are bitwise reproducible.
 *     Every sum runs in a fixed order; the only atomics are the integer
 *     counters (in the workspace) from which the sweep's waves take work
 *     units, and a unit's result does not depend on which wave computes it.
 */
#ifndef OMEGA_H
#define OMEGA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Form factor of the pair (k up, -k+Q down).  OMEGA_ETA_K: Delta_k = Delta
 * eta(k) on the spin-up momentum, as Sec. 2, Eq. (3) writes it (the default;
 * a zero-initialised model gets it).  OMEGA_ETA_REL: Delta eta(k - Q/2), the
 * form factor at the pair's relative momentum (k - (Q - k))/2; the two agree
 * at Q = 0. */
enum { OMEGA_ETA_K = 0, OMEGA_ETA_REL = 1 };

/* Model constants.  t1..t4: hoppings of App. A, Eqs. (A.1)-(A.3) (the paper's
 * values are t1=-1, t2=1.3, t3=t4=-0.85); mu: chemical potential (1.54 gives
 * two electrons per site); V[0], V[1]: pairing strength V_eps of Eq. (5) for
 * the E_- and E_+ band; form: OMEGA_ETA_K or OMEGA_ETA_REL; pad: 0.  All
 * finite, V[i] != 0. */
typedef struct {
    double t1, t2, t3, t4;
    double mu;
    double V[2];
    int32_t form;
    int32_t pad;
} omega_model;

/* One (h, T) point of a phase diagram on an Lx x Ly lattice.
 * h: Zeeman field of Eq. (1) (any finite sign); T: temperature, 0 or a normal
 * positive double; 2 <= Lx, Ly <= 16384 and Lx*Ly <= 2^26. */
typedef struct {
    double h;
    double T;
    int32_t Lx, Ly;
} omega_point;

/* Band selection mask; with both, outputs hold E_- first, then E_+. */
enum { OMEGA_BAND_MINUS = 1, OMEGA_BAND_PLUS = 2, OMEGA_BAND_BOTH = 3 };

/* Arithmetic of the Delta-dependent sweep.  OMEGA_FP64: everything in FP64.
 * OMEGA_FP32_COMP: the Delta-dependent part of each term in FP32 with
 * compensated accumulation; band energies, the Delta-independent part, all
 * cross-block sums and the argmin stay FP64. */
enum { OMEGA_FP64 = 0, OMEGA_FP32_COMP = 1 };

enum {
    OMEGA_OK = 0,
    OMEGA_E_INVAL = -1,       /* an argument is out of range or NULL        */
    OMEGA_E_WORKSPACE = -2,   /* ws_bytes smaller than required             */
    OMEGA_E_HIP = -3,         /* a HIP runtime call or launch failed        */
    OMEGA_E_UNSUPPORTED = -4  /* valid request the library does not provide */
};

/* Bytes of device workspace that omega_grid / omega_argmin (grad = 0) or
 * omega_grad (grad = 1, n_delta and n_q ignored) need for these sizes.
 * Returns 0 if the arguments are invalid. */
size_t omega_workspace_bytes(const omega_point *pts, int n_pts, int n_delta,
                             int n_q, int bands, int precision, int grad);

/* Omega grid, Eq. (5), for every point, selected band, Q and Delta
 * (Algorithm 1's two loops, all at once).
 *   pts        host array [n_pts]
 *   delta_dev  device [n_delta] Delta values (any real; Delta >= 0 physical),
 *              1 <= n_delta <= 2^20
 *   q_dev      device [n_q][2] pair momenta Q = (qx, qy), any real values,
 *              1 <= n_q <= 16384 and n_q * n_delta <= 2^30
 *   omega_dev  device output [n_pts][nb][n_q][n_delta], Delta fastest,
 *              nb = number of bands in `bands`; total Omega (not per site). */
int omega_grid(const omega_model *model, const omega_point *pts, int n_pts,
               const double *delta_dev, int n_delta, const double *q_dev,
               int n_q, int bands, int precision, void *ws_dev,
               size_t ws_bytes, double *omega_dev, void *stream);

/* Launch options of the _ex entry points; NULL, or a zero-initialised
 * struct, gives the defaults of the plain entry points.  None of them changes
 * any result: each unit of work of the persistent sweeps is computed by one
 * wave in a fixed order, whichever wave takes it.
 *   sweep_blocks_per_cu  workgroups per CU of the persistent per-Delta
 *                        sweeps (>= 0; 0: as many as stay resident)
 *   sweep_queues         work queues they take units from (0..16; 0: 8)
 *   sweep_start_event,   hipEvent_t handles (caller-owned, both or neither)
 *   sweep_stop_event     recorded on the call's stream right before the
 *                        call's first per-Delta sweep launch and right after
 *                        its last (with one batch of points: around that
 *                        sweep alone; the paper times the computation part
 *                        only, Sec. 3.3)
 *   count_dev            NULL, or a device pointer to an unsigned 64-bit
 *                        counter to which the sweeps add the number of
 *                        (k, Delta) terms they evaluated directly (terms
 *                        summed through a series in Delta^2 are not counted)
 * The options belong to the call: the library keeps none of them. */
typedef struct {
    int32_t sweep_blocks_per_cu;
    int32_t sweep_queues;
    void *sweep_start_event;
    void *sweep_stop_event;
    unsigned long long *count_dev;
} omega_launch;

/* Omega grid plus the searches of Algorithm 1 (per-Q Delta minimum, then the
 * global minimum), with a tie rule: among grid points with
 * Omega <= Omega_min + tie_rel*|Omega_min| the lexicographically smallest
 * (iDelta, iq) is chosen; per row the smallest iDelta.  Comparisons in FP64;
 * NaN is never chosen; an all-NaN set gives index -1 and Omega NaN.
 *   tie_rel      >= 0 (1e-11 recommended: grid points of one physical state,
 *                e.g. the Delta = 0 row over lattice Q, agree only to rounding)
 *   idx_dev      device output [n_pts][nb][2] = (iDelta, iq)
 *   omin_dev     device output [n_pts][nb], Omega at the chosen point
 *   row_idx_dev  device output [n_pts][nb][n_q] or NULL
 *   omega_dev    device output as in omega_grid, or NULL (grid then lives in
 *                the workspace). */
int omega_argmin(const omega_model *model, const omega_point *pts, int n_pts,
                 const double *delta_dev, int n_delta, const double *q_dev,
                 int n_q, int bands, int precision, double tie_rel,
                 void *ws_dev, size_t ws_bytes, int32_t *idx_dev,
                 double *omin_dev, int32_t *row_idx_dev, double *omega_dev,
                 void *stream);

/* omega_argmin with launch options (NULL: the defaults); OMEGA_E_INVAL for
 * options out of range. */
int omega_argmin_ex(const omega_model *model, const omega_point *pts, int n_pts,
                    const double *delta_dev, int n_delta, const double *q_dev, int n_q,
                    int bands, int precision, double tie_rel, void *ws_dev, size_t ws_bytes,
                    int32_t *idx_dev, double *omin_dev, int32_t *row_idx_dev,
                    double *omega_dev, const omega_launch *launch, void *stream);

/* omega_argmin for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation, results bitwise equal to omega_argmin's, with its
 * scratch taken from an array of OMEGA_NOALLOC_SCRATCH_BYTES that the library
 * holds statically on each device it runs on (allocated when the library's
 * code is loaded on that device, kept until the process ends).  The caller
 * still passes the inputs and outputs; the call allocates nothing, on the
 * device or through any library.  Its device address is looked up on the
 * first call on each device (make that first call outside graph capture).
 *   Returns OMEGA_E_WORKSPACE when the call needs more scratch than the
 *   array holds (omega_workspace_bytes(..., grad = 0) bytes, less the grid's
 *   n_pts*nb*n_q*n_delta*8 bytes when omega_dev is given): e.g. the 1024 x
 *   1024 lattice with 256 Delta x 64 Q x 2 bands needs about 75 MiB.
 *   Every call on one device shares that device's array, and a call leaves
 *   its contents behind (each call initialises what it reads): calls that
 *   overlap on one device (two streams, or two host threads, without
 *   ordering) race and give undefined results. */
#define OMEGA_NOALLOC_SCRATCH_BYTES (128u << 20)
int omega_argmin_noalloc(const omega_model *model, const omega_point *pts, int n_pts,
                         const double *delta_dev, int n_delta, const double *q_dev, int n_q,
                         int bands, int precision, double tie_rel, int32_t *idx_dev,
                         double *omin_dev, int32_t *row_idx_dev, double *omega_dev,
                         void *stream);

/* Omega and its first derivatives at one (Delta, Q) per point and band,
 * obtained by differentiating Eqs. (4)-(5) by hand (dOmega/dE = Fermi
 * function; at R = sqrt(s^2 + Delta^2 eta^2) = 0 and at band-touching points
 * the non-smooth factors are given the symmetric value 0).  FP64 only.
 *   delta_dev  device [n_pts][nb]; q_dev device [n_pts][nb][2]
 *   outputs    device omega_dev, dDelta_dev, dmu_dev [n_pts][nb];
 *              dq_dev [n_pts][nb][2] (d/dqx, d/dqy).  dOmega/dmu = -n_eps. */
int omega_grad(const omega_model *model, const omega_point *pts, int n_pts,
               const double *delta_dev, const double *q_dev, int bands,
               void *ws_dev, size_t ws_bytes, double *omega_dev,
               double *dDelta_dev, double *dq_dev, double *dmu_dev,
               void *stream);

/* ------------------------------------------------------------------------
 * Three-band model of App. B (Daghofer et al.; orbitals d_xz, d_yz, d_xy).
 * The band energies are the eigenvalues of the 3x3 orbital matrix of App. B,
 * which has no closed form the paper uses; as the paper proposes (Sec. 3.2),
 * they are computed numerically once per lattice and stored (a device table
 * [3][Lx][Ly]), and E(Q - k) is read from the same table where Q lies on the
 * lattice (Q = (2 pi m/Lx, 2 pi n/Ly) to 1e-13), else diagonalised at Q - k.
 * Eq. (4)-(5) and Algorithm 1 then apply per band exactly as above.  Bands
 * are numbered 0, 1, 2 in ascending energy at each k (energies in eV in the
 * paper's parametrisation).
 * ------------------------------------------------------------------------ */

/* t[0..11] = t1..t12 and eps0 as in App. B (printed: t1 = -0.08,
 * t2 = 0.1825, t3 = 0.08375, t4 = -0.03, t5 = t6 = 0.15, t7 = -0.12,
 * t8 = 0.06, t9 = 0, t10 = -0.024, t11 = -0.01, t12 = 0.0275,
 * eps0 = 0.75; mu = 0.4748 gives four electrons per site); V[b]: pairing
 * strength of band b in Eq. (5); form: OMEGA_ETA_K or OMEGA_ETA_REL; pad: 0.
 * All finite; V[b] != 0 for selected bands. */
typedef struct {
    double t[12];
    double eps0;
    double mu;
    double V[3];
    int32_t form;
    int32_t pad;
} omega3_model;

/* Band selection of the three-band model; outputs hold the selected bands in
 * ascending order. */
enum { OMEGA3_BAND_0 = 1, OMEGA3_BAND_1 = 2, OMEGA3_BAND_2 = 4, OMEGA3_BAND_ALL = 7 };

/* Band table of App. B on the Lx x Ly lattice: E_dev [3][Lx][Ly] (band, i, j)
 * at kx = 2 pi i/Lx, ky = 2 pi j/Ly, ascending per momentum.  Needs
 * ws_bytes >= 16 (Lx + Ly) bytes of workspace.  The V of `model` is not
 * used here. */
int omega3_bands(const omega3_model *model, int Lx, int Ly, void *ws_dev, size_t ws_bytes,
                 double *E_dev, void *stream);

/* Workspace bytes of omega3_grid / omega3_argmin; 0 if the arguments are
 * invalid.  bands is an OMEGA3_BAND_* mask (1..7). */
size_t omega3_workspace_bytes(const omega_point *pts, int n_pts, int n_delta, int n_q,
                              int bands, int precision);

/* As omega_grid, for the three-band model; nb = bands selected (1..3). */
int omega3_grid(const omega3_model *model, const omega_point *pts, int n_pts,
                const double *delta_dev, int n_delta, const double *q_dev, int n_q,
                int bands, int precision, void *ws_dev, size_t ws_bytes,
                double *omega_dev, void *stream);

/* As omega_argmin, for the three-band model (same tie rule and outputs). */
int omega3_argmin(const omega3_model *model, const omega_point *pts, int n_pts,
                  const double *delta_dev, int n_delta, const double *q_dev, int n_q,
                  int bands, int precision, double tie_rel, void *ws_dev,
                  size_t ws_bytes, int32_t *idx_dev, double *omin_dev,
                  int32_t *row_idx_dev, double *omega_dev, void *stream);

/* omega3_argmin with launch options, as omega_argmin_ex. */
int omega3_argmin_ex(const omega3_model *model, const omega_point *pts, int n_pts,
                     const double *delta_dev, int n_delta, const double *q_dev, int n_q,
                     int bands, int precision, double tie_rel, void *ws_dev,
                     size_t ws_bytes, int32_t *idx_dev, double *omin_dev,
                     int32_t *row_idx_dev, double *omega_dev, const omega_launch *launch,
                     void *stream);

/* ------------------------------------------------------------------------
 * Static Cooper-pair susceptibility, App. C, at omega -> 0:
 *   chi_{eps eps'}(q) = (1/N) sum_k eta(-k-q)^2
 *                       (1 - f(E_{eps k up}) - f(E_{eps',-k-q,down}))
 *                       / (E_{eps k up} + E_{eps',-k-q,down}),
 * f the Fermi function at T, eta(k) = 4 cos kx cos ky (s+- structure factor),
 * E_{eps k sigma} = E_eps(k) - (mu + sigma h).  Where the two energies sum
 * to zero the summand takes its limit 1 / (4 T cosh^2(E/2T)).  T = 0 uses
 * the step function, with 0 where the energies sum to zero.
 * Output chi_dev [n_pts][nb][nb][n_q] (eps, eps' over the selected bands, in
 * the band order of the grid calls).  V of the model is not used.
 * ------------------------------------------------------------------------ */

/* Workspace bytes of omega_pair_chi (bands: OMEGA_BAND_* mask); 0 if the
 * arguments are invalid. */
size_t omega_chi_workspace_bytes(const omega_point *pts, int n_pts, int n_q, int bands);

/* chi of the two-band model for every point, band pair and q_dev [n_q][2]. */
int omega_pair_chi(const omega_model *model, const omega_point *pts, int n_pts,
                   const double *q_dev, int n_q, int bands, void *ws_dev, size_t ws_bytes,
                   double *chi_dev, void *stream);

/* Workspace bytes of omega3_pair_chi (bands: OMEGA3_BAND_* mask). */
size_t omega3_chi_workspace_bytes(const omega_point *pts, int n_pts, int n_q, int bands);

/* chi of the three-band model; E(-k-q) from the band table where q lies on
 * the lattice, else diagonalised. */
int omega3_pair_chi(const omega3_model *model, const omega_point *pts, int n_pts,
                    const double *q_dev, int n_q, int bands, void *ws_dev, size_t ws_bytes,
                    double *chi_dev, void *stream);

/* Pair momenta of the whole zone reduced by symmetry (host only, no GPU
 * work).  Algorithm 1 scans every Q of the first Brillouin zone; on the
 * lattice these are Q = (2 pi m/Lx, 2 pi n/Ly).  k -> -k, kx -> -kx and
 * ky -> -ky (and kx <-> ky when Lx == Ly) map the lattice onto itself and
 * leave E(k) and eta(k)^2 of both models invariant, so Omega(Q) =
 * Omega(-qx, qy) = Omega(qx, -qy) (= Omega(qy, qx) on a square lattice).
 * Writes one representative per orbit, 0 <= m <= Lx/2 and 0 <= n <= Ly/2
 * (and n <= m on a square lattice), in (m, n) lexicographic order, to
 * q_host [count][2], and the orbit size (zone momenta sharing its Omega) to
 * orbit_host [count]; the orbit sizes add up to Lx*Ly.  With q_host == NULL
 * it only counts.  Returns the count, OMEGA_E_INVAL for a bad lattice or
 * OMEGA_E_WORKSPACE if capacity is too small. */
int omega_q_wedge(int Lx, int Ly, double *q_host, int32_t *orbit_host, int capacity);

/* ------------------------------------------------------------------------
 * Larkin-Ovchinnikov (LO) pairing of the two-band model: the M = 2 case of
 * the plane-wave sum of Sec. 2, Eq. (6), pairs of momentum q and -q with
 * equal amplitude, Delta(R_j) = Delta (e^{i q.R_j} + e^{-i q.R_j}), gap
 * Delta eta(k) on the spin-up momentum (OMEGA_ETA_K only).  As the
 * historical and technical note of Sec. 2 describes, with q on a lattice
 * axis the Nambu problem splits into one 2 L x 2 L problem per momentum
 * across q (L the lattice side along q); each of those splits further into
 * cycles of 2 L / gcd(2 s, L) modes (q = 2 pi s / L), which the library
 * diagonalises numerically (cyclic Jacobi, FP64).  Per band:
 *   Omega_LO = -T sum_n ln(1 + e^{-E_n/T}) + sum_k E_{k down}
 *              - (2 / V_eps) sum_j |Delta(R_j)|^2
 * over the 2N Nambu eigenvalues E_n; the last two terms are those of
 * Eq. (5), with sum_j |Delta(R_j)|^2 = 2 N Delta^2 (4 N Delta^2 where 2q is
 * a reciprocal lattice vector: then the two waves coincide and the state
 * is the FF state of gap 2 Delta).  One wave alone reproduces Eq. (5).
 *   q_host   host [n_q][2] lattice indices (m, n) of q = (2 pi m/Lx,
 *            2 pi n/Ly) with m == 0 or n == 0; a cycle may hold at most 128
 *            modes (2 L / gcd(2 s, L) <= 128), else OMEGA_E_UNSUPPORTED
 *   omega_dev device output [n_pts][nb][n_q][n_delta] (total, not per site)
 * ------------------------------------------------------------------------ */

/* Workspace bytes of omega_lo_grid; 0 if the arguments are invalid or a
 * (point, q) is outside what omega_lo_grid takes. */
size_t omega_lo_workspace_bytes(const omega_point *pts, int n_pts, int n_delta,
                                const int32_t *q_host, int n_q, int bands);

int omega_lo_grid(const omega_model *model, const omega_point *pts, int n_pts,
                  const double *delta_dev, int n_delta, const int32_t *q_host, int n_q,
                  int bands, void *ws_dev, size_t ws_bytes, double *omega_dev, void *stream);

/* Static description of an OMEGA_* code (never NULL). */
const char *omega_strerror(int code);

/* Library interface version, currently 4 (2 added the three-band model, 3 the
 * pair susceptibility, 4 the form factor field of the model structs, the LO
 * pairing, and the launch options of the _ex calls in place of process-wide
 * benchmark hooks). */
int omega_version(void);

#ifdef __cplusplus
}
#endif

#endif /* OMEGA_H */
