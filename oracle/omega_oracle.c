/*
 * Reference oracle for the Fulde-Ferrell free energy of the two-band
 * iron-pnictide model (Januszewski, Ptok, Crivelli, Gardas, "GPU-based
 * acceleration of free energy calculations in solid state physics").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, FP64 statement of
 * what the GPU library computes.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no code, header, table
 * or helper with the GPU library, and it never reads anything the GPU library
 * produced.
 *
 * What it follows:
 *   - band energies: App. A, Eqs. (A.1)-(A.4) (two-band model, closed-form
 *     diagonalisation of the 2x2 orbital hopping matrix);
 *   - spin-dependent on-site shift E_{k sigma} = E_k - (mu + sigma h) with
 *     sigma = +1 for spin up: Sec. 2, Eq. (1) and the text under it;
 *   - quasiparticle energies: Sec. 2, Eq. (4), pairing (k up, -k+q down) with
 *     Delta_k = Delta * eta(k), eta(k) = cos kx cos ky (s+- form factor of the
 *     introduction; Sec. 2, Eq. (3) attaches it to the spin-up momentum k).
 *     As a model option the form factor is taken at the pair's relative
 *     momentum instead, eta(k - q/2) = cos(kx - qx/2) cos(ky - qy/2), the
 *     momentum of each partner measured from the pair's centre of mass;
 *     at q = 0 the two coincide;
 *   - free energy per band: Sec. 2, Eq. (5);
 *   - search: Sec. 3.2, Algorithm 1 (for each q: build the two band-energy
 *     arrays over the Brillouin zone, then for each Delta evaluate Eq. (4) and
 *     Eq. (5); keep the per-q minimum, then the global one).  The Delta loop is
 *     parallelised with OpenMP as in the paper's CPU variant (Sec. 3.2).
 *
 * Readings taken where the paper is silent (each is listed in the design
 * notes of the repository):
 *   - k grid kx = 2 pi i / Lx, i = 0..Lx-1 (same for y);
 *   - Sum_k E_{k down} is taken literally (Q-independent);
 *   - -T ln(1 + exp(-E/T)) is evaluated as min(E,0) - T log1p(exp(-|E|/T)),
 *     which is the same function written without overflow; T = 0 gives
 *     min(E,0);
 *   - V < 0 is attractive (the -2 Delta^2 / V term is taken as printed);
 *   - k sums are Neumaier-compensated in fixed i-major order;
 *   - argmin tie rule: among grid points with Omega <= Omega_min +
 *     tie_rel*|Omega_min| the lexicographically smallest (iDelta, iq) wins,
 *     rows take the smallest iDelta; NaN is never selected.
 *
 * Parity pins: band energies, hopping signs / filling, the whole of
 * Eqs. (4)-(5), the normal and BCS limits, the symmetries, gradients and the
 * argmin rule are each checked against an independent statement (a textbook
 * routine, a closed form, brute-force diagonalisation or finite differences)
 * by the CPU test-suite.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double t1, t2, t3, t4; /* hoppings of App. A, energy unit |t1| */
    double mu;             /* chemical potential */
    double V[2];           /* pairing strength for band 0 (E_-) and band 1 (E_+) */
    int32_t form;          /* OR_ETA_K: eta(k); OR_ETA_REL: eta(k - q/2) */
    int32_t pad;
} or_model;

#define OR_ETA_K 0
#define OR_ETA_REL 1

typedef struct {
    double h, T;      /* Zeeman field, temperature (k_B = 1) */
    int32_t Lx, Ly;   /* lattice sizes, N = Lx * Ly momenta */
} or_point;

#define OR_OK 0
#define OR_EINVAL (-1)

static const double OR_PI = 3.14159265358979323846;

/* ---------------------------------------------------------------- helpers */

typedef struct { double s, c; } nsum;

static void nadd(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double nval(const nsum *a) { return a->s + a->c; }

/* -T ln(1 + exp(-E/T)), Eq. (5) summand, written without overflow. */
static double softplus_term(double E, double T)
{
    double lo = E < 0.0 ? E : 0.0;
    if (T == 0.0)
        return lo;
    return lo - T * log1p(exp(-fabs(E) / T));
}

/* s+- form factor of the pair (k up, -k+q down): eta(k) = cos kx cos ky on
 * the spin-up momentum, or eta(k - q/2) at the relative momentum. */
static double form_factor(int form, double kx, double ky, double qx, double qy)
{
    if (form == OR_ETA_REL)
        return cos(kx - 0.5 * qx) * cos(ky - 0.5 * qy);
    return cos(kx) * cos(ky);
}

/* Fermi function f(E) = 1 / (1 + exp(E/T)); T = 0 gives the step (1/2 at 0). */
static double fermi(double E, double T)
{
    if (T == 0.0)
        return E < 0.0 ? 1.0 : (E > 0.0 ? 0.0 : 0.5);
    if (E > 0.0) {
        double e = exp(-E / T);
        return e / (1.0 + e);
    }
    return 1.0 / (1.0 + exp(E / T));
}

/* ---------------------------------------------------------------- App. A */

/* Eq. (A.1)-(A.4): eigenvalue of the 2x2 orbital matrix T_k.
 * band 0 -> E_- (hole-like), band 1 -> E_+ (electron-like). */
double oracle_band_energy(const or_model *m, int band, double kx, double ky)
{
    double cx = cos(kx), cy = cos(ky), sx = sin(kx), sy = sin(ky);
    double T11 = -2.0 * (m->t1 * cx + m->t2 * cy) - 4.0 * m->t3 * cx * cy;
    double T22 = -2.0 * (m->t2 * cx + m->t1 * cy) - 4.0 * m->t3 * cx * cy;
    double T12 = -4.0 * m->t4 * sx * sy;
    double half_sum = 0.5 * (T11 + T22);
    double half_diff = 0.5 * (T11 - T22);
    double root = sqrt(half_diff * half_diff + T12 * T12);
    return band ? half_sum + root : half_sum - root;
}

/* Gradient of the (A.4) eigenvalue with respect to (kx, ky).  Where the two
 * bands touch (root = 0) the non-smooth part is given the symmetric
 * subgradient 0. */
void oracle_band_grad(const or_model *m, int band, double kx, double ky,
                      double *dEx, double *dEy)
{
    double cx = cos(kx), cy = cos(ky), sx = sin(kx), sy = sin(ky);
    double T11 = -2.0 * (m->t1 * cx + m->t2 * cy) - 4.0 * m->t3 * cx * cy;
    double T22 = -2.0 * (m->t2 * cx + m->t1 * cy) - 4.0 * m->t3 * cx * cy;
    double T12 = -4.0 * m->t4 * sx * sy;
    /* derivatives of the matrix elements */
    double dT11x = 2.0 * m->t1 * sx + 4.0 * m->t3 * sx * cy;
    double dT11y = 2.0 * m->t2 * sy + 4.0 * m->t3 * cx * sy;
    double dT22x = 2.0 * m->t2 * sx + 4.0 * m->t3 * sx * cy;
    double dT22y = 2.0 * m->t1 * sy + 4.0 * m->t3 * cx * sy;
    double dT12x = -4.0 * m->t4 * cx * sy;
    double dT12y = -4.0 * m->t4 * sx * cy;
    double half_diff = 0.5 * (T11 - T22);
    double root = sqrt(half_diff * half_diff + T12 * T12);
    double gx = 0.5 * (dT11x + dT22x);
    double gy = 0.5 * (dT11y + dT22y);
    if (root > 0.0) {
        double sgn = band ? 1.0 : -1.0;
        gx += sgn * (half_diff * 0.5 * (dT11x - dT22x) + T12 * dT12x) / root;
        gy += sgn * (half_diff * 0.5 * (dT11y - dT22y) + T12 * dT12y) / root;
    }
    *dEx = gx;
    *dEy = gy;
}

/* ---------------------------------------------------------------- checks */

static int check_model(const or_model *m)
{
    if (!m || (m->form != OR_ETA_K && m->form != OR_ETA_REL))
        return OR_EINVAL;
    const double *v = &m->t1;
    for (int i = 0; i < 7; ++i)
        if (!isfinite(v[i]))
            return OR_EINVAL;
    if (m->V[0] == 0.0 || m->V[1] == 0.0)
        return OR_EINVAL;
    return OR_OK;
}

static int check_point(const or_point *p)
{
    if (!isfinite(p->h) || !isfinite(p->T) || p->T < 0.0)
        return OR_EINVAL;
    if (p->Lx < 2 || p->Ly < 2)
        return OR_EINVAL;
    return OR_OK;
}

static int band_list(int bands, int *list)
{
    int nb = 0;
    if (bands & 1)
        list[nb++] = 0;
    if (bands & 2)
        list[nb++] = 1;
    return nb;
}

/* ------------------------------------------------- Eq. (4)-(5), Alg. 1 */

/* Eq. (4)-(5) summed over the zone for every Delta_i, from the per-k arrays
 * E_{eps k up}, E_{eps,-k+q,down}, E_{eps k down} and eta(k).  The Delta loop
 * is the OpenMP-parallel one; the k sum is Neumaier-compensated in the
 * arrays' (i-major) order. */
static void eq5_sum(long N, const double *e_up, const double *e_dn,
                    const double *e_kd, const double *eta, double V, double T,
                    const double *delta, int n_delta, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int id = 0; id < n_delta; ++id) {
        const double D = delta[id];
        nsum acc = {0.0, 0.0};
        for (long k = 0; k < N; ++k) {
            double gap = D * eta[k];                      /* Delta_{eps k} */
            double half_sum = 0.5 * (e_up[k] + e_dn[k]);
            double half_diff = 0.5 * (e_up[k] - e_dn[k]);
            double root = sqrt(half_sum * half_sum + gap * gap);
            double Ep = half_diff + root;                 /* Eq. (4), + */
            double Em = half_diff - root;                 /* Eq. (4), - */
            nadd(&acc, softplus_term(Ep, T));
            nadd(&acc, softplus_term(Em, T));
            nadd(&acc, e_kd[k]);
        }
        out[id] = nval(&acc) + (double)N * (-2.0 * D * D / V);
    }
}

/* Omega_eps(Delta_i, q) for every Delta_i, one band, one q, one point.
 * Follows Algorithm 1: the arrays E_{k up} and E_{-k+q down} are generated
 * once for the q, then for each Delta Eq. (4) and Eq. (5) are evaluated over
 * the whole zone.  The Delta loop is the OpenMP-parallel one. */
static void omega_row(const or_model *m, const or_point *p, int band,
                      double qx, double qy, const double *delta, int n_delta,
                      double *out)
{
    const int Lx = p->Lx, Ly = p->Ly;
    const long N = (long)Lx * Ly;
    const double h = p->h, T = p->T, mu = m->mu;
    double *e_up = (double *)malloc(sizeof(double) * N);   /* E_{eps k up}        */
    double *e_dn = (double *)malloc(sizeof(double) * N);   /* E_{eps,-k+q,down}   */
    double *e_kd = (double *)malloc(sizeof(double) * N);   /* E_{eps k down}      */
    double *eta = (double *)malloc(sizeof(double) * N);    /* cos kx cos ky       */

#pragma omp parallel for schedule(static)
    for (int i = 0; i < Lx; ++i) {
        double kx = 2.0 * OR_PI * i / Lx;
        for (int j = 0; j < Ly; ++j) {
            double ky = 2.0 * OR_PI * j / Ly;
            long k = (long)i * Ly + j;
            double Ek = oracle_band_energy(m, band, kx, ky);
            double Eqk = oracle_band_energy(m, band, qx - kx, qy - ky);
            e_up[k] = Ek - (mu + h);   /* sigma = +1 */
            e_dn[k] = Eqk - (mu - h);  /* sigma = -1 at -k+q */
            e_kd[k] = Ek - (mu - h);   /* sigma = -1 at k */
            eta[k] = form_factor(m->form, kx, ky, qx, qy);
        }
    }

    eq5_sum(N, e_up, e_dn, e_kd, eta, m->V[band], T, delta, n_delta, out);
    free(e_up);
    free(e_dn);
    free(e_kd);
    free(eta);
}

/* Omega grid, layout [pt][band][q][Delta] (Delta fastest).
 * q is [n_q][2] = (qx, qy).  bands: 1 = E_- only, 2 = E_+ only, 3 = both. */
int oracle_omega_grid(const or_model *m, const or_point *pts, int n_pts,
                      const double *delta, int n_delta, const double *q,
                      int n_q, int bands, double *out)
{
    if (check_model(m) || !pts || !delta || !q || !out)
        return OR_EINVAL;
    if (n_pts <= 0 || n_delta <= 0 || n_q <= 0 || bands < 1 || bands > 3)
        return OR_EINVAL;
    for (int p = 0; p < n_pts; ++p)
        if (check_point(&pts[p]))
            return OR_EINVAL;
    int list[2];
    int nb = band_list(bands, list);
    for (int p = 0; p < n_pts; ++p)
        for (int b = 0; b < nb; ++b)
            for (int iq = 0; iq < n_q; ++iq) {
                double *row = out + (((long)p * nb + b) * n_q + iq) * n_delta;
                omega_row(m, &pts[p], list[b], q[2 * iq], q[2 * iq + 1], delta,
                          n_delta, row);
            }
    return OR_OK;
}

/* Eq. (4)-(5) for one band, one q and one point from tabulated band
 * energies (the paper's recipe for models whose bands are found numerically,
 * Sec. 3.2, e.g. the three-band model of App. B): ek[i*Ly + j] = E_eps(k) and
 * eqk[i*Ly + j] = E_eps(q - k) at kx = 2 pi i / Lx, ky = 2 pi j / Ly;
 * (qx, qy) = q and form (OR_ETA_K or OR_ETA_REL) fix the form factor.
 * out[id] = Omega_eps(delta[id], q).  T >= 0, V != 0. */
int oracle_omega_row_tab(const double *ek, const double *eqk, int Lx, int Ly,
                         double mu, double h, double T, double V, double qx, double qy,
                         int form, const double *delta, int n_delta, double *out)
{
    if (!ek || !eqk || !delta || !out || Lx < 2 || Ly < 2 || n_delta <= 0)
        return OR_EINVAL;
    if (form != OR_ETA_K && form != OR_ETA_REL)
        return OR_EINVAL;
    if (!isfinite(mu) || !isfinite(h) || !isfinite(T) || T < 0.0 || V == 0.0 ||
        !isfinite(V))
        return OR_EINVAL;
    const long N = (long)Lx * Ly;
    double *e_up = (double *)malloc(sizeof(double) * N);
    double *e_dn = (double *)malloc(sizeof(double) * N);
    double *e_kd = (double *)malloc(sizeof(double) * N);
    double *eta = (double *)malloc(sizeof(double) * N);
    for (int i = 0; i < Lx; ++i) {
        double kx = 2.0 * OR_PI * i / Lx;
        for (int j = 0; j < Ly; ++j) {
            double ky = 2.0 * OR_PI * j / Ly;
            long k = (long)i * Ly + j;
            e_up[k] = ek[k] - (mu + h);
            e_dn[k] = eqk[k] - (mu - h);
            e_kd[k] = ek[k] - (mu - h);
            eta[k] = form_factor(form, kx, ky, qx, qy);
        }
    }
    eq5_sum(N, e_up, e_dn, e_kd, eta, V, T, delta, n_delta, out);
    free(e_up);
    free(e_dn);
    free(e_kd);
    free(eta);
    return OR_OK;
}

/* ------------------------------------------- App. C pair susceptibility */

/* Static Cooper-pair susceptibility of App. C at omega -> 0: with
 * E1 = E_{eps k up}, E2 = E_{eps',-k-q,down} and f the Fermi function the
 * retarded pair propagator gives the summand
 *   F(E1, E2) = (1 - f(E1) - f(E2)) / (E1 + E2)
 *             = (tanh(E1/2T) + tanh(E2/2T)) / (2 (E1 + E2)),
 * whose E1 + E2 -> 0 limit is 1 / (4 T cosh^2(E1/2T)).  Near that limit
 * (|E1 + E2| <= T) the sum of tanh is rewritten with
 * tanh a + tanh b = sinh(a + b) / (cosh a cosh b).  T = 0: the step
 * function, (sgn E1 + sgn E2) / (2 (E1 + E2)), and 0 where E1 + E2 = 0. */
static double pair_term(double E1, double E2, double T)
{
    double S = E1 + E2;
    if (T == 0.0) {
        if (S == 0.0)
            return 0.0;
        double s1 = (E1 > 0.0) - (E1 < 0.0), s2 = (E2 > 0.0) - (E2 < 0.0);
        return (s1 + s2) / (2.0 * S);
    }
    double x1 = E1 / (2.0 * T), x2 = E2 / (2.0 * T), u = x1 + x2;
    if (fabs(u) > 0.5)
        return (tanh(x1) + tanh(x2)) / (2.0 * S);
    double shc = u == 0.0 ? 1.0 : sinh(u) / u;
    return shc / (4.0 * T * cosh(x1) * cosh(x2));
}

/* chi_{eps eps'}(q) of App. C from tabulated energies: e1[i*Ly + j] =
 * E_eps(k), e2[i*Ly + j] = E_eps'(-k - q) at kx = 2 pi i/Lx, ky = 2 pi j/Ly;
 * structure factor eta(k) = 4 cos kx cos ky evaluated at -k - q.
 *   chi = (1/N) sum_k eta(-k-q)^2 F(E1 - mu - h, E2 - mu + h). */
int oracle_pair_chi_tab(const double *e1, const double *e2, int Lx, int Ly,
                        double mu, double h, double T, double qx, double qy,
                        double *out)
{
    if (!e1 || !e2 || !out || Lx < 2 || Ly < 2)
        return OR_EINVAL;
    if (!isfinite(mu) || !isfinite(h) || !isfinite(T) || T < 0.0)
        return OR_EINVAL;
    nsum acc = {0.0, 0.0};
    for (int i = 0; i < Lx; ++i) {
        double kx = 2.0 * OR_PI * i / Lx;
        for (int j = 0; j < Ly; ++j) {
            double ky = 2.0 * OR_PI * j / Ly;
            long k = (long)i * Ly + j;
            double eta = 4.0 * cos(-kx - qx) * cos(-ky - qy);
            nadd(&acc, eta * eta * pair_term(e1[k] - (mu + h), e2[k] - (mu - h), T));
        }
    }
    *out = nval(&acc) / ((double)Lx * Ly);
    return OR_OK;
}

/* chi_{eps eps'}(q) of the two-band model for every point, band pair and q:
 * out[((p * nb + a) * nb + b) * n_q + iq], a = eps, b = eps' over the
 * selected bands (bands mask as in oracle_omega_grid). */
int oracle_pair_chi(const or_model *m, const or_point *pts, int n_pts,
                    const double *q, int n_q, int bands, double *out)
{
    if (check_model(m) || !pts || !q || !out || n_pts <= 0 || n_q <= 0)
        return OR_EINVAL;
    if (bands < 1 || bands > 3)
        return OR_EINVAL;
    for (int p = 0; p < n_pts; ++p)
        if (check_point(&pts[p]))
            return OR_EINVAL;
    int list[2];
    int nb = band_list(bands, list);
    for (int p = 0; p < n_pts; ++p) {
        const int Lx = pts[p].Lx, Ly = pts[p].Ly;
        const long N = (long)Lx * Ly;
        double *e1 = (double *)malloc(sizeof(double) * N);
        double *e2 = (double *)malloc(sizeof(double) * N);
        int rc = OR_OK;
        for (int a = 0; a < nb && rc == OR_OK; ++a)
            for (int b = 0; b < nb && rc == OR_OK; ++b)
                for (int iq = 0; iq < n_q && rc == OR_OK; ++iq) {
                    double qx = q[2 * iq], qy = q[2 * iq + 1];
#pragma omp parallel for schedule(static)
                    for (int i = 0; i < Lx; ++i) {
                        double kx = 2.0 * OR_PI * i / Lx;
                        for (int j = 0; j < Ly; ++j) {
                            double ky = 2.0 * OR_PI * j / Ly;
                            e1[(long)i * Ly + j] = oracle_band_energy(m, list[a], kx, ky);
                            e2[(long)i * Ly + j] =
                                oracle_band_energy(m, list[b], -kx - qx, -ky - qy);
                        }
                    }
                    rc = oracle_pair_chi_tab(e1, e2, Lx, Ly, m->mu, pts[p].h, pts[p].T, qx,
                                             qy, out + ((long)(p * nb + a) * nb + b) * n_q + iq);
                }
        free(e1);
        free(e2);
        if (rc != OR_OK)
            return rc;
    }
    return OR_OK;
}

/* ------------------------------------------------------ Alg. 1 search */

/* Alg. 1, the two "find and save" steps, on a given grid [n_set][n_q][n_delta]
 * with the tie rule stated at the top of this file. */
int oracle_argmin_grid(const double *grid, int n_set, int n_q, int n_delta,
                       double tie_rel, int32_t *idx, double *omin,
                       int32_t *row_idx)
{
    if (!grid || !idx || !omin || n_set <= 0 || n_q <= 0 || n_delta <= 0)
        return OR_EINVAL;
    if (!(tie_rel >= 0.0) || !isfinite(tie_rel))
        return OR_EINVAL;
    for (int s = 0; s < n_set; ++s) {
        const double *g = grid + (long)s * n_q * n_delta;
        if (row_idx) {
            for (int iq = 0; iq < n_q; ++iq) {
                const double *row = g + (long)iq * n_delta;
                double best = NAN;
                for (int id = 0; id < n_delta; ++id)
                    if (!isnan(row[id]) && (isnan(best) || row[id] < best))
                        best = row[id];
                int pick = -1;
                if (!isnan(best)) {
                    double thr = best + tie_rel * fabs(best);
                    for (int id = 0; id < n_delta; ++id)
                        if (!isnan(row[id]) && row[id] <= thr) {
                            pick = id;
                            break;
                        }
                }
                row_idx[(long)s * n_q + iq] = pick;
            }
        }
        double best = NAN;
        for (long t = 0; t < (long)n_q * n_delta; ++t)
            if (!isnan(g[t]) && (isnan(best) || g[t] < best))
                best = g[t];
        int pd = -1, pq = -1;
        if (!isnan(best)) {
            double thr = best + tie_rel * fabs(best);
            for (int id = 0; id < n_delta && pd < 0; ++id)
                for (int iq = 0; iq < n_q; ++iq) {
                    double v = g[(long)iq * n_delta + id];
                    if (!isnan(v) && v <= thr) {
                        pd = id;
                        pq = iq;
                        break;
                    }
                }
        }
        idx[2 * s] = pd;
        idx[2 * s + 1] = pq;
        omin[s] = pd >= 0 ? g[(long)pq * n_delta + pd] : NAN;
    }
    return OR_OK;
}

int oracle_omega_argmin(const or_model *m, const or_point *pts, int n_pts,
                        const double *delta, int n_delta, const double *q,
                        int n_q, int bands, double tie_rel, int32_t *idx,
                        double *omin, int32_t *row_idx, double *omega_out)
{
    if (bands < 1 || bands > 3 || n_pts <= 0 || n_q <= 0 || n_delta <= 0)
        return OR_EINVAL;
    int list[2];
    int nb = band_list(bands, list);
    long n = (long)n_pts * nb * n_q * n_delta;
    double *g = omega_out ? omega_out : (double *)malloc(sizeof(double) * n);
    int rc = oracle_omega_grid(m, pts, n_pts, delta, n_delta, q, n_q, bands, g);
    if (rc == OR_OK)
        rc = oracle_argmin_grid(g, n_pts * nb, n_q, n_delta, tie_rel, idx, omin,
                                row_idx);
    if (!omega_out)
        free(g);
    return rc;
}

/* ------------------------------------------------- derivatives of Eq. (5) */

/* For one band and one point: Omega and its partial derivatives with respect
 * to Delta, qx, qy and mu, from differentiating Eq. (4)-(5) by hand:
 *   dOmega/dE for each quasiparticle branch is the Fermi function f(E);
 *   dE+-/dDelta = +- Delta eta^2 / R;
 *   dE+-/dq     = (dE_{q-k}/dq) (-1 +- s/R) / 2;
 *   dE+-/dmu    = -+ s / R, and the literal Sum_k E_{k down} adds -N;
 *   d(-2 N Delta^2 / V)/dDelta = -4 N Delta / V;
 *   with eta(k - q/2), also dE+-/dq = +- (Delta^2 eta / R) deta/dq, with
 *   deta/dqx = sin(kx - qx/2) cos(ky - qy/2) / 2 (likewise qy).
 * R = 0 is given s/R = 0 and Delta eta^2 / R = 0. */
static void grad_one(const or_model *m, const or_point *p, int band, double D,
                     double qx, double qy, double *om, double *gD, double *gqx,
                     double *gqy, double *gmu)
{
    const int Lx = p->Lx, Ly = p->Ly;
    const long N = (long)Lx * Ly;
    const double h = p->h, T = p->T, mu = m->mu, V = m->V[band];
    nsum so = {0, 0}, sd = {0, 0}, sx = {0, 0}, sy = {0, 0}, sm = {0, 0};
    for (int i = 0; i < Lx; ++i) {
        double kx = 2.0 * OR_PI * i / Lx;
        for (int j = 0; j < Ly; ++j) {
            double ky = 2.0 * OR_PI * j / Ly;
            double Ek = oracle_band_energy(m, band, kx, ky);
            double Eqk = oracle_band_energy(m, band, qx - kx, qy - ky);
            double bx, by;
            oracle_band_grad(m, band, qx - kx, qy - ky, &bx, &by);
            double a = Ek - (mu + h), b = Eqk - (mu - h);
            double eta = form_factor(m->form, kx, ky, qx, qy);
            double gap = D * eta;
            double s = 0.5 * (a + b), d = 0.5 * (a - b);
            double R = sqrt(s * s + gap * gap);
            double Ep = d + R, Em = d - R;
            double fp = fermi(Ep, T), fm = fermi(Em, T);
            double sr = R > 0.0 ? s / R : 0.0;
            double dr = R > 0.0 ? D * eta * eta / R : 0.0;
            nadd(&so, softplus_term(Ep, T));
            nadd(&so, softplus_term(Em, T));
            nadd(&so, Ek - (mu - h));
            nadd(&sd, dr * (fp - fm));
            double w = 0.5 * fp * (sr - 1.0) - 0.5 * fm * (sr + 1.0);
            double ex = 0.0, ey = 0.0;   /* form-factor part of dOmega/dq */
            if (m->form == OR_ETA_REL && R > 0.0) {
                double ge = D * gap / R * (fp - fm);    /* dOmega_k / d eta */
                ex = ge * 0.5 * sin(kx - 0.5 * qx) * cos(ky - 0.5 * qy);
                ey = ge * 0.5 * cos(kx - 0.5 * qx) * sin(ky - 0.5 * qy);
            }
            nadd(&sx, bx * w + ex);
            nadd(&sy, by * w + ey);
            nadd(&sm, sr * (fm - fp));
        }
    }
    *om = nval(&so) + (double)N * (-2.0 * D * D / V);
    *gD = nval(&sd) - 4.0 * (double)N * D / V;
    *gqx = nval(&sx);
    *gqy = nval(&sy);
    *gmu = nval(&sm) - (double)N;
}

/* Per point p: (Delta[p], q[p]) -> Omega, dOmega/dDelta, dOmega/dq (2),
 * dOmega/dmu for one band (0 = E_-, 1 = E_+). */
int oracle_omega_grad(const or_model *m, const or_point *pts, int n_pts,
                      const double *delta, const double *q, int band,
                      double *omega, double *dDelta, double *dq, double *dmu)
{
    if (check_model(m) || !pts || !delta || !q || n_pts <= 0)
        return OR_EINVAL;
    if (band != 0 && band != 1)
        return OR_EINVAL;
    if (!omega || !dDelta || !dq || !dmu)
        return OR_EINVAL;
    for (int p = 0; p < n_pts; ++p)
        if (check_point(&pts[p]))
            return OR_EINVAL;
#pragma omp parallel for schedule(dynamic, 1)
    for (int p = 0; p < n_pts; ++p)
        grad_one(m, &pts[p], band, delta[p], q[2 * p], q[2 * p + 1], &omega[p],
                 &dDelta[p], &dq[2 * p], &dq[2 * p + 1], &dmu[p]);
    return OR_OK;
}

/* Root of the gap equation dOmega/dDelta = 0 on (lo, hi] by bisection, for a
 * band, point and q.  Returns NaN when dOmega/dDelta does not change sign. */
double oracle_gap_root(const or_model *m, const or_point *p, int band,
                       double qx, double qy, double lo, double hi, double tol)
{
    double om, g_lo, g_hi, gx, gy, gm;
    grad_one(m, p, band, lo, qx, qy, &om, &g_lo, &gx, &gy, &gm);
    grad_one(m, p, band, hi, qx, qy, &om, &g_hi, &gx, &gy, &gm);
    if (!(g_lo < 0.0 && g_hi > 0.0))
        return NAN;
    for (int it = 0; it < 200 && hi - lo > tol; ++it) {
        double mid = 0.5 * (lo + hi), g_mid;
        grad_one(m, p, band, mid, qx, qy, &om, &g_mid, &gx, &gy, &gm);
        if (g_mid < 0.0)
            lo = mid;
        else
            hi = mid;
    }
    return 0.5 * (lo + hi);
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
