/* Drives every exported routine of the FP64 oracle (oracle/omega_oracle.c,
 * compiled into this program) on small lattices, ragged sizes, NaN inputs
 * and invalid arguments, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer.  Exits 0 when every call returns what it should
 * and every finite input gives a finite result; the sanitizers abort on the
 * first out-of-bounds access, leak or undefined operation. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "omega_oracle.c"

#define CHECK(c)                                                 \
    do {                                                         \
        if (!(c)) {                                              \
            printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);   \
            return 1;                                            \
        }                                                        \
    } while (0)

static int all_finite(const double *x, long n)
{
    for (long i = 0; i < n; ++i)
        if (!isfinite(x[i]))
            return 0;
    return 1;
}

int main(void)
{
    or_model m = {-1.0, 1.3, -0.85, -0.85, 1.54, {-16.0, -7.5}, OR_ETA_K, 0};
    const or_point pts[3] = {{0.1, 0.002, 6, 5}, {0.0, 0.0, 2, 2}, {-0.2, 0.3, 3, 7}};
    const double delta[5] = {0.0, 0.1, 0.25, 0.6, 1.1};
    const double q[3 * 2] = {0.0, 0.0, 0.3, 0.0, 2.0 * OR_PI / 6.0, 2.0 * OR_PI / 5.0};
    enum { NP = 3, NB = 2, NQ = 3, ND = 5 };
    double *grid = malloc(sizeof(double) * NP * NB * NQ * ND);
    double *grid2 = malloc(sizeof(double) * NP * NB * NQ * ND);
    int32_t idx[NP * NB * 2], row_idx[NP * NB * NQ];
    double omin[NP * NB];

    for (int form = OR_ETA_K; form <= OR_ETA_REL; ++form) {
        m.form = form;
        for (int bands = 1; bands <= 3; ++bands) {
            const int nb = bands == 3 ? 2 : 1;
            CHECK(oracle_omega_grid(&m, pts, NP, delta, ND, q, NQ, bands, grid) == OR_OK);
            CHECK(all_finite(grid, (long)NP * nb * NQ * ND));
            CHECK(oracle_omega_argmin(&m, pts, NP, delta, ND, q, NQ, bands, 1e-11, idx, omin,
                                      row_idx, grid2) == OR_OK);
            for (long i = 0; i < (long)NP * nb * NQ * ND; ++i)
                CHECK(grid2[i] == grid[i]);
            for (int s = 0; s < NP * nb; ++s)
                CHECK(idx[2 * s] >= 0 && idx[2 * s] < ND && idx[2 * s + 1] >= 0 &&
                      idx[2 * s + 1] < NQ);
        }
        /* gradient at one (Delta, q) per point and band */
        double d1[NP] = {0.2, 0.0, 0.4}, q1[2 * NP] = {0.1, 0.0, 0.0, 0.0, 0.3, 0.2};
        double om[NP], gd[NP], gq[2 * NP], gm[NP];
        for (int band = 0; band < 2; ++band) {
            CHECK(oracle_omega_grad(&m, pts, NP, d1, q1, band, om, gd, gq, gm) == OR_OK);
            CHECK(all_finite(om, NP) && all_finite(gd, NP) && all_finite(gq, 2 * NP) &&
                  all_finite(gm, NP));
        }
        const double root = oracle_gap_root(&m, &pts[0], 0, 0.0, 0.0, 1e-6, 1.0, 1e-12);
        CHECK(isfinite(root) || isnan(root));
    }
    m.form = OR_ETA_K;

    /* tabulated-band routines on a ragged lattice */
    {
        const int Lx = 5, Ly = 3;
        double ek[15], eqk[15], row[ND], chi;
        for (int i = 0; i < Lx; ++i)
            for (int j = 0; j < Ly; ++j) {
                const double kx = 2.0 * OR_PI * i / Lx, ky = 2.0 * OR_PI * j / Ly;
                ek[i * Ly + j] = oracle_band_energy(&m, 1, kx, ky);
                eqk[i * Ly + j] = oracle_band_energy(&m, 1, 0.4 - kx, -ky);
            }
        CHECK(oracle_omega_row_tab(ek, eqk, Lx, Ly, m.mu, 0.05, 0.01, -7.5, 0.4, 0.0,
                                   OR_ETA_REL, delta, ND, row) == OR_OK);
        CHECK(all_finite(row, ND));
        CHECK(oracle_pair_chi_tab(ek, eqk, Lx, Ly, m.mu, 0.05, 0.0, 0.4, 0.0, &chi) == OR_OK);
        CHECK(isfinite(chi));
        CHECK(oracle_omega_row_tab(ek, eqk, 1, Ly, m.mu, 0.0, 0.01, -7.5, 0.0, 0.0, OR_ETA_K,
                                   delta, ND, row) == OR_EINVAL);
    }

    /* pair susceptibility of the two-band model */
    {
        double chi[NP * 2 * 2 * NQ];
        CHECK(oracle_pair_chi(&m, pts, NP, q, NQ, 3, chi) == OR_OK);
        CHECK(all_finite(chi, NP * 4 * NQ));
    }

    /* argmin over grids with NaN: never chosen; an all-NaN set gives -1 */
    {
        double g[2 * 2 * 3];
        for (int i = 0; i < 12; ++i)
            g[i] = (double)((i * 7) % 5);
        g[3] = NAN;
        for (int i = 6; i < 12; ++i)
            g[i] = NAN;
        int32_t ix[4], rx[4];
        double mn[2];
        CHECK(oracle_argmin_grid(g, 2, 2, 3, 1e-11, ix, mn, rx) == OR_OK);
        CHECK(ix[0] >= 0 && ix[2] == -1 && ix[3] == -1 && isnan(mn[1]));
    }

    /* invalid arguments are refused before any work */
    {
        or_model bad = m;
        bad.V[1] = 0.0;
        CHECK(oracle_omega_grid(&bad, pts, NP, delta, ND, q, NQ, 3, grid) == OR_EINVAL);
        bad = m;
        bad.form = 7;
        CHECK(oracle_omega_grid(&bad, pts, NP, delta, ND, q, NQ, 3, grid) == OR_EINVAL);
        bad = m;
        bad.mu = NAN;
        CHECK(oracle_omega_grid(&bad, pts, NP, delta, ND, q, NQ, 3, grid) == OR_EINVAL);
        or_point bp = {0.0, -1.0, 4, 4};
        CHECK(oracle_omega_grid(&m, &bp, 1, delta, ND, q, NQ, 3, grid) == OR_EINVAL);
        bp.T = 0.0;
        bp.Lx = 1;
        CHECK(oracle_omega_grid(&m, &bp, 1, delta, ND, q, NQ, 3, grid) == OR_EINVAL);
        CHECK(oracle_omega_grid(&m, pts, NP, delta, 0, q, NQ, 3, grid) == OR_EINVAL);
        CHECK(oracle_omega_grid(&m, pts, NP, delta, ND, q, NQ, 4, grid) == OR_EINVAL);
        CHECK(oracle_omega_grid(&m, pts, NP, delta, ND, q, NQ, 3, NULL) == OR_EINVAL);
        CHECK(oracle_argmin_grid(grid, 0, NQ, ND, 1e-11, idx, omin, row_idx) == OR_EINVAL);
    }

    /* NaN Delta propagates into the grid without touching other rows */
    {
        const double dn[2] = {NAN, 0.2};
        double out[2];
        CHECK(oracle_omega_grid(&m, pts, 1, dn, 2, q, 1, 1, out) == OR_OK);
        CHECK(isnan(out[0]) && isfinite(out[1]));
    }

    oracle_set_threads(1);
    CHECK(oracle_max_threads() >= 1);
    free(grid);
    free(grid2);
    printf("ok\n");
    return 0;
}
