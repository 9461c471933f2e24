/* A plain C client of libomega's interface (include/omega.h): the host-only
 * entry points and the host-side validation, no GPU needed.  Exits 0 when
 * every check holds and prints the first failing one otherwise. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "omega.h"

#define CHECK(c)                                                 \
    do {                                                         \
        if (!(c)) {                                              \
            printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);   \
            return 1;                                            \
        }                                                        \
    } while (0)

int main(void)
{
    CHECK(omega_version() == 4);
    CHECK(strcmp(omega_strerror(OMEGA_OK), "success") == 0);
    CHECK(strcmp(omega_strerror(OMEGA_E_WORKSPACE), "workspace too small") == 0);

    /* symmetry wedge of an 8 x 8 lattice: 15 orbits covering 64 momenta */
    double q[2 * 64];
    int32_t orbit[64];
    const int n = omega_q_wedge(8, 8, q, orbit, 64);
    CHECK(n == 15);
    int total = 0;
    for (int i = 0; i < n; ++i)
        total += orbit[i];
    CHECK(total == 64);
    CHECK(q[0] == 0.0 && q[1] == 0.0 && orbit[0] == 1);
    const double pi = 3.14159265358979323846;
    CHECK(fabs(q[2 * 14] - pi) < 1e-15 && fabs(q[2 * 14 + 1] - pi) < 1e-15);
    CHECK(omega_q_wedge(8, 8, NULL, NULL, 0) == 15);
    CHECK(omega_q_wedge(8, 8, q, orbit, 3) == OMEGA_E_WORKSPACE);

    /* workspace queries */
    omega_point pt = {0.1, 0.002, 64, 64};
    const size_t ws = omega_workspace_bytes(&pt, 1, 32, 4, OMEGA_BAND_BOTH, OMEGA_FP64, 0);
    CHECK(ws > 0);
    CHECK(omega_workspace_bytes(&pt, 1, 0, 4, OMEGA_BAND_BOTH, OMEGA_FP64, 0) == 0);
    CHECK(omega3_workspace_bytes(&pt, 1, 32, 4, OMEGA3_BAND_ALL, OMEGA_FP64) > 0);
    CHECK(omega_chi_workspace_bytes(&pt, 1, 4, OMEGA_BAND_BOTH) > 0);

    /* host-side validation fails before anything is enqueued */
    omega_model m = {-1.0, 1.3, -0.85, -0.85, 1.54, {-16.0, -7.5}, OMEGA_ETA_K, 0};
    void *fake = (void *)0x1000;
    CHECK(omega_grid(&m, &pt, 1, fake, 32, fake, 4, 0, OMEGA_FP64, fake, ws, fake, NULL) ==
          OMEGA_E_INVAL);
    CHECK(omega_grid(&m, &pt, 1, fake, 32, fake, 4, OMEGA_BAND_BOTH, OMEGA_FP64, fake, 16,
                     fake, NULL) == OMEGA_E_WORKSPACE);
    m.form = 2;   /* no such form factor */
    CHECK(omega_grid(&m, &pt, 1, fake, 32, fake, 4, OMEGA_BAND_BOTH, OMEGA_FP64, fake, ws,
                     fake, NULL) == OMEGA_E_INVAL);
    m.form = OMEGA_ETA_REL;
    m.V[1] = 0.0;
    CHECK(omega_grid(&m, &pt, 1, fake, 32, fake, 4, OMEGA_BAND_BOTH, OMEGA_FP64, fake, ws,
                     fake, NULL) == OMEGA_E_INVAL);
    omega_point bad = {0.0, -1.0, 64, 64};
    CHECK(omega_workspace_bytes(&bad, 1, 32, 4, OMEGA_BAND_BOTH, OMEGA_FP64, 0) == 0);
    printf("ok\n");
    return 0;
}
