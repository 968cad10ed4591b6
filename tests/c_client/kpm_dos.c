/*
 * A plain C99 client of the library's C ABI (no C++, no Python): KPM density
 * of states of a disordered 3D topological insulator (Sec. 2.2; moments and
 * the Jackson-damped DOS of Sec. 4), with the field generated in the sweep
 * kernels (Sec. 3.3) and random-phase start columns made on the device.
 *
 *   kpm_dos Lx Ly Lz nb M field_seed W vec_seed
 *
 * prints "mu <column> <n> <value>" for every moment, then "dos <E> <rho>" for
 * the column mean on a few energies.  Without a GPU it checks that argument
 * errors come back before any device call, prints "no-device <status>" and
 * exits 0.  Any other failure prints the library's message and exits 1.
 */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "pvdtm.h"

#define CHECK(call)                                                                       \
    do {                                                                                  \
        pv_status st_ = (call);                                                           \
        if (st_ != PV_OK) {                                                               \
            fprintf(stderr, "%s: %s (%s)\n", #call, pv_status_string(st_), pv_last_error()); \
            return 1;                                                                     \
        }                                                                                 \
    } while (0)

int main(int argc, char** argv) {
    if (argc != 9) {
        fprintf(stderr, "usage: %s Lx Ly Lz nb M field_seed W vec_seed\n", argv[0]);
        return 2;
    }
    const int64_t L[3] = {atoll(argv[1]), atoll(argv[2]), atoll(argv[3])};
    const int nb = atoi(argv[4]), M = atoi(argv[5]);
    const uint64_t field_seed = strtoull(argv[6], NULL, 10), vec_seed = strtoull(argv[8], NULL, 10);
    const double W = atof(argv[7]);

    /* the TI stencil of Sec. 2.2 with t = 1, m = 2 */
    static int offsets[PV_MAX_TERMS * 3];
    static double blocks[PV_MAX_TERMS * PV_MAX_ORB * PV_MAX_ORB * 2];
    static double onsite[PV_MAX_ORB * PV_MAX_ORB * 2];
    const double params[4] = {1.0, 2.0, 0.0, 0.0};
    int dim, n_orb, n_terms, pot_mode;
    CHECK(pv_model_stencil(PV_MODEL_TI, params, &dim, &n_orb, &n_terms, offsets, blocks, onsite, &pot_mode));
    pv_lattice_desc d;
    d.dim = dim;
    d.L[0] = L[0];
    d.L[1] = L[1];
    d.L[2] = L[2];
    d.n_orb = n_orb;
    d.periodic[0] = d.periodic[1] = d.periodic[2] = 1;
    d.n_terms = n_terms;
    d.offsets = offsets;
    d.blocks = blocks;
    d.onsite = onsite;
    d.pot_mode = pot_mode;
    d.flags = PV_CHECK_HERMITIAN;
    pv_lattice* lat = NULL;
    CHECK(pv_lattice_create(&d, &lat));
    int64_t n_sites, n_rows;
    int family;
    CHECK(pv_lattice_info(lat, &n_sites, &n_rows, &family));
    CHECK(pv_lattice_set_random_potential(lat, field_seed, W));

    /* argument errors are reported before any device use */
    if (pv_kpm_moments(lat, PV_C128, nb, M + 1, 7.0, 0.0, NULL, NULL, NULL, 0, NULL) != PV_ERR_INVALID_ARG) {
        fprintf(stderr, "odd M was not rejected\n");
        return 1;
    }

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        void* fake = (void*)(uintptr_t)(1u << 20);
        pv_status st = pv_random_block(lat, PV_C128, nb, vec_seed, PV_RANDOM_PHASE, 0, fake, NULL);
        printf("no-device %d\n", (int)st);
        pv_lattice_destroy(lat);
        return st == PV_OK ? 1 : 0;
    }

    const size_t vec_bytes = (size_t)n_rows * (size_t)nb * 16u;
    const size_t ws_bytes = pv_kpm_workspace_size(lat, PV_C128, nb, M);
    void *r = NULL, *ws = NULL;
    double* mu_dev = NULL;
    if (ws_bytes == 0 || hipMalloc(&r, vec_bytes) != hipSuccess || hipMalloc(&ws, ws_bytes) != hipSuccess ||
        hipMalloc((void**)&mu_dev, sizeof(double) * (size_t)nb * (size_t)M) != hipSuccess) {
        fprintf(stderr, "device allocation failed\n");
        return 1;
    }
    CHECK(pv_random_block(lat, PV_C128, nb, vec_seed, PV_RANDOM_PHASE, 0, r, NULL));
    CHECK(pv_kpm_moments(lat, PV_C128, nb, M, 7.0, 0.0, r, mu_dev, ws, ws_bytes, NULL));
    double* mu = (double*)malloc(sizeof(double) * (size_t)nb * (size_t)M);
    double* mean = (double*)calloc((size_t)M, sizeof(double));
    if (!mu || !mean || hipMemcpy(mu, mu_dev, sizeof(double) * (size_t)nb * (size_t)M, hipMemcpyDeviceToHost) != hipSuccess) {
        fprintf(stderr, "copy of the moments failed\n");
        return 1;
    }
    for (int c = 0; c < nb; ++c)
        for (int n = 0; n < M; ++n) {
            printf("mu %d %d %.17g\n", c, n, mu[(size_t)c * M + n]);
            mean[n] += mu[(size_t)c * M + n] / nb;
        }
    double E[5] = {-4.0, -1.0, 0.0, 1.5, 3.0}, rho[5];
    CHECK(pv_kpm_dos(M, mean, 7.0, 0.0, 5, E, rho));
    for (int k = 0; k < 5; ++k) printf("dos %.17g %.17g\n", E[k], rho[k]);
    free(mu);
    free(mean);
    (void)hipFree(r);
    (void)hipFree(ws);
    (void)hipFree(mu_dev);
    pv_lattice_destroy(lat);
    return 0;
}
