/* A plain C11 program that runs one freezing-droplet solve through the library's C ABI
 * alone: no Python and no torch, device memory from the HIP runtime, the default stream.
 *
 *   c_consumer NX NY PRECISION STEPS OUT
 *
 * fills the parameters with lbfs_params_default, allocates lbfs_state_bytes of device
 * memory, initialises (Table 1, initialisation), takes STEPS time steps, and writes to
 * OUT, as native doubles: the step count, time, liquid fraction, solid ratio (Eq. 51),
 * volume, height and max |u| of lbfs_observe, then the order parameter C and the
 * enthalpy He (NX x NY each, row-major) read back with lbfs_read_field. Exit status 0 on
 * success; otherwise the failing call and its status are printed. */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "lbfs.h"

static int fail(const char* what, int status)
{
    fprintf(stderr, "c_consumer: %s: %s (%d)\n", what, lbfs_strerror(status), status);
    return 1;
}

int main(int argc, char** argv)
{
    if (argc != 6) {
        fprintf(stderr, "usage: %s NX NY PRECISION STEPS OUT\n", argv[0]);
        return 2;
    }
    const int nx = atoi(argv[1]), ny = atoi(argv[2]), prec = atoi(argv[3]), steps = atoi(argv[4]);
    lbfs_params p;
    int rc = lbfs_params_default(&p, nx, ny, prec);
    if (rc != LBFS_OK) return fail("lbfs_params_default", rc);
    const size_t bytes = lbfs_state_bytes(&p);
    if (bytes == 0) return fail("lbfs_state_bytes", LBFS_E_INVAL);

    void* dev = NULL;
    if (hipMalloc(&dev, bytes) != hipSuccess) {
        fprintf(stderr, "c_consumer: hipMalloc of %zu bytes failed\n", bytes);
        return 1;
    }
    lbfs_solver* s = NULL;
    rc = lbfs_init(&p, dev, bytes, NULL, &s);
    if (rc != LBFS_OK) return fail("lbfs_init", rc);
    rc = lbfs_step(s, steps);
    if (rc != LBFS_OK) return fail("lbfs_step", rc);
    lbfs_observables o;
    rc = lbfs_observe(s, &o);
    if (rc != LBFS_OK) return fail("lbfs_observe", rc);

    const size_t n = (size_t)nx * (size_t)ny;
    double* host = malloc(2 * n * sizeof(double));
    if (!host) return 1;
    rc = lbfs_read_field(s, LBFS_FIELD_C, host, n);
    if (rc != LBFS_OK) return fail("lbfs_read_field C", rc);
    rc = lbfs_read_field(s, LBFS_FIELD_HE, host + n, n);
    if (rc != LBFS_OK) return fail("lbfs_read_field He", rc);

    const double head[7] = {(double)o.step, o.t, o.liquid_fraction, o.solid_ratio, o.volume, o.height, o.umax};
    FILE* f = fopen(argv[5], "wb");
    if (!f || fwrite(head, sizeof(double), 7, f) != 7 || fwrite(host, sizeof(double), 2 * n, f) != 2 * n) {
        fprintf(stderr, "c_consumer: cannot write %s\n", argv[5]);
        return 1;
    }
    fclose(f);
    printf("c_consumer: %dx%d %s, %d steps, liquid fraction %.6f\n", nx, ny, prec ? "FP64" : "FP32", steps,
           o.liquid_fraction);
    free(host);
    lbfs_destroy(s);
    hipFree(dev);
    return 0;
}
