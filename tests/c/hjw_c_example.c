/* A plain C99 use of the library's C ABI: device memory from the HIP runtime, no
 * Python.  Reads phi0 of an n x n periodic grid over [-2, 2)^2 from a file (FP64,
 * row-major), solves phi_t + (phi_x + phi_y + 1)^2 / 2 = 0 in FP64 to t = 0.02 with
 * CFL 0.5, and writes phi to a file.  Prints the steps taken.
 *
 * usage: hjw_c_example n phi0.bin phi.bin
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "hjw.h"

#define CHECK(call)                                                                  \
    do {                                                                             \
        const hjw_status st_ = (call);                                               \
        if (st_ != HJW_OK) {                                                         \
            fprintf(stderr, "%s failed (%d): %s\n", #call, (int)st_, hjw_last_error()); \
            return 1;                                                                \
        }                                                                            \
    } while (0)

static int read_all(const char *path, double *buf, size_t count) {
    FILE *f = fopen(path, "rb");
    if (!f) return -1;
    const size_t got = fread(buf, sizeof(double), count, f);
    fclose(f);
    return got == count ? 0 : -1;
}

static int write_all(const char *path, const double *buf, size_t count) {
    FILE *f = fopen(path, "wb");
    if (!f) return -1;
    const size_t put = fwrite(buf, sizeof(double), count, f);
    fclose(f);
    return put == count ? 0 : -1;
}

int main(int argc, char **argv) {
    if (argc != 4) {
        fprintf(stderr, "usage: %s n phi0.bin phi.bin\n", argv[0]);
        return 2;
    }
    const int64_t n = atoll(argv[1]);
    const size_t cells = (size_t)(n * n);
    double *phi = malloc(cells * sizeof(double));
    if (!phi || read_all(argv[2], phi, cells) != 0) {
        fprintf(stderr, "cannot read %s\n", argv[2]);
        return 1;
    }
    const int64_t dims[2] = {n, n};
    const double lo[2] = {-2.0, -2.0}, hi[2] = {2.0, 2.0};
    const int bc[2] = {HJW_BC_PERIODIC, HJW_BC_PERIODIC};
    hjw_grid *g = NULL;
    CHECK(hjw_grid_create(2, dims, lo, hi, bc, HJW_FP64, &g));
    size_t bytes = 0;
    CHECK(hjw_workspace_bytes(g, &bytes));
    void *ws = NULL;
    if (hipMalloc(&ws, bytes) != hipSuccess) {
        fprintf(stderr, "hipMalloc of %zu bytes failed\n", bytes);
        return 1;
    }
    CHECK(hjw_bind(g, ws, bytes, NULL));
    const double params[3] = {1.0, 1.0, 1.0};
    CHECK(hjw_set_hamiltonian(g, HJW_H_BURGERS, params, 3));
    CHECK(hjw_set_phi(g, phi, 0));
    hjw_info info;
    CHECK(hjw_step_to(g, 0.02, 0.5, 0, &info));
    CHECK(hjw_get_phi(g, phi, 0));
    hjw_grid_destroy(g);
    (void)hipFree(ws);
    if (write_all(argv[3], phi, cells) != 0) {
        fprintf(stderr, "cannot write %s\n", argv[3]);
        return 1;
    }
    printf("steps %lld t %.17g\n", (long long)info.steps, info.t);
    free(phi);
    return 0;
}
