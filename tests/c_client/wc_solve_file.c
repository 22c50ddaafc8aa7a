/* A client of the solver library that uses nothing but the C ABI of wc.h and
 * the HIP runtime's C API: it reads gauge links and a source (canonical
 * complex128 layouts, raw binary files), solves D x = b on the GPU with the
 * default parameters, and writes x.
 *
 *   wc_solve_file Lx Ly Lz Lt kappa csw tol links.bin source.bin solution.bin
 *
 * Prints one line with the status and the solve's counters; exits 0 only
 * when every call returned WC_OK. */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "wc.h"

static int read_all(const char *path, void *buf, size_t bytes) {
    FILE *f = fopen(path, "rb");
    if (!f) return -1;
    size_t got = fread(buf, 1, bytes, f);
    fclose(f);
    return got == bytes ? 0 : -1;
}

static int write_all(const char *path, const void *buf, size_t bytes) {
    FILE *f = fopen(path, "wb");
    if (!f) return -1;
    size_t put = fwrite(buf, 1, bytes, f);
    fclose(f);
    return put == bytes ? 0 : -1;
}

int main(int argc, char **argv) {
    if (argc != 11) {
        fprintf(stderr, "usage: %s Lx Ly Lz Lt kappa csw tol links.bin source.bin solution.bin\n", argv[0]);
        return 2;
    }
    int dims[4];
    for (int d = 0; d < 4; d++) dims[d] = atoi(argv[1 + d]);
    const double kappa = atof(argv[5]), csw = atof(argv[6]), tol = atof(argv[7]);
    const size_t V = (size_t)dims[0] * dims[1] * dims[2] * dims[3];
    const size_t link_bytes = 4 * V * 9 * 16, spinor_bytes = V * 12 * 16;

    void *U = malloc(link_bytes), *b = malloc(spinor_bytes), *x = malloc(spinor_bytes);
    if (!U || !b || !x || read_all(argv[8], U, link_bytes) || read_all(argv[9], b, spinor_bytes)) {
        fprintf(stderr, "cannot read the input files\n");
        return 2;
    }
    void *U_dev = NULL, *b_dev = NULL, *x_dev = NULL;
    if (hipMalloc(&U_dev, link_bytes) != hipSuccess || hipMalloc(&b_dev, spinor_bytes) != hipSuccess ||
        hipMalloc(&x_dev, spinor_bytes) != hipSuccess) {
        fprintf(stderr, "device allocation failed\n");
        return 2;
    }
    if (hipMemcpy(U_dev, U, link_bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b_dev, b, spinor_bytes, hipMemcpyHostToDevice) != hipSuccess) {
        fprintf(stderr, "copy to the device failed\n");
        return 2;
    }

    wc_lattice *lat = NULL;
    int rc = wc_create_lattice(dims, NULL, &lat);
    if (rc == WC_OK) rc = wc_load_links(lat, U_dev);
    wc_solve_info info;
    if (rc == WC_OK) {
        wc_solve_params p;
        wc_solve_params_default(&p);
        rc = wc_solve(lat, b_dev, kappa, csw, tol, &p, x_dev, 0, &info);
    }
    if (rc != WC_OK) {
        fprintf(stderr, "wc call failed (%d): %s\n", rc, wc_last_error());
    } else {
        printf("status %d outer %d inner %d true_rel_residual %.6e\n", info.status, info.outer_iters,
               info.inner_iters_total, info.true_rel_residual);
        if (hipMemcpy(x, x_dev, spinor_bytes, hipMemcpyDeviceToHost) != hipSuccess ||
            write_all(argv[10], x, spinor_bytes)) {
            fprintf(stderr, "cannot write the solution\n");
            rc = -100;
        }
    }
    wc_destroy_lattice(lat);
    hipFree(U_dev);
    hipFree(b_dev);
    hipFree(x_dev);
    free(U);
    free(b);
    free(x);
    return rc == WC_OK ? 0 : 1;
}
