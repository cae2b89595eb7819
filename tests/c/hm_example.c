/*
 * A C program that uses only the C ABI (include/hmdd.h) and the HIP
 * runtime: a 24 x 16 planar fault of 1 m squares, its H-matrix operator,
 * b = E x for x = 1, a GMRES solve of E y = b, and one step of the
 * interface law for two elements.  Prints one line per stage; exits with
 * a nonzero status on the first error.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "hmdd.h"

#define CHECK(call)                                                             \
    do {                                                                        \
        hm_status st_ = (call);                                                 \
        if (st_ != HM_OK) {                                                     \
            fprintf(stderr, "%s failed (%d): %s\n", #call, (int)st_, hm_last_error()); \
            return 1;                                                           \
        }                                                                       \
    } while (0)

#define HIPCHECK(call)                                                          \
    do {                                                                        \
        if ((call) != hipSuccess) {                                             \
            fprintf(stderr, "%s failed\n", #call);                              \
            return 1;                                                           \
        }                                                                       \
    } while (0)

int main(void)
{
    const int nx = 24, ny = 16;
    const int64_t nv = (int64_t)(nx + 1) * (ny + 1), ne = (int64_t)nx * ny, n = 3 * ne;
    double* xyz = malloc(sizeof(double) * 3 * nv);
    int64_t* conn = malloc(sizeof(int64_t) * 4 * ne);
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            double* p = xyz + 3 * ((int64_t)j * (nx + 1) + i);
            p[0] = i;
            p[1] = j;
            p[2] = 0.0;
        }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            int64_t* c = conn + 4 * ((int64_t)j * nx + i);
            c[0] = (int64_t)j * (nx + 1) + i;
            c[1] = c[0] + 1;
            c[2] = c[1] + nx + 1;
            c[3] = c[0] + nx + 1;
        }

    size_t sizes[] = HM_ABI_SIZES;
    CHECK(hm_abi_check(HM_ABI_N_STRUCTS, sizes));
    hm_mesh* mesh = NULL;
    CHECK(hm_mesh_create(4, nv, xyz, ne, conn, &mesh));
    hm_build_opts bo;
    hm_build_opts_default(&bo);
    bo.leaf_size = 32;
    bo.aca_tol = 1e-8;
    hm_op* op = NULL;
    CHECK(hm_operator_build(mesh, 30e9, 0.25, &bo, NULL, &op));
    hm_op_stats stats;
    CHECK(hm_operator_stats(op, &stats));
    printf("operator: %lld elements, %lld dense and %lld low-rank blocks\n", (long long)stats.n_elements,
           (long long)stats.n_dense_blocks, (long long)stats.n_lowrank_blocks);

    double* x = malloc(sizeof(double) * n);
    double* y = malloc(sizeof(double) * n);
    for (int64_t i = 0; i < n; ++i) x[i] = 1.0;
    double *d_x, *d_b, *d_y;
    HIPCHECK(hipMalloc((void**)&d_x, sizeof(double) * n));
    HIPCHECK(hipMalloc((void**)&d_b, sizeof(double) * n));
    HIPCHECK(hipMalloc((void**)&d_y, sizeof(double) * n));
    HIPCHECK(hipMemcpy(d_x, x, sizeof(double) * n, hipMemcpyHostToDevice));
    CHECK(hm_operator_apply(op, 1, d_x, n, d_b, n, 0u, NULL));
    HIPCHECK(hipMemcpy(y, d_b, sizeof(double) * n, hipMemcpyDeviceToHost));
    printf("product: b[n] of the centre element = %.6e Pa\n", y[3 * (ne / 2 + nx / 2) + 2]);

    hm_solve_opts so;
    hm_solve_opts_default(&so);
    so.rtol = 1e-10;
    hm_solve_report rep;
    CHECK(hm_solve(op, &so, 1, d_b, n, d_y, n, &rep, NULL));
    HIPCHECK(hipMemcpy(y, d_y, sizeof(double) * n, hipMemcpyDeviceToHost));
    double e2 = 0.0, x2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        e2 += (y[i] - x[i]) * (y[i] - x[i]);
        x2 += x[i] * x[i];
    }
    printf("solve: %d iterations, relative error %.3e\n", rep.iterations, sqrt(e2 / x2));

    /* one interface-law step: an elastic and a sliding element of a frictional fault */
    hm_interface_material m = {3.2e10, 3.2e10, 0.6, 0.6, 0.0, 0.0, 0.0, 0.0, 0.0};
    const double dd[6] = {1e-5, 0, 0, 1e-3, 0, 0}, t0[6] = {1e6, 0, -10e6, 5.9e6, 0, -10e6};
    const double zero[6] = {0, 0, 0, 0, 0, 0};
    double* d_in;
    double* d_out;
    int32_t* d_mode;
    HIPCHECK(hipMalloc((void**)&d_in, sizeof(double) * 24));
    HIPCHECK(hipMalloc((void**)&d_out, sizeof(double) * 36));
    HIPCHECK(hipMalloc((void**)&d_mode, sizeof(int32_t) * 2));
    HIPCHECK(hipMemcpy(d_in, dd, sizeof dd, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(d_in + 6, t0, sizeof t0, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(d_in + 12, zero, sizeof zero, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(d_in + 18, zero, sizeof zero, hipMemcpyHostToDevice));
    CHECK(hm_interface_update(1, &m, 2, NULL, d_in, d_in + 6, d_in + 12, d_in + 18, d_out, d_out + 6, d_out + 12,
                              d_out + 18, d_mode, NULL, NULL, NULL));
    double t1[6];
    int32_t mode[2];
    HIPCHECK(hipMemcpy(t1, d_out, sizeof t1, hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(mode, d_mode, sizeof mode, hipMemcpyDeviceToHost));
    printf("interface: modes %d %d, shear tractions %.6e %.6e Pa\n", mode[0], mode[1], t1[0], t1[3]);

    hipFree(d_x);
    hipFree(d_b);
    hipFree(d_y);
    hipFree(d_in);
    hipFree(d_out);
    hipFree(d_mode);
    hm_op_destroy(op);
    hm_mesh_destroy(mesh);
    free(xyz);
    free(conn);
    free(x);
    free(y);
    return 0;
}
