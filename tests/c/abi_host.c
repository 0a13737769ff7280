/* A plain C consumer of the library's C ABI (include/sesub.h), host calls only:
 * mesh creation without a device, the host copies of the reordered mesh and its
 * geometry, plan statistics, the AB3-AM4 coefficients and the error paths.  It
 * prints "key value ..." lines that tests/test_c_abi_host.py compares with the
 * Python binding and with closed forms.  No torch, no Python, no GPU. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sesub.h"

#define CHECK(call)                                                                 \
    do {                                                                            \
        se_status st_ = (call);                                                     \
        if (st_ != SE_OK) {                                                         \
            fprintf(stderr, "%s failed: %d (%s)\n", #call, (int)st_, se_last_error()); \
            return 1;                                                               \
        }                                                                           \
    } while (0)

/* n x n vertex grid of spacing h on [0, (n-1) h]^2, two counter-clockwise
 * triangles per cell */
static void grid(int n, double h, double *x, double *y, int32_t *tri) {
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            x[j * n + i] = i * h;
            y[j * n + i] = j * h;
        }
    int e = 0;
    for (int j = 0; j + 1 < n; ++j)
        for (int i = 0; i + 1 < n; ++i) {
            const int32_t a = j * n + i, b = a + 1, c = a + n, d = c + 1;
            tri[3 * e] = a; tri[3 * e + 1] = b; tri[3 * e + 2] = d; ++e;
            tri[3 * e] = a; tri[3 * e + 1] = d; tri[3 * e + 2] = c; ++e;
        }
}

int main(void) {
    enum { N = 9 };
    const int64_t nv = N * N, ne = 2 * (N - 1) * (N - 1);
    const double h = 1000.0;
    double *x = malloc(sizeof(double) * nv), *y = malloc(sizeof(double) * nv);
    int32_t *tri = malloc(sizeof(int32_t) * 3 * ne);
    grid(N, h, x, y, tri);
    se_mesh_desc desc;
    memset(&desc, 0, sizeof desc);
    desc.nv = nv;
    desc.ne = ne;
    desc.x = x;
    desc.y = y;
    desc.tri = tri;
    se_mesh *mesh = NULL;
    CHECK(se_mesh_create(&desc, -1, &mesh));   /* host only: no device memory */

    int64_t gnv, gne, nnz;
    double mu;
    CHECK(se_mesh_info(mesh, &gnv, &gne, &nnz, &mu));
    printf("info %lld %lld %lld %.17g\n", (long long)gnv, (long long)gne, (long long)nnz, mu);

    int32_t *vperm = malloc(sizeof(int32_t) * nv), *eperm = malloc(sizeof(int32_t) * ne);
    CHECK(se_mesh_perm(mesh, vperm, eperm));
    printf("vperm");
    for (int64_t i = 0; i < nv; ++i) printf(" %d", vperm[i]);
    printf("\neperm");
    for (int64_t i = 0; i < ne; ++i) printf(" %d", eperm[i]);
    printf("\n");

    int32_t *rtri = malloc(sizeof(int32_t) * 3 * ne), *row = malloc(sizeof(int32_t) * (nv + 1)),
            *col = malloc(sizeof(int32_t) * 3 * ne);
    CHECK(se_mesh_csr(mesh, rtri, row, col));
    printf("row_ptr");
    for (int64_t i = 0; i <= nv; ++i) printf(" %d", row[i]);
    printf("\n");

    double *Av = malloc(sizeof(double) * nv), *Ae = malloc(sizeof(double) * ne),
           *gN = malloc(sizeof(double) * 6 * ne);
    CHECK(se_mesh_geometry(mesh, Av, Ae, gN));
    double sav = 0.0, sae = 0.0, gmax = 0.0;
    for (int64_t i = 0; i < nv; ++i) sav += Av[i];
    for (int64_t i = 0; i < ne; ++i) sae += Ae[i];
    for (int64_t i = 0; i < ne; ++i)   /* basis gradients of a triangle sum to zero */
        for (int c = 0; c < 2; ++c) {
            const double s = gN[6 * i + c] + gN[6 * i + 2 + c] + gN[6 * i + 4 + c];
            if (s < 0 ? -s > gmax : s > gmax) gmax = s < 0 ? -s : s;
        }
    printf("areas %.17g %.17g %.17g\n", sav, sae, gmax);

    se_plan_stats_t ps;
    CHECK(se_plan_stats(mesh, 0, 64, 2, 256, &ps));
    printf("plan %d %d %d %d %d %d\n", ps.ntiles, ps.max_tri, ps.max_vtx, ps.tri_per_thread,
           ps.ok_f32, ps.ok_f64);

    double co[4];
    CHECK(se_sesm_coefficients(0.14, 0.0, co));
    printf("sesm %.17g %.17g %.17g %.17g\n", co[0], co[1], co[2], co[3]);

    /* error paths: each returns its status and leaves a message */
    se_mesh *bad = NULL;
    se_status st = se_mesh_create(NULL, -1, &bad);
    printf("err_null %d %d\n", (int)st, (int)(strlen(se_last_error()) > 0));
    tri[0] = (int32_t)nv;   /* vertex index out of range */
    st = se_mesh_create(&desc, -1, &bad);
    printf("err_index %d %d\n", (int)st, (int)(strlen(se_last_error()) > 0));
    tri[0] = 0;
    const int32_t t1 = tri[1];   /* clockwise first triangle: non-positive area */
    tri[1] = tri[2];
    tri[2] = t1;
    st = se_mesh_create(&desc, -1, &bad);
    printf("err_orientation %d %d\n", (int)st, (int)(strlen(se_last_error()) > 0));
    st = se_plan_stats(mesh, 0, 32, 2, 256, &ps);   /* tile below 64 */
    printf("err_plan %d\n", (int)st);
    st = se_sesm_coefficients(0.14, 0.0, NULL);
    printf("err_sesm %d\n", (int)st);
    se_params prm;
    memset(&prm, 0, sizeof prm);
    prm.g = 9.81;
    prm.theta = 0.14;
    se_state state;
    memset(&state, 0, sizeof state);
    se_forcing forcing;
    memset(&forcing, 0, sizeof forcing);
    st = se_subcycle(mesh, &prm, &state, &forcing, 10, 100.0, NULL, NULL);
    printf("err_host_only %d %d\n", (int)st, (int)(strlen(se_last_error()) > 0));

    se_mesh_destroy(mesh);
    free(x); free(y); free(tri); free(vperm); free(eperm); free(rtri); free(row); free(col);
    free(Av); free(Ae); free(gN);
    printf("done\n");
    return 0;
}
