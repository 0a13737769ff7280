/* A plain C caller of the library on the GPU: device memory from hipMalloc, one FP64
 * se_subcycle on the default stream, results copied back.  No torch, no Python.
 *
 *   abi_gpu <input> <output>
 *
 * input (native byte order): int64 nv, ne; int32 nsub, mesh flags (SE_PERIODIC_X ...),
 * parameter flags (SE_LINEAR_H), pad; double tau, g, theta, period_x, period_y, radius;
 * then x[nv], y[nv] (double), tri[3 ne] (int32), eta0[nv], U0[2 ne], R[2 ne], f[ne],
 * H0[nv] (double), all in the caller's numbering.
 * output: eta[nv], U[2 ne], <<U>>[2 ne] (caller's numbering), volume[nsub + 1] (double).
 * tests/test_gpu_c_abi.py writes the input and compares the output with the oracle. */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sesub.h"

#define CHECK(call)                                                                      \
    do {                                                                                 \
        se_status st_ = (call);                                                          \
        if (st_ != SE_OK) {                                                              \
            fprintf(stderr, "%s: status %d (%s)\n", #call, (int)st_, se_last_error());   \
            return 1;                                                                    \
        }                                                                                \
    } while (0)
#define HCHECK(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));                   \
            return 1;                                                                    \
        }                                                                                \
    } while (0)

static void *read_n(FILE *f, size_t bytes) {
    void *p = malloc(bytes ? bytes : 1);
    if (p && bytes && fread(p, 1, bytes, f) != bytes) {
        free(p);
        return NULL;
    }
    return p;
}

int main(int argc, char **argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: abi_gpu <input> <output>\n");
        return 2;
    }
    FILE *in = fopen(argv[1], "rb");
    if (!in) return 2;
    int64_t n2[2];
    int32_t i4[4];
    double d6[6];
    if (fread(n2, 8, 2, in) != 2 || fread(i4, 4, 4, in) != 4 || fread(d6, 8, 6, in) != 6)
        return 2;
    const int64_t nv = n2[0], ne = n2[1];
    const int32_t nsub = i4[0];
    const double tau = d6[0], g = d6[1], theta = d6[2];
    if (nv <= 0 || ne <= 0 || nsub < 1) return 2;
    double *x = read_n(in, 8 * nv), *y = read_n(in, 8 * nv);
    int32_t *tri = read_n(in, 12 * ne);
    double *eta0 = read_n(in, 8 * nv), *U0 = read_n(in, 16 * ne), *R = read_n(in, 16 * ne),
           *f = read_n(in, 8 * ne), *H0 = read_n(in, 8 * nv);
    fclose(in);
    if (!x || !y || !tri || !eta0 || !U0 || !R || !f || !H0) return 2;

    se_mesh_desc desc;
    memset(&desc, 0, sizeof desc);
    desc.nv = nv;
    desc.ne = ne;
    desc.x = x;
    desc.y = y;
    desc.tri = tri;
    desc.flags = (uint32_t)i4[1];
    desc.period_x = d6[3];
    desc.period_y = d6[4];
    desc.radius = d6[5];
    se_mesh *mesh = NULL;
    CHECK(se_mesh_create(&desc, 0, &mesh));
    /* the library's numbering: vperm[new] = caller's vertex, eperm[new] = caller's triangle */
    int32_t *vperm = malloc(4 * nv), *eperm = malloc(4 * ne);
    CHECK(se_mesh_perm(mesh, vperm, eperm));
    double *he = malloc(8 * nv), *hU = malloc(16 * ne), *hR = malloc(16 * ne), *hf = malloc(8 * ne),
           *hH = malloc(8 * nv), *hUa = malloc(16 * ne), *hvol = malloc(8 * (nsub + 1));
    for (int64_t i = 0; i < nv; ++i) {
        he[i] = eta0[vperm[i]];
        hH[i] = H0[vperm[i]];
    }
    for (int64_t e = 0; e < ne; ++e) {
        const int64_t o = eperm[e];
        hU[2 * e] = U0[2 * o];
        hU[2 * e + 1] = U0[2 * o + 1];
        hR[2 * e] = R[2 * o];
        hR[2 * e + 1] = R[2 * o + 1];
        hf[e] = f[o];
    }

    se_params prm;
    memset(&prm, 0, sizeof prm);
    prm.g = g;
    prm.theta = theta;
    prm.precision = SE_F64;
    prm.flags = SE_TRACK_VOLUME | (uint32_t)i4[2];
    size_t wbytes = 0;
    CHECK(se_workspace_bytes(mesh, &prm, nsub, 0, &wbytes));
    void *d_eta, *d_U, *d_R, *d_f, *d_H, *d_Ua, *d_vol, *d_ws;
    HCHECK(hipMalloc(&d_eta, 8 * nv));
    HCHECK(hipMalloc(&d_U, 16 * ne));
    HCHECK(hipMalloc(&d_R, 16 * ne));
    HCHECK(hipMalloc(&d_f, 8 * ne));
    HCHECK(hipMalloc(&d_H, 8 * nv));
    HCHECK(hipMalloc(&d_Ua, 16 * ne));
    HCHECK(hipMalloc(&d_vol, 8 * (nsub + 1)));
    HCHECK(hipMalloc(&d_ws, wbytes));   /* hipMalloc returns 256-byte aligned memory */
    HCHECK(hipMemcpy(d_eta, he, 8 * nv, hipMemcpyHostToDevice));
    HCHECK(hipMemcpy(d_U, hU, 16 * ne, hipMemcpyHostToDevice));
    HCHECK(hipMemcpy(d_R, hR, 16 * ne, hipMemcpyHostToDevice));
    HCHECK(hipMemcpy(d_f, hf, 8 * ne, hipMemcpyHostToDevice));
    HCHECK(hipMemcpy(d_H, hH, 8 * nv, hipMemcpyHostToDevice));

    se_state st = {d_eta, d_U, (double *)d_Ua, (double *)d_vol};
    se_forcing fo = {d_R, d_f, d_H, NULL};
    CHECK(se_subcycle(mesh, &prm, &st, &fo, nsub, tau, d_ws, NULL));
    uint32_t faults = 0;
    CHECK(se_check_faults(mesh, 0, NULL, &faults));
    if (faults) {
        fprintf(stderr, "fault bits %u\n", faults);
        return 1;
    }
    HCHECK(hipMemcpy(he, d_eta, 8 * nv, hipMemcpyDeviceToHost));
    HCHECK(hipMemcpy(hU, d_U, 16 * ne, hipMemcpyDeviceToHost));
    HCHECK(hipMemcpy(hUa, d_Ua, 16 * ne, hipMemcpyDeviceToHost));
    HCHECK(hipMemcpy(hvol, d_vol, 8 * (nsub + 1), hipMemcpyDeviceToHost));

    /* back to the caller's numbering */
    double *oe = malloc(8 * nv), *oU = malloc(16 * ne), *oUa = malloc(16 * ne);
    for (int64_t i = 0; i < nv; ++i) oe[vperm[i]] = he[i];
    for (int64_t e = 0; e < ne; ++e) {
        const int64_t o = eperm[e];
        oU[2 * o] = hU[2 * e];
        oU[2 * o + 1] = hU[2 * e + 1];
        oUa[2 * o] = hUa[2 * e];
        oUa[2 * o + 1] = hUa[2 * e + 1];
    }
    FILE *out = fopen(argv[2], "wb");
    if (!out) return 2;
    fwrite(oe, 8, nv, out);
    fwrite(oU, 16, ne, out);
    fwrite(oUa, 16, ne, out);
    fwrite(hvol, 8, nsub + 1, out);
    fclose(out);

    hipFree(d_eta); hipFree(d_U); hipFree(d_R); hipFree(d_f); hipFree(d_H); hipFree(d_Ua);
    hipFree(d_vol); hipFree(d_ws);
    se_mesh_destroy(mesh);
    free(x); free(y); free(tri); free(eta0); free(U0); free(R); free(f); free(H0);
    free(vperm); free(eperm); free(he); free(hU); free(hR); free(hf); free(hH); free(hUa);
    free(hvol); free(oe); free(oU); free(oUa);
    printf("ok\n");
    return 0;
}
