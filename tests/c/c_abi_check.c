/* The C ABI used from plain C, with no Python or torch: load a mechanism,
 * create a plan, integrate cells held in hipMalloc'd buffers, write the
 * results.  The GPU test runs this program and compares its output with the
 * Python binding's, bit for bit.
 *
 * usage: c_abi_check MECH_TEXT INPUT OUTPUT
 *   INPUT : int64 n, then n T0, n p, N*n Y0 (species-major), n dt (doubles)
 *   OUTPUT: n T1, N*n Y1 (doubles), then n status, n n_acc (int32) */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "stiffchem.h"

static void *read_all(const char *path, size_t *len)
{
    FILE *f = fopen(path, "rb");
    if (!f) return NULL;
    fseek(f, 0, SEEK_END);
    long sz = ftell(f);
    fseek(f, 0, SEEK_SET);
    char *buf = (char *)malloc((size_t)sz + 1);
    if (buf && fread(buf, 1, (size_t)sz, f) != (size_t)sz) {
        free(buf);
        buf = NULL;
    }
    fclose(f);
    if (buf) buf[sz] = 0;
    *len = (size_t)sz;
    return buf;
}

#define CHECK_SC(x)                                                             \
    do {                                                                        \
        sc_status s_ = (x);                                                     \
        if (s_ != SC_OK) {                                                      \
            fprintf(stderr, "%s failed: %d %s\n", #x, (int)s_, sc_last_error()); \
            return 2;                                                           \
        }                                                                       \
    } while (0)
#define CHECK_HIP(x)                                              \
    do {                                                          \
        if ((x) != hipSuccess) {                                  \
            fprintf(stderr, "%s failed\n", #x);                   \
            return 3;                                             \
        }                                                         \
    } while (0)

int main(int argc, char **argv)
{
    if (argc != 4) {
        fprintf(stderr, "usage: %s MECH_TEXT INPUT OUTPUT\n", argv[0]);
        return 1;
    }
    size_t tlen = 0, ilen = 0;
    char *text = (char *)read_all(argv[1], &tlen);
    char *in = (char *)read_all(argv[2], &ilen);
    if (!text || !in || ilen < sizeof(int64_t)) return 1;
    sc_mech *mech = NULL;
    CHECK_SC(sc_mech_load(text, tlen, &mech));
    sc_mech_info info;
    CHECK_SC(sc_mech_info_get(mech, &info));
    const int64_t N = info.n_species;
    const int64_t n = *(const int64_t *)in;
    if ((int64_t)ilen != (int64_t)sizeof(int64_t) + (int64_t)sizeof(double) * n * (N + 3)) {
        fprintf(stderr, "input size does not match n = %lld, N = %lld\n", (long long)n, (long long)N);
        return 1;
    }
    const double *T0 = (const double *)(in + sizeof(int64_t));
    const double *p = T0 + n, *Y0 = p + n, *dt = Y0 + N * n;
    sc_options opt;
    sc_default_options(&opt);
    sc_plan *plan = NULL;
    CHECK_SC(sc_plan_create(mech, 0, &opt, &plan));
    double *dT0, *dp, *dY0, *ddt, *dT1, *dY1;
    int32_t *dst, *dna;
    const size_t vb = sizeof(double) * (size_t)n, yb = sizeof(double) * (size_t)(N * n);
    CHECK_HIP(hipMalloc((void **)&dT0, vb));
    CHECK_HIP(hipMalloc((void **)&dp, vb));
    CHECK_HIP(hipMalloc((void **)&dY0, yb));
    CHECK_HIP(hipMalloc((void **)&ddt, vb));
    CHECK_HIP(hipMalloc((void **)&dT1, vb));
    CHECK_HIP(hipMalloc((void **)&dY1, yb));
    CHECK_HIP(hipMalloc((void **)&dst, sizeof(int32_t) * (size_t)n));
    CHECK_HIP(hipMalloc((void **)&dna, sizeof(int32_t) * (size_t)n));
    CHECK_HIP(hipMemcpy(dT0, T0, vb, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(dp, p, vb, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(dY0, Y0, yb, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(ddt, dt, vb, hipMemcpyHostToDevice));
    CHECK_SC(sc_integrate(plan, n, dT0, dp, dY0, n, ddt, NULL, NULL, dT1, dY1, dst, dna, NULL, NULL));
    CHECK_HIP(hipDeviceSynchronize());
    double *out = (double *)malloc(vb + yb);
    int32_t *iout = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)n);
    if (!out || !iout) return 1;
    CHECK_HIP(hipMemcpy(out, dT1, vb, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(out + n, dY1, yb, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(iout, dst, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(iout + n, dna, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost));
    FILE *f = fopen(argv[3], "wb");
    if (!f) return 1;
    fwrite(out, 1, vb + yb, f);
    fwrite(iout, sizeof(int32_t), 2 * (size_t)n, f);
    fclose(f);
    hipFree(dT0); hipFree(dp); hipFree(dY0); hipFree(ddt);
    hipFree(dT1); hipFree(dY1); hipFree(dst); hipFree(dna);
    sc_plan_free(plan);
    sc_mech_free(mech);
    free(out); free(iout); free(text); free(in);
    printf("c_abi_check: %lld cells integrated\n", (long long)n);
    return 0;
}
