/*
 * qg_example.c -- a C99 program that drives libqg through include/qg.h
 * alone: device buffers from hipMalloc, no Python, no torch.
 *
 * It builds the island channel of the 128 x 64 workload (2 pi x pi box,
 * beta = 1, Re = 1000, inflow 1, porosity 1e-3, sponge rate 10, static
 * Smagorinsky c = 0.17, RK4 with dt = 2e-3, 64-bit): a smoothed circular
 * island (tanh edge over two cells), a sponge ramp at both x ends
 * (thickness lx/16) and a deterministic initial vorticity made of a few
 * Fourier modes.  It then runs 20 steps in one qg_step call (graph replay),
 * takes the diagnostics, and writes the inputs and the result as raw
 * little-endian doubles, row-major (ny, nx):
 *
 *     qg_example OUT_DIR   ->  OUT_DIR/{chi,chi_s,omega0,omega20}.f64
 *
 * and prints the diagnostics on stdout.  Exit status 0 on success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "qg.h"

#define NX 128
#define NY 64
#define NSTEPS 20

#define CHECK_QG(call)                                                      \
    do {                                                                    \
        int rc_ = (call);                                                   \
        if (rc_ != QG_OK) {                                                 \
            fprintf(stderr, "%s failed (%d): %s\n", #call, rc_, qg_last_error()); \
            return 1;                                                       \
        }                                                                   \
    } while (0)

#define CHECK_HIP(call)                                                     \
    do {                                                                    \
        hipError_t e_ = (call);                                             \
        if (e_ != hipSuccess) {                                             \
            fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_)); \
            return 1;                                                       \
        }                                                                   \
    } while (0)

static const double PI = 3.14159265358979323846;

static void make_inputs(double lx, double ly, double* chi, double* chs, double* w0) {
    const double dx = lx / NX, eps = 2.0 * dx, xc = 1.5, yc = 0.5 * ly, radius = 0.3;
    const double ds = lx / 16.0;
    for (int j = 0; j < NY; ++j) {
        for (int i = 0; i < NX; ++i) {
            const double x = i * dx, y = j * (ly / NY);
            const double r = hypot(x - xc, y - yc);
            const double d = fmin(x, lx - x);
            chi[j * NX + i] = 0.5 * (1.0 - tanh((r - radius) / eps));
            chs[j * NX + i] = fmax(0.0, 1.0 - d / ds);
            /* a few modes (kx = 2 pi mx / lx, ky = 2 pi my / ly) */
            w0[j * NX + i] = 0.08 * cos(2.0 * x + 2.0 * y + 0.3) + 0.05 * sin(3.0 * x - 4.0 * y)
                           + 0.04 * cos(5.0 * x + 6.0 * y + 1.1) + 0.03 * sin(7.0 * x + 2.0 * y - 0.4);
        }
    }
}

static int write_field(const char* dir, const char* name, const double* f) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s.f64", dir, name);
    FILE* fp = fopen(path, "wb");
    if (!fp) return 1;
    const size_t n = fwrite(f, sizeof(double), (size_t)NX * NY, fp);
    fclose(fp);
    return n == (size_t)NX * NY ? 0 : 1;
}

int main(int argc, char** argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s OUT_DIR\n", argv[0]);
        return 2;
    }
    qg_params p;
    memset(&p, 0, sizeof p);
    p.nx = NX;
    p.ny = NY;
    p.lx = 2.0 * PI;
    p.ly = PI;
    p.beta = 1.0;
    p.re = 1000.0;
    p.mu = 0.0;
    p.u_in = 1.0;
    p.v_in = 0.0;
    p.eta = 1e-3;
    p.sponge_sigma = 10.0;
    p.dt = 2e-3;
    p.c = 0.17;
    p.closure = QG_CLOSURE_SMAG;
    p.precision = 64;
    p.test_ratio = 2.0;
    p.clip_mode = 0;
    p.fp64_lowk = 8;
    p.scheme = QG_SCHEME_RK4;

    const size_t nbytes = (size_t)NX * NY * sizeof(double);
    double* chi = (double*)malloc(nbytes);
    double* chs = (double*)malloc(nbytes);
    double* w = (double*)malloc(nbytes);
    if (!chi || !chs || !w) return 1;
    make_inputs(p.lx, p.ly, chi, chs, w);
    if (write_field(argv[1], "chi", chi) || write_field(argv[1], "chi_s", chs) ||
        write_field(argv[1], "omega0", w)) {
        fprintf(stderr, "cannot write to %s\n", argv[1]);
        return 1;
    }

    size_t ws_bytes = 0;
    CHECK_QG(qg_workspace_bytes(&p, 1, 0, &ws_bytes));
    void *ws = NULL, *d_chi = NULL, *d_chs = NULL, *d_w = NULL;
    double* d_diag = NULL;
    CHECK_HIP(hipMalloc(&ws, ws_bytes));          /* hipMalloc returns >= 256-byte alignment */
    CHECK_HIP(hipMalloc(&d_chi, nbytes));
    CHECK_HIP(hipMalloc(&d_chs, nbytes));
    CHECK_HIP(hipMalloc(&d_w, nbytes));
    CHECK_HIP(hipMalloc((void**)&d_diag, 8 * sizeof(double)));
    CHECK_HIP(hipMemcpy(d_chi, chi, nbytes, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_chs, chs, nbytes, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_w, w, nbytes, hipMemcpyHostToDevice));

    const void* masks[1] = {d_chi};
    const void* sponges[1] = {d_chs};
    qg_handle* h = NULL;
    CHECK_QG(qg_init(&p, 1, masks, sponges, ws, ws_bytes, 0, NULL, &h));
    CHECK_QG(qg_step(h, d_w, NSTEPS, 0, NULL, 1, NULL));
    CHECK_QG(qg_diag(h, d_w, d_diag, NULL, NULL));
    CHECK_HIP(hipDeviceSynchronize());

    double diag[8];
    CHECK_HIP(hipMemcpy(w, d_w, nbytes, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(diag, d_diag, sizeof diag, hipMemcpyDeviceToHost));
    if (write_field(argv[1], "omega20", w)) return 1;
    printf("workspace %zu bytes\n", ws_bytes);
    printf("energy %.17g enstrophy %.17g C %.17g nu_mean %.17g cfl %.17g nonfinite %g\n", diag[0], diag[1],
           diag[2], diag[4], diag[6], diag[7]);

    qg_destroy(h);
    CHECK_HIP(hipFree(d_diag));
    CHECK_HIP(hipFree(d_w));
    CHECK_HIP(hipFree(d_chs));
    CHECK_HIP(hipFree(d_chi));
    CHECK_HIP(hipFree(ws));
    free(w);
    free(chs);
    free(chi);
    return diag[7] != 0.0;
}
