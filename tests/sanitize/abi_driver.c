/* Calls the C-ABI with invalid arguments under the host address and
 * undefined-behaviour sanitizers: every call must be refused with the
 * documented code by the validation that runs before any device call, so
 * this driver needs no GPU (test infrastructure). */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "elas3d.h"

static int fails = 0;

static void expect(const char* what, int got, int want)
{
    if (got != want) {
        printf("FAIL %s: got %d, want %d (%s)\n", what, got, want, elas3d_last_error(NULL));
        ++fails;
    }
}

int main(void)
{
    elas3d_options o;
    elas3d_options_init(&o);
    double C[2 * 36];
    memset(C, 0, sizeof C);
    for (int d = 0; d < 6; ++d) C[7 * d] = d < 3 ? 300.0 : 80.0;
    int phase[64];
    for (int m = 0; m < 64; ++m) phase[m] = m % 2;
    double strain[6] = {1e-3, 0, 0, 0, 0, 0};
    elas3d_ctx* ctx = (elas3d_ctx*)0x1;
    expect("null out", elas3d_setup(NULL, 4, 4, 4, phase, 2, C, 1, strain, &o), ELAS3D_EBADARG);
    expect("dims", elas3d_setup(&ctx, 1, 4, 4, phase, 2, C, 1, strain, &o), ELAS3D_EBADARG);
    if (ctx != NULL) { printf("FAIL ctx not cleared\n"); ++fails; }
    expect("null phase", elas3d_setup(&ctx, 4, 4, 4, NULL, 2, C, 1, strain, &o), ELAS3D_EBADARG);
    expect("nphase", elas3d_setup(&ctx, 4, 4, 4, phase, 0, C, 1, strain, &o), ELAS3D_EBADARG);
    expect("nrhs", elas3d_setup(&ctx, 4, 4, 4, phase, 2, C, 7, strain, &o), ELAS3D_EBADARG);
    phase[5] = 2;
    expect("phase range", elas3d_setup(&ctx, 4, 4, 4, phase, 2, C, 1, strain, &o), ELAS3D_EBADARG);
    phase[5] = 1;
    C[1] = 5.0;
    expect("asymmetric C", elas3d_setup(&ctx, 4, 4, 4, phase, 2, C, 1, strain, &o), ELAS3D_EBADARG);
    C[1] = 0.0;
    C[40] = NAN;
    expect("NaN C", elas3d_setup(&ctx, 4, 4, 4, phase, 2, C, 1, strain, &o), ELAS3D_EBADARG);
    C[40] = 0.0;
    strain[2] = INFINITY;
    expect("Inf strain", elas3d_setup(&ctx, 4, 4, 4, phase, 2, C, 1, strain, &o), ELAS3D_EBADARG);
    strain[2] = 0.0;
    elas3d_options bad = o;
    bad.precision = 7;
    expect("options", elas3d_setup(&ctx, 4, 4, 4, phase, 2, C, 1, strain, &bad), ELAS3D_EBADARG);
    bad = o;
    bad.tile = 99;
    expect("tile", elas3d_setup(&ctx, 4, 4, 4, phase, 2, C, 1, strain, &bad), ELAS3D_EBADARG);
    expect("solve NULL", elas3d_solve(NULL, 1e-8, 10, 1, NULL), ELAS3D_EBADARG);
    expect("stress NULL", elas3d_stress(NULL, 0, NULL, NULL, NULL, NULL), ELAS3D_EBADARG);
    expect("apply NULL", elas3d_apply(NULL, NULL, NULL), ELAS3D_EBADARG);
    expect("grains dims", elas3d_generate_grains(0, 4, 4, 1, strain, NULL, phase, NULL), ELAS3D_EBADARG);
    double seed_out[3] = {5.0, 0.5, 0.5};
    expect("grains seed", elas3d_generate_grains(4, 4, 4, 1, seed_out, NULL, phase, NULL), ELAS3D_EBADARG);
    expect("grains static output", elas3d_generate_grains_static(4, 4, 4, 1, strain, NULL, phase, &o),
           ELAS3D_EBADARG);
    expect("pores", elas3d_carve_pores(4, 4, 4, NULL, 1, 1, C, -1.0, NULL, NULL, NULL), ELAS3D_EBADARG);
    double gbs[3];
    expect("stream", elas3d_stream_bandwidth(1000, 64, 1, 0, gbs, NULL), ELAS3D_EBADARG);
    expect("group", elas3d_group_create(NULL, NULL), ELAS3D_EBADARG);
    if (elas3d_device_bytes(1, 4, 4, 2, 1, NULL) != 0.0) { printf("FAIL device_bytes\n"); ++fails; }
    if (!elas3d_version() || !elas3d_last_error(NULL)) { printf("FAIL strings\n"); ++fails; }
    elas3d_destroy(NULL);
    printf("%s (%d failures)\n", fails ? "FAILED" : "ok", fails);
    return fails ? 1 : 0;
}
