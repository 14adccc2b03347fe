/* Drives every entry point of the oracle on small inputs under the host
 * address and undefined-behaviour sanitizers (test infrastructure). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_element_stiffness(const double* C, double* ke);
void orc_stiffness_table(int nphase, const double* C, double* ke);
void orc_apply(int, int, int, const int32_t*, const double*, const double*, double*);
void orc_apply_at(int, int, int, const int32_t*, const double*, const double*, const int64_t*, long, double*);
void orc_load(int, int, int, const int32_t*, const double*, const double*, double*, double*);
void orc_load_at(int, int, int, const int32_t*, const double*, const double*, const int64_t*, long, double*);
void orc_precond(int, int, int, const int32_t*, const double*, int, const double*, int, double*);
void orc_precond_at(int, int, int, const int32_t*, const double*, int, const double*, const int64_t*, long,
                    double*);
int orc_pcg(int, int, int, const int32_t*, const double*, const double*, const double*, double, double, int, int,
            double*, double*, double*);
void orc_stress(int, int, int, const int32_t*, int, const double*, const double*, const double*, double*,
                double*);
double orc_energy(int, int, int, const int32_t*, const double*, const double*, const double*);
void orc_grains(int, int, int, int, const double*, const double*, int32_t*);
void orc_grains_at(int, int, int, int, const double*, const double*, const int64_t*, long, int32_t*);
int orc_carve(int, int, int, int32_t*, int32_t, int, const double*, double, int64_t*);
void orc_covered_at(int, int, int, int, const double*, const int64_t*, long, int32_t*);
void orc_von_mises(long, const double*, double*);

static double urand(unsigned* s)
{
    *s = *s * 1664525u + 1013904223u;
    return (*s >> 8) * (1.0 / 16777216.0);
}

int main(void)
{
    const int nx = 5, ny = 4, nz = 3, n = nx * ny * nz, nphase = 3;
    unsigned seed = 7;
    double C[3 * 36];
    memset(C, 0, sizeof C);
    for (int p = 0; p < 2; ++p) { /* SPD: A A^T + 6 I; phase 2 is a void */
        double A[36];
        for (int t = 0; t < 36; ++t) A[t] = urand(&seed) - 0.5;
        for (int r = 0; r < 6; ++r)
            for (int c = 0; c < 6; ++c) {
                double s = r == c ? 6.0 : 0.0;
                for (int k = 0; k < 6; ++k) s += A[6 * r + k] * A[6 * c + k];
                C[36 * p + 6 * r + c] = s;
            }
    }
    int32_t phase[60];
    for (int m = 0; m < n; ++m) phase[m] = (int32_t)(urand(&seed) * 2.999);
    double* ke = malloc(sizeof(double) * 576 * nphase);
    orc_stiffness_table(nphase, C, ke);
    double strain[6] = {1e-3, 0, 2e-4, 0, 1e-4, 0};
    double b[180], r2 = 0, x[180], y[180], w[180], minv[540], info[5], trace[400], sig[360], avg[6];
    orc_load(nx, ny, nz, phase, ke, strain, b, &r2);
    for (int t = 0; t < 3 * n; ++t) x[t] = urand(&seed) - 0.5;
    orc_apply(nx, ny, nz, phase, ke, x, y);
    int64_t sel[4] = {0, 7, 33, n - 1};
    double ya[12], ba[12], ma[36];
    orc_apply_at(nx, ny, nz, phase, ke, x, sel, 4, ya);
    orc_load_at(nx, ny, nz, phase, ke, strain, sel, 4, ba);
    orc_precond(nx, ny, nz, phase, ke, nphase, C, 0, minv);
    orc_precond_at(nx, ny, nz, phase, ke, nphase, C, sel, 4, ma);
    int st = orc_pcg(nx, ny, nz, phase, ke, minv, b, r2, 1e-10, 400, 0, w, info, trace);
    orc_stress(nx, ny, nz, phase, nphase, C, strain, w, sig, avg);
    double en = orc_energy(nx, ny, nz, phase, ke, strain, w);
    double vm[60];
    orc_von_mises(n, sig, vm);
    double seeds[3 * 6], semi[2 * 6];
    for (int g = 0; g < 6; ++g) {
        seeds[3 * g] = urand(&seed) * nx;
        seeds[3 * g + 1] = urand(&seed) * ny;
        seeds[3 * g + 2] = urand(&seed) * nz;
        semi[2 * g] = 0.5 + urand(&seed);
        semi[2 * g + 1] = 0.5 + urand(&seed);
    }
    int32_t gr[60], ga[4], cov[4];
    orc_grains(nx, ny, nz, 6, seeds, semi, gr);
    orc_grains_at(nx, ny, nz, 6, seeds, semi, sel, 4, ga);
    int same = 1;
    for (int t = 0; t < 4; ++t) same = same && ga[t] == gr[sel[t]];
    double pores[2 * 15] = {0.2, 3.9, 1.0, 1.5, 1.0, 0.8, 1, 0, 0, 0, 1, 0, 0, 0, 1,
                            2.5, 2.0, 1.5, 0.9, 0.9, 0.9, 0, -1, 0, 1, 0, 0, 0, 0, 1};
    int64_t nvoid = 0;
    int used = orc_carve(nx, ny, nz, gr, 6, 2, pores, 5.0, &nvoid);
    orc_covered_at(nx, ny, nz, 2, pores, sel, 4, cov);
    free(ke);
    int ok = st == 0 && isfinite(en) && isfinite(avg[0]) && used >= 1 && nvoid >= 5 && same;
    printf("status %d iters %g energy %.6g used %d nvoid %lld ok %d\n", st, info[0], en, used, (long long)nvoid, ok);
    return ok ? 0 : 1;
}
