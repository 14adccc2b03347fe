/*
 * Reference (oracle) implementation of the microstructure generator and the
 * von Mises output.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, serial statements of what the
 * generator kernels compute; only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file.  It shares no code
 * with the product library.
 *
 * Method: ELAS3D-Xtal (arXiv 2602.07354).
 *   - grain assignment by the smallest ellipsoidal distance   Sec. 2.2.2, Eq. (ellipsoid_dist)
 *   - pore overwrite of the grain map                        Sec. 2.2.3, pore-integration algorithm
 *   - von Mises equivalent stress per voxel                  Sec. 2.1.3, Table 1 (stress_fullfield)
 *
 * Readings (listed in the design notes):
 *   - The assignment is the plain definition: the minimum over ALL grains.
 *     The paper's spatial filter (candidate cells grown by 1.5 max radius)
 *     only restricts where it looks; the definition it approximates is
 *     written out here.
 *   - Voxel (i,j,k) is represented by its centre (i+1/2, j+1/2, k+1/2); the
 *     grid is periodic and offsets are minimum images: d = x - s, or
 *     (x -+ L) - s when |x - s| > L/2 (seeds and centres in [0, L)).
 *   - D^2 = (dx*dx + dy*dy) / (rt*rt) + (dz*dz) / (rl*rl), evaluated in that
 *     order in FP64; the lowest grain index wins an exact tie.
 *   - A pore covers a voxel centre when sum_j (e_j / a_j)^2 <= 1 + 1e-12,
 *     e_j = (d0 R[0][j] + d1 R[1][j]) + d2 R[2][j] the offset in the pore's
 *     own axes (R's columns are those axes in the sample frame, a the
 *     semi-axes); the slack keeps centres that sit on the surface inside.
 *   - Pores are carved in order; with a target count of void voxels the
 *     overwrite stops after the first pore with which the count reaches it
 *     (none is carved when it already does).
 *
 * Compiled without floating-point contraction, so that every product and
 * sum above is rounded on its own.
 */
#include <math.h>
#include <stdint.h>

/* Minimum-image offset of a voxel centre x from a point s in a box of
 * length L: x - s, or (x -+ L) - s when |x - s| > L/2 (x -+ L is exact, so
 * the offset is always rounded once). */
static double min_image(double x, double s, double L)
{
    const double d = x - s;
    if (d > 0.5 * L) return (x - L) - s;
    if (d < -0.5 * L) return (x + L) - s;
    return d;
}

/* seeds: 3 per grain (x, y, z in [0, n)), semi: 2 per grain (rt, rl). */
void orc_grains(int nx, int ny, int nz, int ngrain, const double* seeds, const double* semi,
                int32_t* phase)
{
    const double Lx = nx, Ly = ny, Lz = nz;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const double x = i + 0.5, y = j + 0.5, z = k + 0.5;
                double best = INFINITY;
                int32_t arg = 0;
                for (int g = 0; g < ngrain; ++g) {
                    const double dx = min_image(x, seeds[3 * g], Lx);
                    const double dy = min_image(y, seeds[3 * g + 1], Ly);
                    const double dz = min_image(z, seeds[3 * g + 2], Lz);
                    const double rt = semi[2 * g], rl = semi[2 * g + 1];
                    const double d2 = (dx * dx + dy * dy) / (rt * rt) + (dz * dz) / (rl * rl);
                    if (d2 < best) {
                        best = d2;
                        arg = g;
                    }
                }
                phase[i + (long)nx * (j + (long)ny * k)] = arg;
            }
}

/* 1 if pore p (15 doubles: centre 3, semi-axes 3, R row-major 9) covers the
 * centre of voxel (i, j, k). */
static int covers(const double* p, int nx, int ny, int nz, int i, int j, int k)
{
    const double d0 = min_image(i + 0.5, p[0], nx);
    const double d1 = min_image(j + 0.5, p[1], ny);
    const double d2 = min_image(k + 0.5, p[2], nz);
    const double* a = p + 3;
    const double* R = p + 6;
    double s = 0.0;
    for (int c = 0; c < 3; ++c) {
        const double e = (d0 * R[c] + d1 * R[3 + c]) + d2 * R[6 + c];
        const double q = e / a[c];
        s = c == 0 ? q * q : s + q * q;
    }
    return s <= 1.0 + 1e-12;
}

int orc_carve(int nx, int ny, int nz, int32_t* phase, int32_t void_id, int npore,
              const double* pores, double target, int64_t* nvoid)
{
    const long n = (long)nx * ny * nz;
    int64_t count = 0;
    for (long m = 0; m < n; ++m) count += phase[m] == void_id;
    int used = 0;
    for (int p = 0; p < npore; ++p) {
        if (target >= 0.0 && !((double)count < target)) break;
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    const long m = i + (long)nx * (j + (long)ny * k);
                    if (phase[m] != void_id && covers(pores + 15 * (long)p, nx, ny, nz, i, j, k)) {
                        phase[m] = void_id;
                        ++count;
                    }
                }
        used = p + 1;
    }
    *nvoid = count;
    return used;
}

/* sigma: 6 planes of n (Voigt 11, 22, 33, 23, 13, 12). */
void orc_von_mises(long n, const double* sigma, double* vm)
{
    for (long m = 0; m < n; ++m) {
        const double s11 = sigma[m], s22 = sigma[n + m], s33 = sigma[2 * n + m];
        const double s23 = sigma[3 * n + m], s13 = sigma[4 * n + m], s12 = sigma[5 * n + m];
        const double a = s11 - s22, b = s22 - s33, c = s33 - s11;
        vm[m] = sqrt(0.5 * (a * a + b * b + c * c) + 3.0 * (s23 * s23 + s13 * s13 + s12 * s12));
    }
}

/* orc_grains at `count` voxels idx[] only (same definition). */
void orc_grains_at(int nx, int ny, int nz, int ngrain, const double* seeds, const double* semi,
                   const int64_t* idx, long count, int32_t* out)
{
    const double Lx = nx, Ly = ny, Lz = nz;
    for (long t = 0; t < count; ++t) {
        const long m = idx[t];
        const int i = (int)(m % nx), j = (int)((m / nx) % ny), k = (int)(m / ((long)nx * ny));
        const double x = i + 0.5, y = j + 0.5, z = k + 0.5;
        double best = INFINITY;
        int32_t arg = 0;
        for (int g = 0; g < ngrain; ++g) {
            const double dx = min_image(x, seeds[3 * g], Lx);
            const double dy = min_image(y, seeds[3 * g + 1], Ly);
            const double dz = min_image(z, seeds[3 * g + 2], Lz);
            const double rt = semi[2 * g], rl = semi[2 * g + 1];
            const double d2 = (dx * dx + dy * dy) / (rt * rt) + (dz * dz) / (rl * rl);
            if (d2 < best) {
                best = d2;
                arg = g;
            }
        }
        out[t] = arg;
    }
}

/* out[t] = 1 if any of the npore pores covers voxel idx[t]. */
void orc_covered_at(int nx, int ny, int nz, int npore, const double* pores, const int64_t* idx, long count,
                    int32_t* out)
{
    for (long t = 0; t < count; ++t) {
        const long m = idx[t];
        const int i = (int)(m % nx), j = (int)((m / nx) % ny), k = (int)(m / ((long)nx * ny));
        int hit = 0;
        for (int p = 0; p < npore && !hit; ++p) hit = covers(pores + 15 * (long)p, nx, ny, nz, i, j, k);
        out[t] = hit;
    }
}
