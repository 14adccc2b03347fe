/*
 * Reference (oracle) implementation of the periodic voxel elasticity solve.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, serial FP64
 * statement of what the solver computes.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product
 * library never does, and the two share no code.
 *
 * Method: ELAS3D-Xtal (arXiv 2602.07354), Sec. 2.1.
 *   - periodic node indexing                     Sec. 2.1.1, Eq. (pbc_indices)
 *   - per-phase 6x6 stiffness, zero = void       Sec. 2.1.1, Eq. (2)-(3)
 *   - trilinear hex element stiffness K_e        Sec. 2.1.2, Eq. (discrete_energy)
 *   - affine load from the macroscopic strain    Sec. 2.1.2, Eq. (affine_strain)
 *   - gradient g = A w + b                       Sec. 2.1.2, Eq. (quadratic_form)
 *   - point-block Jacobi M^-1                    Sec. 2.1.2, Eq. (block_precond)
 *   - PCG with Fletcher-Reeves directions        Sec. 2.1.2, Algorithm 2
 *   - voxel / global stress                      Sec. 2.1.3, Table 1 (stress_OpenMP)
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - K_e: unit cube, trilinear shape functions, exact 2x2x2 Gauss rule,
 *     Voigt order (11,22,33,23,13,12) with engineering shear.  Local node
 *     a = ax + 2 ay + 4 az sits at (ax, ay, az).
 *   - Node m = (i,j,k) sits at the lower corner of voxel m; voxel (i,j,k) has
 *     nodes ((i+ax)%nx, (j+ay)%ny, (k+az)%nz), m = i + nx (j + ny k).
 *   - Fluctuation form: total displacement u = E.X + w, w starts at 0, and
 *     b = sum_e scatter(K_e u^E_e) with u^E_{e,a} = E . (ax, ay, az).
 *   - Nodes touched only by void voxels get M^-1 = 0 (and stay 0).
 *   - Breakdown when h.Ah <= 0 or not finite.
 *   - Convergence: metric mode stops on ||g||/||b|| <= tol and then checks
 *     the true residual ||A w + b||/||b||, restarting from w if it fails;
 *     paper mode stops on sqrt(gg/gg0) < tol.
 *   - Zero load: ||b|| <= 1e-14 ||b||_ref (uncancelled element forces)
 *     returns converged after 0 iterations.
 *
 * Vector fields are SoA: component c of node m at [c*N + m].
 *
 * The same file also builds with OpenMP (-fopenmp) into a separate library
 * used only to time a threaded CPU baseline (the paper's OpenMP column of
 * Table 4): the node loops then run in parallel and the element scatter of
 * the operator runs layer by layer in two (three for odd nz) colours, so
 * sums are formed in another order.  The serial build, which every pin and
 * parity test uses, ignores the pragmas and keeps the plain loop order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NDOF 24

/* ------------------------------------------------------------------ element */

/* Strain-displacement matrix B (6 x 24) of the unit trilinear hex at (x,y,z). */
static void orc_bmatrix(double x, double y, double z, double B[6][NDOF])
{
    memset(B, 0, sizeof(double) * 6 * NDOF);
    for (int a = 0; a < 8; ++a) {
        int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
        double fx = ax ? x : 1.0 - x, fy = ay ? y : 1.0 - y, fz = az ? z : 1.0 - z;
        double sx = ax ? 1.0 : -1.0, sy = ay ? 1.0 : -1.0, sz = az ? 1.0 : -1.0;
        double dNx = sx * fy * fz, dNy = fx * sy * fz, dNz = fx * fy * sz;
        int c = 3 * a;
        B[0][c] = dNx;                       /* e11 = du1/dx1 */
        B[1][c + 1] = dNy;                   /* e22 */
        B[2][c + 2] = dNz;                   /* e33 */
        B[3][c + 1] = dNz; B[3][c + 2] = dNy; /* 2 e23 */
        B[4][c] = dNz;     B[4][c + 2] = dNx; /* 2 e13 */
        B[5][c] = dNy;     B[5][c + 1] = dNx; /* 2 e12 */
    }
}

/* K_e = int_cube B^T C B dV, 2x2x2 Gauss (exact for this integrand). */
void orc_element_stiffness(const double* C, double* ke)
{
    const double g[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
    double B[6][NDOF], CB[6][NDOF];
    memset(ke, 0, sizeof(double) * NDOF * NDOF);
    for (int q = 0; q < 8; ++q) {
        orc_bmatrix(g[q & 1], g[(q >> 1) & 1], g[(q >> 2) & 1], B);
        for (int r = 0; r < 6; ++r)
            for (int col = 0; col < NDOF; ++col) {
                double s = 0.0;
                for (int t = 0; t < 6; ++t) s += C[r * 6 + t] * B[t][col];
                CB[r][col] = s;
            }
        for (int p = 0; p < NDOF; ++p)
            for (int col = 0; col < NDOF; ++col) {
                double s = 0.0;
                for (int r = 0; r < 6; ++r) s += B[r][p] * CB[r][col];
                ke[p * NDOF + col] += 0.125 * s; /* Gauss weight (1/2)^3 */
            }
    }
}

static int orc_phase_is_void(const double* C)
{
    for (int t = 0; t < 36; ++t)
        if (C[t] != 0.0) return 0;
    return 1;
}

/* K_e for every phase (nphase x 576); void phases get zeros. */
void orc_stiffness_table(int nphase, const double* C, double* ke)
{
    for (int p = 0; p < nphase; ++p) {
        if (orc_phase_is_void(C + 36 * p))
            memset(ke + (size_t)p * 576, 0, sizeof(double) * 576);
        else
            orc_element_stiffness(C + 36 * p, ke + (size_t)p * 576);
    }
}

/* ------------------------------------------------------------------ indexing */

typedef struct {
    int nx, ny, nz;
    long n;
} orc_grid;

static orc_grid mkgrid(int nx, int ny, int nz)
{
    orc_grid g = {nx, ny, nz, (long)nx * ny * nz};
    return g;
}

/* Global node indices of the 8 corners of voxel e (Eq. pbc_indices, 0-based). */
static void orc_element_nodes(const orc_grid* g, long e, long nodes[8])
{
    int i = (int)(e % g->nx), j = (int)((e / g->nx) % g->ny), k = (int)(e / ((long)g->nx * g->ny));
    for (int a = 0; a < 8; ++a) {
        int ii = (i + (a & 1)) % g->nx;
        int jj = (j + ((a >> 1) & 1)) % g->ny;
        int kk = (k + ((a >> 2) & 1)) % g->nz;
        nodes[a] = ii + (long)g->nx * (jj + (long)g->ny * kk);
    }
}

/* Voxel that has node m as its local corner a. */
static long orc_voxel_with_corner(const orc_grid* g, long m, int a)
{
    int i = (int)(m % g->nx), j = (int)((m / g->nx) % g->ny), k = (int)(m / ((long)g->nx * g->ny));
    int ii = (i - (a & 1) + g->nx) % g->nx;
    int jj = (j - ((a >> 1) & 1) + g->ny) % g->ny;
    int kk = (k - ((a >> 2) & 1) + g->nz) % g->nz;
    return ii + (long)g->nx * (jj + (long)g->ny * kk);
}

static void gather(const orc_grid* g, const double* x, const long nodes[8], double xe[NDOF])
{
    for (int a = 0; a < 8; ++a)
        for (int c = 0; c < 3; ++c) xe[3 * a + c] = x[c * g->n + nodes[a]];
}

static void affine_element_field(const double* strain, double ue[NDOF])
{
    /* tensor E from (E11,E22,E33,E23,E13,E12); u_a = E . xi_a */
    double E[3][3] = {{strain[0], strain[5], strain[4]},
                      {strain[5], strain[1], strain[3]},
                      {strain[4], strain[3], strain[2]}};
    for (int a = 0; a < 8; ++a) {
        double xi[3] = {(double)(a & 1), (double)((a >> 1) & 1), (double)((a >> 2) & 1)};
        for (int c = 0; c < 3; ++c) ue[3 * a + c] = E[c][0] * xi[0] + E[c][1] * xi[1] + E[c][2] * xi[2];
    }
}

/* ------------------------------------------------------------------ operator */

/* y += scatter_e(K_e gather_e(x)) for voxel e. */
static void apply_element(const orc_grid* g, const int32_t* phase, const double* ke, const double* x,
                          double* y, long e)
{
    long nodes[8];
    double xe[NDOF];
    const double* K = ke + (size_t)phase[e] * 576;
    orc_element_nodes(g, e, nodes);
    gather(g, x, nodes, xe);
    for (int p = 0; p < NDOF; ++p) {
        double s = 0.0;
        for (int q = 0; q < NDOF; ++q) s += K[p * NDOF + q] * xe[q];
        y[(p % 3) * g->n + nodes[p / 3]] += s;
    }
}

/* y = A x, A = sum_e scatter K_e gather (matrix-free, Algorithm 2 step A). */
void orc_apply(int nx, int ny, int nz, const int32_t* phase, const double* ke,
               const double* x, double* y)
{
    orc_grid g = mkgrid(nx, ny, nz);
    memset(y, 0, sizeof(double) * 3 * g.n);
#ifdef _OPENMP
    /* element layer k writes node planes k and (k+1) % nz only: layers of
       one colour never write the same plane */
    const long plane = (long)nx * ny;
    const int ncol = (nz % 2) ? 3 : 2;
    for (int col = 0; col < ncol; ++col) {
        const int kfirst = col < 2 ? col : nz - 1;
        const int klast = (col == 0 && ncol == 3) ? nz - 2 : nz - 1;
#pragma omp parallel for schedule(dynamic, 1)
        for (int k = kfirst; k <= klast; k += 2)
            for (long e = k * plane; e < (k + 1) * plane; ++e) apply_element(&g, phase, ke, x, y, e);
    }
#else
    for (long e = 0; e < g.n; ++e) apply_element(&g, phase, ke, x, y, e);
#endif
}

/* (A x) at selected nodes only, from the 8 voxels around each node. */
void orc_apply_at(int nx, int ny, int nz, const int32_t* phase, const double* ke,
                  const double* x, const int64_t* sel, long count, double* y)
{
    orc_grid g = mkgrid(nx, ny, nz);
    long nodes[8];
    double xe[NDOF];
    for (long s = 0; s < count; ++s) {
        long m = sel[s];
        double acc[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 8; ++a) {
            long e = orc_voxel_with_corner(&g, m, a);
            const double* K = ke + (size_t)phase[e] * 576;
            orc_element_nodes(&g, e, nodes);
            gather(&g, x, nodes, xe);
            for (int c = 0; c < 3; ++c) {
                double t = 0.0;
                for (int q = 0; q < NDOF; ++q) t += K[(3 * a + c) * NDOF + q] * xe[q];
                acc[c] += t;
            }
        }
        for (int c = 0; c < 3; ++c) y[c * count + s] = acc[c];
    }
}

/* b = sum_e scatter(K_e u^E_e); returns ||b||_ref^2 = sum_e ||K_e u^E_e||^2 in *ref2. */
void orc_load(int nx, int ny, int nz, const int32_t* phase, const double* ke,
              const double* strain, double* b, double* ref2)
{
    orc_grid g = mkgrid(nx, ny, nz);
    memset(b, 0, sizeof(double) * 3 * g.n);
    double ue[NDOF];
    affine_element_field(strain, ue);
    long nodes[8];
    double r2 = 0.0;
    for (long e = 0; e < g.n; ++e) {
        const double* K = ke + (size_t)phase[e] * 576;
        orc_element_nodes(&g, e, nodes);
        for (int p = 0; p < NDOF; ++p) {
            double s = 0.0;
            for (int q = 0; q < NDOF; ++q) s += K[p * NDOF + q] * ue[q];
            b[(p % 3) * g.n + nodes[p / 3]] += s;
            r2 += s * s;
        }
    }
    if (ref2) *ref2 = r2;
}

void orc_load_at(int nx, int ny, int nz, const int32_t* phase, const double* ke,
                 const double* strain, const int64_t* sel, long count, double* b)
{
    orc_grid g = mkgrid(nx, ny, nz);
    double ue[NDOF];
    affine_element_field(strain, ue);
    for (long s = 0; s < count; ++s) {
        long m = sel[s];
        double acc[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 8; ++a) {
            const double* K = ke + (size_t)phase[orc_voxel_with_corner(&g, m, a)] * 576;
            for (int c = 0; c < 3; ++c) {
                double t = 0.0;
                for (int q = 0; q < NDOF; ++q) t += K[(3 * a + c) * NDOF + q] * ue[q];
                acc[c] += t;
            }
        }
        for (int c = 0; c < 3; ++c) b[c * count + s] = acc[c];
    }
}

/* ------------------------------------------------------------ preconditioner */

/* Diagonal 3x3 block A_mm = sum over the 8 voxels of (K_e)_aa; returns the
 * number of non-void voxels around the node. */
static int orc_diag_block(const orc_grid* g, const int32_t* phase, const double* ke,
                          const unsigned char* voidp, long m, double D[9])
{
    int solid = 0;
    memset(D, 0, sizeof(double) * 9);
    for (int a = 0; a < 8; ++a) {
        int p = phase[orc_voxel_with_corner(g, m, a)];
        if (!voidp[p]) solid++;
        const double* K = ke + (size_t)p * 576;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) D[3 * r + c] += K[(3 * a + r) * NDOF + 3 * a + c];
    }
    return solid;
}

/* Cofactor (adjugate / determinant) inverse of a 3x3 block (Eq. block_precond). */
static void orc_inv3(const double A[9], double X[9])
{
    double c00 = A[4] * A[8] - A[5] * A[7];
    double c01 = A[5] * A[6] - A[3] * A[8];
    double c02 = A[3] * A[7] - A[4] * A[6];
    double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    double id = 1.0 / det;
    X[0] = c00 * id;
    X[1] = (A[2] * A[7] - A[1] * A[8]) * id;
    X[2] = (A[1] * A[5] - A[2] * A[4]) * id;
    X[3] = c01 * id;
    X[4] = (A[0] * A[8] - A[2] * A[6]) * id;
    X[5] = (A[2] * A[3] - A[0] * A[5]) * id;
    X[6] = c02 * id;
    X[7] = (A[1] * A[6] - A[0] * A[7]) * id;
    X[8] = (A[0] * A[4] - A[1] * A[3]) * id;
}

static unsigned char* void_flags(int nphase, const double* C)
{
    unsigned char* v = (unsigned char*)malloc((size_t)nphase);
    for (int p = 0; p < nphase; ++p) v[p] = (unsigned char)orc_phase_is_void(C + 36 * p);
    return v;
}

/* minv: N x 9 (row-major 3x3 per node).  identity != 0 gives plain CG's
 * M^-1 = I on active nodes.  Inactive nodes (all 8 voxels void) get 0. */
void orc_precond(int nx, int ny, int nz, const int32_t* phase, const double* ke,
                 int nphase, const double* C, int identity, double* minv)
{
    orc_grid g = mkgrid(nx, ny, nz);
    unsigned char* voidp = void_flags(nphase, C);
#pragma omp parallel for schedule(static)
    for (long m = 0; m < g.n; ++m) {
        double D[9];
        double* X = minv + 9 * m;
        int solid = orc_diag_block(&g, phase, ke, voidp, m, D);
        if (!solid) {
            memset(X, 0, sizeof(double) * 9);
        } else if (identity) {
            memset(X, 0, sizeof(double) * 9);
            X[0] = X[4] = X[8] = 1.0;
        } else {
            orc_inv3(D, X);
        }
    }
    free(voidp);
}

void orc_precond_at(int nx, int ny, int nz, const int32_t* phase, const double* ke,
                    int nphase, const double* C, const int64_t* sel, long count, double* minv)
{
    orc_grid g = mkgrid(nx, ny, nz);
    unsigned char* voidp = void_flags(nphase, C);
    double D[9];
    for (long s = 0; s < count; ++s) {
        double* X = minv + 9 * s;
        if (!orc_diag_block(&g, phase, ke, voidp, sel[s], D))
            memset(X, 0, sizeof(double) * 9);
        else
            orc_inv3(D, X);
    }
    free(voidp);
}

static void apply_minv(long n, const double* minv, const double* g, double* z)
{
#pragma omp parallel for schedule(static)
    for (long m = 0; m < n; ++m) {
        const double* X = minv + 9 * m;
        double g0 = g[m], g1 = g[n + m], g2 = g[2 * n + m];
        z[m] = X[0] * g0 + X[1] * g1 + X[2] * g2;
        z[n + m] = X[3] * g0 + X[4] * g1 + X[5] * g2;
        z[2 * n + m] = X[6] * g0 + X[7] * g1 + X[8] * g2;
    }
}

static double dot(long len, const double* a, const double* b)
{
    double s = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : s)
    for (long t = 0; t < len; ++t) s += a[t] * b[t];
    return s;
}

/* ------------------------------------------------------------------ PCG */

enum { ORC_CONVERGED = 0, ORC_NOT_CONVERGED = 1, ORC_BREAKDOWN = 2 };

/*
 * Algorithm 2 (point-block Jacobi PCG, Fletcher-Reeves directions) on
 * A w = -b, starting from w = 0.  info[0] iterations, info[1] recursive
 * ||g||/||b||, info[2] sqrt(gg/gg0), info[3] true ||A w + b||/||b||,
 * info[4] restarts.  mode 0: metric criterion, 1: paper criterion.
 * Returns the status.  ``trace`` (optional, maxit entries) receives
 * ||g||/||b|| after each iteration.
 */
int orc_pcg(int nx, int ny, int nz, const int32_t* phase, const double* ke,
            const double* minv, const double* b, double bref2, double tol, int maxit,
            int mode, double* w, double* info, double* trace)
{
    orc_grid g0 = mkgrid(nx, ny, nz);
    long n = g0.n, len = 3 * n;
    double* g = (double*)malloc(sizeof(double) * len);
    double* z = (double*)malloc(sizeof(double) * len);
    double* h = (double*)malloc(sizeof(double) * len);
    double* Ah = (double*)malloc(sizeof(double) * len);
    memset(w, 0, sizeof(double) * len);
    memcpy(g, b, sizeof(double) * len);

    double bnorm = sqrt(dot(len, b, b));
    int it = 0, status = ORC_NOT_CONVERGED, restarts = 0;
    double relres = 1.0, relpre = 1.0, truerel = 1.0;
    if (bnorm <= 1e-14 * sqrt(bref2)) {
        status = ORC_CONVERGED;
        relres = relpre = truerel = 0.0;
        goto done;
    }
    for (;;) {
        apply_minv(n, minv, g, z);
        memcpy(h, z, sizeof(double) * len);
        double gg = dot(len, z, g);
        double gg0 = gg;
        int stop = 0;
        while (it < maxit) {
            ++it;
            orc_apply(nx, ny, nz, phase, ke, h, Ah);           /* A. directional stiffness */
            double hAh = dot(len, h, Ah);                      /* B. step size */
            if (!(hAh > 0.0) || !isfinite(hAh)) { status = ORC_BREAKDOWN; stop = 1; break; }
            double lambda = gg / hAh;
#pragma omp parallel for schedule(static)
            for (long t = 0; t < len; ++t) {                   /* C. update */
                w[t] -= lambda * h[t];
                g[t] -= lambda * Ah[t];
            }
            apply_minv(n, minv, g, z);                         /* D. precondition */
            double gg_last = gg;
            gg = dot(len, z, g);
            relres = sqrt(dot(len, g, g)) / bnorm;
            relpre = gg0 > 0.0 ? sqrt(fabs(gg / gg0)) : 0.0;
            if (trace) trace[it - 1] = relres;
            int conv = (mode == 1) ? (relpre < tol) : (relres <= tol);
            if (conv) { status = ORC_CONVERGED; break; }
            double gamma = gg / gg_last;                       /* E. Fletcher-Reeves */
#pragma omp parallel for schedule(static)
            for (long t = 0; t < len; ++t) h[t] = z[t] + gamma * h[t];
        }
        if (stop || status != ORC_CONVERGED || mode == 1) break;
        /* metric mode: confirm with the true residual, restart from w otherwise */
        orc_apply(nx, ny, nz, phase, ke, w, g);
        for (long t = 0; t < len; ++t) g[t] += b[t];
        truerel = sqrt(dot(len, g, g)) / bnorm;
        if (truerel <= tol) break;
        status = ORC_NOT_CONVERGED;
        if (it >= maxit) break;
        ++restarts;
    }
done:
    if (bnorm > 0.0) {
        orc_apply(nx, ny, nz, phase, ke, w, g);
        for (long t = 0; t < len; ++t) g[t] += b[t];
        truerel = sqrt(dot(len, g, g)) / bnorm;
    }
    info[0] = it;
    info[1] = relres;
    info[2] = relpre;
    info[3] = truerel;
    info[4] = restarts;
    free(g); free(z); free(h); free(Ah);
    return status;
}

/* ------------------------------------------------------------------ stress */

/*
 * Voxel stress sigma_e = C_p (E_hat + B(1/2,1/2,1/2) w_e), the voxel average
 * of the trilinear field; voids give 0.  sigma: 6 x N (may be NULL); avg: 6,
 * the mean over all N voxels.
 */
void orc_stress(int nx, int ny, int nz, const int32_t* phase, int nphase, const double* C,
                const double* strain, const double* w, double* sigma, double* avg)
{
    (void)nphase;
    orc_grid g = mkgrid(nx, ny, nz);
    double B[6][NDOF];
    orc_bmatrix(0.5, 0.5, 0.5, B);
    double Ehat[6] = {strain[0], strain[1], strain[2], 2 * strain[3], 2 * strain[4], 2 * strain[5]};
    double sum[6] = {0, 0, 0, 0, 0, 0};
    long nodes[8];
    double we[NDOF];
    for (long e = 0; e < g.n; ++e) {
        const double* Cp = C + 36 * (size_t)phase[e];
        orc_element_nodes(&g, e, nodes);
        gather(&g, w, nodes, we);
        double eps[6];
        for (int r = 0; r < 6; ++r) {
            double s = Ehat[r];
            for (int q = 0; q < NDOF; ++q) s += B[r][q] * we[q];
            eps[r] = s;
        }
        for (int r = 0; r < 6; ++r) {
            double s = 0.0;
            for (int t = 0; t < 6; ++t) s += Cp[6 * r + t] * eps[t];
            if (sigma) sigma[r * g.n + e] = s;
            sum[r] += s;
        }
    }
    for (int r = 0; r < 6; ++r) avg[r] = sum[r] / (double)g.n;
}

/* Total potential energy Pi(w) = 1/2 sum_e (u^E_e + w_e)^T K_e (u^E_e + w_e). */
double orc_energy(int nx, int ny, int nz, const int32_t* phase, const double* ke,
                  const double* strain, const double* w)
{
    orc_grid g = mkgrid(nx, ny, nz);
    double ue[NDOF], we[NDOF], te[NDOF];
    affine_element_field(strain, ue);
    long nodes[8];
    double sum = 0.0;
    for (long e = 0; e < g.n; ++e) {
        const double* K = ke + (size_t)phase[e] * 576;
        orc_element_nodes(&g, e, nodes);
        gather(&g, w, nodes, we);
        for (int q = 0; q < NDOF; ++q) te[q] = ue[q] + we[q];
        double s = 0.0;
        for (int p = 0; p < NDOF; ++p) {
            double r = 0.0;
            for (int q = 0; q < NDOF; ++q) r += K[p * NDOF + q] * te[q];
            s += te[p] * r;
        }
        sum += 0.5 * s;
    }
    return sum;
}

/* Threads of the OpenMP build (timing only); nothing in the serial build. */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
