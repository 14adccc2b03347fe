// gfx950 kernels of the matrix-free point-block Jacobi PCG for periodic voxel
// elasticity (ELAS3D-Xtal, arXiv 2602.07354, Sec. 2.1.2, Algorithm 2).
//
// Element operator.  For a unit voxel with trilinear shape functions the
// product K_e u_e (Eq. discrete_energy) is evaluated without forming the
// 24x24 K_e.  Writing each displacement component in the L2-orthogonal basis
// {1, X, Y, Z, XY, XZ, YZ, XYZ} (X = x - 1/2, ...) of the voxel, the strain
// lives in span{1, X, Y, Z, XY, XZ, YZ} with weights 1, 1/12, 1/144, so the
// element energy splits into seven small quadratic forms of C.  The basis
// coefficients are an 8-point +-1 transform (butterfly) of the nodal values;
// the nodal forces are the adjoint transform of the mode stresses.  This is
// exactly K_e u_e (same bilinear form, 2x2x2 Gauss being exact) at about
// 330 flops per voxel instead of 1152.
//
// Sweep structure.  A workgroup of TX x TY lanes owns an (x,y) column of
// (TX-1) x (TY-1) nodes and marches through a chunk of z planes.  Lane
// (tx,ty) evaluates the voxel column whose upper corner is its own node, so
// one element layer per step; node planes are staged once in LDS and shared
// by the four voxels around each node (neighbour-plane reuse), forces of the
// lower face are carried in registers to the next step (z coupling) and the
// in-plane coupling goes through LDS.  The ring of voxels on the low x/y edge
// of a column is evaluated by two workgroups.
//
// Reductions are two-stage and deterministic: a fixed-order in-block tree
// writes one partial per block, a single-block kernel sums the partials in
// fixed order and updates the device-resident PCG scalars.
#include <type_traits>

#include "elas3d_internal.h"

namespace e3d {

namespace {

constexpr int kBlock = 256;
constexpr int kFinThreads = 256;

// Index of (r,c) in the packed upper triangle of a symmetric 6x6.
__host__ __device__ constexpr int ut(int r, int c)
{
    return r <= c ? r * 6 - (r * (r - 1)) / 2 + (c - r) : c * 6 - (c * (c - 1)) / 2 + (r - c);
}

// ----------------------------------------------------------------- element

// In-place +-1 transform of 8 corner values (corner a = ax + 2ay + 4az).
// Output slot mu holds sum_a prod_{d in mu} s_d(a) v_a, s = 2 a_d - 1; slot 1
// is X, 2 Y, 3 XY, 4 Z, 5 XZ, 6 YZ, 7 XYZ (slot 0, the plain sum, is unused).
template <typename R>
__device__ __forceinline__ void fwd8(R* v)
{
#pragma unroll
    for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
        for (int a = 0; a < 8; ++a)
            if (!(a & bit)) {
                const R lo = v[a], hi = v[a | bit];
                v[a] = lo + hi;
                v[a | bit] = hi - lo;
            }
}

// Adjoint (transpose) of fwd8.
template <typename R>
__device__ __forceinline__ void adj8(R* v)
{
#pragma unroll
    for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
        for (int a = 0; a < 8; ++a)
            if (!(a & bit)) {
                const R lo = v[a], hi = v[a | bit];
                v[a] = lo - hi;
                v[a | bit] = lo + hi;
            }
}

// t = C[sup,sup] e for a support of the 6 Voigt components; a row r whose
// bit is set in ACC adds to the value t[r] holds on entry (its chain of FMAs
// starts there).
template <int N, unsigned ACC = 0u, typename R>
__device__ __forceinline__ void contract(const R* Cu, const int (&sup)[N], const R* e, R* t)
{
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R acc = ((ACC >> r) & 1u) ? fma(Cu[ut(sup[r], sup[0])], e[0], t[r]) : Cu[ut(sup[r], sup[0])] * e[0];
#pragma unroll
        for (int c = 1; c < N; ++c) acc = fma(Cu[ut(sup[r], sup[c])], e[c], acc);
        t[r] = acc;
    }
}

enum { MX = 1, MY = 2, MXY = 3, MZ = 4, MXZ = 5, MYZ = 6, MXYZ = 7 };

// The stiffness table holds C/16 (exact: a power of two).  With H the +-1
// transform of the nodal values, the element energy is
//   1/2 [ (1/16) e1^T C e1 + (1/48) sum_{X,Y,Z} e^T C e + (1/144) sum_{YZ,XZ,XY} e^T C e ]
// (coefficient scales 1/4, 1/2, 1 of the transform times the L2 weights 1,
// 1/12, 1/144 of the modes), so with Cs = C/16 the linear modes carry an
// extra weight 1/3 and the bilinear ones 1/9.  Each class of modes reads and
// writes its own slots of H and G (constant: MX, MY, MZ; linear: MXY, MXZ,
// MYZ; bilinear: MXYZ), so the weights can be applied to G afterwards.
constexpr double kLinearWeight = 1.0 / 3.0, kBilinearWeight = 1.0 / 9.0;

// modal_core: H[c][mu] (slots MX..MXYZ) -> G[c][mu] = dE/dH before the mode
// weights (slots MXY, MXZ, MYZ still to be multiplied by 1/3 and MXYZ by
// 1/9; slot 0 is not written and must be treated as 0).
template <typename R>
__device__ __forceinline__ void modal_core(const R* Cs, const R (&H)[3][8], R (&G)[3][8])
{
    // constant mode: full 6-component strain
    {
        constexpr int sup[6] = {0, 1, 2, 3, 4, 5};
        const R e[6] = {H[0][MX], H[1][MY], H[2][MZ], H[1][MZ] + H[2][MY], H[0][MZ] + H[2][MX],
                        H[0][MY] + H[1][MX]};
        R t[6];
        contract<6>(Cs, sup, e, t);
        G[0][MX] = t[0];
        G[1][MY] = t[1];
        G[2][MZ] = t[2];
        G[1][MZ] = t[3];
        G[2][MY] = t[3];
        G[0][MZ] = t[4];
        G[2][MX] = t[4];
        G[0][MY] = t[5];
        G[1][MX] = t[5];
    }
    // X mode: (yy, zz, yz, xz, xy)
    {
        constexpr int sup[5] = {1, 2, 3, 4, 5};
        const R e[5] = {H[1][MXY], H[2][MXZ], H[1][MXZ] + H[2][MXY], H[0][MXZ], H[0][MXY]};
        R t[5];
        contract<5>(Cs, sup, e, t);
        G[1][MXY] = t[0];
        G[2][MXZ] = t[1];
        G[1][MXZ] = t[2];
        G[2][MXY] = t[2];
        G[0][MXZ] = t[3];
        G[0][MXY] = t[4];
    }
    // Y mode: (xx, zz, yz, xz, xy)
    {
        constexpr int sup[5] = {0, 2, 3, 4, 5};
        const R e[5] = {H[0][MXY], H[2][MYZ], H[1][MYZ], H[0][MYZ] + H[2][MXY], H[1][MXY]};
        R t[5];
        t[0] = G[0][MXY];
        t[4] = G[1][MXY];
        contract<5, 0x11u>(Cs, sup, e, t);
        G[0][MXY] = t[0];
        G[2][MYZ] = t[1];
        G[1][MYZ] = t[2];
        G[0][MYZ] = t[3];
        G[2][MXY] += t[3];
        G[1][MXY] = t[4];
    }
    // Z mode: (xx, yy, yz, xz, xy)
    {
        constexpr int sup[5] = {0, 1, 3, 4, 5};
        const R e[5] = {H[0][MXZ], H[1][MYZ], H[2][MYZ], H[2][MXZ], H[0][MYZ] + H[1][MXZ]};
        R t[5];
        t[0] = G[0][MXZ];
        t[1] = G[1][MYZ];
        t[2] = G[2][MYZ];
        t[3] = G[2][MXZ];
        contract<5, 0x0Fu>(Cs, sup, e, t);
        G[0][MXZ] = t[0];
        G[1][MYZ] = t[1];
        G[2][MYZ] = t[2];
        G[2][MXZ] = t[3];
        G[0][MYZ] += t[4];
        G[1][MXZ] += t[4];
    }
    // YZ mode: (xx, xz, xy)
    {
        constexpr int sup[3] = {0, 4, 5};
        const R e[3] = {H[0][MXYZ], H[2][MXYZ], H[1][MXYZ]};
        R t[3];
        contract<3>(Cs, sup, e, t);
        G[0][MXYZ] = t[0];
        G[2][MXYZ] = t[1];
        G[1][MXYZ] = t[2];
    }
    // XZ mode: (yy, yz, xy)
    {
        constexpr int sup[3] = {1, 3, 5};
        const R e[3] = {H[1][MXYZ], H[2][MXYZ], H[0][MXYZ]};
        R t[3] = {G[1][MXYZ], G[2][MXYZ], G[0][MXYZ]};
        contract<3, 0x7u>(Cs, sup, e, t);
        G[1][MXYZ] = t[0];
        G[2][MXYZ] = t[1];
        G[0][MXYZ] = t[2];
    }
    // XY mode: (zz, yz, xz)
    {
        constexpr int sup[3] = {2, 3, 4};
        const R e[3] = {H[2][MXYZ], H[1][MXYZ], H[0][MXYZ]};
        R t[3] = {G[2][MXYZ], G[1][MXYZ], G[0][MXYZ]};
        contract<3, 0x7u>(Cs, sup, e, t);
        G[2][MXYZ] = t[0];
        G[1][MXYZ] = t[1];
        G[0][MXYZ] = t[2];
    }
}

// f = K_e u for one voxel with the scaled packed stiffness Cs.  u[c][a] is
// destroyed.  f[c][a]: force component c on corner a.
template <typename R>
__device__ __forceinline__ void element_force(const R* Cs, R (&u)[3][8], R (&f)[3][8])
{
    fwd8(u[0]);
    fwd8(u[1]);
    fwd8(u[2]);
    R g[3][8];
    modal_core(Cs, u, g);
    const R lw = R(kLinearWeight), bw = R(kBilinearWeight);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        g[c][0] = R(0);
        g[c][MXY] *= lw;
        g[c][MXZ] *= lw;
        g[c][MYZ] *= lw;
        g[c][MXYZ] *= bw;
        adj8(g[c]);
#pragma unroll
        for (int a = 0; a < 8; ++a) f[c][a] = g[c][a];
    }
}

// 2D transform of a face (corner q = ax + 2ay) into the slots {sum, X, Y, XY}.
template <typename R>
__device__ __forceinline__ void face_fwd(R v0, R v1, R v2, R v3, R (&F)[4])
{
    const R p0 = v0 + v1, d0 = v1 - v0, p1 = v2 + v3, d1 = v3 - v2;
    F[0] = p0 + p1;
    F[2] = p1 - p0;
    F[1] = d0 + d1;
    F[3] = d1 - d0;
}

// Adjoint of face_fwd: face slots -> corner values.
template <typename R>
__device__ __forceinline__ void face_adj(const R (&F)[4], R (&v)[4])
{
    const R o0 = F[0] - F[1], o1 = F[0] + F[1], o2 = F[2] - F[3], o3 = F[2] + F[3];
    v[0] = o0 - o2;
    v[2] = o0 + o2;
    v[1] = o1 - o3;
    v[3] = o1 + o3;
}

// Element operator on face spectra: L, U = face_fwd of the lower (z) and
// upper node planes' corner values; returns the face spectra FL, FU of the
// lower- and upper-face corner forces (face_adj turns them into forces).
template <typename R>
__device__ __forceinline__ void element_force_faces(const R* Cs, const R (&L)[3][4], const R (&U)[3][4],
                                                    R (&FL)[3][4], R (&FU)[3][4])
{
    R H[3][8], G[3][8];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        // z stage: slots without z are sums of the faces, slots with z differences
        H[c][MX] = U[c][1] + L[c][1];
        H[c][MY] = U[c][2] + L[c][2];
        H[c][MXY] = U[c][3] + L[c][3];
        H[c][MZ] = U[c][0] - L[c][0];
        H[c][MXZ] = U[c][1] - L[c][1];
        H[c][MYZ] = U[c][2] - L[c][2];
        H[c][MXYZ] = U[c][3] - L[c][3];
    }
    modal_core(Cs, H, G);
    const R lw = R(kLinearWeight), bw = R(kBilinearWeight);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        // adjoint of the z stage (slot 0 of G is zero), with the mode weights
        FL[c][0] = -G[c][MZ];
        FU[c][0] = G[c][MZ];
        FL[c][1] = fma(-lw, G[c][MXZ], G[c][MX]);
        FU[c][1] = fma(lw, G[c][MXZ], G[c][MX]);
        FL[c][2] = fma(-lw, G[c][MYZ], G[c][MY]);
        FU[c][2] = fma(lw, G[c][MYZ], G[c][MY]);
        const R b3 = bw * G[c][MXYZ];
        FL[c][3] = fma(lw, G[c][MXY], -b3);
        FU[c][3] = fma(lw, G[c][MXY], b3);
    }
}

// 21 packed coefficients of phase p (table stride kCoefStride entries).
__device__ __forceinline__ void load_coef(const double* __restrict__ coef, int p, double (&Cu)[21])
{
    const double2* src = reinterpret_cast<const double2*>(coef + (size_t)p * kCoefStride);
#pragma unroll
    for (int q = 0; q < 10; ++q) {
        const double2 v = src[q];
        Cu[2 * q] = v.x;
        Cu[2 * q + 1] = v.y;
    }
    Cu[20] = coef[(size_t)p * kCoefStride + 20];
}

__device__ __forceinline__ void load_coef(const float* __restrict__ coef, int p, float (&Cu)[21])
{
    const float4* src = reinterpret_cast<const float4*>(coef + (size_t)p * kCoefStride);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const float4 v = src[q];
        Cu[4 * q] = v.x;
        Cu[4 * q + 1] = v.y;
        Cu[4 * q + 2] = v.z;
        Cu[4 * q + 3] = v.w;
    }
    Cu[20] = coef[(size_t)p * kCoefStride + 20];
}

// ---------------------------------------------------------------- reductions

// Fixed-order block sum of NV values; thread 0 writes partials[k*stride + bid].
template <int NV, int NT>
__device__ __forceinline__ void block_partials(double (&v)[NV], double* partials, int stride, int bid)
{
    __shared__ double red[NV][NT / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if (lane == 0) red[k][wid] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = red[k][0];
            for (int w = 1; w < NT / 64; ++w) s += red[k][w];
            partials[(size_t)k * stride + bid] = s;
        }
    }
}

enum FinKind { FIN_STORE = 0, FIN_INIT = 1, FIN_DIRECTION = 2, FIN_UPDATE = 3 };

// Sums NV partial vectors (nblocks each) in fixed order, then:
//   FIN_STORE     out[k] = total[k]
//   FIN_INIT      start of a PCG run (gg, rr)
//   FIN_DIRECTION step size from h.Ah (Algorithm 2, B)
//   FIN_UPDATE    gg, rr after the update; convergence; Fletcher-Reeves gamma (D, E)
template <int NV>
__device__ __forceinline__ void finalize_body(int kind, const double* partials, int stride, int nblocks,
                                              Scalars* S, double* out, const double* norms)
{
    __shared__ double red[NV][kFinThreads / 64];
    // sweeps enqueued after the stop flag was raised did no work: leave the
    // scalars of the finished run untouched
    if ((kind == FIN_DIRECTION || kind == FIN_UPDATE) && S->done) return;
    // Each lane adds its partials in increasing block order.  The loads of
    // kFinBatch consecutive strides are issued together, so that their
    // latencies overlap (one at a time, a grid of 32768 update workgroups
    // took about 90 us to reduce).
    constexpr int kFinBatch = 8;
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    int b = threadIdx.x;
    for (; b + (kFinBatch - 1) * kFinThreads < nblocks; b += kFinBatch * kFinThreads) {
        double x[NV][kFinBatch];
#pragma unroll
        for (int k = 0; k < NV; ++k)
#pragma unroll
            for (int u = 0; u < kFinBatch; ++u) x[k][u] = partials[(size_t)k * stride + b + u * kFinThreads];
#pragma unroll
        for (int k = 0; k < NV; ++k)
#pragma unroll
            for (int u = 0; u < kFinBatch; ++u) v[k] += x[k][u];
    }
    for (; b < nblocks; b += kFinThreads)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += partials[(size_t)k * stride + b];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if (lane == 0) red[k][wid] = x;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double tot[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = red[k][0];
        for (int w = 1; w < kFinThreads / 64; ++w) s += red[k][w];
        tot[k] = s;
    }
    if (kind == FIN_STORE) {
#pragma unroll
        for (int k = 0; k < NV; ++k) out[k] = tot[k];
        return;
    }
    if (kind == FIN_INIT) {
        // tot = {z.g, g.g}; norms = {||b||^2, ||b||_ref^2} of the case
        S->gg = tot[0];
        S->gg0 = tot[0];
        S->rr = tot[NV > 1 ? 1 : 0];
        S->bnorm2 = norms[0];
        S->bref2 = norms[1];
        S->lambda = 0.0;
        S->lambda_prev = 0.0;
        S->gamma = 0.0;
        S->cur = 0;
        S->pending = 0;
        S->done = 0;
        S->status = 1;
        // zero load (homogeneous or all-void grid): nothing to solve
        if (S->bnorm2 <= 1e-28 * S->bref2) {
            S->done = 1;
            S->status = 0;
        } else if (S->it >= S->maxit) {
            S->done = 1;
        }
        return;
    }
    if (kind == FIN_DIRECTION) {
        const double hAh = tot[0];
        S->hAh = hAh;
        // the sweep wrote the new direction to the other buffer; it paid the
        // owed steps if there were two and left a single one owed
        const int owed = S->pending;
        if (!(hAh > 0.0) || !isfinite(hAh)) {
            // the iteration that found the breakdown counts (its operator
            // sweep ran), as in Algorithm 2
            S->it += 1;
            S->status = 2;
            S->done = 1;
            if (owed != 1) {
                S->pending = 0;
                S->lambda = 0.0;
                S->cur ^= 1;
            }  // else lambda h of buffer cur stays owed, for the final update
        } else {
            if (owed == 1)
                S->lambda_prev = S->lambda;  // now in buffer cur ^ 1
            else
                S->pending = 0;
            S->cur ^= 1;
            S->lambda = S->gg / hAh;
        }
        return;
    }
    if (kind == FIN_UPDATE) {
        const double gg_new = tot[0];
        const double rr = tot[NV > 1 ? 1 : 0];
        S->it += 1;
        S->pending += 1;
        S->rr = rr;
        const double gg_last = S->gg;
        S->gg = gg_new;
        bool conv;
        if (S->mode == 1)
            conv = S->gg0 > 0.0 && sqrt(fabs(gg_new / S->gg0)) < S->tol;
        else
            conv = rr <= S->tol * S->tol * S->bnorm2;
        if (!isfinite(gg_new) || !isfinite(rr)) {
            S->status = 2;
            S->done = 1;
        } else if (conv) {
            S->status = 0;
            S->done = 1;
        } else if (S->it >= S->maxit) {
            S->status = 1;
            S->done = 1;
        }
        S->gamma = gg_new / gg_last;
        return;
    }
}

template <int NV>
__global__ void __launch_bounds__(kFinThreads) finalize_kernel(int kind, const double* partials,
                                                               int stride, int nblocks, Scalars* S,
                                                               double* out, const double* norms,
                                                               int rhs_stride)
{
    // block r finalizes RHS r of a batch
    finalize_body<NV>(kind, partials + (size_t)blockIdx.x * rhs_stride, stride, nblocks,
                      S ? S + blockIdx.x : nullptr, out, norms);
}

// One (problem, RHS) of a group's finalize.
struct FinItem {
    const double* partials;
    int stride, nblocks;
    Scalars* S;
};

template <int NV>
__global__ void __launch_bounds__(kFinThreads) finalize_group_kernel(int kind, const FinItem* __restrict__ items)
{
    const FinItem it = items[blockIdx.x];
    finalize_body<NV>(kind, it.partials, it.stride, it.nblocks, it.S, nullptr, nullptr);
}

// ------------------------------------------------------------- node sweeps

__device__ __forceinline__ void node_ijk(int m, const Dims& d, int& i, int& j, int& k)
{
    const int plane = d.nx * d.ny;
    k = m / plane;
    const int r = m - k * plane;
    j = r / d.nx;
    i = r - j * d.nx;
}

// b_m = sum over the 8 voxels around node m of the force that voxel's
// uniform stress C_p E_hat exerts on its corner: (sigma s_a)/4, s_a = 2a-1
// (the element vector K_e u^E_e of the affine field, Eq. affine_strain).
__global__ void __launch_bounds__(kBlock) load_kernel(Dims d, const int32_t* __restrict__ phase,
                                                      const double* __restrict__ sig, double* bx,
                                                      double* by, double* bz, double* partials,
                                                      int stride)
{
    double acc[2] = {0.0, 0.0};
    for (int m = blockIdx.x * kBlock + threadIdx.x; m < d.n; m += gridDim.x * kBlock) {
        int i, j, k;
        node_ijk(m, d, i, j, k);
        double f0 = 0.0, f1 = 0.0, f2 = 0.0;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
            const int ii = i - ax < 0 ? d.nx - 1 : i - ax;
            const int jj = j - ay < 0 ? d.ny - 1 : j - ay;
            const int kk = k - az < 0 ? d.nz - 1 : k - az;
            const double* s = sig + (size_t)phase[ii + d.nx * (jj + d.ny * kk)] * kSigStride;
            const double sx = ax ? 1.0 : -1.0, sy = ay ? 1.0 : -1.0, sz = az ? 1.0 : -1.0;
            f0 += s[0] * sx + s[5] * sy + s[4] * sz;
            f1 += s[5] * sx + s[1] * sy + s[3] * sz;
            f2 += s[4] * sx + s[3] * sy + s[2] * sz;
        }
        f0 *= 0.25;
        f1 *= 0.25;
        f2 *= 0.25;
        const size_t mv = (size_t)m;
        bx[mv] = f0;
        by[mv] = f1;
        bz[mv] = f2;
        acc[0] += f0 * f0 + f1 * f1 + f2 * f2;
        // uncancelled element forces of voxel m: sum_a |sigma s_a / 4|^2 = |sigma|_F^2 / 2
        const double* s = sig + (size_t)phase[m] * kSigStride;
        acc[1] += 0.5 * (s[0] * s[0] + s[1] * s[1] + s[2] * s[2] +
                         2.0 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]));
    }
    block_partials<2, kBlock>(acc, partials, stride, blockIdx.x);
}

// Inverse of the assembled diagonal 3x3 block (Eq. block_precond) of a node
// from the phases of its eight voxels (voxel a = ax + 2 ay + 4 az lies at
// (i - ax, j - ay, k - az)).  The corner block of a phase is
// D + sx sy Oxy + sx sz Oxz + sy sz Oyz (four symmetric pieces per phase,
// ordered xx, yy, zz, yz, xz, xy); nodes whose eight voxels are all void get
// 0, plain CG gets I on the other nodes.
__device__ __forceinline__ void block_inverse(const int (&ph)[8], const double* __restrict__ diag,
                                              const uint8_t* __restrict__ solid, int identity, double (&r)[6])
{
    double A[6] = {0, 0, 0, 0, 0, 0};
    int nsolid = 0;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
        const int p = ph[a];
        nsolid += solid[p];
        const double* t = diag + (size_t)p * kDiagStride;
        const double sxy = (ax == ay) ? 1.0 : -1.0;
        const double sxz = (ax == az) ? 1.0 : -1.0;
        const double syz = (ay == az) ? 1.0 : -1.0;
#pragma unroll
        for (int q = 0; q < 6; ++q) A[q] += t[q] + sxy * t[6 + q] + sxz * t[12 + q] + syz * t[18 + q];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) r[q] = 0.0;
    if (nsolid == 0) return;
    if (identity) {
        r[0] = r[1] = r[2] = 1.0;
        return;
    }
    // symmetric [a b c; b d e; c e f] with a=xx d=yy f=zz e=yz c=xz b=xy
    const double a_ = A[0], d_ = A[1], f_ = A[2], e_ = A[3], c_ = A[4], b_ = A[5];
    const double c00 = d_ * f_ - e_ * e_;
    const double c01 = c_ * e_ - b_ * f_;
    const double c02 = b_ * e_ - c_ * d_;
    const double c11 = a_ * f_ - c_ * c_;
    const double c12 = b_ * c_ - a_ * e_;
    const double c22 = a_ * d_ - b_ * b_;
    const double inv = 1.0 / (a_ * c00 + b_ * c01 + c_ * c02);
    r[0] = c00 * inv;
    r[1] = c11 * inv;
    r[2] = c22 * inv;
    r[3] = c12 * inv;
    r[4] = c02 * inv;
    r[5] = c01 * inv;
}

// Phases of the eight voxels around node m; true when they are all the same.
__device__ __forceinline__ bool node_phases(const Dims& d, const int32_t* __restrict__ phase, int m,
                                            int (&ph)[8])
{
    int i, j, k;
    node_ijk(m, d, i, j, k);
    const int im = i == 0 ? d.nx - 1 : i - 1;
    const int jm = j == 0 ? d.ny - 1 : j - 1;
    const int km = k == 0 ? d.nz - 1 : k - 1;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        const int ii = (a & 1) ? im : i, jj = ((a >> 1) & 1) ? jm : j, kk = (a >> 2) ? km : k;
        ph[a] = phase[ii + d.nx * (jj + d.ny * kk)];
    }
    bool same = true;
#pragma unroll
    for (int a = 1; a < 8; ++a) same = same && ph[a] == ph[0];
    return same;
}

// Nodes of chunk blockIdx.x: base + s * kBlock + threadIdx.x, s = 0..15, so
// that ranks in node order are wave ballots plus a running offset.
static_assert(kPrecondChunk == 16 * kBlock, "a preconditioner chunk is 16 rows of a workgroup");

__global__ void __launch_bounds__(kBlock) precond_count_kernel(Dims d, const int32_t* __restrict__ phase,
                                                               int* __restrict__ counts)
{
    __shared__ int wc[kBlock / 64];
    const size_t base = (size_t)blockIdx.x * kPrecondChunk;
    int cnt = 0;
    for (int s = 0; s < kPrecondChunk / kBlock; ++s) {
        const size_t m = base + (size_t)s * kBlock + threadIdx.x;
        int ph[8];
        if (m < (size_t)d.n && !node_phases(d, phase, (int)m, ph)) ++cnt;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kBlock / 64; ++w) t += wc[w];
        counts[blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(kBlock) precond_fill_kernel(Dims d, const int32_t* __restrict__ phase,
                                                              const double* __restrict__ diag,
                                                              const uint8_t* __restrict__ solid,
                                                              int identity, int nphase,
                                                              const int* __restrict__ offsets,
                                                              uint32_t* __restrict__ idx,
                                                              double* m0, double* m1, double* m2,
                                                              double* m3, double* m4, double* m5)
{
    __shared__ int wc[kBlock / 64];
    const size_t base = (size_t)blockIdx.x * kPrecondChunk;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
    int run = offsets[blockIdx.x];
    for (int s = 0; s < kPrecondChunk / kBlock; ++s) {
        const size_t m = base + (size_t)s * kBlock + threadIdx.x;
        int ph[8];
        const bool live = m < (size_t)d.n;
        const bool bnd = live && !node_phases(d, phase, (int)m, ph);
        const unsigned long long ball = __ballot(bnd);
        if (lane == 0) wc[wid] = __popcll(ball);
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            before += w < wid ? wc[w] : 0;
            total += wc[w];
        }
        __syncthreads();  // wc is rewritten by the next row
        if (live) {
            if (bnd) {
                const int row = nphase + run + before + __popcll(ball & below);
                idx[m] = (uint32_t)row;
                double r[6];
                block_inverse(ph, diag, solid, identity, r);
                const size_t mq = (size_t)row;
                m0[mq] = r[0];
                m1[mq] = r[1];
                m2[mq] = r[2];
                m3[mq] = r[3];
                m4[mq] = r[4];
                m5[mq] = r[5];
            } else {
                idx[m] = (uint32_t)ph[0];
            }
        }
        run += total;
    }
}

__global__ void __launch_bounds__(kBlock) precond_table_kernel(int nphase, const double* __restrict__ diag,
                                                               const uint8_t* __restrict__ solid,
                                                               int identity, double* m0, double* m1,
                                                               double* m2, double* m3, double* m4,
                                                               double* m5)
{
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= nphase) return;
    const int ph[8] = {p, p, p, p, p, p, p, p};
    double r[6];
    block_inverse(ph, diag, solid, identity, r);
    const size_t mq = (size_t)p;
    m0[mq] = r[0];
    m1[mq] = r[1];
    m2[mq] = r[2];
    m3[mq] = r[3];
    m4[mq] = r[4];
    m5[mq] = r[5];
}

__global__ void __launch_bounds__(kBlock) precond_expand_kernel(Dims d, MinvRows<double> M, double* out)
{
    for (int m = blockIdx.x * kBlock + threadIdx.x; m < d.n; m += gridDim.x * kBlock) {
        const size_t row = (size_t)M.idx[m];
#pragma unroll
        for (int q = 0; q < 6; ++q) out[(size_t)q * d.n + m] = M.m[q][row];
    }
}

// Start (or restart) of a PCG run: g = b (or the residual already in g),
// z = M^-1 g, current direction h = 0, w = 0 on a fresh start.  Dots in FP64.
template <typename T>
__global__ void __launch_bounds__(kBlock) pcg_init_kernel(Dims d, FieldsT<T> f, MinvRows<T> M, int fresh,
                                                          int from_residual, double* partials,
                                                          int stride)
{
    double acc[2] = {0.0, 0.0};
    for (int m = blockIdx.x * kBlock + threadIdx.x; m < d.n; m += gridDim.x * kBlock) {
        const int mv = m;
        const size_t mq = (size_t)M.idx[m];
        T g[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            g[c] = from_residual ? f.g[c][mv] : f.b[c][mv];
            if (!from_residual) f.g[c][mv] = g[c];
        }
        const T xx = M.m[0][mq], yy = M.m[1][mq], zz = M.m[2][mq];
        const T yz = M.m[3][mq], xz = M.m[4][mq], xy = M.m[5][mq];
        const T z0 = xx * g[0] + xy * g[1] + xz * g[2];
        const T z1 = xy * g[0] + yy * g[1] + yz * g[2];
        const T z2 = xz * g[0] + yz * g[1] + zz * g[2];
        f.z[0][mv] = z0;
        f.z[1][mv] = z1;
        f.z[2][mv] = z2;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            f.h0[c][mv] = T(0);
            if (fresh) f.w[c][mv] = T(0);
        }
        acc[0] += (double)z0 * g[0] + (double)z1 * g[1] + (double)z2 * g[2];
        acc[1] += (double)g[0] * g[0] + (double)g[1] * g[1] + (double)g[2] * g[2];
    }
    block_partials<2, kBlock>(acc, partials, stride, blockIdx.x);
}

// A load or store of a streamed vector, optionally non-temporal (passed by
// the caches: on grids far larger than the caches nothing streamed is
// re-read from them before it is evicted anyway).
template <bool NT, typename T>
__device__ __forceinline__ T stream_load(const T* p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void stream_store(T v, T* p)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Algorithm 2, C-D for a batch of RHS sharing M^-1 (loaded once per node):
// g -= lambda Ah, z = M^-1 g, partials z.g and g.g (FP64) per RHS.
// (w -= lambda h is deferred to a later direction sweep, which reads h anyway.)
// NT: the node vectors and dictionary indices are streamed non-temporally;
// the M^-1 rows (the per-phase ones are shared by most nodes) are not.
// (by value: the fields stay in scalar registers)
template <typename T, bool NT>
__device__ __forceinline__ void update_body(const Dims d, const FieldsT<T> f, const size_t rs, const int nrhs,
                                            const MinvRows<T> M, const Scalars* S, double* partials,
                                            const int stride, const int bid, const int nblk)
{
    unsigned active = 0;
    T lam[kMaxRhs];
#pragma unroll
    for (int r = 0; r < kMaxRhs; ++r) {
        lam[r] = T(0);
        if (r < nrhs && !S[r].done) {
            active |= 1u << r;
            lam[r] = (T)S[r].lambda;
        }
    }
    if (!active) return;
    double acc[2 * kMaxRhs];
#pragma unroll
    for (int k = 0; k < 2 * kMaxRhs; ++k) acc[k] = 0.0;
    if constexpr (sizeof(T) == 8) {
        // FP64: two consecutive nodes per lane and step, with 16-byte loads
        // and stores of the node vectors (5 % faster at 500^3; FP32 pairs,
        // 8 bytes, were slower), when the node count is even and every
        // field 16-byte aligned (one condition for the whole grid)
        bool pairs = (d.n & 1) == 0 && (rs & 1) == 0 && ((uintptr_t)M.idx & 7) == 0;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            pairs = pairs && (((uintptr_t)f.g[c] | (uintptr_t)f.Ah[c] | (uintptr_t)f.z[c]) & 15) == 0;
        if (pairs) {
            typedef T T2 __attribute__((ext_vector_type(2)));
            typedef uint32_t U2 __attribute__((ext_vector_type(2)));
            for (int q = bid * kBlock + threadIdx.x; q < (d.n >> 1); q += (unsigned)nblk * kBlock) {
                const int m = 2 * q;
                const U2 mq = stream_load<NT>(reinterpret_cast<const U2*>(M.idx + m));
                T mm[2][6];
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    mm[0][k] = M.m[k][mq.x];
                    mm[1][k] = M.m[k][mq.y];
                }
#pragma unroll
                for (int r = 0; r < kMaxRhs; ++r) {
                    if (!(active & (1u << r))) continue;
                    const size_t o = (size_t)r * rs + (size_t)m;
                    T g[2][3], z[2][3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const T2 ah = stream_load<NT>(reinterpret_cast<const T2*>(f.Ah[c] + o));
                        const T2 gg = stream_load<NT>(reinterpret_cast<const T2*>(f.g[c] + o));
                        g[0][c] = fma(-lam[r], ah.x, gg.x);
                        g[1][c] = fma(-lam[r], ah.y, gg.y);
                    }
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const T xx = mm[h][0], yy = mm[h][1], zz = mm[h][2], yz = mm[h][3], xz = mm[h][4],
                                xy = mm[h][5];
                        z[h][0] = xx * g[h][0] + xy * g[h][1] + xz * g[h][2];
                        z[h][1] = xy * g[h][0] + yy * g[h][1] + yz * g[h][2];
                        z[h][2] = xz * g[h][0] + yz * g[h][1] + zz * g[h][2];
                        acc[2 * r] += (double)z[h][0] * g[h][0] + (double)z[h][1] * g[h][1] +
                                      (double)z[h][2] * g[h][2];
                        acc[2 * r + 1] += (double)g[h][0] * g[h][0] + (double)g[h][1] * g[h][1] +
                                          (double)g[h][2] * g[h][2];
                    }
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        stream_store<NT>(T2{g[0][c], g[1][c]}, reinterpret_cast<T2*>(f.g[c] + o));
                        stream_store<NT>(T2{z[0][c], z[1][c]}, reinterpret_cast<T2*>(f.z[c] + o));
                    }
                }
            }
            block_partials<2 * kMaxRhs, kBlock>(acc, partials, stride, bid);
            return;
        }
    }
    // the unsigned step (as gridDim.x * kBlock) keeps the compiler from
    // strength-reducing every field address into its own 64-bit induction
    // variable, which triples the register count
    for (int m = bid * kBlock + threadIdx.x; m < d.n; m += (unsigned)nblk * kBlock) {
        const size_t mq = (size_t)stream_load<NT>(M.idx + m);
        T mm[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) mm[q] = M.m[q][mq];
        const T xx = mm[0], yy = mm[1], zz = mm[2], yz = mm[3], xz = mm[4], xy = mm[5];
#pragma unroll
        for (int r = 0; r < kMaxRhs; ++r) {
            if (!(active & (1u << r))) continue;
            const size_t o = (size_t)r * rs + (size_t)m;
            T g[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) g[c] = fma(-lam[r], stream_load<NT>(f.Ah[c] + o), stream_load<NT>(f.g[c] + o));
            const T z0 = xx * g[0] + xy * g[1] + xz * g[2];
            const T z1 = xy * g[0] + yy * g[1] + yz * g[2];
            const T z2 = xz * g[0] + yz * g[1] + zz * g[2];
#pragma unroll
            for (int c = 0; c < 3; ++c) stream_store<NT>(g[c], f.g[c] + o);
            stream_store<NT>(z0, f.z[0] + o);
            stream_store<NT>(z1, f.z[1] + o);
            stream_store<NT>(z2, f.z[2] + o);
            acc[2 * r] += (double)z0 * g[0] + (double)z1 * g[1] + (double)z2 * g[2];
            acc[2 * r + 1] += (double)g[0] * g[0] + (double)g[1] * g[1] + (double)g[2] * g[2];
        }
    }
    block_partials<2 * kMaxRhs, kBlock>(acc, partials, stride, bid);
}

template <typename T, bool NT>
__global__ void __launch_bounds__(kBlock) update_precond_kernel(Dims d, FieldsT<T> f, size_t rs,
                                                                int nrhs, MinvRows<T> M,
                                                                const Scalars* S, double* partials,
                                                                int stride)
{
    update_body<T, NT>(d, f, rs, nrhs, M, S, partials, stride, blockIdx.x, gridDim.x);
}

// The steps still owed to w at the end of a run, oldest first.
template <typename T>
__global__ void __launch_bounds__(kBlock) final_update_kernel(Dims d, FieldsT<T> f, const Scalars* S)
{
    const int owed = S->pending;
    if (!owed) return;
    const T lam = (T)S->lambda, lamp = (T)S->lambda_prev;
    T* const* h = S->cur ? f.h1 : f.h0;
    T* const* ho = S->cur ? f.h0 : f.h1;
    for (int m = blockIdx.x * kBlock + threadIdx.x; m < d.n; m += gridDim.x * kBlock) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T w = f.w[c][m];
            if (owed == 2) w = fma(-lamp, ho[c][m], w);
            f.w[c][m] = fma(-lam, h[c][m], w);
        }
    }
}

// w += d (FP64 iterate, FP32 correction), after the refinement sweep.
__global__ void __launch_bounds__(kBlock) add_correction_kernel(Dims d, double* w0, double* w1,
                                                                double* w2, const float* d0,
                                                                const float* d1, const float* d2)
{
    for (int m = blockIdx.x * kBlock + threadIdx.x; m < d.n; m += gridDim.x * kBlock) {
        const int mv = m;
        w0[mv] += (double)d0[mv];
        w1[mv] += (double)d1[mv];
        w2[mv] += (double)d2[mv];
    }
}

// Dense stand-in data for timing a sweep: element i gets a value in
// [-1e-3, 1e-3) from a 64-bit integer hash of i (SplitMix64's finaliser), so
// that the timed sweep reads non-zero, varied node values as in a solve.
__global__ void __launch_bounds__(kBlock) tuning_fill_kernel(double* __restrict__ p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
        unsigned long long z = i + 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        p[i] = ((double)(z >> 11) * 0x1.0p-53 - 0.5) * 2e-3;
    }
}

// dst = (float) src, n elements.
__global__ void __launch_bounds__(kBlock) to_float_kernel(const double* __restrict__ src,
                                                          float* __restrict__ dst, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        dst[i] = (float)src[i];
}

// ------------------------------------------------------- tiled operator sweep

#ifndef E3D_XCD_REMAP
#define E3D_XCD_REMAP 1
#endif
constexpr int kXcds = 8;  // MI355X: 8 accelerator dies, each with its own L2

// Workgroups are handed to the XCDs round-robin: of nb consecutive
// workgroups, the b-th and the (b+8)-th run on the same XCD.  This bijection
// of b in [0, nb) gives each XCD a contiguous range of logical tiles
// instead, so that tiles that share halo rows and cache lines run on the
// same L2 at about the same time.
__device__ __forceinline__ int xcd_map(const int b, const int nb)
{
    if (!E3D_XCD_REMAP || nb < kXcds) return b;
    const int per = nb / kXcds, rem = nb % kXcds;
    const int x = b % kXcds, j = b / kXcds;
    return x < rem ? x * (per + 1) + j : rem * (per + 1) + (x - rem) * per + j;
}

__device__ __forceinline__ int xcd_local_block() { return xcd_map(blockIdx.x, gridDim.x); }

// The wave-specialised sweep runs one workgroup per CU, so each XCD holds a
// band of kCusPerXcd consecutive tiles at a time.  This bijection hands the
// XCDs adjacent bands at the same time (groups of kXcds bands of W logical
// workgroups; the tail of nb that fills no whole group keeps the
// contiguous map): the halo rows two bands share are then read by two XCDs
// at about the same time, and the second read is served by the memory-side
// cache shared by all XCDs instead of HBM.
constexpr int kCusPerXcd = 32;  // MI355X: 256 CUs in 8 XCDs
__device__ __forceinline__ int xcd_band_map(const int b, const int nb, const int W)
{
    if (!E3D_XCD_REMAP || nb < kXcds) return b;
    const int full = nb / (kXcds * W) * (kXcds * W);
    if (b < full) {
        const int x = b % kXcds, j = b / kXcds;
        return (j / W) * (kXcds * W) + x * W + (j % W);
    }
    return full + xcd_map(b - full, nb - full);
}

// Operator sweep modes.
enum OpMode { OP_APPLY = 0, OP_FUSED = 1, OP_REFINE = 2 };

template <typename T>
struct OpArgs {
    Dims d;
    int tiles_x, tiles_y, kz;
    const int32_t* phase;
    const T* coef;  // FUSED: table in T; APPLY / REFINE: FP64 table
    // APPLY / REFINE input x (FP64); REFINE adds the FP32 correction xd on the
    // fly (x itself is not written: neighbouring workgroups read it at their
    // halo nodes during the sweep)
    double* x[3];
    const float* xd[3];
    // FUSED: z, the two direction buffers, w
    const T* z[3];
    T* h0[3];
    T* h1[3];
    T* w[3];
    // outputs: y (APPLY: FP64, FUSED: T), yr (REFINE: FP32)
    T* y[3];
    double* yd[3];
    float* yr[3];
    const double* add[3];
    const Scalars* S;
    double* partials;
    int want_norm;
    size_t rs;  // FUSED: elements between consecutive RHS of the batch
    int nrhs;   // FUSED: RHS in the batch (workgroup -> (tile, rhs))
    // wave-specialised sweeps: phase dictionaries of the launch geometry
    const int32_t* wsdict;
    const uint8_t* wsmap;
};

// OP_APPLY : y = A x (+ add) in FP64, optional ||y||^2 partials.
// OP_FUSED : Algorithm 2 steps E and A of one iteration in a single sweep, in
//            T: h_new = z + gamma h_old (written to the other direction
//            buffer), Ah = A h_new and the partial h_new.Ah (FP64); when w
//            owes two steps (WPAY), also w -= lambda_prev h_prev (the
//            buffer's old content) and w -= lambda h_old, in that order.
// OP_REFINE: y = A (x + xd) + add in FP64, stored as FP32, ||y||^2 (the
//            wave-specialised form reads x after xd has been added to it).
#ifndef E3D_OP_MIN_WAVES
#define E3D_OP_MIN_WAVES 1
#endif


// Arithmetic type of an operator sweep.
template <int MODE, typename T>
using OpReal = typename std::conditional<MODE == OP_FUSED, T, double>::type;

// LDS of an operator-sweep workgroup: a node plane with its halo row and
// column, and the in-plane force exchange.
// One workgroup barrier per plane step: the node plane and the force
// exchange are double-buffered by step parity, and the forces of step s are
// summed and stored after the barrier of step s + 1.
template <int TX, int TY, typename R>
struct OpShared {
    R sn[2][3][(TY + 1) * (TX + 1)];
    R sf[2][3][3][TX * TY];
};

// Workgroup lbr (logical, of nblocks) of an operator sweep over a.
template <int TX, int TY, int MODE, typename T, bool WPAY>
__device__ __forceinline__ void op_body(OpArgs<T> a, const int lbr, const int nblocks,
                                        OpShared<TX, TY, OpReal<MODE, T>>& sh)
{
    constexpr bool FUSED = MODE == OP_FUSED;
    using R = OpReal<MODE, T>;
    constexpr int NT = TX * TY, LX = TX + 1, LY = TY + 1;
    auto& SN = sh.sn;
    auto& SF = sh.sf;

    // logical workgroup -> (RHS, tile block): the tiles of one RHS are a
    // contiguous range in the XCD-local order, laid out as in a single-RHS
    // sweep, so neighbouring workgroups stream neighbouring rows of the same
    // vectors (interleaving the RHS of one tile instead measured about 11 %
    // slower on six load cases)
    const int nr = FUSED ? a.nrhs : 1;
    const int ntb = nblocks / nr;  // tile blocks per RHS
    const int rhs = lbr / ntb;
    const int lb = lbr - rhs * ntb;
    R gam = R(0), lam = R(0), lamp = R(0);
    const T* hold[3] = {nullptr, nullptr, nullptr};
    T* hnew[3] = {nullptr, nullptr, nullptr};
    if constexpr (FUSED) {
        const Scalars* S = a.S + rhs;
        if (S->done) return;
        gam = (R)S->gamma;
        lam = (R)S->lambda;
        lamp = (R)S->lambda_prev;
        const int cur = S->cur;
        const size_t off = (size_t)rhs * a.rs;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            hold[c] = (cur ? a.h1[c] : a.h0[c]) + off;
            hnew[c] = (cur ? a.h0[c] : a.h1[c]) + off;
            a.z[c] += off;
            a.w[c] += off;
            a.y[c] += off;
        }
    }
    const R* coef = reinterpret_cast<const R*>(a.coef);

    const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz;
    const int plane = nx * ny;
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
    const int ntiles = a.tiles_x * a.tiles_y;
    const int bz = lb / ntiles, t = lb - bz * ntiles;
    const int by = t / a.tiles_x, bx = t - by * a.tiles_x;
    const int i0 = bx * (TX - 1), j0 = by * (TY - 1);
    const int k0 = bz * a.kz;
    const int kend = min(k0 + a.kz, nz);

    const int gi = i0 + tx, gj = j0 + ty;
    const int own = (gi % nx) + nx * (gj % ny);
    const int elem = ((gi + nx - 1) % nx) + nx * ((gj + ny - 1) % ny);
    const bool out_ok = (tx < TX - 1) && (ty < TY - 1) && (gi < nx) && (gj < ny);
    const bool has_halo = tid < LX + TY;
    // lanes without a halo node re-read their own node (an L1 hit), so that
    // every lane issues the same loads and no load sits behind a branch
    int hslot = 0, hoff = own;
    if (has_halo) {
        const int hx = tid < LX ? tid : 0;
        const int hy = tid < LX ? 0 : tid - LX + 1;
        hslot = hy * LX + hx;
        hoff = ((i0 - 1 + hx + nx) % nx) + nx * ((j0 - 1 + hy + ny) % ny);
    }
    const int oslot = (ty + 1) * LX + (tx + 1);
    // w is needed only where the lane writes it: lanes that own no output
    // node load the w of the nearest owned node of the tile instead (a line
    // another lane of the workgroup loads anyway), so the overlap rows and
    // columns of neighbouring tiles cost no w traffic
    int wown = own;
    if (!out_ok) {
        const int wi = min(gi, min(i0 + TX - 2, nx - 1)), wj = min(gj, min(j0 + TY - 2, ny - 1));
        wown = wi + nx * wj;
    }
    // h of two iterations back, paid to w: the old content of the buffer
    // this sweep overwrites, read by its owner lane before the overwrite.
    // Lanes without an output node read the current direction instead (a
    // buffer nothing writes during the sweep; the value is not used): the
    // two buffers lie the same distance apart in every component (checked
    // at launch), so one offset per lane selects the buffer.
    int poff = 0;
    if constexpr (WPAY) poff = out_ok ? 0 : (int)(hold[0] - hnew[0]);

    // Raw values of the next node plane, prefetched one step ahead and only
    // combined (h_new = z + gamma h_old, or x + xd) when the step that needs
    // them starts, so the loads stay in flight across a whole element layer.
    // All loads are unconditional: the wait counts of the compiler then never
    // make the contraction wait on a prefetch.
    R rz[3], rh[3], rw[3], rp[3], hz[3], hh[3];
    auto fetch = [&](int kk) {
        const int kw = kk < 0 ? kk + nz : (kk >= nz ? kk - nz : kk);
        const int base = kw * plane;
        const int io = (base + own), ih = (base + hoff);
        if constexpr (FUSED) {
            const int iw = (base + wown);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                rh[c] = hold[c][io];
                rz[c] = a.z[c][io];
                if constexpr (WPAY) {
                    rw[c] = a.w[c][iw];
                    rp[c] = hnew[c][(ptrdiff_t)iw + poff];
                }
                hh[c] = hold[c][ih];
                hz[c] = a.z[c][ih];
            }
        } else if constexpr (MODE == OP_REFINE) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                rz[c] = a.x[c][io];
                rh[c] = a.xd[c][io];
                hz[c] = a.x[c][ih];
                hh[c] = a.xd[c][ih];
            }
        } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                rz[c] = a.x[c][io];
                hz[c] = a.x[c][ih];
            }
        }
    };
    // node values (h_new, x + xd or x) of the prefetched plane
    auto own_value = [&](int c) -> R {
        if constexpr (FUSED) return fma(gam, rh[c], rz[c]);
        else if constexpr (MODE == OP_REFINE) return rz[c] + rh[c];
        else return rz[c];
    };
    auto halo_value = [&](int c) -> R {
        if constexpr (FUSED) return fma(gam, hh[c], hz[c]);
        else if constexpr (MODE == OP_REFINE) return hz[c] + hh[c];
        else return hz[c];
    };
    auto layer_phase = [&](int kl) {
        const int klw = kl < 0 ? kl + nz : (kl >= nz ? kl - nz : kl);
        return a.phase[klw * plane + elem];
    };

    // Per lane, in face-spectral form (face_fwd slots): lo = lower node plane
    // of the current element layer, carry = upper-face forces of the previous
    // layer (they act on the same node plane as this layer's lower face).
    R lo[3][4], carry[3][4];
    auto read_face = [&](int b, R (&F)[3][4]) {
        auto& sn = SN[b];
#pragma unroll
        for (int c = 0; c < 3; ++c)
            face_fwd(sn[c][ty * LX + tx], sn[c][ty * LX + tx + 1], sn[c][(ty + 1) * LX + tx],
                     sn[c][(ty + 1) * LX + tx + 1], F[c]);
    };
    double dot = 0.0;
    // y of node plane kl (of the element layers above and below it): the
    // lane's own part m plus its neighbours' parts from buffer b; the dot
    // with h (fused) or y (the other modes)
    auto emit = [&](int b, const R (&m)[3], const R (&hk)[3], int kl) {
        auto& sf = SF[b];
        const int idx = ((kl < 0 ? kl + nz : kl) * plane + own);
        R yv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            R v = m[c] + sf[2][c][tid + 1];
            v += sf[1][c][tid + TX];
            v += sf[0][c][tid + TX + 1];
            if constexpr (!FUSED) {
                if (a.add[0]) v += a.add[c][idx];
            }
            yv[c] = v;
            if constexpr (FUSED) a.y[c][idx] = v;
            else if constexpr (MODE == OP_REFINE) a.yr[c][idx] = (float)v;
            else a.yd[c][idx] = v;
        }
        if constexpr (FUSED) {
            dot += (double)hk[0] * yv[0] + (double)hk[1] * yv[1] + (double)hk[2] * yv[2];
        } else {
            dot += yv[0] * yv[0] + yv[1] * yv[1] + yv[2] * yv[2];
        }
    };
    // prologue: node plane k0-1 gives the lower face of element layer k0-1
    // (in buffer 1, so that step 0 may write buffer 0 at once)
    fetch(k0 - 1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        SN[1][c][oslot] = own_value(c);
        if (has_halo) SN[1][c][hslot] = halo_value(c);
    }
    __syncthreads();
    read_face(1, lo);
    const int nsteps = kend - k0 + 1;
    // coefficients of the current layer, phase of the next one
    R Cu[21];
    load_coef(coef, layer_phase(k0 - 1), Cu);
    int p_next = layer_phase(min(k0, kend - 1));
    fetch(k0);

    R hprev[3] = {R(0), R(0), R(0)};  // own node value of the lower plane
    // the own force part and h of the plane that step s completes, summed
    // and stored after the barrier of step s + 1
    R mine_d[3] = {R(0), R(0), R(0)}, hout_d[3] = {R(0), R(0), R(0)};
    for (int s = 0; s < nsteps; ++s) {
        const int b = s & 1;
        const int ku = k0 + s;
        const int kuw = ku >= nz ? ku - nz : ku;
        R ov[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) ov[c] = own_value(c);
        if (out_ok && ku < kend) {
            const int idx = (kuw * plane + own);
            if constexpr (FUSED) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    hnew[c][idx] = ov[c];
                    if constexpr (WPAY) a.w[c][idx] = fma(-lam, rh[c], fma(-lamp, rp[c], rw[c]));
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            SN[b][c][oslot] = ov[c];
            if (has_halo) SN[b][c][hslot] = halo_value(c);
        }
        __syncthreads();
        if (s > 1 && out_ok) emit(b ^ 1, mine_d, hout_d, k0 - 2 + s);
        R up[3][4];
        read_face(b, up);
        fetch(min(ku + 1, kend));  // the last step re-reads plane kend (unused)

        R FL[3][4], FU[3][4];
        element_force_faces(Cu, lo, up, FL, FU);
        // The coefficients are dead: start loading the next layer's, and the
        // phase id of the layer after it (unconditional, with clamped
        // indices, so that the compiler cannot merge them into the guarded
        // prefetch and keep two copies of Cu live through the contraction).
        __builtin_amdgcn_sched_barrier(0);
        load_coef(coef, p_next, Cu);
        p_next = layer_phase(min(k0 + s + 1, kend - 1));

        R mine[3] = {R(0), R(0), R(0)};
        if (s > 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                R F[4], v[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) F[q] = carry[c][q] + FL[c][q];
                face_adj(F, v);
                SF[b][0][c][tid] = v[0];
                SF[b][1][c][tid] = v[1];
                SF[b][2][c][tid] = v[2];
                mine[c] = v[3];
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                carry[c][q] = FU[c][q];
                lo[c][q] = up[c][q];
            }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            mine_d[c] = mine[c];
            hout_d[c] = hprev[c];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) hprev[c] = ov[c];
    }
    __syncthreads();
    if (nsteps > 1 && out_ok) emit((nsteps - 1) & 1, mine_d, hout_d, k0 - 2 + nsteps);
    if (FUSED || a.want_norm) {
        double v[1] = {dot};
        block_partials<1, NT>(v, a.partials + (size_t)rhs * ntb, ntb, lb);
    }
}

// One operator-sweep workgroup; a fused sweep pays w's owed steps when its
// RHS owes two (the same decision for the whole workgroup).
template <int TX, int TY, int MODE, typename T>
__device__ __forceinline__ void op_dispatch(const OpArgs<T>& a, const int lbr, const int nblocks)
{
    __shared__ OpShared<TX, TY, OpReal<MODE, T>> sh;
    if constexpr (MODE == OP_FUSED) {
        const int ntb = nblocks / a.nrhs;
        if (a.S[lbr / ntb].pending == 2)
            op_body<TX, TY, MODE, T, true>(a, lbr, nblocks, sh);
        else
            op_body<TX, TY, MODE, T, false>(a, lbr, nblocks, sh);
    } else {
        op_body<TX, TY, MODE, T, false>(a, lbr, nblocks, sh);
    }
}

template <int TX, int TY, int MODE, typename T>
__global__ void __launch_bounds__(TX* TY, E3D_OP_MIN_WAVES) op_kernel(OpArgs<T> a)
{
    op_dispatch<TX, TY, MODE, T>(a, xcd_local_block(), gridDim.x);
}

// ----------------------------------------- wave-specialised fused sweep

// The fused sweep above issues every load and store of a plane step from
// the lanes that also compute, and a wavefront's vector-memory counter
// retires in issue order: the coefficients a step needs wait behind the
// stores and loads issued before them, so each step pays a memory latency.
// Here the workgroup is split:
//   - NL loader wavefronts copy the coming node planes of z and h_old, and
//     the phase ranks of the element layers, from HBM into a ring of D
//     planes in LDS with 16-byte direct-to-LDS loads, D - 1 planes ahead (no
//     register holds the data in flight); before the first plane they copy
//     the stiffness rows of the workgroup's phase dictionary (WsTables) into
//     LDS, where they stay for the whole workgroup;
//   - the TX x TY compute lanes read a plane's corner values and their
//     element's phase rank from the ring and its coefficients from the
//     dictionary rows, form h_new = z + gamma h_old there, and only store:
//     they issue no global load inside the z march, so no step waits for
//     memory.
// The paying form (w owes two steps) and the light form are separate
// kernels, each with its own register allocation; the launch starts both and
// the one that does not match the run's state returns at once.
//
// Ring layout of one plane slot: fields f = z0 z1 z2 h0 h1 h2, patch rows
// y = 0 .. TY (node row j0 - 1 + y), each row NCH 16-byte chunks from the
// chunk-aligned node xa <= i0 - 1 (chunks never straddle the periodic wrap,
// as nx is a multiple of the chunk): chunk q = (f * LY + y) * NCH + c; then,
// from a fresh 64-chunk block, the phase ranks of element layer k0 - 1 + u
// (TY rows of TX bytes, element i0 - 1 + x at byte x); in the paying form,
// from the next fresh block, w and the older direction on the owned node
// rows.  A loader instruction moves chunks [64 j, 64 j + 64).
//
// In-plane force exchange: a wavefront is one row of TX = 64 lanes, so the
// part a lane owes its x neighbour is passed by a lane shuffle; the part for
// the row below (v1 of this lane plus v0 of its x neighbour, summed) goes
// through LDS.
template <int TX, int TY, int NL, int D, typename T, bool WPAY, int MODE>
struct WsCfg {
    static constexpr int CH = 16 / (int)sizeof(T);  // elements per chunk
    static constexpr int NCH = TX / CH + 1;         // chunks per patch row
    static constexpr int LY = TY + 1;               // patch rows
    // OP_FUSED: z (3 components) and h_old (3); OP_APPLY and OP_REFINE: x (3)
    static constexpr bool APPLY = MODE != OP_FUSED;
    static constexpr int NF = APPLY ? 3 : 6;
    static constexpr int QN = NF * LY * NCH;        // node chunks per plane
    static constexpr int NIN = (QN + 63) / 64;      // loader instructions of node chunks
    static constexpr int LAYER = TX * TY;           // bytes of a layer of phase ranks
    static constexpr int QP = LAYER / 16;           // its chunks
    static constexpr int NIP = 1;
    // paying form: w and the older direction (3 components each), or the
    // added vector in APPLY, on the owned node rows j0 .. j0 + TY - 2, from
    // the chunk-aligned node <= i0
    static constexpr int QW = WPAY ? NF * (TY - 1) * NCH : 0;
    static constexpr int NIW = (QW + 63) / 64;
    static constexpr int NT = TX * TY;              // compute lanes
    static constexpr int NTOT = NT + 64 * NL;
    static constexpr int NLOAD = NL;                // loader wavefronts
    static constexpr int NI = ((NIN + NIP + NIW) + NL - 1) / NL * NL;  // loader instructions per plane
    static constexpr int PER_W = NI / NL;           // per loader wavefront
    static constexpr int SLOT = NI * 64 * 16;       // ring bytes per plane
    static constexpr int PH_OFF = NIN * 64 * 16;    // byte offset of the phase ranks in a slot
    static constexpr int W_OFF = (NIN + NIP) * 64 * 16;  // byte offset of w / the older direction
    // dictionary rows: kCoefStride elements each, in 16-byte chunks
    // dictionary rows in LDS: RS elements apart (FP64 22, FP32 28), so that
    // the 16-byte reads of lanes on rows of different phases fall on
    // different banks unless the rows' ranks differ by a multiple of 8.  CHR
    // 16-byte chunks per LDS row, copied from the first of the CHG chunks of
    // a table row (kCoefStride elements); an LDS row longer than the table's
    // (FP32) repeats its last chunk as padding
    static constexpr int RS = sizeof(T) == 8 ? 22 : 28;
    static constexpr int CHR = RS * (int)sizeof(T) / 16;
    static constexpr int CHG = kCoefStride * (int)sizeof(T) / 16;
    static constexpr int NCI = (kWsDict * CHR + 63) / 64;  // loader instructions of the rows
    static constexpr int CCB = NCI * 1024;                 // their bytes in LDS
    static_assert(TX == 64, "one wavefront per row of the tile");
    static_assert(NT % 64 == 0, "whole wavefronts");
    static_assert(LAYER % 16 == 0 && QP <= 64, "a layer of ranks in one instruction");
    static_assert(kCoefStride * sizeof(T) % 16 == 0 && RS * sizeof(T) % 16 == 0 && RS >= 21,
                  "rows of whole 16-byte chunks holding the 21 coefficients");
    static_assert(kWsDict <= 256, "ranks are bytes");
    static_assert(NL >= 1 && D >= 3, "loader wavefronts and a ring of at least three planes");
    // vmcnt that lets D - 2 planes of a loader wavefront stay in flight
    static constexpr int WAIT = (D - 2) * PER_W > 63 ? 63 : (D - 2) * PER_W;
    static constexpr int WAIT0 = (D - 1) * PER_W > 63 ? 63 : (D - 1) * PER_W;
};

template <int TX, int TY, int NL, int D, typename T, bool WPAY, int MODE>
struct OpSharedWS {
    using C = WsCfg<TX, TY, NL, D, T, WPAY, MODE>;
    alignas(16) char ring[D][C::SLOT];
    T sf[2][3][C::NT];
    alignas(16) char cc[C::CCB];  // the dictionary's stiffness rows, C::RS elements apart
};

// s_waitcnt on the vector-memory counter only (gfx9 encoding: vmcnt in bits
// 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at their maxima).
template <int N>
__device__ __forceinline__ void wait_vmcnt()
{
    static_assert(N >= 0 && N <= 63, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Stores of the compute wavefronts go through buffer descriptors of one
// plane of a field: a lane with nothing to store passes an offset past the
// descriptor's range, and the hardware drops its write.  Every step then
// issues the same stores on every path, so the memory counter a later wait
// names is exact instead of the smallest count over the paths.
constexpr int kDropOffset = 0x40000000;  // beyond every plane (under 2^27 voxels)
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(T* field, size_t first, int count)
{
    const unsigned long long p = reinterpret_cast<unsigned long long>(field + first);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)p);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(p >> 32));
    T* q = reinterpret_cast<T*>(((unsigned long long)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(q, 0, count * (int)sizeof(T), 0x00020000);
}
typedef unsigned int e3d_u2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void plane_store(double v, __amdgpu_buffer_rsrc_t r, int byte_off)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(e3d_u2, v), r, byte_off, 0, 0);
}
__device__ __forceinline__ void plane_store(float v, __amdgpu_buffer_rsrc_t r, int byte_off)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, byte_off, 0, 0);
}

// Value of the next lane (lane + 1) of the wavefront, through a DPP
// wavefront shift by one lane (a VALU move, no LDS round trip like a lane
// permute); lane 63 gets 0.
__device__ __forceinline__ float next_lane(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ double next_lane(double v)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)u, 0x130, 0xF, 0xF, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), 0x130, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Copy duties of one loader wavefront in the wave-specialised sweep: the
// source of each of its PER_W direct-to-LDS instructions of a ring slot
// (instruction j = cw + NL i of the slot layout above), the plane and layer
// offsets of slot u, and the dictionary rows.  Field bases are held as plain values: a
// select among the argument struct's members would take its address and
// move it to scratch memory.
template <class C, typename T>
struct WsCopier {
    const char* src[C::PER_W];
    const int32_t* dict;
    const T* coef;
    const uint8_t* rmap;
    int cw, lane, k0, nsteps, nz;
    size_t plane;

    // nf: the node-plane fields (slot fields 0 .. NF - 1), of: the owned-row
    // fields of the paying form / the added vector (0 .. NF - 1)
    __device__ __forceinline__ void init(const OpArgs<T>& a, const T* const (&nf)[6], const T* const (&of)[6],
                                         int lb, int cw_, int lane_, int xa, int xw, int j0, int k0_, int nsteps_)
    {
        constexpr int LY = C::LY, NCH = C::NCH, CH = C::CH, TY = C::NT / 64;
        const int nx = a.d.nx, ny = a.d.ny;
        const T *n0 = nf[0], *n1 = nf[1], *n2 = nf[2], *n3 = nf[3], *n4 = nf[4], *n5 = nf[5];
        const T *o0 = of[0], *o1 = of[1], *o2 = of[2], *o3 = of[3], *o4 = of[4], *o5 = of[5];
        auto pick = [](int f, const T* p0, const T* p1, const T* p2, const T* p3, const T* p4, const T* p5) {
            return f == 0 ? p0 : f == 1 ? p1 : f == 2 ? p2 : f == 3 ? p3 : f == 4 ? p4 : p5;
        };
        cw = cw_;
        lane = lane_;
        k0 = k0_;
        nsteps = nsteps_;
        nz = a.d.nz;
        plane = (size_t)nx * ny;
        dict = a.wsdict + (size_t)lb * kWsDict;
        coef = a.coef;
        rmap = a.wsmap + (size_t)lb * ((size_t)(a.kz + 2) * C::LAYER);
#pragma unroll
        for (int i = 0; i < C::PER_W; ++i) {
            const int j = cw + C::NLOAD * i;
            if (j < C::NIN) {
                const int q = 64 * j + lane;
                const int qq = q < C::QN ? q : 0;  // padding lanes copy chunk 0 into the block's tail
                const int f = qq / (LY * NCH), rem = qq - f * (LY * NCH);
                const int y = rem / NCH, c = rem - y * NCH;
                const int gx = ((xa + c * CH) % nx + nx) % nx;
                const int gy = ((j0 - 1 + y) % ny + ny) % ny;
                src[i] = reinterpret_cast<const char*>(pick(f, n0, n1, n2, n3, n4, n5) + (gx + (size_t)nx * gy));
            } else if (j < C::NIN + C::NIP) {
                src[i] = reinterpret_cast<const char*>(rmap + 16 * (lane < C::QP ? lane : 0));
            } else if (j < C::NIN + C::NIP + C::NIW) {
                // owned-row fields (in the fused sweep w and the older
                // direction, the buffer it overwrites: read here before the
                // owner lane writes it)
                const int q = 64 * (j - C::NIN - C::NIP) + lane;
                const int qq = q < C::QW ? q : 0;
                const int f = qq / ((TY - 1) * NCH), rem = qq - f * ((TY - 1) * NCH);
                const int y = rem / NCH, c = rem - y * NCH;
                const int gx = ((xw + c * CH) % nx + nx) % nx;
                const int gy = (j0 + y) % ny;
                src[i] = reinterpret_cast<const char*>(pick(f, o0, o1, o2, o3, o4, o5) + (gx + (size_t)nx * gy));
            } else {
                // padding instruction: the first chunk of field 0's plane (it
                // takes the node-plane offset, in bounds of a T field only)
                src[i] = reinterpret_cast<const char*>(n0);
            }
        }
    }
    // node plane and element layer k0 - 1 + u into the ring slot at dst
    __device__ __forceinline__ void issue(char* dst, int u) const
    {
        const int uc = min(u, nsteps);
        int kw = k0 - 1 + uc;
        kw = kw < 0 ? kw + nz : (kw >= nz ? kw - nz : kw);
        const size_t pn = (size_t)kw * plane * sizeof(T), pp = (size_t)uc * C::LAYER;
#pragma unroll
        for (int i = 0; i < C::PER_W; ++i) {
            const int j = cw + C::NLOAD * i;
            __builtin_amdgcn_global_load_lds((const void*)(src[i] + (j < C::NIN || j >= C::NIN + C::NIP ? pn : pp)),
                                             (void*)(dst + (size_t)j * 1024), 16, 0, 0);
        }
    }
    // this wavefront's share of the dictionary's stiffness rows
    __device__ __forceinline__ void issue_dict(char* ccb) const
    {
#pragma unroll
        for (int m = 0; m < (C::NCI + C::NLOAD - 1) / C::NLOAD; ++m) {
            const int i = cw + C::NLOAD * m;
            if (i < C::NCI) {
                // chunk g of the LDS rows; the tail of the last instruction
                // and the padding chunks of a row copy a chunk of the row
                const int g = 64 * i + lane;
                const int r = min(g / C::CHR, kWsDict - 1), q = min(g - r * C::CHR, C::CHG - 1);
                const T* row = coef + (size_t)dict[r] * kCoefStride + q * C::CH;
                __builtin_amdgcn_global_load_lds((const void*)row, (void*)(ccb + (size_t)i * 1024), 16, 0, 0);
            }
        }
    }
};

// MODE OP_FUSED: the direction + operator sweep (WPAY: the form that pays
// w's two owed steps).  MODE OP_APPLY (FP64): y = A x, plus the added vector
// when WPAY, with the optional ||y||^2 partials; one right-hand side.  MODE
// OP_REFINE: the same operator with the added vector, y stored in FP32 and
// ||y||^2 from the FP64 values (the refinement residual, once the FP32
// correction has been added to x).
template <int TX, int TY, int NL, int D, typename T, bool WPAY, int MODE>
__device__ __forceinline__ void op_body_ws(OpArgs<T> a, const int lbr, const int nblocks,
                                           OpSharedWS<TX, TY, NL, D, T, WPAY, MODE>& sh)
{
    using C = WsCfg<TX, TY, NL, D, T, WPAY, MODE>;
    using R = T;
    constexpr int NT = C::NT, LY = C::LY, NCH = C::NCH, CH = C::CH;
    constexpr bool FUSED = MODE == OP_FUSED;
    constexpr bool REFINE = MODE == OP_REFINE;
    static_assert(FUSED || ((MODE == OP_APPLY || (REFINE && WPAY)) && sizeof(T) == 8),
                  "the fused sweep, or the FP64 operator");

    int ntb = nblocks, rhs = 0, lb = lbr;
    R gam = R(0);
    const Scalars* S = nullptr;
    const T* nf[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    const T* of[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    T* hnew[3] = {nullptr, nullptr, nullptr};
    T* wdst[3] = {nullptr, nullptr, nullptr};
    T* ydst[3];
    float* yrdst[3];
    if constexpr (FUSED) {
        ntb = nblocks / a.nrhs;  // tile blocks per RHS
        rhs = lbr / ntb;
        lb = lbr - rhs * ntb;
        S = a.S + rhs;
        // the other form's kernel serves this sweep, or the run is over
        if (S->done || ((S->pending == 2) != WPAY)) return;
        gam = (R)S->gamma;
        const int cur = S->cur;
        const size_t roff = (size_t)rhs * a.rs;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            hnew[c] = (cur ? a.h0[c] : a.h1[c]) + roff;
            nf[c] = a.z[c] + roff;
            nf[c + 3] = (cur ? a.h1[c] : a.h0[c]) + roff;
            wdst[c] = a.w[c] + roff;
            of[c] = wdst[c];
            of[c + 3] = hnew[c];
            ydst[c] = a.y[c] + roff;
        }
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            nf[c] = reinterpret_cast<const T*>(a.x[c]);
            of[c] = reinterpret_cast<const T*>(a.add[c]);
            ydst[c] = reinterpret_cast<T*>(a.yd[c]);
            yrdst[c] = a.yr[c];
        }
    }

    const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz;
    const int plane = nx * ny;
    const int ntiles = a.tiles_x * a.tiles_y;
    const int bz = lb / ntiles, t = lb - bz * ntiles;
    const int by = t / a.tiles_x, bx = t - by * a.tiles_x;
    const int i0 = bx * (TX - 1), j0 = by * (TY - 1);
    const int k0 = bz * a.kz;
    const int kend = min(k0 + a.kz, nz);
    const int nsteps = kend - k0 + 1;
    // chunk-aligned start of the patch rows (xs = i0 - 1 may be -1)
    const int xs = i0 - 1;
    const int xa = (xs >= 0 ? xs / CH : -((-xs + CH - 1) / CH)) * CH;
    const int xw = (i0 / CH) * CH;  // owned nodes (paying form's w block)
    auto wrapk = [&](int kk) { return kk < 0 ? kk + nz : (kk >= nz ? kk - nz : kk); };
    const int tid = threadIdx.x;
    double dot = 0.0;

    const int lane = tid & 63;
    if (tid >= NT) {
        // ---------------------------------------------------------- loader
        WsCopier<C, T> cp;
        cp.init(a, nf, of, lb, (tid - NT) >> 6, lane, xa, xw, j0, k0, nsteps);
        cp.issue_dict(sh.cc);
#pragma unroll
        for (int u = 0; u < D; ++u) cp.issue(sh.ring[u % D], u);
        wait_vmcnt<C::WAIT0>();  // plane 0 landed
        __builtin_amdgcn_s_barrier();
        for (int s = 0; s < nsteps; ++s) {
            // slot (s - 1) % D was read before the last barrier: refill it
            if (s >= 1) cp.issue(sh.ring[(s - 1 + D) % D], s - 1 + D);
            wait_vmcnt<C::WAIT>();  // plane s + 1 landed
            __builtin_amdgcn_s_barrier();
        }
        wait_vmcnt<0>();  // no copy into LDS may outlive the workgroup
        __builtin_amdgcn_s_barrier();
    } else {
        // --------------------------------------------------------- compute
        R lam = R(0), lamp = R(0);
        if constexpr (FUSED) {
            lam = (R)S->lambda;
            lamp = (R)S->lambda_prev;
        }
        const int tx = tid % TX, ty = tid / TX;
        const int gi = i0 + tx, gj = j0 + ty;
        const int own = (gi % nx) + nx * (gj % ny);
        const bool out_ok = (tx < TX - 1) && (ty < TY - 1) && (gi < nx) && (gj < ny);
        // element offsets of the lane's four corners in a ring slot (field 0)
        // and of its element's phase id
        const int off0 = xs - xa;
        const int e00 = (ty * NCH) * CH + tx + off0, e10 = e00 + 1;
        const int e01 = ((ty + 1) * NCH) * CH + tx + off0, e11 = e01 + 1;
        const int eph = ty * TX + tx;
        // own node in the w block (rows of owned nodes only; lanes that own
        // none read a clamped slot and do not use it)
        const int ew = min(ty, TY - 2) * NCH * CH + min(tx, TX - 2) + (i0 - xw);
        constexpr int FSTRIDE = LY * NCH * CH;       // elements between fields
        constexpr int WSTRIDE = (TY - 1) * NCH * CH;  // between w-block fields
        // corner values of the plane in a ring slot as face spectra (fused:
        // h_new = z + gamma h_old; apply: x), the own node's value and, fused,
        // its h_old
        auto read_plane = [&](int slot, R (&F)[3][4], R (&ownv)[3], R (&ownh)[3]) {
            const R* rg = reinterpret_cast<const R*>(sh.ring[slot]);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const R* zf = rg + c * FSTRIDE;
                if constexpr (FUSED) {
                    const R* hf = rg + (c + 3) * FSTRIDE;
                    const R v00 = fma(gam, hf[e00], zf[e00]);
                    const R v10 = fma(gam, hf[e10], zf[e10]);
                    const R v01 = fma(gam, hf[e01], zf[e01]);
                    const R h11 = hf[e11];
                    const R v11 = fma(gam, h11, zf[e11]);
                    face_fwd(v00, v10, v01, v11, F[c]);
                    ownv[c] = v11;
                    ownh[c] = h11;
                } else {
                    const R v11 = zf[e11];
                    face_fwd(zf[e00], zf[e10], zf[e01], v11, F[c]);
                    ownv[c] = v11;
                    ownh[c] = R(0);
                }
            }
        };
        // phase rank of the lane's element in the layer of a ring slot, and
        // its coefficients from the dictionary rows
        auto slot_rank = [&](int slot) {
            return (int)reinterpret_cast<const uint8_t*>(sh.ring[slot] + C::PH_OFF)[eph];
        };
        auto read_coef = [&](int rank, R (&Cx)[21]) {
            const R* row = reinterpret_cast<const R*>(sh.cc) + rank * C::RS;
#pragma unroll
            for (int q = 0; q < 21; ++q) Cx[q] = row[q];
        };
        auto& SF = sh.sf;
        R lo[3][4], carry[3][4];
        __syncthreads();  // plane and layer k0 - 1 in slot 0, the dictionary rows in LDS
        // rank of the layer the next contraction computes (read a step ahead:
        // the loaders refill a slot during the step after the one that reads it)
        int rank = slot_rank(0);
        {
            R ov[3], oh[3];
            read_plane(0, lo, ov, oh);
        }
        // a step reads the next step's coefficients when it ends (the
        // dictionary rows never change), so a wavefront that reaches the
        // barrier early has them read while the others still compute
        R Cn[21];
        read_coef(rank, Cn);
        R hprev[3] = {R(0), R(0), R(0)};
        R mine_d[3] = {R(0), R(0), R(0)}, hout_d[3] = {R(0), R(0), R(0)};
        // one plane step; the loop below runs two per trip, so the values a
        // step hands to the next (lo, carry and the delayed outputs) change
        // registers between the two instead of being copied back every step
        auto step = [&](const int s) {
            const int b = s & 1;
            const int ku = k0 + s;
            __syncthreads();  // plane ku in slot (s + 1) % D; forces of step s - 1 in SF[b ^ 1]
            // Ah (A x, plus the added vector) of plane ku - 2
            const bool emit = s > 1 && out_ok;
            R yv[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                yv[c] = mine_d[c] + SF[b ^ 1][c][tid + TX];
                if constexpr (!FUSED) yv[c] += hout_d[c];  // the added vector
            }
            if (emit) {
                if constexpr (FUSED)
                    dot += (double)hout_d[0] * yv[0] + (double)hout_d[1] * yv[1] + (double)hout_d[2] * yv[2];
                else
                    dot += (double)yv[0] * yv[0] + (double)yv[1] * yv[1] + (double)yv[2] * yv[2];
            }
            {
                const size_t pk = (size_t)wrapk(ku - 2) * plane;
                if constexpr (REFINE) {
                    const int off = emit ? own * (int)sizeof(float) : kDropOffset;
#pragma unroll
                    for (int c = 0; c < 3; ++c) plane_store((float)yv[c], plane_rsrc(yrdst[c], pk, plane), off);
                } else {
                    const int off = emit ? own * (int)sizeof(T) : kDropOffset;
#pragma unroll
                    for (int c = 0; c < 3; ++c) plane_store(yv[c], plane_rsrc(ydst[c], pk, plane), off);
                }
            }
            const int slot = (s + 1) % D;
            R Cu[21];
#pragma unroll
            for (int q = 0; q < 21; ++q) Cu[q] = Cn[q];
            rank = slot_rank(slot);
            R up[3][4], ov[3], oh[3];
            read_plane(slot, up, ov, oh);
            R FL[3][4], FU[3][4];
            element_force_faces(Cu, lo, up, FL, FU);
            R mine[3] = {R(0), R(0), R(0)};
            if (s > 0) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    R F[4], v[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) F[q] = carry[c][q] + FL[c][q];
                    face_adj(F, v);
                    // own node: v3 + the x neighbour's v2; row below: v1 + the x neighbour's v0
                    mine[c] = v[3] + next_lane(v[2]);
                    SF[b][c][tid] = v[1] + next_lane(v[0]);
                }
            }
            const R* wb = reinterpret_cast<const R*>(sh.ring[slot] + C::W_OFF);
            if constexpr (FUSED) {
                // h_new (and w) of plane ku
                const size_t pk = (size_t)min(ku, nz - 1) * plane;
                const int off = (out_ok && ku < kend) ? own * (int)sizeof(T) : kDropOffset;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    plane_store(ov[c], plane_rsrc(hnew[c], pk, plane), off);
                    if constexpr (WPAY)
                        plane_store(fma(-lam, oh[c], fma(-lamp, wb[(c + 3) * WSTRIDE + ew], wb[c * WSTRIDE + ew])),
                                    plane_rsrc(wdst[c], pk, plane), off);
                }
            } else {
                // the added vector at the own node of plane ku, carried to its emit
#pragma unroll
                for (int c = 0; c < 3; ++c) ov[c] = WPAY ? wb[c * WSTRIDE + ew] : R(0);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    carry[c][q] = FU[c][q];
                    lo[c][q] = up[c][q];
                }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                mine_d[c] = mine[c];
                hout_d[c] = hprev[c];
                hprev[c] = ov[c];
            }
            read_coef(rank, Cn);
        };
        int s = 0;
        for (; s + 1 < nsteps; s += 2) {
            step(s);
            step(s + 1);
        }
        if (s < nsteps) step(s);
        __syncthreads();
        if (nsteps > 1 && out_ok) {
            const int b = (nsteps - 1) & 1;
            const int idx = wrapk(k0 - 2 + nsteps) * plane + own;
            R yv[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                yv[c] = mine_d[c] + SF[b][c][tid + TX];
                if constexpr (!FUSED) yv[c] += hout_d[c];
                if constexpr (REFINE)
                    yrdst[c][idx] = (float)yv[c];
                else
                    ydst[c][idx] = yv[c];
            }
            if constexpr (FUSED)
                dot += (double)hout_d[0] * yv[0] + (double)hout_d[1] * yv[1] + (double)hout_d[2] * yv[2];
            else
                dot += (double)yv[0] * yv[0] + (double)yv[1] * yv[1] + (double)yv[2] * yv[2];
        }
    }
    double v[1] = {dot};
    if (FUSED || a.want_norm) block_partials<1, C::NTOT>(v, a.partials + (size_t)rhs * ntb, ntb, lb);
}

template <int TX, int TY, int NL, int D, typename T, bool WPAY, int MODE>
__global__ void __launch_bounds__(TX* TY + 64 * NL, 1) op_kernel_ws(OpArgs<T> a)
{
    static_assert(sizeof(OpSharedWS<TX, TY, NL, D, T, WPAY, MODE>) + 64 * 8 <= 160 * 1024,
                  "ring, row exchange, dictionary and reduction within a CU's LDS");
    __shared__ OpSharedWS<TX, TY, NL, D, T, WPAY, MODE> sh;
    op_body_ws<TX, TY, NL, D, T, WPAY, MODE>(a, xcd_band_map(blockIdx.x, gridDim.x, kCusPerXcd), gridDim.x, sh);
}

// Copy of a work-list entry held in scalar registers: the entry is the same
// for the whole workgroup, and reading it word by word through readfirstlane
// keeps its pointers out of the vector registers of the sweep.
template <typename A>
__device__ __forceinline__ A load_uniform(const A* __restrict__ p)
{
    static_assert(sizeof(A) % 4 == 0, "work-list entries are whole words");
    A out;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(p);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(A) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
    return out;
}

// Index p of the work-list entry with first[p] <= b < first[p+1].  b is the
// same in every lane; so is the result, which is made explicit so that the
// entry's arguments load into scalar registers.
__device__ __forceinline__ int find_entry(const int* __restrict__ first, int n, int b)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// Up to kGroupPack problems of a group in one kernel argument: the
// arguments stay in the constant kernel-argument segment, which the compiler
// reads with scalar loads wherever a field is used, as for a single-problem
// sweep (the same entries read from a global-memory list end up in vector
// registers and halve the occupancy of the FP64 sweep).
constexpr int kGroupPack = 8;
template <typename T>
struct OpPack {
    OpArgs<T> m[kGroupPack];
    int first[kGroupPack + 1];
    int n;
};

// Fused sweep over a pack of independent problems: problem p owns the
// logical workgroups [first[p], first[p+1]) and runs exactly the workgroups
// its own sweep would.
template <int TX, int TY, typename T>
__global__ void __launch_bounds__(TX* TY, E3D_OP_MIN_WAVES) op_group_kernel(OpPack<T> pk)
{
    // each problem's workgroups are spread over all XCDs (contiguous tile
    // ranges per XCD within the problem), so problems of different sizes do
    // not load some XCDs more than others
    const int b = blockIdx.x;
    const int p = find_entry(pk.first, pk.n, b);
    const int nbp = pk.first[p + 1] - pk.first[p];
    op_dispatch<TX, TY, OP_FUSED, T>(pk.m[p], xcd_map(b - pk.first[p], nbp), nbp);
}

template <typename T>
struct UpdArgs {
    Dims d;
    FieldsT<T> f;
    size_t rs;
    int nrhs;
    MinvRows<T> M;
    const Scalars* S;
    double* partials;
};

// Update sweep over a group's work list: problem p owns workgroups
// [first[p], first[p+1]) and runs them as its own sweep would.
template <typename T>
__global__ void __launch_bounds__(kBlock) update_group_kernel(const UpdArgs<T>* __restrict__ list,
                                                              const int* __restrict__ first, int n)
{
    const int b = blockIdx.x;
    const int p = find_entry(first, n, b);
    const int nb = first[p + 1] - first[p];
    const UpdArgs<T> u = load_uniform(list + p);
    update_body<T, false>(u.d, u.f, u.rs, u.nrhs, u.M, u.S, u.partials, nb, b - first[p], nb);
}

#ifndef E3D_OP_TARGET_BLOCKS
#define E3D_OP_TARGET_BLOCKS 4096
#endif
constexpr int kTX = kTileShapes[0].tx, kTY = kTileShapes[0].ty;

// Ring depth of the wave-specialised sweep: the shape's d planes in FP64,
// two more for the FP32 sweep (half the bytes per plane); one less for the
// paying form, whose planes also carry w and the older direction, and one
// less again for the 8-row shape, whose paying ring of 5 would not fit the
// LDS (op_kernel_ws checks the total).
template <typename T, bool WPAY>
constexpr int ws_depth(int t)
{
    return kTileShapes[t].d + (sizeof(T) == 4 ? 2 : 0) - (WPAY ? (kTileShapes[t].ty > 6 ? 2 : 1) : 0);
}

// Launch of the operator sweep with the workgroup shape of g.tile (the
// wave-specialised shapes exist for the fused sweep only).
template <int MODE, typename T>
hipError_t launch_op_tiled(hipStream_t st, const OpGeom& g, unsigned grid, const OpArgs<T>& a)
{
#define E3D_OP_CASE(I)                                                                        \
    case I:                                                                                   \
        hipLaunchKernelGGL((op_kernel<kTileShapes[I].tx, kTileShapes[I].ty, MODE, T>), dim3(grid), \
                           dim3(kTileShapes[I].tx * kTileShapes[I].ty), 0, st, a);             \
        break;
#define E3D_WS_CASE(I)                                                                        \
    case I:                                                                                   \
        if constexpr (MODE == OP_FUSED && ws_elem_ok(I, sizeof(T))) {                         \
            hipLaunchKernelGGL((op_kernel_ws<kTileShapes[I].tx, kTileShapes[I].ty, kTileShapes[I].nl, \
                                             ws_depth<T, false>(I), T, false, OP_FUSED>),      \
                               dim3(grid), dim3(tile_lanes(I)), 0, st, a);                    \
            hipLaunchKernelGGL((op_kernel_ws<kTileShapes[I].tx, kTileShapes[I].ty, kTileShapes[I].nl, \
                                             ws_depth<T, true>(I), T, true, OP_FUSED>),        \
                               dim3(grid), dim3(tile_lanes(I)), 0, st, a);                    \
        } else {                                                                              \
            return hipErrorInvalidValue;                                                      \
        }                                                                                     \
        break;
    static_assert(kNumTiles == 7, "a launch case per shape");
    switch (g.tile) {
        E3D_OP_CASE(0)
        E3D_OP_CASE(1)
        E3D_OP_CASE(2)
        E3D_OP_CASE(3)
        E3D_OP_CASE(4)
        E3D_WS_CASE(5)
        E3D_WS_CASE(6)
        default:
            return hipErrorInvalidValue;
    }
#undef E3D_OP_CASE
#undef E3D_WS_CASE
    return hipGetLastError();
}

// ------------------------------------------------------------ post-process

struct Strain6 {
    double e[6];  // tensor components E11 E22 E33 E23 E13 E12
};

struct Sig6 {
    double* s[6];
};

// Centroid stress C_p (E_hat + B(1/2) w_e) per voxel, which is the voxel
// average of the trilinear field, and the element energy
// 1/2 (u^E + w)_e^T K_e (u^E + w)_e (Eq. discrete_energy).
// Centroid stress sg of voxel e and, with ENERGY, its element energy en.
template <bool ENERGY>
__device__ __forceinline__ void voxel_stress(const Dims& d, const int32_t* __restrict__ phase,
                                             const double* __restrict__ coef, const Strain6& E,
                                             const Fields& f, int e, double (&sg)[6], double& en)
{
    const double Et[3][3] = {{E.e[0], E.e[5], E.e[4]}, {E.e[5], E.e[1], E.e[3]}, {E.e[4], E.e[3], E.e[2]}};
    {
        int i, j, k;
        node_ijk(e, d, i, j, k);
        const int i1 = i + 1 == d.nx ? 0 : i + 1;
        const int j1 = j + 1 == d.ny ? 0 : j + 1;
        const int k1 = k + 1 == d.nz ? 0 : k + 1;
        const int xs[2] = {i, i1}, ys[2] = {j, j1}, zs[2] = {k, k1};
        double u[3][8], ut_[3][8];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int m = xs[a & 1] + d.nx * (ys[(a >> 1) & 1] + d.ny * zs[a >> 2]);
            const double xi[3] = {(double)(a & 1), (double)((a >> 1) & 1), (double)(a >> 2)};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double wv = f.w[c][m];
                u[c][a] = wv;
                ut_[c][a] = wv + Et[c][0] * xi[0] + Et[c][1] * xi[1] + Et[c][2] * xi[2];
            }
        }
        fwd8(u[0]);
        fwd8(u[1]);
        fwd8(u[2]);
        // centroid strain: gradient coefficients are (transform X/Y/Z slots)/4
        double eps[6] = {E.e[0] + 0.25 * u[0][MX],
                         E.e[1] + 0.25 * u[1][MY],
                         E.e[2] + 0.25 * u[2][MZ],
                         2.0 * E.e[3] + 0.25 * (u[1][MZ] + u[2][MY]),
                         2.0 * E.e[4] + 0.25 * (u[0][MZ] + u[2][MX]),
                         2.0 * E.e[5] + 0.25 * (u[0][MY] + u[1][MX])};
        double Cu[21];
        load_coef(coef, phase[e], Cu);  // C/16
        constexpr int sup[6] = {0, 1, 2, 3, 4, 5};
        contract<6>(Cu, sup, eps, sg);
#pragma unroll
        for (int r = 0; r < 6; ++r) sg[r] *= 16.0;
        en = 0.0;
        if constexpr (ENERGY) {
            double ff[3][8];
            double keep[3][8];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int a = 0; a < 8; ++a) keep[c][a] = ut_[c][a];
            element_force(Cu, ut_, ff);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int a = 0; a < 8; ++a) en += keep[c][a] * ff[c][a];
        }
    }
}

__global__ void __launch_bounds__(kBlock) stress_kernel(Dims d, const int32_t* __restrict__ phase,
                                                        const double* __restrict__ coef, Strain6 E,
                                                        Fields f, Sig6 out, int store,
                                                        double* partials, int stride)
{
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int e = blockIdx.x * kBlock + threadIdx.x; e < d.n; e += gridDim.x * kBlock) {
        double sg[6], en;
        voxel_stress<true>(d, phase, coef, E, f, e, sg, en);
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            if (store) out.s[r][e] = sg[r];
            acc[r] += sg[r];
        }
        acc[6] += 0.5 * en;
    }
    block_partials<7, kBlock>(acc, partials, stride, blockIdx.x);
}

// (value, index) pair order of the von Mises maximum: larger value, then
// lower index.
__device__ __forceinline__ bool vm_better(double v, double i, double bv, double bi)
{
    return v > bv || (v == bv && i < bi);
}

// Von Mises stress of every voxel (optional store) and the block's largest
// value with its lowest voxel index: partials[b] (value), partials[stride+b]
// (index, exact in a double).
__global__ void __launch_bounds__(kBlock) von_mises_kernel(Dims d, const int32_t* __restrict__ phase,
                                                           const double* __restrict__ coef, Strain6 E,
                                                           Fields f, double* vm, double* partials,
                                                           int stride)
{
    double best = -1.0, bidx = 0.0;
    for (int e = blockIdx.x * kBlock + threadIdx.x; e < d.n; e += gridDim.x * kBlock) {
        double sg[6], en;
        voxel_stress<false>(d, phase, coef, E, f, e, sg, en);
        const double a = sg[0] - sg[1], b = sg[1] - sg[2], c = sg[2] - sg[0];
        const double v = sqrt(0.5 * (a * a + b * b + c * c) + 3.0 * (sg[3] * sg[3] + sg[4] * sg[4] + sg[5] * sg[5]));
        if (vm) vm[e] = v;
        if (vm_better(v, (double)e, best, bidx)) {
            best = v;
            bidx = (double)e;
        }
    }
    __shared__ double rv[kBlock / 64], ri[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(best, off), oi = __shfl_xor(bidx, off);
        if (vm_better(ov, oi, best, bidx)) {
            best = ov;
            bidx = oi;
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        rv[wid] = best;
        ri[wid] = bidx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double bv = rv[0], bi = ri[0];
        for (int w = 1; w < kBlock / 64; ++w)
            if (vm_better(rv[w], ri[w], bv, bi)) {
                bv = rv[w];
                bi = ri[w];
            }
        partials[blockIdx.x] = bv;
        partials[stride + blockIdx.x] = bi;
    }
}

__global__ void __launch_bounds__(kFinThreads) von_mises_finalize(const double* partials, int stride,
                                                                  int nblocks, double* out2)
{
    __shared__ double rv[kFinThreads / 64], ri[kFinThreads / 64];
    double best = -1.0, bidx = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kFinThreads)
        if (vm_better(partials[b], partials[stride + b], best, bidx)) {
            best = partials[b];
            bidx = partials[stride + b];
        }
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(best, off), oi = __shfl_xor(bidx, off);
        if (vm_better(ov, oi, best, bidx)) {
            best = ov;
            bidx = oi;
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        rv[wid] = best;
        ri[wid] = bidx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double bv = rv[0], bi = ri[0];
        for (int w = 1; w < kFinThreads / 64; ++w)
            if (vm_better(rv[w], ri[w], bv, bi)) {
                bv = rv[w];
                bi = ri[w];
            }
        out2[0] = bv;
        out2[1] = bi;
    }
}

// u = E.X + w with X = (i, j, k) of the node.
__global__ void __launch_bounds__(kBlock) total_displacement_kernel(Dims d, Strain6 E, Fields f,
                                                                    double* u0, double* u1,
                                                                    double* u2)
{
    for (int m = blockIdx.x * kBlock + threadIdx.x; m < d.n; m += gridDim.x * kBlock) {
        int i, j, k;
        node_ijk(m, d, i, j, k);
        const double X = i, Y = j, Z = k;
        const int mv = m;
        u0[m] = f.w[0][mv] + E.e[0] * X + E.e[5] * Y + E.e[4] * Z;
        u1[m] = f.w[1][mv] + E.e[5] * X + E.e[1] * Y + E.e[3] * Z;
        u2[m] = f.w[2][mv] + E.e[4] * X + E.e[3] * Y + E.e[2] * Z;
    }
}

// Counts phase ids outside [0, nphase) (validation of device-resident input).
__global__ void __launch_bounds__(kBlock) phase_check_kernel(const int32_t* __restrict__ phase, int n,
                                                             int nphase, int* bad)
{
    int cnt = 0;
    for (int m = blockIdx.x * kBlock + threadIdx.x; m < n; m += gridDim.x * kBlock) {
        const int p = phase[m];
        cnt += (p < 0 || p >= nphase) ? 1 : 0;
    }
    if (cnt) atomicAdd(bad, cnt);
}

int sweep_blocks(int n, int max_blocks)
{
    long long b = ((long long)n + kBlock - 1) / kBlock;
    if (b > max_blocks) b = max_blocks;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace

// ------------------------------------------------ phase dictionaries
// One workgroup per box of the wave-specialised geometry (the element
// columns i0 - 1 .. i0 + TX - 2 and rows j0 - 1 .. j0 + TY - 2 of its tile,
// element layers k0 - 1 .. kend, all periodic): the distinct phase ids go
// into an LDS hash set, their ranks in ascending order become the box's
// dictionary, and each element of the box gets its rank as a byte.
constexpr int kWsHash = 1024;  // hash slots (well above kWsDict + one insertion per lane)
template <int TX, int TY>
__global__ void __launch_bounds__(256) ws_dict_kernel(Dims d, int tiles_x, int tiles_y, int kz,
                                                     const int32_t* __restrict__ phase, int32_t* __restrict__ dict,
                                                     uint8_t* __restrict__ map, int* maxcount)
{
    __shared__ int key[kWsHash];
    __shared__ int rank_of[kWsHash];
    __shared__ int count;
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int lb = blockIdx.x;
    const int ntiles = tiles_x * tiles_y;
    const int bz = lb / ntiles, t = lb - bz * ntiles;
    const int by = t / tiles_x, bx = t - by * tiles_x;
    const int i0 = bx * (TX - 1), j0 = by * (TY - 1), k0 = bz * kz;
    const int kend = min(k0 + kz, nz);
    const int layers = kend - k0 + 2;  // u = 0 .. nsteps
    const int nel = layers * TY * TX;
    const int tid = threadIdx.x;
    for (int h = tid; h < kWsHash; h += 256) key[h] = -1;
    if (tid == 0) count = 0;
    __syncthreads();
    auto element_phase = [&](int e) {
        const int u = e / (TY * TX), r = e - u * (TY * TX);
        const int y = r / TX, x = r - y * TX;
        const int gx = ((i0 - 1 + x) % nx + nx) % nx;
        const int gy = ((j0 - 1 + y) % ny + ny) % ny;
        int gz = k0 - 1 + u;
        gz = gz < 0 ? gz + nz : (gz >= nz ? gz - nz : gz);
        return phase[(size_t)gx + (size_t)nx * ((size_t)gy + (size_t)ny * gz)];
    };
    auto slot_of = [](int p) { return (int)(((unsigned)p * 2654435761u) >> 22); };  // 10 bits
    for (int e = tid; e < nel; e += 256) {
        if (*(volatile int*)&count > kWsDict) break;  // too many: stop early (the table never fills)
        const int p = element_phase(e);
        int h = slot_of(p);
        while (true) {
            const int old = atomicCAS(&key[h], -1, p);
            if (old == -1) {
                atomicAdd(&count, 1);
                break;
            }
            if (old == p) break;
            h = (h + 1) & (kWsHash - 1);
        }
    }
    __syncthreads();
    const int c = count;
    if (tid == 0) atomicMax(maxcount, c);
    if (c > kWsDict) return;
    // rank = number of smaller ids in the set
    int first = -1;
    for (int h = tid; h < kWsHash; h += 256) {
        const int k = key[h];
        if (k < 0) continue;
        int r = 0;
        for (int h2 = 0; h2 < kWsHash; ++h2) {
            const int k2 = key[h2];
            r += (k2 >= 0 && k2 < k);
        }
        rank_of[h] = r;
        dict[(size_t)lb * kWsDict + r] = k;
        if (r == 0) first = k;
    }
    // unused entries repeat rank 0 (a valid row to copy)
    __shared__ int first_id;
    if (first >= 0) first_id = first;
    __syncthreads();
    for (int r = c + tid; r < kWsDict; r += 256) dict[(size_t)lb * kWsDict + r] = first_id;
    uint8_t* out = map + (size_t)lb * ((size_t)(kz + 2) * TX * TY);
    for (int e = tid; e < nel; e += 256) {
        const int p = element_phase(e);
        int h = slot_of(p);
        while (key[h] != p) h = (h + 1) & (kWsHash - 1);
        out[e] = (uint8_t)rank_of[h];
    }
}

hipError_t launch_ws_dictionary(hipStream_t st, const Dims& d, const OpGeom& g, const int32_t* phase,
                                int32_t* dict, uint8_t* map, int* maxcount)
{
    if (g.tile < 0 || g.tile >= kNumTiles || !is_ws(g.tile) || g.blocks <= 0) return hipErrorInvalidValue;
    static_assert(kNumTiles == 7 && kTileShapes[5].tx == 64 && kTileShapes[5].ty == 6 &&
                      kTileShapes[6].tx == 64 && kTileShapes[6].ty == 8,
                  "a dictionary kernel per wave-specialised shape");
    if (g.tile == 6)
        hipLaunchKernelGGL((ws_dict_kernel<64, 8>), dim3(g.blocks), dim3(256), 0, st, d, g.tiles_x, g.tiles_y,
                           g.kz, phase, dict, map, maxcount);
    else
        hipLaunchKernelGGL((ws_dict_kernel<64, 6>), dim3(g.blocks), dim3(256), 0, st, d, g.tiles_x, g.tiles_y,
                           g.kz, phase, dict, map, maxcount);
    return hipGetLastError();
}

// ------------------------------------------------------------- launchers

OpGeom op_geometry(const Dims& d, int kz_hint, int tile, int target_blocks)
{
    OpGeom g;
    g.tile = (tile >= 0 && tile < kNumTiles) ? tile : 0;
    const int tx = kTileShapes[g.tile].tx, ty = kTileShapes[g.tile].ty;
    g.tiles_x = (d.nx + tx - 2) / (tx - 1);
    g.tiles_y = (d.ny + ty - 2) / (ty - 1);
    const int ntiles = g.tiles_x * g.tiles_y;
    int kz = kz_hint;
    if (kz <= 0) {
        // enough workgroups to fill 256 CUs several times over
        const int target = target_blocks > 0 ? target_blocks : E3D_OP_TARGET_BLOCKS;
        int chunks = (target + ntiles - 1) / ntiles;
        if (chunks > d.nz) chunks = d.nz;
        kz = (d.nz + chunks - 1) / chunks;
        // Short chunks pay their extra lower plane and start-up on few
        // planes: on small grids lengthen them toward 16 planes while about
        // target/8 workgroups (one round on the chip at the default) remain.
        const long long fill = (long long)ntiles * d.nz / (target / 8 > 0 ? target / 8 : 1);
        const int kz_fill = (int)std::min<long long>(16, fill);
        if (kz < kz_fill) kz = kz_fill;
        if (kz < 4 && d.nz >= 4) kz = 4;
    }
    if (kz > d.nz) kz = d.nz;
    g.kz = kz;
    g.zchunks = (d.nz + kz - 1) / kz;
    g.blocks = ntiles * g.zchunks;
    return g;
}

hipError_t launch_load(hipStream_t st, const Dims& d, const int32_t* phase, const double* sig,
                       double* const b[3], double* partials, double* out2, int max_blocks)
{
    const int nb = sweep_blocks(d.n, max_blocks);
    hipLaunchKernelGGL(load_kernel, dim3(nb), dim3(kBlock), 0, st, d, phase, sig, b[0], b[1], b[2],
                       partials, nb);
    hipLaunchKernelGGL(finalize_kernel<2>, dim3(1), dim3(kFinThreads), 0, st, (int)FIN_STORE,
                       (const double*)partials, nb, nb, (Scalars*)nullptr, out2, (const double*)nullptr, 0);
    return hipGetLastError();
}

hipError_t launch_precond_count(hipStream_t st, const Dims& d, const int32_t* phase, int* counts)
{
    const int nb = (int)(((size_t)d.n + kPrecondChunk - 1) / kPrecondChunk);
    hipLaunchKernelGGL(precond_count_kernel, dim3(nb), dim3(kBlock), 0, st, d, phase, counts);
    return hipGetLastError();
}

hipError_t launch_precond_fill(hipStream_t st, const Dims& d, const int32_t* phase, const Tables& t,
                               int identity, int nphase, const int* offsets, uint32_t* idx,
                               double* const rows[6])
{
    const int nb = (int)(((size_t)d.n + kPrecondChunk - 1) / kPrecondChunk);
    hipLaunchKernelGGL(precond_fill_kernel, dim3(nb), dim3(kBlock), 0, st, d, phase, t.diag, t.solid,
                       identity, nphase, offsets, idx, rows[0], rows[1], rows[2], rows[3], rows[4],
                       rows[5]);
    return hipGetLastError();
}

hipError_t launch_precond_table(hipStream_t st, int nphase, const Tables& t, int identity,
                                double* const rows[6])
{
    const int nb = (nphase + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(precond_table_kernel, dim3(nb), dim3(kBlock), 0, st, nphase, t.diag, t.solid,
                       identity, rows[0], rows[1], rows[2], rows[3], rows[4], rows[5]);
    return hipGetLastError();
}

hipError_t launch_precond_expand(hipStream_t st, const Dims& d, const MinvRows<double>& M, double* out)
{
    const int nb = sweep_blocks(d.n, 8192);
    hipLaunchKernelGGL(precond_expand_kernel, dim3(nb), dim3(kBlock), 0, st, d, M, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pcg_init(hipStream_t st, const Dims& d, const FieldsT<T>& f, const MinvRows<T>& M,
                           int fresh, int from_residual, Scalars* S, double* partials,
                           int max_blocks, const double* norms2)
{
    const int nb = sweep_blocks(d.n, max_blocks);
    hipLaunchKernelGGL(pcg_init_kernel<T>, dim3(nb), dim3(kBlock), 0, st, d, f, M, fresh,
                       from_residual, partials, nb);
    hipLaunchKernelGGL(finalize_kernel<2>, dim3(1), dim3(kFinThreads), 0, st, (int)FIN_INIT,
                       (const double*)partials, nb, nb, S, (double*)nullptr, norms2, 0);
    return hipGetLastError();
}

// The fused sweep selects a direction buffer per lane by one element offset:
// h1 must lie the same distance (under 2^31 elements) from h0 in every
// component.
template <typename T>
static bool direction_buffers_ok(const FieldsT<T>& f)
{
    const ptrdiff_t dh = f.h1[0] - f.h0[0];
    if (dh <= -((ptrdiff_t)1 << 31) || dh >= ((ptrdiff_t)1 << 31)) return false;
    return f.h1[1] - f.h0[1] == dh && f.h1[2] - f.h0[2] == dh;
}

// The wave-specialised sweep copies 16-byte chunks of z and the direction
// buffers: rows a whole number of chunks, every field and RHS offset
// 16-byte aligned.
template <typename T>
static bool ws_fields_ok(const Dims& d, int tile, const FieldsT<T>& f, size_t rs)
{
    if (!is_ws(tile)) return true;
    if (!ws_supported(d, tile, (int)sizeof(T)) || (rs * sizeof(T)) % 16 != 0) return false;
    for (int c = 0; c < 3; ++c)
        if (((uintptr_t)f.z[c] | (uintptr_t)f.h0[c] | (uintptr_t)f.h1[c]) % 16 != 0) return false;
    return true;
}

template <typename T>
hipError_t launch_direction_operator(hipStream_t st, const Dims& d, const OpGeom& g,
                                     const int32_t* phase, const Tables& t, const FieldsT<T>& f,
                                     size_t rs, int nrhs, Scalars* S, double* partials, bool finalize)
{
    if (!direction_buffers_ok(f)) return hipErrorInvalidValue;
    if (g.tile < 0 || g.tile >= kNumTiles || !ws_fields_ok(d, g.tile, f, rs)) return hipErrorInvalidValue;
    if (is_ws(g.tile) &&
        (!t.ws.dict || !t.ws.map || t.ws.tile != g.tile || t.ws.tiles_x != g.tiles_x ||
         t.ws.tiles_y != g.tiles_y || t.ws.kz != g.kz))
        return hipErrorInvalidValue;  // no dictionaries built for this geometry
    OpArgs<T> a = {};
    a.wsdict = t.ws.dict;
    a.wsmap = t.ws.map;
    a.d = d;
    a.tiles_x = g.tiles_x;
    a.tiles_y = g.tiles_y;
    a.kz = g.kz;
    a.phase = phase;
    if constexpr (std::is_same<T, float>::value)
        a.coef = t.coef32;
    else
        a.coef = t.coef;
    for (int c = 0; c < 3; ++c) {
        a.z[c] = f.z[c];
        a.h0[c] = f.h0[c];
        a.h1[c] = f.h1[c];
        a.w[c] = f.w[c];
        a.y[c] = f.Ah[c];
    }
    a.S = S;
    a.partials = partials;
    a.rs = rs;
    a.nrhs = nrhs;
    hipError_t e = launch_op_tiled<OP_FUSED, T>(st, g, (unsigned)(g.blocks * nrhs), a);
    if (e != hipSuccess || !finalize) return e;
    hipLaunchKernelGGL(finalize_kernel<1>, dim3(nrhs), dim3(kFinThreads), 0, st, (int)FIN_DIRECTION,
                       (const double*)partials, g.blocks, g.blocks, S, (double*)nullptr,
                       (const double*)nullptr, g.blocks);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_update_precond(hipStream_t st, const Dims& d, const FieldsT<T>& f, size_t rs,
                                 int nrhs, const MinvRows<T>& M, Scalars* S, double* partials,
                                 int max_blocks, bool finalize, bool nontemporal)
{
    const int nb = sweep_blocks(d.n, max_blocks);
    if (nontemporal)
        hipLaunchKernelGGL((update_precond_kernel<T, true>), dim3(nb), dim3(kBlock), 0, st, d, f, rs, nrhs,
                           M, (const Scalars*)S, partials, nb);
    else
        hipLaunchKernelGGL((update_precond_kernel<T, false>), dim3(nb), dim3(kBlock), 0, st, d, f, rs, nrhs,
                           M, (const Scalars*)S, partials, nb);
    if (!finalize) return hipGetLastError();
    hipLaunchKernelGGL(finalize_kernel<2>, dim3(nrhs), dim3(kFinThreads), 0, st, (int)FIN_UPDATE,
                       (const double*)partials, nb, nb, S, (double*)nullptr, (const double*)nullptr,
                       2 * nb);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_final_update(hipStream_t st, const Dims& d, const FieldsT<T>& f, Scalars* S)
{
    const int nb = sweep_blocks(d.n, 4096);
    hipLaunchKernelGGL(final_update_kernel<T>, dim3(nb), dim3(kBlock), 0, st, d, f, (const Scalars*)S);
    return hipGetLastError();
}

// ------------------------------------------------------------------ groups

namespace {

template <typename T>
struct PlanLayout {
    size_t upd, updfirst, findir, finupd, bytes;
};

template <typename T>
PlanLayout<T> plan_layout(int n, int nfin)
{
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    PlanLayout<T> L;
    L.upd = 0;
    L.updfirst = up(L.upd + sizeof(UpdArgs<T>) * n);
    L.findir = up(L.updfirst + sizeof(int) * (n + 1));
    L.finupd = up(L.findir + sizeof(FinItem) * nfin);
    L.bytes = up(L.finupd + sizeof(FinItem) * nfin);
    return L;
}

}  // namespace

template <typename T>
size_t group_plan_bytes(int n, int nfin)
{
    return plan_layout<T>(n, nfin).bytes;
}

template <typename T>
hipError_t group_prepare(hipStream_t st, const GroupMember<T>* m, int n, char* staging, char* dev,
                         GroupPlan* plan)
{
    int nfin = 0;
    for (int i = 0; i < n; ++i) nfin += m[i].nrhs;
    const PlanLayout<T> L = plan_layout<T>(n, nfin);
    const int npacks = (n + kGroupPack - 1) / kGroupPack;
    plan->packs.assign(sizeof(OpPack<T>) * npacks, 0);
    plan->pack_blocks.assign(npacks, 0);
    OpPack<T>* packs = reinterpret_cast<OpPack<T>*>(plan->packs.data());
    UpdArgs<T>* up = reinterpret_cast<UpdArgs<T>*>(staging + L.upd);
    int* updfirst = reinterpret_cast<int*>(staging + L.updfirst);
    FinItem* fd = reinterpret_cast<FinItem*>(staging + L.findir);
    FinItem* fu = reinterpret_cast<FinItem*>(staging + L.finupd);
    long long ub = 0;
    int k = 0;
    for (int i = 0; i < n; ++i) {
        const GroupMember<T>& g = m[i];
        if (g.g.tile != 0) return hipErrorInvalidValue;  // groups run workgroup shape 0
        if (!direction_buffers_ok(g.f)) return hipErrorInvalidValue;
        OpArgs<T> a = {};
        a.d = g.d;
        a.tiles_x = g.g.tiles_x;
        a.tiles_y = g.g.tiles_y;
        a.kz = g.g.kz;
        a.phase = g.phase;
        if constexpr (std::is_same<T, float>::value)
            a.coef = g.t.coef32;
        else
            a.coef = g.t.coef;
        for (int c = 0; c < 3; ++c) {
            a.z[c] = g.f.z[c];
            a.h0[c] = g.f.h0[c];
            a.h1[c] = g.f.h1[c];
            a.w[c] = g.f.w[c];
            a.y[c] = g.f.Ah[c];
        }
        a.S = g.S;
        a.partials = g.partials;
        a.rs = g.rs;
        a.nrhs = g.nrhs;
        OpPack<T>& pk = packs[i / kGroupPack];
        const int j = i % kGroupPack;
        pk.m[j] = a;
        pk.first[j] = (int)plan->pack_blocks[i / kGroupPack];
        const long long ob = (long long)pk.first[j] + (long long)g.g.blocks * g.nrhs;
        if (ob >= (1LL << 31)) return hipErrorInvalidValue;
        pk.first[j + 1] = (int)ob;
        pk.n = j + 1;
        plan->pack_blocks[i / kGroupPack] = (int)ob;
        const int nb = sweep_blocks(g.d.n, g.upd_blocks);
        UpdArgs<T> u;
        u.d = g.d;
        u.f = g.f;
        u.rs = g.rs;
        u.nrhs = g.nrhs;
        u.M = g.minv;
        u.S = g.S;
        u.partials = g.partials;
        up[i] = u;
        updfirst[i] = (int)ub;
        ub += nb;
        for (int r = 0; r < g.nrhs; ++r, ++k) {
            fd[k] = FinItem{g.partials + (size_t)r * g.g.blocks, g.g.blocks, g.g.blocks, g.S + r};
            fu[k] = FinItem{g.partials + (size_t)r * 2 * nb, nb, nb, g.S + r};
        }
    }
    if (ub >= (1LL << 31)) return hipErrorInvalidValue;
    updfirst[n] = (int)ub;
    plan->dev = dev;
    plan->n = n;
    plan->nfin = nfin;
    plan->upd_blocks = (int)ub;
    plan->off_upd = L.upd;
    plan->off_updfirst = L.updfirst;
    plan->off_findir = L.findir;
    plan->off_finupd = L.finupd;
    return hipMemcpyAsync(dev, staging, L.bytes, hipMemcpyHostToDevice, st);
}

template <typename T>
hipError_t launch_group_iteration(hipStream_t st, const GroupPlan& p)
{
    if (p.n == 0) return hipSuccess;
    const OpPack<T>* packs = reinterpret_cast<const OpPack<T>*>(p.packs.data());
    for (size_t k = 0; k < p.pack_blocks.size(); ++k)
        hipLaunchKernelGGL((op_group_kernel<kTX, kTY, T>), dim3(p.pack_blocks[k]), dim3(kTX * kTY), 0, st,
                           packs[k]);
    hipLaunchKernelGGL(finalize_group_kernel<1>, dim3(p.nfin), dim3(kFinThreads), 0, st, (int)FIN_DIRECTION,
                       reinterpret_cast<const FinItem*>(p.dev + p.off_findir));
    hipLaunchKernelGGL(update_group_kernel<T>, dim3(p.upd_blocks), dim3(kBlock), 0, st,
                       reinterpret_cast<const UpdArgs<T>*>(p.dev + p.off_upd),
                       reinterpret_cast<const int*>(p.dev + p.off_updfirst), p.n);
    hipLaunchKernelGGL(finalize_group_kernel<2>, dim3(p.nfin), dim3(kFinThreads), 0, st, (int)FIN_UPDATE,
                       reinterpret_cast<const FinItem*>(p.dev + p.off_finupd));
    return hipGetLastError();
}

#define E3D_INSTANTIATE(T)                                                                          \
    template hipError_t launch_pcg_init<T>(hipStream_t, const Dims&, const FieldsT<T>&, const MinvRows<T>&, \
                                           int, int, Scalars*, double*, int, const double*);         \
    template hipError_t launch_direction_operator<T>(hipStream_t, const Dims&, const OpGeom&,         \
                                                     const int32_t*, const Tables&,                  \
                                                     const FieldsT<T>&, size_t, int, Scalars*,        \
                                                     double*, bool);                                 \
    template hipError_t launch_update_precond<T>(hipStream_t, const Dims&, const FieldsT<T>&, size_t, \
                                                 int, const MinvRows<T>&, Scalars*, double*, int, bool,     \
                                                 bool);                                                     \
    template hipError_t launch_final_update<T>(hipStream_t, const Dims&, const FieldsT<T>&, Scalars*);     \
    template size_t group_plan_bytes<T>(int, int);                                                   \
    template hipError_t group_prepare<T>(hipStream_t, const GroupMember<T>*, int, char*, char*,       \
                                         GroupPlan*);                                                \
    template hipError_t launch_group_iteration<T>(hipStream_t, const GroupPlan&);
E3D_INSTANTIATE(double)
E3D_INSTANTIATE(float)
#undef E3D_INSTANTIATE

hipError_t launch_apply(hipStream_t st, const Dims& d, const OpGeom& g, const int32_t* phase,
                        const Tables& t, const double* const x[3], double* const y[3],
                        const double* const add[3], double* partials, double* norm2)
{
    if (g.tile < 0 || g.tile >= kNumTiles) return hipErrorInvalidValue;
    if (is_ws(g.tile)) {
        // the wave-specialised operator: its dictionaries, rows of whole
        // 16-byte chunks and 16-byte aligned node vectors
        if (!t.ws.dict || !t.ws.map || t.ws.tile != g.tile || t.ws.tiles_x != g.tiles_x ||
            t.ws.tiles_y != g.tiles_y || t.ws.kz != g.kz || !ws_supported(d, g.tile, 8))
            return hipErrorInvalidValue;
        for (int c = 0; c < 3; ++c)
            if (((uintptr_t)x[c] | (add ? (uintptr_t)add[c] : 0)) % 16 != 0) return hipErrorInvalidValue;
    }
    OpArgs<double> a = {};
    a.d = d;
    a.tiles_x = g.tiles_x;
    a.tiles_y = g.tiles_y;
    a.kz = g.kz;
    a.phase = phase;
    a.coef = t.coef;
    for (int c = 0; c < 3; ++c) {
        a.x[c] = const_cast<double*>(x[c]);  // read only in this mode
        a.yd[c] = y[c];
        a.add[c] = add ? add[c] : nullptr;
    }
    a.partials = partials;
    a.want_norm = norm2 != nullptr;
    a.wsdict = t.ws.dict;
    a.wsmap = t.ws.map;
    a.nrhs = 1;
    if (is_ws(g.tile)) {
        static_assert(kNumTiles == 7 && is_ws(5) && ws_elem_ok(5, 8), "the FP64 wave-specialised shape");
        constexpr int TX = kTileShapes[5].tx, TY = kTileShapes[5].ty, NL = kTileShapes[5].nl,
                      DA = kTileShapes[5].d;  // the operator's ring carries x alone: one depth serves both forms
        if (add)
            hipLaunchKernelGGL((op_kernel_ws<TX, TY, NL, DA, double, true, OP_APPLY>), dim3(g.blocks),
                               dim3(tile_lanes(5)), 0, st, a);
        else
            hipLaunchKernelGGL((op_kernel_ws<TX, TY, NL, DA, double, false, OP_APPLY>), dim3(g.blocks),
                               dim3(tile_lanes(5)), 0, st, a);
    } else {
        hipError_t e = launch_op_tiled<OP_APPLY, double>(st, g, (unsigned)g.blocks, a);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (norm2)
        hipLaunchKernelGGL(finalize_kernel<1>, dim3(1), dim3(kFinThreads), 0, st, (int)FIN_STORE,
                           (const double*)partials, g.blocks, g.blocks, (Scalars*)nullptr, norm2,
                           (const double*)nullptr, 0);
    return hipGetLastError();
}

hipError_t launch_refine(hipStream_t st, const Dims& d, const OpGeom& g, const int32_t* phase,
                         const Tables& t, double* const w[3], const float* const dcorr[3],
                         const double* const b[3], float* const r[3], double* partials,
                         double* norm2)
{
    if (g.tile < 0 || g.tile >= kNumTiles) return hipErrorInvalidValue;
    const bool ws = is_ws(g.tile);
    if (ws) {
        if (!t.ws.dict || !t.ws.map || t.ws.tile != g.tile || t.ws.tiles_x != g.tiles_x ||
            t.ws.tiles_y != g.tiles_y || t.ws.kz != g.kz || !ws_supported(d, g.tile, 8))
            return hipErrorInvalidValue;
        for (int c = 0; c < 3; ++c)
            if (((uintptr_t)w[c] | (uintptr_t)b[c]) % 16 != 0) return hipErrorInvalidValue;
    }
    OpArgs<double> a = {};
    a.d = d;
    a.tiles_x = g.tiles_x;
    a.tiles_y = g.tiles_y;
    a.kz = g.kz;
    a.phase = phase;
    a.coef = t.coef;
    for (int c = 0; c < 3; ++c) {
        a.x[c] = w[c];
        a.xd[c] = dcorr[c];
        a.yr[c] = r[c];
        a.add[c] = b[c];
    }
    a.partials = partials;
    a.want_norm = 1;
    a.wsdict = t.ws.dict;
    a.wsmap = t.ws.map;
    a.nrhs = 1;
    const int nb = sweep_blocks(d.n, 4096);
    if (ws) {
        // w + d is formed once, in place, and the operator reads it: the
        // same FP64 sums as the classic sweep forms at every node it reads
        hipLaunchKernelGGL(add_correction_kernel, dim3(nb), dim3(kBlock), 0, st, d, w[0], w[1], w[2],
                           dcorr[0], dcorr[1], dcorr[2]);
        constexpr int TX = kTileShapes[5].tx, TY = kTileShapes[5].ty, NL = kTileShapes[5].nl,
                      DA = kTileShapes[5].d;
        hipLaunchKernelGGL((op_kernel_ws<TX, TY, NL, DA, double, true, OP_REFINE>), dim3(g.blocks),
                           dim3(tile_lanes(5)), 0, st, a);
    } else {
        hipError_t e = launch_op_tiled<OP_REFINE, double>(st, g, (unsigned)g.blocks, a);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finalize_kernel<1>, dim3(1), dim3(kFinThreads), 0, st, (int)FIN_STORE,
                       (const double*)partials, g.blocks, g.blocks, (Scalars*)nullptr, norm2,
                       (const double*)nullptr, 0);
    if (!ws)
        hipLaunchKernelGGL(add_correction_kernel, dim3(nb), dim3(kBlock), 0, st, d, w[0], w[1], w[2],
                           dcorr[0], dcorr[1], dcorr[2]);
    return hipGetLastError();
}

hipError_t launch_tuning_fill(hipStream_t st, double* p, size_t n)
{
    size_t nb = (n + kBlock - 1) / kBlock;
    if (nb > 8192) nb = 8192;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(tuning_fill_kernel, dim3((unsigned)nb), dim3(kBlock), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_to_float(hipStream_t st, const double* src, float* dst, size_t n)
{
    size_t nb = (n + kBlock - 1) / kBlock;
    if (nb > 8192) nb = 8192;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(to_float_kernel, dim3((unsigned)nb), dim3(kBlock), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_stress(hipStream_t st, const Dims& d, const int32_t* phase, const Tables& t,
                         const double* strain6, const Fields& f, double* const sig[6],
                         double* partials, double* sums7, int max_blocks)
{
    const int nb = sweep_blocks(d.n, max_blocks);
    Strain6 E;
    for (int q = 0; q < 6; ++q) E.e[q] = strain6[q];
    Sig6 o;
    for (int q = 0; q < 6; ++q) o.s[q] = sig ? sig[q] : nullptr;
    hipLaunchKernelGGL(stress_kernel, dim3(nb), dim3(kBlock), 0, st, d, phase, t.coef, E, f, o,
                       sig ? 1 : 0, partials, nb);
    hipLaunchKernelGGL(finalize_kernel<7>, dim3(1), dim3(kFinThreads), 0, st, (int)FIN_STORE,
                       (const double*)partials, nb, nb, (Scalars*)nullptr, sums7,
                       (const double*)nullptr, 0);
    return hipGetLastError();
}

hipError_t launch_von_mises(hipStream_t st, const Dims& d, const int32_t* phase, const Tables& t,
                           const double* strain6, const Fields& f, double* vm, double* partials,
                           double* out2, int max_blocks)
{
    const int nb = sweep_blocks(d.n, max_blocks);
    Strain6 E;
    for (int q = 0; q < 6; ++q) E.e[q] = strain6[q];
    hipLaunchKernelGGL(von_mises_kernel, dim3(nb), dim3(kBlock), 0, st, d, phase, t.coef, E, f, vm, partials,
                       nb);
    hipLaunchKernelGGL(von_mises_finalize, dim3(1), dim3(kFinThreads), 0, st, (const double*)partials, nb, nb,
                       out2);
    return hipGetLastError();
}

hipError_t launch_phase_check(hipStream_t st, const int32_t* phase, int n, int nphase, int* bad)
{
    const int nb = sweep_blocks(n, 2048);
    hipLaunchKernelGGL(phase_check_kernel, dim3(nb), dim3(kBlock), 0, st, phase, n, nphase, bad);
    return hipGetLastError();
}

hipError_t launch_total_displacement(hipStream_t st, const Dims& d, const double* strain6,
                                     const Fields& f, double* const u[3])
{
    const int nb = sweep_blocks(d.n, 4096);
    Strain6 E;
    for (int q = 0; q < 6; ++q) E.e[q] = strain6[q];
    hipLaunchKernelGGL(total_displacement_kernel, dim3(nb), dim3(kBlock), 0, st, d, E, f, u[0], u[1],
                       u[2]);
    return hipGetLastError();
}

}  // namespace e3d
