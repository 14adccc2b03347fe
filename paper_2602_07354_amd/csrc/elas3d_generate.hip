// gfx950 kernels of the microstructure generator (ELAS3D-Xtal, arXiv
// 2602.07354, Sec. 2.2): grain assignment by the smallest ellipsoidal
// distance (Eq. ellipsoid_dist) and the overwrite of the grain map by pores
// (Sec. 2.2.3).
//
// Grain assignment.  The result is the plain definition: every voxel centre
// goes to the grain with the smallest D^2 over all grains (periodic minimum
// images, lowest index on ties).  The paper cuts the search with cells grown
// by 1.5 times the largest radius; here the cells only order the search: a
// lane scans its voxel's cell, then shells of cells at growing Chebyshev
// distance k, and stops once no unscanned seed can beat the best one found.
// Seeds beyond shell k lie at least k*hmin away, so their D^2 is at least
// (k*hmin)^2 / Rmax^2 with Rmax the largest semi-axis of any grain; the lane
// stops when its best D^2 is below that bound (with a relative margin for the
// rounding of the cell binning).  The distance is evaluated in FP64 without
// contraction and in the same order as the definition, so the result equals
// a brute-force scan bit for bit.
//
// Pores.  Pores are given in order and carved until the void count reaches a
// target.  Since a carved voxel stays void, the voxels made void by the
// first P pores are those whose smallest covering pore index is below P.  The
// first pass scatters that index (vector atomicMin over each pore's bounding
// box), the second counts per pore the voxels it is the first to cover
// (among those not void before), the host takes the prefix sum to find P,
// the third writes the void id.  All integer: independent of scheduling.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "elas3d.h"
#include "elas3d_internal.h"

namespace {

constexpr int kGenBlock = 256;
constexpr int kPoreStride = 15;  // centre 3, semi-axes 3, R row-major 9

struct GrainGrid {
    int nx, ny, nz;
    int cx, cy, cz;        // cells per dimension
    double hx, hy, hz;     // cell edges
    double bound_scale;    // (hmin (1 - margin))^2 / Rmax^2
    int kfull;             // shells needed to cover every cell
    const int* start;      // cx*cy*cz + 1 offsets into the sorted seeds
    const double* sx;
    const double* sy;
    const double* sz;
    const double* rt2;
    const double* rl2;
    const int* gid;
};

// Minimum-image offset of x from s in a box of length L, rounded once.
__device__ __forceinline__ double min_image(double x, double s, double L)
{
#pragma clang fp contract(off)
    const double d = x - s;
    if (d > 0.5 * L) return (x - L) - s;
    if (d < -0.5 * L) return (x + L) - s;
    return d;
}

__device__ __forceinline__ int cell_of(double x, double h, int nc)
{
    int c = (int)floor(x / h);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__global__ void __launch_bounds__(kGenBlock) grains_kernel(GrainGrid G, int32_t* __restrict__ phase)
{
#pragma clang fp contract(off)
    const long n = (long)G.nx * G.ny * G.nz;
    const double Lx = G.nx, Ly = G.ny, Lz = G.nz;
    const int lox = (G.cx - 1) / 2, hix = G.cx / 2;
    const int loy = (G.cy - 1) / 2, hiy = G.cy / 2;
    const int loz = (G.cz - 1) / 2, hiz = G.cz / 2;
    for (long m = (long)blockIdx.x * kGenBlock + threadIdx.x; m < n; m += (long)gridDim.x * kGenBlock) {
        const int k = (int)(m / ((long)G.nx * G.ny));
        const int r = (int)(m - (long)k * G.nx * G.ny);
        const int j = r / G.nx, i = r - j * G.nx;
        const double x = i + 0.5, y = j + 0.5, z = k + 0.5;
        const int vx = cell_of(x, G.hx, G.cx), vy = cell_of(y, G.hy, G.cy), vz = cell_of(z, G.hz, G.cz);
        double best = INFINITY;
        int arg = INT_MAX;
        for (int sh = 0; sh <= G.kfull; ++sh) {
            for (int oz = -min(sh, loz); oz <= min(sh, hiz); ++oz)
                for (int oy = -min(sh, loy); oy <= min(sh, hiy); ++oy)
                    for (int ox = -min(sh, lox); ox <= min(sh, hix); ++ox) {
                        if (max(abs(ox), max(abs(oy), abs(oz))) != sh) continue;
                        int cx = vx + ox, cy = vy + oy, cz = vz + oz;
                        cx += cx < 0 ? G.cx : (cx >= G.cx ? -G.cx : 0);
                        cy += cy < 0 ? G.cy : (cy >= G.cy ? -G.cy : 0);
                        cz += cz < 0 ? G.cz : (cz >= G.cz ? -G.cz : 0);
                        const int c = cx + G.cx * (cy + G.cy * cz);
                        for (int q = G.start[c]; q < G.start[c + 1]; ++q) {
                            const double dx = min_image(x, G.sx[q], Lx);
                            const double dy = min_image(y, G.sy[q], Ly);
                            const double dz = min_image(z, G.sz[q], Lz);
                            const double d2 = (dx * dx + dy * dy) / G.rt2[q] + (dz * dz) / G.rl2[q];
                            const int g = G.gid[q];
                            if (d2 < best || (d2 == best && g < arg)) {
                                best = d2;
                                arg = g;
                            }
                        }
                    }
            // every seed not scanned yet lies beyond shell sh
            const double reach = (double)sh * sh * G.bound_scale;
            if (best < reach) break;
        }
        phase[m] = arg;
    }
}

struct PoreBox {
    int lo[3], w[3];  // first raw (unwrapped) voxel index and width per dimension
};

__device__ __forceinline__ bool pore_covers(const double* __restrict__ p, double x, double y, double z,
                                            double Lx, double Ly, double Lz)
{
#pragma clang fp contract(off)
    const double d0 = min_image(x, p[0], Lx);
    const double d1 = min_image(y, p[1], Ly);
    const double d2 = min_image(z, p[2], Lz);
    const double* a = p + 3;
    const double* R = p + 6;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double e = (d0 * R[c] + d1 * R[3 + c]) + d2 * R[6 + c];
        const double q = e / a[c];
        s = c == 0 ? q * q : s + q * q;
    }
    return s <= 1.0 + 1e-12;
}

// first[v] = smallest index of a pore covering voxel v (among voxels that are
// not void); one workgroup per pore, lanes over its bounding box.
__global__ void __launch_bounds__(kGenBlock) pore_first_kernel(int nx, int ny, int nz,
                                                               const int32_t* __restrict__ phase,
                                                               int32_t void_id,
                                                               const double* __restrict__ pores,
                                                               const PoreBox* __restrict__ boxes,
                                                               int npore, int32_t* first)
{
    const double Lx = nx, Ly = ny, Lz = nz;
    for (int p = blockIdx.x; p < npore; p += gridDim.x) {
        const PoreBox b = boxes[p];
        const double* P = pores + (size_t)kPoreStride * p;
        const long cnt = (long)b.w[0] * b.w[1] * b.w[2];
        for (long t = threadIdx.x; t < cnt; t += kGenBlock) {
            const int tz = (int)(t / ((long)b.w[0] * b.w[1]));
            const int rem = (int)(t - (long)tz * b.w[0] * b.w[1]);
            const int ty = rem / b.w[0], tx = rem - ty * b.w[0];
            int i = (b.lo[0] + tx) % nx, j = (b.lo[1] + ty) % ny, k = (b.lo[2] + tz) % nz;
            i += i < 0 ? nx : 0;
            j += j < 0 ? ny : 0;
            k += k < 0 ? nz : 0;
            const long v = i + (long)nx * (j + (long)ny * k);
            if (phase[v] == void_id) continue;
            if (pore_covers(P, i + 0.5, j + 0.5, k + 0.5, Lx, Ly, Lz)) atomicMin(first + v, p);
        }
    }
}

// counts[p] += voxels whose first covering pore is p; void0 += voxels void
// on entry.
__global__ void __launch_bounds__(kGenBlock) pore_count_kernel(long n, const int32_t* __restrict__ phase,
                                                               int32_t void_id,
                                                               const int32_t* __restrict__ first,
                                                               int npore, unsigned long long* counts,
                                                               unsigned long long* void0)
{
    unsigned long long v0 = 0;
    for (long m = (long)blockIdx.x * kGenBlock + threadIdx.x; m < n; m += (long)gridDim.x * kGenBlock) {
        if (phase[m] == void_id)
            ++v0;
        else if (first[m] < npore)
            atomicAdd(counts + first[m], 1ull);
    }
    // one atomic per wave for the entry void count
    for (int off = 32; off > 0; off >>= 1) v0 += __shfl_xor(v0, off);
    if ((threadIdx.x & 63) == 0 && v0) atomicAdd(void0, v0);
}

__global__ void __launch_bounds__(kGenBlock) pore_apply_kernel(long n, int32_t* phase, int32_t void_id,
                                                               const int32_t* __restrict__ first,
                                                               int used)
{
    for (long m = (long)blockIdx.x * kGenBlock + threadIdx.x; m < n; m += (long)gridDim.x * kGenBlock)
        if (first[m] < used) phase[m] = void_id;
}

__global__ void __launch_bounds__(kGenBlock) fill_int_kernel(long n, int32_t* a, int32_t v)
{
    for (long m = (long)blockIdx.x * kGenBlock + threadIdx.x; m < n; m += (long)gridDim.x * kGenBlock) a[m] = v;
}

int grid_for(long n)
{
    long b = (n + kGenBlock - 1) / kGenBlock;
    return (int)std::max(1L, std::min(b, 16384L));
}

int gen_fail(int code, const std::string& msg)
{
    e3d::set_last_error(msg);
    return code;
}

// Device buffers and stream of one generator call, released on scope exit.
struct GenCall {
    hipStream_t stream = nullptr;
    bool own = false;
    std::vector<void*> bufs;
    ~GenCall()
    {
        if (stream) hipStreamSynchronize(stream);
        for (void* p : bufs) hipFree(p);
        if (own && stream) hipStreamDestroy(stream);
    }
    template <typename P>
    hipError_t alloc(P** p, size_t bytes)
    {
        hipError_t e = hipMalloc((void**)p, bytes);
        if (e == hipSuccess) bufs.push_back((void*)*p);
        return e;
    }
};

#define GENCHK(expr)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return gen_fail(ELAS3D_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

int gen_begin(const elas3d_options* opt, GenCall& call)
{
    elas3d_options o;
    if (opt)
        o = *opt;
    else
        elas3d_options_init(&o);
    if (o.device >= 0) GENCHK(hipSetDevice(o.device));
    if (o.stream) {
        call.stream = (hipStream_t)o.stream;
    } else {
        GENCHK(hipStreamCreateWithFlags(&call.stream, hipStreamNonBlocking));
        call.own = true;
    }
    return 0;
}

int check_grid(int32_t nx, int32_t ny, int32_t nz)
{
    if (nx < 1 || ny < 1 || nz < 1) return gen_fail(ELAS3D_EBADARG, "grid dimensions must each be >= 1");
    if (3 * (int64_t)nx * ny * nz >= ((int64_t)1 << 31))
        return gen_fail(ELAS3D_EBADARG, "3*nx*ny*nz must be < 2^31");
    return 0;
}

// Validated inputs of a grain assignment and its search cells: about one
// seed per cell, each at least one voxel wide.
struct GrainPlan {
    int nx, ny, nz;
    int nc[3];
    double h[3];
    long ncell;
    double rmax;
};

int grain_plan(int32_t nx, int32_t ny, int32_t nz, int32_t ngrain, const double* seeds, const double* semi,
               GrainPlan& P)
{
    int rc = check_grid(nx, ny, nz);
    if (rc) return rc;
    if (ngrain < 1) return gen_fail(ELAS3D_EBADARG, "ngrain must be >= 1");
    if (!seeds) return gen_fail(ELAS3D_EBADARG, "seeds is NULL");
    const int dims[3] = {nx, ny, nz};
    double rmax = 0.0;
    for (int g = 0; g < ngrain; ++g) {
        for (int d = 0; d < 3; ++d) {
            const double s = seeds[3 * (size_t)g + d];
            if (!(s >= 0.0 && s < dims[d]))
                return gen_fail(ELAS3D_EBADARG, "seed " + std::to_string(g) + " outside [0, n)");
        }
        const double rt = semi ? semi[2 * (size_t)g] : 1.0, rl = semi ? semi[2 * (size_t)g + 1] : 1.0;
        if (!(rt > 0.0) || !(rl > 0.0) || !std::isfinite(rt) || !std::isfinite(rl))
            return gen_fail(ELAS3D_EBADARG, "semi-axes of grain " + std::to_string(g) + " must be > 0");
        rmax = std::max(rmax, std::max(rt, rl));
    }
    const double spacing = std::cbrt((double)nx * ny * nz / ngrain);
    P.nx = nx;
    P.ny = ny;
    P.nz = nz;
    for (int d = 0; d < 3; ++d) {
        P.nc[d] = (int)std::max(1.0, std::min((double)dims[d], std::floor(dims[d] / spacing)));
        P.h[d] = (double)dims[d] / P.nc[d];
    }
    P.ncell = (long)P.nc[0] * P.nc[1] * P.nc[2];
    P.rmax = rmax;
    return 0;
}

// Counting sort of the seeds by cell (ascending grain id within a cell):
// start[ncell + 1] offsets, gid[ngrain] grain of each sorted slot, cols the
// five SoA columns x, y, z, rt^2, rl^2 (ngrain each); owner and fillp are
// work arrays (ngrain and ncell).
void grain_sort(const double* seeds, const double* semi, int ngrain, const GrainPlan& P, int* start, int* owner,
                int* fillp, int* gid, double* cols)
{
    auto cell = [&](int d, double x) {
        int c = (int)std::floor(x / P.h[d]);
        return c < 0 ? 0 : (c >= P.nc[d] ? P.nc[d] - 1 : c);
    };
    std::fill(start, start + P.ncell + 1, 0);
    for (int g = 0; g < ngrain; ++g) {
        const long c = cell(0, seeds[3 * (size_t)g]) +
                       (long)P.nc[0] * (cell(1, seeds[3 * (size_t)g + 1]) +
                                        (long)P.nc[1] * cell(2, seeds[3 * (size_t)g + 2]));
        owner[g] = (int)c;
        ++start[c + 1];
    }
    for (long c = 0; c < P.ncell; ++c) start[c + 1] += start[c];
    std::copy(start, start + P.ncell, fillp);
    for (int g = 0; g < ngrain; ++g) {
        const int q = fillp[owner[g]]++;
        gid[q] = g;
        cols[q] = seeds[3 * (size_t)g];
        cols[(size_t)ngrain + q] = seeds[3 * (size_t)g + 1];
        cols[2 * (size_t)ngrain + q] = seeds[3 * (size_t)g + 2];
        const double rt = semi ? semi[2 * (size_t)g] : 1.0, rl = semi ? semi[2 * (size_t)g + 1] : 1.0;
        cols[3 * (size_t)ngrain + q] = rt * rt;
        cols[4 * (size_t)ngrain + q] = rl * rl;
    }
}

// Copies the sorted seeds to the device buffers and launches the grain
// kernel on st (asynchronous: the host arrays must stay valid until the
// stream passes the copies, which pageable host memory guarantees on return).
int grain_launch(hipStream_t st, const GrainPlan& P, int ngrain, const int* start, const int* gid,
                 const double* cols, int* dstart, int* dgid, double* dseed, int32_t* out)
{
    GENCHK(hipMemcpyAsync(dstart, start, sizeof(int) * (size_t)(P.ncell + 1), hipMemcpyHostToDevice, st));
    GENCHK(hipMemcpyAsync(dgid, gid, sizeof(int) * (size_t)ngrain, hipMemcpyHostToDevice, st));
    GENCHK(hipMemcpyAsync(dseed, cols, sizeof(double) * 5 * (size_t)ngrain, hipMemcpyHostToDevice, st));
    GrainGrid G{};
    G.nx = P.nx;
    G.ny = P.ny;
    G.nz = P.nz;
    G.cx = P.nc[0];
    G.cy = P.nc[1];
    G.cz = P.nc[2];
    G.hx = P.h[0];
    G.hy = P.h[1];
    G.hz = P.h[2];
    const double hmin = std::min(P.h[0], std::min(P.h[1], P.h[2])) * (1.0 - 1e-9);
    G.bound_scale = hmin * hmin / (P.rmax * P.rmax);
    G.kfull = std::max({P.nc[0] / 2, P.nc[1] / 2, P.nc[2] / 2});
    G.start = dstart;
    G.gid = dgid;
    G.sx = dseed;
    G.sy = dseed + ngrain;
    G.sz = dseed + 2 * (size_t)ngrain;
    G.rt2 = dseed + 3 * (size_t)ngrain;
    G.rl2 = dseed + 4 * (size_t)ngrain;
    const long n = (long)P.nx * P.ny * P.nz;
    hipLaunchKernelGGL(grains_kernel, dim3(grid_for(n)), dim3(kGenBlock), 0, st, G, out);
    GENCHK(hipGetLastError());
    return 0;
}

// ---- the allocation-free grain assignment ------------------------------
// Its sorted seeds live in a static device array (one copy per GPU, held
// until the process ends) and its host staging in static host arrays.
constexpr int kStaticMaxGrains = 1 << 16;
constexpr long kStaticMaxCells = 1L << 17;
constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kOffStart = 0;
constexpr size_t kOffGid = align256(kOffStart + sizeof(int) * (kStaticMaxCells + 1));
constexpr size_t kOffSeed = align256(kOffGid + sizeof(int) * kStaticMaxGrains);
constexpr size_t kStaticBytes = align256(kOffSeed + sizeof(double) * 5 * kStaticMaxGrains);

__device__ __align__(256) char scratch[kStaticBytes];

struct StaticHost {
    int start[kStaticMaxCells + 1];
    int owner[kStaticMaxGrains];
    int fillp[kStaticMaxCells];
    int gid[kStaticMaxGrains];
    double cols[5 * kStaticMaxGrains];
};
StaticHost g_static_host;
std::mutex g_static_mu;
constexpr int kMaxDevices = 64;
char* g_scratch_dev[kMaxDevices] = {};

// Device address of this GPU's copy of the work area (the array's name is
// a host-side stand-in, not a device address), looked up once per device
// with that device current.
int static_scratch(int dev, char** out)
{
    if (dev < 0 || dev >= kMaxDevices) return gen_fail(ELAS3D_EBADARG, "device ordinal out of range");
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        GENCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return gen_fail(ELAS3D_EDEVICE, "no device address for the static work area");
        g_scratch_dev[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_dev[dev];
    return 0;
}

}  // namespace

extern "C" {

int elas3d_generate_grains(int32_t nx, int32_t ny, int32_t nz, int32_t ngrain, const double* seeds,
                           const double* semi, int32_t* phase, const elas3d_options* opt)
{
    if (!phase) return gen_fail(ELAS3D_EBADARG, "phase is NULL");
    GrainPlan P;
    int rc = grain_plan(nx, ny, nz, ngrain, seeds, semi, P);
    if (rc) return rc;
    std::vector<int> start(P.ncell + 1), owner(ngrain), fillp(P.ncell), gid(ngrain);
    std::vector<double> cols(5 * (size_t)ngrain);
    grain_sort(seeds, semi, ngrain, P, start.data(), owner.data(), fillp.data(), gid.data(), cols.data());
    GenCall call;
    rc = gen_begin(opt, call);
    if (rc) return rc;
    int *dstart = nullptr, *dgid = nullptr;
    double* dseed = nullptr;
    GENCHK(call.alloc(&dstart, sizeof(int) * start.size()));
    GENCHK(call.alloc(&dgid, sizeof(int) * (size_t)ngrain));
    GENCHK(call.alloc(&dseed, sizeof(double) * 5 * (size_t)ngrain));
    const long n = (long)nx * ny * nz;
    const bool dev_out = opt && opt->outputs_on_device;
    int32_t* out = phase;
    if (!dev_out) GENCHK(call.alloc(&out, sizeof(int32_t) * (size_t)n));
    rc = grain_launch(call.stream, P, ngrain, start.data(), gid.data(), cols.data(), dstart, dgid, dseed, out);
    if (rc) return rc;
    if (!dev_out)
        GENCHK(hipMemcpyAsync(phase, out, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, call.stream));
    GENCHK(hipStreamSynchronize(call.stream));
    return 0;
}

int elas3d_generate_grains_static(int32_t nx, int32_t ny, int32_t nz, int32_t ngrain, const double* seeds,
                                  const double* semi, int32_t* phase, const elas3d_options* opt)
{
    if (!phase) return gen_fail(ELAS3D_EBADARG, "phase is NULL");
    if (!opt || !opt->outputs_on_device)
        return gen_fail(ELAS3D_EBADARG, "the allocation-free grain assignment writes device memory only: "
                                        "set options.outputs_on_device and pass a device phase buffer");
    if (ngrain > kStaticMaxGrains)
        return gen_fail(ELAS3D_EBADARG, "ngrain above " + std::to_string(kStaticMaxGrains) +
                                            " (the static work area's limit)");
    GrainPlan P;
    int rc = grain_plan(nx, ny, nz, ngrain, seeds, semi, P);
    if (rc) return rc;
    if (P.ncell > kStaticMaxCells)
        return gen_fail(ELAS3D_EBADARG, std::to_string(P.ncell) + " search cells, above " +
                                            std::to_string(kStaticMaxCells) + " (the static work area's limit)");
    // one call at a time in the process: the host staging below and each
    // device's work area are shared by every call
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (opt->device >= 0) GENCHK(hipSetDevice(opt->device));
    int dev = 0;
    GENCHK(hipGetDevice(&dev));
    char* base = nullptr;
    rc = static_scratch(dev, &base);
    if (rc) return rc;
    StaticHost& H = g_static_host;
    grain_sort(seeds, semi, ngrain, P, H.start, H.owner, H.fillp, H.gid, H.cols);
    int* dstart = reinterpret_cast<int*>(base + kOffStart);
    int* dgid = reinterpret_cast<int*>(base + kOffGid);
    double* dseed = reinterpret_cast<double*>(base + kOffSeed);
    hipStream_t st = (hipStream_t)opt->stream;  // NULL: the default stream
    rc = grain_launch(st, P, ngrain, H.start, H.gid, H.cols, dstart, dgid, dseed, phase);
    if (rc) return rc;
    GENCHK(hipStreamSynchronize(st));
    return 0;
}

int elas3d_carve_pores(int32_t nx, int32_t ny, int32_t nz, int32_t* phase, int32_t void_id, int32_t npore,
                       const double* pores, double target, int32_t* used, int64_t* nvoid,
                       const elas3d_options* opt)
{
    int rc = check_grid(nx, ny, nz);
    if (rc) return rc;
    if (!phase || (npore > 0 && !pores)) return gen_fail(ELAS3D_EBADARG, "phase or pores is NULL");
    if (npore < 0) return gen_fail(ELAS3D_EBADARG, "npore must be >= 0");
    if (std::isnan(target)) return gen_fail(ELAS3D_EBADARG, "target is NaN");
    const int dims[3] = {nx, ny, nz};
    std::vector<PoreBox> boxes((size_t)std::max(npore, 1));
    for (int p = 0; p < npore; ++p) {
        const double* P = pores + (size_t)kPoreStride * p;
        for (int q = 0; q < kPoreStride; ++q)
            if (!std::isfinite(P[q])) return gen_fail(ELAS3D_EBADARG, "pore " + std::to_string(p) + " is not finite");
        double half = 0.0;
        for (int d = 0; d < 3; ++d) {
            if (!(P[d] >= 0.0 && P[d] < dims[d]))
                return gen_fail(ELAS3D_EBADARG, "pore centre " + std::to_string(p) + " outside [0, n)");
            if (!(P[3 + d] > 0.0)) return gen_fail(ELAS3D_EBADARG, "pore semi-axes must be > 0");
            half = std::max(half, P[3 + d]);
        }
        for (int d = 0; d < 3; ++d) {
            // voxel centres within `half` of the centre, one voxel of margin
            const double lo = std::floor(P[d] - half - 0.5) - 1.0, hi = std::ceil(P[d] + half - 0.5) + 1.0;
            if (hi - lo + 1.0 >= dims[d]) {
                boxes[p].lo[d] = 0;
                boxes[p].w[d] = dims[d];
            } else {
                boxes[p].lo[d] = (int)lo;
                boxes[p].w[d] = (int)(hi - lo + 1.0);
            }
        }
    }
    GenCall call;
    rc = gen_begin(opt, call);
    if (rc) return rc;
    const long n = (long)nx * ny * nz;
    const bool dev = opt && opt->outputs_on_device;
    int32_t* ph = phase;
    if (!dev) {
        GENCHK(call.alloc(&ph, sizeof(int32_t) * (size_t)n));
        GENCHK(hipMemcpyAsync(ph, phase, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, call.stream));
    }
    int32_t* first = nullptr;
    double* dpores = nullptr;
    PoreBox* dboxes = nullptr;
    unsigned long long* dcnt = nullptr;
    GENCHK(call.alloc(&first, sizeof(int32_t) * (size_t)n));
    GENCHK(call.alloc(&dcnt, sizeof(unsigned long long) * ((size_t)npore + 1)));
    hipLaunchKernelGGL(fill_int_kernel, dim3(grid_for(n)), dim3(kGenBlock), 0, call.stream, n, first,
                       (int32_t)INT_MAX);
    GENCHK(hipGetLastError());
    GENCHK(hipMemsetAsync(dcnt, 0, sizeof(unsigned long long) * ((size_t)npore + 1), call.stream));
    if (npore > 0) {
        GENCHK(call.alloc(&dpores, sizeof(double) * kPoreStride * (size_t)npore));
        GENCHK(call.alloc(&dboxes, sizeof(PoreBox) * (size_t)npore));
        GENCHK(hipMemcpyAsync(dpores, pores, sizeof(double) * kPoreStride * (size_t)npore, hipMemcpyHostToDevice,
                              call.stream));
        GENCHK(hipMemcpyAsync(dboxes, boxes.data(), sizeof(PoreBox) * (size_t)npore, hipMemcpyHostToDevice,
                              call.stream));
        hipLaunchKernelGGL(pore_first_kernel, dim3(std::min(npore, 65535)), dim3(kGenBlock), 0, call.stream, nx,
                           ny, nz, (const int32_t*)ph, void_id, (const double*)dpores, (const PoreBox*)dboxes,
                           npore, first);
        GENCHK(hipGetLastError());
    }
    hipLaunchKernelGGL(pore_count_kernel, dim3(grid_for(n)), dim3(kGenBlock), 0, call.stream, n,
                       (const int32_t*)ph, void_id, (const int32_t*)first, npore, dcnt + 1, dcnt);
    GENCHK(hipGetLastError());
    std::vector<unsigned long long> cnt((size_t)npore + 1);
    GENCHK(hipMemcpyAsync(cnt.data(), dcnt, sizeof(unsigned long long) * cnt.size(), hipMemcpyDeviceToHost,
                          call.stream));
    GENCHK(hipStreamSynchronize(call.stream));
    // pores carved in order until the void count reaches the target
    int64_t count = (int64_t)cnt[0];
    int u = 0;
    while (u < npore && !(target >= 0.0 && !((double)count < target))) {
        count += (int64_t)cnt[(size_t)u + 1];
        ++u;
    }
    hipLaunchKernelGGL(pore_apply_kernel, dim3(grid_for(n)), dim3(kGenBlock), 0, call.stream, n, ph, void_id,
                       (const int32_t*)first, u);
    GENCHK(hipGetLastError());
    if (!dev)
        GENCHK(hipMemcpyAsync(phase, ph, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, call.stream));
    GENCHK(hipStreamSynchronize(call.stream));
    if (used) *used = u;
    if (nvoid) *nvoid = count;
    return 0;
}

}  // extern "C"
