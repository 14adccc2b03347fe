// Host runtime and C-ABI of libelas3d: argument validation, device memory
// budget, per-phase coefficient tables, and the iteration driver of the
// point-block Jacobi PCG (ELAS3D-Xtal, arXiv 2602.07354, Algorithm 2).
//
// The PCG scalars live on the device and are updated by single-block
// finalize kernels, so iterations are enqueued back to back; the host only
// reads the stop flag every `poll_interval` iterations, one batch behind
// the device (a batch enqueued after convergence returns at once).
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "elas3d.h"
#include "elas3d_internal.h"
#include "elas3d_runtime.h"

using namespace e3d::rt;

namespace {

thread_local std::string g_last_error = "";

}  // namespace

void e3d::set_last_error(const std::string& msg) { g_last_error = msg; }

namespace e3d::rt {

int fail(elas3d_ctx* ctx, int code, const std::string& msg)
{
    if (ctx)
        ctx->err = msg;
    else
        g_last_error = msg;
    return code;
}

void default_options(elas3d_options* o)
{
    std::memset(o, 0, sizeof(*o));
    o->precision = ELAS3D_PREC_FP64;
    o->convergence = ELAS3D_CONV_RESIDUAL;
    o->preconditioner = ELAS3D_PRECOND_BLOCK_JACOBI;
    o->device = -1;
    o->graphs = 1;
}

// Device bytes of a context (kept in one place so the budget check and
// elas3d_device_bytes agree).
// Partial sums per value slot: one per workgroup (and RHS) of the largest
// grid any sweep, autotuning candidate or fixed geometry (tile, zchunk) can
// launch.
long long partial_slots(const Dims& d, int nrhs, int tile, int zchunk)
{
    long long most = kMinPartialSlots;
    for (int t = 0; t < e3d::kNumTiles; ++t)
        for (int target : kTuneTargets)
            most = std::max(most, (long long)e3d::op_geometry(d, 0, t, target).blocks * nrhs);
    most = std::max(most, (long long)e3d::op_geometry(d, zchunk, tile).blocks * nrhs);
    return most;
}

double plan_bytes(int32_t nx, int32_t ny, int32_t nz, int nphase, int nrhs, bool mixed, bool batched,
                  int tile, int zchunk)
{
    const int64_t n = (int64_t)nx * ny * nz;
    const double N = (double)n;
    double bytes = 0.0;
    if (mixed)  // FP32 work, table
        bytes += 4.0 * 18.0 * (batched ? nrhs : 1) * N + 4.0 * nphase * e3d::kCoefStride;
    bytes += 4.0 * N;                          // phase ids
    bytes += 8.0 * 3.0 * N * nrhs * 2.0;       // b and w per case
    bytes += 8.0 * 15.0 * N * (batched ? nrhs : 1);  // g, z, h0, h1, Ah
    // M^-1 (symmetric 3x3) rows: at most one per phase and one per node, and
    // the row index of each node
    bytes += (8.0 * 6.0 * (mixed ? 1.5 : 1.0)) * (N + nphase) + 4.0 * N;
    bytes += (double)nphase * 8.0 * (e3d::kCoefStride + e3d::kDiagStride + 1.0) +
             (double)nphase * nrhs * 8.0 * e3d::kSigStride;
    bytes += 8.0 * kPartialValues * (double)partial_slots(Dims{nx, ny, nz, (int)n}, nrhs, tile, zchunk);
    if (tile >= 0 && tile < e3d::kNumTiles && e3d::is_ws(tile)) {
        // the forced wave-specialised shape's phase dictionaries
        const e3d::OpGeom g = e3d::op_geometry(Dims{nx, ny, nz, (int)n}, zchunk, tile);
        bytes += (double)e3d::ws_map_bytes(g) + 4.0 * e3d::kWsDict * g.blocks;
    }
    bytes += 4096.0;
    return bytes;
}

// Voigt index of the tensor pair (i,j).
int voigt(int i, int j)
{
    if (i == j) return i;
    const int s = i + j;
    return s == 3 ? 3 : (s == 2 ? 4 : 5);  // (1,2)->3, (0,2)->4, (0,1)->5
}

int ut(int r, int c)
{
    if (r > c) std::swap(r, c);
    return r * 6 - (r * (r - 1)) / 2 + (c - r);
}

// Per-phase tables (Sec. 2.1.1: a full stiffness per phase).
//  coef: packed upper triangle of C/16 (the weight of the constant strain
//        mode of the element operator; dividing by a power of two is exact).
//  diag: the corner block of the element stiffness for corner signs s,
//        (K_e)_aa,ij = sum_kl s_k s_l C_ikjl I_kl with I_kk = 1/9 and
//        I_kl = 1/12 (k != l) the integrals of products of shape-function
//        derivatives over the voxel, split as D + sx sy Oxy + sx sz Oxz + sy sz Oyz.
//  sig:  C E_hat per load case (uniform stress of the affine field).
void build_tables(const double* C, int nphase, const double* strain, int nrhs,
                  std::vector<double>& coef, std::vector<double>& diag, std::vector<uint8_t>& solid,
                  std::vector<double>& sig)
{
    coef.assign((size_t)nphase * e3d::kCoefStride, 0.0);
    diag.assign((size_t)nphase * e3d::kDiagStride, 0.0);
    solid.assign((size_t)nphase, 0);
    sig.assign((size_t)nrhs * nphase * e3d::kSigStride, 0.0);
    const int pij[6][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}, {0, 2}, {0, 1}};
    for (int p = 0; p < nphase; ++p) {
        const double* Cp = C + 36 * (size_t)p;
        auto T = [&](int i, int j, int k, int l) { return Cp[6 * voigt(i, j) + voigt(k, l)]; };
        bool any = false;
        for (int q = 0; q < 36; ++q) any = any || Cp[q] != 0.0;
        solid[p] = any ? 1 : 0;
        for (int r = 0; r < 6; ++r)
            for (int c = r; c < 6; ++c)
                coef[(size_t)p * e3d::kCoefStride + ut(r, c)] = Cp[6 * r + c] / 16.0;  // exact
        double* dg = diag.data() + (size_t)p * e3d::kDiagStride;
        for (int q = 0; q < 6; ++q) {
            const int i = pij[q][0], j = pij[q][1];
            dg[q] = (T(i, 0, j, 0) + T(i, 1, j, 1) + T(i, 2, j, 2)) / 9.0;
            dg[6 + q] = (T(i, 0, j, 1) + T(i, 1, j, 0)) / 12.0;   // x-y corner term
            dg[12 + q] = (T(i, 0, j, 2) + T(i, 2, j, 0)) / 12.0;  // x-z
            dg[18 + q] = (T(i, 1, j, 2) + T(i, 2, j, 1)) / 12.0;  // y-z
        }
        for (int r = 0; r < nrhs; ++r) {
            const double* E = strain + 6 * r;
            const double Eh[6] = {E[0], E[1], E[2], 2 * E[3], 2 * E[4], 2 * E[5]};
            double* s = sig.data() + ((size_t)r * nphase + p) * e3d::kSigStride;
            for (int a = 0; a < 6; ++a) {
                double acc = 0.0;
                for (int b = 0; b < 6; ++b) acc += Cp[6 * a + b] * Eh[b];
                s[a] = acc;
            }
        }
    }
}

int validate_options(const elas3d_options* o)
{
    if (o->precision != ELAS3D_PREC_FP64 && o->precision != ELAS3D_PREC_MIXED)
        return fail(nullptr, ELAS3D_EBADARG, "options.precision must be ELAS3D_PREC_FP64 or _MIXED");
    if (o->convergence != ELAS3D_CONV_RESIDUAL && o->convergence != ELAS3D_CONV_PAPER)
        return fail(nullptr, ELAS3D_EBADARG, "options.convergence must be RESIDUAL or PAPER");
    if (o->preconditioner != ELAS3D_PRECOND_BLOCK_JACOBI && o->preconditioner != ELAS3D_PRECOND_NONE)
        return fail(nullptr, ELAS3D_EBADARG, "options.preconditioner must be BLOCK_JACOBI or NONE");
    if (o->poll_interval < 0 || o->inner_maxit < 0)
        return fail(nullptr, ELAS3D_EBADARG, "options.poll_interval / inner_maxit must be >= 0");
    if (!(o->hbm_budget_bytes >= 0.0) || !std::isfinite(o->hbm_budget_bytes))
        return fail(nullptr, ELAS3D_EBADARG, "options.hbm_budget_bytes must be finite and >= 0");
    if (!(o->inner_tol >= 0.0) || !(o->inner_tol < 1.0))
        return fail(nullptr, ELAS3D_EBADARG, "options.inner_tol must be in [0, 1)");
    if (o->tile < 0 || o->tile >= e3d::kNumTiles)
        return fail(nullptr, ELAS3D_EBADARG,
                    "options.tile must be in [0, " + std::to_string(e3d::kNumTiles - 1) + "]");
    if (o->zchunk < 0) return fail(nullptr, ELAS3D_EBADARG, "options.zchunk must be >= 0");
    if (o->update_blocks < 0 || o->update_blocks > kMaxUpdateBlocks)
        return fail(nullptr, ELAS3D_EBADARG,
                    "options.update_blocks must be in [0, " + std::to_string(kMaxUpdateBlocks) + "]");
    if (o->update_nontemporal != 0 && o->update_nontemporal != 1)
        return fail(nullptr, ELAS3D_EBADARG, "options.update_nontemporal must be 0 or 1");
    return 0;
}

int validate_setup(int32_t nx, int32_t ny, int32_t nz, const int32_t* phase, int32_t nphase,
                   const double* C, int32_t nrhs, const double* strain, const elas3d_options* o)
{
    if (nx < 2 || ny < 2 || nz < 2)
        return fail(nullptr, ELAS3D_EBADARG, "grid dimensions must each be >= 2");
    const int64_t n = (int64_t)nx * ny * nz;
    if (3 * n >= ((int64_t)1 << 31))
        return fail(nullptr, ELAS3D_EBADARG, "3*nx*ny*nz must be < 2^31");
    if (!phase) return fail(nullptr, ELAS3D_EBADARG, "phase is NULL");
    if (!C) return fail(nullptr, ELAS3D_EBADARG, "C is NULL");
    if (!strain) return fail(nullptr, ELAS3D_EBADARG, "strain is NULL");
    if (nphase < 1) return fail(nullptr, ELAS3D_EBADARG, "nphase must be >= 1");
    if (nrhs < 1 || nrhs > ELAS3D_MAX_RHS)
        return fail(nullptr, ELAS3D_EBADARG, "nrhs must be in [1, 6]");
    int rc = validate_options(o);
    if (rc) return rc;
    {
        // a forced wave-specialised shape streams node rows in whole 16-byte
        // chunks in every precision the context sweeps in
        const Dims d{nx, ny, nz, (int)n};
        const int elem = o->precision == ELAS3D_PREC_MIXED ? 4 : 8;
        if (o->autotune != 1 && !e3d::ws_elem_ok(o->tile, elem))
            return fail(nullptr, ELAS3D_EBADARG,
                        "options.tile " + std::to_string(o->tile) +
                            " is a shape of the FP32 sweep only (mixed precision)");
        if (o->autotune != 1 && !e3d::ws_supported(d, o->tile, elem))
            return fail(nullptr, ELAS3D_EBADARG,
                        "options.tile " + std::to_string(o->tile) + " needs nx to be a multiple of " +
                            std::to_string(16 / elem) + " and nx*ny < 2^27");
    }
    for (int p = 0; p < nphase; ++p) {
        const double* Cp = C + 36 * (size_t)p;
        double amax = 0.0;
        for (int q = 0; q < 36; ++q) {
            if (!std::isfinite(Cp[q]))
                return fail(nullptr, ELAS3D_EBADARG, "C of phase " + std::to_string(p) + " is not finite");
            amax = std::max(amax, std::fabs(Cp[q]));
        }
        for (int r = 0; r < 6; ++r)
            for (int c = r + 1; c < 6; ++c)
                if (std::fabs(Cp[6 * r + c] - Cp[6 * c + r]) > 1e-12 * amax)
                    return fail(nullptr, ELAS3D_EBADARG,
                                "C of phase " + std::to_string(p) + " is not symmetric");
    }
    for (int q = 0; q < 6 * nrhs; ++q)
        if (!std::isfinite(strain[q])) return fail(nullptr, ELAS3D_EBADARG, "strain is not finite");
    if (!o->inputs_on_device) {
        for (int64_t m = 0; m < n; ++m)
            if (phase[m] < 0 || phase[m] >= nphase)
                return fail(nullptr, ELAS3D_EBADARG,
                            "phase id out of range at voxel " + std::to_string(m));
    }
    return 0;
}

void free_ctx(elas3d_ctx* c)
{
    if (!c) return;
    if (c->stream) hipStreamSynchronize(c->stream);
    for (void* p : {(void*)c->phase, (void*)c->coef, (void*)c->diag, (void*)c->solid, (void*)c->sig,
                    (void*)c->bundle64, (void*)c->midx, (void*)c->minv, (void*)c->partials,
                    (void*)c->norms, (void*)c->dscratch, (void*)c->dflag, (void*)c->S,
                    (void*)c->bundle32, (void*)c->minv32, (void*)c->coef32})
        if (p) hipFree(p);
    if (c->hS) hipHostFree(c->hS);
    if (c->hscratch) hipHostFree(c->hscratch);
    for (auto& e : c->wsd) {
        if (e.dict) hipFree(e.dict);
        if (e.map) hipFree(e.map);
    }
    for (auto& g : c->graphs) {
        hipGraphExecDestroy(g.exec);
        hipGraphDestroy(g.graph);
    }
    for (auto& e : c->ev_op) {
        hipEventDestroy(e.a);
        hipEventDestroy(e.b);
    }
    for (auto& e : c->ev_up) {
        hipEventDestroy(e.a);
        hipEventDestroy(e.b);
    }
    if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
    delete c;
}

int ensure_events(elas3d_ctx* c, std::vector<EventPair>& pool, size_t count)
{
    while (pool.size() < count) {
        EventPair e;
        HIPCHK(c, hipEventCreate(&e.a));
        HIPCHK(c, hipEventCreate(&e.b));
        pool.push_back(e);
    }
    return 0;
}

// Copy a device field of ncomp planes (ncomp*N doubles) to the caller's
// buffer: device memory when outputs_on_device, else host memory.
int export_field(elas3d_ctx* c, const double* field, int ncomp, double* out)
{
    const size_t bytes = 8 * (size_t)ncomp * c->N();
    HIPCHK(c, hipMemcpyAsync(out, field, bytes,
                             c->opt.outputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return 0;
}

// Builds (once per geometry) the phase dictionaries of the wave-specialised
// geometry g; fits is false when some workgroup box of g holds more than
// kWsDict distinct phases (nothing is kept then).  Other geometries: fits.
int ws_prepare(elas3d_ctx* c, const e3d::OpGeom& g, bool& fits)
{
    fits = true;
    if (!e3d::is_ws(g.tile)) return 0;
    for (const auto& e : c->wsd)
        if (e.g.tile == g.tile && e.g.tiles_x == g.tiles_x && e.g.tiles_y == g.tiles_y && e.g.kz == g.kz) {
            fits = e.maxcount <= e3d::kWsDict;
            return 0;
        }
    elas3d_ctx::WsDictEntry e{g, nullptr, nullptr, 0};
    auto drop = [&](hipError_t err) {
        if (e.dict) hipFree(e.dict);
        if (e.map) hipFree(e.map);
        return fail(c, ELAS3D_EDEVICE, std::string("phase dictionaries: ") + hipGetErrorString(err));
    };
    hipError_t err = hipMalloc(&e.dict, sizeof(int32_t) * (size_t)g.blocks * e3d::kWsDict);
    if (err == hipSuccess) err = hipMalloc(&e.map, e3d::ws_map_bytes(g));
    if (err == hipSuccess) err = hipMemsetAsync(c->dflag + 1, 0, sizeof(int), c->stream);
    if (err == hipSuccess) err = e3d::launch_ws_dictionary(c->stream, c->d, g, c->phase, e.dict, e.map, c->dflag + 1);
    if (err == hipSuccess)
        err = hipMemcpyAsync(c->hscratch, c->dflag + 1, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (err == hipSuccess) err = hipStreamSynchronize(c->stream);
    if (err != hipSuccess) return drop(err);
    std::memcpy(&e.maxcount, c->hscratch, sizeof(int));
    if (e.maxcount > e3d::kWsDict) {
        hipFree(e.dict);
        hipFree(e.map);
        e.dict = nullptr;
        e.map = nullptr;
        fits = false;
    }
    c->wsd.push_back(e);
    return 0;
}

// Frees the dictionaries of geometries that neither precision's fused sweep
// nor the residual sweep uses (nor `also`, when given).
void ws_release_unused(elas3d_ctx* c, const e3d::OpGeom* also = nullptr)
{
    auto same = [](const e3d::OpGeom& a, const e3d::OpGeom& b) {
        return a.tile == b.tile && a.tiles_x == b.tiles_x && a.tiles_y == b.tiles_y && a.kz == b.kz;
    };
    std::vector<elas3d_ctx::WsDictEntry> keep;
    for (auto& e : c->wsd) {
        bool used = (also && same(e.g, *also)) || same(e.g, c->geom_apply);
        for (const auto& g : c->geom_sweep) used = used || same(e.g, g);
        if (used) {
            keep.push_back(e);
        } else {
            if (e.dict) hipFree(e.dict);
            if (e.map) hipFree(e.map);
        }
    }
    c->wsd.swap(keep);
}

// Process-wide autotuning results: (device, nx, ny, nz, element size, RHS,
// mode) -> (operator sweep geometry, update grid, update non-temporal);
// mode 2 tunes the update sweep only (its geometry entry is not used).
struct TuneChoice {
    e3d::OpGeom geom;
    int upd_blocks, upd_nt;
};
std::mutex g_tune_mu;
std::map<std::array<int, 7>, TuneChoice> g_tune_cache;

// Time every candidate geometry of the two iteration sweeps on the live
// fields and keep the fastest.  Runs right after the start of a run, where
// lambda = gamma = 0, h_old = 0 and w owes nothing: the operator sweep then
// writes h_new = z (which the first iteration writes again) and Ah and
// leaves w alone, and the update sweep leaves g as it is and rewrites
// z = M^-1 g; no finalize kernel runs, so the scalars are untouched.  (The
// sweeps that also pay w's owed steps, every other iteration, are not
// timed.)  Option autotune = 2 keeps the operator sweep's geometry from
// options.tile / zchunk and times the update sweep's candidates only.
template <typename T>
int autotune(elas3d_ctx* c, const FieldsT<T>& f0, size_t rs, int r0, int R, const e3d::MinvRows<T>& M)
{
    const int pi = sizeof(T) == sizeof(double) ? 0 : 1;
    const bool op_too = c->opt.autotune != 2;
    const std::array<int, 7> key = {c->device, c->d.nx, c->d.ny, c->d.nz, (int)sizeof(T), R, op_too ? 1 : 2};
    bool cached = false;
    TuneChoice choice{};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            cached = true;
            choice = it->second;
        }
    }
    if (cached) {
        // the cache is keyed by the grid, not the phases: a wave-specialised
        // choice is kept only when this microstructure's boxes fit its
        // dictionaries, else this context is tuned afresh (and not cached)
        bool fits = true;
        if (op_too) {
            int rc = ws_prepare(c, choice.geom, fits);
            if (rc) return rc;
        }
        if (fits) {
            if (op_too) c->geom_sweep[pi] = choice.geom;
            c->upd_blocks[pi] = choice.upd_blocks;
            c->upd_nt[pi] = choice.upd_nt;
            c->tuned[pi] = 1;
            ws_release_unused(c);
            return 0;
        }
    }
    const Dims& d = c->d;
    const e3d::Tables t = c->tables();
    Scalars* S0 = c->S + r0;
    hipEvent_t ev[2];
    HIPCHK(c, hipEventCreate(&ev[0]));
    HIPCHK(c, hipEventCreate(&ev[1]));
    auto time_it = [&](auto launch, float& ms) -> int {
        HIPCHK(c, launch());  // warm-up
        HIPCHK(c, hipEventRecord(ev[0], c->stream));
        for (int k = 0; k < 3; ++k) HIPCHK(c, launch());
        HIPCHK(c, hipEventRecord(ev[1], c->stream));
        HIPCHK(c, hipEventSynchronize(ev[1]));
        HIPCHK(c, hipEventElapsedTime(&ms, ev[0], ev[1]));
        return 0;
    };
    int rc = 0;
    float best = 1e30f;
    e3d::OpGeom best_g = c->geom_sweep[pi];
    for (int tile = 0; tile < e3d::kNumTiles && !rc && op_too; ++tile)
        for (int target : kTuneTargets) {
            if (!e3d::ws_supported(d, tile, (int)sizeof(T))) break;  // shape not possible on this grid
            const e3d::OpGeom g = e3d::op_geometry(d, 0, tile, target);
            bool fits = true;
            rc = ws_prepare(c, g, fits);
            if (rc) break;
            if (!fits) continue;  // a box with more phases than a dictionary holds
            const e3d::Tables tg = c->tables_for(g);
            float ms = 0.f;
            rc = time_it([&] {
                return e3d::launch_direction_operator<T>(c->stream, d, g, c->phase, tg, f0, rs, R, S0,
                                                         c->partials, false);
            }, ms);
            if (rc) break;
            if (ms < best) {
                best = ms;
                best_g = g;
            }
            ws_release_unused(c, &best_g);  // at most the best candidate's dictionaries stay
        }
    float best_u = 1e30f;
    int best_nb = c->upd_blocks[pi], best_nt = c->upd_nt[pi];
    for (int nt = 0; nt < 2; ++nt)
        for (int nb : kTuneUpdate) {
            if (rc) break;
            float ms = 0.f;
            rc = time_it([&] {
                return e3d::launch_update_precond<T>(c->stream, d, f0, rs, R, M, S0, c->partials, nb, false,
                                                     nt != 0);
            }, ms);
            if (!rc && ms < best_u) {
                best_u = ms;
                best_nb = nb;
                best_nt = nt;
            }
        }
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
    if (rc) return rc;
    c->geom_sweep[pi] = best_g;
    c->upd_blocks[pi] = best_nb;
    c->upd_nt[pi] = best_nt;
    c->tuned[pi] = 1;
    ws_release_unused(c);
    if (!cached) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = {best_g, best_nb, best_nt};
    }
    return 0;
}

// Geometry of the residual and refinement sweeps (one operator application
// each, FP64): with options.autotune = 1, the fastest of the candidate
// workgroup shapes and z-chunkings on the live grid (cached per process by
// device and grid), timed as y = A x + b, as those sweeps run, with x dense
// stand-in data in the FP64 direction buffer that the first direction sweep
// writes before reading, and y the FP64 operator-output field of case 0 (no
// finalize, so no scalar changes; y is rewritten by the first direction
// sweep); with 2, the forced geometry of options.tile / zchunk
// (64x8 lanes when a wave-specialised box holds more phases than its
// dictionary).  The reduction order of ||y||^2 follows the geometry; y itself
// does not depend on it.
// Cached: the fastest shape and the fastest classic one, the fallback for a
// microstructure whose phases do not fit the wave-specialised dictionaries.
std::map<std::array<int, 4>, std::pair<e3d::OpGeom, e3d::OpGeom>> g_apply_cache;

int autotune_apply(elas3d_ctx* c)
{
    const Dims& d = c->d;
    if (c->opt.autotune == 2) {
        // the forced shape (its phase dictionaries were built at setup; the
        // FP32-only shape leaves these FP64 sweeps on 64x8 lanes)
        c->geom_apply = e3d::op_geometry(d, c->opt.zchunk, e3d::ws_elem_ok(c->opt.tile, 8) ? c->opt.tile : 4);
        if (e3d::is_ws(c->geom_apply.tile)) {
            bool fits = true;
            int rc = ws_prepare(c, c->geom_apply, fits);
            if (rc) return rc;
            if (!fits) c->geom_apply = e3d::op_geometry(d, c->opt.zchunk, 4);
        }
        c->apply_tuned = 1;
        return 0;
    }
    const std::array<int, 4> key = {c->device, d.nx, d.ny, d.nz};
    {
        std::pair<e3d::OpGeom, e3d::OpGeom> hit;
        bool found = false;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_apply_cache.find(key);
            if (it != g_apply_cache.end()) {
                hit = it->second;
                found = true;
            }
        }
        if (found) {
            // a wave-specialised choice needs this microstructure's dictionaries
            bool fits = true;
            int rc = ws_prepare(c, hit.first, fits);
            if (rc) return rc;
            c->geom_apply = fits ? hit.first : hit.second;
            c->apply_tuned = 1;
            return 0;
        }
    }
    Fields f = c->fields(0);
    // h1 is contiguous over its three components
    HIPCHK(c, e3d::launch_tuning_fill(c->stream, f.h1[0], 3 * c->N()));
    const double* x[3] = {f.h1[0], f.h1[1], f.h1[2]};
    double* y[3] = {f.Ah[0], f.Ah[1], f.Ah[2]};
    hipEvent_t ev[2];
    HIPCHK(c, hipEventCreate(&ev[0]));
    HIPCHK(c, hipEventCreate(&ev[1]));
    float best = 1e30f, best_classic = 1e30f;
    e3d::OpGeom best_g = c->geom_apply, best_cg = c->geom_apply;
    int rc = 0;
    for (int tile = 0; tile < e3d::kNumTiles && !rc; ++tile)
        for (int target : kTuneTargets) {
            if (!e3d::ws_supported(d, tile, 8)) break;  // shape not possible on this grid
            const e3d::OpGeom g = e3d::op_geometry(d, 0, tile, target);
            bool fits = true;
            rc = ws_prepare(c, g, fits);
            if (rc) break;
            if (!fits) continue;  // a box with more phases than a dictionary holds
            const e3d::Tables t = c->tables_for(g);
            auto launch = [&] { return e3d::launch_apply(c->stream, d, g, c->phase, t, x, y, f.b, c->partials, nullptr); };
            hipError_t e = launch();  // warm-up
            for (int k = 0; k < 3 && e == hipSuccess; ++k) {
                if (k == 0) e = hipEventRecord(ev[0], c->stream);
                if (e == hipSuccess) e = launch();
            }
            if (e == hipSuccess) e = hipEventRecord(ev[1], c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
            if (e != hipSuccess) {
                rc = fail(c, ELAS3D_EDEVICE, std::string("apply autotuning: ") + hipGetErrorString(e));
                break;
            }
            if (ms < best) {
                best = ms;
                best_g = g;
            }
            if (!e3d::is_ws(tile) && ms < best_classic) {
                best_classic = ms;
                best_cg = g;
            }
            ws_release_unused(c, &best_g);  // at most the best candidate's dictionaries stay
        }
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
    if (rc) return rc;
    c->geom_apply = best_g;
    c->apply_tuned = 1;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_apply_cache[key] = {best_g, best_cg};
    return 0;
}

// Enqueue PCG iterations (direction+operator sweep, update sweep) for the
// batch of R right-hand sides [r0, r0+R) in batches of `poll`, until the
// device has raised the stop flag of every RHS; the host looks at the flags of
// batch k while batch k+1 is already queued.  Optional HIP-event timing of
// every launch that did real work.  Then the steps still owed to w are applied.
template <typename T>
int iterate(elas3d_ctx* c, const FieldsT<T>& f0, size_t rs, int r0, int R, const e3d::MinvRows<T>& M, int maxit,
            elas3d_info* info, RunStats* rs_out)
{
    const Dims& d = c->d;
    const int poll = c->opt.poll_interval > 0 ? c->opt.poll_interval : kDefaultPoll;
    const bool timing = c->opt.timing != 0;
    const int pi = sizeof(T) == sizeof(double) ? 0 : 1;
    if (c->opt.autotune && !c->tuned[pi]) {
        int rc = autotune<T>(c, f0, rs, r0, R, M);
        if (rc) return rc;
    }
    const e3d::OpGeom geom = c->geom_sweep[pi];
    const e3d::Tables t = c->tables_for(geom);
    const int upd_blocks = c->upd_blocks[pi];
    const bool upd_nt = c->upd_nt[pi] != 0;
    Scalars* S0 = c->S + r0;
    Scalars* h0 = c->hS;                      // slot 0
    Scalars* h1 = c->hS + e3d::kMaxRhs;       // slot 1
    auto all_done = [&](const Scalars* h) {
        for (int r = 0; r < R; ++r)
            if (!h[r].done) return false;
        return true;
    };
    HIPCHK(c, hipMemcpyAsync(h0, S0, R * sizeof(Scalars), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int min_start = maxit;
    for (int r = 0; r < R; ++r) {
        rs_out[r].it_start = h0[r].it;
        if (!h0[r].done) min_start = std::min(min_start, h0[r].it);
    }
    size_t ev_used = 0;
    if (!all_done(h0)) {
        hipEvent_t batch_ev[2] = {nullptr, nullptr};
        HIPCHK(c, hipEventCreateWithFlags(&batch_ev[0], hipEventDisableTiming));
        HIPCHK(c, hipEventCreateWithFlags(&batch_ev[1], hipEventDisableTiming));
        const long long max_launch = (long long)maxit - min_start + poll;
        long long launched = 0;
        bool recorded[2] = {false, false};
        // a captured batch of `poll` iterations (no timing events inside)
        hipGraphExec_t exec = nullptr;
        if (c->opt.graphs && !timing) {
            const int key[3] = {(int)sizeof(T), r0, R};
            for (auto& g : c->graphs)
                if (g.key[0] == key[0] && g.key[1] == key[1] && g.key[2] == key[2]) exec = g.exec;
            if (!exec) {
                elas3d_ctx::GraphEntry ge{{key[0], key[1], key[2]}, nullptr, nullptr};
                HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
                hipError_t e1 = hipSuccess;
                for (int j = 0; j < poll && e1 == hipSuccess; ++j) {
                    e1 = e3d::launch_direction_operator<T>(c->stream, d, geom, c->phase, t, f0, rs, R,
                                                           S0, c->partials);
                    if (e1 == hipSuccess)
                        e1 = e3d::launch_update_precond<T>(c->stream, d, f0, rs, R, M, S0, c->partials,
                                                           upd_blocks, true, upd_nt);
                }
                hipError_t e2 = hipStreamEndCapture(c->stream, &ge.graph);
                if (e1 != hipSuccess || e2 != hipSuccess)
                    return fail(c, ELAS3D_EDEVICE, std::string("graph capture: ") +
                                                       hipGetErrorString(e1 != hipSuccess ? e1 : e2));
                HIPCHK(c, hipGraphInstantiate(&ge.exec, ge.graph, nullptr, nullptr, 0));
                c->graphs.push_back(ge);
                exec = ge.exec;
            }
        }
        auto enqueue = [&](int slot) -> int {
            if (exec) HIPCHK(c, hipGraphLaunch(exec, c->stream));
            for (int j = 0; j < poll && !exec; ++j) {
                if (timing) {
                    int rc = ensure_events(c, c->ev_op, ev_used + 1);
                    if (rc) return rc;
                    rc = ensure_events(c, c->ev_up, ev_used + 1);
                    if (rc) return rc;
                    HIPCHK(c, hipEventRecord(c->ev_op[ev_used].a, c->stream));
                }
                HIPCHK(c, e3d::launch_direction_operator<T>(c->stream, d, geom, c->phase, t, f0, rs,
                                                            R, S0, c->partials));
                if (timing) {
                    HIPCHK(c, hipEventRecord(c->ev_op[ev_used].b, c->stream));
                    HIPCHK(c, hipEventRecord(c->ev_up[ev_used].a, c->stream));
                }
                HIPCHK(c, e3d::launch_update_precond<T>(c->stream, d, f0, rs, R, M, S0, c->partials,
                                                        upd_blocks, true, upd_nt));
                if (timing) {
                    HIPCHK(c, hipEventRecord(c->ev_up[ev_used].b, c->stream));
                    ++ev_used;
                }
            }
            launched += poll;
            HIPCHK(c, hipMemcpyAsync(slot ? h1 : h0, S0, R * sizeof(Scalars), hipMemcpyDeviceToHost,
                                     c->stream));
            HIPCHK(c, hipEventRecord(batch_ev[slot], c->stream));
            recorded[slot] = true;
            return 0;
        };
        int rc = enqueue(0);
        bool stop = false;
        int k = 0;
        while (!rc && !stop) {
            const int slot = k & 1;
            if (launched < max_launch) rc = enqueue(slot ^ 1);
            if (rc) break;
            hipError_t e = hipEventSynchronize(batch_ev[slot]);
            if (e != hipSuccess) {
                rc = fail(c, ELAS3D_EDEVICE, std::string("hipEventSynchronize: ") + hipGetErrorString(e));
                break;
            }
            if (all_done(slot ? h1 : h0)) stop = true;
            if (!stop && launched >= max_launch) {
                // the last batch is in flight: wait for it
                e = recorded[slot ^ 1] ? hipEventSynchronize(batch_ev[slot ^ 1]) : hipSuccess;
                if (e != hipSuccess) {
                    rc = fail(c, ELAS3D_EDEVICE, std::string("hipEventSynchronize: ") + hipGetErrorString(e));
                    break;
                }
                stop = true;
            }
            ++k;
        }
        hipStreamSynchronize(c->stream);
        hipEventDestroy(batch_ev[0]);
        hipEventDestroy(batch_ev[1]);
        if (rc) return rc;
    }
    for (int r = 0; r < R; ++r)
        HIPCHK(c, e3d::launch_final_update<T>(c->stream, d, e3d::shifted(f0, (size_t)r * rs), S0 + r));
    HIPCHK(c, hipMemcpyAsync(h0, S0, R * sizeof(Scalars), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int real = 0;  // launches before the last RHS of the batch stopped
    for (int r = 0; r < R; ++r) {
        rs_out[r].fin = h0[r];
        real = std::max(real, h0[r].it - rs_out[r].it_start);
    }
    if (timing && info) {
        for (int q = 0; q < real && q < (int)ev_used; ++q) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, c->ev_op[q].a, c->ev_op[q].b) == hipSuccess) {
                info->t_operator_ms += ms;
                info->n_operator += 1;
            }
            if (hipEventElapsedTime(&ms, c->ev_up[q].a, c->ev_up[q].b) == hipSuccess) {
                info->t_update_ms += ms;
                info->n_update += 1;
            }
        }
    }
    return 0;
}

// Start a PCG run of RHS r: load tol/maxit/mode and the iteration counter
// into its device scalars, then the init sweep (fresh: w = 0, g = b;
// otherwise g already holds the residual to continue from).
template <typename T>
int start_run(elas3d_ctx* c, int r, const FieldsT<T>& f, const e3d::MinvRows<T>& M, double tol, int maxit,
              int mode, int it0, int fresh, int from_residual, const double* norms2)
{
    Scalars init{};
    init.tol = tol;
    init.maxit = maxit;
    init.mode = mode;
    init.it = it0;
    // pinned staging slot r: nothing else writes it before the stream passes
    // this copy (every caller synchronises before the next start of RHS r)
    std::memcpy(&c->hS[r], &init, sizeof(Scalars));
    HIPCHK(c, hipMemcpyAsync(c->S + r, &c->hS[r], sizeof(Scalars), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, e3d::launch_pcg_init<T>(c->stream, c->d, f, M, fresh, from_residual, c->S + r,
                                      c->partials, kSweepBlocks, norms2));
    return 0;
}

template int start_run<double>(elas3d_ctx*, int, const FieldsT<double>&, const e3d::MinvRows<double>&, double, int, int,
                               int, int, int, const double*);
template int start_run<float>(elas3d_ctx*, int, const FieldsT<float>&, const e3d::MinvRows<float>&, double, int, int, int,
                              int, int, const double*);

// Mark RHS r of the next batch as finished (its sweeps return at once).
int park(elas3d_ctx* c, int r, const Scalars& fin)
{
    Scalars q = fin;
    q.done = 1;
    q.pending = 0;
    std::memcpy(&c->hS[r], &q, sizeof(Scalars));  // staging slot r, as start_run
    HIPCHK(c, hipMemcpyAsync(c->S + r, &c->hS[r], sizeof(Scalars), hipMemcpyHostToDevice, c->stream));
    return 0;
}

// FP64 PCG (Algorithm 2) on the RHS [r0, r0+R) in lockstep (R = 1 unless the
// context is batched), from w = 0, or continuing from the current w when
// `cont` (g = A w + b already in place).  In residual mode every RHS whose
// recursive and true residual disagree restarts from its w.
int solve_fp64(elas3d_ctx* c, int r0, int R, double tol, int maxit, bool cont, int it0,
               elas3d_info* info, CaseResult* res)
{
    const e3d::MinvRows<double> M = c->minv_rows();
    const e3d::Tables t = c->tables();
    std::vector<int> running(R, 1);
    for (int q = 0; q < R; ++q) {
        int rc = start_run<double>(c, r0 + q, c->fields(r0 + q), M, tol, maxit, c->opt.convergence, it0,
                                   cont ? 0 : 1, cont ? 1 : 0, c->norms + 2 * (r0 + q));
        if (rc) return rc;
    }
    std::vector<RunStats> rs(R);
    for (;;) {
        int rc = iterate<double>(c, c->fields(r0), c->rs64(), r0, R, M, maxit, info, rs.data());
        if (rc) return rc;
        bool again = false;
        for (int q = 0; q < R; ++q) {
            if (!running[q]) continue;
            Fields f = c->fields(r0 + q);
            // true residual r = A w + b (into g, ready for a restart)
            double rr = 0.0;
            rc = true_residual(c, r0 + q, &rr);
            if (rc) return rc;
            CaseResult& cr = res[q];
            cr.fin = rs[q].fin;
            const bool zero_load = cr.fin.bnorm2 <= 1e-28 * cr.fin.bref2;
            cr.rel_true = (zero_load || cr.fin.bnorm2 <= 0.0) ? 0.0 : std::sqrt(rr / cr.fin.bnorm2);
            if (c->opt.convergence == ELAS3D_CONV_RESIDUAL && cr.fin.status == 0 && !zero_load &&
                !(cr.rel_true <= tol)) {
                if (cr.fin.it >= maxit) {
                    cr.fin.status = 1;
                    running[q] = 0;
                    continue;
                }
                ++cr.restarts;
                rc = start_run<double>(c, r0 + q, f, M, tol, maxit, c->opt.convergence, cr.fin.it, 0, 1,
                                       c->norms + 2 * (r0 + q));
                if (rc) return rc;
                again = true;
            } else {
                running[q] = 0;
            }
        }
        if (!again) break;
        // RHS that are finished keep their raised stop flags
    }
    return 0;
}

int refine_launch(elas3d_ctx* c, int r, int q)
{
    Fields f64 = c->fields(r);
    e3d::FieldsT<float> f32 = c->fields32(r);
    double* w[3] = {f64.w[0], f64.w[1], f64.w[2]};
    const float* dc[3] = {f32.w[0], f32.w[1], f32.w[2]};
    float* r32[3] = {f32.g[0], f32.g[1], f32.g[2]};
    HIPCHK(c, e3d::launch_refine(c->stream, c->d, c->geom_apply, c->phase, c->tables_for(c->geom_apply), w, dc, f64.b, r32,
                                 c->partials, c->dscratch + 4 + 2 * q));
    // {||r||^2, ||r||^2}: the norms of the next inner run
    HIPCHK(c, hipMemcpyAsync(c->dscratch + 5 + 2 * q, c->dscratch + 4 + 2 * q, sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
    return 0;
}

int residual_launch(elas3d_ctx* c, int r, double* norm2)
{
    Fields f = c->fields(r);
    const double* wx[3] = {f.w[0], f.w[1], f.w[2]};
    double* gy[3] = {f.g[0], f.g[1], f.g[2]};
    HIPCHK(c, e3d::launch_apply(c->stream, c->d, c->geom_apply, c->phase, c->tables_for(c->geom_apply), wx, gy, f.b, c->partials,
                                norm2));
    return 0;
}

int refine_step(elas3d_ctx* c, int r, int q, double bnorm2, double* rel)
{
    int rc = refine_launch(c, r, q);
    if (rc) return rc;
    HIPCHK(c, hipMemcpyAsync(c->hscratch, c->dscratch + 4 + 2 * q, sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *rel = std::sqrt(c->hscratch[0] / bnorm2);
    return 0;
}

int true_residual(elas3d_ctx* c, int r, double* rr)
{
    Fields f = c->fields(r);
    const double* wx[3] = {f.w[0], f.w[1], f.w[2]};
    double* gy[3] = {f.g[0], f.g[1], f.g[2]};
    HIPCHK(c, e3d::launch_apply(c->stream, c->d, c->geom_apply, c->phase, c->tables_for(c->geom_apply), wx, gy, f.b, c->partials,
                                c->dscratch));
    HIPCHK(c, hipMemcpyAsync(c->hscratch, c->dscratch, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *rr = c->hscratch[0];
    return 0;
}

// Mixed precision (iterative refinement) on the RHS [r0, r0+R): the
// corrections d of A d = -r are solved by the FP32 PCG in lockstep to a
// relative reduction of the inner tolerance, then for each RHS w += d and
// r = A w + b are formed in FP64.  A RHS whose cycle does not halve its true
// residual continues in FP64 PCG from its w.
int solve_mixed(elas3d_ctx* c, int r0, int R, double tol, int maxit, elas3d_info* info,
                CaseResult* res)
{
    const Dims& d = c->d;
    const e3d::MinvRows<float> M32 = c->minv32_rows();
    const e3d::Tables t = c->tables();
    const double inner_tol = c->opt.inner_tol > 0.0 ? c->opt.inner_tol : 1e-4;
    std::vector<double> bnorm2(R), bref2(R), rel(R);
    std::vector<int> iters(R, 0), active(R, 0), fallback(R, 0);
    auto refine = [&](int q) -> int { return refine_step(c, r0 + q, q, bnorm2[q], &rel[q]); };
    for (int q = 0; q < R; ++q) {
        const int r = r0 + q;
        Fields f64 = c->fields(r);
        e3d::FieldsT<float> f32 = c->fields32(r);
        // w = 0, d = 0 (each field is 3N contiguous elements from component 0)
        HIPCHK(c, hipMemsetAsync(f64.w[0], 0, sizeof(double) * 3 * c->N(), c->stream));
        HIPCHK(c, hipMemsetAsync(f32.w[0], 0, sizeof(float) * 3 * c->N(), c->stream));
        HIPCHK(c, hipMemcpyAsync(c->hscratch + 2, c->norms + 2 * r, 2 * sizeof(double),
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        bnorm2[q] = c->hscratch[2];
        bref2[q] = c->hscratch[3];
        res[q] = CaseResult{};
        res[q].fin.bnorm2 = bnorm2[q];
        res[q].fin.bref2 = bref2[q];
        if (bnorm2[q] <= 1e-28 * bref2[q]) {  // zero load: converged
            res[q].fin.status = 0;
            continue;
        }
        int rc = refine(q);  // r = b, rounded
        if (rc) return rc;
        active[q] = rel[q] > tol;
        if (!active[q]) res[q].fin.status = 0;
    }
    std::vector<RunStats> rs(R);
    for (;;) {
        bool any = false;
        for (int q = 0; q < R; ++q)
            if (active[q] && iters[q] < maxit) any = true;
        if (!any) break;
        for (int q = 0; q < R; ++q) {
            const int r = r0 + q;
            if (active[q] && iters[q] < maxit) {
                // inner FP32 PCG from d = 0 on g = r (rounded); relative target:
                // the cycle's, not tighter than the outer tolerance needs
                const double target = std::max(inner_tol, 0.5 * tol / rel[q]);
                int rc = start_run<float>(c, r, c->fields32(r), M32, target, maxit - iters[q],
                                          ELAS3D_CONV_RESIDUAL, 0, 1, 1, c->dscratch + 4 + 2 * q);
                if (rc) return rc;
            } else {
                int rc = park(c, r, Scalars{});
                if (rc) return rc;
            }
        }
        int rc = iterate<float>(c, c->fields32(r0), c->rs32(), r0, R, M32, maxit, info, rs.data());
        if (rc) return rc;
        for (int q = 0; q < R; ++q) {
            if (!(active[q] && iters[q] < maxit)) continue;
            iters[q] += rs[q].fin.it;
            ++res[q].restarts;
            const double prev = rel[q];
            rc = refine(q);  // w += d, r = A w + b
            if (rc) return rc;
            res[q].fin.rr = rs[q].fin.rr;
            res[q].fin.gg = rs[q].fin.gg;
            res[q].fin.gg0 = rs[q].fin.gg0;
            if (rel[q] <= tol) {
                active[q] = 0;
            } else if (rs[q].fin.status == 2 || !(rel[q] < 0.5 * prev)) {
                active[q] = 0;  // stagnation or breakdown of the FP32 solve
                fallback[q] = 1;
            }
        }
    }
    for (int q = 0; q < R; ++q) {
        const int r = r0 + q;
        res[q].fin.it = iters[q];
        res[q].rel_true = (bnorm2[q] <= 1e-28 * bref2[q]) ? 0.0 : rel[q];
        res[q].fin.status = res[q].rel_true <= tol ? 0 : 1;
        if (!fallback[q]) continue;
        // finish in FP64 from w: g = A w + b, then PCG continuing the count
        Fields f = c->fields(r);
        const double* wx[3] = {f.w[0], f.w[1], f.w[2]};
        double* gy[3] = {f.g[0], f.g[1], f.g[2]};
        HIPCHK(c, e3d::launch_apply(c->stream, d, c->geom_apply, c->phase, c->tables_for(c->geom_apply), wx, gy,
                                    f.b, c->partials, c->dscratch));
        CaseResult fr;
        int rc = solve_fp64(c, r, 1, tol, maxit, true, iters[q], info, &fr);
        if (rc) return rc;
        const int cycles = res[q].restarts;
        res[q] = fr;
        res[q].restarts += cycles;
        res[q].fallback = 1;
    }
    return 0;
}

// Solve RHS [r0, r0+R) and record per-RHS statistics.
int solve_batch(elas3d_ctx* c, int r0, int R, double tol, int maxit, elas3d_info* info)
{
    CaseResult res[e3d::kMaxRhs];
    int rc;
    if (c->opt.precision == ELAS3D_PREC_MIXED)
        rc = solve_mixed(c, r0, R, tol, maxit, info, res);
    else
        rc = solve_fp64(c, r0, R, tol, maxit, false, 0, info, res);
    if (rc) return rc;
    return record_results(c, r0, R, res, info);
}

int record_results(elas3d_ctx* c, int r0, int R, const CaseResult* res, elas3d_info* info)
{
    int worst = 0;
    for (int q = 0; q < R; ++q) {
        const int r = r0 + q;
        const Scalars& fin = res[q].fin;
        if (info) {
            const bool zero_load = fin.bnorm2 <= 1e-28 * fin.bref2;
            info->status[r] = fin.status;
            info->iters[r] = fin.it;
            info->restarts[r] = res[q].restarts;
            info->relres_true[r] = res[q].rel_true;
            info->relres_recursive[r] =
                (zero_load || fin.bnorm2 <= 0) ? 0.0 : std::sqrt(fin.rr / fin.bnorm2);
            info->relres_precond[r] =
                (zero_load || fin.gg0 <= 0) ? 0.0 : std::sqrt(std::fabs(fin.gg / fin.gg0));
            info->fp64_fallback[r] = res[q].fallback;
            const int pi = c->opt.precision == ELAS3D_PREC_MIXED ? 1 : 0;
            const e3d::OpGeom& g = c->geom_sweep[pi];
            info->op_tile[0] = e3d::kTileShapes[g.tile].tx;
            info->op_tile[1] = e3d::kTileShapes[g.tile].ty;
            info->op_tile[2] = g.kz;
            info->update_blocks = c->upd_blocks[pi];
            info->update_nontemporal = c->upd_nt[pi];
            info->apply_tile[0] = e3d::kTileShapes[c->geom_apply.tile].tx;
            info->apply_tile[1] = e3d::kTileShapes[c->geom_apply.tile].ty;
            info->apply_tile[2] = c->geom_apply.kz;
            info->op_shape = g.tile;
        }
        c->solved[r] = 1;
        worst = std::max(worst, fin.status);
    }
    return worst;
}

// Two fused sweeps per iteration: direction+operator (read z, h_old, phase;
// write h_new, Ah; every other iteration also read w and the older h and
// write w) and update+precondition (read g, Ah, the M^-1 row index and the
// rows of phase-boundary nodes; write g, z).  Per RHS: the fused sweep moves
// 5.5 vectors + phase on average, the update 4 vectors; M^-1 once per node
// for a batch (the nphase shared rows stay in cache).
void iteration_bytes(const elas3d_ctx* c, int nrhs, elas3d_info* info)
{
    const int rb = c->batched() ? nrhs : 1;
    const double N = (double)c->N();
    const double nbnd = (double)(c->mrows - (size_t)c->nphase);
    info->precond_rows = (int64_t)c->mrows;
    if (c->opt.precision == ELAS3D_PREC_MIXED)
        info->bytes_per_iter = N * rb * ((5.5 * 12.0 + 4.0) + 4 * 12.0) + 4.0 * N + 24.0 * nbnd;
    else
        info->bytes_per_iter = N * rb * ((5.5 * 24.0 + 4.0) + 4 * 24.0) + 4.0 * N + 48.0 * nbnd;
}

// Per-context entry points that use the context's stream or work area
// refuse it while a group runs it.
int grouped(elas3d_ctx* c)
{
    return c->group ? fail(c, ELAS3D_EORDER, "context is a member of a group") : 0;
}

}  // namespace e3d::rt

extern "C" {

void elas3d_options_init(elas3d_options* opt)
{
    if (opt) default_options(opt);
}

const char* elas3d_version(void) { return "elas3d-mi355x 0.1 (gfx950)"; }

const char* elas3d_last_error(const elas3d_ctx* ctx)
{
    if (ctx) return ctx->err.c_str();
    return g_last_error.c_str();
}

double elas3d_device_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t nphase, int32_t nrhs,
                           const elas3d_options* opt)
{
    // the size checks of elas3d_setup
    if (nx < 2 || ny < 2 || nz < 2 || 3 * (int64_t)nx * ny * nz >= ((int64_t)1 << 31) || nphase < 1 ||
        nrhs < 1 || nrhs > ELAS3D_MAX_RHS)
        return 0.0;
    const bool valid_geom = opt && opt->tile >= 0 && opt->tile < e3d::kNumTiles && opt->zchunk >= 0;
    return plan_bytes(nx, ny, nz, nphase, nrhs, opt && opt->precision == ELAS3D_PREC_MIXED,
                      opt && opt->batched, valid_geom ? opt->tile : 0, valid_geom ? opt->zchunk : 0);
}

int elas3d_setup(elas3d_ctx** out, int32_t nx, int32_t ny, int32_t nz, const int32_t* phase,
                 int32_t nphase, const double* C, int32_t nrhs, const double* strain,
                 const elas3d_options* opt_in)
{
    if (!out) return fail(nullptr, ELAS3D_EBADARG, "out is NULL");
    *out = nullptr;
    elas3d_options opt;
    if (opt_in)
        opt = *opt_in;
    else
        default_options(&opt);
    int rc = validate_setup(nx, ny, nz, phase, nphase, C, nrhs, strain, &opt);
    if (rc) return rc;

    auto t0 = std::chrono::steady_clock::now();
    // ---- device calls start here
    int dev = opt.device;
    if (dev >= 0) {
        hipError_t e = hipSetDevice(dev);
        if (e != hipSuccess) return fail(nullptr, ELAS3D_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    } else {
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return fail(nullptr, ELAS3D_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    const int64_t n = (int64_t)nx * ny * nz;
    const bool mixed = opt.precision == ELAS3D_PREC_MIXED;
    const double need = plan_bytes(nx, ny, nz, nphase, nrhs, mixed, opt.batched != 0, opt.tile, opt.zchunk);
    double budget = opt.hbm_budget_bytes;
    if (budget <= 0.0) {
        size_t free_b = 0, total_b = 0;
        hipError_t e = hipMemGetInfo(&free_b, &total_b);
        if (e != hipSuccess) return fail(nullptr, ELAS3D_EDEVICE, std::string("hipMemGetInfo: ") + hipGetErrorString(e));
        budget = 0.95 * (double)free_b;
    }
    if (need > budget) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "needs %.3f GB of device memory, budget is %.3f GB", need / 1e9,
                      budget / 1e9);
        return fail(nullptr, ELAS3D_ENOMEM, buf);
    }

    elas3d_ctx* c = new elas3d_ctx();
    c->device = dev;
    c->opt = opt;
    c->d = Dims{nx, ny, nz, (int)n};
    c->nphase = nphase;
    c->nrhs = nrhs;
    c->strain.assign(strain, strain + 6 * nrhs);
    c->solved.assign(nrhs, 0);
    c->bytes = need;
    c->geom = e3d::op_geometry(c->d, 0);
    c->geom_apply = c->geom;
    for (int q = 0; q < 2; ++q) {
        // a forced FP32-only shape leaves the FP64 sweep (the fallback of a
        // stalled refinement) on 64x8 lanes
        c->geom_sweep[q] = e3d::op_geometry(c->d, opt.zchunk, e3d::ws_elem_ok(opt.tile, q ? 4 : 8) ? opt.tile : 4);
        c->upd_blocks[q] = opt.update_blocks > 0 ? opt.update_blocks : default_update_blocks(c->d.n);
        c->upd_nt[q] = opt.update_nontemporal;
    }
    {
        const long long slots = partial_slots(c->d, nrhs, opt.tile, opt.zchunk);
        if (slots >= (1LL << 31) / kPartialValues) {
            free_ctx(c);
            return fail(nullptr, ELAS3D_EBADARG, "options.zchunk gives too many workgroups");
        }
        c->partial_stride = (int)slots;
    }

    auto bail = [&](hipError_t e, const char* what) {
        std::string m = std::string(what) + ": " + hipGetErrorString(e);
        free_ctx(c);
        return fail(nullptr, ELAS3D_EDEVICE, m);
    };
#define SETUPCHK(expr)                          \
    do {                                        \
        hipError_t e_ = (expr);                 \
        if (e_ != hipSuccess) return bail(e_, #expr); \
    } while (0)

    if (opt.stream) {
        c->stream = (hipStream_t)opt.stream;
    } else {
        SETUPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    const size_t N = (size_t)n;
    SETUPCHK(hipMalloc(&c->phase, 4 * N));
    SETUPCHK(hipMalloc(&c->coef, 8 * (size_t)nphase * e3d::kCoefStride));
    SETUPCHK(hipMalloc(&c->diag, 8 * (size_t)nphase * e3d::kDiagStride));
    SETUPCHK(hipMalloc(&c->solid, (size_t)nphase));
    SETUPCHK(hipMalloc(&c->sig, 8 * (size_t)nrhs * nphase * e3d::kSigStride));
    SETUPCHK(hipMalloc(&c->bundle64, 8 * N * (opt.batched ? 21 * (size_t)nrhs : 6 * (size_t)nrhs + 15)));
    SETUPCHK(hipMalloc(&c->midx, 4 * N));
    if (mixed) {
        SETUPCHK(hipMalloc(&c->bundle32, 4 * 18 * N * (opt.batched ? (size_t)nrhs : 1)));
        SETUPCHK(hipMalloc(&c->coef32, 4 * (size_t)nphase * e3d::kCoefStride));
    }
    SETUPCHK(hipMalloc(&c->partials, 8 * (size_t)kPartialValues * c->partial_stride));
    SETUPCHK(hipMalloc(&c->norms, 8 * 2 * (size_t)nrhs));
    SETUPCHK(hipMalloc(&c->dscratch, 8 * 64));
    SETUPCHK(hipMalloc(&c->dflag, sizeof(int) * 4));
    SETUPCHK(hipMalloc(&c->S, e3d::kMaxRhs * sizeof(Scalars)));
    SETUPCHK(hipHostMalloc(&c->hS, 2 * e3d::kMaxRhs * sizeof(Scalars), hipHostMallocDefault));
    SETUPCHK(hipHostMalloc(&c->hscratch, 64 * sizeof(double), hipHostMallocDefault));

    SETUPCHK(hipMemcpyAsync(c->phase, phase, 4 * N,
                            opt.inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                            c->stream));
    if (opt.inputs_on_device) {
        SETUPCHK(hipMemsetAsync(c->dflag, 0, sizeof(int), c->stream));
        SETUPCHK(e3d::launch_phase_check(c->stream, c->phase, (int)n, nphase, c->dflag));
        int bad = 0;
        SETUPCHK(hipMemcpyAsync(&bad, c->dflag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        SETUPCHK(hipStreamSynchronize(c->stream));
        if (bad) {
            free_ctx(c);
            return fail(nullptr, ELAS3D_EBADARG, std::to_string(bad) + " phase ids out of range");
        }
    }
    std::vector<double> coef, diag, sig;
    std::vector<uint8_t> solid;
    build_tables(C, nphase, strain, nrhs, coef, diag, solid, sig);
    SETUPCHK(hipMemcpyAsync(c->coef, coef.data(), 8 * coef.size(), hipMemcpyHostToDevice, c->stream));
    std::vector<float> coef32;
    if (mixed) {
        coef32.assign(coef.begin(), coef.end());  // rounded to FP32
        SETUPCHK(hipMemcpyAsync(c->coef32, coef32.data(), 4 * coef32.size(), hipMemcpyHostToDevice,
                                c->stream));
    }
    SETUPCHK(hipMemcpyAsync(c->diag, diag.data(), 8 * diag.size(), hipMemcpyHostToDevice, c->stream));
    SETUPCHK(hipMemcpyAsync(c->solid, solid.data(), solid.size(), hipMemcpyHostToDevice, c->stream));
    SETUPCHK(hipMemcpyAsync(c->sig, sig.data(), 8 * sig.size(), hipMemcpyHostToDevice, c->stream));
    for (int r = 0; r < nrhs; ++r) {
        double* bp[3] = {c->comp(c->bptr(r), 0), c->comp(c->bptr(r), 1), c->comp(c->bptr(r), 2)};
        SETUPCHK(e3d::launch_load(c->stream, c->d, c->phase,
                                  c->sig + (size_t)r * nphase * e3d::kSigStride, bp, c->partials,
                                  c->norms + 2 * r, kSweepBlocks));
    }
    // M^-1 as a dictionary: count the phase-boundary nodes of each chunk (in
    // the partial-sum buffer), lay their rows out after the nphase shared
    // ones, then fill the rows and every node's row index
    {
        const int identity = opt.preconditioner == ELAS3D_PRECOND_NONE ? 1 : 0;
        const size_t nchunks = (N + e3d::kPrecondChunk - 1) / e3d::kPrecondChunk;
        if (nchunks > 2 * (size_t)kPartialValues * c->partial_stride) {
            free_ctx(c);
            return fail(nullptr, ELAS3D_EDEVICE, "preconditioner chunk table exceeds the partial-sum buffer");
        }
        int* chunk = reinterpret_cast<int*>(c->partials);
        SETUPCHK(e3d::launch_precond_count(c->stream, c->d, c->phase, chunk));
        std::vector<int> cnt(nchunks);
        SETUPCHK(hipMemcpyAsync(cnt.data(), chunk, sizeof(int) * nchunks, hipMemcpyDeviceToHost, c->stream));
        SETUPCHK(hipStreamSynchronize(c->stream));
        size_t nb = 0;
        for (size_t q = 0; q < nchunks; ++q) {
            const int v = cnt[q];
            cnt[q] = (int)nb;
            nb += (size_t)v;
        }
        c->mrows = (size_t)nphase + nb;
        SETUPCHK(hipMemcpyAsync(chunk, cnt.data(), sizeof(int) * nchunks, hipMemcpyHostToDevice, c->stream));
        SETUPCHK(hipMalloc(&c->minv, 8 * 6 * c->mrows));
        if (mixed) SETUPCHK(hipMalloc(&c->minv32, 4 * 6 * c->mrows));
        const e3d::MinvRows<double> M = c->minv_rows();
        SETUPCHK(e3d::launch_precond_table(c->stream, nphase, c->tables(), identity, M.m));
        SETUPCHK(e3d::launch_precond_fill(c->stream, c->d, c->phase, c->tables(), identity, nphase, chunk,
                                          c->midx, M.m));
        // mixed: the blocks are inverted in FP64 and stored rounded to FP32
        if (mixed) SETUPCHK(e3d::launch_to_float(c->stream, c->minv, c->minv32, 6 * c->mrows));
        SETUPCHK(hipStreamSynchronize(c->stream));  // (cnt is read by the copy)
    }
    // (host input arrays must not be read after return)
    SETUPCHK(hipStreamSynchronize(c->stream));
    if (opt.autotune != 1 && e3d::is_ws(opt.tile)) {
        // the forced wave-specialised shape: its phase dictionaries (the
        // sweep of the precision that runs it)
        bool fits = true;
        int rc2 = ws_prepare(c, c->geom_sweep[e3d::is_ws(c->geom_sweep[0].tile) ? 0 : 1], fits);
        if (!rc2 && !fits) {
            free_ctx(c);
            return fail(nullptr, ELAS3D_EBADARG,
                        "options.tile " + std::to_string(opt.tile) + ": a workgroup box holds more than " +
                            std::to_string(e3d::kWsDict) +
                            " distinct phases; a shorter options.zchunk or another tile");
        }
        if (rc2) {
            std::string m = c->err;
            free_ctx(c);
            return fail(nullptr, rc2, m);
        }
    }
    (void)t0;
#undef SETUPCHK
    *out = c;
    return 0;
}

int elas3d_solve(elas3d_ctx* ctx, double tol, int32_t maxit, int32_t nrhs, elas3d_info* info)
{
    if (!ctx) return fail(nullptr, ELAS3D_EBADARG, "ctx is NULL");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(ctx, ELAS3D_EBADARG, "tol must be finite and >= 0");
    if (maxit < 0) return fail(ctx, ELAS3D_EBADARG, "maxit must be >= 0");
    if (nrhs < 1 || nrhs > ctx->nrhs)
        return fail(ctx, ELAS3D_EBADARG, "nrhs must be in [1, nrhs of setup]");
    if (int rc = grouped(ctx)) return rc;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->nrhs = nrhs;
    }
    HIPCHK(ctx, hipSetDevice(ctx->device));
    auto t0 = std::chrono::steady_clock::now();
    if (ctx->opt.autotune && !ctx->apply_tuned) {
        int rc = autotune_apply(ctx);
        if (rc) return rc;
    }
    int worst = 0;
    if (ctx->batched()) {
        int rc = solve_batch(ctx, 0, nrhs, tol, maxit, info);
        if (rc < 0) return rc;
        worst = rc;
    } else {
        for (int r = 0; r < nrhs; ++r) {
            int rc = solve_batch(ctx, r, 1, tol, maxit, info);
            if (rc < 0) return rc;
            worst = std::max(worst, rc);
        }
    }
    auto t1 = std::chrono::steady_clock::now();
    if (info) {
        info->t_solve_s = std::chrono::duration<double>(t1 - t0).count();
        iteration_bytes(ctx, nrhs, info);
    }
    return worst;
}

int elas3d_stress(elas3d_ctx* ctx, int32_t rhs, double* sigma_voxel, double* sigma_avg,
                  double* u_node, double* energy)
{
    if (!ctx) return fail(nullptr, ELAS3D_EBADARG, "ctx is NULL");
    if (int rc = grouped(ctx)) return rc;
    if (rhs < 0 || rhs >= ctx->nrhs) return fail(ctx, ELAS3D_EBADARG, "rhs out of range");
    if (!ctx->solved[rhs]) return fail(ctx, ELAS3D_EORDER, "load case not solved yet");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const size_t N = ctx->N();
    Fields f = ctx->fields(rhs);
    double* sigd[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    if (sigma_voxel) {
        double* base = ctx->opt.outputs_on_device ? sigma_voxel : ctx->work64(0);  // 15N >= 6N
        for (int q = 0; q < 6; ++q) sigd[q] = base + q * N;
    }
    HIPCHK(ctx, e3d::launch_stress(ctx->stream, ctx->d, ctx->phase, ctx->tables(),
                                   ctx->strain.data() + 6 * rhs, f, sigma_voxel ? sigd : nullptr,
                                   ctx->partials, ctx->dscratch, kSweepBlocks));
    if (sigma_voxel && !ctx->opt.outputs_on_device)
        HIPCHK(ctx, hipMemcpyAsync(sigma_voxel, ctx->work64(0), 8 * 6 * N, hipMemcpyDeviceToHost,
                                   ctx->stream));
    if (u_node) {
        double* base = ctx->opt.outputs_on_device ? u_node : ctx->work64(0) + 6 * N;
        double* ud[3] = {base, base + N, base + 2 * N};
        HIPCHK(ctx, e3d::launch_total_displacement(ctx->stream, ctx->d, ctx->strain.data() + 6 * rhs, f, ud));
        if (!ctx->opt.outputs_on_device)
            HIPCHK(ctx, hipMemcpyAsync(u_node, base, 8 * 3 * N, hipMemcpyDeviceToHost, ctx->stream));
    }
    HIPCHK(ctx, hipMemcpyAsync(ctx->hscratch, ctx->dscratch, 8 * 7, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (sigma_avg)
        for (int q = 0; q < 6; ++q) sigma_avg[q] = ctx->hscratch[q] / (double)N;
    if (energy) *energy = ctx->hscratch[6];
    return 0;
}

int elas3d_von_mises(elas3d_ctx* ctx, int32_t rhs, double* vm, double* vm_max, int64_t* argmax)
{
    if (!ctx) return fail(nullptr, ELAS3D_EBADARG, "ctx is NULL");
    if (int rc = grouped(ctx)) return rc;
    if (rhs < 0 || rhs >= ctx->nrhs) return fail(ctx, ELAS3D_EBADARG, "rhs out of range");
    if (!ctx->solved[rhs]) return fail(ctx, ELAS3D_EORDER, "load case not solved yet");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const size_t N = ctx->N();
    double* dvm = vm ? (ctx->opt.outputs_on_device ? vm : ctx->work64(0)) : nullptr;  // 15N >= N
    HIPCHK(ctx, e3d::launch_von_mises(ctx->stream, ctx->d, ctx->phase, ctx->tables(),
                                      ctx->strain.data() + 6 * rhs, ctx->fields(rhs), dvm, ctx->partials,
                                      ctx->dscratch, kSweepBlocks));
    if (vm && !ctx->opt.outputs_on_device)
        HIPCHK(ctx, hipMemcpyAsync(vm, dvm, 8 * N, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(ctx->hscratch, ctx->dscratch, 8 * 2, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (vm_max) *vm_max = ctx->hscratch[0];
    if (argmax) *argmax = (int64_t)ctx->hscratch[1];
    return 0;
}

int elas3d_apply(elas3d_ctx* ctx, const double* x, double* y)
{
    if (!ctx) return fail(nullptr, ELAS3D_EBADARG, "ctx is NULL");
    if (int rc = grouped(ctx)) return rc;
    if (!x || !y) return fail(ctx, ELAS3D_EBADARG, "x or y is NULL");
    const size_t N = ctx->N();
    // the sweep reads x at neighbouring nodes while it writes y
    if (x < y + 3 * N && y < x + 3 * N) return fail(ctx, ELAS3D_EBADARG, "x and y overlap");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    // caller's device buffers directly, or host data staged through the work
    // area (15N): [x | y]
    const double* xd = x;
    double* yd = y;
    if (!ctx->opt.outputs_on_device) {
        double* xs = ctx->work64(0);
        HIPCHK(ctx, hipMemcpyAsync(xs, x, 8 * 3 * N, hipMemcpyHostToDevice, ctx->stream));
        xd = xs;
        yd = xs + 3 * N;
    }
    const double* xp[3] = {ctx->comp(xd, 0), ctx->comp(xd, 1), ctx->comp(xd, 2)};
    double* yp[3] = {ctx->comp(yd, 0), ctx->comp(yd, 1), ctx->comp(yd, 2)};
    HIPCHK(ctx, e3d::launch_apply(ctx->stream, ctx->d, ctx->geom, ctx->phase, ctx->tables(), xp, yp,
                                  nullptr, ctx->partials, nullptr));
    if (!ctx->opt.outputs_on_device)
        HIPCHK(ctx, hipMemcpyAsync(y, yd, 8 * 3 * N, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return 0;
}

int elas3d_get_load(elas3d_ctx* ctx, int32_t rhs, double* b)
{
    if (!ctx) return fail(nullptr, ELAS3D_EBADARG, "ctx is NULL");
    if (int rc = grouped(ctx)) return rc;
    if (rhs < 0 || rhs >= ctx->nrhs || !b) return fail(ctx, ELAS3D_EBADARG, "bad rhs or NULL output");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    return export_field(ctx, ctx->bptr(rhs), 3, b);
}

int elas3d_get_precond(elas3d_ctx* ctx, double* minv)
{
    if (!ctx) return fail(nullptr, ELAS3D_EBADARG, "ctx is NULL");
    if (int rc = grouped(ctx)) return rc;
    if (!minv) return fail(ctx, ELAS3D_EBADARG, "NULL output");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const size_t N = ctx->N();
    double* dst = ctx->opt.outputs_on_device ? minv : ctx->work64(0);
    HIPCHK(ctx, e3d::launch_precond_expand(ctx->stream, ctx->d, ctx->minv_rows(), dst));
    if (!ctx->opt.outputs_on_device)
        HIPCHK(ctx, hipMemcpyAsync(minv, dst, 8 * 6 * N, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return 0;
}

int elas3d_get_solution(elas3d_ctx* ctx, int32_t rhs, double* w)
{
    if (!ctx) return fail(nullptr, ELAS3D_EBADARG, "ctx is NULL");
    if (int rc = grouped(ctx)) return rc;
    if (rhs < 0 || rhs >= ctx->nrhs || !w) return fail(ctx, ELAS3D_EBADARG, "bad rhs or NULL output");
    if (!ctx->solved[rhs]) return fail(ctx, ELAS3D_EORDER, "load case not solved yet");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    return export_field(ctx, ctx->wptr(rhs), 3, w);
}

void elas3d_destroy(elas3d_ctx* ctx)
{
    if (!ctx) return;
    if (ctx->group) group_forget(ctx->group, ctx);
    if (ctx->group_done) group_forget(ctx->group_done, ctx);
    hipSetDevice(ctx->device);
    free_ctx(ctx);
}

}  // extern "C"
