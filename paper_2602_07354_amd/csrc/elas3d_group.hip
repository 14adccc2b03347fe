// Group engine of libelas3d: continuous batching of independent solves.
//
// Every member is a context with its own grid, tables and fields.  The
// members of a precision lane (FP64 PCG, or the FP32 inner PCG of the
// mixed-precision refinement) are advanced in lockstep by one launch per
// sweep over a work list (e3d::group_prepare / launch_group_iteration), so an
// iteration costs four launches for up to 8 requests in flight.  Between
// batches of iterations the host settles the members whose runs ended: the
// same steps elas3d_solve takes (true-residual restarts; refinement cycles;
// FP64 fallback), then members leave and new ones join.  A member's sweeps
// run exactly the workgroups of its own single-context sweep, so its result
// does not depend on the mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "elas3d.h"
#include "elas3d_internal.h"
#include "elas3d_runtime.h"

using namespace e3d::rt;

namespace {

enum State { RUN64 = 0, RUN32 = 1, FINISHED = 2 };

struct Member {
    elas3d_ctx* c = nullptr;
    hipStream_t own_stream = nullptr;  // the context's stream, restored on leaving
    double tol = 0.0;
    int maxit = 0;
    int R = 0;
    bool mixed = false;
    int state = FINISHED;
    std::chrono::steady_clock::time_point t0;
    CaseResult res[e3d::kMaxRhs];
    int running[e3d::kMaxRhs] = {};  // FP64: RHS whose run is not settled
    // mixed precision
    double bnorm2[e3d::kMaxRhs] = {}, bref2[e3d::kMaxRhs] = {}, rel[e3d::kMaxRhs] = {};
    int iters[e3d::kMaxRhs] = {}, active[e3d::kMaxRhs] = {}, fallback[e3d::kMaxRhs] = {};
    int cycles[e3d::kMaxRhs] = {};    // refinement cycles before an FP64 fallback
    int restarts64[e3d::kMaxRhs] = {};  // true-residual restarts of the FP64 runs
};

double inner_tol_of(const elas3d_ctx* c) { return c->opt.inner_tol > 0.0 ? c->opt.inner_tol : 1e-4; }

}  // namespace

struct elas3d_group {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<Member> members;
    std::vector<std::pair<elas3d_ctx*, elas3d_info>> done;
    char* dev[2] = {nullptr, nullptr};
    size_t dev_cap[2] = {0, 0};
    char* staging[2] = {nullptr, nullptr};
    size_t stg_cap[2] = {0, 0};
    e3d::GroupPlan plan[2];
    bool dirty = true;
    Scalars* hS = nullptr;  // pinned, kMaxRhs per member
    size_t hS_cap = 0;
};

namespace {

int gfail(int code, const std::string& msg) { return fail(nullptr, code, msg); }

#define GCHK(expr)                                                                              \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return gfail(ELAS3D_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Propagate a member's context error as the thread's error.
int mfail(Member& m, int rc)
{
    if (rc < 0) gfail(rc, "member: " + m.c->err);
    return rc;
}

// ---- FP64 lane ---------------------------------------------------------

int start64(Member& m, int q, int it0, bool fresh)
{
    elas3d_ctx* c = m.c;
    const e3d::MinvRows<double> M = c->minv_rows();
    return start_run<double>(c, q, c->fields(q), M, m.tol, m.maxit, c->opt.convergence, it0, fresh ? 1 : 0,
                             fresh ? 0 : 1, c->norms + 2 * q);
}

// ---- mixed precision ---------------------------------------------------

// Refinement sweeps (w += d, r = A w + b) of the RHS with want[q], enqueued
// back to back; one read-back of their norms gives rel[q].
int refine_all(Member& m, const int* want)
{
    elas3d_ctx* c = m.c;
    bool any = false;
    for (int q = 0; q < m.R; ++q) {
        if (!want[q]) continue;
        int rc = refine_launch(c, q, q);
        if (rc) return rc;
        any = true;
    }
    if (!any) return 0;
    HIPCHK(c, hipMemcpyAsync(c->hscratch + 16, c->dscratch + 4, 2 * m.R * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int q = 0; q < m.R; ++q)
        if (want[q]) m.rel[q] = std::sqrt(c->hscratch[16 + 2 * q] / m.bnorm2[q]);
    return 0;
}

// Start the next inner FP32 cycle of every active RHS (park the others);
// false when none is left.
int start_cycle(Member& m, bool* any)
{
    elas3d_ctx* c = m.c;
    const e3d::MinvRows<float> M32 = c->minv32_rows();
    *any = false;
    for (int q = 0; q < m.R; ++q) {
        int rc;
        if (m.active[q] && m.iters[q] < m.maxit) {
            const double target = std::max(inner_tol_of(c), 0.5 * m.tol / m.rel[q]);
            rc = start_run<float>(c, q, c->fields32(q), M32, target, m.maxit - m.iters[q], ELAS3D_CONV_RESIDUAL, 0,
                                  1, 1, c->dscratch + 4 + 2 * q);
            *any = true;
        } else {
            rc = park(c, q, Scalars{});
        }
        if (rc) return rc;
    }
    return 0;
}

// All cycles over: final statistics; RHS that stalled go on in FP64 (the
// FP64 lane), the others are final.
int end_mixed(Member& m)
{
    elas3d_ctx* c = m.c;
    bool any_fb = false;
    for (int q = 0; q < m.R; ++q) {
        m.res[q].fin.it = m.iters[q];
        m.res[q].rel_true = (m.bnorm2[q] <= 1e-28 * m.bref2[q]) ? 0.0 : m.rel[q];
        m.res[q].fin.status = m.res[q].rel_true <= m.tol ? 0 : 1;
        m.running[q] = 0;
        if (m.fallback[q]) any_fb = true;
    }
    if (!any_fb) {
        m.state = FINISHED;
        return 0;
    }
    for (int q = 0; q < m.R; ++q) {
        int rc;
        if (m.fallback[q]) {
            double rr;
            rc = true_residual(c, q, &rr);  // g = A w + b: the FP64 run continues from w
            if (!rc) rc = start64(m, q, m.iters[q], false);
            m.cycles[q] = m.res[q].restarts;
            m.running[q] = 1;
        } else {
            rc = park(c, q, m.res[q].fin);
        }
        if (rc) return rc;
    }
    m.state = RUN64;
    return 0;
}

int admit(Member& m)
{
    elas3d_ctx* c = m.c;
    if (!m.mixed) {
        for (int q = 0; q < m.R; ++q) {
            int rc = start64(m, q, 0, true);
            if (rc) return rc;
            m.running[q] = 1;
        }
        m.state = RUN64;
        return 0;
    }
    for (int q = 0; q < m.R; ++q) {  // w = 0, d = 0
        Fields f64 = c->fields(q);
        FieldsT<float> f32 = c->fields32(q);
        HIPCHK(c, hipMemsetAsync(f64.w[0], 0, sizeof(double) * 3 * c->N(), c->stream));
        HIPCHK(c, hipMemsetAsync(f32.w[0], 0, sizeof(float) * 3 * c->N(), c->stream));
    }
    HIPCHK(c, hipMemcpyAsync(c->hscratch + 32, c->norms, 2 * m.R * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int want[e3d::kMaxRhs] = {};
    for (int q = 0; q < m.R; ++q) {
        m.bnorm2[q] = c->hscratch[32 + 2 * q];
        m.bref2[q] = c->hscratch[33 + 2 * q];
        m.res[q] = CaseResult{};
        m.res[q].fin.bnorm2 = m.bnorm2[q];
        m.res[q].fin.bref2 = m.bref2[q];
        if (m.bnorm2[q] <= 1e-28 * m.bref2[q])  // zero load
            m.res[q].fin.status = 0;
        else
            want[q] = 1;
    }
    int rc = refine_all(m, want);  // r = b, rounded
    if (rc) return rc;
    for (int q = 0; q < m.R; ++q) {
        if (!want[q]) continue;
        m.active[q] = m.rel[q] > m.tol;
        if (!m.active[q]) m.res[q].fin.status = 0;
    }
    bool any = false;
    rc = start_cycle(m, &any);
    if (rc) return rc;
    if (any) {
        m.state = RUN32;
        return 0;
    }
    return end_mixed(m);
}

// Settle a member whose lane run ended (every RHS's stop flag is up).
int settle(Member& m, const Scalars* fin)
{
    elas3d_ctx* c = m.c;
    if (m.state == RUN32) {
        for (int q = 0; q < m.R; ++q)
            HIPCHK(c, e3d::launch_final_update<float>(c->stream, c->d, c->fields32(q), c->S + q));
        int want[e3d::kMaxRhs] = {};
        double prev[e3d::kMaxRhs] = {};
        for (int q = 0; q < m.R; ++q) {
            want[q] = m.active[q] && m.iters[q] < m.maxit;
            prev[q] = m.rel[q];
        }
        int rc = refine_all(m, want);  // w += d, r = A w + b
        if (rc) return rc;
        for (int q = 0; q < m.R; ++q) {
            if (!want[q]) continue;
            m.iters[q] += fin[q].it;
            ++m.res[q].restarts;
            m.res[q].fin.rr = fin[q].rr;
            m.res[q].fin.gg = fin[q].gg;
            m.res[q].fin.gg0 = fin[q].gg0;
            if (m.rel[q] <= m.tol) {
                m.active[q] = 0;
            } else if (fin[q].status == 2 || !(m.rel[q] < 0.5 * prev[q])) {
                m.active[q] = 0;  // stagnation or breakdown of the FP32 solve
                m.fallback[q] = 1;
            }
        }
        bool any = false;
        rc = start_cycle(m, &any);
        if (rc) return rc;
        return any ? 0 : end_mixed(m);
    }
    // FP64 lane: apply the step owed to w, check the true residual
    for (int q = 0; q < m.R; ++q)
        HIPCHK(c, e3d::launch_final_update<double>(c->stream, c->d, c->fields(q), c->S + q));
    // true residuals r = A w + b of the settled RHS (into g, ready for a
    // restart), one read-back
    for (int q = 0; q < m.R; ++q) {
        if (!m.running[q]) continue;
        int rc = residual_launch(c, q, c->dscratch + 32 + q);
        if (rc) return rc;
    }
    HIPCHK(c, hipMemcpyAsync(c->hscratch + 32, c->dscratch + 32, m.R * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    bool again = false;
    for (int q = 0; q < m.R; ++q) {
        if (!m.running[q]) continue;
        const double rr = c->hscratch[32 + q];
        int rc = 0;
        CaseResult cr;
        cr.fin = fin[q];
        const bool zero_load = cr.fin.bnorm2 <= 1e-28 * cr.fin.bref2;
        cr.rel_true = (zero_load || cr.fin.bnorm2 <= 0.0) ? 0.0 : std::sqrt(rr / cr.fin.bnorm2);
        if (c->opt.convergence == ELAS3D_CONV_RESIDUAL && cr.fin.status == 0 && !zero_load &&
            !(cr.rel_true <= m.tol)) {
            if (cr.fin.it >= m.maxit) {
                cr.fin.status = 1;
                m.running[q] = 0;
            } else {
                ++m.restarts64[q];
                rc = start64(m, q, cr.fin.it, false);  // restart from w
                if (rc) return rc;
                again = true;
            }
        } else {
            m.running[q] = 0;
        }
        cr.restarts = m.restarts64[q];
        if (m.mixed) {  // an FP64 fallback after the refinement cycles
            cr.restarts += m.cycles[q];
            cr.fallback = 1;
        }
        m.res[q] = cr;
    }
    if (!again) m.state = FINISHED;
    return 0;
}

template <typename T>
int build_plan(elas3d_group* g, int lane)
{
    std::vector<e3d::GroupMember<T>> mem;
    for (const Member& m : g->members) {
        if (m.state != lane) continue;
        elas3d_ctx* c = m.c;
        e3d::GroupMember<T> gm;
        gm.d = c->d;
        gm.g = c->geom;  // workgroup shape 0, default chunking
        gm.phase = c->phase;
        gm.t = c->tables();
        gm.nrhs = m.R;
        gm.S = c->S;
        gm.partials = c->partials;
        gm.upd_blocks = default_update_blocks(c->d.n);
        if constexpr (sizeof(T) == sizeof(double)) {
            gm.f = c->fields(0);
            gm.rs = c->rs64();
            gm.minv = c->minv_rows();
        } else {
            gm.f = c->fields32(0);
            gm.rs = c->rs32();
            gm.minv = c->minv32_rows();
        }
        mem.push_back(gm);
    }
    int nfin = 0;
    for (auto& gm : mem) nfin += gm.nrhs;
    const size_t bytes = e3d::group_plan_bytes<T>((int)mem.size(), nfin);
    if (bytes > g->dev_cap[lane]) {
        if (g->dev[lane]) hipFree(g->dev[lane]);
        g->dev[lane] = nullptr;
        g->dev_cap[lane] = 0;
        GCHK(hipMalloc(&g->dev[lane], 2 * bytes));
        g->dev_cap[lane] = 2 * bytes;
    }
    if (bytes > g->stg_cap[lane]) {
        if (g->staging[lane]) hipHostFree(g->staging[lane]);
        g->staging[lane] = nullptr;
        g->stg_cap[lane] = 0;
        GCHK(hipHostMalloc(&g->staging[lane], 2 * bytes, hipHostMallocDefault));
        g->stg_cap[lane] = 2 * bytes;
    }
    g->plan[lane] = e3d::GroupPlan{};
    if (mem.empty()) return 0;
    GCHK(e3d::group_prepare<T>(g->stream, mem.data(), (int)mem.size(), g->staging[lane], g->dev[lane],
                               &g->plan[lane]));
    return 0;
}

void leave(elas3d_group* g, Member& m)
{
    m.c->stream = m.own_stream;
    m.c->group = nullptr;
}

int finish(elas3d_group* g, Member& m)
{
    elas3d_ctx* c = m.c;
    elas3d_info info;
    std::memset(&info, 0, sizeof(info));
    info.nrhs = m.R;
    int rc = record_results(c, 0, m.R, m.res, &info);
    if (rc < 0) return mfail(m, rc);
    info.t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - m.t0).count();
    iteration_bytes(c, m.R, &info);
    // the work list changed: the stream must be idle before the context leaves it
    GCHK(hipStreamSynchronize(g->stream));
    leave(g, m);
    c->group_done = g;
    g->done.push_back({c, info});
    return 0;
}

}  // namespace

void e3d::rt::group_forget(elas3d_group* g, elas3d_ctx* c)
{
    hipSetDevice(g->device);
    hipStreamSynchronize(g->stream);  // no sweep of the group is in flight
    for (size_t i = 0; i < g->members.size(); ++i)
        if (g->members[i].c == c) {
            leave(g, g->members[i]);
            g->members.erase(g->members.begin() + (long)i);
            g->dirty = true;
            break;
        }
    for (size_t i = 0; i < g->done.size(); ++i)
        if (g->done[i].first == c) {
            g->done.erase(g->done.begin() + (long)i);
            break;
        }
    c->group_done = nullptr;
}

extern "C" {

int elas3d_group_create(elas3d_group** out, const elas3d_options* opt)
{
    if (!out) return gfail(ELAS3D_EBADARG, "out is NULL");
    *out = nullptr;
    elas3d_options o;
    if (opt)
        o = *opt;
    else
        elas3d_options_init(&o);
    int dev = o.device;
    if (dev >= 0)
        GCHK(hipSetDevice(dev));
    else
        GCHK(hipGetDevice(&dev));
    elas3d_group* g = new elas3d_group();
    g->device = dev;
    if (o.stream) {
        g->stream = (hipStream_t)o.stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete g;
            return gfail(ELAS3D_EDEVICE, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(e));
        }
        g->own_stream = true;
    }
    *out = g;
    return 0;
}

int elas3d_group_add(elas3d_group* g, elas3d_ctx* ctx, double tol, int32_t maxit)
{
    if (!g || !ctx) return gfail(ELAS3D_EBADARG, "group or ctx is NULL");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return gfail(ELAS3D_EBADARG, "tol must be finite and >= 0");
    if (maxit < 0) return gfail(ELAS3D_EBADARG, "maxit must be >= 0");
    if (ctx->group) return gfail(ELAS3D_EORDER, "context is already in a group");
    if (ctx->group_done) return gfail(ELAS3D_EORDER, "context finished in a group and was not returned yet");
    if (ctx->device != g->device) return gfail(ELAS3D_EBADARG, "context is on another device");
    if (ctx->nrhs > 1 && !ctx->batched())
        return gfail(ELAS3D_EBADARG, "a member with several load cases must be set up with options.batched");
    GCHK(hipSetDevice(g->device));
    GCHK(hipStreamSynchronize(ctx->stream));  // its setup is complete
    GCHK(hipStreamSynchronize(g->stream));     // no sweep of the group is in flight
    Member m;
    m.c = ctx;
    m.own_stream = ctx->stream;
    m.tol = tol;
    m.maxit = maxit;
    m.R = ctx->nrhs;
    m.mixed = ctx->opt.precision == ELAS3D_PREC_MIXED;
    m.t0 = std::chrono::steady_clock::now();
    ctx->stream = g->stream;
    ctx->group = g;
    int rc = admit(m);
    if (rc) {
        leave(g, m);
        return mfail(m, rc);
    }
    g->dirty = true;
    if (m.state == FINISHED) return finish(g, m);
    g->members.push_back(m);
    return 0;
}

int elas3d_group_run(elas3d_group* g, int32_t iters, elas3d_ctx** done, elas3d_info* infos, int32_t cap,
                     int32_t* ndone, int32_t* nactive)
{
    if (!g || !ndone || iters < 1 || cap < 0 || (cap > 0 && (!done || !infos)))
        return gfail(ELAS3D_EBADARG, "bad group, iters, cap or NULL output");
    GCHK(hipSetDevice(g->device));
    *ndone = 0;
    const size_t n = g->members.size();
    if (n > 0) {
        if (g->dirty) {
            int rc = build_plan<double>(g, RUN64);
            if (!rc) rc = build_plan<float>(g, RUN32);
            if (rc) return rc;
            g->dirty = false;
        }
        for (int j = 0; j < iters; ++j) {
            GCHK(e3d::launch_group_iteration<double>(g->stream, g->plan[RUN64]));
            GCHK(e3d::launch_group_iteration<float>(g->stream, g->plan[RUN32]));
        }
        if (n * e3d::kMaxRhs > g->hS_cap) {
            if (g->hS) hipHostFree(g->hS);
            g->hS = nullptr;
            g->hS_cap = 0;
            GCHK(hipHostMalloc(&g->hS, 2 * n * e3d::kMaxRhs * sizeof(Scalars), hipHostMallocDefault));
            g->hS_cap = 2 * n * e3d::kMaxRhs;
        }
        for (size_t i = 0; i < n; ++i)
            GCHK(hipMemcpyAsync(g->hS + i * e3d::kMaxRhs, g->members[i].c->S, g->members[i].R * sizeof(Scalars),
                                hipMemcpyDeviceToHost, g->stream));
        GCHK(hipStreamSynchronize(g->stream));
        std::vector<Member> keep;
        keep.reserve(n);
        for (size_t i = 0; i < n; ++i) {
            Member& m = g->members[i];
            const Scalars* fin = g->hS + i * e3d::kMaxRhs;
            bool all = true;
            for (int q = 0; q < m.R; ++q) all = all && fin[q].done;
            if (all) {
                const int before = m.state;
                int rc = settle(m, fin);
                if (rc) {
                    // leave the group broken for this member: return it unsolved
                    leave(g, m);
                    for (size_t k = i + 1; k < n; ++k) keep.push_back(g->members[k]);
                    g->members.swap(keep);
                    g->dirty = true;
                    return mfail(m, rc);
                }
                if (m.state != before) g->dirty = true;
            }
            if (m.state == FINISHED) {
                int rc = finish(g, m);
                if (rc) return rc;
            } else {
                keep.push_back(m);
            }
        }
        g->members.swap(keep);
    }
    int k = 0;
    while (k < cap && !g->done.empty()) {
        done[k] = g->done.front().first;
        done[k]->group_done = nullptr;
        infos[k] = g->done.front().second;
        g->done.erase(g->done.begin());
        ++k;
    }
    *ndone = k;
    if (nactive) *nactive = (int32_t)(g->members.size() + g->done.size());
    return 0;
}

void elas3d_group_destroy(elas3d_group* g)
{
    if (!g) return;
    hipSetDevice(g->device);
    if (g->stream) hipStreamSynchronize(g->stream);
    for (Member& m : g->members) leave(g, m);
    for (auto& d : g->done) d.first->group_done = nullptr;
    for (int l = 0; l < 2; ++l) {
        if (g->dev[l]) hipFree(g->dev[l]);
        if (g->staging[l]) hipHostFree(g->staging[l]);
    }
    if (g->hS) hipHostFree(g->hS);
    if (g->own_stream && g->stream) hipStreamDestroy(g->stream);
    delete g;
}

}  // extern "C"
