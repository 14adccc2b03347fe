// Host runtime shared by the C-ABI translation units of libelas3d: the
// context of one problem and the solver steps that both elas3d_solve and
// the group engine (elas3d_group_*) drive.  Not part of the public ABI.
#pragma once

#include <cstring>
#include <string>
#include <vector>

#include "elas3d.h"
#include "elas3d_internal.h"

namespace e3d::rt {

constexpr int kSweepBlocks = 4096;  // grid of the node-wise sweeps
// autotuning candidates: workgroup targets of the operator sweep (every tile
// shape) and grids of the update sweep
constexpr int kTuneTargets[4] = {2048, 4096, 8192, 16384};
constexpr int kTuneUpdate[6] = {1024, 2048, 4096, 8192, 16384, 32768};
constexpr int kPartialValues = 8;   // partial sums per block, upper bound
constexpr int kMinPartialSlots = 65536;  // blocks' worth of partials, at least
constexpr int kMaxUpdateBlocks = kTuneUpdate[5];  // largest update grid, tuned or set
// the update sweep writes 2 * kMaxRhs partials per workgroup at stride
// (its grid): the largest grid must fit the smallest buffer
static_assert((long long)kMaxUpdateBlocks * 2 * kMaxRhs <= (long long)kPartialValues * kMinPartialSlots,
              "update grids overrun the partials buffer");

// Grid of the update sweep when it is not autotuned (and of every group
// member's): 4096 workgroups, or 1024 on grids of at most 2^21 nodes, where
// fewer workgroups that each loop over more nodes, and a finalize over fewer
// partials, measured faster (96^3, mixed precision: 37 -> 25 us per launch).
inline int default_update_blocks(long long n) { return n <= (1LL << 21) ? 1024 : kSweepBlocks; }
constexpr int kDefaultPoll = 16;

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
};

}  // namespace e3d::rt

using e3d::Dims;
using e3d::Fields;
using e3d::FieldsT;
using e3d::Scalars;

struct elas3d_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    Dims d{};
    int nphase = 0, nrhs = 0;
    elas3d_options opt{};
    std::vector<double> strain;  // nrhs * 6
    e3d::OpGeom geom{};  // default geometry (tile shape 0): group members
    // geometry of the residual and refinement sweeps of elas3d_solve (the
    // default, or the autotuned choice)
    e3d::OpGeom geom_apply{};
    int apply_tuned = 0;
    // direction+operator sweep and update grid per precision (0 FP64, 1 FP32),
    // the defaults or the autotuned choice
    e3d::OpGeom geom_sweep[2]{};
    int upd_blocks[2] = {0, 0};
    int upd_nt[2] = {0, 0};  // update sweep streams non-temporally (autotuned)
    int tuned[2] = {0, 0};

    int32_t* phase = nullptr;
    double* coef = nullptr;
    double* diag = nullptr;
    uint8_t* solid = nullptr;
    double* sig = nullptr;
    // FP64 fields.  Batched: per RHS one bundle [w 3N | b 3N | g z h0 h1 Ah 15N]
    // so that every field of RHS r lies r*21N after RHS 0's.  Otherwise the
    // RHS keep [w | b] (6N each) and share one 15N work area after them.
    double* bundle64 = nullptr;
    // M^-1 as a dictionary: row of each node, and mrows rows of six entries
    // (one per phase, then one per phase-boundary node)
    uint32_t* midx = nullptr;
    size_t mrows = 0;
    double* minv = nullptr;
    // mixed precision: FP32 g, z, h0, h1, Ah, d (18N floats per work slot),
    // M^-1 rows, table
    float* bundle32 = nullptr;
    float* minv32 = nullptr;
    float* coef32 = nullptr;
    double* partials = nullptr;
    int partial_stride = 0;
    double* norms = nullptr;  // nrhs * 2: ||b||^2, ||b||_ref^2
    double* dscratch = nullptr;  // 64 doubles
    int* dflag = nullptr;
    Scalars* S = nullptr;
    Scalars* hS = nullptr;        // pinned, 2 slots of kMaxRhs
    double* hscratch = nullptr;   // pinned, 64 doubles
    std::vector<int> solved;
    elas3d_group* group = nullptr;       // group the context is solved in, if any
    elas3d_group* group_done = nullptr;  // group holding it finished, not yet returned
    double bytes = 0.0;
    std::string err;

    // phase dictionaries of the wave-specialised sweep, one entry per
    // geometry built (maxcount > kWsDict: too many phases, nothing kept)
    struct WsDictEntry {
        e3d::OpGeom g;
        int32_t* dict;
        uint8_t* map;
        int maxcount;
    };
    std::vector<WsDictEntry> wsd;

    std::vector<e3d::rt::EventPair> ev_op, ev_up;
    // captured iteration batches, keyed by (element size, first RHS, RHS count)
    struct GraphEntry {
        int key[3];
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;

    size_t N() const { return (size_t)d.n; }
    // component c (or M^-1 entry q) of a field starting at base
    template <typename P>
    P* comp(P* base, int c) const { return base + (size_t)c * N(); }

    bool batched() const { return opt.batched != 0; }
    size_t rs64() const { return (batched() ? 21 : 6) * N(); }  // RHS stride of the bundles
    size_t rs32() const { return 18 * N(); }
    double* wptr(int r) const { return bundle64 + (size_t)r * rs64(); }
    double* bptr(int r) const { return wptr(r) + 3 * N(); }
    double* work64(int r) const
    {
        return batched() ? wptr(r) + 6 * N() : bundle64 + (size_t)nrhs * 6 * N();
    }
    float* work32(int r) const { return bundle32 + (batched() ? (size_t)r * rs32() : 0); }
    Fields fields(int rhs)
    {
        Fields f;
        double* wk = work64(rhs);
        for (int c = 0; c < 3; ++c) {
            f.w[c] = comp(wptr(rhs), c);
            f.b[c] = comp(bptr(rhs), c);
            f.g[c] = comp(wk, c);
            f.z[c] = comp(wk + 3 * N(), c);
            f.h0[c] = comp(wk + 6 * N(), c);
            f.h1[c] = comp(wk + 9 * N(), c);
            f.Ah[c] = comp(wk + 12 * N(), c);
        }
        return f;
    }
    // entry q of the M^-1 rows starting at base
    template <typename P>
    P* mcomp(P* base, int q) const { return base + (size_t)q * mrows; }
    e3d::MinvRows<double> minv_rows() const
    {
        e3d::MinvRows<double> M;
        M.idx = midx;
        for (int q = 0; q < 6; ++q) M.m[q] = mcomp(minv, q);
        return M;
    }
    e3d::FieldsT<float> fields32(int rhs)
    {
        e3d::FieldsT<float> f;
        float* wk = work32(rhs);
        for (int c = 0; c < 3; ++c) {
            f.g[c] = comp(wk, c);
            f.z[c] = comp(wk + 3 * N(), c);
            f.h0[c] = comp(wk + 6 * N(), c);
            f.h1[c] = comp(wk + 9 * N(), c);
            f.Ah[c] = comp(wk + 12 * N(), c);
            f.w[c] = comp(wk + 15 * N(), c);
            f.b[c] = nullptr;
        }
        return f;
    }
    e3d::MinvRows<float> minv32_rows() const
    {
        e3d::MinvRows<float> M;
        M.idx = midx;
        for (int q = 0; q < 6; ++q) M.m[q] = mcomp(minv32, q);
        return M;
    }
    e3d::Tables tables() const { return e3d::Tables{coef, coef32, diag, solid}; }
    // the tables plus the dictionaries of geometry g, when built
    e3d::Tables tables_for(const e3d::OpGeom& g) const
    {
        e3d::Tables t = tables();
        for (const auto& e : wsd)
            if (e.dict && e.g.tile == g.tile && e.g.tiles_x == g.tiles_x && e.g.tiles_y == g.tiles_y &&
                e.g.kz == g.kz)
                t.ws = e3d::WsTables{e.dict, e.map, g.tile, g.tiles_x, g.tiles_y, g.kz};
        return t;
    }
};


namespace e3d::rt {

// Records msg as the error of ctx (or of the thread when ctx is NULL) and
// returns code.
int fail(elas3d_ctx* ctx, int code, const std::string& msg);

#define HIPCHK(ctx, expr)                                                                       \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return e3d::rt::fail((ctx), ELAS3D_EDEVICE,                                         \
                                 std::string(#expr) + ": " + hipGetErrorString(e_));            \
    } while (0)

struct RunStats {
    Scalars fin{};     // device scalars at the end of the run
    int it_start = 0;  // iteration counter when the run started
};

struct CaseResult {
    Scalars fin{};
    int restarts = 0;
    double rel_true = 0.0;
    int fallback = 0;
};

// Start a PCG run of RHS r (device scalars and the init sweep), enqueued on
// the context's stream through pinned staging slot r of c->hS.
template <typename T>
int start_run(elas3d_ctx* c, int r, const FieldsT<T>& f, const e3d::MinvRows<T>& M, double tol, int maxit, int mode,
              int it0, int fresh, int from_residual, const double* norms2);
// Mark RHS r finished for the sweeps that follow (enqueued, staging slot r).
int park(elas3d_ctx* c, int r, const Scalars& fin);
// FP64 PCG of RHS [r0, r0+R) (see elas3d_api.hip).
int solve_fp64(elas3d_ctx* c, int r0, int R, double tol, int maxit, bool cont, int it0, elas3d_info* info,
               CaseResult* res);
// Mixed precision: w += d, then r = A w + b in FP64 stored as the FP32
// residual of the next inner run (and as its norms); *rel = ||r|| / ||b||.
int refine_step(elas3d_ctx* c, int r, int q, double bnorm2, double* rel);
// The refinement sweep of refine_step, enqueued only: ||r||^2 lands in
// c->dscratch[4 + 2q] (and [5 + 2q]).
int refine_launch(elas3d_ctx* c, int r, int q);
// The residual sweep of true_residual, enqueued only: ||g||^2 into the
// device double norm2.
int residual_launch(elas3d_ctx* c, int r, double* norm2);
// FP64 true residual of RHS r: g = A w + b, returns ||g||^2 in *rr.
int true_residual(elas3d_ctx* c, int r, double* rr);
// Per-RHS statistics of a finished solve into info (may be NULL); marks the
// RHS solved; returns the worst status.
int record_results(elas3d_ctx* c, int r0, int R, const CaseResult* res, elas3d_info* info);
// Algorithmic HBM bytes of one PCG iteration over nrhs cases and the M^-1
// dictionary's size, into info.
void iteration_bytes(const elas3d_ctx* c, int nrhs, elas3d_info* info);
// Withdraw c from the group that runs it or holds it finished (before c is
// destroyed): waits until the group's stream is idle.
void group_forget(elas3d_group* g, elas3d_ctx* c);

}  // namespace e3d::rt
