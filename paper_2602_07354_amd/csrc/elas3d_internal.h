// Internal declarations shared by the kernels and the host runtime of
// libelas3d.  Not part of the public ABI (include/elas3d.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace e3d {

// Per-phase table strides (doubles).  The operator table holds the 21
// upper-triangular entries of the phase's 6x6 Voigt stiffness, the
// preconditioner table the four 3x3 symmetric pieces of the corner block,
// the load table C_p E_hat for each load case.
constexpr int kCoefStride = 24;
constexpr int kDiagStride = 24;
constexpr int kSigStride = 8;

// Problem size.  3N < 2^31, so node and vector-element indices fit in int.
struct Dims {
    int nx, ny, nz;
    int n;
};

// Layout of node vectors in device memory: SoA planes, the layout of the
// C-ABI.  A vector field of T is three planes of N elements, component c of
// node m at c*N + m; kernels address component c through a pointer to its
// plane and node m at m.  The M^-1 dictionary is six planes of its rows.

// Device-resident scalars of one PCG run (Algorithm 2).  Written only by
// the single-block finalize kernels; read by the sweep kernels.
struct Scalars {
    double gg;      // z.g of the current iterate
    double gg0;     // z0.g0 (reference of the paper's criterion)
    double hAh;     // h.Ah of the current direction
    double lambda;  // step size; applied to w lazily by a later direction sweep
    double gamma;   // Fletcher-Reeves coefficient for the next direction
    double rr;      // g.g
    double bnorm2;  // ||b||^2 of the case
    double bref2;   // sum_e ||K_e u^E_e||^2 (scale for the zero-load test)
    double tol;
    double rr_true;  // ||A w + b||^2 from the last residual sweep
    double lambda_prev;  // step size of the older owed step when pending == 2
    int it;          // iterations done
    int maxit;       // iteration cap of this run
    int done;        // nonzero: every later sweep returns at once
    int status;      // 0 converged, 1 not converged, 2 breakdown
    int mode;        // 0 residual criterion, 1 paper criterion
    int cur;         // which of the two direction buffers holds the current h
    // steps w still owes: 0; 1: -lambda h (h in buffer cur); 2: first
    // -lambda_prev h (h in buffer cur ^ 1), then -lambda h (buffer cur).
    // Direction sweeps pay both owed steps when there are two and none
    // otherwise, so w is read and written every other iteration.
    int pending;
    int pad;
};

// Field pointers of one PCG run (component pointers of T, addressed at
// m: double for the FP64 solve, float for the inner solve of the
// mixed-precision refinement, where w is the correction d and g starts as
// the rounded residual).
template <typename T>
struct FieldsT {
    T* w[3];
    T* g[3];
    T* z[3];
    T* h0[3];
    T* h1[3];
    T* Ah[3];
    const T* b[3];
};
using Fields = FieldsT<double>;

constexpr int kMaxRhs = 6;

// The same fields for RHS r of a batch whose buffers lie `rs` elements apart.
template <typename T>
__host__ __device__ inline FieldsT<T> shifted(const FieldsT<T>& f, size_t off)
{
    FieldsT<T> g;
    for (int c = 0; c < 3; ++c) {
        g.w[c] = f.w[c] ? f.w[c] + off : nullptr;
        g.g[c] = f.g[c] ? f.g[c] + off : nullptr;
        g.z[c] = f.z[c] ? f.z[c] + off : nullptr;
        g.h0[c] = f.h0[c] ? f.h0[c] + off : nullptr;
        g.h1[c] = f.h1[c] ? f.h1[c] + off : nullptr;
        g.Ah[c] = f.Ah[c] ? f.Ah[c] + off : nullptr;
        g.b[c] = f.b[c] ? f.b[c] + off : nullptr;
    }
    return g;
}

// The inverse diagonal blocks as a dictionary of rows: node m uses row
// idx[m], whose six symmetric entries (xx, yy, zz, yz, xz, xy) are
// m[q][row].  Rows [0, nphase) belong to the nodes whose eight voxels
// all have phase p (the same block for all of them); each remaining row to
// one node at a phase boundary, in node order.
template <typename T>
struct MinvRows {
    const uint32_t* idx;
    T* m[6];
};

// Phase dictionaries of the wave-specialised sweep, for one launch geometry
// (tiles_x, tiles_y, kz): per workgroup box (the element columns and rows
// its tile reads, element layers k0 - 1 .. kend, periodic), the distinct
// phase ids in ascending order (kWsDict entries, the unused ones repeating
// the first), and per element of the box the rank of its phase in that list
// (one byte; layer u of block b at b * ws_map_block(kz) + u * tx * ty, rows
// of tx bytes).
constexpr int kWsDict = 96;
struct WsTables {
    const int32_t* dict = nullptr;
    const uint8_t* map = nullptr;
    int tile = -1, tiles_x = 0, tiles_y = 0, kz = 0;
};

struct Tables {
    const double* coef;    // nphase * kCoefStride: C/16, packed
    const float* coef32;   // the same rounded to FP32 (mixed precision), or nullptr
    const double* diag;    // nphase * kDiagStride
    const uint8_t* solid;  // nphase: 1 if the phase has stiffness
    WsTables ws{};         // the wave-specialised sweep's dictionaries, when built
};

// Workgroup shapes of the tiled operator sweep: tx x ty lanes evaluate the
// element columns of a tile.  Shape 0 is the default of every sweep; the
// fused direction + operator sweep can be autotuned over all of them, the
// residual and refinement sweeps over those with nl = 0.
//
// nl > 0 marks the wave-specialised form of the fused sweep: the workgroup
// has nl more wavefronts that only stream the next node planes of z and the
// current direction into a ring of d planes in LDS (16-byte direct-to-LDS
// loads), so that several planes are in flight per CU without holding them
// in registers; the tx x ty lanes compute from the ring.  The phases come
// from a dictionary per workgroup built at setup (WsTables): its stiffness
// rows sit in LDS for the whole workgroup, and the ring carries one byte per
// element, the phase's rank in it.  It needs rows of whole 16-byte chunks of
// nodes, 16-byte aligned fields and at most kWsDict distinct phases in every
// workgroup box (ws_supported, launch_ws_dictionary).
// Shape 6 (64 x 8 compute lanes + 2 loaders) exists for the FP32 sweep only:
// its ten wavefronts put two computing ones on every SIMD, and in FP64 its
// ring and row exchange would not fit the LDS of a CU.
constexpr int kNumTiles = 7;
struct TileShape {
    int tx, ty;
    int nl, d;  // d > 0: wave-specialised, with nl loader wavefronts and a ring of d planes
    int elem;   // wave-specialised: 0 for both precisions, 4 for the FP32 sweep only
};
constexpr TileShape kTileShapes[kNumTiles] = {{32, 8, 0, 0, 0},  {16, 16, 0, 0, 0}, {64, 4, 0, 0, 0},
                                              {32, 16, 0, 0, 0}, {64, 8, 0, 0, 0},  {64, 6, 2, 4, 0},
                                              {64, 8, 2, 4, 4}};
// True for the wave-specialised shapes (fused sweep only).
constexpr bool is_ws(int t) { return kTileShapes[t].d > 0; }
// Lanes of a workgroup of shape t.
constexpr int tile_lanes(int t) { return kTileShapes[t].tx * kTileShapes[t].ty + 64 * kTileShapes[t].nl; }
// True when shape t exists for elements of elem_bytes (constexpr: selects
// the kernels that are built).
constexpr bool ws_elem_ok(int t, int elem_bytes) { return kTileShapes[t].elem == 0 || kTileShapes[t].elem == elem_bytes; }
// True when the wave-specialised shape t can run on grid d with elements of
// elem_bytes: a shape for that precision, rows of whole 16-byte chunks and
// planes under 2^27 voxels (its stores address a plane by a 32-bit byte
// offset).
inline bool ws_supported(const Dims& d, int t, int elem_bytes)
{
    return !is_ws(t) || (ws_elem_ok(t, elem_bytes) && d.nx % (16 / elem_bytes) == 0 &&
                         (long long)d.nx * d.ny < (1ll << 27));
}

// Kernel launch geometry of the tiled operator sweep.
struct OpGeom {
    int tile;  // index into kTileShapes
    int tiles_x, tiles_y, zchunks, kz;
    int blocks;
};

// kz_hint > 0 fixes the z chunk; otherwise the chunks are cut so that about
// target_blocks workgroups (0: the default, 4096) cover the grid.
OpGeom op_geometry(const Dims& d, int kz_hint, int tile = 0, int target_blocks = 0);

// Bytes of one workgroup's rank map (kz + 2 layers of tx * ty bytes) and of
// all of them, for a wave-specialised geometry g (tiles per RHS).
inline size_t ws_map_block(const OpGeom& g)
{
    return (size_t)(g.kz + 2) * kTileShapes[g.tile].tx * kTileShapes[g.tile].ty;
}
inline size_t ws_map_bytes(const OpGeom& g) { return (size_t)g.blocks * ws_map_block(g); }

// ---- launchers (elas3d_kernels.hip) -------------------------------------
// Every launcher enqueues on `st` and returns the hipError_t of the launch.

hipError_t launch_load(hipStream_t st, const Dims& d, const int32_t* phase, const double* sig,
                       double* const b[3], double* partials, double* out2 /* bnorm2, bref2 */,
                       int max_blocks);
// Preconditioner build in three steps.  count: boundary nodes (whose eight
// voxels do not all share one phase) of each chunk of kPrecondChunk nodes
// into counts[chunk]; the host takes the exclusive prefix sum.  fill: every
// node's row (its phase, or nphase + offsets[chunk] + its rank in the chunk)
// into M.idx, and the inverted block of each boundary node into its row.
// table: rows [0, nphase).  identity: plain CG (I on nodes with stiffness).
constexpr int kPrecondChunk = 4096;
hipError_t launch_precond_count(hipStream_t st, const Dims& d, const int32_t* phase, int* counts);
hipError_t launch_precond_fill(hipStream_t st, const Dims& d, const int32_t* phase, const Tables& t,
                               int identity, int nphase, const int* offsets, uint32_t* idx,
                               double* const rows[6]);
hipError_t launch_precond_table(hipStream_t st, int nphase, const Tables& t, int identity,
                                double* const rows[6]);
// Dense SoA planes (6 x N, FP64) of the dictionary M.
hipError_t launch_precond_expand(hipStream_t st, const Dims& d, const MinvRows<double>& M,
                                 double* out);
// The PCG sweeps exist for T = double (FP64 solve) and T = float (inner
// solve of the mixed-precision refinement); dot products are FP64 in both.
// norms2: device {||b||^2, ||b||_ref^2} of the run (zero-load test).
template <typename T>
hipError_t launch_pcg_init(hipStream_t st, const Dims& d, const FieldsT<T>& f, const MinvRows<T>& M,
                           int fresh, int from_residual, Scalars* S, double* partials,
                           int max_blocks, const double* norms2);
// The two iteration sweeps run a batch of nrhs right-hand sides in lockstep:
// f describes RHS 0, RHS r lies r*rs elements further in every field, and S
// points to nrhs consecutive scalar sets (a RHS whose flag is done is skipped).
// finalize = false launches the sweep alone (autotuning at the start of a
// run, where lambda = gamma = 0 leave the iterate unchanged).  The update
// sweep runs on at most max_blocks workgroups (it writes 2 * kMaxRhs partial
// sums per workgroup into partials); nontemporal streams its node vectors
// past the caches.
// Phase dictionaries of the wave-specialised geometry g (WsTables): dict
// (g.blocks * kWsDict int32) and map (ws_map_bytes(g)); *maxcount (device,
// zeroed by the caller) becomes the largest number of distinct phases of a
// box, or a number above kWsDict when some box holds more (then dict and map
// are incomplete and must not be used).
hipError_t launch_ws_dictionary(hipStream_t st, const Dims& d, const OpGeom& g, const int32_t* phase,
                                int32_t* dict, uint8_t* map, int* maxcount);
template <typename T>
hipError_t launch_direction_operator(hipStream_t st, const Dims& d, const OpGeom& g,
                                     const int32_t* phase, const Tables& t, const FieldsT<T>& f,
                                     size_t rs, int nrhs, Scalars* S, double* partials,
                                     bool finalize = true);
template <typename T>
hipError_t launch_update_precond(hipStream_t st, const Dims& d, const FieldsT<T>& f, size_t rs,
                                 int nrhs, const MinvRows<T>& M, Scalars* S, double* partials,
                                 int max_blocks, bool finalize = true, bool nontemporal = false);
template <typename T>
hipError_t launch_final_update(hipStream_t st, const Dims& d, const FieldsT<T>& f, Scalars* S);
// Refinement of the mixed-precision solve: r = A (w + d) + b in FP64, stored
// rounded to FP32, ||r||^2 (FP64) into *norm2; then w += d.
hipError_t launch_refine(hipStream_t st, const Dims& d, const OpGeom& g, const int32_t* phase,
                         const Tables& t, double* const w[3], const float* const dcorr[3],
                         const double* const b[3], float* const r[3], double* partials,
                         double* norm2);
hipError_t launch_to_float(hipStream_t st, const double* src, float* dst, size_t n);
// n values in [-1e-3, 1e-3) from a hash of the index (stand-in data for timing)
hipError_t launch_tuning_fill(hipStream_t st, double* p, size_t n);
// y = A x (+ add when add[0] != nullptr); ||y||^2 into *norm2 when norm2 != nullptr.
// APPLY and REFINE run with any workgroup shape (the geometry g).
hipError_t launch_apply(hipStream_t st, const Dims& d, const OpGeom& g, const int32_t* phase,
                        const Tables& t, const double* const x[3], double* const y[3],
                        const double* const add[3], double* partials, double* norm2);
// sums7: device {sum sigma_r (6), energy}; sig may be nullptr.  Uses f.w.
hipError_t launch_stress(hipStream_t st, const Dims& d, const int32_t* phase, const Tables& t,
                         const double* strain6, const Fields& f, double* const sig[6],
                         double* partials, double* sums7, int max_blocks);
// Von Mises stress per voxel into vm (may be nullptr) and {max, argmax}
// (argmax as a double) into the device pair out2.  Uses f.w.
hipError_t launch_von_mises(hipStream_t st, const Dims& d, const int32_t* phase, const Tables& t,
                            const double* strain6, const Fields& f, double* vm, double* partials,
                            double* out2, int max_blocks);
hipError_t launch_total_displacement(hipStream_t st, const Dims& d, const double* strain6,
                                     const Fields& f, double* const u[3]);
// Adds to *bad the number of ids outside [0, nphase).
hipError_t launch_phase_check(hipStream_t st, const int32_t* phase, int n, int nphase, int* bad);
// ---- groups of independent problems in one launch per sweep -------------
// One member of a group: a problem (its own grid, tables and fields) with
// nrhs right-hand sides in lockstep; its sweeps use workgroup shape 0 and
// the geometry g, its update sweep upd_blocks workgroups.
template <typename T>
struct GroupMember {
    Dims d;
    OpGeom g;
    const int32_t* phase;
    Tables t;
    FieldsT<T> f;
    size_t rs;
    int nrhs;
    MinvRows<T> minv;
    Scalars* S;
    double* partials;
    int upd_blocks;
};

// Work lists of a group (built by group_prepare): the direction+operator
// sweep's members in kernel-argument packs of up to 8 (one launch each),
// the update sweep's and the finalizes' lists in device memory.
struct GroupPlan {
    char* dev = nullptr;
    int n = 0, nfin = 0, upd_blocks = 0;
    std::vector<uint8_t> packs;    // the packs, by value
    std::vector<int> pack_blocks;  // workgroups of each pack's launch
    size_t off_upd = 0, off_updfirst = 0, off_findir = 0, off_finupd = 0;
};

// Bytes of the work lists of n members with nfin (member, RHS) pairs.
template <typename T>
size_t group_plan_bytes(int n, int nfin);
// Writes the work lists to `staging` (pinned host memory of
// group_plan_bytes) and enqueues their copy to `dev` on st.
template <typename T>
hipError_t group_prepare(hipStream_t st, const GroupMember<T>* m, int n, char* staging, char* dev,
                         GroupPlan* plan);
// One PCG iteration (direction + operator sweep, update sweep and their
// finalizes) of every member of the plan: four launches for up to 8
// members, one more per further 8.
template <typename T>
hipError_t launch_group_iteration(hipStream_t st, const GroupPlan& plan);

// Message returned by elas3d_last_error(NULL) on this thread (context-free
// entry points).
void set_last_error(const std::string& msg);

}  // namespace e3d
