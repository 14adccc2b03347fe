// Streaming-bandwidth probe: the rates that plain HBM streams reach on this
// device, the practical ceiling for the solver's sweeps (which only stream
// vectors through HBM).  Not part of a solve.
//
// Three kernels over buffers the call allocates: copy (read a, write b), read
// (sum a) and write (fill b).  Every lane moves 16 bytes per access in a
// grid-stride loop, so each wave instruction covers 1 KiB of consecutive
// addresses; the caller picks the grid and whether the accesses are
// non-temporal (streamed past the caches).

#include <hip/hip_runtime.h>

#include <string>

#include "elas3d.h"
#include "elas3d_internal.h"

namespace {

typedef double v2d __attribute__((ext_vector_type(2)));
constexpr int kStreamBlock = 256;

template <bool NT>
__global__ void __launch_bounds__(kStreamBlock) stream_copy_kernel(const v2d* __restrict__ a, v2d* __restrict__ b,
                                                                   size_t n)
{
    const size_t stride = (size_t)gridDim.x * kStreamBlock;
    for (size_t i = (size_t)blockIdx.x * kStreamBlock + threadIdx.x; i < n; i += stride) {
        if constexpr (NT)
            __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
        else
            b[i] = a[i];
    }
}

// The sum decides a store that the zero-filled input never takes, so the
// loads cannot be dropped and nothing is written.
template <bool NT>
__global__ void __launch_bounds__(kStreamBlock) stream_read_kernel(const v2d* __restrict__ a, double* sink, size_t n)
{
    const size_t stride = (size_t)gridDim.x * kStreamBlock;
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * kStreamBlock + threadIdx.x; i < n; i += stride) {
        const v2d v = NT ? __builtin_nontemporal_load(a + i) : a[i];
        s += v.x + v.y;
    }
    if (s != 0.0) sink[0] = s;
}

template <bool NT>
__global__ void __launch_bounds__(kStreamBlock) stream_write_kernel(v2d* __restrict__ b, size_t n)
{
    const size_t stride = (size_t)gridDim.x * kStreamBlock;
    const v2d v = {1.0, 2.0};
    for (size_t i = (size_t)blockIdx.x * kStreamBlock + threadIdx.x; i < n; i += stride) {
        if constexpr (NT)
            __builtin_nontemporal_store(v, b + i);
        else
            b[i] = v;
    }
}

// Device buffers, events and stream of one probe call, released on scope exit.
struct ProbeCall {
    hipStream_t stream = nullptr;
    bool own = false;
    void* a = nullptr;
    void* b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~ProbeCall()
    {
        if (stream) hipStreamSynchronize(stream);
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
        if (a) hipFree(a);
        if (b) hipFree(b);
        if (own && stream) hipStreamDestroy(stream);
    }
};

int probe_fail(int code, const std::string& msg)
{
    e3d::set_last_error(msg);
    return code;
}

#define PROBECHK(expr)                                                                                            \
    do {                                                                                                          \
        hipError_t e_ = (expr);                                                                                   \
        if (e_ != hipSuccess) return probe_fail(ELAS3D_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

}  // namespace

extern "C" {

int elas3d_stream_bandwidth(int64_t bytes, int32_t blocks, int32_t reps, int32_t nontemporal, double* gbs,
                            const elas3d_options* opt)
{
    if (!gbs) return probe_fail(ELAS3D_EBADARG, "gbs is NULL");
    if (bytes < ((int64_t)1 << 20) || bytes % 16 != 0)
        return probe_fail(ELAS3D_EBADARG, "bytes must be >= 1 MiB and a multiple of 16");
    if (blocks < 1 || blocks > (1 << 24)) return probe_fail(ELAS3D_EBADARG, "blocks must be in [1, 2^24]");
    if (reps < 1 || reps > 10000) return probe_fail(ELAS3D_EBADARG, "reps must be in [1, 10000]");
    if (nontemporal != 0 && nontemporal != 1) return probe_fail(ELAS3D_EBADARG, "nontemporal must be 0 or 1");
    elas3d_options o;
    if (opt)
        o = *opt;
    else
        elas3d_options_init(&o);

    ProbeCall call;
    if (o.device >= 0) PROBECHK(hipSetDevice(o.device));
    if (o.stream) {
        call.stream = (hipStream_t)o.stream;
    } else {
        PROBECHK(hipStreamCreateWithFlags(&call.stream, hipStreamNonBlocking));
        call.own = true;
    }
    if (hipMalloc(&call.a, (size_t)bytes) != hipSuccess || hipMalloc(&call.b, (size_t)bytes) != hipSuccess) {
        (void)hipGetLastError();
        return probe_fail(ELAS3D_ENOMEM, "cannot allocate two buffers of " + std::to_string(bytes) + " bytes");
    }
    PROBECHK(hipEventCreate(&call.e0));
    PROBECHK(hipEventCreate(&call.e1));
    PROBECHK(hipMemsetAsync(call.a, 0, (size_t)bytes, call.stream));
    PROBECHK(hipMemsetAsync(call.b, 0, (size_t)bytes, call.stream));

    const size_t n = (size_t)bytes / sizeof(v2d);
    const v2d* a = (const v2d*)call.a;
    v2d* b = (v2d*)call.b;
    double* sink = (double*)call.b;
    auto launch = [&](int kind) {
        const dim3 grid(blocks), block(kStreamBlock);
        if (kind == 0) {
            if (nontemporal) stream_copy_kernel<true><<<grid, block, 0, call.stream>>>(a, b, n);
            else stream_copy_kernel<false><<<grid, block, 0, call.stream>>>(a, b, n);
        } else if (kind == 1) {
            if (nontemporal) stream_read_kernel<true><<<grid, block, 0, call.stream>>>(a, sink, n);
            else stream_read_kernel<false><<<grid, block, 0, call.stream>>>(a, sink, n);
        } else {
            if (nontemporal) stream_write_kernel<true><<<grid, block, 0, call.stream>>>(b, n);
            else stream_write_kernel<false><<<grid, block, 0, call.stream>>>(b, n);
        }
    };
    const double moved[3] = {2.0 * (double)bytes, (double)bytes, (double)bytes};
    for (int kind = 0; kind < 3; ++kind) {
        launch(kind);  // untimed first pass
        PROBECHK(hipGetLastError());
        PROBECHK(hipEventRecord(call.e0, call.stream));
        for (int r = 0; r < reps; ++r) launch(kind);
        PROBECHK(hipGetLastError());
        PROBECHK(hipEventRecord(call.e1, call.stream));
        PROBECHK(hipEventSynchronize(call.e1));
        float ms = 0.0f;
        PROBECHK(hipEventElapsedTime(&ms, call.e0, call.e1));
        gbs[kind] = moved[kind] * reps / (ms * 1e-3) / 1e9;
    }
    return 0;
}

}  // extern "C"
