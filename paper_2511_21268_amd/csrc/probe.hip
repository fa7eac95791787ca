// Streaming-read reference for the rooflines: how fast this GPU streams a
// buffer from HBM with the loads the matrix passes use (16 bytes per lane,
// nontemporal).  Measurement support only; no step of the solve calls it.
#include <hip/hip_runtime.h>
#include <cstdint>
#include "amg.h"

namespace {

typedef double v2d __attribute__((ext_vector_type(2)));
constexpr int PROBE_THREADS = 256;

// each thread sums its 16-byte elements i, i + T, i + 2T, ... (T threads in
// the grid), four loads in flight, and writes its sum to sink[thread]
__global__ __launch_bounds__(PROBE_THREADS) void k_stream_read(const v2d *__restrict__ a, int64_t n,
                                                               double *__restrict__ sink)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const v2d x0 = __builtin_nontemporal_load(a + i), x1 = __builtin_nontemporal_load(a + i + stride);
        const v2d x2 = __builtin_nontemporal_load(a + i + 2 * stride), x3 = __builtin_nontemporal_load(a + i + 3 * stride);
        s += ((x0.x + x0.y) + (x1.x + x1.y)) + ((x2.x + x2.y) + (x3.x + x3.y));
    }
    for (; i < n; i += stride) {
        const v2d x = __builtin_nontemporal_load(a + i);
        s += x.x + x.y;
    }
    sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" amg_status amg_stream_read(const void *buf, int64_t bytes, double *sink, int64_t sink_len, void *stream)
{
    if (!buf || !sink || bytes <= 0 || bytes % 16 != 0 || ((uintptr_t)buf & 15) != 0 || sink_len < PROBE_THREADS)
        return AMG_ERR_ARG;
    const int64_t blocks = sink_len / PROBE_THREADS;
    const unsigned grid = (unsigned)(blocks < 65536 ? blocks : 65536);
    hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(PROBE_THREADS), 0, (hipStream_t)stream,
                       (const v2d *)buf, bytes / 16, sink);
    return hipGetLastError() == hipSuccess ? AMG_OK : AMG_ERR_HIP;
}
