// Streaming-read reference for the rooflines: how fast this GPU streams a
// buffer from HBM with the loads the matrix passes use (16 bytes per lane,
// nontemporal).  Measurement support only; no step of the solve calls it.
#include <hip/hip_runtime.h>
#include <cstdint>
#include "amg.h"

namespace amgk {

typedef double v2d __attribute__((ext_vector_type(2)));
constexpr int PROBE_THREADS = 256;

// Each wave reads contiguous 4 KB chunks (four 1 KB loads of 16 bytes per
// lane, all in flight), chunk c of the buffer on wave c mod W (W waves in the
// grid); every thread sums what it read and writes the sum to sink[thread].
// With a persistent grid of eight 4-wave blocks per compute unit this is the
// fastest plain read of the shapes tried on this GPU (per-lane grid strides
// with 4-16 loads in flight, plain loads, direct-to-LDS copies).
__global__ __launch_bounds__(PROBE_THREADS) void k_stream_read(const v2d *__restrict__ a, int64_t n,
                                                               double *__restrict__ sink)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t nchunks = n / 256;   // 256 elements of 16 bytes
    double s = 0.0;
    for (int64_t c = wave; c < nchunks; c += nwaves) {
        const v2d *p = a + c * 256 + lane;
        const v2d x0 = __builtin_nontemporal_load(p), x1 = __builtin_nontemporal_load(p + 64);
        const v2d x2 = __builtin_nontemporal_load(p + 128), x3 = __builtin_nontemporal_load(p + 192);
        s += ((x0.x + x0.y) + (x1.x + x1.y)) + ((x2.x + x2.y) + (x3.x + x3.y));
    }
    // the last n mod 256 elements: one per thread of the first waves
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = nchunks * 256 + t; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const v2d x = __builtin_nontemporal_load(a + i);
        s += x.x + x.y;
    }
    sink[t] = s;
}

}  // namespace amgk

extern "C" amg_status amg_stream_read(const void *buf, int64_t bytes, double *sink, int64_t sink_len, void *stream)
{
    if (!buf || !sink || bytes <= 0 || bytes % 16 != 0 || ((uintptr_t)buf & 15) != 0 ||
        sink_len < amgk::PROBE_THREADS)
        return AMG_ERR_ARG;
    const int64_t blocks = sink_len / amgk::PROBE_THREADS;
    const unsigned grid = (unsigned)(blocks < 65536 ? blocks : 65536);
    hipLaunchKernelGGL(amgk::k_stream_read, dim3(grid), dim3(amgk::PROBE_THREADS), 0, (hipStream_t)stream,
                       (const amgk::v2d *)buf, bytes / 16, sink);
    return hipGetLastError() == hipSuccess ? AMG_OK : AMG_ERR_HIP;
}
