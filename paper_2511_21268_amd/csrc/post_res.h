// The prolongation fused into the first step of a polynomial post-smoothing
// (Sec. 3 steps 4 and 5 re-associated, as k_sell_post does for l1-Jacobi).
#pragma once
#include "kernels.h"

namespace amgk {

// Prolongation fused with the residual of the first polynomial post-smoothing
// step: up = u + P e (written to y) and r <- r - (K P) e = f - K up in place,
// with acc = ((K P) e)_row over the SELL image of K P as in k_sell_post.
template <typename VT, typename IT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_sell_post_res(
    const Sell<VT, IT> A, const VT *__restrict__ e, const VT *__restrict__ u, VT *__restrict__ r,
    const int32_t *__restrict__ agg, const VT *__restrict__ pc, VT *__restrict__ y)
{
    const int lane = threadIdx.x & 63, wid = wave_id();
    const int64_t s = (int64_t)blockIdx.x * SELL_WAVES + wid;
    if (s >= A.nslices) return;
    const int64_t row = A.row_of(s * SLICE + lane);
    VT acc = 0;
    sell_row<SLICE, 2>(A, s, lane, [&](const VT *v, const int *c) {
#pragma unroll
        for (int t = 0; t < 8; t++) acc = fma(v[t], ld32(e, c[t]), acc);
    });
    if (row < 0) return;
    y[row] = u[row] + pc[row] * e[agg[row]];
    r[row] = r[row] - acc;
}

}  // namespace amgk
