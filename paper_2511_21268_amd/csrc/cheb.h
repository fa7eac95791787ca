// Kernels of the smoothed-aggregation form of the V-cycle (the paper's default
// preconditioner, Sec. 3.1 "Variants and efficiency", Sec. 3.2, Sec. 5.1):
// the fourth-kind Chebyshev acceleration of l1-Jacobi as fused matrix passes,
// and the Jacobi-preconditioned CG on the coarsest level in one workgroup.
//
// Fourth-kind Chebyshev smoother of degree k on K x = f (D the l1 diagonal,
// lambda(D^{-1}K) in (0, 1], so no spectral estimate is needed): the error
// after k steps is W_k(I - 2 D^{-1}K) e_0 / (2k+1), W_k(cos t) =
// sin((k + 1/2) t) / sin(t/2).  From the three-term recurrence of W_k, with
// d_j = x_{j+1} - x_j and r_j = f - K x_j:
//     d_0 = (4/3) D^{-1} r_0,
//     d_j = (2j-1)/(2j+3) d_{j-1} + (8j+4)/(2j+3) D^{-1} r_j,
//     r_j = r_{j-1} - K d_{j-1},   x_{j+1} = x_j + d_j,
// so each step is one matrix pass over K whose gathered vector is d_{j-1}
// and whose epilogue updates x, r and the next direction row by row.
#pragma once
#include "kernels.h"

namespace amgk {

// One Chebyshev matrix pass, acc = (K x)_row:
//   MODE 0 (start from u = x):   r = f - acc;  dn = b invd r
//   MODE 1 (step, x = d_{j-1}):  u += d_{j-1} (u = d_{j-1} when first);
//                                r = (first ? f : r) - acc;
//                                dn = a d_{j-1} + b invd r
//   MODE 2 (last step):          as MODE 1 without dn (leaves the residual
//                                of the smoothed iterate in r)
// x is read by every row (gathered); u, r and dn are per-row, and dn never
// aliases x (the directions ping-pong between two buffers).
template <typename IT, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_sell_cheb(
    const Sell<double, IT> A, const double *__restrict__ x, const double *__restrict__ f, double *__restrict__ r,
    const double *__restrict__ invd, double *__restrict__ u, double *__restrict__ dn, double a, double b,
    int first)
{
    const int lane = threadIdx.x & 63, wid = wave_id();
    const int64_t s = (int64_t)blockIdx.x * SELL_WAVES + wid;
    if (s >= A.nslices) return;
    const int64_t row = A.row_of(s * SLICE + lane);
    double acc = 0.0;
    sell_row<SLICE, 2>(A, s, lane, [&](const double *v, const int *c) {
#pragma unroll
        for (int t = 0; t < 8; t++) acc = fma(v[t], ld32(x, c[t]), acc);
    });
    if (row < 0) return;
    if (MODE == 0) {
        const double rr = f[row] - acc;
        r[row] = rr;
        dn[row] = b * (invd[row] * rr);
    } else {
        const double dold = x[row];
        u[row] = first ? dold : u[row] + dold;
        const double rr = (first ? f[row] : r[row]) - acc;
        r[row] = rr;
        if (MODE == 1) dn[row] = a * dold + b * (invd[row] * rr);
    }
}

// ---- CSR with LPR lanes per row ---------------------------------------------
//
// The coarse matrices and transfer operators of the smoothed hierarchy have few
// rows of hundreds to thousands of entries: one lane per row leaves the GPU
// nearly empty and each lane walks its row serially.  Here LPR consecutive lanes
// (8..64) share a row, stride through its entries (coalesced loads of values and
// int32 columns), and reduce by a butterfly within the group; the group's first
// lane writes, so the result does not depend on which lane is asked.
template <int LPR>
__device__ inline double csr_row(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                 const double *__restrict__ v, const double *__restrict__ x, int64_t row, int sub)
{
    // four independent chains (column load -> gather -> fma) per lane, summed
    // in a fixed order at the end
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    const int64_t e1 = rp[row + 1];
    int64_t e = rp[row] + sub;
    for (; e + 3 * LPR < e1; e += 4 * LPR) {
        const int32_t c0 = __builtin_nontemporal_load(ci + e), c1 = __builtin_nontemporal_load(ci + e + LPR);
        const int32_t c2 = __builtin_nontemporal_load(ci + e + 2 * LPR), c3 = __builtin_nontemporal_load(ci + e + 3 * LPR);
        a0 = fma(__builtin_nontemporal_load(v + e), x[c0], a0);
        a1 = fma(__builtin_nontemporal_load(v + e + LPR), x[c1], a1);
        a2 = fma(__builtin_nontemporal_load(v + e + 2 * LPR), x[c2], a2);
        a3 = fma(__builtin_nontemporal_load(v + e + 3 * LPR), x[c3], a3);
    }
    for (; e < e1; e += LPR) a0 = fma(__builtin_nontemporal_load(v + e), x[__builtin_nontemporal_load(ci + e)], a0);
    double acc = (a0 + a1) + (a2 + a3);
#pragma unroll
    for (int o = LPR / 2; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    return acc;
}

// Chebyshev pass (modes of k_sell_cheb) over a CSR image.
template <int LPR, int MODE>
__global__ __launch_bounds__(256) void k_csr_cheb(int64_t nrows, const int64_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                  const double *__restrict__ x, const double *__restrict__ f,
                                                  double *__restrict__ r, const double *__restrict__ invd,
                                                  double *__restrict__ u, double *__restrict__ dn, double a, double b,
                                                  int first)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t row = t / LPR;
    const int sub = (int)(t % LPR);
    if (row >= nrows) return;   // whole groups leave together
    const double acc = csr_row<LPR>(rp, ci, v, x, row, sub);
    if (sub != 0) return;
    if (MODE == 0) {
        const double rr = f[row] - acc;
        r[row] = rr;
        dn[row] = b * (invd[row] * rr);
    } else {
        const double dold = x[row];
        u[row] = first ? dold : u[row] + dold;
        const double rr = (first ? f[row] : r[row]) - acc;
        r[row] = rr;
        if (MODE == 1) dn[row] = a * dold + b * (invd[row] * rr);
    }
}

// y = acc (EPI_SPMV), f + acc (EPI_ADD) or f - acc (EPI_RESID) over a CSR image.
template <int LPR, int EPI>
__global__ __launch_bounds__(256) void k_csr_apply(int64_t nrows, const int64_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                   const double *__restrict__ x, const double *__restrict__ f,
                                                   double *__restrict__ y)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t row = t / LPR;
    const int sub = (int)(t % LPR);
    if (row >= nrows) return;
    const double acc = csr_row<LPR>(rp, ci, v, x, row, sub);
    if (sub != 0) return;
    if (EPI == EPI_ADD) y[row] = f[row] + acc;
    else if (EPI == EPI_RESID) y[row] = f[row] - acc;
    else y[row] = acc;
}

constexpr int CG_THREADS = 1024;
constexpr int CG_WAVES = CG_THREADS / 64;
constexpr int CG_MAXN = 2000;   // the coarsest level never exceeds 2000 rows

// Sums of two per-thread values over the block, the same bits in every thread:
// butterfly within each wave, lane 0 publishes, every thread adds the wave
// sums in index order.
__device__ inline void cg_sum2(double &a, double &b, double *lds /* 2 * CG_WAVES */)
{
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) { lds[wid] = a; lds[CG_WAVES + wid] = b; }
    __syncthreads();
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < CG_WAVES; w++) { sa += lds[w]; sb += lds[CG_WAVES + w]; }
    a = sa;
    b = sb;
}

// Coarsest-level solve of Sec. 5.1: CG preconditioned by one Jacobi sweep
// (z = dj r, dj = 1 / k_ii) from x = 0, stopped when ||r|| <= tol ||b|| on the
// recursive residual or after itmax iterations, or when (p, K p) <= 0.  One
// workgroup; vectors in LDS; the matrix (CSR, int32) is read from global
// memory (L2-resident at these sizes), one wavefront per row.  Every scalar is
// formed identically in all threads, so the loop exits uniformly.
__global__ __launch_bounds__(CG_THREADS) void k_coarse_cg(int n, const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ ci,
                                                          const double *__restrict__ v,
                                                          const double *__restrict__ dj,
                                                          const double *__restrict__ bvec, double *__restrict__ xout,
                                                          double tol, int itmax)
{
    __shared__ double xs[CG_MAXN], rs[CG_MAXN], ps[CG_MAXN], qs[CG_MAXN];
    __shared__ double red[2 * CG_WAVES];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double bb = 0.0, rz = 0.0;
    for (int i = tid; i < n; i += CG_THREADS) {
        const double bi = bvec[i], zi = dj[i] * bi;
        xs[i] = 0.0;
        rs[i] = bi;
        ps[i] = zi;
        bb += bi * bi;
        rz += bi * zi;
    }
    cg_sum2(bb, rz, red);
    const double nb = sqrt(bb);
    if (nb > 0.0) {
        for (int it = 0; it < itmax; it++) {
            // q = K p, one wavefront per row
            for (int row = wid; row < n; row += CG_WAVES) {
                double s = 0.0;
                for (int e = rp[row] + lane; e < rp[row + 1]; e += 64) s = fma(v[e], ps[ci[e]], s);
                s = wave_sum(s);
                if (lane == 0) qs[row] = s;
            }
            __syncthreads();
            double pq = 0.0, unused = 0.0;
            for (int i = tid; i < n; i += CG_THREADS) pq += ps[i] * qs[i];
            cg_sum2(pq, unused, red);
            if (!(pq > 0.0)) break;
            const double alpha = rz / pq;
            double rr = 0.0, rzn = 0.0;
            for (int i = tid; i < n; i += CG_THREADS) {
                xs[i] = xs[i] + alpha * ps[i];
                const double ri = rs[i] - alpha * qs[i];
                rs[i] = ri;
                rr += ri * ri;
                rzn += ri * (dj[i] * ri);
            }
            cg_sum2(rr, rzn, red);
            if (sqrt(rr) <= tol * nb) break;
            const double beta = rzn / rz;
            rz = rzn;
            for (int i = tid; i < n; i += CG_THREADS) ps[i] = dj[i] * rs[i] + beta * ps[i];
            __syncthreads();
        }
    }
    __syncthreads();
    for (int i = tid; i < n; i += CG_THREADS) xout[i] = xs[i];
}

}  // namespace amgk
