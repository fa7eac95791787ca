// Kernels of the block flexible CG for up to NB = 16 right-hand sides (O'Leary's
// block CG with the coefficients of flexible CG): per iteration
//     Q = K P,  G = P^T Q,  alpha = G^{-1} P^T R,  X += P alpha,  R -= Q alpha,
//     Z = B R,  beta = -G^{-1} Q^T Z,  P = Z + P beta,
// over the columns still active (a converged column leaves the block).  Block
// vectors are the row-major N x 16 arrays of the batched solve.
#pragma once
#include "kernels_blk.h"

namespace amgk {

constexpr int GRAM_BLOCKS = 512;   // fixed grid of the Gram-matrix partials

// Partials of A^T B and A^T C (16 x 16 each; C may be NULL): 16-row tiles of
// A, B, C staged in LDS; thread (i, j) = (t / 16, t % 16) accumulates
// A_ri B_rj over the block's rows in ascending order.  The tiles of a block
// are chunk = blockIdx.x, blockIdx.x + GRAM_BLOCKS, ...
__global__ __launch_bounds__(256) void k_gram2(int64_t n, const double *__restrict__ A, const double *__restrict__ B,
                                               const double *__restrict__ Cm, double *__restrict__ partial)
{
    __shared__ double as[16][NB], bs[16][NB], cs[16][NB];
    const int t = threadIdx.x, i = t >> 4, j = t & 15;
    double g1 = 0.0, g2 = 0.0;
    for (int64_t r0 = (int64_t)blockIdx.x * 16; r0 < n; r0 += (int64_t)gridDim.x * 16) {
        const int64_t row = r0 + i;
        const bool in = row < n;
        as[i][j] = in ? A[row * NB + j] : 0.0;
        bs[i][j] = in ? B[row * NB + j] : 0.0;
        if (Cm) cs[i][j] = in ? Cm[row * NB + j] : 0.0;
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < 16; rr++) {
            g1 = fma(as[rr][i], bs[rr][j], g1);
            if (Cm) g2 = fma(as[rr][i], cs[rr][j], g2);
        }
        __syncthreads();
    }
    partial[(int64_t)blockIdx.x * 512 + t] = g1;
    partial[(int64_t)blockIdx.x * 512 + 256 + t] = g2;
}

// Final Gram sums (blocks in index order) and the small solve on the active
// columns S (bactive):
//   mode 0: G = first Gram (stored in gsave), H = second (P^T R);
//           coef = G_SS^{-1} H_SS                       (alpha)
//   mode 1: G = gsave, W = first Gram (Q^T Z);
//           coef = -G_SS^{-1} W_SS                      (beta)
// coef is 16 x 16 row-major (direction i, column j), zero outside S x S.  A
// non-positive pivot marks every active column broken (flag slot).
__global__ __launch_bounds__(256) void k_bcg_small(int nblk, const double *__restrict__ partial, double *sc,
                                                   double *__restrict__ gsave, double *__restrict__ coef, int mode)
{
    __shared__ double G[256], H[256], L[256], Y[256];
    __shared__ int idx[NB];
    const int t = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int k = 0; k < nblk; k++) {
        a += partial[(int64_t)k * 512 + t];
        b += partial[(int64_t)k * 512 + 256 + t];
    }
    if (mode == 0) {
        G[t] = a;
        gsave[t] = a;
        H[t] = b;
    } else {
        G[t] = gsave[t];
        H[t] = -a;
    }
    coef[t] = 0.0;
    __syncthreads();
    if (t != 0) return;
    int m = 0;
    for (int j = 0; j < NB; j++)
        if (bactive(sc, j)) idx[m++] = j;
    // Cholesky of G_SS
    for (int r = 0; r < m; r++)
        for (int c = 0; c <= r; c++) {
            double s = G[idx[r] * NB + idx[c]];
            for (int k = 0; k < c; k++) s -= L[r * NB + k] * L[c * NB + k];
            if (r == c) {
                if (!(s > 0.0) || !isfinite(s)) {
                    for (int q = 0; q < m; q++) sc[B_FLAG * NB + idx[q]] = 3.0;
                    return;
                }
                L[r * NB + r] = sqrt(s);
            } else {
                L[r * NB + c] = s / L[c * NB + c];
            }
        }
    // Y = G_SS^{-1} H_SS, column by column
    for (int c = 0; c < m; c++) {
        for (int r = 0; r < m; r++) {
            double s = H[idx[r] * NB + idx[c]];
            for (int k = 0; k < r; k++) s -= L[r * NB + k] * Y[k * NB + c];
            Y[r * NB + c] = s / L[r * NB + r];
        }
        for (int r = m - 1; r >= 0; r--) {
            double s = Y[r * NB + c];
            for (int k = r + 1; k < m; k++) s -= L[k * NB + r] * Y[k * NB + c];
            Y[r * NB + c] = s / L[r * NB + r];
        }
    }
    for (int r = 0; r < m; r++)
        for (int c = 0; c < m; c++) coef[idx[r] * NB + idx[c]] = Y[r * NB + c];
}

// X += P alpha ; R -= Q alpha (element-parallel; row r = e / 16, column j);
// per-column partials of (R, R) as k_bcg_update.
__global__ __launch_bounds__(256) void k_bcg_xr(int64_t n, const double *__restrict__ alpha, double *__restrict__ X,
                                                double *__restrict__ R, const double *__restrict__ P,
                                                const double *__restrict__ Q, double *__restrict__ partial)
{
    __shared__ double al[256];
    __shared__ double lds[8 * NB];
    al[threadIdx.x] = alpha[threadIdx.x];
    __syncthreads();
    const int j = threadIdx.x & (NB - 1);
    double s = 0.0;
    const int64_t m = n * NB;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < m; e += (int64_t)gridDim.x * 256) {
        const int64_t r = e >> 4;
        double dx = 0.0, dr = 0.0;
#pragma unroll
        for (int i = 0; i < NB; i++) {
            const double a = al[i * NB + j];
            dx = fma(P[r * NB + i], a, dx);
            dr = fma(Q[r * NB + i], a, dr);
        }
        X[e] = X[e] + dx;
        const double ri = R[e] - dr;
        R[e] = ri;
        s = fma(ri, ri, s);
    }
    blk_col_partials(s, 0.0, lds, partial);
}

// Pn = Z + P beta (element-parallel)
__global__ __launch_bounds__(256) void k_bcg_p(int64_t n, const double *__restrict__ beta, const double *__restrict__ Z,
                                               const double *__restrict__ P, double *__restrict__ Pn)
{
    __shared__ double be[256];
    be[threadIdx.x] = beta[threadIdx.x];
    __syncthreads();
    const int j = threadIdx.x & (NB - 1);
    const int64_t m = n * NB;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < m; e += (int64_t)gridDim.x * 256) {
        const int64_t r = e >> 4;
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < NB; i++) t = fma(P[r * NB + i], be[i * NB + j], t);
        Pn[e] = Z[e] + t;
    }
}

}  // namespace amgk
