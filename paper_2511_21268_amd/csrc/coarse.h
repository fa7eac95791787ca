// Coarsest-level dense Cholesky factorization on the device (FP64), run once
// in amg_setup, and the inverse of the factor used by every coarse solve.
//
// Right-looking blocked algorithm with 16 x 16 tiles in one 256-thread block:
// for each diagonal tile, an unblocked factorization in LDS, a triangular solve
// of the panel below it, and the trailing update A_ij -= L_ik L_jk^T of every
// lower tile on the matrix cores (v_mfma_f64_16x16x4f64, four k-steps per
// 16-wide panel).  The matrix is npad x npad row-major (npad a multiple of 16;
// padding rows and columns hold the identity).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amgk {

typedef double vd4 __attribute__((ext_vector_type(4)));

// MFMA f64 16x16x4 operand layout (lane l of the wave): A element (l%16, l/16),
// B element (l/16, l%16); accumulator register r holds D(l/16 + 4r, l%16)
// (measured on gfx950).
__global__ __launch_bounds__(256) void k_chol_mfma(int npad, double *A, int *status)
{
    __shared__ double D[16][17];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int nb = npad / 16;
    for (int kb = 0; kb < nb; kb++) {
        const int k0 = kb * 16;
        {
            int i = tid >> 4, j = tid & 15;
            D[i][j] = A[(int64_t)(k0 + i) * npad + k0 + j];
        }
        __syncthreads();
        for (int j = 0; j < 16; j++) {
            if (tid == 0) {
                double d = D[j][j];
                if (!(d > 0.0)) { *status = 1; d = 1.0; }
                D[j][j] = sqrt(d);
            }
            __syncthreads();
            if (tid > j && tid < 16) D[tid][j] = D[tid][j] / D[j][j];
            __syncthreads();
            {
                int i = tid >> 4, k = tid & 15;
                if (i > j && k > j && k <= i) D[i][k] = D[i][k] - D[i][j] * D[k][j];
            }
            __syncthreads();
        }
        {
            int i = tid >> 4, j = tid & 15;
            A[(int64_t)(k0 + i) * npad + k0 + j] = j <= i ? D[i][j] : 0.0;
        }
        // panel: X L_kk^T = A_panel, one row per thread
        for (int r = k0 + 16 + tid; r < npad; r += 256) {
            double x[16];
            double *row = A + (int64_t)r * npad + k0;
            for (int j = 0; j < 16; j++) {
                double s = row[j];
                for (int m = 0; m < j; m++) s -= x[m] * D[j][m];
                x[j] = s / D[j][j];
            }
            for (int j = 0; j < 16; j++) row[j] = x[j];
        }
        __syncthreads();
        // trailing update of the lower tiles (ib >= jb > kb) on the matrix cores
        const int nrem = nb - kb - 1;
        const int ntiles = nrem * (nrem + 1) / 2;
        for (int t = wid; t < ntiles; t += 4) {
            int ib = 0, rem = t;      // enumerate (ib, jb) with jb <= ib in the remaining tiles
            while (rem > ib) { rem -= ib + 1; ib++; }
            int jb = rem;
            ib += kb + 1;
            jb += kb + 1;
            double *Ct = A + (int64_t)(ib * 16) * npad + jb * 16;
            const double *Li = A + (int64_t)(ib * 16) * npad + k0;
            const double *Lj = A + (int64_t)(jb * 16) * npad + k0;
            vd4 acc;
            for (int r = 0; r < 4; r++) acc[r] = Ct[(int64_t)((lane >> 4) + 4 * r) * npad + (lane & 15)];
            for (int s = 0; s < 4; s++) {
                double a = -Li[(int64_t)(lane & 15) * npad + 4 * s + (lane >> 4)];
                double b = Lj[(int64_t)(lane & 15) * npad + 4 * s + (lane >> 4)];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
            for (int r = 0; r < 4; r++) Ct[(int64_t)((lane >> 4) + 4 * r) * npad + (lane & 15)] = acc[r];
        }
        __syncthreads();
    }
}

// Inverse of the lower factor by forward substitution, one column per thread;
// writes L^{-1} (row-major, lower) and its transpose.
__global__ __launch_bounds__(256) void k_tri_inv(int n, int npad, const double *__restrict__ L,
                                                 double *__restrict__ Linv, double *__restrict__ LinvT)
{
    for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256) {
        for (int i = 0; i < j; i++) {
            Linv[(int64_t)i * npad + j] = 0.0;
            LinvT[(int64_t)j * npad + i] = 0.0;
        }
        double xjj = 1.0 / L[(int64_t)j * npad + j];
        Linv[(int64_t)j * npad + j] = xjj;
        LinvT[(int64_t)j * npad + j] = xjj;
        for (int i = j + 1; i < n; i++) {
            const double *row = L + (int64_t)i * npad;
            double s = 0.0;
            for (int k = j; k < i; k++) s = fma(row[k], Linv[(int64_t)k * npad + j], s);
            double xij = -s / row[i];
            Linv[(int64_t)i * npad + j] = xij;
            LinvT[(int64_t)j * npad + i] = xij;
        }
    }
}

}  // namespace amgk
