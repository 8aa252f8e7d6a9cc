// lm_dense.hip -- dense Cholesky factor of the kernel matrix K(X) and triangular solves.
//
// Algorithm 1 converts velocities into momenta with K(X)^{-1} at the fixed template X, once
// per iteration.  K(X) is symmetric positive definite (both kernels are positive-definite
// radial functions) and does not change during a match, so it is factored once,
// K + tau I = L L^T, and every iteration then costs two triangular sweeps over L.  At
// N = 65536 the factor is 34 GB, resident in HBM.
//
// Layout: K is row-major n x n (leading dimension n); only the lower triangle is built, read
// or written (the upper triangle of the diagonal tiles may hold scratch).  Blocked
// right-looking factorisation with panels of kPanel = 128 columns:
//   1. lm_potrf_diag_kernel  -- factor the 128 x 128 diagonal block in LDS (one workgroup);
//   2. lm_trinv_kernel       -- invert that triangular block (kept: the sweeps reuse it);
//   3. lm_panel_kernel       -- panel rows below: A_ik <- A_ik L_kk^{-T} (one workgroup per
//                               64 rows, the rows staged in LDS);
//   4. lm_syrk_kernel        -- trailing update A_ij -= A_ik A_jk^T on 64 x 64 lower tiles,
//                               FP64 MFMA (v_mfma_f64_16x16x4f64): the only dense
//                               contraction of the path, N^3/3 flops.
// Solves: blocked forward (L y = b) and backward (L^T x = y) sweeps, one launch per panel;
// in launch k every workgroup subtracts panel k's contribution from its rows, and the
// workgroup that owns block k+1 (k-1 backward) then finishes that block with the stored
// inverse of its diagonal block.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lm_internal.h"
#include "lm_math.h"

namespace lm {

constexpr int kPanel = 128;

// ---------------------------------------------------------------------------------------
// K_ij = G(|X_i - X_j|) (+ tau on the diagonal) for j <= i.  One workgroup per row.
// ---------------------------------------------------------------------------------------
template <int DIM, int KER>
__global__ __launch_bounds__(256) void lm_kbuild_kernel(const double* __restrict__ X, int64_t n, double kq,
                                                        double tau, double* __restrict__ K)
{
    const int64_t i = blockIdx.x;
    double xi[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) xi[c] = X[c * n + i];
    double* row = K + i * n;
    for (int64_t j = threadIdx.x; j <= i; j += blockDim.x) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const double d = xi[c] - X[c * n + j];
            s = __builtin_fma(d, d, s);
        }
        const double a = (KER == LM_KERNEL_CONON) ? __builtin_sqrt(s) * kq : s * kq;
        row[j] = exp_nonpos(a) + (j == i ? tau : 0.0);
    }
}

// ---------------------------------------------------------------------------------------
// Diagonal block: unblocked right-looking Cholesky of the bs x bs block at (k0, k0), held in
// LDS in packed lower-triangular form (bs <= 128: 8256 doubles).  A non-positive pivot sets
// *info = k0 + j + 1 (the factor is then meaningless).
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int pk(int r, int c) { return r * (r + 1) / 2 + c; }

__global__ __launch_bounds__(256) void lm_potrf_diag_kernel(double* __restrict__ K, int64_t n, int64_t k0, int bs,
                                                            int* __restrict__ info)
{
    __shared__ double L[kPanel * (kPanel + 1) / 2];
    const int tid = threadIdx.x;
    const int ne = bs * (bs + 1) / 2;
    for (int e = tid; e < ne; e += blockDim.x) {
        // invert the packed index: row r with r(r+1)/2 <= e
        int r = (int)((__builtin_sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while (pk(r + 1, 0) <= e) ++r;
        while (pk(r, 0) > e) --r;
        const int c = e - pk(r, 0);
        L[e] = K[(k0 + r) * n + k0 + c];
    }
    __syncthreads();
    for (int j = 0; j < bs; ++j) {
        const double d = L[pk(j, j)];
        const bool ok = d > 0.0;
        const double ljj = ok ? __builtin_sqrt(d) : __builtin_nan("");
        __syncthreads();
        if (tid == 0) {
            L[pk(j, j)] = ljj;
            if (!ok && *info == 0) *info = (int)(k0 + j + 1);
        }
        for (int r = j + 1 + tid; r < bs; r += blockDim.x) L[pk(r, j)] /= ljj;
        __syncthreads();
        // trailing update of the block: L[r][c] -= L[r][j] L[c][j], j < c <= r
        const int m = bs - j - 1;
        const int cnt = m * (m + 1) / 2;
        for (int e = tid; e < cnt; e += blockDim.x) {
            int rr = (int)((__builtin_sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
            while (pk(rr + 1, 0) <= e) ++rr;
            while (pk(rr, 0) > e) --rr;
            const int cc = e - pk(rr, 0);
            const int r = j + 1 + rr, c = j + 1 + cc;
            L[pk(r, c)] -= L[pk(r, j)] * L[pk(c, j)];
        }
        __syncthreads();
    }
    for (int e = tid; e < ne; e += blockDim.x) {
        int r = (int)((__builtin_sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while (pk(r + 1, 0) <= e) ++r;
        while (pk(r, 0) > e) --r;
        const int c = e - pk(r, 0);
        K[(k0 + r) * n + k0 + c] = L[e];
    }
}

// ---------------------------------------------------------------------------------------
// Inverse of the lower-triangular diagonal block at (k0, k0): Linv (kPanel x kPanel,
// row-major, zero above the diagonal and outside bs).  Thread j computes column j by forward
// substitution; the block is read from LDS (packed).
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kPanel) void lm_trinv_kernel(const double* __restrict__ K, int64_t n, int64_t k0, int bs,
                                                          double* __restrict__ Linv)
{
    __shared__ double L[kPanel * (kPanel + 1) / 2];
    const int j = threadIdx.x;
    const int ne = bs * (bs + 1) / 2;
    for (int e = j; e < ne; e += blockDim.x) {
        int r = (int)((__builtin_sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while (pk(r + 1, 0) <= e) ++r;
        while (pk(r, 0) > e) --r;
        const int c = e - pk(r, 0);
        L[e] = K[(k0 + r) * n + k0 + c];
    }
    __syncthreads();
    for (int r = 0; r < kPanel; ++r) Linv[r * kPanel + j] = 0.0;
    if (j >= bs) return;
    // x_r = 0 for r < j ; x_j = 1/L_jj ; x_r = -(sum_{l=j}^{r-1} L_rl x_l)/L_rr
    Linv[j * kPanel + j] = 1.0 / L[pk(j, j)];
    for (int r = j + 1; r < bs; ++r) {
        double s = 0.0;
        for (int l = j; l < r; ++l) s = __builtin_fma(L[pk(r, l)], Linv[l * kPanel + j], s);
        Linv[r * kPanel + j] = -s / L[pk(r, r)];
    }
}

// ---------------------------------------------------------------------------------------
// Panel below the diagonal block: rows i in [k0+bs, n), columns [k0, k0+bs):
// A_ik <- A_ik L_kk^{-T}, i.e. A[i][c] = sum_{m <= c} A[i][m] Linv[c][m].  One workgroup per
// 64 rows; the rows are staged in LDS so the update can be written in place.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void lm_panel_kernel(double* __restrict__ K, int64_t n, int64_t k0, int bs,
                                                       const double* __restrict__ Linv)
{
    __shared__ double rows[64][kPanel + 1];
    const int64_t r0 = k0 + bs + (int64_t)blockIdx.x * 64;
    const int nr = (int)((n - r0) < 64 ? (n - r0) : 64);
    for (int e = threadIdx.x; e < 64 * kPanel; e += blockDim.x) {
        const int r = e / kPanel, c = e % kPanel;
        rows[r][c] = (r < nr && c < bs) ? K[(r0 + r) * n + k0 + c] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nr * bs; e += blockDim.x) {
        const int r = e / bs, c = e % bs;
        const double* li = Linv + c * kPanel;
        double s = 0.0;
        for (int m = 0; m <= c; ++m) s = __builtin_fma(rows[r][m], li[m], s);
        K[(r0 + r) * n + k0 + c] = s;
    }
}

// ---------------------------------------------------------------------------------------
// Trailing update A_ij -= sum_m A[i][k0+m] A[j][k0+m] over the lower 64 x 64 tiles of the
// trailing matrix (rows/cols from t0 = k0 + bs).  Workgroup = 4 waves, wave w computes the
// 32 x 32 quarter (w/2, w%2) as 2 x 2 blocks of v_mfma_f64_16x16x4f64.  Operand layout of
// that instruction (lane l), as measured on gfx950: A[l%16][l/16] of the 16x4 left block,
// B[l/16][l%16] of the 4x16 right block, and D[4r + l/16][l%16] in accumulator element r.
// ---------------------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void lm_syrk_kernel(double* __restrict__ K, int64_t n, int64_t k0, int bs)
{
    constexpr int KC = 32;
    __shared__ double Ai[64][KC + 1];
    __shared__ double Aj[64][KC + 1];
    const int64_t t0 = k0 + bs;
    // linear tile id -> (ti, tj), tj <= ti
    const int64_t id = blockIdx.x;
    int64_t ti = (int64_t)((__builtin_sqrt(8.0 * (double)id + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= id) ++ti;
    while (ti * (ti + 1) / 2 > id) --ti;
    const int64_t tj = id - ti * (ti + 1) / 2;
    const int64_t ri = t0 + ti * 64, rj = t0 + tj * 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;

    d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = (d4){0.0, 0.0, 0.0, 0.0};

    for (int kc = 0; kc < bs; kc += KC) {
        // stage 64 x KC of each operand: thread t loads 8 consecutive doubles of one row
        {
            const int r = tid >> 2, c0 = (tid & 3) * 8;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int c = c0 + u;
                const bool okc = kc + c < bs;
                Ai[r][c] = (okc && ri + r < n) ? K[(ri + r) * n + k0 + kc + c] : 0.0;
                Aj[r][c] = (okc && rj + r < n) ? K[(rj + r) * n + k0 + kc + c] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < KC; k4 += 4) {
            double fa[2], fb[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) fa[a] = Ai[wr * 32 + a * 16 + (lane & 15)][k4 + (lane >> 4)];
#pragma unroll
            for (int b = 0; b < 2; ++b) fb[b] = Aj[wc * 32 + b * 16 + (lane & 15)][k4 + (lane >> 4)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = ri + wr * 32 + a * 16 + 4 * r + (lane >> 4);
                const int64_t gj = rj + wc * 32 + b * 16 + (lane & 15);
                if (gi < n && gj <= gi) K[gi * n + gj] -= acc[a][b][r];
            }
}

// ---------------------------------------------------------------------------------------
// Triangular sweeps for `dim` right-hand sides (component-major vectors of length n).
// ---------------------------------------------------------------------------------------

// y_blk = Linv_blk * y_blk (forward, TRANS = false) or Linv_blk^T * y_blk (backward), for
// block `blk`, executed by one workgroup of 256 threads.
template <bool TRANS, int DIM>
__device__ void finish_block(const double* __restrict__ Linv, int64_t n, int nb, int64_t blk,
                             double* __restrict__ y, double* sh)
{
    const int64_t b0 = blk * kPanel;
    const int bs = (int)((n - b0) < kPanel ? (n - b0) : kPanel);
    const double* Li = Linv + blk * kPanel * kPanel;
    for (int e = threadIdx.x; e < DIM * kPanel; e += blockDim.x) {
        const int c = e / kPanel, r = e % kPanel;
        sh[e] = r < bs ? y[c * n + b0 + r] : 0.0;
    }
    __syncthreads();
    double out[3] = {0.0, 0.0, 0.0};
    const int r = threadIdx.x;
    if (r < bs) {
        for (int c = 0; c < DIM; ++c) {
            double s = 0.0;
            if (!TRANS) {
                for (int m = 0; m <= r; ++m) s = __builtin_fma(Li[r * kPanel + m], sh[c * kPanel + m], s);
            } else {
                for (int m = r; m < bs; ++m) s = __builtin_fma(Li[m * kPanel + r], sh[c * kPanel + m], s);
            }
            out[c] = s;
        }
    }
    __syncthreads();
    if (r < bs)
        for (int c = 0; c < DIM; ++c) y[c * n + b0 + r] = out[c];
}

// Launch k of the forward sweep (k = -1: only finish block 0).  Workgroup 0 owns block k+1:
// it subtracts L[block k+1, block k] y_k and finishes y_{k+1}; workgroups >= 1 subtract the
// contribution of y_k from the rows of blocks k+2 .. nb-1, eight rows per wave at a time.
template <int DIM>
__global__ __launch_bounds__(256) void lm_trsv_fwd_kernel(const double* __restrict__ L, const double* __restrict__ Linv,
                                                          int64_t n, int nb, int64_t k, double* __restrict__ y)
{
    __shared__ double sh[3 * kPanel];
    __shared__ double yk[3 * kPanel];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (k >= 0) {
        const int64_t k0 = k * kPanel;
        for (int e = threadIdx.x; e < DIM * kPanel; e += blockDim.x) {
            const int c = e / kPanel, m = e % kPanel;
            yk[e] = (k0 + m < n) ? y[c * n + k0 + m] : 0.0;
        }
        __syncthreads();
        // eight rows per wave at a time: lane l reads 16 consecutive doubles of row (l / 8),
        // so each row's 128 panel entries come in as one coalesced 1 KiB segment
        const int sub = lane >> 3, seg = (lane & 7) * 16;
        int64_t rbeg, rend, rstep;
        if (blockIdx.x == 0) {
            rbeg = (k + 1) * kPanel + wave * 8;
            rend = (k + 2) * kPanel < n ? (k + 2) * kPanel : n;
            rstep = 32;
        } else {
            rbeg = (k + 2) * kPanel + ((int64_t)(blockIdx.x - 1) * 4 + wave) * 8;
            rend = n;
            rstep = (int64_t)(gridDim.x - 1) * 32;
        }
        for (int64_t rb = rbeg; rb < rend; rb += rstep) {
            const int64_t r = rb + sub;
            const bool ok = r < rend;
            const double* lr = L + (ok ? r : rb) * n + k0 + seg;
            double lv[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) lv[u] = lr[u];
            double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
#pragma unroll
                for (int u = 0; u < 16; ++u) s[c] = __builtin_fma(lv[u], yk[c * kPanel + seg + u], s[c]);
#pragma unroll
                for (int o = 4; o > 0; o >>= 1) s[c] += __shfl_xor(s[c], o, 64);
            }
            if (ok && (lane & 7) == 0)
                for (int c = 0; c < DIM; ++c) y[c * n + r] -= s[c];
        }
    }
    if (blockIdx.x == 0 && k + 1 < nb) {
        __threadfence_block();
        __syncthreads();
        finish_block<false, DIM>(Linv, n, nb, k + 1, y, sh);
    }
}

// Launch k of the backward sweep (k = nb: only finish block nb-1).  Workgroup 0 owns block
// k-1: it subtracts L[block k, block k-1]^T x_k and finishes x_{k-1}; workgroups >= 1 handle
// the columns of blocks 0 .. k-2, one column per thread.
template <int DIM>
__global__ __launch_bounds__(256) void lm_trsv_bwd_kernel(const double* __restrict__ L, const double* __restrict__ Linv,
                                                          int64_t n, int nb, int64_t k, double* __restrict__ y)
{
    __shared__ double sh[3 * kPanel];
    __shared__ double xk[3 * kPanel];
    if (k < nb) {
        const int64_t k0 = k * kPanel;
        const int bs = (int)((n - k0) < kPanel ? (n - k0) : kPanel);
        for (int e = threadIdx.x; e < DIM * kPanel; e += blockDim.x) {
            const int c = e / kPanel, m = e % kPanel;
            xk[e] = m < bs ? y[c * n + k0 + m] : 0.0;
        }
        __syncthreads();
        int64_t cbeg, cend, cstep;
        if (blockIdx.x == 0) {
            cbeg = (k - 1) * kPanel + threadIdx.x;
            cend = k * kPanel;
            cstep = blockDim.x;
        } else {
            cbeg = (int64_t)(blockIdx.x - 1) * blockDim.x + threadIdx.x;
            cend = (k - 1) * kPanel;
            cstep = (int64_t)(gridDim.x - 1) * blockDim.x;
        }
        for (int64_t col = cbeg; col < cend; col += cstep) {
            double s[3] = {0.0, 0.0, 0.0};
            const double* lc = L + k0 * n + col;
            // sixteen independent loads in flight per thread (zeros past a ragged block end)
            for (int m0 = 0; m0 < kPanel; m0 += 16) {
                double lv[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) lv[u] = (m0 + u < bs) ? lc[(int64_t)(m0 + u) * n] : 0.0;
                for (int c = 0; c < DIM; ++c)
#pragma unroll
                    for (int u = 0; u < 16; ++u) s[c] = __builtin_fma(lv[u], xk[c * kPanel + m0 + u], s[c]);
            }
            for (int c = 0; c < DIM; ++c) y[c * n + col] -= s[c];
        }
    }
    if (blockIdx.x == 0 && k - 1 >= 0) {
        __threadfence_block();
        __syncthreads();
        finish_block<true, DIM>(Linv, n, nb, k - 1, y, sh);
    }
}

// ---------------------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------------------

__global__ void lm_int_zero_kernel(int* p) { if (threadIdx.x == 0) *p = 0; }

int dense_panels(int64_t n) { return (int)((n + kPanel - 1) / kPanel); }
int64_t dense_linv_elems(int64_t n) { return (int64_t)dense_panels(n) * kPanel * kPanel; }

hipError_t launch_dense_factor(int dim, int kernel, double kq, double tau, const double* X, int64_t n, double* K,
                               double* Linv, int* info, hipStream_t st)
{
    hipLaunchKernelGGL(lm_int_zero_kernel, dim3(1), dim3(64), 0, st, info);
    if (dim == 2) {
        if (kernel == LM_KERNEL_CONON)
            hipLaunchKernelGGL((lm_kbuild_kernel<2, LM_KERNEL_CONON>), dim3((unsigned)n), dim3(256), 0, st, X, n, kq, tau, K);
        else
            hipLaunchKernelGGL((lm_kbuild_kernel<2, LM_KERNEL_GAUSS>), dim3((unsigned)n), dim3(256), 0, st, X, n, kq, tau, K);
    } else {
        if (kernel == LM_KERNEL_CONON)
            hipLaunchKernelGGL((lm_kbuild_kernel<3, LM_KERNEL_CONON>), dim3((unsigned)n), dim3(256), 0, st, X, n, kq, tau, K);
        else
            hipLaunchKernelGGL((lm_kbuild_kernel<3, LM_KERNEL_GAUSS>), dim3((unsigned)n), dim3(256), 0, st, X, n, kq, tau, K);
    }
    const int nb = dense_panels(n);
    for (int b = 0; b < nb; ++b) {
        const int64_t k0 = (int64_t)b * kPanel;
        const int bs = (int)((n - k0) < kPanel ? (n - k0) : kPanel);
        hipLaunchKernelGGL(lm_potrf_diag_kernel, dim3(1), dim3(256), 0, st, K, n, k0, bs, info);
        hipLaunchKernelGGL(lm_trinv_kernel, dim3(1), dim3(kPanel), 0, st, (const double*)K, n, k0, bs,
                           Linv + (int64_t)b * kPanel * kPanel);
        const int64_t rest = n - k0 - bs;
        if (rest <= 0) continue;
        hipLaunchKernelGGL(lm_panel_kernel, dim3((unsigned)((rest + 63) / 64)), dim3(256), 0, st, K, n, k0, bs,
                           (const double*)(Linv + (int64_t)b * kPanel * kPanel));
        const int64_t nt = (rest + 63) / 64;
        hipLaunchKernelGGL(lm_syrk_kernel, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, st, K, n, k0, bs);
    }
    return hipGetLastError();
}

hipError_t launch_dense_solve(const double* L, const double* Linv, int64_t n, int dim, double* y, hipStream_t st)
{
    const int nb = dense_panels(n);
    // enough workgroups to stream a panel at full bandwidth, never more than its rows need
    auto groups = [&](int64_t items, int64_t per_group) -> unsigned {
        int64_t g = 1 + (items + per_group - 1) / per_group;
        return (unsigned)(g < 2049 ? g : 2049);
    };
    for (int64_t k = -1; k < nb - 1; ++k) {
        const int64_t below = n - (k + 2) * kPanel;
        const dim3 g(k < 0 ? 1u : groups(below > 0 ? below : 0, 32));
        if (dim == 2)
            hipLaunchKernelGGL(lm_trsv_fwd_kernel<2>, g, dim3(256), 0, st, L, Linv, n, nb, k, y);
        else
            hipLaunchKernelGGL(lm_trsv_fwd_kernel<3>, g, dim3(256), 0, st, L, Linv, n, nb, k, y);
    }
    for (int64_t k = nb; k > 0; --k) {
        const int64_t above = (k - 1) * kPanel;
        const dim3 g(k == nb ? 1u : groups(above, 256));
        if (dim == 2)
            hipLaunchKernelGGL(lm_trsv_bwd_kernel<2>, g, dim3(256), 0, st, L, Linv, n, nb, k, y);
        else
            hipLaunchKernelGGL(lm_trsv_bwd_kernel<3>, g, dim3(256), 0, st, L, Linv, n, nb, k, y);
    }
    return hipGetLastError();
}

}  // namespace lm
