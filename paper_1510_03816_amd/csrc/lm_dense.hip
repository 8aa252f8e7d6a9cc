// lm_dense.hip -- dense Cholesky factor of the kernel matrix K(X) and triangular solves.
//
// Algorithm 1 converts velocities into momenta with K(X)^{-1} at the fixed template X, once
// per iteration.  K(X) is symmetric positive definite (both kernels are positive-definite
// radial functions) and does not change during a match, so it is factored once,
// K + tau I = L L^T, and every iteration then costs two triangular sweeps over L.  At
// N = 65536 the factor is 34 GB, resident in HBM.
//
// Layout: K is row-major n x n (leading dimension n); only the lower triangle is built, read
// or written.  Blocked right-looking factorisation with panels of kPanel = 128 columns, the
// trailing matrix updated once per block of kOuter panels:
//   1. lm_potrf_inv_kernel -- factor the 128 x 128 diagonal block in LDS and invert it (the
//                             inverse is kept: the panel solve and the sweeps reuse it);
//   2. lm_panel_kernel     -- panel rows below: A_ik <- A_ik L_kk^{-T} (FP64 MFMA);
//   3. lm_syrk_kernel      -- within a block, the next panel's column strip takes the
//                             updates of the block's earlier panels (64 x 64 tiles);
//   4. lm_syrk128_kernel   -- after the block, the trailing update A_ij -= A_ik A_jk^T
//                             (128 x 128 tiles; 64 x 64 once the trailing matrix is small):
//                             the only large dense contraction of the path, N^3/3 flops.
// Solves: blocked forward (L y = b) and backward (L^T x = y) sweeps, one launch per panel;
// in launch k every workgroup subtracts panel k's contribution from its rows, and the
// workgroup that owns block k+1 (k-1 backward) then finishes that block with the stored
// inverse of its diagonal block.  The panel kernel also writes each panel transposed into
// the unused upper triangle, where the forward sweep reads it as contiguous rows.  Large
// factors use the superblock form instead (three launches per 8 blocks, through the stored
// inverses of the diagonal superblocks; below the batched solves).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "lm_internal.h"
#include "lm_math.h"

namespace lm {

constexpr int kPanel = 128;

// Panels per trailing update (the update of a block of kOuter panels reads and writes the
// trailing matrix once; measured on MI355X at N = 65536: 5.8 s for 1 panel, 4.7 s for 2, 4.3 s
// for 8 with the other kernels then in use).
constexpr int kOuter = 8;

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
        row[j] = exp2_nonpos_fine(a) + (j == i ? tau : 0.0);
    }
}

// ---------------------------------------------------------------------------------------
// Diagonal block, factor and inverse in one pass: the bs x bs block at (k0, k0) is held in
// LDS as a full 128 x 129 array.  Cholesky is left-looking by columns: for column c, a group
// of threads per row r >= c (2 while more than 64 rows remain, up to 64 for the last few)
// forms A_rc - sum_{k<c} L_rk L_ck, the pivot thread takes the square root, and the rows
// below divide by it.  A non-positive pivot sets *info = k0 + c + 1 (the factor is then
// meaningless).  The inverse is then formed by forward substitution, two threads per column
// j of Linv, whose entries (r >= j) are kept in the unused upper triangle at A[j][r + 1].
// Outputs: the factor written back over the block, Linv (kPanel x kPanel, row-major, zero
// above the diagonal and outside bs) and its transpose LinvT (the triangular sweeps read rows
// of both).  The dot products keep eight LDS loads in flight (one at a time left every
// iteration waiting out the LDS latency: 0.36 ms per block, now 0.23 ms on MI355X); the
// kernel stays bound by the latency of its dependent column steps.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void lm_potrf_inv_kernel(double* __restrict__ K, int64_t n, int64_t k0, int bs,
                                                           double* __restrict__ Linv, double* __restrict__ LinvT,
                                                           int* __restrict__ info)
{
    __shared__ double A[kPanel][kPanel + 1];
    __shared__ double rdiag[kPanel];
    const int tid = threadIdx.x;
    // global loads are issued in batches of 8 before any is stored (a load-store loop would
    // wait out the memory latency once per element)
    for (int e0 = tid; e0 < kPanel * kPanel; e0 += 8 * 256) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + 256 * u, r = e / kPanel, c = e % kPanel;
            v[u] = (r < bs && c <= r) ? K[(k0 + r) * n + k0 + c] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + 256 * u;
            A[e / kPanel][e % kPanel] = v[u];
        }
    }
    __syncthreads();
    for (int c = 0; c < bs; ++c) {
        // tpr threads per row r >= c (as many as the 256 threads cover, 2 to 64), thread h of a
        // row summing k = h, h + tpr, ... with eight loads in flight and four accumulators
        const int rows = bs - c;
        const int tpr = rows > 64 ? 2 : rows > 32 ? 4 : rows > 16 ? 8 : rows > 8 ? 16 : rows > 4 ? 32 : 64;
        const int h = tid & (tpr - 1), r = c + tid / tpr;
        double v = 0.0;
        if (r < bs) {
            double s4[4] = {0.0, 0.0, 0.0, 0.0};
            int k = h;
            for (; k + 7 * tpr < c; k += 8 * tpr) {
                double x[8], y[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    x[u] = A[r][k + u * tpr];
                    y[u] = A[c][k + u * tpr];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) s4[u & 3] = __builtin_fma(x[u], y[u], s4[u & 3]);
            }
            for (; k < c; k += tpr) s4[0] = __builtin_fma(A[r][k], A[c][k], s4[0]);
            v = (s4[0] + s4[1]) + (s4[2] + s4[3]);
        }
        for (int o = 1; o < tpr; o <<= 1) v += __shfl_xor(v, o);
        if (r < bs) v = A[r][c] - v;
        if (r == c && h == 0) {
            const bool ok = v > 0.0;
            A[c][c] = ok ? __builtin_sqrt(v) : __builtin_nan("");
            if (!ok && *info == 0) *info = (int)(k0 + c + 1);
        }
        __syncthreads();
        if (r > c && r < bs && h == 0) A[r][c] = v / A[c][c];
        __syncthreads();
    }
    for (int e = tid; e < kPanel * kPanel; e += blockDim.x) {
        const int r = e / kPanel, c = e % kPanel;
        if (r < bs && c <= r) K[(k0 + r) * n + k0 + c] = A[r][c];
    }
    // inverse: x_j = 1/L_jj, x_r = -(sum_{l=j}^{r-1} L_rl x_l) / L_rr, two threads per
    // column j (l = j + h, j + h + 2, ...; eight loads in flight, four accumulators).  Both
    // threads of a pair compute and store every x_r, so each reads back only its own stores.
    if (tid < bs) rdiag[tid] = 1.0 / A[tid][tid];
    __syncthreads();
    const int h = tid & 1, j = tid >> 1;
    if (j < bs) {
        A[j][j + 1] = rdiag[j];
        for (int r = j + 1; r < bs; ++r) {
            double s4[4] = {0.0, 0.0, 0.0, 0.0};
            int l = j + h;
            for (; l + 14 < r; l += 16) {
                double x[8], y[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    x[u] = A[r][l + 2 * u];
                    y[u] = A[j][l + 2 * u + 1];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) s4[u & 3] = __builtin_fma(x[u], y[u], s4[u & 3]);
            }
            for (; l < r; l += 2) s4[0] = __builtin_fma(A[r][l], A[j][l + 1], s4[0]);
            double s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
            s += __shfl_xor(s, 1);
            A[j][r + 1] = -s * rdiag[r];
        }
    }
    __syncthreads();
    for (int e = tid; e < kPanel * kPanel; e += blockDim.x) {
        const int r = e / kPanel, c = e % kPanel;
        Linv[e] = (r < bs && c <= r) ? A[c][r + 1] : 0.0;
        LinvT[e] = (c < bs && r <= c) ? A[r][c + 1] : 0.0;    // LinvT[r][c] = Linv[c][r]
    }
}

// ---------------------------------------------------------------------------------------
// FP64 MFMA.  Every dense contraction here uses v_mfma_f64_4x4x4f64 (four independent
// 4x4x4 products per instruction): on gfx950 it sustains about twice the FP64 rate of the
// 16x16x4 form (measured 73 vs 36 TFLOP/s).  Operand layout (measured): lane l works on
// block (l/4)%4 with A[l%4][l/16], B[l/16][l%4] and D[l/16][l%4].  A wave that issues the
// instruction with left operand M[16a + l%16][k] and right operand N[4c + l%4][k] therefore
// accumulates (M N^T) over rows 16a + 4((l/4)%4) + l/16 and column 4c + l%4.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double mfma4(double a, double b, double c)
{
    return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ int mfma4_row(int lane) { return 4 * ((lane >> 2) & 3) + (lane >> 4); }

// ---------------------------------------------------------------------------------------
// Panel below the diagonal block: rows i in [k0+bs, n), columns [k0, k0+bs):
// A_ik <- A_ik L_kk^{-T}, a 64 x 128 by 128 x 128 product per workgroup.  Linv is staged in
// LDS; wave w holds its 16 rows of A as left operands in registers (all 32 k-steps) before
// it writes any of them back, so the update is in place.  Columns at or past bs read as zero
// (Linv is zero there).  Each finished entry L_ik is also stored at (k, i), in the upper
// triangle, which nothing else uses: the forward sweep then reads panel k as 128 contiguous
// rows instead of one 1 KiB segment from each of n - k0 rows 8 n bytes apart.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void lm_panel_kernel(double* __restrict__ K, int64_t n, int64_t k0, int bs,
                                                       const double* __restrict__ Linv)
{
    constexpr int LD = kPanel + 4;     // row pitch of the staged Linv
    __shared__ double Ls[kPanel * LD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < kPanel * kPanel; e += blockDim.x) Ls[(e / kPanel) * LD + e % kPanel] = Linv[e];
    const int64_t rbase = k0 + bs + (int64_t)blockIdx.x * 64 + wave * 16;
    const int64_t row = rbase + (lane & 15);
    const bool okr = row < n;
    double a[kPanel / 4];
#pragma unroll
    for (int s = 0; s < kPanel / 4; ++s) {
        const int m = 4 * s + (lane >> 4);
        a[s] = (okr && m < bs) ? K[row * n + k0 + m] : 0.0;
    }
    __syncthreads();
    double acc[kPanel / 4];
#pragma unroll
    for (int c = 0; c < kPanel / 4; ++c) acc[c] = 0.0;
    // right operand N[col][m] = Linv[col][m]
    const double* lrow = Ls + (lane & 3) * LD + (lane >> 4);
#pragma unroll
    for (int s = 0; s < kPanel / 4; ++s) {
#pragma unroll
        for (int c = 0; c < kPanel / 4; ++c) acc[c] = mfma4(a[s], lrow[4 * c * LD + 4 * s], acc[c]);
    }
    const int64_t gi = rbase + mfma4_row(lane);
#pragma unroll
    for (int c = 0; c < kPanel / 4; ++c) {
        const int col = 4 * c + (lane & 3);
        if (gi < n && col < bs) {
            K[gi * n + k0 + col] = acc[c];
            K[(k0 + col) * n + gi] = acc[c];   // transposed copy in the unused upper triangle
        }
    }
}

// ---------------------------------------------------------------------------------------
// Trailing update A_ij -= sum_m A[i][k0+m] A[j][k0+m], m < bs, over 64 x 64 lower tiles of the
// matrix from row/column t0 (t0 = k0 + bs for the trailing matrix).  With strip = 1 the grid
// covers only the two tile columns of the 128-wide column strip starting at t0 (the update
// of a panel by the earlier panels of its block).  Wave w computes the 32 x 32 quarter
// (w/2, w%2).  Operands are staged through LDS 32 columns at a time.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void lm_syrk_kernel(double* __restrict__ K, int64_t n, int64_t k0, int bs,
                                                      int64_t t0, int strip)
{
    constexpr int KC = 32;
    constexpr int LD = KC + 1;   // odd pitch: a left-operand read's 16 rows fall in distinct banks
    __shared__ double Ai[64 * LD];
    __shared__ double Aj[64 * LD];
    const int64_t id = blockIdx.x;
    int64_t ti, tj;
    if (strip) {
        // tiles (0,0), (1,0), (1,1), (2,0), (2,1), ...
        ti = (id + 1) / 2;
        tj = id == 0 ? 0 : (id + 1) % 2;
    } else {
        // linear tile id -> (ti, tj), tj <= ti
        ti = (int64_t)((__builtin_sqrt(8.0 * (double)id + 1.0) - 1.0) * 0.5);
        while ((ti + 1) * (ti + 2) / 2 <= id) ++ti;
        while (ti * (ti + 1) / 2 > id) --ti;
        tj = id - ti * (ti + 1) / 2;
    }
    const int64_t ri = t0 + ti * 64, rj = t0 + tj * 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;

    double acc[2][8];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[a][c] = 0.0;

    const double* ai = Ai + (wr * 32 + (lane & 15)) * LD + (lane >> 4);
    const double* aj = Aj + (wc * 32 + (lane & 3)) * LD + (lane >> 4);
    for (int kc = 0; kc < bs; kc += KC) {
        // thread t loads column t%32 of rows t/32 + 8u, so a wave's load instruction reads two
        // whole 256-byte row segments
        {
            const int c = tid & 31, r0 = tid >> 5;
            const bool okc = kc + c < bs;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int r = r0 + 8 * u;
                Ai[r * LD + c] = (okc && ri + r < n) ? K[(ri + r) * n + k0 + kc + c] : 0.0;
                Aj[r * LD + c] = (okc && rj + r < n) ? K[(rj + r) * n + k0 + kc + c] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < KC; k4 += 4) {
            double fa[2], fb[8];
#pragma unroll
            for (int a = 0; a < 2; ++a) fa[a] = ai[a * 16 * LD + k4];
#pragma unroll
            for (int c = 0; c < 8; ++c) fb[c] = aj[c * 4 * LD + k4];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 8; ++c) acc[a][c] = mfma4(fa[a], fb[c], acc[a][c]);
        }
        __syncthreads();
    }
    // every old value of the tile is read before the first store, so the loads overlap
    double old[2][8];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int64_t gi = ri + wr * 32 + a * 16 + mfma4_row(lane);
            const int64_t gj = rj + wc * 32 + c * 4 + (lane & 3);
            old[a][c] = (gi < n && gj <= gi) ? K[gi * n + gj] : 0.0;
        }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int64_t gi = ri + wr * 32 + a * 16 + mfma4_row(lane);
            const int64_t gj = rj + wc * 32 + c * 4 + (lane & 3);
            if (gi < n && gj <= gi) K[gi * n + gj] = old[a][c] - acc[a][c];
        }
}

// The same trailing update on 128 x 128 lower tiles, for large trailing matrices: each staged
// operand row then feeds twice the arithmetic.  Wave w computes the 64 x 64 quarter
// (w/2, w%2), 4 x 16 instructions per k-step of 4 with 64 accumulators per lane.  Operands go
// through LDS 32 columns at a time; the next chunk is fetched into registers while the
// current one is multiplied.  A wave stays within 256 registers (246: 128 accumulators, 64
// staged values, one k-step's operands) so that two workgroups share a CU and one multiplies
// while the other stages its next chunk: the fetches are buffer loads from the tile's first
// row with one 32-bit lane offset (rows past n fall outside the buffer's range and read as
// zero) instead of a live pointer per staged row, the k-steps are not unrolled, and the
// epilogue works on a quarter of the tile at a time.  With one workgroup per CU (384
// registers) the N = 65536 factorization took 2.66 s, with two 2.04 s (MI355X).
constexpr int kSyrkRsrcWord3 = 0x00020000;   // raw buffer, 32-bit elements (gfx9 encoding)

__device__ __forceinline__ double syrk_load(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
// A lane whose column lies past the block width loads from 2^31 bytes on, outside every
// operand buffer (at most 2^31 - 1 bytes), which reads as zero without a branch.
__device__ __forceinline__ unsigned syrk_col_off(unsigned off, bool in_block) { return in_block ? off : 0x80000000u; }

__global__ __launch_bounds__(256, 2) void lm_syrk128_kernel(double* __restrict__ K, int64_t n, int64_t k0, int bs,
                                                            int64_t t0)
{
    constexpr int KC = 32;
    // row pitch of the staged operands: with an odd pitch the 16 rows of a left-operand read
    // fall in distinct LDS banks (a pitch of 36 put rows 4 apart in the same bank: 2% slower)
    constexpr int LD = KC + 1;
    __shared__ double Ai[128 * LD];
    __shared__ double Aj[128 * LD];
    const int64_t id = blockIdx.x;
    int64_t ti = (int64_t)((__builtin_sqrt(8.0 * (double)id + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= id) ++ti;
    while (ti * (ti + 1) / 2 > id) --ti;
    const int64_t tj = id - ti * (ti + 1) / 2;
    const int64_t ri = t0 + ti * 128, rj = t0 + tj * 128;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const bool diag = (ti == tj);
    const bool active = !(diag && wc > wr);   // the quarter above a diagonal tile's diagonal is not needed

    // staging: thread t holds column t%KC of rows t/KC + RS u (u < NU) of each operand, so one
    // load instruction of a wave reads whole row segments of KC doubles.  Byte offsets from
    // (row ri or rj, column k0): row r, column c at 8 (r n + c); the buffer holds the tile's
    // rows below n.  128 n 8 bytes fit the 31-bit range for n below 2^21.
    constexpr int RS = 256 / KC, NU = 128 / RS;
    const int sc = tid % KC, sr = tid / KC;
    const int64_t rows_i = (n - ri) < 128 ? (n - ri) : 128;
    const int64_t rows_j = (n - rj) < 128 ? (n - rj) : 128;
    const __amdgpu_buffer_rsrc_t bi =
        __builtin_amdgcn_make_buffer_rsrc(K + ri * n + k0, (short)0, (int)(rows_i * n * 8), kSyrkRsrcWord3);
    const __amdgpu_buffer_rsrc_t bj =
        __builtin_amdgcn_make_buffer_rsrc(K + rj * n + k0, (short)0, (int)(rows_j * n * 8), kSyrkRsrcWord3);
    const unsigned rowstep = (unsigned)(RS * n * 8);   // RS rows, in bytes
    const unsigned lane_off = (unsigned)((sr * n + sc) * 8);
    double pa[NU], pb[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const unsigned off = syrk_col_off(lane_off, sc < bs);
        pa[u] = syrk_load(bi, off + u * rowstep);
        pb[u] = syrk_load(bj, off + u * rowstep);
    }

    double acc[4][16];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 16; ++c) acc[a][c] = 0.0;

    const double* ai = Ai + (wr * 64 + (lane & 15)) * LD + (lane >> 4);
    const double* aj = Aj + (wc * 64 + (lane & 3)) * LD + (lane >> 4);
    for (int kc = 0; kc < bs; kc += KC) {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            Ai[(sr + RS * u) * LD + sc] = pa[u];
            Aj[(sr + RS * u) * LD + sc] = pb[u];
        }
        __syncthreads();
        const int kn = kc + KC;
        if (kn < bs) {
            const unsigned off = syrk_col_off(lane_off + (unsigned)kn * 8, kn + sc < bs);
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                pa[u] = syrk_load(bi, off + u * rowstep);
                pb[u] = syrk_load(bj, off + u * rowstep);
            }
        }
        if (active) {
#pragma unroll 1
            for (int k4 = 0; k4 < KC; k4 += 4) {
                double fa[4], fb[16];
#pragma unroll
                for (int a = 0; a < 4; ++a) fa[a] = ai[a * 16 * LD + k4];
#pragma unroll
                for (int c = 0; c < 16; ++c) fb[c] = aj[c * 4 * LD + k4];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int c = 0; c < 16; ++c)
                        acc[a][c] = mfma4(fa[a], fb[c], acc[a][c]);
            }
        }
        __syncthreads();
    }
    if (!active) return;
    // read-modify-write in four groups of 16 values: each group's loads are all issued before
    // its first store (one load in flight at a time would serialise them), and a group's 32
    // registers fit beside the accumulators within the two-wave budget
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int64_t gi = ri + wr * 64 + a * 16 + mfma4_row(lane);
        double old[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const int64_t gj = rj + wc * 64 + c * 4 + (lane & 3);
            old[c] = (gi < n && gj <= gi) ? K[gi * n + gj] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const int64_t gj = rj + wc * 64 + c * 4 + (lane & 3);
            if (gi < n && gj <= gi) K[gi * n + gj] = old[c] - acc[a][c];
        }
    }
}


// The block's columns of the trailing rows rounded to float once, for the single-precision
// update below: P[(r - t0) w + c] = K[r][k0 + c], t0 <= r < n, c < w (one workgroup per row).
// Every tile pair then stages four bytes per operand instead of eight, from a compact copy.
__global__ __launch_bounds__(256) void lm_panel_f32_kernel(const double* __restrict__ K, int64_t n, int64_t k0, int w,
                                                           int64_t t0, float* __restrict__ P)
{
    const int64_t r = t0 + blockIdx.x;
    for (int c = threadIdx.x; c < w; c += blockDim.x) P[(r - t0) * w + c] = (float)K[r * n + k0 + c];
}

__device__ __forceinline__ float syrk_load_f32(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}

// The same 128 x 128 trailing update with the products in single precision, for factors whose
// solves only steer an iteration (matches with single-precision shoots): the staged operands
// are rounded to float, multiplied on v_mfma_f32_16x16x4f32 (twice the FP64 matrix rate) with
// float accumulation over the block's columns, and the result is subtracted from the FP64
// matrix.  PANEL: the operands come from the float copy lm_panel_f32_kernel made (P, pitch bs,
// row t0 first); else they are read from K as FP64 and rounded as they are staged (the same
// floats either way).  The factor is then accurate to about the single-precision rounding of each update
// (a solve to roughly cond(K) times 1e-6).  Operand layout (measured): lane l supplies A[l%16]
// [l/16] and B[l/16][l%16] and holds D[4 (l/16) + r][l%16], r < 4, of the 16 x 16 block.  Wave
// w computes the 64 x 64 quarter (w/2, w%2) as 4 x 4 blocks, 16 instructions per k-step of 4;
// the staged rows have a pitch of 34 floats, so that the 32 lanes of a half-wave read 16 rows
// at two columns from distinct banks.
typedef float v4f32 __attribute__((ext_vector_type(4)));

template <bool PANEL>
__global__ __launch_bounds__(256, 2) void lm_syrk128_f32_kernel(double* __restrict__ K, int64_t n, int64_t k0,
                                                                int bs, int64_t t0, const float* __restrict__ P)
{
    using S = typename std::conditional<PANEL, float, double>::type;   // a staged value
    constexpr unsigned ES = sizeof(S);
    constexpr int KC = 32;
    constexpr int LD = KC + 2;
    __shared__ float Ai[128 * LD];
    __shared__ float Aj[128 * LD];
    const int64_t id = blockIdx.x;
    int64_t ti = (int64_t)((__builtin_sqrt(8.0 * (double)id + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= id) ++ti;
    while (ti * (ti + 1) / 2 > id) --ti;
    const int64_t tj = id - ti * (ti + 1) / 2;
    const int64_t ri = t0 + ti * 128, rj = t0 + tj * 128;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const bool diag = (ti == tj);
    const bool active = !(diag && wc > wr);

    // staging as in lm_syrk128_kernel (buffer loads from the tile's first row), rounded to
    // float as it is stored unless it comes from the float copy
    constexpr int RS = 256 / KC, NU = 128 / RS;
    const int sc = tid % KC, sr = tid / KC;
    const int64_t rows_i = (n - ri) < 128 ? (n - ri) : 128;
    const int64_t rows_j = (n - rj) < 128 ? (n - rj) : 128;
    const int64_t pitch = PANEL ? bs : n;   // elements between rows of the operand buffer
    const void* base_i = PANEL ? (const void*)(P + (ri - t0) * bs) : (const void*)(K + ri * n + k0);
    const void* base_j = PANEL ? (const void*)(P + (rj - t0) * bs) : (const void*)(K + rj * n + k0);
    const __amdgpu_buffer_rsrc_t bi = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base_i), (short)0,
                                                                        (int)(rows_i * pitch * ES), kSyrkRsrcWord3);
    const __amdgpu_buffer_rsrc_t bj = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base_j), (short)0,
                                                                        (int)(rows_j * pitch * ES), kSyrkRsrcWord3);
    const unsigned rowstep = (unsigned)(RS * pitch * ES);
    const unsigned lane_off = (unsigned)((sr * pitch + sc) * ES);
    auto load = [&](__amdgpu_buffer_rsrc_t r, unsigned off) -> S {
        if constexpr (PANEL)
            return syrk_load_f32(r, off);
        else
            return syrk_load(r, off);
    };
    S pa[NU], pb[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const unsigned off = syrk_col_off(lane_off, sc < bs);
        pa[u] = load(bi, off + u * rowstep);
        pb[u] = load(bj, off + u * rowstep);
    }

    v4f32 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = v4f32{0.f, 0.f, 0.f, 0.f};

    // this lane's operand rows: row 16 a + l%16 of the wave's 64, column k4 + l/16
    const float* ai = Ai + (wr * 64 + (lane & 15)) * LD + (lane >> 4);
    const float* aj = Aj + (wc * 64 + (lane & 15)) * LD + (lane >> 4);
    for (int kc = 0; kc < bs; kc += KC) {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            Ai[(sr + RS * u) * LD + sc] = (float)pa[u];
            Aj[(sr + RS * u) * LD + sc] = (float)pb[u];
        }
        __syncthreads();
        const int kn = kc + KC;
        if (kn < bs) {
            const unsigned off = syrk_col_off(lane_off + (unsigned)kn * ES, kn + sc < bs);
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                pa[u] = load(bi, off + u * rowstep);
                pb[u] = load(bj, off + u * rowstep);
            }
        }
        if (active) {
#pragma unroll 2
            for (int k4 = 0; k4 < KC; k4 += 4) {
                float fa[4], fb[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) fa[a] = ai[a * 16 * LD + k4];
#pragma unroll
                for (int c = 0; c < 4; ++c) fb[c] = aj[c * 16 * LD + k4];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[a], fb[c], acc[a][c], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    if (!active) return;
    // read-modify-write by row block: all 16 loads of a block issued before its first store
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        double old[4][4];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = ri + wr * 64 + a * 16 + 4 * (lane >> 4) + r;
                const int64_t gj = rj + wc * 64 + c * 16 + (lane & 15);
                old[c][r] = (gi < n && gj <= gi) ? K[gi * n + gj] : 0.0;
            }
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = ri + wr * 64 + a * 16 + 4 * (lane >> 4) + r;
                const int64_t gj = rj + wc * 64 + c * 16 + (lane & 15);
                if (gi < n && gj <= gi) K[gi * n + gj] = old[c][r] - (double)acc[a][c][r];
            }
    }
}

// ---------------------------------------------------------------------------------------
// Triangular sweeps for `dim` right-hand sides (component-major vectors of length n).
// ---------------------------------------------------------------------------------------

// y_blk <- M y_blk for block blk, with M = Linv_blk (forward, TRANS = false) or Linv_blk^T
// (backward), by one workgroup of 256 threads.  (M y)_r = sum_m M^T[m][r] y_m reads rows of
// M^T, which is stored: LinvT for the forward sweep, Linv for the backward one.  Thread
// (h, r) sums m over half h for output r with 16 loads in flight (each wave load is one
// 512-byte row segment); the halves are added in order.  part: 3 * kPanel doubles of LDS.
template <bool TRANS, int DIM>
__device__ void finish_block(const double* __restrict__ Linv, int64_t n, int nb, int64_t blk,
                             double* __restrict__ y, int64_t ldy, double* sh, double* part)
{
    const int64_t b0 = blk * kPanel;
    const int bs = (int)((n - b0) < kPanel ? (n - b0) : kPanel);
    const double* Mt = Linv + ((TRANS ? 0 : (int64_t)nb) + blk) * kPanel * kPanel;
    for (int e = threadIdx.x; e < DIM * kPanel; e += blockDim.x) {
        const int c = e / kPanel, r = e % kPanel;
        sh[e] = r < bs ? y[c * ldy + b0 + r] : 0.0;
    }
    __syncthreads();
    const int r = threadIdx.x & (kPanel - 1), h = threadIdx.x >> 7;
    double acc[3] = {0.0, 0.0, 0.0};
    const double* col = Mt + (int64_t)(h * 64) * kPanel + r;
    for (int m0 = 0; m0 < 64; m0 += 16) {
        double lv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) lv[u] = col[(m0 + u) * kPanel];
#pragma unroll
        for (int c = 0; c < DIM; ++c)
#pragma unroll
            for (int u = 0; u < 16; ++u) acc[c] = __builtin_fma(lv[u], sh[c * kPanel + h * 64 + m0 + u], acc[c]);
    }
    if (h == 1)
        for (int c = 0; c < DIM; ++c) part[c * kPanel + r] = acc[c];
    __syncthreads();
    if (h == 0 && r < bs)
        for (int c = 0; c < DIM; ++c) y[c * ldy + b0 + r] = acc[c] + part[c * kPanel + r];
}

// Launch k of the forward sweep (k = -1: only finish block 0): y_r -= sum_m L[r][k0 + m]
// y_k[m] for every row r past block k, reading panel k from its transposed copy, row k0 + m
// of the upper triangle (LT[m][r] = L[r][k0 + m], contiguous in r).  A workgroup takes 64
// consecutive rows r, one per lane; wave w sums m over [32 w, 32 w + 32) (each wave load is
// one 512-byte segment of a row of LT) and the four wave sums are added in wave order.
// Workgroup 0 owns block k+1 (its two 64-row halves, then the block's finish with the
// stored inverse); workgroups >= 1 take the rows of blocks k+2 .. nb-1, 64 at a time.
template <int DIM>
__global__ __launch_bounds__(256) void lm_trsv_fwd_kernel(const double* __restrict__ L, const double* __restrict__ Linv,
                                                          int64_t n, int nb, int64_t k, double* __restrict__ y,
                                                          int64_t ldy)
{
    __shared__ double sh[3 * kPanel];
    __shared__ double yk[3 * kPanel];
    __shared__ double red[4][3][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (k >= 0) {
        const int64_t k0 = k * kPanel;
        for (int e = threadIdx.x; e < DIM * kPanel; e += blockDim.x) {
            const int c = e / kPanel, m = e % kPanel;
            yk[e] = (k0 + m < n) ? y[c * ldy + k0 + m] : 0.0;
        }
        __syncthreads();
        int64_t rbeg, rend, rstep;
        if (blockIdx.x == 0) {
            rbeg = (k + 1) * kPanel;
            rend = (k + 2) * kPanel < n ? (k + 2) * kPanel : n;
            rstep = 64;
        } else {
            rbeg = (k + 2) * kPanel + (int64_t)(blockIdx.x - 1) * 64;
            rend = n;
            rstep = (int64_t)(gridDim.x - 1) * 64;
        }
        const int m0 = wave * 32;
        for (int64_t rb = rbeg; rb < rend; rb += rstep) {
            const int64_t r = rb + lane;
            const bool ok = r < rend;
            const double* lt = L + (k0 + m0) * n + (ok ? r : rb);
            double lv[32];
#pragma unroll
            for (int u = 0; u < 32; ++u) lv[u] = lt[(int64_t)u * n];
            double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < DIM; ++c)
#pragma unroll
                for (int u = 0; u < 32; ++u) s[c] = __builtin_fma(lv[u], yk[c * kPanel + m0 + u], s[c]);
#pragma unroll
            for (int c = 0; c < DIM; ++c) red[wave][c][lane] = s[c];
            __syncthreads();
            if (wave == 0 && ok)
                for (int c = 0; c < DIM; ++c)
                    y[c * ldy + r] -= ((red[0][c][lane] + red[1][c][lane]) + red[2][c][lane]) + red[3][c][lane];
            __syncthreads();
        }
    }
    if (blockIdx.x == 0 && k + 1 < nb) {
        __threadfence_block();
        __syncthreads();
        finish_block<false, DIM>(Linv, n, nb, k + 1, y, ldy, sh, yk);
    }
}

// Launch k of the backward sweep (k = nb: only finish block nb-1).  Workgroup 0 owns block
// k-1: it subtracts L[block k, block k-1]^T x_k (thread (h, r): column r over row half h,
// the halves added in order) and finishes x_{k-1}; workgroups >= 1 handle the columns of
// blocks 0 .. k-2, one column per thread.
template <int DIM>
__global__ __launch_bounds__(256) void lm_trsv_bwd_kernel(const double* __restrict__ L, const double* __restrict__ Linv,
                                                          int64_t n, int nb, int64_t k, double* __restrict__ y,
                                                          int64_t ldy)
{
    __shared__ double sh[3 * kPanel];
    __shared__ double xk[3 * kPanel];
    if (k < nb) {
        const int64_t k0 = k * kPanel;
        const int bs = (int)((n - k0) < kPanel ? (n - k0) : kPanel);
        for (int e = threadIdx.x; e < DIM * kPanel; e += blockDim.x) {
            const int c = e / kPanel, m = e % kPanel;
            xk[e] = m < bs ? y[c * ldy + k0 + m] : 0.0;
        }
        __syncthreads();
        if (blockIdx.x == 0) {
            const int r = threadIdx.x & (kPanel - 1), h = threadIdx.x >> 7;
            const int64_t col = (k - 1) * kPanel + r;
            const double* lc = L + (k0 + h * 64) * n + col;
            double s[3] = {0.0, 0.0, 0.0};
            for (int m0 = 0; m0 < 64; m0 += 16) {
                double lv[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int m = h * 64 + m0 + u;
                    lv[u] = m < bs ? lc[(int64_t)(m0 + u) * n] : 0.0;
                }
                for (int c = 0; c < DIM; ++c)
#pragma unroll
                    for (int u = 0; u < 16; ++u) s[c] = __builtin_fma(lv[u], xk[c * kPanel + h * 64 + m0 + u], s[c]);
            }
            if (h == 1)
                for (int c = 0; c < DIM; ++c) sh[c * kPanel + r] = s[c];
            __syncthreads();
            if (h == 0)
                for (int c = 0; c < DIM; ++c) y[c * ldy + col] -= s[c] + sh[c * kPanel + r];
        } else {
            const int64_t cend = (k - 1) * kPanel;
            const int64_t cstep = (int64_t)(gridDim.x - 1) * blockDim.x;
            for (int64_t col = (int64_t)(blockIdx.x - 1) * blockDim.x + threadIdx.x; col < cend; col += cstep) {
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
                for (int c = 0; c < DIM; ++c) y[c * ldy + col] -= s[c];
            }
        }
    }
    if (blockIdx.x == 0 && k - 1 >= 0) {
        __threadfence_block();
        __syncthreads();
        finish_block<true, DIM>(Linv, n, nb, k - 1, y, ldy, sh, xk);
    }
}

// ---------------------------------------------------------------------------------------
// Batched solves: y_b <- (L_b L_b^T)^{-1} y_b for every flagged problem b of a batch, one
// workgroup per problem, the problem's vector held in LDS (at most kBatchSolveMax points).
// Forward, per 128-row block k: s = y_k - L[k, <k] y_<k (rows spread over the waves, lanes
// striding the columns, four rows at a time), then y_k = Linv_k s.  Backward, per block from
// the last: t = y_k - L[>k, k]^T x_>k (each wave takes every fourth row below the block, lanes
// the block's columns; the wave partials are added in wave order), then x_k = Linv_k^T t.
// Both block finishes read rows (of LinvT, of Linv) with two threads per output.  One
// workgroup sweeps a problem's whole factor, so the loops keep 16 loads in flight per wave
// (with one to four, the 4065-point problem's sweeps took 11.1 ms, latency-bound).
// L_b: row-major n_b x n_b lower triangle at L + loff[b]; Linv_b at Linv + ioff[b] (the
// transposes after the problem's panels of inverses, as launch_dense_factor stores them); y: the
// batch's (dim, ntot) array, problem b in columns offs[b] .. offs[b+1]-1.
// ---------------------------------------------------------------------------------------
constexpr int kBatchSolveMax = 4096;

// v[k0 + r] <- (M t)_r for r < bs, M^T stored at Mt (128 x 128 rows): thread (h, r) sums its
// half of the rows of Mt, the halves added in order (part: scratch, one panel per component).
// t must be zero past bs.
template <int DIM>
__device__ __forceinline__ void batch_finish(const double* __restrict__ Mt, int bs, int k0,
                                             const double (*t)[kPanel], double (*part)[kPanel],
                                             double (*v)[kBatchSolveMax])
{
    const int tid = threadIdx.x, r = tid & (kPanel - 1), h = tid >> 7;
    double acc[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) acc[c] = 0.0;
    const double* col = Mt + (int64_t)(h * 64) * kPanel + r;
    for (int m0 = 0; m0 < 64; m0 += 16) {
        double lv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) lv[u] = col[(m0 + u) * kPanel];
#pragma unroll
        for (int c = 0; c < DIM; ++c)
#pragma unroll
            for (int u = 0; u < 16; ++u) acc[c] = __builtin_fma(lv[u], t[c][h * 64 + m0 + u], acc[c]);
    }
    if (h == 1)
#pragma unroll
        for (int c = 0; c < DIM; ++c) part[c][r] = acc[c];
    __syncthreads();
    if (h == 0 && r < bs)
#pragma unroll
        for (int c = 0; c < DIM; ++c) v[c][k0 + r] = acc[c] + part[c][r];
    __syncthreads();
}

template <int DIM>
__global__ __launch_bounds__(256) void lm_batch_solve_kernel(const double* __restrict__ L,
                                                             const int64_t* __restrict__ loff,
                                                             const double* __restrict__ Linv,
                                                             const int64_t* __restrict__ ioff,
                                                             const int64_t* __restrict__ offs, int64_t ntot,
                                                             double* __restrict__ y, const int* __restrict__ flag)
{
    __shared__ double v[DIM][kBatchSolveMax];
    __shared__ double tmp[4][DIM][kPanel];
    const int b = blockIdx.x;
    if (!flag[b]) return;
    const int64_t off = offs[b];
    const int n = (int)(offs[b + 1] - off);
    const double* Lb = L + loff[b];
    const double* Ib = Linv + ioff[b];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int c = 0; c < DIM; ++c)
        for (int i = tid; i < n; i += blockDim.x) v[c][i] = y[c * ntot + off + i];
    __syncthreads();
    const int nb = (n + kPanel - 1) / kPanel;

    // forward sweep
    for (int k = 0; k < nb; ++k) {
        const int k0 = k * kPanel, bs = (n - k0) < kPanel ? (n - k0) : kPanel;
        for (int r0 = wave * 4; r0 < bs; r0 += 16) {
            double acc[4][DIM];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int c = 0; c < DIM; ++c) acc[u][c] = 0.0;
            // four 64-column chunks per iteration (16 loads in flight), then single chunks;
            // every row's terms are added in increasing j either way
            int j = lane;
            for (; j + 192 < k0; j += 256) {
                double l[4][4];
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        l[q][u] = (r0 + u < bs) ? Lb[(int64_t)(k0 + r0 + u) * n + j + 64 * q] : 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int c = 0; c < DIM; ++c) {
                        const double yj = v[c][j + 64 * q];
#pragma unroll
                        for (int u = 0; u < 4; ++u) acc[u][c] = __builtin_fma(l[q][u], yj, acc[u][c]);
                    }
            }
            for (; j < k0; j += 64) {
                double l[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) l[u] = (r0 + u < bs) ? Lb[(int64_t)(k0 + r0 + u) * n + j] : 0.0;
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    const double yj = v[c][j];
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc[u][c] = __builtin_fma(l[u], yj, acc[u][c]);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    double a = acc[u][c];
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
                    if (lane == 0 && r0 + u < bs) tmp[0][c][r0 + u] = v[c][k0 + r0 + u] - a;
                }
        }
        // zero the staged vector past a ragged last block (the finish multiplies every entry)
        for (int e = bs + tid; e < kPanel; e += blockDim.x)
            for (int c = 0; c < DIM; ++c) tmp[0][c][e] = 0.0;
        __syncthreads();
        // y_k = Linv_k t: rows of the stored transpose LinvT
        batch_finish<DIM>(Ib + ((int64_t)nb + k) * kPanel * kPanel, bs, k0, tmp[0], tmp[1], v);
    }

    // backward sweep
    for (int k = nb - 1; k >= 0; --k) {
        const int k0 = k * kPanel, bs = (n - k0) < kPanel ? (n - k0) : kPanel;
        double acc[2][DIM];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int c = 0; c < DIM; ++c) acc[h][c] = 0.0;
        const bool ok0 = lane < bs, ok1 = 64 + lane < bs;
        // eight of the wave's rows per iteration (16 loads in flight), then single rows; the
        // terms are added in increasing j either way
        int j = k0 + bs + wave;
        for (; j + 28 < n; j += 32) {
            double l0[8], l1[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double* lr = Lb + (int64_t)(j + 4 * q) * n + k0;
                l0[q] = ok0 ? lr[lane] : 0.0;
                l1[q] = ok1 ? lr[64 + lane] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 8; ++q)
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    const double xj = v[c][j + 4 * q];
                    acc[0][c] = __builtin_fma(l0[q], xj, acc[0][c]);
                    acc[1][c] = __builtin_fma(l1[q], xj, acc[1][c]);
                }
        }
        for (; j < n; j += 4) {
            const double* lr = Lb + (int64_t)j * n + k0;
            const double l0 = ok0 ? lr[lane] : 0.0;
            const double l1 = ok1 ? lr[64 + lane] : 0.0;
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const double xj = v[c][j];
                acc[0][c] = __builtin_fma(l0, xj, acc[0][c]);
                acc[1][c] = __builtin_fma(l1, xj, acc[1][c]);
            }
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            tmp[wave][c][lane] = acc[0][c];
            tmp[wave][c][64 + lane] = acc[1][c];
        }
        __syncthreads();
        if (tid < kPanel) {
            for (int c = 0; c < DIM; ++c) {
                const double sum = tmp[0][c][tid] + tmp[1][c][tid] + tmp[2][c][tid] + tmp[3][c][tid];
                tmp[0][c][tid] = (tid < bs) ? v[c][k0 + tid] - sum : 0.0;
            }
        }
        __syncthreads();
        // x_k = Linv_k^T t: rows of Linv
        batch_finish<DIM>(Ib + (int64_t)k * kPanel * kPanel, bs, k0, tmp[0], tmp[1], v);
    }
    for (int c = 0; c < DIM; ++c)
        for (int i = tid; i < n; i += blockDim.x) y[c * ntot + off + i] = v[c][i];
}

int batch_solve_max() { return kBatchSolveMax; }

hipError_t launch_batch_dense_solve(const double* L, const int64_t* loff, const double* Linv, const int64_t* ioff,
                                    const int64_t* offs, int nprob, int dim, int64_t ntot, double* y, const int* flag,
                                    hipStream_t st)
{
    if (dim == 2)
        hipLaunchKernelGGL(lm_batch_solve_kernel<2>, dim3(nprob), dim3(256), 0, st, L, loff, Linv, ioff, offs, ntot, y,
                           flag);
    else
        hipLaunchKernelGGL(lm_batch_solve_kernel<3>, dim3(nprob), dim3(256), 0, st, L, loff, Linv, ioff, offs, ntot, y,
                           flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Batched wide sweeps: the per-block sweeps above for many problems at once, so that a large
// problem of a batch is streamed by many workgroups rather than by the one workgroup of
// lm_batch_solve_kernel (whose loads in flight bound one problem's sweep at about 31 GB/s).
// Launch k of the forward sweep serves every listed problem with more than k + 1 blocks:
// item (b, 0) owns block k+1 (its rows take panel k, then the block's finish with the stored
// inverse), item (b, 1, r) takes the 64 rows r .. r+63 (in blocks k+2 ..) and panel k.
// Launch k of the backward sweep: item (b, 0) subtracts block row k from block k-1 and
// finishes it, item (b, 1, c) takes the 256 columns c .. c+255 (in blocks 0 .. k-2) and block
// row k.  Items of a problem whose flag is 0 do nothing.  A persistent grid walks the
// launch's list, owners first.
// ---------------------------------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(256) void lm_batch_trsv_fwd_kernel(const double* __restrict__ L,
                                                                const int64_t* __restrict__ loff,
                                                                const double* __restrict__ Linv,
                                                                const int64_t* __restrict__ ioff,
                                                                const int64_t* __restrict__ offs, int64_t ntot,
                                                                double* __restrict__ y, const int* __restrict__ flag,
                                                                const int4* __restrict__ items, int nitems, int64_t k)
{
    __shared__ double sh[3 * kPanel];
    __shared__ double yk[3 * kPanel];
    __shared__ double red[4][3][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int4 w = items[it];
        if (!flag[w.x]) continue;
        const int64_t off = offs[w.x], n = offs[w.x + 1] - off;
        const int nb = (int)((n + kPanel - 1) / kPanel);
        const double* Lb = L + loff[w.x];
        double* yb = y + off;
        __syncthreads();   // the previous item is done with yk and sh
        if (k >= 0) {
            const int64_t k0 = k * kPanel;
            for (int e = threadIdx.x; e < DIM * kPanel; e += blockDim.x) {
                const int c = e / kPanel, m = e % kPanel;
                yk[e] = (k0 + m < n) ? yb[c * ntot + k0 + m] : 0.0;
            }
            __syncthreads();
            int64_t rbeg, rend;
            if (w.y == 0) {
                rbeg = (k + 1) * kPanel;
                rend = (k + 2) * kPanel < n ? (k + 2) * kPanel : n;
            } else {
                rbeg = w.z;
                rend = w.z + 64 < n ? w.z + 64 : n;
            }
            const int m0 = wave * 32;
            for (int64_t rb = rbeg; rb < rend; rb += 64) {
                const int64_t r = rb + lane;
                const bool ok = r < rend;
                const double* lt = Lb + (k0 + m0) * n + (ok ? r : rb);
                double lv[32];
#pragma unroll
                for (int u = 0; u < 32; ++u) lv[u] = (k0 + m0 + u < n) ? lt[(int64_t)u * n] : 0.0;
                double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int c = 0; c < DIM; ++c)
#pragma unroll
                    for (int u = 0; u < 32; ++u) s[c] = __builtin_fma(lv[u], yk[c * kPanel + m0 + u], s[c]);
#pragma unroll
                for (int c = 0; c < DIM; ++c) red[wave][c][lane] = s[c];
                __syncthreads();
                if (wave == 0 && ok)
                    for (int c = 0; c < DIM; ++c)
                        yb[c * ntot + r] -= ((red[0][c][lane] + red[1][c][lane]) + red[2][c][lane]) + red[3][c][lane];
                __syncthreads();
            }
        }
        if (w.y == 0) {
            __threadfence_block();
            __syncthreads();
            finish_block<false, DIM>(Linv + ioff[w.x], n, nb, k + 1, yb, ntot, sh, yk);
        }
    }
}

template <int DIM>
__global__ __launch_bounds__(256) void lm_batch_trsv_bwd_kernel(const double* __restrict__ L,
                                                                const int64_t* __restrict__ loff,
                                                                const double* __restrict__ Linv,
                                                                const int64_t* __restrict__ ioff,
                                                                const int64_t* __restrict__ offs, int64_t ntot,
                                                                double* __restrict__ y, const int* __restrict__ flag,
                                                                const int4* __restrict__ items, int nitems, int64_t k)
{
    __shared__ double sh[3 * kPanel];
    __shared__ double xk[3 * kPanel];
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int4 w = items[it];
        if (!flag[w.x]) continue;
        const int64_t off = offs[w.x], n = offs[w.x + 1] - off;
        const int nb = (int)((n + kPanel - 1) / kPanel);
        const double* Lb = L + loff[w.x];
        double* yb = y + off;
        __syncthreads();   // the previous item is done with xk and sh
        if (k < nb) {
            const int64_t k0 = k * kPanel;
            const int bs = (int)((n - k0) < kPanel ? (n - k0) : kPanel);
            for (int e = threadIdx.x; e < DIM * kPanel; e += blockDim.x) {
                const int c = e / kPanel, m = e % kPanel;
                xk[e] = m < bs ? yb[c * ntot + k0 + m] : 0.0;
            }
            __syncthreads();
            if (w.y == 0) {
                const int r = threadIdx.x & (kPanel - 1), h = threadIdx.x >> 7;
                const int64_t col = (k - 1) * kPanel + r;
                const double* lc = Lb + (k0 + h * 64) * n + col;
                double s[3] = {0.0, 0.0, 0.0};
                for (int m0 = 0; m0 < 64; m0 += 16) {
                    double lv[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        const int m = h * 64 + m0 + u;
                        lv[u] = m < bs ? lc[(int64_t)(m0 + u) * n] : 0.0;
                    }
                    for (int c = 0; c < DIM; ++c)
#pragma unroll
                        for (int u = 0; u < 16; ++u)
                            s[c] = __builtin_fma(lv[u], xk[c * kPanel + h * 64 + m0 + u], s[c]);
                }
                if (h == 1)
                    for (int c = 0; c < DIM; ++c) sh[c * kPanel + r] = s[c];
                __syncthreads();
                if (h == 0)
                    for (int c = 0; c < DIM; ++c) yb[c * ntot + col] -= s[c] + sh[c * kPanel + r];
            } else {
                const int64_t cend = (k - 1) * kPanel;
                const int64_t col = w.z + threadIdx.x;
                if (col < cend) {
                    double s[3] = {0.0, 0.0, 0.0};
                    const double* lc = Lb + k0 * n + col;
                    for (int m0 = 0; m0 < kPanel; m0 += 16) {
                        double lv[16];
#pragma unroll
                        for (int u = 0; u < 16; ++u) lv[u] = (m0 + u < bs) ? lc[(int64_t)(m0 + u) * n] : 0.0;
                        for (int c = 0; c < DIM; ++c)
#pragma unroll
                            for (int u = 0; u < 16; ++u) s[c] = __builtin_fma(lv[u], xk[c * kPanel + m0 + u], s[c]);
                    }
                    for (int c = 0; c < DIM; ++c) yb[c * ntot + col] -= s[c];
                }
            }
        }
        if (w.y == 0) {
            __threadfence_block();
            __syncthreads();
            finish_block<true, DIM>(Linv + ioff[w.x], n, nb, k - 1, yb, ntot, sh, xk);
        }
    }
}

void batch_wide_plan(const int64_t* offs, const std::vector<int>& probs, BatchWidePlan* pl)
{
    pl->items.clear();
    int maxnb = 0;
    for (int b : probs) maxnb = std::max(maxnb, dense_panels(offs[b + 1] - offs[b]));
    pl->maxnb = maxnb;
    pl->fwd.assign((size_t)maxnb + 1, 0);
    pl->bwd.assign((size_t)maxnb + 1, 0);
    // forward launch k = -1 .. maxnb - 2 (list k + 1)
    for (int k = -1; k <= maxnb - 2; ++k) {
        pl->fwd[k + 1] = (int)pl->items.size();
        for (int b : probs)
            if (k + 1 < dense_panels(offs[b + 1] - offs[b])) pl->items.push_back(make_int4(b, 0, 0, 0));
        if (k >= 0)
            for (int b : probs) {
                const int64_t n = offs[b + 1] - offs[b];
                for (int64_t r = (int64_t)(k + 2) * kPanel; r < n; r += 64) pl->items.push_back(make_int4(b, 1, (int)r, 0));
            }
    }
    pl->fwd[maxnb] = (int)pl->items.size();
    // backward launch k = maxnb .. 1 (list maxnb - k)
    for (int k = maxnb; k >= 1; --k) {
        pl->bwd[maxnb - k] = (int)pl->items.size();
        for (int b : probs)
            if (k <= dense_panels(offs[b + 1] - offs[b])) pl->items.push_back(make_int4(b, 0, 0, 0));
        for (int b : probs) {
            const int nbb = dense_panels(offs[b + 1] - offs[b]);
            if (k >= nbb) continue;
            for (int64_t c = 0; c < (int64_t)(k - 1) * kPanel; c += 256) pl->items.push_back(make_int4(b, 1, (int)c, 0));
        }
    }
    pl->bwd[maxnb] = (int)pl->items.size();
}

hipError_t launch_batch_wide_solve(const double* L, const int64_t* loff, const double* Linv, const int64_t* ioff,
                                   const int64_t* offs, int dim, int64_t ntot, double* y, const int* flag,
                                   const int4* items, const BatchWidePlan& pl, hipStream_t st)
{
    auto grid = [](int cnt) { return dim3((unsigned)(cnt < 2048 ? cnt : 2048)); };
    for (int k = -1; k <= pl.maxnb - 2; ++k) {
        const int a = pl.fwd[k + 1], cnt = pl.fwd[k + 2] - a;
        if (cnt <= 0) continue;
        if (dim == 2)
            hipLaunchKernelGGL(lm_batch_trsv_fwd_kernel<2>, grid(cnt), dim3(256), 0, st, L, loff, Linv, ioff, offs, ntot,
                               y, flag, items + a, cnt, (int64_t)k);
        else
            hipLaunchKernelGGL(lm_batch_trsv_fwd_kernel<3>, grid(cnt), dim3(256), 0, st, L, loff, Linv, ioff, offs, ntot,
                               y, flag, items + a, cnt, (int64_t)k);
    }
    for (int k = pl.maxnb; k >= 1; --k) {
        const int a = pl.bwd[pl.maxnb - k], cnt = pl.bwd[pl.maxnb - k + 1] - a;
        if (cnt <= 0) continue;
        if (dim == 2)
            hipLaunchKernelGGL(lm_batch_trsv_bwd_kernel<2>, grid(cnt), dim3(256), 0, st, L, loff, Linv, ioff, offs, ntot,
                               y, flag, items + a, cnt, (int64_t)k);
        else
            hipLaunchKernelGGL(lm_batch_trsv_bwd_kernel<3>, grid(cnt), dim3(256), 0, st, L, loff, Linv, ioff, offs, ntot,
                               y, flag, items + a, cnt, (int64_t)k);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Superblock sweeps.  The per-block sweeps above take one launch per 128-row block, and
// each launch ends with one workgroup finishing the next block: at N = 65536 that is 1024
// dependent launches per solve.  Here kSuper consecutive blocks form a superblock s whose
// diagonal part L_ss is inverted once, after the factor: W_s = L_ss^{-1} is block lower
// triangular with W_ii = Linv_i and, for i > m,
//   W_im = -Linv_i sum_{j=m}^{i-1} L_ij W_jm
// (from L_ss W_s = I).  A forward sweep is then, per superblock, three launches:
//   prod: every block product W_im t_m (m <= i) by its own workgroup into a partial buffer;
//   sum:  x_i = sum_m of those partials in increasing m (one workgroup per block) into z;
//   rows: every row past the superblock subtracts L[r, s] x_s, the panel of kSuper * 128
//         columns read from its transposed copy in the upper triangle (contiguous rows).
// The backward sweep mirrors it with W_s^T (blocks (W_mi)^T, m >= i), reading L's rows
// below the diagonal.  The forward sweep writes its result into the scratch z and uses y
// as the accumulator; the backward sweep uses z as the accumulator and writes x into y.
// W_im and W_im^T are stored for every superblock (the products read rows: W^T rows for
// W t, W rows for W^T t), 2 * kSuper(kSuper-1)/2 blocks of 128 x 128 per superblock.
// ---------------------------------------------------------------------------------------
constexpr int kSuper = 8;
constexpr int kSuperPairs = kSuper * (kSuper - 1) / 2;   // off-diagonal blocks of W_s
constexpr int kSuperProds = kSuper * (kSuper + 1) / 2;   // block products of one sweep step

int super_count(int64_t n) { return (dense_panels(n) + kSuper - 1) / kSuper; }
int64_t dense_super_elems(int64_t n) { return 2 * (int64_t)super_count(n) * kSuperPairs * kPanel * kPanel; }
int64_t dense_solve_scratch_elems(int64_t n) { return 3 * n + (int64_t)kSuperProds * 3 * kPanel; }

// Block (i, m), m < i, of W_s, and its transpose.
__host__ __device__ __forceinline__ int64_t super_blk(int64_t s, int i, int m)
{
    return (s * kSuperPairs + i * (i - 1) / 2 + m) * kPanel * kPanel;
}
__host__ __device__ __forceinline__ int64_t super_blk_t(int ns, int64_t s, int i, int m)
{
    return ((int64_t)ns * kSuperPairs) * kPanel * kPanel + super_blk(s, i, m);
}
__device__ __forceinline__ int block_rows(int64_t n, int64_t blk)
{
    const int64_t r = n - blk * kPanel;
    return r < kPanel ? (int)r : kPanel;
}

// acc[u][v] += sum_k A[tr + 16u][k] B[k][tc + 16v] over the 128 x 128 x 128 product of the
// row-major blocks A (leading dimension lda; entries with row >= arows or k >= kdim read as
// zero) and B (ldb; k >= kdim or column >= bcols read as zero), thread (tr, tc) = (tid / 16,
// tid % 16).  k runs in chunks of 16 staged in LDS (A transposed), each added in increasing k.
__device__ void gemm128_acc(const double* __restrict__ A, int64_t lda, int arows, int kdim,
                            const double* __restrict__ B, int64_t ldb, int bcols, double (&acc)[8][8],
                            double (*As)[kPanel + 1], double (*Bs)[kPanel + 1])
{
    const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
    for (int k0 = 0; k0 < kPanel; k0 += 16) {
        double av[8], bv[8];
        {
            const int r = tid >> 1, kk = (tid & 1) * 8;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                av[u] = (r < arows && k0 + kk + u < kdim) ? A[(int64_t)r * lda + k0 + kk + u] : 0.0;
            const int kb = tid >> 4, c = (tid & 15) * 8;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                bv[u] = (k0 + kb < kdim && c + u < bcols) ? B[(int64_t)(k0 + kb) * ldb + c + u] : 0.0;
        }
        __syncthreads();   // the previous chunk's reads are done
        {
            const int r = tid >> 1, kk = (tid & 1) * 8;
#pragma unroll
            for (int u = 0; u < 8; ++u) As[kk + u][r] = av[u];
            const int kb = tid >> 4, c = (tid & 15) * 8;
#pragma unroll
            for (int u = 0; u < 8; ++u) Bs[kb][c + u] = bv[u];
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < 16; ++k) {
            double a[8], b[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                a[u] = As[k][tr + 16 * u];
                b[u] = Bs[k][tc + 16 * u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int v = 0; v < 8; ++v) acc[u][v] = __builtin_fma(a[u], b[v], acc[u][v]);
        }
    }
    __syncthreads();
}

// Step d of building the W_s (all superblocks, blocks i = m + d): S = sum_{j=m}^{i-1} L_ij W_jm
// (W_mm = Linv_m), stored in the slot of W_im^T for the next kernel.
__global__ __launch_bounds__(256) void lm_super_s_kernel(const double* __restrict__ L, const double* __restrict__ Linv,
                                                         double* __restrict__ W, int64_t n, int nb, int ns, int d)
{
    __shared__ double As[16][kPanel + 1];
    __shared__ double Bs[16][kPanel + 1];
    const int64_t s = blockIdx.x / (kSuper - d);
    const int m = (int)(blockIdx.x % (kSuper - d)), i = m + d;
    const int64_t b0 = s * kSuper;
    if (b0 + i >= nb) return;
    const int bi = block_rows(n, b0 + i), bm = block_rows(n, b0 + m);
    double acc[8][8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int v = 0; v < 8; ++v) acc[u][v] = 0.0;
    for (int j = m; j < i; ++j) {
        const double* Aij = L + ((b0 + i) * kPanel) * n + (b0 + j) * kPanel;
        const double* Bjm = (j == m) ? Linv + (b0 + m) * kPanel * kPanel : W + super_blk(s, j, m);
        gemm128_acc(Aij, n, bi, block_rows(n, b0 + j), Bjm, kPanel, bm, acc, As, Bs);
    }
    double* S = W + super_blk_t(ns, s, i, m);
    const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int v = 0; v < 8; ++v) S[(tr + 16 * u) * kPanel + tc + 16 * v] = acc[u][v];
}

// Step d, second half: W_im = -Linv_i S (S read from the W_im^T slot), stored with its
// transpose.  Every read of S is done (gemm128_acc ends with a barrier) before the slot is
// overwritten.
__global__ __launch_bounds__(256) void lm_super_w_kernel(const double* __restrict__ Linv, double* __restrict__ W,
                                                         int64_t n, int nb, int ns, int d)
{
    __shared__ double As[16][kPanel + 1];
    __shared__ double Bs[16][kPanel + 1];
    const int64_t s = blockIdx.x / (kSuper - d);
    const int m = (int)(blockIdx.x % (kSuper - d)), i = m + d;
    const int64_t b0 = s * kSuper;
    if (b0 + i >= nb) return;
    const int bi = block_rows(n, b0 + i), bm = block_rows(n, b0 + m);
    double acc[8][8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int v = 0; v < 8; ++v) acc[u][v] = 0.0;
    double* Wt = W + super_blk_t(ns, s, i, m);
    gemm128_acc(Linv + (b0 + i) * kPanel * kPanel, kPanel, bi, bi, Wt, kPanel, bm, acc, As, Bs);
    double* Wim = W + super_blk(s, i, m);
    const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int r = tr + 16 * u, c = tc + 16 * v;
            Wim[r * kPanel + c] = -acc[u][v];
            Wt[c * kPanel + r] = -acc[u][v];
        }
}

// One superblock step's block products: workgroup p takes pair (a, b), a >= b, with
// p = a(a+1)/2 + b.  Forward: (i, m) = (a, b), out = W_im t_m, reading rows of W_im^T (LinvT
// for i = m).  Backward: (i, m) = (b, a), out = W_mi^T t_m, reading rows of W_mi (Linv for
// i = m).  t_m: block b0 + m of t (zero past n); out: DIM x kPanel doubles at part + p.
// Thread (h, r) sums its half of the rows for output r, 16 loads in flight; halves added in
// order.
template <int DIM, bool BWD>
__global__ __launch_bounds__(256) void lm_super_prod_kernel(const double* __restrict__ Linv, const double* __restrict__ W,
                                                            int64_t n, int nb, int ns, int64_t s,
                                                            const double* __restrict__ t, int64_t ldt,
                                                            double* __restrict__ part)
{
    __shared__ double tv[DIM][kPanel];
    __shared__ double half[DIM][kPanel];
    const int p = blockIdx.x;
    int a = 0;
    while ((a + 1) * (a + 2) / 2 <= p) ++a;
    const int b = p - a * (a + 1) / 2;
    const int i = BWD ? b : a, m = BWD ? a : b;
    const int64_t b0 = s * kSuper;
    const double* Mrows;
    if (i == m)
        Mrows = Linv + ((BWD ? 0 : (int64_t)nb) + b0 + i) * kPanel * kPanel;
    else
        Mrows = BWD ? W + super_blk(s, m, i) : W + super_blk_t(ns, s, i, m);
    const int64_t t0 = (b0 + m) * kPanel;
    const int bm = block_rows(n, b0 + m);
    for (int e = threadIdx.x; e < DIM * kPanel; e += blockDim.x) {
        const int c = e / kPanel, r = e % kPanel;
        tv[c][r] = r < bm ? t[c * ldt + t0 + r] : 0.0;
    }
    __syncthreads();
    const int r = threadIdx.x & (kPanel - 1), h = threadIdx.x >> 7;
    double acc[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) acc[c] = 0.0;
    const double* col = Mrows + (int64_t)(h * 64) * kPanel + r;
    for (int j0 = 0; j0 < 64; j0 += 16) {
        double lv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) lv[u] = col[(j0 + u) * kPanel];
#pragma unroll
        for (int c = 0; c < DIM; ++c)
#pragma unroll
            for (int u = 0; u < 16; ++u) acc[c] = __builtin_fma(lv[u], tv[c][h * 64 + j0 + u], acc[c]);
    }
    if (h == 1)
#pragma unroll
        for (int c = 0; c < DIM; ++c) half[c][r] = acc[c];
    __syncthreads();
    if (h == 0)
#pragma unroll
        for (int c = 0; c < DIM; ++c) part[((int64_t)p * DIM + c) * kPanel + r] = acc[c] + half[c][r];
}

// x_i = sum of the step's partials for block i in increasing m (forward: m = 0 .. i, pairs
// (i, m); backward: m = i .. q-1, pairs (m, i)), written to rows b0 + i of x (ldx).
template <int DIM, bool BWD>
__global__ __launch_bounds__(kPanel) void lm_super_sum_kernel(int64_t n, int64_t s, int q,
                                                              const double* __restrict__ part,
                                                              double* __restrict__ x, int64_t ldx)
{
    const int i = blockIdx.x, r = threadIdx.x;
    const int64_t row = (s * kSuper + i) * kPanel + r;
    if (row >= n) return;
    double v[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) v[c] = 0.0;
    const int mb = BWD ? i : 0, me = BWD ? q : i + 1;
    for (int m = mb; m < me; ++m) {
        const int p = BWD ? m * (m + 1) / 2 + i : i * (i + 1) / 2 + m;
#pragma unroll
        for (int c = 0; c < DIM; ++c) v[c] += part[((int64_t)p * DIM + c) * kPanel + r];
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) x[c * ldx + row] = v[c];
}

// acc[c][col] -= sum_{m < w} L[m0 + m][col] x[c][m] for col in [c0, c1): rows m0 .. m0 + w - 1
// of L, contiguous in col (forward: columns past the superblock, the panel's transposed copy
// in the upper triangle; backward: columns before it, L below the diagonal).  x: rows m0 ..
// m0 + w - 1 of xs (ldx), staged in LDS.  A workgroup takes 64 columns at a time, one per
// lane; wave wv sums m over its quarter of [0, kSuper * kPanel) in batches of 32 loads, and
// the four wave sums are added in wave order.
template <int DIM>
__global__ __launch_bounds__(256) void lm_super_rows_kernel(const double* __restrict__ L, int64_t n, int64_t m0, int w,
                                                            const double* __restrict__ xs, int64_t ldx,
                                                            double* __restrict__ acc, int64_t lda, int64_t c0,
                                                            int64_t c1)
{
    constexpr int kW = kSuper * kPanel;
    __shared__ double xv[DIM][kW];
    __shared__ double red[4][DIM][64];
    for (int e = threadIdx.x; e < DIM * kW; e += blockDim.x) {
        const int c = e / kW, m = e % kW;
        xv[c][m] = m < w ? xs[c * ldx + m0 + m] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q4 = (w + 3) / 4;
    const int mb = wave * q4, me = (mb + q4 < w) ? mb + q4 : w;
    // workgroups are dealt to the 8 XCDs in turn: give each XCD a contiguous run of column
    // groups, so that the row segments one XCD streams at a time are adjacent (9.9 -> 9.3 ms
    // per solve at N = 65536 against the plain order)
    const unsigned G = gridDim.x;
    const unsigned grp = (G % 8u == 0u) ? (blockIdx.x % 8u) * (G / 8u) + blockIdx.x / 8u : blockIdx.x;
    for (int64_t cb = c0 + (int64_t)grp * 64; cb < c1; cb += (int64_t)G * 64) {
        const int64_t col = cb + lane;
        const bool ok = col < c1;
        const double* lp = L + (m0 + mb) * n + (ok ? col : cb);
        double sacc[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) sacc[c] = 0.0;
        int m = mb;
        for (; m + 32 <= me; m += 32, lp += 32 * n) {
            double lv[32];
#pragma unroll
            for (int u = 0; u < 32; ++u) lv[u] = lp[(int64_t)u * n];
#pragma unroll
            for (int c = 0; c < DIM; ++c)
#pragma unroll
                for (int u = 0; u < 32; ++u) sacc[c] = __builtin_fma(lv[u], xv[c][m + u], sacc[c]);
        }
        for (; m < me; ++m, lp += n) {
            const double lv = *lp;
#pragma unroll
            for (int c = 0; c < DIM; ++c) sacc[c] = __builtin_fma(lv, xv[c][m], sacc[c]);
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c) red[wave][c][lane] = sacc[c];
        __syncthreads();
        if (wave == 0 && ok)
#pragma unroll
            for (int c = 0; c < DIM; ++c)
                acc[c * lda + col] -= ((red[0][c][lane] + red[1][c][lane]) + red[2][c][lane]) + red[3][c][lane];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------------------

__global__ void lm_int_zero_kernel(int* p) { if (threadIdx.x == 0) *p = 0; }

int dense_panels(int64_t n) { return (int)((n + kPanel - 1) / kPanel); }
// the inverses of the diagonal blocks, then their transposes
int64_t dense_linv_elems(int64_t n) { return 2 * (int64_t)dense_panels(n) * kPanel * kPanel; }

int64_t dense_panel_f32_elems(int64_t n) { return n * kOuter * kPanel; }

hipError_t launch_dense_factor(int dim, int kernel, double kq, double tau, const double* X, int64_t n, double* K,
                               double* Linv, int* info, hipStream_t st, bool f32_update, float* panel)
{
    if (n <= 0 || n >= kDenseMaxN) return hipErrorInvalidValue;
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
    // Panels of kPanel columns are factored one by one, but the trailing matrix is updated once
    // per block of kOuter panels: within a block, panel s first takes the updates of
    // the block's earlier panels on its own column strip, and the rest of the matrix takes the
    // whole block in one pass.  That pass reads and writes the trailing matrix, so its HBM
    // traffic per flop falls with the block width.
    const int nb = dense_panels(n);
    for (int b0 = 0; b0 < nb; b0 += kOuter) {
        const int64_t kb = (int64_t)b0 * kPanel;
        int64_t kend = kb;
        for (int b = b0; b < nb && b < b0 + kOuter; ++b) {
            const int64_t k0 = (int64_t)b * kPanel;
            const int bs = (int)((n - k0) < kPanel ? (n - k0) : kPanel);
            if (k0 > kb) {
                const int64_t nt = (n - k0 + 63) / 64;
                hipLaunchKernelGGL(lm_syrk_kernel, dim3((unsigned)(2 * nt - 1)), dim3(256), 0, st, K, n, kb,
                                   (int)(k0 - kb), k0, 1);
            }
            double* Lb = Linv + (int64_t)b * kPanel * kPanel;
            double* LbT = Lb + (int64_t)nb * kPanel * kPanel;
            hipLaunchKernelGGL(lm_potrf_inv_kernel, dim3(1), dim3(256), 0, st, K, n, k0, bs, Lb, LbT, info);
            const int64_t below = n - k0 - bs;
            if (below > 0)
                hipLaunchKernelGGL(lm_panel_kernel, dim3((unsigned)((below + 63) / 64)), dim3(256), 0, st, K, n, k0,
                                   bs, (const double*)Lb);
            kend = k0 + bs;
        }
        const int64_t rest = n - kend;
        if (rest <= 0) continue;
        const int width = (int)(kend - kb);
        if (rest >= 1024) {
            const int64_t nt = (rest + 127) / 128;
            if (f32_update && panel) {
                hipLaunchKernelGGL(lm_panel_f32_kernel, dim3((unsigned)rest), dim3(256), 0, st, (const double*)K, n, kb,
                                   width, kend, panel);
                hipLaunchKernelGGL(lm_syrk128_f32_kernel<true>, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, st, K,
                                   n, kb, width, kend, (const float*)panel);
            } else if (f32_update) {
                hipLaunchKernelGGL(lm_syrk128_f32_kernel<false>, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, st,
                                   K, n, kb, width, kend, (const float*)nullptr);
            } else
                hipLaunchKernelGGL(lm_syrk128_kernel, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, st, K, n, kb,
                                   width, kend);
        } else {
            const int64_t nt = (rest + 63) / 64;
            hipLaunchKernelGGL(lm_syrk_kernel, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, st, K, n, kb,
                               width, kend, 0);
        }
    }
    return hipGetLastError();
}

hipError_t launch_dense_solve(const double* L, const double* Linv, int64_t n, int dim, double* y, int64_t ldy,
                              hipStream_t st)
{
    const int nb = dense_panels(n);
    // enough workgroups to stream a panel at full bandwidth, never more than its rows need
    auto groups = [&](int64_t items, int64_t per_group) -> unsigned {
        int64_t g = 1 + (items + per_group - 1) / per_group;
        return (unsigned)(g < 2049 ? g : 2049);
    };
    for (int64_t k = -1; k < nb - 1; ++k) {
        const int64_t below = n - (k + 2) * kPanel;
        const dim3 g(k < 0 ? 1u : groups(below > 0 ? below : 0, 64));
        if (dim == 2)
            hipLaunchKernelGGL(lm_trsv_fwd_kernel<2>, g, dim3(256), 0, st, L, Linv, n, nb, k, y, ldy);
        else
            hipLaunchKernelGGL(lm_trsv_fwd_kernel<3>, g, dim3(256), 0, st, L, Linv, n, nb, k, y, ldy);
    }
    for (int64_t k = nb; k > 0; --k) {
        const int64_t above = (k - 1) * kPanel;
        const dim3 g(k == nb ? 1u : groups(above, 256));
        if (dim == 2)
            hipLaunchKernelGGL(lm_trsv_bwd_kernel<2>, g, dim3(256), 0, st, L, Linv, n, nb, k, y, ldy);
        else
            hipLaunchKernelGGL(lm_trsv_bwd_kernel<3>, g, dim3(256), 0, st, L, Linv, n, nb, k, y, ldy);
    }
    return hipGetLastError();
}

bool dense_super_default(int64_t n) { return dense_panels(n) > kSuper; }

hipError_t launch_dense_super(const double* L, const double* Linv, int64_t n, double* W, hipStream_t st)
{
    const int nb = dense_panels(n), ns = super_count(n);
    for (int d = 1; d < kSuper && d < nb; ++d) {
        const dim3 g((unsigned)(ns * (kSuper - d)));
        hipLaunchKernelGGL(lm_super_s_kernel, g, dim3(256), 0, st, L, Linv, W, n, nb, ns, d);
        hipLaunchKernelGGL(lm_super_w_kernel, g, dim3(256), 0, st, Linv, W, n, nb, ns, d);
    }
    return hipGetLastError();
}

template <int DIM>
static void super_sweeps(const double* L, const double* Linv, const double* W, int64_t n, double* y, int64_t ldy,
                         double* scratch, hipStream_t st)
{
    const int nb = dense_panels(n), ns = super_count(n);
    double* z = scratch;                 // DIM x n, leading dimension n
    double* part = scratch + 3 * n;      // kSuperProds x DIM x kPanel
    auto groups = [](int64_t cols) -> unsigned {
        const int64_t g = (cols + 63) / 64;
        return (unsigned)(g < 2048 ? g : 2048);
    };
    // forward: L z = y (y is the accumulator)
    for (int s = 0; s < ns; ++s) {
        const int64_t b0 = (int64_t)s * kSuper;
        const int q = (int)((nb - b0) < kSuper ? (nb - b0) : kSuper);
        const int64_t m0 = b0 * kPanel;
        const int w = (int)((n - m0) < (int64_t)q * kPanel ? (n - m0) : (int64_t)q * kPanel);
        hipLaunchKernelGGL((lm_super_prod_kernel<DIM, false>), dim3(q * (q + 1) / 2), dim3(256), 0, st, Linv, W, n,
                           nb, ns, (int64_t)s, (const double*)y, ldy, part);
        hipLaunchKernelGGL((lm_super_sum_kernel<DIM, false>), dim3(q), dim3(kPanel), 0, st, n, (int64_t)s, q,
                           (const double*)part, z, n);
        const int64_t c0 = m0 + w;
        if (c0 < n)
            hipLaunchKernelGGL(lm_super_rows_kernel<DIM>, dim3(groups(n - c0)), dim3(256), 0, st, L, n, m0, w,
                               (const double*)z, n, y, ldy, c0, n);
    }
    // backward: L^T x = z (z is the accumulator, x goes to y)
    for (int s = ns - 1; s >= 0; --s) {
        const int64_t b0 = (int64_t)s * kSuper;
        const int q = (int)((nb - b0) < kSuper ? (nb - b0) : kSuper);
        const int64_t m0 = b0 * kPanel;
        const int w = (int)((n - m0) < (int64_t)q * kPanel ? (n - m0) : (int64_t)q * kPanel);
        hipLaunchKernelGGL((lm_super_prod_kernel<DIM, true>), dim3(q * (q + 1) / 2), dim3(256), 0, st, Linv, W, n,
                           nb, ns, (int64_t)s, (const double*)z, n, part);
        hipLaunchKernelGGL((lm_super_sum_kernel<DIM, true>), dim3(q), dim3(kPanel), 0, st, n, (int64_t)s, q,
                           (const double*)part, y, ldy);
        if (m0 > 0)
            hipLaunchKernelGGL(lm_super_rows_kernel<DIM>, dim3(groups(m0)), dim3(256), 0, st, L, n, m0, w,
                               (const double*)y, ldy, z, n, (int64_t)0, m0);
    }
}

hipError_t launch_dense_solve_super(const double* L, const double* Linv, const double* W, int64_t n, int dim,
                                    double* y, int64_t ldy, double* scratch, hipStream_t st)
{
    if (dim == 2)
        super_sweeps<2>(L, Linv, W, n, y, ldy, scratch, st);
    else
        super_sweeps<3>(L, Linv, W, n, y, ldy, scratch, st);
    return hipGetLastError();
}

}  // namespace lm
