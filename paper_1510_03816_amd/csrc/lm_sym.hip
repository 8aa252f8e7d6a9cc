// lm_sym.hip -- the N-particle pair sums with each unordered pair evaluated once (gfx950).
//
// In the right-hand side of the N-particle system (equation "N-particle") the kernel value
// G(|q_i - q_j|), the force weight w(|q_i - q_j|) and the momentum product p_i . p_j are
// symmetric in (i, j) and the distance vector q_i - q_j changes sign, so one evaluation of
// a pair serves both particles:
//     v_i += g p_j,  v_j += g p_i,  f_i += (p_i . p_j) w d,  f_j -= (p_i . p_j) w d,  d = q_i - q_j.
// The shared part (distance, 1/sqrt, exponential, weight, momentum product) is about three
// quarters of a pair's work, so a sweep over the N(N+1)/2 unordered pairs costs about 55% of
// the N^2 ordered ones.  Used for the self-interaction of one point set in double precision
// (right-hand side, RK4 stages, K x); targets distinct from the sources, tile skipping and
// single precision keep the one-sided kernel in lm_kernels.hip.
//
// Decomposition.  The 64-point tiles are grouped into superblocks of B = 2W tiles; a
// workgroup of W wavefronts takes one pair (X, Y), X <= Y, of superblocks.  Wave w owns the
// two row tiles X*B + 2w and X*B + 2w + 1 (one point of each per lane, in registers, with
// their row sums) and the W waves walk the B column tiles of superblock Y together:
//   - the column tile (q, p interleaved) is staged in LDS twice in a row, so that at step k
//     lane l reads entry l + k -- point (l + k) mod 64 -- at an immediate offset, and over 64
//     steps every lane meets every point of the tile once;
//   - the column-side terms go to the wave's own LDS array with ds_add_f64 at the same entry
//     l + k (128 entries, the two halves added at the end), so no two lanes of an instruction
//     touch the same word and each wave's sums have a fixed order;
//   - after the tile, the W waves' arrays are added in wave order and written out.
// In a diagonal superblock (X = Y) a row tile meets the column tiles after it symmetrically,
// itself one-sidedly (all 64 x 64 ordered pairs, the self pair included), and skips the ones
// before it (those pairs are done from the other side).
//
// Partial sums.  A point of superblock Z receives one partial from each superblock pair that
// contains Z: from (Z, Y), Y > Z, as a row (slot Y); from (Y, Z), Y < Z, as a column (slot Y);
// from (Z, Z) both (row: slot Z, column: slot S).  Every one of the S + 1 slots of a point is
// written exactly once per launch, and lm_finish_kernel adds them in slot order, so the
// result is bitwise reproducible.  The force constant is applied when a partial is written.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>

#include "lm_internal.h"
#include "lm_math.h"

namespace lm {

namespace {

constexpr int kSymSteps = 64;     // column points per tile
constexpr int kSymUnroll = 8;     // steps per unrolled loop body

// Doubles per staged column point: q and p, padded by one so that the 64 lanes' reads of
// consecutive entries (stride 14 or 10 words) fall in distinct LDS banks.
__host__ __device__ constexpr int sym_stride(int dim) { return 2 * dim + 1; }

// The symmetric part of a pair: d = q_i - q_j, kernel value g and force weight w (without
// the constant, which is applied to the sums).
template <int DIM, int KER>
__device__ __forceinline__ void sym_pair(const double (&qi)[DIM], const double (&qj)[DIM], double kq,
                                         double (&d)[DIM], double& g, double& w)
{
    // conon: the squared distance starts at 1e-300 (see pair_f64) so the self pair and
    // padding points at the same position give a finite weight times d = 0
    double s = (KER == LM_KERNEL_CONON) ? 1e-300 : 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        d[c] = qi[c] - qj[c];
        s = __builtin_fma(d[c], d[c], s);
    }
    if constexpr (KER == LM_KERNEL_CONON) {
        const double rho = rsqrt_pos(s);
        g = exp_nonpos(s * rho * kq);
        w = g * rho;
    } else {
        g = exp_nonpos(s * kq);
        w = g;
    }
}

// One step: the ROWS row points of this lane against column entry `src` (q then p).  With
// JSIDE the column-side terms are added into the wave's column array at `acc` (component c
// at acc[c * 128]).
template <int DIM, int KER, bool FORCE, int ROWS, bool JSIDE>
__device__ __forceinline__ void sym_step(const double (&qi)[ROWS][DIM], const double (&pi)[ROWS][DIM],
                                         const double* __restrict__ src, double kq, double (&v)[ROWS][DIM],
                                         double (&f)[ROWS][DIM], double* __restrict__ acc)
{
    double qj[DIM], pj[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        qj[c] = src[c];
        pj[c] = src[DIM + c];
    }
    double tv[DIM], tf[DIM];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        double d[DIM], g, w;
        sym_pair<DIM, KER>(qi[r], qj, kq, d, g, w);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            v[r][c] = __builtin_fma(g, pj[c], v[r][c]);
            if (JSIDE) tv[c] = (r == 0) ? g * pi[r][c] : __builtin_fma(g, pi[r][c], tv[c]);
        }
        if constexpr (FORCE) {
            double pp = pi[r][0] * pj[0];
#pragma unroll
            for (int c = 1; c < DIM; ++c) pp = __builtin_fma(pi[r][c], pj[c], pp);
            const double cw = pp * w;
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                f[r][c] = __builtin_fma(cw, d[c], f[r][c]);
                if (JSIDE) tf[c] = (r == 0) ? -cw * d[c] : __builtin_fma(-cw, d[c], tf[c]);
            }
        }
    }
    if constexpr (JSIDE) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            __hip_atomic_fetch_add(acc + c * 128, tv[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (FORCE)
                __hip_atomic_fetch_add(acc + (DIM + c) * 128, tf[c], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
}

// All 64 steps of one (row tile(s), column tile) block.  jb = this lane's first column entry
// (jbuf + lane * sym_stride(DIM)), acc = this lane's first word of the wave's column array.
template <int DIM, int KER, bool FORCE, int ROWS, bool JSIDE>
__device__ __forceinline__ void sym_block(const double (&qi)[ROWS][DIM], const double (&pi)[ROWS][DIM],
                                          const double* __restrict__ jb, double kq, double (&v)[ROWS][DIM],
                                          double (&f)[ROWS][DIM], double* __restrict__ acc)
{
    constexpr int E = sym_stride(DIM);
    for (int k0 = 0; k0 < kSymSteps; k0 += kSymUnroll) {
#pragma unroll
        for (int u = 0; u < kSymUnroll; ++u)
            sym_step<DIM, KER, FORCE, ROWS, JSIDE>(qi, pi, jb + (k0 + u) * E, kq, v, f, acc + k0 + u);
    }
}

// Loads column tile J into jbuf: entry e (0..127) holds point J*64 + (e mod 64), its q then
// its p (the pad word is never read); points past n are zero (zero momentum: they add exactly nothing to real points).
template <int DIM>
__device__ __forceinline__ void sym_stage(double* __restrict__ jbuf, const double* __restrict__ q,
                                          const double* __restrict__ p, int64_t n, int64_t J)
{
    constexpr int E = sym_stride(DIM);
    for (int t = threadIdx.x; t < kSymSteps * 2 * DIM; t += blockDim.x) {
        const int c = t >> 6, l = t & 63;
        const int64_t j = J * kSymSteps + l;
        double x = 0.0;
        if (j < n) x = (c < DIM) ? q[c * n + j] : p[(c - DIM) * n + j];
        jbuf[l * E + c] = x;
        jbuf[(l + 64) * E + c] = x;
    }
}

enum SymMode : int { SYM_SKIP = 0, SYM_ONE = 1, SYM_BOTH = 2 };

// What row tile I does with column tile J in superblock pair (X, Y).
__device__ __forceinline__ int sym_mode(bool diag, int64_t I, int64_t J, int64_t T)
{
    if (I >= T) return SYM_SKIP;
    if (!diag || I < J) return SYM_BOTH;
    return I == J ? SYM_ONE : SYM_SKIP;
}

template <int DIM, int KER, bool FORCE>
__global__ __launch_bounds__(512, kSymOccupancy) void lm_sym_pair_kernel(SymArgs a)
{
    constexpr int E = sym_stride(DIM);           // staged doubles per column point
    constexpr int EC = FORCE ? 2 * DIM : DIM;    // column sums per point
    extern __shared__ double lds[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    const int64_t side = kSymRows * (int64_t)nw;
    double* jbuf = lds;                          // [128][E]
    double* region = lds + 128 * E;              // [nw][EC][128]

    // superblock pair: off-diagonal pairs (X < Y) first, numbered Y(Y-1)/2 + X, then the
    // diagonal ones, which carry half the work
    const int64_t S = a.nsb;
    const int64_t noff = S * (S - 1) / 2;
    const int64_t b = blockIdx.x;
    int64_t X, Y;
    if (b < noff) {
        int64_t y = (int64_t)(0.5 * (1.0 + __builtin_sqrt(1.0 + 8.0 * (double)b)));
        while (y * (y - 1) / 2 > b) --y;
        while ((y + 1) * y / 2 <= b) ++y;
        Y = y;
        X = b - y * (y - 1) / 2;
    } else {
        X = Y = b - noff;
    }
    const bool diag = X == Y;
    const int64_t n = a.n, T = a.tiles;

    int64_t I[kSymRows];
    double qi[kSymRows][DIM], pi[kSymRows][DIM], v[kSymRows][DIM], f[kSymRows][DIM];
#pragma unroll
    for (int r = 0; r < kSymRows; ++r) {
        I[r] = X * side + kSymRows * wave + r;
        const int64_t i = I[r] * kSymSteps + lane;
        const bool live = i < n;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            qi[r][c] = live ? a.q[c * n + i] : 0.0;
            pi[r][c] = live ? a.p[c * n + i] : 0.0;
            v[r][c] = 0.0;
            f[r][c] = 0.0;
        }
    }

    for (int t = threadIdx.x; t < nw * EC * 128; t += blockDim.x) region[t] = 0.0;
    const int64_t J0 = Y * side;
    const int64_t J1 = (J0 + side < T) ? (J0 + side) : T;
    sym_stage<DIM>(jbuf, a.q, a.p, n, J0);
    __syncthreads();

    const double* jb = jbuf + lane * E;
    double* acc = region + wave * EC * 128 + lane;
    const int64_t slot_col = diag ? S : X;
    double* pc = a.part + slot_col * (2 * DIM) * n;
    for (int64_t J = J0; J < J1; ++J) {
        // every row tile meets J from both sides, except near the diagonal
        const bool all = diag ? J > I[kSymRows - 1] : I[kSymRows - 1] < T;
        if (all) {
            sym_block<DIM, KER, FORCE, kSymRows, true>(qi, pi, jb, a.kq, v, f, acc);
        } else {
#pragma unroll
            for (int r = 0; r < kSymRows; ++r) {
                const int m = sym_mode(diag, I[r], J, T);
                if (m == SYM_SKIP) continue;
                double q1[1][DIM], p1[1][DIM], v1[1][DIM], f1[1][DIM];
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    q1[0][c] = qi[r][c];
                    p1[0][c] = pi[r][c];
                    v1[0][c] = v[r][c];
                    f1[0][c] = f[r][c];
                }
                if (m == SYM_BOTH)
                    sym_block<DIM, KER, FORCE, 1, true>(q1, p1, jb, a.kq, v1, f1, acc);
                else
                    sym_block<DIM, KER, FORCE, 1, false>(q1, p1, jb, a.kq, v1, f1, acc);
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    v[r][c] = v1[0][c];
                    f[r][c] = f1[0][c];
                }
            }
        }
        __syncthreads();
        // column sums of tile J: the waves in order, each wave's two halves in order
        for (int t = threadIdx.x; t < EC * 64; t += blockDim.x) {
            const int c = t >> 6, l = t & 63;
            double s = 0.0;
            for (int w = 0; w < nw; ++w) {
                double* rg = region + (w * EC + c) * 128;
                s += rg[l];
                s += rg[l + 64];
                rg[l] = 0.0;
                rg[l + 64] = 0.0;
            }
            const int64_t j = J * kSymSteps + l;
            if (j < n) pc[c * n + j] = (c < DIM) ? s : s * a.wscale;
        }
        if (J + 1 < J1) sym_stage<DIM>(jbuf, a.q, a.p, n, J + 1);
        __syncthreads();
    }

    double* pr = a.part + Y * (2 * DIM) * n;
#pragma unroll
    for (int r = 0; r < kSymRows; ++r) {
        const int64_t i = I[r] * kSymSteps + lane;
        if (I[r] >= T || i >= n) continue;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            pr[c * n + i] = v[r][c];
            if (FORCE) pr[(DIM + c) * n + i] = f[r][c] * a.wscale;
        }
    }
}

template <int DIM, int KER, bool FORCE>
hipError_t launch_sym_t(const SymArgs& a, int waves, hipStream_t st)
{
    constexpr int EC = FORCE ? 2 * DIM : DIM;
    const size_t lds = (size_t)(128 * sym_stride(DIM) + waves * EC * 128) * sizeof(double);
    const int64_t S = a.nsb;
    hipLaunchKernelGGL((lm_sym_pair_kernel<DIM, KER, FORCE>), dim3((unsigned)(S * (S + 1) / 2)),
                       dim3(64 * waves), lds, st, a);
    return hipGetLastError();
}

}  // namespace

SymPlan plan_sym(int64_t n, bool force)
{
    SymPlan sp{};
    const int64_t T = tiles_of(n);
    // LM_SYM_WAVES fixes the workgroup width (tuning runs, tests of every width)
    const char* env = getenv("LM_SYM_WAVES");
    const int fixed = env ? atoi(env) : 0;
    int w = 0;
    if (fixed == 1 || fixed == 2 || fixed == 4 || fixed == 8) {
        w = fixed;
    } else if (T >= kSymWideTiles) {
        w = 4;
    } else if (T >= kSymMinTiles) {
        w = 2;
    } else if (force) {
        w = 1;
    }
    if (w == 0) return sp;
    // partial sums: (S + 1) slots of up to 6 doubles per point; wider superblocks need
    // fewer, and beyond the cap the one-sided kernel (at most 64 slots) is used instead
    for (;; w *= 2) {
        const int64_t S = (T + kSymRows * w - 1) / (kSymRows * w);
        const bool fits = (S + 1) * 6 * n * (int64_t)sizeof(double) <= kSymMaxPartBytes;
        if (fits && S * (S + 1) / 2 < ((int64_t)1 << 31)) {
            sp.waves = w;
            sp.nsb = S;
            return sp;
        }
        if (w >= kSymMaxWaves || fixed) return sp;
    }
}

hipError_t launch_sym_pair(int dim, int kernel, bool force, const SymArgs& a, int waves, hipStream_t st)
{
    if (dim == 2) {
        if (kernel == LM_KERNEL_CONON)
            return force ? launch_sym_t<2, LM_KERNEL_CONON, true>(a, waves, st)
                         : launch_sym_t<2, LM_KERNEL_CONON, false>(a, waves, st);
        return force ? launch_sym_t<2, LM_KERNEL_GAUSS, true>(a, waves, st)
                     : launch_sym_t<2, LM_KERNEL_GAUSS, false>(a, waves, st);
    }
    if (kernel == LM_KERNEL_CONON)
        return force ? launch_sym_t<3, LM_KERNEL_CONON, true>(a, waves, st)
                     : launch_sym_t<3, LM_KERNEL_CONON, false>(a, waves, st);
    return force ? launch_sym_t<3, LM_KERNEL_GAUSS, true>(a, waves, st)
                 : launch_sym_t<3, LM_KERNEL_GAUSS, false>(a, waves, st);
}

}  // namespace lm
