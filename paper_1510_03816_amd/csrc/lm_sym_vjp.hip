// lm_sym_vjp.hip -- the vector-Jacobian product of the N-particle right-hand side with each
// unordered pair evaluated once (gfx950, double precision).
//
// For the cotangent (a, b) of (dq/dt, dp/dt) at (q, p) the pair (k, j) adds to particle k
// (lm_adjoint.hip states the sums; d = q_k - q_j, e = b_k - b_j)
//     ap_k += G a_j + w (e . d) p_j
//     aq_k += [(p_k . p_j)(e . d) u - w ((a_k . p_j) + (a_j . p_k))] d + (p_k . p_j) w e.
// Exchanging k and j flips d and e and leaves e . d, p_k . p_j, a_k . p_j + a_j . p_k, G, w and
// u unchanged, so the same evaluation gives particle j
//     ap_j += G a_k + w (e . d) p_k,        aq_j -= (the aq_k term).
// The shared part (distance, 1/sqrt, exponential, weights, the three products) is most of
// a pair's work, so the unordered sweep costs a little over half of the one-sided kernel's.
//
// Decomposition, staging, column sums and partial-sum slots as in lm_sym.hip: each wave holds
// two row tiles (q, p, a, b of two points per lane, their sums in registers); a column tile is
// staged in LDS twice in a row, (q, p, a, b) interleaved and padded to an odd stride, lane l
// reading entry l + k at step k; the column-side terms go to the wave's own double array
// with ds_add_f64; the waves' arrays are added in wave order after each column tile; every
// point gets one partial per partner superblock (slot layout of lm_vjp_finish_kernel: aq in
// component c, ap in dim + c), added in a fixed order by lm_vjp_finish_kernel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lm_internal.h"
#include "lm_math.h"
#include "lm_sym.h"

namespace lm {

namespace {

// Doubles per staged column point: q, p, a, b and one pad word (odd stride: conflict-free reads).
__host__ __device__ constexpr int vjp_stride(int dim) { return 4 * dim + 1; }

// The shared part of the pair (k, j): d, e and the coefficients g (of a), t1 = w (e . d) (of p),
// td (of d) and te (of e).  Coincident particles (d = 0) keep only the G a term.
template <int DIM, int KER>
__device__ __forceinline__ void vjp_shared(const double (&qk)[DIM], const double (&pk)[DIM], const double (&ak)[DIM],
                                           const double (&bk)[DIM], const double (&qj)[DIM], const double (&pj)[DIM],
                                           const double (&aj)[DIM], const double (&bj)[DIM], double kq, double c1,
                                           double c2, double (&d)[DIM], double (&e)[DIM], double& g, double& t1,
                                           double& td, double& te)
{
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        d[c] = qk[c] - qj[c];
        s = __builtin_fma(d[c], d[c], s);
    }
    double w, u;
    if constexpr (KER == LM_KERNEL_CONON) {
        // w = G/(sigma r), u = w'/r = -w rho (rho + 1/sigma) with rho = 1/r; c1 = 1/sigma
        const double sc = __builtin_fmax(s, 1e-200);
        const double rho = rsqrt_pos(sc);
        g = exp2_nonpos(sc * rho * kq);
        const double gm = s > 0.0 ? g : 0.0;   // coincident particles: w = u = 0
        w = gm * rho * c1;
        u = -w * rho * (rho + c1);
    } else {
        // w = 2G/sigma^2, u = -4G/sigma^4; c1 = 2/sigma^2, c2 = -4/sigma^4
        g = exp2_nonpos(s * kq);
        const double gm = s > 0.0 ? g : 0.0;   // coincident particles: w = u = 0
        w = gm * c1;
        u = gm * c2;
    }
    double ed = 0.0, apj = 0.0, pp = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        e[c] = bk[c] - bj[c];
        ed = __builtin_fma(e[c], d[c], ed);
        apj = __builtin_fma(ak[c], pj[c], __builtin_fma(aj[c], pk[c], apj));
        pp = __builtin_fma(pk[c], pj[c], pp);
    }
    t1 = w * ed;
    td = __builtin_fma(pp * ed, u, -w * apj);
    te = pp * w;
}

// Row data of a lane: q, p, a, b of ROWS points.
template <int DIM, int ROWS>
struct VjpRows {
    double q[ROWS][DIM], p[ROWS][DIM], a[ROWS][DIM], b[ROWS][DIM];
};

// One step: the lane's ROWS row points against column entry `src`; with JSIDE the column-side
// terms go to the wave's column array at `acc` (aq component c at acc[c * 128], ap at
// acc[(DIM + c) * 128]).
template <int DIM, int KER, int ROWS, bool JSIDE>
__device__ __forceinline__ void vjp_step(const VjpRows<DIM, ROWS>& R, const double* __restrict__ src, double kq,
                                         double c1, double c2, double (&gq)[ROWS][DIM], double (&gp)[ROWS][DIM],
                                         double* __restrict__ acc)
{
    double qj[DIM], pj[DIM], aj[DIM], bj[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        qj[c] = src[c];
        pj[c] = src[DIM + c];
        aj[c] = src[2 * DIM + c];
        bj[c] = src[3 * DIM + c];
    }
    double tq[DIM], tp[DIM];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        double d[DIM], e[DIM], g, t1, td, te;
        vjp_shared<DIM, KER>(R.q[r], R.p[r], R.a[r], R.b[r], qj, pj, aj, bj, kq, c1, c2, d, e, g, t1, td, te);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            gp[r][c] = __builtin_fma(g, aj[c], gp[r][c]);
            gp[r][c] = __builtin_fma(t1, pj[c], gp[r][c]);
            const double v = __builtin_fma(td, d[c], te * e[c]);
            gq[r][c] += v;
            if (JSIDE) {
                tp[c] = (r == 0) ? __builtin_fma(g, R.a[r][c], t1 * R.p[r][c])
                                 : __builtin_fma(g, R.a[r][c], __builtin_fma(t1, R.p[r][c], tp[c]));
                tq[c] = (r == 0) ? -v : tq[c] - v;
            }
        }
    }
    if constexpr (JSIDE) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            __hip_atomic_fetch_add(acc + c * 128, tq[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(acc + (DIM + c) * 128, tp[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
}

template <int DIM, int KER, int ROWS, bool JSIDE>
__device__ __forceinline__ void vjp_block(const VjpRows<DIM, ROWS>& R, const double* __restrict__ jb, double kq,
                                          double c1, double c2, double (&gq)[ROWS][DIM], double (&gp)[ROWS][DIM],
                                          double* __restrict__ acc)
{
    constexpr int E = vjp_stride(DIM);
    for (int k0 = 0; k0 < kSymSteps; k0 += kSymUnroll) {
#pragma unroll
        for (int u = 0; u < kSymUnroll; ++u)
            vjp_step<DIM, KER, ROWS, JSIDE>(R, jb + (k0 + u) * E, kq, c1, c2, gq, gp, acc + k0 + u);
    }
}

// Column tile J into jbuf (entry e: point J*64 + (e mod 64), its q, p, a, b; zeros past n,
// which add exactly nothing to real points).
template <int DIM>
__device__ __forceinline__ void vjp_stage(double* __restrict__ jbuf, const VjpArgs& A, int64_t J)
{
    constexpr int E = vjp_stride(DIM);
    const int64_t n = A.n;
    const double* const arrays[4] = {A.q, A.p, A.a, A.b};
#pragma unroll
    for (int arr = 0; arr < 4; ++arr) {
        const double* __restrict__ src = arrays[arr];
        for (int t = threadIdx.x; t < kSymSteps * DIM; t += blockDim.x) {
            const int cc = t >> 6, l = t & 63;
            const int64_t j = J * kSymSteps + l;
            const double x = j < n ? src[cc * n + j] : 0.0;
            jbuf[l * E + arr * DIM + cc] = x;
            jbuf[(l + 64) * E + arr * DIM + cc] = x;
        }
    }
}

template <int DIM, int KER>
__global__ __launch_bounds__(512, 3) void lm_sym_vjp_kernel(VjpArgs A, int64_t NT, int64_t S)
{
    constexpr int E = vjp_stride(DIM);
    constexpr int EC = 2 * DIM;
    extern __shared__ double lds_words[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    const int64_t side = kSymRows * (int64_t)nw;
    double* region = lds_words;                   // [nw][EC][128]
    double* jbuf = region + nw * EC * 128;        // [128][E]

    int64_t X, Y;
    sym_superblocks(blockIdx.x, S, X, Y);
    const bool diag = X == Y;
    const int64_t n = A.n;

    int64_t I[kSymRows];
    VjpRows<DIM, kSymRows> R;
    double gq[kSymRows][DIM], gp[kSymRows][DIM];
#pragma unroll
    for (int r = 0; r < kSymRows; ++r) {
        I[r] = X * side + kSymRows * wave + r;
        const int64_t i = I[r] * kSymSteps + lane;
        const bool live = i < n;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            R.q[r][c] = live ? A.q[c * n + i] : 0.0;
            R.p[r][c] = live ? A.p[c * n + i] : 0.0;
            R.a[r][c] = live ? A.a[c * n + i] : 0.0;
            R.b[r][c] = live ? A.b[c * n + i] : 0.0;
            gq[r][c] = 0.0;
            gp[r][c] = 0.0;
        }
    }

    for (int t = threadIdx.x; t < nw * EC * 128; t += blockDim.x) region[t] = 0.0;
    const int64_t J0 = Y * side;
    const int64_t J1 = (J0 + side < NT) ? (J0 + side) : NT;
    vjp_stage<DIM>(jbuf, A, J0);
    __syncthreads();

    const double* jb = jbuf + lane * E;
    double* acc = region + wave * EC * 128 + lane;
    double* pc = A.part + (diag ? S : X) * (2 * DIM) * n;
    for (int64_t J = J0; J < J1; ++J) {
        const bool all = diag ? J > I[kSymRows - 1] : I[kSymRows - 1] < NT;
        if (all) {
            vjp_block<DIM, KER, kSymRows, true>(R, jb, A.kq, A.c1, A.c2, gq, gp, acc);
        } else {
#pragma unroll
            for (int r = 0; r < kSymRows; ++r) {
                const int m = sym_mode(diag, I[r], J, NT);
                if (m == SYM_SKIP) continue;
                VjpRows<DIM, 1> R1;
                double gq1[1][DIM], gp1[1][DIM];
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    R1.q[0][c] = R.q[r][c];
                    R1.p[0][c] = R.p[r][c];
                    R1.a[0][c] = R.a[r][c];
                    R1.b[0][c] = R.b[r][c];
                    gq1[0][c] = gq[r][c];
                    gp1[0][c] = gp[r][c];
                }
                if (m == SYM_BOTH)
                    vjp_block<DIM, KER, 1, true>(R1, jb, A.kq, A.c1, A.c2, gq1, gp1, acc);
                else
                    vjp_block<DIM, KER, 1, false>(R1, jb, A.kq, A.c1, A.c2, gq1, gp1, acc);
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    gq[r][c] = gq1[0][c];
                    gp[r][c] = gp1[0][c];
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
            if (j < n) pc[c * n + j] = s;
        }
        if (J + 1 < J1) vjp_stage<DIM>(jbuf, A, J + 1);
        __syncthreads();
    }

    double* pr = A.part + Y * (2 * DIM) * n;
#pragma unroll
    for (int r = 0; r < kSymRows; ++r) {
        const int64_t i = I[r] * kSymSteps + lane;
        if (I[r] >= NT || i >= n) continue;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            pr[c * n + i] = gq[r][c];
            pr[(DIM + c) * n + i] = gp[r][c];
        }
    }
}

template <int DIM, int KER>
hipError_t launch_sym_vjp_t(const VjpArgs& a, int waves, int64_t nsb, hipStream_t st)
{
    const size_t lds = ((size_t)waves * 2 * DIM * 128 + (size_t)128 * vjp_stride(DIM)) * sizeof(double);
    hipLaunchKernelGGL((lm_sym_vjp_kernel<DIM, KER>), dim3((unsigned)(nsb * (nsb + 1) / 2)), dim3(64 * waves), lds, st,
                       a, tiles_of(a.n), nsb);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sym_vjp(int dim, int kernel, const VjpArgs& a, int waves, int64_t nsb, hipStream_t st)
{
    if (dim == 2)
        return kernel == LM_KERNEL_CONON ? launch_sym_vjp_t<2, LM_KERNEL_CONON>(a, waves, nsb, st)
                                         : launch_sym_vjp_t<2, LM_KERNEL_GAUSS>(a, waves, nsb, st);
    return kernel == LM_KERNEL_CONON ? launch_sym_vjp_t<3, LM_KERNEL_CONON>(a, waves, nsb, st)
                                     : launch_sym_vjp_t<3, LM_KERNEL_GAUSS>(a, waves, nsb, st);
}

}  // namespace lm
