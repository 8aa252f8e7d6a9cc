// lm_adjoint.hip -- reverse mode of the shooting map: the vector-Jacobian product (VJP) of the
// N-particle right-hand side and the epilogue that chains the four RK4 stages backwards.
//
// For the cotangent (a, b) of (dq/dt, dp/dt) at (q, p), with w = -G'(r)/r, u = w'(r)/r,
// d = q_k - q_j and e = b_k - b_j (differentiating the sums of the N-particle system):
//   ap_k = tau a_k + sum_j G_kj a_j + sum_{j != k} w (e . d) p_j
//   aq_k = sum_{j != k} [ -w ((a_k . p_j) + (a_j . p_k)) d + (p_k . p_j) (w e + (e . d) u d) ]
// Coincident particles contribute only to the first sum, as in the forward sums.
//
// Work decomposition as in lm_pair_kernel: 64 targets k per workgroup (one per lane), the
// sources j split into contiguous chunks per (wave, grid-y), source data wave-uniform (scalar
// loads of q_j, p_j, a_j, b_j into SGPR operands, from an interleaved copy written by
// lm_vjp_pack_kernel), wave partials combined in LDS in wave order, grid-y splits by
// lm_vjp_finish_kernel in a fixed order.  FP64 only.  From the size where the forward sums
// use the symmetric kernel, the VJP does too (lm_sym_vjp.hip: each unordered pair once).
//
// Adjoint of one RK4 step y' = y + dt/6 (k1 + 2k2 + 2k3 + k4), k_s = f(Y_s), given the
// cotangent abar of y' (stages visited 4, 3, 2, 1):
//   Yb4 = J(Y4)^T (dt/6 abar),            next = dt/3 abar + dt   Yb4,  lam  = abar + Yb4
//   Yb3 = J(Y3)^T next,                   next = dt/3 abar + dt/2 Yb3,  lam += Yb3
//   Yb2 = J(Y2)^T next,                   next = dt/6 abar + dt/2 Yb2,  lam += Yb2
//   Yb1 = J(Y1)^T next,                                                 lam += Yb1
// and lam is the cotangent of y.  Each VJP launch does one line in its epilogue.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lm_internal.h"
#include "lm_math.h"

namespace lm {

#ifndef LM_VJP_UNROLL
#define LM_VJP_UNROLL 2
#endif

constexpr int kTileA = kTile;     // same launch plan as the pair kernel
constexpr int kWavesA = kWaves;

template <int DIM, int KER>
__device__ __forceinline__ void vjp_pair(const double (&qk)[DIM], const double (&pk)[DIM], const double (&ak)[DIM],
                                         const double (&bk)[DIM], const double (&qj)[DIM], const double (&pj)[DIM],
                                         const double (&aj)[DIM], const double (&bj)[DIM], double kq, double c1,
                                         double c2, double (&gq)[DIM], double (&gp)[DIM])
{
    double d[DIM];
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        d[c] = qk[c] - qj[c];
        s = __builtin_fma(d[c], d[c], s);
    }
    double g, w, u;
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
        const double e = bk[c] - bj[c];
        ed = __builtin_fma(e, d[c], ed);
        apj = __builtin_fma(ak[c], pj[c], __builtin_fma(aj[c], pk[c], apj));
        pp = __builtin_fma(pk[c], pj[c], pp);
    }
    const double t1 = w * ed;
    const double td = __builtin_fma(pp * ed, u, -w * apj);   // coefficient of d in aq
    const double te = pp * w;                               // coefficient of e in aq
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        gp[c] = __builtin_fma(g, aj[c], gp[c]);
        gp[c] = __builtin_fma(t1, pj[c], gp[c]);
        gq[c] = __builtin_fma(td, d[c], gq[c]);
        gq[c] = __builtin_fma(te, bk[c] - bj[c], gq[c]);
    }
}

// What the owner of target k does with its VJP sums (gq, gp).
template <int DIM>
__device__ __forceinline__ void adj_epilogue(const AdjEpi& e, int64_t n, int64_t k, const double (&gq)[DIM],
                                             const double (&gp)[DIM])
{
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        const int64_t o = c * n + k;
        const double yq = e.cscale * gq[c];
        const double yp = e.cscale * __builtin_fma(e.tau, e.cot_q[o], gp[c]);
        double lq, lp;
        if (e.kind == ADJ_STORE) {
            e.lam_q[o] = yq;
            e.lam_p[o] = yp;
            continue;
        }
        if (e.kind == ADJ_FIRST) {
            lq = e.abar_q[o] + yq;
            lp = e.abar_p[o] + yp;
        } else {
            lq = e.lam_q[o] + yq;
            lp = e.lam_p[o] + yp;
        }
        e.lam_q[o] = lq;
        e.lam_p[o] = lp;
        if (e.kind != ADJ_LAST) {
            e.nxt_q[o] = __builtin_fma(e.ca, e.abar_q[o], e.cy * yq);
            e.nxt_p[o] = __builtin_fma(e.ca, e.abar_p[o], e.cy * yp);
        }
    }
}

template <int DIM, int KER>
__global__ __launch_bounds__(kTileA * kWavesA) void lm_vjp_kernel(VjpArgs A)
{
    const int lane = threadIdx.x & (kTileA - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t n = A.n;
    const int64_t k = (int64_t)blockIdx.x * kTileA + lane;
    const bool live = k < n;
    const int64_t kc = live ? k : n - 1;
    double qk[DIM], pk[DIM], ak[DIM], bk[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        qk[c] = A.q[c * n + kc];
        pk[c] = A.p[c * n + kc];
        ak[c] = A.a[c * n + kc];
        bk[c] = A.b[c * n + kc];
    }
    const int64_t chunk = (int64_t)blockIdx.y * kWavesA + wave;
    const int64_t j0 = chunk * A.jchunk;
    const int64_t j1 = (j0 + A.jchunk < n) ? (j0 + A.jchunk) : n;
    double gq[DIM], gp[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) { gq[c] = 0.0; gp[c] = 0.0; }
    // sources come from the interleaved copy: one base address, 4 DIM consecutive doubles per
    // source, so a source is a few wide scalar loads and the loop needs few SGPRs
    const double* __restrict__ src = A.pack;
    int64_t j = j0;
    for (; j + LM_VJP_UNROLL <= j1; j += LM_VJP_UNROLL) {
#pragma unroll
        for (int uu = 0; uu < LM_VJP_UNROLL; ++uu) {
            const double* sj = src + (j + uu) * (4 * DIM);
            double qj[DIM], pj[DIM], aj[DIM], bj[DIM];
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                qj[c] = sj[c];
                pj[c] = sj[DIM + c];
                aj[c] = sj[2 * DIM + c];
                bj[c] = sj[3 * DIM + c];
            }
            vjp_pair<DIM, KER>(qk, pk, ak, bk, qj, pj, aj, bj, A.kq, A.c1, A.c2, gq, gp);
        }
    }
    for (; j < j1; ++j) {
        const double* sj = src + j * (4 * DIM);
        double qj[DIM], pj[DIM], aj[DIM], bj[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            qj[c] = sj[c];
            pj[c] = sj[DIM + c];
            aj[c] = sj[2 * DIM + c];
            bj[c] = sj[3 * DIM + c];
        }
        vjp_pair<DIM, KER>(qk, pk, ak, bk, qj, pj, aj, bj, A.kq, A.c1, A.c2, gq, gp);
    }

    __shared__ double red[kWavesA][2 * DIM][kTileA];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        red[wave][c][lane] = gq[c];
        red[wave][DIM + c][lane] = gp[c];
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        double sq = red[0][c][lane], sp = red[0][DIM + c][lane];
#pragma unroll
        for (int w = 1; w < kWavesA; ++w) {
            sq += red[w][c][lane];
            sp += red[w][DIM + c][lane];
        }
        gq[c] = sq;
        gp[c] = sp;
    }
    if (!live) return;
    if (gridDim.y > 1) {
        double* part = A.part + (int64_t)blockIdx.y * (2 * DIM) * n;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            part[c * n + k] = gq[c];
            part[(DIM + c) * n + k] = gp[c];
        }
        return;
    }
    adj_epilogue<DIM>(A.epi, n, k, gq, gp);
}

// Adds the partial sums of each target in a fixed order (as lm_finish_kernel: four waves per
// 64 targets, wave w taking slots w, w + 4, ..., the wave sums added in wave order), then
// runs the adjoint epilogue.
template <int DIM>
__global__ __launch_bounds__(256) void lm_vjp_finish_kernel(const double* __restrict__ part, int nsplit, int64_t n,
                                                            AdjEpi e)
{
    constexpr int NV = 2 * DIM;
    __shared__ double red[3][NV][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t k = (int64_t)blockIdx.x * 64 + lane;
    const bool live = k < n;
    const int64_t slot = (int64_t)NV * n;
    double acc[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) acc[c] = 0.0;
    if (live) {
        const double* ps = part + k;
        int s = wave;
        for (; s + 12 < nsplit; s += 16) {
            double x[4][NV];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int c = 0; c < NV; ++c) x[u][c] = ps[(s + 4 * u) * slot + c * n];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int c = 0; c < NV; ++c) acc[c] += x[u][c];
        }
        for (; s < nsplit; s += 4)
#pragma unroll
            for (int c = 0; c < NV; ++c) acc[c] += ps[s * slot + c * n];
    }
    if (wave > 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) red[wave - 1][c][lane] = acc[c];
    __syncthreads();
    if (wave != 0 || !live) return;
    double gq[DIM], gp[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        gq[c] = acc[c];
        gp[c] = acc[DIM + c];
#pragma unroll
        for (int w = 0; w < 3; ++w) {
            gq[c] += red[w][c][lane];
            gp[c] += red[w][DIM + c][lane];
        }
    }
    adj_epilogue<DIM>(e, n, k, gq, gp);
}

__global__ __launch_bounds__(256) void lm_scale_kernel(double* __restrict__ y, double alpha, const double* __restrict__ x,
                                                       int64_t m)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = alpha * x[i];
}

// pack[j][0..4 DIM) = (q_j, p_j, a_j, b_j)
template <int DIM>
__global__ __launch_bounds__(256) void lm_vjp_pack_kernel(const double* __restrict__ q, const double* __restrict__ p,
                                                          const double* __restrict__ a, const double* __restrict__ b,
                                                          int64_t n, double* __restrict__ pack)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        double* o = pack + j * (4 * DIM);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            o[c] = q[c * n + j];
            o[DIM + c] = p[c * n + j];
            o[2 * DIM + c] = a[c * n + j];
            o[3 * DIM + c] = b[c * n + j];
        }
    }
}

template <int DIM, int KER>
static hipError_t launch_vjp_t(const VjpArgs& a, const PairPlan& pl, hipStream_t st)
{
    hipError_t err;
    if (pl.sym_waves > 0) {
        err = launch_sym_vjp(DIM, KER, a, pl.sym_waves, pl.sym_nsb, st);
    } else {
        const int64_t pg = (a.n + 255) / 256;
        hipLaunchKernelGGL((lm_vjp_pack_kernel<DIM>), dim3((unsigned)(pg < 65536 ? pg : 65536)), dim3(256), 0, st, a.q,
                           a.p, a.a, a.b, a.n, a.pack);
        hipLaunchKernelGGL((lm_vjp_kernel<DIM, KER>), dim3((unsigned)pl.itiles, (unsigned)pl.nsplit),
                           dim3(kTileA * kWavesA), 0, st, a);
        err = hipGetLastError();
    }
    if (err != hipSuccess || pl.nsplit == 1) return err;
    const unsigned g = (unsigned)((a.n + 63) / 64);
    hipLaunchKernelGGL((lm_vjp_finish_kernel<DIM>), dim3(g), dim3(256), 0, st, (const double*)a.part, pl.nsplit, a.n,
                       a.epi);
    return hipGetLastError();
}

hipError_t launch_vjp(int dim, int kernel, const VjpArgs& a, const PairPlan& pl, hipStream_t st)
{
    if (dim == 2)
        return kernel == LM_KERNEL_CONON ? launch_vjp_t<2, LM_KERNEL_CONON>(a, pl, st)
                                         : launch_vjp_t<2, LM_KERNEL_GAUSS>(a, pl, st);
    return kernel == LM_KERNEL_CONON ? launch_vjp_t<3, LM_KERNEL_CONON>(a, pl, st)
                                     : launch_vjp_t<3, LM_KERNEL_GAUSS>(a, pl, st);
}

hipError_t launch_scale(double* y, double alpha, const double* x, int64_t m, hipStream_t st)
{
    int64_t b = (m + 255) / 256;
    hipLaunchKernelGGL(lm_scale_kernel, dim3((unsigned)(b < 8192 ? (b < 1 ? 1 : b) : 8192)), dim3(256), 0, st, y,
                       alpha, x, m);
    return hipGetLastError();
}

}  // namespace lm
